/*
 * ddo.c -- CPU oracle for the cumulative damage-diffusion distribution.
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow reference that the GPU library
 * is compared against.  Only tests, the smoke check and the benchmark's CPU
 * baseline may load it.  No code, header, table or constant is shared with
 * the GPU library.
 *
 * What it computes is the plain definition, in long double:
 *   psi(r, t) = sum over visits i with t_i < t of phi_i(r, t)     (Eq. 6)
 *   phi_i     = Q0/(4 pi D) [E1(a/b1) - E1(a/b0)]                  (Eqs. 1-2)
 *   phi_i     = Q0/(4 pi D) ln(b1/b0)            when r = r_i      (Eqs. 3-4)
 * with a = |r - r_i|^2, Ds = r_s^2 = sigma^2, b1 = 2Ds + 4D(t - t_i),
 * b0 = 2Ds while the beam is on (t <= t_i + tau) and
 * b0 = 2Ds + 4D(t - t_i - tau) once it is off.
 * A uniform scan takes t_i = i tau on a probe lattice; a general visit list
 * (ddo_psi_points_general) gives every visit its own position, start time
 * and dwell, and the same sum runs over it.
 *
 * Parity status of every function is pinned by tests (series vs continued
 * fraction vs quadrature vs library E1, heat-kernel time quadrature, a -> 0
 * limit, Fick's law residual, mass balance, symmetry, scaling; for general
 * visit lists: heat-kernel quadrature, the uniform scan, dwell splitting).
 */
#include "ddo.h"

#include <math.h>
#include <pthread.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define EULER_GAMMA_L 0.577215664901532860606512090082402431L
#define PI_L 3.141592653589793238462643383279502884L

/* ------------------------------------------------------------------------ */
/* E1 by its power series about zero (A&S 5.1.11):
 *   E1(x) = -gamma - ln x - sum_{n>=1} (-x)^n / (n * n!).
 * Used for x <= 1 (and in tests, a little beyond, to overlap the CF).     */
long double ddo_e1_series(long double x) {
  long double term = 1.0L; /* (-x)^n / n! */
  long double sum = 0.0L;
  for (int n = 1; n < 400; ++n) {
    term *= -x / (long double)n;
    long double add = term / (long double)n;
    sum += add;
    if (fabsl(add) <= 1e-22L * fabsl(sum)) break;
  }
  return -EULER_GAMMA_L - logl(x) - sum;
}

/* E1 by the continued fraction A&S 5.1.22, written in its even (contracted)
 * form  E1(x) = exp(-x) / G,  G = (x+1) - 1^2/((x+3) - 2^2/((x+5) - ...)),
 * evaluated front to back with the modified Lentz scheme.                  */
long double ddo_e1_cf(long double x) {
  const long double tiny = 1e-4000L;
  long double f = x + 1.0L; /* b0 */
  long double C = f, Dn = 0.0L;
  for (int j = 1; j < 100000; ++j) {
    long double aj = -(long double)j * (long double)j;
    long double bj = x + 2.0L * j + 1.0L;
    Dn = bj + aj * Dn;
    if (Dn == 0.0L) Dn = tiny;
    C = bj + aj / C;
    if (C == 0.0L) C = tiny;
    Dn = 1.0L / Dn;
    long double delta = C * Dn;
    f *= delta;
    if (fabsl(delta - 1.0L) < 1e-21L) break;
  }
  return expl(-x) / f;
}

/* Gauss-Legendre nodes/weights on [-1, 1] by Newton on the Legendre
 * recurrence (used only by the quadrature form of E1).                     */
#define GL_N 12
static void gauss_legendre(long double *xs, long double *ws) {
  for (int i = 0; i < GL_N; ++i) {
    long double z = cosl(PI_L * (i + 0.75L) / (GL_N + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int k = 1; k < GL_N; ++k) {
        long double p2 = ((2.0L * k + 1.0L) * z * p1 - k * p0) / (k + 1.0L);
        p0 = p1;
        p1 = p2;
      }
      dp = GL_N * (z * p1 - p0) / (z * z - 1.0L);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-20L) break;
    }
    xs[i] = z;
    ws[i] = 2.0L / ((1.0L - z * z) * dp * dp);
  }
}

/* E1 by quadrature of its definition, E1(x) = int_x^inf e^-u/u du, after
 * u = e^s:  E1(x) = int_{ln x}^{inf} exp(-e^s) ds.  Composite Gauss-Legendre
 * with panels no wider than 0.05 in s nor 0.25 in u, stopped once the
 * integrand is below 1e-40 of the running sum.                             */
long double ddo_e1_quad(long double x) {
  long double xs[GL_N], ws[GL_N];
  gauss_legendre(xs, ws);
  long double s = logl(x), sum = 0.0L;
  for (int panel = 0; panel < 10000000; ++panel) {
    long double h = 0.25L * expl(-s);
    if (h > 0.05L) h = 0.05L;
    long double mid = s + 0.5L * h, part = 0.0L;
    for (int i = 0; i < GL_N; ++i) part += ws[i] * expl(-expl(mid + 0.5L * h * xs[i]));
    sum += 0.5L * h * part;
    s += h;
    if (expl(-expl(s)) < 1e-40L * sum) break;
  }
  return sum;
}

static long double e1l(long double x) { return x <= 1.0L ? ddo_e1_series(x) : ddo_e1_cf(x); }

double ddo_e1(double x) { return (double)e1l((long double)x); }

/* ------------------------------------------------------------------------ */
/* Dimensionless bracket of Eqs. 1-4 (without Q0/(4 pi D)).                 */
static long double phi_bracket(long double a, long double dt, long double tau, long double Ds,
                               long double D) {
  if (dt <= 0.0L) return 0.0L;                 /* visit not started (Eq. 6 sums to j) */
  long double b1 = 2.0L * Ds + 4.0L * D * dt;  /* beam on since t_i     */
  long double b0 = (dt <= tau) ? 2.0L * Ds     /* Eq. 1: still on       */
                               : 2.0L * Ds + 4.0L * D * (dt - tau); /* Eq. 2: off */
  if (a == 0.0L) return logl(b1 / b0);         /* Eqs. 3-4 at r = r_i   */
  return e1l(a / b1) - e1l(a / b0);
}

double ddo_phi(double a, double dt, double tau, double sigma, double D, double Q0) {
  long double Ds = (long double)sigma * (long double)sigma;
  long double br = phi_bracket(a, dt, tau, Ds, D);
  return (double)((long double)Q0 / (4.0L * PI_L * (long double)D) * br);
}

/* ------------------------------------------------------------------------ */
/* The same bracket in IEEE binary128 (libquadmath), for per-pair checks
 * where E1(a/b1) and E1(a/b0) nearly coincide and the long-double
 * difference loses up to ~log10(E1/phi) digits.  Same series and continued
 * fraction as above, carried to 113-bit precision.                         */
static __float128 e1q(__float128 x) {
  if (x <= 1.0Q) {
    __float128 term = 1.0Q, sum = 0.0Q;
    for (int n = 1; n < 400; ++n) {
      term *= -x / (__float128)n;
      __float128 add = term / (__float128)n;
      sum += add;
      if (fabsq(add) <= 1e-36Q * fabsq(sum)) break;
    }
    return -0.5772156649015328606065120900824024310422Q - logq(x) - sum;
  }
  const __float128 tiny = 1e-4900Q;
  __float128 f = x + 1.0Q, C = f, Dn = 0.0Q;
  for (int j = 1; j < 1000000; ++j) {
    __float128 aj = -(__float128)j * (__float128)j;
    __float128 bj = x + 2.0Q * j + 1.0Q;
    Dn = bj + aj * Dn;
    if (Dn == 0.0Q) Dn = tiny;
    C = bj + aj / C;
    if (C == 0.0Q) C = tiny;
    Dn = 1.0Q / Dn;
    __float128 delta = C * Dn;
    f *= delta;
    if (fabsq(delta - 1.0Q) < 1e-34Q) break;
  }
  return expq(-x) / f;
}

double ddo_e1_q(double x) { return (double)e1q((__float128)x); }

double ddo_phi_bracket_q(double a, double dt, double tau, double sigma, double D) {
  if (dt <= 0.0) return 0.0;
  __float128 Ds = (__float128)sigma * (__float128)sigma;
  __float128 b1 = 2.0Q * Ds + 4.0Q * (__float128)D * (__float128)dt;
  __float128 b0 = (dt <= tau) ? 2.0Q * Ds
                              : 2.0Q * Ds + 4.0Q * (__float128)D * ((__float128)dt - (__float128)tau);
  if (a == 0.0) return (double)logq(b1 / b0);
  return (double)(e1q((__float128)a / b1) - e1q((__float128)a / b0));
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 as published by Steele, Lea & Flood (OOPSLA 2014).            */
uint64_t ddo_splitmix64(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Unbiased integer in [0, n) by Lemire's multiply-and-reject method
 * (ACM TOMACS 2019), fed with the top 32 bits of each SplitMix64 output.   */
static uint32_t bounded(uint64_t *state, uint32_t n) {
  uint32_t x = (uint32_t)(ddo_splitmix64(state) >> 32);
  uint64_t m = (uint64_t)x * (uint64_t)n;
  uint32_t low = (uint32_t)m;
  if (low < n) {
    uint32_t thresh = (uint32_t)(-n) % n;
    while (low < thresh) {
      x = (uint32_t)(ddo_splitmix64(state) >> 32);
      m = (uint64_t)x * (uint64_t)n;
      low = (uint32_t)m;
    }
  }
  return (uint32_t)(m >> 32);
}

int64_t ddo_visits(int order, int32_t nx, int32_t ny, int32_t stride, int32_t frames,
                   uint64_t seed, int32_t *out, int64_t cap) {
  if (nx < 1 || ny < 1) return -1;
  int64_t n = (int64_t)nx * ny;
  if (n > 0x7fffffff) return -1;
  if (order == DDO_RASTER) {
    if (cap < n) return -1;
    for (int64_t v = 0; v < n; ++v) out[v] = (int32_t)v;
    return n;
  }
  if (order == DDO_INTERLEAVED) {
    /* stride^2 sub-lattice passes, offsets (oy, ox) in row-major order; each
     * pass rasters rows oy, oy+s, ... and in each row columns ox, ox+s, ... */
    if (stride < 1 || cap < n) return -1;
    int64_t v = 0;
    for (int oy = 0; oy < stride; ++oy)
      for (int ox = 0; ox < stride; ++ox)
        for (int r = oy; r < ny; r += stride)
          for (int c = ox; c < nx; c += stride) out[v++] = r * nx + c;
    return v;
  }
  if (order == DDO_RANDOM) {
    /* Fisher-Yates from the last slot down, j uniform in [0, i]. */
    if (cap < n) return -1;
    uint64_t st = seed;
    for (int64_t v = 0; v < n; ++v) out[v] = (int32_t)v;
    for (int64_t i = n - 1; i >= 1; --i) {
      uint32_t j = bounded(&st, (uint32_t)(i + 1));
      int32_t tmp = out[i];
      out[i] = out[j];
      out[j] = tmp;
    }
    return n;
  }
  if (order == DDO_MULTIFRAME) {
    /* `frames` consecutive raster frames. */
    if (frames < 1) return -1;
    int64_t total = n * frames;
    if (total > 0x7fffffff || cap < total) return -1;
    for (int64_t v = 0; v < total; ++v) out[v] = (int32_t)(v % n);
    return total;
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* psi at one point: plain loop over every visit that started before t.     */
static long double psi_point(const ddo_scan *s, long double x, long double y, long double t) {
  long double Ds = (long double)s->sigma * (long double)s->sigma;
  long double D = s->D, tau = s->tau_v, p = s->pitch;
  long double sum = 0.0L;
  for (int64_t v = 0; v < s->n_visits; ++v) {
    long double tv = (long double)v * tau;
    if (!(tv < t)) break; /* visits start in order, so the rest are later */
    int32_t id = s->ids[v];
    long double px = (long double)(id % s->nx) * p, py = (long double)(id / s->nx) * p;
    long double dx = x - px, dy = y - py;
    sum += phi_bracket(dx * dx + dy * dy, t - tv, tau, Ds, D);
  }
  return (long double)s->Q0 / (4.0L * PI_L * D) * sum;
}

/* psi at one point of a general visit list: every visit that started before t. */
static long double psi_point_general(const ddo_vlist *g, long double x, long double y,
                                     long double t) {
  long double Ds = (long double)g->sigma * (long double)g->sigma;
  long double D = g->D;
  long double sum = 0.0L;
  for (int64_t v = 0; v < g->n; ++v) {
    long double tv = g->t0[v];
    if (!(tv < t)) continue;
    long double dx = x - (long double)g->x[v], dy = y - (long double)g->y[v];
    sum += phi_bracket(dx * dx + dy * dy, t - tv, (long double)g->dwell[v], Ds, D);
  }
  return (long double)g->Q0 / (4.0L * PI_L * D) * sum;
}

typedef struct {
  const ddo_scan *s;
  const ddo_vlist *g;
  int kind; /* 0 points, 1 arrival, 2 map, 3 points of a general visit list */
  int64_t n;
  const double *x, *y, *t;
  const int64_t *idx;
  double x0, y0, dx, dy;
  int32_t w, h;
  double *out;
  int tid, nth;
} job_t;

static void *worker(void *arg) {
  job_t *j = (job_t *)arg;
  const ddo_scan *s = j->s;
  for (int64_t k = j->tid; k < j->n; k += j->nth) {
    long double x, y, t;
    if (j->kind == 3) {
      j->out[k] = (double)psi_point_general(j->g, j->x[k], j->y[k], j->t[k]);
      continue;
    }
    if (j->kind == 0) {
      x = j->x[k];
      y = j->y[k];
      t = j->t[k];
    } else if (j->kind == 1) {
      int64_t v = j->idx[k];
      int32_t id = s->ids[v];
      x = (long double)(id % s->nx) * s->pitch;
      y = (long double)(id / s->nx) * s->pitch;
      t = (long double)v * (long double)s->tau_v;
    } else {
      int64_t per = (int64_t)j->w * j->h;
      int64_t m = k / per, rem = k % per;
      int64_t v = rem / j->w, u = rem % j->w;
      x = (long double)j->x0 + (long double)u * (long double)j->dx;
      y = (long double)j->y0 + (long double)v * (long double)j->dy;
      t = j->t[m];
    }
    j->out[k] = (double)psi_point(s, x, y, t);
  }
  return NULL;
}

int ddo_default_threads(void) {
  long n = sysconf(_SC_NPROCESSORS_ONLN);
  return n > 0 ? (int)n : 1;
}

static int run_jobs(job_t *tmpl, int nthreads) {
  if (nthreads <= 0) nthreads = ddo_default_threads();
  if (nthreads > 256) nthreads = 256;
  if (tmpl->n < nthreads) nthreads = tmpl->n > 0 ? (int)tmpl->n : 1;
  pthread_t th[256];
  job_t jobs[256];
  for (int i = 0; i < nthreads; ++i) {
    jobs[i] = *tmpl;
    jobs[i].tid = i;
    jobs[i].nth = nthreads;
    if (pthread_create(&th[i], NULL, worker, &jobs[i]) != 0) {
      /* fall back to finishing the rest on this thread */
      for (int k = i; k < nthreads; ++k) {
        jobs[k] = *tmpl;
        jobs[k].tid = k;
        jobs[k].nth = nthreads;
        worker(&jobs[k]);
      }
      for (int k = 0; k < i; ++k) pthread_join(th[k], NULL);
      return 0;
    }
  }
  for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
  return 0;
}

static int scan_ok(const ddo_scan *s) {
  return s && s->ids && s->nx >= 1 && s->ny >= 1 && s->n_visits >= 0 && s->pitch > 0 &&
         s->tau_v > 0 && s->sigma > 0 && s->D > 0;
}

int ddo_psi_points(const ddo_scan *s, int64_t n, const double *x, const double *y,
                   const double *t, double *out, int nthreads) {
  if (!scan_ok(s) || n < 0 || (n > 0 && (!x || !y || !t || !out))) return -1;
  job_t j;
  memset(&j, 0, sizeof j);
  j.s = s; j.kind = 0; j.n = n; j.x = x; j.y = y; j.t = t; j.out = out;
  return run_jobs(&j, nthreads);
}

int ddo_psi_arrival(const ddo_scan *s, int64_t n, const int64_t *visit_idx, double *out,
                    int nthreads) {
  if (!scan_ok(s) || n < 0 || (n > 0 && (!visit_idx || !out))) return -1;
  for (int64_t k = 0; k < n; ++k)
    if (visit_idx[k] < 0 || visit_idx[k] >= s->n_visits) return -1;
  job_t j;
  memset(&j, 0, sizeof j);
  j.s = s; j.kind = 1; j.n = n; j.idx = visit_idx; j.out = out;
  return run_jobs(&j, nthreads);
}

int ddo_psi_map(const ddo_scan *s, double x0, double y0, double dx, double dy, int32_t w,
                int32_t h, const double *t, int32_t nt, double *out, int nthreads) {
  if (!scan_ok(s) || w < 0 || h < 0 || nt < 0 || (nt > 0 && (!t || !out))) return -1;
  job_t j;
  memset(&j, 0, sizeof j);
  j.s = s; j.kind = 2; j.n = (int64_t)w * h * nt; j.t = t; j.out = out;
  j.x0 = x0; j.y0 = y0; j.dx = dx; j.dy = dy; j.w = w; j.h = h;
  return run_jobs(&j, nthreads);
}

int ddo_psi_points_general(const ddo_vlist *g, int64_t n, const double *px, const double *py,
                           const double *pt, double *out, int nthreads) {
  if (!g || g->n < 0 || (g->n > 0 && (!g->x || !g->y || !g->t0 || !g->dwell)) ||
      !(g->sigma > 0) || !(g->D > 0) || n < 0 || (n > 0 && (!px || !py || !pt || !out)))
    return -1;
  for (int64_t v = 0; v < g->n; ++v)
    if (!(g->dwell[v] > 0)) return -1;
  job_t j;
  memset(&j, 0, sizeof j);
  j.g = g; j.kind = 3; j.n = n; j.x = px; j.y = py; j.t = pt; j.out = out;
  return run_jobs(&j, nthreads);
}
