/*
 * ddo.h -- CPU oracle for the cumulative damage-diffusion distribution.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain, obviously
 * correct reference that the GPU library is checked against.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source, header, table or constant with the GPU
 * library and it never calls it.
 *
 * Everything is evaluated in `long double` (x87 80-bit on x86-64) and
 * returned as `double`.  Units are whatever the caller uses consistently
 * (SI in the tests: metres, seconds, m^2/s, u/s).
 *
 * Paper: "Fast Simulation of Damage Diffusion Distribution in Scanning
 * Transmission Electron Microscopy", Sec. II (Eqs. 1-4 single-probe field,
 * Eq. 6 cumulative sum).
 */
#ifndef DDO_H
#define DDO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- exponential integral E1 (Sec. II, definition after Eq. 2) ---------- */
/* Power series of E1 about 0 (Abramowitz & Stegun 5.1.11); x > 0.          */
long double ddo_e1_series(long double x);
/* Continued fraction of E1 (A&S 5.1.22), modified Lentz; x > 0.           */
long double ddo_e1_cf(long double x);
/* Direct quadrature of the defining integral after u = e^s; x > 0.        */
long double ddo_e1_quad(long double x);
/* Oracle E1: series for x <= 1, continued fraction above.  x > 0.         */
double ddo_e1(double x);

/* ---- single-probe field (Sec. II, Eqs. 1-4) ------------------------------
 * phi_i(r, t) for one visit that started at t_i and lasted tau, at squared
 * distance a = |r - r_i|^2 and lag dt = t - t_i; r_s^2 = Ds = sigma^2.
 * Returns 0 for dt <= 0 (visit not yet started).                          */
double ddo_phi(double a, double dt, double tau, double sigma, double D, double Q0);

/* Eqs. 1-4 bracket E1(a/b1) - E1(a/b0) (or ln(b1/b0) at a = 0), without
 * Q0/(4 pi D), evaluated in IEEE binary128 to resolve nearly coincident
 * arguments; and E1 itself in binary128.                                  */
double ddo_phi_bracket_q(double a, double dt, double tau, double sigma, double D);
double ddo_e1_q(double x);

/* ---- scan orders (Sec. I scan strategies) -------------------------------- */
enum { DDO_RASTER = 0, DDO_INTERLEAVED = 1, DDO_RANDOM = 2, DDO_MULTIFRAME = 3 };
/* SplitMix64 step (Steele, Lea & Flood 2014); advances *state.            */
uint64_t ddo_splitmix64(uint64_t *state);
/* Writes the probe id (row * nx + col) of every visit in order into out
 * (capacity cap).  Returns the number of visits, or -1 on bad arguments.  */
int64_t ddo_visits(int order, int32_t nx, int32_t ny, int32_t stride, int32_t frames,
                   uint64_t seed, int32_t *out, int64_t cap);

/* ---- cumulative distribution (Sec. II, Eq. 6) -----------------------------
 * A scan: visit v (0-based) sits on probe id ids[v] at (col*pitch, row*pitch)
 * with col = id % nx, row = id / nx, starts at t_v = v * tau_v and lasts
 * tau_v.  psi(r, t) = sum over visits with t_v < t of phi_v(r, t).           */
typedef struct {
  int32_t nx, ny;
  const int32_t *ids;     /* [n_visits] */
  int64_t n_visits;
  double pitch, tau_v, sigma, D, Q0;
} ddo_scan;

/* psi at n arbitrary points (x[k], y[k], t[k]); nthreads <= 0 -> all cores.
 * Returns 0, or -1 on bad arguments.                                       */
int ddo_psi_points(const ddo_scan *s, int64_t n, const double *x, const double *y,
                   const double *t, double *out, int nthreads);
/* psi at the arrival of each listed visit j (point r_j, time t_j); the sum
 * then runs over visits v < j.                                             */
int ddo_psi_arrival(const ddo_scan *s, int64_t n, const int64_t *visit_idx, double *out,
                    int nthreads);
/* Map: pixel (u, v) at (x0 + u*dx, y0 + v*dy), times t[0..nt-1];
 * out[(m*h + v)*w + u].                                                    */
int ddo_psi_map(const ddo_scan *s, double x0, double y0, double dx, double dy, int32_t w,
                int32_t h, const double *t, int32_t nt, double *out, int nthreads);

/* ---- general visit lists --------------------------------------------------
 * Visit v at (x[v], y[v]) (metres), beam on from t0[v] for dwell[v]
 * seconds; visits in any order, each on its own window.  psi(r, t) = sum
 * over visits with t0[v] < t of phi_v(r, t) (Eqs. 1-4 with the visit's own
 * dwell, Eq. 6).                                                           */
typedef struct {
  int64_t n;
  const double *x, *y, *t0, *dwell; /* [n] */
  double sigma, D, Q0;
} ddo_vlist;

/* psi at n points (px[k], py[k], pt[k]); nthreads <= 0 -> all cores.
 * Returns 0, or -1 on bad arguments.                                       */
int ddo_psi_points_general(const ddo_vlist *g, int64_t n, const double *px, const double *py,
                           const double *pt, double *out, int nthreads);

/* Number of hardware threads the oracle uses for nthreads <= 0.           */
int ddo_default_threads(void);

#ifdef __cplusplus
}
#endif
#endif
