// dd_visits.hip -- FP64 kernels of the general visit list (per-visit
// position, start time and dwell; Eqs. 1-4 per visit, summed by Eq. 6).
//
// Pair term.  With b_hat = 2 + 4 D lag / sigma^2 (the b of Eqs. 1-2 over
// sigma^2), b0 at the end of the visit's beam-on time seen from t and b1 at
// its start, x1 = a/b1 < x0 = a/b0 and dx = x0 - x1 = a db / (b0 b1):
//   E1(x1) - E1(x0) = integral of e^-u / u over [x1, x0]
// and, at a = 0, ln(b1/b0) (Eqs. 3-4).  Every visit has its own b0 and db,
// so the per-lag series rows of the uniform scan do not exist here; the
// term is evaluated per pair in one of four forms:
//   * x1 > 745: zero (both E1 values below the double range);
//   * dx > 1: the difference of the two E1 values (series or continued
//     fraction), which differ by more than a factor e^-dx;
//   * q = db/b0 <= 1 (then x1 >= dx): u = x1 + w, w in [0, dx], as
//     e^-x1 times the integral of e^-w / (x1 + w), a function with no
//     singularity within a distance x1 >= dx of the interval: Gauss-Legendre
//     with 3 to 12 nodes by q and dx (see near_rule);
//   * q > 1: u = x1 e^s, s in [0, L], L = ln(1 + q), as e^-x1 times the
//     integral of exp(-x1 (e^s - 1)) (an entire function, exponent between
//     0 and dx <= 1): 12-node Gauss-Legendre while L <= 2; for L > 2,
//     x0 = dx (1 + 1/q) < 1.16 and L plus the difference of the two E1 power
//     series (18 terms) converges without cancellation.
// An emulation in double precision agrees with a 40-digit E1 difference to
// 1e-13 relative over b0, db in [2, 4e9] and the whole a range.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dd_device.h"
#include "dd_visits.h"

namespace dd {

namespace {

// Gauss-Legendre rule of N nodes on [0, 1] (nodes x, weights w summing to
// 1), computed at compile time: Newton iteration on P_N from the usual
// cosine estimates, then the weights 1 / ((1 - z^2) P_N'(z)^2) halved.
constexpr double ccos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 30; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
template <int N>
struct GLRule {
  double x[N], w[N];
  constexpr GLRule() : x(), w() {
    for (int i = 0; i < N; ++i) {
      double z = ccos(3.141592653589793 * (i + 0.75) / (N + 0.5)), dp = 1.0;
      for (int it = 0; it < 12; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 1; k < N; ++k) {
          const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
          p0 = p1;
          p1 = p2;
        }
        dp = N * (z * p1 - p0) / (z * z - 1.0);
        if (it < 11) z -= p1 / dp;
      }
      x[i] = 0.5 * (1.0 - z);
      w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

// 1/y for normal y > 0: hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp64(double y) {
  double r = __builtin_amdgcn_rcp(y);
  r = fma(r, fma(-y, r, 1.0), r);
  return fma(r, fma(-y, r, 1.0), r);
}

// e^-w for 0 <= w <= wmax by its Taylor polynomial of degree DEG (DEG = 7
// for w <= 0.03, 9 for w <= 0.1: remainder < 3e-17 relative).
template <int DEG>
__device__ __forceinline__ double exp_neg_small(double w) {
  constexpr InvFact f{};
  double p = f.v[DEG];
#pragma unroll
  for (int k = DEG - 1; k >= 0; --k) p = fma(p, -w, f.v[k]);
  return p;
}

// e^-x1 times the integral of e^-w / (x1 + w) over [0, dx] by the N-node
// rule (the near form for q = dx / x1 <= 1); EDEG > 0 takes e^-w from its
// Taylor polynomial (dx <= 0.1), else from exp.  e^-x1 comes from exp2_neg
// (relative error below 1e-13 up to x1 = 745, the FP64 per-term budget).
template <int N, int EDEG>
__device__ __forceinline__ double near_linear(double x1, double dx) {
  constexpr GLRule<N> g{};
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double w = dx * g.x[k];
    const double e = EDEG > 0 ? exp_neg_small<EDEG>(w) : ::exp(-w);
    s = fma(g.w[k], e * rcp64(x1 + w), s);
  }
  return exp2_neg<11>(x1 * kLog2e) * dx * s;
}

// Nodes of the linear near form.  The error of the N-node rule falls with
// q (the pole of 1/(x1 + w) sits q^-1 interval lengths away) and with dx
// (the e^-w factor); a study against a 40-digit E1 difference gives, at
// <= 2e-15 relative: 3 nodes for q <= 0.01 and dx <= 0.03, 4 for q <= 0.03
// and dx <= 0.1, 6 for q <= 0.1, 8 for q <= 0.3, 12 up to q = 1.
__device__ __forceinline__ int near_rule(double q, double dx) {
  if (q <= 0.01 && dx <= 0.03) return 0;
  if (q <= 0.03 && dx <= 0.1) return 1;
  if (q <= 0.1) return 2;
  return q <= 0.3 ? 3 : 4;
}

// The linear near form in FP32 for the mixed precision: e^-w and 1/(x1 + w)
// per node by the hardware exp2 and reciprocal (about 1 ulp each); e^-x1
// with its integer power of two split off in FP64 (x1 reaches 745, beyond
// the FP32 range, and x1 rounded to FP32 would cost x1 * 6e-8 relative).
template <int N>
__device__ __forceinline__ double near_linear_f32(double x1, double dx) {
  constexpr GLRule<N> g{};
  const float x1f = (float)x1, dxf = (float)dx;
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const float w = dxf * (float)g.x[k];
    const float e = __builtin_amdgcn_exp2f(-w * 1.44269504f);
    s = __builtin_fmaf((float)g.w[k], e * __builtin_amdgcn_rcpf(x1f + w), s);
  }
  const double y = x1 * kLog2e;
  const double n = __builtin_rint(y);
  const float f = (float)(n - y);  // |f| <= 1/2
  return __builtin_ldexp((double)(__builtin_amdgcn_exp2f(f) * dxf * s), -(int)n);
}

// Node counts of the FP32 form: rule errors below 4e-8 relative (same study
// as near_rule): 2 nodes for q <= 0.01 and dx <= 0.1, 3 for q <= 0.03 and
// dx <= 0.3, 4 for q <= 0.1, 6 for q <= 0.3, 8 up to q = 1.
__device__ __forceinline__ int near_rule_mixed(double q, double dx) {
  if (q <= 0.01 && dx <= 0.1) return 0;
  if (q <= 0.03 && dx <= 0.3) return 1;
  if (q <= 0.1) return 2;
  return q <= 0.3 ? 3 : 4;
}

// sum_{n>=1} (-1)^n x^n / (n n!) for x <= 1.16 (18 terms, remainder < 2e-17).
__device__ __forceinline__ double e1_series_tail(double x) {
  constexpr E1SeriesCoef k{};
  double s = k.c[17];
#pragma unroll
  for (int n = 16; n >= 0; --n) s = fma(s, x, k.c[n]);
  return x * s;
}

// E1(x1) - E1(x1 + dx) for the pairs outside the linear near form: dx > 1
// (direct difference), or q > 1 (log variable, or the series for L > 2).
__device__ __noinline__ double far_or_log_term(double x1, double dx, double q) {
  if (dx > 1.0) {
    const double x0 = x1 + dx;
    const double e0 = x0 > 745.0 ? 0.0 : e1_f64(x0);
    return e1_f64(x1) - e0;
  }
  const double L = ::log1p(q);
  if (L <= 2.0) {
    constexpr GLRule<12> g{};
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) s = fma(g.w[k], ::exp(-x1 * ::expm1(L * g.x[k])), s);
    return ::exp(-x1) * L * s;
  }
  // E1(x) = -gamma - ln x - tail(x): the difference is L + tail(x0) - tail(x1)
  const double x0 = x1 + dx;
  return L + (e1_series_tail(x0) - e1_series_tail(x1));
}

// The term of a pair that passed the cull (x1 <= 745); active = the pair
// contributes at all.  The linear near form, almost every pair of a long
// scan, runs with the node count the wave's lanes need at most, so that
// the branch is the same for the whole wave.
template <bool MIXED>
__device__ __forceinline__ double pair_term(bool active, double x1, double dx, double q) {
  const bool lin = active && dx <= 1.0 && q <= 1.0 && x1 > 0.0;
  double t = 0.0;
  if (__ballot(lin)) {
    const double u = lin ? x1 : 1.0, v = lin ? dx : 0.0;
    double r;
    if (MIXED) {
      const int need = lin ? near_rule_mixed(q, dx) : -1;
      if (__ballot(need == 4))
        r = near_linear_f32<8>(u, v);
      else if (__ballot(need == 3))
        r = near_linear_f32<6>(u, v);
      else if (__ballot(need == 2))
        r = near_linear_f32<4>(u, v);
      else if (__ballot(need == 1))
        r = near_linear_f32<3>(u, v);
      else
        r = near_linear_f32<2>(u, v);
    } else {
      const int need = lin ? near_rule(q, dx) : -1;
      if (__ballot(need == 4))
        r = near_linear<12, 0>(u, v);
      else if (__ballot(need == 3))
        r = near_linear<8, 0>(u, v);
      else if (__ballot(need == 2))
        r = near_linear<6, 0>(u, v);
      else if (__ballot(need == 1))
        r = near_linear<4, 9>(u, v);
      else
        r = near_linear<3, 7>(u, v);
    }
    t = lin ? r : 0.0;
  }
  if (active && !lin) t = far_or_log_term(x1, dx, q);
  return t;
}

// One block per item: 256 points (one per thread) against the item's visits,
// staged 256 at a time in LDS.  Visits are in start order, so the first one
// that starts at or after the tile's latest time ends the item for the
// whole block.  Map tiles share one time: the per-visit factors (1/b1,
// db/(b0 b1), db/b0) are then formed once per staged visit.
template <bool MAP, bool MIXED>
__global__ __launch_bounds__(kVisTile) void k_visit_pairs(
    const VisList* __restrict__ lists, const VisTile* __restrict__ tiles,
    const VisItem* __restrict__ items, int64_t n_items, double* __restrict__ partial) {
  __shared__ double4 s_v[kVisStage];
  __shared__ double4 s_f[MAP ? kVisStage : 1];
  const int lane = threadIdx.x;
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const VisItem item = items[it];
    const VisTile tile = tiles[item.tile];
    const VisList& L = lists[tile.list];
    const double4* __restrict__ vis = L.vis;
    const double inv_sigma = L.inv_sigma, th4 = L.th4;
    const bool live = lane < tile.n;
    double px = 0.0, py = 0.0, pt = tile.tmax;
    if (MAP) {
      const VisGrid grid = L.grid;
      const int64_t pix = tile.p0 + (live ? lane : 0);
      px = grid.x0 + (double)(pix % grid.w) * grid.dx;
      py = grid.y0 + (double)(pix / grid.w) * grid.dy;
      pt = L.times[tile.m];
    } else if (live) {
      const double4 me = vis[tile.p0 + lane];
      px = me.x;
      py = me.y;
      pt = me.z;
    }
    double sum = 0.0;
    bool done = false;
    for (int64_t v0 = item.v0; v0 < item.v0 + item.nv && !done; v0 += kVisStage) {
      const int64_t left = item.v0 + item.nv - v0;
      const int nk = left < kVisStage ? (int)left : kVisStage;
      __syncthreads();  // the previous stage is no longer read
      if (lane < nk) {
        const double4 v = vis[v0 + lane];
        s_v[lane] = v;
        if (MAP) {
          const double dt = pt - v.z;
          double4 f = make_double4(-1.0, 0.0, 0.0, 0.0);  // rb1 < 0: not started
          if (dt > 0.0) {
            const double on = fmin(dt, v.w), off = dt - on;
            const double b0 = fma(th4, off, 2.0), db = th4 * on, b1 = b0 + db;
            const double r0 = rcp64(b0), r1 = rcp64(b1);
            f = make_double4(r1, db * r0 * r1, db * r0, 0.0);
          }
          s_f[lane] = f;
        }
      }
      __syncthreads();
      for (int j = 0; j < nk; ++j) {
        const double4 v = s_v[j];
        if (v.z >= pt && MAP) {
          done = true;  // uniform: one time for the whole tile
          break;
        }
        if (!MAP && v.z >= tile.tmax) {
          done = true;  // uniform: no later visit starts before any point
          break;
        }
        const double ex = (px - v.x) * inv_sigma, ey = (py - v.y) * inv_sigma;
        const double a = fma(ex, ex, ey * ey);
        if (MAP) {
          const double4 f = s_f[j];
          const double x1 = a * f.x;
          sum += pair_term<MIXED>(live && f.x > 0.0 && x1 <= 745.0, x1, a * f.y, f.z);
        } else {
          const double dt = pt - v.z;
          const bool started = live && dt > 0.0;
          const double on = fmin(dt, v.w), off = dt - on;
          const double b0 = fma(th4, off, 2.0), db = th4 * on;
          const double b1 = b0 + db;
          const double rr = rcp64(started ? b0 * b1 : 4.0);  // 1 / (b0 b1)
          const double x1 = a * (b0 * rr), q = db * (b1 * rr);
          sum += pair_term<MIXED>(started && x1 <= 745.0, x1, x1 * q, q);
        }
      }
    }
    if (live) partial[tile.pbase + (int64_t)item.slot * kVisTile + lane] = sum;
  }
}

template <bool MAP>
__global__ __launch_bounds__(kVisTile) void k_visit_reduce(const VisList* __restrict__ lists,
                                                           const VisTile* __restrict__ tiles,
                                                           const double* __restrict__ partial) {
  const VisTile tile = tiles[blockIdx.x];
  const VisList& L = lists[tile.list];
  const int lane = threadIdx.x;
  if (lane >= tile.n) return;
  double s = 0.0;
  for (int k = 0; k < tile.slots; ++k) s += partial[tile.pbase + (int64_t)k * kVisTile + lane];
  const int64_t dst = MAP ? tile.out0 + lane : L.perm[tile.p0 + lane];
  const double v = L.pref * s;
  L.out[dst] = v;
  flag_nonfinite(L.fl, v, dst);
}

}  // namespace

hipError_t launch_visit_pairs(bool map, bool mixed, const VisList* lists, const VisTile* tiles,
                              const VisItem* items, int64_t n_items, double* partial,
                              hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>(n_items, 1 << 20);
#define DD_VISIT_LAUNCH(M, X)                                                                  \
  k_visit_pairs<M, X><<<blocks, kVisTile, 0, st>>>(lists, tiles, items, n_items, partial)
  if (map && mixed)
    DD_VISIT_LAUNCH(true, true);
  else if (map)
    DD_VISIT_LAUNCH(true, false);
  else if (mixed)
    DD_VISIT_LAUNCH(false, true);
  else
    DD_VISIT_LAUNCH(false, false);
#undef DD_VISIT_LAUNCH
  return hipGetLastError();
}

hipError_t launch_visit_reduce(bool map, const VisList* lists, const VisTile* tiles,
                               int64_t n_tiles, const double* partial, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (map)
    k_visit_reduce<true><<<(unsigned)n_tiles, kVisTile, 0, st>>>(lists, tiles, partial);
  else
    k_visit_reduce<false><<<(unsigned)n_tiles, kVisTile, 0, st>>>(lists, tiles, partial);
  return hipGetLastError();
}

}  // namespace dd
