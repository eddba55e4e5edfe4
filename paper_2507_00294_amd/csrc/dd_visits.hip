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
//     singularity within a distance x1 >= dx of the interval: 12-node
//     Gauss-Legendre;
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

// sum_{n>=1} (-1)^n x^n / (n n!) for x <= 1.16 (18 terms, remainder < 2e-17).
__device__ __forceinline__ double e1_series_tail(double x) {
  constexpr E1SeriesCoef k{};
  double s = k.c[17];
#pragma unroll
  for (int n = 16; n >= 0; --n) s = fma(s, x, k.c[n]);
  return x * s;
}

// E1(x1) - E1(x1 + dx) for one pair; q = db / b0 (see the file comment).
__device__ __forceinline__ double visit_term(double x1, double dx, double q, const VisGL& g) {
  if (dx > 1.0) {
    const double x0 = x1 + dx;
    const double e0 = x0 > 745.0 ? 0.0 : e1_f64(x0);
    return e1_f64(x1) - e0;
  }
  if (q <= 1.0 && x1 > 0.0) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kVisGL; ++k) {
      const double w = dx * g.x[k];
      s = fma(g.w[k], ::exp(-w) / (x1 + w), s);
    }
    return ::exp(-x1) * dx * s;
  }
  const double L = ::log1p(q);
  if (L <= 2.0) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kVisGL; ++k) s = fma(g.w[k], ::exp(-x1 * ::expm1(L * g.x[k])), s);
    return ::exp(-x1) * L * s;
  }
  // E1(x) = -gamma - ln x - tail(x): the difference is L + tail(x0) - tail(x1)
  const double x0 = x1 + dx;
  return L + (e1_series_tail(x0) - e1_series_tail(x1));
}

// One block per item: 256 points (one per thread) against the item's visits,
// staged 256 at a time in LDS.  Visits are in start order, so the first one
// that starts at or after the tile's latest time ends the item for the
// whole block.  Map tiles share one time: the per-visit factors (1/b1,
// db/(b0 b1), db/b0) are then formed once per staged visit.
template <bool MAP>
__global__ __launch_bounds__(kVisTile) void k_visit_pairs(
    const double4* __restrict__ vis, const VisTile* __restrict__ tiles,
    const VisItem* __restrict__ items, int64_t n_items, const double* __restrict__ times,
    VisGrid grid, VisPhys ph, VisGL rule, double* __restrict__ partial) {
  __shared__ double4 s_v[kVisStage];
  __shared__ double4 s_f[MAP ? kVisStage : 1];
  const int lane = threadIdx.x;
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const VisItem item = items[it];
    const VisTile tile = tiles[item.tile];
    const bool live = lane < tile.n;
    double px = 0.0, py = 0.0, pt = tile.tmax;
    if (MAP) {
      const int64_t pix = tile.p0 + (live ? lane : 0);
      px = grid.x0 + (double)(pix % grid.w) * grid.dx;
      py = grid.y0 + (double)(pix / grid.w) * grid.dy;
      pt = times[tile.m];
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
            const double b0 = fma(ph.th4, off, 2.0), db = ph.th4 * on, b1 = b0 + db;
            f = make_double4(1.0 / b1, db / (b0 * b1), db / b0, 0.0);
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
        const double ex = (px - v.x) * ph.inv_sigma, ey = (py - v.y) * ph.inv_sigma;
        const double a = fma(ex, ex, ey * ey);
        if (MAP) {
          const double4 f = s_f[j];
          const double x1 = a * f.x;
          if (live && f.x > 0.0 && x1 <= 745.0) sum += visit_term(x1, a * f.y, f.z, rule);
        } else {
          const double dt = pt - v.z;
          if (live && dt > 0.0) {
            const double on = fmin(dt, v.w), off = dt - on;
            const double b0 = fma(ph.th4, off, 2.0), db = ph.th4 * on, b1 = b0 + db;
            const double x1 = a / b1;
            if (x1 <= 745.0) sum += visit_term(x1, a * (db / (b0 * b1)), db / b0, rule);
          }
        }
      }
    }
    if (live) partial[tile.pbase + (int64_t)item.slot * kVisTile + lane] = sum;
  }
}

__global__ __launch_bounds__(kVisTile) void k_visit_reduce(const VisTile* __restrict__ tiles,
                                                           const double* __restrict__ partial,
                                                           const int64_t* __restrict__ perm,
                                                           double pref, double* __restrict__ out) {
  const VisTile tile = tiles[blockIdx.x];
  const int lane = threadIdx.x;
  if (lane >= tile.n) return;
  double s = 0.0;
  for (int k = 0; k < tile.slots; ++k) s += partial[tile.pbase + (int64_t)k * kVisTile + lane];
  const int64_t dst = perm ? perm[tile.p0 + lane] : tile.out0 + lane;
  out[dst] = pref * s;
}

}  // namespace

hipError_t launch_visit_pairs(bool map, const double4* vis, const VisTile* tiles,
                              const VisItem* items, int64_t n_items, const double* times,
                              VisGrid grid, VisPhys phys, VisGL rule, double* partial,
                              hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>(n_items, 1 << 20);
  if (map)
    k_visit_pairs<true><<<blocks, kVisTile, 0, st>>>(vis, tiles, items, n_items, times, grid,
                                                     phys, rule, partial);
  else
    k_visit_pairs<false><<<blocks, kVisTile, 0, st>>>(vis, tiles, items, n_items, times, grid,
                                                      phys, rule, partial);
  return hipGetLastError();
}

hipError_t launch_visit_reduce(const VisTile* tiles, int64_t n_tiles, const double* partial,
                               const int64_t* perm, double pref, double* out, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  k_visit_reduce<<<(unsigned)n_tiles, kVisTile, 0, st>>>(tiles, partial, perm, pref, out);
  return hipGetLastError();
}

}  // namespace dd
