// dd_kernels.hip -- HIP kernels of libdd for gfx950 (CDNA4, wave64).
//
// The hot path is the all-pairs sum of Eq. 6 (Sec. II): every evaluation
// point adds the pair term of Eqs. 1-4 for every visit that started before it.
// It is a transcendental pair sum, not a contraction, so it runs on the vector
// ALUs (no MFMA).  The design keeps everything that depends only on the lag
// (time since a visit started) uniform across a wavefront:
//
//  * arrival query (evaluation point = visit j at its start time): a wave owns
//    64 R consecutive visits (R per lane) and walks the lag n; the probe of
//    pair (j, n) is visit j - n, so all 64 R pairs of one step share one lag
//    row (read into SGPRs) and each lane slides a window of 2R - 1 probe
//    positions (R loads per R^2 pairs);
//  * map query (evaluation points = pixels at one time): a wave owns 64 R
//    pixels and walks the visits; probe position and lag row are both
//    uniform (SGPR operands), only the pixel coordinates live in VGPRs.
//
// Lags split into a near band (per-pair choice between the series and the
// direct E1 difference) and a far region where every pair of the tile is in
// the series regime; there the series degree M is a template parameter chosen
// per lag segment, so the inner loop has no branches.  Partial sums of work
// items go to fixed slots and are added in a fixed order (bitwise
// reproducible, no floating-point atomics).
#include "dd_items.h"
#include "dd_kernels.h"

namespace dd {

__global__ void __launch_bounds__(256) k_lag_rows(int64_t n0, int64_t count, double f, double kappa,
                                                  double s2, GLNodes gl, double* __restrict__ rows64,
                                                  float* __restrict__ rows32) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x) {
    make_row(f + (double)(n0 + k), kappa, s2, gl, rows64 + k * kRow64, rows32 + k * kRow32);
  }
}

// ---------------------------------------------------------------------------
// Grid-mapped kernels: wavefront w of block b takes item 4 b + w.  RANGE = 1
// marks the launches of a visit-range query: the same code as a whole-scan
// query, instantiated apart so that kernel traces report the two separately.
template <int R, int RANGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_arrival_far32(const float4* __restrict__ pos,
                                                       const float* __restrict__ rows,
                                                       const ArrItem* __restrict__ items, int n_items,
                                                       int64_t V, DegreeBounds bnd,
                                                       double* __restrict__ partial, int64_t pstride,
                                                       int64_t pj0) {
  const int it = blockIdx.x * 4 + wave_id();
  if (it >= n_items) return;
  do_arrival_far32<R, false>(items[it], pos, rows, V, bnd, partial, pstride, pj0);
}

template <int R, int RANGE>
__global__ void __launch_bounds__(256) k_arrival_far64(const double2* __restrict__ pos,
                                                       const double* __restrict__ rows,
                                                       const ArrItem* __restrict__ items, int n_items,
                                                       int64_t V, DegreeBounds bnd,
                                                       double* __restrict__ partial, int64_t pstride,
                                                       int64_t pj0) {
  const int it = blockIdx.x * 4 + wave_id();
  if (it >= n_items) return;
  do_arrival_far64<R>(items[it], pos, rows, V, bnd, partial, pstride, pj0);
}

template <int R, bool MIXED, int RANGE>
__global__ void __launch_bounds__(256) k_arrival_near(const void* __restrict__ pos_v,
                                                      const double* __restrict__ rows64,
                                                      const float* __restrict__ rows32,
                                                      const ArrItem* __restrict__ items, int n_items,
                                                      int64_t V, double* __restrict__ partial,
                                                      int64_t pstride, int64_t pj0) {
  const int it = blockIdx.x * 4 + wave_id();
  if (it >= n_items) return;
  do_arrival_near<R, MIXED>(items[it], pos_v, rows64, rows32, V, partial, pstride, pj0);
}

template <int R, bool MIXED>
__global__ void __launch_bounds__(256) k_map(const void* __restrict__ pos_v,
                                             const float4* __restrict__ pos4,
                                             const double* __restrict__ rows64,
                                             const float* __restrict__ rows32,
                                             const MapItem* __restrict__ items, int n_items,
                                             const MapTime* __restrict__ times, double X0, double Y0,
                                             double DX, double DY, int W, int H, int lattice,
                                             double* __restrict__ partial) {
  const int it = blockIdx.x * 4 + wave_id();
  if (it >= n_items) return;
  const MapItem item = items[it];
  do_map<R, MIXED>(item, times[item.m], pos_v, pos4, rows64, rows32, X0, Y0, DX, DY, W, H,
                   lattice != 0, partial);
}

// ---------------------------------------------------------------------------
// Fixed-order reductions of the partial slots.
// out[i] = pref * (sum of the slots of visit j0 + i), i < n.
__global__ void __launch_bounds__(256) k_reduce_arrival(const double* __restrict__ partial,
                                                        const int32_t* __restrict__ tile_slots,
                                                        int64_t pstride, int64_t pj0, int tile,
                                                        double pref, int64_t j0, int64_t n,
                                                        double* __restrict__ out, OutFlag fl) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = j0 + i;
    const int ns = tile_slots[j / tile];
    double s = 0.0;
    for (int k = 0; k < ns; ++k) s += partial[(int64_t)k * pstride + (j - pj0)];
    const double v = pref * s;
    out[i] = v;
    flag_nonfinite(fl, v, i);
  }
}

// The same sums when a visit has many slots (a visit range with short lag
// chunks): one wave per visit, lane l adding slots l, l + 64, ... in order,
// then a butterfly over the lanes in a fixed pattern (deterministic).
__global__ void __launch_bounds__(256) k_reduce_arrival_wide(const double* __restrict__ partial,
                                                             const int32_t* __restrict__ tile_slots,
                                                             int64_t pstride, int64_t pj0, int tile,
                                                             double pref, int64_t j0, int64_t n,
                                                             double* __restrict__ out, OutFlag fl) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = blockIdx.x * 4 + wave_id(); i < n; i += (int64_t)gridDim.x * 4) {
    const int64_t j = j0 + i;
    const int ns = tile_slots[j / tile];
    double s = 0.0;
    for (int k = lane; k < ns; k += 64) s += partial[(int64_t)k * pstride + (j - pj0)];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    if (lane == 0) {
      const double v = pref * s;
      out[i] = v;
      flag_nonfinite(fl, v, i);
    }
  }
}

__global__ void __launch_bounds__(256) k_reduce_map(const double* __restrict__ partial,
                                                    const MapTime* __restrict__ times, int n_t,
                                                    int64_t npix, double pref,
                                                    double* __restrict__ out, OutFlag fl) {
  const int64_t total = npix * n_t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / npix, pix = e % npix;
    const MapTime tm = times[m];
    double s = 0.0;
    for (int k = 0; k < tm.n_slots; ++k) s += partial[(tm.slot_base + k) * npix + pix];
    const double v = pref * s;
    out[e] = v;
    flag_nonfinite(fl, v, e);
  }
}

// ---------------------------------------------------------------------------
// Pair terms for testing the device math: one thread per (a, lag).
__global__ void __launch_bounds__(256) k_pair_terms(double kappa, double s2, int64_t n,
                                                    const double* __restrict__ a,
                                                    const double* __restrict__ lag, int mixed,
                                                    GLNodes gl, double* __restrict__ out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    double r64[kRow64];
    float r32[kRow32];
    make_row(lag[k], kappa, s2, gl, r64, r32);
    const double ak = a[k];
    double v;
    if (!(lag[k] > 0.0)) {
      v = 0.0;
    } else if (mixed) {
      const float af = (float)ak;
      if (af * r32[kR32_C] <= kThr32)
        v = (double)series_f32<kMNear32>(af, r32);
      else
        v = phi_general_mixed(af, r64, r32);
    } else {
      v = phi_general_f64(ak, r64);
    }
    out[k] = v;
  }
}

// ---------------------------------------------------------------------------
// Launchers.
static inline unsigned grid_for(int64_t n, int64_t cap = 65536) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_lag_rows(int64_t n0, int64_t count, double f, double kappa, double s2,
                           const GLNodes& gl, double* rows64, float* rows32, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lag_rows, dim3(grid_for(count, 4096)), dim3(256), 0, st, n0, count, f,
                     kappa, s2, gl, rows64, rows32);
  return hipGetLastError();
}

template <int R, int RANGE>
static void launch_arrival_r(const ArrivalLaunch& L, hipStream_t st, unsigned blocks) {
  if (L.mixed) {
    hipLaunchKernelGGL((k_arrival_far32<R, RANGE>), dim3(blocks), dim3(256), 0, st, L.pos4,
                       L.rows32, L.items, L.n_items, L.V, L.bounds, L.partial, L.pstride, L.pj0);
  } else {
    hipLaunchKernelGGL((k_arrival_far64<R, RANGE>), dim3(blocks), dim3(256), 0, st,
                       (const double2*)L.pos, L.rows64, L.items, L.n_items, L.V, L.bounds,
                       L.partial, L.pstride, L.pj0);
  }
}

template <int R, int RANGE>
static void launch_arrival_near_r(const ArrivalLaunch& L, hipStream_t st, unsigned blocks) {
  if (L.mixed)
    hipLaunchKernelGGL((k_arrival_near<R, true, RANGE>), dim3(blocks), dim3(256), 0, st, L.pos,
                       L.rows64, L.rows32, L.items, L.n_items, L.V, L.partial, L.pstride, L.pj0);
  else
    hipLaunchKernelGGL((k_arrival_near<R, false, RANGE>), dim3(blocks), dim3(256), 0, st, L.pos,
                       L.rows64, L.rows32, L.items, L.n_items, L.V, L.partial, L.pstride, L.pj0);
}

template <int R>
static void launch_arrival_kind(const ArrivalLaunch& L, hipStream_t st, unsigned blocks) {
  if (L.near)
    L.range ? launch_arrival_near_r<R, 1>(L, st, blocks) : launch_arrival_near_r<R, 0>(L, st, blocks);
  else
    L.range ? launch_arrival_r<R, 1>(L, st, blocks) : launch_arrival_r<R, 0>(L, st, blocks);
}

// Near-band and far-region items are launched separately (L.near).
hipError_t launch_arrival(const ArrivalLaunch& L, hipStream_t st) {
  if (L.n_items <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((L.n_items + 3) / 4);
  switch (L.R) {
    case 2: launch_arrival_kind<2>(L, st, blocks); break;
    case 4: launch_arrival_kind<4>(L, st, blocks); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_map(const MapLaunch& L, hipStream_t st) {
  if (L.n_items <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((L.n_items + 3) / 4);
#define DD_LAUNCH_MAP(RR)                                                                       \
  if (L.mixed)                                                                                  \
    hipLaunchKernelGGL((k_map<RR, true>), dim3(blocks), dim3(256), 0, st, L.pos, L.pos4,       \
                       L.rows64, L.rows32, L.items, L.n_items, L.times, L.X0, L.Y0, L.DX, L.DY, \
                       L.W, L.H, L.lattice ? 1 : 0, L.partial);                                 \
  else                                                                                          \
    hipLaunchKernelGGL((k_map<RR, false>), dim3(blocks), dim3(256), 0, st, L.pos, L.pos4,      \
                       L.rows64, L.rows32, L.items, L.n_items, L.times, L.X0, L.Y0, L.DX, L.DY, \
                       L.W, L.H, L.lattice ? 1 : 0, L.partial);
  switch (L.R) {
    case 1: DD_LAUNCH_MAP(1) break;
    case 2: DD_LAUNCH_MAP(2) break;
    case 4: DD_LAUNCH_MAP(4) break;
    default: return hipErrorInvalidValue;
  }
#undef DD_LAUNCH_MAP
  return hipGetLastError();
}

hipError_t launch_reduce_arrival(const double* partial, const int32_t* tile_slots,
                                 int64_t pstride, int64_t pj0, int tile, double pref, int64_t j0,
                                 int64_t n, double* out, OutFlag fl, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_arrival, dim3(grid_for(n)), dim3(256), 0, st, partial, tile_slots,
                     pstride, pj0, tile, pref, j0, n, out, fl);
  return hipGetLastError();
}

hipError_t launch_reduce_arrival_wide(const double* partial, const int32_t* tile_slots,
                                      int64_t pstride, int64_t pj0, int tile, double pref,
                                      int64_t j0, int64_t n, double* out, OutFlag fl,
                                      hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 3) / 4, 65536);
  hipLaunchKernelGGL(k_reduce_arrival_wide, dim3(blocks), dim3(256), 0, st, partial, tile_slots,
                     pstride, pj0, tile, pref, j0, n, out, fl);
  return hipGetLastError();
}

hipError_t launch_reduce_map(const double* partial, const MapTime* times, int32_t n_t,
                             int64_t npix, double pref, double* out, OutFlag fl, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_map, dim3(grid_for(npix * n_t)), dim3(256), 0, st, partial, times,
                     n_t, npix, pref, out, fl);
  return hipGetLastError();
}

hipError_t launch_pair_terms(double kappa, double s2, int64_t n, const double* a,
                             const double* lag, bool mixed, const GLNodes& gl, double* out,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_terms, dim3(grid_for(n, 4096)), dim3(256), 0, st, kappa, s2, n, a, lag,
                     mixed ? 1 : 0, gl, out);
  return hipGetLastError();
}

}  // namespace dd
