// dd_items.h -- per-work-item device code of libdd, shared by the per-scan
// kernels (dd_kernels.hip) and the persistent batched kernel (dd_batch.hip).
// One wavefront processes one work item; see dd_kernels.hip for the design.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dd_device.h"
#include "dd_internal.h"

namespace dd {

// ---------------------------------------------------------------------------
// Lag rows (see dd_internal.h for the series).  J_m(w) by 24-node
// Gauss-Legendre on [0, 1] when w <= 1 (the integrand's pole at u = -1/w is at
// least 1 away), by the forward recurrence J_{m+1} = (1/(m+1) - J_m) / w when
// w > 1 (errors shrink by 1/w per step).
__device__ inline void make_row(double lam, double kappa, double s2, const GLNodes& gl, double* r64,
                         float* r32) {
  if (!(lam > 0.0)) {
    for (int k = 0; k < kRow64; ++k) r64[k] = 0.0;
    for (int k = 0; k < kRow32; ++k) r32[k] = 0.0f;
    return;
  }
  const double db = 4.0 * kappa * fmin(lam, 1.0);
  const double b0 = s2 + 4.0 * kappa * fmax(lam - 1.0, 0.0);
  const double b1 = b0 + db;
  const double w = db / b0;
  const double rb1 = 1.0 / b1, rb0 = 1.0 / b0;
  const double c = db / (b0 * b1);
  double J[kM64 + 1];
  if (w <= 1.0) {
    for (int m = 0; m <= kM64; ++m) J[m] = 0.0;
    for (int k = 0; k < kGL; ++k) {
      const double u = gl.x[k];
      double f = gl.w[k] / (1.0 + w * u);
      for (int m = 0; m <= kM64; ++m) {
        J[m] += f;
        f *= u;
      }
    }
  } else {
    J[0] = log1p(w) / w;
    for (int m = 0; m < kM64; ++m) J[m + 1] = (1.0 / (m + 1) - J[m]) / w;
  }
  double P[kM64 + 1];
  P[0] = log1p(w);
  double inv_fact = 1.0;
  for (int m = 1; m <= kM64; ++m) {
    inv_fact /= m;
    P[m] = ((m & 1) ? -1.0 : 1.0) * w * J[m] * inv_fact;
  }
  const double rl2 = rb1 * kLog2e;
  r64[kR64_RB1] = rb1;
  r64[kR64_RB0] = rb0;
  r64[kR64_C] = c;
  r64[kR64_RL2] = rl2;
  for (int m = 0; m <= kM64; ++m) r64[kR64_P + m] = P[m];
  for (int k = kR64_P + kM64 + 1; k < kRow64; ++k) r64[k] = 0.0;
  const float rhi = (float)rl2;
  const float rlo = (float)(rl2 - (double)rhi);
  r32[kR32_RHI] = rhi;
  r32[kR32_P0] = (float)P[0];
  double cm = 1.0;
  for (int m = 1; m <= kMaxA; ++m) {
    cm *= c;
    r32[kR32_PA + m - 1] = (float)(P[m] * cm + (m == 1 ? -kLn2 * P[0] * (double)rlo : 0.0));
  }
  r32[kR32_P0N] = (float)(-kLn2 * P[0]);
  r32[kR32_P0NR] = (float)(-kLn2 * P[0] * (double)rlo);
  r32[kR32_C] = (float)c;
  r32[kR32_RLO] = rlo;
  for (int m = 1; m <= kM32; ++m) r32[kR32_P1 + m - 1] = (float)P[m];
  for (int k = kR32_P1 + kM32; k < kRow32; ++k) r32[k] = 0.0f;
  r32[kR32_RA] = (float)(kLog2e * (rb1 - c * (P[1] / P[0])));
}


// ---------------------------------------------------------------------------
// Small helpers.
template <int R>
__device__ __forceinline__ float pairwise_sum(const float (&t)[R]) {
  if constexpr (R == 1) {
    return t[0];
  } else if constexpr (R == 2) {
    return t[0] + t[1];
  } else if constexpr (R == 4) {
    return (t[0] + t[1]) + (t[2] + t[3]);
  } else {
    static_assert(R == 8, "R must be 1, 2, 4 or 8");
    return ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
  }
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ---------------------------------------------------------------------------
// Arrival query, far region, mixed precision.  Lags [lo, hi) with
// (hi - lo) % R == 0; window W[q] holds the probe of visit jl - n0 - (R-1) + q
// as (-2x, -2y, x^2 + y^2), so that a = |e|^2 + |p|^2 - 2 e.p takes three
// exact FP32 operations (lattice coordinates below 2048).  For degrees <= 3
// the rows of the next R lags are fetched (scalar loads) while the current R
// lags are evaluated.
// Forms of the far series by row range (see DegreeBounds): the full form,
// the a-form without the exponent's rounding correction, and the folded
// single exponential P_0 2^{-a RA}.
enum { kFormFull = 0, kFormPlain = 1, kFormFold = 2 };

// The two fields of the folded form.
struct RowF {
  float ra, p0;
};

template <int M, int F = kFormFull>
struct RowSel {
  // folded: RA and P_0; degree <= 3: the 8 bulk fields; higher degrees read
  // the row in place
  using type = typename std::conditional<
      F == kFormFold, RowF,
      typename std::conditional<(M <= kMaxA), RowA, const float*>::type>::type;
};

template <int M, bool CAS = true, int F = kFormFull>
__device__ __forceinline__ typename RowSel<M, F>::type fetch_row(const float* __restrict__ rows,
                                                                 int64_t n) {
  if constexpr (F == kFormFold) {
    const float* row = rows + n * kRow32;
    if constexpr (CAS)
      return RowF{ldc(row + kR32_RA), ldc(row + kR32_P0)};
    else
      return RowF{row[kR32_RA], row[kR32_P0]};
  } else if constexpr (M <= kMaxA) {
    return load_rowa<CAS>(rows + n * kRow32);
  } else {
    return rows + n * kRow32;
  }
}

template <int M, int F = kFormFull>
__device__ __forceinline__ float series_row32(float a, const typename RowSel<M, F>::type& row) {
  if constexpr (F == kFormFold) {
    return row.p0 * __builtin_amdgcn_exp2f(-(a * row.ra));
  } else if constexpr (M <= kMaxA) {
    static_assert(F == kFormFull || F == kFormPlain, "unknown form");
    return series_f32a<M, F == kFormFull>(a, row);
  } else {
    static_assert(F == kFormFull, "the lighter forms need degree <= 3");
    return series_f32<M>(a, row);
  }
}

// The term as its two factors (q returned, t set), for sums that must not
// depend on how the compiler fuses products into additions.
template <int M>
__device__ __forceinline__ float series_row32_q(float a, const typename RowSel<M>::type& row,
                                                float& t) {
  if constexpr (M <= kMaxA)
    return series_f32a_q<M>(a, row, t);
  else
    return series_f32_q<M>(a, row, t);
}

// One chunk of R lags n0 .. n0+R-1 against window W (see arr_far32); the R
// terms of each evaluation point are summed in FP32 by fused multiply-adds
// (R roundings) and then added to its FP64 accumulator.
template <int M, int R, bool EDGE, int F>
__device__ __forceinline__ void arr_chunk32(int n0, int64_t jl, const float4 (&W)[2 * R - 1],
                                            const float (&ex)[R], const float (&ey)[R],
                                            const float (&ee)[R],
                                            const typename RowSel<M, F>::type (&row)[R],
                                            double (&acc)[R]) {
  float part[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float4 p = W[r - s + R - 1];
      const float a = __builtin_fmaf(ex[r], p.x, __builtin_fmaf(ey[r], p.y, ee[r] + p.z));
      float v = series_row32<M, F>(a, row[s]);
      if (EDGE) v = (jl + r >= (int64_t)(n0 + s)) ? v : 0.0f;
      part[r] = (s == 0) ? v : part[r] + v;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] += (double)part[r];
}

// A visit position of the arrival window (per lane); CAS: through the global
// address space, for pointers read from memory.
template <bool CAS>
__device__ __forceinline__ float4 ldpos(const float4* p) {
  if constexpr (CAS)
    return ldg3(p);
  else
    return *p;
}

template <int M, int R, bool EDGE, bool CAS, int F = kFormFull>
__device__ __forceinline__ void arr_far32(int lo, int hi, const float4* __restrict__ pos, int64_t jl,
                                          const float (&ex)[R], const float (&ey)[R],
                                          const float (&ee)[R], const float* __restrict__ rows,
                                          double (&acc)[R]) {
  using Row = typename RowSel<M, F>::type;
  // Two windows alternate: A covers the chunk at n0, B the chunk at n0 + R.
  // Each shares R - 1 positions with the other, copied in registers; loading
  // the whole window per chunk instead costs more than those moves.
  float4 A[2 * R - 1], B[2 * R - 1];
#pragma unroll
  for (int q = 0; q < 2 * R - 1; ++q) A[q] = ldpos<CAS>(pos + (jl - lo - (R - 1) + q));
  Row cur[R];
#pragma unroll
  for (int s = 0; s < R; ++s) cur[s] = fetch_row<M, CAS, F>(rows, lo + s);
  int n0 = lo;
  for (; n0 + 2 * R <= hi; n0 += 2 * R) {
    Row nxt[R];
#pragma unroll
    for (int s = 0; s < R; ++s) nxt[s] = fetch_row<M, CAS, F>(rows, n0 + R + s);
#pragma unroll
    for (int q = R; q < 2 * R - 1; ++q) B[q] = A[q - R];
    const int64_t b1 = jl - (n0 + R) - (R - 1);
#pragma unroll
    for (int q = 0; q < R; ++q) B[q] = ldpos<CAS>(pos + (b1 + q));
    arr_chunk32<M, R, EDGE, F>(n0, jl, A, ex, ey, ee, cur, acc);
#pragma unroll
    for (int s = 0; s < R; ++s) cur[s] = fetch_row<M, CAS, F>(rows, min(n0 + 2 * R + s, hi - 1));
#pragma unroll
    for (int q = R; q < 2 * R - 1; ++q) A[q] = B[q - R];
    const int64_t b2 = jl - (n0 + 2 * R) - (R - 1);
#pragma unroll
    for (int q = 0; q < R; ++q) A[q] = ldpos<CAS>(pos + (b2 + q));
    arr_chunk32<M, R, EDGE, F>(n0 + R, jl, B, ex, ey, ee, nxt, acc);
  }
  if (n0 < hi) arr_chunk32<M, R, EDGE, F>(n0, jl, A, ex, ey, ee, cur, acc);  // one chunk left
}

template <int M, int R, bool EDGE>
__device__ __forceinline__ void arr_far64(int lo, int hi, const double2* __restrict__ pos, int64_t jl,
                                          const double (&ex)[R], const double (&ey)[R],
                                          const double* __restrict__ rows, double (&acc)[R]) {
  double2 W[2 * R - 1];
#pragma unroll
  for (int q = 0; q < 2 * R - 1; ++q) W[q] = pos[jl - lo - (R - 1) + q];
  for (int n0 = lo; n0 < hi; n0 += R) {
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const double* row = rows + (int64_t)(n0 + s) * kRow64;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double2 p = W[r - s + R - 1];
        const double dx = ex[r] - p.x, dy = ey[r] - p.y;
        const double a = fma(dy, dy, dx * dx);
        double v = series_f64<M>(a, row);
        if (EDGE) v = (jl + r >= (int64_t)(n0 + s)) ? v : 0.0;
        acc[r] += v;
      }
    }
#pragma unroll
    for (int q = 2 * R - 2; q >= R; --q) W[q] = W[q - R];
    const int64_t base = jl - (n0 + R) - (R - 1);
#pragma unroll
    for (int q = 0; q < R; ++q) W[q] = pos[base + q];
  }
}

// Degree dispatch for one segment (uniform branch).  PLAIN: the a-form
// without the exponent's rounding correction (degrees <= 3 only; the planner
// starts that range below degree 4).
template <int R, bool EDGE, bool CAS, bool PLAIN = false>
__device__ __forceinline__ void arr_far32_seg(int M, int lo, int hi, const float4* __restrict__ pos,
                                              int64_t jl, const float (&ex)[R], const float (&ey)[R],
                                              const float (&ee)[R], const float* __restrict__ rows,
                                              double (&acc)[R]) {
  if constexpr (PLAIN) {
    switch (M) {
      case 0: arr_far32<0, R, EDGE, CAS, kFormPlain>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
      case 1: arr_far32<1, R, EDGE, CAS, kFormPlain>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
      case 2: arr_far32<2, R, EDGE, CAS, kFormPlain>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
      default: arr_far32<3, R, EDGE, CAS, kFormPlain>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
    }
    return;
  }
  switch (M) {
    case 0: arr_far32<0, R, EDGE, CAS>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
    case 1: arr_far32<1, R, EDGE, CAS>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
    case 2: arr_far32<2, R, EDGE, CAS>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
    case 3: arr_far32<3, R, EDGE, CAS>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
    case 4: arr_far32<4, R, EDGE, CAS>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
    case 5: arr_far32<5, R, EDGE, CAS>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
    default: arr_far32<6, R, EDGE, CAS>(lo, hi, pos, jl, ex, ey, ee, rows, acc); break;
  }
}

template <int R, bool EDGE>
__device__ __forceinline__ void arr_far64_seg(int M, int lo, int hi, const double2* __restrict__ pos,
                                              int64_t jl, const double (&ex)[R], const double (&ey)[R],
                                              const double* __restrict__ rows, double (&acc)[R]) {
#define DD_CASE(k) \
  case k: arr_far64<k, R, EDGE>(lo, hi, pos, jl, ex, ey, rows, acc); break;
  switch (M) {
    DD_CASE(0) DD_CASE(1) DD_CASE(2) DD_CASE(3) DD_CASE(4) DD_CASE(5) DD_CASE(6) DD_CASE(7)
    DD_CASE(8) DD_CASE(9) DD_CASE(10) DD_CASE(11) DD_CASE(12) DD_CASE(13) DD_CASE(14)
    DD_CASE(15) DD_CASE(16)
    default: arr_far64<17, R, EDGE>(lo, hi, pos, jl, ex, ey, rows, acc); break;
  }
#undef DD_CASE
}

// Segment [lo, hi) of degree M within [n_lo, n_hi): M runs from m_max down.
__device__ __forceinline__ void seg_range(const DegreeBounds& b, int M, int n_lo, int n_hi, int& lo,
                                          int& hi) {
  lo = max(n_lo, b.b[M]);
  hi = (M == 0) ? n_hi : min(n_hi, b.b[M - 1]);
}

// One wavefront processes one arrival work item (far region).  The sums of
// visit j go to partial[slot * pstride + j - pj0]: pstride = V and pj0 = 0
// for a whole-scan query; a visit range keeps only the columns of its tiles.
template <int R, bool CAS>
__device__ __forceinline__ void do_arrival_far32(const ArrItem& item, const float4* __restrict__ pos,
                                                 const float* __restrict__ rows, int64_t V,
                                                 const DegreeBounds& bnd,
                                                 double* __restrict__ partial, int64_t pstride,
                                                 int64_t pj0) {
  const int lane = threadIdx.x & 63;
  const int64_t jl = (int64_t)item.tile * (64 * R) + (int64_t)R * lane;
  float ex[R], ey[R], ee[R];
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float4 e = pos[jl + r];
    ex[r] = -0.5f * e.x;
    ey[r] = -0.5f * e.y;
    ee[r] = e.z;
    acc[r] = 0.0;
  }
  const bool edge = (item.slot_flags & kItemEdge) != 0;
  // rows [n_lo, fold) by degree segment, each split at `plain`; then the
  // folded rows [fold, n_hi) whatever their degree segment
  const int n_fold = max(item.n_lo, min(item.n_hi, bnd.fold));
  for (int M = bnd.m_max; M >= 0; --M) {
    int lo, hi;
    seg_range(bnd, M, item.n_lo, n_fold, lo, hi);
    if (lo >= hi) continue;
    const int mid = max(lo, min(hi, bnd.plain));
    if (edge) {
      if (lo < mid) arr_far32_seg<R, true, CAS>(M, lo, mid, pos, jl, ex, ey, ee, rows, acc);
      if (mid < hi) arr_far32_seg<R, true, CAS, true>(M, mid, hi, pos, jl, ex, ey, ee, rows, acc);
    } else {
      if (lo < mid) arr_far32_seg<R, false, CAS>(M, lo, mid, pos, jl, ex, ey, ee, rows, acc);
      if (mid < hi) arr_far32_seg<R, false, CAS, true>(M, mid, hi, pos, jl, ex, ey, ee, rows, acc);
    }
  }
  if (n_fold < item.n_hi) {
    if (edge)
      arr_far32<0, R, true, CAS, kFormFold>(n_fold, item.n_hi, pos, jl, ex, ey, ee, rows, acc);
    else
      arr_far32<0, R, false, CAS, kFormFold>(n_fold, item.n_hi, pos, jl, ex, ey, ee, rows, acc);
  }
  const int64_t base = (int64_t)(item.slot_flags & kSlotMask) * pstride - pj0;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (jl + r < V) partial[base + jl + r] = acc[r];
}

template <int R>
__device__ __forceinline__ void do_arrival_far64(const ArrItem& item, const double2* __restrict__ pos,
                                                 const double* __restrict__ rows, int64_t V,
                                                 const DegreeBounds& bnd,
                                                 double* __restrict__ partial, int64_t pstride,
                                                 int64_t pj0) {
  const int lane = threadIdx.x & 63;
  const int64_t jl = (int64_t)item.tile * (64 * R) + (int64_t)R * lane;
  double ex[R], ey[R], acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double2 e = pos[jl + r];
    ex[r] = e.x;
    ey[r] = e.y;
    acc[r] = 0.0;
  }
  const bool edge = (item.slot_flags & kItemEdge) != 0;
  for (int M = bnd.m_max; M >= 0; --M) {
    int lo, hi;
    seg_range(bnd, M, item.n_lo, item.n_hi, lo, hi);
    if (lo >= hi) continue;
    if (edge)
      arr_far64_seg<R, true>(M, lo, hi, pos, jl, ex, ey, rows, acc);
    else
      arr_far64_seg<R, false>(M, lo, hi, pos, jl, ex, ey, rows, acc);
  }
  const int64_t base = (int64_t)(item.slot_flags & kSlotMask) * pstride - pj0;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (jl + r < V) partial[base + jl + r] = acc[r];
}

// Near band, mixed precision: the pairs that need the general form (series
// variable above the FP32 series' threshold, x1 within the cull) are few and
// scattered over the lanes; evaluated where they occur, the general form runs
// with most lanes idle.  They are queued instead, per lane in LDS (a and the
// lag), and evaluated by the whole wave whenever some lane's queue could
// overflow, and at the end: the queues are packed into one list at offsets
// from a prefix sum of their lengths, lane l evaluates list entries l, l + 64,
// ..., and each lane then adds its own values in the order it queued them
// (deterministic; the general-form terms of a flush enter the FP64 sum after
// the series terms of the same lags).
constexpr int kNearQ = 6;  // queued general-form pairs per lane
struct NearQueue {
  float a[kNearQ][64];
  int32_t n[kNearQ][64];  // lag | (r << 29)
  float fa[64 * kNearQ];  // the packed list
  int32_t fn[64 * kNearQ];
  double fv[64 * kNearQ];
};

__device__ __forceinline__ void near_wave_sync() {
  // a wave's LDS operations complete in order: a compiler barrier at
  // wavefront scope orders its writes before other lanes' reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int R>
__device__ __forceinline__ void near_flush(NearQueue& Q, int& cnt, const double* __restrict__ rows64,
                                           const float* __restrict__ rows32, double (&acc)[R]) {
  const int lane = threadIdx.x & 63;
  const int c = cnt;
  int s = c;  // inclusive prefix sum of the queue lengths over the lanes
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(s, d);
    if (lane >= d) s += t;
  }
  const int base = s - c, total = __shfl(s, 63);
#pragma unroll
  for (int k = 0; k < kNearQ; ++k)
    if (k < c) {
      Q.fa[base + k] = Q.a[k][lane];
      Q.fn[base + k] = Q.n[k][lane];
    }
  near_wave_sync();
  for (int e = lane; e < total; e += 64) {
    const int n = Q.fn[e] & 0x1fffffff;
    Q.fv[e] = phi_general_mixed(Q.fa[e], rows64 + (int64_t)n * kRow64, rows32 + (int64_t)n * kRow32);
  }
  near_wave_sync();
#pragma unroll
  for (int k = 0; k < kNearQ; ++k)
    if (k < c) {
      const int r = Q.fn[base + k] >> 29;
      const double v = Q.fv[base + k];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) acc[rr] += (rr == r) ? v : 0.0;  // no indexed registers
    }
  near_wave_sync();  // the queues and the list are rewritten next
  cnt = 0;
}

// Near band: per-pair regime choice, every pair masked by causality.
template <int R, bool MIXED>
__device__ __forceinline__ void do_arrival_near(const ArrItem& item, const void* __restrict__ pos_v,
                                                const double* __restrict__ rows64,
                                                const float* __restrict__ rows32, int64_t V,
                                                double* __restrict__ partial, int64_t pstride,
                                                int64_t pj0) {
  const int lane = threadIdx.x & 63;
  const int64_t jl = (int64_t)item.tile * (64 * R) + (int64_t)R * lane;
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  if (MIXED) {
    const float2* pos = (const float2*)pos_v;
    float ex[R], ey[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float2 e = pos[jl + r];
      ex[r] = e.x;
      ey[r] = e.y;
    }
    static_assert(R <= 4, "the queue entry holds r in two bits");
    __shared__ NearQueue queues[4];  // one per wave of the 256-thread block
    NearQueue& Q = queues[threadIdx.x >> 6];
    int cnt = 0;
    for (int n = item.n_lo; n < item.n_hi; ++n) {
      if (__ballot(cnt > kNearQ - R)) near_flush<R>(Q, cnt, rows64, rows32, acc);
      const float* r32 = rows32 + (int64_t)n * kRow32;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t i = jl + r - n;
        if (i >= 0 && jl + r < V) {
          const float2 p = pos[i];
          const float dx = ex[r] - p.x, dy = ey[r] - p.y;
          const float a = __builtin_fmaf(dy, dy, dx * dx);
          if (a * ldc(r32 + kR32_C) <= kThr32) {
            acc[r] += (double)series_f32<kMNear32>(a, r32);
          } else if (a * ldc(r32 + kR32_RHI) <= kCull32Log2) {
            Q.a[cnt][lane] = a;
            Q.n[cnt][lane] = n | (r << 29);
            ++cnt;
          }
        }
      }
    }
    if (__ballot(cnt > 0)) near_flush<R>(Q, cnt, rows64, rows32, acc);
  } else {
    const double2* pos = (const double2*)pos_v;
    double ex[R], ey[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double2 e = pos[jl + r];
      ex[r] = e.x;
      ey[r] = e.y;
    }
    for (int n = item.n_lo; n < item.n_hi; ++n) {
      const double* r64 = rows64 + (int64_t)n * kRow64;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t i = jl + r - n;
        if (i >= 0 && jl + r < V) {
          const double2 p = pos[i];
          const double dx = ex[r] - p.x, dy = ey[r] - p.y;
          acc[r] += phi_general_f64(fma(dy, dy, dx * dx), r64);
        }
      }
    }
  }
  const int64_t base = (int64_t)(item.slot_flags & kSlotMask) * pstride - pj0;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (jl + r < V) partial[base + jl + r] = acc[r];
}

// ---------------------------------------------------------------------------
// Map query.  Pixel pix = tile * 64 R + R lane + r at (X0 + u DX, Y0 + v DY),
// u = pix % W, v = pix / W, all at the item's time; visit v = K - n.
// LAT: pixel and probe coordinates are exact small dyadic numbers, so the
// three-operation a = |e|^2 + |p|^2 - 2 e.p is exact; otherwise a is formed
// from the differences (relative error ~1e-7, no cancellation).
template <bool LAT, int R>
__device__ __forceinline__ float map_a32(const float4& p, const float (&ex)[R], const float (&ey)[R],
                                         const float (&ee)[R], int r) {
  if (LAT) return __builtin_fmaf(ex[r], p.x, __builtin_fmaf(ey[r], p.y, ee[r] + p.z));
  const float dx = __builtin_fmaf(0.5f, p.x, ex[r]), dy = __builtin_fmaf(0.5f, p.y, ey[r]);
  return __builtin_fmaf(dy, dy, dx * dx);
}

template <int M, int R, int U, bool LAT>
__device__ __forceinline__ void map_far32(int lo, int hi, int64_t K, const float4* __restrict__ pos,
                                          const float* __restrict__ rows, const float (&ex)[R],
                                          const float (&ey)[R], const float (&ee)[R],
                                          double (&acc)[R]) {
  using Row = typename RowSel<M>::type;
  int n = lo;
  if (n + U <= hi) {
    Row cur[U];
    float4 pc[U];
#pragma unroll
    for (int s = 0; s < U; ++s) {
      cur[s] = fetch_row<M>(rows, n + s);
      pc[s] = ldc(pos + (K - (n + s)));
    }
    for (; n + U <= hi; n += U) {
      Row nxt[U];
      float4 pn[U];
#pragma unroll
      for (int s = 0; s < U; ++s) {
        const int nn = min(n + U + s, hi - 1);
        nxt[s] = fetch_row<M>(rows, nn);
        pn[s] = ldc(pos + (K - nn));
      }
      float t[R][U], qv[R][U];
#pragma unroll
      for (int s = 0; s < U; ++s) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          qv[r][s] = series_row32_q<M>(map_a32<LAT, R>(pc[s], ex, ey, ee, r), cur[s], t[r][s]);
      }
      // Groups of four lags in lag order, each summed by an explicit chain
      // of fused multiply-adds: the arithmetic of a pixel is then the same
      // for every tile width and unroll depth.
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < U; q += 4) {
          float g = t[r][q] * qv[r][q];
          g = __builtin_fmaf(t[r][q + 1], qv[r][q + 1], g);
          g = __builtin_fmaf(t[r][q + 2], qv[r][q + 2], g);
          g = __builtin_fmaf(t[r][q + 3], qv[r][q + 3], g);
          acc[r] += (double)g;
        }
#pragma unroll
      for (int s = 0; s < U; ++s) {
        cur[s] = nxt[s];
        pc[s] = pn[s];
      }
    }
  }
  for (; n < hi; ++n) {
    const float4 p = ldc(pos + (K - n));
    const Row row = fetch_row<M>(rows, n);
#pragma unroll
    for (int r = 0; r < R; ++r)
      acc[r] += (double)series_row32<M>(map_a32<LAT, R>(p, ex, ey, ee, r), row);
  }
}

// One-pixel tiles, degrees <= 3.  A one-pixel tile has too little work per
// lag to hide per-lag scalar loads of rows that are read once (as for a
// single map row), so the rows and probe positions of 64 lags at a time are
// brought into LDS by one vector load per lane, the next 64 in flight while
// the current ones are evaluated, and read back by broadcast.  The arithmetic
// and its order are those of map_far32: groups of four lags from lo, each an
// explicit FMA chain, then single lags.
__device__ __forceinline__ float4* map_r1_stage() {
  __shared__ float4 stage[4 * 2 * 64 * 3];  // wave, buffer, lag, (row lo, row hi, position)
  return stage;
}

template <int M, bool LAT>
__device__ __forceinline__ void map_far32_r1(int lo, int hi, int64_t K, const float4* __restrict__ pos,
                                             const float* __restrict__ rows, const float (&ex)[1],
                                             const float (&ey)[1], const float (&ee)[1],
                                             double (&acc)[1]) {
  static_assert(M <= kMaxA, "row staging holds the 8 fields of degrees <= 3");
  if (lo >= hi) return;
  const int lane = threadIdx.x & 63;
  float4* const st = map_r1_stage() + (threadIdx.x >> 6) * (2 * 64 * 3);
  // lane i fetches lag base + i (clamped into [lo, hi))
  auto fetch = [&](int base, float4& r0, float4& r1, float4& pp) {
    const int n = min(base + lane, hi - 1);
    const float4* row = reinterpret_cast<const float4*>(rows + (int64_t)n * kRow32);
    r0 = row[0];
    r1 = row[1];
    pp = pos[K - n];
  };
  auto put = [&](int buf, const float4& r0, const float4& r1, const float4& pp) {
    float4* d = st + (buf * 64 + lane) * 3;
    d[0] = r0;
    d[1] = r1;
    d[2] = pp;
  };
  auto term = [&](int buf, int j, float& t) {
    const float4* d = st + (buf * 64 + j) * 3;
    const float4 u = d[0], v = d[1], p = d[2];
    const RowA row{u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
    return series_f32a_q<M>(map_a32<LAT, 1>(p, ex, ey, ee, 0), row, t);
  };
  float4 r0, r1, pp;
  fetch(lo, r0, r1, pp);
  put(0, r0, r1, pp);
  __builtin_amdgcn_wave_barrier();
  int buf = 0;
  for (int base = lo; base < hi; base += 64, buf ^= 1) {
    const int cnt = min(64, hi - base);
    const bool more = base + 64 < hi;
    if (more) fetch(base + 64, r0, r1, pp);
    int j = 0;
    for (; j + 4 <= cnt; j += 4) {
      float t0, t1, t2, t3;
      const float q0 = term(buf, j, t0), q1 = term(buf, j + 1, t1);
      const float q2 = term(buf, j + 2, t2), q3 = term(buf, j + 3, t3);
      float g = t0 * q0;
      g = __builtin_fmaf(t1, q1, g);
      g = __builtin_fmaf(t2, q2, g);
      g = __builtin_fmaf(t3, q3, g);
      acc[0] += (double)g;
    }
    for (; j < cnt; ++j) {
      float t;
      const float q = term(buf, j, t);
      acc[0] += (double)(t * q);
    }
    if (more) {
      __builtin_amdgcn_wave_barrier();
      put(buf ^ 1, r0, r1, pp);
      __builtin_amdgcn_wave_barrier();
    }
  }
}

template <int M, int R>
__device__ __forceinline__ void map_far64(int lo, int hi, int64_t K, const double2* __restrict__ pos,
                                          const double* __restrict__ rows, const double (&ex)[R],
                                          const double (&ey)[R], double (&acc)[R]) {
  for (int n = lo; n < hi; ++n) {
    const double2 p = ldc(pos + (K - n));
    const double* row = rows + (int64_t)n * kRow64;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double dx = ex[r] - p.x, dy = ey[r] - p.y;
      double t;
      const double q = series_f64_q<M>(fma(dy, dy, dx * dx), row, t);
      acc[r] = fma(t, q, acc[r]);  // explicit: the same for every tile width
    }
  }
}

template <int R, int U, bool LAT>
__device__ __forceinline__ void map_far32_u(int M, int lo, int hi, int64_t K,
                                            const float4* __restrict__ pos,
                                            const float* __restrict__ rows, const float (&ex)[R],
                                            const float (&ey)[R], const float (&ee)[R],
                                            double (&acc)[R]) {
  switch (M) {
    case 0: map_far32<0, R, U, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); break;
    case 1: map_far32<1, R, U, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); break;
    case 2: map_far32<2, R, U, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); break;
    case 3: map_far32<3, R, U, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); break;
    case 4: map_far32<4, R, U, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); break;
    case 5: map_far32<5, R, U, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); break;
    default: map_far32<6, R, U, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); break;
  }
}

template <int R, bool LAT>
__device__ __forceinline__ void map_far32_seg(int M, int lo, int hi, int64_t K,
                                              const float4* __restrict__ pos,
                                              const float* __restrict__ rows, const float (&ex)[R],
                                              const float (&ey)[R], const float (&ee)[R],
                                              double (&acc)[R]) {
  // One pixel per lane: degrees <= 3 from rows staged in LDS; higher degrees
  // eight lags per step for more loads in flight.  The sum runs over groups
  // of four in lag order either way, so the result does not depend on the
  // tile width.
  if constexpr (R == 1) {
    switch (M) {
      case 0: map_far32_r1<0, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); return;
      case 1: map_far32_r1<1, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); return;
      case 2: map_far32_r1<2, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); return;
      case 3: map_far32_r1<3, LAT>(lo, hi, K, pos, rows, ex, ey, ee, acc); return;
      default: break;
    }
    const int mid = lo + ((hi - lo) & ~7);
    map_far32_u<R, 8, LAT>(M, lo, mid, K, pos, rows, ex, ey, ee, acc);
    lo = mid;
  }
  map_far32_u<R, 4, LAT>(M, lo, hi, K, pos, rows, ex, ey, ee, acc);
}

template <int R>
__device__ __forceinline__ void map_far64_seg(int M, int lo, int hi, int64_t K,
                                              const double2* __restrict__ pos,
                                              const double* __restrict__ rows, const double (&ex)[R],
                                              const double (&ey)[R], double (&acc)[R]) {
#define DD_CASE(k) \
  case k: map_far64<k, R>(lo, hi, K, pos, rows, ex, ey, acc); break;
  switch (M) {
    DD_CASE(0) DD_CASE(1) DD_CASE(2) DD_CASE(3) DD_CASE(4) DD_CASE(5) DD_CASE(6) DD_CASE(7)
    DD_CASE(8) DD_CASE(9) DD_CASE(10) DD_CASE(11) DD_CASE(12) DD_CASE(13) DD_CASE(14)
    DD_CASE(15) DD_CASE(16)
    default: map_far64<17, R>(lo, hi, K, pos, rows, ex, ey, acc); break;
  }
#undef DD_CASE
}

template <int R, bool MIXED>
__device__ __forceinline__ void do_map(const MapItem& item, const MapTime& tm,
                                       const void* __restrict__ pos_v,
                                       const float4* __restrict__ pos4,
                                       const double* __restrict__ rows64,
                                       const float* __restrict__ rows32, double X0, double Y0,
                                       double DX, double DY, int W, int H, bool lattice,
                                       double* __restrict__ partial) {
  const int lane = threadIdx.x & 63;
  const int64_t npix = (int64_t)W * H;
  const int64_t p0 = (int64_t)item.tile * (64 * R) + (int64_t)R * lane;
  double pxd[R], pyd[R], acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t pix = min(p0 + r, npix - 1);
    pxd[r] = X0 + (double)(pix % W) * DX;
    pyd[r] = Y0 + (double)(pix / W) * DY;
    acc[r] = 0.0;
  }
  const double* r64b = rows64 + tm.row_base * kRow64;
  const float* r32b = rows32 + tm.row_base * kRow32;
  if (MIXED) {
    const float2* pos = (const float2*)pos_v;
    float ex[R], ey[R], ee[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ex[r] = (float)pxd[r];
      ey[r] = (float)pyd[r];
      ee[r] = __builtin_fmaf(ey[r], ey[r], ex[r] * ex[r]);
    }
    if (item.near) {
      for (int n = item.n_lo; n < item.n_hi; ++n) {
        const float2 p = ldc(pos + (tm.K - n));
        const float* r32 = r32b + (int64_t)n * kRow32;
        const double* r64 = r64b + (int64_t)n * kRow64;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float dx = ex[r] - p.x, dy = ey[r] - p.y;
          const float a = __builtin_fmaf(dy, dy, dx * dx);
          if (a * ldc(r32 + kR32_C) <= kThr32)
            acc[r] += (double)series_f32<kMNear32>(a, r32);
          else if (a * ldc(r32 + kR32_RHI) <= kCull32Log2)
            acc[r] += phi_general_mixed(a, r64, r32);
        }
      }
    } else {
      for (int M = tm.bounds.m_max; M >= 0; --M) {
        int lo, hi;
        seg_range(tm.bounds, M, item.n_lo, item.n_hi, lo, hi);
        if (lo >= hi) continue;
        if (lattice)
          map_far32_seg<R, true>(M, lo, hi, tm.K, pos4, r32b, ex, ey, ee, acc);
        else
          map_far32_seg<R, false>(M, lo, hi, tm.K, pos4, r32b, ex, ey, ee, acc);
      }
    }
  } else {
    const double2* pos = (const double2*)pos_v;
    if (item.near) {
      for (int n = item.n_lo; n < item.n_hi; ++n) {
        const double2 p = ldc(pos + (tm.K - n));
        const double* r64 = r64b + (int64_t)n * kRow64;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double dx = pxd[r] - p.x, dy = pyd[r] - p.y;
          acc[r] += phi_general_f64(fma(dy, dy, dx * dx), r64);
        }
      }
    } else {
      for (int M = tm.bounds.m_max; M >= 0; --M) {
        int lo, hi;
        seg_range(tm.bounds, M, item.n_lo, item.n_hi, lo, hi);
        if (lo < hi) map_far64_seg<R>(M, lo, hi, tm.K, pos, r64b, pxd, pyd, acc);
      }
    }
  }
  double* out = partial + (tm.slot_base + item.slot) * npix;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (p0 + r < npix) out[p0 + r] = acc[r];
}

}  // namespace dd
