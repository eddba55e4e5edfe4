// dd_batch.hip -- the persistent batched kernel of libdd (many scans in one
// launch) and its fixed-order reduction.
#include <algorithm>

#include "dd_items.h"
#include "dd_kernels.h"

namespace dd {

// ---------------------------------------------------------------------------
// Persistent batched kernels: many scans, one launch per item kind (arrival
// far region, arrival near band, map far region, map near band), so that
// each kernel has the register budget of its own code.  Each wavefront takes the next item from a device counter until
// the list is exhausted (every wave reaches that exit).  The items were
// sorted longest first on the host; each item runs exactly the per-item code
// of the per-scan kernels, so batch results equal per-scan results bit for
// bit.
template <int R, bool MIXED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MIXED && R == 4 ? 3 : 1, 8)))
k_batch_arrival_far(const BatchScan* __restrict__ scans, const BatchItem* __restrict__ items,
                    int n_items, int* __restrict__ counter) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    int it = 0;
    if (lane == 0) it = atomicAdd(counter, 1);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= n_items) break;
    const BatchItem bi = items[it];
    const BatchScan& S = scans[bi.scan];
    const ArrItem ai{bi.tile, bi.n_lo, bi.n_hi, bi.slot_flags};
    if (MIXED)
      do_arrival_far32<R, true>(ai, S.pos4, S.rows32, S.V, S.arr_bounds, S.arr_partial, S.V, 0);
    else
      do_arrival_far64<R>(ai, (const double2*)S.pos, S.rows64, S.V, S.arr_bounds, S.arr_partial,
                          S.V, 0);
  }
}

template <int RN, bool MIXED>
__global__ void __launch_bounds__(256) k_batch_arrival_near(const BatchScan* __restrict__ scans,
                                                            const BatchItem* __restrict__ items,
                                                            int n_items, int* __restrict__ counter) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    int it = 0;
    if (lane == 0) it = atomicAdd(counter, 1);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= n_items) break;
    const BatchItem bi = items[it];
    const BatchScan& S = scans[bi.scan];
    const ArrItem ai{bi.tile, bi.n_lo, bi.n_hi, bi.slot_flags};
    do_arrival_near<RN, MIXED>(ai, S.pos, S.rows64, S.rows32, S.V, S.arr_partial, S.V, 0);
  }
}

// Map items; NEAR selects the near-band items (per-pair regimes) or the
// far-region items (degree segments).
template <int RM, bool MIXED, bool NEAR>
__global__ void __launch_bounds__(256) k_batch_map(const BatchScan* __restrict__ scans,
                                                   const BatchItem* __restrict__ items,
                                                   int n_items, int* __restrict__ counter) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    int it = 0;
    if (lane == 0) it = atomicAdd(counter, 1);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= n_items) break;
    const BatchItem bi = items[it];
    const BatchScan& S = scans[bi.scan];
    const MapItem mi{bi.tile, 0, bi.n_lo, bi.n_hi, bi.slot_flags & kSlotMask, NEAR ? 1 : 0, 0, 0};
    do_map<RM, MIXED>(mi, S.map_time, S.pos, S.pos4, S.rows64, S.rows32, (double)S.map_x0,
                      (double)S.map_y0, (double)S.map_step, (double)S.map_step, S.map_w, S.map_h,
                      true, S.map_partial);
  }
}

__global__ void k_zero_int(int* p) { *p = 0; }

// One pass over the outputs of a whole batch; entry found by binary search
// on the output offsets; slots added in the same order as the per-scan
// reductions.
__global__ void __launch_bounds__(256) k_reduce_batch(const BatchReduce* __restrict__ reds,
                                                      int n_red, int64_t total, OutFlag fl) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = n_red - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (reds[mid].out_off <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    const BatchReduce& Rd = reds[lo];
    const int64_t j = e - Rd.out_off;
    const int ns = Rd.tile_slots ? Rd.tile_slots[j / Rd.tile] : Rd.n_slots;
    double s = 0.0;
    for (int k = 0; k < ns; ++k) s += Rd.partial[(int64_t)k * Rd.n + j];
    const double v = Rd.pref * s;
    Rd.out[j] = v;
    flag_nonfinite(Rd.scan_flag, v, j);
    flag_nonfinite(fl, v, e);
  }
}

static inline unsigned batch_grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

// Persistent grid: enough waves to fill the chip a few times over.
static unsigned persistent_blocks(int32_t n_items) {
  return (unsigned)std::min<int64_t>((n_items + 3) / 4, 256 * 8);
}

hipError_t launch_batch(const BatchScan* scans, const BatchItem* items, int32_t n_items,
                        int* counter, int R, bool mixed, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, counter);
  const unsigned blocks = persistent_blocks(n_items);
#define DD_LAUNCH(A)                                                                            \
  if (R == A) {                                                                                 \
    if (mixed)                                                                                  \
      hipLaunchKernelGGL((k_batch_arrival_far<A, true>), dim3(blocks), dim3(256), 0, st, scans, \
                         items, n_items, counter);                                              \
    else                                                                                        \
      hipLaunchKernelGGL((k_batch_arrival_far<A, false>), dim3(blocks), dim3(256), 0, st,       \
                         scans, items, n_items, counter);                                       \
    return hipGetLastError();                                                                   \
  }
  DD_LAUNCH(4)
  DD_LAUNCH(2)
#undef DD_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_batch_near(const BatchScan* scans, const BatchItem* items, int32_t n_items,
                             int* counter, int RN, bool mixed, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, counter);
  const unsigned blocks = persistent_blocks(n_items);
#define DD_LAUNCH(B)                                                                             \
  if (RN == B) {                                                                                 \
    if (mixed)                                                                                   \
      hipLaunchKernelGGL((k_batch_arrival_near<B, true>), dim3(blocks), dim3(256), 0, st, scans, \
                         items, n_items, counter);                                               \
    else                                                                                         \
      hipLaunchKernelGGL((k_batch_arrival_near<B, false>), dim3(blocks), dim3(256), 0, st,       \
                         scans, items, n_items, counter);                                        \
    return hipGetLastError();                                                                    \
  }
  DD_LAUNCH(2)
  DD_LAUNCH(4)
#undef DD_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_batch_map(const BatchScan* scans, const BatchItem* items, int32_t n_items,
                            int* counter, int RM, bool mixed, bool near, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, counter);
  const unsigned blocks = persistent_blocks(n_items);
#define DD_LAUNCH_ONE(C, MX, NR)                                                                 \
  hipLaunchKernelGGL((k_batch_map<C, MX, NR>), dim3(blocks), dim3(256), 0, st, scans, items,     \
                     n_items, counter)
#define DD_LAUNCH_BATCH_MAP(C)                                                                   \
  if (RM == C) {                                                                                 \
    if (mixed) {                                                                                 \
      if (near)                                                                                  \
        DD_LAUNCH_ONE(C, true, true);                                                            \
      else                                                                                       \
        DD_LAUNCH_ONE(C, true, false);                                                           \
    } else {                                                                                     \
      if (near)                                                                                  \
        DD_LAUNCH_ONE(C, false, true);                                                           \
      else                                                                                       \
        DD_LAUNCH_ONE(C, false, false);                                                          \
    }                                                                                            \
    return hipGetLastError();                                                                    \
  }
  // every tile shape the autotuner may choose: RM in {1, 2, 4}
  DD_LAUNCH_BATCH_MAP(4)
  DD_LAUNCH_BATCH_MAP(2)
  DD_LAUNCH_BATCH_MAP(1)
#undef DD_LAUNCH_BATCH_MAP
#undef DD_LAUNCH_ONE
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_batch(const BatchReduce* reds, int32_t n_red, int64_t total, OutFlag fl,
                               hipStream_t st) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_batch, dim3(batch_grid_for(total)), dim3(256), 0, st, reds, n_red, total, fl);
  return hipGetLastError();
}

}  // namespace dd
