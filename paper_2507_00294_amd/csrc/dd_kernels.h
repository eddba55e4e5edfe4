// dd_kernels.h -- host-callable launchers for the libdd HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "dd_internal.h"

namespace dd {

// Front/back padding (in visits) of the device position arrays, so that the
// sliding probe windows of edge tiles stay inside the allocation.
constexpr int kPosPad = 1024;

// Fills `count` lag rows for lags lambda = f + n, n = n0 .. n0+count-1, into
// rows64[k * kRow64] and rows32[k * kRow32], k = n - n0 (rows with
// lambda <= 0 are zero).
hipError_t launch_lag_rows(int64_t n0, int64_t count, double f, double kappa, double s2,
                           const GLNodes& gl, double* rows64, float* rows32, hipStream_t st);

struct ArrivalLaunch {
  const void* pos;          // float2 (mixed) or double2 (FP64), base = visit 0
  const float4* pos4;       // (-2x, -2y, x^2+y^2, 0) by visit, base = visit 0
  const double* rows64;     // integer-lag rows, row n = lag n
  const float* rows32;
  const ArrItem* items;
  int32_t n_items;
  int64_t V;
  DegreeBounds bounds;
  double* partial;          // [slots][pstride], column j - pj0 for visit j
  int64_t pstride, pj0;     // V and 0 for a whole-scan query
  int R;                    // eval visits per lane (tile = 64 R)
  bool mixed;
  bool near;                // items are near-band items (per-pair regime)
  bool range = false;       // a visit-range query (its own kernel instantiations)
};
hipError_t launch_arrival(const ArrivalLaunch& L, hipStream_t st);

struct MapLaunch {
  const void* pos;          // float2 / double2 probe positions by visit
  const float4* pos4;       // (-2x, -2y, x^2+y^2, 0) by visit
  bool lattice;             // pixel/probe coordinates exact small dyadics
  const double* rows64;
  const float* rows32;
  const MapItem* items;
  int32_t n_items;
  const MapTime* times;
  double X0, Y0, DX, DY;    // pixel grid in pitch units
  int32_t W, H;
  double* partial;          // [slots][W*H]
  int R;
  bool mixed;
};
hipError_t launch_map(const MapLaunch& L, hipStream_t st);

// Fixed-order sums of the partial slots times pref; non-finite results are
// marked in the word of `fl` (fl.word may be null).
hipError_t launch_reduce_arrival(const double* partial, const int32_t* tile_slots,
                                 int64_t pstride, int64_t pj0, int tile, double pref, int64_t j0,
                                 int64_t n, double* out, OutFlag fl, hipStream_t st);
// One wave per visit (for visits with many slots).
hipError_t launch_reduce_arrival_wide(const double* partial, const int32_t* tile_slots,
                                      int64_t pstride, int64_t pj0, int tile, double pref,
                                      int64_t j0, int64_t n, double* out, OutFlag fl,
                                      hipStream_t st);
hipError_t launch_reduce_map(const double* partial, const MapTime* times, int32_t n_t,
                             int64_t npix, double pref, double* out, OutFlag fl, hipStream_t st);

// Persistent batched launches (arrival far-region items; arrival near-band
// items; map far-region or near-band items); `counter` is zeroed on the
// stream first.
hipError_t launch_batch(const BatchScan* scans, const BatchItem* items, int32_t n_items,
                        int* counter, int R, bool mixed, hipStream_t st);
hipError_t launch_batch_near(const BatchScan* scans, const BatchItem* items, int32_t n_items,
                             int* counter, int RN, bool mixed, hipStream_t st);
hipError_t launch_batch_map(const BatchScan* scans, const BatchItem* items, int32_t n_items,
                            int* counter, int RM, bool mixed, bool near, hipStream_t st);
// Also marks each non-finite result in its scan's word and in `fl` (index:
// the flat output index of the call).
hipError_t launch_reduce_batch(const BatchReduce* reds, int32_t n_red, int64_t total, OutFlag fl,
                               hipStream_t st);

hipError_t launch_pair_terms(double kappa, double s2, int64_t n, const double* a,
                             const double* lag, bool mixed, const GLNodes& gl, double* out,
                             hipStream_t st);

}  // namespace dd
