// dd_visits.h -- general visit lists: shared types of the host plan and the
// kernels of dd_visits.hip.  Not part of the public ABI.
//
// A general list gives every visit its own position, start time and dwell;
// the field is the sum of Eqs. 1-4 over the visits that started before the
// query time (Eq. 6).  Positions are kept in metres and times in seconds, so
// that the lag t - t_i and the distance r - r_i are formed from the caller's
// own values before any scaling (a product taken first, e.g. D t / sigma^2,
// would turn the rounding of t into an error of the short lags).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dd_internal.h"

namespace dd {

constexpr int kVisTile = 256;     // evaluation points per tile (one per thread)
constexpr int kVisStage = 256;    // visits staged in LDS at a time
constexpr int kVisMaxSlots = 32;  // visit chunks (partial sums) per tile at most

// Map grid (pixel (u, v) at (x0 + u dx, y0 + v dy), w columns).
struct VisGrid {
  double x0, y0, dx, dy;
  int32_t w, pad;
};

// One visit list of a launch: its visits (x, y, t0, dwell) in start order,
// the start order's caller indices (arrival), the output, the map's grid
// and times (maps), and the scaling of a pair: a_hat = |r - r_i|^2 /
// sigma^2 with inv_sigma, b_hat = 2 + 4 (D / sigma^2) lag with th4 =
// 4 D / sigma^2, psi = pref * sum.  Non-finite results are marked in
// fl's word, indexed by their output index plus fl.base.
struct VisList {
  const double4* vis;
  const int64_t* perm;
  double* out;
  const double* times;
  VisGrid grid;
  double inv_sigma, th4, pref;
  OutFlag fl;
};

// A tile of evaluation points of list `list`.  Arrival: the visits p0 ..
// p0+n-1 in start order, each at its own position and start time.  Map: a
// block of tw columns and n / tw rows of the list's grid at its time index
// m, with top-left pixel p0 (row-major index); its point i is pixel p0 +
// (i / tw) w + i % tw.  Its partial sums sit at pbase + slot * 256.
struct VisTile {
  int64_t p0;
  int64_t pbase;
  int64_t out0;  // map: output index of the first point
  double tmax;   // latest point time of the tile
  int32_t n, m, slots, list;
  int32_t tw, pad;  // map: block width
};

// One work item: a tile against visits v0 .. v0+nv-1 (start order).
struct VisItem {
  int32_t tile, slot;
  int64_t v0;
  int64_t nv;
};

// Partial sums of every item: arrival (map = false) or map points, in FP64
// or with the FP32 near form (mixed).
hipError_t launch_visit_pairs(bool map, bool mixed, const VisList* lists, const VisTile* tiles,
                              const VisItem* items, int64_t n_items, double* partial,
                              hipStream_t st);

// For every point of every tile: out[dst] = pref * (sum over the tile's
// slots, in slot order), with the tile's list's out and pref; dst = perm[p0
// + k] for an arrival (the caller's visit order), out0 + k for a map.
hipError_t launch_visit_reduce(bool map, const VisList* lists, const VisTile* tiles,
                               int64_t n_tiles, const double* partial, hipStream_t st);

}  // namespace dd
