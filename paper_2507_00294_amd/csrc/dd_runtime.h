// dd_runtime.h -- the scan handle and host helpers shared by the libdd
// runtime sources.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/dd.h"
#include "dd_internal.h"

namespace dd {

dd_status fail(dd_status st, const char* fmt, ...);
dd_status hip_fail(hipError_t e, const char* what);
bool host_alloc_ok(size_t bytes);
hipError_t dev_alloc(void** p, size_t bytes);
dd_status ensure_device();
const GLNodes& gl_nodes();
void gauss_legendre01(int n, double* x, double* w);
double row_c(double lam, double kappa, double s2);
int degree_needed(double dx, bool mixed);
double row_dx_bound(double lam, double a_max, double cull, double kappa, double s2);
int64_t first_row_below(double thr, double a_max, double cull, double f, double kappa, double s2,
                        int64_t n_start, int64_t n_end);
DegreeBounds degree_bounds(double a_max, double f, double kappa, double s2, int64_t kf, int align,
                           bool mixed);

// Kernel timing (dd_profiling / dd_profile_read): events around a launch on
// the stream it runs on, plus the launch's algorithmic work.
struct ProfToken {
  int slot = -1;
};
ProfToken prof_begin(const char* kernel, hipStream_t st);
void prof_end(ProfToken tok, hipStream_t st, double pairs, double flops);
bool prof_on();  // whether kernel timing is being recorded

// Floating-point operations per pair of the evaluation form used (FMA = 2):
// mixed degree <= 3 (powers of a, folded correction) 15 + 2M, mixed degree
// >= 4 (powers of dx, exact correction) 17 + 2M, FP64 40 + 2M (13-term
// exp polynomial).
inline double series_flops(int M, bool mixed) {
  if (!mixed) return 36.0 + 2.0 * M;  // exp: degree-11 polynomial (22 flops)
  return (M <= kMaxA ? 15.0 : 17.0) + 2.0 * M;
}

// A grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int dev = -1;
  hipError_t ensure(size_t need) {
    if (need <= bytes && p) return hipSuccess;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    hipError_t e = dev_alloc(&p, need);
    if (e == hipSuccess) bytes = need ? need : 16;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

// Tile-shape choices (autotuned; defaults otherwise).
struct TuneParams {
  int arr_R_mixed = 4, arr_R_f64 = 2;      // far-region tile: 64 R visits
  int arr_RN_mixed = 2, arr_RN_f64 = 2;    // near-band tile
  int arr_K_mixed = 2048, arr_K_f64 = 1024;   // lags per far work item
  int map_R_mixed = 4, map_R_f64 = 1;
  int map_K = 4096;
};
TuneParams& tune();

// Batched solve of many scans (arrival and/or final map, the final map
// restricted to rows [row0, row0 + rows) of each grid; rows < 0 = all).
dd_status run_batch(dd_scan* const* scans, int32_t n, uint32_t mask, bool mixed,
                    double* const* outs, int32_t on_device, hipStream_t st, int32_t row0,
                    int32_t rows);

}  // namespace dd

struct dd_scan {
  dd_scan_desc desc{};
  std::vector<int32_t> ids;
  int64_t V = 0;
  double tau_v = 0, kappa = 0, s2 = 0, pref = 0;

  // Device state (created on first query, on the then-current device).
  int dev = -1;
  dd::DevBuf pos32, pos64, pos4;    // padded probe positions by visit
  dd::DevBuf rows64, rows32;        // integer-lag rows n = 0 .. n_rows-1
  int64_t n_rows = 0;
  dd::DevBuf partial, items, aux, aux2, aux3, tmp_out, maprows64, maprows32;
  // Surrogate input table (per probe: the network inputs, then the own-visit
  // term), built on first use; sur_state 0 = not built, 1 = built, -1 = the
  // scan is outside what the surrogate accepts.
  dd::DevBuf sur;
  int sur_state = 0;
  // Plans of the batched solve, kept on the handle: they depend only on the
  // scan, the precision and the tile shape (and, for the map, its rows), so
  // a scan solved again skips the host planning.  Two map plans are kept
  // (the whole final map and one row subset, as the surrogate's judge uses).
  struct BatchArrPlan {
    bool ok = false, mixed = false, counted = false;
    int R = 0, RN = 0, K = 0, S = 0;
    dd::DegreeBounds bounds{};
    std::vector<dd::ArrItem> near, far;
    std::vector<int32_t> tile_slots;
    double pairs = 0, flops = 0;
  } barr;
  struct BatchMapPlan {
    bool ok = false, mixed = false, counted = false;
    int R = 0;
    int32_t row0 = 0, rows = 0;
    int64_t K = 0, slots = 0, npix = 0;
    uint64_t used = 0;
    dd::MapTime time{};
    std::vector<dd::MapItem> items;
    double pairs = 0, flops = 0;
  } bmap[2];

  void release_device() {
    for (dd::DevBuf* b : {&pos32, &pos64, &pos4, &rows64, &rows32, &partial, &items, &aux, &aux2, &aux3,
                          &tmp_out, &maprows64, &maprows32, &sur})
      b->release();
    sur_state = 0;
    n_rows = 0;
    dev = -1;
  }
  // Uploads positions and integer-lag rows (rows 0 .. V + margin).
  dd_status prepare(hipStream_t st);
};
