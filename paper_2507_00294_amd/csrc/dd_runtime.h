// dd_runtime.h -- the scan handle and host helpers shared by the libdd
// runtime sources.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <vector>

#include "../../include/dd.h"
#include "dd_internal.h"

struct dd_scan;

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
void lean_bounds(DegreeBounds& b, double a_max, double kappa, double s2, int64_t kf, int align);

// Kernel timing (dd_profiling / dd_profile_read): events around a launch on
// the stream it runs on, plus the launch's algorithmic work.
struct ProfToken {
  int slot = -1;
};
ProfToken prof_begin(const char* kernel, hipStream_t st);
void prof_end(ProfToken tok, hipStream_t st, double pairs, double flops);
bool prof_on();  // whether kernel timing is being recorded

// Floating-point operations per pair of the evaluation form used, counted as
// the hardware counters count them (FMA = 2, add, multiply and the
// transcendental v_exp_f32 = 1), with the FP64 accumulation.  Mixed
// precision:
//  * degree M <= 3 (powers of a, folded correction): 13 + 2 max(M, 1) --
//    a 3, x1 log2(e) and its rounding error 3, 2^-x 1, the polynomial
//    2 max(M, 1) (degrees 0 and 1 both take one FMA), the correction 2,
//    the running sum 2 (FMA; every 4th lag a product of 1 and an FP64 add
//    of 1 every 4 lags);
//  * degree M >= 4 (powers of dx, exact correction): 17 + 2M.
// FP64: 29 + 2M (distance 5, dx 1, x1 log2(e) 1, the exponent split 2, the
// degree-9 exp polynomial 18, the polynomial 2M, the sum 2).
inline double series_flops(int M, bool mixed) {
  if (!mixed) return 29.0 + 2.0 * M;
  return M <= kMaxA ? 13.0 + 2.0 * (M > 1 ? M : 1) : 17.0 + 2.0 * M;
}
// The lighter mixed forms: the a-form without the rounding correction (two
// fused multiply-adds fewer) and the folded form (a: 5, product, exponential,
// fused multiply-add into the partial sum: 9).
inline double plain_flops(int M) { return series_flops(M, true) - 4.0; }
constexpr double kFoldFlops = 9.0;

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

// Plan of a scan's arrival query (tile shapes, items, slots), kept on the
// handle; V = -1 until planned.  Its items and tile slots live in the
// handle's device buffers `items` and `aux`.
struct ArrivalPlan {
  int R = 0, RN = 0, K = 0;
  bool mixed = false;
  int64_t V = -1;
  int n_near = 0, n_far = 0, S = 0;
  DegreeBounds bounds{};
  double near_pairs = 0, near_flops = 0, far_pairs = 0, far_flops = 0;
};

// Plan of an arrival query over the visits [j0, j1) (the streaming range):
// work items (near items first), partial-sum slots per tile, and the
// partial columns [pj0, pj0 + pstride) of the range's tiles.
struct RangePlan {
  ArrivalPlan P;
  std::vector<ArrItem> items, far;
  std::vector<int32_t> tile_slots;
  int64_t pj0 = 0, pstride = 0;
};

// An event recorded once, after a call's last launch, on the stream the call
// ran on.  Shared by the handles the call used (a batched call records one).
struct StreamEvent {
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;
  StreamEvent() = default;
  StreamEvent(const StreamEvent&) = delete;
  StreamEvent& operator=(const StreamEvent&) = delete;
  ~StreamEvent() {
    if (ev) (void)hipEventDestroy(ev);
  }
};

// Probe sub-grid of a batched final map: output pixel (u, v), u < w, v < h,
// at probe (x0 + step u, y0 + step v); w < 0 selects the whole probe grid.
struct MapSel {
  int32_t x0 = 0, y0 = 0, step = 1, w = -1, h = -1;
};

// Batched solve of many scans (arrival and/or the final map on the probe
// sub-grid `sel` of each scan).
dd_status run_batch(dd_scan* const* scans, int32_t n, uint32_t mask, bool mixed,
                    double* const* outs, int32_t on_device, hipStream_t st, const MapSel& sel);

struct OutFlag;
// Plans the range query (plan_range) and launches it with its items, tile
// slots and partial sums at the given device addresses (launch_range): the
// allocating and the no-allocation entry points share both steps.
void plan_range(const dd_scan* s, bool mixed, int64_t j0, int64_t j1, bool count, RangePlan& rp);
dd_status launch_range(dd_scan* s, bool mixed, const RangePlan& rp, int64_t j0, int64_t j1,
                       const ArrItem* d_items, const int32_t* d_slots, double* d_partial,
                       double* out_dev, const OutFlag& fl, hipStream_t st, bool profile);
// Cross-stream order and non-finite flag of a query call on one scan.
dd_status begin_call(dd_scan* s, hipStream_t st, OutFlag& fl);

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
  // scan, the precision and the tile shape (and, for the map, its probe
  // sub-grid), so a scan solved again skips the host planning.  Two map
  // plans are kept (the whole final map and one sub-grid, as the
  // surrogate's judge uses).
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
    dd::MapSel sel{};
    int64_t K = 0, slots = 0, npix = 0;
    uint64_t used = 0;
    dd::MapTime time{};
    std::vector<dd::MapItem> items;
    double pairs = 0, flops = 0;
  } bmap[2];

  // Plan of the per-scan arrival query (items in `items`, tile slots in `aux`).
  dd::ArrivalPlan arr_plan;

  // Non-finite output check: the handle's device word (dd::OutFlag) and the
  // seq of its last call.
  dd::DevBuf flag;
  uint64_t seq = 0;

  // Order of the handle's device state across streams: the event after the
  // handle's last call that wrote it, and the handle's own reusable event.
  // A call on another stream first makes its stream wait for `last`, so
  // calls on different streams never overwrite each other's partial sums,
  // items or lag rows.
  std::shared_ptr<dd::StreamEvent> last, own;

  void release_device() {
    for (dd::DevBuf* b : {&pos32, &pos64, &pos4, &rows64, &rows32, &partial, &items, &aux, &aux2, &aux3,
                          &tmp_out, &maprows64, &maprows32, &sur, &flag})
      b->release();
    sur_state = 0;
    n_rows = 0;
    arr_plan = dd::ArrivalPlan{};
    seq = 0;
    last.reset();
    own.reset();
    dev = -1;
  }
  // Uploads positions (and clears the flag word) on the current device.
  dd_status prepare(hipStream_t st);
  // Makes `st` wait for the handle's last call when that ran on another stream.
  dd_status wait_last(hipStream_t st);
  // Records the handle's own event on `st` as its last call.
  dd_status record_last(hipStream_t st);
  // A fresh seq for a call (the flag word is cleared, synchronously, when
  // the 24-bit seq wraps) and the call's flag.
  dd_status next_flag(hipStream_t st, dd::OutFlag& fl);
  // Reads the flag word (st is synchronized first): DD_EDEVICE naming the
  // first non-finite output of call `seq`, else DD_OK.
  dd_status check_flag(hipStream_t st, uint64_t call_seq);
};
