// dd_internal.h -- structures shared by the libdd host runtime and its HIP
// kernels.  Not part of the public ABI (include/dd.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dd {

// ---------------------------------------------------------------------------
// Lag rows.  For one scan (kappa = D tau_v / pitch^2, s2 = 2 sigma_hat^2) and
// one lag lambda (time since the visit started, in dwells), the pair term of
// Eqs. 1-4 in pitch units is
//     phi_hat(a) = E1(a rb1) - E1(a rb0)              (a = |r - r_i|^2 / pitch^2)
//               = exp(-a rb1) * sum_m P_m (a c)^m      (entire series in a c)
// with db = 4 kappa min(lambda, 1), b0 = s2 + 4 kappa max(lambda - 1, 0),
// b1 = b0 + db, w = db / b0, c = w / b1 and
//     P_m = (-1)^m w J_m(w) / m!,  J_m(w) = int_0^1 u^m / (1 + w u) du.
// (Substitute u = x1 e^s in the E1 integral: phi_hat = int_0^L exp(-x1 e^s) ds
// with L = ln(b1/b0); expand exp(-x1 (e^s - 1)) in powers of x1.)  P_0 = L is
// exactly the log form of Eqs. 3-4, reached at a = 0.
// Everything lag-dependent is uniform across a wavefront, so it is computed
// once per lag into a row and read through the scalar cache.

constexpr int kM64 = 17;     // FP64 rows hold P_0..P_17
constexpr int kM32 = 6;      // FP32 rows hold P_0..P_6
constexpr int kRow64 = 24;   // doubles per row: rb1 rb0 c rl2 P0..P17 (+2 pad)
constexpr int kRow32 = 16;   // floats per row, see kR32_*
constexpr int kR64_RB1 = 0, kR64_RB0 = 1, kR64_C = 2, kR64_RL2 = 3, kR64_P = 4;
// FP32 row.  The first 8 floats are everything the bulk (degree <= 3) path
// reads, so one 32-byte scalar load fetches them: rb1 log2(e) rounded (rhi),
// P_0, the series coefficients in powers of a itself (PA_m = P_m c^m,
// m = 1..3), -ln2 P_0, -ln2 P_0 rlo and c.  Then rlo = rb1 log2(e) - rhi,
// P_1..P_6 for the degree >= 4 form in powers of dx = a c, and the exponent
// rate RA = log2(e) (rb1 - c P_1/P_0) of the folded form (see DegreeBounds).
constexpr int kR32_RHI = 0, kR32_P0 = 1, kR32_PA = 2, kR32_P0N = 5, kR32_P0NR = 6, kR32_C = 7,
              kR32_RLO = 8, kR32_P1 = 9, kR32_RA = 15;
constexpr int kMaxA = 3;     // highest degree evaluated in powers of a
static_assert(kR32_PA + kMaxA <= kR32_P0N && kR32_P0NR < kR32_C && kR32_P1 + kM32 - 1 < kR32_RA &&
                  kR32_RA < kRow32,
              "FP32 row fields overlap");
// Row fields of the bulk path, loaded together.
struct RowA {
  float rhi, p0, pa1, pa2, pa3, p0n, p0nr, c;
};

// Series regime thresholds on dx = a c (= a/b0 - a/b1).  Below them the
// series above is used; the truncation bound after P_M is
// e^{2 dx} dx^{M+1} / (M+1)!  relative to the term.
constexpr double kThr64 = 1.0;    // FP64: M = 17 covers dx <= 1 to 5e-15
// Truncation target per term of the FP64 far-region series (degree chosen
// per lag segment): 1e-13, three orders below the FP64 path's 1e-10 bound on
// a sum of positive terms.
constexpr double kTrunc64 = 1e-13;
constexpr float kThr32 = 0.25f;   // FP32: M = 6 covers dx <= 0.25 to 2e-8
constexpr int kMNear32 = 6;
// Mixed path: terms with x1 = a/b1 > 100 (below e^-100 each, fewer than
// 2^30 of them) are dropped; they sum to < 4e-35, far below the 1e-30
// floor of the mixed path's relative-error model.  The test is made on
// x1 log2(e), the quantity the FP32 rows hold.
constexpr float kCull32Log2 = 144.26950408889634f;
// The x1 beyond which a pair's term is negligible, per path (FP64: both E1
// values are below the double range).  The planner bounds a pair's dx by
// min(a_max c, cull w) with w = db/b0 (= b1 c): a term with x1 above the
// cull contributes nothing whatever its dx, so it needs no near-band form;
// evaluated by the far-region series it is below L e^{-x1 (1 - w)}, which is
// zero in the path's precision since w <= thr / cull there.
constexpr double kCullX32 = 100.0;
constexpr double kCullX64 = 745.0;

constexpr int kGL = 24;  // Gauss-Legendre nodes on [0, 1] for J_m(w), w <= 1
struct GLNodes {
  double x[kGL];
  double w[kGL];
};

// Work item of the arrival query: wavefront tile `tile` (T = 64 R consecutive
// visits), lags [n_lo, n_hi), partial slot `slot`; `flags` bit 0 = edge (some
// pairs have lag > visit index and are masked), bit 1 = near (per-pair regime).
struct ArrItem {
  int32_t tile, n_lo, n_hi, slot_flags;
};
constexpr int kItemEdge = 1 << 30;
constexpr int kItemNear = 1 << 29;
constexpr int kSlotMask = (1 << 29) - 1;

// Work item of a map query: pixel tile, time index, lag range, slot.
struct MapItem {
  int32_t tile, m, n_lo, n_hi;
  int32_t slot, near, pad0, pad1;
};

// Degree segments of the far region: for rows n in [bound[M], bound[M-1]) the
// series needs P_0..P_M.  bound[-1] is +inf; bound[kMaxSeg] ... bound[0].
//
// Two lighter forms of the mixed arrival series take the rows where every
// pair's exponent y = x1 log2(e) is small, since the rounding of fl(a rhi)
// then costs little: its error is at most half an ulp of y.
//  * From row `plain` on (y <= 8 and degree <= 3), the a-form runs without
//    the correction of that rounding (two operations fewer per pair); the
//    exponent's error is <= 2^-22, i.e. <= 1.7e-7 of the term.
//  * From row `fold` on (y <= 4, dx <= 2e-4, degree <= 1), the term is
//    P_0 2^{-fl(a RA)}: the linear term of the series moves into the exponent,
//    exp(-x1) (1 + k dx) ~ exp(-x1 + k dx) with k = P_1/P_0, since the two
//    differ by at most 0.3 dx^2 <= 1.2e-8 (|k| <= 1/(2 ln 2) and
//    P_2/P_0 <= 1/(6 ln 2) for q = db/b0 <= 1).  Per pair: a, one product, the
//    exponential and one fused multiply-add into the partial sum.  The
//    exponent's error, from fl(RA) and fl(a RA), is <= 1.5 2^-22, i.e.
//    <= 2.5e-7 of the term.
// Both are >= 2^30 (never) where unused: FP64, maps and short scans.
constexpr int kMaxSeg = 18;
struct DegreeBounds {
  int32_t b[kMaxSeg + 1];  // b[M] for M = 0..kMaxSeg; nondecreasing as M falls
  int32_t m_max;           // degree used at the start of the far region
  int32_t plain, fold;     // first rows of the lighter forms; plain <= fold
};

struct MapTime {
  int64_t K;           // floor(t / tau_v): visit v uses lag row K - v
  int64_t row_base;    // first row of this time's lag table
  int64_t slot_base;   // first partial slot of this time
  int32_t n_slots;     // slots of this time
  int32_t n_min;       // smallest valid row (1 when t is on a dwell boundary)
  DegreeBounds bounds; // series degree by row for this time's table
};


// Batched launch: one descriptor per scan and one item list for all scans.
enum { kBatchArrNear = 0, kBatchArrFar = 1, kBatchMapNear = 2, kBatchMapFar = 3 };
struct BatchScan {
  const void* pos;         // float2 (mixed) or double2 (FP64), base = visit 0
  const float4* pos4;      // (-2x, -2y, x^2+y^2, 0) by visit
  const double* rows64;    // integer-lag rows of this scan
  const float* rows32;
  int64_t V;
  int32_t nx, ny;          // probe grid
  // final map on a probe sub-grid: pixel (u, v), u < map_w, v < map_h, at
  // probe (map_x0 + map_step u, map_y0 + map_step v)
  int32_t map_x0, map_y0, map_step, map_w, map_h;
  DegreeBounds arr_bounds;
  MapTime map_time;        // the final map at t = V tau_v (K = V, f = 0)
  double* arr_partial;     // [slots][V]
  double* map_partial;     // [slots][nx*ny]
};
struct BatchItem {
  int32_t scan, kind, tile, n_lo, n_hi, slot_flags, cost_hi, cost_lo;
};
// Check of non-finite outputs.  A reduction that writes a value that is not
// finite raises *word to (seq << kFlagIndexBits) | (2^kFlagIndexBits - 1 -
// (base + index)) by an atomic max, so the word names the latest flagged
// call (seq, 24 bits) and the smallest bad output index of that call.  No
// word is cleared per call: a call owns a fresh seq.  word == nullptr: no
// check.
constexpr int kFlagIndexBits = 40;
constexpr uint64_t kFlagSeqMax = (1ull << 24) - 1;
struct OutFlag {
  unsigned long long* word;
  unsigned long long seq;
  int64_t base;
};

// Reduction work of a batch: one entry per (scan, query).
struct BatchReduce {
  const double* partial;
  const int32_t* tile_slots;  // arrival: slots per tile; map: nullptr
  int32_t n_slots;            // map: slots of the single time
  int32_t tile;               // arrival tile width
  int64_t n;                  // outputs
  int64_t out_off;            // first output in the flat index space
  double* out;
  double pref;
  OutFlag scan_flag;          // the scan's own word (index: its output index)
};

}  // namespace dd
