// dd_visits.hip -- kernels of the general visit list (per-visit
// position, start time and dwell; Eqs. 1-4 per visit, summed by Eq. 6).
//
// Pair term.  With b_hat = 2 + 4 D lag / sigma^2 (the b of Eqs. 1-2 over
// sigma^2), b0 at the end of the visit's beam-on time seen from t and b1 at
// its start, x1 = a/b1 < x0 = a/b0 and dx = x0 - x1 = a db / (b0 b1):
//   E1(x1) - E1(x0) = integral of e^-u / u over [x1, x0]
// and, at a = 0, ln(b1/b0) (Eqs. 3-4).
//
// Maps (k_visit_map): every pixel of a map shares its time, so each visit
// has one b0 and db for the whole map and its term is a series in dx with
// coefficients of the visit alone (dd_visit_rows.h), built once per visit
// and tile, as the scan's lag rows are once per lag.
//
// Arrival (k_visit_arrival): every pair has its own b0 and db; the bulk of
// a long list takes a short polynomial (see bulk_term), the rest the
// general form, one of four per pair:
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
#include <cstdint>
#include <type_traits>

#include "dd_device.h"
#include "dd_visit_rows.h"
#include "dd_visits.h"

namespace dd {

namespace {

// 1/y for normal y > 0: hardware estimate and STEPS Newton steps (each
// squares the relative error; one suffices for the mixed path's 1e-9 need
// from an estimate good to at least FP32's 2^-23).
template <int STEPS = 2>
__device__ __forceinline__ double rcp64(double y) {
  double r = __builtin_amdgcn_rcp(y);
#pragma unroll
  for (int k = 0; k < STEPS; ++k) r = fma(r, fma(-y, r, 1.0), r);
  return r;
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
    s = fma(g.w[k], e * rcp64<>(x1 + w), s);
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

// ---------------------------------------------------------------------------
// Map query: per-visit series rows.
//
// All pixels of a map share its time, so a visit's b0, db and b1 are the
// same for every pixel and its pair term is the series of dd_visit_rows.h
// with coefficients of the visit alone.  A wave takes one item: a tile of up
// to 256 pixels (4 per lane, pixel lane + 64 k) against the item's visits,
// 64 at a time.  Lane j builds visit j's row in the wave's LDS block, with
// the degree the tile needs; then every lane adds the 64 visits' terms to
// its 4 pixels, reading each row as a broadcast.  Per pair: a in metres^2
// from the positions (the row carries 1/sigma^2), x1 log2(e) and dx as
// products with the row, the series in dx and exp(-x1).
//
// Row degree: the largest dx of a contributing pair of the tile,
// dx_max = min(a_max c, cull q) (a_max over the tile's bounding box; a pair
// beyond the cull, x1 > cull, has dx = x1 q > cull q), gives the degree by
// series_degree at min(dx_max, threshold).  A row with dx_max above the
// series threshold (1 in FP64, 0.25 mixed) is general: a wave with a
// contributing pair above the threshold takes the general form (pair_term)
// for that visit.  Pairs beyond the cull stay in the series with dx clamped
// to the row's bound, where exp(-x1) makes them vanish (below 2^-1074 in
// FP64, e^-100 in FP32).  A visit beyond the cull for the whole box of the
// tile is skipped.

constexpr int kMapWaves = 4;            // waves per block, one item each
constexpr int kMapPix = kVisTile / 64;   // pixels per lane
// Row kinds: the degree M (bits 0-4) of a lean row, with flags; negative:
// no term for the tile.
constexpr int kRowNotStarted = -1;  // the visit starts at or after t
constexpr int kRowCulled = -2;      // x1 > cull for the whole tile
constexpr int kRowCareful = 32;     // clamps, and the per-pair far form
constexpr int kRowP0 = 64;          // mixed: exponent correction through P_0
// A lean row: every pixel of the tile has dx <= threshold and
// x1 log2(e) <= kLeanY (FP64: 2^-y by exp2_lean without a clamp; mixed: y
// converts to a finite FP32 value), so its pairs need no clamp.
template <bool MIXED>
constexpr double kLeanY = MIXED ? 1e30 : 1000.0;

// 1/k (k = 1 .. 63) and (-1)^m / m! (m = 0 .. 23), in constant memory.
struct RowConst {
  double inv[64];
  double sfac[24];
};
__constant__ RowConst kRowConst = [] {
  RowConst c{};
  for (int k = 1; k < 64; ++k) c.inv[k] = 1.0 / k;
  double f = 1.0;
  for (int m = 0; m < 24; ++m) {
    if (m > 0) f *= m;
    c.sfac[m] = ((m & 1) ? -1.0 : 1.0) / f;
  }
  return c;
}();

// A visit's row for one tile, in the wave's LDS block.
template <bool MIXED>
struct MapRow {
  using T = typename std::conditional<MIXED, float, double>::type;
  double vx, vy;  // visit position (m)
  double R;       // log2(e) / (b1 sigma^2): x1 log2(e) = a_m R
  double rb1s;    // 1 / (b1 sigma^2): x1 = a_m rb1s
  T c2;           // db / (b0 b1 sigma^2): dx = a_m c2
  T zmax;         // dx bound of the series, min(dx_max, threshold)
  T p0n;          // -ln2 P_0 (mixed)
  int32_t kind;
  T P[(MIXED ? kM32 : kM64) + 1];
};

// Row of visit v for the tile with bounding box (xlo, xhi, ylo, yhi) at
// time t, written into `row` (LDS) field by field; returns its kind.
template <bool MIXED>
__device__ __forceinline__ int build_map_row(const double4 v, double t, double th4, double is2,
                                             const double4 box, MapRow<MIXED>* row) {
  constexpr int MM = MIXED ? kM32 : kM64;
  constexpr double thr = MIXED ? (double)kThr32 : kThr64;
  constexpr double target = MIXED ? kTrunc32 : kTrunc64;
  constexpr double cull = MIXED ? kCullX32 : kCullX64;
  using T = typename MapRow<MIXED>::T;
  row->vx = v.x;
  row->vy = v.y;
  const double dt = t - v.z;
  if (!(dt > 0.0)) return row->kind = kRowNotStarted;
  const double on = fmin(dt, v.w), off = dt - on;
  const double b0 = fma(th4, off, 2.0), db = th4 * on, b1 = b0 + db;
  const double q = db / b0, rb1s = is2 / b1, c2 = q * rb1s;
  // nearest point of the box: every pixel beyond the cull (a margin of
  // 1e-9 keeps roundings on the safe side)
  const double gx = fmax(0.0, fmax(box.x - v.x, v.x - box.y));
  const double gy = fmax(0.0, fmax(box.z - v.y, v.y - box.w));
  if (fma(gx, gx, gy * gy) * rb1s > cull * (1.0 + 1e-9)) return row->kind = kRowCulled;
  const double fx = fmax(fabs(box.x - v.x), fabs(box.y - v.x));
  const double fy = fmax(fabs(box.z - v.y), fabs(box.w - v.y));
  const double amax = fma(fx, fx, fy * fy);
  const double zmax = fmin(fmin(amax * c2, cull * q), thr);
  const double R = rb1s * kLog2e;
  row->R = R;
  row->rb1s = rb1s;
  row->c2 = (T)c2;
  row->zmax = (T)zmax;
  // P_m = (-1)^m q J_m / m! with J_m by the regime of q (dd_visit_rows.h)
  if (q <= 0.25) {
    // downwards from J_N = 1/(N+1), constants from the table (a loop, not
    // unrolled: 45 FP64 constants held in registers would crowd the pair
    // loop's)
    constexpr int N = MM + 28;
    double j = kRowConst.inv[N + 1];
#pragma unroll 1
    for (int m = N - 1; m >= 0; --m) {
      j = fma(-q, j, kRowConst.inv[m + 1]);
      if (m <= MM) row->P[m] = (T)(kRowConst.sfac[m] * q * j);
    }
  } else if (q <= 1.0) {
    // 24-node Gauss-Legendre rule on [0, 1], one coefficient at a time
    constexpr GLRule<24> g{};
#pragma unroll 1
    for (int m = 0; m <= MM; ++m) {
      double J = 0.0;
#pragma unroll 4
      for (int k = 0; k < 24; ++k) {
        const double u = g.x[k];
        double um = 1.0;
        for (int i = 0; i < m; ++i) um *= u;
        J = fma(g.w[k] / fma(q, u, 1.0), um, J);
      }
      row->P[m] = (T)(kRowConst.sfac[m] * q * J);
    }
  } else {
    // upwards from J_0 = ln(1 + q)/q
    const double rq = 1.0 / q;
    double j = log1p(q) * rq;
#pragma unroll 1
    for (int m = 0; m <= MM; ++m) {
      row->P[m] = (T)(kRowConst.sfac[m] * q * j);
      j = (kRowConst.inv[m + 1] - j) * rq;
    }
  }
  int kind;
  if (!(amax * c2 <= thr && amax * R <= kLeanY<MIXED>)) {
    kind = kRowCareful | MM;
  } else {
    kind = series_degree<MM>(zmax, target);
    // mixed: the P_0 form of the exponent correction (as in the scan's
    // bulk) where dx <= 0.01: its neglected part is below |eps| dx / 2 < 1e-8
    if (MIXED && kind <= 3 && zmax <= 0.01) kind |= kRowP0;
  }
  row->p0n = (T)(-kLn2 * (double)row->P[0]);
  return row->kind = kind;
}

// 2^-y for 0 <= y <= 1000 in double precision: -y = m + h, m = rint(-y), 2^h
// by the degree-9 Chebyshev interpolant of exp2_neg9 (relative error below
// 1.9e-14), without exp2_neg9's clamp.
__device__ __forceinline__ double exp2_lean(double y) {
  constexpr Exp2Cheb<9> e{};
  const double m = __builtin_rint(-y);
  const double h = -y - m;
  double p = e.c[9];
#pragma unroll
  for (int k = 8; k >= 0; --k) p = fma(p, h, e.c[k]);
  return __builtin_ldexp(p, (int)m);
}

__device__ __forceinline__ void map_am(const double (&px)[kMapPix], const double (&py)[kMapPix],
                                       double vx, double vy, double (&am)[kMapPix]) {
#pragma unroll
  for (int k = 0; k < kMapPix; ++k) {
    const double ex = px[k] - vx, ey = py[k] - vy;
    am[k] = fma(ex, ex, ey * ey);
  }
}

// The lean rows of a stage (bit j of `mask`: row j), all at degree M (the
// stage's highest; a higher degree is as accurate), the terms added to acc
// (mixed: each term in FP32, converted).
template <int M, bool MIXED, bool P0C>
__device__ __forceinline__ void map_lean_rows(const MapRow<MIXED>* __restrict__ rows,
                                              uint64_t mask, const double (&px)[kMapPix],
                                              const double (&py)[kMapPix],
                                              double (&acc)[kMapPix]) {
  using T = typename MapRow<MIXED>::T;
  while (mask) {
    const int j = __builtin_ctzll(mask);
    mask &= mask - 1;
    const MapRow<MIXED>* r = rows + j;
    double am[kMapPix];
    map_am(px, py, r->vx, r->vy, am);
    const double R = r->R;
    const T c2 = r->c2;
    T P[M + 1];
#pragma unroll
    for (int m = 0; m <= M; ++m) P[m] = r->P[m];
#pragma unroll
    for (int k = 0; k < kMapPix; ++k) {
      if constexpr (MIXED) {
        const double y = am[k] * R;
        const float yh = (float)y;
        const float yl = (float)(y - (double)yh);
        const float z = (float)am[k] * c2;
        float s = P[M];
#pragma unroll
        for (int m = M - 1; m >= 0; --m) s = __builtin_fmaf(s, z, P[m]);
        if constexpr (P0C)
          s = __builtin_fmaf(r->p0n, yl, s);
        else
          s = __builtin_fmaf(s, yl * (float)(-kLn2), s);
        acc[k] += (double)(__builtin_amdgcn_exp2f(-yh) * s);
      } else {
        const double z = am[k] * c2;
        double s = P[M];
#pragma unroll
        for (int m = M - 1; m >= 0; --m) s = fma(s, z, P[m]);
        acc[k] = fma(exp2_lean(am[k] * R), s, acc[k]);
      }
    }
  }
}

// The careful rows of a stage (bits of `mask`): the clamped series of degree MM at every pixel,
// and, in each pixel slot where some lane has a contributing pair with dx
// above the series threshold, the direct difference E1(x1) - E1(x0) for
// those lanes: the two E1 values differ by more than a factor e^thr there,
// so the difference keeps its digits (the general form of the scan's lag
// rows, phi_general_*).
template <bool MIXED>
__device__ __forceinline__ void map_careful_rows(const MapRow<MIXED>* __restrict__ rows,
                                                 uint64_t mask, const double (&px)[kMapPix],
                                                 const double (&py)[kMapPix],
                                                 const bool (&live)[kMapPix],
                                                 double (&acc)[kMapPix]) {
  constexpr int MM = MIXED ? kM32 : kM64;
  constexpr double thr = MIXED ? (double)kThr32 : kThr64;
  constexpr double cull = MIXED ? kCullX32 : kCullX64;
  while (mask) {
    const int j = __builtin_ctzll(mask);
    mask &= mask - 1;
    const MapRow<MIXED>* r = rows + j;
    double am[kMapPix];
    map_am(px, py, r->vx, r->vy, am);
    // pixel slot by slot, not unrolled (rare rows, long code)
#pragma unroll 1
    for (int k = 0; k < kMapPix; ++k) {
      double a = am[0];
      bool l = live[0];
#pragma unroll
      for (int i = 1; i < kMapPix; ++i)
        if (k == i) {
          a = am[i];
          l = live[i];
        }
      const double x1 = a * r->rb1s, dx = a * (double)r->c2;
      const bool far = l && dx > thr && x1 <= cull;
      double term;
      if constexpr (MIXED) {
        const double y = fmin(a * r->R, 4096.0);
        const float yh = (float)y;
        const float yl = (float)(y - (double)yh);
        const float z = fminf((float)a * r->c2, r->zmax);
        float s = r->P[MM];
#pragma unroll
        for (int m = MM - 1; m >= 0; --m) s = __builtin_fmaf(s, z, r->P[m]);
        s = __builtin_fmaf(s, yl * (float)(-kLn2), s);
        term = (double)(__builtin_amdgcn_exp2f(-yh) * s);
      } else {
        const double z = fmin(dx, r->zmax);
        double s = r->P[MM];
#pragma unroll
        for (int m = MM - 1; m >= 0; --m) s = fma(s, z, r->P[m]);
        term = exp2_neg<11>(a * r->R) * s;
      }
      if (__ballot(far) && far) {
        const double x0 = x1 + dx;
        if constexpr (MIXED)
          term = e1_mixed(x1) - (x0 > 745.0 ? 0.0 : e1_mixed(x0));
        else
          term = e1_f64(x1) - (x0 > 745.0 ? 0.0 : e1_f64(x0));
      }
#pragma unroll
      for (int i = 0; i < kMapPix; ++i)
        if (k == i) acc[i] += term;
    }
  }
}

#define DD_LEAN(MV, P0) \
  case MV:              \
    map_lean_rows<(MV), MIXED, P0>(rows, lean, px, py, acc); \
    break;

// One stage of rows: the lean rows (bits of `lean`) at degree M with the
// P_0 correction form if every one allows it (p0), then the careful rows.
template <bool MIXED>
__device__ __forceinline__ void map_stage(const MapRow<MIXED>* __restrict__ rows, uint64_t lean,
                                          int M, bool p0, uint64_t careful,
                                          const double (&px)[kMapPix],
                                          const double (&py)[kMapPix],
                                          const bool (&live)[kMapPix], double (&acc)[kMapPix]) {
  if (lean) {
    if constexpr (MIXED) {
      if (p0) {
        switch (M) {
          DD_LEAN(0, true) DD_LEAN(1, true) DD_LEAN(2, true)
          default: map_lean_rows<3, MIXED, true>(rows, lean, px, py, acc);
        }
      } else {
        switch (M) {
          DD_LEAN(0, false) DD_LEAN(1, false) DD_LEAN(2, false)
          DD_LEAN(3, false) DD_LEAN(4, false) DD_LEAN(5, false)
          default: map_lean_rows<6, MIXED, false>(rows, lean, px, py, acc);
        }
      }
    } else {
      // degrees rounded up to 1, 2, 3, 4, 6, 8, 11, 14, 17 (fewer variants
      // keep the code small)
      if (M <= 4) {
        switch (M) {
          DD_LEAN(0, false) DD_LEAN(1, false) DD_LEAN(2, false) DD_LEAN(3, false)
          default: map_lean_rows<4, MIXED, false>(rows, lean, px, py, acc);
        }
      } else if (M <= 6) {
        map_lean_rows<6, MIXED, false>(rows, lean, px, py, acc);
      } else if (M <= 8) {
        map_lean_rows<8, MIXED, false>(rows, lean, px, py, acc);
      } else if (M <= 11) {
        map_lean_rows<11, MIXED, false>(rows, lean, px, py, acc);
      } else if (M <= 14) {
        map_lean_rows<14, MIXED, false>(rows, lean, px, py, acc);
      } else {
        map_lean_rows<17, MIXED, false>(rows, lean, px, py, acc);
      }
    }
  }
  if (careful) map_careful_rows<MIXED>(rows, careful, px, py, live, acc);
}
#undef DD_LEAN

// Orders a wave's LDS writes before its later reads by other lanes (and
// the reads before later overwrites): the wave's LDS operations complete in
// order, so a compiler barrier at wavefront scope suffices.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave w of block b takes items 4 b + w, 4 b + w + 4 gridDim.x, ...  The
// item's visits go 64 at a time: lane j builds visit j's row in the wave's
// LDS block; then the stage's lean rows are taken by one loop at their
// highest degree and its careful rows by another.  Mixed: held to 168 VGPRs
// (3 waves per SIMD instead of 2; the few spilled values are outside the
// lean loop).
template <bool MIXED>
__global__ __launch_bounds__(64 * kMapWaves)
__attribute__((amdgpu_waves_per_eu(MIXED ? 3 : 1, 8))) void k_visit_map(
    const VisList* __restrict__ lists, const VisTile* __restrict__ tiles,
    const VisItem* __restrict__ items, int64_t n_items, double* __restrict__ partial) {
  __shared__ MapRow<MIXED> s_rows[kMapWaves][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  MapRow<MIXED>* rows = s_rows[w];
  for (int64_t it = (int64_t)blockIdx.x * kMapWaves + w; it < n_items;
       it += (int64_t)gridDim.x * kMapWaves) {
    const VisItem item = items[it];
    const VisTile tile = tiles[item.tile];
    const VisList& L = lists[tile.list];
    const VisGrid grid = L.grid;
    const double t = L.times[tile.m];
    const double is2 = L.inv_sigma * L.inv_sigma, th4 = L.th4;
    // the tile: a block of tw columns from pixel (u0, v0)
    const int tw = tile.tw;
    const int64_t u0 = tile.p0 % grid.w, v0 = tile.p0 / grid.w;
    double px[kMapPix], py[kMapPix];
    bool live[kMapPix];
#pragma unroll
    for (int k = 0; k < kMapPix; ++k) {
      const int idx = lane + 64 * k;
      live[k] = idx < tile.n;
      const int i = live[k] ? idx : 0;
      px[k] = grid.x0 + (double)(u0 + i % tw) * grid.dx;
      py[k] = grid.y0 + (double)(v0 + i / tw) * grid.dy;
    }
    // bounding box of the tile's pixels (the same products as the pixels')
    const int64_t u1 = u0 + tw - 1, v1 = v0 + (tile.n - 1) / tw;
    const double xa = grid.x0 + (double)u0 * grid.dx, xb = grid.x0 + (double)u1 * grid.dx;
    const double ya = grid.y0 + (double)v0 * grid.dy, yb = grid.y0 + (double)v1 * grid.dy;
    const double4 box = make_double4(fmin(xa, xb), fmax(xa, xb), fmin(ya, yb), fmax(ya, yb));
    double acc[kMapPix];
#pragma unroll
    for (int k = 0; k < kMapPix; ++k) acc[k] = 0.0;
    bool done = false;
    for (int64_t v0 = item.v0; v0 < item.v0 + item.nv && !done; v0 += 64) {
      const int64_t left = item.v0 + item.nv - v0;
      const int nk = left < 64 ? (int)left : 64;
      wave_lds_sync();  // the previous stage's rows are no longer read
      int mykind = kRowNotStarted;
      if (lane < nk) mykind = build_map_row<MIXED>(L.vis[v0 + lane], t, th4, is2, box, rows + lane);
      // visits are in start order: the started ones are a prefix
      const int ns = __popcll(__ballot(mykind != kRowNotStarted));
      if (ns < nk) done = true;
      wave_lds_sync();
      // the stage's lean and careful rows; the lean degree is the highest
      const bool is_lean = mykind >= 0 && !(mykind & kRowCareful);
      const uint64_t lean = __ballot(is_lean);
      const uint64_t careful = __ballot(mykind >= 0 && (mykind & kRowCareful));
      int M = 0;
      if (lean) {
        constexpr int MM = MIXED ? kM32 : kM64;
        const int mine = is_lean ? (mykind & 31) : 0;
        for (int m = MM; m > 0; --m)
          if (__ballot(mine >= m)) {
            M = m;
            break;
          }
      }
      const bool p0 = MIXED && !__ballot(is_lean && !(mykind & kRowP0));
      map_stage<MIXED>(rows, lean, M, p0, careful, px, py, live, acc);
    }
    const int64_t pb = tile.pbase + (int64_t)item.slot * kVisTile;
#pragma unroll
    for (int k = 0; k < kMapPix; ++k)
      if (live[k]) partial[pb + lane + 64 * k] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// Arrival query: the bulk form.
//
// With u = db/b1 and v = x1 u (so q = u/(1-u), dx = x1 q = v/(1-u)), the
// term is e^{-x1} u F(u, v) with
//   F = int_0^1 exp(-v s/(1-u)) / (1 - u(1-s)) ds = sum_{m,n} C_{m,n} v^m u^n,
//   C_{m,n} = (-1)^m sum_{k=0..n} binom(m+n-k-1, n-k) k! / (m+k+1)!
// ((1 - u(1-s))^-1 and (1-u)^-m expanded in u, the exponential in v, and
// int_0^1 s^m (1-s)^k ds = m! k! / (m+k+1)!).  It needs one reciprocal per
// pair (1/b1), and for small u and v a short polynomial: on u <= 2^-8,
// v <= 2^-5 (FP64) the degrees in u for m = 0..6 are 5,5,5,4,3,2,1 with a
// truncation below 1e-14 of the term; on u <= 2^-6, v <= 2^-5 (mixed, in
// FP32) the degrees for m = 0..3 are 4,3,3,1, below 2e-8.  A wave whose
// contributing pairs of a visit are all in that domain takes this form (98%
// of the visit steps of a long raster list); otherwise the general form
// (pair_term).
constexpr double binom_d(int a, int b) {
  if (b == 0) return 1.0;
  if (a < b || a < 0) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
  return r;
}
struct BulkCoef {
  double c[8][8];  // C_{m,n}
  constexpr BulkCoef() : c() {
    for (int m = 0; m < 8; ++m)
      for (int n = 0; n < 8; ++n) {
        double sum = 0.0;
        for (int k = 0; k <= n; ++k) {
          double f = 1.0;  // k! / (m+k+1)!
          for (int i = k + 1; i <= m + k + 1; ++i) f /= i;
          sum += binom_d(m + n - k - 1, n - k) * f;
        }
        c[m][n] = (m & 1) ? -sum : sum;
      }
  }
};
constexpr double kBulkU64 = 1.0 / 256, kBulkV64 = 1.0 / 32;
constexpr float kBulkU32 = 1.0f / 64, kBulkV32 = 1.0f / 32;

// F(u, v) by Horner in u per power of v, then in v.
template <typename T, int NM, int D0, int D1, int D2, int D3, int D4 = -1, int D5 = -1,
          int D6 = -1>
__device__ __forceinline__ T bulk_f(T u, T v) {
  constexpr BulkCoef C{};
  constexpr int deg[7] = {D0, D1, D2, D3, D4, D5, D6};
  T acc = 0;
#pragma unroll
  for (int m = NM - 1; m >= 0; --m) {
    T cm = (T)C.c[m][deg[m]];
#pragma unroll
    for (int n = deg[m] - 1; n >= 0; --n) cm = cm * u + (T)C.c[m][n];
    acc = (m == NM - 1) ? cm : acc * v + cm;
  }
  return acc;
}

// The FP64 bulk's 43 constants (F's coefficients, rows of kBulkStride, and
// the degree-9 exp2 interpolant) do not fit the scalar registers beside the
// kernel's own; the arrival kernel keeps them in LDS (kBulkLds doubles) and
// reads them as wave-uniform loads.  Same values, same operations.
constexpr int kBulkStride = 6, kBulkE = 7 * kBulkStride, kBulkLds = kBulkE + 10;
__device__ __forceinline__ double bulk_const64(int k) {
  constexpr BulkCoef C{};
  constexpr Exp2Cheb<9> E{};
  if (k >= kBulkE) return E.c[k - kBulkE];
  return C.c[k / kBulkStride][k % kBulkStride];
}
__device__ __forceinline__ double bulk_term64_lds(double x1, double u, double v,
                                                  const double* __restrict__ bc) {
  constexpr int deg[7] = {5, 5, 5, 4, 3, 2, 1};
  double g = 0;
#pragma unroll
  for (int m = 6; m >= 0; --m) {
    double cm = bc[m * kBulkStride + deg[m]];
#pragma unroll
    for (int n = deg[m] - 1; n >= 0; --n) cm = cm * u + bc[m * kBulkStride + n];
    g = (m == 6) ? cm : g * v + cm;
  }
  // exp2_lean with the interpolant's coefficients from bc
  const double y = x1 * kLog2e;
  const double mm = __builtin_rint(-y);
  const double h = -y - mm;
  double p = bc[kBulkE + 9];
#pragma unroll
  for (int k = 8; k >= 0; --k) p = fma(p, h, bc[kBulkE + k]);
  return __builtin_ldexp(p, (int)mm) * (u * g);
}

// The bulk term e^{-x1} u F(u, v) (x1 <= cull).
template <bool MIXED>
__device__ __forceinline__ double bulk_term(double x1, double u, double v) {
  if constexpr (MIXED) {
    const double y = x1 * kLog2e;
    const float yh = (float)y;
    const float yl = (float)(y - (double)yh);
    const float uf = (float)u, vf = (float)v;
    float g = bulk_f<float, 4, 4, 3, 3, 1>(uf, vf);
    g = __builtin_fmaf(g, yl * (float)(-kLn2), g);
    return (double)(__builtin_amdgcn_exp2f(-yh) * (uf * g));
  } else {
    const double g = bulk_f<double, 7, 5, 5, 5, 4, 3, 2, 1>(u, v);
    return exp2_lean(x1 * kLog2e) * (u * g);
  }
}

// One arrival pair (point at (px, py) at time pt, visit v): the quantities
// of both forms and whether the pair contributes (act) and lies in the bulk
// domain.
template <bool MIXED>
struct ArrPair {
  double x1, u, w, b0, db;
  bool act, bulk;
  __device__ __forceinline__ void setup(const double4 v, double px, double py, double pt,
                                        bool live, double is2, double th4) {
    constexpr double cull = MIXED ? kCullX32 : kCullX64;
    const double lag = pt - v.z;
    const bool started = live && lag > 0.0;
    const double lg = started ? lag : v.w;  // a valid lag for idle lanes
    const double on = fmin(lg, v.w), off = lg - on;
    b0 = fma(th4, off, 2.0);
    db = th4 * on;
    const double r1 = rcp64<MIXED ? 1 : 2>(b0 + db);
    const double ex = px - v.x, ey = py - v.y;
    x1 = fma(ex, ex, ey * ey) * (is2 * r1);
    u = db * r1;
    w = x1 * u;
    act = started && x1 <= cull;
    bulk = MIXED ? ((float)u <= kBulkU32 && (float)w <= kBulkV32)
                 : (u <= kBulkU64 && w <= kBulkV64);
  }
  // Lanes outside the domain (idle, culled) may compute a non-finite value;
  // the select drops it.
  __device__ __forceinline__ double bulk_value(const double* __restrict__ bc) const {
    double t;
    if constexpr (MIXED)
      t = bulk_term<MIXED>(x1, u, w);
    else
      t = bulk_term64_lds(x1, u, w, bc);
    return act ? t : 0.0;
  }
};

// The term of one pair: the bulk form if the wave's contributing pairs of
// this visit are all in its domain, else the general form.
template <bool MIXED>
__device__ __forceinline__ double arr_pair_term(const double4 v, double px, double py, double pt,
                                                bool live, double is2, double th4,
                                                const double* __restrict__ bc) {
  ArrPair<MIXED> pr;
  pr.setup(v, px, py, pt, live, is2, th4);
  if (!__ballot(pr.act && !pr.bulk)) return pr.bulk_value(bc);
  const double q = pr.db / pr.b0;
  return pair_term<MIXED>(pr.act, pr.x1, pr.x1 * q, q);
}

// One block per item: 256 points (one per thread) against the item's visits,
// staged 256 at a time in LDS.  Visits are in start order, so the first one
// that starts at or after the tile's latest time ends the item for the
// whole block.
// FP64: held to 168 VGPRs (3 waves per SIMD; the constants in LDS took it to
// 182 and 2 waves unhinted).
template <bool MIXED>
__global__ __launch_bounds__(kVisTile)
__attribute__((amdgpu_waves_per_eu(MIXED ? 1 : 3, 8))) void k_visit_arrival(
    const VisList* __restrict__ lists, const VisTile* __restrict__ tiles,
    const VisItem* __restrict__ items, int64_t n_items, double* __restrict__ partial) {
  constexpr double cull = MIXED ? kCullX32 : kCullX64;
  __shared__ double4 s_v[kVisStage];
  __shared__ double s_bc[MIXED ? 1 : kBulkLds];
  const int lane = threadIdx.x;
  if (!MIXED && lane < kBulkLds) s_bc[lane] = bulk_const64(lane);  // read after the stage barrier
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const VisItem item = items[it];
    const VisTile tile = tiles[item.tile];
    const VisList& L = lists[tile.list];
    const double4* __restrict__ vis = L.vis;
    const double is2 = L.inv_sigma * L.inv_sigma, th4 = L.th4;
    const bool live = lane < tile.n;
    double px = 0.0, py = 0.0, pt = tile.tmax;
    if (live) {
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
      if (lane < nk) s_v[lane] = vis[v0 + lane];
      __syncthreads();
      int j = 0;
      // four visits at a time (four independent chains per lane) while all
      // four start before the tile's latest time and the wave's pairs are
      // all in the bulk domain
      for (; j + 4 <= nk && s_v[j + 3].z < tile.tmax; j += 4) {
        ArrPair<MIXED> pr[4];
        bool out = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          pr[i].setup(s_v[j + i], px, py, pt, live, is2, th4);
          out |= pr[i].act && !pr[i].bulk;
        }
        if (!__ballot(out)) {
#pragma unroll
          for (int i = 0; i < 4; ++i) sum += pr[i].bulk_value(s_bc);
        } else {
#pragma unroll 1
          for (int i = 0; i < 4; ++i)
            sum += arr_pair_term<MIXED>(s_v[j + i], px, py, pt, live, is2, th4, s_bc);
        }
      }
      for (; j < nk; ++j) {
        const double4 v = s_v[j];
        if (v.z >= tile.tmax) {
          done = true;  // uniform: no later visit starts before any point
          break;
        }
        sum += arr_pair_term<MIXED>(v, px, py, pt, live, is2, th4, s_bc);
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
  const int64_t dst = MAP ? tile.out0 + (int64_t)(lane / tile.tw) * L.grid.w + lane % tile.tw
                          : L.perm[tile.p0 + lane];
  const double v = L.pref * s;
  L.out[dst] = v;
  flag_nonfinite(L.fl, v, dst);
}

}  // namespace

hipError_t launch_visit_pairs(bool map, bool mixed, const VisList* lists, const VisTile* tiles,
                              const VisItem* items, int64_t n_items, double* partial,
                              hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (map) {
    const unsigned mb =
        (unsigned)std::min<int64_t>((n_items + kMapWaves - 1) / kMapWaves, 1 << 20);
    if (mixed)
      k_visit_map<true><<<mb, 64 * kMapWaves, 0, st>>>(lists, tiles, items, n_items, partial);
    else
      k_visit_map<false><<<mb, 64 * kMapWaves, 0, st>>>(lists, tiles, items, n_items, partial);
    return hipGetLastError();
  }
  const unsigned blocks = (unsigned)std::min<int64_t>(n_items, 1 << 20);
  if (mixed)
    k_visit_arrival<true><<<blocks, kVisTile, 0, st>>>(lists, tiles, items, n_items, partial);
  else
    k_visit_arrival<false><<<blocks, kVisTile, 0, st>>>(lists, tiles, items, n_items, partial);
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
