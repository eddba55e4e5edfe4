// dd_device.h -- device math for the damage-diffusion pair term on gfx950.
//
// The pair term of Eqs. 1-4 (Sec. II) in pitch units is
//   phi_hat = E1(x1) - E1(x0),  x1 = a rb1 < x0 = a rb0,  and ln(b1/b0) at a = 0.
// Three evaluation forms are used, chosen by dx = x0 - x1 = a c:
//   * series  (dx <= threshold): exp(-x1) * sum_m P_m dx^m with per-lag P_m
//     (see dd_internal.h); covers a = 0, the small-argument regime and the
//     near-coincident regime without cancellation;
//   * direct  (dx above threshold): E1(x1) - E1(x0) with E1 from its power
//     series (x <= 2.5) or its continued fraction (x > 2.5); the two values
//     differ by more than a factor e^-dx so the subtraction loses < 2 digits;
//   * FP32 series with a split exponent for the mixed-precision bulk.
#pragma once
#include <hip/hip_runtime.h>

#include "dd_internal.h"

namespace dd {

// Load of read-only data through the constant address space: where the
// address is the same for the whole wave (a lag row, a visit position shared
// by all pixels) it becomes a scalar load, also when the pointer itself was
// read from memory (the batched kernels' per-scan descriptors).  Only for
// device-memory tables that no kernel writes while the caller runs: a pointer
// to a thread's private array or to LDS is not a valid constant address, so
// helpers that may receive such rows (phi_general_f64, series_f64_q,
// series_f32_q, as k_pair_terms calls them) read through plain pointers.
#define DD_CONST_AS __attribute__((address_space(4)))
__device__ __forceinline__ float ldc(const float* p) {
  return *reinterpret_cast<const DD_CONST_AS float*>(reinterpret_cast<uintptr_t>(p));
}
__device__ __forceinline__ double ldc(const double* p) {
  return *reinterpret_cast<const DD_CONST_AS double*>(reinterpret_cast<uintptr_t>(p));
}
__device__ __forceinline__ float2 ldc(const float2* p) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 v = *reinterpret_cast<const DD_CONST_AS v2*>(reinterpret_cast<uintptr_t>(p));
  return make_float2(v[0], v[1]);
}
__device__ __forceinline__ float4 ldc(const float4* p) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  const v4 v = *reinterpret_cast<const DD_CONST_AS v4*>(reinterpret_cast<uintptr_t>(p));
  return make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ double2 ldc(const double2* p) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 v = *reinterpret_cast<const DD_CONST_AS v2*>(reinterpret_cast<uintptr_t>(p));
  return make_double2(v[0], v[1]);
}
#undef DD_CONST_AS

// Per-lane load of the first three fields of a float4 known to be in global
// memory (a plain vector load, not a flat one, also through a pointer read
// from memory); the fourth field is returned as 0.
__device__ __forceinline__ float4 ldg3(const float4* p) {
  typedef float v3 __attribute__((ext_vector_type(3)));
  const v3 v =
      *reinterpret_cast<const __attribute__((address_space(1))) v3*>(reinterpret_cast<uintptr_t>(p));
  return make_float4(v[0], v[1], v[2], 0.0f);
}


constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
constexpr double kEulerGamma = 0.5772156649015329;

// 1/k! for k = 0 .. 23, each the correctly rounded quotient of two exact
// doubles (k! is exact in double up to 18!; beyond, the first rounding).
struct InvFact {
  double v[24];
  constexpr InvFact() : v() {
    double f = 1.0;
    for (int k = 0; k < 24; ++k) {
      if (k > 0) f *= k;
      v[k] = 1.0 / f;
    }
  }
};

// 2^-y for y >= 0 in double precision, y -> 2^-n 2^-f with n = rint(y),
// f in [-1/2, 1/2]; 2^-f = e^{-f ln 2} by its Taylor polynomial of degree
// DEG: relative remainder < 1.3e-14 for DEG = 11 (the FP64 path's per-term
// budget is 1e-13), < 7.4e-9 for DEG = 7 (the mixed path's general form).
// Returns 0 for y > 1100.
template <int DEG = 11>
__device__ __forceinline__ double exp2_neg(double y) {
  constexpr InvFact f{};
  y = fmin(y, 1100.0);
  const double n = __builtin_rint(y);
  const double g = (n - y) * kLn2;  // e^g with |g| <= 0.3466
  double p = f.v[DEG];
#pragma unroll
  for (int k = DEG - 1; k >= 0; --k) p = fma(p, g, f.v[k]);
  return __builtin_ldexp(p, -(int)n);
}

// cos on [0, pi/2] by its Taylor series (compile time).
constexpr double cheb_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 24; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
// 2^h for |h| <= 1/2 by the degree-D polynomial interpolating it at the D + 1
// Chebyshev points of that interval (near-minimax), as monomial coefficients
// in h formed at compile time: Chebyshev coefficients by the discrete cosine
// sum over the nodes (T_k(x_j) by the three-term recurrence), then each T_k
// expanded in powers of x = 2h.  Its error is close to the first omitted
// Chebyshev coefficient, 2 I_{D+1}(ln(2) / 2) ~ (ln(2)/4)^{D+1} / (D+1)! 2:
// 1.3e-14 relative at D = 9, the accuracy the degree-11 Taylor polynomial has.
template <int D>
struct Exp2Cheb {
  double c[D + 1];
  constexpr Exp2Cheb() : c() {
    constexpr int N = D + 1;
    constexpr double pi = 3.141592653589793;
    double x[N] = {}, f[N] = {}, a[N] = {};
    for (int j = 0; j < N; ++j) {
      const double th = pi * (j + 0.5) / N;
      // cos on [0, pi/2] only, by symmetry
      x[j] = th <= pi / 2 ? cheb_cos(th) : -cheb_cos(pi - th);
      // 2^{x/2} = e^{x ln2 / 2} by its Taylor series
      const double g = x[j] * 0.34657359027997264;
      double t = 1.0, s = 1.0;
      for (int k = 1; k < 30; ++k) {
        t *= g / k;
        s += t;
      }
      f[j] = s;
    }
    for (int j = 0; j < N; ++j) {
      double tm = 1.0, tk = x[j];
      a[0] += f[j];
      if (N > 1) a[1] += f[j] * tk;
      for (int k = 2; k < N; ++k) {
        const double tn = 2.0 * x[j] * tk - tm;
        tm = tk;
        tk = tn;
        a[k] += f[j] * tk;
      }
    }
    for (int k = 0; k < N; ++k) a[k] *= (k == 0 ? 1.0 : 2.0) / N;
    // monomial coefficients of T_k in x, accumulated with weights a_k
    double tm[N] = {}, tk[N] = {}, px[N] = {};
    tm[0] = 1.0;          // T_0
    if (N > 1) tk[1] = 1.0;  // T_1
    px[0] += a[0];
    if (N > 1) px[1] += a[1];
    for (int k = 2; k < N; ++k) {
      double tn[N] = {};
      for (int m = 0; m < N; ++m) {
        tn[m] = -tm[m] + (m > 0 ? 2.0 * tk[m - 1] : 0.0);
      }
      for (int m = 0; m < N; ++m) {
        tm[m] = tk[m];
        tk[m] = tn[m];
        px[m] += a[k] * tn[m];
      }
    }
    double sc = 1.0;  // x = 2h
    for (int m = 0; m < N; ++m) {
      c[m] = px[m] * sc;
      sc *= 2.0;
    }
  }
};

// 2^-y for y >= 0 to the FP64 series' per-term budget (1e-13): -y -> m + h,
// m = rint(-y), |h| <= 1/2, 2^h by Exp2Cheb<9> (relative error below 1.9e-14,
// two FMAs fewer than the degree-11 Taylor form of exp2_neg); rounding -y
// rather than y gives the exponent without a negation.  Returns 0 for
// y > 1100.
__device__ __forceinline__ double exp2_neg9(double y) {
  constexpr Exp2Cheb<9> e{};
  const double ny = -fmin(y, 1100.0);
  const double m = __builtin_rint(ny);
  const double h = ny - m;
  double p = e.c[9];
#pragma unroll
  for (int k = 8; k >= 0; --k) p = fma(p, h, e.c[k]);
  return __builtin_ldexp(p, (int)m);
}

// Coefficients (-1)^n / (n n!) of the E1 power series, n = 1..24.
struct E1SeriesCoef {
  double c[24];
  constexpr E1SeriesCoef() : c() {
    double fact = 1.0;
    for (int n = 1; n <= 24; ++n) {
      fact *= n;
      c[n - 1] = ((n & 1) ? -1.0 : 1.0) / (n * fact);
    }
  }
};

// E1(x) for x > 0 in double precision.  Power series about 0 (A&S 5.1.11)
// with NSER terms for x <= 2.5; for x > 2.5 the even continued fraction
//   E1(x) = e^-x / (x+1 - 1/(x+3 - 4/(x+5 - ...)))   (A&S 5.1.22)
// truncated after CFA + CFB/x levels and evaluated by the forward three-term
// recurrence of its convergents (no divisions inside the loop).  The depths
// come from a numerical study against the oracle's E1:
//   e1_f64  (24 terms, 5 + 90/x, exp degree 11): relative error < 3e-15 for
//           x <= 2.5, < 1e-14 above;
//   e1_mixed (18 terms, 4 + 30/x, exp degree 7): < 1e-8, for the mixed path.
template <int NSER, int CFA, int CFB, int EXPDEG>
__device__ __forceinline__ double e1_eval(double x) {
  if (x <= 2.5) {
    constexpr E1SeriesCoef k{};
    double s = k.c[NSER - 1];
#pragma unroll
    for (int n = NSER - 2; n >= 0; --n) s = fma(s, x, k.c[n]);
    return -kEulerGamma - ::log(x) - x * s;
  }
  const int depth = CFA + (int)((double)CFB / x);
  double am1 = 1.0, bm1 = 0.0, a0 = x + 1.0, b0 = 1.0;
  double bj = x + 1.0;
  for (int j = 1; j <= depth; ++j) {
    bj += 2.0;
    const double aj = -(double)j * (double)j;
    const double a1 = fma(bj, a0, aj * am1);
    const double b1 = fma(bj, b0, aj * bm1);
    am1 = a0; bm1 = b0; a0 = a1; b0 = b1;
  }
  return exp2_neg<EXPDEG>(x * kLog2e) * (b0 / a0);
}

__device__ __forceinline__ double e1_f64(double x) { return e1_eval<24, 5, 90, 11>(x); }
__device__ __forceinline__ double e1_mixed(double x) { return e1_eval<18, 4, 30, 7>(x); }

// Series form in double precision with P_0..P_M read from an FP64 row.
// The two factors of the term: returns q and sets t = exp(-x1) (term = t q).
template <int M>
__device__ __forceinline__ double series_f64_q(double a, const double* __restrict__ row,
                                               double& t) {
  const double z = a * row[kR64_C];
  double q = row[kR64_P + M];
#pragma unroll
  for (int m = M - 1; m >= 0; --m) q = fma(q, z, row[kR64_P + m]);
  t = exp2_neg9(a * row[kR64_RL2]);
  return q;
}

template <int M>
__device__ __forceinline__ double series_f64(double a, const double* __restrict__ row) {
  double t;
  const double q = series_f64_q<M>(a, row, t);
  return t * q;
}

// General FP64 pair term: series for dx <= 1, direct difference above.
__device__ __forceinline__ double phi_general_f64(double a, const double* __restrict__ row) {
  const double z = a * row[kR64_C];
  if (z <= kThr64) return series_f64<kM64>(a, row);
  const double x1 = a * row[kR64_RB1];
  if (x1 > 745.0) return 0.0;  // both E1 values below the double range
  const double x0 = a * row[kR64_RB0];
  const double e0 = x0 > 745.0 ? 0.0 : e1_f64(x0);
  return e1_f64(x1) - e0;
}

// General pair term of the mixed path, for the pairs its FP32 series does not
// cover (dx > 0.25), to ~1e-8 relative, a hundredth of the mixed bound:
// dx <= 1: the series of degree 12 (truncation < 2e-9) in FP64 times
// exp(-x1) in the split FP32 form of the bulk (a exact, x1 log2(e) = yh + yl);
// dx > 1: E1(x1) - E1(x0) by e1_mixed (the two values differ by more than a
// factor e, so the difference keeps ~2e-8).
__device__ __forceinline__ double phi_general_mixed(float a, const double* __restrict__ r64,
                                                    const float* __restrict__ r32) {
  const double ad = (double)a;
  const double z = ad * r64[kR64_C];
  if (z <= kThr64) {
    double q = r64[kR64_P + 12];
#pragma unroll
    for (int m = 11; m >= 0; --m) q = fma(q, z, r64[kR64_P + m]);
    const float rhi = r32[kR32_RHI];
    const float yh = a * rhi;
    float yl = __builtin_fmaf(a, rhi, -yh);
    yl = __builtin_fmaf(a, r32[kR32_RLO], yl);
    float t = __builtin_amdgcn_exp2f(-yh);
    t = __builtin_fmaf(t, yl * (float)(-kLn2), t);
    return (double)t * q;
  }
  const double x1 = ad * r64[kR64_RB1];
  if (x1 > 745.0) return 0.0;
  const double x0 = ad * r64[kR64_RB0];
  const double e0 = x0 > 745.0 ? 0.0 : e1_mixed(x0);
  return e1_mixed(x1) - e0;
}

// Mixed-precision series with P_0..P_M from an FP32 row.  `a` is exact
// (lattice distances).  x1 log2(e) = a (rhi + rlo) is formed as yh + yl with
// yh = fl(a rhi) and yl its rounding error plus a rlo, so that
// exp(-x1) = 2^-yh (1 - ln2 yl) keeps its relative error near 1e-7 even when
// x1 is large.  dx = a c stays below the series threshold, where the sum is
// well conditioned.
// The two factors of the term: returns q and sets t = 2^-yh (term = t q).
template <int M>
__device__ __forceinline__ float series_f32_q(float a, const float* __restrict__ row, float& t) {
  const float z = a * row[kR32_C];
  const float rhi = row[kR32_RHI];
  const float yh = a * rhi;
  float yl = __builtin_fmaf(a, rhi, -yh);
  yl = __builtin_fmaf(a, row[kR32_RLO], yl);
  t = __builtin_amdgcn_exp2f(-yh);
  float q;
  if constexpr (M == 0) {
    q = row[kR32_P0];
  } else {
    q = row[kR32_P1 + M - 1];
#pragma unroll
    for (int m = M - 1; m >= 1; --m) q = __builtin_fmaf(q, z, row[kR32_P1 + m - 1]);
    q = __builtin_fmaf(q, z, row[kR32_P0]);
  }
  return __builtin_fmaf(q, yl * (float)(-kLn2), q);
}

template <int M>
__device__ __forceinline__ float series_f32(float a, const float* __restrict__ row) {
  float t;
  const float q = series_f32_q<M>(a, row, t);
  return t * q;
}

// Mixed-precision series for degree M <= 3 in powers of a itself,
//   q = P_0 + PA_1 a + ... + PA_M a^M,   PA_m = P_m c^m,
// with the exponent's rounding correction folded in: with x1 log2(e) =
// yh + e2 + a rlo (yh = fl(a rhi), e2 its exact rounding error),
// exp(-x1) = 2^-yh (1 + eps), eps = -ln2 (e2 + a rlo), and
// t q (1 + eps) ~= t (q + P_0 eps); the neglected t P_0 eps (q/P_0 - 1) is
// below |eps| dx / 2, i.e. under 1e-8 of the term at the dx <= 0.01 where
// degrees <= 3 are used.  P_0 eps enters as -ln2 P_0 rlo added to the linear
// coefficient (row field PA_1 holds PA_1 - ln2 P_0 rlo) and one fma with e2.
// `a` is exact.  COMP = false leaves out the e2 correction, for rows where
// y = x1 log2(e) is small enough that fl(a rhi) alone is accurate enough.
template <int M, bool COMP = true>
__device__ __forceinline__ float series_f32a_q(float a, const RowA& w, float& t) {
  static_assert(M <= kMaxA, "degree too high for the a-form");
  const float yh = a * w.rhi;
  t = __builtin_amdgcn_exp2f(-yh);
  float q;
  if constexpr (M == 0) {
    q = __builtin_fmaf(w.p0nr, a, w.p0);
  } else {
    const float pa[3] = {w.pa1, w.pa2, w.pa3};
    q = pa[M - 1];
#pragma unroll
    for (int m = M - 1; m >= 1; --m) q = __builtin_fmaf(q, a, pa[m - 1]);
    q = __builtin_fmaf(q, a, w.p0);
  }
  if constexpr (!COMP) return q;
  const float e2 = __builtin_fmaf(a, w.rhi, -yh);
  return __builtin_fmaf(w.p0n, e2, q);
}

template <int M, bool COMP = true>
__device__ __forceinline__ float series_f32a(float a, const RowA& w) {
  float t;
  const float q = series_f32a_q<M, COMP>(a, w, t);
  return t * q;
}

// Marks a non-finite output value in the word of `f` (see OutFlag).
__device__ __forceinline__ void flag_nonfinite(const OutFlag& f, double v, int64_t idx) {
  if (__builtin_isfinite(v) || f.word == nullptr) return;
  constexpr unsigned long long lim = (1ull << kFlagIndexBits) - 1;
  unsigned long long i = (unsigned long long)(f.base + idx);
  if (i >= lim) i = lim - 1;
  atomicMax(f.word, (f.seq << kFlagIndexBits) | (lim - i));
}

// The 8 bulk fields of an FP32 row; CAS: through the constant address space
// (scalar loads also where the table pointer was read from memory).
template <bool CAS>
__device__ __forceinline__ RowA load_rowa(const float* __restrict__ row) {
  float4 u, v;
  if constexpr (CAS) {
    u = ldc(reinterpret_cast<const float4*>(row));
    v = ldc(reinterpret_cast<const float4*>(row + 4));
  } else {
    u = *(const float4*)row;
    v = *(const float4*)(row + 4);
  }
  return RowA{u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
}

}  // namespace dd
