// dd_log.h -- a lean double-precision natural logarithm for the renderer.
//
// For positive normal x: x = m 2^e with m in [sqrt(1/2), sqrt(2)), and
//   ln m = 2 artanh(s) = 2 (s + s^3/3 + s^5/5 + ...),  s = (m - 1) / (m + 1),
// with |s| <= 0.1716, so s^2 <= 0.0295 and eleven terms leave a truncation
// below 1e-19 of the value.  ln x = e ln 2 + ln m.  The same code runs on
// the host, where a test checks it against the C library: a few units in the
// last place of ln x, far inside the 1e-12 decision slack of the colour
// scale.  Positive finite x only.
#pragma once

namespace dd {

struct ArtanhSeries {
  double c[11];  // 2 / (2k + 1)
  constexpr ArtanhSeries() : c() {
    for (int k = 0; k < 11; ++k) c[k] = 2.0 / (2 * k + 1);
  }
};

__host__ __device__ inline double ln_pos(double x) {
  constexpr ArtanhSeries a{};
  constexpr double kLn2 = 0.69314718055994530942;
  constexpr double kSqrtHalf = 0.70710678118654752440;
  // a subnormal x is scaled by 2^54 first
  const bool sub = x < 2.2250738585072014e-308;
  if (sub) x *= 18014398509481984.0;
  // x = m 2^e, m in [1/2, 1), from the bits of a normal x
  const unsigned long long bits = __builtin_bit_cast(unsigned long long, x);
  int e = (int)((bits >> 52) & 0x7ffu) - 1022 - (sub ? 54 : 0);
  double m = __builtin_bit_cast(double, (bits & 0x000fffffffffffffull) | 0x3fe0000000000000ull);
  if (m < kSqrtHalf) {
    m *= 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0), z = s * s;
  double p = a.c[10];
  for (int k = 9; k >= 0; --k) p = __builtin_fma(p, z, a.c[k]);
  return __builtin_fma((double)e, kLn2, s * p);
}

}  // namespace dd
