// dd_visit_rows.h -- the series of the per-visit rows that the map query over
// a general visit list builds on the device (see k_visit_map).
//
// At one query time a visit has fixed b0 (its b of Eqs. 1-2 over sigma^2 at
// the end of the beam-on time seen from t), db and b1 = b0 + db, so its pair
// term at squared distance a (units of sigma^2) is the series of the uniform
// scan with coefficients of the visit alone:
//   phi_hat(a) = E1(x1) - E1(x0) = exp(-x1) sum_m P_m dx^m,
//   x1 = a / b1, dx = x0 - x1 = a db / (b0 b1), q = db / b0,
//   P_m = (-1)^m q J_m(q) / m!,   J_m(q) = int_0^1 u^m / (1 + q u) du
// (u = x1 e^s in the E1 integral, then the exponential expanded in powers of
// dx), with P_0 = ln(1 + q), the log form of Eqs. 3-4 at a = 0.  J_m by the
// regime of q:
//   q <= 1/4: J_m = 1/(m+1) - q J_{m+1} downwards from J_N = 1/(N+1),
//     N = M + 28.  J_N lies in [1/((N+1)(1+q)), 1/(N+1)], so the start is off
//     by less than q/(N+1), and each step multiplies that error by q: below
//     q^29/(N+1) < 1e-19 at m <= M, where J_m > 1/(1.25 (m+1)).  The steps'
//     own roundings are damped the same way.
//   1/4 < q <= 1: the 24-node Gauss-Legendre rule (the integrand's pole at
//     u = -1/q is at least one interval length away).
//   q > 1: J_0 = ln(1 + q)/q and J_{m+1} = (1/(m+1) - J_m)/q upwards, whose
//     errors shrink by 1/q per step; 1/(m+1) - J_m >= q/((1+q)(m+2)) >
//     1/(2(m+2)), so the difference cancels no digits.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "dd_internal.h"

namespace dd {

// Gauss-Legendre rule of N nodes on [0, 1] (nodes x, weights w summing to
// 1), computed at compile time: Newton iteration on P_N from the usual
// cosine estimates, then the weights 1 / ((1 - z^2) P_N'(z)^2) halved.
constexpr double ccos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 30; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
template <int N>
struct GLRule {
  double x[N], w[N];
  constexpr GLRule() : x(), w() {
    for (int i = 0; i < N; ++i) {
      double z = ccos(3.141592653589793 * (i + 0.75) / (N + 0.5)), dp = 1.0;
      for (int it = 0; it < 12; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 1; k < N; ++k) {
          const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
          p0 = p1;
          p1 = p2;
        }
        dp = N * (z * p1 - p0) / (z * z - 1.0);
        if (it < 11) z -= p1 / dp;
      }
      x[i] = 0.5 * (1.0 - z);
      w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

// Smallest degree M <= MM whose truncation bound e^{2 dx} dx^{M+1} / (M+1)!
// (relative to the term) is at most `target` at dx >= 0; MM if none is.
template <int MM>
__host__ __device__ inline int series_degree(double dx, double target) {
  double b = exp(2.0 * dx) * dx;
  int M = 0;
  while (M < MM && b > target) {
    ++M;
    b *= dx / (M + 1);
  }
  return M;
}

// Per-term truncation targets of the map rows: FP64 kTrunc64; mixed 2e-8,
// below the FP32 evaluation's own ~1e-7.
constexpr double kTrunc32 = 2e-8;

}  // namespace dd
