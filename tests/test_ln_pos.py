"""Host check of the renderer's logarithm (not a GPU test).

``dd::ln_pos`` in ``csrc/dd_log.h`` takes ln x = e ln 2 + 2 artanh(s),
s = (m - 1)/(m + 1), m in [sqrt(1/2), sqrt(2)), by eleven terms of the
artanh series.  The colour scale needs t = ln(v/lo)/ln(hi/lo) only to well
inside 1e-12 (the decision slack of the render tests).  This test compiles
the header for the host with g++ and compares it with ``logl`` (long double)
over the whole double range, subnormals included."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_00294_amd", "csrc")

SRC = r"""
#include <cmath>
#include <cstdio>
#include <random>
#define __host__
#define __device__
#include "dd_log.h"
int main() {
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  long double rel = 0, ab = 0, sub = 0;
  for (int i = 0; i < 400000; ++i) {
    double x = std::pow(10.0, 307.9 * u(g));
    if (i % 4 == 1) x = 1.0 + 1e-3 * u(g);                 // near 1
    if (i % 4 == 2) x = std::ldexp(1.0 + 0.5 * u(g), -1060);  // subnormal
    const long double r = logl((long double)x), d = dd::ln_pos(x);
    const long double e = fabsl(d - r);
    if (i % 4 == 2) { if (e / fabsl(r) > sub) sub = e / fabsl(r); continue; }
    if (fabsl(r) > 1e-3L && e / fabsl(r) > rel) rel = e / fabsl(r);
    if (e > ab) ab = e;
  }
  const double one = dd::ln_pos(1.0), two = dd::ln_pos(2.0), half = dd::ln_pos(0.5);
  printf("%.6Le %.6Le %.6Le %.17g %.17g %.17g\n", rel, ab, sub, one, two, half);
}
"""


def test_ln_pos_against_libm(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no g++")
    src = tmp_path / "ln.cpp"
    src.write_text(SRC)
    exe = tmp_path / "ln"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    rel, ab, sub, one, two, half = map(float, subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True).stdout.split())
    assert rel < 5e-16, rel   # a few units in the last place
    assert ab < 2e-13, ab     # |ln x| up to 709
    assert sub < 5e-16, sub   # subnormals, scaled first
    assert one == 0.0
    assert abs(two - 0.6931471805599453) <= 1.2e-16 and abs(half + 0.6931471805599453) <= 1.2e-16
