"""Helpers shared by the GPU parity tests: build inputs for both sides from
one ScanSpec and compare with the tolerance model of the parity tests."""
import math

import numpy as np

# Relative error per element: |g - o| / max(|o|, floor), with the floor in
# units of the prefactor Q0/(4 pi D): values below it (deep in the underflow
# range of the precision in use) are compared absolutely.
FLOOR_HAT = {"fp64": 1e-250, "mixed": 1e-30}
TOL = {"fp64": 1e-10, "mixed": 1e-6}


def oracle_scan(ora, spec, visits):
    return ora.Scan(spec.nx, spec.ny, visits, spec.pitch_m, spec.tau_v, spec.sigma_m, spec.D_m2s,
                    spec.Q0_us)


def prefactor(spec):
    return spec.Q0_us / (4 * math.pi * spec.D_m2s)


def rel_err(got, ref, spec, prec):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    floor = FLOOR_HAT[prec] * prefactor(spec)
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


def assert_close(got, ref, spec, prec, what=""):
    err = rel_err(got, ref, spec, prec)
    worst = float(err.max()) if err.size else 0.0
    assert np.all(np.isfinite(got)), what
    assert worst <= TOL[prec], f"{what} {prec}: max rel err {worst:.3e} at {int(err.argmax())}"
    return worst
