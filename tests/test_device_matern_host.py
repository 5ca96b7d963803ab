"""The device Matérn evaluator (csrc/matern_device.hpp, Temme's series for
x <= 2, Miller's backward recurrence for x > 2, the upward recurrence in the
order) compiled for the host and checked against mpmath's besselk, over
x = r/θ2 in [1e-8, 745] and smoothness 0.05 ... 50, including large ν at small
x, where x^ν underflows and K_ν overflows on their own.  No GPU is used: the
header is plain __host__ __device__ code."""
import os
import shutil
import subprocess

import mpmath
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
NORMAL_MIN = 2.2250738585072014e-308


@pytest.fixture(scope="module")
def evaluator(tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("mh") / "matern_host_eval"
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1708_02835_amd", "csrc"),
                           os.path.join(ROOT, "tests", "matern_host_eval.cpp"), "-o", str(exe)])

    def run(pairs, closed=False):
        inp = "".join(f"{nu!r} {x!r}\n" for nu, x in pairs)
        args = [str(exe)] + (["closed"] if closed else [])
        out = subprocess.run(args, input=inp, capture_output=True, text=True, check=True).stdout
        return [float(v) for v in out.split()]
    return run


def _tol(nu, x):
    """2e-13, or more where x^ν e^-x goes through an exponential of a large
    argument: its rounding, ε·|ν log x - x|, carries into the result."""
    return max(2e-13, 4 * 2.2e-16 * (abs(nu * np.log(x)) + x))


def _ref(nu, x):
    mpmath.mp.dps = 40
    return float(mpmath.mpf(2) ** (1 - nu) / mpmath.gamma(nu) * mpmath.mpf(x) ** nu * mpmath.besselk(nu, x))


@pytest.mark.parametrize("nu", [0.05, 0.3, 0.77, 1.0, 1.3, 2.2, 3.2, 7.6, 20.0, 45.0, 49.7, 50.0])
def test_device_evaluator_wide_range(evaluator, nu):
    xs = list(np.geomspace(1e-8, 745.0, 57)) + [1.999999999, 2.0, 2.000000001, 16.0, 16.5, 700.0, 745.0]
    got = evaluator([(nu, x) for x in xs])
    for x, v in zip(xs, got):
        ref = _ref(nu, x)
        assert np.isfinite(v), (nu, x, v)
        if ref >= NORMAL_MIN:
            assert abs(v - ref) <= _tol(nu, x) * ref, (nu, x, v, ref)
        else:
            assert abs(v - ref) <= 64 * 5e-324, (nu, x, v, ref)


def test_device_evaluator_large_order_small_argument(evaluator):
    # x^ν K_ν(x) -> 2^(ν-1) Γ(ν), so C -> θ1 = 1; formerly 0 · inf = NaN here
    pairs = [(45.0, 1e-8), (40.3, 1e-8), (49.7, 1e-5), (50.0, 1e-12), (30.5, 1e-30)]
    for (nu, x), v in zip(pairs, evaluator(pairs)):
        ref = _ref(nu, x)
        assert abs(ref - 1.0) <= 1e-12 and abs(v - ref) <= _tol(nu, x), (nu, x, v, ref)


def test_device_evaluator_far_field(evaluator):
    """Large ν keeps normal values well past x = 745 (x^ν offsets e^-x); the
    evaluator returns 0 past x = 2000, where every ν <= 50 has underflowed,
    including the closed forms at astronomically large x (no 0 · inf)."""
    pairs = [(nu, x) for nu in (20.0, 45.0, 50.0) for x in (760.5, 800.0, 900.0, 1100.0, 1500.0)]
    for (nu, x), v in zip(pairs, evaluator(pairs)):
        ref = _ref(nu, x)
        if ref >= NORMAL_MIN:
            assert abs(v - ref) <= _tol(nu, x) * ref, (nu, x, v, ref)
        else:
            assert abs(v - ref) <= 64 * 5e-324, (nu, x, v, ref)
    far = [(nu, x) for nu in (0.3, 0.5, 1.5, 2.5, 3.2, 50.0) for x in (2000.5, 1e6, 1e200, 1e300)]
    assert all(v == 0.0 for v in evaluator(far))
    for nu in (0.5, 1.5, 2.5, 50.0):
        assert _ref(nu, 2000.0) == 0.0


def test_half_integer_evaluator_matches_general_bit_for_bit(evaluator):
    """The specialised tile generator (half-integer smoothness, Euclidean
    distance) evaluates matern_eval_closed; it must give the general
    evaluator's values exactly, including r = 0 and the far-field cut."""
    xs = [0.0] + list(np.geomspace(1e-12, 2500.0, 301)) + [1.0, 2.0, 2000.0, 2000.0000001]
    for nu in (0.5, 1.5, 2.5):
        pairs = [(nu, x) for x in xs]
        general, closed = evaluator(pairs), evaluator(pairs, closed=True)
        assert all(a == b for a, b in zip(general, closed)), nu
        ref = [float(mpmath.mpf(2) ** (1 - nu) / mpmath.gamma(nu) * mpmath.mpf(x) ** nu * mpmath.besselk(nu, x))
               if 0 < x <= 700 else None for x in xs]
        for x, v, r in zip(xs, closed, ref):
            if r is not None and r >= NORMAL_MIN:
                assert abs(v - r) <= _tol(nu, x) * r, (nu, x, v, r)
