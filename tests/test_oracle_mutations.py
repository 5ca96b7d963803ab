"""Planted-mistake check for the oracle's pins.

Each case copies the oracle source, plants one plausible mistake (a dropped
term, a flipped sign, a wrong index, a transposed operand, a wrong constant),
compiles the copy to a temporary library on the CPU and runs a few of the
independent pins against it.  Every mutant must fail at least one pin; the
unmodified source must pass all of them.  Nothing here touches the GPU.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla

import geoinputs

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")

MUTANTS = {
    "none": None,
    "cholesky_sign": ("s -= li[k] * lj[k];", "s += li[k] * lj[k];"),
    "cholesky_index": ("s -= li[k] * lj[k];", "s -= li[k] * li[k];"),
    "forward_transposed": ("s -= l[i * n + k] * w[k];", "s -= l[k * n + i] * w[k];"),
    "logdet_factor": ("t[i] = 2.0 * log(l[i * n + i]);", "t[i] = log(l[i * n + i]);"),
    "loglik_dropped_term": ("out[0] = -0.5 * quad - 0.5 * logdet - 0.5 * (double)n * log(2.0 * M_PI);",
                            "out[0] = -0.5 * quad - 0.5 * (double)n * log(2.0 * M_PI);"),
    "matern_gamma": ("tgamma(theta3)", "tgamma(theta3 + 1.0)"),
    "matern_power": ("pow(2.0, theta3 - 1.0)", "pow(2.0, theta3)"),
    "bessel_nu": ("sum += 0.5 * (exp(a + nu * t) + exp(a - nu * t));",
                  "sum += 0.5 * (exp(a + 0.5 * nu * t) + exp(a - 0.5 * nu * t));"),
    "bessel_halfweight": ("double sum = 0.5 * exp(peak);", "double sum = exp(peak);"),
    "bessel_sinh": ("(exp(a + nu * t) + exp(a - nu * t))", "(exp(a + nu * t) - exp(a - nu * t))"),
    "bessel_power": ("const double lx = log(x);", "const double lx = log(0.5 * x);"),
    "distance_sign": ("double dx = x1 - x2, dy = y1 - y2;", "double dx = x1 - x2, dy = y1 + y2;"),
    "krige_backward_skipped": ("oracle_backward(a, n, w, v);", "memcpy(v, w, (size_t)n * sizeof(double));"),
    "trmv_upper": ("for (int64_t k = 0; k <= i; ++k) s += l[i * n + k] * e[k];",
                   "for (int64_t k = 0; k <= i; ++k) s += l[k * n + i] * e[k];"),
    "gcd_cos_twice": ("cos(phi1) * cos(phi2)", "cos(phi1) * cos(phi1)"),
    "gcd_full_angle": ("double s1 = sin(0.5 * dphi)", "double s1 = sin(dphi)"),
    "gcd_no_degrees": ("const double deg = M_PI / 180.0;", "const double deg = 1.0;"),
    "gcd_no_factor_two": ("return 2.0 * radius * asin(sqrt(h));", "return radius * asin(sqrt(h));"),
    "variance_sign": ("var[k] = theta1 - oracle_dot(w, n);", "var[k] = theta1 + oracle_dot(w, n);"),
    "variance_backward": ("oracle_forward(a, n, sk, w);", "oracle_backward(a, n, sk, w);"),
    "ind_stride": ("for (int64_t s = 0; s < n; s += block) {", "for (int64_t s = 0; s < n; s += block + 1) {"),
    "ind_sum_sign": ("        l += part[0];", "        l -= part[0];"),
    "krige_ind_no_backward": ("oracle_backward(a, no, w, v);", "memcpy(v, w, (size_t)no * sizeof(double));"),
    "krige_ind_block_edge": ("const int64_t e = (n - s < block) ? n : s + block;",
                             "const int64_t e = (n - s < block) ? n : s + block - 1;"),
    "krige_ind_own_point": ("(metric, radius, x[i], y[i], bx[j], by[j])", "(metric, radius, x[j], y[j], bx[j], by[j])"),
}


def _build(tmp_path, name, mutation):
    src = open(SRC).read()
    if mutation is not None:
        old, new = mutation
        assert src.count(old) >= 1, name
        src = src.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
                           "-D_GNU_SOURCE", str(c), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    D, I64, P = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_matern.restype = D
    lib.oracle_matern.argtypes = [D, D, D, D]
    lib.oracle_loglik.restype = I64
    INT = ctypes.c_int
    lib.oracle_distance.restype = D
    lib.oracle_distance.argtypes = [INT, D, D, D, D, D]
    lib.oracle_loglik.argtypes = [P, P, P, I64, D, D, D, INT, D, P, P]
    lib.oracle_krige.restype = I64
    lib.oracle_krige.argtypes = [P, P, P, I64, P, P, I64, D, D, D, INT, D, P, P]
    lib.oracle_synth.restype = I64
    lib.oracle_synth.argtypes = [P, P, P, I64, D, D, D, INT, D, P]
    lib.oracle_loglik_ind.restype = I64
    lib.oracle_loglik_ind.argtypes = [P, P, P, I64, D, D, D, INT, D, I64, P]
    lib.oracle_krige_ind.restype = I64
    lib.oracle_krige_ind.argtypes = [P, P, P, P, I64, D, D, D, INT, D, I64, P]
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pins(lib):
    """Returns the list of failed pin names."""
    failed = []
    # Matérn closed forms (Sec. 2.2)
    for r, t2 in [(0.05, 0.1), (0.3, 0.2)]:
        x = r / t2
        if abs(lib.oracle_matern(r, 1.3, t2, 0.5) - 1.3 * math.exp(-x)) > 1e-14:
            failed.append("matern_exp")
        if abs(lib.oracle_matern(r, 1.3, t2, 1.5) - 1.3 * (1 + x) * math.exp(-x)) > 1e-14:
            failed.append("matern_32")
    # general and large smoothness against mpmath (x^ν K_ν near its x -> 0
    # limit at large ν, where x^ν underflows and K_ν overflows on their own)
    import mpmath
    mpmath.mp.dps = 30
    for nu, xx in [(0.77, 0.4), (2.2, 3.0), (13.0, 0.5), (45.0, 1e-8), (45.0, 30.0)]:
        want = float(mpmath.mpf(2) ** (1 - nu) / mpmath.gamma(nu) * mpmath.mpf(xx) ** nu * mpmath.besselk(nu, xx))
        if not abs(lib.oracle_matern(xx, 1.0, 1.0, nu) - want) <= 1e-12 * want:
            failed.append("matern_mpmath")
            break
    # l(θ) vs eigendecomposition on a jittered grid
    n = 40
    theta = (1.1, 0.15, 1.5)
    x, y = geoinputs.jittered_grid(n, 7)
    z = geoinputs.normal_vector(n, 7)
    a = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            dx, dy = x[i] - x[j], y[i] - y[j]
            rr = math.sqrt(dx * dx + dy * dy) / theta[1]
            a[i, j] = theta[0] * (1 + rr) * math.exp(-rr)
    lam, u = np.linalg.eigh(a)
    ref_ld = float(np.sum(np.log(lam)))
    ref_q = float(np.sum((u.T @ z) ** 2 / lam))
    ref_l = -0.5 * n * math.log(2 * math.pi) - 0.5 * ref_ld - 0.5 * ref_q
    out = np.zeros(3)
    lib.oracle_loglik(_p(x), _p(y), _p(z), n, *theta, 0, 1.0, _p(out), None)
    if not abs(out[0] - ref_l) <= 1e-9 * abs(ref_l):
        failed.append("loglik_eig")
    # kriging vs dense solve
    xn, yn = geoinputs.uniform_points(4, 7)
    zn, vn = np.zeros(4), np.zeros(4)
    lib.oracle_krige(_p(x), _p(y), _p(z), n, _p(xn), _p(yn), 4, *theta, 0, 1.0, _p(zn), _p(vn))
    s12 = np.empty((4, n))
    for k in range(4):
        for j in range(n):
            dx, dy = xn[k] - x[j], yn[k] - y[j]
            rr = math.sqrt(dx * dx + dy * dy) / theta[1]
            s12[k, j] = theta[0] * (1 + rr) * math.exp(-rr)
    if not np.allclose(zn, s12 @ np.linalg.solve(a, z), rtol=1e-8, atol=1e-10):
        failed.append("krige_dense")
    # prediction variance (Eq. 4) vs dense solve
    dense_var = theta[0] - np.einsum("kj,jk->k", s12, np.linalg.solve(a, s12.T))
    if not np.allclose(vn, dense_var, rtol=1e-8, atol=1e-12):
        failed.append("variance_dense")
    # great-circle distance: equator, meridian, 3-D chord
    R = 6371.0
    if abs(lib.oracle_distance(1, R, 10.0, 0.0, 40.0, 0.0) - R * math.pi / 6) > 1e-9:
        failed.append("gcd_equator")
    if abs(lib.oracle_distance(1, R, -90.0, 10.0, -90.0, 55.0) - R * math.pi / 4) > 1e-9:
        failed.append("gcd_meridian")
    for (l1, p1, l2, p2) in [(-95.0, 33.0, -88.5, 41.2), (-99.0, 44.0, -86.0, 30.5)]:
        u = [np.array([math.cos(math.radians(p)) * math.cos(math.radians(l)),
                       math.cos(math.radians(p)) * math.sin(math.radians(l)), math.sin(math.radians(p))])
             for l, p in ((l1, p1), (l2, p2))]
        want = 2 * R * math.asin(np.linalg.norm(u[0] - u[1]) / 2)
        if abs(lib.oracle_distance(1, R, l1, p1, l2, p2) - want) > 1e-9 * want:
            failed.append("gcd_chord")
    # IND (Sec. 6.8) vs the block-masked dense covariance
    blk = np.arange(n) // 15
    am = np.where(blk[:, None] == blk[None, :], a, 0.0)
    lam_m, u_m = np.linalg.eigh(am)
    ref_ind = -0.5 * n * math.log(2 * math.pi) - 0.5 * float(np.sum(np.log(lam_m))) \
        - 0.5 * float(np.sum((u_m.T @ z) ** 2 / lam_m))
    out_ind = np.zeros(3)
    lib.oracle_loglik_ind(_p(x), _p(y), _p(z), n, *theta, 0, 1.0, 15, _p(out_ind))
    if not abs(out_ind[0] - ref_ind) <= 1e-9 * abs(ref_ind):
        failed.append("ind_masked")
    # kriging under IND vs the conditional mean of the block-masked covariance
    miss = np.zeros(n, dtype=np.int32)
    miss[[2, 9, 17, 31, 38]] = 1
    o, mm = miss == 0, miss != 0
    zi = np.zeros(int(miss.sum()))
    lib.oracle_krige_ind(_p(x), _p(y), _p(z), _p(miss), n, *theta, 0, 1.0, 15, _p(zi))
    if not np.allclose(zi, am[np.ix_(mm, o)] @ np.linalg.solve(am[np.ix_(o, o)], z[o]), rtol=1e-8, atol=1e-10):
        failed.append("krige_ind_masked")
    # synth vs LAPACK factor
    e = geoinputs.normal_vector(n, 8)
    zs = np.zeros(n)
    lib.oracle_synth(_p(x), _p(y), _p(e), n, *theta, 0, 1.0, _p(zs))
    if not np.allclose(zs, sla.cholesky(a, lower=True) @ e, rtol=1e-9, atol=1e-10):
        failed.append("synth_lapack")
    return failed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    lib = _build(tmp_path, name, MUTANTS[name])
    failed = _pins(lib)
    if name == "none":
        assert failed == []
    else:
        assert failed, f"planted mistake {name} passed every pin"
