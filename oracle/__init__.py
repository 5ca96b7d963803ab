"""Plain FP64 CPU oracle for the exact Matérn log-likelihood (arXiv 1708.02835).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  The C source
``oracle.c`` holds every formula with its citation; this module only compiles
it with gcc (single-threaded, ``-O2 -ffp-contract=off``, no fast-math) and
marshals numpy arrays.

Functions (each follows the passage named in ``oracle.c``):

* ``bessel_k(nu, x)`` / ``bessel_k_scaled`` — K_ν from its integral form.
* ``matern(r, theta)`` — Sec. 2.2 Eq. (2).
* ``distance(x1, y1, x2, y2, metric, radius)`` — Euclidean (metric 0) or
  great-circle by the haversine formula (metric 1, Sec. 7.4; x = longitude,
  y = latitude in degrees).
* ``cov_matrix`` / ``cov_symmetric`` — genDistanceMatrix + genCovMatrix.
* ``cholesky``, ``forward``, ``backward``, ``trmv`` — unblocked dense kernels.
* ``loglik`` — Alg. 2 / Eq. (1), returns (l, logdet, quad, info).
* ``krige`` — Alg. 3 / Eq. (5), optionally the variances of Eq. (4).
* ``synth`` — Alg. 1, Z = L e.
* ``loglik_ind`` — the IND approximation of Sec. 6.8 (blocks of consecutive
  locations, off-block covariances annihilated).
* ``krige_ind`` — kriging (Eq. (5)) under the IND approximation of the
  covariance of all locations: each held-out value from its own block.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` next to the source (rebuilt when stale)."""
    stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    D, I64, P = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
    sig = {
        "oracle_bessel_k": (D, [D, D]),
        "oracle_bessel_k_scaled": (D, [D, D]),
        "oracle_matern": (D, [D, D, D, D]),
        "oracle_distance": (D, [ctypes.c_int, D, D, D, D, D]),
        "oracle_cov_matrix": (None, [P, P, I64, P, P, I64, D, D, D, ctypes.c_int, D, P]),
        "oracle_cov_symmetric": (None, [P, P, I64, D, D, D, ctypes.c_int, D, P]),
        "oracle_cholesky": (I64, [P, I64]),
        "oracle_forward": (None, [P, I64, P, P]),
        "oracle_backward": (None, [P, I64, P, P]),
        "oracle_trmv": (None, [P, I64, P, P]),
        "oracle_logdet": (D, [P, I64]),
        "oracle_dot": (D, [P, I64]),
        "oracle_loglik": (I64, [P, P, P, I64, D, D, D, ctypes.c_int, D, P, P]),
        "oracle_krige": (I64, [P, P, P, I64, P, P, I64, D, D, D, ctypes.c_int, D, P, P]),
        "oracle_synth": (I64, [P, P, P, I64, D, D, D, ctypes.c_int, D, P]),
        "oracle_loglik_ind": (I64, [P, P, P, I64, D, D, D, ctypes.c_int, D, I64, P]),
        "oracle_krige_ind": (I64, [P, P, P, P, I64, D, D, D, ctypes.c_int, D, I64, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def bessel_k(nu: float, x: float) -> float:
    return _load().oracle_bessel_k(float(nu), float(x))


def bessel_k_scaled(nu: float, x: float) -> float:
    """e^x K_ν(x)."""
    return _load().oracle_bessel_k_scaled(float(nu), float(x))


def matern(r: float, theta) -> float:
    t1, t2, t3 = (float(t) for t in theta)
    return _load().oracle_matern(float(r), t1, t2, t3)


EUCLIDEAN, GREAT_CIRCLE = 0, 1
EARTH_RADIUS_KM = 6371.0


def distance(x1, y1, x2, y2, metric: int = EUCLIDEAN, radius: float = EARTH_RADIUS_KM) -> float:
    return _load().oracle_distance(int(metric), float(radius), float(x1), float(y1), float(x2), float(y2))


def cov_matrix(x1, y1, x2, y2, theta, metric: int = EUCLIDEAN, radius: float = EARTH_RADIUS_KM) -> np.ndarray:
    x1, y1, x2, y2 = map(_f64, (x1, y1, x2, y2))
    out = np.empty((x1.size, x2.size), dtype=np.float64)
    _load().oracle_cov_matrix(_p(x1), _p(y1), x1.size, _p(x2), _p(y2), x2.size,
                              *map(float, theta), int(metric), float(radius), _p(out))
    return out


def cov_symmetric(x, y, theta, metric: int = EUCLIDEAN, radius: float = EARTH_RADIUS_KM) -> np.ndarray:
    x, y = _f64(x), _f64(y)
    out = np.empty((x.size, x.size), dtype=np.float64)
    _load().oracle_cov_symmetric(_p(x), _p(y), x.size, *map(float, theta), int(metric), float(radius), _p(out))
    return out


def cholesky(a) -> tuple[np.ndarray, int]:
    """Returns (L, info); L is lower triangular with a zero upper triangle."""
    l = np.array(a, dtype=np.float64, order="C", copy=True)
    info = _load().oracle_cholesky(_p(l), l.shape[0])
    return l, int(info)


def forward(l, z) -> np.ndarray:
    l, z = _f64(l), _f64(z)
    w = np.empty_like(z)
    _load().oracle_forward(_p(l), z.size, _p(z), _p(w))
    return w


def backward(l, w) -> np.ndarray:
    l, w = _f64(l), _f64(w)
    v = np.empty_like(w)
    _load().oracle_backward(_p(l), w.size, _p(w), _p(v))
    return v


def trmv(l, e) -> np.ndarray:
    l, e = _f64(l), _f64(e)
    z = np.empty_like(e)
    _load().oracle_trmv(_p(l), e.size, _p(e), _p(z))
    return z


def logdet(l) -> float:
    l = _f64(l)
    return _load().oracle_logdet(_p(l), l.shape[0])


def dot(w) -> float:
    w = _f64(w)
    return _load().oracle_dot(_p(w), w.size)


def loglik(x, y, z, theta, return_factor: bool = False, metric: int = EUCLIDEAN,
           radius: float = EARTH_RADIUS_KM):
    """Alg. 2: returns (l, logdet, quad, info) [, L]."""
    x, y, z = map(_f64, (x, y, z))
    out = np.zeros(3, dtype=np.float64)
    fac = np.empty((x.size, x.size), dtype=np.float64) if return_factor else None
    info = _load().oracle_loglik(_p(x), _p(y), _p(z), x.size, *map(float, theta), int(metric), float(radius),
                                 _p(out), _p(fac) if fac is not None else None)
    res = (float(out[0]), float(out[1]), float(out[2]), int(info))
    return (res + (fac,)) if return_factor else res


def krige(x, y, z, xnew, ynew, theta, return_variance: bool = False, metric: int = EUCLIDEAN,
          radius: float = EARTH_RADIUS_KM):
    """Alg. 3 / Eq. (5): returns (Z1, info), or (Z1, var, info) with the
    prediction variances of Eq. (4)."""
    x, y, z, xnew, ynew = map(_f64, (x, y, z, xnew, ynew))
    out = np.zeros(xnew.size, dtype=np.float64)
    var = np.zeros(xnew.size, dtype=np.float64) if return_variance else None
    info = _load().oracle_krige(_p(x), _p(y), _p(z), x.size, _p(xnew), _p(ynew), xnew.size,
                                *map(float, theta), int(metric), float(radius), _p(out),
                                _p(var) if var is not None else None)
    return (out, var, int(info)) if return_variance else (out, int(info))


def synth(x, y, e, theta, metric: int = EUCLIDEAN, radius: float = EARTH_RADIUS_KM) -> tuple[np.ndarray, int]:
    """Alg. 1: returns (Z = L e, info)."""
    x, y, e = map(_f64, (x, y, e))
    z = np.zeros_like(e)
    info = _load().oracle_synth(_p(x), _p(y), _p(e), x.size, *map(float, theta), int(metric), float(radius),
                                _p(z))
    return z, int(info)


def loglik_ind(x, y, z, theta, block: int, metric: int = EUCLIDEAN, radius: float = EARTH_RADIUS_KM):
    """IND approximation (Sec. 6.8): returns (l, logdet, quad, info) summed over
    diagonal blocks of `block` consecutive locations."""
    x, y, z = map(_f64, (x, y, z))
    out = np.zeros(3, dtype=np.float64)
    info = _load().oracle_loglik_ind(_p(x), _p(y), _p(z), x.size, *map(float, theta), int(metric), float(radius),
                                     int(block), _p(out))
    return float(out[0]), float(out[1]), float(out[2]), int(info)


def krige_ind(x, y, z, missing, theta, block: int, metric: int = EUCLIDEAN, radius: float = EARTH_RADIUS_KM):
    """Kriging under the IND approximation (Sec. 6.8 with Eq. (5)): blocks of
    `block` consecutive locations (observed and held-out alike) are
    independent; each held-out value (missing != 0) is predicted from the
    observed values of its block.  Returns (predictions in location order,
    info)."""
    x, y, z = map(_f64, (x, y, z))
    miss = np.ascontiguousarray(missing, dtype=np.int32)
    out = np.zeros(int(np.count_nonzero(miss)), dtype=np.float64)
    info = _load().oracle_krige_ind(_p(x), _p(y), _p(z), _p(miss), x.size, *map(float, theta), int(metric),
                                    float(radius), int(block), _p(out))
    return out, int(info)
