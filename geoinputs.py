"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds only random draws and the placement of locations; it does no
covariance, factorisation or likelihood arithmetic.  Both the HIP path and the
CPU oracle receive exactly the arrays produced here.

Recipes (Sec. 7.1 of the paper describes the synthetic workload):

* ``jittered_grid(n, seed)`` — irregular locations in the unit square: a g×g
  grid with g = ceil(sqrt(n)), each point moved by independent U(-0.4, 0.4)
  draws in units of the grid spacing, i.e. ((r - 0.5 + X_rl)/g, (l - 0.5 + Y_rl)/g)
  for r, l = 1..g, generated r-major and truncated to the first n points.
  The paper writes the scale as n^(1/2) times the grid coordinates; scaling to
  the unit square changes only the distance unit, which the range θ2 absorbs.
* ``normal_vector(n, seed)`` — e_i ~ N(0, 1) for Z = L e (Alg. 1).
* ``uniform_points(m, seed)`` — m extra locations ~ U[0, 1]^2 (held-out kriging
  targets).
* ``serving_fields(count, seed)`` — per-field sizes and true parameters for the
  many-optimiser workload: n ~ U{1000..16000}, θ1 ~ U[0.5, 2], θ2 ~ U[0.02, 0.3],
  θ3 ~ U{0.5, 1.0, 1.5, 2.5}.

All draws come from numpy's PCG64 generator; each recipe uses its own stream
(seed, tag) so that changing one input never shifts another.
"""
from __future__ import annotations

import math

import numpy as np

_TAG_JITTER = 1
_TAG_NORMAL = 2
_TAG_UNIFORM = 3
_TAG_FIELDS = 4
_TAG_ARRIVALS = 5


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(tag)]))


def grid_side(n: int) -> int:
    g = math.isqrt(n)
    return g if g * g >= n else g + 1


def jittered_grid(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """n jittered grid locations in [0,1]^2 as two float64 arrays (x, y)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    g = grid_side(n)
    rng = _rng(seed, _TAG_JITTER)
    jx = rng.uniform(-0.4, 0.4, size=(g, g))
    jy = rng.uniform(-0.4, 0.4, size=(g, g))
    r = np.arange(1, g + 1, dtype=np.float64)[:, None]
    l = np.arange(1, g + 1, dtype=np.float64)[None, :]
    x = ((r - 0.5 + jx) / g).reshape(-1)[:n]
    y = ((l - 0.5 + jy) / g).reshape(-1)[:n]
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def normal_vector(n: int, seed: int) -> np.ndarray:
    return _rng(seed, _TAG_NORMAL).standard_normal(n)


def uniform_points(m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    rng = _rng(seed, _TAG_UNIFORM)
    return rng.uniform(0.0, 1.0, size=m), rng.uniform(0.0, 1.0, size=m)


def serving_fields(count: int, seed: int, n_lo: int = 1000, n_hi: int = 16000):
    """List of dicts {n, theta} for the many-optimiser serving workload."""
    rng = _rng(seed, _TAG_FIELDS)
    nus = np.array([0.5, 1.0, 1.5, 2.5])
    out = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        theta = (float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.02, 0.3)),
                 float(nus[rng.integers(0, 4)]))
        out.append({"n": n, "theta": theta})
    return out


def arrival_times(count: int, rate: float, seed: int) -> np.ndarray:
    """Poisson-process start times (seconds) for `count` clients at `rate` per second."""
    rng = _rng(seed, _TAG_ARRIVALS)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
