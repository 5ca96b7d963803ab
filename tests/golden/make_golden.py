"""Writes the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py

config1_n1600.txt: the 1,600-point workload of the paper's synthetic
experiments (Sec. 7.1: 40 x 40 jittered grid in the unit square, Matérn
θ = (1, 0.1, 0.5), Z = L e as in Alg. 1, seed 1000): the measurements Z and
the oracle's l(θ), log|Σ| and ZᵀΣ⁻¹Z (Eq. 1, Alg. 2), each printed with 17
significant digits (binary64 round trip).
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import geoinputs  # noqa: E402
import oracle  # noqa: E402

N, SEED, THETA = 1600, 1000, (1.0, 0.1, 0.5)


def main() -> None:
    x, y = geoinputs.jittered_grid(N, SEED)
    e = geoinputs.normal_vector(N, SEED)
    z, info = oracle.synth(x, y, e, THETA)
    assert info == 0
    l, logdet, quad, info = oracle.loglik(x, y, z, THETA)
    assert info == 0
    with open(os.path.join(HERE, "config1_n1600.txt"), "w") as f:
        f.write("# Sec. 7.1 synthetic workload, n = 1600 (40 x 40 jittered grid), theta = (1, 0.1, 0.5),\n")
        f.write("# Z = L e (Alg. 1), geoinputs seed 1000; values from oracle/ (Eq. 1, Alg. 2);\n")
        f.write("# written by tests/golden/make_golden.py\n")
        f.write(f"n {N}\nseed {SEED}\ntheta {THETA[0]!r} {THETA[1]!r} {THETA[2]!r}\n")
        f.write(f"loglik {l:.17g}\nlogdet {logdet:.17g}\nquad {quad:.17g}\n")
        f.write("z\n")
        for v in z:
            f.write(f"{v:.17g}\n")


if __name__ == "__main__":
    main()
