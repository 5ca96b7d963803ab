"""Stored expected values (tests/golden/, written from the oracle by
tests/golden/make_golden.py) for the 1,600-point workload of Sec. 7.1.

CPU: the oracle still reproduces them, and they agree with an evaluation that
shares nothing with the oracle: the ν = 1/2 Matérn in its closed form
θ1 exp(-r/θ2) (Sec. 2.2) factored by LAPACK, whose ZᵀΣ⁻¹Z must also equal
‖e‖² for Z = L e (Alg. 1).  GPU: the device l(θ) and log|Σ| at the FP64
bound."""
import os

import numpy as np
import pytest

import geoinputs
import oracle

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_config1():
    vals, z = {}, []
    with open(os.path.join(HERE, "config1_n1600.txt")) as f:
        in_z = False
        for line in f:
            if line.startswith("#"):
                continue
            parts = line.split()
            if in_z:
                z.append(float(parts[0]))
            elif parts[0] == "z":
                in_z = True
            else:
                vals[parts[0]] = [float(p) for p in parts[1:]]
    n, seed = int(vals["n"][0]), int(vals["seed"][0])
    x, y = geoinputs.jittered_grid(n, seed)
    return dict(n=n, seed=seed, theta=tuple(vals["theta"]), loglik=vals["loglik"][0], logdet=vals["logdet"][0],
                quad=vals["quad"][0], x=x, y=y, z=np.array(z))


def test_oracle_reproduces_golden():
    c = load_config1()
    e = geoinputs.normal_vector(c["n"], c["seed"])
    z, info = oracle.synth(c["x"], c["y"], e, c["theta"])
    assert info == 0 and np.array_equal(z, c["z"])
    l, logdet, quad, info = oracle.loglik(c["x"], c["y"], c["z"], c["theta"])
    assert info == 0 and (l, logdet, quad) == (c["loglik"], c["logdet"], c["quad"])


def test_golden_against_closed_form_and_lapack():
    from scipy.linalg import cho_factor, cho_solve
    c = load_config1()
    th1, th2, _ = c["theta"]
    x, y, z, n = c["x"], c["y"], c["z"], c["n"]
    r = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    sigma = th1 * np.exp(-r / th2)
    cf = cho_factor(sigma, lower=True)
    logdet = 2.0 * np.sum(np.log(np.diag(cf[0])))
    quad = float(z @ cho_solve(cf, z))
    l = -0.5 * quad - 0.5 * logdet - 0.5 * n * np.log(2.0 * np.pi)
    assert abs(logdet - c["logdet"]) <= 1e-12 * abs(logdet)
    assert abs(quad - c["quad"]) <= 1e-12 * quad
    assert abs(l - c["loglik"]) <= 1e-12 * abs(l)
    e = geoinputs.normal_vector(n, c["seed"])
    assert abs(quad - float(e @ e)) <= 1e-10 * quad


@pytest.mark.gpu
def test_device_matches_golden():
    torch = pytest.importorskip("torch")
    import paper_1708_02835_amd as g
    c = load_config1()
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    with g.Context(0) as ctx:
        r = g.loglik_eval(ctx, dev(c["x"]), dev(c["y"]), dev(c["z"]), c["theta"])
    assert r["status"] == g.GL_OK
    assert abs(r["loglik"] - c["loglik"]) <= 1e-10 * abs(c["loglik"])
    assert abs(r["logdet"] - c["logdet"]) <= 1e-10 * abs(c["logdet"])
