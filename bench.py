"""Benchmark: exact Matérn log-likelihood evaluations per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one full l(θ) evaluation (Alg. 2: Σ(θ) generation, tiled Cholesky,
forward solve, log-determinant, quadratic form) at n = 100,000 jittered-grid
locations (g = 317, first 100,000 points), θ = (1, 0.1, 0.5), tile 512, FP64,
with Z = L e simulated at the same θ (Alg. 1) before timing.  Inputs are
resident in HBM when the timed region starts.

Printed as one JSON line: evals/s of the timed FP64 steps, effective Cholesky
TFLOP/s (n³/3 per step), the trailing-update kernel's live roofline fraction
(HIP events around each of its launches; also split into the bulk launches of
the lookahead stream and the critical-column launches) with its HBM traffic
from the committed counter record, and the oracle timed on one host core as
the CPU baseline.  Legs outside the timed region, each skippable: mixed
precision against FP64 at the same size for two θ (with each precision
class's in-situ matrix-core rate from per-class launch timing), the independent-blocks
approximation per super-tile size (l, and 10-fold prediction MSE against the
exact prediction), small-n latency with and without graph replay,
maximum-likelihood estimates FP64 vs mixed, the 1,600-point evaluation
(median latency, oracle agreement), n = 40,000 per tile size with the kernel
time of each phase and 1,000-point kriging, 64 concurrent Nelder-Mead clients
on the request queue against one-at-a-time evaluation, and n = 150,000 with
BF16 off-band updates and 5,000-point kriging from the resident factor.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak (AMD published)
PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=100000)
    p.add_argument("--tile", type=int, default=512)
    p.add_argument("--theta", type=float, nargs=3, default=(1.0, 0.1, 0.5))
    p.add_argument("--seed", type=int, default=3000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision legs")
    p.add_argument("--theta-b", type=float, nargs=3, default=(1.0, 0.3, 1.0),
                   help="second parameter vector of the mixed-precision comparison")
    p.add_argument("--no-theta-b", action="store_true", help="mixed leg: skip the second theta")
    p.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    p.add_argument("--no-ind", action="store_true", help="skip the independent-blocks leg")
    p.add_argument("--no-graph", action="store_true", help="skip the small-n graph-replay latency leg")
    p.add_argument("--no-mle", action="store_true", help="skip the maximum-likelihood (FP64 vs mixed) leg")
    p.add_argument("--no-small", action="store_true", help="skip the n = 1,600 latency leg")
    p.add_argument("--no-n40k", action="store_true", help="skip the n = 40,000 tile-sweep and kriging leg")
    p.add_argument("--no-n150k", action="store_true", help="skip the n = 150,000 BF16 and kriging leg")
    p.add_argument("--mle-n", type=int, default=8100)
    p.add_argument("--serve-clients", type=int, default=64)
    p.add_argument("--serve-evals", type=int, default=100,
                   help="most l(theta) requests of one client's Nelder-Mead search")
    p.add_argument("--serve-replay", type=int, default=10,
                   help="first requests of every client replayed one at a time for comparison")
    p.add_argument("--serve-rate", type=float, default=400.0, help="client arrivals per second (Poisson)")
    p.add_argument("--serve-think-ms", type=float, default=1.0,
                   help="mean exponential pause of a client between a result and its next request")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="only run device-to-device copies of MIB mebibytes (HBM counter calibration)")
    return p.parse_args()


def calibrate_copy(mib: int) -> None:
    """Plain device copies of a known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters of the benchmark kernels (read: mib MiB, write: mib MiB
    per copy)."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_mib": mib, "copies": 3}), flush=True)


def host_info() -> dict:
    """CPU model (from /proc/cpuinfo) and core counts of the machine the
    oracle is timed on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0))}


CPU_SAMPLE_SIZES = (400, 1600, 2800, 4000)


def fit_cubic(ns, ts):
    """Least-squares t = a n³ + b n² through the timed sizes with a, b >= 0
    (both terms are work, never negative; noisy small sizes could otherwise
    give a negative cubic term); returns (a, b)."""
    import numpy as np
    from scipy.optimize import nnls
    A = np.array([[float(n) ** 3, float(n) ** 2] for n in ns])
    scale = A.max(axis=0)
    coef, _ = nnls(A / scale, np.array(ts, dtype=float))
    a, b = coef / scale
    return float(a), float(b)


def cpu_baseline(n_target: int, theta, sizes=CPU_SAMPLE_SIZES) -> dict:
    """Time the oracle (single-threaded FP64 C, one call per size) pinned to
    one host core at n = 400, 1,600, 2,800 and 4,000 (about 10-30 s), fit
    t = a n³ + b n² on the first three sizes, check the fit against the fourth,
    and extrapolate to the benchmark size (labelled as extrapolated).  The
    n = 1,600 time is the 1,600-point single-evaluation workload timed directly."""
    import geoinputs
    import oracle
    oracle.build()
    info = host_info()
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    times = []
    try:
        for n in sizes:
            x, y = geoinputs.jittered_grid(n, 77)
            z = geoinputs.normal_vector(n, 77)
            t0 = time.perf_counter()
            oracle.loglik(x, y, z, theta)
            times.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, old)
    a, b = fit_cubic(sizes[:3], times[:3])
    n4 = sizes[3]
    pred4 = a * n4 ** 3 + b * n4 ** 2
    t_target = a * n_target ** 3 + b * n_target ** 2
    timed = ", ".join(f"n={n}: {t:.2f} s" for n, t in zip(sizes, times))
    return {"value": 1.0 / t_target, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle l(theta) (generation, unblocked Cholesky, solve) timed once per size on host "
                       f"core {core} ({timed}); t = a n^3 + b n^2 fitted on the first three sizes predicts "
                       f"{pred4:.2f} s at n={n4} (residual {(times[3] - pred4) / times[3]:+.1%}); "
                       f"extrapolated to n={n_target}: {t_target:.3g} s per evaluation"),
            "extrapolated": True, "pinned_core": core, **info,
            "sizes": list(sizes), "seconds": times, "fit": {"a_n3": a, "b_n2": b},
            "fit_residual_at_largest": (times[3] - pred4) / times[3],
            "n1600_direct_s": times[1], "seconds_timed": sum(times)}


def measured_traffic(n: int, tile: int):
    """HBM bytes per trailing-update launch from the committed FETCH_SIZE /
    WRITE_SIZE counter runs of this workload, or None when the kernel source
    has changed since they were taken (or they cover another workload)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"trailing_f64_n{n}_hbm_traffic.json")
    if tile != 512 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["hbm_bytes_per_launch"]


# Dense matrix-core peaks (TFLOP/s) of the arithmetic each precision class
# runs on, and the products one of its tile updates takes.
CLASS_PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x6": 2500.0, "bf16x3": 2500.0, "bf16": 2500.0,
              "fp16x3": 2500.0, "fp16": 2500.0}
CLASS_PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x6": 6, "bf16x3": 3, "bf16": 1, "fp16x3": 3, "fp16": 1}


def class_utilisation(g, ctx, xd, yd, z, th, prec, tile):
    """One more evaluation with the trailing updates timed per precision class
    (HIP events around each launch): summed launch ms, algorithmic flops
    (2b³ per tile update), TFLOP/s and the fraction of the class's matrix
    peak, algorithmically and counting the products of the split classes.
    Launches of different streams overlap, so the per-class figures are
    in-situ rates, not a split of the wall time."""
    g.gl_profile_enable(ctx, 1)
    try:
        g.loglik_eval(ctx, xd, yd, z, th, g.gl_opts_default(precision=prec, tile=tile))
        ph = g.gl_profile_phases(ctx)
    finally:
        g.gl_profile_enable(ctx, 0)
    out = {}
    for cls in g.PRECISION_CLASSES:
        v = ph["mixed_" + cls]
        if not v["launches"]:
            continue
        tf = v["flops"] / (v["ms"] * 1e-3) / 1e12
        out[cls] = {"launches": v["launches"], "ms": v["ms"], "flops": v["flops"], "tflops": tf,
                    "peak_tflops": CLASS_PEAK[cls], "frac_of_peak": tf / CLASS_PEAK[cls],
                    "products_per_update": CLASS_PRODUCTS[cls],
                    "frac_of_peak_counting_products": tf * CLASS_PRODUCTS[cls] / CLASS_PEAK[cls]}
    return out


def mixed_legs(g, ctx, xd, yd, ed, zd, theta, theta_b, args, res64, t64, log):
    """Time-to-l(θ) of the mixed-precision modes against FP64 at the same
    size, with the relative error of l and log|Σ| against the FP64 result,
    for θ (Z simulated at θ) and θ_b (Z simulated at θ_b)."""
    import torch
    out = {}

    def run(z, th, prec, steps):
        opts = g.gl_opts_default(precision=prec, tile=args.tile)
        r = g.loglik_eval(ctx, xd, yd, z, th, opts)  # warm-up (also builds the precision map)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = g.loglik_eval(ctx, xd, yd, z, th, opts)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        stats = g.gl_precision_stats(ctx) if prec != g.GL_FP64 else None
        return r, dt, stats

    legs = [("theta_a", theta, zd, min(args.steps, 3))]
    if not args.no_theta_b:
        legs.append(("theta_b", theta_b, None, 1))
    for label, th, z, steps in legs:
        if z is None:
            z, info = g.synth_generate(ctx, xd, yd, ed, th, args.tile)
            if info != 0:
                out[label] = {"theta": list(th), "error": f"field generation failed, info={info}"}
                continue
            r64, t64b, _ = run(z, th, g.GL_FP64, 1)
        else:
            r64, t64b = res64, t64
        leg = {"theta": list(th), "fp64_ms": t64b * 1e3, "loglik_fp64": r64["loglik"]}
        for name, prec in (("fp16", g.GL_MIXED_FP16), ("bf16", g.GL_MIXED_BF16), ("fp32", g.GL_MIXED_FP32)):
            r, dt, stats = run(z, th, prec, steps if name != "fp32" else 1)
            leg[name] = {"ms": dt * 1e3, "speedup_vs_fp64": t64b / dt,
                         "rel_err_loglik": abs(r["loglik"] - r64["loglik"]) / abs(r64["loglik"]),
                         "rel_err_logdet": abs(r["logdet"] - r64["logdet"]) / abs(r64["logdet"]),
                         "status": r["status"],
                         "work_frac": {k: round(stats[k]["work_frac"], 4) for k in g.PRECISION_CLASSES},
                         "thresholds": stats["thresholds"]}
            log(f"mixed {label} {name}: {dt:.3f} s, x{t64b / dt:.2f}, rel err {leg[name]['rel_err_loglik']:.2e}")
            if label == "theta_a":
                leg[name]["class_util"] = class_utilisation(g, ctx, xd, yd, z, th, prec, args.tile)
        if label == "theta_b":
            # Why the adaptive rule keeps θ_b in binary64: forcing the
            # FP32-grade two-part binary16 class on the tiles with normalised
            # norm up to tol_64 (the rest binary64) puts little work in it
            # already at the 1e-4 error level.
            trade = []
            for tol in (0.1, 0.3):
                opts = g.gl_opts_default(precision=g.GL_MIXED_FP16, tile=args.tile, tol_64=tol, tol_lo=0.0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = g.loglik_eval(ctx, xd, yd, z, th, opts)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                st = g.gl_precision_stats(ctx)
                err = abs(r["loglik"] - r64["loglik"]) / abs(r64["loglik"]) if r["status"] == g.GL_OK else None
                trade.append({"tol_64": tol, "status": r["status"], "low_precision_work_frac": 1.0 - st["fp64"]["work_frac"],
                              "rel_err_loglik": err, "speedup_vs_fp64": t64b / dt})
                log(f"mixed theta_b fp16x3 forced up to nu={tol}: low-precision work "
                    f"{trade[-1]['low_precision_work_frac']:.4f}, rel err {err}, x{t64b / dt:.2f}")
            leg["forced_fp16x3"] = trade
        out[label] = leg
    return out


def ind_legs(g, ctx, xd, yd, zd, theta, args, res64, t64, log):
    """Independent-blocks approximation (diagonal super tiles of s tiles) at
    the benchmark size: time and l against the exact FP64 l."""
    import torch
    out = []
    for s in (1, 2, 4, 8, 16):
        opts = g.gl_opts_default(tile=args.tile, ind_tiles=s)
        g.loglik_eval(ctx, xd, yd, zd, theta, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            r = g.loglik_eval(ctx, xd, yd, zd, theta, opts)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out.append({"super_tile": s, "block_points": s * args.tile, "ms": dt * 1e3, "speedup_vs_exact": t64 / dt,
                    "loglik": r["loglik"], "rel_diff_vs_exact": abs(r["loglik"] - res64["loglik"]) / abs(res64["loglik"])})
        log(f"IND s={s}: {dt * 1e3:.1f} ms, l={r['loglik']:.6f}")
    return out


def ind_prediction_leg(g, ctx, args, log):
    """Prediction MSE of 10-fold cross-validation, exact against IND with
    super tiles of s tiles (the paper's exact-versus-IND prediction
    comparison, on a synthetic field of n = 40,000 jittered-grid locations
    with Z = L e simulated at θ), with the time per fold."""
    import numpy as np
    import torch

    import geoinputs
    n, k, theta = 40000, 10, tuple(args.theta)
    x, y = geoinputs.jittered_grid(n, args.seed + 11)
    e = geoinputs.normal_vector(n, args.seed + 11)
    xd, yd, ed = (torch.as_tensor(a).cuda() for a in (x, y, e))
    zd, info = g.synth_generate(ctx, xd, yd, ed, theta, args.tile)
    if info != 0:
        return {"error": f"field generation failed, info={info}"}
    folds = np.random.Generator(np.random.PCG64([args.seed, 12])).permutation(np.arange(n) % k).astype(np.int32)
    out = {"n": n, "folds": k, "theta": list(theta), "tile": args.tile, "runs": []}
    for s in (0, 1, 2, 4, 8, 16):
        opts = g.gl_opts_default(tile=args.tile, ind_tiles=s)
        t0 = time.perf_counter()
        mse, st = g.krige_cv(ctx, xd, yd, zd, theta, folds, opts)
        dt = time.perf_counter() - t0
        run = {"super_tile": s if s else "exact", "block_points": s * args.tile if s else n,
               "mse_mean": float(np.mean(mse)), "mse_folds": [float(v) for v in mse], "status": st,
               "seconds_per_fold": dt / k}
        out["runs"].append(run)
        log(f"IND prediction s={run['super_tile']}: MSE {run['mse_mean']:.5f}, {dt / k * 1e3:.0f} ms per fold")
    return out


def graph_leg(g, ctx, args, log):
    """Latency of repeated small evaluations (an optimiser on one dataset):
    direct launches against the replayed hipGraph, same inputs and θ walk."""
    import numpy as np
    import torch

    import geoinputs
    out = []
    for n in (1000, 2000, 4000):
        x, y = geoinputs.jittered_grid(n, args.seed + n)
        z = geoinputs.normal_vector(n, args.seed + n)
        xd, yd, zd = (torch.as_tensor(a).cuda() for a in (x, y, z))
        thetas = [(1.0, 0.1 * (1 + 0.01 * i), 0.5) for i in range(40)]
        row = {"n": n}
        for mode in (0, 1):
            opts = g.gl_opts_default(graph=mode)
            g.loglik_eval(ctx, xd, yd, zd, thetas[0], opts)
            lat = []
            for th in thetas:
                t0 = time.perf_counter()
                g.loglik_eval(ctx, xd, yd, zd, th, opts)
                lat.append(time.perf_counter() - t0)
            row["graph_ms" if mode else "direct_ms"] = float(np.median(lat) * 1e3)
        row["speedup"] = row["direct_ms"] / row["graph_ms"]
        log(f"graph n={n}: direct {row['direct_ms']:.3f} ms, graph {row['graph_ms']:.3f} ms")
        out.append(row)
    return out


def mle_leg(g, ctx, args, log):
    """θ̂ from FP64 and from the BF16 and FP16 mixed modes: Nelder-Mead over log θ,
    restarted from its own result until it stops improving (a derivative-free
    stand-in for the paper's BOBYQA), same field and start."""
    import numpy as np
    import torch
    from scipy import optimize

    import geoinputs
    n, truth = args.mle_n, tuple(args.theta)
    x, y = geoinputs.jittered_grid(n, args.seed + 7)
    e = geoinputs.normal_vector(n, args.seed + 7)
    xd, yd, ed = (torch.as_tensor(a).cuda() for a in (x, y, e))
    zd, info = g.synth_generate(ctx, xd, yd, ed, truth)
    if info != 0:
        return {"error": f"field generation failed, info={info}"}
    start = np.log([0.7 * truth[0], 1.4 * truth[1], 0.8 * truth[2]])
    out = {"n": n, "theta_true": list(truth), "optimizer": "Nelder-Mead on log theta with restarts, same start"}
    for name, prec in (("fp64", g.GL_FP64), ("bf16", g.GL_MIXED_BF16), ("fp16", g.GL_MIXED_FP16)):
        opts = g.gl_opts_default(precision=prec)

        def negl(v):
            r = g.loglik_eval(ctx, xd, yd, zd, tuple(float(t) for t in np.exp(v)), opts)
            return -r["loglik"] if r["status"] == g.GL_OK else 1e300

        t0 = time.perf_counter()
        xs, res, nfev = start, None, 0
        for _ in range(5):
            r = optimize.minimize(negl, xs, method="Nelder-Mead", options={"xatol": 1e-5, "fatol": 1e-7, "maxfev": 600})
            nfev += r.nfev
            if res is not None and r.fun > res.fun - 1e-6:
                break
            res, xs = r, r.x
        res.nfev = nfev
        dt = time.perf_counter() - t0
        out[name] = {"theta_hat": [float(v) for v in np.exp(res.x)], "loglik": -float(res.fun),
                     "evals": int(res.nfev), "seconds": dt}
        log(f"mle {name}: theta_hat={np.exp(res.x)} in {res.nfev} evals, {dt:.1f} s")
    a = np.array(out["fp64"]["theta_hat"])
    out["max_rel_diff_theta_hat"] = {m: float(np.max(np.abs(np.array(out[m]["theta_hat"]) - a) / a))
                                     for m in ("bf16", "fp16")}
    return out


def small_leg(g, ctx, args, log):
    """The 1,600-point single evaluation (40 x 40 jittered grid, θ = (1, 0.1,
    0.5), Z = L e): latency as the median of 50 timed evaluations after 5
    warm-ups, and l and log|Σ| against the oracle."""
    import numpy as np
    import torch

    import geoinputs
    import oracle
    n, theta = 1600, (1.0, 0.1, 0.5)
    x, y = geoinputs.jittered_grid(n, 1000)
    e = geoinputs.normal_vector(n, 1000)
    xd, yd, ed = (torch.as_tensor(a).cuda() for a in (x, y, e))
    zd, info = g.synth_generate(ctx, xd, yd, ed, theta)
    if info != 0:
        return {"error": f"field generation failed, info={info}"}
    opts = g.gl_opts_default()
    for _ in range(5):
        g.loglik_eval(ctx, xd, yd, zd, theta, opts)
    lat = []
    for _ in range(50):
        t0 = time.perf_counter()
        r = g.loglik_eval(ctx, xd, yd, zd, theta, opts)
        lat.append(time.perf_counter() - t0)
    ref = oracle.loglik(x, y, zd.cpu().numpy(), theta)
    out = {"n": n, "theta": list(theta), "tile": r["tile"], "median_ms": float(np.median(lat) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "evals_per_s": 1.0 / float(np.median(lat)),
           "loglik": r["loglik"], "logdet": r["logdet"],
           "rel_err_loglik_vs_oracle": abs(r["loglik"] - ref[0]) / abs(ref[0]),
           "rel_err_logdet_vs_oracle": abs(r["logdet"] - ref[1]) / abs(ref[1])}
    log(f"n=1600: median {out['median_ms']:.3f} ms, rel err vs oracle {out['rel_err_loglik_vs_oracle']:.1e}")
    return out


def held_out_field(g, ctx, n, m, seed, theta, tile=0):
    """n jittered-grid locations plus m extra ones ~ U[0,1]², Z simulated
    jointly at all n + m (Alg. 1 on the device); returns device tensors of the
    observed part and the held-out part with its true values."""
    import numpy as np
    import torch

    import geoinputs
    x, y = geoinputs.jittered_grid(n, seed)
    xm, ym = geoinputs.uniform_points(m, seed)
    xa, ya = np.concatenate([x, xm]), np.concatenate([y, ym])
    e = geoinputs.normal_vector(n + m, seed)
    xd, yd, ed = (torch.as_tensor(a).cuda() for a in (xa, ya, e))
    zd, info = g.synth_generate(ctx, xd, yd, ed, theta, tile)
    del ed
    if info != 0:
        return None
    obs = (xd[:n].contiguous(), yd[:n].contiguous(), zd[:n].contiguous())
    held = (xd[n:].contiguous(), yd[n:].contiguous(), zd[n:].cpu().numpy())
    return obs, held


def n40k_leg(g, ctx, args, log):
    """The tiled path at n = 40,000 (200 x 200 jittered grid) for θ = (1, 0.1,
    0.5) and (1, 0.03, 1.5): one timed evaluation per tile size 256, 384, 512
    (after a warm-up) with the kernel time of every phase of Alg. 2, and
    kriging of 1,000 held-out locations (Z simulated jointly with them) from the
    tile-512 factor: time and MSE against the simulated truth."""
    import numpy as np
    import torch
    n, m = 40000, 1000
    out = {"n": n, "held_out": m, "runs": []}
    for ti, theta in enumerate(((1.0, 0.1, 0.5), (1.0, 0.03, 1.5))):
        fld = held_out_field(g, ctx, n, m, args.seed + 20 + ti, theta)
        if fld is None:
            out["runs"].append({"theta": list(theta), "error": "field generation failed"})
            continue
        (xd, yd, zd), (xh, yh, truth) = fld
        for tile in (256, 384, 512):
            opts = g.gl_opts_default(tile=tile)
            g.loglik_eval(ctx, xd, yd, zd, theta, opts)
            torch.cuda.synchronize()
            g.gl_profile_enable(ctx, 2)
            g.gl_profile_phases(ctx)
            t0 = time.perf_counter()
            r = g.loglik_eval(ctx, xd, yd, zd, theta, opts)
            dt = time.perf_counter() - t0
            ph = g.gl_profile_phases(ctx)
            g.gl_profile_enable(ctx, 0)
            t1 = time.perf_counter()
            g.loglik_eval(ctx, xd, yd, zd, theta, opts)  # untimed phases: the plain wall time
            dt_plain = time.perf_counter() - t1
            run = {"theta": list(theta), "tile": tile, "seconds": dt_plain, "seconds_with_phase_events": dt,
                   "cholesky_tflops": n ** 3 / 3.0 / dt_plain / 1e12, "loglik": r["loglik"], "status": r["status"],
                   "phase_kernel_ms": {p: round(v["ms"], 3) for p, v in ph.items()}}
            for key in ("trail_bulk", "trail_pair"):
                tr = ph[key]
                if tr["ms"] > 0:
                    run[f"{key}_tflops"] = tr["flops"] / (tr["ms"] * 1e-3) / 1e12
            out["runs"].append(run)
            log(f"n=40000 theta={theta} tile={tile}: {dt_plain:.3f} s, phases {run['phase_kernel_ms']}")
        r = g.loglik_eval(ctx, xd, yd, zd, theta, g.gl_opts_default(tile=512, keep_factor=1))
        if r["status"] == g.GL_OK:
            try:
                g.krige_predict(ctx, r["factor"], xh, yh)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pred = g.krige_predict(ctx, r["factor"], xh, yh)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            finally:
                g.gl_factor_release(ctx, r["factor"])
            pred = pred.cpu().numpy()
            out["runs"].append({"theta": list(theta), "kriging_points": m, "kriging_ms": dt * 1e3,
                                "mse_vs_truth": float(np.mean((pred - truth) ** 2)),
                                "truth_variance": float(np.var(truth))})
            log(f"n=40000 theta={theta}: kriging {m} points {dt * 1e3:.2f} ms, "
                f"MSE {out['runs'][-1]['mse_vs_truth']:.4e}")
        del xd, yd, zd, xh, yh
        torch.cuda.empty_cache()
    return out


def n150k_leg(g, args, log):
    """n = 150,000 jittered locations plus 5,000 held out (Z simulated jointly
    at 155,000 points in FP64), θ = (1, 0.1, 0.5): time-to-l with BF16 off-band
    updates, kriging of the 5,000 points from the device-resident BF16 factor
    (the factor reused: no new factorisation), and the same with the FP64
    factor; MSE of the BF16 predictions against the FP64 ones and against the
    simulated truth."""
    import numpy as np
    import torch
    n, m, theta = 150000, 5000, (1.0, 0.1, 0.5)
    out = {"n": n, "held_out": m, "theta": list(theta)}
    ctx = g.Context(0)
    try:
        t0 = time.perf_counter()
        fld = held_out_field(g, ctx, n, m, args.seed + 30, theta)
        log(f"n=150000: field of {n + m} points simulated ({time.perf_counter() - t0:.1f} s)")
        if fld is None:
            return {"error": "field generation failed"}
        (xd, yd, zd), (xh, yh, truth) = fld
        ctx.close()
        ctx = g.Context(0)  # release the simulation's workspace
        torch.cuda.empty_cache()
        preds = {}
        for name, prec in (("bf16", g.GL_MIXED_BF16), ("fp64", g.GL_FP64)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = g.loglik_eval(ctx, xd, yd, zd, theta, g.gl_opts_default(precision=prec, keep_factor=1))
            t_l = time.perf_counter() - t0
            if r["status"] != g.GL_OK:
                out[name] = {"status": r["status"]}
                continue
            try:
                t0 = time.perf_counter()
                pred = g.krige_predict(ctx, r["factor"], xh, yh)
                torch.cuda.synchronize()
                t_k = time.perf_counter() - t0
                t0 = time.perf_counter()
                pred = g.krige_predict(ctx, r["factor"], xh, yh)  # the factor reused again
                torch.cuda.synchronize()
                t_k2 = time.perf_counter() - t0
            finally:
                g.gl_factor_release(ctx, r["factor"])
            preds[name] = pred.cpu().numpy()
            out[name] = {"time_to_l_s": t_l, "loglik": r["loglik"], "logdet": r["logdet"],
                         "kriging_ms": t_k * 1e3, "kriging_reuse_ms": t_k2 * 1e3,
                         "mse_vs_truth": float(np.mean((preds[name] - truth) ** 2))}
            log(f"n=150000 {name}: l in {t_l:.2f} s, kriging {m} points {t_k * 1e3:.1f} ms "
                f"(again {t_k2 * 1e3:.1f} ms), MSE {out[name]['mse_vs_truth']:.4e}")
            torch.cuda.empty_cache()
        if "bf16" in preds and "fp64" in preds:
            out["bf16"]["speedup_vs_fp64"] = out["fp64"]["time_to_l_s"] / out["bf16"]["time_to_l_s"]
            out["bf16"]["rel_err_loglik"] = abs(out["bf16"]["loglik"] - out["fp64"]["loglik"]) / abs(out["fp64"]["loglik"])
            out["bf16"]["mse_vs_fp64_kriging"] = float(np.mean((preds["bf16"] - preds["fp64"]) ** 2))
        out["truth_variance"] = float(np.var(truth))
    finally:
        ctx.close()
        torch.cuda.empty_cache()
    return out


SERVE_THETA0 = (1.0, 0.1, 1.0)
SERVE_BOUNDS = ((0.01, 5.0), (0.005, 1.5), (0.1, 3.0))


def serving_leg(g, ctx, args, log):
    """Many concurrent maximum-likelihood clients on the request queue, each
    on its own synthetic field (n uniform in 1,000..16,000, true θ drawn per
    client), starting as a Poisson process.  Each client runs a bounded
    Nelder-Mead search over log θ from θ0 = (1, 0.1, 1.0) (a derivative-free
    stand-in for the paper's BOBYQA) in closed loop: every objective value is
    one l(θ) request, issued after the previous result and an exponential
    pause, up to --serve-evals requests.  Reported: evals/s over the makespan,
    submit-to-result latency percentiles, and, for the first requests of every
    client replayed one at a time with loglik_eval, the one-at-a-time rate and
    the largest difference of l."""
    import threading

    import numpy as np
    import torch
    from scipy import optimize

    import geoinputs

    clients, maxfev = args.serve_clients, args.serve_evals
    fields = geoinputs.serving_fields(clients, args.seed)
    rng = np.random.Generator(np.random.PCG64([args.seed, 77]))
    data, dss = [], []
    t_s = time.perf_counter()
    for c, f in enumerate(fields):
        n, th = f["n"], f["theta"]
        x, y = geoinputs.jittered_grid(n, args.seed + 1 + c)
        e = geoinputs.normal_vector(n, args.seed + 1 + c)
        xd, yd, ed = (torch.as_tensor(a).cuda() for a in (x, y, e))
        z, info = g.synth_generate(ctx, xd, yd, ed, th)
        if info != 0:
            z = ed  # Σ(θ) not numerically SPD at the true θ: serve white noise
        data.append((xd, yd, z))
        dss.append(g.gl_dataset_register(ctx, xd, yd, z))
    starts = geoinputs.arrival_times(clients, args.serve_rate, args.seed)
    pauses = rng.exponential(args.serve_think_ms * 1e-3, size=(clients, maxfev + 8))
    lo = np.log([b[0] for b in SERVE_BOUNDS])
    hi = np.log([b[1] for b in SERVE_BOUNDS])
    log(f"serving: {clients} fields ready ({time.perf_counter() - t_s:.2f} s)")

    q = g.lq_create(ctx, g.lq_config_default())
    try:
        # warm-up: one request per client, all at once (workspace pool, code objects)
        for t in [g.lq_submit(q, ds, SERVE_THETA0) for ds in dss]:
            g.lq_wait(q, t)
        lat = [[] for _ in range(clients)]
        hist = [[] for _ in range(clients)]
        found = [None] * clients
        errors = []
        t0 = time.perf_counter()

        def client(c):
            try:
                due = [t0 + starts[c]]

                def negl(v):
                    now = time.perf_counter()
                    if due[0] > now:
                        time.sleep(due[0] - now)
                    th = tuple(float(t) for t in np.exp(np.clip(v, lo, hi)))
                    s0 = time.perf_counter()
                    r = g.lq_wait(q, g.lq_submit(q, dss[c], th))
                    done = time.perf_counter()
                    lat[c].append(done - s0)
                    hist[c].append((th, r))
                    due[0] = done + pauses[c][min(len(hist[c]), maxfev + 7)]
                    return -r["loglik"] if r["status"] == g.GL_OK else 1e300

                res = optimize.minimize(negl, np.log(SERVE_THETA0), method="Nelder-Mead",
                                        bounds=list(zip(lo, hi)),
                                        options={"maxfev": maxfev, "xatol": 1e-5, "fatol": 1e-7})
                found[c] = ([float(t) for t in np.exp(res.x)], bool(res.success))
            except Exception as exc:  # noqa: BLE001
                errors.append(repr(exc))

        threads = [threading.Thread(target=client, args=(c,)) for c in range(clients)]
        for th_ in threads:
            th_.start()
        for th_ in threads:
            th_.join()
        wall = time.perf_counter() - t0
        stats = g.lq_stats(q)
        ticks = g.lq_tick_stats(q)
    finally:
        g.lq_destroy(q)
    if errors:
        raise SystemExit(f"serving clients failed: {errors[:3]}")
    all_lat = np.array([v for c in lat for v in c])
    total = int(all_lat.size)
    log(f"serving: {total} evals in {wall:.2f} s, p50 {np.median(all_lat) * 1e3:.1f} ms")

    # the first requests of every client, one at a time
    replay = min(args.serve_replay, min(len(h) for h in hist))
    opts = g.gl_opts_default()
    for c in range(clients):
        g.loglik_eval(ctx, *data[c], hist[c][0][0], opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    single = [[g.loglik_eval(ctx, *data[c], hist[c][k][0], opts) for k in range(replay)] for c in range(clients)]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t1
    for ds in dss:
        g.gl_dataset_release(ctx, ds)
    worst, statuses = 0.0, {}
    for c in range(clients):
        for th, a in hist[c]:
            statuses[str(a["status"])] = statuses.get(str(a["status"]), 0) + 1
        for k in range(replay):
            a, b = hist[c][k][1], single[c][k]
            if a["status"] == g.GL_OK and b["status"] == g.GL_OK:
                worst = max(worst, abs(a["loglik"] - b["loglik"]) / abs(b["loglik"]))
            elif a["status"] != b["status"]:
                statuses["mismatch"] = statuses.get("mismatch", 0) + 1
    ns = [f["n"] for f in fields]
    single_rate = clients * replay / t_single
    log(f"serving: one at a time {single_rate:.1f} evals/s ({clients * replay} replayed)")
    # statistical, not parity: θ̂ after at most --serve-evals evaluations
    # (Nelder-Mead from (1, 0.1, 1.0) has often not converged by then)
    rel_theta = [float(np.max(np.abs(np.array(found[c][0]) - np.array(fields[c]["theta"])) /
                              np.array(fields[c]["theta"]))) for c in range(clients)]
    converged = sum(1 for c in range(clients) if found[c][1])
    return {"clients": clients, "max_evals_per_client": maxfev, "evals": total,
            "evals_per_client": {"min": min(len(h) for h in hist), "max": max(len(h) for h in hist)},
            "optimizer": "bounded Nelder-Mead on log theta from (1, 0.1, 1.0), closed loop",
            "n_range": [min(ns), max(ns)], "n_mean": float(np.mean(ns)),
            "makespan_s": wall, "evals_per_s": total / wall,
            "p50_ms": float(np.percentile(all_lat, 50) * 1e3),
            "p99_ms": float(np.percentile(all_lat, 99) * 1e3), "max_ms": float(all_lat.max() * 1e3),
            "one_at_a_time_evals_per_s": single_rate, "one_at_a_time_sample": clients * replay,
            "speedup_vs_one_at_a_time": total / wall / single_rate,
            "status_counts": statuses, "max_rel_diff_vs_one_at_a_time": worst,
            "optimizers_converged_within_max_evals": converged,
            "theta_at_end_max_rel_diff_vs_truth": {"median": float(np.median(rel_theta)),
                                                   "max": float(np.max(rel_theta))},
            "peak_inflight": stats["peak_inflight"], "peak_bytes": stats["peak_bytes"],
            "fused_launches": stats["fused_launches"],
            "ticks": {"count": ticks["ticks"],
                      "host_us_per_tick": ticks["host_us"] / max(ticks["ticks"], 1),
                      "device_us_per_tick": ticks["device_ms"] * 1e3 / max(ticks["ticks"], 1),
                      "launches_per_tick": stats["fused_launches"] / max(ticks["ticks"], 1),
                      "idle_between_ticks_frac": ticks["gap_ms"] * 1e-3 / wall},
            "arrivals": f"Poisson, {args.serve_rate:g} clients/s; pause {args.serve_think_ms:g} ms mean"}


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the library has no multi-GPU path (use --gpus 1)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import geoinputs
    import paper_1708_02835_amd as g

    n, theta = args.n, tuple(args.theta)
    x, y = geoinputs.jittered_grid(n, args.seed)
    e = geoinputs.normal_vector(n, args.seed)
    dev = torch.device("cuda:0")
    xd = torch.as_tensor(x).to(dev)
    yd = torch.as_tensor(y).to(dev)
    ed = torch.as_tensor(e).to(dev)
    ctx = g.Context(0)
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)
    t_s = time.perf_counter()
    zd, info = g.synth_generate(ctx, xd, yd, ed, theta, args.tile)
    log(f"synthetic field n={n} ready ({time.perf_counter() - t_s:.2f} s)")
    if info != 0:
        raise SystemExit(f"synthetic field generation failed: info={info}")
    opts = g.gl_opts_default(tile=args.tile)
    for i in range(args.warmup):
        s0 = time.perf_counter()
        g.loglik_eval(ctx, xd, yd, zd, theta, opts)
        log(f"warmup {i} {time.perf_counter() - s0:.3f} s")
    torch.cuda.synchronize()
    g.gl_profile_enable(ctx, 1)
    g.gl_profile_phases(ctx)  # reset
    lat = []
    res = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        res = g.loglik_eval(ctx, xd, yd, zd, theta, opts)
        lat.append(time.perf_counter() - s0)
        log(f"step {len(lat) - 1} {lat[-1]:.3f} s l={res['loglik']:.10g}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ph = g.gl_profile_phases(ctx)
    g.gl_profile_enable(ctx, 0)
    crit, bulk, pair = ph["trail_crit"], ph["trail_bulk"], ph["trail_pair"]
    prof = {k: crit[k] + bulk[k] + pair[k] for k in ("ms", "flops", "launches")}
    if res["status"] != g.GL_OK:
        raise SystemExit(f"evaluation failed: {res}")

    step_s = elapsed / args.steps

    def rate(p):
        """Roofline of one kind of trailing launch: the two-panel passes over
        the far columns and the one-panel updates of the near columns
        (lookahead stream), or the next column's update (critical stream)."""
        a = p["flops"] / (p["ms"] * 1e-3) / 1e12 if p["ms"] > 0 else 0.0
        return {"achieved": a, "frac": a / PEAK_FP64_TFLOPS, "launches": p["launches"],
                "avg_launch_ms": p["ms"] / max(p["launches"], 1), "flops_per_launch": p["flops"] / max(p["launches"], 1),
                "busy_frac_of_wall": p["ms"] * 1e-3 / elapsed}
    chol_flops = n ** 3 / 3.0
    # the dominant kernel: the two-panel trailing passes (most of the flops at
    # this size); the one-panel launches and all trailing launches together
    # are reported beside it
    dom = pair if pair["launches"] else bulk
    launches = max(dom["launches"], 1)
    avg_ms = dom["ms"] / launches
    avg_flops = dom["flops"] / launches
    achieved = avg_flops / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    out = {
        "metric": "l(theta) evals/sec at n=100k, FP64 (exact Matern log-likelihood)",
        "value": args.steps / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"l(theta) FP64, n={n} jittered grid (g={geoinputs.grid_side(n)}), "
                               f"theta={list(theta)}, tile {args.tile}, Z = L e simulated at theta",
                   "n": n, "tile": args.tile, "theta": list(theta), "precision": "fp64"},
        "cholesky_tflops": chol_flops / step_s / 1e12,
        "latency_ms": {"p50": statistics.median(lat) * 1e3, "max": max(lat) * 1e3},
        "loglik": res["loglik"], "logdet": res["logdet"],
        "roofline": {"bound": "mfma",
                     "kernel": "trailing_f64_kernel<%d, true> (SYRK/GEMM trailing update, two panels per pass)"
                               % args.tile if pair["launches"] else "trailing_f64_kernel<%d, false>" % args.tile,
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(n, args.tile),
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                     "launches": dom["launches"], "avg_launch_ms": avg_ms,
                     "flops_per_launch": avg_flops,
                     "flop_share": dom["flops"] / max(prof["flops"], 1.0),
                     "all_trailing": rate(prof), "one_panel_bulk": rate(bulk), "critical_column": rate(crit)},
    }
    if not args.no_mixed:
        out["mixed"] = mixed_legs(g, ctx, xd, yd, ed, zd, theta, tuple(args.theta_b), args, res, step_s, log)
    if not args.no_ind:
        out["ind"] = ind_legs(g, ctx, xd, yd, zd, theta, args, res, step_s, log)
        out["ind_prediction"] = ind_prediction_leg(g, ctx, args, log)
    if not args.no_graph:
        out["graph_replay"] = graph_leg(g, ctx, args, log)
    if not args.no_mle:
        out["mle"] = mle_leg(g, ctx, args, log)
    if not args.no_small:
        out["n1600"] = small_leg(g, ctx, args, log)
    if not args.no_n40k:
        out["n40000"] = n40k_leg(g, ctx, args, log)
    if not args.no_serve:
        out["serving"] = serving_leg(g, ctx, args, log)
    ctx.close()
    if not args.no_n150k:
        del xd, yd, ed, zd
        torch.cuda.empty_cache()
        out["n150000"] = n150k_leg(g, args, log)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(n, theta)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
