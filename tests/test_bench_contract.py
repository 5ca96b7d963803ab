"""The benchmark's command-line contract, checked on the CPU: more than one
GPU is refused with a JSON message, and the HBM-traffic record is only used
for the kernel source it was measured with."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_traffic_record_matches_only_its_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "trailing_f64_n100000_hbm_traffic.json")))
    assert rec["hbm_bytes_per_launch"] > 0
    assert bench.measured_traffic(100000, 256) is None      # another workload
    assert bench.measured_traffic(40000, 512) is None       # no record
    # a record whose hash does not match the source is ignored
    fake = tmp_path / "profiles"
    fake.mkdir()
    bad = dict(rec, source_sha256="0" * 64)
    (fake / "trailing_f64_n100000_hbm_traffic.json").write_text(json.dumps(bad))
    (tmp_path / os.path.dirname(rec["source"])).mkdir(parents=True)
    (tmp_path / rec["source"]).write_bytes(open(os.path.join(ROOT, rec["source"]), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(100000, 512) is None


def test_cpu_baseline_fit_and_record():
    """The CPU-baseline leg on tiny sizes: pinned to one core, four timed
    sizes, a fit on the first three checked against the fourth, host model
    and core counts recorded, and the affinity restored afterwards."""
    sys.path.insert(0, ROOT)
    import bench
    before = os.sched_getaffinity(0)
    r = bench.cpu_baseline(2000, (1.0, 0.1, 0.5), sizes=(200, 400, 600, 800))
    assert os.sched_getaffinity(0) == before
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["extrapolated"] is True
    assert r["sizes"] == [200, 400, 600, 800] and len(r["seconds"]) == 4 and r["value"] > 0
    assert r["pinned_core"] in before and r["nproc"] >= 1 and "cpu_model" in r
    assert abs(r["fit_residual_at_largest"]) < 10


def test_fit_cubic_recovers_exact_coefficients():
    sys.path.insert(0, ROOT)
    import bench
    a, b = bench.fit_cubic((100, 200, 300), [2e-9 * n ** 3 + 3e-7 * n ** 2 for n in (100, 200, 300)])
    assert abs(a - 2e-9) < 1e-15 and abs(b - 3e-7) < 1e-12


def test_class_utilisation_arithmetic():
    """The mixed legs' per-class rates from stand-in phase timings: TFLOP/s
    from algorithmic flops and summed launch time, fractions of the class's
    matrix peak with and without the split classes' extra products, classes
    without launches left out, timing switched off afterwards."""
    sys.path.insert(0, ROOT)
    import bench

    class FakeG:
        PRECISION_CLASSES = ("fp64", "fp32", "bf16x6", "bf16x3", "bf16", "fp16x3", "fp16")
        calls = []

        def gl_profile_enable(self, ctx, on):
            self.calls.append(on)

        def gl_opts_default(self, **kw):
            return kw

        def loglik_eval(self, *a):
            return {}

        def gl_profile_phases(self, ctx):
            ph = {"mixed_" + c: {"ms": 0.0, "flops": 0.0, "launches": 0} for c in self.PRECISION_CLASSES}
            ph["mixed_fp64"] = {"ms": 10.0, "flops": 0.393e12, "launches": 4}   # 39.3 TFLOP/s
            ph["mixed_fp16x3"] = {"ms": 100.0, "flops": 25e12, "launches": 7}  # 250 TFLOP/s
            return ph

    fg = FakeG()
    out = bench.class_utilisation(fg, None, None, None, None, (1, 0.1, 0.5), 3, 512)
    assert set(out) == {"fp64", "fp16x3"} and fg.calls == [1, 0]
    assert abs(out["fp64"]["tflops"] - 39.3) < 1e-9 and abs(out["fp64"]["frac_of_peak"] - 0.5) < 1e-12
    assert abs(out["fp16x3"]["tflops"] - 250.0) < 1e-9
    assert abs(out["fp16x3"]["frac_of_peak"] - 0.1) < 1e-12
    assert abs(out["fp16x3"]["frac_of_peak_counting_products"] - 0.3) < 1e-12
