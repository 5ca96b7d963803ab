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
