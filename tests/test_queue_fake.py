"""The request queue's host code (scheduler thread, admission, cancellation,
kept factors and their least-recently-used release, dataset release with
requests pending, context teardown) built for the CPU against a stand-in HIP
runtime and CPU stand-ins of the kernels (tests/fake_hip/), driven by many
client threads, under ThreadSanitizer and under AddressSanitizer with
UndefinedBehaviorSanitizer and leak checking.  No GPU is used; the driver
checks every delivered result against the closed form the stand-ins compute
(Σ = θ1·I)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
SOURCES = [os.path.join(ROOT, "paper_1708_02835_amd", "csrc", f) for f in ("engine.cpp", "serve.cpp", "batch.cpp")] + \
          [os.path.join(ROOT, "tests", "fake_hip", f) for f in ("fake_hip.cpp", "fake_kernels.cpp", "queue_driver.cpp")]


@pytest.mark.parametrize("sanitize,env", [
    ("thread", {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"}),
    ("address,undefined", {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1",
                           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}),
])
def test_queue_under_sanitizer(tmp_path, sanitize, env):
    if not os.path.exists(CLANG) and not shutil.which(CLANG):
        pytest.skip("clang++ not available")
    exe = tmp_path / "queue_driver"
    cmd = [CLANG, "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "tests", "fake_hip"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1708_02835_amd", "csrc"), *SOURCES, "-o", str(exe), "-lpthread"]
    if "undefined" in sanitize:
        cmd.insert(4, "-fno-sanitize-recover=undefined")
    subprocess.check_call(cmd)
    for run in range(2):
        p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240, env={**os.environ, **env})
        assert p.returncode == 0 and p.stdout.strip().endswith("ok"), (p.stdout[-2000:], p.stderr[-4000:])
        assert "WARNING: ThreadSanitizer" not in p.stderr and "ERROR: AddressSanitizer" not in p.stderr
