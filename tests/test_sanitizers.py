"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the FP64 oracle (C) driven through every entry point on small systems, and the
engine's host-only paths (parameter checks, workspace sizing and carving,
error reporting) through its C ABI.  Each driver also checks a few results;
the tests pass when the drivers exit cleanly with no sanitizer report.  The
engine is built with the sanitizers on its host code only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-6000:]
    assert "ERROR: AddressSanitizer" not in report and "runtime error" not in report, report[-6000:]
    return report


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_driver"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-o", str(exe), os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(HERE, "oracle_driver.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    out = _run(exe, {"OMP_NUM_THREADS": "2", "ASAN_OPTIONS": "detect_leaks=1",
                     "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert "all checks passed" in out


def test_engine_host_paths_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    exe = tmp_path / "engine_host_driver"
    # the sanitizers apply to the host code only (-Xarch_host before each)
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-o", str(exe),
           os.path.join(ROOT, "paper_1310_0998_amd", "csrc", "engine.hip"),
           os.path.join(HERE, "engine_host_driver.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    # the HIP runtime is not instrumented: its allocations are not ours to report
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0",
                     "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert "all checks passed" in out
