"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host-side
C++ (model construction, patterns, bounds) and of the CPU oracle, run over
every model kind and some malformed inputs (CPU only; host code, no GPU
code is built with a sanitizer)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(tmp_path, compiler, srcs, extra):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not found")
    exe = str(tmp_path / "driver")
    subprocess.run([compiler] + SAN + extra + ["-o", exe] + srcs + ["-lm"], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_host_model_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "g++", [os.path.join(HERE, "host_driver.cpp"),
                                           os.path.join(ROOT, "paper_2510_12897_amd", "csrc", "host_model.cpp")],
                         ["-std=c++17", "-I", os.path.join(ROOT, "include"),
                          "-I", os.path.join(ROOT, "paper_2510_12897_amd", "csrc"), "-I", HERE])
    assert "host driver: ok" in out


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc", [os.path.join(HERE, "oracle_driver.c")],
                         ["-std=c99", "-ffp-contract=off", "-I", HERE])
    assert "oracle driver: ok" in out
