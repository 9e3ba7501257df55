"""CPU checks of the benchmark's contract: one GPU only, the algorithmic
byte model of a callback set, and the kernel-code hash that keys the
committed HBM-traffic summary."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2510_12897_amd import opf, synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_10k_set():
    """9,284,048 bytes per 10k-bus set: every input read once, every output
    written once (the figure the roofline divides by)."""
    cs = synth.network(10000, 13500, 2000, 1)
    dims = opf.case_dims(cs)
    assert dims == (78000, 114501, 429001, 140000)
    assert bench.algorithmic_bytes(cs, dims) == 9284048


def test_kernel_hash_ignores_comments_and_whitespace():
    code = "int f(int a) {\n  return a + 1;  // one more\n}\n"
    same = "/* header */\nint f(int a) { return a + 1; }\n"
    other = "int f(int a) { return a + 2; }\n"
    assert bench.kernel_hash([code]) == bench.kernel_hash([same])
    assert bench.kernel_hash([code]) != bench.kernel_hash([other])
