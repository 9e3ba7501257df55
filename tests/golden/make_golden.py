"""Writes the oracle regression fixtures in this folder.

The paper prints no callback values, so these files are not the paper's:
they hold what the oracle computes for three small seeded models, so that a
later change to the oracle's arithmetic shows up as a failing CPU test
(tests/test_golden.py) and has to be argued for.  Calls only oracle/ and
the seeded input generator.  Run from the repository root:

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2510_12897_amd import synth  # noqa: E402


def cases():
    """(name, case, options, periods, copies, point seed, objective weight)."""
    cs = synth.network(14, 20, 5, 0)
    yield "case14_static", cs, {}, 1, 0, 100, 1.0
    pd_t, qd_t = synth.mp_loads(cs, 3, 1)
    yield "case14_mp3", cs, dict(n_periods=3, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2), 3, 0, 101, 0.5
    yield "case14_sc2", cs, dict(n_cont=2, outaged=synth.outages(cs, 2, 2)), 1, 2, 102, 1.0


def compute(cs, opts, T, K, seed, sigma):
    x = synth.point(cs, seed, n_periods=T, n_cont=K)
    m = O.dims(cs, **opts)[1]
    y = synth.multipliers(m, seed)
    return x, y, O.evaluate(cs, x, y, sigma, **opts)


def write(path, res):
    with open(path, "w") as fh:
        fh.write("# oracle regression fixture, written by tests/golden/make_golden.py\n")
        fh.write(f"f {res['f']!r}\n")
        for key in ("g", "c", "jval", "hval"):
            v = np.asarray(res[key], dtype=np.float64)
            fh.write(f"{key} {v.size}\n")
            fh.writelines(f"{float(a)!r}\n" for a in v)
        for key in ("jrow", "jcol", "hrow", "hcol"):
            v = np.asarray(res[key], dtype=np.int64)
            fh.write(f"{key} {v.size}\n")
            fh.write(" ".join(str(int(a)) for a in v) + "\n")


def read(path) -> dict:
    out = {}
    with open(path) as fh:
        lines = [ln.rstrip("\n") for ln in fh if not ln.startswith("#")]
    i = 0
    while i < len(lines):
        key, val = lines[i].split(" ", 1)
        if key == "f":
            out["f"] = float(val)
            i += 1
        elif key in ("g", "c", "jval", "hval"):
            n = int(val)
            out[key] = np.array([float(a) for a in lines[i + 1:i + 1 + n]], dtype=np.float64)
            i += 1 + n
        else:
            n = int(val)
            out[key] = np.array([int(a) for a in lines[i + 1].split()], dtype=np.int64) if n else np.zeros(0, np.int64)
            i += 2
    return out


if __name__ == "__main__":
    for name, cs, opts, T, K, seed, sigma in cases():
        _, _, res = compute(cs, opts, T, K, seed, sigma)
        write(os.path.join(HERE, name + ".txt"), res)
        print("wrote", name)
