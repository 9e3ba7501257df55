"""Shared test utilities: named synthetic cases and the parity tolerance."""
from __future__ import annotations

import numpy as np

from paper_2510_12897_amd import synth

RTOL = 1e-12
ATOL = 1e-14


def case0(variant: bool = False):
    """The 14-bus parity network (spanning tree + extra edges = 20 branches,
    5 generators), network seed 0."""
    return synth.network(14, 20, 5, 0, variant=variant)


def small_cases():
    """Small networks covering the structural corner cases: both branch
    orientations, several generators on one bus, buses without generators,
    a two-bus network, nonunit taps, phase shifts and shunts."""
    yield "c0", synth.network(14, 20, 5, 0)
    yield "c0v", synth.network(14, 20, 5, 0, variant=True)
    yield "two_bus", synth.network(2, 1, 1, 7, variant=True)
    yield "many_gens", synth.network(6, 9, 12, 11, variant=True)
    yield "tree_only", synth.network(9, 8, 3, 13)


def assert_close(v, ref, scale=None, rtol=RTOL, atol=ATOL, what="values"):
    """Scale-aware parity: |v - ref| <= rtol * max(|ref|, scale) + atol,
    where scale is the oracle's sum of |terms| for each output."""
    v = np.asarray(v, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert v.shape == ref.shape, f"{what}: shape {v.shape} vs {ref.shape}"
    mag = np.abs(ref) if scale is None else np.maximum(np.abs(ref), np.asarray(scale))
    err = np.abs(v - ref)
    bad = ~(err <= rtol * mag + atol)
    if bad.any():
        i = int(np.flatnonzero(bad)[0])
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {v.size} outside tolerance; first at {i}: "
            f"got {v[i]!r} expected {ref[i]!r} (scale {mag[i]:.3e}, err {err[i]:.3e})")


def strict_violations(v, ref, rtol=RTOL, atol=ATOL) -> int:
    """Count of entries that fail the strict form |v - ref| <= rtol |ref| + atol."""
    v = np.asarray(v, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return int((np.abs(v - ref) > rtol * np.abs(ref) + atol).sum())
