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


def hub_network(seed: int = 21):
    """420 buses with four hubs whose bus segments (head lane + one lane per
    incident half-edge + one per generator) are 63, 64 and 65 lanes (either
    side of one 64-lane wave) and 124 lanes (two generators and a parallel
    branch at the hub): the last two take the workgroup-wide reduction.
    Chains and 30 random extra branches among the other buses; parameters
    from the seeded generator with taps, shifts and shunts."""
    rng = np.random.default_rng(seed)
    edges = []
    edges += [(0, v) for v in range(1, 62)]          # hub 0: 61 leaves
    edges += [(100, v) for v in range(101, 162)]     # hub 100: 61 leaves
    edges += [(200, v) for v in range(201, 263)]     # hub 200: 62 leaves
    edges += [(300, v) for v in range(301, 420)]     # hub 300: 119 leaves
    edges += [(0, 100), (100, 200), (200, 300)]      # hub degrees 62, 63, 64, 120
    for a, b in ((61, 100), (161, 200), (262, 300)):  # chains 61-62-..-99 etc.
        edges += [(v, v + 1) for v in range(a, b - 1)]
    hubs = {0, 100, 200, 300}
    present = {(min(u, v), max(u, v)) for u, v in edges}
    extra = []
    while len(extra) < 30:
        u, v = (int(z) for z in rng.integers(0, 420, size=2))
        if u == v or u in hubs or v in hubs or (min(u, v), max(u, v)) in present:
            continue
        present.add((min(u, v), max(u, v)))
        extra.append((u, v))
    edges = edges + extra + [(300, 301)]  # a parallel branch at the big hub
    L = len(edges)
    flip = rng.random(L) < 0.5
    perm = rng.permutation(L)
    f_bus = np.array([edges[j][1] if flip[j] else edges[j][0] for j in perm], np.int32)
    t_bus = np.array([edges[j][0] if flip[j] else edges[j][1] for j in perm], np.int32)
    is_extra = np.zeros(L, bool)
    is_extra[419:419 + 30] = True
    G = 20
    cs = synth.network(420, L, G, seed, variant=True)
    leaves = np.array([v for v in range(420) if v not in hubs])
    gen_bus = np.r_[rng.choice(leaves, G - 2), [300, 300]].astype(np.int32)
    cs.update(f_bus=f_bus, t_bus=t_bus, gen_bus=gen_bus, ref_bus=np.array([gen_bus[0]], np.int32),
              extra_branches=np.flatnonzero(is_extra[perm]).astype(np.int32))
    return cs


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


# Strict-form counts of the parity checks of this session, by case tag:
# printed in the session's summary and written as JSON to the file named by
# OPF_PARITY_RECORD, if set (tests/conftest.py).
STRICT_COUNTS = {}


def record_strict(tag, n_strict, n_total):
    STRICT_COUNTS[tag] = dict(strict_violations=int(n_strict), compared=int(n_total))
