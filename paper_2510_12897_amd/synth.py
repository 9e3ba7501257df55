"""Seeded synthetic inputs for the polar AC-OPF callbacks.

This module is the only code shared by the HIP path, its tests and the CPU
oracle.  It draws networks, loads, evaluation points and multipliers; it holds
none of the model's arithmetic (no flows, no derivatives, no pattern rules).

Networks stand in for the PGLib-OPF / GOC3 / epigrids cases the paper
benchmarks on (Sec. IV, Tables I-III), which are not available here.  Sizes
follow the paper's "Large" classes (static nvar > 75k, multi-period
nvar > 500k).  Recipe:

* topology: a uniformly random labelled spanning tree (Pruefer-sequence
  decoding) plus extra edges drawn as uniform bus pairs, rejecting self-loops
  and pairs already present; tree edges get a random orientation, extra edges
  keep the order their endpoints were drawn in; the branch list is then
  shuffled so tree and extra edges interleave.
* branches: r ~ U(0.005, 0.05), x ~ U(0.02, 0.3), line charging
  b ~ U(0, 0.05), tap 1, shift 0, rate_a ~ U(0.5, 2.0) p.u.,
  angle-difference limits +-pi/6.
* generators: buses uniform with replacement, c2 ~ U(0.01, 0.1),
  c1 ~ U(10, 40), c0 = 0, pg in [0, 3], qg in [-1, 1].
* buses: pd ~ U(0, 0.5), qd = 0.3 pd, vm in [0.9, 1.1], gs = bs = 0;
  the reference bus is the bus of generator 0.
* ``variant=True`` (tests only) also draws tap ~ U(0.9, 1.1),
  shift ~ U(-0.1, 0.1), gs, bs ~ U(-0.05, 0.05) and c0 ~ U(0, 10).

All draws use numpy's PCG64 generator seeded by the caller, in the fixed
order written below, so a seed always yields the same arrays.
"""
from __future__ import annotations

import heapq
import math

import numpy as np

__all__ = [
    "network",
    "point",
    "multipliers",
    "mp_loads",
    "outages",
    "scenario_loads",
    "perturbed_loads",
    "storage",
    "devices",
    "BATCH_SIZES",
]

# Bus counts of the eight networks in the uneven batch mix.
BATCH_SIZES = (500, 1000, 2000, 3000, 5000, 8000, 12000, 20000)


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _pruefer_tree(n: int, rng: np.random.Generator):
    """Edges of a uniformly random labelled tree on n nodes."""
    if n < 2:
        return []
    if n == 2:
        return [(0, 1)]
    seq = rng.integers(0, n, size=n - 2)
    degree = np.ones(n, dtype=np.int64)
    for s in seq:
        degree[s] += 1
    leaves = [i for i in range(n) if degree[i] == 1]
    heapq.heapify(leaves)
    edges = []
    for s in seq:
        leaf = heapq.heappop(leaves)
        edges.append((leaf, int(s)))
        degree[s] -= 1
        if degree[s] == 1:
            heapq.heappush(leaves, int(s))
    u = heapq.heappop(leaves)
    v = heapq.heappop(leaves)
    edges.append((u, v))
    return edges


def network(n_bus: int, n_branch: int, n_gen: int, seed, variant: bool = False) -> dict:
    """Draw one synthetic transmission network.

    Returns a dict of numpy arrays named like the C-ABI case fields, plus
    ``extra_branches`` (indices of the non-tree branches, int32) which the
    contingency recipe draws outages from so that no outage islands a bus.
    """
    if n_bus < 2:
        raise ValueError("a network needs at least two buses")
    if n_branch < n_bus - 1:
        raise ValueError("n_branch must be at least n_bus - 1 (spanning tree)")
    if n_branch > n_bus * (n_bus - 1) // 2:
        raise ValueError("too many branches for a simple graph")
    if n_gen < 1:
        raise ValueError("at least one generator is needed")
    rng = _rng(seed)
    tree = _pruefer_tree(n_bus, rng)
    flip = rng.random(len(tree)) < 0.5
    edges = [(v, u) if fl else (u, v) for (u, v), fl in zip(tree, flip)]
    present = {(min(u, v), max(u, v)) for u, v in edges}
    n_extra = n_branch - len(edges)
    extra = []
    while len(extra) < n_extra:
        u, v = (int(z) for z in rng.integers(0, n_bus, size=2))
        key = (min(u, v), max(u, v))
        if u == v or key in present:
            continue
        present.add(key)
        extra.append((u, v))
    all_edges = edges + extra
    is_extra = np.zeros(n_branch, dtype=bool)
    is_extra[len(edges):] = True
    perm = rng.permutation(n_branch)
    f_bus = np.array([all_edges[j][0] for j in perm], dtype=np.int32)
    t_bus = np.array([all_edges[j][1] for j in perm], dtype=np.int32)
    is_extra = is_extra[perm]

    L = n_branch
    r = rng.uniform(0.005, 0.05, L)
    x = rng.uniform(0.02, 0.3, L)
    b = rng.uniform(0.0, 0.05, L)
    rate_a = rng.uniform(0.5, 2.0, L)
    tap = np.ones(L)
    shift = np.zeros(L)

    gen_bus = rng.integers(0, n_bus, size=n_gen).astype(np.int32)
    c2 = rng.uniform(0.01, 0.1, n_gen)
    c1 = rng.uniform(10.0, 40.0, n_gen)
    c0 = np.zeros(n_gen)

    pd = rng.uniform(0.0, 0.5, n_bus)
    qd = 0.3 * pd
    gs = np.zeros(n_bus)
    bs = np.zeros(n_bus)
    if variant:
        tap = rng.uniform(0.9, 1.1, L)
        shift = rng.uniform(-0.1, 0.1, L)
        gs = rng.uniform(-0.05, 0.05, n_bus)
        bs = rng.uniform(-0.05, 0.05, n_bus)
        c0 = rng.uniform(0.0, 10.0, n_gen)

    return dict(
        n_bus=int(n_bus), n_branch=int(L), n_gen=int(n_gen), n_ref=1,
        pd=pd, qd=qd, gs=gs, bs=bs,
        vmin=np.full(n_bus, 0.9), vmax=np.full(n_bus, 1.1),
        ref_bus=np.array([gen_bus[0]], dtype=np.int32),
        f_bus=f_bus, t_bus=t_bus, r=r, x=x, b=b, tap=tap, shift=shift,
        rate_a=rate_a,
        angmin=np.full(L, -math.pi / 6), angmax=np.full(L, math.pi / 6),
        gen_bus=gen_bus,
        pmin=np.zeros(n_gen), pmax=np.full(n_gen, 3.0),
        qmin=np.full(n_gen, -1.0), qmax=np.full(n_gen, 1.0),
        c2=c2, c1=c1, c0=c0,
        extra_branches=np.flatnonzero(is_extra).astype(np.int32),
    )


def point(case: dict, seed, n_periods: int = 1, n_cont: int = 0, form: str = "polar", storage=None,
          devices=None) -> np.ndarray:
    """An evaluation point drawn inside the variable bounds.

    Blocks are concatenated in the model's variable order (va, vm, pg, qg,
    p, q), each block entity-fastest over its replicas (periods or copies);
    with contingency copies the pg block is shared (one replica).  va, which
    is unbounded, is drawn from U(-pi/6, pi/6); p and q of an arc from
    U(-rate_a, rate_a) of its branch.  For the rectangular form the same
    draws give the bus blocks (vr, vi) = (vm cos va, vm sin va).
    """
    rng = _rng(seed)
    nrep = n_periods if n_periods > 1 else n_cont + 1
    npg = 1 if n_cont > 0 else nrep
    N, L, G = case["n_bus"], case["n_branch"], case["n_gen"]
    rate_arc = np.concatenate([case["rate_a"], case["rate_a"]])
    va = rng.uniform(-math.pi / 6, math.pi / 6, N * nrep)
    vm = rng.uniform(np.tile(case["vmin"], nrep), np.tile(case["vmax"], nrep))
    pg = rng.uniform(np.tile(case["pmin"], npg), np.tile(case["pmax"], npg))
    qg = rng.uniform(np.tile(case["qmin"], nrep), np.tile(case["qmax"], nrep))
    p = rng.uniform(-np.tile(rate_arc, nrep), np.tile(rate_arc, nrep))
    q = rng.uniform(-np.tile(rate_arc, nrep), np.tile(rate_arc, nrep))
    assert p.size == 2 * L * nrep and pg.size == G * npg
    if form == "rect":
        va, vm = vm * np.cos(va), vm * np.sin(va)
    elif form != "polar":
        raise ValueError(f"unknown form {form!r}")
    blocks = [va, vm, pg, qg, p, q]
    if storage is not None:  # ps, qs, qsc, se, sc, sd inside their bounds
        st = storage
        rt = np.tile(st["rating"], nrep)
        blocks += [rng.uniform(-rt, rt), rng.uniform(np.tile(st["qmin"], nrep), np.tile(st["qmax"], nrep)),
                   rng.uniform(-rt, rt), rng.uniform(0.0, np.tile(st["emax"], nrep)),
                   rng.uniform(0.0, np.tile(st["chmax"], nrep)), rng.uniform(0.0, np.tile(st["dismax"], nrep))]
    if devices is not None:
        blocks.append(rng.uniform(np.tile(devices["lo"], nrep), np.tile(devices["hi"], nrep)))
    return np.concatenate(blocks)


def multipliers(m: int, seed) -> np.ndarray:
    """Constraint multipliers y ~ N(0, 1)."""
    return _rng(seed).standard_normal(m)


def mp_loads(case: dict, n_periods: int, seed):
    """Per-(bus, period) loads, bus fastest.

    pd[i, t] = pd_i (0.7 + 0.3 sin(2 pi t / 48) + eps[i, t]) with
    eps ~ N(0, 0.02^2); qd uses the same factor.
    """
    rng = _rng(seed)
    N = case["n_bus"]
    t = np.arange(n_periods)
    eps = rng.normal(0.0, 0.02, size=(n_periods, N))
    factor = 0.7 + 0.3 * np.sin(2.0 * math.pi * t / 48.0)[:, None] + eps
    pd_t = (case["pd"][None, :] * factor).reshape(-1)
    qd_t = (case["qd"][None, :] * factor).reshape(-1)
    return pd_t, qd_t


def outages(case: dict, n_cont: int, seed) -> np.ndarray:
    """Outaged branch per contingency copy, drawn without replacement from
    the non-tree branches so that no copy islands a bus."""
    extra = case["extra_branches"]
    if n_cont > extra.size:
        raise ValueError("more contingencies than non-tree branches")
    rng = _rng(seed)
    return np.sort(rng.choice(extra, size=n_cont, replace=False)).astype(np.int32)


def scenario_loads(case: dict, seed):
    """A fresh load scenario for a network: pd ~ U(0, 0.5), qd = 0.3 pd."""
    rng = _rng(seed)
    pd = rng.uniform(0.0, 0.5, case["n_bus"])
    return pd, 0.3 * pd


def perturbed_loads(case: dict, n_samples: int, seed, spread: float = 0.3):
    """Load samples for the warm-start proxy: each sample scales every bus's
    (pd, qd) by its own factor ~ U(1 - spread, 1 + spread).  Returns
    (pd, qd) arrays of shape (n_samples, n_bus)."""
    rng = _rng(seed)
    fac = rng.uniform(1.0 - spread, 1.0 + spread, size=(n_samples, case["n_bus"]))
    return case["pd"][None, :] * fac, case["qd"][None, :] * fac


def storage(case: dict, seed, frac: float = 0.1, loads=None) -> dict:
    """Storage units at the buses with the largest active loads (the top
    `frac` of buses, at least one), as the paper places them for its
    multi-period benchmarks with storage (Sec. IV-C), each with an energy
    rating of 1.5 times its bus's load there.  The paper gives no other
    parameter; drawn here: charge and discharge ratings 0.5 emax, thermal
    rating 0.6 emax, reactive range +-0.5 rating, efficiencies
    ~ U(0.9, 0.95), converter r ~ U(0, 0.02), x ~ U(0, 0.05), standby losses
    ~ U(0, 1e-3) and an initial energy of 0.5 emax.  `loads` (default the
    case's pd) picks the buses."""
    rng = _rng(seed)
    pd = np.asarray(case["pd"] if loads is None else loads, np.float64)
    n = max(1, int(round(frac * case["n_bus"])))
    bus = np.sort(np.argsort(-pd, kind="stable")[:n]).astype(np.int32)
    emax = np.maximum(1.5 * pd[bus], 1e-3)
    rating = 0.6 * emax
    return dict(bus=bus, emax=emax, chmax=0.5 * emax, dismax=0.5 * emax, rating=rating, qmin=-0.5 * rating,
                qmax=0.5 * rating, eta_c=rng.uniform(0.9, 0.95, n), eta_d=rng.uniform(0.9, 0.95, n),
                r=rng.uniform(0.0, 0.02, n), x=rng.uniform(0.0, 0.05, n), ploss=rng.uniform(0.0, 1e-3, n),
                qloss=rng.uniform(0.0, 1e-3, n), e0=0.5 * emax)


def devices(case: dict, n_dev: int, seed) -> dict:
    """Linear user-extension devices shaped like the electrolyzers of the
    paper's user-extension example (Sec. III-D): buses uniform with
    replacement, a load on the active balance (cp = 1; cq = 0, except every
    third device draws reactive power too, cq ~ U(0.1, 0.3)), a negative
    cost ~ U(-50, -10) (hydrogen revenue), power in [0, 0.5], ramp limit
    0.1 and an initial power of 0."""
    rng = _rng(seed)
    bus = rng.integers(0, case["n_bus"], n_dev).astype(np.int32)
    cq = np.where(np.arange(n_dev) % 3 == 2, rng.uniform(0.1, 0.3, n_dev), 0.0)
    return dict(bus=bus, cp=np.ones(n_dev), cq=cq, cost=rng.uniform(-50.0, -10.0, n_dev),
                lo=np.zeros(n_dev), hi=np.full(n_dev, 0.5), ramp=np.full(n_dev, 0.1), init_lo=np.zeros(n_dev),
                init_hi=np.zeros(n_dev))
