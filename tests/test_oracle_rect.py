"""Pins of the oracle's rectangular form (form = :rect, Sec. III-C1; the
ACR formulation of the cited PowerModels).

* At (vr, vi) = vm e^{j va} every flow, balance and thermal row equals the
  polar oracle's row (the two forms describe the same physics), the
  voltage-magnitude row equals vm^2, the reference row vm sin(va) and the
  two angle rows vm_f vm_t (sin th - tan(limit) cos th).
* Flows against S = V conj(I) of the MATPOWER-style branch matrices in
  complex arithmetic, straight from (vr, vi).
* Jacobian and Hessian against central differences (the Hessian as a
  brute-force dense matrix, which also proves pattern coverage).
* Closed-form pattern counts, bounds and the start point; one period and
  zero copies equal the static model.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_12897_amd import synth

from helpers import case0, small_cases
from test_oracle_pins import _branch_matrices, _fd_hessian, _fd_jacobian


def _rect_blocks(cs, nrep=1, T=1):
    N, L, G, R = cs["n_bus"], cs["n_branch"], cs["n_gen"], len(cs["ref_bus"])
    sizes = [("ref", R), ("pfr", L), ("qfr", L), ("pto", L), ("qto", L), ("angu", L), ("angl", L),
             ("balp", N), ("balq", N), ("thf", L), ("tht", L), ("vmag", N)]
    o, out = 0, {}
    for name, s in sizes:
        out[name] = (o, s * nrep)
        o += s * nrep
    out["ramp"] = (o, G * (T - 1))
    return out


def _polar_blocks(cs):
    N, L, R = cs["n_bus"], cs["n_branch"], len(cs["ref_bus"])
    sizes = [("ref", R), ("pfr", L), ("qfr", L), ("pto", L), ("qto", L), ("ang", L),
             ("balp", N), ("balq", N), ("thf", L), ("tht", L)]
    o, out = 0, {}
    for name, s in sizes:
        out[name] = (o, s)
        o += s
    return out


@pytest.mark.parametrize("name,cs", list(small_cases()))
def test_rect_equals_polar_at_the_same_voltages(name, cs):
    N, L = cs["n_bus"], cs["n_branch"]
    xp = synth.point(cs, 11)
    xr = synth.point(cs, 11, form="rect")
    va, vm = xp[:N], xp[N:2 * N]
    np.testing.assert_allclose(xr[:N], vm * np.cos(va), rtol=0, atol=0)
    np.testing.assert_array_equal(xr[2 * N:], xp[2 * N:])
    rp = O.evaluate(cs, xp, want=O.W_CONS | O.W_OBJ)
    rr = O.evaluate(cs, xr, want=O.W_CONS | O.W_OBJ, form="rect")
    assert rr["n"] == rp["n"]
    assert rr["m"] == rp["m"] + L + N
    bp, br = _polar_blocks(cs), _rect_blocks(cs)
    for blk in ("pfr", "qfr", "pto", "qto", "balp", "balq", "thf", "tht"):
        (o1, k), (o2, _) = bp[blk], br[blk]
        np.testing.assert_allclose(rr["c"][o2:o2 + k], rp["c"][o1:o1 + k], rtol=0,
                                   atol=1e-13 * max(1.0, np.abs(rp["cscale"][o1:o1 + k]).max()), err_msg=blk)
    assert rr["f"] == rp["f"]
    o, k = br["vmag"]
    np.testing.assert_allclose(rr["c"][o:o + k], vm ** 2, rtol=1e-14)
    o, k = br["ref"]
    np.testing.assert_allclose(rr["c"][o:o + k], vm[cs["ref_bus"]] * np.sin(va[cs["ref_bus"]]), rtol=1e-14)
    f, t = cs["f_bus"], cs["t_bus"]
    th = va[f] - va[t]
    for blk, lim in (("angu", cs["angmax"]), ("angl", cs["angmin"])):
        o, k = br[blk]
        want = vm[f] * vm[t] * (np.sin(th) - np.tan(lim) * np.cos(th))
        np.testing.assert_allclose(rr["c"][o:o + k], want, rtol=1e-12, atol=1e-14, err_msg=blk)


@pytest.mark.parametrize("name,cs", list(small_cases()))
def test_rect_flows_match_complex_pi_model(name, cs):
    N, L = cs["n_bus"], cs["n_branch"]
    x = synth.point(cs, 12, form="rect")
    x[2 * N + 2 * cs["n_gen"]:] = 0.0  # p = q = 0: the flow rows hold -F
    V = x[:N] + 1j * x[N:2 * N]
    yff, yft, ytf, ytt = _branch_matrices(cs)
    f, t = cs["f_bus"], cs["t_bus"]
    Sf = V[f] * np.conj(yff * V[f] + yft * V[t])
    St = V[t] * np.conj(ytf * V[f] + ytt * V[t])
    c = O.evaluate(cs, x, want=O.W_CONS, form="rect")["c"]
    br = _rect_blocks(cs)
    for blk, ref in (("pfr", Sf.real), ("qfr", Sf.imag), ("pto", St.real), ("qto", St.imag)):
        o, k = br[blk]
        np.testing.assert_allclose(-c[o:o + k], ref, rtol=1e-13, atol=1e-13, err_msg=blk)


def _rect_case(tag):
    if tag == "c0v":
        return case0(variant=True), {}
    if tag == "mp3":
        cs = synth.network(8, 11, 3, 41, variant=True)
        pd_t, qd_t = synth.mp_loads(cs, 3, 42)
        return cs, dict(n_periods=3, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2)
    cs = synth.network(8, 11, 3, 43, variant=True)
    return cs, dict(n_cont=2, outaged=synth.outages(cs, 2, 44))


@pytest.mark.parametrize("tag", ["c0v", "mp3", "sc2"])
def test_rect_jacobian_matches_finite_differences(tag):
    cs, opts = _rect_case(tag)
    opts = dict(opts, form="rect")
    n, m = O.dims(cs, **opts)
    x = synth.point(cs, 6, n_periods=opts.get("n_periods", 1), n_cont=opts.get("n_cont", 0), form="rect")
    r = O.evaluate(cs, x, want=O.W_JAC, **opts)
    Jd = O.dense_jacobian(r)
    Jfd = _fd_jacobian(cs, x, **opts)
    scale = np.zeros((m, n))
    scale[r["jrow"], r["jcol"]] = r["jscale"]
    err = np.abs(Jd - Jfd)
    assert (err <= 2e-6 * (1.0 + scale)).all(), f"max err {err.max():.3e}"
    inpat = np.zeros((m, n), bool)
    inpat[r["jrow"], r["jcol"]] = True
    assert not (np.abs(Jfd) > 1e-6)[~inpat].any()


@pytest.mark.parametrize("tag", ["c0v", "mp3", "sc2"])
def test_rect_hessian_matches_finite_differences(tag):
    cs, opts = _rect_case(tag)
    opts = dict(opts, form="rect")
    n, m = O.dims(cs, **opts)
    x = synth.point(cs, 7, n_periods=opts.get("n_periods", 1), n_cont=opts.get("n_cont", 0), form="rect")
    y = synth.multipliers(m, 7)
    r = O.evaluate(cs, x, y, 0.8, want=O.W_HESS, **opts)
    Hd = O.dense_hessian(r)
    Hfd = _fd_hessian(cs, x, y, 0.8, **opts)
    scale = np.zeros((n, n))
    scale[r["hrow"], r["hcol"]] = r["hscale"]
    scale = np.maximum(scale, scale.T)
    err = np.abs(Hd - Hfd)
    assert (err <= 2e-5 * (1.0 + scale)).all(), f"max err {err.max():.3e}"
    inpat = np.zeros((n, n), bool)
    inpat[r["hrow"], r["hcol"]] = True
    inpat |= inpat.T
    assert not (np.abs(Hfd) > 1e-5)[~inpat].any()
    # no (vr_i, vi_i) entry: the rectangular rows never multiply a bus's
    # two coordinates together
    N = cs["n_bus"] * opts.get("n_periods", 1) * (1 + opts.get("n_cont", 0))
    assert not np.any((r["hrow"] >= N) & (r["hrow"] < 2 * N) & (r["hrow"] - N == r["hcol"]))


@pytest.mark.parametrize("name,cs", list(small_cases()))
def test_rect_pattern_counts(name, cs):
    """Static, simple graph: nnzJ = R + 36L + 6N + 2G (flows 20L, two angle
    rows 8L, balance 4N + 4L + 2G, thermal 4L, magnitude 2N, reference R);
    nnzH = G + 2N + 8L (two bus diagonals, four cross pairs per branch, two
    arc diagonals per arc, the pg diagonal)."""
    N, L, G, R = cs["n_bus"], cs["n_branch"], cs["n_gen"], len(cs["ref_bus"])
    r = O.evaluate(cs, synth.point(cs, 1, form="rect"), want=O.W_JAC | O.W_HESS, form="rect")
    assert r["jrow"].size == R + 36 * L + 6 * N + 2 * G
    assert r["hrow"].size == G + 2 * N + 8 * L
    assert np.all(r["hrow"] >= r["hcol"])
    key = r["hrow"].astype(np.int64) * r["n"] + r["hcol"]
    assert np.all(np.diff(key) > 0)
    keyj = r["jrow"].astype(np.int64) * r["n"] + r["jcol"]
    assert np.all(np.diff(keyj) > 0)


def test_rect_bounds_and_start():
    cs = case0(variant=True)
    K = 2
    out = synth.outages(cs, K, 3)
    b = O.bounds(cs, form="rect", n_cont=K, outaged=out)
    N, L = cs["n_bus"], cs["n_branch"]
    P = K + 1
    np.testing.assert_array_equal(b["x0"][:N * P], 1.0)
    np.testing.assert_array_equal(b["x0"][N * P:2 * N * P], 0.0)
    np.testing.assert_array_equal(b["uvar"][:2 * N * P], np.tile(cs["vmax"], 2 * P))
    np.testing.assert_array_equal(b["lvar"][:2 * N * P], -np.tile(cs["vmax"], 2 * P))
    br = _rect_blocks(cs, nrep=P)
    o, k = br["vmag"]
    np.testing.assert_array_equal(b["lcon"][o:o + k], np.tile(cs["vmin"] ** 2, P))
    np.testing.assert_array_equal(b["ucon"][o:o + k], np.tile(cs["vmax"] ** 2, P))
    for blk, lo, hi in (("angu", -math.inf, 0.0), ("angl", 0.0, math.inf)):
        o, k = br[blk]
        lcon, ucon = b["lcon"][o:o + k].reshape(P, L), b["ucon"][o:o + k].reshape(P, L)
        for s in range(P):
            keep = np.ones(L, bool)
            if s >= 1:
                keep[out[s - 1]] = False
                assert lcon[s, out[s - 1]] == -math.inf and ucon[s, out[s - 1]] == math.inf
            assert np.all(lcon[s, keep] == lo) and np.all(ucon[s, keep] == hi)


def test_rect_one_period_and_zero_copies_equal_static():
    cs = case0(variant=True)
    x = synth.point(cs, 9, form="rect")
    y = synth.multipliers(O.dims(cs, form="rect")[1], 9)
    base = O.evaluate(cs, x, y, 0.5, form="rect")
    for opts in (dict(n_periods=1, ramp_ratio=0.2), dict(n_cont=0)):
        r = O.evaluate(cs, x, y, 0.5, form="rect", **opts)
        for key in ("c", "jval", "hval", "jrow", "jcol", "hrow", "hcol"):
            np.testing.assert_array_equal(r[key], base[key], err_msg=key)
