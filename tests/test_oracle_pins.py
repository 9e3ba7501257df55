"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

The paper prints no callback value, so every pin is mathematical:
* branch flows against the complex-power definition S = V conj(I) of the pi
  model (MATPOWER-style branch admittance matrix), an independent
  formulation in complex numpy arithmetic;
* balance rows against the bus-injection identity S = V conj(Ybus V) with a
  dense Ybus assembled from the branch matrices and the bus shunts;
* the Jacobian against central finite differences of the oracle's c(x), and
  the Hessian against central finite differences of the Lagrangian gradient
  sigma grad f + J^T y (a brute-force dense Hessian, which also proves that no
  nonzero lies outside the pattern);
* closed forms: lossless branches, flat start, the quadratic objective;
* special cases: one period equals the static model, zero copies equal the
  static model, period and copy indexing, outaged branches;
* pattern: closed-form counts, sorted, unique, lower triangle.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_12897_amd import synth

from helpers import case0, small_cases


# ----------------------------------------------------------------- helpers
def _block_views(cs, x, nrep=1, npg=1):
    N, L, G = cs["n_bus"], cs["n_branch"], cs["n_gen"]
    o = 0
    out = {}
    for name, size in (("va", N * nrep), ("vm", N * nrep), ("pg", G * npg), ("qg", G * nrep),
                       ("p", 2 * L * nrep), ("q", 2 * L * nrep)):
        out[name] = (o, size)
        o += size
    assert o == x.size
    return out


def _con_blocks(cs, nrep=1, T=1):
    N, L, G, R = cs["n_bus"], cs["n_branch"], cs["n_gen"], len(cs["ref_bus"])
    sizes = [("ref", R), ("pfr", L), ("qfr", L), ("pto", L), ("qto", L), ("ang", L),
             ("balp", N), ("balq", N), ("thf", L), ("tht", L)]
    o, out = 0, {}
    for name, s in sizes:
        out[name] = (o, s * nrep)
        o += s * nrep
    out["ramp"] = (o, G * (T - 1))
    return out


def _branch_matrices(cs):
    """MATPOWER-style 2x2 branch admittance blocks (Yff, Yft, Ytf, Ytt)."""
    ys = 1.0 / (cs["r"] + 1j * cs["x"])
    tap = cs["tap"] * np.exp(1j * cs["shift"])
    ytt = ys + 1j * cs["b"] / 2
    yff = ytt / (tap * np.conj(tap))
    yft = -ys / np.conj(tap)
    ytf = -ys / tap
    return yff, yft, ytf, ytt


def _complex_flows(cs, va, vm):
    V = vm * np.exp(1j * va)
    f, t = cs["f_bus"], cs["t_bus"]
    yff, yft, ytf, ytt = _branch_matrices(cs)
    If = yff * V[f] + yft * V[t]
    It = ytf * V[f] + ytt * V[t]
    return V[f] * np.conj(If), V[t] * np.conj(It)


def _zero_arc_vars(cs, x):
    bl = _block_views(cs, x)
    x = x.copy()
    for k in ("p", "q"):
        o, s = bl[k]
        x[o:o + s] = 0.0
    return x


# ----------------------------------------------------------------- physics
@pytest.mark.parametrize("name,cs", list(small_cases()))
def test_flows_match_complex_pi_model(name, cs):
    n, m = O.dims(cs)
    x = _zero_arc_vars(cs, synth.point(cs, 1))
    res = O.evaluate(cs, x, want=O.W_CONS)
    bl, cb = _block_views(cs, x), _con_blocks(cs)
    va = x[bl["va"][0]:bl["va"][0] + cs["n_bus"]]
    vm = x[bl["vm"][0]:bl["vm"][0] + cs["n_bus"]]
    Sf, St = _complex_flows(cs, va, vm)
    L = cs["n_branch"]
    c = res["c"]
    # c = p_arc - F(v); with p = q = 0 the rows hold -F
    for blk, ref in (("pfr", Sf.real), ("qfr", Sf.imag), ("pto", St.real), ("qto", St.imag)):
        o = cb[blk][0]
        np.testing.assert_allclose(-c[o:o + L], ref, rtol=1e-13, atol=1e-13, err_msg=blk)


@pytest.mark.parametrize("name,cs", list(small_cases()))
def test_balance_matches_ybus_injection(name, cs):
    """With p, q set to the branch flows, the balance rows equal the bus
    injections V conj(Ybus V) plus loads minus generation."""
    N, L = cs["n_bus"], cs["n_branch"]
    x = _zero_arc_vars(cs, synth.point(cs, 2))
    res0 = O.evaluate(cs, x, want=O.W_CONS)
    cb = _con_blocks(cs)
    bl = _block_views(cs, x)
    F = {blk: -res0["c"][cb[blk][0]:cb[blk][0] + L] for blk in ("pfr", "qfr", "pto", "qto")}
    op, oq = bl["p"][0], bl["q"][0]
    x[op:op + L], x[op + L:op + 2 * L] = F["pfr"], F["pto"]
    x[oq:oq + L], x[oq + L:oq + 2 * L] = F["qfr"], F["qto"]
    res = O.evaluate(cs, x, want=O.W_CONS)
    c = res["c"]
    # flow rows now vanish
    for blk in ("pfr", "qfr", "pto", "qto"):
        o = cb[blk][0]
        assert np.abs(c[o:o + L]).max() < 1e-12
    va = x[bl["va"][0]:bl["va"][0] + N]
    vm = x[bl["vm"][0]:bl["vm"][0] + N]
    V = vm * np.exp(1j * va)
    Y = np.zeros((N, N), complex)
    yff, yft, ytf, ytt = _branch_matrices(cs)
    f, t = cs["f_bus"], cs["t_bus"]
    np.add.at(Y, (f, f), yff)
    np.add.at(Y, (f, t), yft)
    np.add.at(Y, (t, f), ytf)
    np.add.at(Y, (t, t), ytt)
    Y[np.arange(N), np.arange(N)] += cs["gs"] + 1j * cs["bs"]
    Sinj = V * np.conj(Y @ V)
    G = cs["n_gen"]
    pg = x[bl["pg"][0]:bl["pg"][0] + G]
    qg = x[bl["qg"][0]:bl["qg"][0] + G]
    gen_p = np.zeros(N)
    gen_q = np.zeros(N)
    np.add.at(gen_p, cs["gen_bus"], pg)
    np.add.at(gen_q, cs["gen_bus"], qg)
    balp = c[cb["balp"][0]:cb["balp"][0] + N]
    balq = c[cb["balq"][0]:cb["balq"][0] + N]
    np.testing.assert_allclose(balp - cs["pd"] + gen_p, Sinj.real, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(balq - cs["qd"] + gen_q, Sinj.imag, rtol=1e-12, atol=1e-12)


def test_other_rows_closed_form():
    cs = case0(variant=True)
    x = synth.point(cs, 3)
    res = O.evaluate(cs, x, want=O.W_CONS)
    bl, cb = _block_views(cs, x), _con_blocks(cs)
    c = res["c"]
    N, L = cs["n_bus"], cs["n_branch"]
    va = x[:N]
    p = x[bl["p"][0]:bl["p"][0] + 2 * L]
    q = x[bl["q"][0]:bl["q"][0] + 2 * L]
    assert c[cb["ref"][0]] == va[cs["ref_bus"][0]]
    np.testing.assert_array_equal(c[cb["ang"][0]:cb["ang"][0] + L], va[cs["f_bus"]] - va[cs["t_bus"]])
    rate2 = cs["rate_a"] ** 2
    np.testing.assert_allclose(c[cb["thf"][0]:cb["thf"][0] + L], p[:L] ** 2 + q[:L] ** 2 - rate2, rtol=1e-15)
    np.testing.assert_allclose(c[cb["tht"][0]:cb["tht"][0] + L], p[L:] ** 2 + q[L:] ** 2 - rate2, rtol=1e-15)


def test_lossless_branch_invariants():
    """r = 0, b = 0, tap 1, shift 0: p_fr + p_to = 0 for every x, and the
    reactive loss q_fr + q_to equals |V_f - V_t|^2 / x."""
    cs = synth.network(12, 16, 3, 21)
    cs["r"][:] = 0.0
    cs["b"][:] = 0.0
    x = _zero_arc_vars(cs, synth.point(cs, 4))
    res = O.evaluate(cs, x, want=O.W_CONS)
    cb = _con_blocks(cs)
    L, N = cs["n_branch"], cs["n_bus"]
    c = res["c"]
    pf, qf = -c[cb["pfr"][0]:cb["pfr"][0] + L], -c[cb["qfr"][0]:cb["qfr"][0] + L]
    pt, qt = -c[cb["pto"][0]:cb["pto"][0] + L], -c[cb["qto"][0]:cb["qto"][0] + L]
    assert np.abs(pf + pt).max() <= 1e-14 * np.abs(pf).max()
    V = x[N:2 * N] * np.exp(1j * x[:N])
    loss = np.abs(V[cs["f_bus"]] - V[cs["t_bus"]]) ** 2 / cs["x"]
    np.testing.assert_allclose(qf + qt, loss, rtol=1e-10, atol=1e-13)


def test_flat_start_zero_load():
    """vm = 1, va = 0, no load, no shunt, no generation: every branch carries
    no active power, so the active balance is exactly zero; each arc carries
    -b/2 of reactive charging."""
    cs = synth.network(14, 20, 5, 0)
    cs["pd"][:] = 0.0
    cs["qd"][:] = 0.0
    n, m = O.dims(cs)
    x = np.zeros(n)
    bl, cb = _block_views(cs, x), _con_blocks(cs)
    N, L = cs["n_bus"], cs["n_branch"]
    x[N:2 * N] = 1.0
    oq = bl["q"][0]
    x[oq:oq + L] = -cs["b"] / 2
    x[oq + L:oq + 2 * L] = -cs["b"] / 2
    res = O.evaluate(cs, x, want=O.W_CONS)
    c = res["c"]
    assert np.all(c[cb["balp"][0]:cb["balp"][0] + N] == 0.0)
    for name in ("pfr", "pto"):
        assert np.all(c[cb[name][0]:cb[name][0] + L] == 0.0)
    for name in ("qfr", "qto"):
        o = cb[name][0]
        assert np.all(np.abs(c[o:o + L]) <= 4 * np.finfo(float).eps * res["cscale"][o:o + L])
    charge = np.zeros(N)
    np.add.at(charge, cs["f_bus"], -cs["b"] / 2)
    np.add.at(charge, cs["t_bus"], -cs["b"] / 2)
    np.testing.assert_allclose(c[cb["balq"][0]:cb["balq"][0] + N], charge, atol=1e-16)


# ----------------------------------------------------------------- objective
@pytest.mark.parametrize("name,cs", list(small_cases()))
def test_objective_quadratic(name, cs):
    x = synth.point(cs, 5)
    res = O.evaluate(cs, x, sigma=0.7)
    bl = _block_views(cs, x)
    o, G = bl["pg"][0], cs["n_gen"]
    pg = x[o:o + G]
    f = np.sum(cs["c2"] * pg ** 2 + cs["c1"] * pg + cs["c0"])
    assert abs(res["f"] - f) <= 1e-13 * res["fscale"]
    g = np.zeros_like(x)
    g[o:o + G] = 2 * cs["c2"] * pg + cs["c1"]
    np.testing.assert_allclose(res["g"], g, rtol=1e-14, atol=0)
    # f at pg = 0 is the constant term; f is exactly quadratic along pg
    x0 = x.copy()
    x0[o:o + G] = 0.0
    assert O.evaluate(cs, x0, want=O.W_OBJ)["f"] == pytest.approx(cs["c0"].sum(), rel=1e-15)
    # hess of the objective alone: sigma * 2 c2 on the pg diagonal only
    r0 = O.evaluate(cs, x, y=np.zeros(res["m"]), sigma=0.7, want=O.W_HESS)
    on_pg = (r0["hrow"] >= o) & (r0["hrow"] < o + G)
    assert np.all(r0["hval"][~on_pg] == 0.0)
    d = r0["hrow"][on_pg] == r0["hcol"][on_pg]
    assert d.all()
    np.testing.assert_allclose(r0["hval"][on_pg], 0.7 * 2 * cs["c2"], rtol=1e-15)


# ----------------------------------------------------------------- derivatives
def _fd_jacobian(cs, x, h=1e-6, **opts):
    n = x.size
    cols = []
    for j in range(n):
        xp, xm = x.copy(), x.copy()
        step = h * max(1.0, abs(x[j]))
        xp[j] += step
        xm[j] -= step
        cp = O.evaluate(cs, xp, want=O.W_CONS, **opts)["c"]
        cm = O.evaluate(cs, xm, want=O.W_CONS, **opts)["c"]
        cols.append((cp - cm) / (2 * step))
    return np.array(cols).T


def _lagrangian_gradient(cs, x, y, sigma, **opts):
    r = O.evaluate(cs, x, y, sigma, want=O.W_OBJ | O.W_JAC, **opts)
    Jd = O.dense_jacobian(r)
    return sigma * r["g"] + Jd.T @ y


def _fd_hessian(cs, x, y, sigma, h=1e-6, **opts):
    n = x.size
    H = np.zeros((n, n))
    for j in range(n):
        xp, xm = x.copy(), x.copy()
        step = h * max(1.0, abs(x[j]))
        xp[j] += step
        xm[j] -= step
        H[:, j] = (_lagrangian_gradient(cs, xp, y, sigma, **opts)
                   - _lagrangian_gradient(cs, xm, y, sigma, **opts)) / (2 * step)
    return H


DERIV_CASES = [
    ("c0v", dict()),
    ("mp3", dict(n_periods=3, ramp_ratio=0.2)),
    ("sc2", dict(n_cont=2)),
]


def _deriv_case(tag):
    if tag == "c0v":
        cs = case0(variant=True)
        return cs, {}
    if tag == "mp3":
        cs = synth.network(8, 11, 3, 41, variant=True)
        pd_t, qd_t = synth.mp_loads(cs, 3, 42)
        return cs, dict(n_periods=3, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2)
    cs = synth.network(8, 11, 3, 43, variant=True)
    return cs, dict(n_cont=2, outaged=synth.outages(cs, 2, 44))


@pytest.mark.parametrize("tag", ["c0v", "mp3", "sc2"])
def test_jacobian_matches_finite_differences(tag):
    cs, opts = _deriv_case(tag)
    n, m = O.dims(cs, **opts)
    x = synth.point(cs, 6, n_periods=opts.get("n_periods", 1), n_cont=opts.get("n_cont", 0))
    r = O.evaluate(cs, x, want=O.W_JAC, **opts)
    Jd = O.dense_jacobian(r)
    Jfd = _fd_jacobian(cs, x, **opts)
    scale = np.zeros((m, n))
    scale[r["jrow"], r["jcol"]] = r["jscale"]
    err = np.abs(Jd - Jfd)
    assert (err <= 2e-6 * (1.0 + scale)).all(), f"max err {err.max():.3e}"
    # coverage: every finite-difference nonzero lies in the pattern
    inpat = np.zeros((m, n), bool)
    inpat[r["jrow"], r["jcol"]] = True
    assert not (np.abs(Jfd) > 1e-6)[~inpat].any()
    # linear rows hold exact constants
    lin = np.isin(r["jval"], [-1.0, 1.0])
    assert lin.sum() >= m - 2 * cs["n_bus"] * (opts.get("n_periods", 1) + opts.get("n_cont", 0))


@pytest.mark.parametrize("tag", ["c0v", "mp3", "sc2"])
def test_hessian_matches_finite_differences(tag):
    """Brute-force dense Hessian of the Lagrangian by central differences of
    sigma grad f + J^T y; compared with the scattered lower triangle."""
    cs, opts = _deriv_case(tag)
    n, m = O.dims(cs, **opts)
    x = synth.point(cs, 7, n_periods=opts.get("n_periods", 1), n_cont=opts.get("n_cont", 0))
    y = synth.multipliers(m, 7)
    sigma = 0.8
    r = O.evaluate(cs, x, y, sigma, want=O.W_HESS, **opts)
    Hd = O.dense_hessian(r)
    Hfd = _fd_hessian(cs, x, y, sigma, **opts)
    assert np.abs(Hfd - Hfd.T).max() < 1e-5
    scale = np.zeros((n, n))
    scale[r["hrow"], r["hcol"]] = r["hscale"]
    scale = np.maximum(scale, scale.T)
    err = np.abs(Hd - Hfd)
    assert (err <= 2e-5 * (1.0 + scale)).all(), f"max err {err.max():.3e}"
    inpat = np.zeros((n, n), bool)
    inpat[r["hrow"], r["hcol"]] = True
    inpat |= inpat.T
    assert not (np.abs(Hfd) > 1e-5)[~inpat].any(), "nonzero outside the pattern"


def test_hessian_linear_in_multipliers():
    cs = case0(variant=True)
    n, m = O.dims(cs)
    x = synth.point(cs, 8)
    y1, y2 = synth.multipliers(m, 81), synth.multipliers(m, 82)
    a = O.evaluate(cs, x, y1, 0.3, want=O.W_HESS)
    b = O.evaluate(cs, x, y2, 1.1, want=O.W_HESS)
    ab = O.evaluate(cs, x, y1 + y2, 1.4, want=O.W_HESS)
    np.testing.assert_array_equal(a["hrow"], ab["hrow"])
    np.testing.assert_allclose(ab["hval"], a["hval"] + b["hval"], rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------- pattern
def _pattern_counts(N, L, G, R, T=1, K=0):
    if K:
        return (R + 30 * L + 2 * N + 2 * G) * (K + 1), G + (K + 1) * (3 * N + 8 * L)
    return T * (R + 30 * L + 2 * N + 2 * G) + 2 * G * (T - 1), T * (G + 3 * N + 8 * L)


@pytest.mark.parametrize("T,K", [(1, 0), (4, 0), (1, 3)])
def test_pattern_closed_form(T, K):
    cs = synth.network(40, 55, 9, 17)
    opts = dict(n_periods=T, ramp_ratio=0.2)
    if K:
        opts = dict(n_cont=K, outaged=synth.outages(cs, K, 18))
    n, m = O.dims(cs, **opts)
    N, L, G = 40, 55, 9
    nrep = T if T > 1 else K + 1
    assert n == nrep * (2 * N + G + 4 * L) + (1 if K else nrep) * G
    assert m == nrep * (1 + 7 * L + 2 * N) + G * (T - 1)
    x = synth.point(cs, 1, n_periods=T, n_cont=K)
    r = O.evaluate(cs, x, synth.multipliers(m, 1), 1.0, **opts)
    nnzj, nnzh = _pattern_counts(N, L, G, 1, T, K)
    assert r["jrow"].size == nnzj and r["hrow"].size == nnzh
    for rows, cols in ((r["jrow"], r["jcol"]), (r["hrow"], r["hcol"])):
        key = rows.astype(np.int64) * n + cols
        assert (np.diff(key) > 0).all(), "not sorted or not unique"
    assert (r["hrow"] >= r["hcol"]).all()
    assert r["jrow"].max() == m - 1 and r["jcol"].max() <= n - 1


def test_pattern_is_structural():
    """The pattern depends on topology only: zero cost curvature, zero shunts
    and an outaged branch keep their entries."""
    cs = synth.network(20, 28, 4, 19, variant=True)
    x = synth.point(cs, 2)
    n, m = O.dims(cs)
    a = O.evaluate(cs, x, synth.multipliers(m, 2))
    cs2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in cs.items()}
    cs2["c2"][:] = 0
    cs2["gs"][:] = 0
    cs2["bs"][:] = 0
    b = O.evaluate(cs2, x, synth.multipliers(m, 2))
    for k in ("jrow", "jcol", "hrow", "hcol"):
        np.testing.assert_array_equal(a[k], b[k])


# ----------------------------------------------------------------- bounds
def test_bounds_follow_listing():
    cs = case0()
    b = O.bounds(cs)
    x = np.zeros(O.dims(cs)[0])
    bl, cb = _block_views(cs, x), _con_blocks(cs)
    N, L, G = cs["n_bus"], cs["n_branch"], cs["n_gen"]
    assert np.all(np.isinf(b["lvar"][:N])) and np.all(b["x0"][N:2 * N] == 1.0)
    np.testing.assert_array_equal(b["lvar"][N:2 * N], cs["vmin"])
    o = bl["pg"][0]
    np.testing.assert_array_equal(b["uvar"][o:o + G], cs["pmax"])
    o = bl["p"][0]
    np.testing.assert_array_equal(b["uvar"][o:o + L], cs["rate_a"])
    np.testing.assert_array_equal(b["lvar"][o + L:o + 2 * L], -cs["rate_a"])
    eq = np.r_[cb["ref"][0]:cb["ang"][0], cb["balp"][0]:cb["thf"][0]]
    assert np.all(b["lcon"][eq] == 0) and np.all(b["ucon"][eq] == 0)
    th = np.r_[cb["thf"][0]:cb["tht"][0] + L]
    assert np.all(np.isneginf(b["lcon"][th])) and np.all(b["ucon"][th] == 0)
    o = cb["ang"][0]
    np.testing.assert_array_equal(b["lcon"][o:o + L], cs["angmin"])
    # ramp rows and the outaged copy's angle row
    opts = dict(n_periods=3, ramp_ratio=0.2)
    b3 = O.bounds(cs, **opts)
    np.testing.assert_allclose(b3["ucon"][-2 * G:], np.tile(0.2 * cs["pmax"], 2))
    out = np.array([cs["extra_branches"][0]], np.int32)
    bk = O.bounds(cs, n_cont=1, outaged=out)
    cbk = _con_blocks(cs, nrep=2)
    o = cbk["ang"][0] + L + out[0]
    assert np.isinf(bk["lcon"][o]) and np.isinf(bk["ucon"][o])
    assert bk["lcon"][cbk["ang"][0] + out[0]] == cs["angmin"][out[0]]


# ----------------------------------------------------------------- replication
def test_one_period_equals_static():
    cs = case0(variant=True)
    x = synth.point(cs, 9)
    n, m = O.dims(cs)
    y = synth.multipliers(m, 9)
    a = O.evaluate(cs, x, y, 0.9)
    b = O.evaluate(cs, x, y, 0.9, n_periods=1, ramp_ratio=0.2)
    c = O.evaluate(cs, x, y, 0.9, n_cont=0)
    for k in ("g", "c", "jrow", "jcol", "jval", "hrow", "hcol", "hval"):
        np.testing.assert_array_equal(a[k], b[k])
        np.testing.assert_array_equal(a[k], c[k])


def _replicate(cs, x, nrep, shared_pg):
    bl = _block_views(cs, x)
    parts = []
    for k in ("va", "vm", "pg", "qg", "p", "q"):
        o, s = bl[k]
        parts.append(x[o:o + s] if (k == "pg" and shared_pg) else np.tile(x[o:o + s], nrep))
    return np.concatenate(parts)


def test_periods_index_entity_fastest():
    """Identical periods reproduce the static rows per period; the balance
    rows of period t see the loads of period t; ramp rows vanish."""
    cs = case0(variant=True)
    T = 4
    x = synth.point(cs, 10)
    n, m = O.dims(cs)
    base = O.evaluate(cs, x, want=O.W_CONS | O.W_JAC)
    xt = _replicate(cs, x, T, False)
    pd_t = np.tile(cs["pd"], T)
    qd_t = np.tile(cs["qd"], T)
    dp = np.arange(T * cs["n_bus"]) * 1e-3
    mp = O.evaluate(cs, xt, n_periods=T, pd_t=pd_t + dp, qd_t=qd_t, ramp_ratio=0.2,
                    want=O.W_CONS | O.W_JAC)
    cbt = _con_blocks(cs, nrep=T, T=T)
    cb = _con_blocks(cs)
    N = cs["n_bus"]
    for name, (o, s) in cb.items():
        if s == 0:
            continue
        got = mp["c"][cbt[name][0]:cbt[name][0] + T * s].reshape(T, s)
        want = np.tile(base["c"][o:o + s], (T, 1))
        if name == "balp":
            want = want + dp.reshape(T, N)
        np.testing.assert_allclose(got, want, rtol=1e-15, atol=1e-15, err_msg=name)
    ro, rs = cbt["ramp"]
    assert rs == cs["n_gen"] * (T - 1) and np.all(mp["c"][ro:] == 0.0)


def test_contingency_copies():
    """Copies share pg: the objective counts it once; copy s has its outaged
    branch carrying no flow (rows equal the arc variables)."""
    cs = case0(variant=True)
    K = 2
    out = synth.outages(cs, K, 3)
    x = synth.point(cs, 11)
    base = O.evaluate(cs, x, want=O.W_CONS | O.W_OBJ)
    xk = _replicate(cs, x, K + 1, True)
    sc = O.evaluate(cs, xk, n_cont=K, outaged=out, want=O.W_CONS | O.W_OBJ)
    assert sc["f"] == base["f"]
    L = cs["n_branch"]
    cbk = _con_blocks(cs, nrep=K + 1)
    cb = _con_blocks(cs)
    bl = _block_views(cs, x)
    p = x[bl["p"][0]:bl["p"][0] + 2 * L]
    q = x[bl["q"][0]:bl["q"][0] + 2 * L]
    for name in ("pfr", "qfr", "pto", "qto"):
        got = sc["c"][cbk[name][0]:cbk[name][0] + (K + 1) * L].reshape(K + 1, L)
        want = np.tile(base["c"][cb[name][0]:cb[name][0] + L], (K + 1, 1))
        arcvar = {"pfr": p[:L], "qfr": q[:L], "pto": p[L:], "qto": q[L:]}[name]
        for s in range(1, K + 1):
            want[s, out[s - 1]] = arcvar[out[s - 1]]
        np.testing.assert_allclose(got, want, rtol=1e-15, atol=1e-15, err_msg=name)
    for name in ("ref", "ang", "balp", "balq", "thf", "tht"):
        o, s = cb[name]
        got = sc["c"][cbk[name][0]:cbk[name][0] + (K + 1) * s].reshape(K + 1, s)
        np.testing.assert_array_equal(got, np.tile(base["c"][o:o + s], (K + 1, 1)), err_msg=name)


def test_bus_relabelling_permutes_results():
    """Metamorphic: renumbering buses permutes the per-bus rows and columns."""
    cs = synth.network(10, 14, 3, 23, variant=True)
    N = cs["n_bus"]
    perm = np.random.default_rng(0).permutation(N)  # new label of old bus i
    cs2 = dict(cs)
    for k in ("pd", "qd", "gs", "bs", "vmin", "vmax"):
        a = np.empty_like(cs[k])
        a[perm] = cs[k]
        cs2[k] = a
    for k in ("f_bus", "t_bus", "gen_bus", "ref_bus"):
        cs2[k] = perm[cs[k]].astype(np.int32)
    x = synth.point(cs, 12)
    x2 = x.copy()
    x2[perm] = x[:N]
    x2[N + perm] = x[N:2 * N]
    a = O.evaluate(cs, x, want=O.W_CONS | O.W_OBJ)
    b = O.evaluate(cs2, x2, want=O.W_CONS | O.W_OBJ)
    assert a["f"] == b["f"]
    cb = _con_blocks(cs)
    for name in ("balp", "balq"):
        o = cb[name][0]
        got = b["c"][o:o + N][perm]
        np.testing.assert_allclose(got, a["c"][o:o + N], rtol=1e-14, atol=1e-15)
    o = cb["pfr"][0]
    np.testing.assert_array_equal(a["c"][o:cb["balp"][0]], b["c"][o:cb["balp"][0]])
