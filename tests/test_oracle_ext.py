"""Pins of the oracle's storage units and user-extension devices.

Storage follows the model of Geth, Coffrin and Fobes (2020) that the paper
cites for its multi-period formulation with storage (Sec. III-C3); devices
are linear components in the shape of the paper's electrolyzer example
(Sec. III-D, Listing 10).  Every pin is mathematical (the paper prints no
values):
* each storage and device row against an independent numpy evaluation of
  its definition (losses through the complex converter current
  I = conj(S / V), so r |I|^2 is formed without the oracle's expression);
* the state-of-charge chain telescopes: with unit efficiencies the sum of
  a unit's rows over the periods is se_{T-1} - e0 - dt sum (sc - sd);
* the balance rows gain exactly the storage draws and device terms;
* zero units and zero devices reproduce the base model bit for bit;
* the Jacobian against central differences, the Hessian against a
  brute-force dense Hessian (central differences of sigma grad f + J^T y),
  which also proves pattern coverage; closed-form pattern counts; bounds.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_12897_amd import synth

from test_oracle_pins import _fd_hessian, _fd_jacobian


def _ext_case(T=3, comp=True, form="polar", stor=True, dev=True, seed=41):
    cs = synth.network(8, 11, 3, seed, variant=True)
    opts = dict(form=form)
    if T > 1:
        pd_t, qd_t = synth.mp_loads(cs, T, seed + 1)
        opts.update(n_periods=T, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2)
    if stor:
        opts.update(storage=synth.storage(cs, seed + 2, frac=0.25), stor_dt=0.5, stor_comp=comp)
    if dev:
        opts.update(devices=synth.devices(cs, 3, seed + 3))
    return cs, opts


def _point(cs, opts, seed):
    return synth.point(cs, seed, n_periods=opts.get("n_periods", 1), form=opts.get("form", "polar"),
                       storage=opts.get("storage"), devices=opts.get("devices"))


def _layout(cs, opts):
    """Offsets of the variable and row blocks (the documented order)."""
    N, L, G, R = cs["n_bus"], cs["n_branch"], cs["n_gen"], len(cs["ref_bus"])
    T = opts.get("n_periods", 1)
    S = len(opts["storage"]["bus"]) if "storage" in opts else 0
    D = len(opts["devices"]["bus"]) if "devices" in opts else 0
    rect = opts.get("form") == "rect"
    xb, o = {}, 0
    for name, size in (("va", N * T), ("vm", N * T), ("pg", G * T), ("qg", G * T), ("p", 2 * L * T),
                       ("q", 2 * L * T), ("ps", S * T), ("qs", S * T), ("qsc", S * T), ("se", S * T),
                       ("sc", S * T), ("sd", S * T), ("u", D * T)):
        xb[name] = (o, size)
        o += size
    cb, o = {}, 0
    for name, size in (("ref", R * T), ("pfr", L * T), ("qfr", L * T), ("pto", L * T), ("qto", L * T),
                       ("ang", L * T), ("angl", L * T if rect else 0), ("balp", N * T), ("balq", N * T),
                       ("thf", L * T), ("tht", L * T), ("vmag", N * T if rect else 0), ("ramp", G * (T - 1)),
                       ("soc", S * T), ("slp", S * T), ("slq", S * T), ("sth", S * T),
                       ("scmp", S * T if opts.get("stor_comp") else 0), ("dramp", D * (T - 1)), ("dinit", D)):
        cb[name] = (o, size)
        o += size
    return xb, cb, o


def _blk(a, b, name):
    o, s = b[name]
    return a[o:o + s]


def test_layout_sizes():
    for kw in (dict(), dict(comp=False), dict(T=1), dict(form="rect", stor=False), dict(stor=False),
               dict(dev=False)):
        cs, opts = _ext_case(**kw)
        xb, cb, m = _layout(cs, opts)
        n = sum(s for _, s in xb.values())
        assert O.dims(cs, **opts) == (n, m), kw


def test_storage_rows_match_independent_evaluation():
    cs, opts = _ext_case()
    st, T, N = opts["storage"], opts["n_periods"], cs["n_bus"]
    S = len(st["bus"])
    x = _point(cs, opts, 3)
    res = O.evaluate(cs, x, want=O.W_CONS, **opts)
    xb, cb, _ = _layout(cs, opts)
    c = res["c"]
    V = lambda k: _blk(x, xb, k).reshape(T, -1)  # noqa: E731  [period, entity]
    ps, qs, qsc, se, sc, sd = (V(k) for k in ("ps", "qs", "qsc", "se", "sc", "sd"))
    va, vm = V("va"), V("vm")
    Vb = (vm * np.exp(1j * va))[:, st["bus"]]
    I = np.conj((ps + 1j * qs) / Vb)  # converter current
    i2 = np.abs(I) ** 2
    prev = np.vstack([st["e0"][None, :], se[:-1]])
    soc = se - prev - 0.5 * (st["eta_c"] * sc - sd / st["eta_d"])
    slp = ps + sd - sc - st["ploss"] - st["r"] * i2
    slq = qs - qsc - st["qloss"] - st["x"] * i2
    sth = ps ** 2 + qs ** 2 - st["rating"] ** 2
    for name, ref in (("soc", soc), ("slp", slp), ("slq", slq), ("sth", sth), ("scmp", sc * sd)):
        got = _blk(c, cb, name).reshape(T, S)
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14, err_msg=name)


def test_soc_chain_telescopes():
    """Unit efficiencies: summed over the periods the state-of-charge rows
    of a unit leave se_{T-1} - e0 - dt sum_t (sc_t - sd_t)."""
    cs, opts = _ext_case(T=5)
    st = dict(opts["storage"])
    st["eta_c"] = np.ones_like(st["eta_c"])
    st["eta_d"] = np.ones_like(st["eta_d"])
    opts["storage"] = st
    x = _point(cs, opts, 4)
    res = O.evaluate(cs, x, want=O.W_CONS, **opts)
    xb, cb, _ = _layout(cs, opts)
    S = len(st["bus"])
    soc = _blk(res["c"], cb, "soc").reshape(5, S).sum(0)
    se, sc, sd = (_blk(x, xb, k).reshape(5, S) for k in ("se", "sc", "sd"))
    np.testing.assert_allclose(soc, se[-1] - st["e0"] - 0.5 * (sc - sd).sum(0), rtol=1e-12, atol=1e-13)


def test_balance_gains_storage_and_device_terms():
    cs, opts = _ext_case()
    T, N = opts["n_periods"], cs["n_bus"]
    x = _point(cs, opts, 5)
    base_opts = {k: v for k, v in opts.items() if k not in ("storage", "stor_dt", "stor_comp", "devices")}
    xb, cb, _ = _layout(cs, opts)
    nb = O.dims(cs, **base_opts)[0]
    r_ext = O.evaluate(cs, x, want=O.W_CONS, **opts)
    r_base = O.evaluate(cs, x[:nb], want=O.W_CONS, **base_opts)
    xb0, cb0, _ = _layout(cs, base_opts)
    st, dv = opts["storage"], opts["devices"]
    ps, qs, u = (_blk(x, xb, k).reshape(T, -1) for k in ("ps", "qs", "u"))
    for row, draw, coef in (("balp", ps, dv["cp"]), ("balq", qs, dv["cq"])):
        add = np.zeros((T, N))
        for t in range(T):
            np.add.at(add[t], st["bus"], draw[t])
            np.add.at(add[t], dv["bus"], coef * u[t])
        got = _blk(r_ext["c"], cb, row).reshape(T, N) - _blk(r_base["c"], cb0, row).reshape(T, N)
        np.testing.assert_allclose(got, add, rtol=1e-12, atol=1e-14, err_msg=row)
    # device rows and objective
    ramp = _blk(r_ext["c"], cb, "dramp").reshape(T - 1, -1)
    np.testing.assert_array_equal(ramp, u[1:] - u[:-1])
    np.testing.assert_array_equal(_blk(r_ext["c"], cb, "dinit"), u[0])
    rf_e = O.evaluate(cs, x, want=O.W_OBJ, **opts)
    rf_b = O.evaluate(cs, x[:nb], want=O.W_OBJ, **base_opts)
    np.testing.assert_allclose(rf_e["f"] - rf_b["f"], (dv["cost"][None, :] * u).sum(), rtol=1e-12)
    np.testing.assert_array_equal(_blk(rf_e["g"], xb, "u"), np.tile(dv["cost"], T))


def test_no_units_no_devices_is_the_base_model():
    cs, opts = _ext_case()
    base = {k: v for k, v in opts.items() if k not in ("storage", "stor_dt", "stor_comp", "devices")}
    empty_st = {k: v[:0] for k, v in opts["storage"].items()}
    empty_dv = {k: v[:0] for k, v in opts["devices"].items()}
    x = _point(cs, base, 6)
    m = O.dims(cs, **base)[1]
    y = synth.multipliers(m, 6)
    a = O.evaluate(cs, x, y, 0.7, **base)
    b = O.evaluate(cs, x, y, 0.7, storage=empty_st, devices=empty_dv, stor_comp=True, **base)
    for k in ("c", "g", "jrow", "jcol", "jval", "hrow", "hcol", "hval"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    assert a["f"] == b["f"]


@pytest.mark.parametrize("kw", [dict(), dict(comp=False), dict(T=1), dict(form="rect", stor=False)],
                         ids=["mp3_comp", "mp3", "static", "rect_devices"])
def test_ext_jacobian_matches_finite_differences(kw):
    cs, opts = _ext_case(**kw)
    n, m = O.dims(cs, **opts)
    x = _point(cs, opts, 7)
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


@pytest.mark.parametrize("kw", [dict(), dict(T=1), dict(form="rect", stor=False)],
                         ids=["mp3_comp", "static", "rect_devices"])
def test_ext_hessian_matches_finite_differences(kw):
    cs, opts = _ext_case(**kw)
    n, m = O.dims(cs, **opts)
    x = _point(cs, opts, 8)
    y = synth.multipliers(m, 8)
    r = O.evaluate(cs, x, y, 0.6, want=O.W_HESS, **opts)
    Hd = O.dense_hessian(r)
    Hfd = _fd_hessian(cs, x, y, 0.6, **opts)
    scale = np.zeros((n, n))
    scale[r["hrow"], r["hcol"]] = r["hscale"]
    scale = np.maximum(scale, scale.T)
    err = np.abs(Hd - Hfd)
    assert (err <= 2e-5 * (1.0 + scale)).all(), f"max err {err.max():.3e}"
    inpat = np.zeros((n, n), bool)
    inpat[r["hrow"], r["hcol"]] = True
    inpat |= inpat.T
    assert not (np.abs(Hfd) > 1e-5)[~inpat].any(), "nonzero outside the pattern"


def test_ext_pattern_closed_form():
    """Added to the base counts per period: storage J 4 (soc; 3 at t = 0)
    + 5 + 4 + 2 (+ 2 complementarity) per unit and 1 in each balance row;
    H 5 per unit ((ps, ps), (qs, qs), (ps, vm), (qs, vm), (sd, sc); the
    (vm, vm) term merges into the bus diagonal); devices J 1 in each balance
    row (structural, zero coefficients included), 2 per ramp row, 1 per
    initial row."""
    cs, opts = _ext_case(T=4)
    T, S, D = 4, len(opts["storage"]["bus"]), len(opts["devices"]["bus"])
    base = {k: v for k, v in opts.items() if k not in ("storage", "stor_dt", "stor_comp", "devices")}
    x = _point(cs, opts, 9)
    m = O.dims(cs, **opts)[1]
    r = O.evaluate(cs, x, synth.multipliers(m, 9), 1.0, **opts)
    r0 = O.evaluate(cs, x[:O.dims(cs, **base)[0]], synth.multipliers(O.dims(cs, **base)[1], 9), 1.0, **base)
    dj = T * S * (4 + 5 + 4 + 2 + 2 + 2) - S + T * 2 * D + 2 * D * (T - 1) + D
    assert r["jrow"].size - r0["jrow"].size == dj
    # H: per unit and period (ps,ps) (qs,qs) (ps,vm) (qs,vm) (sd,sc); (vm,vm) merges with the bus diagonal
    assert r["hrow"].size - r0["hrow"].size == T * S * 5
    for rows, cols in ((r["jrow"], r["jcol"]), (r["hrow"], r["hcol"])):
        key = rows.astype(np.int64) * x.size + cols
        assert (np.diff(key) > 0).all()
    assert (r["hrow"] >= r["hcol"]).all()


def test_ext_bounds():
    cs, opts = _ext_case()
    b = O.bounds(cs, **opts)
    xb, cb, _ = _layout(cs, opts)
    st, dv, T = opts["storage"], opts["devices"], opts["n_periods"]
    for k, lo, hi in (("ps", -st["rating"], st["rating"]), ("qs", st["qmin"], st["qmax"]),
                      ("qsc", -st["rating"], st["rating"]), ("se", 0 * st["emax"], st["emax"]),
                      ("sc", 0 * st["chmax"], st["chmax"]), ("sd", 0 * st["dismax"], st["dismax"]),
                      ("u", dv["lo"], dv["hi"])):
        np.testing.assert_array_equal(_blk(b["lvar"], xb, k), np.tile(lo, T), err_msg=k)
        np.testing.assert_array_equal(_blk(b["uvar"], xb, k), np.tile(hi, T), err_msg=k)
    for k in ("soc", "slp", "slq"):
        assert not _blk(b["lcon"], cb, k).any() and not _blk(b["ucon"], cb, k).any()
    for k in ("sth", "scmp"):
        assert np.all(_blk(b["lcon"], cb, k) == -np.inf) and not _blk(b["ucon"], cb, k).any()
    np.testing.assert_array_equal(_blk(b["ucon"], cb, "dramp"), np.tile(dv["ramp"], T - 1))
    np.testing.assert_array_equal(_blk(b["lcon"], cb, "dinit"), dv["init_lo"])
    np.testing.assert_array_equal(_blk(b["ucon"], cb, "dinit"), dv["init_hi"])


def test_storage_rejected_where_undefined():
    cs, opts = _ext_case()
    with pytest.raises(O.OracleError):
        O.dims(cs, **dict(opts, form="rect"))
    sc = {k: v for k, v in opts.items() if k not in ("n_periods", "pd_t", "qd_t", "ramp_ratio")}
    with pytest.raises(O.OracleError):
        O.dims(cs, n_cont=1, outaged=np.array([0], np.int32), **sc)
