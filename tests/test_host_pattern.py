"""Host-side logic of libopf, checked on the CPU (no GPU needed):
the library loads and exports every declared entry point, the host-built
sparsity patterns equal the oracle's bit for bit, sizes and bounds agree, and
validation rejects malformed cases with the documented codes."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_12897_amd import opf, synth

from helpers import hub_network, small_cases


def test_library_exports_every_declared_symbol():
    L = opf.lib()
    names = opf.declared_symbols()
    assert len(names) >= 28
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"


def with_parallel_and_isolated(cs):
    """Copy of a case with two parallel branches and one isolated bus."""
    c = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in cs.items()}
    L = c["n_branch"]
    dup = [0, 3]
    for k in ("f_bus", "t_bus", "r", "x", "b", "tap", "shift", "rate_a", "angmin", "angmax"):
        extra = c[k][dup].copy()
        if k == "x":
            extra = extra * 1.7
        if k == "f_bus":  # second copy reversed: exercises mixed orientation
            extra[1] = c["t_bus"][dup[1]]
        if k == "t_bus":
            extra[1] = c["f_bus"][dup[1]]
        c[k] = np.concatenate([c[k], extra])
    c["n_branch"] = L + 2
    for k, val in (("pd", 0.1), ("qd", 0.03), ("gs", 0.01), ("bs", 0.02), ("vmin", 0.9), ("vmax", 1.1)):
        c[k] = np.append(c[k], val)
    c["n_bus"] += 1
    return c


def _cases():
    for name, cs in small_cases():
        yield name, cs, {}
    cs = synth.network(30, 44, 12, 3, variant=True)
    yield "mp4", cs, dict(n_periods=4, pd_t=synth.mp_loads(cs, 4, 1)[0], qd_t=synth.mp_loads(cs, 4, 1)[1],
                          ramp_ratio=0.2)
    yield "mp2_noloads", cs, dict(n_periods=2, ramp_ratio=0.25)
    yield "sc3", cs, dict(n_cont=3, outaged=synth.outages(cs, 3, 2))
    yield "parallel_isolated", with_parallel_and_isolated(synth.network(12, 16, 4, 8, variant=True)), {}
    pc = with_parallel_and_isolated(synth.network(12, 16, 4, 9))
    yield "parallel_sc", pc, dict(n_cont=2, outaged=np.array([0, pc["n_branch"] - 1], np.int32))
    hub = hub_network()
    yield "hub", hub, {}
    yield "hub_sc2", hub, dict(n_cont=2, outaged=hub["extra_branches"][:2])


def _rect(cases):
    """The rectangular form of every case."""
    for name, cs, opts in cases:
        yield name + "_rect", cs, dict(opts, form="rect")


def _ext_cases():
    """Storage units and devices (multi-period and static), devices in the
    rectangular form, and a hub bus whose segment overflows a wave only
    because of its units and devices."""
    cs = synth.network(30, 44, 12, 3, variant=True)
    pd_t, qd_t = synth.mp_loads(cs, 4, 1)
    st, dv = synth.storage(cs, 7, frac=0.2), synth.devices(cs, 9, 8)
    yield "stor_dev_mp4", cs, dict(n_periods=4, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2, storage=st, stor_dt=0.5,
                                   stor_comp=True, devices=dv)
    yield "stor_static", cs, dict(storage=st, stor_dt=1.0)
    yield "dev_rect_mp2", cs, dict(n_periods=2, ramp_ratio=0.2, devices=dv, form="rect")
    hub = hub_network()
    hst = synth.storage(hub, 3, frac=0.05)
    hst["bus"] = np.sort(np.r_[hst["bus"][:-2], [200, 200]]).astype(np.int32)  # two units at the 63-lane hub
    hdv = synth.devices(hub, 6, 4)
    hdv["bus"][:3] = 100  # three devices at the 64-lane hub
    yield "hub_stor_dev_mp2", hub, dict(n_periods=2, ramp_ratio=0.2, storage=hst, stor_dt=0.5, devices=hdv)


CASES = list(_cases())
CASES += list(_rect(CASES))
CASES += list(_ext_cases())


@pytest.mark.parametrize("name,cs,opts", CASES, ids=[c[0] for c in CASES])
def test_host_pattern_matches_oracle_bit_exact(name, cs, opts):
    n, m, nnzj, nnzh = opf.case_dims(cs, **opts)
    assert (n, m) == O.dims(cs, **opts)
    T, K = opts.get("n_periods", 1), opts.get("n_cont", 0)
    x = synth.point(cs, 3, n_periods=T, n_cont=K, form=opts.get("form", "polar"), storage=opts.get("storage"),
                    devices=opts.get("devices"))
    res = O.evaluate(cs, x, synth.multipliers(m, 3), 1.0, want=O.W_JAC | O.W_HESS, **opts)
    jr, jc, hr, hc = opf.case_structure(cs, **opts)
    assert jr.dtype == np.int32 and hr.dtype == np.int32
    np.testing.assert_array_equal(jr, res["jrow"])
    np.testing.assert_array_equal(jc, res["jcol"])
    np.testing.assert_array_equal(hr, res["hrow"])
    np.testing.assert_array_equal(hc, res["hcol"])
    assert nnzj == res["jrow"].size and nnzh == res["hrow"].size


@pytest.mark.parametrize("name,cs,opts", CASES, ids=[c[0] for c in CASES])
def test_host_bounds_match_oracle(name, cs, opts):
    a = opf.case_bounds(cs, **opts)
    b = O.bounds(cs, **opts)
    for k in ("lvar", "uvar", "lcon", "ucon", "x0"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_closed_form_sizes_full_configs():
    """Sizes of the benchmark configurations (simple graphs)."""
    cs = synth.network(10000, 13500, 2000, 1)
    assert opf.case_dims(cs) == (78000, 114501, 429001, 140000)
    cs = synth.network(2000, 2700, 400, 2)
    pd_t, qd_t = synth.mp_loads(cs, 48, 202)
    assert opf.case_dims(cs, n_periods=48, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2) == \
        (748800, 1118048, 4156048, 1344000)
    cs = synth.network(1000, 1350, 200, 31)
    out = synth.outages(cs, 200, 32)
    assert opf.case_dims(cs, n_cont=200, outaged=out) == (1527800, 2301651, 8623101, 2774000)


def test_closed_form_sizes_rect():
    """Rectangular form (simple graph, every bus on a branch): n as polar,
    m = R + 8L + 3N, nnzJ = R + 36L + 6N + 2G, nnzH = G + 2N + 8L."""
    cs = synth.network(10000, 13500, 2000, 1)
    assert opf.case_dims(cs, form="rect") == (78000, 1 + 8 * 13500 + 3 * 10000,
                                              1 + 36 * 13500 + 6 * 10000 + 2 * 2000, 2000 + 2 * 10000 + 8 * 13500)
    _err(cs, opf.OPF_E_ARG, form="cartesian")


def test_form_out_of_range_rejected():
    cs = synth.network(5, 6, 2, 1)
    c, o, keep = opf._case_struct(cs)
    o.form = 7
    assert opf.lib().opf_case_validate(ctypes.byref(c), ctypes.byref(o)) == opf.OPF_E_CASE
    assert b"form" in opf.lib().opf_last_error()


def _err(cs, code, **opts):
    with pytest.raises(opf.OPFError) as e:
        opf.case_validate(cs, **opts)
    assert e.value.code == code, str(e.value)
    return str(e.value)


def test_validation_errors():
    base = synth.network(10, 14, 3, 5)

    def mod(**kw):
        c = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in base.items()}
        for k, v in kw.items():
            c[k] = v(c) if callable(v) else v
        return c

    opf.case_validate(base)
    assert "out of range" in _err(mod(f_bus=lambda c: np.r_[99, c["f_bus"][1:]].astype(np.int32)), opf.OPF_E_CASE)
    assert "itself" in _err(mod(t_bus=lambda c: np.r_[c["f_bus"][0], c["t_bus"][1:]].astype(np.int32)),
                            opf.OPF_E_CASE)
    z = mod(r=lambda c: np.r_[0.0, c["r"][1:]], x=lambda c: np.r_[0.0, c["x"][1:]])
    assert "impedance" in _err(z, opf.OPF_E_CASE)
    assert "tap" in _err(mod(tap=lambda c: np.r_[0.0, c["tap"][1:]]), opf.OPF_E_CASE)
    assert "reference" in _err(mod(ref_bus=np.array([10], np.int32)), opf.OPF_E_CASE)
    assert "reference bus is required" in _err(mod(ref_bus=np.zeros(0, np.int32)), opf.OPF_E_CASE)
    assert "pmin > pmax" in _err(mod(pmin=lambda c: c["pmax"] + 1), opf.OPF_E_CASE)
    assert "vmin > vmax" in _err(mod(vmin=lambda c: c["vmax"] + 1), opf.OPF_E_CASE)
    assert "generator" in _err(mod(gen_bus=lambda c: np.r_[-1, c["gen_bus"][1:]].astype(np.int32)),
                               opf.OPF_E_CASE)
    _err(base, opf.OPF_E_CASE, n_periods=0)
    _err(base, opf.OPF_E_CASE, n_periods=3, n_cont=1, outaged=np.array([0], np.int32))
    assert "outages" in _err(base, opf.OPF_E_CASE, n_cont=1, outaged=np.array([14], np.int32))
    _err(base, opf.OPF_E_ARG, n_cont=1)  # no outage list
    _err(base, opf.OPF_E_ARG, n_periods=2, pd_t=np.ones(20))  # pd_t without qd_t
    _err(base, opf.OPF_E_CASE, n_periods=2, ramp_ratio=-1.0)


def test_degree_limit():
    N = 1030
    cs = synth.network(N, N - 1, 2, 6)
    # a star: every branch touches bus 0
    cs["f_bus"] = np.zeros(N - 1, np.int32)
    cs["t_bus"] = np.arange(1, N, dtype=np.int32)
    assert "1024" in _err(cs, opf.OPF_E_CASE)


def test_null_arrays_rejected():
    cs = synth.network(5, 6, 2, 1)
    c, o, keep = opf._case_struct(cs)
    c.pd = ctypes.POINTER(ctypes.c_double)()
    rc = opf.lib().opf_case_validate(ctypes.byref(c), ctypes.byref(o))
    assert rc == opf.OPF_E_ARG
    assert opf.lib().opf_case_validate(None, None) == opf.OPF_E_ARG


def test_handles_rejected_after_misuse():
    """Calls on a NULL or foreign handle fail with OPF_E_STATE, no GPU needed."""
    L = opf.lib()
    assert L.opf_model_destroy(None) == opf.OPF_OK
    junk = (ctypes.c_uint64 * 64)()
    assert L.opf_cons(ctypes.cast(junk, ctypes.c_void_p), None, None, None) == opf.OPF_E_STATE
    assert L.opf_batch_eval(ctypes.cast(junk, ctypes.c_void_p), *([None] * 9)) == opf.OPF_E_STATE
    assert b"invalid" in L.opf_last_error()
