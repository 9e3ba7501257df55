"""GPU parity: every callback of libopf against the CPU oracle.

Patterns bit-exact; values within the scale-aware tolerance
|v - v*| <= 1e-12 max(|v*|, S) + 1e-14 (S = the oracle's sum of |terms|);
linear rows (constants) bit-exact; separate callbacks, the fused set and
repeated runs bitwise equal to each other.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_12897_amd import opf, synth

from helpers import assert_close, hub_network, record_strict, small_cases, strict_violations
from test_host_pattern import with_parallel_and_isolated

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    for name, cs in small_cases():
        yield name, cs, {}
    cs = synth.network(30, 44, 12, 3, variant=True)
    pd_t, qd_t = synth.mp_loads(cs, 4, 1)
    yield "mp4", cs, dict(n_periods=4, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2)
    yield "mp2_noloads", cs, dict(n_periods=2, ramp_ratio=0.25)
    yield "sc3", cs, dict(n_cont=3, outaged=synth.outages(cs, 3, 2))
    yield "parallel_isolated", with_parallel_and_isolated(synth.network(12, 16, 4, 8, variant=True)), {}
    pc = with_parallel_and_isolated(synth.network(12, 16, 4, 9))
    yield "parallel_sc", pc, dict(n_cont=2, outaged=np.array([0, pc["n_branch"] - 1], np.int32))
    # buses whose segments are 63, 64, 65 and 124 lanes: both sides of the
    # one-wave limit and the workgroup-wide reduction, with replicas too
    hub = hub_network()
    yield "hub", hub, {}
    pd_t, qd_t = synth.mp_loads(hub, 2, 5)
    yield "hub_mp2", hub, dict(n_periods=2, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2)
    yield "hub_sc2", hub, dict(n_cont=2, outaged=hub["extra_branches"][:2])
    # several tiles and a ragged tail: 700 buses -> half-edges span many 256-wide tiles
    yield "ragged700", synth.network(700, 951, 140, 12, variant=True), {}


CASES = list(_cases())

# launch shapes: small models evaluate a set in one launch (bus items
# recompute the branch terms they need); limit 0 forces the two-launch
# shape (branch items leave records) on every model
SHAPES = {"single": 4096, "two": 0}


@pytest.fixture(params=list(SHAPES))
def shape(request):
    opf.set_single_launch_limit(SHAPES[request.param])
    yield request.param
    opf.set_single_launch_limit(4096)


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def check_against_oracle(model, cs, opts, x, y, sigma, tag):
    say(f"[parity] {tag}: n={model.n} m={model.m} nnzj={model.nnzj} nnzh={model.nnzh}")
    res = O.evaluate(cs, x, y, sigma, **opts)
    f, g, c, jv, hv = model.eval_set(to_dev(x), to_dev(y), sigma)
    jr, jc = model.jac_structure()
    hr, hc = model.hess_structure()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(jr.cpu().numpy(), res["jrow"])
    np.testing.assert_array_equal(jc.cpu().numpy(), res["jcol"])
    np.testing.assert_array_equal(hr.cpu().numpy(), res["hrow"])
    np.testing.assert_array_equal(hc.cpu().numpy(), res["hcol"])
    assert_close([f.item()], [res["f"]], [res["fscale"]], what=f"{tag} f")
    assert_close(g.cpu().numpy(), res["g"], np.abs(res["g"]), what=f"{tag} grad")
    assert_close(c.cpu().numpy(), res["c"], res["cscale"], what=f"{tag} c")
    jvh = jv.cpu().numpy()
    assert_close(jvh, res["jval"], res["jscale"], what=f"{tag} J")
    lin = np.isin(res["jval"], [-1.0, 1.0])
    np.testing.assert_array_equal(jvh[lin], res["jval"][lin])
    assert_close(hv.cpu().numpy(), res["hval"], res["hscale"], what=f"{tag} H")
    n_strict = sum(strict_violations(a, b) for a, b in (
        (c.cpu().numpy(), res["c"]), (jvh, res["jval"]), (hv.cpu().numpy(), res["hval"])))
    record_strict(tag, n_strict, c.numel() + jv.numel() + hv.numel())
    say(f"[parity] {tag}: ok (strict-form violations: {n_strict})")
    return f, g, c, jv, hv


@pytest.mark.parametrize("name,cs,opts", CASES, ids=[c[0] for c in CASES])
def test_callbacks_match_oracle(name, cs, opts, shape):
    T, K = opts.get("n_periods", 1), opts.get("n_cont", 0)
    model = opf.Model(cs, **opts)
    for seed, sigma in ((100, 1.0), (101, 0.37), (102, 0.0)):
        x = synth.point(cs, seed, n_periods=T, n_cont=K)
        y = synth.multipliers(model.m, seed)
        check_against_oracle(model, cs, opts, x, y, sigma, f"{name}/seed{seed}/{shape}")
    model.close()


@pytest.mark.parametrize("name,cs,opts", CASES[:4] + CASES[5:8], ids=[c[0] for c in CASES[:4] + CASES[5:8]])
def test_separate_callbacks_equal_fused_set(name, cs, opts, shape):
    say(f"[separate] {name} ({shape} launch)")
    T, K = opts.get("n_periods", 1), opts.get("n_cont", 0)
    model = opf.Model(cs, **opts)
    x = to_dev(synth.point(cs, 7, n_periods=T, n_cont=K))
    y = to_dev(synth.multipliers(model.m, 7))
    f, g, c, jv, hv = model.eval_set(x, y, 0.6)
    f2 = model.obj(x)
    g2 = model.grad(x)
    c2 = model.cons(x)
    j2 = model.jac_coord(x)
    h2 = model.hess_coord(x, y, 0.6)
    f3, g3, c3, j3, h3 = model.eval_set(x, y, 0.6)
    torch.cuda.synchronize()
    for a, b in ((f.view(()), f2), (g, g2), (c, c2), (jv, j2), (hv, h2), (f, f3), (g, g3), (c, c3), (jv, j3),
                 (hv, h3)):
        assert torch.equal(a.view(-1), b.view(-1))
    # a partial set computes only what is asked for
    c4 = torch.full_like(c, 7.0)
    model.eval_set(x, None, 1.0, c=c4, alloc=False)
    torch.cuda.synchronize()
    assert torch.equal(c4, c)
    with pytest.raises(opf.OPFError):
        model.eval_set(x, None, 1.0, hvals=h2, alloc=False)
    model.close()


def test_bounds_on_device_match_oracle():
    cs = synth.network(30, 44, 12, 3, variant=True)
    for opts in ({}, dict(n_periods=3, ramp_ratio=0.2), dict(n_cont=2, outaged=synth.outages(cs, 2, 5))):
        say(f"[bounds] {opts.keys()}")
        model = opf.Model(cs, **opts)
        b = model.bounds()
        ref = O.bounds(cs, **opts)
        torch.cuda.synchronize()
        for k in ("lvar", "uvar", "lcon", "ucon", "x0"):
            np.testing.assert_array_equal(b[k].cpu().numpy(), ref[k], err_msg=k)
        o, ln = model.block("vm")
        assert o == ln and np.all(ref["x0"][o:o + ln] == 1.0)
        model.close()


def test_jtprod_matches_oracle():
    for name, cs, opts in CASES:
        say(f"[jtprod] {name}")
        T, K = opts.get("n_periods", 1), opts.get("n_cont", 0)
        model = opf.Model(cs, **opts)
        x = synth.point(cs, 11, n_periods=T, n_cont=K)
        v = synth.multipliers(model.m, 11)
        res = O.evaluate(cs, x, want=O.W_JAC, **opts)
        ref = np.zeros(model.n)
        np.add.at(ref, res["jcol"], res["jval"] * v[res["jrow"]])
        scale = np.zeros(model.n)
        np.add.at(scale, res["jcol"], (np.abs(res["jval"]) + res["jscale"]) * np.abs(v[res["jrow"]]))
        out = model.jtprod(to_dev(x), to_dev(v))
        torch.cuda.synchronize()
        assert_close(out.cpu().numpy(), ref, scale, what=f"{name} J^T v")
        model.close()


def test_runs_are_bitwise_deterministic(shape):
    cs = synth.network(3000, 4050, 600, 77, variant=True)
    say(f"[determinism] 3000-bus ({shape} launch)")
    model = opf.Model(cs)
    x = to_dev(synth.point(cs, 1))
    y = to_dev(synth.multipliers(model.m, 1))
    a = [t.clone() for t in model.eval_set(x, y, 1.0)]
    for _ in range(3):
        b = model.eval_set(x, y, 1.0)
        torch.cuda.synchronize()
        for u, w in zip(a, b):
            assert torch.equal(u, w)
    model.close()


@pytest.mark.parametrize("which", ["ragged700", "hub_sc2"])
def test_launch_shapes_agree_bitwise(which):
    """The single launch (bus items recompute the branch terms) and the two
    launches (records) agree bit for bit on one model (hub_sc2: buses wider
    than a wave, contingency copies)."""
    name, cs, opts = [c for c in CASES if c[0] == which][0]
    T, K = opts.get("n_periods", 1), opts.get("n_cont", 0)
    x, y = synth.point(cs, 5, n_periods=T, n_cont=K), None
    outs, shapes = [], []
    for lim in (4096, 0):
        opf.set_single_launch_limit(lim)
        model = opf.Model(cs, **opts)
        shapes.append(model.launch_shape()[0])
        y = synth.multipliers(model.m, 5)
        outs.append([t.cpu().numpy() for t in model.eval_set(to_dev(x), to_dev(y), 0.8)])
        model.close()
    opf.set_single_launch_limit(4096)
    assert shapes == [1, 2]
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b, err_msg="single vs two launches")


def test_single_launch_limit_rejects_negative():
    with pytest.raises(opf.OPFError):
        opf.set_single_launch_limit(-1)


def test_launch_shape_query():
    """A model keeps the shape chosen at creation; the item count is the
    closed form of the 14-bus network (1 branch chunk, 1 generator chunk,
    its bus waves)."""
    cs = synth.network(14, 20, 5, 0)
    try:
        opf.set_single_launch_limit(0)
        two = opf.Model(cs)
        opf.set_single_launch_limit(4096)
        one = opf.Model(cs)
        opf.set_single_launch_limit(1)
        tiny = opf.Model(cs)
    finally:
        opf.set_single_launch_limit(4096)
    assert two.launch_shape()[0] == 2 and one.launch_shape()[0] == 1 and tiny.launch_shape()[0] == 2
    assert two.launch_shape()[1] == one.launch_shape()[1] >= 3
    for mdl in (two, one, tiny):
        mdl.close()


def test_bad_arguments_raise():
    cs = synth.network(14, 20, 5, 0)
    model = opf.Model(cs)
    x = torch.zeros(model.n, dtype=torch.float64, device=DEV)
    with pytest.raises(opf.OPFError):
        model.cons(x[:-1])
    with pytest.raises(opf.OPFError):
        model.cons(x.float())
    with pytest.raises(opf.OPFError):
        model.cons(x.cpu())
    rc = opf.lib().opf_hess_coord(model.handle, x.data_ptr(), None, 1.0, x.data_ptr(), None)
    assert rc == opf.OPF_E_ARG
    model.close()
    with pytest.raises(opf.OPFError):
        model.cons(x)


@pytest.mark.parametrize("name,cs,opts", [c for c in CASES if c[0] in ("mp4", "sc3", "hub", "ragged700")],
                         ids=["mp4", "sc3", "hub", "ragged700"])
def test_every_output_entry_written(name, cs, opts, shape):
    """Outputs pre-filled with NaN: one evaluation (fused set and separate
    callbacks) leaves none of them unwritten."""
    T, K = opts.get("n_periods", 1), opts.get("n_cont", 0)
    model = opf.Model(cs, **opts)
    x = to_dev(synth.point(cs, 9, n_periods=T, n_cont=K))
    y = to_dev(synth.multipliers(model.m, 9))

    def nan(n):
        return torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)

    fused = model.eval_set(x, y, 0.5, nan(1), nan(model.n), nan(model.m), nan(model.nnzj), nan(model.nnzh))
    sep = (model.obj(x, nan(1)), model.grad(x, nan(model.n)), model.cons(x, nan(model.m)),
           model.jac_coord(x, nan(model.nnzj)), model.hess_coord(x, y, 0.5, nan(model.nnzh)))
    torch.cuda.synchronize()
    for what, outs in (("fused", fused), ("separate", sep)):
        left = [int(torch.isnan(t).sum()) for t in outs]
        assert left == [0] * 5, f"{name} ({shape} launch) {what}: NaN entries left in f, g, c, J, H: {left}"
    model.close()


def test_allocator_hook_failure_gives_nomem():
    """An allocator hook that fails makes model and batch creation fail
    with OPF_E_NOMEM and leaves no handle behind."""
    cs = synth.network(14, 20, 5, 0)
    calls = []
    good = opf.Model(cs)
    try:
        opf.set_allocator(lambda n: calls.append(n) or 0, lambda p: None)
        with pytest.raises(opf.OPFError) as e:
            opf.Model(cs)
        assert e.value.code == opf.OPF_E_NOMEM and calls
        with pytest.raises(opf.OPFError) as e:
            opf.Batch([good], [0, 0])
        assert e.value.code == opf.OPF_E_NOMEM
    finally:
        opf.set_allocator(None, None)
    good.close()


def test_torch_caching_allocator_hook():
    """Model storage from torch's caching allocator: the same results as
    hipMalloc'd storage, bitwise, and the arena released through the hook
    on destroy; use_torch_allocator builds a working model too."""
    cs = synth.network(300, 410, 60, 3, variant=True)
    x = to_dev(synth.point(cs, 4))
    ref_model = opf.Model(cs)
    y = to_dev(synth.multipliers(ref_model.m, 4))
    ref = ref_model.eval_set(x, y, 0.9)
    live = {}

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n, 0)
        live[p] = n
        return p

    def release(p):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    try:
        opf.set_allocator(alloc, release)
        model = opf.Model(cs)
        opf.use_torch_allocator(0)
        model2 = opf.Model(cs)
    finally:
        opf.set_allocator(None, None)
    assert len(live) == 1
    for mdl in (model, model2):
        got = mdl.eval_set(x, y, 0.9)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
    model.close()
    assert not live
    model2.close()
    ref_model.close()
