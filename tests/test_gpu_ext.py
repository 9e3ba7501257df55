"""GPU parity of the storage units (Sec. III-C3) and the user-extension
devices (Sec. III-D) against the oracle.

Same bar as the other parity tests: patterns bit-exact; values within
|v - v*| <= 1e-12 max(|v*|, S) + 1e-14; constant Jacobian entries
bit-exact; both launch shapes; every output entry written; separate
callbacks, the fused set and the entry point that allocates nothing
bitwise equal; J^T v against the oracle's dense product; the batch
bitwise equal to two-launch plain sets; the 2,000-bus x 48-period model
with storage at its largest loads and devices, at full size.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_12897_amd import opf, synth

from helpers import assert_close, record_strict, strict_violations
from test_host_pattern import _ext_cases

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    yield from _ext_cases()
    cs = synth.network(700, 951, 140, 12, variant=True)
    pd_t, qd_t = synth.mp_loads(cs, 3, 13)
    yield "ragged700_mp3", cs, dict(n_periods=3, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2,
                                    storage=synth.storage(cs, 14), stor_dt=0.5, stor_comp=True,
                                    devices=synth.devices(cs, 150, 15))


CASES = list(_cases())
SHAPES = {"single": 4096, "two": 0}


@pytest.fixture(params=list(SHAPES))
def shape(request):
    opf.set_single_launch_limit(SHAPES[request.param])
    yield request.param
    opf.set_single_launch_limit(4096)


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def point(cs, seed, opts):
    return synth.point(cs, seed, n_periods=opts.get("n_periods", 1), form=opts.get("form", "polar"),
                       storage=opts.get("storage"), devices=opts.get("devices"))


def check(res, out, tag):
    f, g, c, jv, hv = (np.atleast_1d(t.cpu().numpy()) if torch.is_tensor(t) else np.atleast_1d(t) for t in out)
    assert_close(f[:1], [res["f"]], [res["fscale"]], what=f"{tag} f")
    assert_close(g, res["g"], np.abs(res["g"]), what=f"{tag} grad")
    assert_close(c, res["c"], res["cscale"], what=f"{tag} c")
    assert_close(jv, res["jval"], res["jscale"], what=f"{tag} J")
    lin = np.isin(res["jval"], [-1.0, 1.0])
    np.testing.assert_array_equal(jv[lin], res["jval"][lin])
    assert_close(hv, res["hval"], res["hscale"], what=f"{tag} H")
    n_strict = sum(strict_violations(a, b) for a, b in ((c, res["c"]), (jv, res["jval"]), (hv, res["hval"])))
    record_strict(tag, n_strict, len(c) + len(jv) + len(hv))
    say(f"[ext] {tag}: ok (strict-form violations: {n_strict})")


def check_patterns(model, res, tag):
    jr, jc = model.jac_structure()
    hr, hc = model.hess_structure()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(jr.cpu().numpy(), res["jrow"], err_msg=f"{tag} J rows")
    np.testing.assert_array_equal(jc.cpu().numpy(), res["jcol"], err_msg=f"{tag} J cols")
    np.testing.assert_array_equal(hr.cpu().numpy(), res["hrow"], err_msg=f"{tag} H rows")
    np.testing.assert_array_equal(hc.cpu().numpy(), res["hcol"], err_msg=f"{tag} H cols")


@pytest.mark.parametrize("name,cs,opts", CASES, ids=[c[0] for c in CASES])
def test_ext_callbacks_match_oracle(name, cs, opts, shape):
    model = opf.Model(cs, **opts)
    say(f"[ext] {name} ({shape}): n={model.n} m={model.m} nnzj={model.nnzj} nnzh={model.nnzh}")
    for seed, sigma in ((100, 1.0), (101, 0.37), (102, 0.0)):
        x = point(cs, seed, opts)
        y = synth.multipliers(model.m, seed)
        res = O.evaluate(cs, x, y, sigma, **opts)
        if seed == 100:
            check_patterns(model, res, name)
        out = model.eval_set(to_dev(x), to_dev(y), sigma)
        torch.cuda.synchronize()
        check(res, out, f"ext {name}/seed{seed}/{shape}")
    model.close()


@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_ext_every_entry_written_and_calls_agree(name, shape):
    """NaN-filled outputs: the fused set, the separate callbacks and the
    entry point that allocates nothing write every entry, bitwise alike."""
    _, cs, opts = [c for c in CASES if c[0] == name][0]
    model = opf.Model(cs, **opts)
    x = to_dev(point(cs, 7, opts))
    y = to_dev(synth.multipliers(model.m, 7))

    def nan(n):
        return torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)

    fused = model.eval_set(x, y, 0.6, nan(1), nan(model.n), nan(model.m), nan(model.nnzj), nan(model.nnzh))
    sep = (model.obj(x, nan(1)), model.grad(x, nan(model.n)), model.cons(x, nan(model.m)),
           model.jac_coord(x, nan(model.nnzj)), model.hess_coord(x, y, 0.6, nan(model.nnzh)))
    na = model.eval_set_noalloc(x, y, 0.6, nan(1), nan(model.n), nan(model.m), nan(model.nnzj), nan(model.nnzh))
    f_only = model.obj(x, nan(1))
    torch.cuda.synchronize()
    left = [int(torch.isnan(t).sum()) for t in fused]
    assert left == [0] * 5, f"{name} ({shape}): NaN entries left in f, g, c, J, H: {left}"
    for a, b, c in zip(fused, sep, na):
        assert torch.equal(a.view(-1), b.view(-1)) and torch.equal(a.view(-1), c.view(-1))
    assert torch.equal(f_only.view(-1), fused[0].view(-1))
    model.close()


def test_ext_jtprod_matches_oracle():
    for name, cs, opts in CASES:
        say(f"[ext jtprod] {name}")
        model = opf.Model(cs, **opts)
        x = point(cs, 11, opts)
        v = synth.multipliers(model.m, 11)
        res = O.evaluate(cs, x, want=O.W_JAC, **opts)
        ref = np.zeros(model.n)
        np.add.at(ref, res["jcol"], res["jval"] * v[res["jrow"]])
        scale = np.zeros(model.n)
        np.add.at(scale, res["jcol"], (np.abs(res["jval"]) + res["jscale"]) * np.abs(v[res["jrow"]]))
        out = model.jtprod(to_dev(x), to_dev(v))
        torch.cuda.synchronize()
        assert_close(out.cpu().numpy(), ref, scale, what=f"ext {name} J^T v")
        model.close()


def test_ext_bounds_and_blocks_on_device():
    name, cs, opts = CASES[0]
    model = opf.Model(cs, **opts)
    b = model.bounds()
    ref = O.bounds(cs, **opts)
    torch.cuda.synchronize()
    for k in ("lvar", "uvar", "lcon", "ucon", "x0"):
        np.testing.assert_array_equal(b[k].cpu().numpy(), ref[k], err_msg=k)
    T, S, D = opts["n_periods"], len(opts["storage"]["bus"]), len(opts["devices"]["bus"])
    assert model.block("ps")[1] == S * T and model.block("u")[1] == D * T
    assert model.block("u")[0] + D * T == model.n
    assert model.block("soc")[1] == S * T and model.block("dev_init")[1] == D
    assert model.block("dev_init")[0] + D == model.m
    model.close()


def test_ext_batch_bitwise_equal_to_two_launch_plain():
    """Instances of models with storage and devices (own loads per
    instance), both schedules, against two-launch plain sets; J^T v too."""
    opf.set_single_launch_limit(0)
    try:
        specs = [c for c in CASES if c[0] in ("stor_dev_mp4", "stor_static", "hub_stor_dev_mp2")]
        models = [opf.Model(cs, **opts) for _, cs, opts in specs]
    finally:
        opf.set_single_launch_limit(4096)
    inst = [0, 1, 2, 0]
    T = [opts.get("n_periods", 1) for _, _, opts in specs]
    pds, qds = [], []
    for i, j in enumerate(inst):
        cs = specs[j][1]
        fac = 1.0 + 0.05 * (i + 1)
        base_pd = specs[j][2].get("pd_t", np.tile(cs["pd"], T[j]))
        base_qd = specs[j][2].get("qd_t", np.tile(cs["qd"], T[j]))
        pds.append(fac * base_pd)
        qds.append(fac * base_qd)
    batch = opf.Batch(models, inst, np.concatenate(pds), np.concatenate(qds))
    xs = [point(specs[j][1], (106, i), specs[j][2]) for i, j in enumerate(inst)]
    ys = [synth.multipliers(models[j].m, (106, i)) for i, j in enumerate(inst)]
    X, Y = to_dev(np.concatenate(xs)), to_dev(np.concatenate(ys))
    S = torch.linspace(0.5, 1.5, len(inst), dtype=torch.float64, device=DEV)
    for wg in (0, 4, -1):
        batch.set_schedule(wg)
        say(f"[ext batch] schedule {wg}")
        out = (torch.empty(len(inst), dtype=torch.float64, device=DEV),) + tuple(
            torch.empty(k, dtype=torch.float64, device=DEV) for k in (batch.n, batch.m, batch.nnzj, batch.nnzh))
        batch.eval(X, Y, S, *out)
        for i, j in enumerate(inst):
            name, cs, opts = specs[j]
            o2 = dict(opts)
            if T[j] > 1:
                o2["pd_t"], o2["qd_t"] = pds[i], qds[i]
                c2 = cs
            else:
                c2 = dict(cs)
                c2["pd"], c2["qd"] = pds[i], qds[i]
            opf.set_single_launch_limit(0)
            try:
                pm = opf.Model(c2, **o2)
            finally:
                opf.set_single_launch_limit(4096)
            ref = pm.eval_set(to_dev(xs[i]), to_dev(ys[i]), float(S[i]))
            torch.cuda.synchronize()
            assert torch.equal(out[0][i:i + 1], ref[0].view(1)), f"instance {i} f"
            for off, k in ((batch.xoff, 1), (batch.coff, 2), (batch.joff, 3), (batch.hoff, 4)):
                assert torch.equal(out[k][int(off[i]):int(off[i + 1])], ref[k]), f"instance {i} output {k}"
            if wg == 0 and i < 3:
                check(O.evaluate(c2, xs[i], ys[i], float(S[i]), **o2), ref, f"ext batch instance {i}")
            pm.close()
    out_b = batch.jtprod(X, Y)
    torch.cuda.synchronize()
    for i, j in enumerate(inst[:3]):
        ref = models[j].jtprod(to_dev(xs[i]), to_dev(ys[i]))
        torch.cuda.synchronize()
        assert torch.equal(out_b[int(batch.xoff[i]):int(batch.xoff[i + 1])], ref)
    batch.close()
    for mdl in models:
        mdl.close()


def mp48_storage_case():
    """The 2,000-bus x 48-period network with storage at its largest 10 % of
    loads (Sec. IV-C: energy rating 1.5x the bus load) and 100
    electrolyzer-like devices, 30-minute periods."""
    cs = synth.network(2000, 2700, 400, 2)
    pd_t, qd_t = synth.mp_loads(cs, 48, 202)
    opts = dict(n_periods=48, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2, storage=synth.storage(cs, 203),
                stor_dt=0.5, devices=synth.devices(cs, 100, 204))
    return cs, opts


def test_mp48_storage_full_size_matches_oracle():
    cs, opts = mp48_storage_case()
    model = opf.Model(cs, **opts)
    say(f"[ext] mp48 storage: n={model.n} m={model.m} nnzj={model.nnzj} nnzh={model.nnzh}, "
        f"{model.launch_shape()[0]} launches per set")
    x = point(cs, (104, 0), opts)
    y = synth.multipliers(model.m, (104, 0))
    out = model.eval_set(to_dev(x), to_dev(y), 1.0)
    torch.cuda.synchronize()
    res = O.evaluate(cs, x, y, 1.0, **opts)
    check_patterns(model, res, "mp48 storage")
    check(res, out, "ext mp48 storage")
    model.close()
