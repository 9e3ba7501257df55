"""Batched evaluation: one persistent launch over many uneven instances.

Batched results equal the plain per-instance launches bit for bit, under
every schedule the autotuner may pick, across repeated evaluations and
replays of a captured HIP graph, for J^T v too; sampled instances also
match the oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_12897_amd import opf, synth

from helpers import assert_close, hub_network

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(params=["single", "two"])
def shape(request):
    """Launch shape of the models built in the test: small models evaluate
    in one launch by default; limit 0 forces two launches everywhere."""
    opf.set_single_launch_limit(4096 if request.param == "single" else 0)
    yield request.param
    opf.set_single_launch_limit(4096)


def build_mix(sizes=(40, 300, 1200), per=3, with_mp=True, with_sc=True, with_hub=True):
    """Instances of several networks with their own loads, plus one
    multi-period and one contingency model, and two load scenarios of a
    network with hub buses (segments beyond one wave)."""
    nets, models, inst_model, pds, qds, plain = [], [], [], [], [], []
    for j, N in enumerate(sizes):
        cs = synth.network(N, int(round(1.35 * N)), max(1, int(round(0.2 * N))), 500 + j, variant=(j % 2 == 0))
        nets.append((cs, {}))
        models.append(opf.Model(cs))
        for s in range(per):
            pd, qd = synth.scenario_loads(cs, 900 + 10 * j + s)
            c2 = dict(cs)
            c2["pd"], c2["qd"] = pd, qd
            inst_model.append(len(models) - 1)
            pds.append(pd)
            qds.append(qd)
            plain.append((c2, {}))
    if with_mp:
        cs = synth.network(50, 70, 10, 61, variant=True)
        pd_t, qd_t = synth.mp_loads(cs, 3, 62)
        opts = dict(n_periods=3, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2)
        models.append(opf.Model(cs, **opts))
        nets.append((cs, opts))
        for s in range(2):
            a, b = synth.mp_loads(cs, 3, 70 + s)
            inst_model.append(len(models) - 1)
            pds.append(a)
            qds.append(b)
            plain.append((cs, dict(opts, pd_t=a, qd_t=b)))
    if with_sc:
        cs = synth.network(60, 85, 12, 63, variant=True)
        opts = dict(n_cont=3, outaged=synth.outages(cs, 3, 64))
        models.append(opf.Model(cs, **opts))
        nets.append((cs, opts))
        pd, qd = synth.scenario_loads(cs, 80)
        c2 = dict(cs)
        c2["pd"], c2["qd"] = pd, qd
        inst_model.append(len(models) - 1)
        pds.append(pd)
        qds.append(qd)
        plain.append((c2, opts))
    if with_hub:
        cs = hub_network()
        models.append(opf.Model(cs))
        nets.append((cs, {}))
        for s_ in range(2):
            pd, qd = synth.scenario_loads(cs, 90 + s_)
            c2 = dict(cs)
            c2["pd"], c2["qd"] = pd, qd
            inst_model.append(len(models) - 1)
            pds.append(pd)
            qds.append(qd)
            plain.append((c2, {}))
    batch = opf.Batch(models, inst_model, np.concatenate(pds), np.concatenate(qds))
    return batch, models, inst_model, plain


def fill_inputs(batch, plain):
    X = torch.empty(batch.n, dtype=torch.float64, device=DEV)
    Y = torch.empty(batch.m, dtype=torch.float64, device=DEV)
    xs, ys = [], []
    for i, (cs, opts) in enumerate(plain):
        x = synth.point(cs, (7, i), n_periods=opts.get("n_periods", 1), n_cont=opts.get("n_cont", 0))
        y = synth.multipliers(int(batch.coff[i + 1] - batch.coff[i]), (7, i))
        X[batch.xoff[i]:batch.xoff[i + 1]] = torch.as_tensor(x, device=DEV)
        Y[batch.coff[i]:batch.coff[i + 1]] = torch.as_tensor(y, device=DEV)
        xs.append(x)
        ys.append(y)
    sig = torch.linspace(0.5, 1.5, batch.n_inst, dtype=torch.float64, device=DEV)
    return X, Y, sig, xs, ys


def outputs(batch):
    return (torch.full((batch.n_inst,), np.nan, dtype=torch.float64, device=DEV),
            torch.full((batch.n,), np.nan, dtype=torch.float64, device=DEV),
            torch.full((batch.m,), np.nan, dtype=torch.float64, device=DEV),
            torch.full((batch.nnzj,), np.nan, dtype=torch.float64, device=DEV),
            torch.full((batch.nnzh,), np.nan, dtype=torch.float64, device=DEV))


def plain_reference(batch, plain, X, Y, sig):
    ref = outputs(batch)
    F, G, C, J, H = ref
    for i, (cs, opts) in enumerate(plain):
        m = opf.Model(cs, **opts)
        sl = lambda o, a: a[int(o[i]):int(o[i + 1])]  # noqa: E731
        m.eval_set(sl(batch.xoff, X), sl(batch.coff, Y), float(sig[i].item()), F[i:i + 1], sl(batch.xoff, G),
                   sl(batch.coff, C), sl(batch.joff, J), sl(batch.hoff, H))
        torch.cuda.synchronize()
        m.close()
    return ref


def match_plain(out, ref, shape):
    """Batches take the two-launch shape; plain launches take either shape
    (one launch: bus items recompute the branch terms).  Both are bitwise
    equal to the batch: the shared branch-term arithmetic rounds the same
    way in every kernel."""
    for a, b in zip(out, ref):
        assert torch.equal(a, b), f"batch differs from the plain {shape}-launch sets"


def test_batch_equals_plain_bitwise_every_schedule(shape):
    say(f"[batch] build mix ({shape} launch)")
    batch, models, inst_model, plain = build_mix()
    X, Y, sig, xs, ys = fill_inputs(batch, plain)
    ref = plain_reference(batch, plain, X, Y, sig)
    first = None
    for wg in (0, -1, 1, 2, 4, 16, 32):
        say(f"[batch] schedule wg_per_cu={wg}")
        batch.set_schedule(wg)
        out = outputs(batch)
        batch.eval(X, Y, sig, *out)
        torch.cuda.synchronize()
        if first is None:
            first = [t.clone() for t in out]
        for a, b in zip(out, first):  # the schedule never changes a bit
            assert torch.equal(a, b), f"schedule {wg} differs from the first schedule"
        match_plain(out, ref, shape)
    say("[batch] tune")
    sched = batch.tune()
    out = outputs(batch)
    batch.eval(X, Y, sig, *out)
    torch.cuda.synchronize()
    for a, b in zip(out, first):
        assert torch.equal(a, b)
    say(f"[batch] tuned schedule {sched}")
    batch.close()
    for m in models:
        m.close()


def test_batch_repeated_evals_and_partial_outputs():
    opf.set_single_launch_limit(0)  # plain references in the batch's (two-launch) shape
    batch, models, inst_model, plain = build_mix(sizes=(30, 200), per=2, with_mp=False)
    X, Y, sig, xs, ys = fill_inputs(batch, plain)
    ref = plain_reference(batch, plain, X, Y, sig)
    out = outputs(batch)
    for rep in range(4):
        say(f"[batch] replay {rep}")
        for t in out:
            t.fill_(np.nan)  # eager work between replays
        torch.cuda.synchronize()
        batch.eval(X, Y, sig, *out)
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert torch.equal(a, b), f"replay {rep}"
    # only constraints
    C = torch.full((batch.m,), np.nan, dtype=torch.float64, device=DEV)
    batch.eval(X, C=C)
    torch.cuda.synchronize()
    assert torch.equal(C, ref[2])
    with pytest.raises(opf.OPFError):
        batch.eval(X, H=out[4])
    batch.close()
    for m in models:
        m.close()
    opf.set_single_launch_limit(4096)


@pytest.mark.parametrize("wg_per_cu", [0, 4, -1])
def test_batch_eval_captured_in_graph(wg_per_cu):
    """The batch's two launches captured into a HIP graph: every replay, with
    eager work in between, is bitwise the eager evaluation."""
    batch, models, inst_model, plain = build_mix(sizes=(30, 200), per=2, with_mp=False)
    batch.set_schedule(wg_per_cu)
    X, Y, sig, xs, ys = fill_inputs(batch, plain)
    ref = outputs(batch)
    batch.eval(X, Y, sig, *ref)
    torch.cuda.synchronize()
    out = outputs(batch)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        batch.eval(X, Y, sig, *out)
    torch.cuda.synchronize()
    for rep in range(3):
        say(f"[batch] captured graph replay {rep} (wg_per_cu={wg_per_cu})")
        for t in out:
            t.fill_(np.nan)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert torch.equal(a, b), f"replay {rep}"
    del graph
    batch.close()
    for m in models:
        m.close()


def test_batch_jtprod_equals_plain():
    batch, models, inst_model, plain = build_mix(sizes=(25, 400), per=2)
    X, V, _, xs, vs = fill_inputs(batch, plain)
    out = batch.jtprod(X, V)
    torch.cuda.synchronize()
    for i, (cs, opts) in enumerate(plain):
        m = opf.Model(cs, **opts)
        r = m.jtprod(X[batch.xoff[i]:batch.xoff[i + 1]], V[batch.coff[i]:batch.coff[i + 1]])
        torch.cuda.synchronize()
        assert torch.equal(r, out[batch.xoff[i]:batch.xoff[i + 1]]), f"instance {i}"
        m.close()
    batch.close()
    for m in models:
        m.close()


def test_batch_instances_match_oracle():
    batch, models, inst_model, plain = build_mix(sizes=(35, 260), per=2)
    X, Y, sig, xs, ys = fill_inputs(batch, plain)
    out = outputs(batch)
    batch.eval(X, Y, sig, *out)
    torch.cuda.synchronize()
    F, G, C, J, H = (t.cpu().numpy() for t in out)
    for i, (cs, opts) in enumerate(plain):
        say(f"[batch/oracle] instance {i}")
        res = O.evaluate(cs, xs[i], ys[i], float(sig[i].item()), **opts)
        sl = lambda o, a: a[int(o[i]):int(o[i + 1])]  # noqa: E731
        assert_close([F[i]], [res["f"]], [res["fscale"]], what=f"inst {i} f")
        assert_close(sl(batch.coff, C), res["c"], res["cscale"], what=f"inst {i} c")
        assert_close(sl(batch.joff, J), res["jval"], res["jscale"], what=f"inst {i} J")
        assert_close(sl(batch.hoff, H), res["hval"], res["hscale"], what=f"inst {i} H")
        assert_close(sl(batch.xoff, G), res["g"], np.abs(res["g"]), what=f"inst {i} g")
    batch.close()
    for m in models:
        m.close()
