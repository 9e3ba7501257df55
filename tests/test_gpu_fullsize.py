"""GPU parity at full size, in the launch configurations the benchmark times.

Every output (patterns bit for bit, values within the scale-aware
tolerance) of:
  * the 10,000-bus network (13,500 branches, 2,000 generators), plain sets
    replayed from a HIP graph in the one-launch shape;
  * the 2,000-bus x 48-period model and the 1,000-bus model with 200 N-1
    copies (two launches per set);
  * the 64-scenario uneven batch (8 networks of 500 to 20,000 buses x 8 load
    seeds) and the 10,000-bus network at 16 points per batched launch, both
    at the autotuned schedule.
Inputs follow the benchmark's seeded recipe.  The oracle evaluates each set
whole (0.3 s for a 10k-bus set, about 12 s for the 64 scenarios).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_12897_amd import opf, synth

from helpers import assert_close, record_strict, strict_violations

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def check_set(res, out, tag):
    f, g, c, jv, hv = (np.atleast_1d(t.cpu().numpy()) if torch.is_tensor(t) else np.atleast_1d(t) for t in out)
    assert_close(f[:1], [res["f"]], [res["fscale"]], what=f"{tag} f")
    assert_close(g, res["g"], np.abs(res["g"]), what=f"{tag} grad")
    assert_close(c, res["c"], res["cscale"], what=f"{tag} c")
    assert_close(jv, res["jval"], res["jscale"], what=f"{tag} J")
    assert_close(hv, res["hval"], res["hscale"], what=f"{tag} H")
    n_strict = sum(strict_violations(a, b) for a, b in ((c, res["c"]), (jv, res["jval"]), (hv, res["hval"])))
    record_strict(tag, n_strict, len(c) + len(jv) + len(hv))
    say(f"[fullsize] {tag}: strict-form violations {n_strict}")


def check_patterns(model, res, tag):
    jr, jc = model.jac_structure()
    hr, hc = model.hess_structure()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(jr.cpu().numpy(), res["jrow"], err_msg=f"{tag} J rows")
    np.testing.assert_array_equal(jc.cpu().numpy(), res["jcol"], err_msg=f"{tag} J cols")
    np.testing.assert_array_equal(hr.cpu().numpy(), res["hrow"], err_msg=f"{tag} H rows")
    np.testing.assert_array_equal(hc.cpu().numpy(), res["hcol"], err_msg=f"{tag} H cols")


def out_set(model):
    return (torch.empty(1, dtype=torch.float64, device=DEV), torch.empty(model.n, dtype=torch.float64, device=DEV),
            torch.empty(model.m, dtype=torch.float64, device=DEV),
            torch.empty(model.nnzj, dtype=torch.float64, device=DEV),
            torch.empty(model.nnzh, dtype=torch.float64, device=DEV))


def test_headline_10k_graph_replays_match_oracle():
    cs = synth.network(10000, 13500, 2000, 1)
    model = opf.Model(cs)
    assert model.launch_shape()[0] == 1, "the 10k-bus model is benchmarked in the one-launch shape"
    say(f"[fullsize] 10k: n={model.n} m={model.m} nnzj={model.nnzj} nnzh={model.nnzh}")
    n_in = 4
    xs_h = [synth.point(cs, (101, r)) for r in range(n_in)]
    ys_h = [synth.multipliers(model.m, (101, r)) for r in range(n_in)]
    xs, ys = [dev(a) for a in xs_h], [dev(a) for a in ys_h]
    outs = [out_set(model) for _ in range(n_in)]

    def enqueue():  # 8 back-to-back sets rotating over the inputs and outputs
        for k in range(8):
            model.eval_set(xs[k % n_in], ys[k % n_in], 1.0, *outs[k % n_in])

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        enqueue()
    torch.cuda.synchronize()
    eager = [[t.clone() for t in o] for o in outs]
    for r in range(n_in):
        res = O.evaluate(cs, xs_h[r], ys_h[r], 1.0)
        if r == 0:
            check_patterns(model, res, "10k")
        check_set(res, eager[r], f"10k set {r}")
        say(f"[fullsize] 10k set {r}: matches the oracle")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        enqueue()
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:  # eager work between replays
            for t in o:
                t.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for r in range(n_in):
            for a, b in zip(outs[r], eager[r]):
                assert torch.equal(a, b), f"replay {rep} set {r} differs from the eager run"
        say(f"[fullsize] 10k graph replay {rep}: bitwise equal to the eager sets")
    model.close()


@pytest.mark.parametrize("which", ["mp48", "sc200"])
def test_large_models_match_oracle(which):
    if which == "mp48":
        cs = synth.network(2000, 2700, 400, 2)
        pd_t, qd_t = synth.mp_loads(cs, 48, 202)
        opts, T, K = dict(n_periods=48, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2), 48, 0
    else:
        cs = synth.network(1000, 1350, 200, 31)
        opts, T, K = dict(n_cont=200, outaged=synth.outages(cs, 200, 32)), 1, 200
    model = opf.Model(cs, **opts)
    say(f"[fullsize] {which}: n={model.n} m={model.m} nnzj={model.nnzj} nnzh={model.nnzh}, "
        f"{model.launch_shape()[0]} launches per set")
    x = synth.point(cs, (104, 0), n_periods=T, n_cont=K)
    y = synth.multipliers(model.m, (104, 0))
    out = model.eval_set(dev(x), dev(y), 1.0)
    torch.cuda.synchronize()
    res = O.evaluate(cs, x, y, 1.0, **opts)
    check_patterns(model, res, which)
    check_set(res, out, which)
    say(f"[fullsize] {which}: matches the oracle")
    model.close()


def _batch_check(batch, cases, xs, ys, sig, out, tag):
    F, G, C, J, H = (t.cpu().numpy() for t in out)
    for i, (cs, opts) in enumerate(cases):
        res = O.evaluate(cs, xs[i], ys[i], sig, **opts)
        sl = lambda o, a: a[int(o[i]):int(o[i + 1])]  # noqa: E731
        check_set(res, (F[i:i + 1], sl(batch.xoff, G), sl(batch.coff, C), sl(batch.joff, J), sl(batch.hoff, H)),
                  f"{tag} instance {i}")
    say(f"[fullsize] {tag}: {len(cases)} instances match the oracle")


def test_batch64_mix_matches_oracle():
    nets, models, inst, pds, qds, cases = [], [], [], [], [], []
    for j, N in enumerate(synth.BATCH_SIZES):
        cs = synth.network(N, int(round(1.35 * N)), int(round(0.2 * N)), 300 + j)
        nets.append(cs)
        models.append(opf.Model(cs))
        for s in range(8):
            pd, qd = synth.scenario_loads(cs, 3000 + 8 * j + s)
            inst.append(j)
            pds.append(pd)
            qds.append(qd)
            c2 = dict(cs)
            c2["pd"], c2["qd"] = pd, qd
            cases.append((c2, {}))
    batch = opf.Batch(models, inst, np.concatenate(pds), np.concatenate(qds))
    xs = [synth.point(nets[inst[i]], (103, i)) for i in range(batch.n_inst)]
    ys = [synth.multipliers(int(batch.coff[i + 1] - batch.coff[i]), (103, i)) for i in range(batch.n_inst)]
    X, Y = dev(np.concatenate(xs)), dev(np.concatenate(ys))
    S = torch.ones(batch.n_inst, dtype=torch.float64, device=DEV)
    out = (torch.empty(batch.n_inst, dtype=torch.float64, device=DEV),
           torch.empty(batch.n, dtype=torch.float64, device=DEV), torch.empty(batch.m, dtype=torch.float64, device=DEV),
           torch.empty(batch.nnzj, dtype=torch.float64, device=DEV),
           torch.empty(batch.nnzh, dtype=torch.float64, device=DEV))
    sched = batch.tune()
    say(f"[fullsize] batch64: {batch.n_inst} instances, schedule wg_per_cu={sched}")
    batch.eval(X, Y, S, *out)
    torch.cuda.synchronize()
    _batch_check(batch, cases, xs, ys, 1.0, out, "batch64")
    batch.close()
    for m in models:
        m.close()


def test_points16_10k_matches_oracle():
    cs = synth.network(10000, 13500, 2000, 1)
    model = opf.Model(cs)
    B = 16
    batch = opf.Batch([model], np.zeros(B, np.int32))
    xs = [synth.point(cs, (101, i)) for i in range(B)]
    ys = [synth.multipliers(model.m, (101, i)) for i in range(B)]
    X, Y = dev(np.concatenate(xs)), dev(np.concatenate(ys))
    S = torch.ones(B, dtype=torch.float64, device=DEV)
    out = (torch.empty(B, dtype=torch.float64, device=DEV), torch.empty(batch.n, dtype=torch.float64, device=DEV),
           torch.empty(batch.m, dtype=torch.float64, device=DEV),
           torch.empty(batch.nnzj, dtype=torch.float64, device=DEV),
           torch.empty(batch.nnzh, dtype=torch.float64, device=DEV))
    sched = batch.tune()
    say(f"[fullsize] 10k x 16 points: schedule wg_per_cu={sched}")
    batch.eval(X, Y, S, *out)
    torch.cuda.synchronize()
    _batch_check(batch, [(cs, {})] * B, xs, ys, 1.0, out, "10k x 16 points")
    batch.close()
    model.close()
