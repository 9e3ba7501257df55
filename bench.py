#!/usr/bin/env python3
"""Benchmark: FP64 polar AC-OPF callback sets per second on one MI355X.

One callback set = (f, grad f, c, J values, H values) at one (x, y, sigma),
the five NLPModels callbacks an interior-point solver calls per iteration.

Headline workload: the plain single-instance callbacks on a 10,000-bus
synthetic network (13,500 branches, 2,000 generators), one step = 1,000
callback sets at distinct seeded (x, y) pairs, launched back to back from a
HIP graph.  Inputs rotate over 256 pre-generated pairs and outputs over 64
buffer sets, so the working set (~0.7 GB) exceeds the 256 MB Infinity Cache
and the roofline is the HBM one.

Also measured in the same run (the "extra" object): the batched form on the
64-scenario uneven mix (8 networks of 500 to 20,000 buses x 8 load seeds,
one persistent launch) against the plain per-instance launches, the
multi-period model (2,000 buses x 48 periods), the N-1 contingency model
(1,000 buses + 200 outage copies), the rectangular form, the interior-point
consumer of the callbacks (300 buses) and the learned warm-start proxy (300
buses, batches of 4,096 load samples).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "callback sets/s (f,∇f,c,J,∇²L) FP64 batched vs plain; % of HBM roofline"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "eval_set_10k_hbm_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2510_12897_amd", "csrc", f) for f in ("eval_kernels.hip", "dev_model.h")]


def _code_only(text: str) -> str:
    """Source text without comments and whitespace (a comment edit does not
    change the kernels the counters were taken on)."""
    import re

    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return "".join(text.split())


def kernel_hash(texts=None) -> str:
    """sha256 of the kernel sources' code (comments and whitespace removed)."""
    import hashlib

    h = hashlib.sha256()
    if texts is None:
        texts = []
        for f in KERNEL_SOURCES:
            with open(f, encoding="utf-8") as fh:
                texts.append(fh.read())
    for t in texts:
        h.update(_code_only(t).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per callback set from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated), or None when the kernel sources
    have changed since the counters were taken."""
    try:
        fields = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        if fields.get("kernel_source_sha256") != kernel_hash():
            return None
        return int(float(fields["hbm_bytes_per_set"]))
    except (OSError, KeyError, ValueError):
        return None


def algorithmic_bytes(cs: dict, dims, T: int = 1, K: int = 0, mp_loads: bool = False, rect: bool = False,
                      S: int = 0, D: int = 0) -> int:
    """Bytes one callback set must move at least: every input read once and
    every output written once.  Reads: x (8n), y (8m), sigma; branch data
    (8 admittance terms + rate^2 + two int32 buses = 80 B; the rectangular
    form also reads the two angle-limit tangents, 16 B); bus loads and
    shunts (32 B, loads per period when they vary); generator costs and bus
    (28 B); adjacency (half-edges, bus pointers, generator lists); outage
    list; storage units (13 parameters and a bus, 108 B) and devices (3
    coefficients and a bus, 28 B) with their per-bus lists.  Writes: f,
    grad f (8n), c (8m), J (8 nnzj), H (8 nnzh)."""
    n, m, nnzj, nnzh = dims
    N, L, G = cs["n_bus"], cs["n_branch"], cs["n_gen"]
    reads = 8 * n + 8 * m + 8
    reads += (96 if rect else 80) * L
    reads += 16 * N * (T if mp_loads else 1) + 16 * N
    reads += 28 * G
    reads += 4 * 2 * L + 4 * (N + 1) * 2 + 4 * G
    reads += 4 * K
    if S or D:
        reads += 108 * S + 28 * D + 4 * (S + D) + 8 * (N + 1)
    writes = 8 + 8 * n + 8 * m + 8 * nnzj + 8 * nnzh
    return int(reads + writes)


def _nproc() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def _cpu_model_name() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


class PlainRunner:
    """Back-to-back plain callback sets of one model, captured in a HIP graph."""

    def __init__(self, model, xs, ys, n_out: int, sets: int, torch):
        self.torch = torch
        self.model = model
        dev = torch.device("cuda", model.device)
        self.xs, self.ys = xs, ys
        self.outs = [(torch.empty(1, dtype=torch.float64, device=dev),
                      torch.empty(model.n, dtype=torch.float64, device=dev),
                      torch.empty(model.m, dtype=torch.float64, device=dev),
                      torch.empty(model.nnzj, dtype=torch.float64, device=dev),
                      torch.empty(model.nnzh, dtype=torch.float64, device=dev)) for _ in range(n_out)]
        self.sets = sets
        self.graph = None

    def enqueue(self, start: int = 0):
        for k in range(self.sets):
            j = start + k
            x, y = self.xs[j % len(self.xs)], self.ys[j % len(self.ys)]
            f, g, c, jv, hv = self.outs[j % len(self.outs)]
            self.model.eval_set(x, y, 1.0, f, g, c, jv, hv)

    def capture(self):
        torch = self.torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.enqueue()  # warm the code path outside capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=s):
            self.enqueue()
        torch.cuda.synchronize()

    def step(self):
        if self.graph is None:
            self.enqueue()
        else:
            self.graph.replay()


def time_steps(torch, fn, steps: int, warmup: int):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def bench_headline(args, torch, opf, synth, log):
    cs = synth.network(10000, 13500, 2000, 1)
    model = opf.Model(cs, device=0)
    dims = (model.n, model.m, model.nnzj, model.nnzh)
    dev = torch.device("cuda", 0)
    log(f"headline model: n={model.n} m={model.m} nnzj={model.nnzj} nnzh={model.nnzh}")
    n_in = args.inputs
    xs = [torch.as_tensor(synth.point(cs, (101, r)), device=dev) for r in range(n_in)]
    ys = [torch.as_tensor(synth.multipliers(model.m, (101, r)), device=dev) for r in range(n_in)]
    log(f"generated {n_in} seeded (x, y) pairs")
    runner = PlainRunner(model, xs, ys, n_out=64, sets=args.sets_per_step, torch=torch)
    if not args.eager:
        runner.capture()
    secs, wall = time_steps(torch, runner.step, args.steps, args.warmup)
    n_sets = args.steps * args.sets_per_step
    per_set = secs / n_sets
    bytes_set = algorithmic_bytes(cs, dims)
    log(f"headline: {n_sets} sets in {secs * 1e3:.2f} ms (GPU events), {wall * 1e3:.2f} ms wall")
    launches, items = model.launch_shape()
    kernel = (f"set_kernel_single: one launch per callback set ({items} 64-lane work items)" if launches == 1 else
              f"branch_kernel<0> + bus_kernel<0>: two launches per callback set ({items} 64-lane work items)")
    return dict(cs=cs, model=model, dims=dims, xs=xs, ys=ys, secs=secs, wall=wall, n_sets=n_sets, kernel=kernel,
                per_set=per_set, bytes_set=bytes_set)


def bench_cpu_baseline(h, synth, oracle, budget_s: float, log):
    cs = h["cs"]
    xs = [synth.point(cs, (101, r)) for r in range(4)]
    ys = [synth.multipliers(h["model"].m, (101, r)) for r in range(4)]
    done = 0
    t0 = time.perf_counter()
    while True:
        oracle.evaluate(cs, xs[done % 4], ys[done % 4], 1.0)
        done += 1
        el = time.perf_counter() - t0
        if (el >= budget_s and done >= 3) or done >= 1000:
            break
    log(f"oracle: {done} sets in {el:.1f} s")
    return dict(value=done / el, unit="sets/s", cores=1, kind="oracle", threads=1, nproc=_nproc(),
                cpu_model=_cpu_model_name(),
                sample=f"{done} callback sets of the 10k-bus workload (x, y seeds (101, 0..3)), "
                       f"single-threaded C oracle, {el:.1f} s on {_cpu_model_name()}")


def bench_cpu_batch64(synth, oracle, log):
    """The oracle over the 64-scenario mix: every scenario once on one
    thread, then once with one scenario per thread on every host core (the
    oracle is a C library called through ctypes, which releases the
    interpreter lock, so the threads run in parallel)."""
    from concurrent.futures import ThreadPoolExecutor

    cases = []
    for j, N in enumerate(synth.BATCH_SIZES):
        cs = synth.network(N, int(round(1.35 * N)), int(round(0.2 * N)), 300 + j)
        n, m = oracle.dims(cs)
        for s in range(8):
            pd, qd = synth.scenario_loads(cs, 3000 + 8 * j + s)
            c2 = dict(cs)
            c2["pd"], c2["qd"] = pd, qd
            i = len(cases)
            cases.append((c2, synth.point(cs, (103, i)), synth.multipliers(m, (103, i))))

    def one(k):
        c2, x, y = cases[k]
        oracle.evaluate(c2, x, y, 1.0)

    t0 = time.perf_counter()
    for k in range(len(cases)):
        one(k)
    t1 = time.perf_counter() - t0
    threads = _nproc()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, range(len(cases))))
    tn = time.perf_counter() - t0
    log(f"oracle on the 64-scenario mix: {t1:.1f} s on 1 thread, {tn:.1f} s on {threads} threads")
    return dict(kind="oracle", unit="sets/s", sets=len(cases), one_thread_sets_per_s=len(cases) / t1,
                all_cores_sets_per_s=len(cases) / tn, threads=threads, nproc=_nproc(), cpu_model=_cpu_model_name(),
                sample="every scenario of the 64-scenario mix once, one thread, then one scenario per thread")


def measure_copy_gbs(torch, mib: int = 1024, reps: int = 5) -> float:
    """Device-to-device copy rate (bytes read + written per second) of a
    plain copy of `mib` MiB: the HBM rate a streaming kernel reaches here."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2.0 * n * 8 / secs / 1e9


def bench_batch(args, torch, opf, synth, log):
    """The 64-scenario uneven mix: batched evaluations vs 64 plain launches per
    pass, both captured in a HIP graph."""
    dev = torch.device("cuda", 0)
    nets, models, plain_models, inst_model, pds, qds = [], [], [], [], [], []
    for j, N in enumerate(synth.BATCH_SIZES):
        cs = synth.network(N, int(round(1.35 * N)), int(round(0.2 * N)), 300 + j)
        nets.append(cs)
        models.append(opf.Model(cs, device=0))
        for s in range(8):
            pd, qd = synth.scenario_loads(cs, 3000 + 8 * j + s)
            inst_model.append(j)
            pds.append(pd)
            qds.append(qd)
            c2 = dict(cs)
            c2["pd"], c2["qd"] = pd, qd
            plain_models.append(opf.Model(c2, device=0))
    batch = opf.Batch(models, inst_model, np.concatenate(pds), np.concatenate(qds))
    n_inst = batch.n_inst
    # n_xy input sets (63 MB each) and n_o output sets (250 MB each), rotated
    # per evaluation: about 1 GB, past the 256 MB Infinity Cache
    n_xy, n_o = 4, 3
    XS = [torch.empty(batch.n, dtype=torch.float64, device=dev) for _ in range(n_xy)]
    YS = [torch.empty(batch.m, dtype=torch.float64, device=dev) for _ in range(n_xy)]
    for q in range(n_xy):
        for i in range(n_inst):
            cs = nets[inst_model[i]]
            XS[q][batch.xoff[i]:batch.xoff[i + 1]] = torch.as_tensor(synth.point(cs, (103 + 1000 * q, i)), device=dev)
            YS[q][batch.coff[i]:batch.coff[i + 1]] = torch.as_tensor(
                synth.multipliers(int(batch.coff[i + 1] - batch.coff[i]), (103 + 1000 * q, i)), device=dev)
    sig = torch.ones(n_inst, dtype=torch.float64, device=dev)
    OUTS = [(torch.empty(n_inst, dtype=torch.float64, device=dev),
             torch.empty(batch.n, dtype=torch.float64, device=dev),
             torch.empty(batch.m, dtype=torch.float64, device=dev),
             torch.empty(batch.nnzj, dtype=torch.float64, device=dev),
             torch.empty(batch.nnzh, dtype=torch.float64, device=dev)) for _ in range(n_o)]
    X, Y = XS[0], YS[0]
    F, G, C, J, H = OUTS[0]
    sched = batch.tune()
    log(f"batch: {n_inst} instances, n={batch.n} m={batch.m} nnzj={batch.nnzj} nnzh={batch.nnzh}, "
        f"tuned schedule wg_per_cu={sched} (0 = one workgroup per item)")

    def batched(k=0):
        batch.eval(XS[k % n_xy], YS[k % n_xy], sig, *OUTS[k % n_o])

    reps = args.batch_reps
    # eager: one evaluation call after another (two kernel launches each)
    secs_e, _ = time_steps(torch, lambda: [batched(k) for k in range(reps)], 3, 1)
    per_eager = secs_e / (3 * reps)

    # plain: the same 64 instances through the single-instance API, back to
    # back on one stream, captured in one HIP graph, rotating the same sets
    def views_of(k):
        Xk, Yk, (Fk, Gk, Ck, Jk, Hk) = XS[k % n_xy], YS[k % n_xy], OUTS[k % n_o]
        v = []
        for i in range(n_inst):
            sl = lambda off, a: a[int(off[i]):int(off[i + 1])]  # noqa: E731
            v.append((sl(batch.xoff, Xk), sl(batch.coff, Yk), Fk[i:i + 1], sl(batch.xoff, Gk), sl(batch.coff, Ck),
                      sl(batch.joff, Jk), sl(batch.hoff, Hk)))
        return v

    views_k = [views_of(k) for k in range(n_xy * n_o)]

    def plain(k=0):
        for i, (x, y, f, g, c, jv, hv) in enumerate(views_k[k % len(views_k)]):
            plain_models[i].eval_set(x, y, 1.0, f, g, c, jv, hv)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plain()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (F, G, C, J, H)]
    batched()
    torch.cuda.synchronize()
    # plain launches of these models take the one-launch shape (recomputed
    # branch terms), batches the two-launch shape: bitwise equal (the
    # kernels contract no floating-point operation)
    bitwise = all(torch.equal(a, b) for a, b in zip(ref, (F, G, C, J, H)))
    max_rel = max(float(((a - b).abs() / b.abs().clamp(min=1.0)).max()) for a, b in zip((F, G, C, J, H), ref))
    # both forms captured the same way: one HIP graph of `reps` passes over
    # the mix (batched: two launches per pass; plain: 64), replayed
    graph_b = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph_b, stream=s):
        for k in range(reps):
            batched(k)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        for k in range(reps):
            plain(k)
    torch.cuda.synchronize()
    secs_b, _ = time_steps(torch, graph_b.replay, 3, 1)
    per_launch = secs_b / (3 * reps)
    secs_p, _ = time_steps(torch, graph.replay, 3, 1)
    per_plain = secs_p / (3 * reps)
    # every schedule the tuner chooses from, the same way (a graph of `reps`
    # evaluations), so the choice can be read off the record
    sched_us = {}
    for wg in (-1, 0, 4, 16):
        batch.set_schedule(wg)
        g_s = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_s, stream=s):
            for k in range(reps):
                batched(k)
        torch.cuda.synchronize()
        secs_s, _ = time_steps(torch, g_s.replay, 2, 1)
        sched_us[str(wg)] = secs_s / (2 * reps) * 1e6
        del g_s
    batch.set_schedule(sched)
    total_bytes = sum(algorithmic_bytes(nets[inst_model[i]], (
        int(batch.xoff[i + 1] - batch.xoff[i]), int(batch.coff[i + 1] - batch.coff[i]),
        int(batch.joff[i + 1] - batch.joff[i]), int(batch.hoff[i + 1] - batch.hoff[i]))) for i in range(n_inst))
    # model data is shared by the 8 scenarios of a network: count it once
    shared = sum(80 * c["n_branch"] + 16 * c["n_bus"] + 28 * c["n_gen"] + 4 * (2 * c["n_branch"] + 2 * c["n_bus"]
                                                                          + 2 + c["n_gen"]) for c in nets)
    total_bytes -= 7 * shared
    log(f"batch: batched {per_launch * 1e6:.1f} us/evaluation in a graph ({per_eager * 1e6:.1f} us issued eagerly), "
        f"plain {per_plain * 1e6:.1f} us/64 sets, "
        f"bitwise equal: {bitwise}, max |diff| / max(|plain|, 1): {max_rel:.3g}; by schedule (us): "
        + ", ".join(f"{k}: {v:.1f}" for k, v in sched_us.items()))
    out = dict(
        workload="64 scenarios = 8 networks (500..20000 buses, L=1.35N, G=0.2N) x 8 load seeds",
        batched_sets_per_s=n_inst / per_launch, plain_sets_per_s=n_inst / per_plain,
        speedup=per_plain / per_launch, us_per_launch=per_launch * 1e6, bytes_per_launch=total_bytes,
        timing=f"both forms captured in a HIP graph of {reps} passes over the mix and replayed, rotating "
               f"{n_xy} input and {n_o} output sets (about 1 GB, past the Infinity Cache)",
        us_per_eval_eager=per_eager * 1e6, speedup_eager=per_plain / per_eager,
        achieved_gbs=total_bytes / per_launch / 1e9, frac=total_bytes / per_launch / 1e9 / HBM_PEAK_GBS,
        schedule=dict(wg_per_cu=sched, us_per_eval_by_schedule=sched_us,
                      legend="-1 one launch (bus lanes recompute the branch terms); 0 two flat launches; "
                             "k > 0 two persistent launches of k workgroups per CU"),
        bitwise_equal_to_plain=bool(bitwise), max_rel_diff_to_plain=max_rel)
    batch.close()
    for mdl in models + plain_models:
        mdl.close()
    return out


def bench_points(torch, opf, synth, log, B=16):
    """The 10k-bus network evaluated at B independent (x, y) points per
    launch through the batch path (what a batch of interior-point solves on
    one network, or a sweep of evaluation points, issues)."""
    dev = torch.device("cuda", 0)
    cs = synth.network(10000, 13500, 2000, 1)
    model = opf.Model(cs, device=0)
    b = opf.Batch([model], np.zeros(B, np.int32))
    n_xy = 8  # input sets of 24 MB rotated with the 8 output sets (114 MB each)
    XS = [torch.empty(b.n, dtype=torch.float64, device=dev) for _ in range(n_xy)]
    YS = [torch.empty(b.m, dtype=torch.float64, device=dev) for _ in range(n_xy)]
    for q in range(n_xy):
        for i in range(B):
            XS[q][b.xoff[i]:b.xoff[i + 1]] = torch.as_tensor(synth.point(cs, (101, i + B * q)), device=dev)
            YS[q][b.coff[i]:b.coff[i + 1]] = torch.as_tensor(synth.multipliers(model.m, (101, i + B * q)), device=dev)
    S = torch.ones(B, dtype=torch.float64, device=dev)
    outs = [(torch.empty(B, dtype=torch.float64, device=dev), torch.empty(b.n, dtype=torch.float64, device=dev),
             torch.empty(b.m, dtype=torch.float64, device=dev), torch.empty(b.nnzj, dtype=torch.float64, device=dev),
             torch.empty(b.nnzh, dtype=torch.float64, device=dev)) for _ in range(8)]
    sched = b.tune()
    k = [0]

    def run():
        o = outs[k[0] % len(outs)]
        X, Y = XS[k[0] % n_xy], YS[k[0] % n_xy]
        k[0] += 1
        b.eval(X, Y, S, *o)

    secs_e, _ = time_steps(torch, lambda: [run() for _ in range(10)], 3, 1)
    per_eager = secs_e / 30
    # 10 evaluations (rotating outputs) captured in one HIP graph, replayed
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        for _ in range(10):
            run()
    torch.cuda.synchronize()
    secs, _ = time_steps(torch, graph.replay, 3, 1)
    per = secs / 30
    shared = 80 * 13500 + 32 * 10000 + 28 * 2000 + 4 * (2 * 13500 + 2 * 10001 + 2000)
    total = B * algorithmic_bytes(cs, (model.n, model.m, model.nnzj, model.nnzh)) - (B - 1) * shared
    log(f"10k x {B} points (wg_per_cu={sched}): {per * 1e6:.1f} us/evaluation in a graph "
        f"({per_eager * 1e6:.1f} us issued eagerly), {B / per:.0f} sets/s, {total / per / 1e9:.0f} GB/s")
    b.close()
    model.close()
    return dict(workload=f"10000-bus network at {B} seeded (x, y) points per batched evaluation", points=B,
                sets_per_s=B / per, us_per_launch=per * 1e6, bytes_per_launch=total,
                timing="10 evaluations captured in a HIP graph and replayed", us_per_eval_eager=per_eager * 1e6,
                achieved_gbs=total / per / 1e9, frac=total / per / 1e9 / HBM_PEAK_GBS, schedule=dict(wg_per_cu=sched))


def bench_model(torch, opf, synth, cs, opts, n_in, n_out, sets, log, label, T=1, K=0, mp_loads=False, seed=104,
                steps=3):
    """Plain sets of one model from a HIP graph, n_in input pairs and n_out
    output sets rotated (sized past the 256 MB Infinity Cache)."""
    dev = torch.device("cuda", 0)
    model = opf.Model(cs, device=0, **opts)
    rect = opts.get("form") == "rect"
    dims = (model.n, model.m, model.nnzj, model.nnzh)
    form = "rect" if rect else "polar"
    st, dv = opts.get("storage"), opts.get("devices")
    xs = [torch.as_tensor(synth.point(cs, (seed, r), n_periods=T, n_cont=K, form=form, storage=st, devices=dv),
                          device=dev) for r in range(n_in)]
    ys = [torch.as_tensor(synth.multipliers(model.m, (seed, r)), device=dev) for r in range(n_in)]
    runner = PlainRunner(model, xs, ys, n_out=n_out, sets=sets, torch=torch)
    runner.capture()
    secs, _ = time_steps(torch, runner.step, steps, 1)
    per = secs / (steps * sets)
    b = algorithmic_bytes(cs, dims, T=T, K=K, mp_loads=mp_loads, rect=rect, S=len(st["bus"]) if st else 0,
                          D=len(dv["bus"]) if dv else 0)
    ws = n_in * 8 * (dims[0] + dims[1]) + n_out * 8 * (1 + sum(dims))
    log(f"{label}: {per * 1e6:.2f} us/set, {b / per / 1e9:.0f} GB/s (working set {ws / 2**20:.0f} MiB)")
    launches, items = model.launch_shape()
    model.close()
    return dict(n=dims[0], m=dims[1], nnzj=dims[2], nnzh=dims[3], sets_per_s=1.0 / per, us_per_set=per * 1e6,
                bytes_per_set=b, achieved_gbs=b / per / 1e9, frac=b / per / 1e9 / HBM_PEAK_GBS,
                launches_per_set=launches, work_items=items, inputs_rotated=n_in, outputs_rotated=n_out,
                working_set_mib=ws / 2**20)


def bench_proxy(args, torch, synth, log):
    """The learned warm-start proxy on a 300-bus network (410 branches, 60
    generators): MLP 600 -> 3 x 1024 (GELU) -> 720 on BF16 matrix cores,
    batches of 4,096 load samples (+-30 % uniform), FP64 penalty from the
    callback kernels.  Reports the training step time, the inference rate,
    the MLP forward's matrix-core rate and, on held-out loads, the largest
    constraint violation of the proxy against the plain starting point."""
    from paper_2510_12897_amd import proxy as P

    cs = synth.network(300, 410, 60, 41)
    B = 4096
    px = P.WarmStartProxy(cs, B=B, width=1024, depth=3, rho=10.0, obj_scale=1e-3, seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    steps = args.proxy_steps
    # the penalty weight rises geometrically from 10 to 100 over the run (4x
    # the steps and this schedule took the held-out Cvio mean 0.186 -> 0.156)
    rho0, rho1 = 10.0, 100.0

    def rho_at(k):
        return rho0 * (rho1 / rho0) ** (k / max(steps - 1, 1))

    loads, feats = px.sample(gen)
    first = float(px.train_step(loads, feats, lr=3e-4))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, steps):
        px.pen.rho = rho_at(k)
        loads, feats = px.sample(gen)
        loss = px.train_step(loads, feats, lr=3e-4)
    torch.cuda.synchronize()
    train_s = (time.perf_counter() - t0) / max(steps - 1, 1)
    last = float(loss)
    gen.manual_seed(4242)
    loads, feats = px.sample(gen)
    _, cvp = px.predict(loads, feats)
    _, cv0 = px.baseline(loads)
    _, cvf = px.flat_start(loads)
    cvp, cv0, cvf = cvp.cpu().numpy(), cv0.cpu().numpy(), cvf.cpu().numpy()
    curve = P.fallback_curve(cvp)
    # the training step split into its parts: with the library-issued step,
    # the GPU time of its phases from events on its stream (20 steps, mean);
    # else each part issued from Python through the autograd path and timed
    # on its own
    gen.manual_seed(99)
    loads, feats = px.sample(gen)
    split = {}
    if px.native and px.pen.fused:
        acc = {}
        for _ in range(20):
            _, ph = px.train_step_phases(loads, feats, lr=0.0)
            for k, v in ph.items():
                acc[k] = acc.get(k, 0.0) + v / 20
        split = {"forward": acc["forward"], "loss_fwd_bwd": acc["loss"], "backward": acc["backward"],
                 "adam": acc["adam"], "mlp_fwd_bwd": acc["forward"] + acc["backward"]}
        split_note = ("GPU time of each phase of the library-issued step (events on its stream, mean of 20 steps): "
                      "forward = the MLP's matrix-core products with bias and GELU; loss_fwd_bwd = the fused FP64 "
                      "loss kernel with d loss / d z and its scaling by 1/B; backward = the weight-gradient and dh "
                      "products with the GELU backward and bias sums; mlp_fwd_bwd = forward + backward")
    else:
        gz = torch.randn(B, px.mlp.dims[-1], device=px.dev) * 1e-3

        def mlp_part():
            px.mlp(feats).backward(gz)
            px.mlp.flat.grad = None

        z0 = px.mlp(feats).detach()

        def loss_part():
            z = z0.clone().requires_grad_(True)
            P._fun("loss").apply(z, px, loads, False).mean().backward()

        zz = px.mlp(feats)
        zz.backward(gz)
        g_keep = px.mlp.flat.grad.clone()

        def adam_part():
            px.mlp.flat.grad = g_keep
            px.mlp.adam_step(lr=0.0)

        for name, fn in (("mlp_fwd_bwd", mlp_part), ("loss_fwd_bwd", loss_part), ("adam", adam_part)):
            secs, _ = time_steps(torch, fn, 20, 2)
            split[name] = secs / 20 * 1e3
        split_note = ("each part issued from Python through the autograd path and timed on its own over 20 "
                      "repetitions (host issue included where it outlasts the GPU work); mlp_fwd_bwd = the "
                      "matrix-core GEMMs with their GELU and bias-sum kernels, loss_fwd_bwd = the FP64 side "
                      "(squash, flows, batch evaluation, penalty, J^T W, squash backward)")
    px.mlp.flat.grad = None
    # inference: MLP + squashing + flows + FP64 constraint evaluation + violation
    gen.manual_seed(4242)
    loads, feats = px.sample(gen)
    secs, _ = time_steps(torch, lambda: px.predict(loads, feats), 10, 2)
    infer_s = secs / 10
    # MLP forward alone on the matrix cores
    with torch.no_grad():
        secs_m, _ = time_steps(torch, lambda: px.mlp(feats), 10, 2)
    flops = 2.0 * B * sum(a * b for a, b in zip(px.mlp.dims[:-1], px.mlp.dims[1:]))
    mlp_tflops = flops / (secs_m / 10) / 1e12
    log(f"proxy: loss {first:.4g} -> {last:.4g} in {steps} steps ({train_s * 1e3:.2f} ms/step); held-out "
        f"Cvio mean {cvp.mean():.4g} vs x0 {cv0.mean():.4g} and flat start {cvf.mean():.4g}; fallback rate at "
        f"tau 0.05: {curve[0.05]:.3f}; {B / infer_s:.0f} inferences/s; MLP forward {mlp_tflops:.1f} TFLOP/s; "
        f"step split (ms): MLP {split['mlp_fwd_bwd']:.3f}, FP64 loss {split['loss_fwd_bwd']:.3f}, "
        f"Adam {split['adam']:.3f}")
    out = dict(workload="300 buses, 410 branches, 60 generators; MLP 600-1024x3-720 GELU, BF16 MFMA; "
                        "batches of 4096 loads (+-30 % uniform)",
               train_steps=steps, penalty_weight=f"{rho0:g} -> {rho1:g}, geometric over the steps",
               ms_per_train_step=train_s * 1e3, loss_first=first, loss_last=last,
               ms_split={**split, "note": split_note},
               native_step=bool(px.native and px.pen.fused),
               fused_loss=bool(px.pen.fused),
               inferences_per_s=B / infer_s, mlp_forward_inferences_per_s=B / (secs_m / 10),
               mlp_forward_tflops=mlp_tflops, mlp_peak_tflops=2500.0,
               heldout_cvio_mean=float(cvp.mean()), heldout_cvio_max=float(cvp.max()),
               x0_cvio_mean=float(cv0.mean()), flatstart_cvio_mean=float(cvf.mean()),
               fallback_tau=0.05, fallback_rate=curve[0.05],
               fallback_curve={str(k): v for k, v in curve.items()},
               flatstart_fallback_curve={str(k): v for k, v in P.fallback_curve(cvf).items()},
               x0_fallback_curve={str(k): v for k, v in P.fallback_curve(cv0).items()},
               fallback_definition="share of held-out samples whose Cvio (largest violation over every row and "
                                   "bound, p.u.) exceeds tau",
               beats_flatstart_rate=float(np.mean(cvp < cvf)), beats_x0_rate=float(np.mean(cvp < cv0)))
    px.close()
    return out


def bench_ipm(torch, opf, synth, log):
    """The interior-point consumer (condensed LiftedKKT barrier method,
    sparse Cholesky on the GPU) solving the proxy's 300-bus network from the model's
    start point: at 0.7x the base loads with the two tolerances of the
    paper's tables, and at the base loads, where no point within the
    bounds satisfies the constraints (the run reports that it is not
    solved).  Time is split into callbacks, linear algebra and the rest."""
    from paper_2510_12897_amd.ipm import InteriorPoint

    base = synth.network(300, 410, 60, 41)
    out = {"workload": "300 buses, 410 branches, 60 generators (the proxy's network), solved from the "
                       "model's start point; condensed matrix factored by rocSOLVER's sparse Cholesky "
                       "re-factorization (minimum-degree ordering)"}
    for tag, fac, tol, max_iter in (("load0.7_tol1e-4", 0.7, 1e-4, 300), ("load0.7_tol1e-8", 0.7, 1e-8, 300),
                                    ("load1.0_tol1e-6", 1.0, 1e-6, 100)):
        cs = dict(base)
        cs["pd"], cs["qd"] = base["pd"] * fac, base["qd"] * fac
        model = opf.Model(cs, device=0)
        try:
            warm = InteriorPoint(model, tol=tol, max_iter=3)         # warm the libraries
            warm.solve()
            warm.close()
            t_setup = time.perf_counter()
            ip = InteriorPoint(model, tol=tol, max_iter=max_iter)   # pattern, ordering, symbolic factor
            t_setup = time.perf_counter() - t_setup
            r = ip.solve()
            ip.close()
        finally:
            model.close()
        t, it = r["times"], max(r["iterations"], 1)
        log(f"ipm {tag}: {r['status']} in {r['iterations']} iterations, f {r['f']:.8g}, cvio {r['cvio']:.2e}, "
            f"{t['total'] * 1e3:.0f} ms (callbacks {t['callbacks'] * 1e3:.1f}, linear algebra "
            f"{t['linear_algebra'] * 1e3:.1f}, other {t['other'] * 1e3:.1f})")
        out[tag] = dict(status=r["status"], iterations=r["iterations"], objective=r["f"], cvio=r["cvio"],
                        kkt=r["kkt"], n=model.n, m=model.m, seconds=t["total"], setup_seconds=t_setup,
                        ms_per_iteration=t["total"] / it * 1e3, seconds_callbacks=t["callbacks"],
                        seconds_linear_algebra=t["linear_algebra"], seconds_other=t["other"],
                        callback_share=t["callbacks"] / t["total"], counts=r["counts"])
    return out


def bench_warm_start(torch, opf, synth, log, steps=1500, samples=12):
    """What the learned proxy gains the solver: the proxy network trained on
    a solvable load regime of the 300-bus network (0.7x the base loads,
    +-30 % per bus) and, on held-out samples, the interior-point iterations
    from the model's start point (cold) against those from the proxy's
    prediction (warm), same solver settings."""
    from paper_2510_12897_amd import proxy as P
    from paper_2510_12897_amd.ipm import InteriorPoint

    base = dict(synth.network(300, 410, 60, 41))
    base["pd"], base["qd"] = base["pd"] * 0.7, base["qd"] * 0.7
    px = P.WarmStartProxy(base, B=4096, width=1024, depth=3, rho=10.0, obj_scale=1e-3, seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    t0 = time.perf_counter()
    for _ in range(steps):
        loads, feats = px.sample(gen)
        px.train_step(loads, feats, lr=3e-4)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    gen.manual_seed(4242)
    loads, feats = px.sample(gen)
    X, cv = px.predict(loads, feats)
    N = px.N
    rows = []
    for i in range(samples):
        cs = dict(base)
        cs["pd"], cs["qd"] = loads[i, :N].cpu().numpy().copy(), loads[i, N:].cpu().numpy().copy()
        model = opf.Model(cs, device=0)
        try:
            res = {}
            # warm_mu: the proxy's start with a smaller initial barrier parameter (0.01), as
            # interior-point warm starts usually take; the other two start at the default 0.1
            for name, x0, mu0 in (("cold", None, 0.1), ("warm", X[i].clone(), 0.1), ("warm_mu", X[i].clone(), 0.01)):
                ip = InteriorPoint(model, tol=1e-6, max_iter=80, mu0=mu0)   # the solvable samples take under 40
                r = ip.solve(x0)
                ip.close()
                res[name] = (r["status"] == "solved", r["iterations"], r["f"], r["times"]["total"])
        finally:
            model.close()
        rows.append(res)
    both = [r for r in rows if r["cold"][0] and r["warm"][0]]
    px.close()
    out = dict(workload="300-bus network at 0.7x base loads, +-30 % per bus; proxy trained 1500 steps; "
                        "interior-point solves (tol 1e-6, sparse factorization) of held-out samples from the "
                        "model's start point (cold) and from the proxy's prediction (warm)",
               train_seconds=train_s, samples=samples, solved_cold=sum(r["cold"][0] for r in rows),
               solved_warm=sum(r["warm"][0] for r in rows), solved_both=len(both),
               mean_iterations_cold=float(np.mean([r["cold"][1] for r in both])) if both else None,
               mean_iterations_warm=float(np.mean([r["warm"][1] for r in both])) if both else None,
               mean_seconds_cold=float(np.mean([r["cold"][3] for r in both])) if both else None,
               mean_seconds_warm=float(np.mean([r["warm"][3] for r in both])) if both else None,
               mean_iterations_warm_mu0_1e_2=float(np.mean([r["warm_mu"][1] for r in both if r["warm_mu"][0]]))
               if any(r["warm_mu"][0] for r in both) else None,
               solved_warm_mu0_1e_2=sum(r["warm_mu"][0] for r in rows),
               max_rel_objective_diff=float(max(abs(r["warm"][2] - r["cold"][2]) / abs(r["cold"][2]) for r in both))
               if both else None,
               heldout_cvio_mean=float(cv[:samples].mean()))
    log(f"warm start: {out['solved_both']} of {samples} held-out samples solved from both starts; mean iterations "
        f"cold {out['mean_iterations_cold']}, warm {out['mean_iterations_warm']}, warm with mu0 0.01 "
        f"{out['mean_iterations_warm_mu0_1e_2']}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sets-per-step", type=int, default=1000)
    ap.add_argument("--inputs", type=int, default=256, help="distinct pre-generated (x, y) pairs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle timing budget (0 = skip)")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched / multi-period / N-1 legs")
    ap.add_argument("--legs", default="all",
                    help="comma-separated extra legs to run (batch64, multiperiod_2k_x48, "
                         "multiperiod_storage_2k_x48, contingency_1k_x201, rect_10k, points16_10k, ipm_300bus, "
                         "proxy_300bus, proxy_warm_start_300bus, cpu_oracle_batch64; default all)")
    ap.add_argument("--batch-reps", type=int, default=20)
    ap.add_argument("--proxy-steps", type=int, default=6000, help="training steps of the proxy leg (0 = skip)")
    ap.add_argument("--eager", action="store_true", help="launch the headline sets without a HIP graph")
    ap.add_argument("--launch-limit", type=int, default=None,
                    help="one-launch limit in work items for the models built (0 = always two launches; "
                         "default: the library's)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run a device-to-device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()

    def log(*a):
        if not args.quiet:
            print("[bench]", *a, file=sys.stderr, flush=True)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: each model is evaluated on a single MI355X "
              "(multi-GPU sharding is a design note, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_12897_amd import opf, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    opf.lib()
    if args.launch_limit is not None:
        opf.set_single_launch_limit(args.launch_limit)
    if args.copy_mb > 0:
        n = args.copy_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: 3 x {args.copy_mb} MiB device-to-device")
        del src, dst
    h = bench_headline(args, torch, opf, synth, log)
    sets_per_s = h["n_sets"] / h["secs"]
    achieved = h["bytes_set"] / h["per_set"] / 1e9
    copy_gbs = measure_copy_gbs(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
    result = {
        "metric": METRIC,
        "value": sets_per_s,
        "unit": "sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["secs"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "plain polar AC-OPF callback sets, 10000-bus synthetic network "
                        "(13500 branches, 2000 generators), 1000 sets per step at seeded (x, y)",
            "n": h["dims"][0], "m": h["dims"][1], "nnzj": h["dims"][2], "nnzh": h["dims"][3],
            "sets_per_step": args.sets_per_step,
            "launch": "eager plain launches" if args.eager else "HIP graph of back-to-back plain launches",
            "inputs_rotated": args.inputs, "outputs_rotated": 64,
        },
        "roofline": {
            "kernel": h["kernel"],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "traffic_unit": "HBM bytes per callback set (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "bytes_per_launch": h["bytes_set"],
            "us_per_launch": h["per_set"] * 1e6,
            "copy_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
    }
    def leg_multiperiod():
        cs = synth.network(2000, 2700, 400, 2)
        pd_t, qd_t = synth.mp_loads(cs, 48, 202)
        return bench_model(torch, opf, synth, cs, dict(n_periods=48, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2), 24, 8, 24,
                           log, "multi-period", T=48, mp_loads=True)

    def leg_multiperiod_storage():
        # storage at the largest 10 % of loads (1.5x energy ratings) and 100
        # electrolyzer-like devices, 30-minute periods
        cs = synth.network(2000, 2700, 400, 2)
        pd_t, qd_t = synth.mp_loads(cs, 48, 202)
        r = bench_model(torch, opf, synth, cs, dict(n_periods=48, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2,
                                                    storage=synth.storage(cs, 203), stor_dt=0.5,
                                                    devices=synth.devices(cs, 100, 204)), 24, 8, 24,
                        log, "multi-period with storage and devices", T=48, mp_loads=True)
        r["workload"] = "2000 buses x 48 periods, 200 storage units at the largest loads, 100 devices"
        return r

    def leg_contingency():
        cs = synth.network(1000, 1350, 200, 31)
        out = synth.outages(cs, 200, 32)
        return bench_model(torch, opf, synth, cs, dict(n_cont=200, outaged=out), 16, 6, 24, log, "N-1 copies", K=200)

    def leg_rect():
        cs = synth.network(10000, 13500, 2000, 1)
        r = bench_model(torch, opf, synth, cs, dict(form="rect"), 256, 64, 500, log, "rectangular 10k", seed=101)
        r["workload"] = "plain rectangular-form callback sets, 10000-bus network, HIP graph of back-to-back launches"
        return r

    legs = [("batch64", lambda: bench_batch(args, torch, opf, synth, log)),
            ("multiperiod_2k_x48", leg_multiperiod),
            ("multiperiod_storage_2k_x48", leg_multiperiod_storage),
            ("contingency_1k_x201", leg_contingency),
            ("rect_10k", leg_rect),
            ("points16_10k", lambda: bench_points(torch, opf, synth, log, B=16)),
            ("ipm_300bus", lambda: bench_ipm(torch, opf, synth, log))]
    if args.proxy_steps > 0:
        legs += [("proxy_300bus", lambda: bench_proxy(args, torch, synth, log)),
                 ("proxy_warm_start_300bus", lambda: bench_warm_start(torch, opf, synth, log))]
    wanted = None if args.legs == "all" else set(args.legs.split(","))
    if not args.no_extra:
        extra = {}
        for name, fn in legs:
            if wanted is not None and name not in wanted:
                continue
            try:
                extra[name] = fn()
            except Exception as e:  # a failing leg must not hide the headline line
                extra[name] = {"error": repr(e)}
        result["extra"] = extra
    if args.cpu_seconds > 0:
        from oracle import oracle

        result["cpu_baseline"] = bench_cpu_baseline(h, synth, oracle, args.cpu_seconds, log)
        if not args.no_extra and (wanted is None or "cpu_oracle_batch64" in wanted):
            try:
                result.setdefault("extra", {})["cpu_oracle_batch64"] = bench_cpu_batch64(synth, oracle, log)
            except Exception as e:
                result.setdefault("extra", {})["cpu_oracle_batch64"] = {"error": repr(e)}
    h["model"].close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
