"""The entry point that allocates nothing (opf_eval_set_noalloc) against
opf_eval_set: same kernels, so every output must be bitwise equal.  Two
calls in a row share the library's fixed scratch array, the second on a
smaller model, in both launch shapes; a model whose scratch exceeds the
array is refused with OPF_E_ARG."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2510_12897_amd import opf, synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _outputs(model, fill):
    return [torch.full((k,), fill, dtype=torch.float64, device=DEV)
            for k in (1, model.n, model.m, model.nnzj, model.nnzh)]


def _call(fn, model, x, y, sigma, outs):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(model.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), ctypes.c_double(sigma),
            *[ctypes.c_void_p(t.data_ptr()) for t in outs], stream)
    if rc != 0:
        raise opf.OPFError(rc, opf.lib().opf_last_error().decode())


def _point(model, cs, seed, **opts):
    x = torch.as_tensor(synth.point(cs, seed, **opts), device=DEV)
    y = torch.as_tensor(synth.multipliers(model.m, seed), device=DEV)
    return x, y


@pytest.mark.parametrize("limit", [4096, 0], ids=["one_launch", "two_launch"])
def test_noalloc_matches_eval_set_twice(limit):
    lib = opf.lib()
    opf.set_single_launch_limit(limit)
    try:
        big = synth.network(2000, 2700, 400, 41, variant=True)
        small = synth.network(300, 410, 60, 42, variant=True)
        pd_t, qd_t = synth.mp_loads(small, 3, 7)
        mopts = dict(n_periods=3, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2)
        cases = [("2000-bus", big, {}), ("300-bus x 3 periods", small, mopts)]
        for k, (name, cs, opts) in enumerate(cases):
            say(f"[noalloc] limit={limit} call {k + 1}: {name}")
            model = opf.Model(cs, device=0, **opts)
            x, y = _point(model, cs, 500 + k, **({"n_periods": opts["n_periods"]} if opts else {}))
            ref = _outputs(model, np.nan)
            got = _outputs(model, -7.0)
            _call(lib.opf_eval_set, model, x, y, 0.75, ref)
            _call(lib.opf_eval_set_noalloc, model, x, y, 0.75, got)
            torch.cuda.synchronize()
            for tag, a, b in zip(("f", "g", "c", "J", "H"), got, ref):
                assert torch.equal(a, b), f"{name}: {tag} differs from opf_eval_set"
            model.close()
    finally:
        opf.set_single_launch_limit(4096)


def test_noalloc_rejects_oversized_model():
    cs = synth.network(1000, 1350, 200, 43)
    say("[noalloc] 1000-bus model with 300 contingency copies (scratch beyond the fixed array)")
    model = opf.Model(cs, device=0, n_cont=300, outaged=synth.outages(cs, 300, 44))
    x, y = _point(model, cs, 510, n_cont=300)
    outs = _outputs(model, 0.0)
    with pytest.raises(opf.OPFError) as ei:
        _call(opf.lib().opf_eval_set_noalloc, model, x, y, 1.0, outs)
    assert ei.value.code == opf.OPF_E_ARG and "scratch" in str(ei.value)
    model.close()
