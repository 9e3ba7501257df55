"""The interior-point consumer driven by the HIP callbacks on the GPU,
against the same solver driven by the oracle on the CPU."""
from __future__ import annotations

import numpy as np
import pytest

from helpers import case0
from ipm_models import OracleModel
from paper_2510_12897_amd import opf, synth
from paper_2510_12897_amd.ipm import InteriorPoint

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _pair(case, tol, **opts):
    m = opf.Model(case, 0, **opts)
    try:
        rg = InteriorPoint(m, tol=tol).solve()
    finally:
        m.close()
    rc = InteriorPoint(OracleModel(case, **opts), tol=tol).solve()
    say(f"[ipm] gpu {rg['status']} it {rg['iterations']} f {rg['f']:.12g} | "
        f"cpu {rc['status']} it {rc['iterations']} f {rc['f']:.12g}")
    return rg, rc


@pytest.mark.parametrize("form", ["polar", "rect"])
def test_14_bus_solve_matches_the_oracle_driven_solve(form):
    rg, rc = _pair(case0(), 1e-8, form=form)
    assert rg["status"] == rc["status"] == "solved"
    assert abs(rg["f"] - rc["f"]) <= 1e-9 * abs(rc["f"])
    np.testing.assert_allclose(rg["x"].cpu().numpy(), rc["x"].numpy(), atol=1e-6)
    assert rg["cvio"] <= 1.01e-8


def test_300_bus_at_reduced_load_solves():
    case = dict(synth.network(300, 410, 60, 4))
    case["pd"], case["qd"] = case["pd"] * 0.7, case["qd"] * 0.7
    rg, rc = _pair(case, 1e-6)
    assert rg["status"] == rc["status"] == "solved"
    assert abs(rg["f"] - rc["f"]) <= 1e-7 * abs(rc["f"])
    assert rg["cvio"] <= 1.01e-6
    t = rg["times"]
    say(f"[ipm] 300-bus: {rg['iterations']} iterations, callbacks {t['callbacks']:.3f} s, "
        f"linear algebra {t['linear_algebra']:.3f} s, other {t['other']:.3f} s")


def test_multiperiod_storage_solve_matches():
    case = case0()
    pd, qd = synth.mp_loads(case, 4, 3)
    opts = dict(n_periods=4, pd_t=pd, qd_t=qd, ramp_ratio=0.2, storage=synth.storage(case, 5, frac=0.3))
    rg, rc = _pair(case, 1e-6, **opts)
    assert rg["status"] == rc["status"] == "solved"
    assert abs(rg["f"] - rc["f"]) <= 1e-7 * abs(rc["f"])


def test_solve_repeats_bit_for_bit():
    """Every reduction of the solver goes through the fixed pattern in a
    fixed order (no atomics): two solves take the same iterations and end
    at the same point, bit for bit."""
    case = dict(synth.network(300, 410, 60, 41))
    case["pd"], case["qd"] = case["pd"] * 0.7, case["qd"] * 0.7
    m = opf.Model(case, 0)
    try:
        r1 = InteriorPoint(m, tol=1e-8).solve()
        r2 = InteriorPoint(m, tol=1e-8).solve()
    finally:
        m.close()
    say(f"[ipm] repeat: {r1['status']} {r1['iterations']} / {r2['status']} {r2['iterations']}")
    assert r1["status"] == r2["status"] == "solved"
    assert r1["iterations"] == r2["iterations"]
    assert r1["f"] == r2["f"]
    assert bool((r1["x"] == r2["x"]).all())


def _ipm_pattern(case):
    """The condensed matrix's pattern of a model: Hessian plus J^T J."""
    m = opf.Model(case, 0)
    try:
        jr, jc = (t.cpu().numpy() for t in m.jac_structure())
        hr, hc = (t.cpu().numpy() for t in m.hess_structure())
        n = m.n
    finally:
        m.close()
    pr, pc = [hr], [hc]
    order = np.argsort(jr, kind="stable")
    starts = np.searchsorted(jr[order], np.arange(jr.max() + 2))
    for r in range(jr.max() + 1):
        cols = jc[order[starts[r]:starts[r + 1]]]
        a, b = np.meshgrid(cols, cols)
        pr.append(a.ravel())
        pc.append(b.ravel())
    return np.concatenate(pr), np.concatenate(pc), n


def test_sparse_cholesky_factors_and_solves():
    """rocSOLVER's sparse re-factorization with the library's ordering and
    symbolic factor: two matrices of the interior-point pattern (the first
    through the analysis, the second re-factored) solve like a dense
    solve; a matrix that is not positive definite is reported."""
    import torch
    from paper_2510_12897_amd.sparse_chol import SparseCholesky
    case = synth.network(300, 410, 60, 41)
    rows, cols, n = _ipm_pattern(case)
    dev = torch.device("cuda", 0)
    ch = SparseCholesky(rows, cols, n, dev)
    say(f"[sparse] n {n}, lower nnz {ch.src.size}, factor nnz {ch.nnzT}")
    rng = np.random.default_rng(2)
    rr, cc = ch.src // n, ch.src % n
    try:
        for trial in range(3):
            v = rng.uniform(-1.0, 1.0, ch.src.size)
            A = np.zeros((n, n))
            A[rr, cc] = v
            A = np.tril(A, -1)
            A = A + A.T
            d = np.abs(A).sum(1) + 1.0 + trial
            A += np.diag(d)
            v[rr == cc] = d
            assert ch.factor(torch.as_tensor(v, device=dev))
            b = rng.standard_normal(n)
            x = ch.solve(torch.as_tensor(b, device=dev)).cpu().numpy()
            ref = np.linalg.solve(A, b)
            err = np.abs(x - ref).max() / np.abs(ref).max()
            say(f"[sparse] trial {trial}: max relative error {err:.2e}")
            assert err < 1e-12
        # an indefinite matrix of the pattern fails to factor
        v = np.zeros(ch.src.size)
        v[rr == cc] = -1.0
        assert not ch.factor(torch.as_tensor(v, device=dev))
    finally:
        ch.close()


def test_sparse_and_dense_linear_solvers_reach_one_optimum():
    case = dict(synth.network(300, 410, 60, 41))
    case["pd"], case["qd"] = case["pd"] * 0.7, case["qd"] * 0.7
    m = opf.Model(case, 0)
    try:
        ips = InteriorPoint(m, tol=1e-8, linear_solver="sparse")
        rs = ips.solve()
        ips.close()
        rd = InteriorPoint(m, tol=1e-8, linear_solver="dense").solve()
    finally:
        m.close()
    say(f"[ipm] sparse {rs['status']} it {rs['iterations']} f {rs['f']:.12g} la {rs['times']['linear_algebra']:.3f} s | "
        f"dense {rd['status']} it {rd['iterations']} f {rd['f']:.12g} la {rd['times']['linear_algebra']:.3f} s")
    assert rs["status"] == rd["status"] == "solved"
    # the equality rows are relaxed by the tolerance (LiftedKKT): two
    # solutions agree to about tol * sum |lam|
    slack = 1e-8 * float(rd["lam"].abs().sum())
    assert abs(rs["f"] - rd["f"]) <= 2 * slack + 1e-10 * abs(rd["f"])
    assert rs["cvio"] <= 1.01e-8


def test_trained_proxy_start_cuts_solver_iterations():
    """The learned proxy's purpose, measured in solver terms: trained on a
    solvable load regime of the 300-bus network (0.7x base, +-30 % per bus),
    its predictions start the interior-point method closer to the optimum
    than the model's start point does: fewer iterations to the same
    optimum on held-out loads."""
    import torch
    from paper_2510_12897_amd import proxy as P
    base = dict(synth.network(300, 410, 60, 41))
    base["pd"], base["qd"] = base["pd"] * 0.7, base["qd"] * 0.7
    px = P.WarmStartProxy(base, B=4096, width=1024, depth=3, rho=10.0, obj_scale=1e-3, seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    for _ in range(1500):
        px.train_step(*px.sample(gen), lr=3e-4)
    gen.manual_seed(4242)
    loads, feats = px.sample(gen)
    X, _ = px.predict(loads, feats)
    N = px.N
    cold, warm = [], []
    for i in range(8):
        cs = dict(base)
        cs["pd"], cs["qd"] = loads[i, :N].cpu().numpy().copy(), loads[i, N:].cpu().numpy().copy()
        m = opf.Model(cs, 0)
        try:
            ipc, ipw = InteriorPoint(m, tol=1e-6, max_iter=80), InteriorPoint(m, tol=1e-6, max_iter=80)
            rc, rw = ipc.solve(), ipw.solve(X[i].clone())
            ipc.close()
            ipw.close()
        finally:
            m.close()
        say(f"[warm] sample {i}: cold {rc['status']} {rc['iterations']}, warm {rw['status']} {rw['iterations']}")
        if rc["status"] == rw["status"] == "solved":
            cold.append(rc["iterations"])
            warm.append(rw["iterations"])
            assert abs(rw["f"] - rc["f"]) <= 1e-6 * abs(rc["f"])
    px.close()
    assert len(cold) >= 3
    assert np.mean(warm) <= 0.9 * np.mean(cold)
