"""The interior-point consumer of the callbacks, on the CPU: textbook
problems with known solutions, the 14-bus network against an independent
solver (scipy's SLSQP), polar against rectangular form, and an infeasible
load level."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from helpers import case0
from ipm_models import HS071, BoundQP, OracleModel
from oracle import oracle as orc
from paper_2510_12897_amd import synth
from paper_2510_12897_amd.ipm import InteriorPoint


def test_hs071_reaches_the_published_optimum():
    r = InteriorPoint(HS071(), tol=1e-8).solve()
    assert r["status"] == "solved"
    assert abs(r["f"] - HS071.F_STAR) < 2e-7
    np.testing.assert_allclose(r["x"].numpy(), HS071.X_STAR, atol=2e-6)
    # x1 sits at its lower bound with a positive bound dual; the others are free
    assert r["zl"][0] > 0.1 and float(r["zl"][1:].max()) < 1e-6


@pytest.mark.parametrize("b", [0.0, 0.4, -0.6])
def test_qp_closed_form_solution_and_multipliers(b):
    r = InteriorPoint(BoundQP(b), tol=1e-9).solve()
    assert r["status"] == "solved"
    np.testing.assert_allclose(r["x"].numpy(), [(1 + b) / 2, (3 - b) / 2], atol=1e-7)
    assert abs(r["f"] - (1 + b * b) / 2) < 1e-7
    np.testing.assert_allclose(r["lam"].numpy(), [1.0, -b], atol=1e-6)


def _scipy_opf(case):
    """The same OPF solved by SLSQP, with the oracle's values and dense
    Jacobian as its callbacks."""
    from scipy.optimize import Bounds, minimize
    b = orc.bounds(case)
    eq = b["lcon"] == b["ucon"]
    lo = np.isfinite(b["lcon"]) & ~eq
    hi = np.isfinite(b["ucon"]) & ~eq

    def c(x):
        return orc.evaluate(case, x, want=orc.W_CONS)["c"]

    def J(x):
        return orc.dense_jacobian(orc.evaluate(case, x, want=orc.W_CONS | orc.W_JAC))

    cons = [dict(type="eq", fun=lambda x: c(x)[eq] - b["lcon"][eq], jac=lambda x: J(x)[eq]),
            dict(type="ineq", fun=lambda x: c(x)[lo] - b["lcon"][lo], jac=lambda x: J(x)[lo]),
            dict(type="ineq", fun=lambda x: b["ucon"][hi] - c(x)[hi], jac=lambda x: -J(x)[hi])]
    r = minimize(lambda x: orc.evaluate(case, x, want=orc.W_OBJ)["f"], b["x0"],
                 jac=lambda x: orc.evaluate(case, x, want=orc.W_OBJ)["g"], constraints=cons,
                 bounds=Bounds(b["lvar"], b["uvar"]), method="SLSQP", options=dict(maxiter=1000, ftol=1e-12))
    assert r.success, r.message
    return r


def test_opf_14_bus_matches_slsqp_and_satisfies_kkt():
    case = case0()
    r = InteriorPoint(OracleModel(case), tol=1e-8).solve()
    assert r["status"] == "solved"
    ref = _scipy_opf(case)
    # the equality rows are relaxed by the tolerance (LiftedKKT), which moves
    # the optimum by about tol * sum |lam|
    slack = 1e-8 * float(r["lam"].abs().sum())
    assert abs(r["f"] - ref.fun) <= 2 * slack + 1e-9 * abs(ref.fun)
    assert r["cvio"] <= 1.01e-8
    # stationarity of the Lagrangian, recomputed here from the oracle
    x, lam = r["x"].numpy(), r["lam"].numpy()
    ev = orc.evaluate(case, x, lam)
    grad_l = ev["g"] + orc.dense_jacobian(ev).T @ lam
    zl, zu = r["zl"].numpy(), r["zu"].numpy()
    assert np.abs(grad_l - zl + zu).max() < 1e-6
    assert zl.min() >= 0 and zu.min() >= 0
    # away from its bounds a variable's bound duals vanish
    b = orc.bounds(case)
    free = (x - b["lvar"] > 1e-3) & (b["uvar"] - x > 1e-3)
    assert np.abs(grad_l[free]).max() < 1e-5


def test_rectangular_form_reaches_the_polar_optimum():
    case = case0()
    rp = InteriorPoint(OracleModel(case), tol=1e-8).solve()
    rr = InteriorPoint(OracleModel(case, form="rect"), tol=1e-8).solve()
    assert rp["status"] == rr["status"] == "solved"
    assert abs(rp["f"] - rr["f"]) < 1e-8 * abs(rp["f"])


def test_multiperiod_storage_model_solves():
    case = case0()
    T = 4
    pd, qd = synth.mp_loads(case, T, 3)
    st = synth.storage(case, 5, frac=0.3)
    opts = dict(n_periods=T, pd_t=pd, qd_t=qd, ramp_ratio=0.2, storage=st)
    r = InteriorPoint(OracleModel(case, **opts), tol=1e-6).solve()
    assert r["status"] == "solved"
    assert r["cvio"] <= 1.01e-6


def test_overloaded_network_is_not_reported_solved():
    case = dict(case0())
    case["pd"] = case["pd"] * 20.0
    case["qd"] = case["qd"] * 20.0
    r = InteriorPoint(OracleModel(case), tol=1e-6, max_iter=60).solve()
    assert r["status"] != "solved"
    assert r["cvio"] > 1e-2


def test_dense_limit_is_enforced():
    with pytest.raises(ValueError, match="dense limit"):
        InteriorPoint(OracleModel(case0()), max_dense_n=10)


def test_condensed_matrix_matches_dense_products():
    """K assembled through the pair list equals W + Sigma_x + J^T Sigma_s J
    formed densely from the oracle."""
    case = case0()
    mdl = OracleModel(case)
    ip = InteriorPoint(mdl)
    rng = np.random.default_rng(3)
    b = orc.bounds(case)
    x = np.clip(b["x0"] + rng.normal(0, 0.05, mdl.n), b["lvar"], b["uvar"])
    y = rng.normal(size=mdl.m)
    ev = orc.evaluate(case, x, y)
    Sx = torch.from_numpy(rng.uniform(0, 2, mdl.n))
    Ss = torch.from_numpy(rng.uniform(0, 2, mdl.m))
    rhs = torch.from_numpy(rng.normal(size=mdl.n))
    dx, delta, _ = ip._assemble_factor(torch.from_numpy(ev["hval"]), torch.from_numpy(ev["jval"]), Sx, Ss, rhs, 0.0)
    J = orc.dense_jacobian(ev)
    K = orc.dense_hessian(ev) + np.diag(Sx.numpy()) + J.T @ np.diag(Ss.numpy()) @ J + delta * np.eye(mdl.n)
    np.testing.assert_allclose(K @ dx.numpy(), rhs.numpy(), rtol=0, atol=1e-8 * np.abs(K).max() * np.abs(dx.numpy()).max())


def test_linear_solver_choice_is_checked():
    mdl = OracleModel(case0())
    assert InteriorPoint(mdl).linear_solver == "dense"          # the CPU default
    with pytest.raises(ValueError, match="GPU only"):
        InteriorPoint(mdl, linear_solver="sparse")
    with pytest.raises(ValueError, match="linear_solver"):
        InteriorPoint(mdl, linear_solver="qr")


def test_warm_start_from_the_optimum_takes_few_iterations():
    """Started at a solution, the method stops after few iterations at the
    same optimum (the primal start is used as given, pushed inside its
    bounds)."""
    mdl = OracleModel(case0())
    r = InteriorPoint(mdl, tol=1e-6).solve()
    rw = InteriorPoint(mdl, tol=1e-6).solve(r["x"].clone())
    assert rw["status"] == "solved"
    assert rw["iterations"] < r["iterations"]
    assert abs(rw["f"] - r["f"]) <= 1e-6 * abs(r["f"])
