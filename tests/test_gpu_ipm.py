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
