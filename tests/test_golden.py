"""Oracle regression fixtures (tests/golden/): the oracle must keep
reproducing the values it wrote for three small seeded models (static,
three periods with ramp rows, two N-1 copies).  The paper prints no callback
values, so these pin the oracle to its own committed past, not to the
paper: a change to its arithmetic fails here and has to name the passage
that justifies it when the fixtures are rewritten."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden as MG  # noqa: E402

CASES = list(MG.cases())


@pytest.mark.parametrize("name,cs,opts,T,K,seed,sigma", CASES, ids=[c[0] for c in CASES])
def test_oracle_reproduces_fixture(name, cs, opts, T, K, seed, sigma):
    ref = MG.read(os.path.join(HERE, "golden", name + ".txt"))
    _, _, res = MG.compute(cs, opts, T, K, seed, sigma)
    for key in ("jrow", "jcol", "hrow", "hcol"):
        np.testing.assert_array_equal(np.asarray(res[key], dtype=np.int64), ref[key], err_msg=key)
    np.testing.assert_allclose(res["f"], ref["f"], rtol=1e-15, atol=0)
    for key in ("g", "c", "jval", "hval"):
        np.testing.assert_allclose(np.asarray(res[key]), ref[key], rtol=1e-15, atol=1e-300, err_msg=key)
