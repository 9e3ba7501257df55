"""The seeded input generator: topology and parameter recipe."""
import math

import numpy as np
import pytest

from paper_2510_12897_amd import synth


def _connected(n, f, t):
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for u, v in zip(f, t):
        parent[find(u)] = find(v)
    return len({find(i) for i in range(n)}) == 1


@pytest.mark.parametrize("N,L,G", [(14, 20, 5), (2, 1, 1), (500, 675, 100), (3000, 4050, 600)])
def test_network_topology(N, L, G):
    cs = synth.network(N, L, G, 5)
    f, t = cs["f_bus"], cs["t_bus"]
    assert f.dtype == np.int32 and f.shape == (L,) and t.shape == (L,)
    assert ((0 <= f) & (f < N) & (0 <= t) & (t < N)).all()
    assert (f != t).all(), "self-loop"
    pairs = {(min(a, b), max(a, b)) for a, b in zip(f, t)}
    assert len(pairs) == L, "parallel branches"
    assert _connected(N, f, t)
    # removing any single extra branch keeps the network connected
    extra = cs["extra_branches"]
    assert extra.size == L - (N - 1)
    for e in extra[:5]:
        keep = np.ones(L, bool)
        keep[e] = False
        assert _connected(N, f[keep], t[keep])
    # both orientations occur (exercises both column orders of a flow row)
    if L > 10:
        assert (f < t).any() and (f > t).any()
    assert cs["ref_bus"][0] == cs["gen_bus"][0]


def test_parameter_ranges():
    cs = synth.network(2000, 2700, 400, 3)
    assert (cs["r"] >= 0.005).all() and (cs["r"] <= 0.05).all()
    assert (cs["x"] >= 0.02).all() and (cs["x"] <= 0.3).all()
    assert (cs["b"] >= 0).all() and (cs["b"] <= 0.05).all()
    assert (cs["rate_a"] >= 0.5).all() and (cs["rate_a"] <= 2.0).all()
    assert (cs["tap"] == 1).all() and (cs["shift"] == 0).all()
    assert (cs["c2"] >= 0.01).all() and (cs["c2"] <= 0.1).all()
    assert (cs["c1"] >= 10).all() and (cs["c1"] <= 40).all()
    assert (cs["c0"] == 0).all()
    assert (cs["pd"] >= 0).all() and (cs["pd"] <= 0.5).all()
    np.testing.assert_array_equal(cs["qd"], 0.3 * cs["pd"])
    assert np.allclose(cs["angmax"], math.pi / 6)
    v = synth.network(50, 70, 10, 3, variant=True)
    assert (np.abs(v["tap"] - 1) <= 0.1).all() and (np.abs(v["shift"]) <= 0.1).all()
    assert (np.abs(v["gs"]) <= 0.05).all() and (v["gs"] != 0).any()


def test_reproducible():
    a = synth.network(300, 410, 60, 4)
    b = synth.network(300, 410, 60, 4)
    for k in a:
        np.testing.assert_array_equal(np.asarray(a[k]), np.asarray(b[k]))
    c = synth.network(300, 410, 60, 5)
    assert not np.array_equal(a["f_bus"], c["f_bus"])
    np.testing.assert_array_equal(synth.point(a, 9), synth.point(a, 9))


def test_point_inside_bounds():
    cs = synth.network(30, 40, 6, 1)
    for T, K in [(1, 0), (3, 0), (1, 2)]:
        x = synth.point(cs, 2, n_periods=T, n_cont=K)
        nrep = T if T > 1 else K + 1
        npg = 1 if K else nrep
        N, L, G = 30, 40, 6
        assert x.size == nrep * (2 * N + G + 4 * L) + npg * G
        vm = x[N * nrep: 2 * N * nrep]
        assert ((vm >= 0.9) & (vm <= 1.1)).all()


def test_mp_loads_profile():
    cs = synth.network(40, 50, 8, 2)
    pd_t, qd_t = synth.mp_loads(cs, 48, 202)
    fac = pd_t.reshape(48, 40) / cs["pd"][None, :]
    prof = 0.7 + 0.3 * np.sin(2 * np.pi * np.arange(48) / 48)
    resid = fac - prof[:, None]
    assert abs(resid.std() - 0.02) < 0.003
    np.testing.assert_allclose(qd_t.reshape(48, 40), cs["qd"][None, :] * fac)


def test_outages_from_extra_branches():
    cs = synth.network(1000, 1350, 200, 31)
    o = synth.outages(cs, 200, 32)
    assert o.size == 200 and np.unique(o).size == 200
    assert np.isin(o, cs["extra_branches"]).all()
