"""Pins of the proxy's CPU oracle to definitions and closed forms."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_bf16_rounding_exact_cases():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)  # BF16 spacing at 1
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -7 + 2.0 ** -8, -2.5, 0.0,
                     3.0e38], dtype=np.float32)
    got = M.bf16_round(vals)
    # halfway to the next BF16 goes to the even neighbour; above halfway goes up
    np.testing.assert_array_equal(got[:4], np.array([one, one, one + ulp, one + 2 * ulp], np.float32))
    assert got[4] == -2.5 and got[5] == 0.0
    # every result has 7 fraction bits at most
    rnd = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    bits = M.bf16_round(rnd).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
    assert np.all(np.abs(M.bf16_round(rnd) - rnd) <= np.abs(rnd) * 2.0 ** -8 * 1.0001)


def test_gelu_definition():
    xs = np.linspace(-6, 6, 97)
    ref = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in xs])
    np.testing.assert_allclose(M.gelu(xs), ref, rtol=1e-15, atol=1e-15)
    assert M.gelu(0.0) == 0.0
    assert M.gelu_grad(0.0) == pytest.approx(0.5, abs=1e-15)
    np.testing.assert_allclose(M.gelu(np.array([8.0])), [8.0], rtol=1e-14)   # GELU(x) -> x
    np.testing.assert_allclose(M.gelu(np.array([-8.0])), [0.0], atol=1e-13)  # GELU(x) -> 0
    h = 1e-6
    fd = (M.gelu(xs + h) - M.gelu(xs - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(xs), fd, rtol=1e-7, atol=1e-9)


def test_adam_first_step_and_convergence():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = M.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=0.0)
    # with zero state the bias-corrected first step is -lr * sign(g)
    np.testing.assert_allclose(p, -0.1 * np.sign(g), rtol=1e-12)
    # minimises a convex quadratic
    x, m, v = np.array([3.0, -4.0]), np.zeros(2), np.zeros(2)
    for t in range(1, 3001):
        x, m, v = M.adam(x, 2 * x, m, v, t, lr=0.05)
    assert np.abs(x).max() < 1e-3


def test_squash_and_gradient():
    rng = np.random.default_rng(1)
    N, G = 5, 2
    box = dict(N=N, G=G, vmin=np.full(N, 0.9), vmax=np.full(N, 1.1), pmin=np.zeros(G), pmax=np.full(G, 3.0),
               qmin=np.full(G, -1.0), qmax=np.ones(G), is_ref=np.array([0, 1, 0, 0, 0]))
    z = rng.standard_normal((3, 2 * N + 2 * G))
    va, vm, pg, qg = M.squash(z, box, math.pi / 6)
    assert np.all((vm > 0.9) & (vm < 1.1)) and np.all(va[:, 1] == 0) and np.all(np.abs(va) < math.pi / 6)
    assert np.all((pg > 0) & (pg < 3)) and np.all((qg > -1) & (qg < 1))
    gs = [rng.standard_normal(a.shape) for a in (va, vm, pg, qg)]
    dz = M.squash_grad(z, box, math.pi / 6, *gs)
    h = 1e-6
    for j in range(z.shape[1]):
        zp, zm = z.copy(), z.copy()
        zp[:, j] += h
        zm[:, j] -= h
        fp = sum((a * g).sum(1) for a, g in zip(M.squash(zp, box, math.pi / 6), gs))
        fm = sum((a * g).sum(1) for a, g in zip(M.squash(zm, box, math.pi / 6), gs))
        np.testing.assert_allclose(dz[:, j], (fp - fm) / (2 * h), rtol=1e-6, atol=1e-9)


def test_penalty_gradient_and_cvio():
    rng = np.random.default_rng(2)
    c = rng.standard_normal(12)
    lcon = np.r_[np.zeros(6), np.full(6, -np.inf)]
    ucon = np.zeros(12)
    flow = np.zeros(12, bool)
    flow[1:3] = True
    pq = rng.standard_normal(4) * 2
    lpq, upq = -np.ones(4), np.ones(4)
    pen, w, gpq, cvio = M.penalty(c, lcon, ucon, flow, pq, lpq, upq, 3.0)
    h = 1e-6
    for r in range(12):
        cp, cm = c.copy(), c.copy()
        cp[r] += h
        cm[r] -= h
        d = (M.penalty(cp, lcon, ucon, flow, pq, lpq, upq, 3.0)[0] - M.penalty(cm, lcon, ucon, flow, pq, lpq, upq,
                                                                                3.0)[0]) / (2 * h)
        assert w[r] == pytest.approx(d, abs=1e-6)
    assert np.all(w[1:3] == 0)
    expect = max(np.abs(c[:6]).max(), np.clip(c[6:], 0, None).max(), np.clip(np.abs(pq) - 1, 0, None).max())
    assert cvio == pytest.approx(expect)
    np.testing.assert_allclose(gpq, 6.0 * np.sign(pq) * np.clip(np.abs(pq) - 1, 0, None))
