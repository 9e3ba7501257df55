"""Pins of the oracle's tolerance scale S (the sum of |contributions|).

The parity tolerance accepts |v - v*| <= 1e-12 max(|v*|, S) + 1e-14, so S
must be exactly the sum of the absolute values of the terms that make up
each output, no more: a looser S loosens every comparison that uses it.
Here S is written out by hand for every row type from the flow template
F = alpha u^2 + beta w^2 + u w (a cos th + b sin th) (u = vm_f, w = vm_t,
th = va_f - va_t), with the admittance terms taken from the complex branch
matrices of the pi model, and for the linear, balance, thermal, ramp and
objective terms of Listing 3.  Jacobian scales are the sums of |terms| of
each partial derivative; Hessian scales the sums over every row (weighted
by |y|) and the objective (weighted by |sigma|) that contributes to a
merged entry.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_12897_amd import synth

from helpers import case0

RT = 1e-13


def _coeffs(cs):
    ys = 1.0 / (cs["r"] + 1j * cs["x"])
    tap = cs["tap"] * np.exp(1j * cs["shift"])
    ytt = ys + 1j * cs["b"] / 2
    yff = ytt / (tap * np.conj(tap))
    yft = -ys / np.conj(tap)
    ytf = -ys / tap
    # (alpha, beta, a, b) of the four flows: p_fr, q_fr, p_to, q_to, from
    # S_f = V_f conj(Yff V_f + Yft V_t) and S_t = V_t conj(Ytf V_f + Ytt V_t).
    return [
        (yff.real, 0 * ys.real, yft.real, yft.imag),
        (-yff.imag, 0 * ys.real, -yft.imag, yft.real),
        (0 * ys.real, ytt.real, ytf.real, -ytf.imag),
        (0 * ys.real, -ytt.imag, -ytf.imag, -ytf.real),
    ]


def _literal_scales(cs, x, y, sigma, T=1):
    """Hand-written S for c, J and H of a static (T = 1) or multi-period
    model, returned as dicts keyed by row and by (row, col)."""
    N, L, G, R = cs["n_bus"], cs["n_branch"], cs["n_gen"], len(cs["ref_bus"])
    xva, xvm, xpg = 0, N * T, 2 * N * T
    xqg = xpg + G * T
    xp = xqg + G * T
    xq = xp + 2 * L * T
    col = dict(va=lambda i, t: xva + i + N * t, vm=lambda i, t: xvm + i + N * t,
               pg=lambda k, t: xpg + k + G * t, qg=lambda k, t: xqg + k + G * t,
               p=lambda a, t: xp + a + 2 * L * t, q=lambda a, t: xq + a + 2 * L * t)
    coef = _coeffs(cs)
    f, tb = cs["f_bus"], cs["t_bus"]
    cS, jS, hS = {}, {}, {}

    def hadd(r, c1, c2, v):
        key = (max(c1, c2), min(c1, c2))
        hS[key] = hS.get(key, 0.0) + v

    blocks = [R, L, L, L, L, L, N, N, L, L]
    start = np.concatenate([[0], np.cumsum(np.array(blocks) * T)])
    fscale = 0.0
    for t in range(T):
        # objective (Listing 3): c2 pg^2 + c1 pg + c0
        for k in range(G):
            pg = x[col["pg"](k, t)]
            fscale += abs(cs["c2"][k]) * pg * pg + abs(cs["c1"][k] * pg) + abs(cs["c0"][k])
            hadd(None, col["pg"](k, t), col["pg"](k, t), abs(sigma) * 2 * abs(cs["c2"][k]))
        # reference angle
        for j in range(R):
            row = start[0] + j + R * t
            c = col["va"](cs["ref_bus"][j], t)
            cS[row] = abs(x[c])
            jS[(row, c)] = 1.0
        # four flow definitions: p_a - F
        for blk in range(4):
            al, be, aa, bb = coef[blk]
            for l in range(L):
                row = start[1 + blk] + l + L * t
                arc = l if blk < 2 else L + l
                av = col["p" if blk % 2 == 0 else "q"](arc, t)
                cu, cw = col["vm"](f[l], t), col["vm"](tb[l], t)
                caf, cat = col["va"](f[l], t), col["va"](tb[l], t)
                u, w = abs(x[cu]), abs(x[cw])
                th = x[caf] - x[cat]
                C, S = abs(np.cos(th)), abs(np.sin(th))
                A, B, a, b = abs(al[l]), abs(be[l]), abs(aa[l]), abs(bb[l])
                kc, ks = a * C + b * S, a * S + b * C
                cS[row] = abs(x[av]) + A * u * u + B * w * w + u * w * kc
                jS[(row, av)] = 1.0
                jS[(row, cu)] = 2 * A * u + w * kc
                jS[(row, cw)] = 2 * B * w + u * kc
                jS[(row, caf)] = u * w * ks
                jS[(row, cat)] = u * w * ks
                ay = abs(y[row])
                hadd(row, cu, cu, ay * 2 * A)
                hadd(row, cw, cw, ay * 2 * B)
                hadd(row, cu, cw, ay * kc)
                for c1 in (caf, cat):
                    hadd(row, cu, c1, ay * w * ks)
                    hadd(row, cw, c1, ay * u * ks)
                hadd(row, caf, caf, ay * u * w * kc)
                hadd(row, cat, cat, ay * u * w * kc)
                hadd(row, caf, cat, ay * u * w * kc)
        # angle difference
        for l in range(L):
            row = start[5] + l + L * t
            caf, cat = col["va"](f[l], t), col["va"](tb[l], t)
            cS[row] = abs(x[caf]) + abs(x[cat])
            jS[(row, caf)] = 1.0
            jS[(row, cat)] = 1.0
        # balance: load + shunt vm^2 + sum of arc variables + sum of generator outputs
        pdt = cs.get("_pd_t")
        for isp, blk in ((True, 6), (False, 7)):
            load = (cs["_pd_t"] if isp else cs["_qd_t"])[t] if pdt is not None else (cs["pd"] if isp else cs["qd"])
            shunt = cs["gs"] if isp else cs["bs"]
            for i in range(N):
                row = start[blk] + i + N * t
                cv = col["vm"](i, t)
                vm = abs(x[cv])
                s = abs(load[i]) + abs(shunt[i]) * vm * vm
                jS[(row, cv)] = 2 * abs(shunt[i]) * vm
                for a in range(2 * L):
                    if (f[a] if a < L else tb[a - L]) == i:
                        ca = col["p" if isp else "q"](a, t)
                        s += abs(x[ca])
                        jS[(row, ca)] = 1.0
                for k in range(G):
                    if cs["gen_bus"][k] == i:
                        cg = col["pg" if isp else "qg"](k, t)
                        s += abs(x[cg])
                        jS[(row, cg)] = 1.0
                cS[row] = s
                hadd(row, cv, cv, abs(y[row]) * 2 * abs(shunt[i]))
        # thermal limits p^2 + q^2 - rate^2
        for side, blk in ((0, 8), (1, 9)):
            for l in range(L):
                row = start[blk] + l + L * t
                a = l + side * L
                cp, cq = col["p"](a, t), col["q"](a, t)
                cS[row] = x[cp] ** 2 + x[cq] ** 2 + cs["rate_a"][l] ** 2
                jS[(row, cp)] = 2 * abs(x[cp])
                jS[(row, cq)] = 2 * abs(x[cq])
                hadd(row, cp, cp, abs(y[row]) * 2)
                hadd(row, cq, cq, abs(y[row]) * 2)
    # ramp rows pg_t - pg_{t-1}, t >= 1
    for t in range(1, T):
        for k in range(G):
            row = start[10] + k + G * (t - 1)
            c1, c0 = col["pg"](k, t), col["pg"](k, t - 1)
            cS[row] = abs(x[c1]) + abs(x[c0])
            jS[(row, c1)] = 1.0
            jS[(row, c0)] = 1.0
    return fscale, cS, jS, hS


def _check(cs, x, y, sigma, T=1, **opts):
    ref = O.evaluate(cs, x, y, sigma, **opts)
    fscale, cS, jS, hS = _literal_scales(cs, x, y, sigma, T)
    assert ref["fscale"] == pytest.approx(fscale, rel=RT)
    m = ref["m"]
    want_c = np.array([cS[r] for r in range(m)])
    np.testing.assert_allclose(ref["cscale"], want_c, rtol=RT, atol=0)
    assert len(jS) == ref["jrow"].size
    want_j = np.array([jS[(int(r), int(c))] for r, c in zip(ref["jrow"], ref["jcol"])])
    np.testing.assert_allclose(ref["jscale"], want_j, rtol=RT, atol=0)
    assert len(hS) == ref["hrow"].size
    want_h = np.array([hS[(int(r), int(c))] for r, c in zip(ref["hrow"], ref["hcol"])])
    np.testing.assert_allclose(ref["hscale"], want_h, rtol=RT, atol=0)
    return ref


@pytest.mark.parametrize("variant", [False, True])
def test_scale_static_every_row_type(variant):
    cs = case0(variant=variant)
    n, m = O.dims(cs)
    x = synth.point(cs, 100)
    y = synth.multipliers(m, 100)
    ref = _check(cs, x, y, 0.37)
    # the scale of a flow row is at least |c|, and strictly larger when its
    # terms cancel: the rows this form exists for
    assert np.all(ref["cscale"] >= np.abs(ref["c"]) * (1 - 1e-15))


def test_scale_multiperiod_ramp_rows():
    cs = case0(variant=True)
    T = 3
    pd_t, qd_t = synth.mp_loads(cs, T, 202)
    opts = dict(n_periods=T, pd_t=pd_t, qd_t=qd_t, ramp_ratio=0.2)
    n, m = O.dims(cs, **opts)
    x = synth.point(cs, 5, n_periods=T)
    y = synth.multipliers(m, 6)
    cs2 = dict(cs, _pd_t=pd_t.reshape(T, -1), _qd_t=qd_t.reshape(T, -1))
    _check(cs2, x, y, -0.8, T=T, **opts)


def test_scale_negative_sigma_and_zero_multipliers():
    cs = case0(variant=True)
    n, m = O.dims(cs)
    x = synth.point(cs, 7)
    ref = _check(cs, x, np.zeros(m), -2.5)
    # with y = 0 only the objective's pg diagonal carries a scale
    pg0 = 2 * cs["n_bus"]
    on_pg = (ref["hrow"] == ref["hcol"]) & (ref["hrow"] >= pg0) & (ref["hrow"] < pg0 + cs["n_gen"])
    assert np.all(ref["hscale"][~on_pg] == 0)
    np.testing.assert_allclose(ref["hscale"][on_pg], 5.0 * np.abs(cs["c2"]), rtol=1e-15)
