"""CPU oracle of the warm-start proxy's arithmetic.

TEST INFRASTRUCTURE ONLY: used by the tests and the smoke check; the HIP
library never loads it and it imports nothing from the HIP package.

* BF16 rounding: round-to-nearest-even of the FP32 bit pattern to its top 16
  bits (the bfloat16 format: sign, 8 exponent bits, 7 fraction bits).
* GEMM: products of BF16-rounded operands accumulated in FP64 (the matrix
  cores accumulate in FP32; tests allow for that difference).
* GELU: x * Phi(x) with the exact normal CDF, Phi(x) = (1 + erf(x / sqrt 2)) / 2
  (Hendrycks and Gimpel, 2016).
* Adam: the bias-corrected update of Kingma and Ba (2015), Algorithm 1.
* Squashing of the network output into the variable boxes, and its
  derivative.
* The penalty on the constraint values: squared violations of the non-flow
  rows and of the arc-variable bounds, its gradient with respect to c, and
  the largest violation (the paper's Cvio, Sec. IV-A5).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def bf16_round(x) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def gemm(A, B) -> np.ndarray:
    """A @ B with BF16-rounded operands, accumulated in FP64."""
    return bf16_round(A).astype(np.float64) @ bf16_round(B).astype(np.float64)


def gelu(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (t counts from 1); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-np.asarray(z, dtype=np.float64)))


def squash(z, box, va_span):
    """z [B, 2N+2G] (vm, va, pg, qg blocks) -> (va, vm, pg, qg) in FP64."""
    N, G = box["N"], box["G"]
    z = np.asarray(z, dtype=np.float64)
    vm = box["vmin"] + (box["vmax"] - box["vmin"]) * sigmoid(z[:, :N])
    va = va_span * np.tanh(z[:, N:2 * N]) * (1 - box["is_ref"])
    pg = box["pmin"] + (box["pmax"] - box["pmin"]) * sigmoid(z[:, 2 * N:2 * N + G])
    qg = box["qmin"] + (box["qmax"] - box["qmin"]) * sigmoid(z[:, 2 * N + G:])
    return va, vm, pg, qg


def squash_grad(z, box, va_span, g_va, g_vm, g_pg, g_qg):
    """(d (va, vm, pg, qg) / dz)^T g, laid out like z."""
    N, G = box["N"], box["G"]
    z = np.asarray(z, dtype=np.float64)
    s_vm = sigmoid(z[:, :N])
    t_va = np.tanh(z[:, N:2 * N])
    s_pg = sigmoid(z[:, 2 * N:2 * N + G])
    s_qg = sigmoid(z[:, 2 * N + G:])
    return np.concatenate([
        g_vm * (box["vmax"] - box["vmin"]) * s_vm * (1 - s_vm),
        g_va * va_span * (1 - t_va ** 2) * (1 - box["is_ref"]),
        g_pg * (box["pmax"] - box["pmin"]) * s_pg * (1 - s_pg),
        g_qg * (box["qmax"] - box["qmin"]) * s_qg * (1 - s_qg),
    ], axis=1)


def violation(v, lo, hi):
    """Signed distance to [lo, hi] (0 inside)."""
    v = np.asarray(v, dtype=np.float64)
    return np.where(v < lo, v - lo, np.where(v > hi, v - hi, 0.0))


def penalty(c, lcon, ucon, flow_rows, pq, lpq, upq, rho):
    """Penalty rho (sum over non-flow rows of viol^2 + sum of p, q bound
    viol^2), its gradients (w on c, zero on the flow rows; gpq on p, q) and
    the largest violation over all rows and the p, q bounds."""
    dv = violation(c, lcon, ucon)
    db = violation(pq, lpq, upq)
    keep = ~flow_rows
    pen = rho * ((dv[..., keep] ** 2).sum(-1) + (db ** 2).sum(-1))
    w = np.where(keep, 2.0 * rho * dv, 0.0)
    gpq = 2.0 * rho * db
    cvio = np.maximum(np.abs(dv).max(-1), np.abs(db).max(-1))
    return pen, w, gpq, cvio
