"""Learned warm-start proxy: a multilayer perceptron from bus loads to
(vm, va, pg, qg), trained self-supervised on the FP64 penalty that the
callback kernels compute.

The paper names learned proxies for OPF as related work whose feasibility is
the open problem (Sec. I); here the FP64 constraint evaluator decides it:
every prediction is completed (arc flows p, q := F(vm, va)) and scored by
the constraint kernels, and a prediction whose largest violation (Cvio,
Sec. IV-A5) exceeds a threshold tau is discarded, the solver then starting
without it (fallback_curve gives that share for several tau).

Every step runs in libopf's kernels (argument marshalling only here):

* the MLP's linear layers are BF16 matrix-core GEMMs with FP32 accumulation
  (``prox_gemm_bf16_mixed``: a BF16 copy of the weights kept by the Adam
  step, hidden activations stored as BF16), the hidden activations an
  exact-erf GELU fused into the GEMM epilogue; its backward is three more GEMM layouts, ``prox_colsum``
  for the biases and ``prox_gelu_bwd``; the optimiser is ``prox_adam``;
* ``Squash`` maps the network output into the variable boxes
  (``prox_squash_fwd`` / ``prox_squash_bwd``);
* ``Penalty`` completes the arc flows (``opf_batch_flows``), evaluates f,
  grad f and c for the whole batch (``opf_batch_eval``) and the penalty
  (``prox_penalty``); its backward is the hand-written vector-Jacobian
  product J^T (w + w2): w the penalty weights, w2 the weights on the flow
  rows that carry the arc-flow gradient back through p = F(vm, va), built
  in closed form by the penalty pass itself when a gradient will follow
  (``prox_penalty`` with ``vjp``), then one ``opf_batch_jtprod`` and
  ``prox_vjp_sum`` (which adds the objective gradient 2 c2 pg + c1);
* training takes Squash and Penalty as one autograd node (the arc flows
  written into the squashed X itself, ``prox_loss_bwd`` for the objective
  and squashing backward in one pass).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import opf
from .opf import OPF_E_ARG, OPFError, _check, lib


def _torch():
    import torch
    return torch


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def gemm(variant, A, lda, B, ldb, C, ldc, M, N, K, bias=None, act=None, accumulate=False, splits=1, work=None):
    """C[M,N] (+)= A B on the BF16 matrix cores (layouts: see prox_gemm_bf16);
    splits > 1 runs the split-K form with `work` (splits * M * N floats)."""
    if splits == 1:
        _check(lib().prox_gemm_bf16(int(variant), _p(A), int(lda), _p(B), int(ldb), _p(C), int(ldc), int(M), int(N),
                                    int(K), _p(bias), _p(act), int(bool(accumulate)), _stream()))
    else:
        _check(lib().prox_gemm_bf16_splitk(int(variant), _p(A), int(lda), _p(B), int(ldb), _p(C), int(ldc), int(M),
                                           int(N), int(K), _p(bias), _p(act), int(bool(accumulate)), int(splits),
                                           _p(work), _stream()))


def gemm_mixed(variant, A, a_bf16, lda, B, b_bf16, ldb, C, ldc, M, N, K, bias=None, act=None, act_bf16=False,
               accumulate=False, splits=1, work=None):
    """gemm with either operand stored as BF16 (a_bf16 / b_bf16) and the
    GELU output stored as BF16 (act_bf16)."""
    _check(lib().prox_gemm_bf16_mixed(int(variant), _p(A), int(bool(a_bf16)), int(lda), _p(B), int(bool(b_bf16)),
                                      int(ldb), _p(C), int(ldc), int(M), int(N), int(K), _p(bias), _p(act),
                                      int(bool(act_bf16)), int(bool(accumulate)), int(splits), _p(work), _stream()))


def gemm_gelu_bwd(A, a_bf16, lda, B, b_bf16, ldb, pre, ldp, out, ldo, M, N, K, part):
    """out (BF16) = (A B) * gelu'(pre) for row-major A [M, K], B [K, N], and
    the 128-row column partial sums of the product in part."""
    _check(lib().prox_gemm_gelu_bwd(_p(A), int(bool(a_bf16)), int(lda), _p(B), int(bool(b_bf16)), int(ldb), _p(pre),
                                    int(ldp), _p(out), int(ldo), int(M), int(N), int(K), _p(part), _stream()))


def gemm_splits(M, N, K):
    """The library's split count for an M x N x K product."""
    s = lib().prox_gemm_splits(int(M), int(N), int(K))
    if s < 1:
        _check(s)
    return s


# ------------------------------------------------------------------ the MLP
class MLP:
    """x [B, n_in] -> z [B, n_out]: `depth` hidden layers of `width` with
    GELU, then a linear output layer.  Parameters live in one flat FP32
    buffer (weights [out, in] row-major, then the bias, per layer).

    With bf16_storage (the default) the matrix cores read a BF16 copy of
    the parameters (kept by the Adam step, refreshed when the FP32 buffer
    is written from outside) and the hidden activations are stored as BF16:
    the operands are rounded once when written instead of each time a tile
    is staged, so the products are the same and read half the bytes."""

    def __init__(self, n_in: int, n_out: int, width: int = 1024, depth: int = 3, seed: int = 0, device: int = 0,
                 bf16_storage: bool = True):
        torch = _torch()
        for d in (n_in, n_out, width):
            if d % 4:
                raise OPFError(OPF_E_ARG, f"layer widths must be multiples of 4 (got {d})")
        self.dims = [n_in] + [width] * depth + [n_out]
        self.device = torch.device("cuda", device)
        self.layout = []  # (w_off, b_off, n_out, n_in) per layer
        off = 0
        for k in range(len(self.dims) - 1):
            fi, fo = self.dims[k], self.dims[k + 1]
            self.layout.append((off, off + fo * fi, fo, fi))
            off += fo * fi + fo
        self.n_params = off
        # He-style initialisation of the hidden layers drawn on the host from
        # a seeded generator; the output layer starts at zero, so the first
        # prediction is the centre of every box (va = 0, vm, pg, qg mid-range)
        rng = np.random.default_rng(seed)
        host = np.zeros(off, np.float32)
        for k, (wo, bo, fo, fi) in enumerate(self.layout[:-1]):
            host[wo:wo + fo * fi] = rng.standard_normal(fo * fi).astype(np.float32) * math.sqrt(2.0 / fi)
        self.flat = torch.from_numpy(host).to(self.device).requires_grad_(True)
        self.m1 = torch.zeros_like(self.flat, requires_grad=False)
        self.m2 = torch.zeros_like(self.flat, requires_grad=False)
        self.step = 0
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=self.device)  # Adam's count, read on the device
        self.bf16_storage = bool(bf16_storage)
        self.flat_bf16 = None
        self._bf16_version = None
        if self.bf16_storage:
            self.flat_bf16 = torch.empty(off, dtype=torch.bfloat16, device=self.device)
            self.sync_bf16()

    def sync_bf16(self):
        """Round the FP32 parameters into the BF16 copy."""
        _check(lib().prox_to_bf16(_p(self.flat.detach()), self.n_params, _p(self.flat_bf16), _stream()))
        self._bf16_version = self.flat._version

    def mma_weight(self, k):
        """(weight [out, in] as the matrix cores read it, stored as BF16).
        The forward reads it k-contiguous, so a BF16 copy needs its input
        width a multiple of 8; other layers read the FP32 buffer."""
        wo, bo, fo, fi = self.layout[k]
        if self.bf16_storage and fi % 8 == 0:
            return self.flat_bf16[wo:wo + fo * fi].view(fo, fi), True
        return self.weight(k), False

    def act_bf16(self, k):
        """Whether hidden layer k stores its activations as BF16 (the next
        layer reads them k-contiguous: width a multiple of 8)."""
        return self.bf16_storage and self.layout[k][2] % 8 == 0

    def weight(self, k):
        wo, bo, fo, fi = self.layout[k]
        return self.flat.detach()[wo:wo + fo * fi].view(fo, fi)

    def bias(self, k):
        wo, bo, fo, fi = self.layout[k]
        return self.flat.detach()[bo:bo + fo]

    def __call__(self, x):
        # without a backward to come (no grad mode, or nothing requiring a
        # gradient) the hidden layers store only their activations
        torch = _torch()
        keep = torch.is_grad_enabled() and (x.requires_grad or self.flat.requires_grad)
        return _MLPFunction.apply(x, self.flat, self, keep)

    def desc(self):
        """The prox_mlp_desc of this MLP (its buffers stay owned here; built
        again whenever a buffer's address changed)."""
        ptrs = (self.flat.data_ptr(), self.flat_bf16.data_ptr() if self.bf16_storage else None,
                self.m1.data_ptr(), self.m2.data_ptr(), self.step_dev.data_ptr())
        if getattr(self, "_desc", None) is None or self._desc[2] != ptrs:
            dims = (ctypes.c_int32 * len(self.dims))(*self.dims)
            self._desc = (opf.MlpDesc(len(self.dims) - 1, dims, *ptrs), dims, ptrs)
        return self._desc[0]

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        if self.flat.grad is None:
            raise OPFError(OPF_E_ARG, "no gradient: run backward first")
        self.step += 1
        if self.bf16_storage and self._bf16_version != self.flat._version:
            self.sync_bf16()
        # the step count lives on the device (the bias corrections need no
        # host value, so the step could be recorded once and replayed)
        _check(lib().prox_adam_dev(_p(self.flat), _p(self.flat.grad), _p(self.m1), _p(self.m2), self.n_params,
                                   float(lr), float(beta1), float(beta2), float(eps), _p(self.step_dev),
                                   _p(self.flat_bf16) if self.bf16_storage else None, _stream()))
        self.flat.grad = None


class _MLPFunction:
    """autograd.Function over the whole MLP (built lazily so that the module
    imports without torch)."""
    _cls = None

    @classmethod
    def apply(cls, x, flat, mlp, keep=True):
        if cls._cls is None:
            cls._cls = _make_mlp_function()
        return cls._cls.apply(x, flat, mlp, keep)


def _make_mlp_function():
    torch = _torch()

    class F(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, flat, mlp, keep):
            x = x.contiguous()
            if x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != mlp.dims[0]:
                raise OPFError(OPF_E_ARG, f"input must be float32 [B, {mlp.dims[0]}]")
            Bn = x.shape[0]
            if mlp.bf16_storage and mlp._bf16_version != mlp.flat._version:
                mlp.sync_bf16()  # the FP32 parameters were written from outside
            acts, pres = [x], []
            h = x
            nl = len(mlp.layout)
            for k in range(nl):
                wo, bo, fo, fi = mlp.layout[k]
                # a hidden layer's FP32 pre-activation serves only the backward
                pre = torch.empty(Bn, fo, dtype=torch.float32, device=x.device) if keep or k == nl - 1 else None
                ab = k < nl - 1 and mlp.act_bf16(k)
                act = None
                if k < nl - 1:
                    act = torch.empty(Bn, fo, dtype=torch.bfloat16 if ab else torch.float32, device=x.device)
                W, w_bf16 = mlp.mma_weight(k)
                gemm_mixed(0, h, h.dtype == torch.bfloat16, fi, W, w_bf16, fi, pre, fo, Bn, fo, fi, bias=mlp.bias(k),
                           act=act, act_bf16=ab)
                pres.append(pre)
                h = act if act is not None else pre
                if act is not None:
                    acts.append(act)
            ctx.mlp = mlp
            ctx.acts, ctx.pres = acts, pres
            return h

        @staticmethod
        def backward(ctx, gz):
            mlp = ctx.mlp
            gz = gz.contiguous()
            Bn = gz.shape[0]
            gflat = torch.empty(mlp.n_params, dtype=torch.float32, device=gz.device)
            nl = len(mlp.layout)
            dpre = gz
            chunks = (Bn + 127) // 128
            work = torch.empty(chunks * max(mlp.dims), dtype=torch.float32, device=gz.device)
            splits = [gemm_splits(fo, fi, Bn) for (_, _, fo, fi) in mlp.layout]
            sk = max(s * fo * fi if s > 1 else 0 for s, (_, _, fo, fi) in zip(splits, mlp.layout))
            skw = torch.empty(max(sk, 4), dtype=torch.float32, device=gz.device)
            parts = False  # work holds the first column-sum pass of dpre
            for k in range(nl - 1, -1, -1):
                wo, bo, fo, fi = mlp.layout[k]
                h_in = ctx.acts[k]
                d_bf16 = dpre.dtype == torch.bfloat16
                # dW [fo, fi] = dpre^T h_in (split over the batch); db = column sums of dpre
                gemm_mixed(2, dpre, d_bf16, fo, h_in, h_in.dtype == torch.bfloat16, fi, gflat[wo:wo + fo * fi], fi,
                           fo, fi, Bn, splits=splits[k], work=skw)
                if parts:
                    _check(lib().prox_colsum_parts(_p(work), chunks, fo, _p(gflat[bo:bo + fo]), ctypes.c_float(1.0),
                                                   _stream()))
                else:
                    _check(lib().prox_colsum(_p(dpre), Bn, fo, _p(work), _p(gflat[bo:bo + fo]), ctypes.c_float(1.0),
                                             _stream()))
                if k == 0:
                    break
                W, w_bf16 = mlp.mma_weight(k)
                if fi % 8 == 0:  # the BF16 result is the next product's k-contiguous operand
                    # dpre of layer k - 1 = (dpre W) * gelu'(pre of k - 1), in BF16 (the rounding every
                    # product applies to it), with its column sums' first pass in work
                    d = torch.empty(Bn, fi, dtype=torch.bfloat16, device=gz.device)
                    gemm_gelu_bwd(dpre, d_bf16, fo, W, w_bf16, fi, ctx.pres[k - 1], fi, d, fi, Bn, fi, fo, work)
                    parts = True
                else:
                    # dh [B, fi] = dpre W, then through the GELU of layer k - 1
                    dh = torch.empty(Bn, fi, dtype=torch.float32, device=gz.device)
                    gemm_mixed(1, dpre, d_bf16, fo, W, w_bf16, fi, dh, fi, Bn, fi, fo)
                    d = torch.empty_like(dh)
                    _check(lib().prox_gelu_bwd(_p(ctx.pres[k - 1]), _p(dh), _p(d), dh.numel(), _stream()))
                    parts = False
                dpre = d
            return None, gflat, None, None

    return F


# ------------------------------------------------------------------ squashing
def _make_squash_function():
    torch = _torch()

    class F(torch.autograd.Function):
        @staticmethod
        def forward(ctx, z, prox):
            z = z.contiguous()
            Bn = z.shape[0]
            X = torch.empty(Bn, prox.model.n, dtype=torch.float64, device=z.device)
            _check(lib().prox_squash_fwd(prox.model.handle, _p(z), Bn, float(prox.va_span), _p(X), _stream()))
            ctx.save_for_backward(z)
            ctx.prox = prox
            return X

        @staticmethod
        def backward(ctx, gX):
            (z,) = ctx.saved_tensors
            gX = gX.contiguous()
            dz = torch.empty_like(z)
            _check(lib().prox_squash_bwd(ctx.prox.model.handle, _p(z), z.shape[0], float(ctx.prox.va_span), _p(gX),
                                         None, None, 0.0, _p(dz), ctypes.c_float(1.0), _stream()))
            return dz, None

    return F


def _make_penalty_function():
    torch = _torch()

    class F(torch.autograd.Function):
        @staticmethod
        def forward(ctx, X, pen):
            Xf = X.detach().clone()
            pen.batch.flows(Xf)
            B, m = pen.B, pen.model.m
            dev = X.device
            Fo = torch.empty(B, dtype=torch.float64, device=dev)
            C = torch.empty(B * m, dtype=torch.float64, device=dev)
            Xflat = Xf.view(-1)
            pen.batch.eval(Xflat, F=Fo, C=C)
            loss = torch.empty(B, dtype=torch.float64, device=dev)
            cvio = torch.empty(B, dtype=torch.float64, device=dev)
            W = torch.empty(B * m, dtype=torch.float64, device=dev)
            gpq = torch.empty(B * 4 * pen.L, dtype=torch.float64, device=dev)
            # with a gradient to come, the flow rows of W get the VJP weights
            # in the same pass (prox_vjp_weights' closed form)
            vjp = int(bool(ctx.needs_input_grad[0]))
            _check(lib().prox_penalty(pen.model.handle, _p(C), _p(Xflat), _p(Fo), float(pen.obj_scale),
                                      float(pen.rho), B, vjp, _p(loss), _p(cvio), _p(W), _p(gpq), _stream()))
            pen.last = {"x": Xf, "f": Fo, "c": C.view(B, m), "cvio": cvio}
            ctx.save_for_backward(Xflat, W)
            ctx.pen = pen
            return loss

        @staticmethod
        def backward(ctx, gloss):
            Xflat, W = ctx.saved_tensors
            pen = ctx.pen
            B, n = pen.B, pen.model.n
            gX1 = pen.batch.jtprod(Xflat, W)  # W holds the VJP weights on the flow rows
            gX = torch.empty(B, n, dtype=torch.float64, device=Xflat.device)
            wb = gloss.detach().to(torch.float64).contiguous()
            _check(lib().prox_vjp_sum(pen.model.handle, _p(Xflat), _p(gX1), None, float(pen.obj_scale), _p(wb), B,
                                      _p(gX), _stream()))
            return gX, None

    return F


def _make_loss_function():
    """z -> per-instance loss in one autograd node.  On a model that
    prox_loss_fused takes, one launch computes the loss, Cvio and d loss / d z
    with each sample in one workgroup's LDS, and the backward scales that
    gradient by the incoming one (prox_scale_rows).  Otherwise: squashing, arc
    flows written into the same X, batch evaluation and penalty forward; J^T W
    and the fused objective / squashing backward (prox_loss_bwd) backward.
    Both give the values of Squash followed by Penalty (to rounding) without
    the copy of X and the [B, n] gradient in between.  keep: also leave x and
    c(x) of every sample in pen.last ("x": x only, in the one-launch form)."""
    torch = _torch()

    class F(torch.autograd.Function):
        @staticmethod
        def forward(ctx, z, prox, loads, keep):
            pen, va_span = prox.pen, prox.squash.va_span
            z = z.contiguous()
            B, n, m = pen.B, pen.model.n, pen.model.m
            dev = z.device
            vjp = bool(ctx.needs_input_grad[0])
            loss = torch.empty(B, dtype=torch.float64, device=dev)
            cvio = torch.empty(B, dtype=torch.float64, device=dev)
            ctx.fused = pen.fused
            if pen.fused:
                loads = loads.to(torch.float64).contiguous()
                gz = torch.empty(z.shape, dtype=torch.float64, device=dev) if vjp else None
                X = torch.empty(B, n, dtype=torch.float64, device=dev) if keep else None
                C = torch.empty(B, m, dtype=torch.float64, device=dev) if keep and keep != "x" else None
                _check(lib().prox_loss_fused(pen.model.handle, _p(z), B, float(va_span), _p(loads), float(pen.rho),
                                             float(pen.obj_scale), _p(loss), _p(cvio), _p(gz), _p(X), _p(C),
                                             _stream()))
                pen.last = {"x": X, "f": None, "c": C, "cvio": cvio}
                if vjp:
                    ctx.save_for_backward(gz)
                return loss
            pen.set_loads(loads[:, :pen.N], loads[:, pen.N:])
            X = torch.empty(B, n, dtype=torch.float64, device=dev)
            # the arc variables are left for the flows, which write every one
            _check(lib().prox_squash_fwd_vars(pen.model.handle, _p(z), B, float(va_span), _p(X), _stream()))
            pen.batch.flows(X)
            Xflat = X.view(-1)
            Fo = torch.empty(B, dtype=torch.float64, device=dev)
            C = torch.empty(B * m, dtype=torch.float64, device=dev)
            pen.batch.eval(Xflat, F=Fo, C=C)
            W = torch.empty(B * m, dtype=torch.float64, device=dev)
            # with a gradient to come, d pen / d (p, q) stays on chip when it fits
            gpq = None if vjp and 4 * pen.L <= 7680 else torch.empty(B * 4 * pen.L, dtype=torch.float64, device=dev)
            _check(lib().prox_penalty(pen.model.handle, _p(C), _p(Xflat), _p(Fo), float(pen.obj_scale),
                                      float(pen.rho), B, int(vjp), _p(loss), _p(cvio), _p(W), _p(gpq), _stream()))
            pen.last = {"x": X, "f": Fo, "c": C.view(B, m), "cvio": cvio}
            ctx.save_for_backward(z, Xflat, W)
            ctx.pen, ctx.va_span = pen, va_span
            return loss

        @staticmethod
        def backward(ctx, gloss):
            wb = gloss.detach().to(torch.float64).contiguous()
            if ctx.fused:
                (gz,) = ctx.saved_tensors
                B, D = gz.shape
                dz = torch.empty(B, D, dtype=torch.float32, device=gz.device)
                _check(lib().prox_scale_rows(_p(gz), _p(wb), B, D, _p(dz), _stream()))
                return dz, None, None, None
            z, Xflat, W = ctx.saved_tensors
            pen = ctx.pen
            gX1 = pen.batch.jtprod(Xflat, W)
            dz = torch.empty_like(z)
            _check(lib().prox_loss_bwd(pen.model.handle, _p(z), pen.B, float(ctx.va_span), _p(Xflat), _p(gX1),
                                       float(pen.obj_scale), _p(wb), _p(dz), _stream()))
            return dz, None, None, None

    return F


_FUN = {}


def _fun(name):
    if name not in _FUN:
        _FUN[name] = {"squash": _make_squash_function, "penalty": _make_penalty_function,
                      "loss": _make_loss_function}[name]()
    return _FUN[name]


# thresholds (p.u.) of the fallback curve: a prediction whose Cvio exceeds
# tau is discarded and the solver starts without it
FALLBACK_TAUS = (0.01, 0.02, 0.05, 0.1, 0.2, 0.5)


def fallback_curve(cvio, taus=FALLBACK_TAUS) -> dict:
    """{tau: share of samples whose Cvio (the largest violation over every
    row and bound, Sec. IV-A5) exceeds tau}."""
    cvio = np.asarray(cvio, dtype=np.float64)
    return {float(t): float(np.mean(cvio > t)) for t in taus}


class Penalty:
    """The FP64 penalty of B instances of one static model with per-instance
    loads: loss_b = rho * (squared violations of the non-flow rows and of the
    arc-variable bounds) + obj_scale * f_b at x_b with p, q := F(vm, va)."""

    def __init__(self, case: dict, B: int, rho: float = 10.0, obj_scale: float = 1e-3, device: int = 0):
        self.case = case
        self.model = opf.Model(case, device=device)
        self.B, self.L, self.N, self.G = int(B), int(case["n_branch"]), int(case["n_bus"]), int(case["n_gen"])
        self.rho, self.obj_scale = float(rho), float(obj_scale)
        pd = np.tile(np.asarray(case["pd"], np.float64), self.B)
        qd = np.tile(np.asarray(case["qd"], np.float64), self.B)
        self.batch = opf.Batch([self.model], np.zeros(self.B, np.int32), pd, qd)
        fits = lib().prox_loss_fused_fits(self.model.handle)
        _check(min(fits, 0))
        # the loss node's one-launch form (prox_loss_fused) when the model
        # has what it takes; else the chain of batch launches
        self.fused = fits == 1
        self.last = None

    def set_loads(self, pd, qd):
        """pd, qd: float64 device tensors [B, N]."""
        self.batch.set_loads(pd.contiguous().view(-1), qd.contiguous().view(-1))

    def __call__(self, X):
        """Per-instance loss [B] of X [B, n] (FP64; its p, q are ignored)."""
        return _fun("penalty").apply(X, self)

    def close(self):
        self.batch.close()
        self.model.close()


class Squash:
    def __init__(self, model, va_span: float = 0.3):
        self.model = model
        self.va_span = float(va_span)

    def __call__(self, z):
        return _fun("squash").apply(z, self)


class WarmStartProxy:
    """MLP + squashing + penalty for one network: loads (pd, qd) -> x."""

    def __init__(self, case: dict, B: int, width: int = 1024, depth: int = 3, rho: float = 10.0,
                 obj_scale: float = 1e-3, va_span: float = 0.3, seed: int = 0, device: int = 0):
        torch = _torch()
        N, G = int(case["n_bus"]), int(case["n_gen"])
        if N % 2 or G % 2:
            raise OPFError(OPF_E_ARG, "the proxy needs an even number of buses and of generators")
        self.case, self.N, self.G, self.B = case, N, G, int(B)
        self.pen = Penalty(case, B, rho=rho, obj_scale=obj_scale, device=device)
        self.squash = Squash(self.pen.model, va_span)
        self.mlp = MLP(2 * N, 2 * N + 2 * G, width=width, depth=depth, seed=seed, device=device)
        self.dev = torch.device("cuda", device)
        base = np.concatenate([np.asarray(case["pd"], np.float64), np.asarray(case["qd"], np.float64)])
        self.base = torch.as_tensor(base, device=self.dev)
        self.spread = 0.3
        scale = self.spread / math.sqrt(3.0) * np.abs(base)
        self.inv_scale = torch.as_tensor(np.where(scale > 0, 1.0 / np.maximum(scale, 1e-300), 0.0), device=self.dev)
        b = self.pen.model.bounds()
        self.x0 = b["x0"]
        self.native = True  # train_step through prox_train_step where it applies
        self._ws = None

    # -- data: seeded +-spread uniform scalings of the base loads (one factor per bus)
    def sample(self, gen):
        """(loads [B, 2N] FP64, features [B, 2N] FP32) from B uniform draws
        per bus of gen (prox_sample_loads: the values of sample_reference in
        one launch)."""
        torch = _torch()
        r = torch.rand(self.B, self.N, generator=gen, device=self.dev, dtype=torch.float64)
        loads = torch.empty(self.B, 2 * self.N, dtype=torch.float64, device=self.dev)
        feats = torch.empty(self.B, 2 * self.N, dtype=torch.float32, device=self.dev)
        _check(lib().prox_sample_loads(_p(r), _p(self.base), _p(self.inv_scale), float(self.spread), self.B, self.N,
                                       _p(loads), _p(feats), _stream()))
        return loads, feats

    def sample_reference(self, gen):
        """sample as torch operations (the tests' reference)."""
        torch = _torch()
        u = torch.rand(self.B, self.N, generator=gen, device=self.dev, dtype=torch.float64) * 2.0 - 1.0
        fac = 1.0 + self.spread * torch.cat([u, u], dim=1)
        loads = self.base[None, :] * fac
        feats = ((loads - self.base[None, :]) * self.inv_scale[None, :]).to(torch.float32)
        return loads, feats

    def loss(self, loads, feats, keep=False):
        """Per-sample loss [B] of the network's prediction on these loads
        (keep: also leave x and c(x) in pen.last; "x": x only where the loss
        runs as one launch)."""
        return _fun("loss").apply(self.mlp(feats), self, loads, keep)

    def loss_unfused(self, loads, feats):
        """loss through Squash and Penalty as two autograd nodes (the same
        values; kept as the reference for the fused node)."""
        self.pen.set_loads(loads[:, :self.N], loads[:, self.N:])
        X = self.squash(self.mlp(feats))
        return self.pen(X)

    def train_step(self, loads, feats, lr=3e-4):
        """One step on the mean loss: forward, backward and Adam.  On a model
        that the fused loss takes, one library call issues every launch
        (prox_train_step); else the autograd path.  Both give the same
        parameters bit for bit."""
        B = feats.shape[0]
        if self.native and self.pen.fused and B % 4 == 0:
            return self._train_step_native(loads, feats, lr)
        return self.train_step_autograd(loads, feats, lr)

    def train_step_autograd(self, loads, feats, lr=3e-4):
        lb = self.loss(loads, feats)
        loss = lb.mean()
        loss.backward()
        self.mlp.adam_step(lr=lr)
        return loss.detach()

    def train_step_phases(self, loads, feats, lr=3e-4):
        """The library-issued step with the GPU time of its phases (ms):
        (mean loss, {forward, loss, backward, adam}); waits for the step."""
        ph = (ctypes.c_float * 4)()
        loss = self._train_step_native(loads, feats, lr, ph)
        return loss, dict(zip(("forward", "loss", "backward", "adam"), (float(v) for v in ph)))

    def _train_step_native(self, loads, feats, lr, phases=None):
        torch = _torch()
        mlp = self.mlp
        B = feats.shape[0]
        # the library reads these through raw pointers: their shapes are checked here
        if tuple(feats.shape) != (B, mlp.dims[0]) or tuple(loads.shape) != (B, 2 * self.N):
            raise OPFError(OPF_E_ARG, f"feats must be [B, {mlp.dims[0]}] and loads [B, {2 * self.N}]")
        if feats.device != self.dev or loads.device != self.dev:
            raise OPFError(OPF_E_ARG, "feats and loads must be on the proxy's device")
        if self._ws is None or self._ws[0] != B:
            nbytes = ctypes.c_int64()
            _check(lib().prox_train_step_bytes(ctypes.byref(mlp.desc()), B, ctypes.byref(nbytes)))
            self._ws = (B, torch.empty(nbytes.value, dtype=torch.uint8, device=self.dev),
                        torch.empty(B, dtype=torch.float64, device=self.dev),
                        torch.empty(B, dtype=torch.float64, device=self.dev))
        _, ws, lb, cv = self._ws
        mlp.step += 1
        if mlp.bf16_storage and mlp._bf16_version != mlp.flat._version:
            mlp.sync_bf16()  # the FP32 parameters were written from outside
        feats = feats.to(torch.float32).contiguous()
        loads = loads.to(torch.float64).contiguous()
        _check(lib().prox_train_step(self.pen.model.handle, ctypes.byref(mlp.desc()), _p(feats), _p(loads), B,
                                     float(self.squash.va_span), float(self.pen.rho), float(self.pen.obj_scale),
                                     float(lr), 0.9, 0.999, 1e-8, _p(ws), ws.numel(), _p(lb), _p(cv), phases,
                                     _stream()))
        self.pen.last = {"x": None, "f": None, "c": None, "cvio": cv}
        return lb.mean()

    def predict(self, loads, feats):
        """(x with p, q := flows, largest violation per sample) under no grad."""
        torch = _torch()
        with torch.no_grad():
            self.loss(loads, feats, keep="x")
        return self.pen.last["x"], self.pen.last["cvio"]

    def baseline(self, loads):
        """The plain starting point x0 scored on the same loads: (x, cvio)."""
        return self._score(loads, self.x0)

    def flat_start(self, loads):
        """The flat start scored on the same loads: vm = 1, va = 0, pg and qg
        at the middle of their bounds, p and q the branch flows: (x, cvio)."""
        torch = _torch()
        b = self.pen.model.bounds()
        x = self.x0.clone()
        for blk in ("pg", "qg"):
            o, n = self.pen.model.block(blk)
            x[o:o + n] = 0.5 * (b["lvar"][o:o + n] + b["uvar"][o:o + n])
        torch.cuda.synchronize()
        return self._score(loads, x)

    def _score(self, loads, x):
        torch = _torch()
        with torch.no_grad():
            self.pen.set_loads(loads[:, :self.N], loads[:, self.N:])
            X = x[None, :].expand(self.B, -1).contiguous()
            self.pen(X)
        return self.pen.last["x"], self.pen.last["cvio"]

    def close(self):
        self.pen.close()
