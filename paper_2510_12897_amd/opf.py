"""Python binding of libopf (ctypes; argument marshalling only).

Every callback runs in the HIP kernels of libopf.so; this module only turns
torch tensors into device pointers and the current torch stream into a
hipStream_t.  There is no CPU fallback: if the library is missing the import
of a Model fails with OPFError.

Cases are dicts of numpy arrays with the field names of ``opf_case``
(``synth.network`` produces them); options are the keyword arguments
``n_periods``, ``pd_t``, ``qd_t``, ``ramp_ratio``, ``n_cont``, ``outaged`` and
``form`` ("polar", the default, or "rect" for bus variables (vr, vi)),
``storage`` (a dict of per-unit arrays named as the fields of opf_storage),
``stor_dt``, ``stor_comp`` and ``devices`` (per-device arrays named as the
fields of opf_devices).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libopf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "opf.h")

OPF_OK, OPF_E_ARG, OPF_E_CASE, OPF_E_NOMEM, OPF_E_HIP, OPF_E_STATE = 0, -1, -2, -3, -4, -5

# bus blocks: va, vm (polar) or vr, vi (rectangular form), same positions
VAR_BLOCKS = {"va": 0, "vm": 1, "pg": 2, "qg": 3, "p": 4, "q": 5, "vr": 0, "vi": 1,
              "ps": 6, "qs": 7, "qsc": 8, "se": 9, "sc": 10, "sd": 11, "u": 12}
CON_BLOCKS = {name: 16 + k for k, name in enumerate(
    ["ref", "p_fr", "q_fr", "p_to", "q_to", "angle", "bal_p", "bal_q", "thermal_fr", "thermal_to", "ramp",
     "angle_lo", "vmag", "soc", "stor_loss_p", "stor_loss_q", "stor_thermal", "stor_comp", "dev_ramp", "dev_init"])}
FORMS = {"polar": 0, "rect": 1}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


class OPFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"opf error {code}: {msg}")
        self.code = code


class _Case(ctypes.Structure):
    _fields_ = [
        ("n_bus", ctypes.c_int32), ("n_branch", ctypes.c_int32),
        ("n_gen", ctypes.c_int32), ("n_ref", ctypes.c_int32),
        ("pd", _dp), ("qd", _dp), ("gs", _dp), ("bs", _dp), ("vmin", _dp), ("vmax", _dp),
        ("ref_bus", _ip), ("f_bus", _ip), ("t_bus", _ip),
        ("r", _dp), ("x", _dp), ("b", _dp), ("tap", _dp), ("shift", _dp), ("rate_a", _dp),
        ("angmin", _dp), ("angmax", _dp),
        ("gen_bus", _ip),
        ("pmin", _dp), ("pmax", _dp), ("qmin", _dp), ("qmax", _dp),
        ("c2", _dp), ("c1", _dp), ("c0", _dp),
    ]


STOR_FIELDS = ("emax", "chmax", "dismax", "rating", "qmin", "qmax", "eta_c", "eta_d", "r", "x", "ploss", "qloss",
               "e0")
DEV_FIELDS = ("cp", "cq", "cost", "lo", "hi", "ramp", "init_lo", "init_hi")


class _Storage(ctypes.Structure):
    _fields_ = ([("n", ctypes.c_int32), ("bus", _ip)] + [(k, _dp) for k in STOR_FIELDS]
                + [("dt", ctypes.c_double), ("comp", ctypes.c_int32)])


class _Devices(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("bus", _ip)] + [(k, _dp) for k in DEV_FIELDS]


class MlpDesc(ctypes.Structure):
    """prox_mlp_desc: the proxy MLP's device buffers (include/opf.h)."""
    _fields_ = [("n_layers", ctypes.c_int32), ("dims", ctypes.POINTER(ctypes.c_int32)), ("flat", _vp),
                ("flat_bf16", _vp), ("m1", _vp), ("m2", _vp), ("step", _vp)]


class _Opts(ctypes.Structure):
    _fields_ = [
        ("n_periods", ctypes.c_int32), ("pd_t", _dp), ("qd_t", _dp),
        ("ramp_ratio", ctypes.c_double), ("n_cont", ctypes.c_int32), ("outaged_branch", _ip),
        ("form", ctypes.c_int32), ("storage", ctypes.POINTER(_Storage)), ("devices", ctypes.POINTER(_Devices)),
    ]


_lib = None


def declared_symbols() -> list:
    """Names of every function declared in include/opf.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:opf|prox)_[a-z0-9_]+)\s*\(", text)))


def lib():
    """Load libopf.so (built by ``paper_2510_12897_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OPFError(OPF_E_STATE, f"{LIB_PATH} is missing: run `python -m paper_2510_12897_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "opf_last_error": ([], ctypes.c_char_p),
        "opf_set_single_launch_limit": ([ctypes.c_int64], ctypes.c_int),
        "opf_case_validate": ([P(_Case), P(_Opts)], ctypes.c_int),
        "opf_case_dims": ([P(_Case), P(_Opts), _i64p, _i64p, _i64p, _i64p], ctypes.c_int),
        "opf_case_structure": ([P(_Case), P(_Opts), _vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_case_bounds": ([P(_Case), P(_Opts), _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_model_create": ([P(_Case), P(_Opts), ctypes.c_int, P(_vp)], ctypes.c_int),
        "opf_model_destroy": ([_vp], ctypes.c_int),
        "opf_model_dims": ([_vp, _i64p, _i64p, _i64p, _i64p], ctypes.c_int),
        "opf_model_launches": ([_vp, P(ctypes.c_int32), _i64p], ctypes.c_int),
        "opf_model_blocks": ([_vp, ctypes.c_int32, _i64p, _i64p], ctypes.c_int),
        "opf_bounds": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_obj": ([_vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_grad": ([_vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_cons": ([_vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_jac_structure": ([_vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_jac_coord": ([_vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_hess_structure": ([_vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_hess_coord": ([_vp, _vp, _vp, ctypes.c_double, _vp, _vp], ctypes.c_int),
        "opf_eval_set": ([_vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_jtprod": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_eval_set_noalloc": ([_vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_batch_create": ([P(_vp), ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32, P(_vp)], ctypes.c_int),
        "opf_batch_destroy": ([_vp], ctypes.c_int),
        "opf_batch_offsets": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_batch_tune": ([_vp, _vp], ctypes.c_int),
        "opf_batch_schedule": ([_vp, P(ctypes.c_int32)], ctypes.c_int),
        "opf_batch_set_schedule": ([_vp, ctypes.c_int32], ctypes.c_int),
        "opf_batch_eval": ([_vp] + [_vp] * 8 + [_vp], ctypes.c_int),
        "opf_batch_jtprod": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_batch_set_loads": ([_vp, _vp, _vp, _vp], ctypes.c_int),
        "opf_batch_flows": ([_vp, _vp, _vp], ctypes.c_int),
        "prox_gemm_bf16": ([ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int,
                            ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp], ctypes.c_int),
        "prox_gemm_bf16_splitk": ([ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int,
                                   _vp, _vp], ctypes.c_int),
        "prox_gemm_bf16_mixed": ([ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int,
                                  _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp], ctypes.c_int),
        "prox_to_bf16": ([_vp, ctypes.c_int64, _vp, _vp], ctypes.c_int),
        "prox_gemm_splits": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "prox_gelu_bwd": ([_vp, _vp, _vp, ctypes.c_int64, _vp], ctypes.c_int),
        "prox_colsum": ([_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_float, _vp], ctypes.c_int),
        "prox_colsum_parts": ([_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_float, _vp], ctypes.c_int),
        "prox_gemm_gelu_bwd": ([_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int,
                                _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp], ctypes.c_int),
        "prox_adam": ([_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                       ctypes.c_float, ctypes.c_int, _vp], ctypes.c_int),
        "prox_adam_dev": ([_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, _vp, _vp, _vp], ctypes.c_int),
        "prox_squash_fwd": ([_vp, _vp, ctypes.c_int, ctypes.c_double, _vp, _vp], ctypes.c_int),
        "prox_squash_fwd_vars": ([_vp, _vp, ctypes.c_int, ctypes.c_double, _vp, _vp], ctypes.c_int),
        "prox_squash_bwd": ([_vp, _vp, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp, ctypes.c_double, _vp,
                             ctypes.c_float, _vp], ctypes.c_int),
        "prox_penalty": ([_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp, _vp,
                          _vp, _vp, _vp], ctypes.c_int),
        "prox_vjp_weights": ([_vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp], ctypes.c_int),
        "prox_vjp_sum": ([_vp, _vp, _vp, _vp, ctypes.c_double, _vp, ctypes.c_int, _vp, _vp], ctypes.c_int),
        "prox_loss_bwd": ([_vp, _vp, ctypes.c_int, ctypes.c_double, _vp, _vp, ctypes.c_double, _vp, _vp, _vp],
                          ctypes.c_int),
        "prox_loss_fused": ([_vp, _vp, ctypes.c_int, ctypes.c_double, _vp, ctypes.c_double, ctypes.c_double, _vp,
                             _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "prox_loss_fused_fits": ([_vp], ctypes.c_int),
        "prox_scale_rows": ([_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp], ctypes.c_int),
        "prox_sample_loads": ([_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp],
                              ctypes.c_int),
        "prox_train_step_bytes": ([P(MlpDesc), ctypes.c_int, _i64p], ctypes.c_int),
        "prox_train_step": ([_vp, P(MlpDesc), _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp,
                             ctypes.c_int64, _vp, _vp, P(ctypes.c_float), _vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
# every callback pair ever installed: a model calls its creation-time hook
# again when it is destroyed, so none may be freed
_hooks = []


def set_allocator(alloc=None, release=None):
    """Device memory hook for models and batches created afterwards:
    alloc(nbytes) -> int device address (0 on failure, which makes create
    fail with OPF_E_NOMEM), release(address).  None, None restores hipMalloc
    / hipFree."""
    L = lib()
    L.opf_set_allocator.argtypes = [_ALLOC_FN, _RELEASE_FN, ctypes.c_void_p]
    L.opf_set_allocator.restype = None
    if alloc is None:
        L.opf_set_allocator(_ALLOC_FN(), _RELEASE_FN(), None)
        return
    a = _ALLOC_FN(lambda n, ctx: int(alloc(int(n)) or 0) or None)
    r = _RELEASE_FN(lambda p, ctx: release(int(p)) if p else None)
    L.opf_set_allocator(a, r, None)
    _hooks.append((a, r))


def use_torch_allocator(device: int = 0):
    """Route model and batch storage through torch's caching allocator on
    `device` (its current stream at allocation time)."""
    torch = _torch()

    def alloc(n):
        return torch.cuda.caching_allocator_alloc(n, device)

    def release(p):
        torch.cuda.caching_allocator_delete(p)

    set_allocator(alloc, release)


def set_single_launch_limit(waves: int):
    """Models created afterwards evaluate a callback set in one launch when it
    is at most `waves` work items (0: always two launches)."""
    _check(lib().opf_set_single_launch_limit(int(waves)))


def _check(rc: int):
    if rc != OPF_OK:
        raise OPFError(rc, lib().opf_last_error().decode())


# ---------------------------------------------------------------- marshalling
def _case_struct(case: dict, n_periods=1, pd_t=None, qd_t=None, ramp_ratio=0.0, n_cont=0, outaged=None,
                 form="polar", storage=None, stor_dt=1.0, stor_comp=False, devices=None):
    keep = []

    def d(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(_dp)

    def i(a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        keep.append(a)
        return a.ctypes.data_as(_ip)

    c = _Case()
    c.n_bus, c.n_branch, c.n_gen = int(case["n_bus"]), int(case["n_branch"]), int(case["n_gen"])
    c.n_ref = len(case["ref_bus"])
    for k in ("pd", "qd", "gs", "bs", "vmin", "vmax", "r", "x", "b", "tap", "shift", "rate_a",
              "angmin", "angmax", "pmin", "pmax", "qmin", "qmax", "c2", "c1", "c0"):
        setattr(c, k, d(case[k]))
    for k in ("ref_bus", "f_bus", "t_bus", "gen_bus"):
        setattr(c, k, i(case[k]))
    o = _Opts()
    o.n_periods = int(n_periods)
    o.pd_t = d(pd_t) if pd_t is not None else _dp()
    o.qd_t = d(qd_t) if qd_t is not None else _dp()
    o.ramp_ratio = float(ramp_ratio)
    o.n_cont = int(n_cont)
    o.outaged_branch = i(outaged) if outaged is not None else _ip()
    if form not in FORMS:
        raise OPFError(OPF_E_ARG, f"unknown form {form!r} (polar or rect)")
    o.form = FORMS[form]
    if storage is not None:
        st = _Storage()
        st.n = len(storage["bus"])
        st.bus = i(storage["bus"])
        for k in STOR_FIELDS:
            setattr(st, k, d(storage[k]))
        st.dt = float(stor_dt)
        st.comp = int(bool(stor_comp))
        keep.append(st)
        o.storage = ctypes.pointer(st)
    if devices is not None:
        dv = _Devices()
        dv.n = len(devices["bus"])
        dv.bus = i(devices["bus"])
        for k in DEV_FIELDS:
            setattr(dv, k, d(devices[k]))
        keep.append(dv)
        o.devices = ctypes.pointer(dv)
    return c, o, keep


def case_validate(case: dict, **opts):
    c, o, keep = _case_struct(case, **opts)
    _check(lib().opf_case_validate(ctypes.byref(c), ctypes.byref(o)))


def case_dims(case: dict, **opts):
    """(n, m, nnzj, nnzh) computed on the host."""
    c, o, keep = _case_struct(case, **opts)
    v = [ctypes.c_int64() for _ in range(4)]
    _check(lib().opf_case_dims(ctypes.byref(c), ctypes.byref(o), *[ctypes.byref(z) for z in v]))
    return tuple(z.value for z in v)


def case_structure(case: dict, **opts):
    """Host-built Jacobian and Hessian patterns (numpy int32 arrays)."""
    n, m, nnzj, nnzh = case_dims(case, **opts)
    c, o, keep = _case_struct(case, **opts)
    out = [np.empty(max(k, 1), np.int32) for k in (nnzj, nnzj, nnzh, nnzh)]
    _check(lib().opf_case_structure(ctypes.byref(c), ctypes.byref(o), *[a.ctypes.data for a in out]))
    return out[0][:nnzj], out[1][:nnzj], out[2][:nnzh], out[3][:nnzh]


def case_bounds(case: dict, **opts) -> dict:
    n, m, _, _ = case_dims(case, **opts)
    c, o, keep = _case_struct(case, **opts)
    out = {"lvar": np.empty(n), "uvar": np.empty(n), "lcon": np.empty(max(m, 1)),
           "ucon": np.empty(max(m, 1)), "x0": np.empty(n)}
    _check(lib().opf_case_bounds(ctypes.byref(c), ctypes.byref(o),
                                 *[out[k].ctypes.data for k in ("lvar", "uvar", "lcon", "ucon", "x0")]))
    out["lcon"], out["ucon"] = out["lcon"][:m], out["ucon"][:m]
    return out


# ---------------------------------------------------------------- device side
def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, n=None, dtype=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor of the expected size and dtype."""
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise OPFError(OPF_E_ARG, f"{name} must be a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise OPFError(OPF_E_ARG, f"{name} must have dtype {dtype}, not {t.dtype}")
    if not t.is_contiguous():
        raise OPFError(OPF_E_ARG, f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise OPFError(OPF_E_ARG, f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


class Model:
    """One AC-OPF model resident on a GPU, with the NLPModels callbacks."""

    def __init__(self, case: dict, device: int = 0, **opts):
        lib()
        c, o, keep = _case_struct(case, **opts)
        h = _vp()
        _check(lib().opf_model_create(ctypes.byref(c), ctypes.byref(o), int(device), ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        self.opts = dict(opts)
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib().opf_model_dims(h, *[ctypes.byref(z) for z in v]))
        self.n, self.m, self.nnzj, self.nnzh = (z.value for z in v)

    def launch_shape(self):
        """(launches per callback set: 1 or 2, 64-lane work items per set)."""
        n, k = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().opf_model_launches(self._h, ctypes.byref(n), ctypes.byref(k)))
        return n.value, k.value

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().opf_model_destroy(self._h))
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- helpers
    def _dev(self):
        return _torch().device("cuda", self.device)

    def _new(self, n, dtype=None):
        torch = _torch()
        return torch.empty(max(n, 0), dtype=dtype or torch.float64, device=self._dev())

    def block(self, name: str):
        """(offset, length) of a variable block (va, vm, pg, qg, p, q) or a
        constraint block (ref, p_fr, ..., ramp)."""
        which = VAR_BLOCKS.get(name, CON_BLOCKS.get(name))
        if which is None:
            raise OPFError(OPF_E_ARG, f"unknown block {name!r}")
        o, n = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().opf_model_blocks(self._h, which, ctypes.byref(o), ctypes.byref(n)))
        return o.value, n.value

    # -- callbacks (Listing 1)
    def bounds(self) -> dict:
        out = {k: self._new(self.n) for k in ("lvar", "uvar", "x0")}
        out.update({k: self._new(self.m) for k in ("lcon", "ucon")})
        _check(lib().opf_bounds(self._h, *[_ptr(out[k]) for k in ("lvar", "uvar", "lcon", "ucon", "x0")],
                                _stream()))
        return out

    def obj(self, x, out=None):
        torch = _torch()
        out = self._new(1) if out is None else out
        _check(lib().opf_obj(self._h, _ptr(x, self.n, torch.float64, "x"), _ptr(out, 1, torch.float64, "f"),
                             _stream()))
        return out.view(()) if out.numel() == 1 else out

    def grad(self, x, out=None):
        torch = _torch()
        out = self._new(self.n) if out is None else out
        _check(lib().opf_grad(self._h, _ptr(x, self.n, torch.float64, "x"), _ptr(out, self.n, torch.float64, "g"),
                              _stream()))
        return out

    def cons(self, x, out=None):
        torch = _torch()
        out = self._new(self.m) if out is None else out
        _check(lib().opf_cons(self._h, _ptr(x, self.n, torch.float64, "x"), _ptr(out, self.m, torch.float64, "c"),
                              _stream()))
        return out

    def jac_structure(self):
        torch = _torch()
        rows, cols = self._new(self.nnzj, torch.int32), self._new(self.nnzj, torch.int32)
        _check(lib().opf_jac_structure(self._h, _ptr(rows), _ptr(cols), _stream()))
        return rows, cols

    def jac_coord(self, x, out=None):
        torch = _torch()
        out = self._new(self.nnzj) if out is None else out
        _check(lib().opf_jac_coord(self._h, _ptr(x, self.n, torch.float64, "x"),
                                   _ptr(out, self.nnzj, torch.float64, "vals"), _stream()))
        return out

    def hess_structure(self):
        torch = _torch()
        rows, cols = self._new(self.nnzh, torch.int32), self._new(self.nnzh, torch.int32)
        _check(lib().opf_hess_structure(self._h, _ptr(rows), _ptr(cols), _stream()))
        return rows, cols

    def hess_coord(self, x, y, obj_weight: float = 1.0, out=None):
        torch = _torch()
        out = self._new(self.nnzh) if out is None else out
        _check(lib().opf_hess_coord(self._h, _ptr(x, self.n, torch.float64, "x"),
                                    _ptr(y, self.m, torch.float64, "y"), float(obj_weight),
                                    _ptr(out, self.nnzh, torch.float64, "vals"), _stream()))
        return out

    def eval_set(self, x, y, obj_weight: float = 1.0, f=None, g=None, c=None, jvals=None, hvals=None,
                 alloc: bool = True):
        """All five callbacks in one launch.  With alloc=True missing outputs
        are allocated; with alloc=False only the given ones are computed."""
        torch = _torch()
        if alloc:
            f = self._new(1) if f is None else f
            g = self._new(self.n) if g is None else g
            c = self._new(self.m) if c is None else c
            jvals = self._new(self.nnzj) if jvals is None else jvals
            hvals = self._new(self.nnzh) if hvals is None else hvals
        _check(lib().opf_eval_set(
            self._h, _ptr(x, self.n, torch.float64, "x"), _ptr(y, self.m, torch.float64, "y"),
            float(obj_weight), _ptr(f, 1, torch.float64, "f"), _ptr(g, self.n, torch.float64, "g"),
            _ptr(c, self.m, torch.float64, "c"), _ptr(jvals, self.nnzj, torch.float64, "jvals"),
            _ptr(hvals, self.nnzh, torch.float64, "hvals"), _stream()))
        return f, g, c, jvals, hvals

    def eval_set_noalloc(self, x, y, obj_weight: float = 1.0, f=None, g=None, c=None, jvals=None, hvals=None):
        """eval_set through the entry point that allocates nothing (its
        scratch is the library's fixed per-device array); only the given
        outputs are computed."""
        torch = _torch()
        _check(lib().opf_eval_set_noalloc(
            self._h, _ptr(x, self.n, torch.float64, "x"), _ptr(y, self.m, torch.float64, "y"),
            float(obj_weight), _ptr(f, 1, torch.float64, "f"), _ptr(g, self.n, torch.float64, "g"),
            _ptr(c, self.m, torch.float64, "c"), _ptr(jvals, self.nnzj, torch.float64, "jvals"),
            _ptr(hvals, self.nnzh, torch.float64, "hvals"), _stream()))
        return f, g, c, jvals, hvals

    def jtprod(self, x, v, out=None):
        torch = _torch()
        out = self._new(self.n) if out is None else out
        _check(lib().opf_jtprod(self._h, _ptr(x, self.n, torch.float64, "x"), _ptr(v, self.m, torch.float64, "v"),
                                _ptr(out, self.n, torch.float64, "out"), _stream()))
        return out


class Batch:
    """Many instances (of possibly different models) evaluated by one
    persistent kernel launch."""

    def __init__(self, models, inst_model, inst_pd=None, inst_qd=None):
        lib()
        self.models = list(models)
        arr = (_vp * len(self.models))(*[m.handle for m in self.models])
        im = np.ascontiguousarray(inst_model, dtype=np.int32)
        self.n_inst = int(im.size)
        self._keep = [arr, im]
        pd = qd = None
        if inst_pd is not None:
            pd = np.ascontiguousarray(inst_pd, dtype=np.float64).reshape(-1)
            qd = np.ascontiguousarray(inst_qd, dtype=np.float64).reshape(-1)
            self._keep += [pd, qd]
        h = _vp()
        _check(lib().opf_batch_create(arr, len(self.models), im.ctypes.data,
                                      pd.ctypes.data if pd is not None else None,
                                      qd.ctypes.data if qd is not None else None, self.n_inst,
                                      ctypes.byref(h)))
        self._h = h
        self.device = self.models[0].device
        offs = [np.zeros(self.n_inst + 1, np.int64) for _ in range(4)]
        _check(lib().opf_batch_offsets(h, *[o.ctypes.data for o in offs]))
        self.xoff, self.coff, self.joff, self.hoff = offs
        self.n, self.m, self.nnzj, self.nnzh = (int(o[-1]) for o in offs)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().opf_batch_destroy(self._h))
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tune(self):
        _check(lib().opf_batch_tune(self._h, _stream()))
        return self.schedule()

    def schedule(self) -> int:
        """-1: one launch; 0: two flat launches (one workgroup per item);
        else two persistent launches of this many workgroups per CU."""
        wg = ctypes.c_int32()
        _check(lib().opf_batch_schedule(self._h, ctypes.byref(wg)))
        return wg.value

    def set_schedule(self, wg_per_cu: int):
        _check(lib().opf_batch_set_schedule(self._h, int(wg_per_cu)))

    def _new(self, n):
        torch = _torch()
        return torch.empty(max(n, 0), dtype=torch.float64, device=torch.device("cuda", self.device))

    def eval(self, X, Y=None, sigma=None, F=None, G=None, C=None, J=None, H=None):
        torch = _torch()
        d = torch.float64
        _check(lib().opf_batch_eval(
            self._h, _ptr(X, self.n, d, "X"), _ptr(Y, self.m, d, "Y"), _ptr(sigma, self.n_inst, d, "sigma"),
            _ptr(F, self.n_inst, d, "F"), _ptr(G, self.n, d, "G"), _ptr(C, self.m, d, "C"),
            _ptr(J, self.nnzj, d, "J"), _ptr(H, self.nnzh, d, "H"), _stream()))
        return F, G, C, J, H

    def jtprod(self, X, V, OUT=None):
        torch = _torch()
        d = torch.float64
        OUT = self._new(self.n) if OUT is None else OUT
        _check(lib().opf_batch_jtprod(self._h, _ptr(X, self.n, d, "X"), _ptr(V, self.m, d, "V"),
                                      _ptr(OUT, self.n, d, "OUT"), _stream()))
        return OUT

    def set_loads(self, pd, qd):
        """Replace every instance's loads (device tensors laid out like the
        inst_pd / inst_qd given at creation)."""
        torch = _torch()
        _check(lib().opf_batch_set_loads(self._h, _ptr(pd, None, torch.float64, "pd"),
                                         _ptr(qd, None, torch.float64, "qd"), _stream()))

    def flows(self, X):
        """Overwrite the arc variables of X (in place) by the branch flows at
        X's voltages."""
        torch = _torch()
        _check(lib().opf_batch_flows(self._h, _ptr(X, self.n, torch.float64, "X"), _stream()))
        return X
