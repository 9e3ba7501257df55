"""Python access to the CPU oracle (opf_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The HIP library never loads it, and this module
imports nothing from the HIP package.

Cases are dicts of numpy arrays with the field names of the network
generator; options are keyword arguments ``n_periods``, ``pd_t``, ``qd_t``,
``ramp_ratio``, ``n_cont``, ``outaged``, ``form`` ("polar", the default,
or "rect": bus variables (vr, vi) in place of (va, vm)), ``storage`` (a dict
of per-unit arrays: bus, emax, chmax, dismax, rating, qmin, qmax, eta_c,
eta_d, r, x, ploss, qloss, e0), ``stor_dt``, ``stor_comp`` and ``devices``
(per-device arrays: bus, cp, cq, cost, lo, hi, ramp, init_lo, init_hi).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "opf_oracle.c")
LIB_PATH = os.path.join(HERE, "libopf_oracle.so")

W_OBJ, W_CONS, W_JAC, W_HESS = 1, 2, 4, 8
W_ALL = W_OBJ | W_CONS | W_JAC | W_HESS

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build() -> str:
    """Compile the oracle with gcc: plain C99, no FMA contraction."""
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                           "-Wall", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Case(ctypes.Structure):
    _fields_ = [
        ("n_bus", ctypes.c_int32), ("n_branch", ctypes.c_int32),
        ("n_gen", ctypes.c_int32), ("n_ref", ctypes.c_int32),
        ("pd", _dp), ("qd", _dp), ("gs", _dp), ("bs", _dp), ("vmin", _dp), ("vmax", _dp),
        ("ref_bus", _ip), ("f_bus", _ip), ("t_bus", _ip),
        ("r", _dp), ("x", _dp), ("b", _dp), ("tap", _dp), ("shift", _dp),
        ("rate_a", _dp), ("angmin", _dp), ("angmax", _dp),
        ("gen_bus", _ip),
        ("pmin", _dp), ("pmax", _dp), ("qmin", _dp), ("qmax", _dp),
        ("c2", _dp), ("c1", _dp), ("c0", _dp),
        ("n_periods", ctypes.c_int32), ("pd_t", _dp), ("qd_t", _dp),
        ("ramp_ratio", ctypes.c_double),
        ("n_cont", ctypes.c_int32), ("outaged", _ip),
        ("form", ctypes.c_int32),
        ("n_stor", ctypes.c_int32), ("stor_bus", _ip),
        ("stor_emax", _dp), ("stor_chmax", _dp), ("stor_dismax", _dp), ("stor_rating", _dp),
        ("stor_qmin", _dp), ("stor_qmax", _dp), ("stor_eta_c", _dp), ("stor_eta_d", _dp),
        ("stor_r", _dp), ("stor_x", _dp), ("stor_ploss", _dp), ("stor_qloss", _dp), ("stor_e0", _dp),
        ("stor_dt", ctypes.c_double), ("stor_comp", ctypes.c_int32),
        ("n_dev", ctypes.c_int32), ("dev_bus", _ip),
        ("dev_cp", _dp), ("dev_cq", _dp), ("dev_cost", _dp), ("dev_lo", _dp), ("dev_hi", _dp),
        ("dev_ramp", _dp), ("dev_init_lo", _dp), ("dev_init_hi", _dp),
    ]


STOR_FIELDS = ("emax", "chmax", "dismax", "rating", "qmin", "qmax", "eta_c", "eta_d", "r", "x", "ploss", "qloss",
               "e0")
DEV_FIELDS = ("cp", "cq", "cost", "lo", "hi", "ramp", "init_lo", "init_hi")


class _Result(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64),
        ("nnzj", ctypes.c_int64), ("nnzh", ctypes.c_int64),
        ("f", ctypes.c_double), ("fscale", ctypes.c_double),
        ("g", _dp), ("c", _dp), ("cscale", _dp),
        ("jrow", _ip), ("jcol", _ip), ("jval", _dp), ("jscale", _dp),
        ("hrow", _ip), ("hcol", _ip), ("hval", _dp), ("hscale", _dp),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.or_eval.restype = ctypes.POINTER(_Result)
        L.or_eval.argtypes = [ctypes.POINTER(_Case), _dp, _dp, ctypes.c_double, ctypes.c_int]
        L.or_free.argtypes = [ctypes.POINTER(_Result)]
        L.or_dims.argtypes = [ctypes.POINTER(_Case), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)]
        L.or_bounds.argtypes = [ctypes.POINTER(_Case), _dp, _dp, _dp, _dp, _dp]
        L.or_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


FORMS = {"polar": 0, "rect": 1}


def _make_case(case: dict, n_periods=1, pd_t=None, qd_t=None, ramp_ratio=0.0,
               n_cont=0, outaged=None, form="polar", storage=None, stor_dt=1.0, stor_comp=False, devices=None):
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
    c.n_bus, c.n_branch, c.n_gen = case["n_bus"], case["n_branch"], case["n_gen"]
    c.n_ref = len(case["ref_bus"])
    for k in ("pd", "qd", "gs", "bs", "vmin", "vmax", "r", "x", "b", "tap", "shift",
              "rate_a", "angmin", "angmax", "pmin", "pmax", "qmin", "qmax", "c2", "c1", "c0"):
        setattr(c, k, d(case[k]))
    for k in ("ref_bus", "f_bus", "t_bus", "gen_bus"):
        setattr(c, k, i(case[k]))
    c.n_periods = int(n_periods)
    c.pd_t = d(pd_t) if pd_t is not None else _dp()
    c.qd_t = d(qd_t) if qd_t is not None else _dp()
    c.ramp_ratio = float(ramp_ratio)
    c.n_cont = int(n_cont)
    c.outaged = i(outaged if outaged is not None else np.zeros(1, np.int32))
    c.form = FORMS[form]
    if storage is not None and len(storage["bus"]) > 0:
        c.n_stor = len(storage["bus"])
        c.stor_bus = i(storage["bus"])
        for k in STOR_FIELDS:
            setattr(c, "stor_" + k, d(storage[k]))
    c.stor_dt = float(stor_dt)
    c.stor_comp = int(bool(stor_comp))
    if devices is not None and len(devices["bus"]) > 0:
        c.n_dev = len(devices["bus"])
        c.dev_bus = i(devices["bus"])
        for k in DEV_FIELDS:
            setattr(c, "dev_" + k, d(devices[k]))
    return c, keep


def dims(case: dict, **opts):
    c, keep = _make_case(case, **opts)
    n, m = ctypes.c_int64(), ctypes.c_int64()
    if lib().or_dims(ctypes.byref(c), ctypes.byref(n), ctypes.byref(m)):
        raise OracleError(lib().or_error().decode())
    return n.value, m.value


def bounds(case: dict, **opts) -> dict:
    n, m = dims(case, **opts)
    c, keep = _make_case(case, **opts)
    out = {k: np.empty(n) for k in ("lvar", "uvar", "x0")}
    out.update({k: np.empty(max(m, 1)) for k in ("lcon", "ucon")})
    rc = lib().or_bounds(ctypes.byref(c), *(out[k].ctypes.data_as(_dp)
                                            for k in ("lvar", "uvar", "lcon", "ucon", "x0")))
    if rc:
        raise OracleError(lib().or_error().decode())
    out["lcon"], out["ucon"] = out["lcon"][:m], out["ucon"][:m]
    return out


def _arr(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def evaluate(case: dict, x, y=None, sigma: float = 1.0, want: int = W_ALL, **opts) -> dict:
    """All callbacks at (x, y, sigma).

    Returns a dict with f, fscale, g, c, cscale and the sorted COO triplets
    (jrow, jcol, jval, jscale) and (hrow, hcol, hval, hscale).
    """
    n, m = dims(case, **opts)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.shape != (n,):
        raise OracleError(f"x has shape {x.shape}, expected ({n},)")
    if y is None:
        y = np.zeros(m)
    y = np.ascontiguousarray(y, dtype=np.float64)
    if y.shape != (m,):
        raise OracleError(f"y has shape {y.shape}, expected ({m},)")
    c, keep = _make_case(case, **opts)
    ybuf = y if m > 0 else np.zeros(1)
    rp = lib().or_eval(ctypes.byref(c), x.ctypes.data_as(_dp), ybuf.ctypes.data_as(_dp),
                       float(sigma), int(want))
    if not rp:
        raise OracleError(lib().or_error().decode())
    try:
        r = rp.contents
        out = dict(n=n, m=m, f=r.f, fscale=r.fscale)
        out["g"] = _arr(r.g, n, np.float64) if (want & (W_OBJ | W_HESS)) else None
        if want & W_CONS:
            out["c"] = _arr(r.c, m, np.float64)
            out["cscale"] = _arr(r.cscale, m, np.float64)
        if want & W_JAC:
            k = r.nnzj
            out.update(jrow=_arr(r.jrow, k, np.int32), jcol=_arr(r.jcol, k, np.int32),
                       jval=_arr(r.jval, k, np.float64), jscale=_arr(r.jscale, k, np.float64))
        if want & W_HESS:
            k = r.nnzh
            out.update(hrow=_arr(r.hrow, k, np.int32), hcol=_arr(r.hcol, k, np.int32),
                       hval=_arr(r.hval, k, np.float64), hscale=_arr(r.hscale, k, np.float64))
    finally:
        lib().or_free(rp)
    return out


def dense_jacobian(res: dict) -> np.ndarray:
    J = np.zeros((res["m"], res["n"]))
    J[res["jrow"], res["jcol"]] = res["jval"]
    return J


def dense_hessian(res: dict) -> np.ndarray:
    """Symmetric dense Hessian assembled from the lower triangle."""
    H = np.zeros((res["n"], res["n"]))
    H[res["hrow"], res["hcol"]] = res["hval"]
    off = res["hrow"] != res["hcol"]
    H[res["hcol"][off], res["hrow"][off]] = res["hval"][off]
    return H
