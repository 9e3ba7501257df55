"""Sparse Cholesky factorization of a matrix with a fixed pattern, for the
interior-point solver's condensed matrix: the symbolic work once on the host,
the numeric factorization and the solves on the GPU every iteration.

The paper's GPU solver configuration factors its condensed KKT matrix with a
sparse direct solver (Sec. IV-A3, cuDSS).  On ROCm the matching library
routines are rocSOLVER's sparse re-factorization (``rocsolver_dcsrrf_*`` in
Cholesky mode): given the pattern of the factor and a fill-reducing
ordering, they factor any matrix of the same pattern on the device.  What
they need is built here:

* the lower triangle of the matrix pattern (diagonal included) in CSR,
  rows sorted;
* a fill-reducing ordering q: the multiple minimum degree ordering on
  A + A^T that SuperLU (scipy) computes, taken from one factorization of a
  diagonally dominant matrix with the same pattern (the ordering depends
  on the pattern only);
* the pattern of the Cholesky factor L of A[q][:, q] from the elimination
  tree (Liu: the pattern of row i of L is the union of the tree paths from
  the nonzeros of row i of the permuted lower triangle up to i);
* the analysis, from the first matrix and its factor (a dense Cholesky on
  the device, read at the symbolic pattern).

Every later matrix of the pattern is then re-factored and solved on the
device (``factor``, ``solve``).  ``symbolic`` and ``minimum_degree_order``
run without a GPU.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np


def _torch():
    import torch
    return torch


def lower_csr(rows: np.ndarray, cols: np.ndarray, n: int):
    """(ptr, ind, src) of the lower triangle of the symmetric pattern given
    by the (row, col) pairs (either triangle, duplicates allowed), diagonal
    always included; src[k] = the flat index row * n + col of entry k."""
    r = np.asarray(rows, np.int64)
    c = np.asarray(cols, np.int64)
    lo = np.maximum(r, c) * n + np.minimum(r, c)
    flat = np.unique(np.concatenate([lo, np.arange(n, dtype=np.int64) * (n + 1)]))
    ri, ci = flat // n, flat % n
    ptr = np.zeros(n + 1, np.int64)
    np.add.at(ptr, ri + 1, 1)
    ptr = np.cumsum(ptr)
    return ptr, ci.astype(np.int64), flat


def minimum_degree_order(ptr: np.ndarray, ind: np.ndarray, n: int) -> np.ndarray:
    """Fill-reducing order q (new position k holds old index q[k]) of the
    symmetric pattern whose lower triangle is (ptr, ind): SuperLU's multiple
    minimum degree on A + A^T, read from the column permutation of one
    factorization of a diagonally dominant matrix with this pattern."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import splu

    rows = np.repeat(np.arange(n), np.diff(ptr))
    off = rows != ind
    r = np.concatenate([rows[off], ind[off]])
    c = np.concatenate([ind[off], rows[off]])
    deg = np.bincount(r, minlength=n).astype(np.float64)
    A = sp.csc_matrix((np.concatenate([-np.ones(r.size), deg + 1.0]),
                       (np.concatenate([r, np.arange(n)]), np.concatenate([c, np.arange(n)]))), shape=(n, n))
    lu = splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    # with the diagonal pivots SuperLU factors A[pc][:, pc] with pc = perm_c
    # read as "old index of new position": the inverse map of perm_c
    q = np.empty(n, np.int64)
    q[lu.perm_c] = np.arange(n)
    return q


def symbolic(ptr: np.ndarray, ind: np.ndarray, n: int, q: np.ndarray):
    """Pattern of the Cholesky factor of B = A[q][:, q] for the lower CSR
    pattern (ptr, ind) of A: returns (ptrL, indL) in CSR, rows sorted,
    diagonal included, and (ptrB, indB, perm) with the lower CSR pattern of
    B and perm[k] = the position in A's lower CSR of B's entry k."""
    pinv = np.empty(n, np.int64)
    pinv[q] = np.arange(n)
    rows = np.repeat(np.arange(n), np.diff(ptr))
    ri, ci = pinv[rows], pinv[ind]
    br, bc = np.maximum(ri, ci), np.minimum(ri, ci)
    key = br * n + bc
    perm = np.argsort(key, kind="stable")
    br, bc = br[perm], bc[perm]
    ptrB = np.zeros(n + 1, np.int64)
    np.add.at(ptrB, br + 1, 1)
    ptrB = np.cumsum(ptrB)
    indB = bc
    # elimination tree (Liu, with path compression)
    parent = np.full(n, -1, np.int64)
    ancestor = np.full(n, -1, np.int64)
    for i in range(n):
        for j in indB[ptrB[i]:ptrB[i + 1]]:
            if j >= i:
                continue
            while j != -1 and j < i:
                nxt = ancestor[j]
                ancestor[j] = i
                if nxt == -1:
                    parent[j] = i
                    break
                j = nxt
    # row patterns: tree paths from each nonzero up to i
    mark = np.full(n, -1, np.int64)
    rows_L = []
    for i in range(n):
        mark[i] = i
        rp = [i]
        for j in indB[ptrB[i]:ptrB[i + 1]]:
            while j != -1 and mark[j] != i:
                rp.append(j)
                mark[j] = i
                j = parent[j]
        rows_L.append(np.sort(np.asarray(rp, np.int64)))
    ptrL = np.zeros(n + 1, np.int64)
    ptrL[1:] = np.cumsum([r.size for r in rows_L])
    indL = np.concatenate(rows_L) if n else np.zeros(0, np.int64)
    return ptrL, indL, ptrB, indB, perm


class _Roc:
    """ctypes entry points of rocBLAS (handle, stream) and rocSOLVER (the
    sparse re-factorization)."""
    _inst = None

    def __init__(self):
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        self.blas = ctypes.CDLL(os.path.join(rocm, "lib", "librocblas.so"))
        self.sol = ctypes.CDLL(os.path.join(rocm, "lib", "librocsolver.so"))
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        self.blas.rocblas_create_handle.argtypes = [ctypes.POINTER(vp)]
        self.blas.rocblas_destroy_handle.argtypes = [vp]
        self.blas.rocblas_set_stream.argtypes = [vp, vp]
        self.sol.rocsolver_create_rfinfo.argtypes = [ctypes.POINTER(vp), vp]
        self.sol.rocsolver_destroy_rfinfo.argtypes = [vp]
        self.sol.rocsolver_set_rfinfo_mode.argtypes = [vp, ctypes.c_int]
        self.sol.rocsolver_dcsrrf_analysis.argtypes = [vp, i32, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, i32,
                                                       vp]
        self.sol.rocsolver_dcsrrf_refactchol.argtypes = [vp, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp]
        self.sol.rocsolver_dcsrrf_solve.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, i32, vp]
        for f in (self.blas.rocblas_create_handle, self.blas.rocblas_destroy_handle, self.blas.rocblas_set_stream,
                  self.sol.rocsolver_create_rfinfo, self.sol.rocsolver_destroy_rfinfo,
                  self.sol.rocsolver_set_rfinfo_mode, self.sol.rocsolver_dcsrrf_analysis,
                  self.sol.rocsolver_dcsrrf_refactchol, self.sol.rocsolver_dcsrrf_solve):
            f.restype = ctypes.c_int

    @classmethod
    def get(cls):
        if cls._inst is None:
            cls._inst = _Roc()
        return cls._inst


RFINFO_MODE_CHOLESKY = 272


def _ok(status, what):
    if status != 0:
        raise RuntimeError(f"{what} failed (rocblas_status {status})")


class SparseCholesky:
    """Re-factorization of matrices with one symmetric pattern on the GPU.

    ``rows``, ``cols``: the pattern (either triangle, duplicates allowed).
    The caller passes values in the order of the lower-triangle CSR pattern
    (``src`` holds each entry's flat index row * n + col, ``diag`` the
    diagonal's positions)."""

    # the first factorization (which seeds the analysis) is a dense one: n^2
    # doubles on the device
    MAX_SETUP_N = 40000

    def __init__(self, rows, cols, n: int, device):
        torch = _torch()
        self.n = int(n)
        if self.n > self.MAX_SETUP_N:
            raise ValueError(f"sparse Cholesky: the dense first factorization limits n to {self.MAX_SETUP_N} "
                             f"(got {self.n})")
        self.dev = device
        self.ptr, self.ind, self.src = lower_csr(rows, cols, self.n)
        self.q = minimum_degree_order(self.ptr, self.ind, self.n)
        self.ptrL, self.indL, self.ptrB, self.indB, self.perm = symbolic(self.ptr, self.ind, self.n, self.q)
        self.nnzT = int(self.indL.size)
        if max(2 * self.ind.size, self.nnzT) >= 2 ** 31:
            raise ValueError("sparse Cholesky: pattern too large for 32-bit indices")
        # the routines take A in its own order (they apply q themselves), as
        # the full symmetric pattern: lower entries and their mirrors
        rows = np.repeat(np.arange(self.n), np.diff(self.ptr))
        off = np.nonzero(rows != self.ind)[0]
        fr = np.concatenate([rows, self.ind[off]])
        fc = np.concatenate([self.ind, rows[off]])
        from_lower = np.concatenate([np.arange(rows.size), off])
        order = np.lexsort((fc, fr))
        fr, fc, from_lower = fr[order], fc[order], from_lower[order]
        ptrA = np.zeros(self.n + 1, np.int64)
        np.add.at(ptrA, fr + 1, 1)
        self.ptrA, self.indA = np.cumsum(ptrA), fc
        self.nnzA = int(fc.size)
        i32 = dict(dtype=torch.int32, device=device)
        self.d_ptrA = torch.as_tensor(self.ptrA, **i32)
        self.d_indA = torch.as_tensor(self.indA, **i32)
        self.d_full = torch.as_tensor(from_lower, dtype=torch.int64, device=device)
        self._diagL = torch.as_tensor(self.ptrL[1:] - 1, dtype=torch.int64, device=device)
        self._lenL = torch.as_tensor(np.diff(self.ptrL), dtype=torch.int64, device=device)
        self.d_ptrB = torch.as_tensor(self.ptrB, **i32)
        self.d_indB = torch.as_tensor(self.indB, **i32)
        self.d_ptrL = torch.as_tensor(self.ptrL, **i32)
        self.d_indL = torch.as_tensor(self.indL, **i32)
        self.d_q = torch.as_tensor(self.q, **i32)
        self.d_perm = torch.as_tensor(self.perm, dtype=torch.int64, device=device)
        self.valL = torch.zeros(self.nnzT, dtype=torch.float64, device=device)
        rowsL = np.repeat(np.arange(self.n), np.diff(self.ptrL))
        self._flatL = torch.as_tensor(rowsL * self.n + self.indL, dtype=torch.int64, device=device)
        self.diag = torch.as_tensor(np.searchsorted(self.src, np.arange(self.n) * (self.n + 1)), dtype=torch.int64,
                                    device=device)
        self._h = None
        self._rf = None


    # A's lower CSR values (caller order) -> B = A[q][:, q] lower CSR values
    def _valB(self, valA):
        return valA[self.d_perm].contiguous()

    def _stream(self):
        return ctypes.c_void_p(_torch().cuda.current_stream(self.dev).cuda_stream)

    def _setup(self, valA):
        """Analysis from the first matrix: its factor from a dense Cholesky
        of B = A[q][:, q] on the device, read at the symbolic pattern."""
        torch = _torch()
        roc = _Roc.get()
        n = self.n
        Bd = torch.zeros(n * n, dtype=torch.float64, device=self.dev)
        rowsB = torch.repeat_interleave(torch.arange(n, device=self.dev), torch.diff(self.d_ptrB.long()))
        Bd[rowsB * n + self.d_indB.long()] = self._valB(valA)
        Bd = Bd.view(n, n)
        Bd = torch.tril(Bd) + torch.tril(Bd, -1).mT
        L, info = torch.linalg.cholesky_ex(Bd)
        if int(info) != 0:
            return False
        self.valL.copy_(L.reshape(-1)[self._flatL])
        h = ctypes.c_void_p()
        _ok(roc.blas.rocblas_create_handle(ctypes.byref(h)), "rocblas_create_handle")
        self._h = h
        rf = ctypes.c_void_p()
        _ok(roc.sol.rocsolver_create_rfinfo(ctypes.byref(rf), h), "rocsolver_create_rfinfo")
        self._rf = rf
        _ok(roc.sol.rocsolver_set_rfinfo_mode(rf, RFINFO_MODE_CHOLESKY), "rocsolver_set_rfinfo_mode")
        _ok(roc.blas.rocblas_set_stream(h, self._stream()), "rocblas_set_stream")
        valF = valA[self.d_full].contiguous()
        # one right-hand side: the analysis also prepares the solve phase
        self._rhs0 = torch.zeros(n, dtype=torch.float64, device=self.dev)
        _ok(roc.sol.rocsolver_dcsrrf_analysis(h, n, 1, self.nnzA, _p(self.d_ptrA), _p(self.d_indA), _p(valF),
                                              self.nnzT, _p(self.d_ptrL), _p(self.d_indL), _p(self.valL), None,
                                              _p(self.d_q), _p(self._rhs0), n, rf), "rocsolver_dcsrrf_analysis")
        return True

    def factor(self, valA) -> bool:
        """Factor the matrix whose lower CSR values (this pattern's order)
        are valA; False if it is not numerically positive definite (a
        non-finite or non-positive pivot)."""
        torch = _torch()
        if self._rf is None:
            return self._setup(valA)
        roc = _Roc.get()
        _ok(roc.blas.rocblas_set_stream(self._h, self._stream()), "rocblas_set_stream")
        valF = valA[self.d_full].contiguous()
        _ok(roc.sol.rocsolver_dcsrrf_refactchol(self._h, self.n, self.nnzA, _p(self.d_ptrA), _p(self.d_indA),
                                                _p(valF), self.nnzT, _p(self.d_ptrL), _p(self.d_indL),
                                                _p(self.valL), _p(self.d_q), self._rf),
            "rocsolver_dcsrrf_refactchol")
        return self._is_factor_of(valA)

    def _is_factor_of(self, valA) -> bool:
        """Whether valL is the Cholesky factor of this matrix.  The routine
        reports no failed pivot (on a matrix that is not positive definite
        it still returns a finite factor), so the factor is checked: for
        the exact factor of B = A[q][:, q], the squares of row i of L sum to
        B_ii, a sum of positive terms that rounding keeps to a few ulps
        whatever the conditioning; a pivot the routine had to replace
        breaks it."""
        torch = _torch()
        if not bool(torch.isfinite(self.valL).all()):
            return False
        bdiag = valA[self.diag][self.d_q.long()]
        if not bool((bdiag > 0).all()):
            return False
        sq = torch.segment_reduce(self.valL * self.valL, "sum", lengths=self._lenL)
        return bool(((sq - bdiag).abs() <= 1e-10 * bdiag).all())

    def solve(self, b):
        """x with A x = b for the last factored A (b: float64 device vector)."""
        roc = _Roc.get()
        x = b.clone().contiguous()
        _ok(roc.blas.rocblas_set_stream(self._h, self._stream()), "rocblas_set_stream")
        _ok(roc.sol.rocsolver_dcsrrf_solve(self._h, self.n, 1, self.nnzT, _p(self.d_ptrL), _p(self.d_indL),
                                           _p(self.valL), None, _p(self.d_q), _p(x), self.n, self._rf),
            "rocsolver_dcsrrf_solve")
        return x

    def close(self):
        roc = _Roc.get()
        if self._rf is not None:
            roc.sol.rocsolver_destroy_rfinfo(self._rf)
            self._rf = None
        if self._h is not None:
            roc.blas.rocblas_destroy_handle(self._h)
            self._h = None


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())
