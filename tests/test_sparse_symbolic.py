"""Host side of the sparse Cholesky re-factorization: the lower CSR
pattern, the minimum-degree ordering and the symbolic factor, against a
dense factorization and SuperLU's own fill count."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from helpers import case0
from ipm_models import OracleModel
from paper_2510_12897_amd.sparse_chol import lower_csr, minimum_degree_order, symbolic


def _spd(ptr, ind, n, seed):
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), np.diff(ptr))
    A = np.zeros((n, n))
    A[rows, ind] = rng.uniform(-1.0, 1.0, ind.size)
    A = np.tril(A, -1)
    A = A + A.T
    return A + np.diag(np.abs(A).sum(1) + 1.0)


def _patterns():
    rng = np.random.default_rng(0)
    yield "random", rng.integers(0, 300, 900), rng.integers(0, 300, 900), 300
    # the interior-point matrix of the 14-bus network: Hessian plus J^T J
    m = OracleModel(case0())
    jr, jc = (t.numpy() for t in m.jac_structure())
    hr, hc = (t.numpy() for t in m.hess_structure())
    pr, pc = [hr], [hc]
    for r in np.unique(jr):
        cols = jc[jr == r]
        a, b = np.meshgrid(cols, cols)
        pr.append(a.ravel())
        pc.append(b.ravel())
    yield "ipm14", np.concatenate(pr), np.concatenate(pc), m.n


@pytest.mark.parametrize("name,rows,cols,n", list(_patterns()), ids=lambda v: v if isinstance(v, str) else "")
def test_symbolic_factor_covers_the_dense_factor(name, rows, cols, n):
    ptr, ind, src = lower_csr(rows, cols, n)
    # lower triangle, diagonal included, rows sorted
    rr = np.repeat(np.arange(n), np.diff(ptr))
    assert np.all(ind <= rr) and np.all(np.diff(src) > 0)
    assert set(np.arange(n) * (n + 1)) <= set(src.tolist())
    q = minimum_degree_order(ptr, ind, n)
    assert np.array_equal(np.sort(q), np.arange(n))
    ptrL, indL, ptrB, indB, perm = symbolic(ptr, ind, n, q)
    A = _spd(ptr, ind, n, 3)
    B = A[np.ix_(q, q)]
    L = np.linalg.cholesky(B)
    rowsL = np.repeat(np.arange(n), np.diff(ptrL))
    pat = np.zeros((n, n), bool)
    pat[rowsL, indL] = True
    assert not np.any((np.abs(L) > 0) & ~pat), "a nonzero of the factor outside the symbolic pattern"
    # rows sorted, diagonal last in each row
    assert np.all(indL[ptrL[1:] - 1] == np.arange(n))
    # the permuted lower pattern and the map from A's entries
    rowsB = np.repeat(np.arange(n), np.diff(ptrB))
    assert np.array_equal(A[rr, ind][perm], B[rowsB, indB])
    # the fill is SuperLU's own for this ordering
    lu = splu(sp.csc_matrix(A), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
              options=dict(SymmetricMode=True))
    assert indL.size == lu.L.nnz
    # and far below the natural order's on the random pattern
    if name == "random":
        assert indL.size < 0.5 * symbolic(ptr, ind, n, np.arange(n))[1].size
