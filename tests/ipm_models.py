"""Models with the callback surface the interior-point solver consumes,
computed on the CPU: the oracle behind that surface, and textbook problems
with derivatives written out by hand."""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as orc


class OracleModel:
    """The oracle's callbacks behind the ``opf.Model`` surface (CPU tensors)."""

    def __init__(self, case: dict, **opts):
        self.case, self.opts = case, opts
        self.n, self.m = orc.dims(case, **opts)
        r = orc.evaluate(case, orc.bounds(case, **opts)["x0"], **opts)
        self._j = tuple(torch.from_numpy(r[k].astype(np.int64)) for k in ("jrow", "jcol"))
        self._h = tuple(torch.from_numpy(r[k].astype(np.int64)) for k in ("hrow", "hcol"))

    def bounds(self):
        return {k: torch.from_numpy(v.copy()) for k, v in orc.bounds(self.case, **self.opts).items()}

    def jac_structure(self):
        return self._j

    def hess_structure(self):
        return self._h

    def eval_set(self, x, y, w):
        r = orc.evaluate(self.case, x.numpy(), y.numpy(), w, **self.opts)
        return (torch.tensor(r["f"], dtype=torch.float64), torch.from_numpy(r["g"]), torch.from_numpy(r["c"]),
                torch.from_numpy(r["jval"]), torch.from_numpy(r["hval"]))

    def obj(self, x):
        return torch.tensor(orc.evaluate(self.case, x.numpy(), want=orc.W_OBJ, **self.opts)["f"],
                            dtype=torch.float64)

    def cons(self, x):
        return torch.from_numpy(orc.evaluate(self.case, x.numpy(), want=orc.W_CONS, **self.opts)["c"])


class HS071:
    """Problem 71 of Hock and Schittkowski's test collection:
    min x1 x4 (x1 + x2 + x3) + x3  s.t.  x1 x2 x3 x4 >= 25,
    x1^2 + x2^2 + x3^2 + x4^2 = 40,  1 <= x <= 5,  start (1, 5, 5, 1).
    The collection gives f* = 17.0140173 at x* = (1, 4.7429994,
    3.8211503, 1.3794082)."""

    n, m = 4, 2
    F_STAR = 17.0140173
    X_STAR = (1.0, 4.7429994, 3.8211503, 1.3794082)

    def bounds(self):
        t = torch.tensor
        d = torch.float64
        return dict(lvar=t([1.0] * 4, dtype=d), uvar=t([5.0] * 4, dtype=d), x0=t([1.0, 5.0, 5.0, 1.0], dtype=d),
                    lcon=t([25.0, 40.0], dtype=d), ucon=t([float("inf"), 40.0], dtype=d))

    def jac_structure(self):
        return torch.tensor([0, 0, 0, 0, 1, 1, 1, 1]), torch.tensor([0, 1, 2, 3, 0, 1, 2, 3])

    def hess_structure(self):
        r = [i for i in range(4) for j in range(i + 1)]
        c = [j for i in range(4) for j in range(i + 1)]
        return torch.tensor(r), torch.tensor(c)

    def obj(self, x):
        x1, x2, x3, x4 = x.tolist()
        return torch.tensor(x1 * x4 * (x1 + x2 + x3) + x3, dtype=torch.float64)

    def cons(self, x):
        x1, x2, x3, x4 = x.tolist()
        return torch.tensor([x1 * x2 * x3 * x4, x1 * x1 + x2 * x2 + x3 * x3 + x4 * x4], dtype=torch.float64)

    def eval_set(self, x, y, w):
        x1, x2, x3, x4 = x.tolist()
        y1, y2 = y.tolist()
        g = [x4 * (2 * x1 + x2 + x3), x1 * x4, x1 * x4 + 1.0, x1 * (x1 + x2 + x3)]
        jv = [x2 * x3 * x4, x1 * x3 * x4, x1 * x2 * x4, x1 * x2 * x3, 2 * x1, 2 * x2, 2 * x3, 2 * x4]
        # lower triangle, row-major: (0,0) (1,0) (1,1) (2,0) (2,1) (2,2) (3,0) (3,1) (3,2) (3,3)
        hf = [2 * x4, x4, 0.0, x4, 0.0, 0.0, 2 * x1 + x2 + x3, x1, x1, 0.0]
        hc1 = [0.0, x3 * x4, 0.0, x2 * x4, x1 * x4, 0.0, x2 * x3, x1 * x3, x1 * x2, 0.0]
        hc2 = [2.0, 0.0, 2.0, 0.0, 0.0, 2.0, 0.0, 0.0, 0.0, 2.0]
        hv = [w * a + y1 * b + y2 * c for a, b, c in zip(hf, hc1, hc2)]
        t = lambda v: torch.tensor(v, dtype=torch.float64)   # noqa: E731
        return self.obj(x), t(g), self.cons(x), t(jv), t(hv)


class BoundQP:
    """min (x0 - 1)^2 + (x1 - 2)^2  s.t.  x0 + x1 <= 2,  x0 - x1 = -1 + b,
    x >= 0.  For |b| < 1 the inequality is active: the minimiser is
    ((1 + b) / 2, (3 - b) / 2), f* = (1 + b^2) / 2, and the multipliers of
    grad f + J^T lam = 0 are lam = (1, -b)."""

    n, m = 2, 2

    def __init__(self, b: float = 0.0):
        self.b = float(b)

    def bounds(self):
        d = torch.float64
        inf = float("inf")
        return dict(lvar=torch.tensor([0.0, 0.0], dtype=d), uvar=torch.tensor([inf, inf], dtype=d),
                    x0=torch.tensor([0.0, 0.0], dtype=d), lcon=torch.tensor([-inf, -1.0 + self.b], dtype=d),
                    ucon=torch.tensor([2.0, -1.0 + self.b], dtype=d))

    def jac_structure(self):
        return torch.tensor([0, 0, 1, 1]), torch.tensor([0, 1, 0, 1])

    def hess_structure(self):
        return torch.tensor([0, 1]), torch.tensor([0, 1])

    def obj(self, x):
        return ((x[0] - 1) ** 2 + (x[1] - 2) ** 2).to(torch.float64)

    def cons(self, x):
        return torch.stack([x[0] + x[1], x[0] - x[1]])

    def eval_set(self, x, y, w):
        g = torch.stack([2 * (x[0] - 1), 2 * (x[1] - 2)])
        jv = torch.tensor([1.0, 1.0, 1.0, -1.0], dtype=torch.float64)
        hv = torch.tensor([2.0 * w, 2.0 * w], dtype=torch.float64)
        return self.obj(x), g, self.cons(x), jv, hv
