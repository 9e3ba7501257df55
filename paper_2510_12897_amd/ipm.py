"""A GPU-resident interior-point solver that consumes the callbacks: the
solver configuration of Sec. IV-A3 that runs MadNLP with the LiftedKKT
condensed system on the GPU.

Every callback (f, grad f, c, J, H of the Lagrangian) is one call into the
model (for an ``opf.Model``: libopf's kernels), and every solver vector stays
on the model's device.  The linear algebra is dense: the condensed matrix

    K = W + Sigma_x + J^T Sigma_s J  (+ delta I)

is assembled on the device (the J^T Sigma_s J products through a pair list
built once from the Jacobian pattern; every sum through the fixed pattern
in a fixed order, so a solve repeats bit for bit) and factored either as a
sparse matrix on the GPU (``linear_solver="sparse"``, the default on a GPU:
``sparse_chol.SparseCholesky``, rocSOLVER's sparse Cholesky
re-factorization with a minimum-degree ordering, as the paper's GPU
configuration factors K with a sparse direct solver) or dense
(``"dense"``: torch's Cholesky, the CPU path, up to ``max_dense_n``
variables).  It reports where its time goes: callbacks, linear algebra,
and the rest.

The algorithm is a primal-dual barrier method in the form of Waechter and
Biegler's Ipopt, with the LiftedKKT treatment of equalities (Pacaud and
Shin, condensed-space interior-point methods):

* every constraint row gets a slack s with c(x) - s = 0 and lcon <= s <=
  ucon; an equality row's bounds are relaxed by ``relax`` (default: the
  tolerance) on each side, so every slack has an interior and the
  condensed K is positive definite once W is regularised;
* the Newton step of the barrier KKT system condenses onto dx:
      K dx = -r_x - J^T (Sigma_s r_c + r_s),  ds = J dx + r_c,
      dlam = Sigma_s ds + r_s,
  with r_x = grad f + J^T lam - mu/(x - l) + mu/(u - x),
  r_s = -lam - mu/(s - lcon) + mu/(ucon - s), r_c = c(x) - s, and the
  Sigma the bound-dual over distance ratios; delta grows (1e-8, then x 8)
  until the Cholesky factorization succeeds;
* fraction-to-the-boundary rule with tau = max(0.99, 1 - mu), separate
  primal and bound-dual step lengths, backtracking on the l1 merit function
  f - mu sum log(distances) + nu |c(x) - s|_1 with an Armijo condition;
  when the first trial point is rejected, up to four second-order
  corrections (Ipopt's: the constraint residual of the trial point added to
  the right-hand side, solved with the same factorization) before
  backtracking;
* monotone barrier update mu <- max(tol / 10, min(0.2 mu, mu^1.5)) once the
  barrier problem is solved to 10 mu; bound duals are kept within a factor
  1e10 of mu / distance; stop when the scaled KKT error is at most tol.

``model`` is anything with the ``opf.Model`` callback surface: ``n``, ``m``,
``bounds()``, ``jac_structure()``, ``hess_structure()``,
``eval_set(x, y, w)``, ``obj(x)`` and ``cons(x)`` returning tensors on one
device.
"""
from __future__ import annotations

import math
import time

import numpy as np


def _torch():
    import torch
    return torch


class _SegSum:
    """out[idx[k]] = sum of values[perm] over segment k, in a fixed order:
    a reduction through a sparsity pattern fixed once, without atomics, so
    that the solver's iterates repeat bit for bit from run to run."""

    def __init__(self, dst: np.ndarray, size: int, device):
        torch = _torch()
        perm = np.argsort(dst, kind="stable")
        sd = dst[perm]
        idx, lengths = np.unique(sd, return_counts=True)
        self.perm = torch.from_numpy(perm).to(device)
        self.idx = torch.from_numpy(idx.astype(np.int64)).to(device)
        self.lengths = torch.from_numpy(lengths.astype(np.int64)).to(device)
        self.size = int(size)

    def __call__(self, values, out=None):
        torch = _torch()
        sums = torch.segment_reduce(values[self.perm], "sum", lengths=self.lengths)
        if out is None:
            out = torch.zeros(self.size, dtype=values.dtype, device=values.device)
        else:
            out.zero_()
        out[self.idx] = sums
        return out


class InteriorPoint:
    """Solve min f(x) s.t. lcon <= c(x) <= ucon, lvar <= x <= uvar."""

    def __init__(self, model, tol: float = 1e-6, relax: float | None = None, max_iter: int = 300,
                 mu0: float = 0.1, max_dense_n: int = 40000, linear_solver: str = "auto", verbose: bool = False):
        torch = _torch()
        self.model = model
        self.tol = float(tol)
        self.relax = self.tol if relax is None else float(relax)
        self.max_iter, self.mu0, self.verbose = int(max_iter), float(mu0), verbose
        n, m = int(model.n), int(model.m)
        self.n, self.m = n, m
        b = model.bounds()
        self.lv, self.uv, self.x0 = b["lvar"], b["uvar"], b["x0"]
        self.lc0, self.uc0 = b["lcon"], b["ucon"]
        self.dev = self.lv.device
        if linear_solver == "auto":
            linear_solver = "sparse" if self.dev.type == "cuda" else "dense"
        if linear_solver not in ("dense", "sparse"):
            raise ValueError(f"ipm: linear_solver must be 'dense', 'sparse' or 'auto', not {linear_solver!r}")
        if linear_solver == "sparse" and self.dev.type != "cuda":
            raise ValueError("ipm: the sparse factorization runs on the GPU only")
        if linear_solver == "dense" and n > max_dense_n:
            raise ValueError(f"ipm: {n} variables exceed the dense limit max_dense_n = {max_dense_n}")
        self.linear_solver = linear_solver
        eq = self.lc0 == self.uc0
        self.lc = torch.where(eq, self.lc0 - self.relax, self.lc0)
        self.uc = torch.where(eq, self.uc0 + self.relax, self.uc0)
        self.hxl, self.hxu = torch.isfinite(self.lv), torch.isfinite(self.uv)
        self.hsl, self.hsu = torch.isfinite(self.lc), torch.isfinite(self.uc)
        self.n_bounds = int(self.hxl.sum() + self.hxu.sum() + self.hsl.sum() + self.hsu.sum())
        jr, jc = (t.long() for t in model.jac_structure())
        hr, hc = (t.long() for t in model.hess_structure())
        self.jr, self.jc = jr, jc
        jr_h, jc_h = jr.cpu().numpy(), jc.cpu().numpy()
        hr_h, hc_h = hr.cpu().numpy(), hc.cpu().numpy()
        # J^T v (sums by column) and J v (sums by row) in a fixed order
        self.sum_cols = _SegSum(jc_h, n, self.dev)
        self.sum_rows = _SegSum(jr_h, m, self.dev)
        # ordered pairs (a, b) of Jacobian entries in one row r:
        # K[col a, col b] += Sigma_s[r] J_a J_b
        p_a, p_b, p_row = self._pairs(jr_h, jc_h)
        if linear_solver == "dense":
            # K index of every Hessian value, both triangles, and of every pair
            off_h = hr_h != hc_h
            h_src = np.concatenate([np.arange(hr_h.size), np.nonzero(off_h)[0]])
            h_dst = np.concatenate([hr_h * n + hc_h, (hc_h * n + hr_h)[off_h]])
            p_dst = jc_h[p_a] * n + jc_h[p_b]
            size = n * n
            self.K = torch.empty(n * n, dtype=torch.float64, device=self.dev)
        else:
            from .sparse_chol import SparseCholesky
            # the lower triangle only: Hessian values as given (lower), pairs
            # with col a >= col b
            keep = jc_h[p_a] >= jc_h[p_b]
            p_a, p_b, p_row = p_a[keep], p_b[keep], p_row[keep]
            self.chol = SparseCholesky(np.concatenate([hr_h, jc_h[p_a]]), np.concatenate([hc_h, jc_h[p_b]]), n,
                                       self.dev)
            h_src = np.arange(hr_h.size)
            h_dst = np.searchsorted(self.chol.src, np.maximum(hr_h, hc_h) * n + np.minimum(hr_h, hc_h))
            p_dst = np.searchsorted(self.chol.src, jc_h[p_a] * n + jc_h[p_b])
            size = self.chol.src.size
        dev_t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(self.dev)   # noqa: E731
        self.h_src, self.p_a, self.p_b, self.p_row = dev_t(h_src), dev_t(p_a), dev_t(p_b), dev_t(p_row)
        # every contribution to K (Hessian values, then pair products) summed
        # per entry in a fixed order
        self.sum_k = _SegSum(np.concatenate([h_dst, p_dst]), size, self.dev)
        self.times = {"callbacks": 0.0, "linear_algebra": 0.0, "other": 0.0}
        self.counts = {"eval_set": 0, "obj_cons": 0, "factorizations": 0, "soc": 0}

    def _pairs(self, jr, jc):
        order = np.argsort(jr, kind="stable")
        starts = np.searchsorted(jr[order], np.arange(self.m + 1))
        cnt = np.diff(starts)
        tot = int((cnt.astype(np.int64) ** 2).sum())
        a = np.empty(tot, np.int64)
        b = np.empty(tot, np.int64)
        r = np.empty(tot, np.int64)
        pos = 0
        for c in np.unique(cnt):
            if c == 0:
                continue
            sel = np.nonzero(cnt == c)[0]
            ent = order[starts[sel][:, None] + np.arange(c)[None, :]]      # (rows, c) entry indices
            w = ent.shape[0] * c * c
            a[pos:pos + w] = np.repeat(ent, c, axis=1).ravel()
            b[pos:pos + w] = np.tile(ent, (1, c)).ravel()
            r[pos:pos + w] = np.repeat(sel, c * c)
            pos += w
        return a, b, r

    def close(self):
        """Release the sparse factorization's library handles."""
        if getattr(self, "chol", None) is not None:
            self.chol.close()
            self.chol = None

    # ---------------------------------------------------------------- helpers
    def _sync(self):
        if self.dev.type == "cuda":
            _torch().cuda.synchronize(self.dev)

    def _timed(self, part, fn, *a):
        self._sync()
        t0 = time.perf_counter()
        out = fn(*a)
        self._sync()
        self.times[part] += time.perf_counter() - t0
        return out

    def _eval(self, x, lam):
        self.counts["eval_set"] += 1
        return self.model.eval_set(x, lam, 1.0)

    def _obj_cons(self, x):
        self.counts["obj_cons"] += 1
        return self.model.obj(x), self.model.cons(x)

    def _interior(self, v, lo, hi, hl, hu, k1=1e-2, k2=1e-2):
        """Move v into the interior of [lo, hi] (Ipopt's initial-point
        push: at least k1 max(1, |bound|) from a bound, at most k2 of the
        gap)."""
        torch = _torch()
        lo0 = torch.where(hl, lo, torch.zeros_like(lo))
        hi0 = torch.where(hu, hi, torch.zeros_like(hi))
        both = hl & hu
        pl = k1 * torch.clamp(lo0.abs(), min=1.0)
        pu = k1 * torch.clamp(hi0.abs(), min=1.0)
        pl = torch.where(both, torch.minimum(pl, k2 * (hi0 - lo0)), pl)
        pu = torch.where(both, torch.minimum(pu, k2 * (hi0 - lo0)), pu)
        v = torch.where(hl, torch.maximum(v, lo0 + pl), v)
        v = torch.where(hu, torch.minimum(v, hi0 - pu), v)
        return v

    def _dist(self, x, s):
        """Distances to the four bound sets (1 where a bound is absent)."""
        torch = _torch()
        one = torch.ones((), dtype=torch.float64, device=self.dev)
        return (torch.where(self.hxl, x - self.lv, one), torch.where(self.hxu, self.uv - x, one),
                torch.where(self.hsl, s - self.lc, one), torch.where(self.hsu, self.uc - s, one))

    def _jt(self, jv, v):
        """J^T v."""
        return self.sum_cols(jv * v[self.jr])

    def _jv(self, jv, v):
        """J v."""
        return self.sum_rows(jv * v[self.jc])

    def _kkt(self, mu, g, c, jv, x, s, lam, z):
        """Scaled KKT error of the barrier problem at mu (Ipopt's E_mu with
        s_max = 100), as a 0-d device tensor (no host synchronization)."""
        torch = _torch()
        zl, zu, vl, vu = z
        dlx, dux, dls, dus = self._dist(x, s)
        rdx = g + self._jt(jv, lam) - zl + zu
        rds = -lam - vl + vu
        comp = torch.stack([torch.where(self.hxl, dlx * zl - mu, 0.0).abs().max(),
                            torch.where(self.hxu, dux * zu - mu, 0.0).abs().max(),
                            torch.where(self.hsl, dls * vl - mu, 0.0).abs().max() if self.m else rdx.new_zeros(()),
                            torch.where(self.hsu, dus * vu - mu, 0.0).abs().max() if self.m else rdx.new_zeros(())]).max()
        nz = self.n_bounds
        zsum = zl.abs().sum() + zu.abs().sum() + vl.abs().sum() + vu.abs().sum()
        s_d = torch.clamp((lam.abs().sum() + zsum) / max(self.m + nz, 1), min=100.0) / 100.0
        s_c = torch.clamp(zsum / max(nz, 1), min=100.0) / 100.0
        e_d = torch.maximum(rdx.abs().max(), rds.abs().max()) if self.m else rdx.abs().max()
        e_p = (c - s).abs().max() if self.m else rdx.new_zeros(())
        return torch.stack([e_d / s_d, e_p, comp / s_c]).max()

    def _assemble_factor(self, hv, jv, Sx, Ss, rhs, delta0):
        """Assemble K, factor it (raising delta until it factors) and solve
        K dx = rhs: (dx, delta, solve) with solve(r) = K^-1 r from the same
        factorization."""
        torch = _torch()
        n = self.n
        contrib = torch.cat([hv[self.h_src], Ss[self.p_row] * jv[self.p_a] * jv[self.p_b]])
        if self.linear_solver == "sparse":
            vals = self.sum_k(contrib)
            vals[self.chol.diag] += Sx
            delta = delta0
            while True:
                v = vals
                if delta > 0:
                    v = vals.clone()
                    v[self.chol.diag] += delta
                self.counts["factorizations"] += 1
                if self.chol.factor(v):
                    break
                delta = 1e-8 if delta == 0.0 else 8.0 * delta
                if delta > 1e40:
                    raise FloatingPointError("ipm: no regularisation makes the condensed matrix positive definite")
            return self.chol.solve(rhs), delta, self.chol.solve
        K = self.K
        self.sum_k(contrib, out=K)
        Kd = K.view(n, n)
        Kd.diagonal().add_(Sx)
        delta = delta0
        while True:
            if delta > 0:
                Kd.diagonal().add_(delta)
            L, info = torch.linalg.cholesky_ex(Kd)
            self.counts["factorizations"] += 1
            if int(info) == 0:
                break
            if delta > 0:
                Kd.diagonal().sub_(delta)
            delta = 1e-8 if delta == 0.0 else 8.0 * delta
            if delta > 1e40:
                raise FloatingPointError("ipm: no regularisation makes the condensed matrix positive definite")
        return self._solve(L, rhs), delta, lambda r: self._solve(L, r)

    @staticmethod
    def _solve(L, rhs):
        """K^-1 rhs from the Cholesky factor: two triangular solves (several
        times faster on ROCm than cholesky_solve's default path here)."""
        torch = _torch()
        w = torch.linalg.solve_triangular(L, rhs[:, None], upper=False)
        return torch.linalg.solve_triangular(L.mT, w, upper=True)[:, 0]

    # ---------------------------------------------------------------- solve
    def solve(self, x0=None) -> dict:
        """Run the iteration from x0 (default: the model's start point).

        Returns a dict: x, s, lam (constraint multipliers), zl, zu (bound
        duals of x), f, status ("solved", "max_iter" or "stalled" after five
        line searches in a row that found no acceptable step), iterations,
        kkt (final scaled KKT error), cvio (largest violation of the
        unrelaxed constraint bounds), mu, times (seconds by part), counts.
        """
        torch = _torch()
        m = self.m
        f64 = dict(dtype=torch.float64, device=self.dev)
        t_start = time.perf_counter()
        for k in self.times:
            self.times[k] = 0.0
        for k in self.counts:
            self.counts[k] = 0
        x = self._interior((self.x0 if x0 is None else x0).to(**f64).clone(), self.lv, self.uv, self.hxl, self.hxu)
        lam = torch.zeros(m, **f64)
        f, g, c, jv, hv = self._timed("callbacks", self._eval, x, lam)
        s = self._interior(c.clone(), self.lc, self.uc, self.hsl, self.hsu)
        zl, zu = self.hxl.to(torch.float64), self.hxu.to(torch.float64)
        vl, vu = self.hsl.to(torch.float64), self.hsu.to(torch.float64)
        mu, nu, delta = self.mu0, 1.0, 0.0
        status, kkt, fails, it = "max_iter", float("inf"), 0, 0
        last_step = "-"
        for it in range(self.max_iter + 1):
            t0 = time.perf_counter()
            z = (zl, zu, vl, vu)
            kkt = float(self._kkt(0.0, g, c, jv, x, s, lam, z))
            if self.verbose:
                print(f"[ipm] it {it:3d} f {float(f):.10g} kkt {kkt:.3e} mu {mu:.1e} delta {delta:.1e} "
                      f"step {last_step}", flush=True)
            if kkt <= self.tol or it == self.max_iter:
                status = "solved" if kkt <= self.tol else status
                self.times["other"] += time.perf_counter() - t0
                break
            while mu > self.tol / 10 and float(self._kkt(mu, g, c, jv, x, s, lam, z)) <= 10.0 * mu:
                mu = max(self.tol / 10, min(0.2 * mu, mu ** 1.5))
            dlx, dux, dls, dus = self._dist(x, s)
            Sx = torch.where(self.hxl, zl / dlx, 0.0) + torch.where(self.hxu, zu / dux, 0.0)
            Ss = torch.where(self.hsl, vl / dls, 0.0) + torch.where(self.hsu, vu / dus, 0.0)
            Jt_lam = self._jt(jv, lam)
            bx = -torch.where(self.hxl, mu / dlx, 0.0) + torch.where(self.hxu, mu / dux, 0.0)
            bs = -torch.where(self.hsl, mu / dls, 0.0) + torch.where(self.hsu, mu / dus, 0.0)
            rx = g + Jt_lam + bx
            rs = bs - lam
            rc = c - s
            self.times["other"] += time.perf_counter() - t0

            def newton():
                rhs = -(rx + self._jt(jv, Ss * rc + rs))
                d0 = 0.0 if delta == 0.0 else max(1e-20, delta / 3.0)
                dx, dlt, solve_k = self._assemble_factor(hv, jv, Sx, Ss, rhs, d0)
                ds = self._jv(jv, dx) + rc
                return dx, ds, dlt, solve_k

            dx, ds, delta, solve_k = self._timed("linear_algebra", newton)
            t0 = time.perf_counter()
            tau = max(0.99, 1.0 - mu)
            has = (self.hxl, self.hxu, self.hsl, self.hsu)

            inf = torch.full((), float("inf"), **f64)

            def max_step(d, dd, h):
                # largest a with d + a dd >= (1 - tau) d wherever h (device scalar)
                return torch.where(h & (dd < 0), -tau * d / dd, inf).min() if d.numel() else inf

            def primal_step(dx_, ds_):
                return min(1.0, float(torch.stack([max_step(dlx, dx_, self.hxl), max_step(dux, -dx_, self.hxu),
                                                   max_step(dls, ds_, self.hsl),
                                                   max_step(dus, -ds_, self.hsu)]).min()))

            def merit(f_, x_, s_, c_):
                # device scalar
                lg = sum(torch.where(h, torch.log(d), 0.0).sum() for d, h in zip(self._dist(x_, s_), has))
                return f_ - mu * lg + nu * (c_ - s_).abs().sum()

            a_p = primal_step(dx, ds)
            if m:
                nu = max(nu, 1.1 * float((lam + Ss * ds + rs).abs().max()))
            phi0 = merit(f, x, s, c)
            # directional derivative of the merit function along (dx, ds)
            dphi = torch.clamp((g + bx) @ dx + bs @ ds - nu * rc.abs().sum(), max=0.0)
            self.times["other"] += time.perf_counter() - t0

            def trial(a, dx_, ds_):
                xt, st = x + a * dx_, s + a * ds_
                ft, ct = self._timed("callbacks", self._obj_cons, xt)
                t1 = time.perf_counter()
                phit = merit(ft, xt, st, ct)
                ok = bool(torch.isfinite(phit) & (phit <= phi0 + 1e-4 * a * dphi))
                self.times["other"] += time.perf_counter() - t1
                return ok, ct - st

            alpha, accepted, soc = a_p, False, 0
            ok, rt = trial(alpha, dx, ds)
            if ok:
                accepted = True
            elif m:
                # second-order correction (Ipopt's): the step that also
                # removes the trial point's constraint residual to first
                # order, from the same factorization; at most 4 rounds while
                # the residual keeps falling
                rc_soc, theta = a_p * rc + rt, float(rt.abs().sum())
                for _ in range(4):
                    soc += 1
                    dx_s = self._timed("linear_algebra", lambda: solve_k(-(rx + self._jt(jv, Ss * rc_soc + rs))))
                    ds_s = self._jv(jv, dx_s) + rc_soc
                    a_s = primal_step(dx_s, ds_s)
                    ok_s, rt_s = trial(a_s, dx_s, ds_s)
                    if ok_s and math.isfinite(a_s):
                        # Armijo against the original step, then take the corrected one
                        dx, ds, alpha, accepted = dx_s, ds_s, a_s, True
                        break
                    theta_s = float(rt_s.abs().sum())
                    if not theta_s < 0.99 * theta:
                        break
                    rc_soc, theta = a_s * rc_soc + rt_s, theta_s
            if not accepted:
                alpha = a_p
                for _ in range(40):
                    alpha *= 0.5
                    ok, _ = trial(alpha, dx, ds)
                    if ok:
                        accepted = True
                        break
            fails = 0 if accepted else fails + 1
            self.counts["soc"] = self.counts.get("soc", 0) + soc
            if fails >= 5:
                status = "stalled"
                break
            t0 = time.perf_counter()
            dlam = Ss * ds + rs
            dzl = torch.where(self.hxl, (mu - zl * dx) / dlx - zl, 0.0)
            dzu = torch.where(self.hxu, (mu + zu * dx) / dux - zu, 0.0)
            dvl = torch.where(self.hsl, (mu - vl * ds) / dls - vl, 0.0)
            dvu = torch.where(self.hsu, (mu + vu * ds) / dus - vu, 0.0)
            a_d = min(1.0, float(torch.stack([max_step(zl, dzl, self.hxl), max_step(zu, dzu, self.hxu),
                                              max_step(vl, dvl, self.hsl), max_step(vu, dvu, self.hsu)]).min()))
            last_step = f"a_p {a_p:.2e} alpha {alpha:.2e} a_d {a_d:.2e} soc {soc} nu {nu:.1e}"
            x, s = x + alpha * dx, s + alpha * ds
            lam = lam + alpha * dlam
            dlx, dux, dls, dus = self._dist(x, s)

            def keep(zz, dzz, d, h):
                # bound dual step, then kept within a factor 1e10 of mu / distance
                zz = zz + a_d * dzz
                return torch.where(h, torch.maximum(torch.minimum(zz, 1e10 * mu / d), mu / (1e10 * d)), 0.0)

            zl, zu = keep(zl, dzl, dlx, self.hxl), keep(zu, dzu, dux, self.hxu)
            vl, vu = keep(vl, dvl, dls, self.hsl), keep(vu, dvu, dus, self.hsu)
            self.times["other"] += time.perf_counter() - t0
            f, g, c, jv, hv = self._timed("callbacks", self._eval, x, lam)
        cvio = 0.0
        if m:
            cvio = float(torch.maximum(torch.clamp(self.lc0 - c, min=0.0), torch.clamp(c - self.uc0, min=0.0)).max())
        return dict(x=x, s=s, lam=lam, zl=zl, zu=zu, f=float(f), status=status, iterations=it, kkt=kkt, cvio=cvio,
                    mu=mu, times=dict(self.times, total=time.perf_counter() - t_start), counts=dict(self.counts))
