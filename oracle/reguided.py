"""Non-linear (re-guided) filters: the first of the two ways to iterate the BF
and the GF (Sections 2 and 3): every step rebuilds the graph with the current
iterate as the guidance, so the graph changes from step to step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading (the paper names the variant but prints no algorithm for it):
  power: x_{k+1} = D(x_k)^-1 W(x_k) x_k, eq. (3) with the guidance replaced by
    the previous result at every pass (the first pass uses x_0 itself).
  CG: Algorithm 2 with L and D rebuilt from the current iterate at the start
    of every step k (L_k = L(x_k), D_k = D(x_k); step 1 uses x_0).  The
    recursion is kept as printed: r is updated (r <- r - alpha q), not
    recomputed from L_k; s = D_k^-1 r; the flexible beta
    s^T (r - r_old) / (s_old^T r_old) (the reading of the garbled
    denominator used by `solvers.cg_filter`), which the end of Section 5 names
    as the form meant for L and D that change; q = L_k p; r_0 = -L(x_0) x_0.
    Breakdown and tolerance tests as in `solvers.cg_filter`, with the floor
    taken from x_0^T D(x_0) x_0 and the tolerance relative to the first
    s^T r.  The reported residual is sqrt(s^T r) of the last step taken (the
    residual of the final iterate would need one more rebuild).
For FP32 data the iterate is rounded to FP32 before each rebuild
(`data_prec="f32"`), since the GPU builds its graph from the stored FP32
iterate; all arithmetic stays FP64.
"""
from __future__ import annotations

import numpy as np

from .operator import build_operator
from .solvers import BREAKDOWN_TOL, CgInfo


def _round(x, data_prec: str):
    x = np.asarray(x, dtype=np.float64)
    return x.astype(np.float32).astype(np.float64) if data_prec == "f32" else x


def _build(kind, x, shape, radius, sigma_s, sigma_r, eps, data_prec, stencil, norm):
    return build_operator(kind, _round(x, data_prec).reshape(shape), radius, sigma_s, sigma_r, eps, stencil, norm)


def power_filter_reguided(kind: str, x0, shape, kmax: int, radius: int, sigma_s: float = 0.0,
                          sigma_r: float = 0.0, eps: float = 0.0, data_prec: str = "f64",
                          stencil: str = "square", norm: str = "d"):
    """kmax passes of x <- D(x)^-1 W(x) x (the non-linear iterated BF / GF;
    the RW form of the chosen normalization, see `build_operator`)."""
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    for _ in range(kmax):
        op = _build(kind, x, shape, radius, sigma_s, sigma_r, eps, data_prec, stencil, norm)
        x = op.apply_rw(x)
    return x


def cg_filter_reguided(kind: str, x0, shape, kmax: int, radius: int, sigma_s: float = 0.0,
                       sigma_r: float = 0.0, eps: float = 0.0, tol: float = 0.0, data_prec: str = "f64",
                       stencil: str = "square", norm: str = "d"):
    """Algorithm 2 with the graph rebuilt from the current iterate every step."""
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    op = _build(kind, x, shape, radius, sigma_s, sigma_r, eps, data_prec, stencil, norm)
    floor = (BREAKDOWN_TOL[data_prec] ** 2) * float(x @ (op.d * x))
    r = -op.apply_l(x)
    info = CgInfo()
    p = s_old = r_old = None
    rho0 = None
    for k in range(1, kmax + 1):
        if k > 1:
            op = _build(kind, x, shape, radius, sigma_s, sigma_r, eps, data_prec, stencil, norm)
        s = r / op.d
        rho = float(s @ r)
        if k == 1:
            rho0 = rho
            info.res0 = np.sqrt(max(rho0, 0.0))
        info.history.append(rho)
        if not (np.isfinite(rho) and rho > floor):
            info.status = "breakdown"
            info.res = np.sqrt(max(rho, 0.0)) if np.isfinite(rho) else rho
            return x, info
        if tol > 0.0 and np.sqrt(rho) <= tol * np.sqrt(rho0):
            info.status = "ok"
            info.res = np.sqrt(rho)
            return x, info
        if k == 1:
            p = s
        else:
            beta = float(s @ (r - r_old)) / float(s_old @ r_old)
            p = s + beta * p
        q = op.apply_l(p)
        pq = float(p @ q)
        if not (np.isfinite(pq) and pq > 0.0):
            info.status = "breakdown"
            info.res = np.sqrt(rho)
            return x, info
        alpha = rho / pq
        x = x + alpha * p
        r_old = r
        s_old = s
        r = r - alpha * q
        info.iters = k
    info.res = np.sqrt(max(info.history[-1], 0.0)) if info.history else 0.0
    if tol > 0.0 and info.res > tol * info.res0:
        info.status = "notconv"
    return x, info
