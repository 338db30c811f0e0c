"""Iteration drivers: the polynomial filters (paper Sections 4-6).

All three work on a fixed graph operator (oracle.operator.GraphOperator) and
take the noisy signal x0 as the starting vector.

Power iteration (Section 4): x_{k+1} = D^-1 W x_k.

Preconditioned CG for L x = 0 with preconditioner D (Algorithm 2).
  Reading of the beta line: the printed denominator s_old^T s_old is read as
  s_old^T r_old.  This is the standard PCG normalisation that the paper says
  Algorithm 2 only slightly modifies; with it, x-space PCG with preconditioner
  D is the same iteration as plain CG on L_sym in z = D^1/2 x, and the
  numerator s^T (r - r_old) is the flexible (Polak-Ribiere type) variant the
  paper describes.
  Initial residual r = -L x0 (right-hand side zero).
  Stopping / breakdown (our reading; the paper runs exactly kmax steps):
    before step k compute rho = s^T r.  rho <= (tau ||z0||)^2, with
    ||z0||^2 = x0^T D x0 and tau = 1e-13 (FP64 data) or 1e-6 (FP32 data), or
    rho non-finite: breakdown (x kept, status "breakdown"); the residual is
    then at the rounding level of the input, which is what a constant x0
    gives.  If tol > 0
    and sqrt(rho) <= tol * sqrt(rho_0): converged, stop.  After q = L p:
    p^T q <= 0 or non-finite: breakdown, stop.  At the end, tol > 0 and the
    final residual above tol * res0: status "notconv".

Block LOBPCG as a low-pass filter (Algorithm 3, Section 6), generalised to a
block of m vectors (our reading; the paper gives the single-vector method):
  operator A = L_sym in z-space, B = I, preconditioner T = I (which is T = D^-1
  in x-space);
  start block: the noisy signal modulated by m smooth functions of position,
  X0[:, j] = z0 * phi_j with phi_0 = 1 and phi_j Legendre polynomials of the
  normalised pixel coordinates (products P_a(t_row) P_b(t_col) ordered by
  total degree a + b, then by a); z0 = X0 e_1 lies in the start space, so the
  filter is the identity at k = 0, and for m = 1 this is Algorithm 3's start.
  (A Krylov basis of z0 would not do: its residual block adds a single new
  direction per step, so the block would collapse to rank m + 1.)
  If the start block (after the constraint projection) has rank < m the
  filter reports a breakdown and returns x0;
  constraint (optional): x orthogonal to the null vector of L, which in
  z-space is Y = D^1/2 e / ||D^1/2 e||; z0's Y-component is removed from the
  start and every W is projected against Y;
  each step: R = AX - X Theta, W = T R (projected), Rayleigh-Ritz on
  S = [X, W, P] with the FP64 Gram pair (S^T A S, S^T S), keeping the m
  smallest Ritz pairs; P = [W, P] C_{W,P}; AX, AP by the same combinations;
  the Rayleigh-Ritz step orthonormalises S by a Cholesky factorisation of the
  unit-diagonal-scaled S^T S that drops every column whose pivot falls below
  drop_tol (1e-10 for FP64 data, 1e-6 for FP32 data), and drops as zero a
  column whose norm is below tau (the CG breakdown tau) times the largest
  column norm;
  output: the projection y = X X^T z0 (+ Y Y^T z0 with the constraint),
  returned in x-space as D^-1/2 y.  It is the identity at k = 0 and tends to
  the GFT low-pass U_m U_m^T z0 (Section 4) as the Ritz block converges.
  tol > 0 stops once every column's residual ||A x_j - theta_j x_j|| <= tol;
  until then a column whose residual is already <= tol is soft-locked: its
  x_j stays in the Rayleigh-Ritz basis but its W column is zero (so the
  Rayleigh-Ritz step drops it and counts the drop).
  AX is carried by the update's linear combinations and recomputed as A X
  after every `refresh`-th step (20; 0 never), so that the rounding the
  recurrence accumulates does not set a floor under the residual (C-10, C-16:
  in exact arithmetic both give the same AX).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DROP_TOL = {"f64": 1e-10, "f32": 1e-6}
AX_REFRESH = 20
BREAKDOWN_TOL = {"f64": 1e-13, "f32": 1e-6}


# --------------------------------------------------------------------------
# power iteration
# --------------------------------------------------------------------------
def power_filter(op, x0, kmax: int):
    """kmax passes of x <- D^-1 W x (iterated BF / GF with fixed weights)."""
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    for _ in range(kmax):
        x = op.apply_rw(x)
    return x


# --------------------------------------------------------------------------
# CG (Algorithm 2)
# --------------------------------------------------------------------------
@dataclass
class CgInfo:
    iters: int = 0
    status: str = "ok"
    res0: float = 0.0
    res: float = 0.0
    history: list = field(default_factory=list)


def cg_filter(op, x0, kmax: int, tol: float = 0.0, data_prec: str = "f64"):
    """Algorithm 2 in x-space: PCG for L x = 0 with preconditioner D."""
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    d = op.d
    floor = (BREAKDOWN_TOL[data_prec] ** 2) * float(x @ (d * x))
    r = -op.apply_l(x)
    info = CgInfo()
    p = s_old = r_old = None
    rho0 = None
    for k in range(1, kmax + 1):
        s = r / d
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
    rho = float((r / d) @ r)
    info.res = np.sqrt(max(rho, 0.0))
    if tol > 0.0 and info.res > tol * info.res0:
        info.status = "notconv"
    return x, info


def cg_filter_block(op, X0, kmax: int, tol: float = 0.0, data_prec: str = "f64"):
    """Algorithm 2 on each column of an n x m block (the channels of a colour
    signal share one graph): the columns are independent CG runs, each with
    its own stopping decisions.  Returns (Y, [CgInfo per column])."""
    X0 = np.asarray(X0, dtype=np.float64)
    out = np.empty_like(X0)
    infos = []
    for j in range(X0.shape[1]):
        out[:, j], info = cg_filter(op, X0[:, j], kmax, tol, data_prec)
        infos.append(info)
    return out, infos


def cg_filter_normalized(op, x0, kmax: int, tol: float = 0.0, data_prec: str = "f64"):
    """The same iteration written for L_sym z = 0 in z = D^1/2 x with T = I
    (s = r); returns x = D^-1/2 z."""
    z = op.sqrt_d * np.asarray(x0, dtype=np.float64).ravel()
    floor = (BREAKDOWN_TOL[data_prec] ** 2) * float(z @ z)
    r = -op.apply_lsym(z)
    info = CgInfo()
    p = r_old = None
    rho0 = None
    for k in range(1, kmax + 1):
        rho = float(r @ r)
        if k == 1:
            rho0 = rho
            info.res0 = np.sqrt(rho0)
        info.history.append(rho)
        if not (np.isfinite(rho) and rho > floor):
            info.status = "breakdown"
            info.res = np.sqrt(max(rho, 0.0)) if np.isfinite(rho) else rho
            return z / op.sqrt_d, info
        if tol > 0.0 and np.sqrt(rho) <= tol * np.sqrt(rho0):
            info.res = np.sqrt(rho)
            return z / op.sqrt_d, info
        if k == 1:
            p = r
        else:
            beta = float(r @ (r - r_old)) / float(r_old @ r_old)
            p = r + beta * p
        q = op.apply_lsym(p)
        pq = float(p @ q)
        if not (np.isfinite(pq) and pq > 0.0):
            info.status = "breakdown"
            info.res = np.sqrt(rho)
            return z / op.sqrt_d, info
        alpha = rho / pq
        z = z + alpha * p
        r_old = r
        r = r - alpha * q
        info.iters = k
    info.res = float(np.sqrt(r @ r))
    if tol > 0.0 and info.res > tol * info.res0:
        info.status = "notconv"
    return z / op.sqrt_d, info


# --------------------------------------------------------------------------
# LOBPCG (Algorithm 3, block form)
# --------------------------------------------------------------------------
@dataclass
class LobpcgInfo:
    iters: int = 0
    status: str = "ok"
    dropped: int = 0          # columns removed by the Rayleigh-Ritz Cholesky
    res: np.ndarray = None    # final per-column residual norms
    theta_history: list = field(default_factory=list)
    res_history: list = field(default_factory=list)    # residual norms each step starts from
    drop_history: list = field(default_factory=list)   # columns dropped by each step


def modulation_degrees(ndim: int, m: int):
    """Polynomial degrees (a, b) of the start-block modulations phi_j:
    total degree ascending, then row degree a ascending (1D: (j,))."""
    if ndim == 1:
        return [(j,) for j in range(m)]
    out = []
    s = 0
    while len(out) < m:
        for a in range(s + 1):
            if len(out) < m:
                out.append((a, s - a))
        s += 1
    return out


def modulated_start(shape, z0, m: int):
    """X0[:, j] = z0 * phi_j (see module docstring), phi_j evaluated with
    numpy's Legendre series at t = 2 (i + 1/2) / n - 1 per axis."""
    from numpy.polynomial import legendre
    z0 = np.asarray(z0, dtype=np.float64).ravel()
    axes = [2.0 * (np.arange(s) + 0.5) / s - 1.0 for s in shape]
    X0 = np.empty((z0.size, m))
    for j, degs in enumerate(modulation_degrees(len(shape), m)):
        phi = np.ones(())
        for t, deg in zip(axes, degs):
            coef = np.zeros(deg + 1)
            coef[deg] = 1.0
            phi = np.multiply.outer(phi, legendre.legval(t, coef))
        X0[:, j] = z0 * phi.ravel()
    return X0


def rayleigh_ritz(GA, GB, m: int, drop_tol: float, zero_tol: float = 0.0):
    """Rayleigh-Ritz for the pencil (GA, GB) of a trial basis S
    (GA = S^T A S, GB = S^T S): the m smallest Ritz values and coefficient
    vectors C with S C B-orthonormal.

    Steps: symmetrise; a column whose squared norm GB_jj is <= zero_tol^2 times
    the largest GB_jj is dropped as zero (rounding-level residuals, an empty
    projected start column); scale the rest to unit diagonal
    (delta = diag(GB)^-1/2); Cholesky factor the scaled GB column by column,
    dropping a column whose pivot (squared distance from the span of the kept
    columns) is <= drop_tol; reduce A to L^-1 A_K L^-T; dense symmetric
    eigensolve; back-transform; fix the sign of each column of C so that its
    largest-magnitude entry (the first one on ties) is positive (the Ritz
    vectors, and so the residuals a non-linear preconditioner sees, then have
    a sign that does not depend on the eigensolver).
    Returns (theta[m] ascending, C[k x m] with zero rows at dropped columns,
    kept[k] bool)."""
    GA = 0.5 * (np.asarray(GA) + np.asarray(GA).T)
    GB = 0.5 * (np.asarray(GB) + np.asarray(GB).T)
    k = GA.shape[0]
    diag = np.diag(GB).copy()
    kept = np.zeros(k, dtype=bool)
    delta = np.zeros(k)
    good = diag > (zero_tol ** 2) * max(float(diag.max()), 0.0)
    delta[good] = 1.0 / np.sqrt(diag[good])
    B = delta[:, None] * GB * delta[None, :]
    A = delta[:, None] * GA * delta[None, :]
    # bordered Cholesky with column dropping: L L^T = B[K, K]
    idx = []
    L = np.zeros((0, 0))
    for j in range(k):
        if not good[j]:
            continue
        b = B[j, idx]
        c = np.zeros(len(idx))
        for t in range(len(idx)):            # forward substitution L c = b
            c[t] = (b[t] - L[t, :t] @ c[:t]) / L[t, t]
        piv = B[j, j] - c @ c
        if piv > drop_tol:
            Ln = np.zeros((len(idx) + 1, len(idx) + 1))
            Ln[:len(idx), :len(idx)] = L
            Ln[len(idx), :len(idx)] = c
            Ln[len(idx), len(idx)] = np.sqrt(piv)
            L = Ln
            idx.append(j)
    idx = np.array(idx, dtype=np.int64)
    kept[idx] = True
    Linv = np.linalg.inv(L)
    M = Linv @ A[np.ix_(idx, idx)] @ Linv.T
    M = 0.5 * (M + M.T)
    theta, Z = np.linalg.eigh(M)
    CK = Linv.T @ Z[:, :m]
    C = np.zeros((k, m))
    C[idx, :] = delta[idx, None] * CK
    for j in range(C.shape[1]):
        i = int(np.argmax(np.abs(C[:, j])))
        if C[i, j] < 0.0:
            C[:, j] = -C[:, j]
    return theta[:m], C, kept


def precondition(T, R):
    """W = T(R) column by column with the fallback rule of the learned
    preconditioner (our reading): a column whose output has a non-finite
    entry or for which r^T T(r) <= 0 (T(r) not a descent direction of the
    Rayleigh quotient) uses T = I instead."""
    W = np.asarray(T(R), dtype=np.float64)
    out = R.copy()
    for j in range(R.shape[1]):
        w = W[:, j]
        if np.all(np.isfinite(w)) and float(R[:, j] @ w) > 0.0:
            out[:, j] = w
    return out


def lobpcg_filter(op, x0, m: int, kmax: int, tol: float = 0.0, constraint: bool = False,
                  data_prec: str = "f64", X0=None, precond=None, refresh: int = AX_REFRESH):
    """Block LOBPCG low-pass filter (see module docstring).
    precond: None (T = I) or a callable R (n, m) -> T(R) used with the
    fallback rule of `precondition` (flexible LOBPCG: T may change or be
    non-linear; the Rayleigh-Ritz step over [X, W, P] needs no other change).
    Returns (x_out, theta, X, info); X columns have sign x_j^T z0 >= 0."""
    drop_tol = DROP_TOL[data_prec]
    x0 = np.asarray(x0, dtype=np.float64).ravel()
    z0 = op.sqrt_d * x0
    A = op.apply_lsym
    Y = op.sqrt_d / np.linalg.norm(op.sqrt_d) if constraint else None
    info = LobpcgInfo()
    if X0 is None:
        X = modulated_start(op.shape, z0, m)
    else:
        X = np.array(X0, dtype=np.float64).reshape(op.n, m)
    if constraint:
        X = X - np.outer(Y, Y @ X)
    AX = A(X)
    zero_tol = BREAKDOWN_TOL[data_prec]
    theta, C, kept = rayleigh_ritz(X.T @ AX, X.T @ X, m, drop_tol, zero_tol)
    if np.count_nonzero(kept) < m:
        info.status = "breakdown"
        info.res = np.zeros(m)
        return x0.copy(), np.zeros(m), X, info
    X = X @ C
    AX = AX @ C
    P = AP = None
    res = np.linalg.norm(AX - X * theta[None, :], axis=0)
    for k in range(kmax):
        R = AX - X * theta[None, :]
        res = np.linalg.norm(R, axis=0)
        if tol > 0.0 and np.max(res) <= tol:
            break
        W = R if precond is None else precondition(precond, R)
        if tol > 0.0:
            # soft locking: a column already at the tolerance adds no search
            # direction (its zero column is then dropped by rayleigh_ritz)
            W = np.where((res <= tol)[None, :], 0.0, W)
        if constraint:
            W = W - np.outer(Y, Y @ W)
        AW = A(W)
        if P is None:
            S = np.column_stack([X, W])
            AS = np.column_stack([AX, AW])
        else:
            S = np.column_stack([X, W, P])
            AS = np.column_stack([AX, AW, AP])
        theta, C, kept = rayleigh_ritz(S.T @ AS, S.T @ S, m, drop_tol, zero_tol)
        info.dropped += int(np.count_nonzero(~kept))
        info.res_history.append(res.copy())
        info.drop_history.append(int(np.count_nonzero(~kept)))
        Cp = C.copy()
        Cp[:m, :] = 0.0
        X, AX, P, AP = S @ C, AS @ C, S @ Cp, AS @ Cp
        if refresh > 0 and (k + 1) % refresh == 0:
            AX = A(X)
        info.iters = k + 1
        info.theta_history.append(theta.copy())
        res = np.linalg.norm(AX - X * theta[None, :], axis=0)
    info.res = res
    if tol > 0.0 and np.max(res) > tol:
        info.status = "notconv"
    y = X @ (X.T @ z0)
    if constraint:
        y = y + Y * (Y @ z0)
    signs = np.where(X.T @ z0 >= 0.0, 1.0, -1.0)
    return y / op.sqrt_d, theta, X * signs[None, :], info


def lobpcg_residual(op, X, theta):
    """Residual block R = L_sym X - X diag(theta) of given Ritz pairs
    (Algorithm 3, residual line, in z-space)."""
    X = np.asarray(X, dtype=np.float64)
    return op.apply_lsym(X) - X * np.asarray(theta, dtype=np.float64)[None, :]


@dataclass
class ShiftedCgInfo:
    iters: int = 0
    status: str = "ok"
    res: float = 0.0


def shifted_cg(op, alpha: float, b, kmax: int, tol: float):
    """Plain CG for (L_sym + alpha I) y = b from y = 0 (the training targets
    of the learned preconditioner; the recurrences of Algorithm 2 with T = I
    on an SPD matrix, including its beta numerator r^T (r - r_old)).  Stops
    when ||b - (L_sym + alpha I) y|| <= tol ||b|| (recursive residual) or
    after kmax steps; p^T q <= 0 is a breakdown.  Returns (y, info)."""
    b = np.asarray(b, dtype=np.float64).ravel()
    y = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = float(r @ r)
    bn = np.sqrt(rho)
    info = ShiftedCgInfo()
    for k in range(kmax):
        if np.sqrt(rho) <= tol * bn:
            break
        q = op.apply_lsym(p) + alpha * p
        pq = float(p @ q)
        if not (pq > 0.0):
            info.status = "breakdown"
            break
        a = rho / pq
        y = y + a * p
        r_old = r
        r = r - a * q
        rho_new = float(r @ r)
        p = r + (float(r @ (r - r_old)) / rho) * p
        rho = rho_new
        info.iters = k + 1
    info.res = float(np.sqrt(rho))
    if info.status == "ok" and np.sqrt(rho) > tol * bn:
        info.status = "notconv"
    return y, info
