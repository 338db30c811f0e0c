"""Pins of the oracle's filters (power iteration, Algorithm 2 CG, Algorithm 3
block LOBPCG) against dense eigendecomposition, brute-force Krylov
minimisation, library eigensolvers and invariants on small graphs."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle.spectral import dense_normalized, eig_lsym, gft_lowpass
from synth import piecewise_constant_1d, scene_2d


def _bf_1d(n=80, seed=1, r=3):
    _, x = piecewise_constant_1d(n, 0.1, seed)
    return oracle.build_operator("bf", x, r, 3.0, 0.2), x


def _bf_2d(h=10, w=12, seed=2, r=2):
    _, x = scene_2d(h, w, 0.05, seed)
    return oracle.build_operator("bf", x, r, 2.0, 0.15), x.ravel()


def _gf_2d(h=9, w=11, seed=3, r=2):
    _, x = scene_2d(h, w, 0.05, seed)
    return oracle.build_operator("gf", x, r, eps=1e-2), x.ravel()


OPS = [_bf_1d, _bf_2d, _gf_2d]


# ---------------------------------------------------------------- power iteration
@pytest.mark.parametrize("make", OPS)
def test_power_iteration_is_spectral_filter(make):
    """z_k = U (1 - Lambda)^k U^T z0 (Section 4, eq. (8))."""
    op, x = make()
    lam, U = eig_lsym(op)
    k = 7
    zk = op.sqrt_d * oracle.power_filter(op, x, k)
    ref = U @ ((1.0 - lam) ** k * (U.T @ (op.sqrt_d * x)))
    np.testing.assert_allclose(zk, ref, rtol=1e-11, atol=1e-12)


def test_power_iteration_mass_and_maximum_principle():
    op, x = _bf_2d()
    xk = oracle.power_filter(op, x, 25)
    assert abs(op.d @ xk - op.d @ x) < 1e-11 * abs(op.d @ x)
    assert xk.min() >= x.min() - 1e-14 and xk.max() <= x.max() + 1e-14


# ---------------------------------------------------------------- CG
@pytest.mark.parametrize("make", OPS)
def test_cg_xspace_equals_zspace(make):
    op, x = make()
    a, ia = oracle.cg_filter(op, x, 12)
    b, ib = oracle.cg_filter_normalized(op, x, 12)
    np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-12)
    assert ia.iters == ib.iters == 12


def _krylov_orthobasis(A, v, k):
    K = np.empty((v.size, k))
    K[:, 0] = v
    for j in range(1, k):
        K[:, j] = A @ K[:, j - 1]
    Q, _ = np.linalg.qr(K)
    return Q


@pytest.mark.parametrize("make", OPS)
@pytest.mark.parametrize("k", [1, 3, 6])
def test_cg_is_energy_minimiser_over_krylov_space(make, k):
    """CG's k-th iterate minimises z^T L_sym z over z0 + K_k(L_sym, r0)
    (brute force with an explicit Krylov basis and a dense solve)."""
    op, x = make()
    _, Ls = dense_normalized(op)
    Ls = 0.5 * (Ls + Ls.T)
    z0 = op.sqrt_d * x
    Q = _krylov_orthobasis(Ls, -Ls @ z0, k)
    c = np.linalg.solve(Q.T @ Ls @ Q, -(Q.T @ Ls @ z0))
    zref = z0 + Q @ c
    xk, _ = oracle.cg_filter(op, x, k)
    np.testing.assert_allclose(op.sqrt_d * xk, zref, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("make", OPS)
def test_cg_ritz_value_polynomial(make):
    """z_k = p_k(L_sym) z0 with p_k(lambda) = prod_j (1 - lambda/theta_j), theta_j
    the Ritz values of L_sym on K_k(L_sym, r0) (the CG polynomial filter of
    Section 5)."""
    op, x = make()
    lam, U = eig_lsym(op)
    _, Ls = dense_normalized(op)
    Ls = 0.5 * (Ls + Ls.T)
    z0 = op.sqrt_d * x
    k = 5
    Q = _krylov_orthobasis(Ls, -Ls @ z0, k)
    theta = np.linalg.eigvalsh(Q.T @ Ls @ Q)
    pk = np.prod(1.0 - lam[:, None] / theta[None, :], axis=1)
    ref = U @ (pk * (U.T @ z0))
    xk, _ = oracle.cg_filter(op, x, k)
    np.testing.assert_allclose(op.sqrt_d * xk, ref, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("make", OPS)
def test_cg_mass_conservation_and_energy_decrease(make):
    op, x = make()
    mass0 = op.d @ x
    prev = None
    for k in range(1, 10):
        xk, _ = oracle.cg_filter(op, x, k)
        assert abs(op.d @ xk - mass0) <= 1e-11 * abs(mass0)
        e = xk @ op.apply_l(xk)
        if prev is not None:
            assert e <= prev * (1 + 1e-12)
        prev = e


def test_cg_constant_input_breaks_down_and_returns_input():
    op = oracle.build_operator("bf", np.linspace(0, 1, 30), 2, 2.0, 0.3)
    x0 = np.full(30, 0.4)
    xk, info = oracle.cg_filter(op, x0, 10)
    # r0 = -L x0 is zero up to rounding: either exact breakdown at k=1 or
    # tiny steps; the result must stay x0
    np.testing.assert_allclose(xk, x0, rtol=0, atol=1e-12)
    xk2, info2 = oracle.cg_filter(oracle.build_operator("bf", x0, 2, 2.0, 0.3), x0, 10)
    assert info2.status == "breakdown" and info2.iters == 0
    np.testing.assert_array_equal(xk2, x0)


def test_cg_finite_termination_tiny_graph():
    """With as many steps as distinct eigenvalues, CG reaches the null-space
    component: x = (e^T D x0 / e^T D e) e on a connected graph."""
    x = np.array([0.1, 0.9, 0.4, 0.6, 0.2, 0.8])
    op = oracle.build_operator("bf", x, 2, 2.0, 0.5)
    xk, info = oracle.cg_filter(op, x, 6, tol=1e-13)
    np.testing.assert_allclose(xk, (op.d @ x) / op.d.sum(), rtol=1e-8)


def test_cg_tolerance_stop():
    op, x = _bf_1d(200)
    xk, info = oracle.cg_filter_normalized(op, x, 500, tol=1e-6)
    assert info.status == "ok" and info.iters < 500
    assert info.res <= 1e-6 * info.res0


# ---------------------------------------------------------------- Rayleigh-Ritz
def test_rayleigh_ritz_matches_generalized_eigh():
    rng = np.random.default_rng(3)
    S = rng.standard_normal((40, 9))
    A0 = rng.standard_normal((40, 40))
    A = A0 @ A0.T
    GA, GB = S.T @ A @ S, S.T @ S
    theta, C, kept = oracle.rayleigh_ritz(GA, GB, 3, 1e-10)
    assert kept.all()
    ref = sla.eigh(GA, GB, eigvals_only=True)[:3]
    np.testing.assert_allclose(theta, ref, rtol=1e-10)
    np.testing.assert_allclose(C.T @ GB @ C, np.eye(3), atol=1e-10)
    np.testing.assert_allclose(C.T @ GA @ C, np.diag(theta), atol=1e-8 * theta.max())


def test_rayleigh_ritz_drops_dependent_columns():
    rng = np.random.default_rng(4)
    S = rng.standard_normal((30, 5))
    S = np.column_stack([S, S[:, 1] * 3.0, np.zeros(30)])  # duplicate and zero column
    A = np.diag(np.arange(1.0, 31.0))
    theta, C, kept = oracle.rayleigh_ritz(S.T @ A @ S, S.T @ S, 2, 1e-10)
    assert list(kept) == [True] * 5 + [False, False]
    ref = sla.eigh(S[:, :5].T @ A @ S[:, :5], S[:, :5].T @ S[:, :5], eigvals_only=True)[:2]
    np.testing.assert_allclose(theta, ref, rtol=1e-10)


def _start_block_reference(shape, z0, m):
    """The modulated start block rebuilt with scipy's Legendre evaluator."""
    from scipy.special import eval_legendre
    degs = oracle.modulation_degrees(len(shape), m)
    axes = [2.0 * (np.arange(s) + 0.5) / s - 1.0 for s in shape]
    cols = []
    for d in degs:
        if len(shape) == 1:
            phi = eval_legendre(d[0], axes[0])
        else:
            phi = np.outer(eval_legendre(d[0], axes[0]), eval_legendre(d[1], axes[1])).ravel()
        cols.append(z0 * phi)
    return np.column_stack(cols)


def test_modulation_degree_order():
    assert oracle.modulation_degrees(2, 8) == [(0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0), (0, 3), (1, 2)]
    assert oracle.modulation_degrees(1, 3) == [(0,), (1,), (2,)]


@pytest.mark.parametrize("shape,m", [((50,), 3), ((7, 9), 8)])
def test_modulated_start_block(shape, m):
    z0 = np.random.default_rng(5).uniform(0.5, 1.0, size=int(np.prod(shape)))
    X0 = oracle.modulated_start(shape, z0, m)
    np.testing.assert_array_equal(X0[:, 0], z0)          # phi_0 = 1: z0 in the start space
    np.testing.assert_allclose(X0, _start_block_reference(shape, z0, m), rtol=1e-13, atol=1e-14)
    assert np.linalg.matrix_rank(X0) == m


# ---------------------------------------------------------------- LOBPCG
@pytest.mark.parametrize("make", OPS)
def test_lobpcg_identity_at_zero_iterations(make):
    op, x = make()
    y, _, _, _ = oracle.lobpcg_filter(op, x, 3, 0)
    np.testing.assert_allclose(y, x, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("make", OPS)
@pytest.mark.parametrize("constraint", [False, True])
def test_lobpcg_first_steps_are_rayleigh_ritz_on_explicit_spans(make, constraint):
    """The first two LOBPCG steps equal Rayleigh-Ritz of L_sym on the explicit
    trial spaces span{X0, W0} and span{X1, W1, P1} (generalised eigensolves
    from scipy on dense matrices)."""
    op, x = make()
    m = 3
    _, Ls = dense_normalized(op)
    Ls = 0.5 * (Ls + Ls.T)
    z0 = op.sqrt_d * x
    Y = op.sqrt_d / np.linalg.norm(op.sqrt_d)
    proj = (lambda B: B - np.outer(Y, Y @ B)) if constraint else (lambda B: B)
    X0 = proj(_start_block_reference(op.shape, z0, m))
    lam, Z = sla.eigh(X0.T @ Ls @ X0, X0.T @ X0)
    X = X0 @ Z
    W = proj(Ls @ X - X * lam)
    S = np.column_stack([X, W])
    lam1, Z1 = sla.eigh(S.T @ Ls @ S, S.T @ S)
    X1 = S @ Z1[:, :m]
    P1 = W @ Z1[m:, :m]
    W1 = proj(Ls @ X1 - X1 * lam1[:m])
    S2 = np.column_stack([X1, W1, P1])
    lam2 = sla.eigh(S2.T @ Ls @ S2, S2.T @ S2, eigvals_only=True)[:m]
    _, th1, _, _ = oracle.lobpcg_filter(op, x, m, 1, constraint=constraint)
    _, th2, _, info = oracle.lobpcg_filter(op, x, m, 2, constraint=constraint)
    assert info.dropped == 0
    np.testing.assert_allclose(th1, lam1[:m], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(th2, lam2, rtol=1e-8, atol=1e-11)


@pytest.mark.parametrize("make", OPS)
@pytest.mark.parametrize("constraint", [False, True])
def test_lobpcg_converges_to_lowest_modes(make, constraint):
    """Many iterations: Theta -> the m smallest eigenvalues of L_sym (the
    smallest non-trivial ones under the constraint), y -> the GFT low-pass
    U_m U_m^T z0; Courant-Fischer bounds hold all along."""
    op, x = make()
    m = 3
    lam, U = eig_lsym(op)
    z0 = op.sqrt_d * x
    y, theta, X, info = oracle.lobpcg_filter(op, x, m, 400, tol=1e-10, constraint=constraint)
    if constraint:
        ref_lam = lam[1:m + 1]
        ref_y = gft_lowpass(U[:, 1:], z0, m) + U[:, 0] * (U[:, 0] @ z0)
    else:
        ref_lam = lam[:m]
        ref_y = gft_lowpass(U, z0, m)
    np.testing.assert_allclose(theta, ref_lam, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(op.sqrt_d * y, ref_y, rtol=1e-5, atol=1e-6 * np.linalg.norm(z0))
    for th in info.theta_history:
        assert np.all(th >= ref_lam - 1e-10)
    sums = [t.sum() for t in info.theta_history]
    assert all(b <= a + 1e-12 for a, b in zip(sums, sums[1:]))


def test_lobpcg_against_scipy_lobpcg():
    from scipy.sparse.linalg import lobpcg as sp_lobpcg
    op, x = _bf_1d(120, r=4)
    _, Ls = dense_normalized(op)
    Ls = 0.5 * (Ls + Ls.T)
    _, theta, _, _ = oracle.lobpcg_filter(op, x, 4, 500, tol=1e-10)
    X0 = np.random.default_rng(0).standard_normal((op.n, 4))
    ref, _ = sp_lobpcg(Ls, X0, largest=False, tol=1e-10, maxiter=2000)
    np.testing.assert_allclose(np.sort(theta), np.sort(ref), rtol=1e-6, atol=1e-9)


def test_lobpcg_single_vector_reduces_to_algorithm3_output():
    """m = 1: y = x_k (x_k^T D x0) / (x_k^T D x_k) in x-space."""
    op, x = _bf_1d(60)
    y, theta, X, _ = oracle.lobpcg_filter(op, x, 1, 5)
    xk = X[:, 0] / op.sqrt_d
    ref = xk * (xk @ (op.d * x)) / (xk @ (op.d * xk))
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-13)


def test_lobpcg_constant_input_breakdown():
    op = oracle.build_operator("bf", np.linspace(0, 1, 20), 2, 2.0, 0.3)
    x0 = np.full(20, 0.3)
    y, _, _, info = oracle.lobpcg_filter(op, x0, 2, 5, constraint=True)
    assert info.status == "breakdown"
    np.testing.assert_array_equal(y, x0)


def test_rayleigh_ritz_sign_convention():
    """Each coefficient column has its largest-magnitude entry positive, and
    the rest of the result is the plain eigen-decomposition's (up to sign)."""
    rng = np.random.default_rng(21)
    S = rng.standard_normal((40, 6))
    A = rng.standard_normal((40, 40))
    A = A @ A.T
    GA, GB = S.T @ A @ S, S.T @ S
    theta, C, kept = oracle.rayleigh_ritz(GA, GB, 3, 1e-12)
    for j in range(3):
        i = int(np.argmax(np.abs(C[:, j])))
        assert C[i, j] > 0
    w, V = sla.eigh(GA, GB)
    np.testing.assert_allclose(theta, w[:3], rtol=1e-10)
    np.testing.assert_allclose(np.abs(C), np.abs(V[:, :3]), rtol=1e-8, atol=1e-10)


def test_lobpcg_ax_refresh_changes_only_rounding():
    """The explicit AX refresh (every 20 steps by default) is an identity in
    exact arithmetic: runs refreshing every step, every 20 steps and never
    agree to rounding after 60 steps, and the refreshed run's reported
    residuals are those of the explicit L_sym X."""
    import oracle
    from synth import scene_2d
    g = scene_2d(30, 36, 0.05, 17)[1]
    op = oracle.build_operator("bf", g, 2, 2.0, 0.1)
    outs = [oracle.lobpcg_filter(op, g.ravel(), 3, 60, refresh=r) for r in (0, 1, 20)]
    for y, th, X, info in outs[1:]:
        assert np.linalg.norm(y - outs[0][0]) <= 1e-10 * np.linalg.norm(outs[0][0])
        np.testing.assert_allclose(th, outs[0][1], rtol=1e-10, atol=1e-14)
    y, th, X, info = outs[2]
    R = op.apply_lsym(X) - X * th[None, :]
    np.testing.assert_allclose(np.linalg.norm(R, axis=0), info.res, rtol=1e-6, atol=1e-14)


def test_exact_shifted_solve_preconditioner_bound():
    """The preconditioner the learned network imitates, applied exactly:
    T = (L_sym + alpha I)^-1 by a sparse LU factorisation.  On a 64 x 64
    scene (BF 11 x 11, m = 4, the constraint, tol 1e-6) it cuts the LOBPCG
    step count at alpha = 1e-2 to a third of the plain method's or less, and
    the count grows with alpha (a larger shift flattens the spectrum less
    near the wanted small eigenvalues).  This is the ceiling any imitation
    of T can reach."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    g = scene_2d(64, 64, 0.05, 5900)[1]
    op = oracle.build_operator("bf", g, 5, 2.0, 0.1)
    Dm = sp.diags(1.0 / op.sqrt_d)
    L = sp.identity(op.n) - Dm @ op.W @ Dm
    plain = oracle.lobpcg_filter(op, g.ravel(), 4, 5000, tol=1e-6, constraint=True)[3]
    steps = []
    for alpha in (1e-2, 1e-1, 1.0):
        lu = spl.splu(sp.csc_matrix(L + alpha * sp.identity(op.n)))
        info = oracle.lobpcg_filter(op, g.ravel(), 4, 5000, tol=1e-6, constraint=True,
                                    precond=lambda R, lu=lu: lu.solve(np.ascontiguousarray(R)))[3]
        assert info.status == "ok"
        steps.append(info.iters)
    print("plain", plain.iters, "exact T at alpha 1e-2, 1e-1, 1:", steps)
    assert plain.status == "ok"
    assert 3 * steps[0] <= plain.iters
    assert steps[0] <= steps[1] <= steps[2] <= plain.iters


def test_lobpcg_soft_locking():
    """tol > 0: a column whose residual is already at the tolerance has a
    zero W column, so every step that starts from such a residual drops at
    least that many columns; the locked run still converges to the lowest
    eigenpairs of the dense operator, and with tol = 0 nothing is locked."""
    g = scene_2d(20, 20, 0.05, 3)[1]
    op = oracle.build_operator("bf", g, 2, 2.0, 0.3)
    tol = 1e-9
    y, th, X, info = oracle.lobpcg_filter(op, g.ravel(), 3, 500, tol=tol)
    assert info.status == "ok"
    locked_steps = 0
    for res, drops in zip(info.res_history, info.drop_history):
        nl = int(np.count_nonzero(res <= tol))
        assert drops >= nl
        locked_steps += nl > 0
    assert locked_steps >= 3
    lam = eig_lsym(op)[0]
    np.testing.assert_allclose(th, lam[:3], atol=1e-12)
    assert np.max(info.res) <= tol
    # the same iteration without a tolerance: nothing is locked, so its first
    # steps (before any column reaches 1e-9) drop nothing more than the locked run
    _, _, _, free = oracle.lobpcg_filter(op, g.ravel(), 3, info.iters)
    first = next(k for k, r in enumerate(info.res_history) if np.any(r <= tol))
    assert free.drop_history[:first] == info.drop_history[:first]
    assert sum(free.drop_history) < info.dropped
