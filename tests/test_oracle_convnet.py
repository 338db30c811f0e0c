"""Pins of the oracle's learned-preconditioner pieces (network forward and
backward, BF16 rounding, Adam, the shifted solve for the training targets and
the preconditioner slot of flexible block LOBPCG, Algorithm 3) against
library routines, finite differences, closed forms and dense linear algebra."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

import oracle
from oracle import convnet as cn
from oracle.spectral import dense_normalized, eig_lsym
from synth import convnet_init, scene_2d


def _img(h=9, w=11, seed=3):
    _, x = scene_2d(h, w, 0.05, seed)
    return x


def _bf(h=10, w=12, seed=2, r=2):
    _, x = scene_2d(h, w, 0.05, seed)
    return oracle.build_operator("bf", x, r, 2.0, 0.15), x


# ------------------------------------------------------------------ bfloat16
def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    v = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cn.bf16_round(v.astype(np.float64)), ref)


def test_bf16_round_ties_to_even():
    one = 1.0
    assert cn.bf16_round(np.array([one + 2.0 ** -8]))[0] == 1.0            # tie -> even (1.0)
    assert cn.bf16_round(np.array([one + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6  # tie -> even
    assert cn.bf16_round(np.array([one + 2.0 ** -8 + 2.0 ** -20]))[0] == 1.0 + 2.0 ** -7
    assert cn.bf16_round(np.array([-3.0]))[0] == -3.0


# ------------------------------------------------------------------ convolutions
def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((3, 7, 9))
    Wt = rng.standard_normal((4, 3, 3, 3))
    ref = np.stack([sum(ndi.correlate(a[c], Wt[o, c], mode="constant", cval=0.0) for c in range(3))
                    for o in range(4)])
    np.testing.assert_allclose(cn.conv3x3(a, Wt), ref, rtol=1e-13, atol=1e-13)


def test_conv3x3_adjoint_dot_product():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((3, 6, 5))
    d = rng.standard_normal((4, 6, 5))
    Wt = rng.standard_normal((4, 3, 3, 3))
    lhs = float(np.sum(cn.conv3x3(a, Wt) * d))
    rhs = float(np.sum(a * cn.conv3x3_adjoint(d, Wt)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_weight_grad_is_derivative_of_linear_conv():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3, 5, 6))
    d = rng.standard_normal((2, 5, 6))
    g = cn.conv3x3_weight_grad(d, a)
    for (o, c, ky, kx) in [(0, 0, 0, 0), (1, 2, 1, 1), (0, 1, 2, 0), (1, 0, 2, 2)]:
        E = np.zeros((2, 3, 3, 3))
        E[o, c, ky, kx] = 1.0
        assert abs(g[o, c, ky, kx] - float(np.sum(cn.conv3x3(a, E) * d))) <= 1e-12


# ------------------------------------------------------------------ network
def test_loss_grad_matches_central_differences():
    rng = np.random.default_rng(4)
    w = convnet_init(7).astype(np.float64)
    B, H, W = 2, 6, 7
    x = rng.standard_normal((B, H, W))
    g = rng.uniform(0, 1, (B, H, W))
    t = rng.standard_normal((B, H, W))
    _, grad = cn.loss_and_grad(w, x, t, g, bf16=False)
    idx = np.concatenate([rng.choice(cn.N_W1, 8, replace=False),
                          cn.N_W1 + rng.choice(cn.N_W2, 16, replace=False),
                          cn.N_W1 + cn.N_W2 + rng.choice(cn.N_W3, 8, replace=False)])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (cn.loss_and_grad(wp, x, t, g, bf16=False)[0] - cn.loss_and_grad(wm, x, t, g, bf16=False)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * (abs(grad[i]) + 1e-3 * np.abs(grad).max()), (i, fd, grad[i])


def test_identity_network_is_identity():
    r = np.random.default_rng(5).standard_normal((8, 9))
    g = _img(8, 9)
    w = cn.identity_weights()
    np.testing.assert_allclose(cn.precond_apply(w, r, g, bf16=False), r, rtol=1e-15, atol=1e-15)
    s = cn.rms(r)
    np.testing.assert_array_equal(cn.precond_apply(w, r, g, bf16=True), s * cn.bf16_round(r / s))


def test_precond_positively_homogeneous():
    rng = np.random.default_rng(6)
    r = rng.standard_normal((7, 8))
    g = _img(7, 8)
    w = convnet_init(1).astype(np.float64)
    a = cn.precond_apply(w, r, g, bf16=False)
    b = cn.precond_apply(w, 37.5 * r, g, bf16=False)
    np.testing.assert_allclose(b, 37.5 * a, rtol=1e-13, atol=1e-13 * np.abs(b).max())
    np.testing.assert_array_equal(cn.precond_apply(w, np.zeros((7, 8)), g), np.zeros((7, 8)))


def test_forward_rounding_points():
    """With BF16 on, x, a1, a2 are exactly representable and y differs from
    the unrounded network by the size BF16 rounding implies."""
    rng = np.random.default_rng(7)
    w = convnet_init(2).astype(np.float64)
    r, g = rng.standard_normal((10, 12)), _img(10, 12)
    f = cn.forward(w, r, g, bf16=True)
    for k in ("x", "a1", "a2"):
        np.testing.assert_array_equal(cn.bf16_round(f[k]), f[k])
    y0 = cn.forward(w, r, g, bf16=False)["y"]
    rel = np.linalg.norm(f["y"] - y0) / np.linalg.norm(y0)
    assert 1e-5 < rel < 3e-2


# ------------------------------------------------------------------ Adam
def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2
    exactly, so every step moves by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(8)
    w0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        w, m, v = cn.adam_step(w, m, v, g, t, lr=1e-3)
    np.testing.assert_allclose(w, w0 - 5 * 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------ shifted solve
def test_shifted_cg_matches_dense_solve():
    op, _ = _bf()
    b = np.random.default_rng(9).standard_normal(op.n)
    y, info = oracle.shifted_cg(op, 1e-2, b, 2000, 1e-12)
    A = dense_normalized(op)[1] + 1e-2 * np.eye(op.n)
    ref = np.linalg.solve(A, b)
    assert info.status == "ok"
    assert np.linalg.norm(y - ref) <= 1e-9 * np.linalg.norm(ref)


def test_shifted_cg_zero_rhs_and_cap():
    op, _ = _bf()
    y, info = oracle.shifted_cg(op, 1e-2, np.zeros(op.n), 10, 1e-10)
    assert info.iters == 0 and np.all(y == 0.0)
    b = np.random.default_rng(10).standard_normal(op.n)
    _, info = oracle.shifted_cg(op, 1e-2, b, 3, 1e-14)
    assert info.iters == 3 and info.status == "notconv"


def test_lobpcg_residual_matches_dense():
    op, x = _bf()
    X = np.random.default_rng(11).standard_normal((op.n, 3))
    th = np.array([0.1, 0.2, 0.3])
    Ls = dense_normalized(op)[1]
    np.testing.assert_allclose(oracle.lobpcg_residual(op, X, th), Ls @ X - X * th, rtol=1e-12, atol=1e-13)


# ------------------------------------------------------------------ flexible LOBPCG
@pytest.mark.parametrize("constraint", [False, True])
def test_lobpcg_identity_network_equals_plain(constraint):
    op, x = _bf()
    T = cn.make_precond(cn.identity_weights(), x, x.shape, bf16=False)
    a = oracle.lobpcg_filter(op, x.ravel(), 3, 8, constraint=constraint)
    b = oracle.lobpcg_filter(op, x.ravel(), 3, 8, constraint=constraint, precond=T)
    np.testing.assert_allclose(b[0], a[0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b[1], a[1], rtol=1e-12, atol=1e-13)


def test_lobpcg_fallback_equals_plain():
    """A negated identity (r^T T r < 0) and a network with a NaN weight both
    fall back to T = I in every column: bitwise the plain method."""
    op, x = _bf()
    neg = cn.identity_weights()
    neg[cn.N_W1 + cn.N_W2:] *= -1.0
    nan = convnet_init(3).astype(np.float64)
    nan[100] = np.nan
    a = oracle.lobpcg_filter(op, x.ravel(), 3, 6, constraint=True)
    for w in (neg, nan):
        T = cn.make_precond(w, x, x.shape)
        b = oracle.lobpcg_filter(op, x.ravel(), 3, 6, constraint=True, precond=T)
        np.testing.assert_array_equal(b[0], a[0])
        np.testing.assert_array_equal(b[1], a[1])


def test_flexible_lobpcg_with_shift_invert_converges_faster():
    """T = (L_sym + alpha I)^-1 (the network's training target) speeds up
    convergence to the smallest non-trivial eigenpairs of L_sym."""
    op, x = _bf(14, 16, seed=5, r=2)
    lam, _ = eig_lsym(op)
    A = dense_normalized(op)[1] + 1e-2 * np.eye(op.n)
    Ainv = np.linalg.inv(A)
    T = lambda R: Ainv @ R
    tol = 1e-8
    _, th_p, _, ip = oracle.lobpcg_filter(op, x.ravel(), 3, 3000, tol=tol, constraint=True)
    _, th_t, _, it = oracle.lobpcg_filter(op, x.ravel(), 3, 3000, tol=tol, constraint=True, precond=T)
    assert ip.status == "ok" and it.status == "ok"
    np.testing.assert_allclose(th_t, lam[1:4], rtol=0, atol=1e-10)
    np.testing.assert_allclose(th_p, lam[1:4], rtol=0, atol=1e-10)
    assert 2 * it.iters < ip.iters, (it.iters, ip.iters)
