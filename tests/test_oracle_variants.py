"""Pins of the oracle's BF options for the image experiment of Section 7:
the cross (5-point-type) lattice and the (diag L)^-1/2 L (diag L)^-1/2
normalization of Section 4."""
import numpy as np
import pytest

import oracle
from oracle.pointwise import _bf_w
from oracle.spectral import dense_normalized
from synth import piecewise_constant_1d, scene_2d


def _img(h=9, w=11, seed=31):
    return scene_2d(h, w, 0.1, seed)[1]


def test_cross_lattice_pattern_and_weights():
    """Radius 1: every pixel is joined to itself and its 4 axis neighbours
    (3 at corners, 4 at edges, 5 inside) with the weights of eq. (2)."""
    g = _img()
    W = oracle.bf_weight_matrix(g, 1, 1.5, 0.1, stencil="cross").tocsr()
    H, Wd = g.shape
    nnz = np.diff(W.indptr).reshape(H, Wd)
    expect = np.full((H, Wd), 5)
    expect[0, :] -= 1
    expect[-1, :] -= 1
    expect[:, 0] -= 1
    expect[:, -1] -= 1
    assert np.array_equal(nnz, expect)
    rng = np.random.default_rng(0)
    for i in rng.choice(g.size, 25, replace=False):
        p = np.array(np.unravel_index(i, g.shape))
        for j in W.indices[W.indptr[i]:W.indptr[i + 1]]:
            q = np.array(np.unravel_index(j, g.shape))
            assert abs(np.abs(q - p).sum()) <= 1
            assert W[i, j] == pytest.approx(_bf_w(g, p, q[None, :], 1.5, 0.1)[0], rel=1e-15)


def test_cross_radius_r_axes_only():
    g = _img()
    W = oracle.bf_weight_matrix(g, 3, 2.0, 0.2, stencil="cross").tocsr()
    coo = W.tocoo()
    pi = np.array(np.unravel_index(coo.row, g.shape))
    pj = np.array(np.unravel_index(coo.col, g.shape))
    o = pj - pi
    assert np.all((o[0] == 0) | (o[1] == 0)) and np.abs(o).max() == 3


def test_cross_equals_square_in_1d():
    _, x = piecewise_constant_1d(50, 0.1, 3)
    a = oracle.bf_weight_matrix(x, 3, 2.0, 0.2, stencil="cross")
    b = oracle.bf_weight_matrix(x, 3, 2.0, 0.2)
    assert (a != b).nnz == 0


@pytest.mark.parametrize("stencil", ["square", "cross"])
def test_diagl_normalization_against_dense(stencil):
    """L_sym = (diag L)^-1/2 L (diag L)^-1/2 with L = D - W formed densely;
    its diagonal is 1; RW = (diag L)^-1 (W - I) (the Jacobi form)."""
    g = _img()
    op = oracle.build_operator("bf", g, 2 if stencil == "square" else 1, 2.0, 0.1, stencil=stencil, norm="diagl")
    Wd = op.W.toarray()
    off = Wd - np.diag(np.diag(Wd))
    assert np.all(np.diag(Wd) == 1.0)
    L = np.diag(off.sum(axis=1)) - off  # the self-loops cancel in D - W
    s = 1.0 / np.sqrt(np.diag(L))
    Ls_ref = s[:, None] * L * s[None, :]
    _, Ls = dense_normalized(op)
    np.testing.assert_allclose(Ls, Ls_ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(np.diag(Ls), 1.0, rtol=0, atol=1e-14)
    x = np.random.default_rng(1).standard_normal(op.n)
    rw_ref = ((Wd - np.eye(op.n)) @ x) / np.diag(L)
    np.testing.assert_allclose(op.apply_rw(x), rw_ref, rtol=0, atol=1e-13)
    lam = np.linalg.eigvalsh(0.5 * (Ls + Ls.T))
    assert lam[0] > -1e-13 and lam[-1] < 2.0 + 1e-13
    z1 = op.sqrt_d  # (diag L)^1/2 1 is the null vector
    assert np.linalg.norm(op.apply_lsym(z1)) <= 1e-13 * np.linalg.norm(z1)


def test_cross_diagl_does_not_depend_on_sigma_d():
    """On the cross lattice every neighbour is at distance 1, so sigma_d only
    scales the off-diagonal weights; the (diag L) normalization removes the
    scale (this is why the paper gives only sigma_r)."""
    g = _img()
    a = oracle.build_operator("bf", g, 1, 1.0, 0.1, stencil="cross", norm="diagl")
    b = oracle.build_operator("bf", g, 1, np.inf, 0.1, stencil="cross", norm="diagl")
    np.testing.assert_allclose(dense_normalized(a)[1], dense_normalized(b)[1], rtol=0, atol=1e-14)


def test_diagl_cg_xspace_equals_zspace():
    """Algorithm 2 with preconditioner diag L equals CG on the (diag L)
    normalized Laplacian in z = (diag L)^1/2 x."""
    g = _img()
    op = oracle.build_operator("bf", g, 1, 2.0, 0.1, stencil="cross", norm="diagl")
    x = g.ravel()
    y1, i1 = oracle.cg_filter(op, x, 15)
    y2, i2 = oracle.cg_filter_normalized(op, x, 15)
    assert i1.iters == i2.iters == 15
    np.testing.assert_allclose(y1, y2, rtol=0, atol=1e-12 * np.abs(y1).max())


def test_gf_rejects_bf_options():
    g = _img()
    with pytest.raises(ValueError):
        oracle.build_operator("gf", g, 2, eps=1e-2, stencil="cross")
    with pytest.raises(ValueError):
        oracle.build_operator("gf", g, 2, eps=1e-2, norm="diagl")


def test_diagl_isolated_vertex_and_small_diag():
    """A pixel whose neighbours all differ by far more than sigma_r: its
    off-diagonal weights underflow to 0, diag L_i = 0, row and column i of L
    vanish and the scale 1 is used there, so the pixel is a fixed point of the
    power and CG filters.  A pixel with diag L_i ~ 1e-9 keeps full relative
    precision in diag L (no d_i - 1 cancellation)."""
    g = np.zeros((7, 8))
    g[3, 4] = 50.0                      # exp(-50^2 / 0.02) underflows to 0
    g[1, 1] = 0.1 * np.sqrt(2 * 20.7)   # w = exp(-20.7) ~ 1e-9 to each of 4 neighbours
    op = oracle.build_operator("bf", g, 1, 1.0, 0.1, stencil="cross", norm="diagl")
    i_iso = 3 * 8 + 4
    i_small = 1 * 8 + 1
    assert op.dl[i_iso] == 0.0 and op.d[i_iso] == 1.0
    w = np.exp(-(g[1, 1] ** 2) / (2 * 0.1 ** 2))
    assert op.dl[i_small] == pytest.approx(4 * w * np.exp(-0.5), rel=1e-14)  # spatial factor, sigma_s = 1
    x = np.random.default_rng(4).standard_normal(op.n)
    assert op.apply_l(x)[i_iso] == 0.0
    assert op.apply_lsym(x)[i_iso] == 0.0
    assert op.apply_rw(x)[i_iso] == x[i_iso]
    y, info = oracle.cg_filter(op, g.ravel(), 10)
    assert y[i_iso] == g.ravel()[i_iso]
    _, Ls = dense_normalized(op)
    assert abs(Ls[i_small, i_small] - 1.0) <= 1e-14
    ev = np.linalg.eigvalsh(0.5 * (Ls + Ls.T))
    assert ev[0] > -1e-12 and ev[-1] < 2.0 + 1e-12


def test_diagl_power_filter_is_jacobi():
    """RW under the (diag L) normalization is one Jacobi sweep for L x = 0:
    x_i <- sum_{j != i} w_ij x_j / sum_{j != i} w_ij (the BF average without
    the centre pixel), checked by brute force."""
    g = _img(6, 7, 5)
    op = oracle.build_operator("bf", g, 2, 1.5, 0.2, stencil="square", norm="diagl")
    x = np.random.default_rng(2).standard_normal(op.n)
    gf = g.ravel()
    H, Wd = g.shape
    ref = np.empty(op.n)
    for i in range(op.n):
        yi, xi = divmod(i, Wd)
        num = den = 0.0
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                if (dy, dx) == (0, 0) or not (0 <= yi + dy < H and 0 <= xi + dx < Wd):
                    continue
                j = (yi + dy) * Wd + xi + dx
                w = np.exp(-(dy * dy + dx * dx) / (2 * 1.5 ** 2)) * np.exp(-(gf[i] - gf[j]) ** 2 / (2 * 0.2 ** 2))
                num += w * x[j]
                den += w
        ref[i] = num / den
    np.testing.assert_allclose(op.apply_rw(x), ref, rtol=0, atol=1e-13)


def test_reguided_variants_without_range_kernel_equal_linear():
    """sigma_r = inf: the cross / (diag L) graph no longer depends on the
    guidance, so the re-guided filters equal the linear ones on that graph."""
    g = _img(8, 9, 6)
    x = g.ravel()
    op = oracle.build_operator("bf", g, 1, 1.3, np.inf, stencil="cross", norm="diagl")
    kw = dict(radius=1, sigma_s=1.3, sigma_r=np.inf, stencil="cross", norm="diagl")
    lin = x.copy()
    for _ in range(4):
        lin = op.apply_rw(lin)
    np.testing.assert_allclose(oracle.power_filter_reguided("bf", x, g.shape, 4, **kw), lin, rtol=0, atol=1e-14)
    ylin, _ = oracle.cg_filter(op, x, 8)
    yrg, info = oracle.cg_filter_reguided("bf", x, g.shape, 8, **kw)
    assert info.iters == 8
    np.testing.assert_allclose(yrg, ylin, rtol=0, atol=1e-12)
