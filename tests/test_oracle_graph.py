"""Pins of the oracle's graph operators (BF eq. (2), GF Algorithm 1 / eq. (6),
the normalized forms of Section 4) against facts that do not come from the
oracle itself: library convolutions, closed forms, brute force and
invariants."""
import itertools

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from oracle.operator import FORM_LSYM, FORM_N, FORM_RW
from oracle.spectral import dense_normalized
from synth import piecewise_constant_1d, scene_2d


def _img(h=12, w=15, seed=0, sigma=0.05):
    return scene_2d(h, w, sigma, seed)[1]


# ---------------------------------------------------------------- BF weights
def test_bf_weights_symmetric_selfloop_range():
    g = _img()
    W = oracle.bf_weight_matrix(g, 2, 2.0, 0.1)
    assert (W != W.T).nnz == 0                      # exactly symmetric
    assert np.all(W.diagonal() == 1.0)              # w_ii = exp(0) exp(0)
    assert W.data.min() > 0.0 and W.data.max() <= 1.0


def test_bf_window_size_and_truncation():
    g = _img(9, 11)
    r = 2
    W = oracle.bf_weight_matrix(g, r, 2.0, 0.1).tocsr()
    nnz = np.diff(W.indptr).reshape(g.shape)
    # interior rows have the full (2r+1)^2 window, corners only (r+1)^2
    assert nnz[4, 5] == (2 * r + 1) ** 2
    assert nnz[0, 0] == (r + 1) ** 2
    assert nnz[0, 5] == (r + 1) * (2 * r + 1)


def test_bf_large_sigma_r_is_truncated_gaussian_convolution():
    """sigma_r -> inf removes the photometric factor: D^-1 W x becomes a
    Gaussian convolution normalised over the in-grid part of the window,
    which scipy.ndimage computes independently."""
    g = _img(13, 17, seed=3)
    x = _img(13, 17, seed=4)
    r, ss = 3, 1.7
    op = oracle.build_operator("bf", g, r, ss, np.inf)
    yy, xx = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1), indexing="ij")
    kern = np.exp(-(yy ** 2 + xx ** 2) / (2 * ss ** 2))
    num = ndi.correlate(x, kern, mode="constant", cval=0.0)
    den = ndi.correlate(np.ones_like(x), kern, mode="constant", cval=0.0)
    np.testing.assert_allclose(op.apply_rw(x.ravel()), (num / den).ravel(), rtol=1e-13, atol=1e-14)


def test_bf_tiny_sigma_r_on_distinct_values_is_identity():
    x = np.linspace(0.0, 1.0, 40) ** 1.3
    op = oracle.build_operator("bf", x, 4, 2.0, 1e-4)
    np.testing.assert_allclose(op.apply_rw(x), x, rtol=0, atol=1e-300)
    np.testing.assert_allclose(op.d, 1.0)


def test_bf_weight_direction_independent():
    """Reflecting the signal reflects the graph (isotropic window)."""
    g = _img(8, 10, seed=5)
    W = oracle.bf_weight_matrix(g, 2, 1.5, 0.2).toarray()
    Wf = oracle.bf_weight_matrix(g[::-1, ::-1], 2, 1.5, 0.2).toarray()
    perm = np.arange(g.size)[::-1]
    np.testing.assert_allclose(Wf, W[np.ix_(perm, perm)], rtol=0, atol=0)


def test_bf_single_edge_hand_value():
    """Two-sample signal, radius 1: w_01 = exp(-1/(2 ss^2)) exp(-(dx)^2/(2 sr^2))."""
    x = np.array([0.2, 0.5])
    W = oracle.bf_weight_matrix(x, 1, 2.0, 0.3).toarray()
    expected = np.exp(-1.0 / 8.0) * np.exp(-0.09 / 0.18)   # = exp(-0.625)
    assert abs(W[0, 1] - 0.5352614285189903) < 1e-15
    assert abs(expected - 0.5352614285189903) < 1e-15
    np.testing.assert_allclose(oracle.degrees(W), [1.5352614285189903] * 2, rtol=1e-15)


# ------------------------------------------------- normalized operator (BF)
@pytest.mark.parametrize("shape,r", [((60,), 5), ((9, 13), 2)])
def test_normalized_bf_invariants(shape, r):
    g = np.random.default_rng(1).uniform(size=shape)
    op = oracle.build_operator("bf", g, r, 2.0, 0.2)
    n = op.n
    ones = np.ones(n)
    np.testing.assert_allclose(op.apply_rw(ones), ones, rtol=0, atol=2e-15)   # rows of D^-1 W sum to 1
    np.testing.assert_allclose(op.apply_n(op.sqrt_d), op.sqrt_d, rtol=1e-14)  # N D^1/2 e = D^1/2 e
    np.testing.assert_allclose(op.apply_l(ones), 0.0, atol=1e-13)             # L e = 0
    N, Ls = dense_normalized(op)
    np.testing.assert_allclose(N, N.T, rtol=0, atol=1e-15)
    lam = np.linalg.eigvalsh(0.5 * (N + N.T))
    assert lam.min() >= -1 - 1e-12 and lam.max() <= 1 + 1e-12
    assert np.linalg.eigvalsh(0.5 * (Ls + Ls.T)).min() > -1e-12            # L_sym PSD
    # forms agree: RW = D^-1/2 N D^1/2, L_sym = I - N
    x = np.random.default_rng(2).standard_normal(n)
    np.testing.assert_allclose(op.apply(FORM_RW, x), op.apply(FORM_N, op.sqrt_d * x) / op.sqrt_d, rtol=1e-13)
    np.testing.assert_allclose(op.apply(FORM_LSYM, x), x - N @ x, rtol=1e-12, atol=1e-13)


def test_gershgorin_remark_spectral_range_only():
    """Section 2 ties smoothing to max d_i <= 2; for the normalized operator
    the spectrum of D^-1 W lies in [-1, 1] whatever the degrees are."""
    g = np.random.default_rng(3).uniform(size=(7, 7))
    op = oracle.build_operator("bf", g, 3, 5.0, 1.0)
    assert op.d.max() > 2.0
    N, _ = dense_normalized(op)
    lam = np.linalg.eigvalsh(0.5 * (N + N.T))
    assert lam.max() <= 1 + 1e-12 and lam.min() >= -1 - 1e-12


# ---------------------------------------------------------------- GF
def _box_brute(v, r):
    out = np.zeros_like(v)
    for idx in itertools.product(*[range(s) for s in v.shape]):
        sl = tuple(slice(max(0, i - r), min(s, i + r + 1)) for i, s in zip(idx, v.shape))
        out[idx] = v[sl].sum()
    return out


@pytest.mark.parametrize("shape,r", [((17,), 3), ((6, 9), 2), ((5, 4), 4)])
def test_box_sum_matches_brute_force(shape, r):
    v = np.random.default_rng(4).standard_normal(shape)
    np.testing.assert_allclose(oracle.box_sum(v, r), _box_brute(v, r), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("shape,r,eps", [((23,), 2, 1e-2), ((7, 8), 1, 1e-2), ((6, 7), 2, 1e-3)])
def test_gf_algorithm1_equals_eq6_matrix(shape, r, eps):
    """Two independent formulas for the same operator: Algorithm 1 applied to
    x equals D^-1 W x with W built window by window as in eq. (6)."""
    g = np.random.default_rng(5).uniform(size=shape)
    x = np.random.default_rng(6).standard_normal(shape)
    W = oracle.gf_weight_matrix_dense(g, r, eps)
    d = W.sum(axis=1)
    np.testing.assert_allclose(d, oracle.gf_degrees(shape, r).ravel(), rtol=1e-13)
    np.testing.assert_allclose(W, W.T, rtol=0, atol=1e-15)
    y = oracle.guided_filter(x, g, r, eps).ravel()
    np.testing.assert_allclose(y, (W @ x.ravel()) / d, rtol=1e-12, atol=1e-13)
    op = oracle.build_operator("gf", g, r, eps=eps)
    np.testing.assert_allclose(op.apply_w(x.ravel()), W @ x.ravel(), rtol=1e-12, atol=1e-13)
    # interior entries match eq. (6) with the fixed 1/|omega|^2
    N = W / np.sqrt(np.outer(d, d))
    lam = np.linalg.eigvalsh(0.5 * (N + N.T))
    assert lam.min() > -1e-12 and lam.max() < 1 + 1e-12   # 0 <= W <= D (Loewner)


def test_gf_has_negative_entries():
    g = np.random.default_rng(7).uniform(size=(6, 6))
    W = oracle.gf_weight_matrix_dense(g, 1, 1e-3)
    assert W.min() < 0.0


def test_gf_large_eps_is_double_box_filter():
    """eps -> inf sends a to 0 and b to mean_x: y = mean(mean(x)), a double
    truncated box filter, computed here with scipy.ndimage."""
    g = np.random.default_rng(8).uniform(size=(11, 14))
    x = np.random.default_rng(9).standard_normal((11, 14))
    r = 2
    kern = np.ones((2 * r + 1, 2 * r + 1))
    cnt = ndi.correlate(np.ones_like(x), kern, mode="constant")
    box = lambda v: ndi.correlate(v, kern, mode="constant") / cnt
    np.testing.assert_allclose(oracle.guided_filter(x, g, r, 1e12), box(box(x)), rtol=1e-9, atol=1e-10)


def test_gf_zero_eps_reproduces_affine_functions_of_guidance():
    g = np.random.default_rng(10).uniform(size=(9, 12))
    x = 0.7 * g - 0.2
    np.testing.assert_allclose(oracle.guided_filter(x, g, 2, 0.0), x, rtol=0, atol=1e-12)


def test_gf_normalized_forms():
    g = np.random.default_rng(11).uniform(size=(8, 9))
    op = oracle.build_operator("gf", g, 2, eps=1e-2)
    ones = np.ones(op.n)
    np.testing.assert_allclose(op.apply_rw(ones), ones, atol=1e-13)
    np.testing.assert_allclose(op.apply_n(op.sqrt_d), op.sqrt_d, rtol=1e-12)
    N, _ = dense_normalized(op)
    np.testing.assert_allclose(N, N.T, atol=1e-14)


def test_gf_stats_against_brute_force():
    g = np.random.default_rng(12).uniform(size=(7, 6))
    r, eps = 2, 1e-2
    mu, inv = oracle.gf_stats(g, r, eps)
    for (i, j) in [(0, 0), (3, 2), (6, 5), (2, 5)]:
        win = g[max(0, i - r):i + r + 1, max(0, j - r):j + r + 1]
        assert abs(mu[i, j] - win.mean()) < 1e-14
        assert abs(inv[i, j] - 1.0 / (win.var() + eps)) < 1e-10


# ---------------------------------------------------------------- generators / PSNR
def test_noisy_psnr_closed_form():
    """PSNR of the noisy input is -20 log10 sigma (peak 1), e.g. 20.0 dB for
    the noise variance 0.01 of Section 7's image experiment (printed there as
    20.1, see tests/golden/paper_values.json)."""
    import json, os
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    for sigma in (0.1, 0.05, 0.08):
        clean, noisy = scene_2d(1024, 1024, sigma, 2)
        assert abs(oracle.psnr(noisy, clean) - (-20 * np.log10(sigma))) < 0.02
    clean, noisy = scene_2d(1024, 1024, np.sqrt(golden["noise_variance"]), 2)
    assert abs(oracle.psnr(noisy, clean) - golden["noisy_psnr_db"]) < 0.15


def test_generator_structure():
    clean, noisy = piecewise_constant_1d(4096, 0.1, 1)
    assert np.unique(clean).size == 9
    assert np.count_nonzero(np.diff(clean)) == 8
    assert clean.min() >= 0 and clean.max() <= 1
    c1, _ = scene_2d(64, 64, 0.05, 7)
    c2, _ = scene_2d(64, 64, 0.05, 7)
    assert np.array_equal(c1, c2)


# ------------------------------------------------------------------ pointwise forms
@pytest.mark.parametrize("shape", [(9, 11), (40,), (6, 5)])
def test_pointwise_bf_lsym_matches_full_operator(shape):
    """The point-by-point L_sym of eq. (2) equals the sparse-matrix oracle at
    every point, borders and corners included."""
    from oracle.pointwise import bf_lsym_at
    from synth import piecewise_constant_1d
    g = scene_2d(shape[0], shape[1], 0.05, 31)[1] if len(shape) == 2 else piecewise_constant_1d(shape[0], 0.1, 31)[1]
    op = oracle.build_operator("bf", g, 2, 2.0, 0.15)
    z = np.random.default_rng(32).standard_normal(op.n)
    ref = op.apply_lsym(z)
    got = bf_lsym_at(g, z, np.arange(op.n), 2, 2.0, 0.15)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("shape", [(9, 10), (30,)])
def test_pointwise_gf_lsym_matches_full_operator(shape):
    """The point-by-point L_sym of Algorithm 1 equals the oracle's operator."""
    from oracle.pointwise import gf_lsym_at
    from synth import piecewise_constant_1d
    g = scene_2d(shape[0], shape[1], 0.05, 33)[1] if len(shape) == 2 else piecewise_constant_1d(shape[0], 0.1, 33)[1]
    op = oracle.build_operator("gf", g, 2, eps=1e-2)
    z = np.random.default_rng(34).standard_normal(op.n)
    ref = op.apply_lsym(z)
    got = gf_lsym_at(g, z, np.arange(op.n), 2, 1e-2)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-12)


def test_sample_points_cover_corners():
    from oracle.pointwise import sample_points
    pts = sample_points((50, 70), 40, 1)
    for c in (0, 69, 49 * 70, 50 * 70 - 1):
        assert c in pts
    assert len(set(pts.tolist())) == len(pts) and pts.max() < 3500
