"""Pins of the colour guidance (Section 2: the BF's photometric distance
measured in CIE-Lab for colour images): the sRGB -> CIE-Lab conversion
against published values, and the multi-channel BF weights of eq. (2)."""
import numpy as np
import pytest

import oracle
from oracle.colour import srgb_matrix, srgb_to_lab


def test_srgb_matrix_matches_the_standard():
    """IEC 61966-2-1 prints the linear sRGB -> XYZ matrix to 4 digits."""
    printed = np.array([[0.4124, 0.3576, 0.1805],
                        [0.2126, 0.7152, 0.0722],
                        [0.0193, 0.1192, 0.9505]])
    assert np.abs(srgb_matrix() - printed).max() <= 5e-5 + 1e-12


@pytest.mark.parametrize("rgb,lab", [
    ((1.0, 0.0, 0.0), (53.2408, 80.0925, 67.2032)),     # published sRGB primaries in CIE-Lab (D65)
    ((0.0, 1.0, 0.0), (87.7347, -86.1827, 83.1793)),
    ((0.0, 0.0, 1.0), (32.2970, 79.1875, -107.8602)),
    ((1.0, 1.0, 1.0), (100.0, 0.0, 0.0)),
    ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
])
def test_published_lab_values(rgb, lab):
    """Published tables differ in the 3rd decimal by the white point they
    tabulate D65 with; 0.01 covers that."""
    np.testing.assert_allclose(srgb_to_lab(np.array(rgb)), lab, atol=0.01)


def test_neutral_axis_and_dark_segment():
    """Greys have a* = b* = 0; below (6/29)^3 the CIE formula is linear,
    L* = (29/3)^3 Y = 903.3 Y."""
    g = np.linspace(0.0, 1.0, 11)
    lab = srgb_to_lab(np.stack([g, g, g], axis=1))
    assert np.abs(lab[:, 1:]).max() <= 1e-12
    assert np.all(np.diff(lab[:, 0]) > 0)
    y = 0.002 / 12.92  # sRGB 0.002 is on the linear part of the transfer curve too
    assert srgb_to_lab(np.array([0.002, 0.002, 0.002]))[0] == pytest.approx(903.2963 * y, rel=1e-5)


def _colour_image(h, w, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(h, w, 3))


def test_multichannel_weights_brute_force():
    """w_ij with |g_i - g_j| the Euclidean distance of the channel vectors."""
    g = srgb_to_lab(_colour_image(7, 9, 1))
    W = oracle.bf_weight_matrix(g, 2, 1.5, 20.0, channels=3).tocsr()
    H, Wd = g.shape[:2]
    rng = np.random.default_rng(2)
    for i in rng.choice(H * Wd, 12, replace=False):
        yi, xi = divmod(int(i), Wd)
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                yj, xj = yi + dy, xi + dx
                if not (0 <= yj < H and 0 <= xj < Wd):
                    continue
                d2 = float(np.sum((g[yi, xi] - g[yj, xj]) ** 2))
                w = np.exp(-(dy * dy + dx * dx) / (2 * 1.5 ** 2)) * np.exp(-d2 / (2 * 20.0 ** 2))
                assert W[i, yj * Wd + xj] == pytest.approx(w, rel=1e-14)


def test_multichannel_reduces_to_scalar():
    """Three equal channels g: the distance is sqrt(3) |g_i - g_j|, so the
    weights equal the scalar BF's with sigma_r / sqrt(3); one channel is the
    scalar BF; the channel order does not matter."""
    rng = np.random.default_rng(3)
    g = rng.uniform(0, 1, size=(8, 10))
    g3 = np.stack([g, g, g], axis=-1)
    a = oracle.bf_weight_matrix(g3, 2, 2.0, 0.3, channels=3)
    b = oracle.bf_weight_matrix(g, 2, 2.0, 0.3 / np.sqrt(3.0))
    assert abs(a - b).max() <= 1e-15
    c = oracle.bf_weight_matrix(g[..., None], 2, 2.0, 0.3)
    assert abs(c - oracle.bf_weight_matrix(g, 2, 2.0, 0.3)).max() == 0.0
    lab = srgb_to_lab(_colour_image(6, 8, 4))
    p = oracle.bf_weight_matrix(lab[..., [2, 0, 1]], 1, 1.0, 15.0, channels=3)
    q = oracle.bf_weight_matrix(lab, 1, 1.0, 15.0, channels=3)
    assert abs(p - q).max() <= 1e-15


def test_colour_operator_filters_channels_independently():
    """One graph (from the Lab guidance) for all channels: filtering an
    n x 3 block equals filtering each channel; the block CG oracle is the
    per-column CG."""
    rgb = _colour_image(9, 11, 5)
    op = oracle.build_operator("bf", srgb_to_lab(rgb), 2, 2.0, 20.0, channels=3)
    assert op.shape == (9, 11)
    X = rgb.reshape(-1, 3)
    Y = op.apply_rw(X)
    for c in range(3):
        np.testing.assert_allclose(Y[:, c], op.apply_rw(X[:, c]), rtol=0, atol=1e-15)
    Yb, infos = oracle.cg_filter_block(op, X, 10)
    for c in range(3):
        yc, ic = oracle.cg_filter(op, X[:, c], 10)
        np.testing.assert_array_equal(Yb[:, c], yc)
        assert infos[c].iters == ic.iters


def test_pointwise_multichannel_matches_matrix():
    from oracle.pointwise import bf_lsym_at
    from oracle.spectral import dense_normalized
    lab = srgb_to_lab(_colour_image(8, 9, 6))
    op = oracle.build_operator("bf", lab, 2, 2.0, 20.0, channels=3)
    z = np.random.default_rng(7).standard_normal((op.n, 2))
    _, Ls = dense_normalized(op)
    pts = [0, 5, 40, 71]
    np.testing.assert_allclose(bf_lsym_at(lab, z, pts, 2, 2.0, 20.0, channels=3), (Ls @ z)[pts], rtol=0,
                               atol=1e-13)
