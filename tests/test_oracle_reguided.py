"""Pins of the re-guided (non-linear) filters of the oracle: against the
linear filters where they must agree (the first step, guidance-independent
weights), fixed points and the conserved D-weighted sum of the GF."""
import numpy as np
import pytest

import oracle
from synth import piecewise_constant_1d, scene_2d


def _sig1d(n=60, seed=11):
    _, x = piecewise_constant_1d(n, 0.1, seed)
    return x, (n,)


def _sig2d(h=9, w=10, seed=12):
    _, x = scene_2d(h, w, 0.05, seed)
    return x.ravel(), (h, w)


CASES = [
    ("bf", _sig1d, dict(radius=3, sigma_s=3.0, sigma_r=0.2)),
    ("bf", _sig2d, dict(radius=2, sigma_s=2.0, sigma_r=0.15)),
    ("gf", _sig1d, dict(radius=3, eps=1e-2)),
    ("gf", _sig2d, dict(radius=2, eps=1e-2)),
]


@pytest.mark.parametrize("kind,sig,par", CASES)
def test_zero_steps_identity(kind, sig, par):
    x, shape = sig()
    assert np.array_equal(oracle.power_filter_reguided(kind, x, shape, 0, **par), x)
    y, info = oracle.cg_filter_reguided(kind, x, shape, 0, **par)
    assert np.array_equal(y, x) and info.iters == 0


@pytest.mark.parametrize("kind,sig,par", CASES)
def test_first_step_is_the_linear_step(kind, sig, par):
    """Step 1 uses the graph of x0 itself: one step of the linear filters."""
    x, shape = sig()
    op = oracle.build_operator(kind, x.reshape(shape), par["radius"], par.get("sigma_s", 0.0),
                               par.get("sigma_r", 0.0), par.get("eps", 0.0))
    np.testing.assert_allclose(oracle.power_filter_reguided(kind, x, shape, 1, **par), op.apply_rw(x),
                               rtol=0, atol=1e-15)
    y, info = oracle.cg_filter_reguided(kind, x, shape, 1, **par)
    yl, il = oracle.cg_filter(op, x, 1)
    np.testing.assert_allclose(y, yl, rtol=0, atol=1e-14)
    assert info.iters == il.iters == 1


@pytest.mark.parametrize("sig", [_sig1d, _sig2d])
def test_bf_without_range_kernel_equals_linear(sig):
    """sigma_r = inf: the BF weights do not depend on the guidance, so the
    re-guided filters equal the linear ones at every step."""
    x, shape = sig()
    par = dict(radius=2, sigma_s=2.0, sigma_r=np.inf)
    op = oracle.build_operator("bf", x.reshape(shape), 2, 2.0, np.inf)
    np.testing.assert_allclose(oracle.power_filter_reguided("bf", x, shape, 6, **par),
                               oracle.power_filter(op, x, 6), rtol=0, atol=1e-13)
    y, info = oracle.cg_filter_reguided("bf", x, shape, 6, **par)
    yl, il = oracle.cg_filter(op, x, 6)
    np.testing.assert_allclose(y, yl, rtol=0, atol=1e-12)
    assert info.iters == il.iters == 6


@pytest.mark.parametrize("sig", [_sig1d, _sig2d])
def test_gf_with_huge_eps_equals_linear(sig):
    """eps -> inf: a_k -> 0 and the GF becomes the guidance-independent box
    filter, so re-guiding changes nothing (up to O(1/eps))."""
    x, shape = sig()
    par = dict(radius=2, eps=1e12)
    op = oracle.build_operator("gf", x.reshape(shape), 2, eps=1e12)
    np.testing.assert_allclose(oracle.power_filter_reguided("gf", x, shape, 5, **par),
                               oracle.power_filter(op, x, 5), rtol=0, atol=1e-9)
    y, _ = oracle.cg_filter_reguided("gf", x, shape, 5, **par)
    yl, _ = oracle.cg_filter(op, x, 5)
    np.testing.assert_allclose(y, yl, rtol=0, atol=1e-9)


@pytest.mark.parametrize("kind,sig,par", CASES)
def test_constant_signal_is_fixed(kind, sig, par):
    """W 1 = D 1 for every guidance: a constant is a fixed point of the power
    filter, and CG stops at once (r0 = -L 1 c = 0) with x unchanged."""
    x, shape = sig()
    c = np.full_like(x, 0.37)
    np.testing.assert_allclose(oracle.power_filter_reguided(kind, c, shape, 4, **par), c, rtol=0, atol=1e-15)
    y, info = oracle.cg_filter_reguided(kind, c, shape, 4, **par)
    assert info.status == "breakdown" and np.array_equal(y, c)


@pytest.mark.parametrize("sig", [_sig1d, _sig2d])
def test_gf_conserves_degree_weighted_sum(sig):
    """GF degrees N_i/|w| do not depend on the guidance, so 1^T D x is kept
    by every power step (1^T D D^-1 W x = (W 1)^T x) and by CG (1^T L = 0 for
    every L_k, so 1^T r stays 0 and so does 1^T D p)."""
    x, shape = sig()
    d = oracle.build_operator("gf", x.reshape(shape), 2, eps=1e-2).d
    m0 = float(d @ x)
    y = oracle.power_filter_reguided("gf", x, shape, 6, radius=2, eps=1e-2)
    assert abs(float(d @ y) - m0) <= 1e-12 * abs(m0)
    y, info = oracle.cg_filter_reguided("gf", x, shape, 6, radius=2, eps=1e-2)
    assert info.iters == 6 and abs(float(d @ y) - m0) <= 1e-12 * abs(m0)


@pytest.mark.parametrize("sig", [_sig1d, _sig2d])
def test_bf_power_step_conserves_its_own_degree_sum(sig):
    """One BF pass with the graph of x_k keeps 1^T D(x_k) x."""
    x, shape = sig()
    y = oracle.power_filter_reguided("bf", x, shape, 2, radius=2, sigma_s=2.0, sigma_r=0.15)
    x1 = oracle.power_filter_reguided("bf", x, shape, 1, radius=2, sigma_s=2.0, sigma_r=0.15)
    d1 = oracle.build_operator("bf", x1.reshape(shape), 2, 2.0, 0.15).d
    assert abs(float(d1 @ y) - float(d1 @ x1)) <= 1e-12 * abs(float(d1 @ x1))


@pytest.mark.parametrize("kind,sig,par", CASES)
def test_reguidance_changes_the_filter(kind, sig, par):
    """With guidance-dependent weights, later steps differ from the linear
    filter's (the graph really is rebuilt)."""
    x, shape = sig()
    op = oracle.build_operator(kind, x.reshape(shape), par["radius"], par.get("sigma_s", 0.0),
                               par.get("sigma_r", 0.0), par.get("eps", 0.0))
    a = oracle.power_filter_reguided(kind, x, shape, 4, **par)
    b = oracle.power_filter(op, x, 4)
    assert np.linalg.norm(a - b) > 1e-6 * np.linalg.norm(b)
    y, _ = oracle.cg_filter_reguided(kind, x, shape, 4, **par)
    yl, _ = oracle.cg_filter(op, x, 4)
    assert np.linalg.norm(y - yl) > 1e-6 * np.linalg.norm(yl)


# ---------------------------------------------------------------------------
# step 2 on a graph that changes, carried out by hand
# ---------------------------------------------------------------------------
def _bf_dense(g, shape, r, sd, sr):
    """Eq. (2) written out point by point over the square window of radius
    r (self-loop included, truncated at the border): an independent dense W."""
    import itertools
    import math
    g = np.asarray(g, dtype=np.float64).ravel()
    pts = list(itertools.product(*[range(s) for s in shape]))
    n = len(pts)
    W = np.zeros((n, n))
    for i, pi in enumerate(pts):
        for j, pj in enumerate(pts):
            if max(abs(a - b) for a, b in zip(pi, pj)) <= r:
                dist2 = sum((a - b) ** 2 for a, b in zip(pi, pj))
                W[i, j] = math.exp(-dist2 / (2.0 * sd * sd) - (g[i] - g[j]) ** 2 / (2.0 * sr * sr))
    return W


def _two_steps_by_hand(x0, shape, r, sd, sr, mistake=None):
    """Algorithm 2, steps 1 and 2, with L_k = D_k - W_k and D_k built from the
    current iterate x_k before step k (the reading of the re-guided CG).
    `mistake` plants a plausible misreading, for the checks that the pin
    tells them apart:
      "stale": step 2 keeps the graph of x_0 (the iterate before the last
               update), i.e. the linear filter;
      "recompute_r": step 2 takes r_1 = -L_1 x_1 instead of the updated r;
      "new_d_old_s": the beta denominator uses s_old = D_1^-1 r_old."""
    def graph(x):
        W = _bf_dense(x, shape, r, sd, sr)
        d = W.sum(axis=1)
        return np.diag(d) - W, d

    L0, d0 = graph(x0)
    r0 = -L0 @ x0
    s0 = r0 / d0
    p0 = s0
    q0 = L0 @ p0
    a0 = (s0 @ r0) / (p0 @ q0)
    x1 = x0 + a0 * p0
    r1 = r0 - a0 * q0
    L1, d1 = graph(x0 if mistake == "stale" else x1)
    if mistake == "recompute_r":
        r1 = -L1 @ x1
    s1 = r1 / d1
    s_old = r0 / d1 if mistake == "new_d_old_s" else s0
    beta = (s1 @ (r1 - r0)) / (s_old @ r0)
    p1 = s1 + beta * p0
    q1 = L1 @ p1
    a1 = (s1 @ r1) / (p1 @ q1)
    return x1 + a1 * p1


@pytest.mark.parametrize("x0,shape,r,sd,sr", [
    (np.array([0.10, 0.18, 0.85, 0.80, 0.95, 0.22, 0.15]), (7,), 2, 1.5, 0.3),
    (np.array([0.10, 0.20, 0.90, 0.15, 0.80, 0.85, 0.30, 0.25, 0.95]), (3, 3), 1, 1.0, 0.35),
])
def test_bf_cg_step_two_by_hand(x0, shape, r, sd, sr):
    """Step 2 of the re-guided BF CG on a graph that changes (the weights of
    eq. (2) written out densely from x_1, Algorithm 2's recursion carried out
    by hand): the oracle agrees to rounding, and each planted misreading
    (the graph of x_0 at step 2, r recomputed from L_1, the beta denominator
    with D_1) lands far outside that."""
    expect = _two_steps_by_hand(x0, shape, r, sd, sr)
    y, info = oracle.cg_filter_reguided("bf", x0, shape, 2, radius=r, sigma_s=sd, sigma_r=sr)
    assert info.iters == 2
    np.testing.assert_allclose(y, expect, rtol=0, atol=1e-13)
    for mistake in ("stale", "recompute_r", "new_d_old_s"):
        wrong = _two_steps_by_hand(x0, shape, r, sd, sr, mistake)
        assert np.abs(wrong - expect).max() > 1e-4, mistake
