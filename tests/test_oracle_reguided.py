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
