"""Pins of the oracle's self-sensitivity band (tests/sensitivity.py): the
reversal it uses is a pure relabelling of the graph, so the band measures
summation order and nothing else, and it does notice a run that is not."""
import numpy as np
import pytest

import oracle
from sensitivity import band, flip_grid, flip_points, reference, rel
from synth import piecewise_constant_1d, scene_2d


def _perm(n):
    return np.arange(n)[::-1]


@pytest.mark.parametrize("shape,r,stencil", [((40,), 4, "square"), ((9, 13), 2, "square"), ((9, 13), 3, "cross")])
def test_reversed_bf_graph_is_the_relabelled_graph_bitwise(shape, r, stencil):
    """W of the reversed guidance equals P W P^T entry for entry (every
    weight of eq. (2) has the same exponent argument), including the border
    truncation."""
    g = (piecewise_constant_1d(shape[0], 0.1, 3)[1] if len(shape) == 1
         else scene_2d(shape[0], shape[1], 0.05, 3)[1])
    W = oracle.bf_weight_matrix(g, r, 2.0, 0.15, stencil).toarray()
    Wr = oracle.bf_weight_matrix(flip_grid(g), r, 2.0, 0.15, stencil).toarray()
    p = _perm(W.shape[0])
    assert np.array_equal(Wr, W[np.ix_(p, p)])


def test_reversed_gf_operator_is_the_relabelled_operator():
    """The GF's windows and counts are symmetric under the reversal: its
    apply on the reversed grid is the reversed apply to rounding."""
    g = scene_2d(11, 14, 0.05, 4)[1]
    op = oracle.build_operator("gf", g, 3, eps=1e-2)
    opr = oracle.build_operator("gf", flip_grid(g), 3, eps=1e-2)
    x = np.random.default_rng(5).standard_normal(op.n)
    assert np.array_equal(opr.d, flip_points(op.d))
    assert rel(flip_points(opr.apply_n(flip_points(x))), op.apply_n(x)) <= 1e-14


@pytest.mark.parametrize("shape,m", [((50,), 3), ((8, 12), 4)])
def test_reversed_start_block_spans_the_relabelled_start(shape, m):
    """Legendre polynomials have parity: the start block of the reversed
    problem is the relabelled start block with column signs (-1)^degree."""
    z0 = np.random.default_rng(6).standard_normal(int(np.prod(shape)))
    X = oracle.modulated_start(shape, z0, m)
    Xr = oracle.modulated_start(shape, flip_points(z0), m)
    signs = np.array([(-1.0) ** sum(d) for d in oracle.modulation_degrees(len(shape), m)])
    np.testing.assert_allclose(flip_points(Xr), X * signs[None, :], rtol=0, atol=1e-15)


def test_band_of_filters_is_at_rounding_level():
    """Power, CG and LOBPCG bands of a small FP64 case sit near the rounding
    unit and above zero for the iterations (their sums really are
    reordered)."""
    g = piecewise_constant_1d(600, 0.1, 7)[1]

    def power(x):
        return oracle.power_filter(oracle.build_operator("bf", x, 4, 3.0, 0.2), x, 20)

    def cg(x):
        return oracle.cg_filter(oracle.build_operator("bf", x, 4, 3.0, 0.2), x, 20)[0]

    def lob(x):
        return oracle.lobpcg_filter(oracle.build_operator("bf", x, 4, 3.0, 0.2), x, 3, 20)[0]

    bp, bc, bl = band(power, g), band(cg, g), band(lob, g)
    assert bp <= 1e-14
    assert 0.0 < bc <= 1e-12 and 0.0 < bl <= 1e-11


def test_band_notices_a_run_that_is_not_a_relabelling():
    """A run that reverses the signal but keeps the guidance of the original
    order (a mistake the reversal would have to expose) has a band of order
    one."""
    g = piecewise_constant_1d(300, 0.1, 8)[1]
    op = oracle.build_operator("bf", g, 3, 3.0, 0.2)

    def cg_fixed_graph(x):
        return oracle.cg_filter(op, x, 10)[0]

    assert band(cg_fixed_graph, g) > 1e-2


def test_reference_and_gate_floor():
    g = piecewise_constant_1d(200, 0.1, 9)[1]

    def cg(x):
        return oracle.cg_filter(oracle.build_operator("bf", x, 2, 3.0, 0.2), x, 5)

    ref = reference(cg, g)
    assert ref.extra.iters == ref.extra_reversed.iters == 5 and ref.gate == max(1e-12, 10.0 * ref.band)
    np.testing.assert_array_equal(ref.y, oracle.cg_filter(oracle.build_operator("bf", g, 2, 3.0, 0.2), g, 5)[0])
