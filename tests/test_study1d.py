"""The 1D study's input (Section 6: piecewise linear with steep ascents and
descents, plus 0.1 randn noise): structure of the seeded generator."""
import numpy as np

from synth import STUDY_1D, piecewise_linear_1d, study_signal


def test_piecewise_linear_structure():
    for n in STUDY_1D["sizes"]:
        clean, noisy = study_signal(n)
        assert clean.shape == noisy.shape == (n,)
        d2 = np.abs(np.diff(clean, 2))
        kinks = np.flatnonzero(d2 > 1e-12)
        # 6 ramps, each bounded by two kinks, each kink touching <= 2 second differences
        assert 6 <= kinks.size <= 24
        steps = np.abs(np.diff(clean))
        assert np.sort(steps)[-6:].min() >= 0.3 / 6 - 1e-12   # a ramp moves >= 0.3 over <= 6 samples
        assert abs(np.std(noisy - clean) - 0.1) <= 0.01


def test_deterministic_and_seeded():
    a = piecewise_linear_1d(500, 0.1, 3)
    b = piecewise_linear_1d(500, 0.1, 3)
    c = piecewise_linear_1d(500, 0.1, 4)
    assert np.array_equal(a[1], b[1]) and not np.array_equal(a[0], c[0])
