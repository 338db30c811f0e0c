"""Self-sensitivity band of the FP64 oracle: the bound of the FP64 parity
gates of the iterative filters (CG, LOBPCG, the re-guided and block filters).

TEST INFRASTRUCTURE ONLY: it calls nothing but `oracle/`.

An iterative filter amplifies rounding: two correct FP64 implementations
that sum the same terms in different orders agree only to some band that
grows with the step count and with the conditioning of each step (CG's
alpha and beta, the Rayleigh-Ritz factorisation of a nearly dependent
[X, W, P]).  The band of a case is measured on the oracle itself: the
filter run on the problem as given and on the same problem with the grid
points in reverse order (a 1D signal reversed, an image turned by 180
degrees, i.e. point i relabelled n - 1 - i).  The reversal is a pure
relabelling of the graph: the BF window, the truncation at the border, the
GF windows and their counts, the cross lattice and both normalizations are
symmetric under it, so every weight of eq. (2) is the same number (same
exponent argument) and only the order of every sum changes (degrees, sparse
row sums, dot products, Gram entries).  The LOBPCG start block of the
reversed problem is the relabelled one up to column signs (Legendre
polynomials have parity), which spans the same space.

The band is rel(y, flip(y_reversed)) in the 2-norm and max-norm sense of
the parity tests, and an FP64 GPU output is gated at max(1e-12, 10 band):
the kernels sum in yet another order, and ten times what the oracle's own
reordering moves is the margin.  `tests/golden/make_sensitivity_band.py`
writes the bands of the named configurations to
`tests/golden/sensitivity_band.json` (a record; the tests measure their own
cases when they run).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FLOOR = 1e-12
FACTOR = 10.0


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den2 = max(np.linalg.norm(b), 1e-300)
    deni = max(np.abs(b).max(), 1e-300)
    return max(np.linalg.norm(a - b) / den2, np.abs(a - b).max() / deni)


def flip_grid(g):
    """A grid-shaped array (1D signal or 2D image, optionally with a trailing
    channel axis of a colour guidance) with its points in reverse order."""
    g = np.asarray(g)
    return g[::-1] if g.ndim == 1 else g[::-1, ::-1]


def flip_points(v):
    """A flat vector (n) or point-major block (n x m) with its points in
    reverse order (row-major reversal of a 2D grid is the 180 degree turn)."""
    return np.asarray(v)[::-1]


def band(run, *grids) -> float:
    """rel(run(*grids), flip(run(*flipped grids))) for a filter `run` that
    maps grid-shaped inputs to a flat output (or point-major block)."""
    y = np.asarray(run(*grids), dtype=np.float64)
    yr = np.asarray(run(*[flip_grid(g) for g in grids]), dtype=np.float64)
    return rel(y, flip_points(yr))


@dataclass
class Reference:
    """The oracle's output y of a case (and `extra`, whatever else its
    forward run returned), the same of the reversed run (`extra_reversed`),
    the band and the FP64 gate max(1e-12, 10 band)."""
    y: np.ndarray
    extra: object
    extra_reversed: object
    band: float
    gate: float


def reference(run, *grids) -> Reference:
    """Runs `run` forward and reversed: run(*grids) returns (y, extra), y the
    output compared with the GPU (flat or point-major).  A decision that the
    oracle's own reversed run takes differently (a column drop of a
    Rayleigh-Ritz step on the rounding threshold) is not fixed by the method
    at FP64 and cannot be asked of the GPU either: compare `extra` with
    `extra_reversed` before asserting such a decision."""
    y, extra = run(*grids)
    yr, extra_r = run(*[flip_grid(g) for g in grids])
    b = rel(np.asarray(y, dtype=np.float64), flip_points(np.asarray(yr, dtype=np.float64)))
    return Reference(y=y, extra=extra, extra_reversed=extra_r, band=b, gate=max(FLOOR, FACTOR * b))

