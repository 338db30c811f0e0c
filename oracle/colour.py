"""CIE-Lab coordinates of sRGB colours, for the colour guidance that Section 2
suggests for the BF's photometric distance (Tomasi and Manduchi measure it in
CIE-Lab).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions (written out from the standards, FP64):
  sRGB (IEC 61966-2-1): a component c in [0, 1] is linearised as c / 12.92 for
    c <= 0.04045, else ((c + 0.055) / 1.055)^2.4.  Linear RGB -> XYZ by the
    matrix whose columns are the XYZ of the three primaries, with
    chromaticities R (0.64, 0.33), G (0.30, 0.60), B (0.15, 0.06), scaled so
    that RGB = (1, 1, 1) gives the white point D65, chromaticity
    (0.3127, 0.3290), Y = 1.
  CIE 1976 L*a*b* relative to that white (X_n, Y_n, Z_n):
    f(t) = t^(1/3) for t > (6/29)^3, else t / (3 (6/29)^2) + 4/29;
    L* = 116 f(Y/Y_n) - 16, a* = 500 (f(X/X_n) - f(Y/Y_n)),
    b* = 200 (f(Y/Y_n) - f(Z/Z_n)).
Reading: the white point is the one the matrix is built for (so sRGB white
maps to L* = 100, a* = b* = 0 up to rounding); inputs outside [0, 1] are
converted by the same formulas (no clipping).
"""
from __future__ import annotations

import numpy as np


def _xyz_of_chromaticity(x: float, y: float) -> np.ndarray:
    """XYZ with Y = 1 of the chromaticity (x, y)."""
    return np.array([x / y, 1.0, (1.0 - x - y) / y])


def srgb_matrix() -> np.ndarray:
    """Linear sRGB -> XYZ (D65, Y of white = 1), from the primaries."""
    P = np.column_stack([_xyz_of_chromaticity(0.64, 0.33), _xyz_of_chromaticity(0.30, 0.60),
                         _xyz_of_chromaticity(0.15, 0.06)])
    white = _xyz_of_chromaticity(0.3127, 0.3290)
    scale = np.linalg.solve(P, white)  # luminance of each primary at full drive
    return P * scale[None, :]


def srgb_to_linear(c):
    c = np.asarray(c, dtype=np.float64)
    hi = np.maximum(c, 0.04045)  # the power branch only ever sees its own domain
    return np.where(c <= 0.04045, c / 12.92, ((hi + 0.055) / 1.055) ** 2.4)


def _f(t):
    d = 6.0 / 29.0
    return np.where(t > d ** 3, np.cbrt(t), t / (3.0 * d * d) + 4.0 / 29.0)


def srgb_to_lab(rgb):
    """CIE-Lab of sRGB values: rgb has a trailing axis of 3 components in
    [0, 1]; returns the same shape with (L*, a*, b*)."""
    rgb = np.asarray(rgb, dtype=np.float64)
    M = srgb_matrix()
    xyz = srgb_to_linear(rgb) @ M.T
    white = M @ np.ones(3)
    fx, fy, fz = (_f(xyz[..., k] / white[k]) for k in range(3))
    return np.stack([116.0 * fy - 16.0, 500.0 * (fx - fy), 200.0 * (fy - fz)], axis=-1)
