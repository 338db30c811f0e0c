"""Denoising quality measure used in Section 7 (PSNR of a filtered image
against the clean one).  Reading: peak value 1 (signals live in [0, 1]),
no clipping of the noisy input, MSE over all pixels."""
from __future__ import annotations

import numpy as np


def psnr(estimate, clean, peak: float = 1.0) -> float:
    """10 log10(peak^2 / MSE)."""
    e = np.asarray(estimate, dtype=np.float64).ravel() - np.asarray(clean, dtype=np.float64).ravel()
    mse = float(np.mean(e * e))
    return 10.0 * np.log10(peak * peak / mse)
