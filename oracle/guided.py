"""Guided filter (paper Section 3): Algorithm 1 and its implicit matrix,
eqs. (5)-(6).

Readings:
  * rho in Algorithm 1 is the window *width*; a radius r means rho = 2r + 1
    and |omega| = (2r+1)^d.
  * f_mean averages over the window truncated at the border, i.e. divides by
    that window's own pixel count N_k.  eq. (6) writes a fixed 1/|omega|^2,
    which is the interior case (N_k = |omega|).  The matrix that reproduces
    Algorithm 1 with truncated windows is
        W_ij = (1/|omega|) sum_{k: i,j in omega_k} (1/N_k)
                 (1 + (g_i - mu_k)(g_j - mu_k) / (sigma_k^2 + eps)),
    equal to eq. (6) in the interior.  Its row sums are d_i = N_i / |omega|
    (N_i = number of windows containing i), so D^-1 W x is exactly
    Algorithm 1's output, and D = I in the interior as Section 3 states.
  * sigma_k^2 is the population variance of g over omega_k, as Algorithm 1
    computes it (corr_g - mean_g^2).
"""
from __future__ import annotations

import itertools

import numpy as np


def box_sum(v: np.ndarray, radius: int) -> np.ndarray:
    """Sum of v over the border-truncated square window of half-width radius
    centred at every pixel (separable: one 1D window sum per axis)."""
    out = np.asarray(v, dtype=np.float64)
    for axis in range(out.ndim):
        n = out.shape[axis]
        acc = np.zeros_like(out)
        for o in range(-radius, radius + 1):
            # acc[i] += out[i + o] for all i with 0 <= i + o < n
            lo, hi = max(0, -o), min(n, n - o)
            if hi <= lo:
                continue
            dst = [slice(None)] * out.ndim
            src = [slice(None)] * out.ndim
            dst[axis] = slice(lo, hi)
            src[axis] = slice(lo + o, hi + o)
            acc[tuple(dst)] += out[tuple(src)]
        out = acc
    return out


def box_count(shape, radius: int) -> np.ndarray:
    """N_k: number of grid pixels inside the truncated window of pixel k."""
    return box_sum(np.ones(shape), radius)


def f_mean(v: np.ndarray, radius: int) -> np.ndarray:
    """Mean filter f_mean(v, rho) of Algorithm 1, rho = 2*radius + 1."""
    return box_sum(v, radius) / box_count(np.shape(v), radius)


def guided_filter(x: np.ndarray, g: np.ndarray, radius: int, eps: float) -> np.ndarray:
    """Algorithm 1, step by step, with truncated-window means."""
    mean_g = f_mean(g, radius)
    mean_x = f_mean(x, radius)
    corr_g = f_mean(g * g, radius)
    corr_gx = f_mean(g * x, radius)
    var_g = corr_g - mean_g * mean_g
    cov_gx = corr_gx - mean_g * mean_x
    a = cov_gx / (var_g + eps)
    b = mean_x - a * mean_g
    mean_a = f_mean(a, radius)
    mean_b = f_mean(b, radius)
    return mean_a * g + mean_b


def gf_stats(g: np.ndarray, radius: int, eps: float):
    """Per-window statistics of the fixed guidance (Algorithm 1, the lines
    that depend on g only): mu_k = mean_g and 1/(var_g + eps)."""
    mean_g = f_mean(g, radius)
    var_g = f_mean(g * g, radius) - mean_g * mean_g
    return mean_g, 1.0 / (var_g + eps)


def gf_degrees(shape, radius: int) -> np.ndarray:
    """d_i = N_i / |omega| (closed form of the row sums of W, see above)."""
    ndim = len(shape)
    return box_count(shape, radius) / float((2 * radius + 1) ** ndim)


def gf_weight_matrix_dense(g: np.ndarray, radius: int, eps: float) -> np.ndarray:
    """Explicit dense W(g) of eq. (6) (truncated-window reading), built window
    by window: each window omega_k adds its rank-two-plus-constant block.
    O(n^2) memory: small grids only."""
    g = np.asarray(g, dtype=np.float64)
    shape = g.shape
    n = g.size
    ndim = len(shape)
    omega = float((2 * radius + 1) ** ndim)
    gflat = g.ravel()
    W = np.zeros((n, n))
    for k in itertools.product(*[range(s) for s in shape]):
        ranges = [range(max(0, kk - radius), min(s, kk + radius + 1)) for kk, s in zip(k, shape)]
        members = np.array([np.ravel_multi_index(p, shape) for p in itertools.product(*ranges)])
        nk = members.size
        gk = gflat[members]
        mu = gk.mean()
        var = np.mean((gk - mu) ** 2)
        dev = gk - mu
        W[np.ix_(members, members)] += (1.0 + np.outer(dev, dev) / (var + eps)) / nk
    return W / omega
