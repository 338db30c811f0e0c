"""Bilateral-filter graph (paper Section 2).

Readings (the paper leaves these open):
  * Window: a square (Chebyshev) window |o|_inf <= r around each pixel, so a
    K = (2r+1)^d point neighbourhood; the spatial term of eq. (2) uses the
    Euclidean distance ||o||^2 in pixel units.  The image experiment of
    Section 7 uses the 5-point stencil instead: the cross of radius 1.
  * Self-loop: eq. (1) sums over all j including j = i, and eq. (3) must
    reproduce that average, so w_ii = exp(0) * exp(0) = 1 belongs to W and D.
  * Boundary: windows are truncated at the border (no padding), which keeps
    W exactly symmetric; d_i sums only in-grid neighbours.
  * Guidance: the weights use a guidance signal g (the noisy input itself in
    the self-guided case), computed once (the linear filter of Section 2).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def window_offsets(ndim: int, radius: int, stencil: str = "square"):
    """All offsets o of the neighbourhood, including o = 0: the square window
    |o|_inf <= radius, or the cross (the offsets along one axis, |o_k| <=
    radius; radius 1 in 2D is the 5-point stencil of the image experiment of
    Section 7).  In 1D both are the same interval."""
    rng = range(-radius, radius + 1)
    if stencil == "square" or ndim == 1:
        return [np.array(o, dtype=np.int64) for o in itertools.product(rng, repeat=ndim)]
    if stencil != "cross":
        raise ValueError(stencil)
    offs = [np.zeros(ndim, dtype=np.int64)]
    for axis in range(ndim):
        for k in rng:
            if k != 0:
                o = np.zeros(ndim, dtype=np.int64)
                o[axis] = k
                offs.append(o)
    return offs


def bf_weight_matrix(g: np.ndarray, radius: int, sigma_s: float, sigma_r: float,
                     stencil: str = "square", channels: int = 1) -> sp.csr_matrix:
    """Adjacency W of the BF graph, eq. (2):

        w_ij = exp(-||p_i - p_j||^2 / (2 sigma_s^2)) * exp(-|g_i - g_j|^2 / (2 sigma_r^2))

    for every j in the (border-truncated) neighbourhood of i (`stencil`, see
    `window_offsets`), w_ii = 1 included.  Pixels are numbered row-major; p_i
    are integer grid coordinates.  sigma_s = inf or sigma_r = inf switch the
    corresponding factor to 1.  channels > 1: g has a trailing axis of that
    length (a colour guidance, e.g. CIE-Lab as Section 2 suggests for colour
    images) and |g_i - g_j| is the Euclidean distance of the channel vectors.
    """
    g = np.asarray(g, dtype=np.float64)
    if channels > 1:
        if g.shape[-1] != channels:
            raise ValueError("guidance must end with an axis of `channels` values")
        shape = g.shape[:-1]
        gf = g.reshape(-1, channels)
    else:
        shape = g.shape
        gf = g.reshape(-1, 1)
    n = gf.shape[0]
    coords = np.indices(shape).reshape(len(shape), -1).T  # (n, ndim) grid positions p_i
    rows, cols, vals = [], [], []
    for o in window_offsets(len(shape), radius, stencil):
        nb = coords + o
        inside = np.all((nb >= 0) & (nb < np.array(shape)), axis=1)
        i = np.flatnonzero(inside)
        j = np.ravel_multi_index(tuple(nb[inside].T), shape)
        dist2 = float(np.dot(o, o))
        spatial = np.exp(-dist2 / (2.0 * sigma_s ** 2)) if np.isfinite(sigma_s) else 1.0
        if np.isfinite(sigma_r):
            photometric = np.exp(-np.sum((gf[i] - gf[j]) ** 2, axis=1) / (2.0 * sigma_r ** 2))
        else:
            photometric = np.ones(i.size)
        rows.append(i)
        cols.append(j)
        vals.append(spatial * photometric)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def degrees(W) -> np.ndarray:
    """d_i = sum_j w_ij (Section 2, the diagonal of D)."""
    return np.asarray(W.sum(axis=1)).ravel()
