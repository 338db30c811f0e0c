"""The normalized operators at single grid points, from their definitions,
for checking large grids on a sample of points (the full matrices of
`graph` and `guided` do not fit at 1024^2 and above).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  BF (eq. (2), Section 4): (L_sym z)_i = z_i - d_i^-1/2 sum_j w_ij d_j^-1/2 z_j
      with w_ij of eq. (2) over the border-truncated window (w_ii = 1) and
      d_j = sum_k w_jk, every weight evaluated from eq. (2) directly.
  GF (Algorithm 1, eqs. (5)-(6)): (N z)_i = d_i^1/2 GF(D^-1/2 z)_i with
      GF(u)_i = (1/N_i) sum_{k: i in w_k} (a_k g_i + b_k),
      a_k = (mean_k(g u) - mu_k mean_k(u)) / (var_k(g) + eps),
      b_k = mean_k(u) - a_k mu_k, means over the truncated window w_k,
      d_j = N_j / |w| (N_j = number of windows containing j); L_sym = I - N.
Both take the grid as a 1D or 2D array g (row-major point numbering) and a
list of flat point indices.
"""
from __future__ import annotations

import itertools

import numpy as np


def _coords(shape, i):
    return np.array(np.unravel_index(int(i), shape), dtype=np.int64)


def _window(shape, p, radius):
    """Grid points of the truncated square window around p: (coords, flat)."""
    ranges = [range(max(0, int(c) - radius), min(int(s), int(c) + radius + 1)) for c, s in zip(p, shape)]
    pts = np.array(list(itertools.product(*ranges)), dtype=np.int64)
    return pts, np.ravel_multi_index(tuple(pts.T), shape)


def _bf_w(g, p, qs, sigma_s, sigma_r, channels=1):
    """eq. (2) between point p and the points qs (coords); with channels > 1
    g has a trailing channel axis and the photometric distance is the
    Euclidean distance of the channel vectors."""
    o = qs - p[None, :]
    dist2 = np.sum(o * o, axis=1).astype(np.float64)
    gp = g[tuple(p)]
    gq = g[tuple(qs.T)]
    d2 = np.sum((gq - gp[None, :]) ** 2, axis=1) if channels > 1 else (gp - gq) ** 2
    spatial = np.exp(-dist2 / (2.0 * sigma_s ** 2)) if np.isfinite(sigma_s) else 1.0
    photometric = np.exp(-d2 / (2.0 * sigma_r ** 2)) if np.isfinite(sigma_r) else 1.0
    return spatial * photometric


def bf_degree_at(g, p, radius, sigma_s, sigma_r, channels=1):
    grid = g.shape[:-1] if channels > 1 else g.shape
    qs, _ = _window(grid, p, radius)
    return float(np.sum(_bf_w(g, p, qs, sigma_s, sigma_r, channels)))


def bf_lsym_at(g, z, points, radius: int, sigma_s: float, sigma_r: float, channels: int = 1):
    """(L_sym z) at the given flat indices of the BF graph of guidance g
    (channels > 1: g has a trailing channel axis); z is (n,) or (n, m), the
    result (len(points),) or (len(points), m)."""
    g = np.asarray(g, dtype=np.float64)
    grid = g.shape[:-1] if channels > 1 else g.shape
    n = int(np.prod(grid))
    z = np.asarray(z, dtype=np.float64)
    zf = z.reshape(n, -1)
    out = np.empty((len(points), zf.shape[1]))
    for t, i in enumerate(points):
        p = _coords(grid, i)
        qs, qflat = _window(grid, p, radius)
        w = _bf_w(g, p, qs, sigma_s, sigma_r, channels)
        di = float(np.sum(w))
        dq = np.array([bf_degree_at(g, q, radius, sigma_s, sigma_r, channels) for q in qs])
        out[t] = zf[i] - (w / np.sqrt(dq)) @ zf[qflat] / np.sqrt(di)
    return out.reshape(len(points)) if z.ndim == 1 else out


def _counts(shape, coords, radius):
    """N_j for points j (coords, one row each): window points per axis, multiplied."""
    c = np.ones(coords.shape[0])
    for a, s in enumerate(shape):
        lo = np.maximum(coords[:, a] - radius, 0)
        hi = np.minimum(coords[:, a] + radius, s - 1)
        c = c * (hi - lo + 1)
    return c


def gf_lsym_at(g, z, points, radius: int, eps: float):
    """(L_sym z) at the given flat indices of the GF operator of guidance g;
    z is (n,) or (n, m)."""
    g = np.asarray(g, dtype=np.float64)
    shape = g.shape
    ndim = g.ndim
    omega = float((2 * radius + 1) ** ndim)
    z = np.asarray(z, dtype=np.float64)
    zf = z.reshape(g.size, -1)
    gflat = g.ravel()
    out = np.empty((len(points), zf.shape[1]))
    for t, i in enumerate(points):
        p = _coords(shape, i)
        ks, _ = _window(shape, p, radius)          # windows w_k that contain i
        acc = np.zeros(zf.shape[1])
        for k in ks:
            memc, mem = _window(shape, k, radius)  # members of w_k
            dmem = _counts(shape, memc, radius) / omega
            u = zf[mem] / np.sqrt(dmem)[:, None]
            gm = gflat[mem]
            mu = gm.mean()
            var = (gm * gm).mean() - mu * mu
            a = ((gm[:, None] * u).mean(axis=0) - mu * u.mean(axis=0)) / (var + eps)
            b = u.mean(axis=0) - a * mu
            acc += a * gflat[i] + b
        ni = ks.shape[0]
        di = ni / omega
        out[t] = zf[i] - np.sqrt(di) * acc / ni
    return out.reshape(len(points)) if z.ndim == 1 else out


def sample_points(shape, count: int, seed):
    """Seeded sample of flat indices: the corners and border midpoints of the
    grid plus uniform interior points."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    special = set()
    if len(shape) == 2:
        H, W = shape
        for y in (0, 1, H // 2, H - 2, H - 1):
            for x in (0, 1, W // 2, W - 2, W - 1):
                if 0 <= y < H and 0 <= x < W:
                    special.add(y * W + x)
    else:
        special.update({0, 1, n // 2, n - 2, n - 1})
    rest = rng.choice(n, size=max(count - len(special), 0), replace=False)
    return np.array(sorted(special | set(int(v) for v in rest)), dtype=np.int64)
