"""Seeded synthetic inputs: noisy piecewise-constant 1D signals and noisy
piecewise-smooth 2D scenes.

These generators stand in for the paper's test data (Section 7 uses a
piecewise-linear 1D signal with additive Gaussian noise and an unnamed test
image with Gaussian noise of variance 0.01; neither is available).  They hold
none of the filtering method's arithmetic: they only draw random numbers and
paint shapes.  Both the CPU oracle and the GPU library consume their output.

G1  1D: 8 distinct breakpoints drawn from {1, ..., n-1} without replacement,
    9 constant pieces with levels U[0,1], plus sigma * N(0,1) noise (no clip).
G3  1D piecewise linear with steep ascents and descents: 6 edges at distinct
    positions on a grid of spacing 2 max(width) + 2 (ends kept clear); each
    edge is a linear ramp over U{2..6} samples that moves the level by
    U[0.3, 0.7], up where the level is below 0.5 and down otherwise; between
    edges the signal runs linearly with slope U[-0.5, 0.5] / n per sample from
    the start level U[0,1]; linear interpolation between these knots; plus
    sigma * N(0,1) noise (the paper's 0.1 * randn(N, 1) at sigma = 0.1).
G4  2D colour (sRGB in [0, 1]): G2's construction with RGB colours instead of
    intensities (background gradient between two colours U[0,1]^3, shape
    colours U[0,1]^3), plus sigma * N(0,1) noise on every channel.
G2  2D: linear-gradient background g0 + (g1-g0) * t(p) along a random
    direction, then 40 random rectangles / disks (probability 1/2 each) in
    painter's order with intensities U[0,1], centres uniform over the image,
    half-sides / radius U[0.02, 0.15] * side, pixel-centre inclusion; plus
    sigma * N(0,1) noise (no clip).
"""
from __future__ import annotations

import numpy as np

__all__ = ["piecewise_constant_1d", "piecewise_linear_1d", "scene_2d", "scene_2d_rgb", "batch_items", "lobpcg_gaussian_block", "convnet_init"]


def piecewise_constant_1d(n: int, sigma: float, seed, n_breaks: int = 8):
    """Return (clean, noisy) float64 arrays of length n (G1)."""
    rng = np.random.default_rng(seed)
    n_breaks = min(n_breaks, max(n - 1, 0))
    clean = np.empty(n, dtype=np.float64)
    if n_breaks > 0:
        cuts = np.sort(rng.choice(np.arange(1, n), size=n_breaks, replace=False))
    else:
        cuts = np.zeros(0, dtype=np.int64)
    levels = rng.uniform(0.0, 1.0, size=n_breaks + 1)
    edges = np.concatenate(([0], cuts, [n]))
    for k in range(n_breaks + 1):
        clean[edges[k]:edges[k + 1]] = levels[k]
    noisy = clean + sigma * rng.standard_normal(n)
    return clean, noisy


def piecewise_linear_1d(n: int, sigma: float, seed, n_edges: int = 6):
    """Return (clean, noisy) float64 arrays of length n (G3)."""
    rng = np.random.default_rng(seed)
    widths = rng.integers(2, 7, size=n_edges)
    gap = 2 * int(widths.max()) + 2
    slots = np.arange(gap, n - gap, gap)
    starts = np.sort(rng.choice(slots, size=min(n_edges, slots.size), replace=False))
    level = rng.uniform(0.0, 1.0)
    kx, ky = [0.0], [level]
    prev = 0
    for s0, w in zip(starts, widths[:starts.size]):
        slope = rng.uniform(-0.5, 0.5) / n
        kx.append(float(s0))
        ky.append(level + slope * (s0 - prev))
        step = rng.uniform(0.3, 0.7)
        level = ky[-1] + (step if ky[-1] < 0.5 else -step)
        prev = int(s0 + w)
        kx.append(float(prev))
        ky.append(level)
    slope = rng.uniform(-0.5, 0.5) / n
    kx.append(float(n - 1))
    ky.append(level + slope * (n - 1 - prev))
    clean = np.interp(np.arange(n, dtype=np.float64), kx, ky)
    noisy = clean + sigma * rng.standard_normal(n)
    return clean, noisy


def scene_2d(height: int, width: int, sigma: float, seed, n_shapes: int = 40):
    """Return (clean, noisy) float64 arrays of shape (height, width) (G2)."""
    rng = np.random.default_rng(seed)
    side = float(max(height, width))
    yy, xx = np.meshgrid(np.arange(height) + 0.5, np.arange(width) + 0.5, indexing="ij")
    g0, g1 = rng.uniform(0.0, 1.0, size=2)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    t = np.cos(phi) * xx + np.sin(phi) * yy
    tmin, tmax = t.min(), t.max()
    t = (t - tmin) / (tmax - tmin) if tmax > tmin else np.zeros_like(t)
    img = g0 + (g1 - g0) * t
    for _ in range(n_shapes):
        is_rect = rng.uniform() < 0.5
        cy = rng.uniform(0.0, height)
        cx = rng.uniform(0.0, width)
        level = rng.uniform(0.0, 1.0)
        if is_rect:
            hy = rng.uniform(0.02, 0.15) * side
            hx = rng.uniform(0.02, 0.15) * side
            y0, y1 = int(max(0, np.floor(cy - hy))), int(min(height, np.ceil(cy + hy) + 1))
            x0, x1 = int(max(0, np.floor(cx - hx))), int(min(width, np.ceil(cx + hx) + 1))
            sub_y, sub_x = yy[y0:y1, x0:x1], xx[y0:y1, x0:x1]
            mask = (np.abs(sub_y - cy) <= hy) & (np.abs(sub_x - cx) <= hx)
        else:
            rad = rng.uniform(0.02, 0.15) * side
            y0, y1 = int(max(0, np.floor(cy - rad))), int(min(height, np.ceil(cy + rad) + 1))
            x0, x1 = int(max(0, np.floor(cx - rad))), int(min(width, np.ceil(cx + rad) + 1))
            sub_y, sub_x = yy[y0:y1, x0:x1], xx[y0:y1, x0:x1]
            mask = (sub_y - cy) ** 2 + (sub_x - cx) ** 2 <= rad * rad
        img[y0:y1, x0:x1][mask] = level
    noisy = img + sigma * rng.standard_normal((height, width))
    return img, noisy


def scene_2d_rgb(height: int, width: int, sigma: float, seed, n_shapes: int = 40):
    """Return (clean, noisy) float64 arrays of shape (height, width, 3) (G4)."""
    rng = np.random.default_rng(seed)
    side = float(max(height, width))
    yy, xx = np.meshgrid(np.arange(height) + 0.5, np.arange(width) + 0.5, indexing="ij")
    c0, c1 = rng.uniform(0.0, 1.0, size=(2, 3))
    phi = rng.uniform(0.0, 2.0 * np.pi)
    t = np.cos(phi) * xx + np.sin(phi) * yy
    tmin, tmax = t.min(), t.max()
    t = (t - tmin) / (tmax - tmin) if tmax > tmin else np.zeros_like(t)
    img = c0[None, None, :] + (c1 - c0)[None, None, :] * t[..., None]
    for _ in range(n_shapes):
        is_rect = rng.uniform() < 0.5
        cy = rng.uniform(0.0, height)
        cx = rng.uniform(0.0, width)
        colour = rng.uniform(0.0, 1.0, size=3)
        if is_rect:
            hy = rng.uniform(0.02, 0.15) * side
            hx = rng.uniform(0.02, 0.15) * side
            y0, y1 = int(max(0, np.floor(cy - hy))), int(min(height, np.ceil(cy + hy) + 1))
            x0, x1 = int(max(0, np.floor(cx - hx))), int(min(width, np.ceil(cx + hx) + 1))
            sub_y, sub_x = yy[y0:y1, x0:x1], xx[y0:y1, x0:x1]
            mask = (np.abs(sub_y - cy) <= hy) & (np.abs(sub_x - cx) <= hx)
        else:
            rad = rng.uniform(0.02, 0.15) * side
            y0, y1 = int(max(0, np.floor(cy - rad))), int(min(height, np.ceil(cy + rad) + 1))
            x0, x1 = int(max(0, np.floor(cx - rad))), int(min(width, np.ceil(cx + rad) + 1))
            sub_y, sub_x = yy[y0:y1, x0:x1], xx[y0:y1, x0:x1]
            mask = (sub_y - cy) ** 2 + (sub_x - cx) ** 2 <= rad * rad
        img[y0:y1, x0:x1][mask] = colour
    noisy = img + sigma * rng.standard_normal((height, width, 3))
    return img, noisy


def lobpcg_gaussian_block(n: int, m: int, seed):
    """Seeded standard-normal n x m block (used only where a caller wants an
    explicit LOBPCG start block instead of the Krylov start)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, m))


def batch_items(seed: int = 4, n_images: int = 256, n_signals: int = 64,
                side_range=(64, 1024), len_range=(2 ** 10, 2 ** 20), max_pixels=None):
    """Per-item recipe of the uneven batch workload.

    Image sides are log-uniform in side_range (square images), signal lengths
    log-uniform in len_range, noise sigma ~ U[0.03, 0.1].  Each item carries
    its own operator parameters: kind BF or GF with probability 1/2; BF radius
    in {1..5}, sigma_d ~ U[1,3], sigma_r ~ U[0.05,0.3]; GF radius in {1..8},
    eps log-uniform in [1e-3, 1e-1]; solver CG or LOBPCG (m=4) with
    probability 1/2; kmax = 50, tol = 1e-6.  Item i uses sub-seed (seed, i).
    Returns a list of dicts (signals are produced lazily by `item_signal`).
    """
    rng = np.random.default_rng(seed)
    items = []
    total = n_images + n_signals
    for i in range(total):
        is_img = i < n_images
        if is_img:
            s = int(round(np.exp(rng.uniform(np.log(side_range[0]), np.log(side_range[1])))))
            shape = (s, s)
        else:
            n = int(round(np.exp(rng.uniform(np.log(len_range[0]), np.log(len_range[1])))))
            shape = (n,)
        sigma = float(rng.uniform(0.03, 0.1))
        kind = "bf" if rng.uniform() < 0.5 else "gf"
        if kind == "bf":
            radius = int(rng.integers(1, 6))
            sigma_d = float(rng.uniform(1.0, 3.0))
            sigma_r = float(rng.uniform(0.05, 0.3))
            eps = 0.0
        else:
            radius = int(rng.integers(1, 9))
            sigma_d = sigma_r = 0.0
            eps = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e-1))))
        method = "cg" if rng.uniform() < 0.5 else "lobpcg"
        items.append(dict(index=i, shape=shape, sigma=sigma, kind=kind, radius=radius,
                          sigma_d=sigma_d, sigma_r=sigma_r, eps=eps, method=method,
                          m=4 if method == "lobpcg" else 1, kmax=50, tol=1e-6,
                          seed=(seed, i)))
    if max_pixels is not None:
        items = [it for it in items if int(np.prod(it["shape"])) <= max_pixels]
    return items


def item_signal(item):
    """(clean, noisy) for one batch item."""
    if len(item["shape"]) == 1:
        return piecewise_constant_1d(item["shape"][0], item["sigma"], item["seed"])
    return scene_2d(item["shape"][0], item["shape"][1], item["sigma"], item["seed"])


def convnet_init(seed, hidden: int = 16, inputs: int = 2):
    """Seeded initial weights of the 3-layer 3x3 convolutional network, flat
    in layer order (layer1 hidden x inputs x 3 x 3, layer2 hidden x hidden x
    3 x 3, layer3 hidden x 3 x 3).  He-normal scale sqrt(2 / fan_in) for the
    two ReLU layers, sqrt(1 / fan_in) for the linear output layer; float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, gain in (((hidden, inputs, 3, 3), 2.0), ((hidden, hidden, 3, 3), 2.0), ((1, hidden, 3, 3), 1.0)):
        fan_in = shape[1] * 9
        parts.append(rng.standard_normal(shape).ravel() * np.sqrt(gain / fan_in))
    return np.concatenate(parts).astype(np.float32)
