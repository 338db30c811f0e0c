"""Named workloads: input recipes plus the operator and solver parameters the
experiments use.  Sizes and parameters only; no filter arithmetic.

signal_1d_4096   1D, n=4096, G1, sigma=0.1, seed 1; BF radius 5, sigma_d=3,
                 sigma_r=0.2, FP64; 30 iterations of power / CG / LOBPCG(m=3).
image_1024_bf11  2D 1024x1024, G2, sigma=0.05, seed 2; BF 11x11, sigma_d=2,
                 sigma_r=0.1, FP32 (FP64 Rayleigh-Ritz); CG 50, LOBPCG(m=4) 50.
image_4096_bf7   2D 4096x4096, G2, sigma=0.08, seed 3; BF 7x7, sigma_d=2,
                 sigma_r=0.15; LOBPCG(m=8) 100.
image_4096_gf8   same image; GF radius 8, eps=1e-2; LOBPCG(m=8) 100.
image_2048_bf11  2D 2048x2048 evaluation images (seeds 5900..5903); BF 11x11,
                 sigma_d=2, sigma_r=0.1; LOBPCG(m=4) with the constraint, tol 1e-6.
image_1024_cross5  2D 1024x1024, G2, sigma=0.1 (noise variance 0.01, so a
                 noisy PSNR of about 20 dB), seed 7; BF on the 5-point (cross,
                 radius 1) lattice, sigma_r=0.1, sigma_d=1 (a common factor
                 of every weight, which the (diag L) normalization removes),
                 normalized by diag L, FP32; 20 steps of CG and of LOBPCG
                 (m=1) with and without the constraint.
image_1024_rgb_bf11  2D 1024x1024 colour (G4), sigma=0.05 per channel, seed
                 12; guidance: the noisy image in CIE-Lab; BF 11x11, sigma_d=2,
                 sigma_r=5 (Delta E units), FP32; the three RGB channels
                 filtered as one block: 10 CG steps, 20 power passes.
STUDY_1D         the 1D filter study of Section 6: G3 signals with N = 500
                 and 1000 samples, sigma=0.1, seed 11; self-guided BF
                 (re-guided, window width 3: radius 1, sigma_d=1,
                 sigma_r=0.1) 500 passes; self-guided GF (re-guided, window
                 width 5: radius 2, eps=0.01) 20 passes; BF-CG 20 steps with
                 the noiseless signal as the guidance (same BF parameters,
                 preconditioner D); the GF-accelerated filters (CG and LOBPCG
                 m=1, 20 steps, noiseless guidance) and BF-LOBPCG 20; FP64.
"""
from __future__ import annotations

from .generators import piecewise_constant_1d, piecewise_linear_1d, scene_2d, scene_2d_rgb

WORKLOADS = {
    "signal_1d_4096": dict(shape=(4096,), sigma=0.1, seed=1, kind="bf", radius=5,
                           sigma_d=3.0, sigma_r=0.2, eps=0.0, prec="f64",
                           power_iters=30, cg_iters=30, lobpcg_iters=30, lobpcg_m=3),
    "image_1024_bf11": dict(shape=(1024, 1024), sigma=0.05, seed=2, kind="bf", radius=5,
                            sigma_d=2.0, sigma_r=0.1, eps=0.0, prec="f32",
                            cg_iters=50, lobpcg_iters=50, lobpcg_m=4),
    "image_4096_bf7": dict(shape=(4096, 4096), sigma=0.08, seed=3, kind="bf", radius=3,
                           sigma_d=2.0, sigma_r=0.15, eps=0.0, prec="f32",
                           lobpcg_iters=100, lobpcg_m=8),
    "image_4096_gf8": dict(shape=(4096, 4096), sigma=0.08, seed=3, kind="gf", radius=8,
                           sigma_d=0.0, sigma_r=0.0, eps=1e-2, prec="f32",
                           lobpcg_iters=100, lobpcg_m=8),
    "image_2048_bf11": dict(shape=(2048, 2048), sigma=0.05, seed=5900, kind="bf", radius=5,
                            sigma_d=2.0, sigma_r=0.1, eps=0.0, prec="f32",
                            lobpcg_m=4, tol=1e-6, max_iters=20000, constraint=True),
    "image_1024_cross5": dict(shape=(1024, 1024), sigma=0.1, seed=7, kind="bf", radius=1,
                              sigma_d=1.0, sigma_r=0.1, eps=0.0, prec="f32", stencil="cross", norm="diagl",
                              cg_iters=20, lobpcg_iters=20, lobpcg_m=1),
    "image_1024_rgb_bf11": dict(shape=(1024, 1024), sigma=0.05, seed=12, kind="bf", radius=5,
                                sigma_d=2.0, sigma_r=5.0, eps=0.0, prec="f32", channels=3,
                                cg_iters=10, power_iters=20),
}


STUDY_1D = dict(sizes=(500, 1000), sigma=0.1, seed=11, prec="f64",
                bf=dict(radius=1, sigma_d=1.0, sigma_r=0.1, passes=500),
                gf=dict(radius=2, eps=0.01, passes=20),
                krylov_steps=20)


def study_signal(n: int):
    """(clean, noisy) G3 signal of the 1D study with n samples."""
    return piecewise_linear_1d(n, STUDY_1D["sigma"], STUDY_1D["seed"])


def make_signal(name: str, shape=None, seed=None):
    """(clean, noisy) float64 input of a named workload; `shape`/`seed`
    override the defaults (used for crops at test sizes)."""
    w = WORKLOADS[name]
    shape = tuple(shape) if shape is not None else w["shape"]
    seed = w["seed"] if seed is None else seed
    if len(shape) == 1:
        return piecewise_constant_1d(shape[0], w["sigma"], seed)
    if w.get("channels", 1) == 3:
        return scene_2d_rgb(shape[0], shape[1], w["sigma"], seed)
    return scene_2d(shape[0], shape[1], w["sigma"], seed)
