"""Plain FP64 CPU oracle for the accelerated graph spectral polynomial filters
(Knyazev & Malyshev, "Accelerated graph-based spectral polynomial filters").

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links
this package: only the test-suite, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library; the only common
input is the seeded generator package `synth`, which holds none of the
method's arithmetic.

Contents (each function cites the passage it follows):
  graph      BF weights, eq. (2); adjacency W, degrees D, Laplacian L = D - W,
             eq. (4); normalized operator D^-1/2 W D^-1/2 (Section 4).
  guided     guided filter, Algorithm 1; its implicit matrix, eqs. (5)-(6).
  operator   one object per graph operator with the three apply forms
             (normalized N, L_sym = I - N, random-walk D^-1 W, eq. (3)).
  solvers    power iteration (Section 4), preconditioned CG for Lx = 0
             (Algorithm 2), block LOBPCG as a low-pass filter (Algorithm 3,
             Section 6).
  reguided   the non-linear (re-guided) power and CG filters: the graph is
             rebuilt from the current iterate every step (Sections 2-3,
             the first way to iterate BF and GF; Algorithm 2's flexible beta).
  spectral   dense spectral factorization eq. (8) and GFT low-pass filters.
  quality    PSNR.
  colour     sRGB -> CIE-Lab (the colour guidance of Section 2).
  convnet    FP64 reference of the learned convolutional preconditioner
             (forward, backward, Adam) with BF16 rounding emulation.

Readings where the paper is silent or ambiguous are stated at each function.
"""
from .graph import window_offsets, bf_weight_matrix, degrees
from .guided import box_sum, box_count, f_mean, guided_filter, gf_stats, gf_weight_matrix_dense, gf_degrees
from .operator import GraphOperator, build_operator
from .solvers import (power_filter, cg_filter, cg_filter_block, cg_filter_normalized, modulated_start, modulation_degrees,
                      rayleigh_ritz, lobpcg_filter, CgInfo, LobpcgInfo, precondition, lobpcg_residual,
                      shifted_cg, ShiftedCgInfo)
from . import convnet
from .reguided import power_filter_reguided, cg_filter_reguided
from .quality import psnr
from .colour import srgb_to_lab

__all__ = [
    "window_offsets", "bf_weight_matrix", "degrees",
    "box_sum", "box_count", "f_mean", "guided_filter", "gf_stats", "gf_weight_matrix_dense", "gf_degrees",
    "GraphOperator", "build_operator",
    "power_filter", "cg_filter", "cg_filter_block", "cg_filter_normalized", "modulated_start", "modulation_degrees", "rayleigh_ritz",
    "lobpcg_filter", "CgInfo", "LobpcgInfo", "psnr", "precondition", "lobpcg_residual", "shifted_cg",
    "ShiftedCgInfo", "convnet",
    "power_filter_reguided", "cg_filter_reguided", "srgb_to_lab",
]
