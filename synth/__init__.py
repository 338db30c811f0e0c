"""Seeded synthetic workloads shared by the CPU oracle and the GPU path.

This package draws random inputs only; it contains none of the filter's
arithmetic and imports neither `oracle` nor `paper_1509_02468_amd`.
"""
from .generators import (piecewise_constant_1d, piecewise_linear_1d, scene_2d, scene_2d_rgb, batch_items, item_signal,
                         lobpcg_gaussian_block, convnet_init)
from .workloads import WORKLOADS, STUDY_1D, make_signal, study_signal

__all__ = ["piecewise_constant_1d", "piecewise_linear_1d", "scene_2d", "scene_2d_rgb", "batch_items", "item_signal",
           "lobpcg_gaussian_block", "convnet_init", "WORKLOADS", "STUDY_1D", "make_signal", "study_signal"]
