"""MI355X-native graph spectral polynomial filters (Knyazev & Malyshev,
"Accelerated graph-based spectral polynomial filters").

The compute path is the HIP library libgsf.so (C ABI in include/gsf.h); this
package is its thin ctypes binding.  There is no CPU fallback: calls fail if
the library has not been built.
"""
from .gsf import (OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EBREAKDOWN, ESCRATCH, BF, GF, F32, F64,
                  FORM_N, FORM_LSYM, FORM_RW, FORM_L, METHOD_POWER, METHOD_CG, METHOD_LOBPCG,
                  STENCIL_SQUARE, STENCIL_CROSS, NORM_D, NORM_DIAGL, LIB_PATH, GsfError, Operator, Batch, Precond, NetTrainer, NET_WEIGHTS, build_operator,
                  batch_filter, tune_table_save, tune_table_load, tune_table_clear, block_gram, rayleigh_ritz, reguided_filter, reguided_workspace, srgb_to_lab, load_library)

__all__ = ["OK", "EINVAL", "ENOMEM", "EDEVICE", "ENOTCONV", "EBREAKDOWN", "ESCRATCH", "BF", "GF", "F32", "F64",
           "FORM_N", "FORM_LSYM", "FORM_RW", "FORM_L", "METHOD_POWER", "METHOD_CG", "METHOD_LOBPCG",
           "STENCIL_SQUARE", "STENCIL_CROSS", "NORM_D", "NORM_DIAGL", "LIB_PATH", "GsfError", "Operator", "Batch", "Precond", "NetTrainer", "NET_WEIGHTS", "build_operator",
           "batch_filter", "tune_table_save", "tune_table_load", "tune_table_clear", "block_gram", "rayleigh_ritz", "reguided_filter", "reguided_workspace", "srgb_to_lab", "load_library"]
