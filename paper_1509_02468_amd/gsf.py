"""ctypes binding of libgsf (argument marshalling only; every step runs in the
HIP library).  Device buffers are torch CUDA tensors (ROCm); torch is used for
device memory and streams only.

Names mirror the C ABI in include/gsf.h: build_operator, apply, power_filter,
cg_filter, lobpcg_filter, the learned preconditioner (net_* training entry
points, Precond, shifted_cg, lobpcg_residual, make_pair), batching (Batch),
plus the diagnostic block_gram / rayleigh_ritz.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsf.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EBREAKDOWN, ESCRATCH = range(7)
BF, GF = 0, 1
F32, F64 = 0, 1
FORM_N, FORM_LSYM, FORM_RW, FORM_L = 0, 1, 2, 3
METHOD_POWER, METHOD_CG, METHOD_LOBPCG = 0, 1, 2
STENCIL_SQUARE, STENCIL_CROSS = 0, 1
NORM_D, NORM_DIAGL = 0, 1
_STENCILS = {"square": STENCIL_SQUARE, "cross": STENCIL_CROSS, STENCIL_SQUARE: STENCIL_SQUARE,
             STENCIL_CROSS: STENCIL_CROSS}
_NORMS = {"d": NORM_D, "diagl": NORM_DIAGL, NORM_D: NORM_D, NORM_DIAGL: NORM_DIAGL}
STATUS_NAMES = {OK: "ok", EINVAL: "einval", ENOMEM: "enomem", EDEVICE: "edevice",
                ENOTCONV: "notconv", EBREAKDOWN: "breakdown", ESCRATCH: "escratch"}


class OperatorDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ndim", ctypes.c_int32), ("dims", ctypes.c_int64 * 2),
                ("prec", ctypes.c_int32), ("radius", ctypes.c_int32), ("sigma_d", ctypes.c_double),
                ("sigma_r", ctypes.c_double), ("gf_eps", ctypes.c_double), ("stencil", ctypes.c_int32),
                ("norm", ctypes.c_int32), ("channels", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class OperatorLayout(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ndim", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("n", ctypes.c_int64), ("nplanes", ctypes.c_int32),
                ("planes", ctypes.c_void_p), ("inv_sqrt_d", ctypes.c_void_p), ("sqrt_d", ctypes.c_void_p),
                ("degree", ctypes.c_void_p), ("guidance", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("inv", ctypes.c_void_p), ("plane_stride", ctypes.c_int64)]


class CgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("res0", ctypes.c_double),
                ("res", ctypes.c_double)]


class LobpcgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("dropped", ctypes.c_int32),
                ("m", ctypes.c_int32), ("res", ctypes.c_double * 8), ("theta", ctypes.c_double * 8),
                ("fallbacks", ctypes.c_int32), ("pad", ctypes.c_int32)]


class BatchItem(ctypes.Structure):
    _fields_ = [("op", OperatorDesc), ("guidance", ctypes.c_void_p), ("x0", ctypes.c_void_p),
                ("x_out", ctypes.c_void_p), ("method", ctypes.c_int32), ("m", ctypes.c_int32),
                ("kmax", ctypes.c_int32), ("constraint", ctypes.c_int32), ("tol", ctypes.c_double)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("res0", ctypes.c_double),
                ("res", ctypes.c_double)]


_lib = None


class GsfError(RuntimeError):
    def __init__(self, status, where, detail=""):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}{detail}")
        self.status = status


def load_library(path: str = LIB_PATH):
    """Load libgsf.so (raises if it has not been built; there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1509_02468_amd.build`")
    # torch first: it brings its own HIP runtime, and libgsf must bind to that
    # same runtime (loaded first, the library's link-time runtime is a second
    # instance in the process, whose first launch then finds no device)
    _torch()
    lib = ctypes.CDLL(path)
    vp, sz, i32, i64, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "gsf_version": ([], i32),
        "gsf_status_string": ([i32], ctypes.c_char_p),
        "gsf_last_device_error": ([], i32),
        "gsf_device_error_string": ([i32], ctypes.c_char_p),
        "gsf_operator_workspace_bytes": ([P(OperatorDesc), P(sz)], i32),
        "gsf_build_operator": ([P(OperatorDesc), vp, vp, sz, vp, P(vp)], i32),
        "gsf_operator_get_layout": ([vp, P(OperatorLayout)], i32),
        "gsf_destroy_operator": ([vp], None),
        "gsf_apply": ([vp, i32, i32, vp, i64, vp, i64, vp], i32),
        "gsf_solver_workspace_bytes": ([vp, i32, i32, P(sz)], i32),
        "gsf_power_filter": ([vp, vp, vp, i32, vp, sz, vp], i32),
        "gsf_cg_filter": ([vp, vp, vp, i32, dbl, vp, sz, P(CgInfo), vp], i32),
        "gsf_cg_filter_noalloc": ([vp, vp, vp, i32, dbl, P(CgInfo), vp], i32),
        "gsf_power_filter_block": ([vp, i32, vp, vp, i32, vp, sz, vp], i32),
        "gsf_cg_filter_block": ([vp, i32, vp, vp, i32, dbl, vp, sz, P(CgInfo), vp], i32),
        "gsf_srgb_to_lab": ([i32, i64, vp, vp, vp], i32),
        "gsf_joint_workspace_bytes": ([vp, i32, P(sz)], i32),
        "gsf_apply_joint": ([vp, i32, i32, vp, vp, vp, vp, vp], i32),
        "gsf_joint_filter": ([vp, vp, vp, i32, vp, vp, i32, i32, i32, vp, sz, P(CgInfo), P(LobpcgInfo), vp], i32),
        "gsf_reguided_workspace_bytes": ([P(OperatorDesc), i32, P(sz)], i32),
        "gsf_reguided_filter": ([P(OperatorDesc), i32, vp, vp, i32, dbl, vp, sz, P(CgInfo), vp], i32),
        "gsf_lobpcg_filter": ([vp, vp, vp, i32, i32, dbl, i32, vp, vp, P(dbl), vp, sz, P(LobpcgInfo), vp], i32),
        "gsf_block_gram": ([i32, i64, i32, i32, P(vp), P(vp), vp, vp, vp, sz, vp], i32),
        "gsf_block_gram_workspace_bytes": ([i64, P(sz)], i32),
        "gsf_rayleigh_ritz": ([i32, i32, vp, vp, dbl, dbl, vp, vp, vp, vp, vp, sz, vp], i32),
        "gsf_rr_workspace_bytes": ([], sz),
        "gsf_tune_apply": ([vp, i32, vp, vp, i32, P(ctypes.c_int), P(ctypes.c_float), vp], i32),
        "gsf_set_apply_rows": ([vp, i32, i32], i32),
        "gsf_batch_workspace_bytes": ([P(BatchItem), i32, P(sz)], i32),
        "gsf_batch_create": ([P(BatchItem), i32, vp, sz, i32, P(vp)], i32),
        "gsf_batch_run": ([vp, vp], i32),
        "gsf_batch_get_info": ([vp, P(BatchInfo), vp], i32),
        "gsf_batch_destroy": ([vp], None),
        "gsf_batch_filter": ([P(BatchItem), i32, vp, sz, P(BatchInfo), vp], i32),
        "gsf_net_workspace_bytes": ([i32, i64, i64, P(sz)], i32),
        "gsf_net_forward": ([vp, i32, vp, i64, i64, vp, vp, vp, sz, vp], i32),
        "gsf_net_loss_grad": ([vp, i32, vp, i64, i64, vp, vp, vp, vp, vp, sz, vp], i32),
        "gsf_net_adam": ([i64, i32, dbl, dbl, dbl, dbl, vp, vp, vp, vp, vp, vp], i32),
        "gsf_net_to_bf16": ([i64, vp, vp, vp], i32),
        "gsf_net_pair_workspace_bytes": ([vp, P(sz)], i32),
        "gsf_net_make_pair": ([vp, vp, i64, vp, i64, vp, vp, vp, vp, sz, vp], i32),
        "gsf_precond_create": ([vp, vp, vp, P(vp)], i32),
        "gsf_get_apply_rows": ([vp, i32, P(i32)], i32),
        "gsf_tune_table_save": ([ctypes.c_char_p, P(i32)], i32),
        "gsf_tune_table_load": ([ctypes.c_char_p, P(i32)], i32),
        "gsf_tune_table_clear": ([], None),
        "gsf_precond_create_shifted": ([vp, dbl, i32, P(vp)], i32),
        "gsf_precond_destroy": ([vp], None),
        "gsf_precond_workspace_bytes": ([vp, i32, P(sz)], i32),
        "gsf_precond_apply": ([vp, i32, vp, vp, vp, sz, vp], i32),
        "gsf_shifted_cg": ([vp, dbl, vp, i64, vp, i32, dbl, vp, sz, P(CgInfo), vp], i32),
        "gsf_lobpcg_residual": ([vp, i32, vp, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status, where):
    if status not in (OK, ENOTCONV, EBREAKDOWN):
        detail = ""
        if status == EDEVICE and _lib is not None:
            code = _lib.gsf_last_device_error()
            if code:
                detail = f" (HIP error {code}: {_lib.gsf_device_error_string(code).decode()})"
        raise GsfError(status, where, detail)
    return status


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype(prec):
    torch = _torch()
    return torch.float32 if prec == F32 else torch.float64


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def make_desc(kind, shape, radius, sigma_d=0.0, sigma_r=0.0, eps=0.0, prec=F32, stencil="square", norm="d",
              channels=1):
    """gsf_operator_desc; stencil "square" / "cross" and norm "d" / "diagl"
    (or the GSF_STENCIL_* / GSF_NORM_* values); channels of the guidance."""
    d = OperatorDesc()
    d.kind = BF if kind in ("bf", BF) else GF
    d.ndim = len(shape)
    d.dims[0] = shape[0]
    d.dims[1] = shape[1] if len(shape) == 2 else 1
    d.prec = prec
    d.radius = radius
    d.sigma_d = sigma_d
    d.sigma_r = sigma_r
    d.gf_eps = eps
    d.stencil = _STENCILS[stencil]
    d.norm = _NORMS[norm]
    d.channels = channels
    return d


def reguided_workspace(kind, shape, method, radius, sigma_d=0.0, sigma_r=0.0, eps=0.0, prec=F32, stencil="square",
                       norm="d"):
    """Device workspace (uint8 tensor) for reguided_filter with these parameters."""
    torch = _torch()
    lib = load_library()
    d = make_desc(kind, tuple(int(v) for v in shape), radius, sigma_d, sigma_r, eps, prec, stencil, norm)
    nbytes = ctypes.c_size_t()
    _check(lib.gsf_reguided_workspace_bytes(ctypes.byref(d), method, ctypes.byref(nbytes)), "reguided_workspace_bytes")
    return torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device="cuda")


def reguided_filter(kind, shape, x0, method, kmax, radius, sigma_d=0.0, sigma_r=0.0, eps=0.0, prec=F32, tol=0.0,
                    out=None, ws=None, info=True, stream=None, stencil="square", norm="d"):
    """Re-guided (non-linear) power or CG filter (gsf_reguided_filter): the
    graph is rebuilt from the current iterate before every step.  x0: device
    tensor of n values of the precision's dtype.  Returns (x, CgInfo or None)."""
    torch = _torch()
    lib = load_library()
    d = make_desc(kind, tuple(int(v) for v in shape), radius, sigma_d, sigma_r, eps, prec, stencil, norm)
    if ws is None:
        ws = reguided_workspace(kind, shape, method, radius, sigma_d, sigma_r, eps, prec, stencil, norm)
    y = out if out is not None else torch.empty_like(x0)
    inf = CgInfo()
    st = lib.gsf_reguided_filter(ctypes.byref(d), method, _ptr(x0), _ptr(y), kmax, tol, _ptr(ws), ws.numel(),
                                 ctypes.byref(inf) if info else None, _stream(stream))
    _check(st, "reguided_filter")
    return y, (inf if info else None)


def srgb_to_lab(rgb, out=None, stream=None):
    """CIE-Lab of an n x 3 sRGB device tensor (float32 or float64), by
    gsf_srgb_to_lab."""
    torch = _torch()
    lib = load_library()
    if rgb.dim() != 2 or rgb.shape[1] != 3 or not rgb.is_contiguous():
        raise ValueError("rgb must be a contiguous n x 3 device tensor")
    prec = F32 if rgb.dtype == torch.float32 else F64
    y = out if out is not None else torch.empty_like(rgb)
    _check(lib.gsf_srgb_to_lab(prec, rgb.shape[0], _ptr(rgb), _ptr(y), _stream(stream)), "srgb_to_lab")
    return y


class Batch:
    """Many items filtered by one graph launch (gsf_batch_*).  Each item is a
    dict with kind, shape, radius, sigma_d, sigma_r, eps, guidance, x0 (device
    tensors of the batch dtype), method ("power", "cg", "lobpcg"), m, kmax,
    tol, constraint; outputs are allocated here (item["out"])."""

    METHODS = {"power": METHOD_POWER, "cg": METHOD_CG, "lobpcg": METHOD_LOBPCG}

    @classmethod
    def describe(cls, items, prec):
        """The gsf_batch_item array of `items` (outputs allocated into item["out"])."""
        torch = _torch()
        arr = (BatchItem * len(items))()
        for k, it in enumerate(items):
            it.setdefault("out", torch.empty_like(it["x0"]))
            b = arr[k]
            b.op = make_desc(it["kind"], it["shape"], it["radius"], it.get("sigma_d", 0.0), it.get("sigma_r", 0.0),
                             it.get("eps", 0.0), prec, it.get("stencil", "square"), it.get("norm", "d"))
            b.guidance = it["guidance"].data_ptr()
            b.x0 = it["x0"].data_ptr()
            b.x_out = it["out"].data_ptr()
            b.method = cls.METHODS[it["method"]]
            b.m = it.get("m", 1)
            b.kmax = it["kmax"]
            b.constraint = int(bool(it.get("constraint", False)))
            b.tol = it.get("tol", 0.0)
        return arr

    @staticmethod
    def workspace(arr, count):
        torch = _torch()
        nbytes = ctypes.c_size_t()
        _check(load_library().gsf_batch_workspace_bytes(arr, count, ctypes.byref(nbytes)), "batch_workspace_bytes")
        return torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda"), nbytes.value

    def __init__(self, items, prec=F32, autotune=True, graphs=False):
        torch = _torch()
        lib = load_library()
        self.items = items
        self.arr = self.describe(items, prec)
        self.ws, nb = self.workspace(self.arr, len(items))
        nbytes = ctypes.c_size_t(nb)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        flags = (1 if autotune else 0) | (2 if graphs else 0)
        _check(lib.gsf_batch_create(self.arr, len(items), _ptr(self.ws), nbytes.value, flags, ctypes.byref(h)),
               "batch_create")
        self.handle = h

    def run(self, stream=None):
        _check(_lib.gsf_batch_run(self.handle, _stream(stream)), "batch_run")

    def info(self, stream=None):
        out = (BatchInfo * len(self.items))()
        _check(_lib.gsf_batch_get_info(self.handle, out, _stream(stream)), "batch_get_info")
        return [(o.iters, o.status, o.res0, o.res) for o in out]

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gsf_batch_destroy(self.handle)
            self.handle = None


def batch_filter(items, prec=F32, stream=None):
    """gsf_batch_filter: the whole batch in one call (synchronizes the stream);
    returns [(iters, status, res0, res)] per item, outputs in item["out"]."""
    arr = Batch.describe(items, prec)
    ws, nb = Batch.workspace(arr, len(items))
    out = (BatchInfo * len(items))()
    _check(load_library().gsf_batch_filter(arr, len(items), _ptr(ws), nb, out, _stream(stream)), "batch_filter")
    return [(o.iters, o.status, o.res0, o.res) for o in out]


class Operator:
    """A built graph operator (BF eq. (2) or GF Algorithm 1) on the GPU.
    Owns its device workspace (a torch uint8 tensor)."""

    def __init__(self, kind, shape, guidance, radius, sigma_d=0.0, sigma_r=0.0, eps=0.0, prec=F32,
                 stream=None, ws=None, stencil="square", norm="d", channels=1):
        torch = _torch()
        lib = load_library()
        shape = tuple(int(s) for s in shape)
        self.shape, self.prec, self.kind, self.radius = shape, prec, kind, radius
        self.n = int(np.prod(shape))
        d = make_desc(kind, shape, radius, sigma_d, sigma_r, eps, prec, stencil, norm, channels)
        self.desc = d
        nbytes = ctypes.c_size_t()
        _check(lib.gsf_operator_workspace_bytes(ctypes.byref(d), ctypes.byref(nbytes)), "operator_workspace_bytes")
        if ws is not None and ws.numel() >= nbytes.value:
            self.ws = ws
        else:
            self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
        g = guidance
        if not isinstance(g, torch.Tensor):
            g = torch.as_tensor(np.ascontiguousarray(g))
        g = g.to(device="cuda", dtype=_dtype(prec)).contiguous().reshape(-1)
        if g.numel() != self.n * max(int(channels), 1):
            raise ValueError("guidance size does not match shape and channels")
        h = ctypes.c_void_p()
        _check(lib.gsf_build_operator(ctypes.byref(d), _ptr(g), _ptr(self.ws), nbytes.value, _stream(stream),
                                      ctypes.byref(h)), "build_operator")
        self.handle = h
        self._guidance = g  # keep alive until the build has run

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gsf_destroy_operator(self.handle)
            self.handle = None

    @property
    def dtype(self):
        return _dtype(self.prec)

    def layout(self):
        lay = OperatorLayout()
        _check(_lib.gsf_operator_get_layout(self.handle, ctypes.byref(lay)), "operator_get_layout")
        return lay

    def _view(self, ptr, count, dtype):
        """Copy `count` elements at device address ptr (inside the workspace)."""
        torch = _torch()
        base = self.ws.data_ptr()
        off = int(ptr) - base
        esz = torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + count * esz].view(dtype).clone()

    def planes(self):
        torch = _torch()
        lay = self.layout()
        esz = torch.tensor([], dtype=self.dtype).element_size()
        return torch.stack([self._view(lay.planes + q * lay.plane_stride * esz, self.n, self.dtype)
                            for q in range(lay.nplanes)])

    def inv_sqrt_d(self):
        return self._view(self.layout().inv_sqrt_d, self.n, self.dtype)

    def sqrt_d(self):
        return self._view(self.layout().sqrt_d, self.n, self.dtype)

    def degree(self):
        return self._view(self.layout().degree, self.n, _torch().float64)

    def gf_stats(self):
        lay = self.layout()
        return self._view(lay.mu, self.n, self.dtype), self._view(lay.inv, self.n, self.dtype)

    # -- entry points --------------------------------------------------------
    @staticmethod
    def _ld(t, m):
        """Elements between consecutive points of a vector (m = 1) or of an
        n x m block whose rows are contiguous (a column slice of a wider
        point-major array is allowed)."""
        if t.dim() == 1:
            if not t.is_contiguous():
                raise ValueError("a vector must be contiguous")
            return 1
        if t.stride(1) != 1 or t.stride(0) < m:
            raise ValueError("a block needs contiguous rows (stride 1 within a point)")
        return t.stride(0)

    def apply(self, x, form=FORM_N, out=None, stream=None):
        torch = _torch()
        m = 1 if x.dim() == 1 else x.shape[1]
        if x.dtype != self.dtype or not x.is_cuda:
            raise ValueError("x must be a device tensor of the operator dtype")
        y = out if out is not None else torch.empty(x.shape, dtype=x.dtype, device=x.device)
        _check(_lib.gsf_apply(self.handle, form, m, _ptr(x), self._ld(x, m), _ptr(y), self._ld(y, m),
                              _stream(stream)), "apply")
        return y

    def apply_joint(self, x, x2, form=FORM_LSYM, out=None, out2=None, stream=None):
        """(F x, F x2) for an n x m block x and a vector x2 in one pass (gsf_apply_joint)."""
        torch = _torch()
        m = 1 if x.dim() == 1 else x.shape[1]
        y = out if out is not None else torch.empty_like(x)
        y2 = out2 if out2 is not None else torch.empty_like(x2)
        _check(_lib.gsf_apply_joint(self.handle, form, m, _ptr(x), _ptr(y), _ptr(x2), _ptr(y2), _stream(stream)),
               "apply_joint")
        return y, y2

    def tune_apply(self, m=1, reps=20, stream=None):
        """Pick the apply tile height for block width m (see gsf_tune_apply);
        returns (rows per thread, [us per launch for 1, 2, 4])."""
        torch = _torch()
        x = torch.randn((self.n, m) if m > 1 else (self.n,), dtype=self.dtype, device="cuda")
        y = torch.empty_like(x)
        best = ctypes.c_int()
        times = (ctypes.c_float * 3)()
        _check(_lib.gsf_tune_apply(self.handle, m, _ptr(x), _ptr(y), reps, ctypes.byref(best), times,
                                   _stream(stream)), "tune_apply")
        return best.value, list(times)

    def apply_rows(self, m):
        """Rows per thread the BF apply of block width m uses (gsf_get_apply_rows)."""
        v = ctypes.c_int()
        _check(_lib.gsf_get_apply_rows(self.handle, m, ctypes.byref(v)), "get_apply_rows")
        return v.value

    def set_apply_rows(self, m, rows_per_thread):
        """Pin the BF apply tile height for block width m (see gsf_set_apply_rows)."""
        _check(_lib.gsf_set_apply_rows(self.handle, m, rows_per_thread), "set_apply_rows")

    def workspace(self, method, m=1):
        torch = _torch()
        nbytes = ctypes.c_size_t()
        _check(_lib.gsf_solver_workspace_bytes(self.handle, method, m, ctypes.byref(nbytes)), "solver_workspace_bytes")
        return torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device="cuda")

    def power_filter(self, x0, kmax, out=None, ws=None, stream=None):
        torch = _torch()
        y = out if out is not None else torch.empty_like(x0)
        ws = ws if ws is not None else self.workspace(METHOD_POWER)
        _check(_lib.gsf_power_filter(self.handle, _ptr(x0), _ptr(y), kmax, _ptr(ws), ws.numel(), _stream(stream)),
               "power_filter")
        return y

    def power_filter_block(self, x0, kmax, out=None, ws=None, stream=None):
        """Power filter of every column of an n x m block (gsf_power_filter_block)."""
        torch = _torch()
        m = x0.shape[1]
        y = out if out is not None else torch.empty_like(x0)
        ws = ws if ws is not None else self.workspace(METHOD_POWER, m)
        _check(_lib.gsf_power_filter_block(self.handle, m, _ptr(x0), _ptr(y), kmax, _ptr(ws), ws.numel(),
                                           _stream(stream)), "power_filter_block")
        return y

    def cg_filter_block(self, x0, kmax, tol=0.0, out=None, ws=None, info=True, stream=None):
        """CG filter of every column of an n x m block (gsf_cg_filter_block);
        returns (y, list of m CgInfo or None)."""
        torch = _torch()
        m = x0.shape[1]
        y = out if out is not None else torch.empty_like(x0)
        ws = ws if ws is not None else self.workspace(METHOD_CG, m)
        infos = (CgInfo * m)()
        st = _lib.gsf_cg_filter_block(self.handle, m, _ptr(x0), _ptr(y), kmax, tol, _ptr(ws), ws.numel(),
                                      infos if info else None, _stream(stream))
        _check(st, "cg_filter_block")
        return y, (list(infos) if info else None)

    def joint_workspace(self, m):
        torch = _torch()
        nbytes = ctypes.c_size_t()
        _check(_lib.gsf_joint_workspace_bytes(self.handle, m, ctypes.byref(nbytes)), "joint_workspace_bytes")
        return torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device="cuda")

    def joint_filter(self, x0_cg, kmax_cg, x0_lob, m, kmax_lob, constraint=False, out_cg=None, out_lob=None,
                     ws=None, info=True, stream=None):
        """CG and LOBPCG filters side by side (gsf_joint_filter); returns
        (x_cg, x_lob, CgInfo or None, LobpcgInfo or None)."""
        torch = _torch()
        ycg = out_cg if out_cg is not None else torch.empty_like(x0_cg)
        ylob = out_lob if out_lob is not None else torch.empty_like(x0_lob)
        ws = ws if ws is not None else self.joint_workspace(m)
        ci, li = CgInfo(), LobpcgInfo()
        st = _lib.gsf_joint_filter(self.handle, _ptr(x0_cg), _ptr(ycg), kmax_cg, _ptr(x0_lob), _ptr(ylob), m,
                                   kmax_lob, int(bool(constraint)), _ptr(ws), ws.numel(),
                                   ctypes.byref(ci) if info else None, ctypes.byref(li) if info else None,
                                   _stream(stream))
        _check(st, "joint_filter")
        return ycg, ylob, (ci if info else None), (li if info else None)

    def cg_filter(self, x0, kmax, tol=0.0, out=None, ws=None, info=True, stream=None):
        torch = _torch()
        y = out if out is not None else torch.empty_like(x0)
        ws = ws if ws is not None else self.workspace(METHOD_CG)
        inf = CgInfo()
        st = _lib.gsf_cg_filter(self.handle, _ptr(x0), _ptr(y), kmax, tol, _ptr(ws), ws.numel(),
                                ctypes.byref(inf) if info else None, _stream(stream))
        _check(st, "cg_filter")
        return y, (inf if info else None)

    def cg_filter_noalloc(self, x0, kmax, tol=0.0, out=None, info=True, stream=None):
        """gsf_cg_filter_noalloc: the CG filter in the library's static scratch."""
        torch = _torch()
        y = out if out is not None else torch.empty_like(x0)
        inf = CgInfo()
        st = _lib.gsf_cg_filter_noalloc(self.handle, _ptr(x0), _ptr(y), kmax, tol,
                                        ctypes.byref(inf) if info else None, _stream(stream))
        _check(st, "cg_filter_noalloc")
        return y, (inf if info else None)

    def lobpcg_filter(self, x0, m, kmax, tol=0.0, constraint=False, out=None, ritz=None, ws=None, info=True,
                      stream=None, precond=None, ritz_vals=None):
        """ritz_vals: None or a ctypes array of m doubles that receives the
        Ritz values (gsf_lobpcg_filter's ritz_vals_host)."""
        torch = _torch()
        y = out if out is not None else torch.empty_like(x0)
        ws = ws if ws is not None else self.workspace(METHOD_LOBPCG, m)
        inf = LobpcgInfo()
        st = _lib.gsf_lobpcg_filter(self.handle, _ptr(x0), _ptr(y), m, kmax, tol, int(bool(constraint)),
                                    precond.handle if precond is not None else None,
                                    _ptr(ritz) if ritz is not None else None,
                                    ritz_vals if ritz_vals is not None else None, _ptr(ws), ws.numel(),
                                    ctypes.byref(inf) if info else None, _stream(stream))
        _check(st, "lobpcg_filter")
        return y, (inf if info else None)

    def shifted_cg(self, alpha, b, kmax, tol, ldb=1, out=None, ws=None, info=True, stream=None):
        """y = (L_sym + alpha I)^-1 b by CG (b: n values at stride ldb)."""
        torch = _torch()
        y = out if out is not None else torch.empty(self.n, dtype=self.dtype, device="cuda")
        ws = ws if ws is not None else self.workspace(METHOD_CG)
        inf = CgInfo()
        st = _lib.gsf_shifted_cg(self.handle, alpha, _ptr(b), ldb, _ptr(y), kmax, tol, _ptr(ws), ws.numel(),
                                 ctypes.byref(inf) if info else None, _stream(stream))
        _check(st, "shifted_cg")
        return y, (inf if info else None)

    def lobpcg_residual(self, X, theta, out=None, stream=None):
        """R = L_sym X - X diag(theta) for an n x m block."""
        torch = _torch()
        m = X.shape[1]
        R = out if out is not None else torch.empty_like(X)
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64)[:m])
        _check(_lib.gsf_lobpcg_residual(self.handle, m, _ptr(X), th.ctypes.data_as(ctypes.c_void_p), _ptr(R),
                                        _stream(stream)), "lobpcg_residual")
        return R

    def make_pair(self, r, y, g, inputs, targets, ldr=1, ldy=1, stream=None):
        """Training pair (r/s, g), y/s into FP32 views inputs (2n), targets (n)."""
        torch = _torch()
        nbytes = ctypes.c_size_t()
        _check(_lib.gsf_net_pair_workspace_bytes(self.handle, ctypes.byref(nbytes)), "net_pair_workspace_bytes")
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
        _check(_lib.gsf_net_make_pair(self.handle, _ptr(r), ldr, _ptr(y), ldy, _ptr(g), _ptr(inputs),
                                      _ptr(targets), _ptr(ws), ws.numel(), _stream(stream)), "net_make_pair")
        return ws  # caller keeps it alive until the stream has run


NET_WEIGHTS = 2736


class Precond:
    """Learned preconditioner handle (gsf_precond_create): borrows the
    operator grid, the guidance tensor and the BF16 weight tensor (uint16 or
    bfloat16 storage), which must stay alive.  Precond.shifted(op, alpha,
    inner) is the shifted-solve reference T (gsf_precond_create_shifted)."""

    @classmethod
    def shifted(cls, op, alpha, inner):
        lib = load_library()
        self = cls.__new__(cls)
        self.op, self.g, self.w = op, None, None
        h = ctypes.c_void_p()
        _check(lib.gsf_precond_create_shifted(op.handle, float(alpha), int(inner), ctypes.byref(h)),
               "precond_create_shifted")
        self.handle = h
        return self

    def __init__(self, op, guidance, w_bf16):
        lib = load_library()
        torch = _torch()
        g = guidance.to(device="cuda", dtype=op.dtype).contiguous().reshape(-1)
        if g.numel() != op.n or w_bf16.numel() != NET_WEIGHTS or not w_bf16.is_cuda:
            raise ValueError("guidance / weights do not match")
        self.op, self.g, self.w = op, g, w_bf16
        h = ctypes.c_void_p()
        _check(lib.gsf_precond_create(op.handle, _ptr(g), _ptr(w_bf16), ctypes.byref(h)), "precond_create")
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gsf_precond_destroy(self.handle)
            self.handle = None

    def apply(self, R, out=None, stream=None):
        torch = _torch()
        m = 1 if R.dim() == 1 else R.shape[1]
        W = out if out is not None else torch.empty_like(R)
        nbytes = ctypes.c_size_t()
        _check(_lib.gsf_precond_workspace_bytes(self.handle, m, ctypes.byref(nbytes)), "precond_workspace_bytes")
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
        _check(_lib.gsf_precond_apply(self.handle, m, _ptr(R), _ptr(W), _ptr(ws), ws.numel(), _stream(stream)),
               "precond_apply")
        self._ws = ws
        return W


class NetTrainer:
    """Device state of the network's training: FP32 master weights, Adam
    moments, the BF16 copy and the scratch of the loss / gradient kernels."""

    def __init__(self, w_init, batch, rows, cols):
        torch = _torch()
        lib = load_library()
        w = torch.as_tensor(np.asarray(w_init, dtype=np.float32)).to("cuda")
        if w.numel() != NET_WEIGHTS:
            raise ValueError("weight vector has the wrong length")
        self.w = w.contiguous()
        self.mom = torch.zeros_like(self.w)
        self.vel = torch.zeros_like(self.w)
        self.grad = torch.zeros_like(self.w)
        self.wb = torch.empty(NET_WEIGHTS, dtype=torch.int16, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.batch, self.rows, self.cols = batch, rows, cols
        nbytes = ctypes.c_size_t()
        _check(lib.gsf_net_workspace_bytes(batch, rows, cols, ctypes.byref(nbytes)), "net_workspace_bytes")
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
        self.t = 0
        _check(lib.gsf_net_to_bf16(NET_WEIGHTS, _ptr(self.w), _ptr(self.wb), _stream()), "net_to_bf16")

    def loss_grad(self, idx, inputs, targets, stream=None):
        """loss (device double) and grad for the samples idx (int32 device)."""
        _check(_lib.gsf_net_loss_grad(_ptr(self.wb), idx.numel(), _ptr(idx), self.rows, self.cols, _ptr(inputs),
                                      _ptr(targets), _ptr(self.grad), _ptr(self.loss), _ptr(self.ws),
                                      self.ws.numel(), _stream(stream)), "net_loss_grad")
        return self.loss, self.grad

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.t += 1
        _check(_lib.gsf_net_adam(NET_WEIGHTS, self.t, lr, b1, b2, eps, _ptr(self.w), _ptr(self.mom), _ptr(self.vel),
                                 _ptr(self.grad), _ptr(self.wb), _stream(stream)), "net_adam")

    def forward(self, idx, inputs, stream=None):
        torch = _torch()
        y = torch.empty(idx.numel() * self.rows * self.cols, dtype=torch.float32, device="cuda")
        nbytes = ctypes.c_size_t()
        _check(_lib.gsf_net_workspace_bytes(idx.numel(), self.rows, self.cols, ctypes.byref(nbytes)),
               "net_workspace_bytes")
        ws = self.ws if nbytes.value <= self.ws.numel() else torch.empty(int(nbytes.value), dtype=torch.uint8,
                                                                         device="cuda")
        _check(_lib.gsf_net_forward(_ptr(self.wb), idx.numel(), _ptr(idx), self.rows, self.cols, _ptr(inputs),
                                    _ptr(y), _ptr(ws), ws.numel(), _stream(stream)), "net_forward")
        return y


def tune_table_save(path):
    """Write the tuned apply tiles to a JSON file (gsf_tune_table_save); returns the entry count."""
    lib = load_library()
    n = ctypes.c_int()
    _check(lib.gsf_tune_table_save(os.fsencode(path), ctypes.byref(n)), "tune_table_save")
    return n.value


def tune_table_load(path):
    """Read tuned apply tiles from a JSON file (gsf_tune_table_load); returns the entry count."""
    lib = load_library()
    n = ctypes.c_int()
    _check(lib.gsf_tune_table_load(os.fsencode(path), ctypes.byref(n)), "tune_table_load")
    return n.value


def tune_table_clear():
    load_library().gsf_tune_table_clear()


def build_operator(kind, shape, guidance, radius, sigma_d=0.0, sigma_r=0.0, eps=0.0, prec=F32, stream=None):
    return Operator(kind, shape, guidance, radius, sigma_d, sigma_r, eps, prec, stream)


def block_gram(S_blocks, AS_blocks, prec=F32, stream=None):
    """(S^T A S, S^T S) through the MFMA Gram kernel; S_blocks/AS_blocks are
    lists of n x m device tensors."""
    torch = _torch()
    lib = load_library()
    n, m = S_blocks[0].shape
    nb = len(S_blocks)
    need = ctypes.c_size_t()
    _check(lib.gsf_block_gram_workspace_bytes(n, ctypes.byref(need)), "block_gram_workspace_bytes")
    ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
    sp = (ctypes.c_void_p * 3)(*[b.data_ptr() for b in S_blocks] + [0] * (3 - nb))
    ap = (ctypes.c_void_p * 3)(*[b.data_ptr() for b in AS_blocks] + [0] * (3 - nb))
    ns = nb * m
    GA = np.zeros((ns, ns))
    GB = np.zeros((ns, ns))
    _check(lib.gsf_block_gram(prec, n, m, nb, sp, ap, GA.ctypes.data_as(ctypes.c_void_p),
                              GB.ctypes.data_as(ctypes.c_void_p), _ptr(ws), ws.numel(), _stream(stream)),
           "block_gram")
    return GA, GB


def rayleigh_ritz(GA, GB, m, drop_tol, zero_tol=0.0, stream=None):
    """Device FP64 Rayleigh-Ritz step on a host Gram pair."""
    torch = _torch()
    lib = load_library()
    ns = GA.shape[0]
    GA = np.ascontiguousarray(GA, dtype=np.float64)
    GB = np.ascontiguousarray(GB, dtype=np.float64)
    theta = np.zeros(m)
    C = np.zeros((ns, m))
    kept = np.zeros(ns, dtype=np.int32)
    nkept = np.zeros(1, dtype=np.int32)
    ws = torch.empty(int(lib.gsf_rr_workspace_bytes()), dtype=torch.uint8, device="cuda")
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib.gsf_rayleigh_ritz(ns, m, vp(GA), vp(GB), drop_tol, zero_tol, vp(theta), vp(C), vp(kept), vp(nkept),
                                 _ptr(ws), ws.numel(), _stream(stream)), "rayleigh_ritz")
    return theta, C, kept.astype(bool), int(nkept[0])
