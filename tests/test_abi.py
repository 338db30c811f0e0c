"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/gsf.h, and validates arguments before
touching the device."""
import ctypes
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsf.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsf_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1509_02468_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libgsf.so not built")
    return pkg.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_status_strings(lib):
    assert lib.gsf_version() >= 1
    assert lib.gsf_status_string(0) == b"ok"
    assert lib.gsf_status_string(99) == b"unknown status"
    # no device error recorded in this thread; HIP's text for a code
    assert lib.gsf_last_device_error() == 0
    assert lib.gsf_device_error_string(0) == b"no error"


def _desc(**kw):
    from paper_1509_02468_amd.gsf import OperatorDesc
    d = OperatorDesc()
    d.kind, d.ndim, d.prec, d.radius = kw.get("kind", 0), kw.get("ndim", 2), kw.get("prec", 0), kw.get("radius", 5)
    d.dims[0], d.dims[1] = kw.get("dims", (64, 80))
    d.sigma_d, d.sigma_r, d.gf_eps = kw.get("sigma_d", 2.0), kw.get("sigma_r", 0.1), kw.get("eps", 0.01)
    d.stencil, d.norm = kw.get("stencil", 0), kw.get("norm", 0)
    d.channels, d.reserved = kw.get("channels", 0), kw.get("reserved", 0)
    return d


def test_operator_workspace_sizes(lib):
    n = 64 * 80
    sz = ctypes.c_size_t()
    assert lib.gsf_operator_workspace_bytes(ctypes.byref(_desc()), ctypes.byref(sz)) == 0
    # 60 half-window planes + diag + sqrt(d) in FP32, + FP64 degrees
    assert sz.value >= (60 + 2) * n * 4 + n * 8
    assert lib.gsf_operator_workspace_bytes(ctypes.byref(_desc(prec=1)), ctypes.byref(sz)) == 0
    assert sz.value >= (60 + 2) * n * 8 + n * 8
    assert lib.gsf_operator_workspace_bytes(ctypes.byref(_desc(kind=1, radius=8)), ctypes.byref(sz)) == 0
    assert sz.value >= 8 * n * 4 + n * 8


@pytest.mark.parametrize("bad", [dict(radius=0), dict(radius=9), dict(ndim=3), dict(kind=2), dict(prec=5),
                                 dict(dims=(0, 5)), dict(sigma_r=0.0), dict(sigma_d=-1.0),
                                 dict(sigma_r=float("nan")), dict(kind=1, eps=-1.0),
                                 dict(kind=1, eps=float("inf")), dict(stencil=2), dict(stencil=-1),
                                 dict(norm=2), dict(kind=1, stencil=1), dict(kind=1, norm=1),
                                 dict(channels=-1), dict(channels=9), dict(kind=1, channels=3),
                                 dict(reserved=1)])
def test_invalid_descriptors_rejected(lib, bad):
    sz = ctypes.c_size_t()
    assert lib.gsf_operator_workspace_bytes(ctypes.byref(_desc(**bad)), ctypes.byref(sz)) == 1


def test_descriptor_layout_matches_header():
    """The ctypes struct matches gsf_operator_desc: 72 bytes with the stencil,
    norm, channels and reserved fields last."""
    from paper_1509_02468_amd.gsf import OperatorDesc
    assert ctypes.sizeof(OperatorDesc) == 72
    assert OperatorDesc.stencil.offset == 56 and OperatorDesc.norm.offset == 60
    assert OperatorDesc.channels.offset == 64 and OperatorDesc.reserved.offset == 68


def test_cross_stencil_workspace(lib):
    """2D cross: 2r planes instead of ((2r+1)^2 - 1)/2; 1D cross = square."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.gsf_operator_workspace_bytes(ctypes.byref(_desc(radius=2, stencil=1)), ctypes.byref(a)) == 0
    assert lib.gsf_operator_workspace_bytes(ctypes.byref(_desc(radius=2)), ctypes.byref(b)) == 0
    n = 64 * 80
    assert a.value < b.value and a.value >= (4 + 2) * n * 4 + n * 8
    assert b.value - a.value >= (12 - 4) * n * 4
    assert lib.gsf_operator_workspace_bytes(ctypes.byref(_desc(ndim=1, dims=(500, 1), radius=3, stencil=1)),
                                            ctypes.byref(a)) == 0
    assert lib.gsf_operator_workspace_bytes(ctypes.byref(_desc(ndim=1, dims=(500, 1), radius=3)),
                                            ctypes.byref(b)) == 0
    assert a.value == b.value


def test_size_limits(lib):
    """BF: fewer than 2^30 points and the padded plane addressable with 32-bit
    byte offsets ((n + r (W + 1)) * element size <= 2^32); GF: fewer than 2^27."""
    sz = ctypes.c_size_t()

    def ok(**kw):
        return lib.gsf_operator_workspace_bytes(ctypes.byref(_desc(**kw)), ctypes.byref(sz)) == 0
    assert ok(dims=(1 << 14, (1 << 16) - 64), prec=0)         # 2^30 - 2^20 points, FP32
    assert not ok(dims=(1 << 15, 1 << 15), prec=0)            # 2^30 points
    assert ok(dims=(1 << 14, (1 << 15) - 64), prec=1)         # 2^29 - 2^20 points, FP64
    assert not ok(dims=(1 << 14, (1 << 15) + 8), prec=1)      # above 2^29, FP64
    assert not ok(ndim=1, dims=((1 << 29) + 1, 1), prec=1)
    assert ok(ndim=1, dims=((1 << 29) - 8, 1), prec=1)
    assert ok(kind=1, dims=(1 << 13, (1 << 14) - 1))
    assert not ok(kind=1, dims=(1 << 13, 1 << 14))


def test_reguided_argument_checks(lib):
    """The re-guided filter validates before any device work."""
    sz = ctypes.c_size_t()
    d = _desc()
    assert lib.gsf_reguided_workspace_bytes(ctypes.byref(d), 2, ctypes.byref(sz)) == 1   # LOBPCG: no
    assert lib.gsf_reguided_workspace_bytes(ctypes.byref(d), 0, ctypes.byref(sz)) == 0
    power = sz.value
    assert lib.gsf_reguided_workspace_bytes(ctypes.byref(d), 1, ctypes.byref(sz)) == 0
    # BF: the passes evaluate the weights where they use them, so the power
    # filter's workspace is the degrees (FP64) and one vector, no weight planes
    assert sz.value > power >= 64 * 80 * (8 + 4) and power < 64 * 80 * 16 + 2 * 256
    assert lib.gsf_reguided_workspace_bytes(ctypes.byref(_desc(radius=0)), 1, ctypes.byref(sz)) == 1
    fake = ctypes.c_void_p(0x1000)
    assert lib.gsf_reguided_filter(ctypes.byref(d), 1, None, fake, 5, 0.0, fake, 1 << 30, None, None) == 1
    assert lib.gsf_reguided_filter(ctypes.byref(d), 1, fake, fake, -1, 0.0, fake, 1 << 30, None, None) == 1
    assert lib.gsf_reguided_filter(ctypes.byref(d), 1, fake, fake, 5, -1.0, fake, 1 << 30, None, None) == 1
    assert lib.gsf_reguided_filter(ctypes.byref(d), 3, fake, fake, 5, 0.0, fake, 1 << 30, None, None) == 1
    assert lib.gsf_reguided_filter(ctypes.byref(d), 1, fake, fake, 5, 0.0, fake, 16, None, None) == 2


def test_build_rejects_small_workspace_and_nulls(lib):
    d = _desc()
    out = ctypes.c_void_p()
    # NULL guidance / workspace: EINVAL before any device call
    assert lib.gsf_build_operator(ctypes.byref(d), None, None, 0, None, ctypes.byref(out)) == 1
    # non-null fake pointers with a too small size: ENOMEM (nothing is launched)
    fake = ctypes.c_void_p(0x1000)
    assert lib.gsf_build_operator(ctypes.byref(d), fake, fake, 16, None, ctypes.byref(out)) == 2


def test_solver_calls_reject_null_operator(lib):
    sz = ctypes.c_size_t()
    assert lib.gsf_solver_workspace_bytes(None, 1, 1, ctypes.byref(sz)) == 1
    assert lib.gsf_apply(None, 0, 1, None, 0, None, 0, None) == 1
    assert lib.gsf_rr_workspace_bytes() > 0


def test_gram_workspace_query(lib):
    sz = ctypes.c_size_t()
    assert lib.gsf_block_gram_workspace_bytes(ctypes.c_int64(1 << 20), ctypes.byref(sz)) == 0
    assert sz.value > 0
    assert lib.gsf_block_gram_workspace_bytes(ctypes.c_int64(0), ctypes.byref(sz)) == 1


def test_learned_preconditioner_argument_checks(lib):
    """The network and training entry points validate before touching the
    device (EINVAL = 1, ENOMEM = 2)."""
    sz = ctypes.c_size_t()
    assert lib.gsf_net_workspace_bytes(0, 64, 64, ctypes.byref(sz)) == 1
    assert lib.gsf_net_workspace_bytes(16, 0, 64, ctypes.byref(sz)) == 1
    assert lib.gsf_net_workspace_bytes(16, 512, 512, ctypes.byref(sz)) == 0
    # a1, a2 (BF16 x 16) + dz1, dz2 (FP32 x 16) + y, dy per pixel
    assert sz.value >= 16 * 512 * 512 * (2 * 32 + 2 * 64 + 2 * 4)
    v = ctypes.c_void_p(16)
    assert lib.gsf_net_forward(None, 1, v, 8, 8, v, v, v, 1 << 30, None) == 1
    assert lib.gsf_net_forward(v, 1, v, 8, 8, v, v, v, 16, None) == 2
    assert lib.gsf_net_loss_grad(v, 0, v, 8, 8, v, v, v, v, v, 1 << 30, None) == 1
    assert lib.gsf_net_adam(0, 1, 1e-3, 0.9, 0.999, 1e-8, v, v, v, v, v, None) == 1
    assert lib.gsf_net_adam(10, 0, 1e-3, 0.9, 0.999, 1e-8, v, v, v, v, v, None) == 1
    assert lib.gsf_net_adam(10, 1, 1e-3, 1.0, 0.999, 1e-8, v, v, v, v, v, None) == 1
    assert lib.gsf_net_to_bf16(0, v, v, None) == 1
    h = ctypes.c_void_p()
    assert lib.gsf_precond_create(None, v, v, ctypes.byref(h)) == 1
    d = ctypes.c_double
    assert lib.gsf_precond_create_shifted(None, d(1e-2), 10, ctypes.byref(h)) == 1
    assert lib.gsf_precond_create_shifted(v, d(0.0), 10, ctypes.byref(h)) == 1
    assert lib.gsf_precond_create_shifted(v, d(float("nan")), 10, ctypes.byref(h)) == 1
    assert lib.gsf_precond_create_shifted(v, d(1e-2), 0, ctypes.byref(h)) == 1
    assert lib.gsf_precond_create_shifted(v, d(1e-2), 10, None) == 1
    assert lib.gsf_precond_workspace_bytes(None, 4, ctypes.byref(sz)) == 1
    assert lib.gsf_precond_apply(None, 4, v, v, v, 1 << 30, None) == 1
    assert lib.gsf_shifted_cg(None, 1e-2, v, 1, v, 10, 1e-10, v, 1 << 30, None, None) == 1
    assert lib.gsf_lobpcg_residual(None, 4, v, v, v, None) == 1
    assert lib.gsf_net_make_pair(None, v, 1, v, 1, v, v, v, v, 1 << 30, None) == 1
    assert lib.gsf_net_pair_workspace_bytes(None, ctypes.byref(sz)) == 1


def test_block_and_colour_argument_checks(lib):
    """Host-side validation of the multi-channel entry points (no launch)."""
    sz = ctypes.c_size_t()
    assert lib.gsf_srgb_to_lab(0, -1, None, None, None) == 1
    assert lib.gsf_srgb_to_lab(2, 10, None, None, None) == 1
    assert lib.gsf_srgb_to_lab(0, 0, None, None, None) == 0
    assert lib.gsf_srgb_to_lab(0, 10, None, None, None) == 1
    assert lib.gsf_power_filter_block(None, 3, None, None, 5, None, 0, None) == 1
    assert lib.gsf_cg_filter_block(None, 3, None, None, 5, 0.0, None, 0, None, None) == 1
    d = _desc(channels=3)
    assert lib.gsf_reguided_workspace_bytes(ctypes.byref(d), 0, ctypes.byref(sz)) == 1
    assert lib.gsf_operator_workspace_bytes(ctypes.byref(d), ctypes.byref(sz)) == 0


def test_joint_argument_checks(lib):
    sz = ctypes.c_size_t()
    assert lib.gsf_joint_workspace_bytes(None, 4, ctypes.byref(sz)) == 1
    assert lib.gsf_joint_filter(None, None, None, 5, None, None, 4, 5, 0, None, 0, None, None, None) == 1


def test_identity_weights_layout():
    """The package's identity network is the oracle's (same weight layout:
    W1 [16][2][3][3], W2 [16][16][3][3], W3 [16][3][3])."""
    from oracle import convnet as cn
    from paper_1509_02468_amd import learned
    assert np.array_equal(learned.identity_weights().astype(np.float64), cn.identity_weights())


def test_tune_table_json_round_trip(lib, tmp_path):
    """The tuned-tile table survives a save / clear / load cycle through its
    JSON file; malformed or out-of-range files are rejected and leave the
    table unchanged (host only: no operator, no device)."""
    import json
    import paper_1509_02468_amd as pkg
    pkg.tune_table_clear()
    src = tmp_path / "tiles.json"
    entries = [dict(prec=0, geometry=1, radius=5, width=4, size_class=1, rows_per_thread=2),
               dict(prec=1, geometry=0, radius=3, width=1, size_class=3, rows_per_thread=4)]
    src.write_text(json.dumps({"gsf_apply_tiles": entries}))
    assert pkg.tune_table_load(str(src)) == 2
    out = tmp_path / "saved.json"
    assert pkg.tune_table_save(str(out)) == 2
    key = lambda e: tuple(e[k] for k in ("prec", "geometry", "radius", "width", "size_class"))
    assert sorted(json.loads(out.read_text())["gsf_apply_tiles"], key=key) == sorted(entries, key=key)
    for bad in ({"gsf_apply_tiles": [dict(entries[0], rows_per_thread=3)]},
                {"gsf_apply_tiles": [dict(entries[0], width=5)]},
                {"gsf_apply_tiles": [{"prec": 0, "geometry": 1}]},
                {"tiles": entries}):
        src.write_text(json.dumps(bad))
        with pytest.raises(pkg.GsfError):
            pkg.tune_table_load(str(src))
    assert pkg.tune_table_save(str(out)) == 2
    with pytest.raises(pkg.GsfError):
        pkg.tune_table_load(str(tmp_path / "missing.json"))
    assert lib.gsf_tune_table_save(None, None) == 1
    pkg.tune_table_clear()
    assert pkg.tune_table_save(str(out)) == 0
    assert json.loads(out.read_text()) == {"gsf_apply_tiles": []}
