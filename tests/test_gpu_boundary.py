"""Call shapes of the C ABI: gsf_apply on strided column slices of wider
point-major arrays (ldx, ldy), the Ritz values returned to the host by
gsf_lobpcg_filter, and the single-call gsf_batch_filter, each against the
plain form of the same call (bitwise: the same kernels run)."""
import ctypes

import numpy as np
import pytest

from synth import batch_items, item_signal, piecewise_constant_1d, scene_2d

pytestmark = pytest.mark.gpu


def _dev(x, prec, gsf):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float32 if prec == gsf.F32 else torch.float64,
                        device="cuda")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,shape,par", [
    ("bf", (67, 130), dict(radius=5, sigma_d=2.0, sigma_r=0.1)),
    ("bf", (40, 90), dict(radius=1, sigma_d=1.0, sigma_r=0.1, stencil="cross", norm="diagl")),
    ("bf", (3000,), dict(radius=4, sigma_d=3.0, sigma_r=0.2)),
    ("gf", (70, 131), dict(radius=3, eps=1e-2)),
])
def test_apply_on_column_slices(gsf, kind, shape, par, prec):
    """y[:, 2:2+m] = F x[:, 1:1+m] with ldx = 6, ldy = 7 equals the dense
    apply of the same columns, and the other columns of y stay untouched."""
    import torch
    g = piecewise_constant_1d(shape[0], 0.1, 5)[1] if len(shape) == 1 else scene_2d(*shape, 0.05, 5)[1]
    op = gsf.Operator(kind, shape, _dev(g.ravel(), prec, gsf), prec=prec, **par)
    n = op.n
    X = _dev(np.random.default_rng(1).standard_normal((n, 6)), prec, gsf)
    for m in (1, 3, 4):
        Y = torch.full((n, 7), float("nan"), dtype=X.dtype, device="cuda")
        for form in (gsf.FORM_N, gsf.FORM_LSYM, gsf.FORM_RW, gsf.FORM_L):
            op.apply(X[:, 1:1 + m], form, out=Y[:, 2:2 + m])
            ref = op.apply(X[:, 1:1 + m].contiguous(), form)
            assert torch.equal(Y[:, 2:2 + m], ref), (form, m)
        assert bool(torch.isnan(Y[:, :2]).all()) and bool(torch.isnan(Y[:, 2 + m:]).all())


def test_apply_rejects_short_strides_and_overlap(gsf):
    import torch
    g = scene_2d(40, 50, 0.05, 6)[1]
    op = gsf.Operator("bf", (40, 50), _dev(g.ravel(), 1, gsf), radius=2, sigma_d=2.0, sigma_r=0.1, prec=1)
    X = torch.zeros((op.n, 4), dtype=torch.float64, device="cuda")
    lib = gsf.load_library()
    # ldx below m
    assert lib.gsf_apply(op.handle, 0, 4, X.data_ptr(), 3, X.data_ptr(), 4, None) == gsf.EINVAL
    # output columns inside the input's extent
    assert lib.gsf_apply(op.handle, 0, 2, X.data_ptr(), 4, X.data_ptr() + 16, 4, None) == gsf.EINVAL


@pytest.mark.parametrize("prec", [0, 1])
def test_lobpcg_ritz_values_to_host(gsf, prec):
    g = scene_2d(50, 60, 0.05, 7)[1]
    op = gsf.Operator("bf", (50, 60), _dev(g.ravel(), prec, gsf), radius=3, sigma_d=2.0, sigma_r=0.1, prec=prec)
    x = _dev(g.ravel(), prec, gsf)
    vals = (ctypes.c_double * 4)()
    y, info = op.lobpcg_filter(x, 4, 12, ritz_vals=vals)
    y2, info2 = op.lobpcg_filter(x, 4, 12)
    assert list(vals) == list(info.theta[:4]) == list(info2.theta[:4])
    assert np.array_equal(y.cpu().numpy(), y2.cpu().numpy())
    vals2 = (ctypes.c_double * 3)()
    op.lobpcg_filter(x, 3, 8, info=False, ritz_vals=vals2)   # no info: the values alone
    assert list(vals2) == list(op.lobpcg_filter(x, 3, 8)[1].theta[:3])


def test_batch_filter_single_call(gsf):
    """gsf_batch_filter equals a plan created, run and read without
    autotuning (same kernels: bitwise), with the same per-item info."""
    import torch
    recipe = batch_items(seed=45, n_images=6, n_signals=3, side_range=(24, 120), len_range=(300, 3000))
    items, items2 = [], []
    for it in recipe:
        _, noisy = item_signal(it)
        gd = torch.tensor(noisy.ravel(), dtype=torch.float32, device="cuda")
        d = dict(kind=it["kind"], shape=it["shape"], radius=it["radius"], sigma_d=it["sigma_d"],
                 sigma_r=it["sigma_r"], eps=it["eps"], guidance=gd, x0=gd, method=it["method"], m=it["m"], kmax=10,
                 tol=it["tol"])
        items.append(dict(d))
        items2.append(dict(d))
    info = gsf.batch_filter(items, prec=gsf.F32)
    b = gsf.Batch(items2, prec=gsf.F32, autotune=False)
    b.run()
    torch.cuda.synchronize()
    assert info == b.info()
    for a, c in zip(items, items2):
        assert torch.equal(a["out"], c["out"])
