"""GPU checks at the full sizes of the named workloads, in the launch
configurations the benchmark uses (every BF apply tile height, the tuned one
included), on sampled outputs that the oracle computes point by point from
eq. (2) / Algorithm 1, and on properties that hold at any size for the CG and
LOBPCG filters.

Tolerances: FP32 data, normwise over the sampled outputs, 1e-5 (inputs are
rounded to FP32 before the oracle sees them, so the comparison measures the
kernels' arithmetic); FP64 data 1e-12.
"""
import numpy as np
import pytest

from oracle.pointwise import bf_lsym_at, gf_lsym_at, sample_points
from synth import make_signal, WORKLOADS

pytestmark = pytest.mark.gpu


def nrel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _op(gsf, name, prec):
    import torch
    w = WORKLOADS[name]
    _, x = make_signal(name)
    if prec == gsf.F32:
        x = x.astype(np.float32).astype(np.float64)
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    xd = torch.tensor(x.ravel(), dtype=dt, device="cuda")
    op = gsf.Operator(w["kind"], w["shape"], xd, w["radius"], w["sigma_d"], w["sigma_r"], w["eps"], prec)
    return op, x, xd, w


def _block(gsf, n, m, prec, seed):
    import torch
    z = np.random.default_rng(seed).standard_normal((n, m))
    if prec == gsf.F32:
        z = z.astype(np.float32).astype(np.float64)
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    return z, torch.tensor(z, dtype=dt, device="cuda")


@pytest.mark.parametrize("rows", [1, 2, 4])
@pytest.mark.parametrize("m", [1, 4])
def test_bf11_1024_apply_sampled(gsf, m, rows):
    """The benchmark's operator (1024^2, BF 11x11, FP32), every tile height."""
    op, x, _, w = _op(gsf, "image_1024_bf11", gsf.F32)
    op.set_apply_rows(m, rows)
    z, zd = _block(gsf, op.n, m, gsf.F32, 11 + m)
    y = op.apply(zd if m > 1 else zd[:, 0].contiguous(), gsf.FORM_LSYM).cpu().numpy().reshape(op.n, m)
    pts = sample_points(w["shape"], 96, 12)
    ref = bf_lsym_at(x, z, pts, w["radius"], w["sigma_d"], w["sigma_r"])
    e = nrel(y[pts], ref)
    print(f"bf11 1024^2 m={m} rows={rows}: {e:.2e}")
    assert e <= 1e-5


def test_bf11_1024_apply_tuned_tile(gsf):
    """The tile the benchmark picks (the tuner's choice) for m = 1 and 4."""
    op, x, _, w = _op(gsf, "image_1024_bf11", gsf.F32)
    pts = sample_points(w["shape"], 64, 13)
    for m in (1, 4):
        best, _ = op.tune_apply(m, reps=5)
        z, zd = _block(gsf, op.n, m, gsf.F32, 20 + m)
        y = op.apply(zd if m > 1 else zd[:, 0].contiguous(), gsf.FORM_LSYM).cpu().numpy().reshape(op.n, m)
        e = nrel(y[pts], bf_lsym_at(x, z, pts, w["radius"], w["sigma_d"], w["sigma_r"]))
        print(f"tuned m={m} rows={best}: {e:.2e}")
        assert e <= 1e-5


@pytest.mark.parametrize("prec", [0, 1])
def test_bf7_4096_apply_sampled(gsf, prec):
    """The precision-study BF operator at 4096^2 (7x7), m = 8."""
    op, x, _, w = _op(gsf, "image_4096_bf7", prec)
    z, zd = _block(gsf, op.n, 8, prec, 31)
    y = op.apply(zd, gsf.FORM_LSYM).cpu().numpy()
    pts = sample_points(w["shape"], 48, 32)
    e = nrel(y[pts], bf_lsym_at(x, z, pts, w["radius"], w["sigma_d"], w["sigma_r"]))
    print(f"bf7 4096^2 prec {prec}: {e:.2e}")
    assert e <= (1e-5 if prec == 0 else 1e-12)


@pytest.mark.parametrize("prec,m", [(0, 1), (0, 8), (1, 4)])
def test_gf8_4096_apply_sampled(gsf, prec, m):
    """The precision-study GF operator at 4096^2 (radius 8, eps 1e-2)."""
    op, x, _, w = _op(gsf, "image_4096_gf8", prec)
    z, zd = _block(gsf, op.n, m, prec, 41 + m)
    y = op.apply(zd if m > 1 else zd[:, 0].contiguous(), gsf.FORM_LSYM).cpu().numpy().reshape(op.n, m)
    pts = sample_points(w["shape"], 40, 42)
    e = nrel(y[pts], gf_lsym_at(x, z, pts, w["radius"], w["eps"]))
    print(f"gf8 4096^2 prec {prec} m {m}: {e:.2e}")
    assert e <= (1e-5 if prec == 0 else 1e-12)


def test_cg_1024_properties(gsf):
    """CG(50) on the benchmark workload: the D-weighted mean is kept (the
    constant is the null vector of L, so every update is D-orthogonal to it)
    and the energy x^T L x decreases; the reported residuals are consistent."""
    import torch
    op, x, xd, w = _op(gsf, "image_1024_bf11", gsf.F32)
    out, info = op.cg_filter(xd, 50)
    d = op.degree().cpu().numpy()
    xo = out.double().cpu().numpy()
    mass0, mass1 = float(np.sum(d * x.ravel())), float(np.sum(d * xo))
    assert abs(mass1 - mass0) <= 1e-5 * float(np.sum(np.abs(d * x.ravel())))
    sq = op.sqrt_d()

    def energy(v):
        z = (sq * v).contiguous()
        return float((z.double() * op.apply(z, gsf.FORM_LSYM).double()).sum())
    e0, e1 = energy(xd), energy(out)
    print(f"cg 1024^2: energy {e0:.4e} -> {e1:.4e}, res {info.res0:.3e} -> {info.res:.3e}")
    assert e1 < 0.2 * e0 and info.res < info.res0 and info.iters == 50


def test_lobpcg_1024_properties(gsf):
    """LOBPCG(m = 4, 50) on the benchmark workload: ascending Ritz values in
    [0, 2], orthonormal Ritz vectors, reported residuals equal to the
    explicit ones, and the output equal to the projection X X^T z0."""
    import torch
    op, x, xd, w = _op(gsf, "image_1024_bf11", gsf.F32)
    m = 4
    X = torch.empty((op.n, m), dtype=torch.float32, device="cuda")
    out, info = op.lobpcg_filter(xd, m, 50, ritz=X)
    th = np.array(list(info.theta)[:m])
    assert np.all(np.diff(th) >= 0) and th[0] >= -1e-6 and th[-1] <= 2.0
    Xd = X.double()
    G = (Xd.T @ Xd).cpu().numpy()
    assert np.abs(G - np.eye(m)).max() <= 1e-4
    R = op.lobpcg_residual(X, list(th))
    res = R.double().norm(dim=0).cpu().numpy()
    print(f"lobpcg 1024^2: theta {th}, res {list(info.res)[:m]} explicit {res}")
    assert np.all(np.abs(res - np.array(list(info.res)[:m])) <= 1e-3 * np.maximum(res, 1e-3))
    sq = op.sqrt_d().double()
    z0 = sq * xd.double()
    y = Xd @ (Xd.T @ z0)
    assert nrel((sq * out.double()).cpu().numpy(), y.cpu().numpy()) <= 1e-4


def test_batch_full_recipe_equals_single_calls(gsf):
    """The full uneven batch (256 images 64..1024 px, 64 signals 2^10..2^20):
    every item's output equals its single-item call bitwise."""
    import torch
    from synth import batch_items, item_signal
    recipe = batch_items()
    items = []
    for it in recipe:
        _, x = item_signal(it)
        xd = torch.tensor(x.astype(np.float32).ravel(), device="cuda")
        items.append(dict(kind=it["kind"], shape=it["shape"], radius=it["radius"], sigma_d=it["sigma_d"],
                          sigma_r=it["sigma_r"], eps=it["eps"], method=it["method"], m=it["m"], kmax=it["kmax"],
                          tol=it["tol"], guidance=xd, x0=xd))
    batch = gsf.Batch(items, prec=gsf.F32, autotune=True)
    batch.run()
    torch.cuda.synchronize()
    bad = 0
    for k in list(range(0, len(items), 7)) + [len(items) - 1]:
        it = items[k]
        op = gsf.Operator(it["kind"], it["shape"], it["guidance"], it["radius"], it["sigma_d"], it["sigma_r"],
                          it["eps"], gsf.F32)
        if it["method"] == "cg":
            solo, _ = op.cg_filter(it["x0"], it["kmax"], tol=it["tol"], info=False)
        else:
            solo, _ = op.lobpcg_filter(it["x0"], it["m"], it["kmax"], tol=it["tol"], info=False)
        bad += int(not torch.equal(solo, it["out"]))
    assert bad == 0
