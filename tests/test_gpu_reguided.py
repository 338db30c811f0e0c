"""GPU parity of the re-guided (non-linear) filters and of the Laplacian apply
form they use, through the C ABI, against the FP64 oracle.

Tolerances (relative, 2-norm and max-norm): FP64 data 1e-12 (power) and
max(1e-12, 10 band) (CG), the band being the oracle's own self-sensitivity
(the case on the grid in reverse point order, tests/sensitivity.py; every
step rebuilds the graph from the iterate, so summation-order differences
also pass through the weights of eq. (2), which move by ~|g_i - g_j| /
sigma_r^2 times a change of the guidance, and the band measures that
growth); FP32 data, against the oracle fed the FP32-rounded iterate before
each rebuild, 1e-5 for power and CG.  The L form of the apply: 1e-12 FP64,
1e-5 FP32 (a single apply, as the other forms).
"""
import numpy as np
import pytest

import oracle
from sensitivity import reference
from synth import piecewise_constant_1d, scene_2d

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den2 = max(np.linalg.norm(b), 1e-300)
    deni = max(np.abs(b).max(), 1e-300)
    return max(np.linalg.norm(a - b) / den2, np.abs(a - b).max() / deni)


def _signal(shape, seed):
    if len(shape) == 1:
        return piecewise_constant_1d(shape[0], 0.1, seed)[1]
    return scene_2d(shape[0], shape[1], 0.05, seed)[1].ravel()


# (kind, shape, seed, params): several tiles plus ragged tails
CASES = [
    ("bf", (3000,), 21, dict(radius=4, sigma_d=3.0, sigma_r=0.2)),
    ("bf", (67, 130), 22, dict(radius=3, sigma_d=2.0, sigma_r=0.15)),
    ("gf", (1500,), 23, dict(radius=4, eps=1e-2)),
    ("gf", (70, 131), 24, dict(radius=3, eps=1e-2)),
]


def _rg_cg(kind, x0, shape, k, **okw):
    """The oracle's re-guided CG with its self-sensitivity band."""
    return reference(lambda g: oracle.cg_filter_reguided(kind, g.ravel(), shape, k, **okw),
                     np.asarray(x0, dtype=np.float64).reshape(shape))


def _dev(x, prec, gsf):
    import torch
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def _oracle_kw(par):
    return dict(radius=par["radius"], sigma_s=par.get("sigma_d", 0.0), sigma_r=par.get("sigma_r", 0.0),
                eps=par.get("eps", 0.0))


def _gpu_kw(par):
    return dict(radius=par["radius"], sigma_d=par.get("sigma_d", 0.0), sigma_r=par.get("sigma_r", 0.0),
                eps=par.get("eps", 0.0))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m", [1, 3])
@pytest.mark.parametrize("kind,shape,seed,par", CASES)
def test_apply_laplacian_form(gsf, kind, shape, seed, par, m, prec):
    """y = L x = D x - W x (eq. (4)) on x-space vectors."""
    g = _signal(shape, seed)
    if prec == gsf.F32:
        g = g.astype(np.float32).astype(np.float64)
    op = gsf.Operator(kind, shape, _dev(g, prec, gsf), **_gpu_kw(par), prec=prec)
    ref_op = oracle.build_operator(kind, g.reshape(shape), **{k: v for k, v in _oracle_kw(par).items()})
    x = np.random.default_rng(seed).standard_normal((op.n, m))
    if prec == gsf.F32:
        x = x.astype(np.float32).astype(np.float64)
    xd = _dev(x if m > 1 else x[:, 0], prec, gsf)
    y = op.apply(xd, gsf.FORM_L).cpu().numpy().reshape(op.n, m)
    ref = np.stack([ref_op.apply_l(x[:, j]) for j in range(m)], axis=1)
    e = rel(y, ref)
    print(f"L form {kind} {shape} m={m} prec={prec}: {e:.2e}")
    assert e <= (1e-12 if prec == gsf.F64 else 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,shape,seed,par", CASES)
def test_reguided_power_parity(gsf, kind, shape, seed, par, prec):
    x0 = _signal(shape, seed)
    if prec == gsf.F32:
        x0 = x0.astype(np.float32).astype(np.float64)
    k = 6
    y, info = gsf.reguided_filter(kind, shape, _dev(x0, prec, gsf), gsf.METHOD_POWER, k, **_gpu_kw(par), prec=prec)
    ref = oracle.power_filter_reguided(kind, x0, shape, k, **_oracle_kw(par),
                                       data_prec="f32" if prec == gsf.F32 else "f64")
    e = rel(y.cpu().numpy(), ref)
    print(f"re-guided power {kind} {shape} prec={prec}: {e:.2e}")
    assert info.iters == k and e <= (1e-12 if prec == gsf.F64 else 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,shape,seed,par", CASES)
def test_reguided_cg_parity(gsf, kind, shape, seed, par, prec):
    x0 = _signal(shape, seed)
    if prec == gsf.F32:
        x0 = x0.astype(np.float32).astype(np.float64)
    k = 12
    y, info = gsf.reguided_filter(kind, shape, _dev(x0, prec, gsf), gsf.METHOD_CG, k, **_gpu_kw(par), prec=prec)
    rr = _rg_cg(kind, x0, shape, k, **_oracle_kw(par), data_prec="f32" if prec == gsf.F32 else "f64")
    ref, rinfo = rr.y, rr.extra
    e = rel(y.cpu().numpy(), ref)
    print(f"re-guided CG {kind} {shape} prec={prec}: {e:.2e} (band {rr.band:.1e}), iters {info.iters} vs "
          f"{rinfo.iters}, res {info.res:.3e} vs {rinfo.res:.3e}")
    assert info.status == gsf.OK and rinfo.status == "ok"
    assert info.iters == rinfo.iters == k
    assert e <= (rr.gate if prec == gsf.F64 else 1e-5)
    assert abs(info.res0 - rinfo.res0) <= (1e-12 if prec == gsf.F64 else 1e-5) * rinfo.res0


@pytest.mark.parametrize("prec", [0, 1])
def test_reguided_cg_tolerance_stop(gsf, prec):
    """tol > 0: stops at the same step as the oracle, status OK."""
    kind, shape, seed, par = CASES[1]
    x0 = _signal(shape, seed)
    if prec == gsf.F32:
        x0 = x0.astype(np.float32).astype(np.float64)
    y, info = gsf.reguided_filter(kind, shape, _dev(x0, prec, gsf), gsf.METHOD_CG, 500, **_gpu_kw(par), prec=prec,
                                  tol=1e-3)
    rr = _rg_cg(kind, x0, shape, 500, **_oracle_kw(par), tol=1e-3, data_prec="f32" if prec == gsf.F32 else "f64")
    ref, rinfo = rr.y, rr.extra
    e = rel(y.cpu().numpy(), ref)
    print(f"re-guided CG to 1e-3 prec={prec}: {info.iters} vs {rinfo.iters} steps, {e:.2e}")
    assert info.status == gsf.OK and rinfo.status == "ok"
    if prec == gsf.F64:
        assert info.iters == rinfo.iters == rr.extra_reversed.iters and e <= rr.gate
    else:
        # the FP32 residual may cross the tolerance a step or two apart from
        # the oracle's (a decision on rounding); the same step gives the bar
        assert abs(info.iters - rinfo.iters) <= 2
        assert e <= (1e-5 if info.iters == rinfo.iters else 1e-4)


@pytest.mark.parametrize("shape,seed", [((3000,), 25), ((67, 130), 26)])
def test_reguided_bf_without_range_kernel_equals_linear_gpu(gsf, shape, seed):
    """sigma_r = inf: the graph does not depend on the guidance, so the
    re-guided filters equal the linear ones (x-space against z-space CG)."""
    x0 = _signal(shape, seed)
    par = dict(radius=3, sigma_d=2.0, sigma_r=float("inf"))
    xd = _dev(x0, gsf.F64, gsf)
    op = gsf.Operator("bf", shape, xd, **par, prec=gsf.F64)
    lin = op.power_filter(xd, 5).cpu().numpy()
    rg, _ = gsf.reguided_filter("bf", shape, xd, gsf.METHOD_POWER, 5, **par, prec=gsf.F64)
    assert rel(rg.cpu().numpy(), lin) <= 1e-12
    lin, li = op.cg_filter(xd, 10)
    rg, ri = gsf.reguided_filter("bf", shape, xd, gsf.METHOD_CG, 10, **par, prec=gsf.F64)
    e = rel(rg.cpu().numpy(), lin.cpu().numpy())
    print(f"sigma_r = inf {shape}: re-guided CG vs linear CG {e:.2e}")
    assert ri.iters == li.iters == 10 and e <= 1e-10


@pytest.mark.parametrize("kind,shape,seed,par", CASES)
def test_reguided_edge_cases(gsf, kind, shape, seed, par):
    """kmax = 0 copies x0; a constant is a fixed point of the power filter and
    stops CG at once (r0 = 0) with x unchanged; in-place (x_out = x0) works."""
    import torch
    x0 = _signal(shape, seed)
    xd = _dev(x0, gsf.F64, gsf)
    y, info = gsf.reguided_filter(kind, shape, xd, gsf.METHOD_CG, 0, **_gpu_kw(par), prec=gsf.F64)
    assert torch.equal(y, xd) and info.iters == 0
    c = _dev(np.full(x0.size, 0.37), gsf.F64, gsf)
    y, _ = gsf.reguided_filter(kind, shape, c, gsf.METHOD_POWER, 3, **_gpu_kw(par), prec=gsf.F64)
    assert rel(y.cpu().numpy(), np.full(x0.size, 0.37)) <= 1e-14
    y, info = gsf.reguided_filter(kind, shape, c, gsf.METHOD_CG, 3, **_gpu_kw(par), prec=gsf.F64)
    assert info.status == gsf.EBREAKDOWN and torch.equal(y, c)
    ref = oracle.power_filter_reguided(kind, x0, shape, 2, **_oracle_kw(par))
    xin = xd.clone()
    gsf.reguided_filter(kind, shape, xin, gsf.METHOD_POWER, 2, **_gpu_kw(par), prec=gsf.F64, out=xin)
    assert rel(xin.cpu().numpy(), ref) <= 1e-12


def test_reguided_fullsize_properties(gsf):
    """The 1024^2 BF 11x11 FP32 workload: step 1 of the re-guided CG equals one
    step of the linear CG (the graph of x0); the GF re-guided filters keep
    1^T D x (its degrees N_i/|w| do not depend on the guidance)."""
    import torch
    from synth import WORKLOADS, make_signal
    w = WORKLOADS["image_1024_bf11"]
    _, x = make_signal("image_1024_bf11")
    xd = torch.tensor(x.astype(np.float32).ravel(), device="cuda")
    par = dict(radius=w["radius"], sigma_d=w["sigma_d"], sigma_r=w["sigma_r"])
    op = gsf.Operator("bf", w["shape"], xd, **par, prec=gsf.F32)
    lin, _ = op.cg_filter(xd, 1)
    rg, ri = gsf.reguided_filter("bf", w["shape"], xd, gsf.METHOD_CG, 1, **par, prec=gsf.F32)
    e = rel(rg.cpu().numpy(), lin.cpu().numpy())
    print(f"1024^2 re-guided CG step 1 vs linear: {e:.2e}")
    assert ri.iters == 1 and e <= 1e-5
    rg5, ri5 = gsf.reguided_filter("bf", w["shape"], xd, gsf.METHOD_CG, 5, **par, prec=gsf.F32)
    assert ri5.iters == 5 and bool(torch.isfinite(rg5).all())
    shape = w["shape"]
    d = oracle.gf_degrees(shape, 4).ravel()
    m0 = float(d @ x.astype(np.float32).astype(np.float64).ravel())
    for method in (gsf.METHOD_POWER, gsf.METHOD_CG):
        y, _ = gsf.reguided_filter("gf", shape, xd, method, 5, radius=4, eps=1e-2, prec=gsf.F32)
        m1 = float(d @ y.double().cpu().numpy())
        print(f"1024^2 GF re-guided method {method}: 1^T D x {m0:.6e} -> {m1:.6e}")
        assert abs(m1 - m0) <= 1e-5 * abs(m0)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [700, 20000])
def test_reguided_power_1d_both_paths(gsf, n, prec):
    """1D BF re-guided power filter: a signal that fits in one workgroup's LDS
    runs in one launch (n = 700), a longer one on the multi-kernel path
    (n = 20000 > 16384 FP32 / 8192 FP64 samples); both against the oracle,
    with the (diag L) normalization too."""
    x0 = piecewise_constant_1d(n, 0.1, 30 + n)[1]
    if prec == gsf.F32:
        x0 = x0.astype(np.float32).astype(np.float64)
    dp = "f32" if prec == gsf.F32 else "f64"
    for norm in ("d", "diagl"):
        par = dict(radius=3, sigma_d=2.0, sigma_r=0.15)
        y, info = gsf.reguided_filter("bf", (n,), _dev(x0, prec, gsf), gsf.METHOD_POWER, 25, **par, prec=prec,
                                      norm=norm)
        ref = oracle.power_filter_reguided("bf", x0, (n,), 25, radius=3, sigma_s=2.0, sigma_r=0.15, data_prec=dp,
                                           norm=norm)
        e = rel(y.cpu().numpy(), ref)
        print(f"re-guided power 1D n={n} prec={prec} norm={norm}: {e:.2e}")
        assert info.iters == 25 and e <= (1e-12 if prec == gsf.F64 else 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("stencil,norm", [("square", "d"), ("square", "diagl"), ("cross", "d"), ("cross", "diagl")])
def test_reguided_bf_interior_and_border_tiles(gsf, stencil, norm, prec):
    """The BF passes evaluate the weights from a 64 x 16 tile of the iterate
    and its halo in LDS, with a branch-free body for tiles whose halo lies on
    the grid: 100 x 200 with radius 5 has such interior tiles as well as
    border tiles on all four sides and ragged ones.  Power (4 passes) and CG
    (6 steps) against the oracle; the FP32 weights use the hardware base-2
    exponential (relative error a few units of 2^-24 times 1 + the exponent's
    magnitude), well inside the bounds stated at the top."""
    shape = (100, 200)
    x0 = scene_2d(shape[0], shape[1], 0.05, 77)[1].ravel()
    if prec == gsf.F32:
        x0 = x0.astype(np.float32).astype(np.float64)
    dp = "f32" if prec == gsf.F32 else "f64"
    gp = dict(radius=5, sigma_d=3.0, sigma_r=0.15, stencil=stencil, norm=norm)
    op_ = dict(radius=5, sigma_s=3.0, sigma_r=0.15, stencil=stencil, norm=norm, data_prec=dp)
    y, info = gsf.reguided_filter("bf", shape, _dev(x0, prec, gsf), gsf.METHOD_POWER, 4, **gp, prec=prec)
    ref = oracle.power_filter_reguided("bf", x0, shape, 4, **op_)
    e = rel(y.cpu().numpy(), ref)
    y, info = gsf.reguided_filter("bf", shape, _dev(x0, prec, gsf), gsf.METHOD_CG, 6, **gp, prec=prec)
    rr = _rg_cg("bf", x0, shape, 6, **op_)
    ref, rinfo = rr.y, rr.extra
    ec = rel(y.cpu().numpy(), ref)
    print(f"re-guided BF 100x200 r=5 {stencil}/{norm} prec={prec}: power {e:.2e}, CG {ec:.2e} (band {rr.band:.1e})")
    assert e <= (1e-12 if prec == gsf.F64 else 1e-5)
    assert info.iters == rinfo.iters == 6 and ec <= (rr.gate if prec == gsf.F64 else 1e-5)
    assert abs(info.res0 - rinfo.res0) <= (1e-12 if prec == gsf.F64 else 1e-5) * rinfo.res0


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", [(40, 90), (5000,)])
def test_reguided_bf_largest_radius(gsf, shape, prec):
    """Radius 8 (the largest window): the LDS tile holds the largest halo
    (80 x 32 points of the iterate and of the CG vector in 2D)."""
    x0 = _signal(shape, 78)
    if prec == gsf.F32:
        x0 = x0.astype(np.float32).astype(np.float64)
    dp = "f32" if prec == gsf.F32 else "f64"
    y, _ = gsf.reguided_filter("bf", shape, _dev(x0, prec, gsf), gsf.METHOD_POWER, 3, radius=8, sigma_d=4.0,
                               sigma_r=0.2, prec=prec)
    ref = oracle.power_filter_reguided("bf", x0, shape, 3, radius=8, sigma_s=4.0, sigma_r=0.2, data_prec=dp)
    e = rel(y.cpu().numpy(), ref)
    y, info = gsf.reguided_filter("bf", shape, _dev(x0, prec, gsf), gsf.METHOD_CG, 4, radius=8, sigma_d=4.0,
                                  sigma_r=0.2, prec=prec)
    rr = _rg_cg("bf", x0, shape, 4, radius=8, sigma_s=4.0, sigma_r=0.2, data_prec=dp)
    ref, rinfo = rr.y, rr.extra
    ec = rel(y.cpu().numpy(), ref)
    print(f"re-guided BF radius 8 {shape} prec={prec}: power {e:.2e}, CG {ec:.2e} (band {rr.band:.1e})")
    assert e <= (1e-12 if prec == gsf.F64 else 1e-5)
    assert info.iters == rinfo.iters == 4 and ec <= (rr.gate if prec == gsf.F64 else 1e-5)


@pytest.mark.parametrize("shape", [(1, 1), (1, 50), (50, 1), (2,), (3, 7)])
def test_reguided_bf_tiny_grids(gsf, shape):
    """Grids smaller than one tile and than the window, single rows and
    columns: every tile is a border tile and most window points are off the
    grid.  A single point has no edge (power leaves it unchanged, CG breaks
    down at once: r_0 = 0); two points converge in one CG step and then break
    down.  FP64 against the oracle, statuses and step counts included."""
    x0 = np.random.default_rng(int(np.prod(shape))).random(int(np.prod(shape)))
    par = dict(radius=2, sigma_d=1.5, sigma_r=0.2)
    y, _ = gsf.reguided_filter("bf", shape, _dev(x0, gsf.F64, gsf), gsf.METHOD_POWER, 3, **par, prec=gsf.F64)
    ref = oracle.power_filter_reguided("bf", x0, shape, 3, radius=2, sigma_s=1.5, sigma_r=0.2)
    assert rel(y.cpu().numpy(), ref) <= 1e-12
    y, info = gsf.reguided_filter("bf", shape, _dev(x0, gsf.F64, gsf), gsf.METHOD_CG, 4, **par, prec=gsf.F64)
    rr = _rg_cg("bf", x0, shape, 4, radius=2, sigma_s=1.5, sigma_r=0.2)
    ref, rinfo = rr.y, rr.extra
    st = {"ok": gsf.OK, "breakdown": gsf.EBREAKDOWN}[rinfo.status]
    print(f"re-guided BF tiny {shape}: status {info.status} vs {rinfo.status}, iters {info.iters} vs {rinfo.iters}")
    assert info.status == st and info.iters == rinfo.iters
    assert rel(y.cpu().numpy(), ref) <= rr.gate
