"""GPU parity of the BF options of the image experiment (Section 7 and the
normalization of Section 4): the cross (5-point-type) lattice and the
(diag L)^-1/2 L (diag L)^-1/2 normalization, through the C ABI, against the
FP64 oracle.

Tolerances as for the default operator (relative, 2-norm and max-norm): FP64
1e-12 for weights, degrees, apply and power iteration, max(1e-12, 10 band)
for the CG, LOBPCG and re-guided outputs (the band is the oracle's own
self-sensitivity: the case on the grid in reverse point order,
tests/sensitivity.py); FP32 1e-5 for every output.  For FP32 runs the oracle
gets the FP32-rounded input.  The full-size experiment compares the whole 1024^2
outputs (the oracle's sparse 5-point operator finishes in seconds there) and
the PSNRs they give.
"""
import numpy as np
import pytest

import oracle
from sensitivity import reference
from synth import WORKLOADS, make_signal, piecewise_constant_1d, scene_2d

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den2 = max(np.linalg.norm(b), 1e-300)
    deni = max(np.abs(b).max(), 1e-300)
    return max(np.linalg.norm(a - b) / den2, np.abs(a - b).max() / deni)


def _dev(x, prec, gsf):
    import torch
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def _round(x, prec, gsf):
    return x.astype(np.float32).astype(np.float64) if prec == gsf.F32 else x


# (shape, seed, radius, sigma_d, sigma_r, stencil, norm): several tiles and
# ragged tails; radius 1 is the 5-point stencil, radius 8 the largest window
CASES = [
    ((67, 130), 41, 1, 1.0, 0.1, "cross", "diagl"),
    ((67, 130), 42, 1, 1.0, 0.1, "cross", "d"),
    ((33, 200), 43, 3, 2.0, 0.15, "cross", "diagl"),
    ((70, 131), 44, 2, 2.0, 0.1, "square", "diagl"),
    ((3000,), 45, 4, 3.0, 0.2, "cross", "diagl"),
    ((40, 150), 46, 8, 4.0, 0.2, "square", "d"),      # the largest window: widest LDS halo
    ((45, 100), 47, 8, 4.0, 0.2, "cross", "diagl"),
]


def _signal(shape, seed, sigma=0.1):
    if len(shape) == 1:
        return piecewise_constant_1d(shape[0], sigma, seed)[1]
    return scene_2d(shape[0], shape[1], sigma, seed)[1]


def _oracle_op(case, g):
    shape, seed, r, sd, sr, stencil, norm = case
    return oracle.build_operator("bf", g, r, sd, sr, stencil=stencil, norm=norm)


def _build(gsf, case, prec):
    shape, seed, r, sd, sr, stencil, norm = case
    x = _round(_signal(shape, seed), prec, gsf)
    op = gsf.Operator("bf", shape, _dev(x.ravel(), prec, gsf), radius=r, sigma_d=sd, sigma_r=sr, prec=prec,
                      stencil=stencil, norm=norm)
    ref = oracle.build_operator("bf", x.reshape(shape), r, sd, sr, stencil=stencil, norm=norm)
    return op, ref, x.ravel()


def _offsets(ndim, r, stencil):
    if ndim == 1:
        return [(o,) for o in range(1, r + 1)]
    if stencil == "cross":
        return [(0, dx) for dx in range(1, r + 1)] + [(dy, 0) for dy in range(1, r + 1)]
    return [(0, dx) for dx in range(1, r + 1)] + [(dy, dx) for dy in range(1, r + 1) for dx in range(-r, r + 1)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_build_parity(gsf, case, prec):
    """Planes hold w_{i,i+o} of eq. (2) for the stencil's half window; the
    degree is the FP64 sum of exactly the stored off-diagonal weights (own
    planes and mirrored entries; diag L, 1 where it is 0) or of all of them
    plus the self-loop (D).  FP32 data (the one-pass build's FP32
    exponential): a weight w = e^-a is within about (2 + 2a) 2^-24 w of the
    oracle's, at most 4e-7 of the largest weight (bound 5e-7)."""
    op, ref, _ = _build(gsf, case, prec)
    shape, r, stencil = ref.shape, ref.radius, case[5]
    W = ref.W.tocsr()
    tol = 1e-12 if prec == gsf.F64 else 1e-5
    planes = op.planes().cpu().numpy().astype(np.float64)
    offs = _offsets(len(shape), r, stencil)
    assert planes.shape[0] == len(offs)
    coords = np.indices(shape).reshape(len(shape), -1).T
    d_st = np.zeros(ref.n)
    for q, o in enumerate(offs):
        nb = coords + np.array(o)
        inside = np.all((nb >= 0) & (nb < np.array(shape)), axis=1)
        i = np.flatnonzero(inside)
        j = np.ravel_multi_index(tuple(nb[inside].T), shape)
        expect = np.zeros(ref.n)
        expect[i] = np.asarray(W[i, j]).ravel()
        assert rel(planes[q], expect) <= (1e-15 if prec == gsf.F64 else 5e-7), (q, o)
        d_st[i] += planes[q][i]
        d_st[j] += planes[q][i]
    if case[6] == "diagl":
        d_st = np.where(d_st > 0.0, d_st, 1.0)
    else:
        d_st += 1.0
    deg = op.degree().cpu().numpy()
    np.testing.assert_allclose(deg, d_st, rtol=1e-13)
    assert rel(deg, ref.d) <= tol   # the oracle's normalizing degree (diag L: 1 where 0)
    assert rel(op.sqrt_d().cpu().numpy(), ref.sqrt_d) <= tol
    assert rel(op.inv_sqrt_d().cpu().numpy(), 1.0 / ref.sqrt_d) <= tol


@pytest.mark.parametrize("m", [1, 3, 8])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", CASES)
def test_apply_parity_all_forms(gsf, case, prec, m):
    op, ref, _ = _build(gsf, case, prec)
    v = _round(np.random.default_rng(7 + m).standard_normal((op.n, m)), prec, gsf)
    vd = _dev(v if m > 1 else v[:, 0], prec, gsf)
    for form in (gsf.FORM_N, gsf.FORM_LSYM, gsf.FORM_RW, gsf.FORM_L):
        y = op.apply(vd, form).cpu().numpy().reshape(op.n, m)
        r = np.stack([ref.apply(form, v[:, j]) for j in range(m)], axis=1)
        e = rel(y, r)
        print(f"apply {case[0]} {case[5]}/{case[6]} form {form} m={m} prec={prec}: {e:.2e}")
        assert e <= (1e-12 if prec == gsf.F64 else 1e-5), (form, e)


@pytest.mark.parametrize("rows", [1, 2, 4])
def test_apply_rows_per_thread_agree(gsf, rows):
    """Every rows-per-thread choice of the cross kernel gives the same result
    (the tuner may pick any of them)."""
    op, ref, x = _build(gsf, CASES[2], gsf.F64)
    for m in (1, 4):
        v = np.random.default_rng(m).standard_normal((op.n, m))
        op.set_apply_rows(m, rows)
        y = op.apply(_dev(v if m > 1 else v[:, 0], gsf.F64, gsf), gsf.FORM_LSYM).cpu().numpy().reshape(op.n, m)
        r = np.stack([ref.apply_lsym(v[:, j]) for j in range(m)], axis=1)
        assert rel(y, r) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[4]])
def test_power_and_cg_parity(gsf, case, prec):
    op, ref, x = _build(gsf, case, prec)
    y = op.power_filter(_dev(x, prec, gsf), 15).cpu().numpy()
    r = x.copy()
    for _ in range(15):
        r = ref.apply_rw(r)
    assert rel(y, r) <= (1e-12 if prec == gsf.F64 else 1e-5)
    y, info = op.cg_filter(_dev(x, prec, gsf), 20)
    rr = reference(lambda g: oracle.cg_filter(_oracle_op(case, g), g.ravel(), 20,
                                              data_prec="f32" if prec == gsf.F32 else "f64"),
                   x.reshape(case[0]))
    r, rinfo = rr.y, rr.extra
    e = rel(y.cpu().numpy(), r)
    print(f"cg {case[0]} {case[5]}/{case[6]} prec={prec}: {e:.2e} (band {rr.band:.1e})")
    assert info.iters == rinfo.iters == 20 and info.status == gsf.OK
    assert e <= (rr.gate if prec == gsf.F64 else 1e-5)
    assert abs(info.res0 - rinfo.res0) <= 1e-6 * rinfo.res0


@pytest.mark.parametrize("prec,m,constraint", [(1, 1, False), (1, 1, True), (1, 4, True), (0, 1, True),
                                               (0, 4, False)])
def test_lobpcg_parity(gsf, prec, m, constraint):
    import torch
    op, ref, x = _build(gsf, CASES[0], prec)
    ritz = torch.empty((op.n, m), dtype=op.dtype, device="cuda")
    y, info = op.lobpcg_filter(_dev(x, prec, gsf), m, 20, constraint=constraint, ritz=ritz)

    def run(g):
        r, th, _, rinfo = oracle.lobpcg_filter(_oracle_op(CASES[0], g), g.ravel(), m, 20, constraint=constraint,
                                               data_prec="f64" if prec == gsf.F64 else "f32")
        return r, (th, rinfo)

    rr = reference(run, x.reshape(CASES[0][0]))
    r, (th, rinfo) = rr.y, rr.extra
    assert info.iters == rinfo.iters == 20
    if rinfo.dropped == rr.extra_reversed[1].dropped:
        assert info.dropped == rinfo.dropped
    theta = np.array(info.theta[:m])
    e = rel(y.cpu().numpy(), r)
    print(f"lobpcg m={m} constraint={constraint} prec={prec}: {e:.2e} (band {rr.band:.1e}), theta {theta} vs {th}")
    if prec == gsf.F64:
        np.testing.assert_allclose(theta, th, rtol=max(1e-9, rr.gate), atol=1e-12)
        assert e <= rr.gate
    else:
        assert np.abs(theta - th).max() <= 2e-5
        assert e <= 1e-5


def test_isolated_vertex(gsf):
    """A pixel whose neighbours all differ by far more than sigma_r has only
    zero off-diagonal weights: its normalizing value is 1, every filter keeps
    it, and the rest matches the oracle."""
    g = scene_2d(40, 70, 0.05, 46)[1]
    g[20, 33] = 50.0
    i = 20 * 70 + 33
    op = gsf.Operator("bf", g.shape, _dev(g.ravel(), gsf.F64, gsf), radius=1, sigma_d=1.0, sigma_r=0.1,
                      prec=gsf.F64, stencil="cross", norm="diagl")
    ref = oracle.build_operator("bf", g, 1, 1.0, 0.1, stencil="cross", norm="diagl")
    assert ref.dl[i] == 0.0 and op.degree().cpu().numpy()[i] == 1.0
    xd = _dev(g.ravel(), gsf.F64, gsf)

    def cross(v):
        return oracle.build_operator("bf", v, 1, 1.0, 0.1, stencil="cross", norm="diagl")

    y, info = op.cg_filter(xd, 10)
    rr = reference(lambda v: oracle.cg_filter(cross(v), v.ravel(), 10), g)
    yv = y.cpu().numpy()
    assert yv[i] == 50.0 and rel(yv, rr.y) <= rr.gate
    y = op.power_filter(xd, 5).cpu().numpy()
    assert y[i] == 50.0
    yl, _ = op.lobpcg_filter(xd, 1, 10, constraint=True)
    rl = reference(lambda v: oracle.lobpcg_filter(cross(v), v.ravel(), 1, 10, constraint=True)[0:2], g)
    assert rel(yl.cpu().numpy(), rl.y) <= rl.gate


def test_gf_rejects_bf_options(gsf):
    x = _dev(np.zeros(64 * 64), gsf.F32, gsf)
    for kw in (dict(stencil="cross"), dict(norm="diagl")):
        with pytest.raises(gsf.GsfError):
            gsf.Operator("gf", (64, 64), x, radius=2, eps=1e-2, **kw)


@pytest.mark.parametrize("prec", [0, 1])
def test_reguided_variants_parity(gsf, prec):
    """The re-guided filters on the cross / (diag L) graph (the graph rebuilt
    from the iterate every step): FP64 1e-12 power, max(1e-12, 10 band) CG;
    FP32 1e-5 both."""
    shape, seed = (67, 130), 47
    x0 = _round(_signal(shape, seed), prec, gsf).ravel()
    kw = dict(radius=1, sigma_d=1.0, sigma_r=0.1, stencil="cross", norm="diagl")
    dp = "f32" if prec == gsf.F32 else "f64"
    y, info = gsf.reguided_filter("bf", shape, _dev(x0, prec, gsf), gsf.METHOD_POWER, 6, prec=prec, **kw)
    r = oracle.power_filter_reguided("bf", x0, shape, 6, radius=1, sigma_s=1.0, sigma_r=0.1, data_prec=dp,
                                     stencil="cross", norm="diagl")
    assert rel(y.cpu().numpy(), r) <= (1e-12 if prec == gsf.F64 else 1e-5)
    y, info = gsf.reguided_filter("bf", shape, _dev(x0, prec, gsf), gsf.METHOD_CG, 12, prec=prec, **kw)
    rr = reference(lambda v: oracle.cg_filter_reguided("bf", v.ravel(), shape, 12, radius=1, sigma_s=1.0,
                                                       sigma_r=0.1, data_prec=dp, stencil="cross", norm="diagl"),
                   x0.reshape(shape))
    r, rinfo = rr.y, rr.extra
    e = rel(y.cpu().numpy(), r)
    print(f"re-guided CG cross/diagl prec={prec}: {e:.2e} (band {rr.band:.1e})")
    assert info.iters == rinfo.iters == 12 and e <= (rr.gate if prec == gsf.F64 else 1e-5)


def psnr(y, clean):
    """10 log10(peak^2 / MSE) with peak 1 (the clean image lies in [0, 1])."""
    return 10.0 * np.log10(1.0 / np.mean((np.asarray(y, dtype=np.float64).ravel() - clean.ravel()) ** 2))


def test_image_experiment_fullsize(gsf):
    """The image experiment of Section 7 on the 1024^2 synthetic scene with
    noise variance 0.01: 5-point lattice, BF weights with sigma_r = 0.1,
    (diag L) normalization, 20 steps of CG and of LOBPCG (m = 1) with and
    without the constraint, FP32.  Whole outputs against the oracle; the
    noisy PSNR is about 20 dB and every filter raises it (the paper reports
    about 20 -> 21 dB on its natural test image; the piecewise-smooth scene
    has no texture to lose, so the gain here is larger)."""
    import torch
    w = WORKLOADS["image_1024_cross5"]
    clean, noisy = make_signal("image_1024_cross5")
    xr = noisy.astype(np.float32).astype(np.float64)
    kw = dict(radius=w["radius"], sigma_d=w["sigma_d"], sigma_r=w["sigma_r"], stencil=w["stencil"], norm=w["norm"])
    op = gsf.Operator("bf", w["shape"], _dev(xr.ravel(), gsf.F32, gsf), prec=gsf.F32, **kw)
    ref = oracle.build_operator("bf", xr, w["radius"], w["sigma_d"], w["sigma_r"], stencil=w["stencil"],
                                norm=w["norm"])
    xd = _dev(xr.ravel(), gsf.F32, gsf)
    p0 = psnr(xr, clean)
    assert 19.9 <= p0 <= 20.1
    y, info = op.cg_filter(xd, w["cg_iters"])
    r, _ = oracle.cg_filter(ref, xr.ravel(), w["cg_iters"], data_prec="f32")
    e = rel(y.cpu().numpy(), r)
    pg, pr = psnr(y.cpu().numpy(), clean), psnr(r, clean)
    print(f"image experiment: noisy {p0:.2f} dB; CG 20: {pg:.3f} dB (oracle {pr:.3f}), rel err {e:.2e}")
    assert e <= 1e-5 and abs(pg - pr) <= 1e-3 and pg >= p0 + 1.0
    for constraint in (False, True):
        ritz = torch.empty((op.n, 1), dtype=torch.float32, device="cuda")
        y, info = op.lobpcg_filter(xd, w["lobpcg_m"], w["lobpcg_iters"], constraint=constraint, ritz=ritz)
        r, th, _, _ = oracle.lobpcg_filter(ref, xr.ravel(), w["lobpcg_m"], w["lobpcg_iters"], constraint=constraint,
                                           data_prec="f32")
        e = rel(y.cpu().numpy(), r)
        pg, pr = psnr(y.cpu().numpy(), clean), psnr(r, clean)
        print(f"image experiment: LOBPCG 20 constraint={constraint}: {pg:.3f} dB (oracle {pr:.3f}), "
              f"rel err {e:.2e}, theta {info.theta[0]:.4e} vs {th[0]:.4e}")
        assert e <= 1e-5 and abs(pg - pr) <= 1e-3 and pg >= p0 + 1.0
