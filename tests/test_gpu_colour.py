"""GPU parity of the colour path (Section 2: the BF's photometric distance in
CIE-Lab for colour images) and of the multi-channel block filters, through
the C ABI, against the FP64 oracle.

Tolerances: CIE-Lab conversion 1e-12 (FP64) and 1e-5 (FP32) relative to the
Lab range (100); weights, degrees and applies as for the scalar guidance (FP64
1e-12, FP32 1e-5); block power 1e-12 / 1e-5; block CG max(1e-12, 10 band) /
1e-5, the band being the oracle's own self-sensitivity (the case on the grid
in reverse point order; tests/sensitivity.py), as for the single-vector CG.  For FP32 runs the oracle gets the FP32-rounded inputs and
the Lab guidance the GPU computed (rounded to FP32), so the comparison
measures the filter's arithmetic; the conversion is checked on its own.
"""
import numpy as np
import pytest

import oracle
from sensitivity import reference
from synth import WORKLOADS, make_signal, scene_2d_rgb

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return max(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300),
               np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _dev(x, prec, gsf):
    import torch
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def _round(x, prec, gsf):
    return x.astype(np.float32).astype(np.float64) if prec == gsf.F32 else x


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [1, 1000, 70001])
def test_srgb_to_lab_parity(gsf, prec, n):
    rng = np.random.default_rng(n)
    rgb = rng.uniform(-0.1, 1.1, size=(n, 3))   # noisy values leave [0, 1]; no clipping
    rgb[:3] = [[1, 0, 0], [0, 1, 0], [0, 0, 1]][:n]
    rgb = _round(rgb, prec, gsf)
    lab = gsf.srgb_to_lab(_dev(rgb, prec, gsf)).cpu().numpy()
    ref = oracle.srgb_to_lab(rgb)
    e = np.abs(lab - ref).max() / 100.0
    print(f"Lab n={n} prec={prec}: {e:.2e}")
    assert e <= (1e-12 if prec == gsf.F64 else 1e-5)


def test_srgb_to_lab_in_place(gsf):
    rgb = np.random.default_rng(5).uniform(0, 1, size=(4097, 3))
    t = _dev(rgb, gsf.F64, gsf)
    gsf.srgb_to_lab(t, out=t)
    assert np.abs(t.cpu().numpy() - oracle.srgb_to_lab(rgb)).max() <= 1e-10


def _colour_case(gsf, shape, seed, prec, radius=3, sigma_r=5.0):
    _, noisy = scene_2d_rgb(shape[0], shape[1], 0.05, seed)
    x = _round(noisy, prec, gsf)
    labd = gsf.srgb_to_lab(_dev(x.reshape(-1, 3), prec, gsf))
    lab = labd.double().cpu().numpy().reshape(shape + (3,))
    op = gsf.Operator("bf", shape, labd, radius=radius, sigma_d=2.0, sigma_r=sigma_r, prec=prec, channels=3)
    ref = oracle.build_operator("bf", lab, radius, 2.0, sigma_r, channels=3)
    return op, ref, x.reshape(-1, 3)


CASES = [((67, 130), 31), ((33, 200), 32)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,seed", CASES)
def test_colour_build_parity(gsf, shape, seed, prec):
    """Planes against the oracle's W of the Lab guidance; degrees as the FP64
    row sums of exactly the stored weights (own planes and mirrored entries)
    and against the oracle's d.  FP32 data: the one-pass build's FP32 squared
    distance and exponential put a weight e^-a within about (4 + 3a) 2^-24 of
    the oracle's, at most 1e-6 of the largest weight (bound 2e-6)."""
    op, ref, _ = _colour_case(gsf, shape, seed, prec)
    W = ref.W.tocsr()
    planes = op.planes().cpu().numpy().astype(np.float64)
    r = ref.radius
    offs = [(0, dx) for dx in range(1, r + 1)] + [(dy, dx) for dy in range(1, r + 1) for dx in range(-r, r + 1)]
    coords = np.indices(shape).reshape(2, -1).T
    d_st = np.ones(ref.n)
    for q, o in enumerate(offs):
        nb = coords + np.array(o)
        inside = np.all((nb >= 0) & (nb < np.array(shape)), axis=1)
        i = np.flatnonzero(inside)
        j = np.ravel_multi_index(tuple(nb[inside].T), shape)
        expect = np.zeros(ref.n)
        expect[i] = np.asarray(W[i, j]).ravel()
        assert rel(planes[q], expect) <= (1e-15 if prec == gsf.F64 else 2e-6), (q, o)
        d_st[i] += planes[q][i]
        d_st[j] += planes[q][i]
    deg = op.degree().cpu().numpy()
    np.testing.assert_allclose(deg, d_st, rtol=1e-13)
    assert rel(deg, ref.d) <= (1e-13 if prec == gsf.F64 else 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,seed", CASES)
def test_colour_apply_parity(gsf, shape, seed, prec):
    op, ref, x = _colour_case(gsf, shape, seed, prec)
    xd = _dev(x, prec, gsf)
    for form in (gsf.FORM_N, gsf.FORM_LSYM, gsf.FORM_RW, gsf.FORM_L):
        y = op.apply(xd, form).cpu().numpy()
        e = rel(y, ref.apply(form, x))
        assert e <= (1e-12 if prec == gsf.F64 else 1e-5), (form, e)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,seed", CASES)
def test_block_filters_parity(gsf, shape, seed, prec):
    op, ref, x = _colour_case(gsf, shape, seed, prec)
    xd = _dev(x, prec, gsf)
    y = op.power_filter_block(xd, 12).cpu().numpy()
    r = x.copy()
    for _ in range(12):
        r = ref.apply_rw(r)
    e = rel(y, r)
    print(f"block power {shape} prec={prec}: {e:.2e}")
    assert e <= (1e-12 if prec == gsf.F64 else 1e-5)
    y, infos = op.cg_filter_block(xd, 15)
    dp = "f32" if prec == gsf.F32 else "f64"
    rr = reference(lambda lab, v: oracle.cg_filter_block(oracle.build_operator("bf", lab, ref.radius, 2.0, 5.0,
                                                                               channels=3),
                                                         v.reshape(-1, 3), 15, data_prec=dp),
                   ref.guidance, x.reshape(shape + (3,)))
    r, rinfos = rr.y, rr.extra
    e = rel(y.cpu().numpy(), r)
    print(f"block CG {shape} prec={prec}: {e:.2e} (band {rr.band:.1e})")
    assert e <= (rr.gate if prec == gsf.F64 else 1e-5)
    for c in range(3):
        assert infos[c].iters == rinfos[c].iters == 15 and infos[c].status == gsf.OK
        assert abs(infos[c].res0 - rinfos[c].res0) <= 1e-6 * rinfos[c].res0


def test_block_cg_equals_single_column_runs(gsf):
    """Each column of the block CG (power filter) is the single-vector CG
    (power filter) of that column, up to summation order (the dot products;
    the apply tile, which may differ with the block width); m = 1..8."""
    op, ref, x = _colour_case(gsf, (67, 130), 33, gsf.F64)
    rng = np.random.default_rng(3)
    for m in (1, 2, 5, 8):
        X = np.concatenate([x, rng.standard_normal((op.n, 5))], axis=1)[:, :m]
        Xd = _dev(X, gsf.F64, gsf)
        Y, infos = op.cg_filter_block(Xd, 12)
        for c in range(m):
            yc, ic = op.cg_filter(Xd[:, c].contiguous(), 12)
            assert rel(Y[:, c].cpu().numpy(), yc.cpu().numpy()) <= 1e-12
            assert infos[c].iters == ic.iters
        P = op.power_filter_block(Xd, 7)
        for c in range(m):
            pc = op.power_filter(Xd[:, c].contiguous(), 7)
            assert rel(P[:, c].cpu().numpy(), pc.cpu().numpy()) <= 1e-13


def test_block_cg_columns_stop_independently(gsf):
    """A constant column breaks down at once and keeps its value; with a
    tolerance, columns stop at their own steps (as the oracle's per-column
    runs), the others continue."""
    op, ref, x = _colour_case(gsf, (67, 130), 34, gsf.F64)
    X = x.copy()
    X[:, 1] = 0.25
    Xd = _dev(X, gsf.F64, gsf)
    Y, infos = op.cg_filter_block(Xd, 10)
    assert infos[1].status == gsf.EBREAKDOWN and infos[1].iters == 0
    assert np.array_equal(Y[:, 1].cpu().numpy(), X[:, 1])
    assert infos[0].status == gsf.OK and infos[0].iters == 10
    shape = ref.shape

    def block_cg(lab, v, kmax, tol=0.0):
        return oracle.cg_filter_block(oracle.build_operator("bf", lab, ref.radius, 2.0, 5.0, channels=3),
                                      v.reshape(-1, 3), kmax, tol)

    rr = reference(lambda lab, v: block_cg(lab, v, 10), ref.guidance, X.reshape(shape + (3,)))
    assert rel(Y.cpu().numpy()[:, [0, 2]], rr.y[:, [0, 2]]) <= rr.gate
    Xt = x.copy()
    Xt[:, 2] *= 1e-3                      # a different scale: the relative tolerance still stops it
    Y, infos = op.cg_filter_block(_dev(Xt, gsf.F64, gsf), 400, tol=1e-4)
    rr = reference(lambda lab, v: block_cg(lab, v, 400, 1e-4), ref.guidance, Xt.reshape(shape + (3,)))
    r, rinfos = rr.y, rr.extra
    for c in range(3):
        print(f"column {c}: {infos[c].iters} vs {rinfos[c].iters} steps")
        assert infos[c].iters == rinfos[c].iters == rr.extra_reversed[c].iters
    assert rel(Y.cpu().numpy(), r) <= rr.gate


def test_colour_fullsize(gsf):
    """The 1024^2 colour workload: the Lab guidance built on the GPU, the
    operator's L_sym at sampled points against the pointwise oracle (eq. (2)
    with the Euclidean Lab distance), the block filters against per-channel
    runs, and the PSNR gain."""
    from oracle.pointwise import bf_lsym_at, sample_points
    w = WORKLOADS["image_1024_rgb_bf11"]
    clean, noisy = make_signal("image_1024_rgb_bf11")
    shape = w["shape"]
    x = noisy.astype(np.float32)
    xd = _dev(x.reshape(-1, 3), gsf.F32, gsf)
    labd = gsf.srgb_to_lab(xd)
    lab = labd.double().cpu().numpy().reshape(shape + (3,))
    assert np.abs(lab - oracle.srgb_to_lab(x.astype(np.float64))).max() <= 1e-3
    op = gsf.Operator("bf", shape, labd, radius=w["radius"], sigma_d=w["sigma_d"], sigma_r=w["sigma_r"],
                      prec=gsf.F32, channels=3)
    z = np.random.default_rng(8).standard_normal((op.n, 3)).astype(np.float32)
    y = op.apply(_dev(z, gsf.F32, gsf), gsf.FORM_LSYM).cpu().numpy()
    pts = sample_points(shape, 40, 9)
    ref = bf_lsym_at(lab, z.astype(np.float64), pts, w["radius"], w["sigma_d"], w["sigma_r"], channels=3)
    e = np.abs(y[pts] - ref).max() / np.abs(ref).max()
    print(f"1024^2 colour L_sym at {len(pts)} points: {e:.2e}")
    assert e <= 1e-5
    Y, infos = op.cg_filter_block(xd, w["cg_iters"])
    for c in range(3):
        yc, _ = op.cg_filter(xd[:, c].contiguous(), w["cg_iters"])
        assert rel(Y[:, c].cpu().numpy(), yc.cpu().numpy()) <= 1e-5

    def psnr(v):
        return 10 * np.log10(1.0 / np.mean((np.asarray(v, dtype=np.float64).ravel() - clean.ravel()) ** 2))
    p0, p1 = psnr(x), psnr(Y.cpu().numpy())
    P = op.power_filter_block(xd, w["power_iters"]).cpu().numpy()
    print(f"1024^2 colour: noisy {p0:.2f} dB, block CG {p1:.2f} dB, block power {psnr(P):.2f} dB")
    assert p1 >= p0 + 3.0 and psnr(P) >= p0 + 3.0


@pytest.mark.parametrize("prec", [0, 1])
def test_block_filters_on_gf_operator(gsf, prec):
    """The block filters run on any operator: a GF operator (scalar guidance)
    filtering a 3-channel block, against the oracle column by column."""
    shape = (60, 90)
    rgb = scene_2d_rgb(*shape, 0.05, 35)[1].reshape(-1, 3)
    g = rgb.mean(axis=1)
    rgb, g = _round(rgb, prec, gsf), _round(g, prec, gsf)
    op = gsf.Operator("gf", shape, _dev(g, prec, gsf), radius=3, eps=1e-2, prec=prec)
    ref = oracle.build_operator("gf", g.reshape(shape), 3, eps=1e-2)
    xd = _dev(rgb, prec, gsf)
    y = op.power_filter_block(xd, 6).cpu().numpy()
    r = rgb.copy()
    for _ in range(6):
        r = ref.apply_rw(r)
    assert rel(y, r) <= (1e-12 if prec == gsf.F64 else 1e-5)
    y, infos = op.cg_filter_block(xd, 12)
    dp = "f32" if prec == gsf.F32 else "f64"
    rr = reference(lambda gg, v: oracle.cg_filter_block(oracle.build_operator("gf", gg, 3, eps=1e-2),
                                                        v.reshape(-1, 3), 12, data_prec=dp),
                   g.reshape(shape), rgb.reshape(shape + (3,)))
    e = rel(y.cpu().numpy(), rr.y)
    print(f"GF block CG prec={prec}: {e:.2e} (band {rr.band:.1e})")
    assert e <= (rr.gate if prec == gsf.F64 else 1e-5)
    assert all(i.iters == 12 for i in infos)
