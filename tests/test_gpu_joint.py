"""The joint CG + LOBPCG driver (Algorithms 2 and 3 side by side on one
operator, sharing each step's stencil pass where the operator offers a joint
apply): its outputs against the single filters on the GPU and against the
oracle.  Tolerances: the CG dot products are summed in another order (the
joint apply's tiles), so CG agrees with the single filter to 1e-12 (FP64) /
1e-5 (FP32) and LOBPCG, which sees the same operations, bitwise or to the
same bounds; against the oracle as for the single filters (FP64: max(1e-12,
10 band) with the oracle's self-sensitivity band, tests/sensitivity.py)."""
import numpy as np
import pytest

import oracle
from sensitivity import reference
from synth import piecewise_constant_1d, scene_2d

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return max(np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max())


def _dev(x, prec, gsf):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float32 if prec == gsf.F32 else torch.float64,
                        device="cuda")


CASES = [
    ("bf", (67, 130), 3, dict(radius=3, sigma_d=2.0, sigma_r=0.1), 4),   # joint apply (square window, m = 4)
    ("bf", (40, 70), 4, dict(radius=5, sigma_d=2.0, sigma_r=0.1), 1),    # joint apply, m = 1
    ("bf", (3000,), 5, dict(radius=4, sigma_d=3.0, sigma_r=0.2), 4),     # 1D joint apply
    ("bf", (50, 90), 6, dict(radius=2, sigma_d=2.0, sigma_r=0.1), 3),    # m = 3: two applies
    ("gf", (60, 70), 7, dict(radius=2, eps=1e-2), 4),                    # GF: two applies
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,shape,seed,par,m", CASES)
def test_joint_equals_single_filters(gsf, kind, shape, seed, par, m, prec):
    x = piecewise_constant_1d(shape[0], 0.1, seed)[1] if len(shape) == 1 else scene_2d(*shape, 0.05, seed)[1]
    x = x.astype(np.float32).astype(np.float64) if prec == gsf.F32 else x
    xd = _dev(x.ravel(), prec, gsf)
    op = gsf.Operator(kind, shape, xd, **par, prec=prec)
    # a second signal of the same kind for CG, so that a mix-up of the inputs shows
    z = piecewise_constant_1d(shape[0], 0.1, seed + 100)[1] if len(shape) == 1 else \
        scene_2d(*shape, 0.05, seed + 100)[1]
    z0 = _dev(z.ravel(), prec, gsf)
    for kcg, klob in ((12, 12), (15, 9), (6, 14)):
        for constraint in (False, True):
            ycg, ylob, ci, li = op.joint_filter(z0, kcg, xd, m, klob, constraint=constraint)
            rcg, rci = op.cg_filter(z0, kcg)
            rlob, rli = op.lobpcg_filter(xd, m, klob, constraint=constraint)
            ecg, elob = rel(ycg.cpu().numpy(), rcg.cpu().numpy()), rel(ylob.cpu().numpy(), rlob.cpu().numpy())
            print(f"joint {kind} {shape} m={m} prec={prec} k=({kcg},{klob}) c={constraint}: cg {ecg:.1e} "
                  f"lobpcg {elob:.1e}")
            assert ci.iters == rci.iters == kcg and li.iters == rli.iters == klob
            assert ecg <= (1e-12 if prec == gsf.F64 else 1e-5)
            assert elob <= (1e-12 if prec == gsf.F64 else 1e-5)


def test_joint_against_oracle(gsf):
    shape, seed = (67, 130), 8
    x = scene_2d(*shape, 0.05, seed)[1]
    par = dict(radius=3, sigma_d=2.0, sigma_r=0.1)
    xd = _dev(x.ravel(), gsf.F64, gsf)
    op = gsf.Operator("bf", shape, xd, **par, prec=gsf.F64)
    ycg, ylob, ci, li = op.joint_filter(xd, 20, xd, 4, 20, constraint=True)

    def lob(g):
        y, th, _, info = oracle.lobpcg_filter(oracle.build_operator("bf", g, 3, 2.0, 0.1), g.ravel(), 4, 20,
                                              constraint=True)
        return y, (th, info)

    rcg = reference(lambda g: oracle.cg_filter(oracle.build_operator("bf", g, 3, 2.0, 0.1), g.ravel(), 20), x)
    rlob = reference(lob, x)
    th, rinfo = rlob.extra
    assert rel(ycg.cpu().numpy(), rcg.y) <= rcg.gate
    assert rel(ylob.cpu().numpy(), rlob.y) <= rlob.gate
    if rinfo.dropped == rlob.extra_reversed[1].dropped:
        assert li.dropped == rinfo.dropped
    np.testing.assert_allclose(np.array(li.theta[:4]), th, rtol=max(1e-9, rlob.gate), atol=1e-12)


def test_joint_apply_rows_agree(gsf):
    """The joint apply follows the tile chosen for the m-column block: every
    choice gives the single-filter results."""
    shape = (67, 130)
    x = scene_2d(*shape, 0.05, 9)[1]
    xd = _dev(x.ravel(), gsf.F64, gsf)
    op = gsf.Operator("bf", shape, xd, radius=3, sigma_d=2.0, sigma_r=0.1, prec=gsf.F64)
    rcg, _ = op.cg_filter(xd, 10)
    rlob, _ = op.lobpcg_filter(xd, 4, 10)
    for rows in (1, 2, 4):
        op.set_apply_rows(4, rows)
        ycg, ylob, _, _ = op.joint_filter(xd, 10, xd, 4, 10)
        assert rel(ycg.cpu().numpy(), rcg.cpu().numpy()) <= 1e-12
        assert rel(ylob.cpu().numpy(), rlob.cpu().numpy()) <= 1e-12


def test_joint_fullsize_bench_configuration(gsf):
    """The bench step's configuration (1024^2, BF 11x11, FP32, CG 50 and
    LOBPCG m = 4 50 steps, the tile the tuner picks): the joint driver against
    the two single filters, whose full-size parity with the oracle the
    full-size tests establish."""
    import torch
    from synth import WORKLOADS, make_signal
    w = WORKLOADS["image_1024_bf11"]
    _, noisy = make_signal("image_1024_bf11")
    x0 = torch.tensor(noisy.ravel().astype(np.float32), device="cuda")
    op = gsf.Operator("bf", w["shape"], x0, w["radius"], w["sigma_d"], w["sigma_r"], 0.0, gsf.F32)
    op.tune_apply(1, reps=5)
    op.tune_apply(w["lobpcg_m"], reps=5)
    ycg, ylob, ci, li = op.joint_filter(x0, w["cg_iters"], x0, w["lobpcg_m"], w["lobpcg_iters"])
    rcg, rci = op.cg_filter(x0, w["cg_iters"])
    rlob, rli = op.lobpcg_filter(x0, w["lobpcg_m"], w["lobpcg_iters"])
    ecg, elob = rel(ycg.cpu().numpy(), rcg.cpu().numpy()), rel(ylob.cpu().numpy(), rlob.cpu().numpy())
    print(f"joint 1024^2: cg {ecg:.2e}, lobpcg {elob:.2e}, theta {list(li.theta[:4])}")
    assert ci.iters == rci.iters == w["cg_iters"] and li.iters == rli.iters == w["lobpcg_iters"]
    assert ecg <= 1e-5 and elob <= 1e-5
    np.testing.assert_allclose(np.array(li.theta[:4]), np.array(rli.theta[:4]), rtol=1e-6)


def test_joint_edge_cases(gsf):
    """kmax = 0 on either side (the other filter runs alone; zero steps return
    the input for CG and the start-block projection for LOBPCG, as the single
    filters do); a constant CG input breaks down at once while LOBPCG runs on."""
    shape = (40, 70)
    x = scene_2d(*shape, 0.05, 12)[1]
    xd = _dev(x.ravel(), gsf.F64, gsf)
    op = gsf.Operator("bf", shape, xd, radius=2, sigma_d=2.0, sigma_r=0.1, prec=gsf.F64)
    for kcg, klob in ((0, 8), (8, 0), (0, 0)):
        ycg, ylob, ci, li = op.joint_filter(xd, kcg, xd, 4, klob)
        rcg, _ = op.cg_filter(xd, kcg)
        rlob, _ = op.lobpcg_filter(xd, 4, klob)
        assert rel(ycg.cpu().numpy(), rcg.cpu().numpy()) <= 1e-13
        assert rel(ylob.cpu().numpy(), rlob.cpu().numpy()) <= 1e-13
        assert ci.iters == kcg and li.iters == klob
    c = _dev(np.full(op.n, 0.3), gsf.F64, gsf)
    ycg, ylob, ci, li = op.joint_filter(c, 10, xd, 4, 10)
    assert ci.status == gsf.EBREAKDOWN and ci.iters == 0
    np.testing.assert_allclose(ycg.cpu().numpy(), 0.3, rtol=1e-15)  # z = D^1/2 x and back
    rlob, _ = op.lobpcg_filter(xd, 4, 10)
    assert li.iters == 10 and rel(ylob.cpu().numpy(), rlob.cpu().numpy()) <= 1e-13
