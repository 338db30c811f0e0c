"""Graph capture of whole filter calls: the solver loops issue kernels and
device-to-device copies only (state set by kernels, no memset nodes, no host
reads when no summary is asked for), so a caller can record gsf_power_filter,
gsf_cg_filter and gsf_lobpcg_filter into one HIP graph and replay it.  Every
replay, with unrelated eager work and synchronisations between replays,
equals the eager calls bitwise.  Also the tuned-tile table's file round trip
on a built operator."""
import numpy as np
import pytest

from synth import piecewise_constant_1d, scene_2d

pytestmark = pytest.mark.gpu

CASES = [
    ("bf", (4096,), dict(radius=5, sigma_d=3.0, sigma_r=0.2)),     # one-workgroup CG path
    ("bf", (96, 130), dict(radius=5, sigma_d=2.0, sigma_r=0.1)),
    ("gf", (90, 120), dict(radius=4, eps=1e-2)),                    # one-pass GF apply (CG, power)
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,shape,par", CASES)
def test_filters_replay_in_a_graph(gsf, kind, shape, par, prec):
    import torch
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    x = piecewise_constant_1d(shape[0], 0.1, 3)[1] if len(shape) == 1 else scene_2d(*shape, 0.05, 3)[1]
    x0 = torch.tensor(np.ascontiguousarray(x).ravel(), dtype=dt, device="cuda")
    op = gsf.Operator(kind, shape, x0, **par, prec=prec)
    m, k = 4, 15
    wp, wc, wl = op.workspace(gsf.METHOD_POWER), op.workspace(gsf.METHOD_CG), op.workspace(gsf.METHOD_LOBPCG, m)
    yp, yc, yl = torch.empty_like(x0), torch.empty_like(x0), torch.empty_like(x0)

    def calls():
        op.power_filter(x0, k, out=yp, ws=wp)
        op.cg_filter(x0, k, out=yc, ws=wc, info=False)
        op.lobpcg_filter(x0, m, k, out=yl, ws=wl, info=False)

    calls()
    torch.cuda.synchronize()
    ref = [v.clone() for v in (yp, yc, yl)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        calls()
    for rep in range(3):
        for v in (yp, yc, yl):
            v.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 18, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        for name, v, r in zip(("power", "cg", "lobpcg"), (yp, yc, yl), ref):
            assert torch.equal(v, r), (rep, name)
    del junk


def test_tuned_tiles_survive_a_file_round_trip(gsf, tmp_path):
    import torch
    shape = (256, 256)
    g = torch.tensor(scene_2d(*shape, 0.05, 4)[1].ravel(), dtype=torch.float32, device="cuda")
    op = gsf.Operator("bf", shape, g, radius=5, sigma_d=2.0, sigma_r=0.1, prec=gsf.F32)
    gsf.tune_table_clear()
    default = op.apply_rows(4)
    choice = 1 if default != 1 else 4
    op.set_apply_rows(4, choice)
    assert op.apply_rows(4) == choice
    path = tmp_path / "tiles.json"
    assert gsf.tune_table_save(str(path)) >= 1
    gsf.tune_table_clear()
    assert op.apply_rows(4) == default
    assert gsf.tune_table_load(str(path)) >= 1
    assert op.apply_rows(4) == choice
    best, times = op.tune_apply(4, reps=3)
    assert op.apply_rows(4) == best and len(times) == 3
    assert op.apply_rows(1) in (1, 2, 4)
    gsf.tune_table_clear()
