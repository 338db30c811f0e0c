"""A seeded sweep of whole filters against the oracle: power iteration, CG
(Algorithm 2) and block LOBPCG (Algorithm 3) on BF and GF operators of
uneven 1D and 2D grids, with random radius, block width, step count,
constraint and tolerance, in FP32 and FP64.  The gates are those of the
fixed parity cases: FP32 outputs within 1e-5 relative, FP64 outputs within
max(1e-12, 10 x) the oracle's own band under a relabelling of the points;
the decisions (steps taken, columns dropped) are compared first wherever the
oracle's forward and reversed runs take them the same way.

FP32 LOBPCG: a column whose residual nears the FP32 resolution of the apply
(about 2^-24 of the column) has a W column made mostly of rounding, and the
Rayleigh-Ritz step drops it on the FP32 pivot threshold (1e-6) where the FP64
run keeps it.  Each such drop moves the output by a discrete amount that no
FP32 run can avoid, so the FP32 gate is max(1e-5, 10 x) the oracle's own
change between its FP32 and FP64 drop thresholds on the case (zero while no
column is dropped)."""
import numpy as np
import pytest

import oracle
from sensitivity import reference, rel
from synth import piecewise_constant_1d, scene_2d

pytestmark = pytest.mark.gpu


def _cases(count=60, seed=77):
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        kind = "bf" if rng.uniform() < 0.6 else "gf"
        if rng.uniform() < 0.35:
            shape = (int(rng.integers(200, 5000)),)
        else:
            shape = (int(rng.integers(8, 60)), int(rng.integers(8, 90)))
        prec = int(rng.integers(0, 2))
        out.append(dict(c=c, kind=kind, shape=shape, radius=int(rng.integers(1, 6)),
                        method=("power", "cg", "lobpcg")[c % 3], m=int(rng.integers(1, 5)),
                        k=int(rng.integers(3, 25)), prec=prec, constraint=bool(rng.uniform() < 0.5),
                        tol=float(rng.choice([0.0, 1e-4])) if prec == 1 else 0.0))
    return out


def _label(d):
    return f"{d['c']}-{d['kind']}-{d['method']}-{'x'.join(map(str, d['shape']))}-p{d['prec']}"


@pytest.mark.parametrize("case", _cases(), ids=_label)
def test_filter_sweep(gsf, case):
    import torch
    c, kind, shape, prec, k, m = case["c"], case["kind"], case["shape"], case["prec"], case["k"], case["m"]
    if len(shape) == 1:
        x = piecewise_constant_1d(shape[0], 0.1, 300 + c)[1]
    else:
        x = scene_2d(shape[0], shape[1], 0.05, 300 + c, n_shapes=6)[1]
    if prec == 0:
        x = x.astype(np.float32).astype(np.float64)
    par = dict(radius=case["radius"], sigma_d=2.0, sigma_r=0.2) if kind == "bf" else \
        dict(radius=case["radius"], eps=1e-2)
    print(f"case {case}", flush=True)
    xd = torch.tensor(x.ravel(), dtype=torch.float32 if prec == 0 else torch.float64, device="cuda")
    op = gsf.Operator(kind, shape, xd, prec=prec, **par)
    dp = "f64" if prec == 1 else "f32"
    grid = x.reshape(shape)

    def oop(g):
        return oracle.build_operator(kind, g, par["radius"], sigma_s=par.get("sigma_d", 0.0),
                                     sigma_r=par.get("sigma_r", 0.0), eps=par.get("eps", 0.0))

    if case["method"] == "power":
        y = op.power_filter(xd, k).cpu().numpy()
        ref = reference(lambda g: (oracle.power_filter(oop(g), g.ravel(), k), None), grid)
        e = rel(y, ref.y)
        gate = ref.gate if prec == 1 else 1e-5
    elif case["method"] == "cg":
        y, info = op.cg_filter(xd, k, tol=case["tol"])
        ref = reference(lambda g: oracle.cg_filter(oop(g), g.ravel(), k, tol=case["tol"], data_prec=dp), grid)
        if ref.extra.iters == ref.extra_reversed.iters:
            assert info.iters == ref.extra.iters, (info.iters, ref.extra.iters)
        e = rel(y.cpu().numpy(), ref.y)
        gate = ref.gate if prec == 1 else 1e-5
    else:
        y, info = op.lobpcg_filter(xd, m, k, tol=case["tol"], constraint=case["constraint"])

        def run(g):
            yy, th, _, rinfo = oracle.lobpcg_filter(oop(g), g.ravel(), m, k, tol=case["tol"],
                                                    constraint=case["constraint"], data_prec=dp)
            return yy, (th, rinfo)

        ref = reference(run, grid)
        th, rinfo = ref.extra
        _, rrev = ref.extra_reversed
        if rinfo.status == "breakdown":
            assert info.status == gsf.EBREAKDOWN
            return
        if rinfo.iters == rrev.iters:
            assert info.iters == rinfo.iters, (info.iters, rinfo.iters)
        if rinfo.dropped == rrev.dropped:
            assert info.dropped == rinfo.dropped, (info.dropped, rinfo.dropped)
        theta = np.array(list(info.theta)[:m])
        if prec == 1:
            np.testing.assert_allclose(theta, th, rtol=max(1e-9, ref.gate), atol=1e-12)
            gate = ref.gate
        else:
            assert np.abs(theta - th).max() <= 2e-5
            y64 = oracle.lobpcg_filter(oop(grid), x, m, k, tol=case["tol"], constraint=case["constraint"],
                                       data_prec="f64")[0]
            drop_band = rel(ref.y, y64)
            gate = max(1e-5, 10.0 * drop_band)
            print(f"  FP32 drop-threshold band {drop_band:.2e}")
        e = rel(y.cpu().numpy(), ref.y)
    print(f"  rel err {e:.2e} gate {gate:.1e}")
    assert e <= gate, e
