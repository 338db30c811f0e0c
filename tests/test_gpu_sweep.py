"""A seeded sweep of operator applies against the oracle, for edge cases the
fixed parity cases may miss: BF and GF, 1D and 2D grids of uneven sizes
(from a single point up to several tiles and strips wide, with ragged
edges), every radius 1..8, block widths 1..8, FP32 and FP64, all four forms
(N, L_sym, D^-1 W, L).  Bars: 1e-5 relative for FP32, 1e-12 for FP64, relative
to the larger of the output's and the input's scale (a Laplacian form
vanishes on a constant).  Each case is printed before it runs."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-12}


def _cases(count=120, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        kind = "bf" if c % 2 == 0 else "gf"
        ndim = 1 if rng.uniform() < 0.3 else 2
        radius = int(rng.integers(1, 9))
        if ndim == 1:
            shape = (int(rng.integers(1, 3000)),)
        else:
            shape = (int(rng.integers(1, 80)), int(rng.integers(1, 330)))
        m = int(rng.choice([1, 1, 2, 3, 4, 5, 8]))
        prec = int(rng.integers(0, 2))
        out.append((c, kind, shape, radius, m, prec))
    return out


@pytest.mark.parametrize("c,kind,shape,radius,m,prec", _cases())
def test_apply_sweep(gsf, c, kind, shape, radius, m, prec):
    import torch
    rng = np.random.default_rng(1000 + c)
    g = rng.uniform(0.0, 1.0, shape)
    # a piecewise guidance: a few level steps so that weights vary
    g = np.round(g * 3.0) / 3.0 + 0.05 * rng.standard_normal(shape)
    dt = torch.float32 if prec == 0 else torch.float64
    if prec == 0:
        g = g.astype(np.float32).astype(np.float64)
    par = dict(radius=radius, sigma_d=2.0, sigma_r=0.2) if kind == "bf" else dict(radius=radius, eps=1e-2)
    print(f"case {c}: {kind} {shape} r={radius} m={m} prec={prec}", flush=True)
    op = gsf.Operator(kind, shape, torch.tensor(g.ravel(), dtype=dt, device="cuda"), **par, prec=prec)
    ref = oracle.build_operator(kind, g, radius, sigma_s=par.get("sigma_d", 0.0), sigma_r=par.get("sigma_r", 0.0),
                                eps=par.get("eps", 0.0))
    X = rng.standard_normal((op.n, m))
    if prec == 0:
        X = X.astype(np.float32).astype(np.float64)
    Xd = torch.tensor(X if m > 1 else X[:, 0], dtype=dt, device="cuda")
    for form in (gsf.FORM_N, gsf.FORM_LSYM, gsf.FORM_RW, gsf.FORM_L):
        Y = op.apply(Xd, form).cpu().numpy().reshape(op.n, m)
        R = ref.apply(form, X)
        scale2 = max(np.linalg.norm(R), np.linalg.norm(X))
        scalei = max(np.abs(R).max(), np.abs(X).max())
        e = max(np.linalg.norm(Y - R) / scale2, np.abs(Y - R).max() / scalei)
        assert e <= TOL[prec], (form, e)
