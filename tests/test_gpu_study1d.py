"""GPU parity of the 1D filter study (Section 6) through the C ABI, against
the FP64 oracle, on both signal lengths: self-guided BF (500 re-guided
passes), self-guided GF (20 re-guided passes), BF-CG with the noiseless
guidance (20 steps), and the GF-accelerated CG and LOBPCG and BF-LOBPCG
(20 steps, noiseless guidance).

Tolerances (relative, 2-norm and max-norm), FP64: CG and LOBPCG max(1e-12,
10 band) as for the other filters (the band is the oracle's own
self-sensitivity: the case with its samples in reverse order,
tests/sensitivity.py); the re-guided passes feed every result back into
the weights, where a change of the guidance moves a weight by about
|g_i - g_j| / sigma_r^2 (~10) times as much, so 1e-12 for both the 500 BF and
the 20 GF passes (measured: 1.4e-15 and 2.3e-15; the passes contract the
differences more than the weights amplify them).
"""
import numpy as np
import pytest

import oracle
from sensitivity import reference
from synth import STUDY_1D, study_signal

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return max(np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max())


def _dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


BF = STUDY_1D["bf"]
GF = STUDY_1D["gf"]
K = STUDY_1D["krylov_steps"]


@pytest.mark.parametrize("n", STUDY_1D["sizes"])
def test_self_guided_bf_and_gf(gsf, n):
    clean, noisy = study_signal(n)
    y, info = gsf.reguided_filter("bf", (n,), _dev(noisy), gsf.METHOD_POWER, BF["passes"], radius=BF["radius"],
                                  sigma_d=BF["sigma_d"], sigma_r=BF["sigma_r"], prec=gsf.F64)
    r = oracle.power_filter_reguided("bf", noisy, (n,), BF["passes"], radius=BF["radius"], sigma_s=BF["sigma_d"],
                                     sigma_r=BF["sigma_r"])
    e = rel(y.cpu().numpy(), r)
    print(f"N={n} self-guided BF x{BF['passes']}: {e:.2e}")
    assert info.iters == BF["passes"] and e <= 1e-12
    y, info = gsf.reguided_filter("gf", (n,), _dev(noisy), gsf.METHOD_POWER, GF["passes"], radius=GF["radius"],
                                  eps=GF["eps"], prec=gsf.F64)
    r = oracle.power_filter_reguided("gf", noisy, (n,), GF["passes"], radius=GF["radius"], eps=GF["eps"])
    e = rel(y.cpu().numpy(), r)
    print(f"N={n} self-guided GF x{GF['passes']}: {e:.2e}")
    assert info.iters == GF["passes"] and e <= 1e-12


@pytest.mark.parametrize("n", STUDY_1D["sizes"])
def test_krylov_filters_noiseless_guidance(gsf, n):
    """BF-CG (the paper's), and the GF-accelerated CG / LOBPCG and BF-LOBPCG,
    all with the noiseless signal as the guidance."""
    clean, noisy = study_signal(n)
    gd, xd = _dev(clean), _dev(noisy)
    bf = gsf.Operator("bf", (n,), gd, radius=BF["radius"], sigma_d=BF["sigma_d"], sigma_r=BF["sigma_r"],
                      prec=gsf.F64)
    gf = gsf.Operator("gf", (n,), gd, radius=GF["radius"], eps=GF["eps"], prec=gsf.F64)
    def rbf(g):
        return oracle.build_operator("bf", g, BF["radius"], BF["sigma_d"], BF["sigma_r"])

    def rgf(g):
        return oracle.build_operator("gf", g, GF["radius"], eps=GF["eps"])

    for name, op, mk in (("BF", bf, rbf), ("GF", gf, rgf)):
        y, info = op.cg_filter(xd, K)
        rr = reference(lambda g, v: oracle.cg_filter(mk(g), v, K), clean, noisy)
        r, rinfo = rr.y, rr.extra
        e = rel(y.cpu().numpy(), r)
        print(f"N={n} {name}-CG {K}: {e:.2e} (band {rr.band:.1e})")
        assert info.iters == rinfo.iters == K and e <= rr.gate
        y, info = op.lobpcg_filter(xd, 1, K)
        rr = reference(lambda g, v: (lambda o: (o[0], o[1]))(oracle.lobpcg_filter(mk(g), v, 1, K)), clean, noisy)
        r, th = rr.y, rr.extra
        e = rel(y.cpu().numpy(), r)
        print(f"N={n} {name}-LOBPCG {K}: {e:.2e} (band {rr.band:.1e}), theta {info.theta[0]:.6e} vs {th[0]:.6e}")
        assert info.iters == K and e <= rr.gate
        np.testing.assert_allclose(info.theta[0], th[0], rtol=max(1e-9, rr.gate), atol=1e-12)


def test_study_errors_below_noise(gsf):
    """Every filter of the study leaves a smaller error than the noise
    (the paper: high-quality denoising by all three)."""
    for n in STUDY_1D["sizes"]:
        clean, noisy = study_signal(n)
        e0 = np.sqrt(np.mean((noisy - clean) ** 2))
        y, _ = gsf.reguided_filter("bf", (n,), _dev(noisy), gsf.METHOD_POWER, BF["passes"], radius=BF["radius"],
                                   sigma_d=BF["sigma_d"], sigma_r=BF["sigma_r"], prec=gsf.F64)
        e1 = np.sqrt(np.mean((y.cpu().numpy() - clean) ** 2))
        y, _ = gsf.reguided_filter("gf", (n,), _dev(noisy), gsf.METHOD_POWER, GF["passes"], radius=GF["radius"],
                                   eps=GF["eps"], prec=gsf.F64)
        e2 = np.sqrt(np.mean((y.cpu().numpy() - clean) ** 2))
        op = gsf.Operator("bf", (n,), _dev(clean), radius=BF["radius"], sigma_d=BF["sigma_d"],
                          sigma_r=BF["sigma_r"], prec=gsf.F64)
        y, _ = op.cg_filter(_dev(noisy), K)
        e3 = np.sqrt(np.mean((y.cpu().numpy() - clean) ** 2))
        print(f"N={n}: noise {e0:.4f}, BF x500 {e1:.4f}, GF x20 {e2:.4f}, BF-CG 20 {e3:.4f}")
        assert max(e1, e2, e3) < e0
