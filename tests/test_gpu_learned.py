"""GPU parity of the learned preconditioner (the preconditioner slot of
Algorithm 3): the network's training kernels (forward, loss, gradients,
Adam), the fused MFMA inference kernel, the training-pair kernels (shifted
CG, residual block, scaling) and flexible LOBPCG with T, against the FP64
oracle with the same BF16 rounding points, called through the C ABI.

Tolerances.  The oracle rounds weights, inputs and the two hidden
activations to BF16 exactly where the kernels do and is exact elsewhere; the
kernels accumulate in FP32.  A 144-term FP32 dot product of BF16 operands is
off by at most ~144 * 2^-24 (~1e-5) of its absolute sum, which moves the
subsequent BF16 rounding of an activation by one BF16 unit (2^-8 relative) in
a small fraction of elements (those within 1e-5 of a rounding midpoint,
~1e-5 / 2^-8 ~ 3e-3 of them at most).  Each such flip perturbs the output by
under 2^-8 of one term, so the network output is bounded normwise by
2^-8 * sqrt(3e-3) ~ 2e-4; we gate at 1e-3 normwise for outputs and
gradients.  Everything outside the network (shifted CG, residual, pairs,
Adam in FP32 against FP64) is compared at the precision of its arithmetic.
"""
import numpy as np
import pytest

import oracle
from oracle import convnet as cn
from oracle.spectral import dense_normalized
from synth import convnet_init, scene_2d

pytestmark = pytest.mark.gpu

NET_TOL = 1e-3


def nrel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dev(x, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _samples(B, H, W, seed):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((B, H, W))
    g = np.stack([scene_2d(H, W, 0.05, seed + 100 + b)[1] for b in range(B)])
    t = rng.standard_normal((B, H, W)) * 3.0
    return r, g, t


def _train_arrays(r, g, t):
    import torch
    B = r.shape[0]
    inp = np.stack([r.reshape(B, -1), g.reshape(B, -1)], axis=-1).astype(np.float32)
    return _dev(inp, torch.float32), _dev(t.reshape(B, -1).astype(np.float32), torch.float32)


def _bf16_bits(w):
    import torch
    wt = torch.tensor(np.asarray(w, dtype=np.float32)).to(torch.bfloat16)
    return wt.view(torch.int16).to("cuda")


@pytest.mark.parametrize("shape", [(37, 45), (16, 16), (1, 300)])
def test_net_forward_matches_oracle(gsf, shape):
    import torch
    H, W = shape
    B = 3
    r, g, t = _samples(B, H, W, 1)
    w = convnet_init(11)
    inp, tg = _train_arrays(r, g, t)
    tr = gsf.NetTrainer(w, B, H, W)
    idx = _dev(np.array([2, 0, 1], dtype=np.int32), torch.int32)
    y = tr.forward(idx, inp).reshape(B, H, W).cpu().numpy()
    wr = w.astype(np.float64)
    for b, s in enumerate([2, 0, 1]):
        ref = cn.forward(wr, r[s].astype(np.float32), g[s].astype(np.float32))["y"]
        e = nrel(y[b], ref)
        print(f"forward {shape} sample {s}: rel {e:.2e}")
        assert e <= NET_TOL


@pytest.mark.parametrize("shape", [(37, 45), (20, 33)])
def test_net_loss_grad_matches_oracle(gsf, shape):
    import torch
    H, W = shape
    B = 4
    r, g, t = _samples(B, H, W, 2)
    w = convnet_init(12)
    inp, tg = _train_arrays(r, g, t)
    tr = gsf.NetTrainer(w, B, H, W)
    idx = _dev(np.arange(B, dtype=np.int32)[::-1].copy(), torch.int32)
    loss, grad = tr.loss_grad(idx, inp, tg)
    loss = float(loss.cpu()[0])
    grad = grad.cpu().numpy()
    order = list(range(B))[::-1]
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    ref_loss, ref_grad = cn.loss_and_grad(w.astype(np.float64), f32(r[order]), f32(t[order]), f32(g[order]))
    el, eg = abs(loss - ref_loss) / ref_loss, nrel(grad, ref_grad)
    per_layer = [nrel(grad[a:b], ref_grad[a:b]) for a, b in ((0, 288), (288, 2592), (2592, 2736))]
    print(f"loss_grad {shape}: loss rel {el:.2e}, grad rel {eg:.2e}, per layer {per_layer}")
    assert el <= NET_TOL
    assert eg <= NET_TOL and max(per_layer) <= 3 * NET_TOL


def test_adam_matches_oracle(gsf):
    import torch
    rng = np.random.default_rng(3)
    w0 = convnet_init(13)
    tr = gsf.NetTrainer(w0, 1, 8, 8)
    w_ref, m_ref, v_ref = w0.astype(np.float64), np.zeros(w0.size), np.zeros(w0.size)
    for t in range(1, 4):
        g = (rng.standard_normal(w0.size) * 1e-2).astype(np.float32)
        tr.grad.copy_(_dev(g, torch.float32))
        tr.adam(lr=1e-3)
        w_ref, m_ref, v_ref = cn.adam_step(w_ref, m_ref, v_ref, g.astype(np.float64), t, lr=1e-3)
    w_gpu = tr.w.cpu().numpy()
    assert nrel(w_gpu, w_ref) <= 1e-6
    assert np.abs(w_gpu - w_ref).max() <= 1e-6
    wb = tr.wb.view(torch.bfloat16).float().cpu().numpy()
    np.testing.assert_array_equal(wb, cn.bf16_round(w_gpu.astype(np.float64)))


@pytest.mark.parametrize("prec_name", ["f32", "f64"])
@pytest.mark.parametrize("shape,m", [((61, 75), 3), ((28, 28), 1), ((100, 57), 4), ((1, 500), 2)])
def test_precond_apply_matches_oracle(gsf, prec_name, shape, m):
    """Fused MFMA inference: T(R) column by column (tiles of 28 x 28 with
    ragged edges, 1D as one row)."""
    import torch
    prec = gsf.F32 if prec_name == "f32" else gsf.F64
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    H, W = shape
    g = scene_2d(H, W, 0.05, 7)[1] if H > 1 else np.random.default_rng(7).uniform(0, 1, (1, W))
    R = np.random.default_rng(8).standard_normal((H * W, m)) * np.array([1.0, 1e-3, 40.0, 2.0])[:m]
    if prec == gsf.F32:
        R = R.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    op = gsf.Operator("bf", (H, W) if H > 1 else (W,), _dev(g.ravel(), dt), 2, 2.0, 0.1, prec=prec)
    w = convnet_init(14)
    T = gsf.Precond(op, _dev(g.ravel(), dt), _bf16_bits(w))
    out = T.apply(_dev(R, dt)).cpu().numpy()
    for j in range(m):
        ref = cn.precond_apply(w.astype(np.float64), R[:, j].reshape(H, W), g.reshape(H, W)).ravel()
        e = nrel(out[:, j], ref)
        print(f"precond {prec_name} {shape} col {j}: rel {e:.2e}")
        assert e <= NET_TOL


def test_fused_inference_equals_training_forward(gsf):
    """The fused MFMA kernel and the per-layer training kernels compute the
    same network (up to FP32 summation order)."""
    import torch
    H, W = 90, 70
    g = scene_2d(H, W, 0.05, 9)[1].astype(np.float32)
    r = np.random.default_rng(10).standard_normal(H * W).astype(np.float32)
    s = np.sqrt(np.mean(r.astype(np.float64) ** 2))
    op = gsf.Operator("bf", (H, W), _dev(g.ravel(), torch.float32), 2, 2.0, 0.1, prec=gsf.F32)
    w = convnet_init(15)
    T = gsf.Precond(op, _dev(g.ravel(), torch.float32), _bf16_bits(w))
    fused = T.apply(_dev(r.reshape(-1, 1), torch.float32)).cpu().numpy().ravel()
    tr = gsf.NetTrainer(w, 1, H, W)
    inp = np.stack([(r / s).astype(np.float32), g.ravel()], axis=-1)[None]
    y = tr.forward(_dev(np.zeros(1, np.int32), torch.int32), _dev(inp, torch.float32)).cpu().numpy()
    e = nrel(fused, s * y)
    print(f"fused vs training forward: {e:.2e}")
    assert e <= NET_TOL


def test_shifted_cg_matches_oracle(gsf):
    import torch
    H, W = 45, 52
    g = scene_2d(H, W, 0.05, 11)[1]
    op = gsf.Operator("bf", (H, W), _dev(g.ravel(), torch.float64), 3, 2.0, 0.1, prec=gsf.F64)
    oop = oracle.build_operator("bf", g, 3, 2.0, 0.1)
    B = np.random.default_rng(12).standard_normal((H * W, 3))
    Bd = _dev(B, torch.float64)
    y, info = op.shifted_cg(1e-2, Bd[:, 1], 5000, 1e-10, ldb=3)
    ref, rinfo = oracle.shifted_cg(oop, 1e-2, B[:, 1], 5000, 1e-10)
    e = nrel(y.cpu().numpy(), ref)
    print(f"shifted CG: iters {info.iters} vs {rinfo.iters}, rel {e:.2e}")
    assert info.status == gsf.OK and rinfo.status == "ok"
    assert abs(info.iters - rinfo.iters) <= 1
    assert e <= 1e-9
    # fixed step count: same iterates
    y5, _ = op.shifted_cg(1e-2, Bd[:, 1], 5, 0.0, ldb=3)
    ref5, _ = oracle.shifted_cg(oop, 1e-2, B[:, 1], 5, 0.0)
    assert nrel(y5.cpu().numpy(), ref5) <= 1e-12
    # zero right-hand side
    z, zi = op.shifted_cg(1e-2, torch.zeros(H * W, dtype=torch.float64, device="cuda"), 10, 1e-10)
    assert zi.iters == 0 and zi.status == gsf.OK and float(z.abs().max()) == 0.0


def test_residual_and_pair_match_oracle(gsf):
    import torch
    H, W = 33, 41
    g = scene_2d(H, W, 0.05, 13)[1]
    op = gsf.Operator("bf", (H, W), _dev(g.ravel(), torch.float64), 2, 2.0, 0.1, prec=gsf.F64)
    oop = oracle.build_operator("bf", g, 2, 2.0, 0.1)
    X = np.random.default_rng(14).standard_normal((H * W, 4))
    th = [0.01, 0.02, 0.5, 1.2]
    R = op.lobpcg_residual(_dev(X, torch.float64), th)
    Rr = oracle.lobpcg_residual(oop, X, th)
    assert nrel(R.cpu().numpy(), Rr) <= 1e-12
    y = _dev(np.random.default_rng(15).standard_normal(H * W), torch.float64)
    inp = torch.empty((H * W, 2), dtype=torch.float32, device="cuda")
    tg = torch.empty(H * W, dtype=torch.float32, device="cuda")
    keep = op.make_pair(R[:, 2], y, _dev(g.ravel(), torch.float64), inp, tg, ldr=4)
    torch.cuda.synchronize()
    del keep
    s = cn.rms(Rr[:, 2])
    np.testing.assert_allclose(inp[:, 0].cpu().numpy(), (Rr[:, 2] / s).astype(np.float32), rtol=1e-6, atol=0)
    np.testing.assert_array_equal(inp[:, 1].cpu().numpy(), g.ravel().astype(np.float32))
    np.testing.assert_allclose(tg.cpu().numpy(), (y.cpu().numpy() / s).astype(np.float32), rtol=1e-6, atol=0)


def _lob_case(gsf, prec, H=40, W=48, seed=16):
    import torch
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    g = scene_2d(H, W, 0.05, seed)[1]
    if prec == gsf.F32:
        g = g.astype(np.float32).astype(np.float64)
    op = gsf.Operator("bf", (H, W), _dev(g.ravel(), dt), 2, 2.0, 0.1, prec=prec)
    oop = oracle.build_operator("bf", g, 2, 2.0, 0.1)
    return op, oop, g, _dev(g.ravel(), dt)


@pytest.mark.parametrize("kind", ["nan", "negated"])
def test_lobpcg_fallback_equals_plain(gsf, kind):
    """Every column falls back to T = I: bitwise the plain method."""
    op, oop, g, gd = _lob_case(gsf, gsf.F64)
    if kind == "nan":
        w = convnet_init(17)
        w[500] = np.nan
    else:
        w = cn.identity_weights().astype(np.float32)
        w[cn.N_W1 + cn.N_W2:] *= -1.0
    T = gsf.Precond(op, gd, _bf16_bits(w))
    m, k = 3, 6
    plain, pinfo = op.lobpcg_filter(gd, m, k, constraint=True)
    learned, linfo = op.lobpcg_filter(gd, m, k, constraint=True, precond=T)
    assert linfo.fallbacks == m * k
    assert pinfo.fallbacks == 0
    np.testing.assert_array_equal(learned.cpu().numpy(), plain.cpu().numpy())
    assert list(linfo.theta) == list(pinfo.theta)


@pytest.mark.parametrize("constraint", [False, True])
def test_lobpcg_identity_network_matches_oracle(gsf, constraint):
    """T(r) = s * bf16(r / s) (the identity network): FP64 run against the
    oracle with the same network."""
    op, oop, g, gd = _lob_case(gsf, gsf.F64)
    w = cn.identity_weights()
    T = gsf.Precond(op, gd, _bf16_bits(w))
    m, k = 3, 8
    out, info = op.lobpcg_filter(gd, m, k, constraint=constraint, precond=T)
    ref = oracle.lobpcg_filter(oop, g.ravel(), m, k, constraint=constraint,
                               precond=cn.make_precond(w, g, g.shape))
    e = nrel(out.cpu().numpy(), ref[0])
    et = np.abs(np.array(list(info.theta)[:m]) - ref[1]).max()
    print(f"identity net LOBPCG (constraint={constraint}): y rel {e:.2e}, theta abs {et:.2e}, "
          f"fallbacks {info.fallbacks}")
    assert info.fallbacks == 0
    assert e <= 1e-9 and et <= 1e-10


def test_lobpcg_random_network_matches_oracle(gsf):
    """A non-linear network (the identity plus a random perturbation, so that
    r^T T(r) > 0 and T is used in every column), GPU against oracle.  T is
    computed with FP32 accumulation on the GPU, so a rare BF16 flip inside
    the network moves a column of W by ~5e-5 (see the precond parity test);
    early LOBPCG steps with nearly equal Ritz values amplify that, so the
    comparison is after one preconditioned step (y within 1e-3) and at
    convergence, where the result is unique (Ritz values within 1e-9, y
    within tol / gap)."""
    op, oop, g, gd = _lob_case(gsf, gsf.F64, H=24, W=28, seed=18)
    w = (cn.identity_weights() + 0.1 * convnet_init(18)).astype(np.float32)
    T = gsf.Precond(op, gd, _bf16_bits(w))
    Tref = cn.make_precond(w, g, g.shape)
    m = 3
    out, info = op.lobpcg_filter(gd, m, 1, constraint=True, precond=T)
    ref = oracle.lobpcg_filter(oop, g.ravel(), m, 1, constraint=True, precond=Tref)
    e1 = nrel(out.cpu().numpy(), ref[0])
    assert info.fallbacks == 0
    assert e1 <= 1e-3
    tol = 1e-9
    out, info = op.lobpcg_filter(gd, m, 3000, tol=tol, constraint=True, precond=T)
    ref = oracle.lobpcg_filter(oop, g.ravel(), m, 3000, tol=tol, constraint=True, precond=Tref)
    lam = np.linalg.eigvalsh(dense_normalized(oop)[1])
    e = nrel(out.cpu().numpy(), ref[0])
    et = np.abs(np.array(list(info.theta)[:m]) - ref[1]).max()
    print(f"random net LOBPCG: one step y rel {e1:.2e}; converged in {info.iters} vs {ref[3].iters} steps: "
          f"y rel {e:.2e}, theta abs {et:.2e}, fallbacks {info.fallbacks}")
    assert info.status == gsf.OK and ref[3].status == "ok"
    gap = lam[m + 1] - lam[m]
    assert et <= 1e-9 and np.abs(ref[1] - lam[1:m + 1]).max() <= 1e-9
    assert e <= max(1e-6, 100 * tol / gap)


def _shifted_T(oop, alpha, inner):
    """The oracle's shifted-solve T: `inner` plain CG steps on
    (L_sym + alpha I) y = r from y = 0, column by column."""
    def T(R):
        return np.column_stack([oracle.shifted_cg(oop, alpha, R[:, j], inner, 0.0)[0] for j in range(R.shape[1])])
    return T


@pytest.mark.parametrize("prec_name", ["f32", "f64"])
def test_shifted_precond_apply_matches_oracle(gsf, prec_name):
    """The shifted-solve reference T on a block with uneven column scales and
    one zero column (whose solve stops at once: y = 0).  FP64 to 1e-11
    relative; FP32 to 1e-5 (twelve CG steps on a system with condition
    number <= (2 + alpha) / alpha, data rounded to FP32)."""
    import torch
    prec = gsf.F32 if prec_name == "f32" else gsf.F64
    dt = torch.float32 if prec == gsf.F32 else torch.float64
    H, W, m, alpha, inner = 37, 45, 4, 1e-2, 12
    g = scene_2d(H, W, 0.05, 31)[1]
    R = np.random.default_rng(32).standard_normal((H * W, m)) * np.array([1.0, 1e-3, 40.0, 0.0])
    if prec == gsf.F32:
        R = R.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    op = gsf.Operator("bf", (H, W), _dev(g.ravel(), dt), 3, 2.0, 0.1, prec=prec)
    oop = oracle.build_operator("bf", g, 3, 2.0, 0.1)
    T = gsf.Precond.shifted(op, alpha, inner)
    out = T.apply(_dev(R, dt)).cpu().numpy()
    ref = _shifted_T(oop, alpha, inner)(R)
    assert np.all(out[:, 3] == 0.0)
    for j in range(3):
        e = nrel(out[:, j], ref[:, j])
        print(f"shifted T {prec_name} col {j}: rel {e:.2e}")
        assert e <= (1e-11 if prec == gsf.F64 else 1e-5)


@pytest.mark.parametrize("constraint", [False, True])
def test_lobpcg_shifted_precond_matches_oracle(gsf, constraint):
    """Flexible LOBPCG with the shifted-solve T, FP64 against the oracle
    with the same T (gate max(1e-12, 10 band), the band of the oracle run on
    the reversed grid), Ritz values and the per-column fallback count."""
    from sensitivity import reference
    op, oop, g, gd = _lob_case(gsf, gsf.F64)
    alpha, inner, m, k = 1e-2, 10, 3, 8
    T = gsf.Precond.shifted(op, alpha, inner)
    out, info = op.lobpcg_filter(gd, m, k, constraint=constraint, precond=T)

    def run(gg):
        o = oracle.build_operator("bf", gg, 2, 2.0, 0.1)
        y, th, _, rinfo = oracle.lobpcg_filter(o, gg.ravel(), m, k, constraint=constraint,
                                               precond=_shifted_T(o, alpha, inner))
        return y, (th, rinfo)
    ref = reference(run, g)
    th, rinfo = ref.extra
    e = nrel(out.cpu().numpy(), ref.y)
    print(f"shifted-T LOBPCG (constraint={constraint}): y rel {e:.2e} (gate {ref.gate:.1e}), "
          f"fallbacks {info.fallbacks}, dropped {info.dropped}/{rinfo.dropped}")
    assert info.fallbacks == 0 and info.iters == k
    assert e <= ref.gate
    np.testing.assert_allclose(np.array(list(info.theta)[:m]), th, rtol=max(1e-10, ref.gate), atol=1e-13)


def test_shifted_precond_bound_cuts_lobpcg_steps(gsf):
    """What the learned T is trained to imitate pays: with the shifted solve
    (alpha = 1e-2, 30 inner CG steps) LOBPCG reaches tol 1e-6 in at most a
    third of the plain method's steps on a 96 x 96 scene (BF 11 x 11, m = 4,
    the constraint).  The oracle's exact-solve study of the same setting
    (tests/test_oracle_solvers.py) gives the unrounded bound."""
    import torch
    side = 96
    g = scene_2d(side, side, 0.05, 5900)[1]
    gd = torch.tensor(g.ravel(), dtype=torch.float64, device="cuda")
    op = gsf.Operator("bf", (side, side), gd, 5, 2.0, 0.1, prec=gsf.F64)
    T = gsf.Precond.shifted(op, 1e-2, 30)
    ip = op.lobpcg_filter(gd, 4, 5000, tol=1e-6, constraint=True)[1]
    it = op.lobpcg_filter(gd, 4, 5000, tol=1e-6, constraint=True, precond=T)[1]
    print(f"96^2 LOBPCG steps to 1e-6: plain {ip.iters}, shifted-solve T {it.iters} (fallbacks {it.fallbacks})")
    assert ip.status == gsf.OK and it.status == gsf.OK
    assert 3 * it.iters <= ip.iters


def test_training_reduces_loss(gsf):
    """A few Adam steps on pairs generated by the method itself (residuals of
    LOBPCG, targets from the shifted CG) lower the loss."""
    from paper_1509_02468_amd import learned
    imgs = [scene_2d(48, 48, 0.05, 500 + i)[1] for i in range(4)]
    inputs, targets, cgi = learned.generate_pairs(imgs, 5, 2.0, 0.1, m=4, snapshots=(0, 5, 10, 15))
    assert inputs.shape == (16, 48 * 48, 2) and max(cgi) < 5000
    trainer, losses = learned.train(inputs, targets, 48, 48, convnet_init(19), epochs=12, batch=4, lr=3e-3)
    print("losses", losses)
    assert losses[-1] < 0.7 * losses[0]


@pytest.fixture(scope="module")
def trained(gsf):
    """A network trained on 12 scenes of 96 x 96 (residuals of LOBPCG steps
    0, 10, 20, 40, 80 and 160, targets (L_sym + 1e-2 I)^-1 r), with the
    losses of the zero and the identity networks on the same pairs."""
    from paper_1509_02468_amd import learned
    side = 96
    imgs = [scene_2d(side, side, 0.05, 600 + i)[1] for i in range(12)]
    inputs, targets, _ = learned.generate_pairs(imgs, 5, 2.0, 0.1, m=4, snapshots=(0, 10, 20, 40, 80, 160))
    trainer, losses = learned.train(inputs, targets, side, side, convnet_init(21), epochs=30, batch=8, lr=3e-3)
    zero = learned.dataset_loss(np.zeros(gsf.NET_WEIGHTS, dtype=np.float32), inputs, targets, side, side, batch=8)
    ident = learned.dataset_loss(learned.identity_weights(), inputs, targets, side, side, batch=8)
    final = learned.dataset_loss(trainer.w.cpu().numpy(), inputs, targets, side, side, batch=8)
    print(f"training loss {losses[0]:.2f} -> {losses[-1]:.2f}; on all pairs: trained {final:.2f}, "
          f"zero net {zero:.2f}, identity net {ident:.2f}")
    return dict(side=side, trainer=trainer, losses=losses, zero=zero, ident=ident, final=final)


def test_trained_network_gain_over_identity(gsf, trained):
    """What the trained network gains over T = I: on the training pairs its
    loss is below those of the zero and the identity networks, and on
    residuals of an unseen scene T(r) is closer in angle to the target
    (L_sym + alpha I)^-1 r than r itself (cosine averaged over the residual
    columns of several LOBPCG steps)."""
    import torch
    side, trainer = trained["side"], trained["trainer"]
    assert trained["final"] < min(trained["zero"], trained["ident"])
    g = scene_2d(side, side, 0.05, 699)[1]
    gd = torch.tensor(g.ravel(), dtype=torch.float64, device="cuda")
    op = gsf.Operator("bf", (side, side), gd, 5, 2.0, 0.1, prec=gsf.F64)
    T = gsf.Precond(op, gd, trainer.wb)
    X = torch.empty((side * side, 4), dtype=torch.float64, device="cuda")
    c_id, c_net = [], []
    for k in (0, 10, 30, 100):
        _, info = op.lobpcg_filter(gd, 4, k, constraint=True, ritz=X)
        R = op.lobpcg_residual(X, list(info.theta)[:4])
        TR = T.apply(R)
        for j in range(4):
            t, _ = op.shifted_cg(1e-2, R[:, j], 5000, 1e-10, ldb=4)
            r, w = R[:, j].contiguous(), TR[:, j].contiguous()
            c_id.append(float(r @ t / (r.norm() * t.norm())))
            c_net.append(float(w @ t / (w.norm() * t.norm())))
    print(f"cos to target: identity {np.mean(c_id):.3f}, network {np.mean(c_net):.3f}")
    assert np.mean(c_net) > np.mean(c_id) + 0.1


@pytest.mark.xfail(strict=True, reason="the network's 7 x 7 receptive field is smaller than one application "
                   "of the 11 x 11 operator, so it cannot imitate the non-local (L_sym + alpha I)^-1 whose "
                   "exact form does cut the steps (test_shifted_precond_bound_cuts_lobpcg_steps)")
def test_learned_precond_cuts_lobpcg_steps(gsf, trained):
    """The learned T against the plain method on an unseen 96 x 96 scene
    (tol 1e-6, m = 4, the constraint): it would pay if it cut the steps by
    more than 1.5 (its cost is about half a LOBPCG step) and the wall time
    with it."""
    import time
    import torch
    side, trainer = trained["side"], trained["trainer"]
    g = scene_2d(side, side, 0.05, 699)[1]
    gd = torch.tensor(g.ravel(), dtype=torch.float64, device="cuda")
    op = gsf.Operator("bf", (side, side), gd, 5, 2.0, 0.1, prec=gsf.F64)
    T = gsf.Precond(op, gd, trainer.wb)
    res = {}
    for name, P in (("plain", None), ("learned", T)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = op.lobpcg_filter(gd, 4, 5000, tol=1e-6, constraint=True, precond=P)[1]
        res[name] = (info.iters, time.perf_counter() - t0, info.fallbacks, info.status)
    print(f"LOBPCG to 1e-6 (steps, s, fallbacks, status): {res}")
    assert res["learned"][3] == gsf.OK
    assert 1.5 * res["learned"][0] <= res["plain"][0]
    assert res["learned"][1] < res["plain"][1]
