"""Training driver of the learned preconditioner (the preconditioner slot of
Algorithm 3): training pairs from the method itself, Adam on the GPU.

Pairs: for each training image, block LOBPCG (m columns, with the constraint)
is run for k steps for each k of a snapshot list (SNAPSHOTS: 0, 5, ..., 45;
TRAJECTORY: 0, 5, 10, 20, ..., 1280, residuals from the whole run to a
tolerance); the residual block R = L_sym X - X Theta of the returned Ritz
pairs gives one column r (column s mod m for the s-th snapshot), and its
target t = (L_sym + alpha I)^-1 r comes from CG to a relative residual of
cg_tol.  Both are scaled by s = RMS(r) (the network sees r / s and learns
t / s).  All arithmetic runs in libgsf (this module only sequences the
calls and keeps the device buffers).
"""
from __future__ import annotations

import numpy as np

from . import gsf

SNAPSHOTS = tuple(range(0, 50, 5))
# residuals from the whole run to the tolerance, not only its first steps
TRAJECTORY = (0, 5, 10, 20, 40, 80, 160, 320, 640, 1280)


def identity_weights():
    """Weights of the network with net(r, g) = r exactly (u = relu(u) -
    relu(-u) through the two hidden layers): the T = I baseline."""
    w = np.zeros(gsf.NET_WEIGHTS, dtype=np.float32)
    w1, w2, w3 = 0, 16 * 2 * 9, 16 * 2 * 9 + 16 * 16 * 9
    centre = 4  # (ky, kx) = (1, 1)
    w[w1 + (0 * 2 + 0) * 9 + centre] = 1.0    # channel 0 <- +r
    w[w1 + (1 * 2 + 0) * 9 + centre] = -1.0   # channel 1 <- -r
    w[w2 + (0 * 16 + 0) * 9 + centre] = 1.0
    w[w2 + (1 * 16 + 1) * 9 + centre] = 1.0
    w[w3 + 0 * 9 + centre] = 1.0
    w[w3 + 1 * 9 + centre] = -1.0
    return w


def dataset_loss(w, inputs, targets, rows, cols, batch=16):
    """Mean loss of the weights w (FP32, rounded to BF16 as in training)
    over the whole training set, in batches of `batch` samples: the zero
    network gives mean(t^2), the identity network mean((r - t)^2)."""
    import torch
    P = inputs.shape[0]
    trainer = gsf.NetTrainer(w, batch, rows, cols)
    total, count = 0.0, 0
    for b0 in range(0, P - batch + 1, batch):
        idx = torch.arange(b0, b0 + batch, dtype=torch.int32, device="cuda")
        loss, _ = trainer.loss_grad(idx, inputs, targets)
        total += float(loss[0]) * batch
        count += batch
    return total / max(count, 1)


def generate_pairs(images, radius, sigma_d, sigma_r, m=4, snapshots=SNAPSHOTS, alpha=1e-2, cg_tol=1e-10,
                   cg_kmax=20000, prec=gsf.F64):
    """images: list of noisy 2D arrays of one shape (the guidance of their own
    BF operator).  Returns device tensors inputs [P, H*W, 2], targets
    [P, H*W] (float32) and per-pair CG iteration counts."""
    import torch
    shape = tuple(images[0].shape)
    n = int(np.prod(shape))
    P = len(images) * len(snapshots)
    inputs = torch.empty((P, n, 2), dtype=torch.float32, device="cuda")
    targets = torch.empty((P, n), dtype=torch.float32, device="cuda")
    cg_iters = []
    p = 0
    for img in images:
        g = torch.as_tensor(np.ascontiguousarray(img, dtype=np.float64)).to("cuda", gsf._dtype(prec)).reshape(-1)
        op = gsf.Operator("bf", shape, g, radius, sigma_d, sigma_r, prec=prec)
        lws = op.workspace(gsf.METHOD_LOBPCG, m)
        cws = op.workspace(gsf.METHOD_CG)
        X = torch.empty((n, m), dtype=op.dtype, device="cuda")
        out = torch.empty_like(g)
        y = torch.empty_like(g)
        for s_idx, k in enumerate(snapshots):
            _, info = op.lobpcg_filter(g, m, k, constraint=True, out=out, ritz=X, ws=lws)
            R = op.lobpcg_residual(X, list(info.theta)[:m])
            j = s_idx % m
            col = R[:, j]
            _, cinfo = op.shifted_cg(alpha, col, cg_kmax, cg_tol, ldb=m, out=y, ws=cws)
            cg_iters.append(cinfo.iters)
            keep = op.make_pair(col, y, g, inputs[p], targets[p], ldr=m)
            torch.cuda.synchronize()
            del keep
            p += 1
    return inputs, targets, cg_iters


def train(inputs, targets, rows, cols, w_init, epochs=20, batch=16, lr=1e-3, seed=0, log=None):
    """Adam on mini-batches of a seeded permutation per epoch.  Returns the
    trainer (FP32 master weights .w, BF16 copy .wb) and the mean loss per
    epoch."""
    import torch
    P = inputs.shape[0]
    trainer = gsf.NetTrainer(w_init, batch, rows, cols)
    rng = np.random.default_rng(seed)
    nb = P // batch
    losses = torch.zeros((epochs, nb), dtype=torch.float64, device="cuda")
    for e in range(epochs):
        perm = torch.as_tensor(rng.permutation(P)[:nb * batch].astype(np.int32)).to("cuda")
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            loss, _ = trainer.loss_grad(idx, inputs, targets)
            losses[e, b].copy_(loss[0])
            trainer.adam(lr)
        if log is not None:
            log(e, float(losses[e].mean()))
    return trainer, losses.mean(dim=1).cpu().numpy()
