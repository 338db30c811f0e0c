"""FP64 reference of the learned preconditioner T (the extension of the
preconditioner slot of Algorithm 3; the paper uses T = D^-1 and names better
preconditioners as future work in its conclusion).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network (our reading, the paper is silent):
  input  x = (r / s, g): the residual column scaled by s = RMS(r) and the
         guidance image, both on the image grid;
  layer 1  z1 = conv3x3(x; W1), 2 -> 16 channels, a1 = relu(z1);
  layer 2  z2 = conv3x3(a1; W2), 16 -> 16 channels, a2 = relu(z2);
  layer 3  y = conv3x3(a2; W3), 16 -> 1 channel;
  T(r) = s * y.
  conv3x3 is a cross-correlation with zero padding at the image border:
  z[o, i, j] = sum_c sum_{dy, dx in -1..1} W[o, c, dy+1, dx+1] a[c, i+dy, j+dx].
  No biases (T is then positively homogeneous: T(c r) = c T(r) for c > 0,
  which the RMS scaling makes exact).
Flat weight layout (2736 values): W1[o][c][ky][kx] (16x2x3x3), then
W2[o][c][ky][kx] (16x16x3x3), then W3[c][ky][kx] (16x3x3).

Precision (rounding points shared with the GPU kernels): the weights, the
input x and the activations a1, a2 are rounded to bfloat16 (round to nearest,
ties to even); everything else is exact here (FP64) and FP32 on the GPU.
`bf16=False` turns the rounding off (used by the finite-difference pins).

Training target: y* = (L_sym + alpha I)^-1 r with alpha = 1e-2 (the shifted
solve `shifted_cg`), loss = mean over samples and pixels of (y - y*/s)^2.
Gradients flow through the rounded weights unchanged (the master copy is the
FP32 weight vector that Adam updates).  ReLU derivative: 1 where the stored
activation is > 0.  relu(NaN) = NaN, so a NaN inside the network reaches the
output (and triggers the T = I fallback of the solver).

Adam (Kingma and Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

C_IN, C_HID = 2, 16
N_W1 = C_HID * C_IN * 9
N_W2 = C_HID * C_HID * 9
N_W3 = C_HID * 9
N_WEIGHTS = N_W1 + N_W2 + N_W3


def bf16_round(x):
    """Round to the nearest bfloat16 value (8 significant bits), ties to even.
    Values stay float64 (exactly representable in bfloat16).  Non-finite
    values pass through."""
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()
    fin = np.isfinite(x) & (x != 0.0)
    mant, expo = np.frexp(x[fin])  # x = mant * 2^expo, 0.5 <= |mant| < 1
    out[fin] = np.ldexp(np.rint(mant * 256.0) / 256.0, expo)
    return out


def split_weights(w):
    w = np.asarray(w, dtype=np.float64).ravel()
    assert w.size == N_WEIGHTS
    W1 = w[:N_W1].reshape(C_HID, C_IN, 3, 3)
    W2 = w[N_W1:N_W1 + N_W2].reshape(C_HID, C_HID, 3, 3)
    W3 = w[N_W1 + N_W2:].reshape(1, C_HID, 3, 3)
    return W1, W2, W3


def shift(a, dy: int, dx: int):
    """b[..., i, j] = a[..., i + dy, j + dx], zero outside the image."""
    b = np.zeros_like(a)
    H, W = a.shape[-2:]
    ys, yd = (slice(dy, H), slice(0, H - dy)) if dy >= 0 else (slice(0, H + dy), slice(-dy, H))
    xs, xd = (slice(dx, W), slice(0, W - dx)) if dx >= 0 else (slice(0, W + dx), slice(-dx, W))
    b[..., yd, xd] = a[..., ys, xs]
    return b


def conv3x3(a, Wt):
    """a: (C, H, W); Wt: (O, C, 3, 3) -> (O, H, W), zero-padded correlation."""
    O = Wt.shape[0]
    out = np.zeros((O,) + a.shape[1:])
    for ky in range(3):
        for kx in range(3):
            s = shift(a, ky - 1, kx - 1)
            out += np.tensordot(Wt[:, :, ky, kx], s, axes=(1, 0))
    return out


def conv3x3_adjoint(d, Wt):
    """Adjoint of conv3x3 in its input: d (O, H, W) -> (C, H, W)."""
    C = Wt.shape[1]
    out = np.zeros((C,) + d.shape[1:])
    for ky in range(3):
        for kx in range(3):
            s = shift(d, 1 - ky, 1 - kx)
            out += np.tensordot(Wt[:, :, ky, kx], s, axes=(0, 0))
    return out


def conv3x3_weight_grad(d, a):
    """d (O, H, W) output gradient, a (C, H, W) layer input -> dW (O, C, 3, 3)."""
    g = np.zeros((d.shape[0], a.shape[0], 3, 3))
    for ky in range(3):
        for kx in range(3):
            s = shift(a, ky - 1, kx - 1)
            g[:, :, ky, kx] = np.tensordot(d, s, axes=([1, 2], [1, 2]))
    return g


def forward(w, r_scaled, g, bf16: bool = True):
    """One sample: r_scaled, g (H, W) -> dict with x, a1, a2 and output y."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1, W2, W3 = (rnd(t) for t in split_weights(w))
    x = rnd(np.stack([np.asarray(r_scaled, np.float64), np.asarray(g, np.float64)]))
    a1 = rnd(np.maximum(conv3x3(x, W1), 0.0))
    a2 = rnd(np.maximum(conv3x3(a1, W2), 0.0))
    y = conv3x3(a2, W3)[0]
    return {"x": x, "a1": a1, "a2": a2, "y": y, "W": (W1, W2, W3)}


def loss_and_grad(w, inputs, targets, guidance, bf16: bool = True):
    """Mean squared error over all samples and pixels and its gradient in the
    flat weight layout.  inputs, targets: (B, H, W) scaled residuals and
    scaled targets; guidance: (B, H, W)."""
    B = len(inputs)
    npix = B * np.asarray(inputs[0]).size
    loss = 0.0
    grad = np.zeros(N_WEIGHTS)
    for b in range(B):
        f = forward(w, inputs[b], guidance[b], bf16)
        W1, W2, W3 = f["W"]
        e = f["y"] - np.asarray(targets[b], np.float64)
        loss += float(np.sum(e * e))
        dy = (2.0 / npix) * e[None]
        g3 = conv3x3_weight_grad(dy, f["a2"])
        dz2 = conv3x3_adjoint(dy, W3) * (f["a2"] > 0.0)
        g2 = conv3x3_weight_grad(dz2, f["a1"])
        dz1 = conv3x3_adjoint(dz2, W2) * (f["a1"] > 0.0)
        g1 = conv3x3_weight_grad(dz1, f["x"])
        grad += np.concatenate([g1.ravel(), g2.ravel(), g3.ravel()])
    return loss / npix, grad


def adam_step(w, m, v, grad, t: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step number t >= 1); returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def rms(r):
    r = np.asarray(r, dtype=np.float64)
    return float(np.sqrt(np.mean(r * r)))


def precond_apply(w, r, g, bf16: bool = True):
    """T(r) = s * net(r / s, g) with s = RMS(r) (0 for r = 0)."""
    r = np.asarray(r, dtype=np.float64)
    s = rms(r)
    if s == 0.0:
        return np.zeros_like(r)
    return s * forward(w, r / s, g, bf16)["y"]


def make_precond(w, g, shape, bf16: bool = True):
    """Column-wise preconditioner callable for oracle.solvers.lobpcg_filter:
    R (n, m) -> T(R), each column reshaped to the image `shape`."""
    g = np.asarray(g, dtype=np.float64).reshape(shape)

    def T(R):
        out = np.empty_like(R)
        for j in range(R.shape[1]):
            out[:, j] = precond_apply(w, R[:, j].reshape(shape), g, bf16).ravel()
        return out
    return T


def identity_weights():
    """A network with net(x) = x[0] exactly: relu(u) - relu(-u) = u."""
    W1, W2, W3 = (np.zeros(s) for s in ((C_HID, C_IN, 3, 3), (C_HID, C_HID, 3, 3), (1, C_HID, 3, 3)))
    W1[0, 0, 1, 1], W1[1, 0, 1, 1] = 1.0, -1.0
    W2[0, 0, 1, 1], W2[1, 1, 1, 1] = 1.0, 1.0
    W3[0, 0, 1, 1], W3[0, 1, 1, 1] = 1.0, -1.0
    return np.concatenate([W1.ravel(), W2.ravel(), W3.ravel()])
