"""Graph operators in the three forms the filters use.

For adjacency W and degrees D (Section 2, eq. (4): L = D - W):
  random-walk form   D^-1 W x = x - D^-1 L x      (eq. (3): one BF / GF pass)
  normalized form    N z = D^-1/2 W D^-1/2 z
  normalized Laplacian  L_sym z = z - N z = D^-1/2 L D^-1/2 z

Reading of the normalization (Section 4 writes (diag L)^-1/2 L (diag L)^-1/2):
by default we normalize by D, the degree matrix that includes the self-loop.
Then D^-1 W = D^-1/2 N D^1/2 is exactly the BF of eq. (3), and D is exactly the
preconditioner of Algorithm 2; z = D^1/2 x maps between the two.

The variant norm="diagl" (BF only) normalizes by diag L instead, as printed in
Section 4: L_sym = (diag L)^-1/2 L (diag L)^-1/2, N = I - L_sym,
RW x = x - (diag L)^-1 L x, and diag L takes D's place everywhere else (the
preconditioner of Algorithm 2, z = (diag L)^1/2 x).  The self-loop cancels in
L = D - W, so diag L_i = sum_{j != i} w_ij; it is summed from the off-diagonal
weights themselves (forming d_i - 1 would cancel all digits of a small
diag L_i, and the normalization divides by it).  Reading for a vertex whose
off-diagonal weights are all zero (diag L_i = 0): row and column i of L
vanish, so any positive scale leaves L_sym's entries unchanged; we take 1 (the
vertex is a fixed point of every filter and z_i = x_i).
The attribute d holds the normalizing diagonal; L = diag(dl) - A with
(dl, A) = (D, W) for norm "d" and (diag L, W - I) for "diagl".
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .graph import bf_weight_matrix, degrees
from .guided import guided_filter, gf_degrees, gf_stats

FORM_N, FORM_LSYM, FORM_RW, FORM_L = 0, 1, 2, 3


@dataclass
class GraphOperator:
    kind: str                 # "bf" or "gf"
    shape: tuple
    guidance: np.ndarray      # float64, grid shape
    radius: int
    sigma_s: float = 0.0
    sigma_r: float = 0.0
    eps: float = 0.0
    W: object = None          # scipy.sparse (BF) or None (GF: implicit)
    d: np.ndarray = None      # flat normalizing diagonal (D, or diag L with 0 -> 1)
    sqrt_d: np.ndarray = None
    stencil: str = "square"
    norm: str = "d"
    dl: np.ndarray = None     # flat diagonal of L's degree part: D (norm "d") or diag L
    W_off: object = None      # norm "diagl": W without its diagonal (the self-loops)

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    # -- adjacency ------------------------------------------------------
    def apply_w(self, x):
        """W x for a flat vector (or n x m block)."""
        x = np.asarray(x, dtype=np.float64)
        if self.kind == "bf":
            return self.W @ x
        # GF: W = D (D^-1 W) and D^-1 W x is Algorithm 1 with fixed guidance.
        if x.ndim == 2:
            return np.stack([self.apply_w(x[:, j]) for j in range(x.shape[1])], axis=1)
        gx = guided_filter(x.reshape(self.shape), self.guidance, self.radius, self.eps).ravel()
        return self.d * gx

    def _scale(self, v, s):
        return v * (s[:, None] if np.ndim(v) == 2 else s)

    # -- the three forms --------------------------------------------------
    def apply_rw(self, x):
        """D^-1 W x (eq. (3)); norm "diagl": x - (diag L)^-1 L x."""
        if self.norm == "diagl":
            return np.asarray(x, dtype=np.float64) - self._scale(self.apply_l(x), 1.0 / self.d)
        return self._scale(self.apply_w(x), 1.0 / self.d)

    def apply_n(self, z):
        """N z = D^-1/2 W D^-1/2 z; norm "diagl": z - L_sym z."""
        if self.norm == "diagl":
            return np.asarray(z, dtype=np.float64) - self.apply_lsym(z)
        inv = 1.0 / self.sqrt_d
        return self._scale(self.apply_w(self._scale(z, inv)), inv)

    def apply_lsym(self, z):
        """L_sym z = z - N z; norm "diagl": (diag L)^-1/2 L (diag L)^-1/2 z (Section 4)."""
        if self.norm == "diagl":
            inv = 1.0 / self.sqrt_d
            return self._scale(self.apply_l(self._scale(z, inv)), inv)
        return np.asarray(z, dtype=np.float64) - self.apply_n(z)

    def apply_l(self, x):
        """L x = D x - W x (eq. (4)); norm "diagl": diag L x - (W - I) x."""
        x = np.asarray(x, dtype=np.float64)
        if self.norm == "diagl":
            return self._scale(x, self.dl) - self.W_off @ x
        return self._scale(x, self.dl) - self.apply_w(x)

    def apply(self, form: int, v):
        return {FORM_N: self.apply_n, FORM_LSYM: self.apply_lsym, FORM_RW: self.apply_rw, FORM_L: self.apply_l}[form](v)

    # -- normalized planes (for parity with a stored-operator build) --------
    def gf_window_stats(self):
        """(mu_k, 1/(sigma_k^2 + eps)) of the fixed guidance (GF only)."""
        return gf_stats(self.guidance, self.radius, self.eps)


def build_operator(kind: str, guidance, radius: int, sigma_s: float = 0.0,
                   sigma_r: float = 0.0, eps: float = 0.0, stencil: str = "square",
                   norm: str = "d", channels: int = 1) -> GraphOperator:
    """Build the graph operator of the BF (eq. (2)) or the GF (eqs. (5)-(6))
    from a fixed guidance signal (the linear filters of Sections 2-3).
    stencil ("square", or "cross" for the 5-point-type lattice of Section 7)
    and norm ("d", or "diagl" for (diag L)^-1/2 L (diag L)^-1/2 of Section 4)
    are BF options, as is channels > 1 (a guidance with a trailing axis of
    that many channels, e.g. CIE-Lab, see `bf_weight_matrix`)."""
    g = np.asarray(guidance, dtype=np.float64)
    if norm not in ("d", "diagl"):
        raise ValueError(norm)
    W_off = None
    if kind == "bf":
        W = bf_weight_matrix(g, radius, sigma_s, sigma_r, stencil, channels)
        d = degrees(W)
        if norm == "diagl":
            W_off = (W - sp.diags(W.diagonal())).tocsr()  # exact: every w_ii is 1
            W_off.eliminate_zeros()
            dl = degrees(W_off)
            d = np.where(dl > 0.0, dl, 1.0)
        else:
            dl = d
    elif kind == "gf":
        if stencil != "square" or norm != "d" or channels != 1:
            raise ValueError("stencil, norm and channel options are BF-only")
        W = None
        d = dl = gf_degrees(g.shape, radius).ravel()
    else:
        raise ValueError(kind)
    shape = g.shape[:-1] if channels > 1 else g.shape
    return GraphOperator(kind=kind, shape=shape, guidance=g, radius=radius,
                         sigma_s=sigma_s, sigma_r=sigma_r, eps=eps, W=W, d=d,
                         sqrt_d=np.sqrt(d), stencil=stencil, norm=norm, dl=dl, W_off=W_off)
