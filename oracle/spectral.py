"""Dense spectral tools for small graphs (Section 4): the factorization
L = U Lambda U^T of eq. (8) applied to the normalized Laplacian, the graph
Fourier transform x_hat = U^T x, and ideal low-pass filters.  O(n^3): n of a
few hundred at most."""
from __future__ import annotations

import numpy as np


def dense_normalized(op):
    """Dense N = D^-1/2 W D^-1/2 and L_sym = I - N of a small operator."""
    n = op.n
    eye = np.eye(n)
    N = op.apply_n(eye)
    return N, eye - N


def eig_lsym(op):
    """Ascending eigenvalues and orthonormal eigenvectors of L_sym, eq. (8)."""
    _, Ls = dense_normalized(op)
    Ls = 0.5 * (Ls + Ls.T)
    return np.linalg.eigh(Ls)


def gft_lowpass(U, z, m: int):
    """Keep the m lowest graph frequencies of z: U_m U_m^T z."""
    Um = U[:, :m]
    return Um @ (Um.T @ z)
