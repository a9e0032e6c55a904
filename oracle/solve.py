"""Dense separable solve (oracle).

The FEM system of eq. (bvp glob 2) has the unique solution (L is SPD)

    v = (x)_i V_i  diag(1 / (sum_i 4 h_i^-2 lambda_{i,k_i}^{(l_i)} + alpha))  (x)_i V_i^T  f^h,

where V_i has C_i-orthonormal columns with V_i^T A_i V_i = diag(lambda_i)
(eq. (decomp v 2); step (1) of algorithm (a) cancels because V^-1 = V^T C).
The oracle applies V_i^T and V_i along every axis as plain dense products,
in FP64.
"""
import numpy as np

from .spectral import basis


def _along(M, F, axis):
    """Apply matrix M along ``axis`` of F: out[..q..] = sum_r M[q, r] F[..r..]."""
    return np.moveaxis(np.tensordot(M, F, axes=([1], [axis])), 0, axis)


def denominators(lams, Xs, Ks, alpha):
    """Outer sum alpha + sum_i 4 h_i^-2 lam_i over the N-D coefficient grid."""
    den = np.array(alpha, dtype=np.float64)
    for i, lam in enumerate(lams):
        s = 4.0 * Ks[i] ** 2 / Xs[i] ** 2
        shape = [1] * len(lams)
        shape[i] = lam.size
        den = den + s * lam.reshape(shape)
    return den


def solve(fh, ns, Ks, Xs, alpha=0.0, route="structured"):
    """Solve eq. (bvp glob 2) for one right-hand side f^h of shape (m_0..m_{N-1})."""
    fh = np.asarray(fh, dtype=np.float64)
    N = fh.ndim
    bases = [basis(ns[i], Ks[i], route) for i in range(N)]
    den = denominators([b[1] for b in bases], Xs, Ks, alpha)
    if np.any(den <= 0):
        raise ValueError("operator is not positive definite for this alpha")
    G = fh
    for i in range(N):
        G = _along(bases[i][0].T, G, i)
    G = G / den
    for i in range(N):
        G = _along(bases[i][0], G, i)
    return G
