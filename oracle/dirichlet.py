"""Non-homogeneous Dirichlet data (oracle; test infrastructure only, never
called by the library's product path).

Section 2, paragraph 4 reduces the general case u = b on the boundary to
zero data through a modified right-hand side.  With g_b the FEM function that
takes the values b at the boundary grid points and 0 inside, the interior
values u_0 of the solution solve

    L u_0 = f^h - (L_ext g_b) restricted to the interior points,

where L_ext is the scaled operator of eq. (bvp glob 2) assembled over all
grid points including the boundary.  Written out as stated: the 1D scaled
stiffness and mass over the nK + 1 points of an axis, assembled from the
exact local matrices (rounded once), applied along every axis.
"""
import numpy as np

from .element import local_matrices


def assemble_1d_extended(n, K):
    """Scaled stiffness and mass over all nK + 1 grid points of an axis (dense FP64)."""
    A, C = local_matrices(n)
    size = n * K + 1
    Ae = np.zeros((size, size))
    Ce = np.zeros((size, size))
    Al = np.array([[float(x) for x in r] for r in A])
    Cl = np.array([[float(x) for x in r] for r in C])
    for j in range(K):
        sl = slice(n * j, n * j + n + 1)
        Ae[sl, sl] += Al
        Ce[sl, sl] += Cl
    return Ae, Ce


def _along(M, F, axis):
    return np.moveaxis(np.tensordot(M, F, axes=([1], [axis])), 0, axis)


def lift_rhs(b_ext, f, ns, Ks, Xs, alpha):
    """f^h - (L_ext g_b)|interior for boundary values on the extended grid b_ext
    (shape (m_0 + 2, ..., m_{N-1} + 2); its interior entries are ignored)."""
    N = len(ns)
    g = np.array(b_ext, dtype=np.float64)
    g[tuple(slice(1, -1) for _ in range(N))] = 0.0
    mats = [assemble_1d_extended(ns[i], Ks[i]) for i in range(N)]
    out = np.zeros_like(g)
    for i in range(N):
        t = g
        for j in range(N):
            t = _along(mats[j][0] if j == i else mats[j][1], t, j)
        out += 4.0 * (Ks[i] / Xs[i]) ** 2 * t
    if alpha != 0.0:
        t = g
        for j in range(N):
            t = _along(mats[j][1], t, j)
        out += alpha * t
    inner = out[tuple(slice(1, -1) for _ in range(N))]
    return (0.0 if f is None else f) - inner
