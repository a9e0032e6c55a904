"""Global 1D pencil and N-D FEM operator (oracle).

Indexing of S_K^(n) (Section 2, paragraph 1): a vector holds the values at
the interior mesh nodes x_j (j = 1..K-1) and at the n-1 interior points
x_{j-1} + (l/n) h of every element j = 1..K.  The oracle stores it in
physical order, i.e. by the position g = 1..nK-1 of the point g*h/n, at array
index q = g - 1.  Node j sits at q = n*j - 1; interior point l of element j
sits at q = n*(j-1) + l - 1.

The scaled pencil of eq. (eig_glob) is assembled from the reference-element
matrices without any h factor (the physical eigenvalue is 4 h^-2 lambda).
The N-D operator is that of eq. (bvp glob 2):

    L = sum_i 4 h_i^-2  A_i (x) prod_{j != i} C_j  +  alpha prod_j C_j,

with axis 0 outermost (C order).  ``apply_operator`` is a matrix-free FP64
apply in which every stiffness factor is evaluated in difference form,
(A v)_k = sum_{l != k} A_kl (v_l - v_k) per element, so that the constants
along that axis are exactly in its kernel, as they are for the exact matrix
(the local stiffness has zero row sums).
"""
from fractions import Fraction

import numpy as np
import scipy.sparse as sp

from .element import local_matrices


def dim(n, K):
    """Number of unknowns per axis, nK - 1."""
    return n * K - 1


def node_index(n, j):
    return n * j - 1


def bubble_index(n, j, l):
    return n * (j - 1) + l - 1


def local_float(n):
    """Local A, C rounded once to FP64 (numpy arrays)."""
    A, C = local_matrices(n)
    return (np.array([[float(x) for x in r] for r in A]),
            np.array([[float(x) for x in r] for r in C]))


def assemble_1d_exact(n, K):
    """Exact global (scaled) stiffness and mass as lists of Fractions (tiny K only)."""
    A, C = local_matrices(n)
    m = dim(n, K)
    Ag = [[Fraction(0)] * m for _ in range(m)]
    Cg = [[Fraction(0)] * m for _ in range(m)]
    for j in range(1, K + 1):
        for r in range(n + 1):
            qr = n * (j - 1) + r - 1
            if not 0 <= qr < m:
                continue
            for s in range(n + 1):
                qs = n * (j - 1) + s - 1
                if not 0 <= qs < m:
                    continue
                Ag[qr][qs] += A[r][s]
                Cg[qr][qs] += C[r][s]
    return Ag, Cg


def assemble_1d(n, K):
    """Global (scaled) stiffness and mass, dense FP64; every entry is the
    exact assembled rational rounded once."""
    As, Cs = assemble_1d_sparse(n, K)
    return As.toarray(), Cs.toarray()


def assemble_1d_sparse(n, K):
    """Same matrices as ``assemble_1d`` in CSR form."""
    A, C = local_matrices(n)
    m = dim(n, K)
    ea, ec = {}, {}
    for j in range(1, K + 1):
        for r in range(n + 1):
            qr = n * (j - 1) + r - 1
            if not 0 <= qr < m:
                continue
            for s in range(n + 1):
                qs = n * (j - 1) + s - 1
                if not 0 <= qs < m:
                    continue
                ea[(qr, qs)] = ea.get((qr, qs), Fraction(0)) + A[r][s]
                ec[(qr, qs)] = ec.get((qr, qs), Fraction(0)) + C[r][s]
    keys = sorted(ea)
    rows = np.array([k[0] for k in keys])
    cols = np.array([k[1] for k in keys])
    Av = np.array([float(ea[k]) for k in keys])
    Cv = np.array([float(ec[k]) for k in keys])
    return (sp.csr_matrix((Av, (rows, cols)), shape=(m, m)),
            sp.csr_matrix((Cv, (rows, cols)), shape=(m, m)))


def operator_sparse(ns, Ks, Xs, alpha):
    """Sparse FP64 matrix of eq. (bvp glob 2) (C order, axis 0 outermost)."""
    N = len(ns)
    mats = [assemble_1d_sparse(ns[i], Ks[i]) for i in range(N)]
    total = None
    for i in range(N):
        h = Xs[i] / Ks[i]
        term = None
        for j in range(N):
            M = mats[j][0] if j == i else mats[j][1]
            term = M if term is None else sp.kron(term, M, format="csr")
        term = term * (4.0 / h ** 2)
        total = term if total is None else total + term
    if alpha != 0.0:
        term = None
        for j in range(N):
            term = mats[j][1] if term is None else sp.kron(term, mats[j][1], format="csr")
        total = total + alpha * term
    return total.tocsr()


def _apply_local_1d(u, axis, M, n, K, difference):
    """Apply the assembled 1D operator with local matrix M along ``axis``.

    Element j (1..K) covers padded positions n(j-1)..nj; the two ends of the
    padded axis are the Dirichlet zeros.  With ``difference`` the product is
    evaluated as sum_{l != k} M_kl (v_l - v_k), valid for zero-row-sum M.
    """
    v = np.moveaxis(u, axis, 0)
    shape = v.shape
    pad = np.zeros((n * K + 1,) + shape[1:])
    pad[1:-1] = v
    out = np.zeros_like(pad)
    for k in range(n + 1):
        vk = pad[k:k + n * K:n]
        acc = np.zeros_like(vk)
        for l in range(n + 1):
            if difference:
                if l == k:
                    continue
                acc += M[k, l] * (pad[l:l + n * K:n] - vk)
            else:
                acc += M[k, l] * pad[l:l + n * K:n]
        out[k:k + n * K:n] += acc
    return np.moveaxis(out[1:-1], 0, axis)


def apply_mass_1d(u, axis, n, K):
    _, C = local_float(n)
    return _apply_local_1d(u, axis, C, n, K, difference=False)


def apply_stiffness_1d(u, axis, n, K):
    A, _ = local_float(n)
    return _apply_local_1d(u, axis, A, n, K, difference=True)


def apply_operator(u, ns, Ks, Xs, alpha):
    """L u for the operator of eq. (bvp glob 2), FP64, matrix-free.

    For each stiffness term the mass factors along the other axes are applied
    first and the stiffness (difference form) last.
    """
    N = u.ndim
    out = np.zeros_like(u)
    for i in range(N):
        w = u
        for j in range(N):
            if j != i:
                w = apply_mass_1d(w, j, ns[j], Ks[j])
        w = apply_stiffness_1d(w, i, ns[i], Ks[i])
        out += (4.0 * Ks[i] ** 2 / Xs[i] ** 2) * w
    if alpha != 0.0:
        w = u
        for j in range(N):
            w = apply_mass_1d(w, j, ns[j], Ks[j])
        out += alpha * w
    return out


def apply_mass(u, ns, Ks):
    """prod_j C_j u (mass along every axis), FP64."""
    w = u
    for j in range(u.ndim):
        w = apply_mass_1d(w, j, ns[j], Ks[j])
    return w
