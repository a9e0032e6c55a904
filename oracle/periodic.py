"""Periodic and Neumann axes (oracle).  TEST INFRASTRUCTURE ONLY.

The Introduction notes that boundary conditions other than Dirichlet fit the
method.  On a periodic axis the points x = 0 and x = X are one point, so the
space holds the values at every point g h / n, g = 0..nK-1 (array index
q = g): the mesh node j at q = n j and the interior points l = 1..n-1 of
element j + 1 at q = n j + l.  Element j = 1..K couples the positions
n (j-1) .. n j, the last one taken modulo nK (element K ends at node 0).

A Neumann axis (natural boundary conditions at both ends) holds the values
at every point g h / n, g = 0..nK, boundary nodes included: element j
couples the positions n (j-1) .. n j and nothing is removed.

The oracle is the plain definition: the periodic (or Neumann) pencil assembled from the
exact local matrices of Section 2, paragraph 1 (every entry rounded once),
the N-D operator of eq. (bvp glob 2) with the periodic matrices on the
periodic axes, and a sparse direct solve of it, corrected with residuals
evaluated exactly (integer arithmetic over the rational local matrices) so
that the result is the exact system's solution rounded to FP64.  No eigen
decomposition, no FFT: it shares nothing with the Bloch-wave route of the
GPU library.
"""
import math
from fractions import Fraction

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assembly
from .element import local_matrices


def dim(n, K):
    """Number of unknowns of a periodic axis, nK."""
    return n * K


def assemble_1d_sparse(n, K):
    """Scaled periodic stiffness and mass (reference element [-1, 1], no h
    factor), CSR, every entry the exact assembled rational rounded once."""
    A, C = local_matrices(n)
    m = dim(n, K)
    ea, ec = {}, {}
    for j in range(1, K + 1):
        for r in range(n + 1):
            qr = (n * (j - 1) + r) % m
            for s in range(n + 1):
                qs = (n * (j - 1) + s) % m
                ea[(qr, qs)] = ea.get((qr, qs), Fraction(0)) + A[r][s]
                ec[(qr, qs)] = ec.get((qr, qs), Fraction(0)) + C[r][s]
    keys = sorted(ea)
    rows = np.array([k[0] for k in keys])
    cols = np.array([k[1] for k in keys])
    Av = np.array([float(ea[k]) for k in keys])
    Cv = np.array([float(ec[k]) for k in keys])
    return (sp.csr_matrix((Av, (rows, cols)), shape=(m, m)),
            sp.csr_matrix((Cv, (rows, cols)), shape=(m, m)))


def assemble_1d(n, K):
    """Dense form of ``assemble_1d_sparse``."""
    As, Cs = assemble_1d_sparse(n, K)
    return As.toarray(), Cs.toarray()


def assemble_1d_neumann_sparse(n, K):
    """Scaled Neumann stiffness and mass (all nK + 1 points), CSR, every entry
    the exact assembled rational rounded once."""
    A, C = local_matrices(n)
    m = n * K + 1
    ea, ec = {}, {}
    for j in range(1, K + 1):
        for r in range(n + 1):
            qr = n * (j - 1) + r
            for s in range(n + 1):
                qs = n * (j - 1) + s
                ea[(qr, qs)] = ea.get((qr, qs), Fraction(0)) + A[r][s]
                ec[(qr, qs)] = ec.get((qr, qs), Fraction(0)) + C[r][s]
    keys = sorted(ea)
    rows = np.array([k[0] for k in keys])
    cols = np.array([k[1] for k in keys])
    Av = np.array([float(ea[k]) for k in keys])
    Cv = np.array([float(ec[k]) for k in keys])
    return (sp.csr_matrix((Av, (rows, cols)), shape=(m, m)),
            sp.csr_matrix((Cv, (rows, cols)), shape=(m, m)))


def axis_matrices(n, K, bc):
    """(A, C) of one axis, bc "dirichlet", "periodic" or "neumann" (CSR)."""
    if bc == "periodic":
        return assemble_1d_sparse(n, K)
    if bc == "neumann":
        return assemble_1d_neumann_sparse(n, K)
    if bc == "dirichlet":
        return assembly.assemble_1d_sparse(n, K)
    raise ValueError(f"unknown boundary condition {bc!r}")


def axis_dim(n, K, bc):
    if bc == "neumann":
        return n * K + 1
    return dim(n, K) if bc == "periodic" else assembly.dim(n, K)


def operator_sparse(ns, Ks, Xs, alpha, bcs):
    """Sparse FP64 matrix of eq. (bvp glob 2) with the given boundary
    condition per axis (C order, axis 0 outermost)."""
    N = len(ns)
    mats = [axis_matrices(ns[i], Ks[i], bcs[i]) for i in range(N)]
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
    return total.tocsc()


def apply_operator(u, ns, Ks, Xs, alpha, bcs):
    """L u by products along every axis (any size; u shaped like the grid)."""
    u = np.asarray(u, dtype=np.float64)
    N = u.ndim
    mats = [axis_matrices(ns[i], Ks[i], bcs[i]) for i in range(N)]

    def along(M, F, axis):
        Fm = np.moveaxis(F, axis, 0)
        out = (M @ Fm.reshape(Fm.shape[0], -1)).reshape(Fm.shape)
        return np.moveaxis(out, 0, axis)

    total = np.zeros_like(u)
    for i in range(N):
        h = Xs[i] / Ks[i]
        G = u
        for j in range(N):
            G = along(mats[j][0] if j == i else mats[j][1], G, j)
        total += (4.0 / h ** 2) * G
    if alpha != 0.0:
        G = u
        for j in range(N):
            G = along(mats[j][1], G, j)
        total += alpha * G
    return total


def _exact_rows(n, K, bc):
    """The exact scaled A and C of one axis as integer matrices over a common
    denominator: (rows_A, d_A, rows_C, d_C) with rows as lists of
    (column, integer) pairs and A = rows_A / d_A."""
    A, C = local_matrices(n)
    m = axis_dim(n, K, bc)
    ra = [dict() for _ in range(m)]
    rc = [dict() for _ in range(m)]

    def index(g):   # array index of position g, None if not an unknown
        if bc == "periodic":
            return g % m
        if bc == "neumann":
            return g
        return None if g in (0, n * K) else g - 1

    for j in range(1, K + 1):
        for r in range(n + 1):
            qr = index(n * (j - 1) + r)
            if qr is None:
                continue
            for t in range(n + 1):
                qt = index(n * (j - 1) + t)
                if qt is None:
                    continue
                ra[qr][qt] = ra[qr].get(qt, Fraction(0)) + A[r][t]
                rc[qr][qt] = rc[qr].get(qt, Fraction(0)) + C[r][t]

    def integral(rows):
        d = 1
        for row in rows:
            for v in row.values():
                d = math.lcm(d, v.denominator)
        return [sorted((c, int(v * d)) for c, v in row.items()) for row in rows], d

    rows_a, da = integral(ra)
    rows_c, dc = integral(rc)
    return rows_a, da, rows_c, dc


def _along_int(rows, V, axis):
    """Integer matrix (rows) times an object array of Python ints along ``axis``."""
    Vm = np.moveaxis(V, axis, 0)
    out = np.empty_like(Vm)
    for q, row in enumerate(rows):
        acc = Vm[row[0][0]] * row[0][1]
        for c, val in row[1:]:
            acc = acc + Vm[c] * val
        out[q] = acc
    return np.moveaxis(out, 0, axis)


def _to_ints(x):
    """x = V / 2^E exactly, V an object array of Python ints."""
    pairs = [float(t).as_integer_ratio() for t in np.asarray(x).ravel()]
    E = max(d.bit_length() - 1 for _, d in pairs)
    V = np.empty(len(pairs), dtype=object)
    V[:] = [num << (E - (d.bit_length() - 1)) for num, d in pairs]
    return V.reshape(np.shape(x)), E


def residual_exact(v, fh, ns, Ks, Xs, alpha, bcs):
    """f^h - L v evaluated exactly (the FP64 inputs v, f^h, X_i and alpha at
    their exact binary values, the local matrices exact rationals) in
    integer arithmetic over a common denominator, rounded once to FP64."""
    v = np.asarray(v, dtype=np.float64)
    N = v.ndim
    V, Ev = _to_ints(v)
    F, Ef = _to_ints(np.asarray(fh, dtype=np.float64))
    mats = [_exact_rows(ns[i], Ks[i], bcs[i]) for i in range(N)]
    terms = []   # (integer array T, scale as a Fraction): term = T * scale
    for i in range(N):
        T, den = V, 2 ** Ev
        for j in range(N):
            rows, d = (mats[j][0], mats[j][1]) if j == i else (mats[j][2], mats[j][3])
            T = _along_int(rows, T, j)
            den *= d
        terms.append((T, 4 * Fraction(Ks[i]) ** 2 / Fraction(Xs[i]) ** 2 / den))
    if alpha != 0.0:
        T, den = V, 2 ** Ev
        for j in range(N):
            T = _along_int(mats[j][2], T, j)
            den *= mats[j][3]
        terms.append((T, Fraction(alpha) / den))
    lcd = 2 ** Ef
    for _, sc in terms:
        lcd = math.lcm(lcd, sc.denominator)
    R = F * (lcd >> Ef)
    for T, sc in terms:
        R = R - T * (sc.numerator * (lcd // sc.denominator))
    out = np.empty(R.size, dtype=np.float64)
    out[:] = [int(x) / lcd for x in R.ravel()]   # int / int rounds correctly
    return out.reshape(v.shape)


def solve(fh, ns, Ks, Xs, alpha, bcs, steps=6):
    """v with L v = f^h (small grids only): a sparse direct solve with the
    FP64-rounded matrix, then residual correction with the residual taken
    exactly (``residual_exact``) until the correction is below 2^-53 of v.
    The rounded matrix alone would carry an error of about cond(L) 2^-53
    (its stiffness no longer annihilates the constants exactly); the
    corrected v is the solution of the exact FEM system rounded to FP64.
    L is SPD unless no axis is Dirichlet and alpha = 0 (constants in the
    kernel)."""
    fh = np.asarray(fh, dtype=np.float64)
    if all(b != "dirichlet" for b in bcs) and not alpha > 0:
        raise ValueError("without a Dirichlet axis the operator needs alpha > 0")
    lu = spla.splu(operator_sparse(ns, Ks, Xs, alpha, bcs))
    v = lu.solve(fh.reshape(-1)).reshape(fh.shape)
    for _ in range(steps):
        r = residual_exact(v, fh, ns, Ks, Xs, alpha, bcs)
        d = lu.solve(r.reshape(-1)).reshape(fh.shape)
        v = v + d
        if np.linalg.norm(d) <= 2.0 ** -53 * np.linalg.norm(v):
            break
    return v
