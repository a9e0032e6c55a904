"""Reference element of the nth-order Lagrange FEM, exact and in high precision.

Follows Section 2, paragraph 1 of the paper: the reference element is
sigma_0 = [-1, 1] with the Lagrange basis {e_l} of P_n fixed by
e_l(-1 + 2k/n) = delta_kl, and the local matrices are

    A_kl = int_{sigma_0} e_k'(x) e_l'(x) dx,   C_kl = int_{sigma_0} e_k(x) e_l(x) dx.

Their 3x3 block form (eq. (matrAC)) splits off the two end nodes from the
n-1 interior ("bubble") nodes; P is the reflection of R^{n-1} that reverses
the order of the interior nodes.  The element eigenproblems of eq. (eig_elem)
are solved here in mpmath (high precision), with the normalisation
C~ e^(l) . e^(l) = 1 stated after Lemma 1.

Everything is exact rational arithmetic (fractions.Fraction) except the
eigenproblems, which use mpmath at a caller-chosen precision.
"""
from fractions import Fraction
from functools import lru_cache

import mpmath as mp


def lagrange_nodes(n):
    """Equispaced interpolation nodes -1 + 2k/n, k = 0..n, as exact rationals."""
    return [Fraction(-1) + Fraction(2 * k, n) for k in range(n + 1)]


def _pmul(p, q):
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _pderiv(p):
    return [i * p[i] for i in range(1, len(p))] or [Fraction(0)]


def _pint_m11(p):
    """Exact integral over [-1, 1] of sum_i p[i] x^i."""
    return sum((Fraction(2, i + 1) * c for i, c in enumerate(p) if i % 2 == 0), Fraction(0))


@lru_cache(maxsize=None)
def lagrange_basis(n):
    """Monomial coefficients (ascending powers) of e_0..e_n, exact."""
    xs = lagrange_nodes(n)
    basis = []
    for l in range(n + 1):
        p = [Fraction(1)]
        for m in range(n + 1):
            if m != l:
                d = xs[l] - xs[m]
                p = _pmul(p, [-xs[m] / d, Fraction(1) / d])
        basis.append(tuple(p))
    return tuple(basis)


@lru_cache(maxsize=None)
def local_matrices(n):
    """Exact local stiffness A and mass C, each an (n+1)x(n+1) tuple of Fractions."""
    if n < 1:
        raise ValueError("order n must be >= 1")
    basis = lagrange_basis(n)
    ders = [_pderiv(list(b)) for b in basis]
    A = tuple(tuple(_pint_m11(_pmul(ders[k], ders[l])) for l in range(n + 1)) for k in range(n + 1))
    C = tuple(tuple(_pint_m11(_pmul(list(basis[k]), list(basis[l]))) for l in range(n + 1))
              for k in range(n + 1))
    return A, C


def blocks(M):
    """Split a local matrix into the blocks of eq. (matrAC).

    Returns (m0, m, M_tilde, mn, m_check): m0 = M[0][0], m = M[1:n, 0],
    M_tilde = M[1:n, 1:n], mn = M[0][n], m_check = M[1:n, n].
    """
    n = len(M) - 1
    m0 = M[0][0]
    mvec = [M[r][0] for r in range(1, n)]
    Mt = [[M[r][c] for c in range(1, n)] for r in range(1, n)]
    mn = M[0][n]
    mchk = [M[r][n] for r in range(1, n)]
    return m0, mvec, Mt, mn, mchk


def to_mp(M):
    """Fraction matrix -> mpmath matrix (at the current mp precision)."""
    return mp.matrix([[mp.mpf(x.numerator) / x.denominator for x in row] for row in M])


def generalized_eigh_mp(A, C):
    """Eigenpairs of the symmetric-definite pencil A x = lam C x in mpmath.

    A, C: mpmath matrices (real symmetric or complex Hermitian), C > 0.
    Returns (lam ascending as a list of mpf, X with C-orthonormal columns).
    Plain reduction: C = L L^H, eigenpairs of L^-1 A L^-H, back-substitute.
    """
    L = mp.cholesky(C)
    Li = L ** -1
    M = Li * A * Li.H
    M = (M + M.H) / 2
    size = M.rows
    is_real = all(mp.im(M[i, j]) == 0 for i in range(size) for j in range(size))
    if is_real:
        M = mp.matrix([[mp.re(M[i, j]) for j in range(size)] for i in range(size)])
        E, Q = mp.eigsy(M)
    else:
        E, Q = mp.eighe(M)
    order = sorted(range(size), key=lambda i: E[i])
    lam = [mp.re(E[i]) for i in order]
    X = Li.H * Q
    cols = mp.matrix(size, size)
    for new, old in enumerate(order):
        for r in range(size):
            cols[r, new] = X[r, old]
    return lam, cols


def interior_eigen(n, dps=40):
    """Eigenpairs of the interior-node problem  A~ e = lam C~ e  (eq. (eig_elem)).

    Returns (lam0, E): lam0 ascending (n-1 mpf values), E an (n-1)x(n-1)
    mpmath matrix whose column l is e^(l) with C~ e^(l) . e^(l) = 1.  The
    sign of each column is fixed so that its lowest-index entry of magnitude
    at least half the largest is positive (Lemma 1 leaves the sign free; the
    basis only enters the solve through products that contain it twice, and
    a rule with a margin does not depend on rounding).
    """
    with mp.workdps(dps):
        A, C = local_matrices(n)
        _, _, At, _, _ = blocks(A)
        _, _, Ct, _, _ = blocks(C)
        lam, X = generalized_eigh_mp(to_mp(At), to_mp(Ct))
        X = mp.matrix([[mp.re(X[i, j]) for j in range(X.cols)] for i in range(X.rows)])
        for j in range(X.cols):
            top = max(abs(X[i, j]) for i in range(X.rows))
            lead = next(i for i in range(X.rows) if abs(X[i, j]) >= top / 2)
            if X[lead, j] < 0:
                for i in range(X.rows):
                    X[i, j] = -X[i, j]
        return lam, X


def element_eigenvalues(n, dps=40):
    """Spectrum S_n of the full element pencil A e = lam C e (eq. (eig_elem))."""
    with mp.workdps(dps):
        A, C = local_matrices(n)
        lam, _ = generalized_eigh_mp(to_mp(A), to_mp(C))
        return lam
