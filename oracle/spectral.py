"""1D eigenpairs of the FEM pencil A v = lambda C v (oracle).

Two independent routes to the spectrum of eq. (eig_glob):

(i)  ``eigen_dense``: the plain dense generalized eigensolve of the assembled
     FP64 matrices (scipy.linalg.eigh).  Accurate only while
     u * lambda_max / lambda_min is small (small K), because the smallest
     eigenvalues are O(K^-2) while the entries are O(1)..O(10^3).

(ii) ``eigen_structured``: high precision, following Theorem 1 (first of the
     two theorems of Section 2).  The pencil is invariant under shifting by
     one element, so for the wave number phi = pi k / K the values at mesh
     node j and in element j of a Bloch wave are U e^{i phi j} and
     B e^{i phi j}; the element vector of element j is then
     e^{i phi j} T [U; B] with T = [[e^{-i phi}, 0], [0, I], [1, 0]], and the
     n eigenvalues lambda_k^(l) are those of the n x n Hermitian pencil
     (T^H A T, T^H C T).  This is the same set of n roots as the secular
     equation eq. (theta) at theta_k = cos(pi k / K) (static condensation of
     the interior nodes); the oracle does not use eq. (theta).  The
     eigenvalues are computed in mpmath (the paper computes its eigenvalues
     in quadruple precision, Section 2, paragraph 5), then p_k^(l) solves
     G~(lambda) p = -g(lambda) (Theorem 1, item 3) in mpmath, and the
     eigenvectors s_k^(l), s_0^(l) are built as Theorem 1 states.  Their
     C-norms are computed directly (s^T C s), not by the closed form the
     theorem on the transforms gives.

``basis`` returns a dense FP64 matrix V with C-orthonormal columns and the
matching eigenvalues; ``solve`` uses it.
"""
import os
import multiprocessing as mproc
from functools import lru_cache

import mpmath as mp
import numpy as np
import scipy.linalg as sla

from .element import local_matrices, blocks, to_mp, generalized_eigh_mp, interior_eigen
from .assembly import assemble_1d, assemble_1d_sparse, dim

# mpmath working precision (decimal digits) of the structured route; quad
# precision is about 34 digits.
DPS = 40
_CACHE_VERSION = 3


def eigen_dense(n, K):
    """Route (i): dense FP64 generalized eigensolve. Returns (lam asc, V)."""
    A, C = assemble_1d(n, K)
    lam, V = sla.eigh(A, C)
    return lam, V


def bloch_pencil(n, phi, dps=DPS):
    """The n x n Hermitian pencil (T^H A T, T^H C T) at wave number phi (mpmath)."""
    with mp.workdps(dps):
        A, C = local_matrices(n)
        Am, Cm = to_mp(A), to_mp(C)
        T = mp.matrix(n + 1, n)
        T[0, 0] = mp.expj(-phi)
        T[n, 0] = mp.mpf(1)
        for r in range(1, n):
            T[r, r] = mp.mpf(1)
        return T.H * Am * T, T.H * Cm * T


def _wave_k(args):
    """Eigenvalues lambda_k^(l) (l = 1..n, ascending) and p_k^(l) for one k."""
    n, K, k, dps = args
    with mp.workdps(dps):
        phi = mp.pi * k / K
        Ab, Cb = bloch_pencil(n, phi, dps)
        lam, _ = generalized_eigh_mp(Ab, Cb)
        A, C = local_matrices(n)
        a0, a, At, an, achk = blocks(A)
        c0, c, Ct, cn, cchk = blocks(C)
        ps = []
        for lm in lam:
            if n == 1:
                ps.append([])
                continue
            G = to_mp(At) - lm * to_mp(Ct)
            g = mp.matrix([mp.mpf(x.numerator) / x.denominator for x in a]) - \
                lm * mp.matrix([mp.mpf(x.numerator) / x.denominator for x in c])
            p = mp.lu_solve(G, -g)
            ps.append([p[i] for i in range(n - 1)])
        return k, [mp.nstr(x, dps) for x in lam], [[mp.nstr(x, dps) for x in p] for p in ps]


def _cache_dir():
    d = os.environ.get("HOFEM_ORACLE_CACHE")
    if d:
        return d
    return os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        ".oracle_cache")


@lru_cache(maxsize=32)
def eigen_structured(n, K, dps=DPS, workers=None):
    """Route (ii).  Returns a dict of FP64 arrays (values rounded once from
    ``dps``-digit mpmath results):

      lam0 (n-1,)          eigenvalues lambda_0^(l) of the interior-node pencil
      E    (n-1, n-1)      column l = e^(l), C~-normalised
      lam  (K-1, n)        lam[k-1, l-1] = lambda_k^(l), ascending in l
      p    (K-1, n, n-1)   p[k-1, l-1] = p_k^(l)

    Results are cached in-process and, as a plain .npz written by this
    function, on disk (directory ``$HOFEM_ORACLE_CACHE`` or ``.oracle_cache``
    beside this package).
    """
    path = os.path.join(_cache_dir(), f"eig_n{n}_K{K}_d{dps}_v{_CACHE_VERSION}.npz")
    if os.path.exists(path):
        z = np.load(path)
        return {key: z[key] for key in z.files}
    lam0m, Em = interior_eigen(n, dps) if n > 1 else ([], mp.matrix(0, 0))
    tasks = [(n, K, k, dps) for k in range(1, K)]
    if workers is None:
        workers = min(len(tasks), os.cpu_count() or 1, 16)
    if workers > 1 and len(tasks) > 8:
        ctx = mproc.get_context("fork")
        with ctx.Pool(workers) as pool:
            res = pool.map(_wave_k, tasks, chunksize=max(1, len(tasks) // (4 * workers)))
    else:
        res = [_wave_k(t) for t in tasks]
    res.sort(key=lambda r: r[0])
    lam = np.array([[float(mp.mpf(x)) for x in r[1]] for r in res]).reshape(K - 1, n)
    p = np.array([[[float(mp.mpf(x)) for x in pl] for pl in r[2]] for r in res]).reshape(K - 1, n, n - 1)
    out = {
        "lam0": np.array([float(x) for x in lam0m]),
        "E": np.array([[float(Em[i, j]) for j in range(n - 1)] for i in range(n - 1)]).reshape(n - 1, n - 1),
        "lam": lam,
        "p": p,
    }
    try:
        os.makedirs(_cache_dir(), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, **out)
        os.replace(tmp, path)
    except OSError:
        pass
    return out


def _sin_table(K):
    """sin(pi t / K) for t = 0..2K-1, arguments reduced exactly before rounding."""
    t = np.arange(2 * K)
    return np.sin(np.pi * t / K)


def eigenvectors_structured(n, K, data=None):
    """Unnormalised eigenvectors of Theorem 1 as a dense (m, m) FP64 matrix.

    Column order: the n-1 vectors s_0^(l) first, then s_k^(l) for
    k = 1..K-1, l = 1..n.  Returns (S, lam) with lam the matching scaled
    eigenvalues.
    """
    if data is None:
        data = eigen_structured(n, K)
    m = dim(n, K)
    S = np.zeros((m, m))
    lam = np.zeros(m)
    tab = _sin_table(K)
    # k = 0: zero at the nodes, (-P)^{j-1} e^(l) in element j.
    col = 0
    for l in range(n - 1):
        e = data["E"][:, l]
        for j in range(1, K + 1):
            v = e if (j - 1) % 2 == 0 else -e[::-1]
            S[n * (j - 1): n * (j - 1) + n - 1, col] = v
        lam[col] = data["lam0"][l]
        col += 1
    # k >= 1: sin(pi k j / K) at node j; p sin(pi k (j-1)/K) + P p sin(pi k j/K)
    # in element j (P reverses the order of the interior points).
    ks = np.arange(1, K)
    js = np.arange(0, K + 1)
    sines = tab[np.outer(ks, js) % (2 * K)]            # (K-1, K+1): sin(pi k j / K)
    node_rows = n * np.arange(1, K) - 1
    cols = (n - 1) + n * (ks - 1)[:, None] + np.arange(n)[None, :]   # (K-1, n)
    for l in range(n):
        c = cols[:, l]
        S[np.ix_(node_rows, c)] = sines[:, 1:K].T
        lam[c] = data["lam"][:, l]
        if n > 1:
            p = data["p"][:, l, :]                        # (K-1, n-1)
            for j in range(1, K + 1):
                rows = n * (j - 1) + np.arange(n - 1)
                left = sines[:, j - 1]                     # sin(pi k (j-1)/K)
                right = sines[:, j]                        # sin(pi k j / K)
                S[np.ix_(rows, c)] = (p * left[:, None] + p[:, ::-1] * right[:, None]).T
    return S, lam


@lru_cache(maxsize=8)
def basis(n, K, route="structured"):
    """C-orthonormal eigenvector matrix V (m, m) and eigenvalues lam (m,).

    route: "structured" (high precision, any K) or "dense" (FP64 eigh, small K).
    """
    if route == "dense":
        lam, V = eigen_dense(n, K)
        return V, lam
    S, lam = eigenvectors_structured(n, K)
    _, Cs = assemble_1d_sparse(n, K)
    norms2 = np.einsum("ij,ij->j", S, Cs @ S)
    V = S / np.sqrt(norms2)[None, :]
    return V, lam
