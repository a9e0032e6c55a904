"""Variable-coefficient operator -div(a grad u) + alpha u (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper proposes the fast solver as a preconditioner for general
second-order elliptic problems (Section 1) and evaluates integrals of the
data by the (n+1)-point Gauss rule per variable (Section 2, paragraph 5).
This module defines the matching FEM operator on the same space and in the
same scaled form as eq. (bvp glob 2): on every element, mapped to [-1, 1]^N,

    L_a = sum_i 4 h_i^-2  int a  d_i u  d_i phi  +  alpha int u phi,

both integrals by the (n_i+1)-point Gauss-Legendre rule in every variable,
with a given at those Gauss points.  For a = 1 the rule is exact and L_a is
the operator of eq. (bvp glob 2).

Coefficient layout: ``a_full[E, Q]`` with E the C-order index of the element
(e_0, .., e_{N-1}) and Q the C-order index of the Gauss point (q_0, ..).

Two independent realisations: ``operator_sparse`` assembles the global
matrix element by element from Kronecker products of 1D basis tables (the
definition, small meshes only); ``apply`` is a vectorised matrix-free numpy
apply for any size.  ``solve`` is a sparse direct solve of the assembled
matrix.
"""
import functools
import itertools

import mpmath
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_DPS = 40


@functools.lru_cache(maxsize=None)
def _gauss_mp(npts):
    """Gauss-Legendre nodes (increasing) and weights at _DPS digits: Newton on
    P_npts from numpy's FP64 nodes; w = 2 / ((1 - x^2) P'(x)^2)."""
    x0, _ = np.polynomial.legendre.leggauss(npts)
    xs, ws = [], []
    with mpmath.workdps(_DPS):
        for z in x0:
            z = mpmath.mpf(float(z))
            for _ in range(8):
                p, dp = _legendre_mp(npts, z)
                z = z - p / dp
            p, dp = _legendre_mp(npts, z)
            xs.append(z)
            ws.append(2 / ((1 - z * z) * dp * dp))
    return xs, ws


def _legendre_mp(m, z):
    """P_m(z) and P_m'(z) by the three-term recurrence."""
    p0, p1 = mpmath.mpf(1), z
    for k in range(2, m + 1):
        p0, p1 = p1, ((2 * k - 1) * z * p1 - (k - 1) * p0) / k
    if m == 0:
        return p0, mpmath.mpf(0)
    return p1, m * (z * p1 - p0) / (z * z - 1)


def gauss_rule(n):
    """(n+1)-point Gauss-Legendre nodes (increasing) and weights on [-1, 1],
    each rounded once to FP64."""
    xs, ws = _gauss_mp(n + 1)
    return np.array([float(x) for x in xs]), np.array([float(w) for w in ws])


def basis_tables(n):
    """B[q, r] = e_r(xi_q), D[q, r] = e_r'(xi_q) at the Gauss nodes xi_q (see
    _basis_tables)."""
    B, D = _basis_tables(n)
    return B.copy(), D.copy()


@functools.lru_cache(maxsize=None)
def _basis_tables(n):
    """The tables of basis_tables from
    the product form of the Lagrange basis at _DPS digits, rounded once:
    e_r(x) = prod_{k != r} (x - x_k) / (x_r - x_k),
    e_r'(x) = sum_{j != r} 1 / (x_r - x_j) prod_{k != r, j} (x - x_k) / (x_r - x_k)."""
    xs, _ = _gauss_mp(n + 1)
    B = np.zeros((n + 1, n + 1))
    D = np.zeros((n + 1, n + 1))
    with mpmath.workdps(_DPS):
        nodes = [mpmath.mpf(-1) + mpmath.mpf(2 * k) / n for k in range(n + 1)]
        for q, x in enumerate(xs):
            for r in range(n + 1):
                v = mpmath.mpf(1)
                for k in range(n + 1):
                    if k != r:
                        v *= (x - nodes[k]) / (nodes[r] - nodes[k])
                d = mpmath.mpf(0)
                for j in range(n + 1):
                    if j == r:
                        continue
                    t = 1 / (nodes[r] - nodes[j])
                    for k in range(n + 1):
                        if k != r and k != j:
                            t *= (x - nodes[k]) / (nodes[r] - nodes[k])
                    d += t
                B[q, r] = float(v)
                D[q, r] = float(d)
    return B, D


def gauss_points(n, K, X):
    """Physical coordinates of the Gauss points, shape (K, n+1)."""
    xi, _ = gauss_rule(n)
    h = X / K
    return (np.arange(K)[:, None] + (xi[None, :] + 1.0) / 2.0) * h


def expand_separable(c0, c1, tables):
    """a_full for a = c0 + c1 prod_i t_i(x_i) from per-axis tables t_i[e_i, q_i]."""
    N = len(tables)
    prod = np.ones([1] * (2 * N))
    for i, t in enumerate(tables):
        shape = [1] * (2 * N)
        shape[i] = t.shape[0]
        shape[N + i] = t.shape[1]
        prod = prod * t.reshape(shape)
    Ks = [t.shape[0] for t in tables]
    bs = [t.shape[1] for t in tables]
    return (c0 + c1 * prod).reshape(int(np.prod(Ks)), int(np.prod(bs)))


def _kron_all(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def local_matrix(ns, hs, alpha, a_el):
    """Element matrix over the (n_i+1)^N local nodes (C order) for the Gauss
    values a_el (C order over the Gauss points)."""
    N = len(ns)
    tabs = [basis_tables(n) for n in ns]
    w = _kron_all([gauss_rule(n)[1] for n in ns])
    out = None
    for i in range(N):
        G = _kron_all([tabs[j][1] if j == i else tabs[j][0] for j in range(N)])
        term = (4.0 / hs[i] ** 2) * (G.T @ ((w * a_el)[:, None] * G))
        out = term if out is None else out + term
    if alpha != 0.0:
        Bf = _kron_all([t[0] for t in tabs])
        out = out + alpha * (Bf.T @ (w[:, None] * Bf))
    return out


def operator_sparse(ns, Ks, Xs, alpha, a_full):
    """Assembled FP64 matrix of L_a on the interior unknowns (C order)."""
    N = len(ns)
    hs = [Xs[i] / Ks[i] for i in range(N)]
    ms = [ns[i] * Ks[i] - 1 for i in range(N)]
    strides = [int(np.prod(ms[i + 1:])) for i in range(N)]
    local_pos = list(itertools.product(*[range(n + 1) for n in ns]))
    rows, cols, vals = [], [], []
    for E, es in enumerate(itertools.product(*[range(K) for K in Ks])):
        Ael = local_matrix(ns, hs, alpha, a_full[E])
        gidx = []
        for rs in local_pos:
            g = [ns[i] * es[i] + rs[i] for i in range(N)]
            if all(1 <= g[i] <= ns[i] * Ks[i] - 1 for i in range(N)):
                gidx.append(sum((g[i] - 1) * strides[i] for i in range(N)))
            else:
                gidx.append(-1)
        gidx = np.array(gidx)
        keep = np.nonzero(gidx >= 0)[0]
        r = np.repeat(gidx[keep], keep.size)
        c = np.tile(gidx[keep], keep.size)
        rows.append(r)
        cols.append(c)
        vals.append(Ael[np.ix_(keep, keep)].ravel())
    M = int(np.prod(ms))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(M, M))


def _contract(x, M, axis):
    """y[..., q, ...] = sum_r M[q, r] x[..., r, ...] along ``axis``."""
    return np.moveaxis(np.tensordot(M, x, axes=([1], [axis])), 0, axis)


def apply(u, ns, Ks, Xs, alpha, a_full):
    """L_a u, matrix-free: gather element values, integrate at the Gauss
    points, scatter-add (FP64).  u: grid array, or (nrhs, grid)."""
    N = len(ns)
    grid = tuple(n * K - 1 for n, K in zip(ns, Ks))
    batched = u.ndim == N + 1
    ub = u if batched else u[None]
    R = ub.shape[0]
    full = np.zeros((R,) + tuple(n * K + 1 for n, K in zip(ns, Ks)))
    full[(slice(None),) + tuple(slice(1, n * K) for n, K in zip(ns, Ks))] = ub
    bs = [n + 1 for n in ns]
    # element values U[R, e_0.., r_0..]
    U = np.empty((R,) + tuple(Ks) + tuple(bs))
    for rs in itertools.product(*[range(b) for b in bs]):
        sl = tuple(slice(rs[i], rs[i] + ns[i] * Ks[i], ns[i]) for i in range(N))
        U[(Ellipsis,) + tuple(rs)] = full[(slice(None),) + sl]
    tabs = [basis_tables(n) for n in ns]
    w = _kron_all([gauss_rule(n)[1] for n in ns]).reshape(bs)
    a = a_full.reshape(tuple(Ks) + tuple(bs))
    hs = [Xs[i] / Ks[i] for i in range(N)]
    out_el = np.zeros_like(U)
    ax = lambda i: 1 + N + i                       # axis of local index i in U
    for i in range(N):
        g = U
        for j in range(N):
            g = _contract(g, tabs[j][1] if j == i else tabs[j][0], ax(j))
        g = g * ((4.0 / hs[i] ** 2) * w * a)[None]
        for j in range(N):
            g = _contract(g, (tabs[j][1] if j == i else tabs[j][0]).T, ax(j))
        out_el += g
    if alpha != 0.0:
        g = U
        for j in range(N):
            g = _contract(g, tabs[j][0], ax(j))
        g = g * (alpha * w)[None, ...]
        for j in range(N):
            g = _contract(g, tabs[j][0].T, ax(j))
        out_el += g
    acc = np.zeros_like(full)
    for rs in itertools.product(*[range(b) for b in bs]):
        sl = tuple(slice(rs[i], rs[i] + ns[i] * Ks[i], ns[i]) for i in range(N))
        acc[(slice(None),) + sl] += out_el[(Ellipsis,) + tuple(rs)]
    out = acc[(slice(None),) + tuple(slice(1, n * K) for n, K in zip(ns, Ks))]
    assert out.shape[1:] == grid
    return out if batched else out[0]


def load(fvals, ns, Ks):
    """Scaled load vector sum_E int f phi (reference variables) from the values
    of f at the Gauss points, fvals[E, Q] (same layout as a_full)."""
    N = len(ns)
    bs = [n + 1 for n in ns]
    tabs = [basis_tables(n) for n in ns]
    w = _kron_all([gauss_rule(n)[1] for n in ns]).reshape(bs)
    g = fvals.reshape(tuple(Ks) + tuple(bs)) * w
    for j in range(N):
        g = _contract(g, tabs[j][0].T, N + j)
    full = np.zeros(tuple(n * K + 1 for n, K in zip(ns, Ks)))
    for rs in itertools.product(*[range(b) for b in bs]):
        sl = tuple(slice(rs[i], rs[i] + ns[i] * Ks[i], ns[i]) for i in range(N))
        full[sl] += g[(Ellipsis,) + tuple(rs)]
    return full[tuple(slice(1, n * K) for n, K in zip(ns, Ks))]


def gauss_values(func, ns, Ks, Xs):
    """func(x_0, .., x_{N-1}) at every Gauss point, layout [E, Q]."""
    N = len(ns)
    pts = [gauss_points(ns[i], Ks[i], Xs[i]) for i in range(N)]
    coords = []
    for i in range(N):
        shape = [1] * (2 * N)
        shape[i] = Ks[i]
        shape[N + i] = ns[i] + 1
        coords.append(pts[i].reshape(shape))
    v = func(*coords)
    full_shape = tuple(Ks) + tuple(n + 1 for n in ns)
    v = np.broadcast_to(v, full_shape)
    return np.ascontiguousarray(v).reshape(int(np.prod(Ks)), int(np.prod([n + 1 for n in ns])))


def solve(f, ns, Ks, Xs, alpha, a_full):
    """u = L_a^{-1} f by a sparse direct solve (small meshes)."""
    L = operator_sparse(ns, Ks, Xs, alpha, a_full).tocsc()
    return spla.spsolve(L, f.ravel()).reshape(f.shape)
