"""Pins of the periodic- and Neumann-axis oracle (oracle.periodic) to facts
outside it.

* the stiffness annihilates the constants; the mass integrates 1 to the
  length (2K on reference elements);
* the matrices commute with the shift by one cell (translation invariance);
* n = 1: the spectrum is the closed form 3(1 - cos phi) / (2 (2 + cos phi)),
  phi = 2 pi k / K;
* odd extension: the periodic problem on 2K elements with a right-hand side
  odd about x = 0 restricts to the Dirichlet problem on K elements (the
  Dirichlet oracle is pinned to the paper's Table 1 and to closed forms);
  also along one axis of a 2D problem with the other axis Dirichlet;
* convergence: a smooth periodic solution is reproduced at order >= n + 1;
* brute force: on tiny, badly conditioned systems the corrected solve equals
  exact rational elimination of the exact FEM system to 4 ulps;
* Neumann axes: constants in the stiffness kernel, total mass 2K, the n = 1
  closed form 3(1 - cos t)/(2(2 + cos t)), t = pi k / K, k = 0..K, even
  reflection (the periodic problem of 2K elements with the reflected
  right-hand side, boundary rows doubled, restricts to the Neumann
  solution), convergence at order >= n + 1 for a smooth solution with zero
  end slopes, and exact elimination.
"""
import numpy as np
import pytest

import workloads
from oracle import assembly, periodic
from oracle import solve as osolve


@pytest.mark.parametrize("n,K", [(1, 4), (2, 5), (4, 3), (9, 4)])
def test_constants_and_total_mass(n, K):
    A, C = periodic.assemble_1d(n, K)
    one = np.ones(n * K)
    assert np.max(np.abs(A @ one)) < 1e-13 * np.max(np.abs(A))
    assert abs(one @ C @ one - 2.0 * K) < 1e-12 * K
    assert np.allclose(A, A.T, rtol=0, atol=0) and np.allclose(C, C.T, rtol=0, atol=0)


@pytest.mark.parametrize("n,K", [(2, 4), (3, 5), (7, 3)])
def test_shift_by_one_cell(n, K):
    A, C = periodic.assemble_1d(n, K)
    P = np.roll(np.eye(n * K), n, axis=0)
    assert np.array_equal(P @ A @ P.T, A)
    assert np.array_equal(P @ C @ P.T, C)


@pytest.mark.parametrize("K", [3, 8, 16])
def test_linear_spectrum_closed_form(K):
    import scipy.linalg as sla
    A, C = periodic.assemble_1d(1, K)
    got = np.sort(sla.eigh(A, C, eigvals_only=True))
    phi = 2.0 * np.pi * np.arange(K) / K
    want = np.sort(3.0 * (1.0 - np.cos(phi)) / (2.0 * (2.0 + np.cos(phi))))
    assert np.max(np.abs(got - want)) < 1e-13


def odd_extension(fd, n, K, axis):
    """Right-hand side on the periodic axis of 2K elements, odd about x = 0:
    positions 1..nK-1 hold fd, nK+1..2nK-1 its negated mirror, 0 and nK zero."""
    fd = np.moveaxis(np.asarray(fd), axis, 0)
    m = n * K - 1
    out = np.zeros((2 * n * K,) + fd.shape[1:])
    out[1:m + 1] = fd
    out[m + 2:] = -fd[::-1]
    return np.moveaxis(out, 0, axis)


@pytest.mark.parametrize("n,K,alpha", [(1, 8, 0.5), (2, 4, 0.7), (3, 8, 2.0), (5, 4, 0.1)])
def test_odd_extension_1d(n, K, alpha):
    X = 1.3
    fd = workloads.uniform_rhs((assembly.dim(n, K),), seed=3)
    want = osolve.solve(fd, (n,), (K,), (X,), alpha)
    fp = odd_extension(fd, n, K, 0)
    got = periodic.solve(fp, (n,), (2 * K,), (2 * X,), alpha, ("periodic",))
    m = n * K - 1
    assert abs(got[0]) < 1e-13 * np.max(np.abs(got))
    assert abs(got[m + 1]) < 1e-13 * np.max(np.abs(got))
    assert np.max(np.abs(got[1:m + 1] - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("alpha", [0.0, 1.5])
def test_odd_extension_2d_mixed(alpha):
    ns, Ks, Xs = (3, 2), (4, 8), (1.0, 0.7)
    fd = workloads.uniform_rhs(workloads.shape(ns, Ks), seed=4)
    want = osolve.solve(fd, ns, Ks, Xs, alpha)
    fp = odd_extension(fd, ns[0], Ks[0], 0)
    got = periodic.solve(fp, ns, (2 * Ks[0], Ks[1]), (2 * Xs[0], Xs[1]), alpha,
                         ("periodic", "dirichlet"))
    m = ns[0] * Ks[0] - 1
    assert np.max(np.abs(got[1:m + 1] - want)) < 1e-12 * np.max(np.abs(want))
    assert np.max(np.abs(got[0])) < 1e-12 * np.max(np.abs(want))


def test_all_periodic_needs_alpha():
    with pytest.raises(ValueError):
        periodic.solve(np.ones(8), (2,), (4,), (1.0,), 0.0, ("periodic",))


@pytest.mark.parametrize("n", [1, 2, 3])
def test_smooth_periodic_solution_converges(n):
    # -u'' + alpha u = f on [0, X) with u = cos(2 pi x / X) + sin(4 pi x / X);
    # right-hand side: the mass times the interpolant of f (eq. (bvp glob 2)
    # scaled by 2/h, whose load is (2/h) (f, e_q) ~ C I f)
    X, alpha = 1.0, 3.0
    errs = []
    for K in (8, 16, 32):
        x = np.arange(n * K) * X / (n * K)
        w1, w2 = 2 * np.pi / X, 4 * np.pi / X
        u = np.cos(w1 * x) + np.sin(w2 * x)
        f = (w1 ** 2 + alpha) * np.cos(w1 * x) + (w2 ** 2 + alpha) * np.sin(w2 * x)
        _, C = periodic.assemble_1d(n, K)
        v = periodic.solve(C @ f, (n,), (K,), (X,), alpha, ("periodic",))
        errs.append(np.max(np.abs(v - u)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > n + 1 - 0.3), (errs, rates)


def test_apply_operator_matches_matrix():
    ns, Ks, Xs, bcs = (2, 3), (4, 2), (1.0, 2.0), ("periodic", "dirichlet")
    shp = tuple(periodic.axis_dim(n, K, b) for n, K, b in zip(ns, Ks, bcs))
    u = workloads.uniform_rhs(shp, seed=5)
    L = periodic.operator_sparse(ns, Ks, Xs, 0.4, bcs)
    got = periodic.apply_operator(u, ns, Ks, Xs, 0.4, bcs)
    assert np.allclose(got.ravel(), L @ u.ravel(), rtol=0, atol=1e-12 * np.max(np.abs(got)))


def _exact_dense_1d(n, K, bc):
    """Exact rational A, C of one axis by brute-force assembly (lists)."""
    from fractions import Fraction
    from oracle.element import local_matrices
    A, C = local_matrices(n)
    m = {"periodic": n * K, "neumann": n * K + 1}.get(bc, n * K - 1)
    Ag = [[Fraction(0)] * m for _ in range(m)]
    Cg = [[Fraction(0)] * m for _ in range(m)]
    for j in range(K):
        for r in range(n + 1):
            for s in range(n + 1):
                gr, gs = n * j + r, n * j + s
                if bc == "periodic":
                    qr, qs = gr % m, gs % m
                elif bc == "neumann":
                    qr, qs = gr, gs
                elif 0 < gr < n * K and 0 < gs < n * K:
                    qr, qs = gr - 1, gs - 1
                else:
                    continue
                Ag[qr][qs] += A[r][s]
                Cg[qr][qs] += C[r][s]
    return Ag, Cg


def _kron(P, Q):
    return [[a * b for a in ra for b in rb] for ra in P for rb in Q]


def _exact_solve(L, f):
    from fractions import Fraction
    m = len(L)
    M = [row[:] + [Fraction(fv)] for row, fv in zip(L, f)]
    for c in range(m):
        p = next(r for r in range(c, m) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(c + 1, m):
            if M[r][c] != 0:
                t = M[r][c] / M[c][c]
                M[r] = [x - t * y for x, y in zip(M[r], M[c])]
    x = [None] * m
    for c in range(m - 1, -1, -1):
        x[c] = (M[c][m] - sum(M[c][k] * x[k] for k in range(c + 1, m))) / M[c][c]
    return x


@pytest.mark.parametrize("ns,Ks,Xs,alpha,bcs", [
    ((3,), (4,), (1.0,), 1e-3, ("periodic",)),
    ((2, 2), (3, 2), (1.0, 0.5), 0.0, ("periodic", "dirichlet")),
    ((4,), (2,), (2.0,), 1e-4, ("periodic",)),
    ((3,), (4,), (1.0,), 1e-3, ("neumann",)),
    ((2, 2), (2, 3), (1.0, 0.5), 0.0, ("neumann", "dirichlet")),
])
def test_corrected_solve_is_the_exact_solution(ns, Ks, Xs, alpha, bcs):
    # brute force: exact rational elimination of the exact FEM system
    from fractions import Fraction
    mats = [_exact_dense_1d(n, K, b) for n, K, b in zip(ns, Ks, bcs)]
    L = None
    for i in range(len(ns)):
        s = 4 * Fraction(Ks[i]) ** 2 / Fraction(Xs[i]) ** 2
        T = None
        for j in range(len(ns)):
            M = mats[j][0] if j == i else mats[j][1]
            T = M if T is None else _kron(T, M)
        T = [[s * x for x in row] for row in T]
        L = T if L is None else [[a + b for a, b in zip(r1, r2)] for r1, r2 in zip(L, T)]
    if alpha:
        T = None
        for j in range(len(ns)):
            T = mats[j][1] if T is None else _kron(T, mats[j][1])
        L = [[a + Fraction(alpha) * b for a, b in zip(r1, r2)] for r1, r2 in zip(L, T)]
    shp = tuple(periodic.axis_dim(n, K, b) for n, K, b in zip(ns, Ks, bcs))
    f = workloads.uniform_rhs(shp, seed=9)
    want = np.array([float(x) for x in _exact_solve(L, f.ravel().tolist())]).reshape(shp)
    got = periodic.solve(f, ns, Ks, Xs, alpha, bcs)
    assert np.max(np.abs(got - want)) <= 4 * np.finfo(float).eps * np.max(np.abs(want))


@pytest.mark.parametrize("n,K", [(1, 4), (2, 5), (4, 3), (9, 4)])
def test_neumann_constants_and_total_mass(n, K):
    A, C = [M.toarray() for M in periodic.axis_matrices(n, K, "neumann")]
    one = np.ones(n * K + 1)
    assert np.max(np.abs(A @ one)) < 1e-13 * np.max(np.abs(A))
    assert abs(one @ C @ one - 2.0 * K) < 1e-12 * K


@pytest.mark.parametrize("K", [3, 8, 16])
def test_neumann_linear_spectrum_closed_form(K):
    import scipy.linalg as sla
    A, C = [M.toarray() for M in periodic.axis_matrices(1, K, "neumann")]
    got = np.sort(sla.eigh(A, C, eigvals_only=True))
    t = np.pi * np.arange(K + 1) / K
    want = np.sort(3.0 * (1.0 - np.cos(t)) / (2.0 * (2.0 + np.cos(t))))
    assert np.max(np.abs(got - want)) < 1e-13


def even_extension(fn, n, K, axis):
    """Right-hand side on the periodic axis of 2K elements, even about x = 0:
    position g' holds fn at g' (g' <= nK) or 2nK - g', the boundary values
    (g = 0, nK) doubled."""
    fn = np.moveaxis(np.asarray(fn, dtype=np.float64), axis, 0)
    m = n * K
    w = fn.copy()
    w[0] *= 2.0
    w[m] *= 2.0
    out = np.concatenate([w[:m + 1], w[1:m][::-1]], axis=0)
    return np.moveaxis(out, 0, axis)


@pytest.mark.parametrize("n,K,alpha", [(1, 8, 0.5), (2, 4, 0.7), (3, 8, 2.0), (5, 4, 0.1)])
def test_neumann_even_extension_1d(n, K, alpha):
    X = 1.3
    fn = workloads.uniform_rhs((n * K + 1,), seed=13)
    want = periodic.solve(fn, (n,), (K,), (X,), alpha, ("neumann",))
    got = periodic.solve(even_extension(fn, n, K, 0), (n,), (2 * K,), (2 * X,), alpha, ("periodic",))
    assert np.max(np.abs(got[:n * K + 1] - want)) < 1e-12 * np.max(np.abs(want))
    assert np.max(np.abs(got[n * K + 1:] - want[1:n * K][::-1])) < 1e-12 * np.max(np.abs(want))


def test_neumann_even_extension_2d_mixed():
    ns, Ks, Xs, alpha = (2, 3), (4, 4), (1.0, 0.7), 0.0
    fn = workloads.uniform_rhs((ns[0] * Ks[0] + 1, ns[1] * Ks[1] - 1), seed=14)
    want = periodic.solve(fn, ns, Ks, Xs, alpha, ("neumann", "dirichlet"))
    got = periodic.solve(even_extension(fn, ns[0], Ks[0], 0), ns, (2 * Ks[0], Ks[1]),
                         (2 * Xs[0], Xs[1]), alpha, ("periodic", "dirichlet"))
    assert np.max(np.abs(got[:ns[0] * Ks[0] + 1] - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("n", [1, 2, 3])
def test_neumann_smooth_solution_converges(n):
    # -u'' + alpha u = f on [0, X] with u = cos(pi x / X) + 0.5 cos(3 pi x / X)
    # (zero slope at both ends); right-hand side C I f as in the periodic test
    X, alpha = 1.0, 2.0
    errs = []
    for K in (8, 16, 32):
        x = np.arange(n * K + 1) * X / (n * K)
        w1, w3 = np.pi / X, 3 * np.pi / X
        u = np.cos(w1 * x) + 0.5 * np.cos(w3 * x)
        f = (w1 ** 2 + alpha) * np.cos(w1 * x) + 0.5 * (w3 ** 2 + alpha) * np.cos(w3 * x)
        C = periodic.axis_matrices(n, K, "neumann")[1].toarray()
        v = periodic.solve(C @ f, (n,), (K,), (X,), alpha, ("neumann",))
        errs.append(np.max(np.abs(v - u)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > n + 1 - 0.3), (errs, rates)
