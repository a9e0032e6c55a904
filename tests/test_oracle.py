"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  They check the oracle against values the
paper prints (the interior spectra S~_2..S~_5, Table 1), textbook special
cases (linear element, the n = 1 closed form), invariants (C-orthonormality,
A-diagonalisation, Rayleigh-quotient upper bounds), brute force on tiny
inputs (a full mpmath eigensolve of the exactly assembled pencil, sparse
direct solves) and convergence rates.
"""
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import assembly, element, load, solve, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Reference element (Section 2, paragraph 1)
# --------------------------------------------------------------------------

def test_linear_element_is_textbook():
    # n = 1: the classical linear element on [-1, 1].
    A, C = element.local_matrices(1)
    assert A == ((Fraction(1, 2), Fraction(-1, 2)), (Fraction(-1, 2), Fraction(1, 2)))
    assert C == ((Fraction(2, 3), Fraction(1, 3)), (Fraction(1, 3), Fraction(2, 3)))


def test_quadratic_element_is_textbook():
    # n = 2 on [-1, 1] with nodes -1, 0, 1: stiffness (1/6)[[7,-8,1],[-8,16,-8],[1,-8,7]],
    # mass (1/15)[[4,2,-1],[2,16,2],[-1,2,4]].
    A, C = element.local_matrices(2)
    Aref = [[7, -8, 1], [-8, 16, -8], [1, -8, 7]]
    Cref = [[4, 2, -1], [2, 16, 2], [-1, 2, 4]]
    assert all(A[i][j] == Fraction(Aref[i][j], 6) for i in range(3) for j in range(3))
    assert all(C[i][j] == Fraction(Cref[i][j], 15) for i in range(3) for j in range(3))


@pytest.mark.parametrize("n", range(1, 10))
def test_local_matrix_identities(n):
    A, C = element.local_matrices(n)
    for i in range(n + 1):
        assert sum(A[i]) == 0                                   # constants in the kernel
        for j in range(n + 1):
            assert A[i][j] == A[j][i] and C[i][j] == C[j][i]     # symmetric
            assert A[i][j] == A[n - i][n - j]                    # persymmetric (reflection)
            assert C[i][j] == C[n - i][n - j]
    assert sum(sum(r) for r in C) == 2                           # integral of 1 over [-1, 1]


def _solve_exact(M, b):
    """Gauss-Jordan elimination over the rationals."""
    size = len(b)
    aug = [list(M[i]) + [b[i]] for i in range(size)]
    for col in range(size):
        piv = next(r for r in range(col, size) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        for r in range(size):
            if r != col and aug[r][col] != 0:
                f = aug[r][col] / aug[col][col]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[col])]
    return [aug[i][size] / aug[i][i] for i in range(size)]


@pytest.mark.parametrize("n", range(2, 10))
def test_static_condensation_gives_linear_element(n):
    # Eliminating the interior nodes of the stiffness leaves the linear element
    # exactly: condensed matrix [[1/2, -1/2], [-1/2, 1/2]].
    A, _ = element.local_matrices(n)
    a0, a, At, an, achk = element.blocks(A)
    y = _solve_exact(At, a)
    s00 = a0 - sum(x * z for x, z in zip(a, y))
    s0n = an - sum(x * z for x, z in zip(achk, y))
    assert s00 == Fraction(1, 2) and s0n == Fraction(-1, 2)


def _golden_interior():
    out = {}
    with open(os.path.join(GOLDEN, "interior_spectra.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, expr = line.split()
            val = eval(expr, {"sqrt": mp.sqrt, "__builtins__": {}})
            out.setdefault(int(n), []).append(mp.mpf(val))
    return out


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_interior_spectrum_matches_printed_values(n):
    with mp.workdps(40):
        want = sorted(_golden_interior()[n])
        got, _ = element.interior_eigen(n, dps=40)
        assert len(got) == len(want)
        for g, w in zip(got, want):
            assert abs(g - w) < mp.mpf(10) ** -30


@pytest.mark.parametrize("n", range(2, 10))
def test_element_spectra_simple_and_parity(n):
    # Lemma 1 and the remark after eq. (theta): simple eigenvalues for n <= 9,
    # e^(l) even for odd l and odd for even l, C~-normalised.
    lam, E = element.interior_eigen(n, dps=40)
    full = element.element_eigenvalues(n, dps=40)
    with mp.workdps(40):
        for a, b in zip(lam, lam[1:]):
            assert b - a > mp.mpf(10) ** -6
        assert abs(full[0]) < mp.mpf(10) ** -30                   # one zero eigenvalue
        for a, b in zip(full, full[1:]):
            assert b - a > mp.mpf(10) ** -6
    _, C = element.local_matrices(n)
    _, _, Ct, _, _ = element.blocks(C)
    with mp.workdps(40):
        Ctm = element.to_mp(Ct)
        for l in range(n - 1):
            e = [E[i, l] for i in range(n - 1)]
            sign = 1 if (l + 1) % 2 == 1 else -1
            for i in range(n - 1):
                assert abs(e[n - 2 - i] - sign * e[i]) < mp.mpf(10) ** -30
            ev = mp.matrix(e)
            assert abs((ev.T * Ctm * ev)[0] - 1) < mp.mpf(10) ** -30


# --------------------------------------------------------------------------
# 1D spectrum (Theorem 1)
# --------------------------------------------------------------------------

def _exact_pencil_mp(n, K):
    Ag, Cg = assembly.assemble_1d_exact(n, K)
    return element.to_mp(Ag), element.to_mp(Cg)


@pytest.mark.parametrize("n,K", [(2, 3), (2, 4), (3, 4), (4, 3), (1, 5)])
def test_structured_spectrum_equals_bruteforce_mp(n, K):
    # Brute force: full high-precision eigensolve of the exactly assembled pencil.
    with mp.workdps(40):
        A, C = _exact_pencil_mp(n, K)
        want, _ = element.generalized_eigh_mp(A, C)
    data = spectral.eigen_structured(n, K, workers=1)
    got = np.sort(np.concatenate([data["lam0"], data["lam"].ravel()]))
    assert got.size == len(want)
    assert np.allclose(got, [float(w) for w in want], rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,K", [(2, 8), (3, 8), (5, 8), (9, 8), (2, 16), (4, 16), (9, 16)])
def test_structured_spectrum_equals_dense_fp64(n, K):
    lam_d, _ = spectral.eigen_dense(n, K)
    data = spectral.eigen_structured(n, K, workers=1)
    got = np.sort(np.concatenate([data["lam0"], data["lam"].ravel()]))
    assert np.max(np.abs(got - lam_d)) <= 1e-12 * lam_d.max()


def test_n1_closed_form():
    # n = 1: lambda_k = (a0 + theta an) / (c0 + theta cn) = 3 (1 - theta) / (2 (2 + theta)).
    K = 16
    data = spectral.eigen_structured(1, K, workers=1)
    th = np.cos(np.pi * np.arange(1, K) / K)
    assert np.allclose(data["lam"][:, 0], 3 * (1 - th) / (2 * (2 + th)), rtol=1e-14, atol=0)


@pytest.mark.parametrize("n,K", [(2, 64), (3, 64), (4, 128), (9, 64), (9, 1024)])
def test_smallest_eigenvalue_closed_form(n, K):
    # The scaled smallest eigenvalue approximates pi^2 h^2 / 4 = pi^2 / (4 K^2)
    # from above (conforming Galerkin, min-max), with relative error O(h^{2n}).
    data = spectral.eigen_structured(n, K)
    lam1 = data["lam"][0, 0]
    exact = np.pi ** 2 / (4.0 * K ** 2)
    rel = (lam1 - exact) / exact
    assert rel > -4e-15
    assert rel < (np.pi / K) ** (2 * n) + 4e-15


@pytest.mark.parametrize("n,K", [(2, 16), (4, 32), (6, 16), (9, 16), (3, 64)])
def test_basis_invariants(n, K):
    V, lam = spectral.basis(n, K)
    A, C = assembly.assemble_1d(n, K)
    m = assembly.dim(n, K)
    assert np.max(np.abs(V.T @ C @ V - np.eye(m))) < 1e-13
    assert np.max(np.abs(V.T @ A @ V - np.diag(lam))) < 1e-13 * lam.max()


def test_eigenpair_residual_high_precision():
    # (A - lambda C) s = 0 to 30 digits with exactly assembled matrices.
    n, K = 4, 8
    with mp.workdps(40):
        A, C = _exact_pencil_mp(n, K)
        for k in (1, 3, 7):
            _, lams, ps = spectral._wave_k((n, K, k, 40))
            for lam_s, p_s in zip(lams, ps):
                lam = mp.mpf(lam_s)
                p = [mp.mpf(x) for x in p_s]
                s = mp.matrix(n * K - 1, 1)
                for j in range(1, K):
                    s[n * j - 1] = mp.sin(mp.pi * k * j / K)
                for j in range(1, K + 1):
                    for c in range(1, n):
                        s[n * (j - 1) + c - 1] = (p[c - 1] * mp.sin(mp.pi * k * (j - 1) / K)
                                                  + p[n - c - 1] * mp.sin(mp.pi * k * j / K))
                r = (A - lam * C) * s
                assert mp.mnorm(r, 1) < mp.mpf(10) ** -30


@pytest.mark.parametrize("n,K", [(2, 16), (5, 32), (9, 32)])
def test_norm_formula_of_transform_theorem(n, K):
    # ||s_k^(l)||_C^2 = K (b0 + bn theta_k), b0 = c0 + (C~p + 2c).p,
    # bn = cn + (C~p + 2c).Pp (second theorem, item 2); ||s_0^(l)||^2 = K.
    S, lam = spectral.eigenvectors_structured(n, K)
    _, Cs = assembly.assemble_1d_sparse(n, K)
    direct = np.einsum("ij,ij->j", S, Cs @ S)
    _, Cl = assembly.local_float(n)
    c0, cn = Cl[0, 0], Cl[0, n]
    c = Cl[1:n, 0]
    Ct = Cl[1:n, 1:n]
    data = spectral.eigen_structured(n, K)
    assert np.allclose(direct[: n - 1], K, rtol=1e-13)
    for k in range(1, K):
        th = np.cos(np.pi * k / K)
        for l in range(n):
            p = data["p"][k - 1, l]
            w = Ct @ p + 2 * c
            formula = K * (c0 + w @ p + (cn + w @ p[::-1]) * th)
            assert abs(direct[(n - 1) + n * (k - 1) + l] - formula) < 1e-12 * abs(formula)


def test_planted_reflection_mistake_is_caught():
    # Build the k >= 1 eigenvectors with P dropped (p in place of P p): the
    # C-orthogonality invariant must fail, so this pin would catch it.
    n, K = 4, 8
    data = spectral.eigen_structured(n, K, workers=1)
    bad = dict(data)
    S_good, _ = spectral.eigenvectors_structured(n, K, data)
    m = assembly.dim(n, K)
    S_bad = S_good.copy()
    tab = np.sin(np.pi * np.arange(2 * K) / K)
    for k in range(1, K):
        for l in range(n):
            col = (n - 1) + n * (k - 1) + l
            p = bad["p"][k - 1, l]
            for j in range(1, K + 1):
                rows = n * (j - 1) + np.arange(n - 1)
                S_bad[rows, col] = p * tab[(k * (j - 1)) % (2 * K)] + p * tab[(k * j) % (2 * K)]
    A, C = assembly.assemble_1d(n, K)
    def off(S):
        G = S.T @ C @ S
        d = np.sqrt(np.diag(G))
        return np.max(np.abs(G / np.outer(d, d) - np.eye(m)))
    assert off(S_good) < 1e-13
    assert off(S_bad) > 1e-3


# --------------------------------------------------------------------------
# Solve (eq. (bvp glob 2), eq. (decomp v 2))
# --------------------------------------------------------------------------

def _refined_sparse_solve(f, ns, Ks, Xs, alpha):
    L = assembly.operator_sparse(ns, Ks, Xs, alpha).tocsc()
    lu = spla.splu(L)
    x = lu.solve(f.ravel())
    for _ in range(3):   # FP64 difference-form residual (kernel-exact) refinement
        r = f - assembly.apply_operator(x.reshape(f.shape), ns, Ks, Xs, alpha)
        x = x + lu.solve(r.ravel())
    return x.reshape(f.shape)


@pytest.mark.parametrize("ns,Ks,Xs,alpha", [
    ([2, 2], [16, 16], [1.0, 1.0], 0.0),
    ([3, 3], [8, 8], [1.0, 1.0], 1.0),
    ([4, 4], [8, 8], [1.0, 2.0], 0.0),
    ([6, 6], [4, 4], [1.0, 1.0], 0.0),
    ([9, 9], [4, 4], [1.0, 1.0], 0.0),
    ([2, 3], [8, 4], [1.0, 0.5], 3.0),
    ([3, 3, 3], [4, 4, 4], [1.0, 1.0, 1.0], 0.0),
    ([2, 4, 2], [4, 2, 8], [1.0, 2.0, 1.0], -5.0),
    ([5], [16], [1.0], 0.0),
])
def test_solve_matches_refined_sparse_direct(ns, Ks, Xs, alpha):
    rng = np.random.default_rng(0)
    shape = [n * K - 1 for n, K in zip(ns, Ks)]
    f = rng.uniform(-1, 1, shape)
    ref = _refined_sparse_solve(f, ns, Ks, Xs, alpha)
    got = solve.solve(f, ns, Ks, Xs, alpha)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12
    # The residual of the oracle's answer, in the kernel-exact FP64 apply.
    r = f - assembly.apply_operator(got, ns, Ks, Xs, alpha)
    assert np.linalg.norm(r) / np.linalg.norm(f) < 1e-10


def test_solve_1d_matches_banded_cholesky():
    n, K, X = 7, 32, 2.0
    A, C = assembly.assemble_1d(n, K)
    L = (4 * K * K / X ** 2) * A + 0.5 * C
    m = L.shape[0]
    ab = np.zeros((n + 1, m))
    for d in range(n + 1):
        ab[n - d, d:] = np.diagonal(L, d)
    f = np.random.default_rng(1).uniform(-1, 1, m)
    ref = sla.solveh_banded(ab, f)
    got = solve.solve(f, [n], [K], [X], 0.5)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


def test_dense_and_structured_routes_agree_on_solve():
    ns, Ks, Xs = [3, 3], [8, 8], [1.0, 1.0]
    f = np.random.default_rng(2).uniform(-1, 1, (23, 23))
    a = solve.solve(f, ns, Ks, Xs, 0.0, route="structured")
    b = solve.solve(f, ns, Ks, Xs, 0.0, route="dense")
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-12


def _table1():
    rows = {}
    with open(os.path.join(GOLDEN, "table1.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            vals = line.split()
            rows[int(vals[0])] = [float(v) for v in vals[1:]]
    return rows


@pytest.mark.parametrize("kappa,n", [(3, n) for n in range(1, 10)] + [(4, n) for n in range(1, 10)]
                         + [(5, n) for n in range(1, 7)] + [(6, 1), (7, 1)])
def test_table1(kappa, n):
    paper = _table1()[kappa][n - 1]
    K = 2 ** kappa
    f = load.load_separable(load.table1_rhs_terms(), [n, n], [K, K], [1.0, 1.0])
    v = solve.solve(f, [n, n], [K, K], [1.0, 1.0], alpha=1.0)
    u = load.interpolate_separable(load.table1_solution_terms(), [n, n], [K, K], [1.0, 1.0])
    err = np.max(np.abs(v - u))
    if paper > 1e-12:
        # discretisation-dominated entries: two printed digits
        assert abs(err - paper) <= 0.06 * paper + 0.05e-12, (err, paper)
    else:
        # round-off-dominated entries: at or below the paper's floor
        assert err <= max(paper, 1e-14) * 1.5, (err, paper)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_convergence_rate_manufactured_sine(n):
    # Configuration of the small 2D case: u = sin(pi x) sin(2 pi y), f = 5 pi^2 u.
    # The max-norm error over the grid points falls at least like h^(n+1).
    s1 = lambda x: np.sin(np.pi * x)
    s2 = lambda x: np.sin(2 * np.pi * x)
    errs = []
    Ks = [8, 16, 32]
    for K in Ks:
        f = load.load_separable([(5 * np.pi ** 2, [s1, s2])], [n, n], [K, K], [1.0, 1.0])
        v = solve.solve(f, [n, n], [K, K], [1.0, 1.0])
        u = load.interpolate_separable([(1.0, [s1, s2])], [n, n], [K, K], [1.0, 1.0])
        errs.append(np.max(np.abs(v - u)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > n + 1 - 0.1, rates
