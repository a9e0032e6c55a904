"""Pins of the oracle's variable-coefficient operator (CPU only).

Each pin checks the oracle against something other than itself:
* a = 1 reproduces the exactly integrated operator of eq. (bvp glob 2);
* the energy u^T L_a u equals the closed-form integral of a |grad u|^2 +
  alpha u^2 (rational arithmetic) for polynomial u and a for which the Gauss
  rule is exact, with an asymmetric a so that a swapped axis fails;
* the matrix-free apply equals the assembled matrix;
* the discrete solution of -div(a grad u) + alpha u = f converges to the
  manufactured u at the order of the element (sign, coefficient placement
  and load all enter).
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import assembly, varcoef


# -- exact polynomial integration over a box ---------------------------------

def p_mul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return out


def p_add(p, q):
    out = dict(p)
    for e, c in q.items():
        out[e] = out.get(e, 0) + c
    return out


def p_der(p, i):
    out = {}
    for e, c in p.items():
        if e[i] > 0:
            e2 = list(e)
            e2[i] -= 1
            out[tuple(e2)] = out.get(tuple(e2), 0) + c * e[i]
    return out


def p_int_box(p, Xs):
    tot = Fraction(0)
    for e, c in p.items():
        t = Fraction(c)
        for k, X in zip(e, Xs):
            t *= Fraction(X) ** (k + 1) / (k + 1)
        tot += t
    return tot


def p_eval(p, xs):
    tot = 0.0
    for e, c in p.items():
        t = float(c)
        for k, x in zip(e, xs):
            t = t * x ** k
        tot = tot + t
    return tot


def var(i, N, c=1):
    e = [0] * N
    e[i] = 1
    return {tuple(e): Fraction(c)}


def const(N, c):
    return {tuple([0] * N): Fraction(c)}


def energy_case(N):
    """u, a as exact polynomials on the box, orders and meshes."""
    if N == 2:
        Xs = (Fraction(1), Fraction(2))
        ns, Ks = (2, 3), (3, 4)
        x, y = var(0, 2), var(1, 2)
        u = p_mul(p_mul(x, p_add(const(2, Xs[0]), var(0, 2, -1))),
                  p_mul(p_mul(y, p_add(const(2, Xs[1]), var(1, 2, -1))),
                        p_add(const(2, Fraction(1, 2)), y)))
        a = p_add(p_add(const(2, 1), x), var(1, 2, 2))
    else:
        Xs = (Fraction(1), Fraction(3, 2), Fraction(1))
        ns, Ks = (2, 2, 3), (2, 3, 2)
        x, y, z = var(0, 3), var(1, 3), var(2, 3)
        u = p_mul(p_mul(x, p_add(const(3, Xs[0]), var(0, 3, -1))),
                  p_mul(p_mul(y, p_add(const(3, Xs[1]), var(1, 3, -1))),
                        p_mul(z, p_mul(p_add(const(3, Xs[2]), var(2, 3, -1)),
                                       p_add(const(3, 1), z)))))
        a = p_add(p_add(p_add(const(3, 2), x), var(1, 3, 2)), var(2, 3, Fraction(-1, 2)))
    return Xs, ns, Ks, u, a


@pytest.mark.parametrize("N", [2, 3])
def test_energy_closed_form(N):
    Xs, ns, Ks, u, a = energy_case(N)
    alpha = 0.75
    # exact: int a |grad u|^2 + alpha u^2 over the box
    integrand = p_mul(const(N, Fraction(3, 4)), p_mul(u, u))
    for i in range(N):
        du = p_der(u, i)
        integrand = p_add(integrand, p_mul(a, p_mul(du, du)))
    exact = float(p_int_box(integrand, Xs))
    Xf = [float(X) for X in Xs]
    a_full = varcoef.gauss_values(lambda *c: p_eval(a, c), ns, Ks, Xf)
    grids = np.meshgrid(*[np.arange(1, n * K) * (X / (n * K)) for n, K, X in zip(ns, Ks, Xf)],
                        indexing="ij")
    uh = p_eval(u, grids)
    L = varcoef.operator_sparse(ns, Ks, Xf, alpha, a_full)
    scale = np.prod([X / K / 2.0 for X, K in zip(Xf, Ks)])
    got = float(uh.ravel() @ (L @ uh.ravel())) * scale
    assert abs(got - exact) <= 1e-12 * abs(exact)
    # and the matrix-free apply gives the same energy
    got2 = float(np.sum(uh * varcoef.apply(uh, ns, Ks, Xf, alpha, a_full))) * scale
    assert abs(got2 - exact) <= 1e-12 * abs(exact)


@pytest.mark.parametrize("ns,Ks,Xs,alpha", [
    ((3,), (5,), (1.0,), 0.3),
    ((2, 3), (3, 4), (1.0, 2.0), 0.7),
    ((2, 2, 3), (2, 3, 2), (1.0, 1.5, 0.5), 0.0),
])
def test_unit_coefficient_is_constant_operator(ns, Ks, Xs, alpha):
    nel = int(np.prod(Ks))
    npts = int(np.prod([n + 1 for n in ns]))
    L1 = varcoef.operator_sparse(ns, Ks, Xs, alpha, np.ones((nel, npts)))
    L0 = assembly.operator_sparse(ns, Ks, Xs, alpha)
    d = abs(L1 - L0).max()
    assert d <= 1e-12 * abs(L0).max()
    # a = c scales the stiffness part only
    c = 2.5
    Lc = varcoef.operator_sparse(ns, Ks, Xs, alpha, np.full((nel, npts), c))
    Ls = assembly.operator_sparse(ns, Ks, Xs, 0.0)
    ref = c * Ls + (L0 - Ls)
    assert abs(Lc - ref).max() <= 1e-12 * abs(ref).max()


@pytest.mark.parametrize("ns,Ks,Xs,alpha", [
    ((3, 2), (3, 4), (1.0, 0.5), 0.2),
    ((2, 3, 2), (2, 2, 3), (1.0, 1.0, 2.0), 0.0),
    ((4,), (6,), (2.0,), 1.5),
])
def test_apply_matches_assembled(ns, Ks, Xs, alpha):
    rng = np.random.default_rng(3)
    nel = int(np.prod(Ks))
    npts = int(np.prod([n + 1 for n in ns]))
    a_full = 0.5 + rng.random((nel, npts))
    grid = tuple(n * K - 1 for n, K in zip(ns, Ks))
    u = rng.uniform(-1, 1, (2,) + grid)
    L = varcoef.operator_sparse(ns, Ks, Xs, alpha, a_full)
    got = varcoef.apply(u, ns, Ks, Xs, alpha, a_full)
    for r in range(2):
        ref = (L @ u[r].ravel()).reshape(grid)
        assert np.max(np.abs(got[r] - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_expand_separable_layout():
    ns, Ks, Xs = (2, 3), (3, 2), (1.0, 2.0)
    t0 = lambda x: np.sin(2 * np.pi * x) + 0.1 * x
    t1 = lambda y: np.cos(np.pi * y) - y
    tabs = [t0(varcoef.gauss_points(ns[0], Ks[0], Xs[0])),
            t1(varcoef.gauss_points(ns[1], Ks[1], Xs[1]))]
    got = varcoef.expand_separable(1.0, 0.5, tabs)
    ref = varcoef.gauss_values(lambda x, y: 1.0 + 0.5 * t0(x) * t1(y), ns, Ks, Xs)
    assert np.array_equal(got, ref)


def _manufactured(n, K, alpha):
    """-div(a grad u) + alpha u = f on [0,1]^2, a = 1 + 0.5 sin(2 pi x) sin(2 pi y),
    u = sin(pi x) sin(pi y); returns the max nodal error of the FEM solution."""
    pi = np.pi
    s, c = np.sin, np.cos
    a = lambda x, y: 1.0 + 0.5 * s(2 * pi * x) * s(2 * pi * y)
    ax = lambda x, y: pi * c(2 * pi * x) * s(2 * pi * y)
    ay = lambda x, y: pi * s(2 * pi * x) * c(2 * pi * y)
    u = lambda x, y: s(pi * x) * s(pi * y)
    ux = lambda x, y: pi * c(pi * x) * s(pi * y)
    uy = lambda x, y: pi * s(pi * x) * c(pi * y)
    f = lambda x, y: (a(x, y) * 2 * pi ** 2 * u(x, y) - ax(x, y) * ux(x, y)
                      - ay(x, y) * uy(x, y) + alpha * u(x, y))
    ns, Ks, Xs = (n, n), (K, K), (1.0, 1.0)
    a_full = varcoef.gauss_values(a, ns, Ks, Xs)
    fh = varcoef.load(varcoef.gauss_values(f, ns, Ks, Xs), ns, Ks)
    uh = varcoef.solve(fh, ns, Ks, Xs, alpha, a_full)
    g = np.arange(1, n * K) / (n * K)
    X, Y = np.meshgrid(g, g, indexing="ij")
    return np.max(np.abs(uh - u(X, Y)))


@pytest.mark.parametrize("n,Ks", [(2, (4, 8, 16)), (3, (4, 8))])
def test_manufactured_convergence(n, Ks):
    errs = [_manufactured(n, K, 0.5) for K in Ks]
    for e0, e1 in zip(errs, errs[1:]):
        assert e0 / e1 > 0.75 * 2 ** (n + 1)
    assert errs[-1] < 1e-3 * 4.0 ** -(n - 2)


def test_load_of_polynomial_is_exact():
    # int f phi for f = x^2 y (degree within the rule): compare with the
    # separable 1D loads of the constant-coefficient oracle.
    from oracle import load
    ns, Ks, Xs = (2, 3), (3, 2), (1.0, 2.0)
    fv = varcoef.gauss_values(lambda x, y: x ** 2 * y, ns, Ks, Xs)
    got = varcoef.load(fv, ns, Ks)
    ref = load.load_separable([(1.0, [lambda x: x ** 2, lambda y: y])], ns, Ks, Xs)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("N,n,K", [(2, 3, 4), (3, 2, 4)])
def test_oracle_pcg_matches_sparse_direct(N, n, K):
    # CG preconditioned by the constant-coefficient solve converges to the
    # sparse direct solution; with 0.5 <= a <= 1.5 the preconditioned
    # operator has condition number <= 3, so the CG bound gives at most
    # about 22 iterations to 1e-10 (energy norm)
    from oracle import pcg
    ns, Ks, Xs = [n] * N, [K] * N, [1.0] * N
    rng = np.random.default_rng(3)
    a = rng.uniform(0.5, 1.5, (K ** N, (n + 1) ** N))
    f = rng.uniform(-1, 1, tuple(n * K - 1 for _ in range(N)))
    u, it, res = pcg.pcg(f, ns, Ks, Xs, 0.0, a, rtol=1e-10)
    want = varcoef.solve(f, ns, Ks, Xs, 0.0, a)
    assert res <= 1e-10 and 1 <= it <= 22
    assert np.linalg.norm(u - want) / np.linalg.norm(want) < 1e-9
    # a = 1: the preconditioner is exact, the start is the solution
    u1, it1, _ = pcg.pcg(f, ns, Ks, Xs, 0.0, np.ones_like(a), rtol=1e-10)
    assert it1 == 0
