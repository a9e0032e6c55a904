"""Pins of the oracle's non-homogeneous Dirichlet lift (CPU).

A tensor product of polynomials of degree <= n per variable lies in the FEM
space, and its (n+1)-point Gauss load vector is exact, so the FEM solution
with its boundary values reproduces it at every grid point up to rounding:
a check that does not depend on the lift's own formula."""
import numpy as np
import pytest

from oracle import dirichlet, load, solve as osolve


def poly(coeffs):
    P = np.polynomial.Polynomial(coeffs)
    return P, P.deriv(2)


def ext_grid(n, K, X):
    return np.arange(0, n * K + 1) * (X / (n * K))


@pytest.mark.parametrize("ns,Ks,Xs,alpha", [
    ([2, 3], [4, 8], [1.0, 0.5], 0.0),
    ([4, 4], [8, 4], [1.0, 1.0], 2.0),
    ([9], [8], [2.0], 0.0),
    ([2, 2, 3], [4, 4, 2], [1.0, 1.0, 1.0], 1.0),
])
def test_polynomial_with_boundary_values_is_reproduced(ns, Ks, Xs, alpha):
    rng = np.random.default_rng(5)
    facs = [poly(rng.uniform(-1, 1, n + 1)) for n in ns]   # degree n, nonzero at both ends
    N = len(ns)
    # f = -Lap u + alpha u for u = prod_i p_i(x_i)
    terms = []
    for i in range(N):
        terms.append((-1.0, [facs[j][1] if j == i else facs[j][0] for j in range(N)]))
    if alpha:
        terms.append((alpha, [facs[j][0] for j in range(N)]))
    f = load.load_separable(terms, ns, Ks, Xs)
    # boundary values on the extended grid
    u_ext = facs[0][0](ext_grid(ns[0], Ks[0], Xs[0]))
    for i in range(1, N):
        u_ext = np.multiply.outer(u_ext, facs[i][0](ext_grid(ns[i], Ks[i], Xs[i])))
    rhs = dirichlet.lift_rhs(u_ext, f, ns, Ks, Xs, alpha)
    u0 = osolve.solve(rhs, ns, Ks, Xs, alpha)
    want = u_ext[tuple(slice(1, -1) for _ in range(N))]
    assert np.max(np.abs(u0 - want)) < 1e-11 * np.max(np.abs(want))


def test_zero_boundary_values_leave_f():
    f = np.random.default_rng(1).uniform(-1, 1, (7, 15))
    b = np.zeros((9, 17))
    b[3:5, 4:9] = 5.0                   # interior entries are ignored
    assert np.array_equal(dirichlet.lift_rhs(b, f, [2, 4], [4, 4], [1.0, 1.0], 1.5), f)
