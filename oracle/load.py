"""Right-hand sides and grid coordinates (oracle).

f^h in eq. (bvp glob 2) is the FEM average of f: the load vector
int f phi_q dx divided by prod_i (h_i / 2), so that f^h = (x)C_i g when f is
the FEM interpolant of nodal values g.  The paper computes it with the
(n+1)-point Gauss rule in every variable (Section 2, paragraph 5); so does
this module, per element, for separable factors g(x_i).  Sums of separable
terms give sums of outer products of 1D load vectors.
"""
import numpy as np

from .element import lagrange_basis


def grid(n, K, X):
    """Coordinates of the nK-1 interior points q*h/n, q = 1..nK-1 (h = X/K)."""
    return np.arange(1, n * K) * (X / (n * K))


def _basis_values(n, xi):
    """e_r(xi) for r = 0..n at the points xi (FP64, from exact coefficients)."""
    out = np.zeros((n + 1, xi.size))
    for r, coeffs in enumerate(lagrange_basis(n)):
        c = np.array([float(x) for x in coeffs])
        out[r] = np.polynomial.polynomial.polyval(xi, c)
    return out


def load_1d(g, n, K, X, npts=None):
    """1D scaled load vector: sum over elements of int g e_r dxi (reference
    variable), by ``npts``-point Gauss-Legendre (default n+1) per element.

    Equals (int_0^X g phi_q dx) / (h/2) for every interior point q.
    """
    npts = n + 1 if npts is None else npts
    xi, w = np.polynomial.legendre.leggauss(npts)
    h = X / K
    E = _basis_values(n, xi)                      # (n+1, npts)
    b = np.zeros(n * K + 1)
    for j in range(1, K + 1):
        x = (j - 1) * h + (xi + 1.0) * (h / 2.0)
        gv = g(x)
        b[n * (j - 1): n * j + 1] += E @ (w * gv)
    return b[1:-1]


def load_separable(terms, ns, Ks, Xs, npts=None):
    """f^h for f = sum_t coef_t prod_i g_{t,i}(x_i).

    terms: list of (coef, [g_0, ..., g_{N-1}]) with callables g_{t,i}.
    """
    out = None
    for coef, gs in terms:
        vecs = [load_1d(gs[i], ns[i], Ks[i], Xs[i], npts) for i in range(len(ns))]
        t = vecs[0]
        for v in vecs[1:]:
            t = np.multiply.outer(t, v)
        t = coef * t
        out = t if out is None else out + t
    return out


def interpolate_separable(terms, ns, Ks, Xs):
    """Nodal values of f = sum_t coef_t prod_i g_{t,i}(x_i) on the grid."""
    out = None
    for coef, gs in terms:
        vecs = [gs[i](grid(ns[i], Ks[i], Xs[i])) for i in range(len(ns))]
        t = vecs[0]
        for v in vecs[1:]:
            t = np.multiply.outer(t, v)
        t = coef * t
        out = t if out is None else out + t
    return out


# The experiment of Section 2, paragraph 5 (Table 1): N = 2, alpha = 1,
# X = 1, exact solution u = sin(pi x1) sin(pi x2) (x1 + x2 - 1).  Then
# f = -Lap u + u = (2 pi^2 + 1) u - 2 pi (cos(pi x1) sin(pi x2) + sin(pi x1) cos(pi x2)).
def table1_solution_terms():
    s = lambda x: np.sin(np.pi * x)
    xs = lambda x: x * np.sin(np.pi * x)
    return [(1.0, [xs, s]), (1.0, [s, xs]), (-1.0, [s, s])]


def table1_rhs_terms():
    s = lambda x: np.sin(np.pi * x)
    c = lambda x: np.cos(np.pi * x)
    xs = lambda x: x * np.sin(np.pi * x)
    k = 2.0 * np.pi ** 2 + 1.0
    return [(k, [xs, s]), (k, [s, xs]), (-k, [s, s]),
            (-2.0 * np.pi, [c, s]), (-2.0 * np.pi, [s, c])]
