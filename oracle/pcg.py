"""Preconditioned conjugate gradients for -div(a grad u) + alpha u = f
(oracle; test infrastructure only, never called by the library's product
path).

The paper proposes the fast solver as a preconditioner for more general
elliptic problems (Section 1).  Plain CG on the FP64 matrix-free operator of
``varcoef.apply`` (Gauss quadrature of the variable coefficient), each step
preconditioned by the exact constant-coefficient solve of ``solve`` (the
operator with a = 1).  The start is the preconditioned right-hand side, as in
the library.  Stops when ||f - L_a u||_2 <= rtol ||f||_2.
"""
import numpy as np

from . import solve as osolve, varcoef


def pcg(f, ns, Ks, Xs, alpha, a_full, rtol=1e-10, max_iter=200):
    """Returns (u, iterations, relative residual)."""
    f = np.asarray(f, dtype=np.float64)
    L = lambda v: varcoef.apply(v, ns, Ks, Xs, alpha, a_full)
    P = lambda v: osolve.solve(v, ns, Ks, Xs, alpha)
    nf = np.linalg.norm(f)
    u = P(f)
    r = f - L(u)
    it = 0
    res = np.linalg.norm(r) / nf
    if res <= rtol:
        return u, it, res
    z = P(r)
    p = z.copy()
    rz = float(np.vdot(r, z))
    while it < max_iter:
        q = L(p)
        step = rz / float(np.vdot(p, q))
        u = u + step * p
        r = r - step * q
        it += 1
        res = np.linalg.norm(r) / nf
        if res <= rtol:
            break
        z = P(r)
        rz_new = float(np.vdot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return u, it, res
