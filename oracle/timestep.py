"""Implicit time stepping with the FEM solve (oracle; test infrastructure
only, never called by the library's product path).

The paper proposes the fast solver for implicit methods for time-dependent
problems (Section 1).  Two schemes, each step one system of eq. (bvp glob 2)
whose alpha carries the time step:

  heat, u_t - Lap u = f, backward Euler, alpha = 1/dt:
      L u^{n+1} = f^h + alpha ((x)_i C_i) u^n
  wave, u_tt - Lap u = f, implicit three-level scheme, alpha = 1/dt^2:
      L u^{n+1} = f^h + alpha ((x)_i C_i) (2 u^n - u^{n-1})

Each step is written out as stated: the mass product by ``apply_mass`` and
the dense separable solve of ``solve``.
"""
import numpy as np

from . import assembly, solve as osolve

HEAT, WAVE = 0, 1


def steps(u0, f, ns, Ks, Xs, alpha, scheme, nsteps, uprev=None):
    """Returns (u^N, u^{N-1}) after nsteps steps from u^0 = u0 (and u^{-1} = uprev
    for the wave scheme); f may be None (zero load)."""
    u = np.array(u0, dtype=np.float64)
    up = None if uprev is None else np.array(uprev, dtype=np.float64)
    for _ in range(nsteps):
        w = u if scheme == HEAT else 2.0 * u - up
        rhs = alpha * assembly.apply_mass(w, ns, Ks)
        if f is not None:
            rhs = rhs + f
        new = osolve.solve(rhs, ns, Ks, Xs, alpha)
        up, u = u, new
    return u, up
