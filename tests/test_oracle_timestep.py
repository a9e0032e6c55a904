"""Pins of the oracle's implicit time stepping (CPU).

A discrete eigenvector v of the 2D FEM pencil (from a dense FP64
generalized eigensolve of the assembled 1D matrices, scipy's eigh, not the
oracle's structured route), with L_0 v = mu (x)C v, is multiplied by
r = alpha / (alpha + mu) per backward Euler step and follows the scalar
recurrence c_{n+1} = r (2 c_n - c_{n-1}) under the wave scheme; with a
steady load the heat iteration converges to the stationary solve."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assembly, solve as osolve, timestep


def eigvec_2d(n, K, i, j):
    A, C = assembly.assemble_1d(n, K)
    lam, V = sla.eigh(A, C)            # scaled 1D eigenvalues, C-orthonormal columns
    s = 4.0 * K * K                    # 4 h^-2 on the unit interval
    mu = s * (lam[i] + lam[j])
    return np.outer(V[:, i], V[:, j]), mu


@pytest.mark.parametrize("n,K,i,j", [(2, 8, 0, 0), (3, 4, 2, 5), (4, 4, 7, 1)])
def test_heat_eigenvector_decays_by_closed_factor(n, K, i, j):
    v, mu = eigvec_2d(n, K, i, j)
    alpha = 37.0                       # dt = 1/37
    u, _ = timestep.steps(v, None, [n, n], [K, K], [1.0, 1.0], alpha, timestep.HEAT, 5)
    want = (alpha / (alpha + mu)) ** 5 * v
    assert np.linalg.norm(u - want) <= 1e-12 * np.linalg.norm(v) * max(1.0, (alpha / (alpha + mu)) ** 5)


@pytest.mark.parametrize("n,K,i,j", [(2, 8, 1, 0), (3, 4, 0, 3)])
def test_wave_eigenvector_follows_scalar_recurrence(n, K, i, j):
    v, mu = eigvec_2d(n, K, i, j)
    alpha = 400.0                      # dt = 1/20
    r = alpha / (alpha + mu)
    c = [0.7, 1.0]                     # c_{-1}, c_0
    for _ in range(6):
        c.append(r * (2 * c[-1] - c[-2]))
    u, up = timestep.steps(v, None, [n, n], [K, K], [1.0, 1.0], alpha, timestep.WAVE, 6,
                           uprev=0.7 * v)
    assert np.linalg.norm(u - c[-1] * v) < 1e-12 * np.linalg.norm(v)
    assert np.linalg.norm(up - c[-2] * v) < 1e-12 * np.linalg.norm(v)


def test_heat_reaches_the_stationary_solution():
    ns, Ks, Xs = [3, 2], [4, 8], [1.0, 1.0]
    f = np.random.default_rng(0).uniform(-1, 1, (11, 15))
    u, _ = timestep.steps(np.zeros_like(f), f, ns, Ks, Xs, 1.0, timestep.HEAT, 40)
    want = osolve.solve(f, ns, Ks, Xs, 0.0)
    assert np.linalg.norm(u - want) / np.linalg.norm(want) < 1e-12
