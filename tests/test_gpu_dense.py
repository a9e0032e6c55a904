"""GPU parity of axes whose K is not a power of two (dense eigenvector
transforms on the FP64 matrix cores) against the oracle's exact dense solve.

Relative l2 <= 1e-12 in 1D, 2D and 3D, odd and even K, mixed with
power-of-two (FFT) axes and with Neumann and periodic axes, two right-hand
sides; the scaled mass product
against the oracle; the workspace required and the unsupported modes
refused.
"""
import numpy as np
import pytest

import workloads
from oracle import assembly
from oracle import solve as osolve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

H = pytest.importorskip("paper_1609_07758_amd")

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


CASES = [
    # (orders, Ks, X, alpha)
    ((3,), (12,), (1.0,), 0.0),
    ((2,), (3,), (1.0,), 0.5),
    ((1,), (6,), (2.0,), 0.0),
    ((5,), (6,), (1.0,), 1.0),
    ((9,), (96,), (1.0,), 0.0),
    ((2, 3), (6, 10), (1.0, 0.5), 0.0),
    ((9, 4), (4, 12), (1.0, 1.0), 0.0),      # FFT axis 0, dense axis 1
    ((3, 3), (12, 16), (1.0, 1.0), 2.0),     # dense axis 0, FFT axis 1
    ((9, 9), (48, 40), (1.0, 1.0), 0.0),
    ((2, 3, 2), (6, 4, 10), (1.0, 1.0, 1.0), 0.0),
    ((3, 2, 4), (8, 12, 8), (1.0, 2.0, 1.0), 1.0),
]


def solve_gpu(orders, Ks, X, alpha, f, nrhs=1):
    S = H.Solver(orders, Ks, X, alpha)
    try:
        u = S.solve(torch.from_numpy(np.ascontiguousarray(f)).to(DEV).reshape(-1), nrhs=nrhs)
        return u.cpu().numpy().reshape(f.shape)
    finally:
        S.close()


@pytest.mark.parametrize("orders,Ks,X,alpha", CASES)
def test_dense_solve_matches_oracle(orders, Ks, X, alpha):
    shp = workloads.shape(orders, Ks)
    f = workloads.uniform_rhs(shp, seed=11)
    got = solve_gpu(orders, Ks, X, alpha, f)
    assert rel(got, osolve.solve(f, orders, Ks, X, alpha)) < 1e-12


# a dense (K not a power of two) Dirichlet axis beside Neumann and periodic axes
MIXED = [
    ((3, 2), (12, 8), (1.0, 1.0), 1.0, ("dirichlet", "neumann")),
    ((2, 4), (8, 6), (1.0, 0.5), 0.5, ("neumann", "dirichlet")),
    ((2, 3), (10, 8), (1.0, 1.0), 1.0, ("dirichlet", "periodic")),
    ((2, 2, 3), (6, 8, 4), (1.0, 1.0, 1.0), 1.0, ("dirichlet", "neumann", "periodic")),
    ((3,), (12,), (1.0,), 1.0, ("neumann",)),                       # dense Neumann axes
    ((2, 3), (6, 10), (1.0, 1.0), 1.0, ("neumann", "neumann")),
    ((2, 4), (6, 16), (1.0, 1.0), 0.0, ("neumann", "dirichlet")),
    ((5, 2), (16, 12), (2.0, 1.0), 0.5, ("periodic", "neumann")),
    ((2,), (6,), (1.0,), 1.0, ("periodic",)),                        # dense periodic axes
    ((3,), (5,), (1.0,), 0.5, ("periodic",)),                        # odd K
    ((2, 3), (10, 7), (1.0, 1.0), 0.0, ("periodic", "dirichlet")),
    ((4, 2), (12, 6), (1.0, 1.0), 1.0, ("periodic", "neumann")),
]


@pytest.mark.parametrize("orders,Ks,X,alpha,bcs", MIXED)
def test_dense_axis_with_neumann_and_periodic_axes(orders, Ks, X, alpha, bcs):
    from oracle import periodic
    shp = tuple(periodic.axis_dim(n, K, b) for n, K, b in zip(orders, Ks, bcs))
    f = workloads.uniform_rhs(shp, seed=15)
    S = H.Solver(orders, Ks, X, alpha, bcs=bcs)
    try:
        u = S.solve(torch.from_numpy(f).to(DEV).reshape(-1)).cpu().numpy().reshape(shp)
    finally:
        S.close()
    assert rel(u, periodic.solve(f, orders, Ks, X, alpha, bcs)) < 1e-12


def test_dense_two_rhs():
    orders, Ks, X, alpha = (2, 3), (6, 10), (1.0, 1.0), 0.0
    shp = workloads.shape(orders, Ks)
    f = np.stack([workloads.uniform_rhs(shp, seed=12 + r) for r in range(2)])
    got = solve_gpu(orders, Ks, X, alpha, f, nrhs=2)
    for r in range(2):
        assert rel(got[r], osolve.solve(f[r], orders, Ks, X, alpha)) < 1e-12


def test_dense_refusals_and_mass():
    orders, Ks = (3, 2), (12, 6)
    S = H.Solver(orders, Ks, (1.0, 1.0), 1.0)
    try:
        g = workloads.uniform_rhs(S.shape, seed=13)
        gd = torch.from_numpy(g).to(DEV)
        u = torch.empty_like(gd)
        with pytest.raises(H.HofemError) as e:   # one grid of workspace is required
            H.hofem_solve(S.handle, "fp64", gd, u, 1, None, 0, 0.0, None, False, True)
        assert e.value.status == -1
        for mode in ("fp32_ir", "fp64_b"):
            with pytest.raises(H.HofemError) as e:
                S.solve(gd, mode=mode)
            assert e.value.status == -2
        got = S.apply_mass(gd).cpu().numpy()
    finally:
        S.close()
    assert rel(got, assembly.apply_mass(g, orders, Ks)) < 1e-14


@pytest.mark.slow
def test_dense_large_2d():
    # n = 9, K = 384 per axis: 3455 x 3455 unknowns, four 3455^3 products
    orders, Ks, X, alpha = (9, 9), (384, 384), (1.0, 1.0), 0.0
    shp = workloads.shape(orders, Ks)
    f = workloads.uniform_rhs(shp, seed=14)
    got = solve_gpu(orders, Ks, X, alpha, f)
    e = rel(got, osolve.solve(f, orders, Ks, X, alpha))
    print(f"dense large 2D: rel l2 {e:.3e}")
    assert e < 1e-12
