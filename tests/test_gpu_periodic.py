"""GPU parity of periodic axes (Bloch-wave line passes, FP64) and Neumann
axes (cosine transforms with band-edge blocks, FP64) against the oracle.

Small grids: the sparse direct solve of the assembled operator
(oracle.periodic), relative l2 <= 1e-12, in 1D, 2D and 3D with every mix of
periodic and Dirichlet axes, several right-hand sides, K = 2 up to 1024.
Full size (n = 9, K = 1024 on both axes of the 2D box): a right-hand side odd
about x = 0 and y = 0 restricts to the Dirichlet problem on half the box,
which the Dirichlet oracle solves exactly (relative l2 <= 1e-12, the even
part zero); and for a generic right-hand side the normwise backward error
||f - L u|| / (||L||_inf ||u|| + ||f||) stays below 1e-15.  The oracle's exact
solution rounded to FP64 scores about 3e-18 by this measure at n = 9, K = 32,
a relative perturbation of 1e-12 about 8e-14.
"""
import numpy as np
import pytest

import workloads
from oracle import periodic
from oracle import solve as osolve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

H = pytest.importorskip("paper_1609_07758_amd")

DEV = "cuda:0"
P, D, NM = "periodic", "dirichlet", "neumann"


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def grid(ns, Ks, bcs):
    return tuple(periodic.axis_dim(n, K, b) for n, K, b in zip(ns, Ks, bcs))


CASES = [
    # (orders, Ks, X, alpha, bcs)
    ((1,), (2,), (1.0,), 0.5, (P,)),
    ((1,), (8,), (1.0,), 2.0, (P,)),
    ((2,), (4,), (1.0,), 0.5, (P,)),
    ((3,), (16,), (2.0,), 1.0, (P,)),
    ((5,), (64,), (1.0,), 3.0, (P,)),
    ((4,), (2,), (1.0,), 0.25, (P,)),
    ((9,), (1024,), (1.0,), 1.0, (P,)),
    ((8,), (128,), (1.0,), 0.01, (P,)),
    ((3, 2), (16, 8), (1.0, 1.0), 1.0, (P, P)),
    ((2, 3), (16, 8), (1.0, 0.5), 0.0, (P, D)),
    ((4, 2), (8, 32), (1.0, 1.0), 0.0, (D, P)),
    ((9, 9), (32, 16), (1.0, 1.0), 0.5, (P, P)),
    ((7, 6), (4, 2), (1.0, 1.0), 0.0, (D, P)),
    ((1, 5), (64, 4), (2.0, 1.0), -1.0, (D, P)),
    ((2, 3, 2), (8, 4, 8), (1.0, 1.0, 1.0), 0.0, (P, D, P)),
    ((3, 3, 3), (8, 8, 4), (1.0, 1.0, 1.0), 1.0, (P, P, P)),
    ((2, 2, 4), (4, 8, 4), (1.0, 2.0, 1.0), 0.0, (D, D, P)),
    ((4, 2, 2), (4, 4, 16), (1.0, 1.0, 1.0), 0.0, (P, D, D)),
]


@pytest.mark.parametrize("orders,Ks,X,alpha,bcs", CASES)
def test_periodic_solve_matches_oracle(orders, Ks, X, alpha, bcs):
    shp = grid(orders, Ks, bcs)
    f = workloads.uniform_rhs(shp, seed=1)
    S = H.Solver(orders, Ks, X, alpha, bcs=bcs)
    try:
        assert S.shape == shp
        u = S.solve(torch.from_numpy(f).to(DEV)).cpu().numpy()
    finally:
        S.close()
    want = periodic.solve(f, orders, Ks, X, alpha, bcs)
    assert rel(u, want) < 1e-12


def test_periodic_several_rhs():
    orders, Ks, X, alpha, bcs = (3, 2), (8, 16), (1.0, 1.0), 0.0, (D, P)
    shp = grid(orders, Ks, bcs)
    f = workloads.uniform_rhs((3,) + shp, seed=2)
    S = H.Solver(orders, Ks, X, alpha, bcs=bcs)
    try:
        u = S.solve(torch.from_numpy(f).to(DEV).reshape(-1), nrhs=3).cpu().numpy().reshape(f.shape)
    finally:
        S.close()
    for r in range(3):
        assert rel(u[r], periodic.solve(f[r], orders, Ks, X, alpha, bcs)) < 1e-12


def test_periodic_forward_inverse_invert_the_mass():
    # V V^T = C^-1 along every axis: inverse(forward(C u)) = u
    orders, Ks, bcs = (3, 4), (8, 4), (P, P)
    shp = grid(orders, Ks, bcs)
    u0 = workloads.uniform_rhs(shp, seed=6)
    Cs = [periodic.axis_matrices(n, K, b)[1] for n, K, b in zip(orders, Ks, bcs)]
    f = (Cs[0] @ (Cs[1] @ u0.T).T)
    S = H.Solver(orders, Ks, (1.0, 1.0), 1.0, bcs=bcs)
    try:
        fd = torch.from_numpy(np.ascontiguousarray(f)).to(DEV)
        c = torch.empty_like(fd)
        u = torch.empty_like(fd)
        H.hofem_forward(S.handle, "fp64", fd, c)
        H.hofem_inverse(S.handle, "fp64", c, u)
        got = u.cpu().numpy()
    finally:
        S.close()
    assert rel(got, u0) < 1e-12


def test_periodic_unsupported_paths():
    S = H.Solver((2, 2), (8, 8), (1.0, 1.0), 1.0, bcs=(P, D))
    try:
        f = torch.zeros(S.size, dtype=torch.float64, device=DEV)
        for mode in ("fp32_ir", "fp64_b", "fp32_pcg"):
            with pytest.raises(H.HofemError) as e:
                S.solve(f, mode=mode)
            assert e.value.status == -2
        with pytest.raises(H.HofemError) as e:   # the Dirichlet lift
            H.hofem_dirichlet_rhs(S.handle, torch.zeros(10 * 18, dtype=torch.float64, device=DEV), None,
                                  f, 1, None)
        assert e.value.status == -2
    finally:
        S.close()
    with pytest.raises(H.HofemError) as e:
        H.Solver((2,), (8,), (1.0,), 0.0, bcs=(P,))
    assert e.value.status == -3


def odd_extension(fd, n, K, axis):
    fd = np.moveaxis(np.asarray(fd), axis, 0)
    m = n * K - 1
    out = np.zeros((2 * n * K,) + fd.shape[1:])
    out[1:m + 1] = fd
    out[m + 2:] = -fd[::-1]
    return np.moveaxis(out, 0, axis)


@pytest.mark.slow
def test_periodic_full_size_odd_extension():
    # n = 9, K = 1024 on both periodic axes of [0, 2)^2, alpha = 1: an odd
    # right-hand side solves the Dirichlet problem of n = 9, K = 512 on [0, 1]^2
    n, Kd = 9, 512
    fd = workloads.uniform_rhs((n * Kd - 1, n * Kd - 1), seed=7)
    fp = np.ascontiguousarray(odd_extension(odd_extension(fd, n, Kd, 0), n, Kd, 1))
    S = H.Solver((n, n), (2 * Kd, 2 * Kd), (2.0, 2.0), 1.0, bcs=(P, P))
    try:
        u = S.solve(torch.from_numpy(fp).to(DEV)).cpu().numpy()
    finally:
        S.close()
    want = osolve.solve(fd, (n, n), (Kd, Kd), (1.0, 1.0), 1.0)
    m = n * Kd - 1
    inner = u[1:m + 1, 1:m + 1]
    e = rel(inner, want)
    print(f"odd extension, full size: rel l2 {e:.3e}")
    assert e < 1e-12
    scale = np.max(np.abs(want))
    assert np.max(np.abs(u[0])) < 1e-12 * scale and np.max(np.abs(u[:, 0])) < 1e-12 * scale
    assert np.max(np.abs(u[m + 1])) < 1e-12 * scale
    assert rel(u[m + 2:, m + 2:], want[::-1, ::-1]) < 1e-12


@pytest.mark.slow
def test_periodic_full_size_backward_error():
    orders, Ks, X, alpha, bcs = (9, 9), (1024, 1024), (1.0, 1.0), 1.0, (P, P)
    shp = grid(orders, Ks, bcs)
    f = workloads.uniform_rhs(shp, seed=8)
    S = H.Solver(orders, Ks, X, alpha, bcs=bcs)
    try:
        u = S.solve(torch.from_numpy(f).to(DEV)).cpu().numpy()
    finally:
        S.close()
    r = f - periodic.apply_operator(u, orders, Ks, X, alpha, bcs)
    mats = [periodic.axis_matrices(n, K, b) for n, K, b in zip(orders, Ks, bcs)]
    inf = lambda M: float(abs(M).sum(axis=1).max())
    s = [4.0 * K ** 2 / x ** 2 for K, x in zip(Ks, X)]
    Linf = (s[0] * inf(mats[0][0]) * inf(mats[1][1]) + s[1] * inf(mats[0][1]) * inf(mats[1][0])
            + alpha * inf(mats[0][1]) * inf(mats[1][1]))
    eta = np.linalg.norm(r) / (Linf * np.linalg.norm(u) + np.linalg.norm(f))
    print(f"backward error, full size: {eta:.3e}")
    assert eta < 1e-15


# Neumann axes (direct cosine passes: every order, K = 2 up to 1024, mixed
# with Dirichlet and periodic axes)
NEUMANN = [
    ((1,), (4,), (1.0,), 0.5, (NM,)),
    ((2,), (8,), (1.0,), 2.0, (NM,)),
    ((3,), (16,), (2.0,), 1.0, (NM,)),
    ((9,), (512,), (1.0,), 1.0, (NM,)),
    ((9,), (1024,), (1.0,), 1.0, (NM,)),
    ((8,), (1024,), (1.0,), 0.5, (NM,)),
    ((6,), (32,), (1.0,), 1.0, (NM,)),
    ((7,), (64,), (3.0,), 1.0, (NM,)),
    ((5,), (2,), (1.0,), 0.25, (NM,)),
    ((1,), (2,), (1.0,), 1.0, (NM,)),
    ((4, 9), (8, 1024), (1.0, 1.0), 0.0, (D, NM)),
    ((9, 2), (256, 16), (1.0, 1.0), 0.0, (NM, D)),
    ((3, 2), (8, 16), (1.0, 1.0), 0.0, (NM, D)),
    ((2, 4), (16, 8), (1.0, 0.5), 0.0, (D, NM)),
    ((4, 3), (8, 8), (1.0, 1.0), 1.0, (NM, NM)),
    ((2, 3), (16, 8), (1.0, 1.0), 0.5, (NM, P)),
    ((2, 3, 2), (8, 4, 8), (1.0, 1.0, 1.0), 0.0, (NM, D, P)),
    ((3, 2, 2), (4, 8, 4), (1.0, 1.0, 1.0), 1.0, (NM, NM, NM)),
]


@pytest.mark.parametrize("orders,Ks,X,alpha,bcs", NEUMANN)
def test_neumann_solve_matches_oracle(orders, Ks, X, alpha, bcs):
    shp = grid(orders, Ks, bcs)
    f = workloads.uniform_rhs(shp, seed=3)
    S = H.Solver(orders, Ks, X, alpha, bcs=bcs)
    try:
        assert S.shape == shp
        u = S.solve(torch.from_numpy(f).to(DEV)).cpu().numpy()
    finally:
        S.close()
    want = periodic.solve(f, orders, Ks, X, alpha, bcs)
    assert rel(u, want) < 1e-12


def test_neumann_several_rhs_round_trip_and_refusals():
    orders, Ks, X, alpha, bcs = (3, 2), (8, 16), (1.0, 1.0), 0.0, (NM, D)
    shp = grid(orders, Ks, bcs)
    f = workloads.uniform_rhs((2,) + shp, seed=4)
    S = H.Solver(orders, Ks, X, alpha, bcs=bcs)
    try:
        assert H.hofem_solver_workspace_bytes(S.handle, "fp64", 2) == 0   # the passes run on the grid itself
        fd = torch.from_numpy(f).to(DEV).reshape(-1)
        u = torch.empty_like(fd)
        H.hofem_solve(S.handle, "fp64", fd, u, 2, None, 0, 0.0, None, False, True)
        u = u.cpu().numpy().reshape(f.shape)
        c = S.forward(fd, nrhs=2)                  # forward then inverse: C^-1 (V V^T = C^-1)
        back = S.inverse(c, nrhs=2).cpu().numpy().reshape(f.shape)
        for mode, x in (("fp32", fd.float()), ("fp32_ir", fd)):
            with pytest.raises(H.HofemError) as e:
                S.solve(x, mode=mode, nrhs=2)
            assert e.value.status == -2
    finally:
        S.close()
    Cs = [periodic.axis_matrices(n, K, b)[1] for n, K, b in zip(orders, Ks, bcs)]
    for r in range(2):
        assert rel(Cs[0] @ (Cs[1] @ back[r].T).T, f[r]) < 1e-13
        assert rel(u[r], periodic.solve(f[r], orders, Ks, X, alpha, bcs)) < 1e-12


@pytest.mark.slow
def test_neumann_full_size_backward_error():
    # n = 9, K = 1024 on both Neumann axes (9217 x 9217 = 84,953,089 unknowns)
    orders, Ks, X, alpha, bcs = (9, 9), (1024, 1024), (1.0, 1.0), 1.0, (NM, NM)
    shp = grid(orders, Ks, bcs)
    f = workloads.uniform_rhs(shp, seed=9)
    S = H.Solver(orders, Ks, X, alpha, bcs=bcs)
    try:
        u = S.solve(torch.from_numpy(f).to(DEV)).cpu().numpy()
    finally:
        S.close()
    r = f - periodic.apply_operator(u, orders, Ks, X, alpha, bcs)
    mats = [periodic.axis_matrices(n, K, b) for n, K, b in zip(orders, Ks, bcs)]
    inf = lambda M: float(abs(M).sum(axis=1).max())
    s = [4.0 * K ** 2 / x ** 2 for K, x in zip(Ks, X)]
    Linf = (s[0] * inf(mats[0][0]) * inf(mats[1][1]) + s[1] * inf(mats[0][1]) * inf(mats[1][0])
            + alpha * inf(mats[0][1]) * inf(mats[1][1]))
    eta = np.linalg.norm(r) / (Linf * np.linalg.norm(u) + np.linalg.norm(f))
    print(f"Neumann backward error, full size: {eta:.3e}")
    assert eta < 1e-15

# the FP64 operator and mass product with periodic and Neumann axes (one
# kernel per axis and term): against the oracle's assembled operator
OP_CASES = [
    ((3,), (16,), (1.0,), 0.5, (NM,)),
    ((2,), (8,), (2.0,), 1.0, (P,)),
    ((3, 2), (8, 16), (1.0, 0.5), 1.0, (NM, D)),
    ((2, 4), (16, 8), (1.0, 1.0), 1.0, (P, NM)),
    ((2, 2, 3), (4, 8, 4), (1.0, 1.0, 1.0), 2.0, (NM, P, D)),
    ((9, 2), (8, 6), (1.0, 1.0), 1.0, (NM, P)),                      # dense periodic axis
]


@pytest.mark.parametrize("orders,Ks,X,alpha,bcs", OP_CASES)
def test_operator_and_mass_with_periodic_and_neumann_axes(orders, Ks, X, alpha, bcs):
    shp = grid(orders, Ks, bcs)
    u = workloads.uniform_rhs((2,) + shp, seed=21)
    S = H.Solver(orders, Ks, X, alpha, bcs=bcs)
    try:
        assert (H.hofem_operator_workspace_bytes(S.handle) > 0) == (len(orders) > 1)
        ud = torch.from_numpy(u).to(DEV).reshape(-1)
        Lu = S.apply_operator(ud, nrhs=2).cpu().numpy().reshape(u.shape)
        Mu = S.apply_mass(ud, nrhs=2).cpu().numpy().reshape(u.shape)
    finally:
        S.close()
    Cs = [periodic.axis_matrices(n, K, b)[1] for n, K, b in zip(orders, Ks, bcs)]
    for r in range(2):
        want = periodic.apply_operator(u[r], orders, Ks, X, alpha, bcs)
        assert rel(Lu[r], want) < 1e-13
        m = u[r]
        for a, C in enumerate(Cs):
            v = np.moveaxis(m, a, 0)
            m = np.moveaxis((C @ v.reshape(v.shape[0], -1)).reshape(v.shape), 0, a)
        assert rel(Mu[r], m) < 1e-14
