"""GPU tests of the variable-coefficient operator and of preconditioned CG
(the fast solver used as a preconditioner), through the C ABI, against the
CPU oracle (oracle.varcoef).

Tolerances: operator applies agree with the oracle to 1e-13 of the largest
output; CG solutions satisfy ||f - L_a u|| <= rtol ||f|| with the residual
recomputed by the oracle (slack 1% of rtol plus FP64 rounding), and agree
with the oracle's sparse direct solution to rtol times the condition bound
measured by the oracle on the same mesh.
"""
import numpy as np
import pytest

import workloads
from oracle import solve as osolve, varcoef

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

H = pytest.importorskip("paper_1609_07758_amd")

DEV = "cuda:0"


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=DEV, dtype=torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def sine_tables(orders, Ks, X, ks):
    c0, c1, ts = workloads.sine_coefficient(ks)
    tabs = [ts[i](varcoef.gauss_points(orders[i], Ks[i], X[i])) for i in range(len(orders))]
    return c0, c1, tabs


def coef_kind1(orders, Ks, X, ks):
    c0, c1, tabs = sine_tables(orders, Ks, X, ks)
    dev = [gpu(t) for t in tabs]
    coef = H.make_coef(1, c0, c1, t=tuple(dev) + (None,) * (3 - len(dev)))
    return coef, varcoef.expand_separable(c0, c1, tabs), dev


def coef_kind2(orders, Ks, seed):
    nel = int(np.prod(Ks))
    npts = int(np.prod([n + 1 for n in orders]))
    a_full = 0.5 + np.random.default_rng(seed).random((nel, npts))
    dev = gpu(a_full)
    return H.make_coef(2, a=dev), a_full, dev


OPCASES = [
    ((5,), (16,), (1.0,), 0.5),
    ((3, 2), (8, 16), (1.0, 2.0), 0.0),
    ((9, 9), (4, 8), (1.0, 1.0), 1.0),
    ((3, 3, 3), (4, 8, 4), (1.0, 1.0, 1.0), 0.0),
    ((2, 4, 3), (4, 4, 2), (1.0, 0.5, 2.0), 2.0),
]


@pytest.mark.parametrize("orders,Ks,X,alpha", OPCASES)
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_coef_operator_matches_oracle(orders, Ks, X, alpha, kind):
    shp = workloads.shape(orders, Ks)
    u = np.random.default_rng(1).uniform(-1, 1, (2,) + shp)
    S = H.Solver(orders, Ks, X, alpha)
    keep = None
    if kind == 0:
        coef = H.make_coef(0)
        a_full = np.ones((int(np.prod(Ks)), int(np.prod([n + 1 for n in orders]))))
    elif kind == 1:
        coef, a_full, keep = coef_kind1(orders, Ks, X, workloads.wavenumbers(len(orders), 5))
    else:
        coef, a_full, keep = coef_kind2(orders, Ks, 7)
    out = host(S.apply_coef_operator(gpu(u), coef, nrhs=2))
    want = varcoef.apply(u, orders, Ks, X, alpha, a_full)
    assert np.max(np.abs(out - want)) <= 1e-13 * np.max(np.abs(want))
    del keep


def oracle_residual(f, u, orders, Ks, X, alpha, a_full):
    r = f - varcoef.apply(u, orders, Ks, X, alpha, a_full)
    return float(np.linalg.norm(r) / np.linalg.norm(f))


@pytest.mark.parametrize("orders,Ks,X,alpha", [
    ((3, 3), (16, 16), (1.0, 1.0), 0.0),
    ((2, 5), (32, 8), (1.0, 2.0), 1.0),
    ((3, 3, 3), (8, 8, 8), (1.0, 1.0, 1.0), 0.0),
])
def test_pcg_matches_direct_solve(orders, Ks, X, alpha):
    shp = workloads.shape(orders, Ks)
    f = workloads.uniform_rhs(shp, seed=0)
    coef, a_full, keep = coef_kind1(orders, Ks, X, workloads.wavenumbers(len(orders), 0))
    S = H.Solver(orders, Ks, X, alpha)
    rtol = 1e-12
    u, info, st = S.pcg(gpu(f), coef=coef, rtol=rtol, max_iter=200)
    got = host(u)
    assert st == H.HOFEM_OK
    assert 0 < info.iterations < 200
    assert info.rel_residual <= rtol
    assert oracle_residual(f, got, orders, Ks, X, alpha, a_full) <= 1.01 * rtol + 1e-14
    want = varcoef.solve(f, orders, Ks, X, alpha, a_full)
    # error <= cond * residual; cond(L_a) <= (max a / min a) cond(L) and the
    # preconditioned iteration stops on the true residual
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    assert err <= 1e-7
    del keep


def test_pcg_unit_coefficient_equals_fast_solve():
    orders, Ks, X, alpha = (4, 4), (32, 16), (1.0, 1.0), 0.5
    shp = workloads.shape(orders, Ks)
    f = workloads.uniform_rhs(shp, seed=2)
    S = H.Solver(orders, Ks, X, alpha)
    u, info, st = S.pcg(gpu(f), coef=None, rtol=1e-13, max_iter=50)
    want = osolve.solve(f, orders, Ks, X, alpha)
    got = host(u)
    assert float(np.linalg.norm(got - want) / np.linalg.norm(want)) <= 1e-12
    assert info.iterations <= 6          # the preconditioner is the inverse up to FP32


def test_fp32_pcg_mode_reaches_1e12():
    orders, Ks, X, alpha = (9, 9), (64, 32), (1.0, 1.0), 0.0
    shp = workloads.shape(orders, Ks)
    f = workloads.uniform_rhs(shp, seed=0)
    S = H.Solver(orders, Ks, X, alpha)
    fd = gpu(f)
    u = host(S.solve(fd, mode="fp32_pcg", tol=1e-13, max_iter=30))
    want = osolve.solve(f, orders, Ks, X, alpha)
    assert float(np.linalg.norm(u - want) / np.linalg.norm(want)) <= 1e-12


def test_pcg_batch_and_kind2():
    orders, Ks, X, alpha = (2, 3), (16, 8), (1.0, 1.0), 0.0
    shp = workloads.shape(orders, Ks)
    f = np.stack([workloads.uniform_rhs(shp, seed=s) for s in (0, 1)])
    coef, a_full, keep = coef_kind2(orders, Ks, 11)
    S = H.Solver(orders, Ks, X, alpha)
    u, info, st = S.pcg(gpu(f), coef=coef, nrhs=2, rtol=1e-11, max_iter=200)
    got = host(u)
    for r in range(2):
        assert oracle_residual(f[r], got[r], orders, Ks, X, alpha, a_full) <= 1.01e-11
    del keep


def test_pcg_noconv_and_errors():
    orders, Ks, X, alpha = (3, 3), (16, 16), (1.0, 1.0), 0.0
    shp = workloads.shape(orders, Ks)
    f = gpu(workloads.uniform_rhs(shp, seed=0))
    coef, a_full, keep = coef_kind1(orders, Ks, X, (3, 3))
    S = H.Solver(orders, Ks, X, alpha)
    u, info, st = S.pcg(f, coef=coef, rtol=1e-14, max_iter=2, raise_noconv=False)
    assert st == H.HOFEM_ENOCONV and info.iterations == 2
    with pytest.raises(RuntimeError):
        S.pcg(f, u=f, coef=coef)                       # in place is rejected
    bad = H.make_coef(1, 1.0, 0.5, t=(keep[0], None, None))
    with pytest.raises(RuntimeError):
        S.pcg(f, coef=bad)                             # missing axis table
    del keep


def test_varcoef_3d_full_size():
    """The 3D variable-coefficient problem at full size: PCG to 1e-10 with the
    residual recomputed by the oracle, matrix-free, on the host."""
    cfg = workloads.CONFIGS["varcoef_3d"]
    orders, Ks, X, alpha = cfg["orders"], cfg["Ks"], cfg["X"], cfg["alpha"]
    shp = workloads.shape(orders, Ks)
    f = workloads.uniform_rhs(shp, seed=0)
    coef, a_full, keep = coef_kind1(orders, Ks, X, workloads.wavenumbers(3, 0))
    S = H.Solver(orders, Ks, X, alpha)
    u, info, st = S.pcg(gpu(f), coef=coef, rtol=1e-10, max_iter=300)
    got = host(u)
    print(f"varcoef_3d: {info.iterations} iterations, rel residual {info.rel_residual:.3e}")
    assert st == H.HOFEM_OK and info.rel_residual <= 1e-10
    assert oracle_residual(f, got, orders, Ks, X, alpha, a_full) <= 1.01e-10
    del keep
