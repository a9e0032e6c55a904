"""GPU tests of implicit time stepping (hofem_stepper_*): backward Euler for
the heat equation and the implicit three-level scheme for the wave equation,
against the oracle's step-by-step solves (relative l2 <= 1e-12), also with
periodic and Neumann axes, with the HIP-graph replays equal to the eager
steps on every replay."""
import numpy as np
import pytest

import workloads
from oracle import timestep as ots

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

H = pytest.importorskip("paper_1609_07758_amd")

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


CASES = [
    # (scheme, orders, Ks, X, alpha, nsteps, with load)
    ("heat", (3, 3), (8, 8), (1.0, 1.0), 50.0, 7, True),
    ("heat", (9, 2), (4, 16), (1.0, 0.5), 400.0, 4, False),
    ("wave", (2, 3, 2), (4, 4, 8), (1.0, 1.0, 1.0), 900.0, 6, True),
    ("wave", (4, 4), (16, 16), (1.0, 1.0), 2500.0, 5, False),
    ("heat", (3, 3, 3), (4, 4, 4), (1.0, 1.0, 1.0), 30.0, 3, True),
]


@pytest.mark.parametrize("scheme,orders,Ks,X,alpha,nsteps,load", CASES)
def test_steps_match_oracle(scheme, orders, Ks, X, alpha, nsteps, load):
    S = H.Solver(orders, Ks, X, alpha)
    u0 = workloads.uniform_rhs(S.shape, seed=80)
    up0 = workloads.uniform_rhs(S.shape, seed=81) if scheme == "wave" else None
    f = workloads.uniform_rhs(S.shape, seed=82) if load else None
    T = H.Stepper(S, scheme)
    u = torch.from_numpy(u0).to(DEV)
    up = torch.from_numpy(up0).to(DEV) if up0 is not None else None
    fd = torch.from_numpy(f).to(DEV) if f is not None else None
    T.run(u, nsteps, f=fd, uprev=up, use_graph=False)
    torch.cuda.synchronize()
    want, want_prev = ots.steps(u0, f, orders, Ks, X, alpha, ots.HEAT if scheme == "heat" else ots.WAVE,
                                nsteps, uprev=up0)
    assert rel(u.cpu().numpy(), want) < 1e-12
    if scheme == "wave":
        assert rel(up.cpu().numpy(), want_prev) < 1e-12
    T.close()


# periodic and Neumann axes: the step's mass product runs axis by axis; the
# expected steps are the oracle's solves of the same step equations with its
# assembled mass matrices
BC_CASES = [
    # (scheme, orders, Ks, X, alpha, nsteps, with load, bcs)
    ("heat", (3, 2), (8, 16), (1.0, 1.0), 50.0, 4, True, ("neumann", "dirichlet")),
    ("heat", (2, 3), (16, 8), (1.0, 1.0), 100.0, 3, False, ("periodic", "periodic")),
    ("wave", (2, 2), (8, 8), (1.0, 1.0), 400.0, 4, True, ("neumann", "neumann")),
    ("wave", (3,), (32,), (1.0,), 900.0, 5, False, ("periodic",)),
    ("heat", (4,), (16,), (2.0,), 20.0, 3, True, ("neumann",)),
    ("heat", (2, 2, 2), (4, 8, 4), (1.0, 1.0, 1.0), 30.0, 3, True, ("neumann", "periodic", "dirichlet")),
]


def oracle_bc_steps(u0, up0, f, orders, Ks, X, alpha, bcs, scheme, nsteps):
    from oracle import periodic
    Cs = [periodic.axis_matrices(n, K, b)[1] for n, K, b in zip(orders, Ks, bcs)]

    def mass(w):
        for a, C in enumerate(Cs):
            v = np.moveaxis(w, a, 0)
            w = np.moveaxis((C @ v.reshape(v.shape[0], -1)).reshape(v.shape), 0, a)
        return w

    u, up = u0.copy(), None if up0 is None else up0.copy()
    for _ in range(nsteps):
        w = u if scheme == "heat" else 2.0 * u - up
        rhs = alpha * mass(w) + (f if f is not None else 0.0)
        un = periodic.solve(rhs, orders, Ks, X, alpha, bcs)
        if scheme == "wave":
            up = u
        u = un
    return u, up


@pytest.mark.parametrize("scheme,orders,Ks,X,alpha,nsteps,load,bcs", BC_CASES)
def test_steps_with_periodic_and_neumann_axes(scheme, orders, Ks, X, alpha, nsteps, load, bcs):
    S = H.Solver(orders, Ks, X, alpha, bcs=bcs)
    u0 = workloads.uniform_rhs(S.shape, seed=83)
    up0 = workloads.uniform_rhs(S.shape, seed=84) if scheme == "wave" else None
    f = workloads.uniform_rhs(S.shape, seed=85) if load else None
    T = H.Stepper(S, scheme)
    u = torch.from_numpy(u0).to(DEV)
    up = torch.from_numpy(up0).to(DEV) if up0 is not None else None
    fd = torch.from_numpy(f).to(DEV) if f is not None else None
    T.run(u, nsteps, f=fd, uprev=up, use_graph=True)
    torch.cuda.synchronize()
    want, want_prev = oracle_bc_steps(u0, up0, f, orders, Ks, X, alpha, bcs, scheme, nsteps)
    assert rel(u.cpu().numpy(), want) < 1e-12
    if scheme == "wave":
        assert rel(up.cpu().numpy(), want_prev) < 1e-12
    T.close()
    S.close()


@pytest.mark.parametrize("scheme", ["heat", "wave"])
def test_graph_replays_equal_eager(scheme):
    orders, Ks, X = (4, 4), (8, 16), (1.0, 1.0)
    S = H.Solver(orders, Ks, X, 200.0)
    u0 = torch.from_numpy(workloads.uniform_rhs(S.shape, seed=90)).to(DEV)
    up0 = torch.from_numpy(workloads.uniform_rhs(S.shape, seed=91)).to(DEV)
    f = torch.from_numpy(workloads.uniform_rhs(S.shape, seed=92)).to(DEV)
    T = H.Stepper(S, scheme)
    # eager reference: 4 steps, then 3 more
    ue, upe = u0.clone(), up0.clone()
    T.run(ue, 4, f=f, uprev=upe, use_graph=False)
    torch.cuda.synchronize()
    ue4, upe4 = ue.clone(), upe.clone()
    T.run(ue, 3, f=f, uprev=upe, use_graph=False)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for rep in range(3):
        u, up = u0.clone(), up0.clone()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            T.run(u, 4, f=f, uprev=up, use_graph=True, stream=s.cuda_stream)
            s.synchronize()
            assert torch.equal(u, ue4), rep
            if scheme == "wave":
                assert torch.equal(up, upe4), rep
            tmp = torch.randn(1 << 18, device=DEV, dtype=torch.float64)   # eager work between
            float(tmp.sum())
            T.run(u, 3, f=f, uprev=up, use_graph=True, stream=s.cuda_stream)
            s.synchronize()
        assert torch.equal(u, ue), rep
    T.close()


def test_stepper_errors():
    S0 = H.Solver((2, 2), (4, 4), (1.0, 1.0), 0.0)
    with pytest.raises(RuntimeError):
        H.Stepper(S0, "heat")                   # alpha = 0: no time step
    S = H.Solver((2, 2), (4, 4), (1.0, 1.0), 10.0)
    with pytest.raises(RuntimeError):
        H.hofem_stepper_create(S.handle, 7)      # unknown scheme
    T = H.Stepper(S, "wave")
    u = torch.zeros(S.size, dtype=torch.float64, device=DEV)
    with pytest.raises(RuntimeError):
        T.run(u, 2)                              # wave scheme without the previous level
    T.close()
    Sd = H.Solver((2,), (6,), (1.0,), 10.0)
    with pytest.raises(RuntimeError):
        H.Stepper(Sd, "heat")                   # K not a power of two: no FFT passes
    Sd.close()
