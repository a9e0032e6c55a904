"""GPU tests of the batched form (many independent problems per call).

Every problem's solution must equal, bit for bit, the single-problem solve
of the same right-hand sides (the batch runs the same kernels on grouped
slabs), and sampled problems must match the CPU oracle to 1e-12 (FP64).
Graph replays are checked against the eager result on every replay, with
eager work and host synchronisation between them.
"""
import numpy as np
import pytest

import workloads
from oracle import solve as osolve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

H = pytest.importorskip("paper_1609_07758_amd")

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def make_batch(pairs, nrhs_list, X=(1.0, 1.0), alpha=0.0):
    solvers = {}
    probs = []
    for (n, K), r in zip(pairs, nrhs_list):
        if (n, K) not in solvers:
            solvers[(n, K)] = H.Solver((n, n), (K, K), X, alpha)
        probs.append((solvers[(n, K)], r))
    return H.Batch(probs), solvers


def fill(batch, rhs, dtype):
    f = torch.empty(batch.total, dtype=dtype, device=DEV)
    for p, arr in enumerate(rhs):
        batch.view(f, p).copy_(torch.from_numpy(arr))
    return f


SMALL = [(2, 8), (3, 16), (2, 8), (4, 8), (3, 16), (2, 8), (4, 8), (3, 16)]
NRHS = [2, 1, 2, 3, 1, 1, 3, 2]


def small_rhs(seed=5):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-1, 1, (r, n * K - 1, n * K - 1)) for (n, K), r in zip(SMALL, NRHS)]


def test_layout_and_groups():
    batch, _ = make_batch(SMALL, NRHS)
    # groups: distinct (solver, nrhs) pairs
    assert batch.groups == len(set(zip(SMALL, NRHS)))
    sizes = [r * (n * K - 1) ** 2 for (n, K), r in zip(SMALL, NRHS)]
    offs = batch.offsets
    assert offs[-1] == sum(sizes)
    spans = sorted((offs[p], offs[p] + sizes[p]) for p in range(len(SMALL)))
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert a1 == b0          # a partition of [0, total)
    assert spans[0][0] == 0


@pytest.mark.parametrize("mode", ["fp64", "fp32", "fp32_ir"])
def test_small_batch_equals_single_solves(mode):
    batch, _ = make_batch(SMALL, NRHS)
    rhs = small_rhs()
    dt = torch.float32 if mode == "fp32" else torch.float64
    f = fill(batch, rhs, dt)
    u = torch.zeros_like(f)
    batch.solve(f, u, mode=mode, max_iter=3, use_graph=False)
    torch.cuda.synchronize()
    for p, ((n, K), r) in enumerate(zip(SMALL, NRHS)):
        S = batch.problems[p][0]
        fp = batch.view(f, p).contiguous()
        up = S.solve(fp, mode=mode, nrhs=r, max_iter=3, tol=0.0)
        torch.cuda.synchronize()
        assert torch.equal(batch.view(u, p), up), p
        if mode != "fp32":
            # FP64, and three refinement steps on these small grids
            for j in range(r):
                want = osolve.solve(rhs[p][j], (n, n), (K, K), (1.0, 1.0), 0.0)
                assert rel(batch.view(u, p)[j].cpu().numpy(), want) < 1e-12


def test_graph_replays_match_eager():
    batch, _ = make_batch(SMALL, NRHS)
    rhs = small_rhs(7)
    f = fill(batch, rhs, torch.float64)
    u_eager = torch.zeros_like(f)
    batch.solve(f, u_eager, mode="fp32_ir", max_iter=2, use_graph=False)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    u = torch.zeros_like(f)
    with torch.cuda.stream(s):
        for rep in range(4):
            u.zero_()
            batch.solve(f, u, mode="fp32_ir", max_iter=2, use_graph=True, stream=s.cuda_stream)
            s.synchronize()
            assert torch.equal(u, u_eager), rep
            # eager work between replays
            tmp = torch.randn(1 << 20, device=DEV, dtype=torch.float64)
            float(tmp.sum())
    # new right-hand side values in the same buffer: the replay reads them
    f2 = fill(batch, small_rhs(8), torch.float64)
    f.copy_(f2)
    u2_eager = torch.zeros_like(f)
    batch.solve(f, u2_eager, mode="fp32_ir", max_iter=2, use_graph=False)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        batch.solve(f, u, mode="fp32_ir", max_iter=2, use_graph=True, stream=s.cuda_stream)
        s.synchronize()
    assert torch.equal(u, u2_eager)


def test_3d_solver_shared_by_two_groups_graph():
    # One 3D solver in two groups (nrhs 1 and 2): the groups run on forked
    # streams in the graph, each with the operator's element buffer in its
    # own workspace region; every replay equals the eager result and the
    # oracle.
    orders, Ks, X = (3, 3, 3), (4, 4, 8), (1.0, 1.0, 1.0)
    S = H.Solver(orders, Ks, X, 0.5)
    T = H.Solver((2, 2, 2), (4, 4, 4), X, 0.0)
    probs = [(S, 1), (T, 1), (S, 2), (S, 1)]
    batch = H.Batch(probs)
    assert batch.groups == 3
    rng = np.random.default_rng(12)
    rhs = [rng.uniform(-1, 1, (r,) + s.shape) for s, r in probs]
    f = fill(batch, rhs, torch.float64)
    u_eager = torch.zeros_like(f)
    batch.solve(f, u_eager, mode="fp32_ir", max_iter=4, use_graph=False)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    u = torch.zeros_like(f)
    with torch.cuda.stream(st):
        for rep in range(3):
            u.zero_()
            batch.solve(f, u, mode="fp32_ir", max_iter=4, use_graph=True, stream=st.cuda_stream)
            st.synchronize()
            assert torch.equal(u, u_eager), rep
    for p, (s_, r) in enumerate(probs):
        o = s_.orders
        for j in range(r):
            want = osolve.solve(rhs[p][j], o, s_.Ks, X, s_.alpha)
            assert rel(batch.view(u, p)[j].cpu().numpy(), want) < 1e-12, (p, j)


def test_batch_with_periodic_neumann_and_dense_groups():
    # groups of periodic, Neumann, non-power-of-two (dense) and plain solvers
    # in one FP64 batch, eager and from the graph, against the oracle
    from oracle import periodic
    X = (1.0, 1.0)
    specs = [((2, 3), (8, 16), 1.0, ("neumann", "dirichlet")),
             ((3, 2), (16, 8), 1.0, ("periodic", "periodic")),
             ((2, 2), (6, 12), 0.0, ("dirichlet", "dirichlet")),
             ((3, 3), (8, 8), 0.0, ("dirichlet", "dirichlet")),
             ((2, 2), (6, 8), 1.0, ("neumann", "periodic"))]
    solvers = [H.Solver(o, K, X, a, bcs=b) for o, K, a, b in specs]
    probs = [(solvers[0], 2), (solvers[1], 1), (solvers[2], 1), (solvers[3], 2), (solvers[4], 1),
             (solvers[0], 1)]
    batch = H.Batch(probs)
    rng = np.random.default_rng(13)
    rhs = [rng.uniform(-1, 1, (r,) + s.shape) for s, r in probs]
    f = fill(batch, rhs, torch.float64)
    u_eager = torch.zeros_like(f)
    batch.solve(f, u_eager, mode="fp64", use_graph=False)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    u = torch.zeros_like(f)
    with torch.cuda.stream(st):
        for rep in range(2):
            u.zero_()
            batch.solve(f, u, mode="fp64", use_graph=True, stream=st.cuda_stream)
            st.synchronize()
            assert torch.equal(u, u_eager), rep
    for p, (s_, r) in enumerate(probs):
        o, K, a, b = specs[solvers.index(s_)]
        for j in range(r):
            want = periodic.solve(rhs[p][j], o, K, X, a, b)
            assert rel(batch.view(u, p)[j].cpu().numpy(), want) < 1e-12, (p, j)


def test_batch_errors():
    batch, _ = make_batch(SMALL[:2], NRHS[:2])
    f = torch.zeros(batch.total, dtype=torch.float64, device=DEV)
    with pytest.raises(RuntimeError):
        batch.solve(f, f, mode="fp32_ir", max_iter=1)           # in place
    with pytest.raises(RuntimeError):
        H.hofem_batch_solve(batch.handle, 3, f, f.clone(), None, 0, 1, False)   # PCG not batched
    with pytest.raises(RuntimeError):
        H.hofem_batch_create([(None, 1)])


def test_batch_2d_full_size():
    """The 256-problem batch: every problem equals its single solve; the
    smallest and largest problems and one in between match the oracle."""
    cfg = workloads.BATCH
    pairs = workloads.batch_problems(cfg["count"], seed=0)
    batch, solvers = make_batch(pairs, [cfg["nrhs"]] * len(pairs))
    f = torch.empty(batch.total, dtype=torch.float64, device=DEV)
    rhs_gen = workloads.batch_rhs(pairs, cfg["nrhs"], seed=0)
    sizes = [(n * K - 1) for n, K in pairs]
    smallest, largest = int(np.argmin(sizes)), int(np.argmax(sizes))
    middle = int(np.argsort(sizes)[len(sizes) // 2])
    keep = {}
    for p, arr in enumerate(rhs_gen):
        batch.view(f, p).copy_(torch.from_numpy(arr))
        if p in (smallest, largest, middle):
            keep[p] = arr
    u = torch.empty_like(f)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        batch.solve(f, u, mode="fp64", use_graph=True, stream=s.cuda_stream)   # eager (first)
        u2 = torch.empty_like(f)
        batch.solve(f, u2, mode="fp64", use_graph=True, stream=s.cuda_stream)  # captured
        s.synchronize()
    assert torch.equal(u, u2)
    print(f"batch_2d: {len(pairs)} problems, {batch.groups} groups, {batch.total} unknowns")
    for p in range(len(pairs)):
        S = batch.problems[p][0]
        up = S.solve(batch.view(f, p).contiguous(), mode="fp64", nrhs=cfg["nrhs"])
        assert torch.equal(batch.view(u, p), up), p
    for p, arr in keep.items():
        n, K = pairs[p]
        for j in (0, cfg["nrhs"] - 1):
            want = osolve.solve(arr[j], (n, n), (K, K), cfg["X"], cfg["alpha"])
            assert rel(batch.view(u, p)[j].cpu().numpy(), want) < 1e-12, (p, n, K)
