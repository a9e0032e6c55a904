"""GPU tests of the launch-shape autotuner: every candidate shape of every
pass gives oracle parity (1e-12 in FP64, 1e-5 in FP32), the tuner keeps the
fastest measured shape per pass, and its disk cache restores the choice."""
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
KIND = {0: "forward", 1: "inverse", 2: "fused"}


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def passes(N):
    # (kind, axis) of the solve: forward N-1..1, fused 0, inverse 1..N-1
    return [(0, a) for a in range(N - 1, 0, -1)] + [(2, 0)] + [(1, a) for a in range(1, N)]


SHAPES = [
    ((9, 9), (64, 64), (1.0, 1.0), 0.0, 1),    # padded FP64 lines
    ((2, 9), (4, 512), (1.0, 1.0), 0.5, 1),    # tight FP64 rows, row-pair intermediate
    ((3, 7), (2, 512), (1.0, 1.0), 0.0, 2),    # tight rows across two right-hand sides
    ((4, 4, 4), (8, 8, 8), (1.0, 1.0, 1.0), 1.0, 1),
    ((5,), (256,), (1.0,), 0.0, 3),
]


@pytest.mark.parametrize("orders,Ks,X,alpha,nrhs", SHAPES)
@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_every_candidate_shape_matches_oracle(orders, Ks, X, alpha, nrhs, mode):
    S = H.Solver(orders, Ks, X, alpha)
    f = np.stack([workloads.uniform_rhs(S.shape, seed=100 + r) for r in range(nrhs)])
    want = [osolve.solve((f[r].astype(np.float32).astype(np.float64) if mode == "fp32" else f[r]),
                         orders, Ks, X, alpha) for r in range(nrhs)]
    dt = torch.float32 if mode == "fp32" else torch.float64
    fd = torch.from_numpy(f).to(DEV, dt)
    tol = 1e-5 if mode == "fp32" else 1e-12
    fp64 = mode == "fp64"
    tried = 0
    for kind, axis in passes(len(orders)):
        cands = H.hofem_pass_shape_candidates(S.handle, kind, axis, fp64, nrhs)
        assert len(cands) >= 1
        for cb, thr in cands:
            H.hofem_pass_set_shape(S.handle, kind, axis, fp64, cb, thr)
            try:
                u = S.solve(fd, mode=mode, nrhs=nrhs)
            except RuntimeError:
                # a shape the row-pair intermediate cannot use is refused
                # before any kernel runs
                continue
            got = u.double().cpu().numpy().reshape((nrhs,) + S.shape)
            for r in range(nrhs):
                assert rel(got[r], want[r]) < tol, (KIND[kind], axis, cb, thr)
            tried += 1
        H.hofem_pass_set_shape(S.handle, kind, axis, fp64, 0, 0)
    assert tried >= len(passes(len(orders)))
    S.close()


def test_autotune_and_cache(tmp_path):
    orders, Ks, X = (4, 4), (64, 64), (1.0, 1.0)
    S = H.Solver(orders, Ks, X, 0.0)
    f = torch.from_numpy(workloads.uniform_rhs(S.shape, seed=7)).to(DEV)
    u = torch.empty_like(f)
    rep = H.hofem_solver_autotune(S.handle, "fp64", f, u, 1, None, 2)
    assert len(rep) == 3
    for e in rep:
        assert e["ms_tuned"] <= e["ms_default"] and e["ms_tuned"] > 0
        assert e["threads"] in (256, 512) and e["cb"] >= 1
    got = S.solve(f, mode="fp64").cpu().numpy()
    assert rel(got, osolve.solve(f.cpu().numpy(), orders, Ks, X, 0.0)) < 1e-12
    path = str(tmp_path / "tune.txt")
    H.hofem_solver_tune_save(S.handle, path)
    text = open(path).read().split("\n")
    assert all(l.startswith(H.hofem_kernel_hash()) for l in text if l)
    H.hofem_solver_tune_reset(S.handle)
    assert H.hofem_solver_tune_load(S.handle, path, "fp64", 1) == 3
    assert H.hofem_solver_tune_load(S.handle, path, "fp64", 2) == 0    # other line counts
    assert H.hofem_solver_tune_load(S.handle, str(tmp_path / "none.txt"), "fp64", 1) == 0
    S.close()
