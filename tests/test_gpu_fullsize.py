"""Parity at full size, in the launch configurations the benchmark times.

large_2d (n = 9, K = 1024 per axis, 84,916,225 unknowns) and cube_3d (n = 4,
K = 128 per axis, 133,432,831 unknowns): the FP64 solve by algorithms (a)
and (b), the FP32 solve with
four FP64 refinement steps and the FP32-preconditioned CG form (relative
update 1e-13) against the oracle's exact dense solve, relative l2 <= 1e-12
over all unknowns; the unrefined FP32 solve within 1e-5.
"""
import numpy as np
import pytest

import workloads
from oracle import load, solve as osolve

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

H = pytest.importorskip("paper_1609_07758_amd")

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def check(cfg, f):
    S = H.Solver(cfg["orders"], cfg["Ks"], cfg["X"], cfg["alpha"])
    fd = torch.from_numpy(f).to(DEV)
    u64 = S.solve(fd, mode="fp64").cpu().numpy()
    ub = S.solve(fd, mode="fp64_b").cpu().numpy()
    uir = S.solve(fd, mode="fp32_ir", max_iter=4, tol=0.0).cpu().numpy()
    u32 = S.solve(fd.float(), mode="fp32").double().cpu().numpy()
    upcg, info, st = S.solve(fd, mode="fp32_pcg", max_iter=40, tol=1e-13, want_info=True)
    torch.cuda.synchronize()
    upcg = upcg.cpu().numpy()
    del fd
    S.close()
    want = osolve.solve(f, cfg["orders"], cfg["Ks"], cfg["X"], cfg["alpha"])
    e64, eir, e32, epcg = rel(u64, want), rel(uir, want), rel(u32, want), rel(upcg, want)
    eb = rel(ub, want)
    print(f"fp64 {e64:.3e}  algorithm (b) {eb:.3e}  fp32+4 steps {eir:.3e}  fp32 {e32:.3e}  "
          f"fp32_pcg {epcg:.3e} ({info.iterations} iterations)")
    assert e64 <= 1e-12
    assert eb <= 1e-12
    assert eir <= 1e-12
    assert e32 <= 1e-5
    assert epcg <= 1e-12


def test_large_2d_full_size():
    cfg = workloads.CONFIGS["large_2d"]
    f = workloads.uniform_rhs(workloads.shape(cfg["orders"], cfg["Ks"]), seed=0)
    check(cfg, f)


def test_cube_3d_full_size():
    # f^h: (n+1)-point Gauss load of f = 11 pi^2 sin(pi x) sin(pi y) sin(3 pi z)
    # plus N(0, 1e-3^2) noise on every entry
    cfg = workloads.CONFIGS["cube_3d"]
    s1 = lambda x: np.sin(np.pi * x)
    s3 = lambda x: np.sin(3 * np.pi * x)
    f = load.load_separable([(11 * np.pi ** 2, [s1, s1, s3])], cfg["orders"], cfg["Ks"], cfg["X"])
    f += workloads.normal_noise(f.shape, 1e-3, seed=0)
    check(cfg, f)
