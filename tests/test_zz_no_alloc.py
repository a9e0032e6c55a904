"""The FP32-with-refinement entry point that allocates nothing
(hofem_solve_ir_noalloc, its workspace in the library's fixed device
scratch) against the entry point that takes a caller workspace
(hofem_solve, mode FP32_IR): the same kernels in the same order, so equal
bit for bit, and within 1e-12 of the oracle.  Two calls in a row on the
shared scratch, the second with a smaller problem; a 3D problem whose
operator keeps its plane-product grids in the scratch; a problem too large for
the scratch is refused before any work."""
import ctypes

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


def one_case(orders, Ks, X, alpha, nrhs, seed):
    S = H.Solver(orders, Ks, X, alpha)
    f = np.stack([workloads.uniform_rhs(S.shape, seed=seed + r) for r in range(nrhs)])
    fd = torch.from_numpy(f).to(DEV)
    ref = S.solve(fd, mode="fp32_ir", nrhs=nrhs, max_iter=4, tol=0.0)   # caller workspace
    u = torch.full_like(fd, float("nan"))
    stream = torch.cuda.current_stream().cuda_stream
    st = H._lib.hofem_solve_ir_noalloc(S.handle, ctypes.c_void_p(fd.data_ptr()),
                                       ctypes.c_void_p(u.data_ptr()), nrhs, 4, 0.0,
                                       ctypes.c_void_p(stream), None)
    assert st == H.HOFEM_OK, H._lib.hofem_status_string(st)
    torch.cuda.synchronize()
    assert torch.equal(u, ref)
    got = u.cpu().numpy()
    for r in range(nrhs):
        assert rel(got[r], osolve.solve(f[r], orders, Ks, X, alpha)) < 1e-12
    S.close()


def test_noalloc_equals_workspace_entry_point_twice_then_smaller():
    one_case((9, 9), (32, 32), (1.0, 1.0), 0.0, 2, seed=40)    # 287^2 x 2 right-hand sides
    one_case((3, 2), (8, 16), (1.0, 2.0), 0.5, 1, seed=50)     # then a smaller problem


def test_noalloc_3d_element_buffer_in_scratch():
    one_case((3, 3, 3), (4, 8, 8), (1.0, 1.0, 1.0), 0.0, 1, seed=60)
    one_case((2, 2, 2), (4, 4, 4), (1.0, 1.0, 1.0), 1.0, 2, seed=70)


def test_noalloc_rejects_too_large():
    S = H.Solver((9, 9), (1024, 1024), (1.0, 1.0), 0.0)   # 85M unknowns: 340 MB of FP32 residual
    f = torch.zeros(4, dtype=torch.float64, device=DEV)
    u = torch.zeros(4, dtype=torch.float64, device=DEV)
    st = H._lib.hofem_solve_ir_noalloc(S.handle, ctypes.c_void_p(f.data_ptr()),
                                       ctypes.c_void_p(u.data_ptr()), 1, 4, 0.0, None, None)
    assert st == H.HOFEM_ETOOBIG
    assert H._lib.hofem_status_string(st).startswith(b"problem exceeds")
    torch.cuda.synchronize()
    assert torch.count_nonzero(u) == 0
    S.close()
