"""Host-side tests of the C ABI (no GPU needed).

The library loads, exports every entry point that include/hofem.h declares,
rejects invalid arguments with the documented codes, and its binary128 host
precompute reproduces the oracle's high-precision eigen data.
"""
import ctypes
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from oracle import assembly, element, spectral

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hofem.h")

H = pytest.importorskip("paper_1609_07758_amd")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hofem_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(H.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(H.SIGNATURES)


@pytest.mark.parametrize("n,K", [(0, 16), (10, 16), (2, 1), (2, 2048), (-1, 8), (9, 1000)])
def test_plan_rejects_unsupported(n, K):
    h = ctypes.c_void_p()
    assert H._lib.hofem_plan1d_create(n, K, ctypes.byref(h)) == H.HOFEM_EUNSUPPORTED


def test_null_and_size_errors():
    assert H._lib.hofem_plan1d_create(2, 16, None) == H.HOFEM_EINVAL
    p = H.Plan1D(3, 8)
    out = np.zeros(5)
    ptr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert H._lib.hofem_plan1d_table(p.handle, 0, ptr, 5) == H.HOFEM_EINVAL     # wrong length
    assert H._lib.hofem_plan1d_table(p.handle, 9, ptr, 5) == H.HOFEM_EINVAL     # bad table id
    assert H._lib.hofem_solver_create(0, None, None, 0.0, None) == H.HOFEM_EINVAL
    arr = (ctypes.c_void_p * 1)(p.handle.value)
    xs = (ctypes.c_double * 1)(1.0)
    h = ctypes.c_void_p()
    assert H._lib.hofem_solver_create(4, arr, xs, 0.0, ctypes.byref(h)) == H.HOFEM_EUNSUPPORTED
    bad = (ctypes.c_double * 1)(-1.0)
    assert H._lib.hofem_solver_create(1, arr, bad, 0.0, ctypes.byref(h)) == H.HOFEM_EINVAL
    # alpha below -pi^2 / X^2 (scaled): the smallest denominator is negative
    assert H._lib.hofem_solver_create(1, arr, xs, -1e4, ctypes.byref(h)) == H.HOFEM_ENOTPOSDEF
    # a plan whose tables were never uploaded to a device
    assert H._lib.hofem_solver_create(1, arr, xs, 0.0, ctypes.byref(h)) == H.HOFEM_EINVAL
    assert H._lib.hofem_solve(None, 0, None, None, 1, None, 0, 0, 0.0, None, None) == H.HOFEM_EINVAL
    assert H._lib.hofem_apply_mass(None, None, None, 1, None, 0, None) == H.HOFEM_EINVAL
    assert H._lib.hofem_apply_operator(None, None, None, 1, None, 0, None) == H.HOFEM_EINVAL
    size = ctypes.c_size_t()
    assert H._lib.hofem_operator_workspace_bytes(None, ctypes.byref(size)) == H.HOFEM_EINVAL


def test_plan_table_image_size_and_upload_errors():
    p = H.Plan1D(9, 1024)
    nbytes = H.hofem_plan1d_table_bytes(p.handle)
    # FP64 lambda, p + norms in FP64 and FP32, twiddles, sines: about 1.4 MB
    n, K = 9, 1024
    assert nbytes % 256 == 0 and 8 * n * K < nbytes < 2 * 1024 * 1024
    assert H._lib.hofem_plan1d_table_bytes(p.handle, None) == H.HOFEM_EINVAL
    assert H._lib.hofem_plan1d_upload(p.handle, None, nbytes, None) == H.HOFEM_EINVAL
    # too few bytes and a misaligned buffer are rejected before any copy
    assert H._lib.hofem_plan1d_upload(p.handle, ctypes.c_void_p(4096), nbytes - 256, None) == H.HOFEM_EINVAL
    assert H._lib.hofem_plan1d_upload(p.handle, ctypes.c_void_p(4096 + 8), nbytes, None) == H.HOFEM_EINVAL
    assert H.hofem_solver_size is not None
    assert H._lib.hofem_status_string(H.HOFEM_ENOCONV) == b"refinement did not converge"


@pytest.mark.parametrize("n,K", [(1, 16), (2, 16), (3, 8), (4, 32), (6, 16), (9, 8), (9, 64),
                                 (3, 12), (5, 6), (2, 3), (9, 10)])
def test_plan_tables_match_oracle(n, K):
    p = H.Plan1D(n, K)
    o = spectral.eigen_structured(n, K)
    # coefficient order: the k = 0 modes, then for each l the wave numbers k = 1..K-1
    lam = np.concatenate([o["lam0"], o["lam"].T.ravel()])
    # both sides round high-precision values once: equal up to one rounding
    assert np.allclose(p.table("lam"), lam, rtol=2.3e-16, atol=0)
    if n > 1:
        assert np.allclose(p.table("p").reshape(K - 1, n, n - 1), o["p"], rtol=0, atol=4e-16 * np.abs(o["p"]).max())
        assert np.allclose(p.table("E").reshape(n - 1, n - 1), o["E"], rtol=0, atol=4e-16 * np.abs(o["E"]).max())
    # norms against the direct C-norm of the oracle's eigenvectors
    S, _ = spectral.eigenvectors_structured(n, K, o)
    _, Cs = assembly.assemble_1d_sparse(n, K)
    direct = np.einsum("ij,ij->j", S, Cs @ S)[n - 1:]
    assert np.allclose(p.table("inorm"), 1.0 / direct, rtol=1e-14, atol=0)


@pytest.mark.parametrize("n", range(1, 10))
def test_local_matrices_match_exact(n):
    p = H.Plan1D(n, 4)
    A, C = element.local_matrices(n)
    Af = np.array([[float(x) for x in r] for r in A]).ravel()
    Cf = np.array([[float(x) for x in r] for r in C]).ravel()
    assert np.allclose(p.table("A"), Af, rtol=4.5e-16, atol=1e-300)
    assert np.allclose(p.table("C"), Cf, rtol=4.5e-16, atol=1e-300)


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_tables_match_oracle(n):
    # nodes increasing, weights, basis values / derivatives at the nodes
    from oracle import varcoef
    p = H.Plan1D(n, 4)
    x, w = varcoef.gauss_rule(n)
    B, D = varcoef.basis_tables(n)
    assert np.all(np.diff(p.table("gx")) > 0)
    # both sides round once from >= 34 digits: equal up to one rounding
    for name, ref in (("gx", x), ("gw", w), ("B", B.ravel()), ("D", D.ravel())):
        assert np.allclose(p.table(name), ref, rtol=2.3e-16, atol=1e-30), name


def test_one_hip_runtime_in_process():
    """The binding and torch share one HIP runtime (a second copy would own
    no device once torch's has initialised)."""
    import torch  # noqa: F401
    maps = open("/proc/self/maps").read().split("\n")
    hip = {l.split()[-1] for l in maps if "libamdhip64" in l}
    hsa = {l.split()[-1] for l in maps if "libhsa-runtime64" in l}
    assert len(hip) == 1, hip
    assert len(hsa) <= 1, hsa


@pytest.mark.parametrize("n,K", [(1, 8), (2, 4), (3, 16), (5, 8), (9, 4), (4, 2)])
def test_periodic_plan_tables(n, K):
    # Bloch waves of the periodic plan are eigenvectors of the assembled
    # periodic pencil (oracle.periodic), C-normalised to K, with the listed
    # eigenvalues; the eigenvalues are the pencil's full spectrum.
    import scipy.linalg as sla
    from oracle import periodic
    P = H.Plan1D(n, K, "periodic")
    try:
        assert P.m == n * K
        lam = P.table("lam")
        wr, wi = P.table("wr"), P.table("wi")
        with pytest.raises(H.HofemError):
            P.table("p")
    finally:
        P.close()
    A, C = periodic.assemble_1d(n, K)
    dense = np.sort(sla.eigh(A, C, eigvals_only=True))
    assert np.max(np.abs(np.sort(lam) - dense)) < 1e-11 * max(1.0, dense[-1])
    assert lam[0] == 0.0
    w = (wr + 1j * wi).reshape(K // 2 + 1, n, n)
    j = np.arange(K)
    for k in range(K // 2 + 1):
        ph = np.exp(2j * np.pi * k * j / K)
        for l in range(n):
            v = (ph[:, None] * w[k, l][None, :]).reshape(-1)
            t = 0 if k == 0 else (K - 1 if 2 * k == K else 2 * k - 1)
            lv = lam[l * K + t]
            r = A @ v - lv * (C @ v)
            assert np.linalg.norm(r) < 1e-11 * max(1.0, lv) * np.linalg.norm(C @ v)
            assert abs(np.vdot(v, C @ v) - K) < 1e-12 * K
            if 0 < k < K // 2:
                assert lam[l * K + t + 1] == lv


def test_periodic_plan_rejects_bad_bc():
    h = ctypes.c_void_p()
    lib = ctypes.CDLL(H.LIB_PATH)
    assert lib.hofem_plan1d_create_bc(2, 8, 3, ctypes.byref(h)) == -1
    assert lib.hofem_plan1d_create_bc(2, 2048, 1, ctypes.byref(h)) == -2


def neumann_basis(P):
    """The Neumann eigenvectors the plan's tables define (columns, in the
    Neumann coefficient order), their eigenvalues and C-norms: for k =
    1..K-1 the cosine counterparts of Theorem 1's vectors with the Dirichlet
    p_k^(l), then the n + 1 band-edge cells repeated along the axis."""
    n, K = P.n, P.K
    m = n * K + 1
    lam, p, inorm, band = P.table("lam"), P.table("p"), P.table("inorm"), P.table("band")
    V = np.zeros((m, m))
    nrm = np.zeros(m)
    for l in range(n):
        for k in range(1, K):
            q = l * (K - 1) + (k - 1)
            pk = p[((k - 1) * n + l) * (n - 1):((k - 1) * n + l + 1) * (n - 1)]
            V[0::n, q] = np.cos(np.pi * k * np.arange(K + 1) / K)
            for e in range(1, K + 1):
                for s in range(1, n):
                    V[n * (e - 1) + s, q] = (np.cos(np.pi * k * (e - 1) / K) * pk[s - 1]
                                             + np.cos(np.pi * k * e / K) * pk[n - s - 1])
            nrm[q] = 1.0 / inorm[(k - 1) * n + l]
    nb0 = n // 2 + 1
    for b in range(n + 1):
        q = n * (K - 1) + b
        sg = 1.0 if b < nb0 else -1.0
        w = band[b * n:(b + 1) * n]
        V[0::n, q] = w[0] * sg ** np.arange(K + 1)
        for e in range(1, K + 1):
            for s in range(1, n):
                V[n * (e - 1) + s, q] = w[s] * sg ** (e - 1)
        nrm[q] = K
    return V, lam, nrm


@pytest.mark.parametrize("n,K", [(1, 8), (2, 8), (3, 16), (4, 8), (8, 16), (9, 32), (3, 12), (2, 5)])
def test_neumann_plan_eigenbasis_matches_oracle(n, K):
    # the tables define a complete C-orthogonal eigenbasis of the oracle's
    # assembled Neumann pencil: A V = C V diag(lam), V^T C V = diag(norms)
    from oracle import periodic
    P = H.Plan1D(n, K, "neumann")
    try:
        assert P.m == n * K + 1
        V, lam, nrm = neumann_basis(P)
        D = H.Plan1D(n, K)
        try:   # p and 1/||s||^2 are those of the Dirichlet plan
            assert np.array_equal(P.table("p"), D.table("p"))
            assert np.array_equal(P.table("inorm"), D.table("inorm"))
        finally:
            D.close()
    finally:
        P.close()
    A, C = [M.toarray() for M in periodic.axis_matrices(n, K, "neumann")]
    scale = np.abs(A).max()
    assert np.abs(A @ V - (C @ V) * lam).max() < 1e-11 * scale * np.abs(V).max()
    G = V.T @ C @ V
    assert np.abs(G - np.diag(nrm)).max() < 1e-12 * nrm.max()
    assert lam[n * (K - 1)] == 0.0 and lam.min() == 0.0   # the constants
    assert np.sort(lam)[1] > 0                             # nothing else in the kernel


@pytest.mark.parametrize("n,K", [(3, 12), (2, 5), (9, 6)])
def test_neumann_dense_tables(n, K):
    # K not a power of two: the plan also holds the eigenvectors as the dense
    # S (columns in the Neumann coefficient order) and S diag(1/||v||^2)
    P = H.Plan1D(n, K, "neumann")
    try:
        m = P.m
        V, lam, nrm = neumann_basis(P)
        S, St = P.table("S").reshape(m, m), P.table("St").reshape(m, m)
    finally:
        P.close()
    assert np.abs(S - V).max() < 1e-14
    assert np.abs(St - V / nrm).max() < 1e-14


@pytest.mark.parametrize("n,K", [(2, 6), (3, 5), (1, 7), (4, 12)])
def test_periodic_dense_tables_match_oracle(n, K):
    # K not a power of two, periodic: S holds the real eigenvectors (real and
    # imaginary parts of the Bloch waves), A S = C S diag(lam); St^T C S = I
    from oracle import periodic
    P = H.Plan1D(n, K, "periodic")
    try:
        m = P.m
        lam = P.table("lam")
        S, St = P.table("S").reshape(m, m), P.table("St").reshape(m, m)
    finally:
        P.close()
    A, C = [M.toarray() for M in periodic.axis_matrices(n, K, "periodic")]
    assert np.abs(A @ S - (C @ S) * lam).max() < 1e-11 * np.abs(A).max() * np.abs(S).max()
    assert np.abs(St.T @ C @ S - np.eye(m)).max() < 1e-12


def test_neumann_plan_tables_and_limits():
    P = H.Plan1D(3, 8, "neumann")
    try:
        assert P.table("band").size == 4 * 3
        assert P.table("lam").size == 25
        with pytest.raises(H.HofemError):
            P.table("wr")                     # Bloch vectors: periodic plans only
    finally:
        P.close()
    D = H.Plan1D(3, 8)
    try:
        with pytest.raises(H.HofemError):
            D.table("band")                   # band-edge cells: Neumann plans only
    finally:
        D.close()
    h = ctypes.c_void_p()
    lib = ctypes.CDLL(H.LIB_PATH)
    assert lib.hofem_plan1d_create_bc(9, 1024, 2, ctypes.byref(h)) == 0
    lib.hofem_plan1d_destroy(h)
    assert lib.hofem_plan1d_create_bc(2, 2048, 2, ctypes.byref(h)) == -2
    assert lib.hofem_plan1d_create_bc(9, 455, 2, ctypes.byref(h)) == -2   # dense: m = 4096 > 4095
    assert lib.hofem_plan1d_create_bc(9, 454, 2, ctypes.byref(h)) == 0    # m = 4087
    lib.hofem_plan1d_destroy(h)


def test_non_power_of_two_plans():
    # axes whose K is not a power of two take dense transforms (m <= 4095)
    P = H.Plan1D(3, 12)
    try:
        assert P.m == 35
    finally:
        P.close()
    h = ctypes.c_void_p()
    lib = ctypes.CDLL(H.LIB_PATH)
    assert lib.hofem_plan1d_create_bc(9, 455, 0, ctypes.byref(h)) == 0   # m = 4094
    lib.hofem_plan1d_destroy(h)
    assert lib.hofem_plan1d_create_bc(9, 456, 0, ctypes.byref(h)) == -2   # m = 4103
    for bc in (1, 2):                            # periodic and Neumann axes too
        assert lib.hofem_plan1d_create_bc(2, 12, bc, ctypes.byref(h)) == 0
        lib.hofem_plan1d_destroy(h)
    assert lib.hofem_plan1d_create_bc(9, 455, 1, ctypes.byref(h)) == 0    # periodic m = 4095
    lib.hofem_plan1d_destroy(h)
    assert lib.hofem_plan1d_create_bc(9, 456, 1, ctypes.byref(h)) == -2   # m = 4104


@pytest.mark.parametrize("n,K", [(3, 12), (2, 3), (5, 6)])
def test_dense_eigenvectors_match_oracle(n, K):
    # the dense transform matrices of a non-power-of-two plan: the columns of
    # S are Theorem 1's eigenvectors (the oracle's structured route), St
    # scales them by 1 / ||s||_C^2
    P = H.Plan1D(n, K)
    try:
        m = P.m
        S = P.table("S").reshape(m, m)
        St = P.table("St").reshape(m, m)
    finally:
        P.close()
    o = spectral.eigen_structured(n, K)
    So, _ = spectral.eigenvectors_structured(n, K, o)
    # the oracle lists the k >= 1 columns k-major, the library l-major
    perm = list(range(n - 1)) + [(n - 1) + (k - 1) * n + (l - 1)
                                 for l in range(1, n + 1) for k in range(1, K)]
    So = So[:, perm]
    assert np.allclose(S, So, rtol=0, atol=1e-14 * np.abs(So).max())
    A, C = assembly.assemble_1d(n, K)
    G = St.T @ C @ S   # = identity: St^T is the inverse of S
    assert np.allclose(G, np.eye(m), rtol=0, atol=1e-12)
