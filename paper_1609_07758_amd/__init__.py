"""Python binding of libhofem, the MI355X fast direct solver for nth-order
Lagrange FEM on boxes (Zlotnik & Zlotnik, arXiv:1609.07758, Section 2).

The functions below carry the names of the C entry points declared in
include/hofem.h and only marshal arguments: every step of a solve runs in the
library's HIP kernels.  Device buffers are torch tensors on the current HIP
device (torch provides memory and streams only).  The library must have been
built (``python paper_1609_07758_amd/csrc/build.py``); importing the binding
without it raises ImportError, and there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

# torch goes first: its bundled HIP runtime carries the same soname
# (libamdhip64.so.7) that libhofem.so needs, so the library binds to the very
# runtime that owns torch's memory and streams.  Loaded the other way round,
# the system runtime comes in first and torch then maps a second HIP and HSA
# runtime of its own, whichever initialises last sees no device.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhofem.so")

HOFEM_OK = 0
HOFEM_EINVAL = -1
HOFEM_EUNSUPPORTED = -2
HOFEM_ENOTPOSDEF = -3
HOFEM_ENOCONV = -4
HOFEM_EHIP = -5
HOFEM_ENOMEM = -6
HOFEM_ETOOBIG = -7

MODES = {"fp64": 0, "fp32": 1, "fp32_ir": 2, "fp32_pcg": 3, "fp64_b": 4}
TABLES = {"lam": 0, "p": 1, "inorm": 2, "E": 3, "A": 4, "C": 5, "gx": 6, "gw": 7, "B": 8, "D": 9,
          "wr": 10, "wi": 11, "S": 12, "St": 13, "band": 14}
BCS = {"dirichlet": 0, "periodic": 1, "neumann": 2}

# Names and signatures of every entry point of include/hofem.h.
_c_int, _c_double, _c_size, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p


class hofem_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_update", ctypes.c_double),
                ("rel_residual", ctypes.c_double)]


class hofem_batch_problem(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_void_p), ("nrhs", ctypes.c_int)]


class hofem_coef(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("c0", ctypes.c_double), ("c1", ctypes.c_double),
                ("t_dev", ctypes.c_void_p * 3), ("a_dev", ctypes.c_void_p)]


class hofem_pass_time(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("axis", ctypes.c_int), ("fp64", ctypes.c_int),
                ("launches", ctypes.c_longlong), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


PASS_KINDS = {0: "forward", 1: "inverse", 2: "fused", 3: "operator", 4: "update", 5: "banded"}


class hofem_tune_entry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("axis", ctypes.c_int), ("fp64", ctypes.c_int),
                ("cb", ctypes.c_int), ("threads", ctypes.c_int), ("nlines", ctypes.c_longlong),
                ("ms_default", ctypes.c_double), ("ms_tuned", ctypes.c_double)]


SIGNATURES = {
    "hofem_plan1d_create": (_c_int, [_c_int, _c_int, ctypes.POINTER(_vp)]),
    "hofem_plan1d_create_bc": (_c_int, [_c_int, _c_int, _c_int, ctypes.POINTER(_vp)]),
    "hofem_plan1d_destroy": (None, [_vp]),
    "hofem_plan1d_dim": (_c_int, [_vp, ctypes.POINTER(_c_int)]),
    "hofem_plan1d_table": (_c_int, [_vp, _c_int, ctypes.POINTER(_c_double), _c_size]),
    "hofem_plan1d_table_bytes": (_c_int, [_vp, ctypes.POINTER(_c_size)]),
    "hofem_plan1d_upload": (_c_int, [_vp, _vp, _c_size, _vp]),
    "hofem_solver_create": (_c_int, [_c_int, ctypes.POINTER(_vp), ctypes.POINTER(_c_double), _c_double,
                                     ctypes.POINTER(_vp)]),
    "hofem_solver_destroy": (None, [_vp]),
    "hofem_solver_size": (_c_int, [_vp, ctypes.POINTER(_c_size)]),
    "hofem_solver_workspace_bytes": (_c_int, [_vp, _c_int, _c_int, ctypes.POINTER(_c_size)]),
    "hofem_solve": (_c_int, [_vp, _c_int, _vp, _vp, _c_int, _vp, _c_size, _c_int, _c_double, _vp,
                             ctypes.POINTER(hofem_info)]),
    "hofem_solve_ir_noalloc": (_c_int, [_vp, _vp, _vp, _c_int, _c_int, _c_double, _vp,
                                        ctypes.POINTER(hofem_info)]),
    "hofem_forward": (_c_int, [_vp, _c_int, _vp, _vp, _c_int, _vp]),
    "hofem_inverse": (_c_int, [_vp, _c_int, _vp, _vp, _c_int, _vp]),
    "hofem_operator_workspace_bytes": (_c_int, [_vp, ctypes.POINTER(_c_size)]),
    "hofem_apply_operator": (_c_int, [_vp, _vp, _vp, _c_int, _vp, _c_size, _vp]),
    "hofem_apply_mass": (_c_int, [_vp, _vp, _vp, _c_int, _vp, _c_size, _vp]),
    "hofem_dirichlet_rhs": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _vp]),
    "hofem_stepper_create": (_c_int, [_vp, _c_int, ctypes.POINTER(_vp)]),
    "hofem_stepper_destroy": (None, [_vp]),
    "hofem_stepper_workspace_bytes": (_c_int, [_vp, _c_int, ctypes.POINTER(_c_size)]),
    "hofem_stepper_run": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _c_int, _vp, _c_size, _c_int, _vp]),
    "hofem_batch_create": (_c_int, [ctypes.POINTER(hofem_batch_problem), _c_int,
                                    ctypes.POINTER(_vp)]),
    "hofem_batch_destroy": (None, [_vp]),
    "hofem_batch_offsets": (_c_int, [_vp, ctypes.POINTER(_c_size), _c_size]),
    "hofem_batch_groups": (_c_int, [_vp, ctypes.POINTER(_c_int)]),
    "hofem_batch_workspace_bytes": (_c_int, [_vp, _c_int, ctypes.POINTER(_c_size)]),
    "hofem_batch_solve": (_c_int, [_vp, _c_int, _vp, _vp, _vp, _c_size, _c_int, _c_int, _vp]),
    "hofem_pcg_workspace_bytes": (_c_int, [_vp, ctypes.POINTER(hofem_coef), ctypes.POINTER(_c_size)]),
    "hofem_pcg": (_c_int, [_vp, ctypes.POINTER(hofem_coef), _vp, _vp, _c_int, _c_double, _c_int,
                           _vp, _c_size, _vp, ctypes.POINTER(hofem_info)]),
    "hofem_apply_coef_operator": (_c_int, [_vp, ctypes.POINTER(hofem_coef), _vp, _vp, _c_int, _vp,
                                           _c_size, _vp]),
    "hofem_solver_set_timing": (_c_int, [_vp, _c_int]),
    "hofem_solver_set_graph": (_c_int, [_vp, _c_int]),
    "hofem_solver_pass_times": (_c_int, [_vp, ctypes.POINTER(hofem_pass_time), _c_int,
                                         ctypes.POINTER(_c_int)]),
    "hofem_pass_shape_candidates": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int,
                                             ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), _c_int,
                                             ctypes.POINTER(_c_int)]),
    "hofem_pass_set_shape": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int, _c_int]),
    "hofem_solver_autotune": (_c_int, [_vp, _c_int, _vp, _vp, _c_int, _vp, _c_size, _c_int, _vp,
                                       ctypes.POINTER(hofem_tune_entry), _c_int,
                                       ctypes.POINTER(_c_int)]),
    "hofem_solver_tune_save": (_c_int, [_vp, ctypes.c_char_p]),
    "hofem_solver_tune_load": (_c_int, [_vp, ctypes.c_char_p, _c_int, _c_int, ctypes.POINTER(_c_int)]),
    "hofem_solver_tune_reset": (_c_int, [_vp]),
    "hofem_kernel_hash": (ctypes.c_char_p, []),
    "hofem_status_string": (ctypes.c_char_p, [_c_int]),
    "hofem_last_hip_error": (_c_int, []),
}


class HofemError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.hofem_status_string(status).decode() if _lib else str(status)
        if status == HOFEM_EHIP and _lib:
            msg += f" (hipError {_lib.hofem_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "'python paper_1609_07758_amd/csrc/build.py'")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _check(status, where):
    if status != HOFEM_OK:
        raise HofemError(status, where)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


# ---- C entry points, same names ------------------------------------------

def hofem_plan1d_create(n, K):
    h = ctypes.c_void_p()
    _check(_lib.hofem_plan1d_create(int(n), int(K), ctypes.byref(h)), "hofem_plan1d_create")
    return h


def hofem_plan1d_create_bc(n, K, bc):
    h = ctypes.c_void_p()
    b = BCS[bc] if isinstance(bc, str) else int(bc)
    _check(_lib.hofem_plan1d_create_bc(int(n), int(K), b, ctypes.byref(h)),
           "hofem_plan1d_create_bc")
    return h


def hofem_plan1d_destroy(plan):
    _lib.hofem_plan1d_destroy(plan)


def hofem_plan1d_dim(plan):
    m = ctypes.c_int()
    _check(_lib.hofem_plan1d_dim(plan, ctypes.byref(m)), "hofem_plan1d_dim")
    return m.value


def hofem_plan1d_table(plan, which, count):
    out = np.zeros(count, dtype=np.float64)
    w = TABLES[which] if isinstance(which, str) else int(which)
    _check(_lib.hofem_plan1d_table(plan, w, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   out.size), "hofem_plan1d_table")
    return out


def hofem_plan1d_table_bytes(plan):
    b = ctypes.c_size_t()
    _check(_lib.hofem_plan1d_table_bytes(plan, ctypes.byref(b)), "hofem_plan1d_table_bytes")
    return b.value


def hofem_plan1d_upload(plan, buf, stream=None):
    """Copies the plan's device tables into `buf` (a uint8 device tensor)."""
    _check(_lib.hofem_plan1d_upload(plan, _ptr(buf), buf.numel() * buf.element_size(),
                                    _stream(stream)), "hofem_plan1d_upload")


def hofem_solver_create(plans, X, alpha):
    N = len(plans)
    arr = (ctypes.c_void_p * N)(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
    xs = (ctypes.c_double * N)(*[float(x) for x in X])
    h = ctypes.c_void_p()
    _check(_lib.hofem_solver_create(N, arr, xs, float(alpha), ctypes.byref(h)), "hofem_solver_create")
    return h


def hofem_solver_destroy(solver):
    _lib.hofem_solver_destroy(solver)


def hofem_solver_size(solver):
    s = ctypes.c_size_t()
    _check(_lib.hofem_solver_size(solver, ctypes.byref(s)), "hofem_solver_size")
    return s.value


def hofem_solver_workspace_bytes(solver, mode, nrhs=1):
    s = ctypes.c_size_t()
    _check(_lib.hofem_solver_workspace_bytes(solver, MODES[mode], int(nrhs), ctypes.byref(s)),
           "hofem_solver_workspace_bytes")
    return s.value


def hofem_solve(solver, mode, f, u, nrhs=1, ws=None, max_iter=0, tol=0.0, stream=None,
                want_info=False, raise_noconv=True):
    info = hofem_info() if want_info else None
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    st = _lib.hofem_solve(solver, MODES[mode], _ptr(f), _ptr(u), int(nrhs), _ptr(ws), wsb,
                          int(max_iter), float(tol), _stream(stream),
                          ctypes.byref(info) if info is not None else None)
    if st == HOFEM_ENOCONV and not raise_noconv:
        return info, st
    _check(st, "hofem_solve")
    return info, st


def hofem_solve_ir_noalloc(solver, f, u, nrhs=1, max_iter=4, tol=0.0, stream=None,
                           want_info=False):
    """FP32 solve with FP64 refinement whose workspace is the library's own scratch."""
    info = hofem_info() if want_info else None
    st = _lib.hofem_solve_ir_noalloc(solver, _ptr(f), _ptr(u), int(nrhs), int(max_iter),
                                     float(tol), _stream(stream),
                                     ctypes.byref(info) if info is not None else None)
    return info, st


def hofem_forward(solver, mode, x, y, nrhs=1, stream=None):
    _check(_lib.hofem_forward(solver, MODES[mode], _ptr(x), _ptr(y), int(nrhs), _stream(stream)),
           "hofem_forward")


def hofem_inverse(solver, mode, x, y, nrhs=1, stream=None):
    _check(_lib.hofem_inverse(solver, MODES[mode], _ptr(x), _ptr(y), int(nrhs), _stream(stream)),
           "hofem_inverse")


def hofem_operator_workspace_bytes(solver):
    b = ctypes.c_size_t()
    _check(_lib.hofem_operator_workspace_bytes(solver, ctypes.byref(b)),
           "hofem_operator_workspace_bytes")
    return b.value


def hofem_apply_operator(solver, u, out, nrhs=1, ws=None, stream=None):
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    _check(_lib.hofem_apply_operator(solver, _ptr(u), _ptr(out), int(nrhs), _ptr(ws), wsb,
                                     _stream(stream)), "hofem_apply_operator")


def hofem_apply_mass(solver, g, out, nrhs=1, ws=None, stream=None):
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    _check(_lib.hofem_apply_mass(solver, _ptr(g), _ptr(out), int(nrhs), _ptr(ws), wsb,
                                 _stream(stream)), "hofem_apply_mass")


def make_coef(kind=0, c0=1.0, c1=0.0, t=(None, None, None), a=None):
    """hofem_coef from torch device tensors (t: per-axis tables, a: full table)."""
    c = hofem_coef()
    c.kind = int(kind)
    c.c0 = float(c0)
    c.c1 = float(c1)
    for i in range(3):
        ti = t[i] if i < len(t) else None
        c.t_dev[i] = ti.data_ptr() if ti is not None else None
    c.a_dev = a.data_ptr() if a is not None else None
    return c


def hofem_pcg_workspace_bytes(solver, coef=None):
    s = ctypes.c_size_t()
    _check(_lib.hofem_pcg_workspace_bytes(solver, ctypes.byref(coef) if coef else None,
                                          ctypes.byref(s)), "hofem_pcg_workspace_bytes")
    return s.value


def hofem_pcg(solver, coef, f, u, nrhs=1, rtol=1e-10, max_iter=100, ws=None, stream=None,
              raise_noconv=True):
    info = hofem_info()
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    st = _lib.hofem_pcg(solver, ctypes.byref(coef) if coef else None, _ptr(f), _ptr(u), int(nrhs),
                        float(rtol), int(max_iter), _ptr(ws), wsb, _stream(stream),
                        ctypes.byref(info))
    if st == HOFEM_ENOCONV and not raise_noconv:
        return info, st
    _check(st, "hofem_pcg")
    return info, st


def hofem_apply_coef_operator(solver, coef, u, out, nrhs=1, ws=None, stream=None):
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    _check(_lib.hofem_apply_coef_operator(solver, ctypes.byref(coef) if coef else None, _ptr(u),
                                          _ptr(out), int(nrhs), _ptr(ws), wsb, _stream(stream)),
           "hofem_apply_coef_operator")


def hofem_batch_create(problems):
    """problems: sequence of (solver handle, nrhs)."""
    arr = (hofem_batch_problem * len(problems))()
    for i, (h, nrhs) in enumerate(problems):
        arr[i].solver = h
        arr[i].nrhs = int(nrhs)
    b = ctypes.c_void_p()
    _check(_lib.hofem_batch_create(arr, len(problems), ctypes.byref(b)), "hofem_batch_create")
    return b


def hofem_batch_destroy(batch):
    _lib.hofem_batch_destroy(batch)


def hofem_batch_offsets(batch, count):
    out = (ctypes.c_size_t * (count + 1))()
    _check(_lib.hofem_batch_offsets(batch, out, count + 1), "hofem_batch_offsets")
    return [int(x) for x in out]


def hofem_batch_groups(batch):
    g = ctypes.c_int()
    _check(_lib.hofem_batch_groups(batch, ctypes.byref(g)), "hofem_batch_groups")
    return g.value


def hofem_batch_workspace_bytes(batch, mode):
    b = ctypes.c_size_t()
    _check(_lib.hofem_batch_workspace_bytes(batch, MODES[mode] if isinstance(mode, str) else mode,
                                            ctypes.byref(b)), "hofem_batch_workspace_bytes")
    return b.value


def hofem_batch_solve(batch, mode, f, u, ws=None, max_iter=0, use_graph=True, stream=None):
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    m = MODES[mode] if isinstance(mode, str) else mode
    _check(_lib.hofem_batch_solve(batch, m, _ptr(f), _ptr(u), _ptr(ws), wsb, int(max_iter),
                                  1 if use_graph else 0, _stream(stream)), "hofem_batch_solve")


def hofem_dirichlet_rhs(solver, b_ext, f, out, nrhs=1, stream=None):
    _check(_lib.hofem_dirichlet_rhs(solver, _ptr(b_ext), _ptr(f), _ptr(out), int(nrhs),
                                    _stream(stream)), "hofem_dirichlet_rhs")


SCHEMES = {"heat": 0, "wave": 1}


def hofem_stepper_create(solver, scheme):
    h = ctypes.c_void_p()
    _check(_lib.hofem_stepper_create(solver, SCHEMES[scheme] if isinstance(scheme, str) else scheme,
                                     ctypes.byref(h)), "hofem_stepper_create")
    return h


def hofem_stepper_destroy(stepper):
    _lib.hofem_stepper_destroy(stepper)


def hofem_stepper_workspace_bytes(stepper, nrhs=1):
    b = ctypes.c_size_t()
    _check(_lib.hofem_stepper_workspace_bytes(stepper, int(nrhs), ctypes.byref(b)),
           "hofem_stepper_workspace_bytes")
    return b.value


def hofem_stepper_run(stepper, f, u, uprev, nrhs, nsteps, ws, use_graph=True, stream=None):
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    _check(_lib.hofem_stepper_run(stepper, _ptr(f), _ptr(u), _ptr(uprev), int(nrhs), int(nsteps),
                                  _ptr(ws), wsb, 1 if use_graph else 0, _stream(stream)),
           "hofem_stepper_run")


class Stepper:
    """Implicit time stepping ('heat': backward Euler, alpha = 1/dt; 'wave':
    implicit three-level scheme, alpha = 1/dt^2) with a Solver's fast solve."""

    def __init__(self, solver, scheme="heat", nrhs=1):
        import torch
        self.solver = solver
        self.scheme = scheme
        self.nrhs = int(nrhs)
        self.handle = hofem_stepper_create(solver.handle, scheme)
        self.ws = torch.empty(hofem_stepper_workspace_bytes(self.handle, self.nrhs),
                              dtype=torch.uint8, device="cuda")

    def run(self, u, nsteps, f=None, uprev=None, use_graph=True, stream=None):
        hofem_stepper_run(self.handle, f, u, uprev, self.nrhs, nsteps, self.ws, use_graph, stream)
        return u

    def close(self):
        if getattr(self, "handle", None) is not None:
            hofem_stepper_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent problems solved together: problems = [(Solver, nrhs), ...].

    The right-hand sides and solutions live in packed 1D device buffers;
    problem p occupies nrhs * grid values from offsets[p] on, as [nrhs][grid]
    (offsets[-1] is the total)."""

    def __init__(self, problems):
        self.problems = [(s, int(r)) for s, r in problems]
        self.handle = hofem_batch_create([(s.handle, r) for s, r in self.problems])
        self.offsets = hofem_batch_offsets(self.handle, len(self.problems))
        self.groups = hofem_batch_groups(self.handle)
        self.total = self.offsets[-1]

    def view(self, buf, p):
        s, r = self.problems[p]
        o = self.offsets[p]
        return buf[o:o + r * s.size].view((r,) + s.shape)

    def workspace(self, mode, device="cuda"):
        import torch
        return torch.empty(hofem_batch_workspace_bytes(self.handle, mode), dtype=torch.uint8,
                           device=device)

    def solve(self, f, u, mode="fp64", ws=None, max_iter=0, use_graph=True, stream=None):
        import torch
        dt = torch.float32 if mode == "fp32" else torch.float64
        for name, t in (("f", f), ("u", u)):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != dt or t.numel() != self.total:
                raise ValueError(f"{name} must be a contiguous {dt} device tensor of {self.total}")
        if ws is None and hofem_batch_workspace_bytes(self.handle, mode) > 0:
            ws = self.workspace(mode, f.device)
        hofem_batch_solve(self.handle, mode, f, u, ws, max_iter, use_graph, stream)
        return u

    def close(self):
        if getattr(self, "handle", None) is not None:
            hofem_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hofem_solver_set_timing(solver, enable):
    _check(_lib.hofem_solver_set_timing(solver, 1 if enable else 0), "hofem_solver_set_timing")


def hofem_solver_pass_times(solver, max_entries=64):
    arr = (hofem_pass_time * max_entries)()
    cnt = ctypes.c_int()
    _check(_lib.hofem_solver_pass_times(solver, arr, max_entries, ctypes.byref(cnt)),
           "hofem_solver_pass_times")
    return [dict(kind=PASS_KINDS.get(a.kind, str(a.kind)), axis=a.axis, fp64=bool(a.fp64),
                 launches=a.launches, ms=a.ms, bytes=a.bytes) for a in arr[:cnt.value]]


def hofem_pass_shape_candidates(solver, kind, axis, fp64, nrhs=1):
    cb = (ctypes.c_int * 64)()
    thr = (ctypes.c_int * 64)()
    cnt = ctypes.c_int()
    k = {"forward": 0, "inverse": 1, "fused": 2}.get(kind, kind)
    _check(_lib.hofem_pass_shape_candidates(solver, k, int(axis), 1 if fp64 else 0, int(nrhs), cb, thr,
                                            64, ctypes.byref(cnt)), "hofem_pass_shape_candidates")
    return [(cb[i], thr[i]) for i in range(min(cnt.value, 64))]


def hofem_pass_set_shape(solver, kind, axis, fp64, cb, threads):
    k = {"forward": 0, "inverse": 1, "fused": 2}.get(kind, kind)
    _check(_lib.hofem_pass_set_shape(solver, k, int(axis), 1 if fp64 else 0, int(cb), int(threads)),
           "hofem_pass_set_shape")


def hofem_solver_autotune(solver, mode, f, u, nrhs=1, ws=None, reps=3, stream=None):
    arr = (hofem_tune_entry * 16)()
    cnt = ctypes.c_int()
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    _check(_lib.hofem_solver_autotune(solver, MODES[mode], _ptr(f), _ptr(u), int(nrhs), _ptr(ws), wsb,
                                      int(reps), _stream(stream), arr, 16, ctypes.byref(cnt)),
           "hofem_solver_autotune")
    return [dict(kind=PASS_KINDS.get(e.kind, str(e.kind)), axis=e.axis, fp64=bool(e.fp64), cb=e.cb,
                 threads=e.threads, nlines=e.nlines, ms_default=e.ms_default, ms_tuned=e.ms_tuned)
            for e in arr[:min(cnt.value, 16)]]


def hofem_solver_tune_save(solver, path):
    _check(_lib.hofem_solver_tune_save(solver, os.fsencode(path)), "hofem_solver_tune_save")


def hofem_solver_tune_load(solver, path, mode, nrhs=1):
    n = ctypes.c_int()
    _check(_lib.hofem_solver_tune_load(solver, os.fsencode(path), MODES[mode], int(nrhs),
                                       ctypes.byref(n)), "hofem_solver_tune_load")
    return n.value


def hofem_solver_tune_reset(solver):
    _check(_lib.hofem_solver_tune_reset(solver), "hofem_solver_tune_reset")


def hofem_kernel_hash():
    return _lib.hofem_kernel_hash().decode()


# ---- convenience wrappers -------------------------------------------------

class Plan1D:
    """1D eigen data for order n and K elements (host, binary128 precompute);
    bc "dirichlet", "periodic" or "neumann"."""

    def __init__(self, n, K, bc="dirichlet"):
        self.n, self.K, self.bc = int(n), int(K), bc
        self.handle = hofem_plan1d_create_bc(n, K, bc)
        self.m = hofem_plan1d_dim(self.handle)

    def upload(self, device="cuda"):
        """Device tables in a caller-owned uint8 tensor (kept alive by the caller)."""
        import torch
        buf = torch.empty(hofem_plan1d_table_bytes(self.handle), dtype=torch.uint8, device=device)
        hofem_plan1d_upload(self.handle, buf)
        return buf

    def table(self, which):
        n, K = self.n, self.K
        counts = {"lam": self.m, "p": (K - 1) * n * (n - 1), "inorm": (K - 1) * n,
                  "E": (n - 1) ** 2, "A": (n + 1) ** 2, "C": (n + 1) ** 2,
                  "gx": n + 1, "gw": n + 1, "B": (n + 1) ** 2, "D": (n + 1) ** 2,
                  "wr": (K // 2 + 1) * n * n, "wi": (K // 2 + 1) * n * n,
                  "S": self.m * self.m, "St": self.m * self.m, "band": (n + 1) * n}
        return hofem_plan1d_table(self.handle, which, counts[which])

    def close(self):
        if self.handle is not None:
            hofem_plan1d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Solver of (sum_i 4 h_i^-2 A_i (x) C_others + alpha (x)C) v = f^h on a box."""

    def __init__(self, orders, Ks, X, alpha=0.0, bcs=None):
        self.orders = [int(n) for n in orders]
        self.Ks = [int(k) for k in Ks]
        self.X = [float(x) for x in X]
        self.alpha = float(alpha)
        self.bcs = list(bcs) if bcs is not None else ["dirichlet"] * len(self.orders)
        if len(self.bcs) != len(self.orders):
            raise ValueError("one boundary condition per axis")
        self.handle = None
        plans = {}
        keys = list(zip(self.orders, self.Ks, self.bcs))
        for key in keys:
            if key not in plans:
                plans[key] = Plan1D(*key)
        # the plans' device tables: caller-owned, alive as long as the solver
        self._tables = [p.upload() for p in plans.values()]
        axis_plans = [plans[key] for key in keys]
        self.shape = tuple(p.m for p in axis_plans)
        self.handle = hofem_solver_create([p.handle for p in axis_plans], self.X, self.alpha)
        for p in plans.values():
            p.close()
        self.size = hofem_solver_size(self.handle)

    def pcg_workspace(self, coef=None, device="cuda"):
        import torch
        b = hofem_pcg_workspace_bytes(self.handle, coef)
        return torch.empty(b, dtype=torch.uint8, device=device)

    def pcg(self, f, u=None, coef=None, nrhs=1, rtol=1e-10, max_iter=100, ws=None, stream=None,
            raise_noconv=True):
        """CG on -div(a grad u) + alpha u = f preconditioned by the FP32 fast solve."""
        import torch
        self._check_grid(f, torch.float64, nrhs, "f")
        u = torch.empty_like(f) if u is None else u
        if ws is None:
            ws = self.pcg_workspace(coef, f.device)
        info, st = hofem_pcg(self.handle, coef, f, u, nrhs, rtol, max_iter, ws, stream,
                             raise_noconv)
        return u, info, st

    def apply_coef_operator(self, u, coef, out=None, nrhs=1, ws=None, stream=None):
        import torch
        out = torch.empty_like(u) if out is None else out
        if ws is None:
            ws = self.pcg_workspace(coef, u.device)
        hofem_apply_coef_operator(self.handle, coef, u, out, nrhs, ws, stream)
        return out

    def workspace(self, mode, nrhs=1, device="cuda"):
        import torch
        b = hofem_solver_workspace_bytes(self.handle, mode, nrhs)
        if b == 0:
            return None
        return torch.empty(b, dtype=torch.uint8, device=device)

    def _check_grid(self, t, dtype, nrhs, name):
        import torch
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous device tensor")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}")
        if t.numel() != self.size * nrhs:
            raise ValueError(f"{name} has {t.numel()} elements, expected {self.size * nrhs}")
        return t

    def solve(self, f, u=None, mode="fp64", nrhs=1, max_iter=3, tol=0.0, ws=None, stream=None,
              want_info=False, raise_noconv=True):
        import torch
        dt = torch.float32 if mode == "fp32" else torch.float64
        self._check_grid(f, dt, nrhs, "f")
        if u is None:
            u = torch.empty_like(f)
        self._check_grid(u, dt, nrhs, "u")
        if ws is None:   # (FP64 needs one only with a dense axis)
            ws = self.workspace(mode, nrhs, f.device)
        info, st = hofem_solve(self.handle, mode, f, u, nrhs, ws, max_iter, tol, stream, want_info,
                               raise_noconv)
        return (u, info, st) if want_info else u

    def forward(self, x, y=None, mode="fp64", nrhs=1, stream=None):
        import torch
        y = torch.empty_like(x) if y is None else y
        hofem_forward(self.handle, mode, x, y, nrhs, stream)
        return y

    def inverse(self, x, y=None, mode="fp64", nrhs=1, stream=None):
        import torch
        y = torch.empty_like(x) if y is None else y
        hofem_inverse(self.handle, mode, x, y, nrhs, stream)
        return y

    def operator_workspace(self, device="cuda"):
        import torch
        b = hofem_operator_workspace_bytes(self.handle)
        return torch.empty(b, dtype=torch.uint8, device=device) if b else None

    def apply_operator(self, u, out=None, nrhs=1, ws=None, stream=None):
        import torch
        out = torch.empty_like(u) if out is None else out
        if ws is None:
            ws = self.operator_workspace(u.device)
        hofem_apply_operator(self.handle, u, out, nrhs, ws, stream)
        return out

    def apply_mass(self, g, out=None, nrhs=1, ws=None, stream=None):
        """f^h = (x)_i C_i g: right-hand side of the FEM interpolant of nodal values g."""
        import torch
        out = torch.empty_like(g) if out is None else out
        if ws is None:
            ws = self.operator_workspace(g.device)
        hofem_apply_mass(self.handle, g, out, nrhs, ws, stream)
        return out

    def dirichlet_rhs(self, b_ext, f=None, out=None, nrhs=1, stream=None):
        """f^h with the boundary values of b_ext (extended grid, m_i + 2 per axis) moved in."""
        import torch
        if out is None:
            out = torch.empty((nrhs,) + self.shape if nrhs > 1 else self.shape,
                              dtype=torch.float64, device=b_ext.device)
        hofem_dirichlet_rhs(self.handle, b_ext, f, out, nrhs, stream)
        return out

    def autotune(self, mode="fp64", nrhs=1, reps=3, cache=None, f=None, u=None, stream=None):
        """Tunes the passes' launch shapes for `mode` on synthetic data (or f, u);
        with `cache`, shapes found there are applied and fresh results saved."""
        import torch
        if cache is not None and hofem_solver_tune_load(self.handle, cache, mode, nrhs) > 0:
            return None
        dt = torch.float32 if mode == "fp32" else torch.float64
        if f is None:
            g = torch.Generator(device="cuda").manual_seed(0)
            f = torch.rand(nrhs * self.size, dtype=dt, device="cuda", generator=g) * 2 - 1
        if u is None:
            u = torch.empty_like(f)
        ws = self.workspace(mode, nrhs, f.device) if mode == "fp32_ir" else None
        rep = hofem_solver_autotune(self.handle, mode, f, u, nrhs, ws, reps, stream)
        if cache is not None:
            hofem_solver_tune_save(self.handle, cache)
        return rep

    def set_timing(self, enable=True):
        hofem_solver_set_timing(self.handle, enable)

    def set_graph(self, enable=True):
        """Replay non-synchronising solves from a HIP graph (captured on the second call)."""
        _check(_lib.hofem_solver_set_graph(self.handle, 1 if enable else 0), "hofem_solver_set_graph")

    def pass_times(self):
        return hofem_solver_pass_times(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            hofem_solver_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
