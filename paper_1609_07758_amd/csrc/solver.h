// Internal services of the solver (capi.hip) for the other entry points of
// the library (time stepping).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "hofem.h"

namespace hofem {

// Unknowns of one right-hand side and the operator's alpha.
size_t solver_unknowns(const hofem_solver_s* S);
double solver_alpha(const hofem_solver_s* S);
int solver_device(const hofem_solver_s* S);
// Every axis has Dirichlet data and K a power of two (the operator kernels
// of the FP32 refinement, CG and the Dirichlet mass update need them).
bool solver_all_dirichlet(const hofem_solver_s* S);
// Bytes of the operator's element buffer (0 where it needs none; a multiple of 256).
size_t solver_op_elem_bytes(const hofem_solver_s* S);
// FP64 solve by algorithm (a) of nrhs right-hand sides, in -> out (in == out allowed).
int solver_solve_fp64(hofem_solver_s* S, const double* in, double* out, int nrhs, hipStream_t st);
// Axes, and whether one has K not a power of two (dense transforms).
int solver_dims(const hofem_solver_s* S);
bool solver_has_dense(const hofem_solver_s* S);
// One axis of the grid for the per-axis products of any boundary condition:
// condition (0 Dirichlet, 1 periodic, 2 Neumann), order, elements, unknowns
// m, stride of the axis in the C-order grid of one right-hand side, and the
// local mass and stiffness matrices on [-1, 1] (row major, (n+1)^2 <= 100
// values each).
struct AxisLocal {
  int bc, n, K, m;
  long long inner;
  double C[100];
  double A[100];
};
int solver_axis_local(const hofem_solver_s* S, int axis, AxisLocal* out);
// out = cc (C_axis (x) I) in + ca (A_axis (x) I) in + add (add may be NULL or
// out itself) along one axis of `total` points (several right-hand sides in
// sequence), each point summing the local rows of the one or two elements
// that hold it, the stiffness in difference form sum_{r != l} A_lr (v_r - v_l).
hipError_t launch_axis_local(const AxisLocal& a, const double* in, double* out, const double* add,
                             double cc, double ca, long long total, hipStream_t s);
// out = f + coef ((x)_i C_i) w (f == NULL: out = coef (x)C w), FP64, by the
// operator kernels with the stiffness scales set to zero; elem: element
// buffer of solver_op_elem_bytes.  w != out.
int solver_mass_update(hofem_solver_s* S, const double* f, const double* w, double* out,
                       double coef, double* elem, int nrhs, hipStream_t st);

}  // namespace hofem
