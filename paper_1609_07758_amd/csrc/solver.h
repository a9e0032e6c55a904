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
// Every axis has Dirichlet data and K a power of two (time stepping needs the
// Dirichlet operator and the FFT passes).
bool solver_all_dirichlet(const hofem_solver_s* S);
// Bytes of the operator's element buffer (0 where it needs none; a multiple of 256).
size_t solver_op_elem_bytes(const hofem_solver_s* S);
// FP64 solve by algorithm (a) of nrhs right-hand sides, in -> out (in == out allowed).
int solver_solve_fp64(hofem_solver_s* S, const double* in, double* out, int nrhs, hipStream_t st);
// out = f + coef ((x)_i C_i) w (f == NULL: out = coef (x)C w), FP64, by the
// operator kernels with the stiffness scales set to zero; elem: element
// buffer of solver_op_elem_bytes.  w != out.
int solver_mass_update(hofem_solver_s* S, const double* f, const double* w, double* out,
                       double coef, double* elem, int nrhs, hipStream_t st);

}  // namespace hofem
