// Implicit time stepping with the fast solve: the paper's use of the fast
// direct solver inside implicit methods for time-dependent problems
// (Section 1; Section 2, paragraph 4 on other equations).
//
// Heat equation u_t - Lap u = f, backward Euler with step dt and
// alpha = 1/dt: the scaled FEM system of eq. (bvp glob 2) for one step is
//   L u^{n+1} = f^h + alpha ((x)_i C_i) u^n.
// Wave equation u_tt - Lap u = f, the implicit three-level scheme
// (u^{n+1} - 2u^n + u^{n-1}) / dt^2 - Lap u^{n+1} = f with alpha = 1/dt^2:
//   L u^{n+1} = f^h + alpha ((x)_i C_i) (2u^n - u^{n-1}).
// A step is one mass update (with Dirichlet axes only: by the operator
// kernels with the stiffness scales set to zero; with periodic or Neumann
// axes: one mass kernel per axis), one FP64 solve by algorithm (a) (2N - 1
// passes) and, for the wave scheme, one vector kernel.  A step is captured
// once into a HIP graph and replayed.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "hofem.h"
#include "kernels.h"
#include "solver.h"

using namespace hofem;

struct hofem_stepper_s {
  hofem_solver S = nullptr;
  int scheme = 0;
  // graph of one step for the last (buffers, nrhs)
  hipGraphExec_t exec = nullptr;
  const double* g_f = nullptr;
  double* g_u = nullptr;
  double* g_up = nullptr;
  void* g_ws = nullptr;
  int g_nrhs = 0;
  bool warm = false;
};

namespace {

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// w = 2 u - up, then up = u (the wave scheme's shift of time levels)
__global__ void wave_shift(const double* __restrict__ u, double* __restrict__ up,
                           double* __restrict__ w, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double a = u[i];
    w[i] = 2.0 * a - up[i];
    up[i] = a;
  }
}

// out = f + coef ((x)_i C_i) w, one axis after another (w != out; tmp: one
// grid, used when there are two or more axes).
int mass_chain(hofem_stepper_s* T, const double* f, const double* w, double* out, double coef,
               double* tmp, int nrhs, hipStream_t st) {
  const int N = solver_dims(T->S);
  const long long total = (long long)solver_unknowns(T->S) * nrhs;
  const double* src = w;
  for (int ax = 0; ax < N; ++ax) {
    AxisLocal al;
    const int rc = solver_axis_local(T->S, ax, &al);
    if (rc != HOFEM_OK) return rc;
    double* dst = ((N - 1 - ax) % 2 == 0) ? out : tmp;
    const bool last = ax == N - 1;
    const hipError_t e = launch_axis_local(al, src, dst, last ? f : nullptr, last ? coef : 1.0, 0.0, total, st);
    if (e != hipSuccess) return record_hip_error(e);
    src = dst;
  }
  return HOFEM_OK;
}

size_t ws_bytes_of(const hofem_stepper_s* T, int nrhs) {
  const size_t grid = al256(solver_unknowns(T->S) * (size_t)nrhs * sizeof(double));
  const size_t levels = grid * (T->scheme == HOFEM_SCHEME_WAVE ? 2 : 1);
  if (solver_all_dirichlet(T->S)) return levels + solver_op_elem_bytes(T->S);
  return levels + (solver_dims(T->S) >= 2 ? grid : 0);   // the mass chain's second grid
}

int one_step(hofem_stepper_s* T, const double* f, double* u, double* up, int nrhs, void* ws,
             hipStream_t st) {
  const long long n = (long long)solver_unknowns(T->S) * nrhs;
  const size_t grid = al256((size_t)n * sizeof(double));
  unsigned char* p = static_cast<unsigned char*>(ws);
  double* rhs = reinterpret_cast<double*>(p);
  p += grid;
  const double* w = u;
  if (T->scheme == HOFEM_SCHEME_WAVE) {
    double* wb = reinterpret_cast<double*>(p);
    p += grid;
    const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(wave_shift, dim3(blocks), dim3(256), 0, st, u, up, wb, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return record_hip_error(e);
    w = wb;
  }
  const int rc = solver_all_dirichlet(T->S)
                     ? solver_mass_update(T->S, f, w, rhs, solver_alpha(T->S),
                                          reinterpret_cast<double*>(p), nrhs, st)
                     : mass_chain(T, f, w, rhs, solver_alpha(T->S), reinterpret_cast<double*>(p),
                                  nrhs, st);
  if (rc != HOFEM_OK) return rc;
  return solver_solve_fp64(T->S, rhs, u, nrhs, st);
}

void drop_graph(hofem_stepper_s* T) {
  if (T->exec) (void)hipGraphExecDestroy(T->exec);
  T->exec = nullptr;
}

}  // namespace

extern "C" {

int hofem_stepper_create(hofem_solver solver, int scheme, hofem_stepper* out) {
  if (!solver || !out) return HOFEM_EINVAL;
  if (scheme != HOFEM_SCHEME_HEAT && scheme != HOFEM_SCHEME_WAVE) return HOFEM_EINVAL;
  if (!(solver_alpha(solver) > 0)) return HOFEM_EINVAL;   // alpha = 1/dt or 1/dt^2
  if (solver_has_dense(solver)) return HOFEM_EUNSUPPORTED;   // K not a power of two
  hofem_stepper T = new (std::nothrow) hofem_stepper_s;
  if (!T) return HOFEM_ENOMEM;
  T->S = solver;
  T->scheme = scheme;
  *out = T;
  return HOFEM_OK;
}

void hofem_stepper_destroy(hofem_stepper T) {
  if (!T) return;
  drop_graph(T);
  delete T;
}

int hofem_stepper_workspace_bytes(hofem_stepper T, int nrhs, size_t* bytes) {
  if (!T || !bytes || nrhs < 1) return HOFEM_EINVAL;
  *bytes = ws_bytes_of(T, nrhs);
  return HOFEM_OK;
}

int hofem_stepper_run(hofem_stepper T, const double* f_dev, double* u_dev, double* uprev_dev,
                      int nrhs, int nsteps, void* ws_dev, size_t ws_bytes, int use_graph,
                      void* stream) {
  if (!T || !u_dev || nrhs < 1 || nsteps < 0 || !ws_dev) return HOFEM_EINVAL;
  if (ws_bytes < ws_bytes_of(T, nrhs)) return HOFEM_EINVAL;
  if (T->scheme == HOFEM_SCHEME_WAVE && (!uprev_dev || uprev_dev == u_dev)) return HOFEM_EINVAL;
  if (f_dev && f_dev == u_dev) return HOFEM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* up = T->scheme == HOFEM_SCHEME_WAVE ? uprev_dev : nullptr;
  int done = 0;
  if (!use_graph || !T->warm || st == nullptr) {
    // eager steps; the first one also performs the one-time kernel set-up
    // that must not happen inside a capture (the legacy default stream
    // cannot be captured)
    const int eager = (use_graph && st != nullptr) ? std::min(nsteps, 1) : nsteps;
    for (; done < eager; ++done) {
      const int rc = one_step(T, f_dev, u_dev, up, nrhs, ws_dev, st);
      if (rc != HOFEM_OK) return rc;
    }
    if (done > 0) T->warm = true;
    if (done == nsteps) return HOFEM_OK;
  }
  if (!(T->exec && T->g_f == f_dev && T->g_u == u_dev && T->g_up == up && T->g_ws == ws_dev &&
        T->g_nrhs == nrhs)) {
    drop_graph(T);
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return record_hip_error(e);
    const int rc = one_step(T, f_dev, u_dev, up, nrhs, ws_dev, st);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (rc != HOFEM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return record_hip_error(e);
    e = hipGraphInstantiate(&T->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      T->exec = nullptr;
      return record_hip_error(e);
    }
    T->g_f = f_dev;
    T->g_u = u_dev;
    T->g_up = up;
    T->g_ws = ws_dev;
    T->g_nrhs = nrhs;
  }
  for (; done < nsteps; ++done) {
    const hipError_t e = hipGraphLaunch(T->exec, st);
    if (e != hipSuccess) return record_hip_error(e);
  }
  return HOFEM_OK;
}

}  // extern "C"
