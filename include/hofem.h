/*
 * hofem.h -- C ABI of the MI355X (gfx950) fast direct solver for nth-order
 * Lagrange finite elements on rectangular boxes with Dirichlet data (and,
 * per axis, periodic or Neumann conditions; see enum hofem_bc).
 *
 * The method is that of A. Zlotnik and I. Zlotnik, "A direct fast FFT-based
 * implementation for high order finite element method on rectangular
 * parallelepipeds for PDE" (arXiv:1609.07758), Section 2:
 *
 *   (sum_i 4 h_i^-2 A_i (x)_{j!=i} C_j + alpha (x)_j C_j) v = f^h       eq. (bvp glob 2)
 *
 * is solved by expanding f^h in the C-orthogonal eigenvectors of the 1D
 * pencils A_i v = lambda C_i v (Theorem 1), dividing by the sums of scaled
 * eigenvalues (eq. (decomp v 2)) and transforming back (algorithm (a)).  The
 * direct and inverse transforms along an axis use n sine transforms of
 * length K-1 coupled by n x n blocks per wave number (transform theorem).
 *
 * Conventions shared by all calls
 * ------------------------------
 * Grid layout.  Per Dirichlet axis i the unknowns are the values at the
 * m_i = n_i K_i - 1 interior points q h_i / n_i (q = 1..m_i, h_i = X_i / K_i):
 * mesh nodes and element-interior Lagrange nodes, in physical order; the
 * Dirichlet zeros are implicit (periodic and Neumann axes: enum hofem_bc).  An N-D grid is dense C order [nrhs][m_0]...[m_{N-1}] (the last
 * axis is contiguous).  The right-hand side is the algebraic f^h of
 * eq. (bvp glob 2): the load vector int f phi divided by prod_i (h_i / 2).
 *
 * Memory.  Pointers named *_dev are device pointers on the current HIP
 * device, owned by the caller: grids, workspaces and the plans' device
 * tables (hofem_plan1d_upload).  Pointers named *_host are host memory owned
 * by the caller.  Handles are host structures owned by the library and
 * released by the matching destroy call.  No call allocates device memory:
 * temporary storage is the caller's workspace, sized by the
 * *_workspace_bytes calls.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  Calls enqueue work and return without synchronising, except
 * where `info` is non-NULL (the call then waits for the stream to read the
 * iteration statistics back).
 *
 * Errors.  Every int-returning call returns HOFEM_OK or a negative status.
 * Argument errors are detected before any work is enqueued and leave all
 * outputs untouched.  HOFEM_EHIP reports a failed HIP runtime call; its code
 * is available from hofem_last_hip_error().
 */
#ifndef HOFEM_H
#define HOFEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum hofem_status {
  HOFEM_OK = 0,
  HOFEM_EINVAL = -1,        /* invalid argument (null pointer, size, ...) */
  HOFEM_EUNSUPPORTED = -2,  /* valid but unsupported parameters (n, K, N) */
  HOFEM_ENOTPOSDEF = -3,    /* alpha makes the operator indefinite */
  HOFEM_ENOCONV = -4,       /* refinement did not reach the tolerance */
  HOFEM_EHIP = -5,          /* HIP runtime failure */
  HOFEM_ENOMEM = -6,        /* host or device allocation failed */
  HOFEM_ETOOBIG = -7        /* the problem exceeds hofem_solve_ir_noalloc's fixed scratch */
};

/* Arithmetic of a solve. */
enum hofem_mode {
  HOFEM_MODE_FP64 = 0,     /* FP64 transforms; f, u are double */
  HOFEM_MODE_FP32 = 1,     /* FP32 transforms with FP32 accumulation; f, u are float */
  HOFEM_MODE_FP32_IR = 2,  /* FP32 transforms + FP64 iterative refinement; f, u are double */
  HOFEM_MODE_FP32_PCG = 3, /* CG on the FP64 operator preconditioned by the FP32 solve;
                              f, u are double */
  HOFEM_MODE_FP64_B = 4    /* algorithm (b): FP64 transforms along axes 0..N-2, banded
                              solves along axis N-1; f, u are double */
};

typedef struct hofem_plan1d_s* hofem_plan1d;
typedef struct hofem_solver_s* hofem_solver;

/* Statistics of the last solve (filled when `info` is non-NULL). */
typedef struct {
  int iterations;          /* refinement / CG steps taken (0 for direct modes) */
  double rel_update;       /* ||last correction||_2 / ||u||_2 */
  double rel_residual;     /* ||f - L u||_2 / ||f||_2 (CG modes), else 0 */
} hofem_info;

/* Coefficient a(x) of -div(a grad u) + alpha u for hofem_pcg. */
typedef struct {
  int kind;                /* 0: a = 1 (the solver's own operator)
                              1: a(x) = c0 + c1 prod_i t_i(x_i), t_i tabulated
                              2: a tabulated at every Gauss point */
  double c0, c1;           /* kind 1 */
  const double* t_dev[3];  /* kind 1: t_i at the (n_i+1)-point Gauss nodes of every element
                              of axis i, index e_i (n_i+1) + q (K_i (n_i+1) values); the
                              nodes of an element in increasing order, i.e. the physical
                              points (e_i + (1 + xi_q) / 2) h_i with xi_q = table gx */
  const double* a_dev;     /* kind 2: index E (n+1)^N + Q with E the C-order index of the
                              element (e_0..e_{N-1}) and Q that of the Gauss point */
} hofem_coef;

/* ---- 1D eigen data (host) -------------------------------------------- */

/* Eigen data of the 1D pencil A v = lambda C v of eq. (eig_glob) for order
 * n and K elements (Section 2, paragraphs 1-3): the n roots of eq. (theta)
 * for every theta_k = cos(pi k / K), the vectors p_k^(l) of Lemma 2, the
 * norms ||s_k^(l)||_C^2 of the transform theorem, and the interior-node
 * eigenpairs of eq. (eig_elem).  Computed on the host in binary128 and
 * rounded once.  1 <= n <= 9 (simple element spectra are verified up to 9),
 * 2 <= K <= 1024, and nK - 1 <= 4095 when K is not a power of two.
 * Returns HOFEM_EUNSUPPORTED otherwise.  A plan changes only in hofem_plan1d_upload; otherwise it is
 * read-only and may be shared between threads. */
int hofem_plan1d_create(int n, int K, hofem_plan1d* out);

/* Boundary condition of an axis: the Introduction notes that other standard
 * conditions fit the method.  A periodic axis identifies x = 0 with x = X:
 * its m = nK unknowns are, for cell j = 0..K-1, the mesh node j (q = n j) and
 * the interior points s = 1..n-1 of element j+1 (q = n j + s).  The pencil is
 * then block circulant; its eigenvectors are Bloch waves w_{k,l} e^{i 2 pi k j/K}
 * with w_{k,l} (n complex values, w^H C_k w = 1) the eigenvectors of the n x n
 * Hermitian pencil of wave number k = 0..K/2 (K - k gives the conjugates).
 * Coefficients of a periodic axis are real, l-major: q = l K + t with t = 0
 * for k = 0, t = 2k-1 and 2k for the real and imaginary parts of k = 1..K/2-1,
 * t = K-1 for k = K/2; lambda_{k,l} is listed at every t of k.  Periodic axes
 * run in HOFEM_MODE_FP64 only (hofem_solve, hofem_forward, hofem_inverse;
 * K not a power of two: the dense transforms below);
 * every other entry point returns HOFEM_EUNSUPPORTED for a solver with a
 * periodic axis.  An all-periodic solver needs alpha > 0 (the constants have
 * lambda = 0): otherwise hofem_solver_create returns HOFEM_ENOTPOSDEF. */
enum hofem_bc { HOFEM_BC_DIRICHLET = 0, HOFEM_BC_PERIODIC = 1, HOFEM_BC_NEUMANN = 2 };

/* A Neumann axis (natural boundary conditions at x = 0 and x = X) holds the
 * m = nK + 1 values at the points g h / n, g = 0..nK, boundary nodes
 * included, in physical order.  Its eigenvectors follow Theorem 1 with
 * cosines for sines: for k = 1..K-1 and l = 1..n, node j: cos(pi k j / K),
 * point s of element e: cos(pi k (e-1)/K) p_s + cos(pi k e/K) p_{n-s}, with
 * the eigenvalue, p_k^(l) and norm ||s_k^(l)||_C^2 of the Dirichlet wave
 * number k (they satisfy the boundary rows because a boundary node belongs
 * to one element: its condensed diagonal is half the interior one).  The
 * other n + 1 are band-edge vectors: a cell (node a, interior values
 * w_1..w_{n-1}) repeated with the factor 1 (theta = 0; w_s = w_{n-s}) or
 * (-1)^j (theta = pi; w_s = -w_{n-s}), the eigenvectors of the cell pencil
 * restricted to those even cells, w^T C_cell w = 1 (so ||v||_C^2 = K).
 * The passes take DCT-I transforms of length K + 1 by K-point FFTs.
 * Coefficient order: q = (l-1)(K-1) + (k-1) for k = 1..K-1, then n(K-1) + b
 * for the band-edge vectors (b < n/2 + 1 at theta = 0, the rest at pi).
 * Neumann axes run in HOFEM_MODE_FP64 only (hofem_solve, hofem_forward,
 * hofem_inverse; K not a power of two: the dense transforms below, m <= 4095);
 * the other restrictions are those of periodic axes (a solver without a
 * Dirichlet axis needs alpha > 0). */

/* hofem_plan1d_create with a boundary condition (enum hofem_bc; else
 * HOFEM_EINVAL).  hofem_plan1d_create(n, K, out) is
 * hofem_plan1d_create_bc(n, K, HOFEM_BC_DIRICHLET, out). */
int hofem_plan1d_create_bc(int n, int K, int bc, hofem_plan1d* out);
void hofem_plan1d_destroy(hofem_plan1d plan);

/* Number of unknowns of the plan's axis: m = nK - 1 (Dirichlet), nK (periodic),
 * nK + 1 (Neumann). */
int hofem_plan1d_dim(hofem_plan1d plan, int* m);

/* Host copies of the plan's tables, for inspection and tests.  `which`:
 *   0  scaled eigenvalues lambda in coefficient order (m values)
 *   1  p_k^(l): index ((k-1) n + l-1) (n-1) + i          ((K-1) n (n-1) values)
 *   2  1 / ||s_k^(l)||_C^2: index (k-1) n + l-1          ((K-1) n values)
 *   3  e^(l) as columns: index i (n-1) + l-1              ((n-1)^2 values)
 *   4  local stiffness A on [-1, 1], row major           ((n+1)^2 values)
 *   5  local mass C on [-1, 1], row major                ((n+1)^2 values)
 *   6  nodes x_q of the (n+1)-point Gauss-Legendre rule, increasing (n+1 values)
 *   7  its weights w_q                                    (n+1 values)
 *   8  basis values e_r(x_q) at index q (n+1) + r         ((n+1)^2 values)
 *   9  basis derivatives e_r'(x_q) at index q (n+1) + r   ((n+1)^2 values)
 *  10  periodic plans: Re w_{k,l,s} at index (k n + l) n + s, k = 0..K/2 ((K/2+1) n^2)
 *  11  periodic plans: Im w_{k,l,s}, the same layout
 *  12  plans with K not a power of two: S, the unnormalised eigenvectors of
 *      Theorem 1 as columns in coefficient order, row major (m^2 values)
 *  13  the same plans: S diag(1 / ||s||_C^2) (1/K for the k = 0 columns)
 *  14  Neumann plans: the n + 1 band-edge cells (a, w_1..w_{n-1}) at index
 *      b n + s, theta = 0 first ((n+1) n values)
 * Tables 1 and 2 exist for Dirichlet and Neumann plans, 10 and 11 for
 * periodic plans only, 12 and 13 for dense ones, 14 for Neumann ones
 * (HOFEM_EINVAL otherwise); table 0 holds the m eigenvalues in the axis's
 * own coefficient order (periodic and Neumann orders above).
 *
 * K need not be a power of two for a Dirichlet or Neumann axis: with
 * m <= 4095 the plan then also holds S (columns in the axis's coefficient
 * order) and its scaled form, and the solver applies
 * them along that axis as dense products on the FP64 matrix cores (there is
 * no power-of-two FFT); an FP64 solve of such a solver takes a workspace of
 * one grid (hofem_solver_workspace_bytes), and only the FP64 solve, the
 * operators, the mass product and the Dirichlet lift accept it
 * (HOFEM_EUNSUPPORTED elsewhere).  The same holds for periodic axes
 * (m = nK <= 4095; the columns are the real and imaginary parts of the Bloch
 * waves, scaled as the periodic coefficients are) and Neumann axes.
 * The coefficient index of a line is q = l-1 for k = 0 (l = 1..n-1) and
 * q = (n-1) + (l-1)(K-1) + (k-1) for k = 1..K-1 (l = 1..n): for each l the
 * wave numbers are consecutive.  `len` must equal the count; otherwise
 * HOFEM_EINVAL. */
int hofem_plan1d_table(hofem_plan1d plan, int which, double* out_host, size_t len);

/* Bytes of the plan's device tables: the eigenvalues (FP64), the vectors
 * p_k^(l) with the norms 1/||s_k^(l)||_C^2 (FP64 and FP32, blocked by 64
 * wave numbers), e^(l), the FFT twiddles and sin(pi t/K) (FP64 and FP32),
 * the local matrices and the Gauss rule tables (FP64).  Under 2 MB for
 * n = 9, K = 1024.  A multiple of 256. */
int hofem_plan1d_table_bytes(hofem_plan1d plan, size_t* bytes);

/* Copies the plan's device tables into dev_buf (caller-owned device memory
 * on the current device, 256-byte aligned, at least
 * hofem_plan1d_table_bytes) and records it in the plan; returns after the
 * copy has completed (the call waits for `stream`).  dev_buf must stay
 * allocated and unchanged while any solver created from this plan is in use.
 * Uploading again re-targets the plan for solvers created afterwards.
 * HOFEM_EINVAL for a NULL or misaligned buffer or too few bytes. */
int hofem_plan1d_upload(hofem_plan1d plan, void* dev_buf, size_t bytes, void* stream);

/* ---- N-D solver (device) ---------------------------------------------- */

/* Solver for eq. (bvp glob 2) on (0,X_0) x ... x (0,X_{N-1}), 1 <= N <= 3,
 * with one plan per axis (plans[i] for axis i; the same plan may be used for
 * several axes) and the constant alpha.  Checks that every denominator
 * alpha + sum_i 4 h_i^-2 lambda_i is positive (the condition on alpha of
 * eq. (diff bvp pr2)), else HOFEM_ENOTPOSDEF.  Every plan must have been
 * uploaded (hofem_plan1d_upload) on the current device, else HOFEM_EINVAL;
 * the solver reads the tables in those device buffers.  The plan handles may
 * be destroyed after this call, their device buffers may not. */
int hofem_solver_create(int N, const hofem_plan1d* plans, const double* X, double alpha,
                        hofem_solver* out);
void hofem_solver_destroy(hofem_solver solver);

/* Total number of unknowns prod_i m_i of one right-hand side. */
int hofem_solver_size(hofem_solver solver, size_t* unknowns);

/* Workspace bytes that hofem_solve needs for `mode` and `nrhs`. */
int hofem_solver_workspace_bytes(hofem_solver solver, int mode, int nrhs, size_t* bytes);

/* Solve eq. (bvp glob 2) for nrhs right-hand sides by algorithm (a):
 * direct transforms along axes N-1..1, then along axis 0 the direct
 * transform, the division by alpha + sum_i 4 h_i^-2 lambda_i and the
 * inverse transform in one pass, then inverse transforms along axes 1..N-1.
 * Step (1) of algorithm (a) (the mass solve) is not performed: applying the
 * direct transforms to f^h itself gives the same coefficients, because the
 * transforms take y = C w as their input.
 * Mode HOFEM_MODE_FP64_B runs algorithm (b) of Section 2, paragraph 4
 * instead: direct transforms along axes 0..N-2, then along axis N-1 for
 * every combination of the other axes' modes the banded SPD system
 * (4 h^-2 A + mu C) v = phi of eq. (sys x1 2), mu = alpha + sum of the other
 * axes' 4 h_i^-2 lambda_i (static condensation of the element-interior
 * points, cyclic reduction of the mesh-node system), then inverse
 * transforms along axes N-2..0.  Same result, FP64, no workspace.
 *   f_dev, u_dev : [nrhs][m_0]..[m_{N-1}], double (FP64, FP32_IR) or float
 *                  (FP32).  u_dev == f_dev (in place) is allowed for FP64
 *                  and FP32, not for FP32_IR.
 *   ws_dev       : workspace of at least hofem_solver_workspace_bytes
 *                  (may be NULL when that is 0).
 *   max_iter,tol : FP32_IR only: at most max_iter refinement steps after the
 *                  first FP32 solve, stopping once ||delta||_2 <= tol ||u||_2
 *                  (tol <= 0: exactly max_iter steps).  Each step computes
 *                  the residual f^h - L u in FP64 with the stiffness in
 *                  difference form and adds the FP32 solve of it to u.
 *                  Returns HOFEM_ENOCONV (u holds the last iterate) when
 *                  tol > 0 and the tolerance was not reached; detecting
 *                  this needs `info` or tol > 0 (the call then waits).
 * Calls that overlap on one solver must use the same stream. */
int hofem_solve(hofem_solver solver, int mode, const void* f_dev, void* u_dev, int nrhs,
                void* ws_dev, size_t ws_bytes, int max_iter, double tol, void* stream,
                hofem_info* info);

/* With enable != 0, hofem_solve calls that do not synchronise (modes FP64,
 * FP32, FP64_B, and FP32_IR with tol <= 0; info NULL; a non-NULL stream)
 * run from a HIP graph: the first call of each mode runs eagerly, the next
 * one captures the whole solve (every pass and refinement step) and later
 * calls with the same mode, buffers, nrhs and max_iter replay it with one
 * graph launch.  Results do not depend on the setting.  A solve captured
 * into the graph records no timing events.  Off by default. */
int hofem_solver_set_graph(hofem_solver solver, int enable);

/* Direct F_n-transforms along every axis (step (2) of algorithm (a)):
 * out = coefficients w_{k l} of eq. (decomp phi 2) of C^-1 in, in coefficient
 * order per axis (see hofem_plan1d_table).  mode FP64 (double) or FP32
 * (float).  in_dev == out_dev allowed. */
int hofem_forward(hofem_solver solver, int mode, const void* in_dev, void* out_dev, int nrhs,
                  void* stream);

/* Inverse F_n-transforms along every axis (step (3) of algorithm (a)):
 * out = sum of coefficient * eigenvector products.  in_dev == out_dev allowed. */
int hofem_inverse(hofem_solver solver, int mode, const void* in_dev, void* out_dev, int nrhs,
                  void* stream);

/* Preconditioned conjugate gradients for -div(a grad u) + alpha u = f in the
 * scaled form of eq. (bvp glob 2) (the operator's stiffness part becomes
 * sum_i 4 h_i^-2 int a d_i u d_i phi on every element, by the (n+1)-point Gauss
 * rule per axis), preconditioned by the FP32 fast solve of the solver's own
 * constant-coefficient operator: the paper's use of the fast algorithm as a
 * preconditioner for general second-order elliptic equations (Section 1).
 * FP64 vectors, FP64 matrix-free operator (derivative factors in difference
 * form, applied first), deterministic reductions.  Starts from the FP32 fast
 * solve of f; stops when ||f - L u||_2 <= rtol ||f||_2 (rtol > 0) or after
 * max_iter steps; returns HOFEM_ENOCONV when rtol > 0 was not reached (u
 * holds the last iterate).  Waits for the stream once per step.
 * coef == NULL means kind 0.  f_dev, u_dev: [nrhs][m_0]..[m_{N-1}] double,
 * f_dev != u_dev; right-hand sides are solved one after another. */
int hofem_pcg_workspace_bytes(hofem_solver solver, const hofem_coef* coef, size_t* bytes);
int hofem_pcg(hofem_solver solver, const hofem_coef* coef, const double* f_dev, double* u_dev,
              int nrhs, double rtol, int max_iter, void* ws_dev, size_t ws_bytes, void* stream,
              hofem_info* info);

/* out = L_a u (f NULL) for the variable-coefficient operator of hofem_pcg
 * (FP64; needs hofem_pcg_workspace_bytes of workspace for kind 1 and 2). */
int hofem_apply_coef_operator(hofem_solver solver, const hofem_coef* coef, const double* u_dev,
                              double* out_dev, int nrhs, void* ws_dev, size_t ws_bytes,
                              void* stream);

/* Workspace bytes of hofem_apply_operator and hofem_apply_mass: for N = 3
 * with equal orders two grids of one right-hand side (the planes' stiffness
 * and mass products), 2 prod m_i doubles (rounded up to 256 bytes); with a
 * periodic or Neumann axis N - 1 grids of one right-hand side (each rounded
 * up to 256 bytes); 0 otherwise. */
int hofem_operator_workspace_bytes(hofem_solver solver, size_t* bytes);

/* out = L u with L the operator of eq. (bvp glob 2), FP64, matrix-free
 * (sum-factorised products of the 1D element matrices), the stiffness
 * factors in difference form sum_{l != k} A_kl (v_l - v_k) so that
 * constants are exactly in their kernel.  Any boundary conditions: with a
 * periodic or Neumann axis the products run one kernel per axis and term
 * (assembled along each axis from the local matrices, wrapping around on a
 * periodic axis, boundary nodes included on a Neumann axis).  u_dev !=
 * out_dev.  ws_dev: at least hofem_operator_workspace_bytes (may be NULL
 * when that is 0); HOFEM_EINVAL otherwise. */
int hofem_apply_operator(hofem_solver solver, const double* u_dev, double* out_dev, int nrhs,
                         void* ws_dev, size_t ws_bytes, void* stream);

/* out = ((x)_i C_i) g: the mass product of eq. (bvp glob 2), which turns
 * nodal values g of a function into the algebraic right-hand side f^h of
 * its FEM interpolant (f^h = C g along every axis, the load vector of the
 * interpolant divided by prod_i (h_i / 2)).  FP64, same kernels, layout and
 * workspace as hofem_apply_operator; g_dev != out_dev. */
int hofem_apply_mass(hofem_solver solver, const double* g_dev, double* out_dev, int nrhs,
                     void* ws_dev, size_t ws_bytes, void* stream);

/* Non-homogeneous Dirichlet data u = b on the boundary (Section 2,
 * paragraph 4: the general case reduces to zero data through a modified
 * f^h).  With g_b the FEM function that takes the values b at the boundary
 * grid points and 0 inside,
 *   out = f^h - (L g_b) at the interior points,
 * L the scaled operator of eq. (bvp glob 2) assembled with the boundary
 * points (element matrices sum_i 4 h_i^-2 A_i (x) C_others + alpha (x) C).
 * Solving L u_0 = out (any mode) gives the interior values of the solution;
 * on the boundary it is b.  b_ext_dev: the extended grid
 * [nrhs][m_0 + 2]..[m_{N-1} + 2] (double) of all grid points including the
 * boundary, in the same C order; only its boundary entries (index 0 or
 * m_i + 1 along some axis) are read.  f_dev: [nrhs][m_0]..[m_{N-1}] or NULL
 * (zero load); out_dev may equal f_dev, not b_ext_dev.  FP64. */
int hofem_dirichlet_rhs(hofem_solver solver, const double* b_ext_dev, const double* f_dev,
                        double* out_dev, int nrhs, void* stream);

/* ---- implicit time stepping -------------------------------------------- */

/* Implicit time stepping with the fast solve, the use the paper names for
 * time-dependent problems (Section 1; Section 2, paragraph 4).  Each step is
 * one system of eq. (bvp glob 2) of the stepper's solver, whose alpha carries
 * the time step dt:
 *   HOFEM_SCHEME_HEAT  u_t - Lap u = f, backward Euler, alpha = 1/dt:
 *                      L u^{n+1} = f^h + alpha ((x)_i C_i) u^n
 *   HOFEM_SCHEME_WAVE  u_tt - Lap u = f, the implicit three-level scheme
 *                      (u^{n+1} - 2u^n + u^{n-1})/dt^2 - Lap u^{n+1} = f,
 *                      alpha = 1/dt^2:
 *                      L u^{n+1} = f^h + alpha ((x)_i C_i)(2u^n - u^{n-1})
 * A step is one mass product (by the operator kernels, or one kernel per
 * axis when an axis is periodic or Neumann) and one FP64 solve by algorithm
 * (a) (plus one vector kernel for the wave scheme).  Any boundary conditions
 * of enum hofem_bc; axes whose K is not a power of two are refused
 * (HOFEM_EUNSUPPORTED). */
enum hofem_scheme { HOFEM_SCHEME_HEAT = 0, HOFEM_SCHEME_WAVE = 1 };

typedef struct hofem_stepper_s* hofem_stepper;

/* A stepper for `solver` (alpha > 0, else HOFEM_EINVAL).  The solver must
 * outlive the stepper. */
int hofem_stepper_create(hofem_solver solver, int scheme, hofem_stepper* out);
void hofem_stepper_destroy(hofem_stepper stepper);

/* Workspace of hofem_stepper_run for nrhs right-hand sides: one FP64 grid
 * (two for the wave scheme) and the operator's workspace (with a periodic or
 * Neumann axis in 2D and 3D: one more grid instead). */
int hofem_stepper_workspace_bytes(hofem_stepper stepper, int nrhs, size_t* bytes);

/* Advances u_dev (in: u^n, out: u^{n+nsteps}) by nsteps steps.  f_dev: the
 * load f^h, constant in time ([nrhs][grid] double), or NULL for zero.
 * uprev_dev: the wave scheme's previous level (in: u^{n-1}, out:
 * u^{n+nsteps-1}; unused and may be NULL for the heat scheme).  u_dev,
 * uprev_dev and f_dev must be distinct.  use_graph != 0 and a non-NULL
 * stream: the first step of the first call runs eagerly, then one step is
 * captured into a HIP graph (once per set of buffers and nrhs) and replayed
 * for the remaining steps; results do not depend on use_graph.  Calls on one
 * stepper must not overlap. */
int hofem_stepper_run(hofem_stepper stepper, const double* f_dev, double* u_dev,
                      double* uprev_dev, int nrhs, int nsteps, void* ws_dev, size_t ws_bytes,
                      int use_graph, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hofem_solve
 * in mode HOFEM_MODE_FP32_IR (f_dev, u_dev double, f_dev != u_dev; max_iter,
 * tol, info as there) with its workspace taken from a scratch buffer of
 * 64 MiB that the library holds in device memory, one per device, from the
 * library's load until the process ends.  The problem must fit it:
 * hofem_solver_workspace_bytes(solver, HOFEM_MODE_FP32_IR, nrhs) <= 64 MiB
 * (the FP32 residual grid of nrhs right-hand sides, 16 KB of norm partials
 * and, in 3D with equal orders, the operator's two plane-product grids; about 16
 * million unknowns in all), else HOFEM_ETOOBIG before any work.  Allocates
 * nothing and records no timing events.  Every call on a device shares that
 * device's scratch: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.  The scratch keeps the
 * last call's contents; each call writes every scratch byte it reads. */
int hofem_solve_ir_noalloc(hofem_solver solver, const double* f_dev, double* u_dev, int nrhs,
                           int max_iter, double tol, void* stream, hofem_info* info);

/* ---- batched form -------------------------------------------------------- */

/* One problem of a batch: the solver of its operator and its number of
 * right-hand sides.  Problems that share a solver handle and nrhs form a
 * group that is solved by one batched launch per pass, so a caller with many
 * problems of few distinct (orders, K, box, alpha) should create one solver
 * per distinct operator and reuse the handle. */
typedef struct {
  hofem_solver solver;
  int nrhs;
} hofem_batch_problem;

typedef struct hofem_batch_s* hofem_batch;

/* Groups `count` problems (the batched form of algorithm (a) over many
 * independent problems) and fixes the packed device layout of their
 * right-hand sides and solutions: problem p occupies nrhs * prod m_i values
 * of one packed buffer from offsets[p] on, [nrhs][m_0]..[m_{N-1}] (see
 * hofem_batch_offsets; problems that share a group are adjacent).  The solvers must outlive
 * the batch.  Creates kSideStreams = 4 HIP streams (default priority) and
 * events on the current device; HOFEM_EINVAL for a NULL solver or nrhs < 1. */
int hofem_batch_create(const hofem_batch_problem* probs, int count, hofem_batch* out);
void hofem_batch_destroy(hofem_batch batch);

/* out_host[0..count-1] = value offset of each problem in the packed layout,
 * out_host[count] = total values.  len must equal count + 1. */
int hofem_batch_offsets(hofem_batch batch, size_t* out_host, size_t len);

/* Number of groups (distinct (solver, nrhs) pairs). */
int hofem_batch_groups(hofem_batch batch, int* groups);

/* Device workspace for hofem_batch_solve in `mode` (FP64, FP32 or FP32_IR):
 * the sum of the groups' hofem_solver_workspace_bytes (0 for the direct
 * modes unless a group's solver has an axis whose K is not a power of two).
 * Every group runs hofem_solve on its slab, so each mode accepts the solvers
 * hofem_solve accepts in it (FP64: any boundary conditions and K). */
int hofem_batch_workspace_bytes(hofem_batch batch, int mode, size_t* bytes);

/* Solves every problem of the batch: f_dev, u_dev are packed buffers (double
 * for FP64 and FP32_IR, float for FP32), f_dev != u_dev for FP32_IR, which
 * runs exactly max_iter refinement steps (no tolerance test, no host
 * synchronisation).  use_graph != 0: the first call per mode runs eagerly;
 * later calls capture the whole batch once into a HIP graph (groups on
 * forked streams, joined back into `stream`) and replay it while mode,
 * buffers and max_iter stay the same (stream NULL, the legacy default
 * stream, always runs eagerly).  Results do not depend on use_graph.
 * Calls on one batch must not overlap. */
int hofem_batch_solve(hofem_batch batch, int mode, const void* f_dev, void* u_dev, void* ws_dev,
                      size_t ws_bytes, int max_iter, int use_graph, void* stream);

/* ---- per-pass timing (profiling aid) ----------------------------------- */

/* Kinds of device work the solver enqueues. */
enum hofem_pass_kind {
  HOFEM_PASS_FORWARD = 0,   /* direct transform along one axis */
  HOFEM_PASS_INVERSE = 1,   /* inverse transform along one axis */
  HOFEM_PASS_FUSED = 2,     /* direct transform, division, inverse transform */
  HOFEM_PASS_OPERATOR = 3,  /* FP64 residual / operator apply */
  HOFEM_PASS_UPDATE = 4,    /* refinement update and norms */
  HOFEM_PASS_BANDED = 5     /* banded solves of algorithm (b) along one axis */
};

typedef struct {
  int kind;                 /* hofem_pass_kind */
  int axis;                 /* axis of a transform pass, -1 otherwise */
  int fp64;                 /* 1: FP64 arithmetic, 0: FP32 */
  long long launches;       /* launches recorded since the last read */
  double ms;                /* their summed duration (HIP events, milliseconds) */
  double bytes;             /* algorithmic bytes of one launch: one read and one
                               write of every value the pass streams */
} hofem_pass_time;

/* When enabled, every kernel launch of this solver is bracketed by HIP events
 * recorded on the call's stream (event objects only: no device allocation).
 * At most 4096 launches are recorded between two reads; later launches are
 * not timed. */
int hofem_solver_set_timing(hofem_solver solver, int enable);

/* Waits for the recorded events, writes up to `max_entries` aggregates (one
 * per kind, axis and precision, in first-launch order) to out_host, sets
 * *count to their number and clears the record. */
int hofem_solver_pass_times(hofem_solver solver, hofem_pass_time* out_host, int max_entries,
                            int* count);

/* ---- autotuner of the line passes' launch shapes ------------------------- */

/* A pass's launch shape: lines per workgroup and workgroup size. */
typedef struct {
  int kind;             /* HOFEM_PASS_FORWARD, _INVERSE or _FUSED */
  int axis;
  int fp64;             /* 1: FP64 pass, 0: FP32 */
  int cb;               /* lines per workgroup */
  int threads;          /* lanes per workgroup (256 or 512) */
  long long nlines;     /* lines of the pass it was tuned for (0: forced) */
  double ms_default;    /* one solve with the default shape (ms) */
  double ms_tuned;      /* one solve with the chosen shape (ms) */
} hofem_tune_entry;

/* Launch shapes the pass (kind, axis, precision) of a solve of nrhs
 * right-hand sides can run with, the default first: out to cb_host /
 * threads_host (at most max_entries), their number to *count.  Every shape
 * gives the same result up to rounding order. */
int hofem_pass_shape_candidates(hofem_solver solver, int kind, int axis, int fp64, int nrhs,
                                int* cb_host, int* threads_host, int max_entries, int* count);

/* Forces a shape on one pass of this solver (cb = 0: back to the default).
 * A shape the pass cannot run makes later solves fail with HOFEM_EHIP. */
int hofem_pass_set_shape(hofem_solver solver, int kind, int axis, int fp64, int cb, int threads);

/* Autotunes the launch shapes of the passes of `mode` (FP64, FP32 or
 * FP32_IR) for nrhs right-hand sides, one pass after another: every
 * candidate shape is timed over `reps` whole solves (HIP events on `stream`;
 * one refinement step for FP32_IR) on the given buffers and workspace, and
 * the fastest is kept for the solver's later solves.  Waits for the stream.
 * Reports one entry per pass (at most max_entries) and their number. */
int hofem_solver_autotune(hofem_solver solver, int mode, const void* f_dev, void* u_dev, int nrhs,
                          void* ws_dev, size_t ws_bytes, int reps, void* stream,
                          hofem_tune_entry* out_host, int max_entries, int* count);

/* Tuning cache on disk (text, one line per tuned pass, keyed by the kernel
 * build's hash, n, K, precision, pass kind, stride and line count): save
 * merges the solver's tuned shapes into `path`; load applies the matching
 * entries for a solve of `mode` with nrhs right-hand sides (*applied: how
 * many; a missing file applies none).  reset drops every tuned or forced
 * shape. */
int hofem_solver_tune_save(hofem_solver solver, const char* path);
int hofem_solver_tune_load(hofem_solver solver, const char* path, int mode, int nrhs, int* applied);
int hofem_solver_tune_reset(hofem_solver solver);

/* Hash of the line-pass kernel sources this library was built from. */
const char* hofem_kernel_hash(void);

/* Human-readable name of a status code (static string). */
const char* hofem_status_string(int status);

/* hipError_t of the last failed HIP call in this thread (0 if none). */
int hofem_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HOFEM_H */
