// Internal interface between the solver (capi.hip) and the device kernels
// (line passes in linepass.h / linepass.hip, operators in operator.hip,
// vector kernels in pcg.hip).  Plain structs of device pointers and sizes.
#pragma once

#include <hip/hip_runtime.h>

namespace hofem {

// Records e as the thread's last HIP error (hofem_last_hip_error) and
// returns HOFEM_EHIP.
int record_hip_error(hipError_t e);

// Device tables of one axis in one precision (T = float or double).
//
// Coefficient order of a line (m = nK - 1 entries): q = l-1 for the k = 0
// modes (l = 1..n-1), q = (n-1) + (l-1)(K-1) + (k-1) for k = 1..K-1 and
// l = 1..n, i.e. for each l the wave numbers k are consecutive.
//
// The per-wave-number tables are blocked by 64 wave numbers (one wavefront)
// and hold their entries in groups of g = 16 bytes / element size (pairs in
// FP64, quadruples in FP32): entry e of wave number k sits at
// (((k-1)/64 * NEG + e/g) * 64 + (k-1) % 64) * g + e % g with NE = n(n-1) + n,
// NEG = ceil(NE / g), e = (l-1)(n-1) + (i-1) for component i of p_k^(l) and
// e = n(n-1) + l-1 for 1 / ||s_k^(l)||^2, so that a wavefront handling 64
// consecutive k reads g entries per lane with one 16-byte load, 64
// consecutive groups.
struct AxisTab {
  const void* blk;     // blocked p and 1/||s||^2 (T)
  const void* E;       // e^(l) columns, i (n-1) + l-1
  const void* tw;      // cos, sin (2 pi t / K) interleaved, t < K
  const void* sn;      // sin(pi t / K), t < K
  const double* lam;   // scaled eigenvalues in coefficient order (FP64)
  int n, K, m;
  const double* band;  // Neumann axes: the n + 1 band-edge vectors (cells of n values)
};

// PASS_INV_ACC: the inverse pass adding its result to a double output
// (FP32 compute, float in; a refinement step's correction).
enum PassKind { PASS_FWD = 0, PASS_INV = 1, PASS_FUSED = 2, PASS_INV_ACC = 5 };

// Arguments of one line pass along one axis of a C-order grid.
struct PassArgs {
  const void* in;
  void* out;
  AxisTab tab;
  long long inner;     // stride of the axis (product of the later extents)
  long long nlines;    // number of lines (total elements / m)
  int cb;              // lines per workgroup (set by the launcher)
  // requested launch shape (the autotuner's candidates): lines per
  // workgroup and workgroup size, 0 = the default of shape_for; a request
  // the kernel cannot run is refused with hipErrorInvalidValue
  int cb_req, threads_req;
  // Row-pair interleaved intermediate of a 2D solve: the first ilv rows of
  // the grid (an even count; rows of all right-hand sides in sequence) are
  // stored in pairs, row 2g + h of column t at 2g * M1 + 2t + h, the rest
  // plain.  A pass along the rows then moves its two lines as one
  // contiguous block, a pass along the columns moves 32 bytes (FP64) per
  // row pair instead of 16 per row.  ilv_in / ilv_out: for the input /
  // output, 0 = plain.  Along the rows (inner == 1) only with two lines per
  // workgroup, and ilv_out only in the forward pass; along the columns
  // ilv_out only in the passes that end with the scatter.
  long long ilv_in;
  long long ilv_out;
  // Denominator of the fused pass: alpha + scale * lam[q] + sum over the
  // other axes of oscale[i] * olam[i][(t / odiv[i]) % omod[i]], t = line % inner.
  double alpha;
  double scale;
  int nother;
  const double* olam[2];
  double oscale[2];
  long long odiv[2];
  long long omod[2];
};

// Per-order launchers, each defined in its own translation unit.
template <int N>
hipError_t launch_pass_order(int kind, int dt, const PassArgs& a, hipStream_t s);
template <> hipError_t launch_pass_order<1>(int, int, const PassArgs&, hipStream_t);
template <> hipError_t launch_pass_order<2>(int, int, const PassArgs&, hipStream_t);
template <> hipError_t launch_pass_order<3>(int, int, const PassArgs&, hipStream_t);
template <> hipError_t launch_pass_order<4>(int, int, const PassArgs&, hipStream_t);
template <> hipError_t launch_pass_order<5>(int, int, const PassArgs&, hipStream_t);
template <> hipError_t launch_pass_order<6>(int, int, const PassArgs&, hipStream_t);
template <> hipError_t launch_pass_order<7>(int, int, const PassArgs&, hipStream_t);
template <> hipError_t launch_pass_order<8>(int, int, const PassArgs&, hipStream_t);
template <> hipError_t launch_pass_order<9>(int, int, const PassArgs&, hipStream_t);

// Launch one pass.  dt: 0 = FP64 compute (double in/out),
// 1 = FP32 compute with float in/out, 2 = FP32 compute, double in, float out,
// 3 = FP32 compute, float in, double out (stored), 4 = FP32 compute, float
// in, double out accumulated (out += result), 5 = FP32 compute, double in,
// double out (stored).
hipError_t launch_pass(int kind, int dt, const PassArgs& a, hipStream_t s);
// Lines per workgroup of a pass along a contiguous axis of order n with K
// elements and nlines lines.
int pass_lines_per_workgroup(int n, int K, bool f64, long long nlines);
// Launch shapes a pass of order n, K can run with (lines per workgroup,
// workgroup size), the default first; at most `max` of them.
int pass_shape_candidates(int n, int K, bool f64, long long nlines, bool one_line, int* cb,
                          int* threads, int max);

// FP64 matrix-free operator r = f - L u (f may be NULL: r = L u), N = 1..3.
struct OpArgs {
  const double* u;
  const double* f;
  void* out;           // double (out_f32 == 0) or float (out_f32 == 1)
  int out_f32;
  int N;
  int n[3], K[3], m[3];
  double scale[3];     // 4 h_i^-2
  double alpha;
  const double* A[3];  // local stiffness (n_i+1)^2, device
  const double* C[3];  // local mass (n_i+1)^2, device
  const double* hA[3]; // the same, host copies (passed by value to kernels)
  const double* hC[3];
  int nrhs;
  // 3D with equal orders: two grids of one right-hand side (the planes' 2D
  // mass products and operators; op3_elem_doubles), device
  double* elem;
};
hipError_t launch_operator(const OpArgs& a, hipStream_t s);
// Element buffer the 3D operator needs (0 when it needs none).
size_t op3_elem_doubles(const OpArgs& a);
// out = f - (L_ext b)|interior for Dirichlet values b on the extended grid
// [nrhs][m_0+2]..[m_{N-1}+2] (f may be NULL).
hipError_t launch_dirichlet_lift(const OpArgs& a, const double* bext, const double* f,
                                 double* out, hipStream_t s);

// Banded solves of algorithm (b) along the contiguous axis: every line L
// (nlines of them, m = nK - 1 values each, contiguous) solves
// (scale A + mu C) v = in with mu = alpha + sum_i oscale[i] *
// olam[i][(t / odiv[i]) % omod[i]], t = L % others; in == out allowed.
struct BandArgs {
  const double* in;
  double* out;
  int n, K, m;
  double scale;
  const double* A;     // local stiffness (n+1)^2, device
  const double* C;     // local mass (n+1)^2, device
  long long nlines;
  long long others;    // lines per right-hand side
  double alpha;
  int nother;
  const double* olam[2];
  double oscale[2];
  long long odiv[2];
  long long omod[2];
};
hipError_t launch_banded(const BandArgs& a, hipStream_t s);

// Line passes along periodic axes (FP64; kind PASS_FWD, PASS_INV or
// PASS_FUSED): tab.blk holds the Bloch eigenvectors w_{k,l,s} (complex FP64,
// index (k n + l) n + s, k = 0..K/2), tab.tw the twiddles, tab.lam the
// eigenvalues in the periodic coefficient order.
hipError_t launch_periodic(int kind, const PassArgs& a, hipStream_t s);

// Line passes along Neumann axes (FP64; kind PASS_FWD, PASS_INV or
// PASS_FUSED).  A line holds the m = nK + 1 values of the axis (node j at
// q = n j, j = 0..K; interior point s of element e at q = n (e-1) + s);
// coefficients in the Neumann order q = (l-1)(K-1) + (k-1) for k = 1..K-1,
// then n(K-1) + b for the band-edge vectors b = 0..n.  tab: the Dirichlet
// tables of (n, K) (blocked p and 1/||s||^2, twiddles, sines), tab.lam the
// eigenvalues in the Neumann order, tab.band the band-edge vectors.
hipError_t launch_neumann(int kind, const PassArgs& a, hipStream_t s);

// C_b = op(A_b) op(B_b) in FP64 on the matrix cores (dense transforms of
// axes whose K is not a power of two): row-major M x K, K x N, M x N after
// op, op = transpose when ta / tb; b = 0..batch-1 with element strides
// sa, sb, sc.
struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  long long lda, ldb, ldc;
  long long sa, sb, sc, batch;
};
hipError_t launch_dgemm(const GemmArgs& g, bool ta, bool tb, hipStream_t s);
// x[o][q][t] /= a.alpha + a.scale a.tab.lam[q] + the other axes' terms (as
// in the fused pass), x of shape [outer][m][inner].
hipError_t launch_dense_divide(double* x, long long outer, int m, long long inner, const PassArgs& a,
                               hipStream_t s);

// u += delta over `count` elements with per-workgroup partial sums of
// delta^2 and u^2 (nparts workgroups), reduced to out[0..1] by a second
// launch (fixed order: deterministic).
hipError_t launch_norms(const float* delta, double* u, long long count, double* partial,
                        int nparts, double* out, hipStream_t s);

// u += (double) delta, elementwise.
hipError_t launch_axpy(const float* delta, double* u, long long count, hipStream_t s);

// FP64 variable-coefficient operator out = f - L_a u (or L_a u when f is NULL).
struct VarOpArgs {
  const double* u;
  const double* f;
  double* out;
  int N;
  int n[3], K[3];
  long long stride[3];   // grid strides of a right-hand side
  long long per_rhs;
  int nrhs;
  double scale[3];       // 4 h_i^-2
  double alpha;
  const double* B[3];    // e_r(x_q), (n+1)^2
  const double* D[3];    // e_r'(x_q), (n+1)^2
  const double* Dh[3];   // differentiation on the Gauss nodes, (n+1)^2
  const double* w[3];    // Gauss weights, n+1
  int kind;              // 0: a = 1, 1: a = c0 + c1 prod_i t_i, 2: a at every Gauss point
  double c0, c1;
  const double* t[3];    // kind 1: t_i at [element][q], K_i (n_i+1) values
  const double* afull;   // kind 2: [element][q_0..q_{N-1}]
};
size_t varop_elem_bytes(const VarOpArgs& a);
hipError_t launch_varop(const VarOpArgs& a, double* elem_buf, hipStream_t s);

// PCG vector kernels (np partial sums, reduced in a fixed order).
hipError_t launch_dot2(const double* x, const double* y, const double* z, long long n,
                       double* partial, int np, double* out2, hipStream_t s);
hipError_t launch_cg_update(double* x, double* r, const double* p, const double* q,
                            const double* z, long long n, const double* scal, double* partial,
                            int np, double* out2, double* out1, hipStream_t s);
hipError_t launch_cg_dir(double* p, const double* z, long long n, const double* scal,
                         hipStream_t s);
// scal[0] = scal[2] / scal[3] (op 0: alpha = rz / pq);
// scal[1] = scal[5] / scal[2], scal[2] = scal[5] (op 1: beta, rz <- rz_new)
hipError_t launch_scalar_op(double* scal, int op, hipStream_t s);
// records a step's statistics and the first converged step (scal[16..19, 32..63])
hipError_t launch_cg_record(double* scal, hipStream_t s);
// sets the convergence thresholds (scal[16..19]) from ||f||^2 in scal[9]
hipError_t launch_cg_init(double* scal, double rtol, double utol, hipStream_t s);

}  // namespace hofem
