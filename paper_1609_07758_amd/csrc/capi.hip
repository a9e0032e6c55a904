// C ABI of the solver: plans, device tables, pass schedule, refinement loop.
//
// Pass schedule of algorithm (a) (Section 2, paragraph 4) for N axes
// (axis N-1 contiguous): direct transforms along N-1, ..., 1; along axis 0
// one fused pass (direct transform, division by alpha + sum_i 4 h_i^-2
// lambda_i, inverse transform); inverse transforms along 1, ..., N-1.  Each
// pass reads and writes the grid once.  Step (1) of the algorithm (the mass
// solve) is not needed: the direct transform takes y = C w as its input, and
// f^h is exactly that y for w = phi^h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <mutex>
#include <new>
#include <vector>

#include "hofem.h"
#include "kernels.h"
#include "plan1d.h"
#include "solver.h"

using namespace hofem;

// Byte offsets of one plan's tables in its device image (256-byte aligned).
struct PlanOff {
  size_t lam, blk64, E64, tw64, sn64, blk32, E32, tw32, sn32, A, C, B, D, Dh, gw;
  size_t S = 0, St = 0;   // dense axes (K not a power of two)
  size_t band = 0;        // Neumann axes: band-edge vectors
};

struct hofem_plan1d_s {
  Plan1DData d;
  std::vector<unsigned char> image;   // device table image, built at creation
  PlanOff off{};
  const unsigned char* dev = nullptr; // the image in the caller's device buffer
  int device = -1;                    // device of that buffer
};

namespace {

thread_local int g_last_hip = 0;
// Set while an entry point that must not allocate runs: no timing events.
thread_local bool g_no_events = false;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return HOFEM_EHIP;
}

}  // namespace

int hofem::record_hip_error(hipError_t e) { return hip_fail(e); }

namespace {

#define HIPCHK(x)                               \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return hip_fail(e_);  \
  } while (0)

struct DevAxis {
  int bc = 0;                   // 0: Dirichlet, 1: periodic, 2: Neumann
  // order, elements and unknowns of the axis (nK - 1, nK, nK + 1)
  int n = 0, K = 0, m = 0;
  // K not a power of two: transforms by the dense matrices S (inverse) and
  // St = S diag(1 / ||s||^2) (forward: St^T y)
  int dense = 0;
  const double* S = nullptr;
  const double* St = nullptr;
  double X = 0, scale = 0;
  AxisTab t64{}, t32{};
  const double* A = nullptr;
  const double* C = nullptr;
  std::vector<double> hA, hC;   // host copies of A and C (kernel arguments)
  const double* B = nullptr;    // basis values at the Gauss nodes
  const double* D = nullptr;    // basis derivatives at the Gauss nodes
  const double* Dh = nullptr;   // differentiation on the Gauss nodes
  const double* gw = nullptr;   // Gauss weights
};

// Packs host arrays into one byte buffer with 256-byte aligned offsets.
struct Packer {
  std::vector<unsigned char> bytes;
  size_t add(const void* src, size_t n) {
    size_t off = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(off + std::max<size_t>(n, 8), 0);
    if (n) std::memcpy(bytes.data() + off, src, n);
    return off;
  }
  size_t add_f64(const std::vector<double>& v) { return add(v.data(), v.size() * sizeof(double)); }
  size_t add_f32(const std::vector<double>& v) {
    std::vector<float> f(v.size());
    for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
    return add(f.data(), f.size() * sizeof(float));
  }
};

constexpr int kNormParts = 1024;

}  // namespace

struct TimedLaunch {
  int kind, axis, fp64;
  double bytes;
  hipEvent_t start, stop;
};

struct hofem_solver_s {
  int N = 0;
  double alpha = 0;
  int device = 0;
  DevAxis ax[3];
  size_t per_rhs = 0;   // unknowns of one right-hand side
  double* dense_tmp = nullptr;   // scratch grid of the dense passes (set per solve)
  // per-pass timing
  bool timing = false;
  std::vector<hipEvent_t> event_pool;
  std::vector<TimedLaunch> records;
  // launch shapes chosen by the autotuner (or forced), per (kind, axis, fp64)
  std::vector<hofem_tune_entry> tune;
  // HIP-graph replay of whole solves (hofem_solver_set_graph): one graph for
  // the last (mode, buffers, nrhs, steps); modes run eagerly once first
  bool use_graph = false;
  bool capturing = false;
  bool warm[8] = {false, false, false, false, false, false, false, false};
  hipGraphExec_t exec = nullptr;
  int g_mode = -1, g_nrhs = 0, g_iter = -1;
  const void* g_f = nullptr;
  void* g_u = nullptr;
  void* g_ws = nullptr;
};

namespace {

constexpr size_t kMaxRecords = 4096;

// Brackets one launch with events when timing is enabled.
struct LaunchTimer {
  hofem_solver_s* S;
  hipStream_t st;
  TimedLaunch rec{};
  bool on = false;
  LaunchTimer(hofem_solver_s* s, hipStream_t stream, int kind, int axis, int fp64, double bytes)
      : S(s), st(stream) {
    if (g_no_events || S->capturing || !S->timing || S->records.size() >= kMaxRecords) return;
    const size_t need = 2 * (S->records.size() + 1);
    while (S->event_pool.size() < need) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      S->event_pool.push_back(e);
    }
    rec = TimedLaunch{kind, axis, fp64, bytes, S->event_pool[need - 2], S->event_pool[need - 1]};
    on = hipEventRecord(rec.start, st) == hipSuccess;
  }
  void done() {
    if (on && hipEventRecord(rec.stop, st) == hipSuccess) S->records.push_back(rec);
    on = false;
  }
};

// il_in / il_out: the pass reads / writes the row-pair interleaved 2D
// intermediate (PassArgs::ilv_in / ilv_out).
struct PassSpec {
  int axis, kind;
  bool il_in = false, il_out = false;
};

PassArgs make_args(const hofem_solver_s* S, int axis, int kind, bool f64, const void* in, void* out,
                   int nrhs) {
  PassArgs a{};
  a.in = in;
  a.out = out;
  const DevAxis& X = S->ax[axis];
  a.tab = f64 ? X.t64 : X.t32;
  long long inner = 1, others = 1;
  for (int i = 0; i < S->N; ++i) {
    if (i > axis) inner *= S->ax[i].m;
    if (i != axis) others *= S->ax[i].m;
  }
  a.inner = inner;
  a.nlines = others * nrhs;
  if (kind == PASS_FUSED) {
    a.alpha = S->alpha;
    a.scale = X.scale;
    a.nother = 0;
    for (int i = 0; i < S->N; ++i) {
      if (i == axis) continue;
      long long div = 1;
      for (int j = i + 1; j < S->N; ++j)
        if (j != axis) div *= S->ax[j].m;
      a.olam[a.nother] = S->ax[i].t64.lam;
      a.oscale[a.nother] = S->ax[i].scale;
      a.odiv[a.nother] = div;
      a.omod[a.nother] = S->ax[i].m;
      ++a.nother;
    }
  }
  return a;
}

// A pass along an axis whose K is not a power of two: the transforms are the
// dense products with St^T (forward) and S (inverse) on the matrix cores;
// the fused pass divides in between.  In place through the solver's dense
// scratch grid.
int dense_pass(hofem_solver_s* S, int axis, int kind, const PassArgs& a, const void* in, void* out,
               hipStream_t st) {
  const DevAxis& X = S->ax[axis];
  const int m = X.m;
  const long long inner = a.inner, outer = a.nlines / inner;
  double* tmp = S->dense_tmp;
  if (!tmp) return HOFEM_EINVAL;
  auto apply = [&](const double* src, double* dst, bool fwd) -> hipError_t {
    GemmArgs g{};
    g.K = m;
    if (inner == 1) {
      // rows: dst (outer x m) = src St (forward) or src S^T (inverse)
      g.A = src;
      g.B = fwd ? X.St : X.S;
      g.C = dst;
      g.M = (int)outer;
      g.N = m;
      g.lda = g.ldb = g.ldc = m;
      g.batch = 1;
      return launch_dgemm(g, false, !fwd, st);
    }
    // strided: per block o of the outer axes, dst_o (m x inner) = St^T src_o or S src_o
    g.A = fwd ? X.St : X.S;
    g.B = src;
    g.C = dst;
    g.M = m;
    g.N = (int)inner;
    g.lda = m;
    g.ldb = g.ldc = inner;
    g.sb = g.sc = (long long)m * inner;
    g.batch = outer;
    return launch_dgemm(g, fwd, false, st);
  };
  if (outer > 0x7fffffffLL || inner > 0x7fffffffLL) return HOFEM_EUNSUPPORTED;
  const double* src = static_cast<const double*>(in);
  double* dst = static_cast<double*>(out);
  const size_t bytes = (size_t)outer * m * inner * sizeof(double);
  if (kind == PASS_FUSED) {
    HIPCHK(apply(src, tmp, true));
    HIPCHK(launch_dense_divide(tmp, outer, m, inner, a, st));
    HIPCHK(apply(tmp, dst, false));
  } else if (src != dst) {
    HIPCHK(apply(src, dst, kind == PASS_FWD));
  } else {
    HIPCHK(apply(src, tmp, kind == PASS_FWD));
    HIPCHK(hipMemcpyAsync(dst, tmp, bytes, hipMemcpyDeviceToDevice, st));
  }
  return HOFEM_OK;
}

// Runs a list of passes: the first reads in0, the last writes outl, the
// others work in place on buf.  dt codes as in launch_pass.
int run_list(hofem_solver_s* S, const std::vector<PassSpec>& list, bool f64, const void* in0,
             void* buf, void* outl, int dt_first, int dt_mid, int dt_last, int dt_single, int nrhs,
             hipStream_t st) {
  for (size_t i = 0; i < list.size(); ++i) {
    const void* in = (i == 0) ? in0 : buf;
    void* out = (i + 1 == list.size()) ? outl : buf;
    int dt;
    if (list.size() == 1) dt = dt_single;
    else if (i == 0) dt = dt_first;
    else if (i + 1 == list.size()) dt = dt_last;
    else dt = dt_mid;
    PassArgs a = make_args(S, list[i].axis, list[i].kind, f64, in, out, nrhs);
    if (a.nlines == 0) continue;
    const int tkind = list[i].kind == PASS_INV_ACC ? PASS_INV : list[i].kind;
    for (const hofem_tune_entry& t : S->tune) {
      if (t.kind == tkind && t.axis == list[i].axis && t.fp64 == (f64 ? 1 : 0)) {
        a.cb_req = t.cb;
        a.threads_req = t.threads;
      }
    }
    if (list[i].il_in || list[i].il_out) {
      const long long rows = ((long long)S->ax[0].m * nrhs) & ~1LL;
      if (list[i].il_in) a.ilv_in = rows;
      if (list[i].il_out) a.ilv_out = rows;
    }
    static const int in_bytes[6] = {8, 4, 8, 4, 4, 8}, out_bytes[6] = {8, 4, 4, 8, 16, 8};
    const double bytes = (double)S->per_rhs * nrhs * (in_bytes[dt] + out_bytes[dt]);
    LaunchTimer tm(S, st, list[i].kind == PASS_INV_ACC ? PASS_INV : list[i].kind, list[i].axis,
                   f64 ? 1 : 0, bytes);
    if (S->ax[list[i].axis].dense) {
      if (dt != 0) return HOFEM_EUNSUPPORTED;   // dense axes: FP64 passes only
      const int rc = dense_pass(S, list[i].axis, list[i].kind, a, in, out, st);
      if (rc != HOFEM_OK) return rc;
    } else if (S->ax[list[i].axis].bc != 0) {
      if (dt != 0) return HOFEM_EUNSUPPORTED;   // periodic / Neumann axes: FP64 passes only
      if (S->ax[list[i].axis].bc == 1) HIPCHK(launch_periodic(list[i].kind, a, st));
      else HIPCHK(launch_neumann(list[i].kind, a, st));
    } else {
      HIPCHK(launch_pass(list[i].kind, dt, a, st));
    }
    tm.done();
  }
  return HOFEM_OK;
}

// Passes of a solve.  In 2D, when the row passes take two lines per
// workgroup, the intermediate between the passes is row-pair interleaved:
// the row passes then move contiguous blocks and the column pass moves
// twice the bytes per access.
// The decision uses the launch shape of the forward row pass for all nrhs
// right-hand sides (m_0 nrhs rows), as the launcher computes it.
std::vector<PassSpec> solve_list(const hofem_solver_s* S, bool f64, int nrhs) {
  const int N = S->N;
  std::vector<PassSpec> l;
  for (int a = N - 1; a >= 1; --a) l.push_back({a, PASS_FWD});
  l.push_back({0, PASS_FUSED});
  for (int a = 1; a < N; ++a) l.push_back({a, PASS_INV});
  if (N == 2 && S->ax[0].bc == 0 && S->ax[1].bc == 0 && !S->ax[0].dense && !S->ax[1].dense &&
      pass_lines_per_workgroup(S->ax[1].n, S->ax[1].K, f64, (long long)S->ax[0].m * nrhs) == 2) {
    l[0].il_out = true;
    l[1].il_in = l[1].il_out = true;
    l[2].il_in = true;
  }
  return l;
}

OpArgs op_args(const hofem_solver_s* S, const double* u, const double* f, void* out, int out_f32,
               int nrhs);

// Bytes of the 3D operator's element buffer (0 where the operator needs none),
// rounded up to 256.
size_t op_elem_bytes(const hofem_solver_s* S) {
  const size_t b = op3_elem_doubles(op_args(S, nullptr, nullptr, nullptr, 0, 1)) * sizeof(double);
  return (b + 255) & ~size_t(255);
}

// FP32_IR workspace: the FP32 correction grid, the norm partials, the
// operator's element buffer.
// Algorithm (b): transforms along axes 0..N-2, banded solves along N-1.
int solve_alg_b(hofem_solver_s* S, const double* f, double* u, int nrhs, hipStream_t st) {
  const int N = S->N, b = N - 1;
  const DevAxis& X = S->ax[b];
  std::vector<PassSpec> fw, inv;
  for (int a = 0; a < b; ++a) fw.push_back({a, PASS_FWD});
  for (int a = b - 1; a >= 0; --a) inv.push_back({a, PASS_INV});
  const double* bin = f;
  if (!fw.empty()) {
    const int rc = run_list(S, fw, true, f, u, u, 0, 0, 0, 0, nrhs, st);
    if (rc != HOFEM_OK) return rc;
    bin = u;
  }
  BandArgs a{};
  a.in = bin;
  a.out = u;
  a.n = X.n;
  a.K = X.K;
  a.m = X.m;
  a.scale = X.scale;
  a.A = X.A;
  a.C = X.C;
  a.others = 1;
  for (int i = 0; i < b; ++i) a.others *= S->ax[i].m;
  a.nlines = a.others * nrhs;
  a.alpha = S->alpha;
  a.nother = 0;
  for (int i = 0; i < b; ++i) {
    long long div = 1;
    for (int j = i + 1; j < b; ++j) div *= S->ax[j].m;
    a.olam[a.nother] = S->ax[i].t64.lam;
    a.oscale[a.nother] = S->ax[i].scale;
    a.odiv[a.nother] = div;
    a.omod[a.nother] = S->ax[i].m;
    ++a.nother;
  }
  {
    LaunchTimer tm(S, st, HOFEM_PASS_BANDED, b, 1, (double)S->per_rhs * nrhs * 16);
    HIPCHK(launch_banded(a, st));
    tm.done();
  }
  if (!inv.empty()) return run_list(S, inv, true, u, u, u, 0, 0, 0, 0, nrhs, st);
  return HOFEM_OK;
}

// Every axis Dirichlet (the operator, refinement, CG, algorithm (b), the
// Dirichlet lift and time stepping are built for Dirichlet axes only).
bool all_dirichlet(const hofem_solver_s* S) {
  for (int i = 0; i < S->N; ++i)
    if (S->ax[i].bc != 0) return false;
  return true;
}

bool has_dense(const hofem_solver_s* S) {
  for (int i = 0; i < S->N; ++i)
    if (S->ax[i].dense) return true;
  return false;
}

// Scratch grid of the dense passes.
size_t dense_bytes(const hofem_solver_s* S, int nrhs) {
  return has_dense(S) ? (S->per_rhs * (size_t)nrhs * sizeof(double) + 255) & ~size_t(255) : 0;
}

size_t ir_workspace(const hofem_solver_s* S, int nrhs) {
  size_t b = S->per_rhs * (size_t)nrhs * sizeof(float);
  b = (b + 255) & ~size_t(255);
  b += ((2 * kNormParts + 2) * sizeof(double) + 255) & ~size_t(255);
  b += op_elem_bytes(S);
  return b;
}

// Operator arguments; elem: the element buffer (op_elem_bytes of the
// caller's workspace; unused where that is 0).
int make_op(hofem_solver_s* S, const double* u, const double* f, void* out, int out_f32, int nrhs,
            double* elem, OpArgs* op) {
  OpArgs o = op_args(S, u, f, out, out_f32, nrhs);
  if (op3_elem_doubles(o) && !elem) return HOFEM_EINVAL;
  o.elem = elem;
  *op = o;
  return HOFEM_OK;
}

OpArgs op_args(const hofem_solver_s* S, const double* u, const double* f, void* out, int out_f32,
               int nrhs) {
  OpArgs o{};
  o.u = u;
  o.f = f;
  o.out = out;
  o.out_f32 = out_f32;
  o.N = S->N;
  for (int i = 0; i < S->N; ++i) {
    o.n[i] = S->ax[i].n;
    o.K[i] = S->ax[i].K;
    o.m[i] = S->ax[i].m;
    o.scale[i] = S->ax[i].scale;
    o.A[i] = S->ax[i].A;
    o.C[i] = S->ax[i].C;
    o.hA[i] = S->ax[i].hA.data();
    o.hC[i] = S->ax[i].hC.data();
  }
  o.alpha = S->alpha;
  o.nrhs = nrhs;
  o.elem = nullptr;
  return o;
}

VarOpArgs make_varop(const hofem_solver_s* S, const hofem_coef* c, const double* u,
                     const double* f, double* out, int nrhs) {
  VarOpArgs v{};
  v.u = u;
  v.f = f;
  v.out = out;
  v.N = S->N;
  long long per = 1;
  for (int i = S->N - 1; i >= 0; --i) {
    v.stride[i] = per;
    per *= S->ax[i].m;
  }
  v.per_rhs = per;
  v.nrhs = nrhs;
  for (int i = 0; i < S->N; ++i) {
    v.n[i] = S->ax[i].n;
    v.K[i] = S->ax[i].K;
    v.scale[i] = S->ax[i].scale;
    v.B[i] = S->ax[i].B;
    v.D[i] = S->ax[i].D;
    v.Dh[i] = S->ax[i].Dh;
    v.w[i] = S->ax[i].gw;
    v.t[i] = c ? c->t_dev[i] : nullptr;
  }
  v.alpha = S->alpha;
  v.kind = c ? c->kind : 0;
  v.c0 = c ? c->c0 : 1.0;
  v.c1 = c ? c->c1 : 0.0;
  v.afull = c ? c->a_dev : nullptr;
  return v;
}

constexpr int kPcgParts = 1024;

struct PcgWs {
  double *r, *z, *p, *q, *elem, *partial, *scal;
  float* w32;
};

size_t pcg_bytes(const hofem_solver_s* S, const hofem_coef* c) {
  const size_t n = S->per_rhs;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t b = 4 * al(n * sizeof(double)) + al(n * sizeof(float));
  if (c && c->kind != 0) b += al(varop_elem_bytes(make_varop(S, c, nullptr, nullptr, nullptr, 1)));
  else b += op_elem_bytes(S);
  b += al(3 * kPcgParts * sizeof(double)) + al(64 * sizeof(double));   // partials, scalars
  return b;
}

PcgWs pcg_carve(const hofem_solver_s* S, const hofem_coef* c, void* ws) {
  const size_t n = S->per_rhs;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  unsigned char* p = static_cast<unsigned char*>(ws);
  PcgWs w{};
  w.r = reinterpret_cast<double*>(p); p += al(n * sizeof(double));
  w.z = reinterpret_cast<double*>(p); p += al(n * sizeof(double));
  w.p = reinterpret_cast<double*>(p); p += al(n * sizeof(double));
  w.q = reinterpret_cast<double*>(p); p += al(n * sizeof(double));
  w.w32 = reinterpret_cast<float*>(p); p += al(n * sizeof(float));
  if (c && c->kind != 0) {
    w.elem = reinterpret_cast<double*>(p);
    p += al(varop_elem_bytes(make_varop(S, c, nullptr, nullptr, nullptr, 1)));
  } else {
    w.elem = reinterpret_cast<double*>(p);
    p += op_elem_bytes(S);
  }
  w.partial = reinterpret_cast<double*>(p); p += al(3 * kPcgParts * sizeof(double));
  w.scal = reinterpret_cast<double*>(p);
  return w;
}

// out = f - A u (f != NULL) or A u, for one right-hand side
int pcg_apply(hofem_solver_s* S, const hofem_coef* c, const PcgWs& w, const double* u,
              const double* f, double* out, hipStream_t st) {
  const long long count = (long long)S->per_rhs;
  if (!c || c->kind == 0) {
    OpArgs o;
    const int rc = make_op(S, u, f, out, 0, 1, w.elem, &o);
    if (rc != HOFEM_OK) return rc;
    LaunchTimer tm(S, st, HOFEM_PASS_OPERATOR, -1, 1, (double)count * (f ? 24 : 16));
    HIPCHK(launch_operator(o, st));
    tm.done();
  } else {
    VarOpArgs v = make_varop(S, c, u, f, out, 1);
    LaunchTimer tm(S, st, HOFEM_PASS_OPERATOR, -1, 1, (double)count * (f ? 24 : 16));
    HIPCHK(launch_varop(v, w.elem, st));
    tm.done();
  }
  return HOFEM_OK;
}

// CG on one right-hand side; stops on the relative residual (rtol > 0) or
// the relative update (utol > 0).
int pcg_run(hofem_solver_s* S, const hofem_coef* c, const PcgWs& w, const double* f, double* x,
            double rtol, double utol, int max_iter, hipStream_t st, int* iters, double* rel_res,
            double* rel_upd, bool* converged) {
  const long long n = (long long)S->per_rhs;
  const std::vector<PassSpec> list = solve_list(S, false, 1);
  const int np = (int)std::max<long long>(1, std::min<long long>(kPcgParts, (n + 255) / 256));
  double* sc = w.scal;
  auto precond = [&](const double* in, double* out) {
    return run_list(S, list, false, in, w.w32, out, 2, 1, 3, 5, 1, st);
  };
  int rc = precond(f, x);                                   // x0 = S32 f
  if (rc != HOFEM_OK) return rc;
  if ((rc = pcg_apply(S, c, w, x, f, w.r, st)) != HOFEM_OK) return rc;   // r = f - A x
  if ((rc = precond(w.r, w.z)) != HOFEM_OK) return rc;      // z = S32 r
  HIPCHK(hipMemcpyAsync(w.p, w.z, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(launch_dot2(w.r, w.z, w.r, n, w.partial, np, sc + 2, st));   // rz, (rr -> sc[3])
  HIPCHK(launch_dot2(f, f, nullptr, n, w.partial, np, sc + 9, st));    // ff
  HIPCHK(launch_cg_init(sc, rtol, utol, st));
  double h[64];
  HIPCHK(hipMemcpyAsync(h, sc, 16 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double ff = h[9] > 0 ? h[9] : 1.0;
  *rel_res = std::sqrt(h[3] / ff);
  *rel_upd = 0.0;
  *iters = 0;
  *converged = (rtol > 0 && *rel_res <= rtol);
  // The device records the first step that meets the tolerance and freezes
  // the iterate from then on; the host looks only at predicted steps (the
  // criterion falls about geometrically), at most 8 steps apart.
  auto crit = [&](const double* hs) {   // criterion value of a history slot and its target
    return rtol > 0 ? hs[0] : (hs[1] > 0 ? hs[2] * hs[2] * hs[3] / hs[1] : 0.0);
  };
  const double target = rtol > 0 ? rtol * rtol * ff : utol * utol;
  double prev = rtol > 0 ? h[3] : -1.0;
  int next_check = std::min(max_iter, 1);
  auto t_look = std::chrono::steady_clock::now();
  int it_look = 0;
  for (int it = 1; it <= max_iter && !*converged; ++it) {
    if ((rc = pcg_apply(S, c, w, w.p, nullptr, w.q, st)) != HOFEM_OK) return rc;   // q = A p
    HIPCHK(launch_dot2(w.p, w.q, w.p, n, w.partial, np, sc + 3, st));              // pq, pp
    HIPCHK(launch_scalar_op(sc, 0, st));                                           // alpha
    {
      LaunchTimer tm(S, st, HOFEM_PASS_UPDATE, -1, 1, (double)n * 48);
      // rr, xx, and r z_old for the flexible beta
      HIPCHK(launch_cg_update(x, w.r, w.p, w.q, w.z, n, sc, w.partial, np, sc + 7, sc + 10, st));
      tm.done();
    }
    HIPCHK(launch_cg_record(sc, st));
    if (it == next_check || it == max_iter) {
      HIPCHK(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      const int conv = (int)h[16];
      const int at = conv > 0 ? conv : it;
      const double* hs = h + 32 + 4 * ((at - 1) & 7);
      *iters = at;
      *rel_res = std::sqrt(hs[0] / ff);
      *rel_upd = hs[1] > 0 ? std::fabs(hs[2]) * std::sqrt(hs[3] / hs[1]) : 0.0;
      if (conv > 0) {
        *converged = true;
        break;
      }
      // next look: a look costs one host round trip (tens of microseconds),
      // a step taken after convergence costs a step; where steps are cheap,
      // look half way to where the criterion is predicted to reach its target
      // (geometric extrapolation from the last two steps), otherwise after
      // every step
      const auto t_now = std::chrono::steady_clock::now();
      const double step_ms =
          std::chrono::duration<double, std::milli>(t_now - t_look).count() / (it - it_look);
      t_look = t_now;
      it_look = it;
      const double now = crit(hs);
      const double before = it >= 2 ? crit(h + 32 + 4 * ((it - 2) & 7)) : prev;
      int steps = 1;
      if (step_ms < 0.25 && before > 0 && now > 0 && now < before && target > 0 && now > target) {
        const double need = std::log(target / now) / std::log(now / before);
        steps = std::min((int)std::floor(need / 2.0), it);
      }
      next_check = std::min(max_iter, it + std::max(1, std::min(8, steps)));
      prev = now;
    }
    if (it == max_iter) break;
    if ((rc = precond(w.r, w.z)) != HOFEM_OK) return rc;                           // z = S32 r
    HIPCHK(launch_dot2(w.r, w.z, nullptr, n, w.partial, np, sc + 5, st));          // rz_new
    HIPCHK(launch_scalar_op(sc, 1, st));                                           // beta
    HIPCHK(launch_cg_dir(w.p, w.z, n, sc, st));                                    // p = z + beta p
  }
  if (rtol <= 0 && utol <= 0) *converged = true;
  return HOFEM_OK;
}

bool coef_ok(const hofem_solver_s* S, const hofem_coef* c) {
  if (!c || c->kind == 0) return true;
  if (c->kind == 1) {
    for (int i = 0; i < S->N; ++i)
      if (!c->t_dev[i]) return false;
    return std::isfinite(c->c0) && std::isfinite(c->c1);
  }
  return c->kind == 2 && c->a_dev != nullptr;
}

}  // namespace

namespace {

// Device table image of one plan: per-wave-number tables blocked by 64 wave
// numbers with entries in 16-byte groups (pairs in FP64, quadruples in FP32;
// layout in kernels.h), the other tables plain, FP64 and FP32 copies.
std::vector<unsigned char> pack_plan(const Plan1DData& d, PlanOff* off) {
  Packer pk;
  const int n = d.n, K = d.K;
  if (d.bc == 1) {
    // periodic: eigenvalues, Bloch eigenvectors (complex FP64, blocked by
    // 64 wave numbers: entry e = l n + s of wave number k at
    // ((k / 64) n^2 + e) 64 + k % 64, so that a wavefront reads one entry
    // of 64 consecutive k with one contiguous 1 KB access), twiddles, local
    // and Gauss tables; the FP32 and Dirichlet-only slots point at the
    // twiddles (no pass reads them)
    const size_t nk = (size_t)K / 2 + 1, ne = (size_t)n * n, nblk = (nk + 63) / 64;
    std::vector<double> w(2 * nblk * ne * 64, 0.0);
    for (size_t k = 0; k < nk; ++k)
      for (size_t e = 0; e < ne; ++e) {
        const size_t at = ((k / 64) * ne + e) * 64 + k % 64;
        w[2 * at] = d.wr[k * ne + e];
        w[2 * at + 1] = d.wi[k * ne + e];
      }
    off->lam = pk.add_f64(d.lam);
    off->blk64 = pk.add_f64(w);
    off->tw64 = pk.add_f64(d.tw);
    off->E64 = off->sn64 = off->blk32 = off->E32 = off->tw32 = off->sn32 = off->tw64;
    off->A = pk.add_f64(d.A);
    off->C = pk.add_f64(d.C);
    off->B = pk.add_f64(d.B);
    off->D = pk.add_f64(d.D);
    off->Dh = pk.add_f64(d.Dh);
    off->gw = pk.add_f64(d.gw);
    if (d.dense) {
      off->S = pk.add_f64(d.S);
      off->St = pk.add_f64(d.St);
    }
    pk.bytes.resize((pk.bytes.size() + 255) & ~size_t(255), 0);
    return pk.bytes;
  }
  auto blocked = [&](size_t ge) {
    const size_t NE = (size_t)n * (n - 1) + n, NEG = (NE + ge - 1) / ge;
    const size_t nblk = ((size_t)K - 1 + 63) / 64;
    std::vector<double> blk(nblk * NEG * 64 * ge, 0.0);
    auto put = [&](int k, size_t e, double v) {
      const size_t b = (size_t)(k - 1) / 64, o = (size_t)(k - 1) % 64;
      blk[((b * NEG + e / ge) * 64 + o) * ge + e % ge] = v;
    };
    for (int k = 1; k < K; ++k) {
      for (int l = 0; l < n; ++l) {
        for (int c = 0; c < n - 1; ++c)
          put(k, (size_t)l * (n - 1) + c, d.p[((size_t)(k - 1) * n + l) * (n - 1) + c]);
        put(k, (size_t)n * (n - 1) + l, d.inorm[(size_t)(k - 1) * n + l]);
      }
    }
    return blk;
  };
  off->lam = pk.add_f64(d.lam);
  off->blk64 = pk.add_f64(blocked(2));
  off->E64 = pk.add_f64(d.E);
  off->tw64 = pk.add_f64(d.tw);
  off->sn64 = pk.add_f64(d.sn);
  off->blk32 = pk.add_f32(blocked(4));
  off->E32 = pk.add_f32(d.E);
  off->tw32 = pk.add_f32(d.tw);
  off->sn32 = pk.add_f32(d.sn);
  off->A = pk.add_f64(d.A);
  off->C = pk.add_f64(d.C);
  off->B = pk.add_f64(d.B);
  off->D = pk.add_f64(d.D);
  off->Dh = pk.add_f64(d.Dh);
  off->gw = pk.add_f64(d.gw);
  if (d.dense) {
    off->S = pk.add_f64(d.S);
    off->St = pk.add_f64(d.St);
  }
  if (d.bc == 2) off->band = pk.add_f64(d.band);
  pk.bytes.resize((pk.bytes.size() + 255) & ~size_t(255), 0);
  return pk.bytes;
}

}  // namespace

namespace hofem {

size_t solver_unknowns(const hofem_solver_s* S) { return S->per_rhs; }
bool solver_all_dirichlet(const hofem_solver_s* S) { return all_dirichlet(S) && !has_dense(S); }
int solver_dims(const hofem_solver_s* S) { return S->N; }
bool solver_has_dense(const hofem_solver_s* S) { return has_dense(S); }
int solver_axis_local(const hofem_solver_s* S, int axis, AxisLocal* out) {
  if (axis < 0 || axis >= S->N) return HOFEM_EINVAL;
  const DevAxis& X = S->ax[axis];
  const size_t nb = (size_t)X.n + 1;
  if (nb * nb > 100 || X.hC.size() != nb * nb || X.hA.size() != nb * nb) return HOFEM_EINVAL;
  out->bc = X.bc;
  out->n = X.n;
  out->K = X.K;
  out->m = X.m;
  long long inner = 1;
  for (int b = axis + 1; b < S->N; ++b) inner *= S->ax[b].m;
  out->inner = inner;
  for (size_t i = 0; i < nb * nb; ++i) {
    out->C[i] = X.hC[i];
    out->A[i] = X.hA[i];
  }
  return HOFEM_OK;
}

double solver_alpha(const hofem_solver_s* S) { return S->alpha; }
int solver_device(const hofem_solver_s* S) { return S->device; }
size_t solver_op_elem_bytes(const hofem_solver_s* S) { return op_elem_bytes(S); }

int solver_solve_fp64(hofem_solver_s* S, const double* in, double* out, int nrhs, hipStream_t st) {
  const std::vector<PassSpec> list = solve_list(S, true, nrhs);
  return run_list(S, list, true, in, out, out, 0, 0, 0, 0, nrhs, st);
}

int solver_mass_update(hofem_solver_s* S, const double* f, const double* w, double* out,
                       double coef, double* elem, int nrhs, hipStream_t st) {
  OpArgs o;
  // out = f - L' w with L' = -coef (x)C (f given), or out = L' w with
  // L' = coef (x)C (f NULL)
  const int rc = make_op(S, w, f, out, 0, nrhs, elem, &o);
  if (rc != HOFEM_OK) return rc;
  for (int i = 0; i < S->N; ++i) o.scale[i] = 0.0;
  o.alpha = f ? -coef : coef;
  LaunchTimer tm(S, st, HOFEM_PASS_OPERATOR, -1, 1, (double)S->per_rhs * nrhs * (f ? 24 : 16));
  HIPCHK(launch_operator(o, st));
  tm.done();
  return HOFEM_OK;
}

}  // namespace hofem

extern "C" {

const char* hofem_status_string(int status) {
  switch (status) {
    case HOFEM_OK: return "ok";
    case HOFEM_EINVAL: return "invalid argument";
    case HOFEM_EUNSUPPORTED: return "unsupported parameters";
    case HOFEM_ENOTPOSDEF: return "operator not positive definite for this alpha";
    case HOFEM_ENOCONV: return "refinement did not converge";
    case HOFEM_EHIP: return "HIP runtime error";
    case HOFEM_ENOMEM: return "out of memory";
    case HOFEM_ETOOBIG: return "problem exceeds the library's fixed scratch buffer";
    default: return "unknown status";
  }
}

int hofem_last_hip_error(void) { return g_last_hip; }

int hofem_plan1d_create(int n, int K, hofem_plan1d* out) {
  return hofem_plan1d_create_bc(n, K, HOFEM_BC_DIRICHLET, out);
}

int hofem_plan1d_create_bc(int n, int K, int bc, hofem_plan1d* out) {
  if (!out) return HOFEM_EINVAL;
  if (bc != HOFEM_BC_DIRICHLET && bc != HOFEM_BC_PERIODIC && bc != HOFEM_BC_NEUMANN) return HOFEM_EINVAL;
  const bool pow2 = (K & (K - 1)) == 0;
  if (n < 1 || n > 9 || K < 2 || K > 1024) return HOFEM_EUNSUPPORTED;
  // K not a power of two: dense transforms (m <= 4095)
  const int mdim = bc == HOFEM_BC_DIRICHLET ? n * K - 1 : bc == HOFEM_BC_PERIODIC ? n * K : n * K + 1;
  if (!pow2 && mdim > kDenseMax) return HOFEM_EUNSUPPORTED;
  hofem_plan1d p = new (std::nothrow) hofem_plan1d_s;
  if (!p) return HOFEM_ENOMEM;
  int rc = bc == HOFEM_BC_PERIODIC  ? plan1d_build_periodic(n, K, &p->d)
           : bc == HOFEM_BC_NEUMANN ? plan1d_build_neumann(n, K, &p->d)
                                    : plan1d_build(n, K, &p->d);
  if (rc == 0 && !pow2) rc = plan1d_build_dense(&p->d);
  if (rc != 0) {
    delete p;
    return HOFEM_EUNSUPPORTED;
  }
  p->image = pack_plan(p->d, &p->off);
  *out = p;
  return HOFEM_OK;
}

int hofem_plan1d_table_bytes(hofem_plan1d plan, size_t* bytes) {
  if (!plan || !bytes) return HOFEM_EINVAL;
  *bytes = plan->image.size();
  return HOFEM_OK;
}

int hofem_plan1d_upload(hofem_plan1d plan, void* dev_buf, size_t bytes, void* stream) {
  if (!plan || !dev_buf || bytes < plan->image.size()) return HOFEM_EINVAL;
  if (reinterpret_cast<uintptr_t>(dev_buf) & 255) return HOFEM_EINVAL;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHK(hipMemcpyAsync(dev_buf, plan->image.data(), plan->image.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  plan->dev = static_cast<const unsigned char*>(dev_buf);
  plan->device = dev;
  return HOFEM_OK;
}

void hofem_plan1d_destroy(hofem_plan1d plan) { delete plan; }

int hofem_plan1d_dim(hofem_plan1d plan, int* m) {
  if (!plan || !m) return HOFEM_EINVAL;
  *m = plan->d.m;
  return HOFEM_OK;
}

int hofem_plan1d_table(hofem_plan1d plan, int which, double* out_host, size_t len) {
  if (!plan || !out_host) return HOFEM_EINVAL;
  const Plan1DData& d = plan->d;
  const int n = d.n, K = d.K;
  const std::vector<double>* v = nullptr;
  size_t count = 0;
  // p and 1/||s||^2 of the Dirichlet and Neumann axes, Bloch vectors of the
  // periodic ones, band-edge vectors of the Neumann ones
  const bool sine_tabs = which == 1 || which == 2, periodic_only = which == 10 || which == 11;
  if ((sine_tabs && d.bc == 1) || (periodic_only && d.bc != 1) || (which == 14 && d.bc != 2))
    return HOFEM_EINVAL;
  switch (which) {
    case 0: v = &d.lam; count = d.m; break;
    case 1: v = &d.p; count = (size_t)(K - 1) * n * (n - 1); break;
    case 2: v = &d.inorm; count = (size_t)(K - 1) * n; break;
    case 3: v = &d.E; count = (size_t)(n - 1) * (n - 1); break;
    case 4: v = &d.A; count = (size_t)(n + 1) * (n + 1); break;
    case 5: v = &d.C; count = (size_t)(n + 1) * (n + 1); break;
    case 6: v = &d.gx; count = (size_t)(n + 1); break;
    case 7: v = &d.gw; count = (size_t)(n + 1); break;
    case 8: v = &d.B; count = (size_t)(n + 1) * (n + 1); break;
    case 9: v = &d.D; count = (size_t)(n + 1) * (n + 1); break;
    case 10: v = &d.wr; count = (size_t)(K / 2 + 1) * n * n; break;
    case 11: v = &d.wi; count = (size_t)(K / 2 + 1) * n * n; break;
    case 12: v = &d.S; count = d.dense ? (size_t)d.m * d.m : 0; break;
    case 13: v = &d.St; count = d.dense ? (size_t)d.m * d.m : 0; break;
    case 14: v = &d.band; count = (size_t)(n + 1) * n; break;
    default: return HOFEM_EINVAL;
  }
  if ((which == 12 || which == 13) && !d.dense) return HOFEM_EINVAL;
  if (len != count) return HOFEM_EINVAL;
  if (count) std::memcpy(out_host, v->data(), count * sizeof(double));
  return HOFEM_OK;
}

int hofem_solver_create(int N, const hofem_plan1d* plans, const double* X, double alpha,
                        hofem_solver* out) {
  if (!out || !plans || !X) return HOFEM_EINVAL;
  if (N < 1 || N > 3) return HOFEM_EUNSUPPORTED;
  if (!std::isfinite(alpha)) return HOFEM_EINVAL;
  for (int i = 0; i < N; ++i) {
    if (!plans[i]) return HOFEM_EINVAL;
    if (!(X[i] > 0) || !std::isfinite(X[i])) return HOFEM_EINVAL;
  }
  // Every denominator alpha + sum_i 4 h_i^-2 lambda_i must be positive; the
  // smallest is alpha + sum_i 4 h_i^-2 min lambda_i.
  double dmin = alpha;
  for (int i = 0; i < N; ++i) {
    const Plan1DData& d = plans[i]->d;
    const double h = X[i] / d.K;
    dmin += 4.0 / (h * h) * *std::min_element(d.lam.begin(), d.lam.end());
  }
  if (!(dmin > 0)) return HOFEM_ENOTPOSDEF;
  // the tables must be on the current device
  for (int i = 0; i < N; ++i)
    if (!plans[i]->dev) return HOFEM_EINVAL;
  int cur = 0;
  const hipError_t ge = hipGetDevice(&cur);
  if (ge != hipSuccess) return hip_fail(ge);
  for (int i = 0; i < N; ++i)
    if (plans[i]->device != cur) return HOFEM_EINVAL;

  hofem_solver S = new (std::nothrow) hofem_solver_s;
  if (!S) return HOFEM_ENOMEM;
  S->N = N;
  S->alpha = alpha;
  S->per_rhs = 1;
  S->device = cur;
  for (int i = 0; i < N; ++i) {
    const hofem_plan1d_s* P = plans[i];
    const Plan1DData& d = P->d;
    DevAxis& ax = S->ax[i];
    ax.bc = d.bc;
    ax.n = d.n;
    ax.K = d.K;
    ax.m = d.m;
    ax.X = X[i];
    const double h = X[i] / d.K;
    ax.scale = 4.0 / (h * h);
    S->per_rhs *= (size_t)d.m;
    ax.hA = d.A;
    ax.hC = d.C;
    const unsigned char* b = P->dev;
    const PlanOff& o = P->off;
    const double* lam = reinterpret_cast<const double*>(b + o.lam);
    const double* band = d.bc == 2 ? reinterpret_cast<const double*>(b + o.band) : nullptr;
    ax.t64 = AxisTab{b + o.blk64, b + o.E64, b + o.tw64, b + o.sn64, lam, ax.n, ax.K, ax.m, band};
    ax.t32 = AxisTab{b + o.blk32, b + o.E32, b + o.tw32, b + o.sn32, lam, ax.n, ax.K, ax.m, band};
    ax.A = reinterpret_cast<const double*>(b + o.A);
    ax.C = reinterpret_cast<const double*>(b + o.C);
    ax.B = reinterpret_cast<const double*>(b + o.B);
    ax.D = reinterpret_cast<const double*>(b + o.D);
    ax.Dh = reinterpret_cast<const double*>(b + o.Dh);
    ax.gw = reinterpret_cast<const double*>(b + o.gw);
    ax.dense = d.dense;
    if (d.dense) {
      ax.S = reinterpret_cast<const double*>(b + o.S);
      ax.St = reinterpret_cast<const double*>(b + o.St);
    }
  }
  *out = S;
  return HOFEM_OK;
}

int hofem_solver_set_graph(hofem_solver S, int enable) {
  if (!S) return HOFEM_EINVAL;
  S->use_graph = enable != 0;
  if (!S->use_graph && S->exec) {
    (void)hipGraphExecDestroy(S->exec);
    S->exec = nullptr;
  }
  return HOFEM_OK;
}

void hofem_solver_destroy(hofem_solver solver) {
  if (!solver) return;
  if (solver->exec) (void)hipGraphExecDestroy(solver->exec);
  for (hipEvent_t e : solver->event_pool) (void)hipEventDestroy(e);
  delete solver;
}

int hofem_solver_set_timing(hofem_solver S, int enable) {
  if (!S) return HOFEM_EINVAL;
  S->timing = enable != 0;
  return HOFEM_OK;
}

int hofem_solver_pass_times(hofem_solver S, hofem_pass_time* out_host, int max_entries,
                            int* count) {
  if (!S || !count || max_entries < 0 || (max_entries > 0 && !out_host)) return HOFEM_EINVAL;
  std::vector<hofem_pass_time> agg;
  for (const TimedLaunch& r : S->records) {
    HIPCHK(hipEventSynchronize(r.stop));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.start, r.stop));
    auto it = std::find_if(agg.begin(), agg.end(), [&](const hofem_pass_time& a) {
      return a.kind == r.kind && a.axis == r.axis && a.fp64 == r.fp64;
    });
    if (it == agg.end()) {
      agg.push_back(hofem_pass_time{r.kind, r.axis, r.fp64, 0, 0.0, r.bytes});
      it = agg.end() - 1;
    }
    it->launches += 1;
    it->ms += ms;
  }
  S->records.clear();
  const int n = std::min<int>((int)agg.size(), max_entries);
  for (int i = 0; i < n; ++i) out_host[i] = agg[i];
  *count = n;
  return HOFEM_OK;
}

int hofem_solver_size(hofem_solver solver, size_t* unknowns) {
  if (!solver || !unknowns) return HOFEM_EINVAL;
  *unknowns = solver->per_rhs;
  return HOFEM_OK;
}

int hofem_solver_workspace_bytes(hofem_solver solver, int mode, int nrhs, size_t* bytes) {
  if (!solver || !bytes || nrhs < 1) return HOFEM_EINVAL;
  switch (mode) {
    case HOFEM_MODE_FP64:
      *bytes = dense_bytes(solver, nrhs);
      return HOFEM_OK;
    case HOFEM_MODE_FP32:
    case HOFEM_MODE_FP64_B: *bytes = 0; return HOFEM_OK;
    case HOFEM_MODE_FP32_IR: *bytes = ir_workspace(solver, nrhs); return HOFEM_OK;
    case HOFEM_MODE_FP32_PCG: *bytes = pcg_bytes(solver, nullptr); return HOFEM_OK;
    default: return HOFEM_EINVAL;
  }
}

int hofem_solve(hofem_solver S, int mode, const void* f_dev, void* u_dev, int nrhs, void* ws_dev,
                size_t ws_bytes, int max_iter, double tol, void* stream, hofem_info* info) {
  if (!S || !f_dev || !u_dev || nrhs < 1) return HOFEM_EINVAL;
  if (mode != HOFEM_MODE_FP64 && (!all_dirichlet(S) || has_dense(S))) return HOFEM_EUNSUPPORTED;
  if (mode == HOFEM_MODE_FP64 && has_dense(S)) {
    if (!ws_dev || ws_bytes < dense_bytes(S, nrhs)) return HOFEM_EINVAL;
    S->dense_tmp = static_cast<double*>(ws_dev);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  // graph replay: solves without host synchronisation, on a stream that can
  // be captured
  const bool graphable = mode == HOFEM_MODE_FP64 || mode == HOFEM_MODE_FP32 ||
                         mode == HOFEM_MODE_FP64_B || (mode == HOFEM_MODE_FP32_IR && tol <= 0);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (S->use_graph && st != nullptr && hipStreamIsCapturing(st, &cap) != hipSuccess) return HOFEM_EHIP;
  if (S->use_graph && !S->capturing && graphable && !info && st != nullptr && mode >= 0 &&
      mode < 8 && max_iter >= 0 && cap == hipStreamCaptureStatusNone) {
    if (!S->warm[mode]) {
      // eager first: one-time kernel set-up must not happen inside a capture
      S->capturing = true;   // (no timing events and no nested graph)
      const int rc = hofem_solve(S, mode, f_dev, u_dev, nrhs, ws_dev, ws_bytes, max_iter, tol,
                                 stream, nullptr);
      S->capturing = false;
      if (rc == HOFEM_OK) S->warm[mode] = true;
      return rc;
    }
    if (!(S->exec && S->g_mode == mode && S->g_f == f_dev && S->g_u == u_dev && S->g_ws == ws_dev &&
          S->g_nrhs == nrhs && S->g_iter == max_iter)) {
      if (S->exec) (void)hipGraphExecDestroy(S->exec);
      S->exec = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      S->capturing = true;
      const int rc = hofem_solve(S, mode, f_dev, u_dev, nrhs, ws_dev, ws_bytes, max_iter, tol,
                                 stream, nullptr);
      S->capturing = false;
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(st, &graph);
      if (rc != HOFEM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (e != hipSuccess) return hip_fail(e);
      const hipError_t ei = hipGraphInstantiate(&S->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        S->exec = nullptr;
        return hip_fail(ei);
      }
      S->g_mode = mode;
      S->g_f = f_dev;
      S->g_u = u_dev;
      S->g_ws = ws_dev;
      S->g_nrhs = nrhs;
      S->g_iter = max_iter;
    }
    HIPCHK(hipGraphLaunch(S->exec, st));
    return HOFEM_OK;
  }
  if (mode == HOFEM_MODE_FP64_B) {
    const int rc = solve_alg_b(S, static_cast<const double*>(f_dev), static_cast<double*>(u_dev),
                               nrhs, st);
    if (rc != HOFEM_OK) return rc;
    if (info) *info = hofem_info{0, 0.0, 0.0};
    return HOFEM_OK;
  }
  const std::vector<PassSpec> list = solve_list(S, mode == HOFEM_MODE_FP64, nrhs);
  if (mode == HOFEM_MODE_FP64 || mode == HOFEM_MODE_FP32) {
    const bool f64 = mode == HOFEM_MODE_FP64;
    const int dt = f64 ? 0 : 1;
    int rc = run_list(S, list, f64, f_dev, u_dev, u_dev, dt, dt, dt, dt, nrhs, st);
    if (rc != HOFEM_OK) return rc;
    if (info) {
      info->iterations = 0;
      info->rel_update = 0.0;
      info->rel_residual = 0.0;
    }
    return HOFEM_OK;
  }
  if (mode == HOFEM_MODE_FP32_PCG) {
    if (max_iter < 0 || !std::isfinite(tol) || f_dev == u_dev) return HOFEM_EINVAL;
    if (!ws_dev || ws_bytes < pcg_bytes(S, nullptr)) return HOFEM_EINVAL;
    const PcgWs w = pcg_carve(S, nullptr, ws_dev);
    int its = 0;
    double rr = 0, ru = 0;
    bool conv = true;
    for (int r = 0; r < nrhs; ++r) {
      bool c1 = false;
      const int rc = pcg_run(S, nullptr, w, static_cast<const double*>(f_dev) + r * S->per_rhs,
                             static_cast<double*>(u_dev) + r * S->per_rhs, 0.0, tol, max_iter, st,
                             &its, &rr, &ru, &c1);
      if (rc != HOFEM_OK) return rc;
      conv = conv && c1;
    }
    if (info) {
      info->iterations = its;
      info->rel_update = ru;
      info->rel_residual = rr;
    }
    return conv ? HOFEM_OK : HOFEM_ENOCONV;
  }
  if (mode != HOFEM_MODE_FP32_IR) return HOFEM_EINVAL;
  if (max_iter < 0 || !std::isfinite(tol)) return HOFEM_EINVAL;
  if (f_dev == u_dev) return HOFEM_EINVAL;
  const size_t need = ir_workspace(S, nrhs);
  if (!ws_dev || ws_bytes < need) return HOFEM_EINVAL;
  const long long count = (long long)S->per_rhs * nrhs;
  float* r32 = static_cast<float*>(ws_dev);
  size_t roff = (S->per_rhs * (size_t)nrhs * sizeof(float) + 255) & ~size_t(255);
  double* partial = reinterpret_cast<double*>(static_cast<unsigned char*>(ws_dev) + roff);
  double* sums = partial + 2 * kNormParts;
  double* elem = reinterpret_cast<double*>(
      static_cast<unsigned char*>(ws_dev) + roff +
      (((2 * kNormParts + 2) * sizeof(double) + 255) & ~size_t(255)));
  // First FP32 solve: f^h (FP64) -> u (FP64).
  int rc = run_list(S, list, false, f_dev, r32, u_dev, 2, 1, 3, 5, nrhs, st);
  if (rc != HOFEM_OK) return rc;
  const int parts = (int)std::max<long long>(1, std::min<long long>(kNormParts, (count + 255) / 256));
  int it = 0;
  bool converged = tol <= 0;
  double host[2] = {0.0, 0.0};
  bool have = false;
  std::vector<PassSpec> acc_list = list;
  acc_list.back().kind = PASS_INV_ACC;
  for (; it < max_iter;) {
    OpArgs o;
    rc = make_op(S, static_cast<const double*>(u_dev), static_cast<const double*>(f_dev), r32, 1,
                 nrhs, elem, &o);
    if (rc != HOFEM_OK) return rc;
    {
      LaunchTimer tm(S, st, HOFEM_PASS_OPERATOR, -1, 1, (double)count * (8 + 8 + 4));
      HIPCHK(launch_operator(o, st));
      tm.done();
    }
    if (tol <= 0 && it + 1 < max_iter && list.size() > 1) {
      // a step whose norms nobody reads: the last (inverse) pass adds the
      // correction to u itself
      rc = run_list(S, acc_list, false, r32, r32, u_dev, 1, 1, 4, 4, nrhs, st);
      if (rc != HOFEM_OK) return rc;
      ++it;
      continue;
    }
    rc = run_list(S, list, false, r32, r32, r32, 1, 1, 1, 1, nrhs, st);
    if (rc != HOFEM_OK) return rc;
    {
      LaunchTimer tm(S, st, HOFEM_PASS_UPDATE, -1, 1, (double)count * (4 + 8 + 8));
      HIPCHK(launch_norms(r32, static_cast<double*>(u_dev), count, partial, parts, sums, st));
      tm.done();
    }
    ++it;
    have = false;
    if (tol > 0) {
      HIPCHK(hipMemcpyAsync(host, sums, sizeof(host), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      have = true;
      const double rel = host[1] > 0 ? std::sqrt(host[0] / host[1]) : 0.0;
      if (rel <= tol) {
        converged = true;
        break;
      }
    }
  }
  if (info) {
    info->iterations = it;
    info->rel_update = 0.0;
    info->rel_residual = 0.0;
    if (it > 0) {
      if (!have) {
        HIPCHK(hipMemcpyAsync(host, sums, sizeof(host), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
      }
      info->rel_update = host[1] > 0 ? std::sqrt(host[0] / host[1]) : 0.0;
    }
  }
  return converged ? HOFEM_OK : HOFEM_ENOCONV;
}

int hofem_forward(hofem_solver S, int mode, const void* in_dev, void* out_dev, int nrhs,
                  void* stream) {
  if (!S || !in_dev || !out_dev || nrhs < 1) return HOFEM_EINVAL;
  if (mode != HOFEM_MODE_FP64 && !all_dirichlet(S)) return HOFEM_EUNSUPPORTED;
  if (mode != HOFEM_MODE_FP64 && mode != HOFEM_MODE_FP32) return HOFEM_EINVAL;
  if (has_dense(S)) return HOFEM_EUNSUPPORTED;   // no workspace argument
  const bool f64 = mode == HOFEM_MODE_FP64;
  const int dt = f64 ? 0 : 1;
  std::vector<PassSpec> l;
  for (int a = S->N - 1; a >= 0; --a) l.push_back({a, PASS_FWD});
  return run_list(S, l, f64, in_dev, out_dev, out_dev, dt, dt, dt, dt, nrhs,
                  static_cast<hipStream_t>(stream));
}

int hofem_inverse(hofem_solver S, int mode, const void* in_dev, void* out_dev, int nrhs,
                  void* stream) {
  if (!S || !in_dev || !out_dev || nrhs < 1) return HOFEM_EINVAL;
  if (mode != HOFEM_MODE_FP64 && !all_dirichlet(S)) return HOFEM_EUNSUPPORTED;
  if (mode != HOFEM_MODE_FP64 && mode != HOFEM_MODE_FP32) return HOFEM_EINVAL;
  if (has_dense(S)) return HOFEM_EUNSUPPORTED;   // no workspace argument
  const bool f64 = mode == HOFEM_MODE_FP64;
  const int dt = f64 ? 0 : 1;
  std::vector<PassSpec> l;
  for (int a = 0; a < S->N; ++a) l.push_back({a, PASS_INV});
  return run_list(S, l, f64, in_dev, out_dev, out_dev, dt, dt, dt, dt, nrhs,
                  static_cast<hipStream_t>(stream));
}

int hofem_pcg_workspace_bytes(hofem_solver S, const hofem_coef* coef, size_t* bytes) {
  if (!S || !bytes || !coef_ok(S, coef)) return HOFEM_EINVAL;
  *bytes = pcg_bytes(S, coef);
  return HOFEM_OK;
}

int hofem_pcg(hofem_solver S, const hofem_coef* coef, const double* f_dev, double* u_dev, int nrhs,
              double rtol, int max_iter, void* ws_dev, size_t ws_bytes, void* stream,
              hofem_info* info) {
  if (!S || !f_dev || !u_dev || nrhs < 1 || f_dev == u_dev || max_iter < 0 ||
      !std::isfinite(rtol) || !coef_ok(S, coef))
    return HOFEM_EINVAL;
  if (!all_dirichlet(S) || has_dense(S)) return HOFEM_EUNSUPPORTED;
  if (!ws_dev || ws_bytes < pcg_bytes(S, coef)) return HOFEM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const PcgWs w = pcg_carve(S, coef, ws_dev);
  int its = 0;
  double rr = 0, ru = 0;
  bool conv = true;
  for (int r = 0; r < nrhs; ++r) {
    bool c1 = false;
    const int rc = pcg_run(S, coef, w, f_dev + r * S->per_rhs, u_dev + r * S->per_rhs, rtol, 0.0,
                           max_iter, st, &its, &rr, &ru, &c1);
    if (rc != HOFEM_OK) return rc;
    conv = conv && c1;
  }
  if (info) {
    info->iterations = its;
    info->rel_update = ru;
    info->rel_residual = rr;
  }
  return conv ? HOFEM_OK : HOFEM_ENOCONV;
}

int hofem_apply_coef_operator(hofem_solver S, const hofem_coef* coef, const double* u_dev,
                              double* out_dev, int nrhs, void* ws_dev, size_t ws_bytes,
                              void* stream) {
  if (!S || !u_dev || !out_dev || nrhs < 1 || u_dev == out_dev || !coef_ok(S, coef))
    return HOFEM_EINVAL;
  if (!all_dirichlet(S)) return HOFEM_EUNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!ws_dev || ws_bytes < pcg_bytes(S, coef)) return HOFEM_EINVAL;
  const PcgWs w = pcg_carve(S, coef, ws_dev);
  if (!coef || coef->kind == 0) {
    OpArgs o;
    const int rc = make_op(S, u_dev, nullptr, out_dev, 0, nrhs, w.elem, &o);
    if (rc != HOFEM_OK) return rc;
    HIPCHK(launch_operator(o, st));
    return HOFEM_OK;
  }
  for (int r = 0; r < nrhs; ++r) {
    VarOpArgs v = make_varop(S, coef, u_dev + r * S->per_rhs, nullptr, out_dev + r * S->per_rhs, 1);
    HIPCHK(launch_varop(v, w.elem, st));
  }
  return HOFEM_OK;
}

// With a periodic or Neumann axis the operator and the mass product run one
// kernel per axis (and per term), one right-hand side at a time, through
// N - 1 grids of one right-hand side.
static size_t axes_op_bytes(const hofem_solver_s* S) {
  return (size_t)(S->N - 1) * ((S->per_rhs * sizeof(double) + 255) & ~size_t(255));
}

int hofem_operator_workspace_bytes(hofem_solver S, size_t* bytes) {
  if (!S || !bytes) return HOFEM_EINVAL;
  *bytes = all_dirichlet(S) ? op_elem_bytes(S) : axes_op_bytes(S);
  return HOFEM_OK;
}

namespace {

// out = L u, or with mass_only the mass product (x)_i C_i u (the operator's
// stiffness scales set to 0 and alpha to 1: the stiffness terms then vanish
// exactly).
// Any boundary conditions: L u = sum_i T_i u with T_0 = (s_0 A_0 + alpha C_0)
// (x) C_1 ... and T_i = C_0 (x) .. s_i A_i .. (x) C_{N-1} (mass only: one term
// of mass factors), each term a chain of one kernel per axis ending in out.
int apply_op_axes(hofem_solver S, const double* u, double* out, int nrhs, double* ws, hipStream_t st,
                  bool mass_only) {
  const int N = S->N;
  const long long M = (long long)S->per_rhs;
  const size_t grid = ((size_t)M * sizeof(double) + 255) & ~size_t(255);
  double* tmp[2] = {ws, ws ? ws + grid / sizeof(double) : nullptr};
  AxisLocal al[3];
  for (int a = 0; a < N; ++a) {
    const int rc = solver_axis_local(S, a, &al[a]);
    if (rc != HOFEM_OK) return rc;
  }
  const int terms = mass_only ? 1 : N;
  for (int r = 0; r < nrhs; ++r) {
    const double* ur = u + (size_t)r * M;
    double* orr = out + (size_t)r * M;
    for (int i = 0; i < terms; ++i) {
      const double* src = ur;
      for (int a = 0; a < N; ++a) {
        double cc = 1.0, ca = 0.0;
        if (!mass_only && a == i) {
          cc = i == 0 ? S->alpha : 0.0;
          ca = S->ax[a].scale;
        }
        const bool last = a == N - 1;
        double* dst = last ? orr : tmp[a % 2];
        HIPCHK(launch_axis_local(al[a], src, dst, (last && i > 0) ? orr : nullptr, cc, ca, M, st));
        src = dst;
      }
    }
  }
  return HOFEM_OK;
}

int apply_op(hofem_solver S, const double* u_dev, double* out_dev, int nrhs, void* ws_dev,
             size_t ws_bytes, void* stream, bool mass_only) {
  if (!S || !u_dev || !out_dev || nrhs < 1 || u_dev == out_dev) return HOFEM_EINVAL;
  if (!all_dirichlet(S)) {
    const size_t need = axes_op_bytes(S);
    if (need && (!ws_dev || ws_bytes < need)) return HOFEM_EINVAL;
    return apply_op_axes(S, u_dev, out_dev, nrhs, static_cast<double*>(ws_dev),
                         static_cast<hipStream_t>(stream), mass_only);
  }
  const size_t need = op_elem_bytes(S);
  if (need && (!ws_dev || ws_bytes < need)) return HOFEM_EINVAL;
  OpArgs o;
  const int rc = make_op(S, u_dev, nullptr, out_dev, 0, nrhs, static_cast<double*>(ws_dev), &o);
  if (rc != HOFEM_OK) return rc;
  if (mass_only) {
    for (int i = 0; i < S->N; ++i) o.scale[i] = 0.0;
    o.alpha = 1.0;
  }
  HIPCHK(launch_operator(o, static_cast<hipStream_t>(stream)));
  return HOFEM_OK;
}

}  // namespace

int hofem_dirichlet_rhs(hofem_solver S, const double* b_ext_dev, const double* f_dev,
                        double* out_dev, int nrhs, void* stream) {
  if (!S || !b_ext_dev || !out_dev || nrhs < 1) return HOFEM_EINVAL;
  if (static_cast<const void*>(b_ext_dev) == static_cast<const void*>(out_dev)) return HOFEM_EINVAL;
  if (!all_dirichlet(S)) return HOFEM_EUNSUPPORTED;
  OpArgs o = op_args(S, nullptr, nullptr, out_dev, 0, nrhs);
  HIPCHK(launch_dirichlet_lift(o, b_ext_dev, f_dev, out_dev, static_cast<hipStream_t>(stream)));
  return HOFEM_OK;
}

int hofem_apply_operator(hofem_solver S, const double* u_dev, double* out_dev, int nrhs,
                         void* ws_dev, size_t ws_bytes, void* stream) {
  return apply_op(S, u_dev, out_dev, nrhs, ws_dev, ws_bytes, stream, false);
}

int hofem_apply_mass(hofem_solver S, const double* g_dev, double* out_dev, int nrhs, void* ws_dev,
                     size_t ws_bytes, void* stream) {
  return apply_op(S, g_dev, out_dev, nrhs, ws_dev, ws_bytes, stream, true);
}

}  // extern "C"

// ---- autotuner of the line passes' launch shapes ----------------------------
namespace {

#ifndef HOFEM_KERNEL_HASH
#define HOFEM_KERNEL_HASH "unhashed"
#endif

struct PassKey {
  int kind, axis, fp64;
};

// The distinct (kind, axis, precision) passes of a mode's solve.
std::vector<PassKey> mode_passes(const hofem_solver_s* S, int mode, int nrhs) {
  std::vector<PassKey> keys;
  const bool f64 = mode == HOFEM_MODE_FP64;
  for (const PassSpec& p : solve_list(S, f64, nrhs)) {
    const PassKey k{p.kind == PASS_INV_ACC ? PASS_INV : p.kind, p.axis, f64 ? 1 : 0};
    bool seen = false;
    for (const PassKey& q : keys) seen = seen || (q.kind == k.kind && q.axis == k.axis && q.fp64 == k.fp64);
    if (!seen) keys.push_back(k);
  }
  return keys;
}

long long pass_lines(const hofem_solver_s* S, int axis, int nrhs) {
  long long others = 1;
  for (int i = 0; i < S->N; ++i)
    if (i != axis) others *= S->ax[i].m;
  return others * nrhs;
}

void set_shape(hofem_solver_s* S, const PassKey& k, int cb, int threads, long long nlines = 0) {
  if (S->exec) {   // a captured solve keeps its launch shapes: capture again
    (void)hipGraphExecDestroy(S->exec);
    S->exec = nullptr;
  }
  for (auto it = S->tune.begin(); it != S->tune.end(); ++it) {
    if (it->kind == k.kind && it->axis == k.axis && it->fp64 == k.fp64) {
      S->tune.erase(it);
      break;
    }
  }
  if (cb > 0) S->tune.push_back(hofem_tune_entry{k.kind, k.axis, k.fp64, cb, threads, nlines, 0.0, 0.0});
}

}  // namespace

extern "C" {

int hofem_pass_shape_candidates(hofem_solver S, int kind, int axis, int fp64, int nrhs,
                                int* cb_host, int* threads_host, int max_entries, int* count) {
  if (!S || !count || axis < 0 || axis >= S->N || nrhs < 1 || max_entries < 0) return HOFEM_EINVAL;
  if (kind != PASS_FWD && kind != PASS_INV && kind != PASS_FUSED) return HOFEM_EINVAL;
  if (max_entries > 0 && (!cb_host || !threads_host)) return HOFEM_EINVAL;
  const DevAxis& X = S->ax[axis];
  const bool rows = axis == S->N - 1;
  *count = pass_shape_candidates(X.n, X.K, fp64 != 0, pass_lines(S, axis, nrhs),
                                 kind == PASS_INV && fp64 && rows, cb_host, threads_host,
                                 max_entries);
  return HOFEM_OK;
}

int hofem_pass_set_shape(hofem_solver S, int kind, int axis, int fp64, int cb, int threads) {
  if (!S || axis < 0 || axis >= S->N || cb < 0) return HOFEM_EINVAL;
  if (kind != PASS_FWD && kind != PASS_INV && kind != PASS_FUSED) return HOFEM_EINVAL;
  if (cb > 0 && threads != 256 && threads != 512) return HOFEM_EINVAL;
  set_shape(S, PassKey{kind, axis, fp64 ? 1 : 0}, cb, threads);
  return HOFEM_OK;
}

int hofem_solver_autotune(hofem_solver S, int mode, const void* f_dev, void* u_dev, int nrhs,
                          void* ws_dev, size_t ws_bytes, int reps, void* stream,
                          hofem_tune_entry* out_host, int max_entries, int* count) {
  if (!S || !f_dev || !u_dev || nrhs < 1 || reps < 1 || !count || max_entries < 0) return HOFEM_EINVAL;
  if (mode != HOFEM_MODE_FP64 && mode != HOFEM_MODE_FP32 && mode != HOFEM_MODE_FP32_IR) return HOFEM_EINVAL;
  if (mode == HOFEM_MODE_FP32_IR && f_dev == u_dev) return HOFEM_EINVAL;
  if (max_entries > 0 && !out_host) return HOFEM_EINVAL;
  if (!all_dirichlet(S) || has_dense(S)) return HOFEM_EUNSUPPORTED;   // FFT line passes only
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return HOFEM_EHIP;
  }
  const bool timing = S->timing;
  S->timing = false;
  // one solve of the mode (one refinement step for FP32_IR), ms per solve;
  // < 0 when the shape cannot run
  auto measure = [&]() -> double {
    auto one = [&]() {
      return hofem_solve(S, mode, f_dev, u_dev, nrhs, ws_dev, ws_bytes, 1, 0.0, st, nullptr);
    };
    if (one() != HOFEM_OK) return -1.0;
    if (hipEventRecord(e0, st) != hipSuccess) return -1.0;
    for (int r = 0; r < reps; ++r)
      if (one() != HOFEM_OK) return -1.0;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
    return ms / reps;
  };
  int rc = HOFEM_OK;
  std::vector<hofem_tune_entry> done;
  for (const PassKey& k : mode_passes(S, mode, nrhs)) {
    set_shape(S, k, 0, 0);
    const double t_def = measure();
    if (t_def < 0) {
      rc = HOFEM_EHIP;
      break;
    }
    int cand_cb[64], cand_thr[64];
    int nc = 0;
    hofem_pass_shape_candidates(S, k.kind, k.axis, k.fp64, nrhs, cand_cb, cand_thr, 64, &nc);
    int best_cb = 0, best_thr = 0;
    double best = t_def;
    for (int c = 1; c < nc; ++c) {       // candidate 0 is the default
      set_shape(S, k, cand_cb[c], cand_thr[c]);
      const double t = measure();
      (void)hipGetLastError();
      if (t >= 0 && t < best) {
        best = t;
        best_cb = cand_cb[c];
        best_thr = cand_thr[c];
      }
    }
    const long long nl = pass_lines(S, k.axis, nrhs);
    set_shape(S, k, best_cb, best_thr, nl);
    if (best_cb == 0) {
      // the default won: record it as such
      best_cb = cand_cb[0];
      best_thr = cand_thr[0];
    }
    done.push_back(hofem_tune_entry{k.kind, k.axis, k.fp64, best_cb, best_thr, nl, t_def, best});
  }
  S->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != HOFEM_OK) return rc;
  const int n = std::min<int>((int)done.size(), max_entries);
  for (int i = 0; i < n; ++i) out_host[i] = done[i];
  *count = (int)done.size();
  return HOFEM_OK;
}

// Tuning cache on disk: one text line per tuned pass,
//   <kernel hash> <n> <K> <fp64> <kind> <rows> <nlines> <cb> <threads> <ms default> <ms tuned>
// (rows: the pass runs along the contiguous axis).  A shape applies to a
// pass of the same kernels, order, K, precision, kind, stride and line count.
int hofem_solver_tune_save(hofem_solver S, const char* path) {
  if (!S || !path) return HOFEM_EINVAL;
  std::vector<std::string> lines;
  auto key_of = [](const std::string& l) {
    std::istringstream is(l);
    std::string k, w;
    for (int i = 0; i < 7 && (is >> w); ++i) k += w + " ";
    return k;
  };
  std::vector<std::string> fresh;
  for (const hofem_tune_entry& t : S->tune) {
    if (t.nlines <= 0) continue;   // forced shapes are not cached
    const DevAxis& X = S->ax[t.axis];
    std::ostringstream os;
    os << HOFEM_KERNEL_HASH << " " << X.n << " " << X.K << " " << t.fp64 << " " << t.kind << " "
       << (t.axis == S->N - 1 ? 1 : 0) << " " << t.nlines << " " << t.cb << " " << t.threads << " "
       << t.ms_default << " " << t.ms_tuned;
    fresh.push_back(os.str());
  }
  {
    std::ifstream in(path);
    std::string l;
    while (std::getline(in, l)) {
      if (l.empty()) continue;
      bool replaced = false;
      for (const std::string& f : fresh) replaced = replaced || key_of(f) == key_of(l);
      if (!replaced) lines.push_back(l);
    }
  }
  for (const std::string& f : fresh) lines.push_back(f);
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return HOFEM_EINVAL;
    for (const std::string& l : lines) out << l << "\n";
    if (!out) return HOFEM_EINVAL;
  }
  if (std::rename(tmp.c_str(), path) != 0) return HOFEM_EINVAL;
  return HOFEM_OK;
}

int hofem_solver_tune_load(hofem_solver S, const char* path, int mode, int nrhs, int* applied) {
  if (!S || !path || nrhs < 1 || !applied) return HOFEM_EINVAL;
  if (mode != HOFEM_MODE_FP64 && mode != HOFEM_MODE_FP32 && mode != HOFEM_MODE_FP32_IR) return HOFEM_EINVAL;
  *applied = 0;
  std::ifstream in(path);
  if (!in) return HOFEM_OK;   // no cache yet
  struct Row {
    std::string hash;
    int n, K, fp64, kind, rows;
    long long nlines;
    int cb, threads;
  };
  std::vector<Row> rows;
  std::string l;
  while (std::getline(in, l)) {
    std::istringstream is(l);
    Row r;
    if (is >> r.hash >> r.n >> r.K >> r.fp64 >> r.kind >> r.rows >> r.nlines >> r.cb >> r.threads)
      rows.push_back(r);
  }
  for (const PassKey& k : mode_passes(S, mode, nrhs)) {
    const DevAxis& X = S->ax[k.axis];
    const long long nl = pass_lines(S, k.axis, nrhs);
    const int isrow = k.axis == S->N - 1 ? 1 : 0;
    for (const Row& r : rows) {
      if (r.hash == HOFEM_KERNEL_HASH && r.n == X.n && r.K == X.K && r.fp64 == k.fp64 &&
          r.kind == k.kind && r.rows == isrow && r.nlines == nl) {
        set_shape(S, k, r.cb, r.threads, nl);
        ++*applied;
        break;
      }
    }
  }
  return HOFEM_OK;
}

int hofem_solver_tune_reset(hofem_solver S) {
  if (!S) return HOFEM_EINVAL;
  S->tune.clear();
  if (S->exec) {
    (void)hipGraphExecDestroy(S->exec);
    S->exec = nullptr;
  }
  return HOFEM_OK;
}

const char* hofem_kernel_hash(void) { return HOFEM_KERNEL_HASH; }

}  // extern "C"

// ---- FP32_IR with the library's own scratch (no allocation) ---------------
namespace {

// Scratch of hofem_solve_ir_noalloc: one copy per device, held until the
// process ends.  Host code never uses the symbol itself (a host stand-in),
// only its device address from hipGetSymbolAddress, kept per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch (looked up once per device, with
// that device current).
int scratch_of_device(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return HOFEM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return HOFEM_OK;
}

}  // namespace

extern "C" {

int hofem_solve_ir_noalloc(hofem_solver S, const double* f_dev, double* u_dev, int nrhs,
                           int max_iter, double tol, void* stream, hofem_info* info) {
  if (!S || !f_dev || !u_dev || nrhs < 1 || f_dev == u_dev) return HOFEM_EINVAL;
  if (max_iter < 0 || !std::isfinite(tol)) return HOFEM_EINVAL;
  if (ir_workspace(S, nrhs) > kScratchBytes) return HOFEM_ETOOBIG;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != S->device) return HOFEM_EINVAL;
  void* ws = nullptr;
  const int rc = scratch_of_device(dev, &ws);
  if (rc != HOFEM_OK) return rc;
  // every byte the refinement reads from the scratch is written first in
  // the same call (the residual grid by the operator, the norm partials by
  // the norm kernels, the 3D plane-product grids by the operator), so nothing
  // needs clearing
  g_no_events = true;
  const int st = hofem_solve(S, HOFEM_MODE_FP32_IR, f_dev, u_dev, nrhs, ws, kScratchBytes,
                             max_iter, tol, stream, info);
  g_no_events = false;
  return st;
}

}  // extern "C"
