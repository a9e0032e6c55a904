// FP64 operator of eq. (bvp glob 2) and the small kernels of the refinement
// loop (update with norms, reduction).

#include <algorithm>

#include "kernels.h"
#include "solver.h"

namespace hofem {
namespace {

// ---------------------------------------------------------------------------
// FP64 operator of eq. (bvp glob 2), matrix-free, one thread per output point.
//
// Element e of axis i covers positions g = n_i (e-1) .. n_i e (g = 0 and
// g = n_i K_i are the Dirichlet zeros).  A point lies in one element along an
// axis (interior point) or two (mesh node).  For every element containing
// it, the element's row is applied sum-factorised: the stiffness factor of a
// term acts first, on u itself, in difference form
// sum_{r != r0} A_{r0 r} (u_r - u_{r0}); the mass factors of the other axes
// act on its result.  This keeps the differences of a smooth u exact and the
// constants along the stiffness axis exactly in the kernel.
// ---------------------------------------------------------------------------

struct OpGeom {
  long long stride[3];
};

template <int N>
__device__ __forceinline__ double op_u(const OpArgs& a, const double* u, const OpGeom& G,
                                       const int* e, int r0, int r1, int r2) {
  int rr[3] = {r0, r1, r2};
  long long idx = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int g = a.n[i] * (e[i] - 1) + rr[i];
    if (g <= 0 || g >= a.n[i] * a.K[i]) return 0.0;
    idx += (long long)(g - 1) * G.stride[i];
  }
  return u[idx];
}

template <int N>
__device__ double op_element(const OpArgs& a, const double* u, const OpGeom& G, const int* e,
                             const int* r) {
  const double* A0 = a.A[0];
  const double* C0 = a.C[0];
  const int n0 = a.n[0], b0 = n0 + 1;
  double acc = 0.0;
  if (N == 1) {
    const double ur = op_u<1>(a, u, G, e, r[0], 0, 0);
    double t = 0.0, mm = 0.0;
    for (int p0 = 0; p0 <= n0; ++p0) {
      const double v = op_u<1>(a, u, G, e, p0, 0, 0);
      if (p0 != r[0]) t += A0[r[0] * b0 + p0] * (v - ur);
      mm += C0[r[0] * b0 + p0] * v;
    }
    acc = a.scale[0] * t + a.alpha * mm;
  } else if (N == 2) {
    const double* A1 = a.A[1];
    const double* C1 = a.C[1];
    const int n1 = a.n[1], b1 = n1 + 1;
    for (int p1 = 0; p1 <= n1; ++p1) {   // stiffness along axis 0, mass along 1
      const double ur = op_u<2>(a, u, G, e, r[0], p1, 0);
      double t = 0.0;
      for (int p0 = 0; p0 <= n0; ++p0)
        if (p0 != r[0]) t += A0[r[0] * b0 + p0] * (op_u<2>(a, u, G, e, p0, p1, 0) - ur);
      acc += a.scale[0] * C1[r[1] * b1 + p1] * t;
    }
    for (int p0 = 0; p0 <= n0; ++p0) {   // stiffness along axis 1 and mass, then mass along 0
      const double ur = op_u<2>(a, u, G, e, p0, r[1], 0);
      double t = 0.0, mm = 0.0;
      for (int p1 = 0; p1 <= n1; ++p1) {
        const double v = op_u<2>(a, u, G, e, p0, p1, 0);
        if (p1 != r[1]) t += A1[r[1] * b1 + p1] * (v - ur);
        mm += C1[r[1] * b1 + p1] * v;
      }
      acc += C0[r[0] * b0 + p0] * (a.scale[1] * t + a.alpha * mm);
    }
  } else {
    const double* A1 = a.A[1];
    const double* C1 = a.C[1];
    const double* A2 = a.A[2];
    const double* C2 = a.C[2];
    const int n1 = a.n[1], b1 = n1 + 1, n2 = a.n[2], b2 = n2 + 1;
    for (int p1 = 0; p1 <= n1; ++p1)
      for (int p2 = 0; p2 <= n2; ++p2) {
        const double ur = op_u<3>(a, u, G, e, r[0], p1, p2);
        double t = 0.0;
        for (int p0 = 0; p0 <= n0; ++p0)
          if (p0 != r[0]) t += A0[r[0] * b0 + p0] * (op_u<3>(a, u, G, e, p0, p1, p2) - ur);
        acc += a.scale[0] * C1[r[1] * b1 + p1] * C2[r[2] * b2 + p2] * t;
      }
    for (int p0 = 0; p0 <= n0; ++p0)
      for (int p2 = 0; p2 <= n2; ++p2) {
        const double ur = op_u<3>(a, u, G, e, p0, r[1], p2);
        double t = 0.0;
        for (int p1 = 0; p1 <= n1; ++p1)
          if (p1 != r[1]) t += A1[r[1] * b1 + p1] * (op_u<3>(a, u, G, e, p0, p1, p2) - ur);
        acc += a.scale[1] * C0[r[0] * b0 + p0] * C2[r[2] * b2 + p2] * t;
      }
    for (int p0 = 0; p0 <= n0; ++p0)
      for (int p1 = 0; p1 <= n1; ++p1) {
        const double ur = op_u<3>(a, u, G, e, p0, p1, r[2]);
        double t = 0.0, mm = 0.0;
        for (int p2 = 0; p2 <= n2; ++p2) {
          const double v = op_u<3>(a, u, G, e, p0, p1, p2);
          if (p2 != r[2]) t += A2[r[2] * b2 + p2] * (v - ur);
          mm += C2[r[2] * b2 + p2] * v;
        }
        acc += C0[r[0] * b0 + p0] * C1[r[1] * b1 + p1] * (a.scale[2] * t + a.alpha * mm);
      }
  }
  return acc;
}

template <int N>
__global__ __launch_bounds__(256) void op_kernel(OpArgs a, long long total) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  OpGeom G;
  long long per = 1;
  for (int i = N - 1; i >= 0; --i) {
    G.stride[i] = per;
    per *= a.m[i];
  }
  const long long rhs = idx / per;
  long long rem = idx - rhs * per;
  const double* u = a.u + rhs * per;
  int ne[3] = {1, 1, 1}, el[3][2], rl[3][2];
  for (int i = 0; i < N; ++i) {
    const int q = (int)(rem / G.stride[i]);
    rem -= (long long)q * G.stride[i];
    const int g = q + 1, ni = a.n[i];
    if (g % ni == 0) {
      ne[i] = 2;
      el[i][0] = g / ni;      rl[i][0] = ni;   // right end of element g/n
      el[i][1] = g / ni + 1;  rl[i][1] = 0;    // left end of the next one
    } else {
      el[i][0] = g / ni + 1;  rl[i][0] = g % ni;
    }
  }
  double acc = 0.0;
  for (int c0 = 0; c0 < ne[0]; ++c0)
    for (int c1 = 0; c1 < (N > 1 ? ne[1] : 1); ++c1)
      for (int c2 = 0; c2 < (N > 2 ? ne[2] : 1); ++c2) {
        int e[3] = {el[0][c0], N > 1 ? el[1][c1] : 1, N > 2 ? el[2][c2] : 1};
        int r[3] = {rl[0][c0], N > 1 ? rl[1][c1] : 0, N > 2 ? rl[2][c2] : 0};
        acc += op_element<N>(a, u, G, e, r);
      }
  const double res = a.f ? a.f[idx] - acc : acc;
  if (a.out_f32) static_cast<float*>(a.out)[idx] = (float)res;
  else static_cast<double*>(a.out)[idx] = res;
}

// ---------------------------------------------------------------------------
// 2D operator by element tiles.  A workgroup owns the points of TE0 x TE1
// elements (positions n(E-1)+1 .. n(E-1+TE) per axis); the element after the
// tile along each axis also touches owned points (its first node line), so
// the workgroup stages u for (TE0+1) x (TE1+1) elements in LDS.
//   Phase 1, per element e and local index i:
//     D0_e[i][r1] = sum_{r0 != i} A0[i][r0] (u[r0][r1] - u[i][r1])   (stiffness along 0)
//     D1_e[r0][i] = sum_{r1 != i} A1[i][r1] (u[r0][r1] - u[r0][i])   (stiffness along 1)
//     M1_e[r0][i] = sum_{r1} C1[i][r1] u[r0][r1]                     (mass along 1)
//   Phase 2, per owned point, summed over the 1, 2 or 4 elements holding it
//   (local indices a0, a1):
//     s0 sum_{r1} C1[a1][r1] D0_e[a0][r1] + sum_{r0} C0[a0][r0] (s1 D1_e[r0][a1] + alpha M1_e[r0][a1])
// which is the element row of s0 A0 (x) C1 + s1 C0 (x) A1 + alpha C0 (x) C1 with
// every stiffness factor applied to u first.
// ---------------------------------------------------------------------------

struct Tile2 {
  int TE0, TE1, nt0, nt1;
};

__global__ __launch_bounds__(256) void op2_tiled_kernel(OpArgs a, Tile2 tl) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n0 = a.n[0], n1 = a.n[1], b0 = n0 + 1, b1 = n1 + 1;
  const int K0 = a.K[0], K1 = a.K[1], m0 = a.m[0], m1 = a.m[1];
  const int t0 = blockIdx.x / tl.nt1, t1 = blockIdx.x - t0 * tl.nt1;
  const long long roff = (long long)blockIdx.y * m0 * m1;
  const int E0 = t0 * tl.TE0 + 1, E1 = t1 * tl.TE1 + 1;        // first element (1-based)
  const int ne0 = min(tl.TE0 + 1, K0 - E0 + 1), ne1 = min(tl.TE1 + 1, K1 - E1 + 1);
  const int P0 = n0 * ne0 + 1, P1 = n1 * ne1 + 1;              // staged points per axis
  const int g00 = n0 * (E0 - 1), g10 = n1 * (E1 - 1);          // position of local point 0
  const int eb = b0 * b1;                                       // values per element block

  double* A0 = reinterpret_cast<double*>(smem);
  double* C0 = A0 + 100;
  double* A1 = C0 + 100;
  double* C1 = A1 + 100;
  double* U = C1 + 100;                                         // [P0][P1]
  double* I = U + ((P0 * P1 + 1) & ~1);                          // [elements][3][b0 b1]
  const int tid = threadIdx.x, nthr = blockDim.x;

  for (int i = tid; i < b0 * b0; i += nthr) {
    A0[i] = a.A[0][i];
    C0[i] = a.C[0][i];
  }
  for (int i = tid; i < b1 * b1; i += nthr) {
    A1[i] = a.A[1][i];
    C1[i] = a.C[1][i];
  }
  const double* __restrict__ u = a.u + roff;
  for (int i = tid; i < P0 * P1; i += nthr) {
    const int i0 = i / P1, i1 = i - i0 * P1;
    const int g0 = g00 + i0, g1 = g10 + i1;
    double v = 0.0;
    if (g0 >= 1 && g0 <= m0 && g1 >= 1 && g1 <= m1) v = u[(long long)(g0 - 1) * m1 + (g1 - 1)];
    U[i] = v;
  }
  __syncthreads();

  // phase 1
  const int bmax = b0 > b1 ? b0 : b1;
  const int tasks = ne0 * ne1 * bmax;
  for (int task = tid; task < tasks; task += nthr) {
    const int el = task / bmax, i = task - el * bmax;
    const int l0 = el / ne1, l1 = el - l0 * ne1;
    const double* Ue = U + (l0 * n0) * P1 + l1 * n1;             // element origin
    double* D0 = I + (size_t)el * 3 * eb;
    double* D1 = D0 + eb;
    double* M1 = D1 + eb;
    if (i < b0) {
      const double* Ai = A0 + i * b0;
      for (int r1 = 0; r1 < b1; ++r1) {
        const double ui = Ue[i * P1 + r1];
        double t = 0.0;
        for (int r0 = 0; r0 < b0; ++r0)
          if (r0 != i) t += Ai[r0] * (Ue[r0 * P1 + r1] - ui);
        D0[i * b1 + r1] = t;
      }
    }
    if (i < b1) {
      const double* Ai = A1 + i * b1;
      const double* Ci = C1 + i * b1;
      for (int r0 = 0; r0 < b0; ++r0) {
        const double* row = Ue + r0 * P1;
        const double ui = row[i];
        double t = 0.0, mm = 0.0;
        for (int r1 = 0; r1 < b1; ++r1) {
          const double v = row[r1];
          if (r1 != i) t += Ai[r1] * (v - ui);
          mm += Ci[r1] * v;
        }
        D1[r0 * b1 + i] = t;
        M1[r0 * b1 + i] = mm;
      }
    }
  }
  __syncthreads();

  // phase 2: owned points p = 1 .. n TE per axis (local), inside the domain
  const double s0 = a.scale[0], s1 = a.scale[1], al = a.alpha;
  const int own0 = n0 * tl.TE0, own1 = n1 * tl.TE1;
  const int cnt = own0 * own1;
  const double* __restrict__ f = a.f ? a.f + roff : nullptr;
  for (int i = tid; i < cnt; i += nthr) {
    const int p0 = i / own1 + 1, p1 = i - (p0 - 1) * own1 + 1;
    const int g0 = g00 + p0, g1 = g10 + p1;
    if (g0 > m0 || g1 > m1) continue;
    int el0[2], a0s[2], n0e = 1, el1[2], a1s[2], n1e = 1;
    if (p0 % n0 == 0) {
      el0[0] = p0 / n0 - 1; a0s[0] = n0;
      el0[1] = p0 / n0;     a0s[1] = 0;
      n0e = (el0[1] < ne0) ? 2 : 1;
    } else {
      el0[0] = p0 / n0; a0s[0] = p0 % n0;
    }
    if (p1 % n1 == 0) {
      el1[0] = p1 / n1 - 1; a1s[0] = n1;
      el1[1] = p1 / n1;     a1s[1] = 0;
      n1e = (el1[1] < ne1) ? 2 : 1;
    } else {
      el1[0] = p1 / n1; a1s[0] = p1 % n1;
    }
    double acc = 0.0;
    for (int c0 = 0; c0 < n0e; ++c0)
      for (int c1 = 0; c1 < n1e; ++c1) {
        const int el = el0[c0] * ne1 + el1[c1];
        const int a0 = a0s[c0], a1 = a1s[c1];
        const double* D0 = I + (size_t)el * 3 * eb;
        const double* D1 = D0 + eb;
        const double* M1 = D1 + eb;
        double t = 0.0;
        for (int r1 = 0; r1 < b1; ++r1) t += C1[a1 * b1 + r1] * D0[a0 * b1 + r1];
        double w = 0.0;
        for (int r0 = 0; r0 < b0; ++r0)
          w += C0[a0 * b0 + r0] * (s1 * D1[r0 * b1 + a1] + al * M1[r0 * b1 + a1]);
        acc += s0 * t + w;
      }
    const long long idx = (long long)(g0 - 1) * m1 + (g1 - 1);
    const double res = f ? f[idx] - acc : acc;
    if (a.out_f32) static_cast<float*>(a.out)[roff + idx] = (float)res;
    else static_cast<double*>(a.out)[roff + idx] = res;
  }
}

// ---------------------------------------------------------------------------
// 2D operator for equal orders NO, sum-factorised along the two axes with the
// assembled 1D matrices (A_g = sum_e A_e, C_g = sum_e C_e):
//   L u = s0 (A0_g (x) C1_g) u + (C0_g (x) (s1 A1_g + alpha C1_g)) u
//       = s0 A0_g P + C0_g D,   P = C1_g u,  D = s1 A1_g u + alpha P
// (P and D along axis 1, then the axis-0 products).  A tile owns TE0 x TE1
// elements, i.e. the points (NO E0, NO (E0 + TE0)] x (NO E1, NO (E1 + TE1)].
//   1. one task per (row, element e along axis 1) of the rows the tile needs
//      (NO E0 .. NO (E0 + TE0 + 1)): reads the element's points and the next
//      element's from global memory and writes P and D at the element's
//      interior points and right node (the node gets both elements' rows);
//   2. one task per (owned column, element e along axis 0), columns fastest
//      (coalesced f reads and r writes): r = f - s0 A0_g P - C0_g D at the
//      element's interior rows and right node.
// Stiffness products use the difference form sum_{q != r} A[r][q] (x_q - x_r)
// (rows of A sum to zero).  Every output has one writer: deterministic.
// ---------------------------------------------------------------------------

constexpr int kOpSfThreads = 512;

// The 1D matrices of the two axes by value: kernel arguments are constant
// memory, read with scalar loads as uniform operands.
struct OpMats {
  double A0[100], C0[100], A1[100], C1[100];
};

template <int NO>
struct OpSfShape {
  static constexpr int B = NO + 1;
  static constexpr int TE1 = 64 / NO;                 // owned columns NO TE1 <= 64
  static constexpr int W = NO * TE1;
  static constexpr int rows(int te0) { return NO * (te0 + 1) + 1; }
  static constexpr bool fits(int te0) {
    return 2 * rows(te0) * W * 8 <= 80 * 1024 && rows(te0) * TE1 <= 2 * kOpSfThreads;
  }
  static constexpr int pick() {
    int t = 1;
    for (int c = 1; c <= 64; ++c)
      if (fits(c)) t = c;
    return t;
  }
  static constexpr int TE0 = pick();
  static constexpr int R = rows(TE0);
  static constexpr int LDS = 2 * R * W * 8;
};

// MASS: also writes (C0_g (x) C1_g) u, the plain mass product, to a.elem
// (double; the planes of the 3D operator need both).
template <int NO, bool MASS = false>
__global__ __launch_bounds__(kOpSfThreads) __attribute__((amdgpu_waves_per_eu(4))) void op2_sf_kernel(
    OpArgs a, OpMats mt, int nt1) {
  using SH = OpSfShape<NO>;
  constexpr int B = SH::B, TE0 = SH::TE0, TE1 = SH::TE1, W = SH::W, R = SH::R;
  extern __shared__ __align__(16) unsigned char smem[];
  double* P = reinterpret_cast<double*>(smem);   // [R][W]
  double* D = P + R * W;                         // [R][W]
  const int K0 = a.K[0], K1 = a.K[1], m0 = a.m[0], m1 = a.m[1];
  // Workgroups are dealt to the eight XCDs in turn; give each XCD a
  // contiguous run of tiles (row-major), so that the halo rows and columns a
  // tile shares with its neighbours are read once into that XCD's L2.
  const int nblk = (int)gridDim.x, qx = nblk >> 3, rx = nblk & 7;
  const int xcd = (int)blockIdx.x & 7, jx = (int)blockIdx.x >> 3;
  const int tile = xcd * qx + (xcd < rx ? xcd : rx) + jx;
  const int t0 = tile / nt1, t1 = tile - t0 * nt1;
  const long long roff = (long long)blockIdx.y * m0 * m1;
  const int E0 = t0 * TE0, E1 = t1 * TE1;   // elements before the tile
  const int tid = threadIdx.x;
  // The 1D matrices are uniform operands (scalar loads of the kernel
  // arguments); the task loops run with uniform bounds and mask their data
  // accesses.
  const double* A0 = mt.A0;
  const double* C0 = mt.C0;
  const double* A1 = mt.A1;
  const double* C1 = mt.C1;
  const double s0 = a.scale[0], s1 = a.scale[1], al = a.alpha;
  const double* __restrict__ u = a.u + roff;
  const double* __restrict__ f = a.f ? a.f + roff : nullptr;

  // f of this lane's first phase-2 task, loaded now: its latency overlaps
  // phase 1 instead of following the barrier
  double fpre[NO];
  {
    const int e = tid / W, cl = tid - e * W;
    const int g1 = NO * E1 + cl + 1, E = E0 + e + 1;
    const bool ok = f && tid < W * TE0 && g1 <= m1 && E <= K0;
#pragma unroll
    for (int r = 1; r <= NO; ++r) {
      const int g0 = NO * (E - 1) + r;
      fpre[r - 1] = (ok && g0 <= m0) ? f[(long long)(g0 - 1) * m1 + (g1 - 1)] : 0.0;
    }
  }

  // 1. axis 1: P = C1_g u, D = s1 A1_g u + alpha P on rows NO E0 + i
  for (int t0 = 0; t0 < R * TE1; t0 += kOpSfThreads) {
    const int task = t0 + tid;
    const bool task_ok = task < R * TE1;
    const int i = task_ok ? task / TE1 : 0, e = task_ok ? task - i * TE1 : 0;
    const int g0 = NO * E0 + i;                  // row (0 and m0 + 1: boundary)
    const int E = E1 + e + 1;                    // element along axis 1 (1-based)
    double x[B], y[B];                           // element E, element E + 1
    const bool row_ok = task_ok && g0 >= 1 && g0 <= m0 && E <= K1;
    const double* ur = u + (long long)(g0 - 1) * m1;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int ga = NO * (E - 1) + q, gb = NO * E + q;
      x[q] = (row_ok && ga >= 1 && ga <= m1) ? ur[ga - 1] : 0.0;
      y[q] = (row_ok && gb >= 1 && gb <= m1 && q > 0) ? ur[gb - 1] : 0.0;
    }
    y[0] = x[NO];
    double* Pr = P + i * W + NO * e;             // local column NO e + r - 1 for point r
    double* Dr = D + i * W + NO * e;
#pragma unroll
    for (int r = 1; r < NO; ++r) {
      double c = 0.0, d = 0.0;
#pragma unroll
      for (int q = 0; q < B; ++q) {
        c += C1[r * B + q] * x[q];
        if (q != r) d += A1[r * B + q] * (x[q] - x[r]);
      }
      if (task_ok) {
        Pr[r - 1] = c;
        Dr[r - 1] = s1 * d + al * c;
      }
    }
    {   // right node: last row of element E plus first row of element E + 1
      double c = 0.0, d = 0.0;
#pragma unroll
      for (int q = 0; q < B; ++q) {
        c += C1[NO * B + q] * x[q] + C1[q] * y[q];
        if (q != NO) d += A1[NO * B + q] * (x[q] - x[NO]);
        if (q != 0) d += A1[q] * (y[q] - y[0]);
      }
      if (task_ok) {
        Pr[NO - 1] = c;
        Dr[NO - 1] = s1 * d + al * c;
      }
    }
  }
  __syncthreads();

  // 2. axis 0: r = f - s0 A0_g P - C0_g D at rows NO (E - 1) + r, E = E0 + e + 1
  for (int t0 = 0; t0 < W * TE0; t0 += kOpSfThreads) {
    const int task = t0 + tid;
    const int e = task / W, cl = task - e * W;
    const int g1 = NO * E1 + cl + 1;             // column
    const int E = E0 + e + 1;
    const bool ok = task < W * TE0 && g1 <= m1 && E <= K0;
    double p[B], d[B], pn[B], dn[B];
    // (the plain mass product needs C1_g u without alpha: P holds it)
    const int l0 = ok ? NO * e : 0;              // local row of the element's first point
    const int lc = ok ? cl : 0;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      p[q] = P[(l0 + q) * W + lc];
      d[q] = D[(l0 + q) * W + lc];
      pn[q] = P[(l0 + NO + q) * W + lc];
      dn[q] = D[(l0 + NO + q) * W + lc];
    }
#pragma unroll
    for (int r = 1; r <= NO; ++r) {
      const int g0 = NO * (E - 1) + r;
      double ap = 0.0, cd = 0.0;
#pragma unroll
      for (int q = 0; q < B; ++q) {
        if (q != r) ap += A0[r * B + q] * (p[q] - p[r]);
        cd += C0[r * B + q] * d[q];
      }
      if (r == NO) {   // the node also takes the first row of element E + 1
#pragma unroll
        for (int q = 1; q < B; ++q) ap += A0[q] * (pn[q] - pn[0]);
#pragma unroll
        for (int q = 0; q < B; ++q) cd += C0[q] * dn[q];
      }
      const double lu = s0 * ap + cd;
      double cm = 0.0;   // C0_g P: the mass product (MASS)
      if constexpr (MASS) {
#pragma unroll
        for (int q = 0; q < B; ++q) cm += C0[r * B + q] * p[q];
        if (r == NO) {
#pragma unroll
          for (int q = 0; q < B; ++q) cm += C0[q] * pn[q];
        }
      }
      if (ok && g0 <= m0) {
        const long long idx = (long long)(g0 - 1) * m1 + (g1 - 1);
        if constexpr (MASS) a.elem[roff + idx] = cm;
        const double fv = t0 == 0 ? fpre[r - 1] : (f ? f[idx] : 0.0);
        const double res = f ? fv - lu : lu;
        if (a.out_f32) static_cast<float*>(a.out)[roff + idx] = (float)res;
        else static_cast<double*>(a.out)[roff + idx] = res;
      }
    }
  }
}

template <int NO, bool MASS = false>
hipError_t launch_op2_sf(const OpArgs& a, hipStream_t s) {
  using SH = OpSfShape<NO>;
  static bool raised = false;   // benign race: every caller sets the same value
  if (!raised) {
    hipError_t e = hipFuncSetAttribute((const void*)op2_sf_kernel<NO, MASS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, SH::LDS);
    if (e != hipSuccess) return e;
    raised = true;
  }
  if (!a.hA[0] || !a.hC[0] || !a.hA[1] || !a.hC[1]) return hipErrorInvalidValue;
  OpMats mt;
  for (int i = 0; i < SH::B * SH::B; ++i) {
    mt.A0[i] = a.hA[0][i];
    mt.C0[i] = a.hC[0][i];
    mt.A1[i] = a.hA[1][i];
    mt.C1[i] = a.hC[1][i];
  }
  const int nt0 = (a.K[0] + SH::TE0 - 1) / SH::TE0, nt1 = (a.K[1] + SH::TE1 - 1) / SH::TE1;
  if (MASS && !a.elem) return hipErrorInvalidValue;
  hipLaunchKernelGGL((op2_sf_kernel<NO, MASS>), dim3((unsigned)(nt0 * nt1), (unsigned)a.nrhs),
                     dim3(kOpSfThreads), SH::LDS, s, a, mt, nt1);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3D operator for equal orders NO, by planes and lines:
//   L u = s0 A0 (x) C1 (x) C2 u + C0 (x) [ s1 A1 (x) C2 + C1 (x) (s2 A2 + alpha C2) ] u
//       = s0 A0_g Z1 + C0_g Z2,   Z1 = (C1 (x) C2) u,   Z2 = L12 u
// along axis 0, where Z1 and Z2 are the 2D mass product and the 2D operator
// (with alpha) of every plane of constant axis-0 index: one run of the tiled
// 2D kernel computes both (its planes as right-hand sides), and op3_axis0_kernel
// applies the axis-0 factors element by element (stiffness in difference
// form) and subtracts from f.  Z1, Z2: the operator's element buffer
// (2 grids of one right-hand side); every output has one writer.
// ---------------------------------------------------------------------------

// One lane per (point of the axis-1/2 plane, run of kOp3Run elements along
// axis 0): element e's outputs at positions n(e-1)+r, r = 1..n (the node n e
// also takes the first row of element e+1).  The lane walks its run and keeps
// the next element's values for the following one, so every position of Z1
// and Z2 is read about once (a lane per element read its neighbour's rows
// again, from HBM: the lane that owns them runs a plane's worth of work later).
constexpr int kOp3Run = 16;

template <int NO>
__global__ __launch_bounds__(256) void op3_axis0_kernel(const double* __restrict__ Z1,
                                                        const double* __restrict__ Z2,
                                                        const double* __restrict__ f, void* out,
                                                        int out_f32, int K0, int m0, long long plane,
                                                        double s0, OpMats mt) {
  constexpr int B = NO + 1;
  const int nrun = (K0 + kOp3Run - 1) / kOp3Run;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= plane * nrun) return;
  const long long pt = t % plane;
  const int e0 = (int)(t / plane) * kOp3Run + 1;
  const int e1 = e0 + kOp3Run - 1 < K0 ? e0 + kOp3Run - 1 : K0;
  auto zat = [&](const double* Z, int g) -> double {   // position g = 0..nK0 (0 and nK0: boundary)
    return (g >= 1 && g <= m0) ? Z[(long long)(g - 1) * plane + pt] : 0.0;
  };
  const double* A0 = mt.A0;
  const double* C0 = mt.C0;
  double z1[B], z2[B], z1n[B], z2n[B];
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int g = NO * (e0 - 1) + q;
    z1[q] = zat(Z1, g);
    z2[q] = zat(Z2, g);
  }
  for (int e = e0; e <= e1; ++e) {
    z1n[0] = z1[NO];
    z2n[0] = z2[NO];
#pragma unroll
    for (int q = 1; q < B; ++q) {
      const int g = NO * e + q;
      z1n[q] = e < K0 ? zat(Z1, g) : 0.0;
      z2n[q] = e < K0 ? zat(Z2, g) : 0.0;
    }
    if (e == K0) {   // no element e+1: its row 0 (the boundary) contributes nothing
      z1n[0] = 0.0;
      z2n[0] = 0.0;
    }
#pragma unroll
    for (int r = 1; r <= NO; ++r) {
      const int g = NO * (e - 1) + r;
      if (g > m0) break;
      double ap = 0.0, cd = 0.0;
#pragma unroll
      for (int q = 0; q < B; ++q) {
        if (q != r) ap += A0[r * B + q] * (z1[q] - z1[r]);
        cd += C0[r * B + q] * z2[q];
      }
      if (r == NO) {   // the node also takes row 0 of element e+1
#pragma unroll
        for (int q = 1; q < B; ++q) ap += A0[q] * (z1n[q] - z1n[0]);
#pragma unroll
        for (int q = 0; q < B; ++q) cd += C0[q] * z2n[q];
      }
      const long long idx = (long long)(g - 1) * plane + pt;
      const double lu = s0 * ap + cd;
      const double res = f ? f[idx] - lu : lu;
      if (out_f32) static_cast<float*>(out)[idx] = (float)res;
      else static_cast<double*>(out)[idx] = res;
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      z1[q] = z1n[q];
      z2[q] = z2n[q];
    }
  }
}

template <int NO>
hipError_t launch_op3_order(const OpArgs& a, hipStream_t s) {
  const long long plane = (long long)a.m[1] * a.m[2];
  const long long per = (long long)a.m[0] * plane;
  if (!a.hA[0] || !a.hC[0] || a.m[0] > 65535) return hipErrorInvalidValue;
  double* Z1 = a.elem;
  double* Z2 = a.elem + per;
  OpMats mt{};
  for (int i = 0; i < (NO + 1) * (NO + 1); ++i) {
    mt.A0[i] = a.hA[0][i];
    mt.C0[i] = a.hC[0][i];
  }
  // the planes of constant axis-0 index as the 2D kernel's right-hand sides
  OpArgs b{};
  b.N = 2;
  b.f = nullptr;
  b.out_f32 = 0;
  b.nrhs = a.m[0];
  for (int i = 0; i < 2; ++i) {
    b.n[i] = a.n[i + 1];
    b.K[i] = a.K[i + 1];
    b.m[i] = a.m[i + 1];
    b.A[i] = a.A[i + 1];
    b.C[i] = a.C[i + 1];
    b.hA[i] = a.hA[i + 1];
    b.hC[i] = a.hC[i + 1];
  }
  const long long lanes = plane * ((a.K[0] + kOp3Run - 1) / kOp3Run);
  const unsigned blocks = (unsigned)((lanes + 255) / 256);
  b.scale[0] = a.scale[1];
  b.scale[1] = a.scale[2];
  b.alpha = a.alpha;
  b.out = Z2;
  b.elem = Z1;   // the mass product C1 (x) C2 u, from the same tiles
  for (int r = 0; r < a.nrhs; ++r) {
    b.u = a.u + r * per;
    hipError_t e = launch_op2_sf<NO, true>(b, s);
    if (e != hipSuccess) return e;
    const double* f = a.f ? a.f + r * per : nullptr;
    void* out = a.out_f32 ? (void*)(static_cast<float*>(a.out) + r * per)
                          : (void*)(static_cast<double*>(a.out) + r * per);
    hipLaunchKernelGGL(op3_axis0_kernel<NO>, dim3(blocks), dim3(256), 0, s, Z1, Z2, f, out, a.out_f32,
                       a.K[0], a.m[0], plane, a.scale[0], mt);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// LDS bytes of a 2D tile of TE0 x TE1 owned elements.
size_t tile2_lds(int n0, int n1, int TE0, int TE1) {
  const size_t P0 = (size_t)n0 * (TE0 + 1) + 1, P1 = (size_t)n1 * (TE1 + 1) + 1;
  const size_t els = (size_t)(TE0 + 1) * (TE1 + 1);
  return (400 + ((P0 * P1 + 1) & ~size_t(1)) + els * 3 * (n0 + 1) * (n1 + 1)) * sizeof(double);
}

// u += delta and per-workgroup partial sums of delta^2 and u^2 (u after the update).
__global__ __launch_bounds__(256) void axpy_norms_kernel(const float* delta, double* u,
                                                         long long count, double* partial) {
  __shared__ double sd[4], su[4];
  double dd = 0.0, uu = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (long long)gridDim.x * 256) {
    const double d = (double)delta[i];
    const double v = u[i] + d;
    u[i] = v;
    dd += d * d;
    uu += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    dd += __shfl_xor(dd, off, 64);
    uu += __shfl_xor(uu, off, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sd[wave] = dd;
    su[wave] = uu;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sd[0] + sd[1] + sd[2] + sd[3];
    partial[2 * blockIdx.x + 1] = su[0] + su[1] + su[2] + su[3];
  }
}

__global__ void reduce_pairs_kernel(const double* partial, int nparts, double* out) {
  __shared__ double sd[256], su[256];
  double dd = 0.0, uu = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) {
    dd += partial[2 * i];
    uu += partial[2 * i + 1];
  }
  sd[threadIdx.x] = dd;
  su[threadIdx.x] = uu;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sd[threadIdx.x] += sd[threadIdx.x + s];
      su[threadIdx.x] += su[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sd[0];
    out[1] = su[0];
  }
}

__global__ __launch_bounds__(256) void axpy_kernel(const float* delta, double* u, long long count) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (long long)gridDim.x * 256)
    u[i] += (double)delta[i];
}

// Boundary lift of non-homogeneous Dirichlet data (Section 2, paragraph 4:
// the general case reduces to zero data through f^h).  For every interior
// point q: out[q] = f[q] - sum over the elements E containing q and the
// local nodes c of E on the boundary of K_E[r(q), c] b[c], with K_E the
// scaled element matrix sum_d s_d A_d (x)_{e != d} C_e + alpha (x)_e C_e and
// b the boundary values on the extended grid (m_d + 2 points per axis).
// Points whose elements do not touch the boundary keep f.
template <int N>
__global__ void dirichlet_lift_kernel(OpArgs a, const double* __restrict__ bext,
                                      const double* __restrict__ f, double* __restrict__ out,
                                      long long total) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= total) return;
  long long rem = t;
  int g[3];                       // extended index along each axis, 1..m_d
  long long eper = 1;
  for (int d = N - 1; d >= 0; --d) {
    g[d] = (int)(rem % a.m[d]) + 1;
    rem /= a.m[d];
    eper *= a.m[d] + 2;
  }
  const long long rhs = rem;
  // candidate elements along each axis: one (interior point of an element)
  // or two (mesh node)
  int e0[3], ne[3];
  bool near = false;
  for (int d = 0; d < N; ++d) {
    const int n = a.n[d];
    if (g[d] % n == 0) {
      e0[d] = g[d] / n - 1;
      ne[d] = 2;
    } else {
      e0[d] = g[d] / n;
      ne[d] = 1;
    }
    if (e0[d] == 0 || e0[d] + ne[d] - 1 == a.K[d] - 1) near = true;
  }
  const double fv = f ? f[t] : 0.0;
  if (!near) {
    out[t] = fv;
    return;
  }
  const double* bx = bext + rhs * eper;
  double acc = 0.0;
  const int ncomb = (N > 0 ? ne[0] : 1) * (N > 1 ? ne[1] : 1) * (N > 2 ? ne[2] : 1);
  for (int comb = 0; comb < ncomb; ++comb) {
    int cc = comb;
    int r[3], e[3];
    for (int d = N - 1; d >= 0; --d) {
      e[d] = e0[d] + cc % ne[d];
      cc /= ne[d];
      r[d] = g[d] - a.n[d] * e[d];
    }
    // local nodes c of element e on the boundary
    int nl = 1;
    for (int d = 0; d < N; ++d) nl *= a.n[d] + 1;
    for (int lc = 0; lc < nl; ++lc) {
      int c[3], G[3];
      int x = lc;
      bool bnd = false;
      for (int d = N - 1; d >= 0; --d) {
        c[d] = x % (a.n[d] + 1);
        x /= a.n[d] + 1;
        G[d] = a.n[d] * e[d] + c[d];
        if (G[d] == 0 || G[d] == a.m[d] + 1) bnd = true;
      }
      if (!bnd) continue;
      long long bi = 0;
      for (int d = 0; d < N; ++d) bi = bi * (a.m[d] + 2) + G[d];
      const double bv = bx[bi];
      // K_E[r, c]
      double mass = 1.0;
      for (int d = 0; d < N; ++d) mass *= a.C[d][r[d] * (a.n[d] + 1) + c[d]];
      double kv = a.alpha * mass;
      for (int d = 0; d < N; ++d) {
        double term = a.scale[d] * a.A[d][r[d] * (a.n[d] + 1) + c[d]];
        for (int o = 0; o < N; ++o)
          if (o != d) term *= a.C[o][r[o] * (a.n[o] + 1) + c[o]];
        kv += term;
      }
      acc += kv * bv;
    }
  }
  out[t] = fv - acc;
}

}  // namespace

hipError_t launch_operator(const OpArgs& a, hipStream_t s) {
  long long total = a.nrhs;
  for (int i = 0; i < a.N; ++i) total *= a.m[i];
  if (total == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  switch (a.N) {
    case 1: hipLaunchKernelGGL(op_kernel<1>, dim3(blocks), dim3(256), 0, s, a, total); break;
    case 2: {
      if (a.n[0] == a.n[1]) {
        switch (a.n[0]) {
          case 1: return launch_op2_sf<1>(a, s);
          case 2: return launch_op2_sf<2>(a, s);
          case 3: return launch_op2_sf<3>(a, s);
          case 4: return launch_op2_sf<4>(a, s);
          case 5: return launch_op2_sf<5>(a, s);
          case 6: return launch_op2_sf<6>(a, s);
          case 7: return launch_op2_sf<7>(a, s);
          case 8: return launch_op2_sf<8>(a, s);
          case 9: return launch_op2_sf<9>(a, s);
          default: break;
        }
      }
      // unequal orders: largest square-ish tile that keeps LDS within 64 KB
      Tile2 tl{1, 1, 0, 0};
      for (int te = 16; te >= 1; --te) {
        if (tile2_lds(a.n[0], a.n[1], te, te) <= 64 * 1024) {
          tl.TE0 = tl.TE1 = te;
          break;
        }
      }
      tl.nt0 = (a.K[0] + tl.TE0 - 1) / tl.TE0;
      tl.nt1 = (a.K[1] + tl.TE1 - 1) / tl.TE1;
      const size_t lds = tile2_lds(a.n[0], a.n[1], tl.TE0, tl.TE1);
      static bool raised = false;
      if (!raised) {
        hipError_t e = hipFuncSetAttribute((const void*)op2_tiled_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        raised = true;
      }
      hipLaunchKernelGGL(op2_tiled_kernel, dim3((unsigned)(tl.nt0 * tl.nt1), (unsigned)a.nrhs),
                         dim3(256), lds, s, a, tl);
      break;
    }
    case 3:
      if (a.elem && a.n[0] == a.n[1] && a.n[1] == a.n[2]) {
        switch (a.n[0]) {
          case 1: return launch_op3_order<1>(a, s);
          case 2: return launch_op3_order<2>(a, s);
          case 3: return launch_op3_order<3>(a, s);
          case 4: return launch_op3_order<4>(a, s);
          case 5: return launch_op3_order<5>(a, s);
          case 6: return launch_op3_order<6>(a, s);
          case 7: return launch_op3_order<7>(a, s);
          case 8: return launch_op3_order<8>(a, s);
          case 9: return launch_op3_order<9>(a, s);
          default: break;
        }
      }
      hipLaunchKernelGGL(op_kernel<3>, dim3(blocks), dim3(256), 0, s, a, total);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_norms(const float* delta, double* u, long long count, double* partial,
                        int nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(axpy_norms_kernel, dim3(nparts), dim3(256), 0, s, delta, u, count, partial);
  hipLaunchKernelGGL(reduce_pairs_kernel, dim3(1), dim3(256), 0, s, partial, nparts, out);
  return hipGetLastError();
}

hipError_t launch_axpy(const float* delta, double* u, long long count, hipStream_t s) {
  long long blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, delta, u, count);
  return hipGetLastError();
}

hipError_t launch_dirichlet_lift(const OpArgs& a, const double* bext, const double* f,
                                 double* out, hipStream_t s) {
  long long total = a.nrhs;
  for (int i = 0; i < a.N; ++i) total *= a.m[i];
  if (total == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  switch (a.N) {
    case 1: hipLaunchKernelGGL(dirichlet_lift_kernel<1>, dim3(blocks), dim3(256), 0, s, a, bext, f, out, total); break;
    case 2: hipLaunchKernelGGL(dirichlet_lift_kernel<2>, dim3(blocks), dim3(256), 0, s, a, bext, f, out, total); break;
    case 3: hipLaunchKernelGGL(dirichlet_lift_kernel<3>, dim3(blocks), dim3(256), 0, s, a, bext, f, out, total); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {

// One axis of any boundary condition: global point g = 0..nK of the axis
// (element e = 1..K holds the points n(e-1)..ne, local index g - n(e-1));
// the unknowns are g = 1..nK-1 (Dirichlet; the boundary values are zero),
// g = 0..nK-1 with nK identified with 0 (periodic) or g = 0..nK (Neumann).
__global__ __launch_bounds__(256) void axis_local_kernel(AxisLocal a, const double* __restrict__ in,
                                                         double* out, const double* add, double cc,
                                                         double ca, long long total) {
  const int n = a.n, K = a.K, nb = n + 1, nK = n * K;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int q = (int)((i / a.inner) % a.m);
    const long long base = i - (long long)q * a.inner;   // point 0 of this line
    const int g = a.bc == 0 ? q + 1 : q;
    const int j = g / n, s = g - j * n;
    auto val = [&](int h) -> double {
      int qq = h;
      if (a.bc == 0) {
        if (h <= 0 || h >= nK) return 0.0;
        qq = h - 1;
      } else if (a.bc == 1 && h == nK) {
        qq = 0;
      }
      return in[base + (long long)qq * a.inner];
    };
    const double vg = in[i];
    double acc = 0.0;
    auto elem = [&](int e, int loc) {
      for (int r = 0; r < nb; ++r) {
        const double v = val(n * (e - 1) + r);
        acc += cc * a.C[loc * nb + r] * v;
        if (r != loc) acc += ca * a.A[loc * nb + r] * (v - vg);
      }
    };
    if (s == 0) {   // node j: the end of element j and the start of element j + 1
      if (j >= 1) elem(j, n);
      else if (a.bc == 1) elem(K, n);   // periodic: node 0 also ends element K
      if (j <= K - 1) elem(j + 1, 0);
    } else {
      elem(j + 1, s);
    }
    out[i] = acc + (add ? add[i] : 0.0);
  }
}

}  // namespace

hipError_t launch_axis_local(const AxisLocal& a, const double* in, double* out, const double* add,
                             double cc, double ca, long long total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(axis_local_kernel, dim3(blocks), dim3(256), 0, s, a, in, out, add, cc, ca, total);
  return hipGetLastError();
}

size_t op3_elem_doubles(const OpArgs& a) {
  if (a.N != 3 || a.n[0] != a.n[1] || a.n[1] != a.n[2]) return 0;
  return 2 * (size_t)a.m[0] * a.m[1] * a.m[2];   // Z1, Z2 of one right-hand side
}

}  // namespace hofem
