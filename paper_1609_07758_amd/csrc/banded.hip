// Algorithm (b) of Section 2, paragraph 4: the direct and inverse
// F_n-transforms along all axes but one, and along that axis, for every
// combination of the other axes' modes, the banded SPD system of
// eq. (sys x1 2),
//   (4 h^-2 A + mu C) v = phi,   mu = alpha + sum_{i != b} 4 h_i^-2 lambda_i,
// of size nK - 1 and half-bandwidth n.  The banded axis here is the
// contiguous one (axis N-1), so a line is one contiguous block.
//
// One line per 256-lane workgroup, held in LDS.  The system is solved by
// static condensation: the n-1 interior points of an element couple only to
// its two end nodes, so with the element matrix E = 4 h^-2 A_loc + mu C_loc,
//   v_b(e) = t_e - W_0 v_{e-1} - W_n v_e,  t_e = E_bb^-1 phi_b(e),
//   W_0 = E_bb^-1 E_b0,  W_n = E_bb^-1 E_bn,
// and the mesh nodes satisfy the tridiagonal system
//   tau v_{j-1} + 2 sigma v_j + tau v_{j+1} = phi_j - E_nb t_j - E_0b t_{j+1}
// with sigma = E_00 - E_0b W_0, tau = E_0n - E_0b W_n (E is symmetric and
// persymmetric).  That system (K - 1 = 2^p - 1 unknowns, equal elements) is
// solved by cyclic reduction in LDS: p - 1 reduction levels, one equation,
// p - 1 substitution levels.  E_bb is factored once per line (Cholesky, one
// lane).  FP64 throughout.
//
// The stiffness has zero row sums, so the row sum of the node equations,
// delta = sigma + tau, is mu [(C 1)_0 - E_0b E_bb^-1 (C 1)_b] (from
// E 1 = mu C 1); it is formed that way rather than as the difference of the
// large sigma and tau, whose rounding (the local stiffness is rounded to
// FP64) would swamp the small eigenvalues of the node system (relative
// errors up to 3e-8 at n = 9, K = 1024 and small mu).  Cyclic reduction
// then carries each level as (a, s) with s = b + 2a the row sum:
// a' = -a^2/b, s' = s (s - 4a)/b, b = s - 2a (a < 0 < s: no cancellation).

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace hofem {
namespace {

constexpr int kBandThreads = 256;
constexpr int kMaxLevels = 12;

template <int NO>
struct BandConst {
  static constexpr int NB = NO > 1 ? NO - 1 : 1;
  double L[NB * NB];     // Cholesky factor of E_bb (lower), diagonal inverted
  double W0[NB], Wn[NB]; // E_bb^-1 E_b0, E_bb^-1 E_bn
  double E0b[NB], Enb[NB];
  double ca[kMaxLevels], cb[kMaxLevels];   // cyclic-reduction coefficients per level
};

// Per-line constants (one lane).
template <int NO>
__device__ void band_constants(const BandArgs& a, double mu, BandConst<NO>& c) {
  constexpr int B = NO + 1;
  constexpr int NB = NO - 1;
  double E[B * B];
  for (int r = 0; r < B * B; ++r) E[r] = a.scale * a.A[r] + mu * a.C[r];
  double delta, tau;   // row sum sigma + tau of the node equations, off-diagonal
  if constexpr (NO == 1) {
    delta = mu * (a.C[0] + a.C[1]);
    tau = E[1];
  } else {
    // Cholesky of E_bb (rows and columns 1..n-1)
    double* Lf = c.L;
    for (int i = 0; i < NB; ++i) {
      for (int j = 0; j <= i; ++j) {
        double s = E[(i + 1) * B + (j + 1)];
        for (int k = 0; k < j; ++k) s -= Lf[i * NB + k] * Lf[j * NB + k];
        if (i == j) {
          Lf[i * NB + i] = sqrt(s);
        } else {
          Lf[i * NB + j] = s / Lf[j * NB + j];
        }
      }
    }
    for (int i = 0; i < NB; ++i) Lf[i * NB + i] = 1.0 / Lf[i * NB + i];
    // W0 = E_bb^-1 E_b0, Wn = E_bb^-1 E_bn, Wc = E_bb^-1 (C 1)_b by two
    // triangular solves each
    double Wc[NB];
    for (int col = 0; col < 3; ++col) {
      double* w = col == 0 ? c.W0 : col == 1 ? c.Wn : Wc;
      double z[NB];
      for (int i = 0; i < NB; ++i) {
        double s;
        if (col == 2) {
          s = 0.0;
          for (int r = 0; r < B; ++r) s += a.C[(i + 1) * B + r];
        } else {
          s = E[(i + 1) * B + (col == 0 ? 0 : NO)];
        }
        for (int k = 0; k < i; ++k) s -= Lf[i * NB + k] * z[k];
        z[i] = s * Lf[i * NB + i];
      }
      for (int i = NB - 1; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < NB; ++k) s -= Lf[k * NB + i] * w[k];
        w[i] = s * Lf[i * NB + i];
      }
    }
    double c10 = 0.0;
    for (int r = 0; r < B; ++r) c10 += a.C[r];
    tau = E[NO];
    double rs = c10;
    for (int i = 0; i < NB; ++i) {
      c.E0b[i] = E[i + 1];
      c.Enb[i] = E[NO * B + i + 1];
      tau -= c.E0b[i] * c.Wn[i];
      rs -= c.E0b[i] * Wc[i];
    }
    delta = mu * rs;
  }
  double ca = tau, cs = 2.0 * delta;
  for (int l = 0; l < kMaxLevels; ++l) {
    const double cb = cs - 2.0 * ca;
    c.ca[l] = ca;
    c.cb[l] = cb;
    cs = cs * (cs - 4.0 * ca) / cb;
    ca = -ca * ca / cb;
  }
}

template <int NO>
__global__ __launch_bounds__(kBandThreads) void banded_kernel(BandArgs a) {
  extern __shared__ __align__(16) double sm[];
  constexpr int NB = NO - 1;
  const int m = a.m, K = a.K, tid = threadIdx.x, nthr = blockDim.x;
  const long long L = blockIdx.x;
  double* y = sm;
  BandConst<NO>* cst = reinterpret_cast<BandConst<NO>*>(sm + ((m + 1) & ~1));
  const double* src = a.in + L * m;
  double* dst = a.out + L * m;
  for (int q = tid; q < m; q += nthr) y[q] = src[q];
  if (tid == 0) {
    // mu of this line: alpha + the other axes' scaled eigenvalues
    const long long t = L % a.others;
    double mu = a.alpha;
    for (int i = 0; i < a.nother; ++i) mu += a.oscale[i] * a.olam[i][(t / a.odiv[i]) % a.omod[i]];
    band_constants<NO>(a, mu, *cst);
  }
  __syncthreads();
  const BandConst<NO>& c = *cst;
  // node j (1..K-1) sits at q = n j - 1, interior point s of element e at
  // q = n (e-1) + s - 1
  if constexpr (NO > 1) {
    // t_e = E_bb^-1 phi_b(e) in place of phi_b(e); the condensed node
    // right-hand sides phi_j - E_nb t_j - E_0b t_{j+1}, applied by even then
    // odd elements (each node has one of each)
    constexpr int EPT = 8;   // elements per lane per round
    // every lane runs the same number of rounds (barriers inside)
    for (int base = 0; base < K; base += nthr * EPT) {
      const int e0 = 1 + base + tid * EPT;
      double c0[EPT], cn[EPT];
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int e = e0 + u;
        c0[u] = cn[u] = 0.0;
        if (e > K) continue;
        double* yb = y + NO * (e - 1);
        double z[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          double s = yb[i];
#pragma unroll
          for (int k = 0; k < i; ++k) s -= c.L[i * NB + k] * z[k];
          z[i] = s * c.L[i * NB + i];
        }
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
          double s = z[i];
#pragma unroll
          for (int k = i + 1; k < NB; ++k) s -= c.L[k * NB + i] * z[k];
          z[i] = s * c.L[i * NB + i];
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          yb[i] = z[i];
          c0[u] += c.E0b[i] * z[i];
          cn[u] += c.Enb[i] * z[i];
        }
      }
      __syncthreads();
      for (int par = 0; par < 2; ++par) {
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
          const int e = e0 + u;
          if (e > K || (e & 1) != par) continue;
          if (e <= K - 1) y[NO * e - 1] -= cn[u];         // node e: element e is on its left
          if (e >= 2) y[NO * (e - 1) - 1] -= c0[u];       // node e-1: element e on its right
        }
        __syncthreads();
      }
    }
  }
  // cyclic reduction on the node system, K - 1 = 2^p - 1 unknowns
  int p = 0;
  while ((1 << p) < K) ++p;
  auto node = [&](int j) -> double& { return y[NO * j - 1]; };
  for (int l = 0; l + 1 < p; ++l) {
    const int h = 1 << l;
    const double r = c.ca[l] / c.cb[l];
    for (int j = 2 * h * (tid + 1); j < K; j += 2 * h * nthr)
      node(j) -= r * (node(j - h) + node(j + h));
    __syncthreads();
  }
  if (tid == 0 && K > 1) node(K / 2) /= c.cb[p - 1];
  __syncthreads();
  for (int l = p - 2; l >= 0; --l) {
    const int h = 1 << l;
    for (int j = h * (2 * tid + 1); j < K; j += 2 * h * nthr) {
      const double vl = j - h > 0 ? node(j - h) : 0.0;
      const double vr = j + h < K ? node(j + h) : 0.0;
      node(j) = (node(j) - c.ca[l] * (vl + vr)) / c.cb[l];
    }
    __syncthreads();
  }
  // interior points: v_b(e) = t_e - W_0 v_{e-1} - W_n v_e
  if constexpr (NO > 1) {
    for (int e = 1 + tid; e <= K; e += nthr) {
      const double vl = e >= 2 ? y[NO * (e - 1) - 1] : 0.0;
      const double vr = e <= K - 1 ? y[NO * e - 1] : 0.0;
      double* yb = y + NO * (e - 1);
#pragma unroll
      for (int i = 0; i < NB; ++i) yb[i] -= c.W0[i] * vl + c.Wn[i] * vr;
    }
    __syncthreads();
  }
  for (int q = tid; q < m; q += nthr) dst[q] = y[q];
}

template <int NO>
hipError_t launch_band_order(const BandArgs& a, hipStream_t s) {
  const size_t lds = ((size_t)((a.m + 1) & ~1)) * sizeof(double) + sizeof(BandConst<NO>);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static bool raised = false;   // benign race: every caller sets the same value
  if (!raised) {
    const hipError_t e = hipFuncSetAttribute((const void*)banded_kernel<NO>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    raised = true;
  }
  hipLaunchKernelGGL(banded_kernel<NO>, dim3((unsigned)a.nlines), dim3(kBandThreads), lds, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_banded(const BandArgs& a, hipStream_t s) {
  if (a.nlines == 0) return hipSuccess;
  if (a.K < 2 || (a.K & (a.K - 1)) || a.nlines > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (a.n) {
    case 1: return launch_band_order<1>(a, s);
    case 2: return launch_band_order<2>(a, s);
    case 3: return launch_band_order<3>(a, s);
    case 4: return launch_band_order<4>(a, s);
    case 5: return launch_band_order<5>(a, s);
    case 6: return launch_band_order<6>(a, s);
    case 7: return launch_band_order<7>(a, s);
    case 8: return launch_band_order<8>(a, s);
    case 9: return launch_band_order<9>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hofem
