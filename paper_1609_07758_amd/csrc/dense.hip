// Dense eigenvector transforms of axes whose K is not a power of two: the
// solve v = (x)V diag(1 / (alpha + sum_i 4 h_i^-2 lambda_i)) (x)V^T f^h of
// eq. (decomp v 2) with V applied along the axis as a matrix product (there
// is no power-of-two FFT for it), on the FP64 matrix cores.
//
// dgemm: C_b = op(A_b) op(B_b), FP64, row-major operands with leading
// dimensions and batch strides, op = transpose when TA / TB.  A workgroup of
// eight wavefronts owns a 128 x 128 tile of C (each operand element is read
// once per 128 columns or rows of C, which keeps the products off the
// memory bound); each wavefront a 32 x 64 block as 2 x 4 blocks of
// v_mfma_f64_16x16x4 (A operand: lane l holds A[l % 16][l / 16] of the
// 16 x 4 slice, B operand: B[l / 16][l % 16] of the 4 x 16 slice, result:
// lane l holds D[l / 16 + 4 r][l % 16], r = 0..3).  K advances in slices of
// 16 staged through LDS, zero-filled outside the matrices, so any M, N, K
// work; each lane fetches the next slice into registers while the matrix
// cores work on the current one.  The register budget of four wavefronts
// per SIMD lets two workgroups share a CU.
#include "kernels.h"

namespace hofem {
namespace {

constexpr int kBM = 128, kBN = 128, kBK = 16;
constexpr int kThreads = 512;                     // 8 wavefronts: 4 along M x 2 along N
constexpr int kWM = 32, kWN = 64;                 // a wavefront's block of C
constexpr int kBI = kWM / 16, kBJ = kWN / 16;     // its 16 x 16 MFMA blocks
constexpr int kPadM = kBM + 2, kPadN = kBN + 2;   // LDS row pitch (doubles)
constexpr int kLoad = kBM * kBK / kThreads;       // values of each operand a lane stages per slice

typedef double double4_t __attribute__((ext_vector_type(4)));

template <bool TA, bool TB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void dgemm_kernel(GemmArgs g) {
  __shared__ double As[kBK][kPadM];   // As[k][i] = op(A)[i][k]
  __shared__ double Bs[kBK][kPadN];   // Bs[k][j] = op(B)[k][j]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  // this lane's staging positions: kLoad consecutive values of each operand
  // per slice (i or k contiguous for A, k or j for B)
  const int a_i0 = TA ? kLoad * (tid & 31) : tid >> 2, a_k0 = TA ? tid >> 5 : kLoad * (tid & 3);
  const int b_k0 = TB ? kLoad * (tid & 3) : tid >> 5, b_j0 = TB ? tid >> 2 : kLoad * (tid & 31);
  for (long long b = blockIdx.z; b < g.batch; b += gridDim.z) {
    const double* __restrict__ A = g.A + b * g.sa;
    const double* __restrict__ B = g.B + b * g.sb;
    double* __restrict__ C = g.C + b * g.sc;
    double4_t acc[kBI][kBJ];
#pragma unroll
    for (int bi = 0; bi < kBI; ++bi)
#pragma unroll
      for (int bj = 0; bj < kBJ; ++bj) acc[bi][bj] = double4_t{0.0, 0.0, 0.0, 0.0};
    // slice k0 of op(A) and op(B) into registers (zero outside the matrices)
    double ra[kLoad], rb[kLoad];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int u = 0; u < kLoad; ++u) {
        const int gi = m0 + a_i0 + (TA ? u : 0), gk = k0 + a_k0 + (TA ? 0 : u);
        ra[u] = (gi < g.M && gk < g.K) ? (TA ? A[(long long)gk * g.lda + gi] : A[(long long)gi * g.lda + gk])
                                       : 0.0;
        const int gk2 = k0 + b_k0 + (TB ? u : 0), gj = n0 + b_j0 + (TB ? 0 : u);
        rb[u] = (gk2 < g.K && gj < g.N) ? (TB ? B[(long long)gj * g.ldb + gk2] : B[(long long)gk2 * g.ldb + gj])
                                        : 0.0;
      }
    };
    fetch(0);
    for (int k0 = 0; k0 < g.K; k0 += kBK) {
#pragma unroll
      for (int u = 0; u < kLoad; ++u) {
        As[a_k0 + (TA ? 0 : u)][a_i0 + (TA ? u : 0)] = ra[u];
        Bs[b_k0 + (TB ? u : 0)][b_j0 + (TB ? 0 : u)] = rb[u];
      }
      __syncthreads();
      if (k0 + kBK < g.K) fetch(k0 + kBK);   // the next slice's loads overlap this slice's products
#pragma unroll
      for (int kk = 0; kk < kBK; kk += 4) {
        const int kr = kk + (lane >> 4), c = lane & 15;
        double av[kBI], bv[kBJ];
#pragma unroll
        for (int bi = 0; bi < kBI; ++bi) av[bi] = As[kr][kWM * wy + 16 * bi + c];
#pragma unroll
        for (int bj = 0; bj < kBJ; ++bj) bv[bj] = Bs[kr][kWN * wx + 16 * bj + c];
#pragma unroll
        for (int bi = 0; bi < kBI; ++bi)
#pragma unroll
          for (int bj = 0; bj < kBJ; ++bj)
            acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bv[bj], acc[bi][bj], 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < kBI; ++bi)
#pragma unroll
      for (int bj = 0; bj < kBJ; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = m0 + kWM * wy + 16 * bi + (lane >> 4) + 4 * r;
          const int gj = n0 + kWN * wx + 16 * bj + (lane & 15);
          if (gi < g.M && gj < g.N) C[(long long)gi * g.ldc + gj] = acc[bi][bj][r];
        }
  }
}

// x[o][q][t] /= alpha + scale lam[q] + sum_i oscale[i] olam[i][(t / odiv[i]) % omod[i]]
// over a grid [outer][m][inner] (outer = right-hand sides: the fused pass runs
// along axis 0).
__global__ __launch_bounds__(256) void dense_divide_kernel(double* __restrict__ x, long long total,
                                                           int m, long long inner, PassArgs a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long t = i % inner;
  const int q = (int)((i / inner) % m);
  double d = a.alpha + a.scale * a.tab.lam[q];
  for (int k = 0; k < a.nother; ++k) d += a.oscale[k] * a.olam[k][(t / a.odiv[k]) % a.omod[k]];
  x[i] /= d;
}

}  // namespace

hipError_t launch_dgemm(const GemmArgs& g, bool ta, bool tb, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((g.N + kBN - 1) / kBN), (unsigned)((g.M + kBM - 1) / kBM),
                  (unsigned)(g.batch < 65535 ? g.batch : 65535));
  auto fn = ta ? (tb ? dgemm_kernel<true, true> : dgemm_kernel<true, false>)
              : (tb ? dgemm_kernel<false, true> : dgemm_kernel<false, false>);
  hipLaunchKernelGGL(fn, grid, dim3(kThreads), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_dense_divide(double* x, long long outer, int m, long long inner, const PassArgs& a,
                               hipStream_t s) {
  const long long total = outer * m * inner;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(dense_divide_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, x, total,
                     m, inner, a);
  return hipGetLastError();
}

}  // namespace hofem
