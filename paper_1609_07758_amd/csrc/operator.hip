// FP64 operator of eq. (bvp glob 2) and the small kernels of the refinement
// loop (update with norms, reduction).

#include "kernels.h"

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

}  // namespace

hipError_t launch_operator(const OpArgs& a, hipStream_t s) {
  long long total = a.nrhs;
  for (int i = 0; i < a.N; ++i) total *= a.m[i];
  if (total == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  switch (a.N) {
    case 1: hipLaunchKernelGGL(op_kernel<1>, dim3(blocks), dim3(256), 0, s, a, total); break;
    case 2: hipLaunchKernelGGL(op_kernel<2>, dim3(blocks), dim3(256), 0, s, a, total); break;
    case 3: hipLaunchKernelGGL(op_kernel<3>, dim3(blocks), dim3(256), 0, s, a, total); break;
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

}  // namespace hofem
