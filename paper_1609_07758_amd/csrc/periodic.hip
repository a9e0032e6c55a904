// Line passes along periodic axes (FP64).  A line holds the m = nK values of
// one axis: cell j = 0..K-1 holds node j (q = n j) and the interior points
// s = 1..n-1 of element j+1 (q = n j + s).  The pencil is block circulant, so
// its eigenvectors are Bloch waves v_j = w_{k,l} e^{i phi_k j},
// phi_k = 2 pi k / K (w from the n x n Hermitian pencil of wave number k,
// normalised w^H C^(k) w = 1, so that v^H C v = K):
//   direct:  X_s(k) = sum_j y[n j + s] e^{-i phi_k j}   (a real FFT per s)
//            c_{k,l} = (1/K) sum_s conj(w_{k,l,s}) X_s(k),  k = 0..K/2
//   inverse: U_s(k) = sum_l c_{k,l} w_{k,l,s},
//            y[n j + s] = sum_{k=0}^{K-1} U_s(k) e^{i phi_k j}
//            (U_s(K-k) = conj U_s(k): real output)
// Coefficients are stored real, l-major: q = l K + t with t = 0 for k = 0,
// t = 2k-1 and 2k for the real and imaginary parts of k = 1..K/2-1, t = K-1
// for k = K/2.  Components are FFT-ed in pairs (s, s+1) as one complex
// sequence y_s + i y_{s+1}, separated by conjugate symmetry; the K-point
// FFT is the wavefront-level Stockham transform of the Dirichlet passes.
// One line per 256-lane workgroup, in LDS.

#include "linepass.h"

namespace hofem {
namespace {

using lp::cx;

constexpr int kPerThreads = 256;

template <int LOG2K, int MODE>
__global__ __launch_bounds__(kPerThreads) void periodic_pass(PassArgs a) {
  using S = lp::FftShape<LOG2K, 4>;
  constexpr int K = S::K, R = S::R, G = S::G;
  constexpr int TPW = 64 / G;
  const int n = a.tab.n, m = a.tab.m;
  const int NP = (n + 1) / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* slots = reinterpret_cast<cx<double>*>(smem);     // [NP][K]
  double* flat = reinterpret_cast<double*>(slots + (size_t)NP * K);   // [m] (inverse pass)
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63, nwaves = nthr >> 6;
  const long long L = blockIdx.x;
  const long long inner = a.inner;
  const long long o = L / inner, tcol = L - o * inner;
  const long long base = o * (long long)m * inner + tcol;
  const double* __restrict__ src = static_cast<const double*>(a.in);
  double* __restrict__ dst = static_cast<double*>(a.out);
  const cx<double>* __restrict__ W = static_cast<const cx<double>*>(a.tab.blk);
  const cx<double>* __restrict__ TW = static_cast<const cx<double>*>(a.tab.tw);
  auto slot = [&](int p, int i) -> cx<double>& { return slots[(size_t)p * K + lp::sw(i)]; };

  if (MODE == PASS_FWD || MODE == PASS_FUSED) {
    for (int q = tid; q < m; q += nthr) {
      const int j = q / n, s = q - j * n;
      const double v = src[base + (long long)q * inner];
      cx<double>& e = slot(s >> 1, j);
      if (s & 1) {
        e.y = v;
      } else {
        e.x = v;
        if (s == n - 1) e.y = 0.0;   // odd n: the last pair has one component
      }
    }
  } else {
    for (int q = tid; q < m; q += nthr) flat[q] = src[base + (long long)q * inner];
  }
  __syncthreads();

  auto transforms = [&]() {   // K-point FFT of every pair, rounds of TPW per wave
    for (int t0 = 0; t0 < NP; t0 += nwaves * TPW) {
      const int task = t0 + wave * TPW + lane / G;
      if (task < NP) {
        int j = lane & (G - 1);
        cx<double> v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) v[t] = slot(task, j + G * t);
        lp::wave_sync();
        lp::task_fft<double, LOG2K, 4>(v, slots + (size_t)task * K, j, TW);
      }
    }
  };
  if (MODE == PASS_FWD || MODE == PASS_FUSED) {
    transforms();
    __syncthreads();
  }

  // per wave number k = 0..K/2: the n x n complex blocks (each k owns
  // entries k and K-k of every pair: no other thread touches them)
  const double invK = 1.0 / K;
  const double sc = a.scale;
  double dline = a.alpha;
  if (MODE == PASS_FUSED) {
    const long long t = tcol;   // position among the other axes
    for (int i = 0; i < a.nother; ++i) dline += a.oscale[i] * a.olam[i][(t / a.odiv[i]) % a.omod[i]];
  }
  for (int k = tid; k <= K / 2; k += nthr) {
    const int kk = (K - k) & (K - 1);
    const int tre = k == 0 ? 0 : (2 * k == K ? K - 1 : 2 * k - 1);   // real part's t
    const bool cplx = k != 0 && 2 * k != K;
    cx<double> c[9];
    if (MODE == PASS_FWD || MODE == PASS_FUSED) {
      cx<double> X[10];
      for (int p = 0; p < NP; ++p) {
        const cx<double> u = slot(p, k), w = slot(p, kk);
        X[2 * p] = {0.5 * (u.x + w.x), 0.5 * (u.y - w.y)};
        X[2 * p + 1] = {0.5 * (u.y + w.y), -0.5 * (u.x - w.x)};
      }
      for (int l = 0; l < n; ++l) {
        double cr = 0.0, ci = 0.0;
        const cx<double>* wl = W + ((size_t)k * n + l) * n;
        for (int s = 0; s < n; ++s) {
          const cx<double> ws = wl[s];
          cr += ws.x * X[s].x + ws.y * X[s].y;   // conj(w) X
          ci += ws.x * X[s].y - ws.y * X[s].x;
        }
        c[l] = {cr * invK, cplx ? ci * invK : 0.0};
      }
      if (MODE == PASS_FWD) {
        for (int l = 0; l < n; ++l) {
          dst[base + ((long long)l * K + tre) * inner] = c[l].x;
          if (cplx) dst[base + ((long long)l * K + tre + 1) * inner] = c[l].y;
        }
        continue;
      }
      for (int l = 0; l < n; ++l) {
        const double den = dline + sc * a.tab.lam[(size_t)l * K + tre];
        c[l] = {c[l].x / den, c[l].y / den};
      }
    } else {
      for (int l = 0; l < n; ++l)
        c[l] = {flat[(size_t)l * K + tre], cplx ? flat[(size_t)l * K + tre + 1] : 0.0};
    }
    // U_s = sum_l c_l w_{k,l,s}; inverse-FFT input as conj(Z), Z = U_s + i U_{s+1}
    for (int p = 0; p < NP; ++p) {
      cx<double> U0 = {0.0, 0.0}, U1 = {0.0, 0.0};
      for (int l = 0; l < n; ++l) {
        const cx<double>* wl = W + ((size_t)k * n + l) * n;
        const cx<double> w0 = wl[2 * p];
        U0.x += c[l].x * w0.x - c[l].y * w0.y;
        U0.y += c[l].x * w0.y + c[l].y * w0.x;
        if (2 * p + 1 < n) {
          const cx<double> w1 = wl[2 * p + 1];
          U1.x += c[l].x * w1.x - c[l].y * w1.y;
          U1.y += c[l].x * w1.y + c[l].y * w1.x;
        }
      }
      slot(p, k) = {U0.x - U1.y, -(U0.y + U1.x)};
      if (kk != k) slot(p, kk) = {U0.x + U1.y, U0.y - U1.x};
    }
  }
  if (MODE == PASS_FWD) return;
  __syncthreads();
  transforms();   // FFT of conj(Z) = conj of the inverse transform
  __syncthreads();
  for (int q = tid; q < m; q += nthr) {
    const int j = q / n, s = q - j * n;
    const cx<double> e = slot(s >> 1, j);
    dst[base + (long long)q * inner] = (s & 1) ? -e.y : e.x;
  }
}

template <int LOG2K, int MODE>
hipError_t launch_per_k(const PassArgs& a, hipStream_t s) {
  constexpr int K = 1 << LOG2K;
  const int NP = (a.tab.n + 1) / 2;
  size_t lds = (size_t)NP * K * sizeof(cx<double>);
  if (MODE == PASS_INV) lds += (size_t)a.tab.m * sizeof(double);
  if (lds > 160 * 1024 || a.tab.n < 1 || a.tab.n > 9 || a.tab.K != K) return hipErrorInvalidValue;
  auto fn = periodic_pass<LOG2K, MODE>;
  static bool raised = false;   // benign race: every caller sets the same value
  if (!raised) {
    const hipError_t e = hipFuncSetAttribute((const void*)fn,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    raised = true;
  }
  if (a.nlines > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3((unsigned)a.nlines), dim3(kPerThreads), lds, s, a);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_per_mode(const PassArgs& a, hipStream_t s) {
  switch (a.tab.K) {
    case 2: return launch_per_k<1, MODE>(a, s);
    case 4: return launch_per_k<2, MODE>(a, s);
    case 8: return launch_per_k<3, MODE>(a, s);
    case 16: return launch_per_k<4, MODE>(a, s);
    case 32: return launch_per_k<5, MODE>(a, s);
    case 64: return launch_per_k<6, MODE>(a, s);
    case 128: return launch_per_k<7, MODE>(a, s);
    case 256: return launch_per_k<8, MODE>(a, s);
    case 512: return launch_per_k<9, MODE>(a, s);
    case 1024: return launch_per_k<10, MODE>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_periodic(int kind, const PassArgs& a, hipStream_t s) {
  if (a.nlines == 0) return hipSuccess;
  switch (kind) {
    case PASS_FWD: return launch_per_mode<PASS_FWD>(a, s);
    case PASS_INV: return launch_per_mode<PASS_INV>(a, s);
    case PASS_FUSED: return launch_per_mode<PASS_FUSED>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hofem
