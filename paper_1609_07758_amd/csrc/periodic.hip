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
//
// A workgroup owns cb lines in LDS.  After the transforms a lane owns one
// wave number k of one line together with its mirror K - k (k = 0 also
// takes K/2): every Bloch vector w_{k,l} is read once (64 consecutive k per
// wavefront, one contiguous access per entry) and used both for the
// coefficient and, in the fused and inverse passes, for the inverse sum.

#include "linepass.h"

namespace hofem {
namespace {

using lp::cx;

constexpr int kPerMaxThreads = 512;
constexpr int kPerMaxCB = 32;

struct PerShape {
  int cb, threads;
  size_t lds;
};

// Lines per workgroup: as many as 160 KB of LDS holds (a power of two, at
// most kPerMaxCB and the line count); 512 lanes when there are two or more.
// (The inverse pass reads its coefficients straight from global memory in
// the block phase, each once, so every pass needs only the sequences.)
inline PerShape per_shape(int n, int K, int mode, long long nlines) {
  const int NP = (n + 1) / 2;
  (void)mode;
  const size_t per_line = (size_t)NP * K * sizeof(cx<double>);
  long long cb = 1;
  while (cb * 2 <= kPerMaxCB && (size_t)(cb * 2) * per_line <= 160 * 1024 && cb * 2 <= nlines) cb *= 2;
  PerShape s;
  s.cb = (int)cb;
  s.threads = cb >= 2 ? 512 : 256;
  s.lds = (size_t)cb * per_line;
  return s;
}

template <int N, int LOG2K, int MODE>
__global__ __launch_bounds__(kPerMaxThreads) void periodic_pass(PassArgs a) {
  using S = lp::FftShape<LOG2K, 4>;
  constexpr int K = S::K, R = S::R, G = S::G;
  constexpr int H = K / 2;
  constexpr int TPW = 64 / G;
  constexpr int n = N, m = N * K;
  constexpr int NP = (N + 1) / 2;
  const int cb = a.cb, lcb = __builtin_ctz(cb);
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* slots = reinterpret_cast<cx<double>*>(smem);            // [cb][NP][K]
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63, nwaves = nthr >> 6;
  // XCD-aware numbering, as in the Dirichlet passes: each XCD walks one
  // contiguous range of lines
  const unsigned nb = gridDim.x, xcd = blockIdx.x % lp::kXcds, per = nb / lp::kXcds,
                 rem = nb % lp::kXcds;
  const unsigned wg = xcd * per + min(xcd, rem) + blockIdx.x / lp::kXcds;
  const long long L0 = (long long)wg * cb;
  const int cv = (int)min((long long)cb, a.nlines - L0);
  const long long inner = a.inner;
  const bool cfast = inner != 1;   // strided axis: adjacent lanes take adjacent lines
  const double* __restrict__ src = static_cast<const double*>(a.in);
  double* __restrict__ dst = static_cast<double*>(a.out);
  const cx<double>* __restrict__ W = static_cast<const cx<double>*>(a.tab.blk);
  const cx<double>* __restrict__ TW = static_cast<const cx<double>*>(a.tab.tw);
  auto lbase = [&](int c) -> long long {
    const long long L = L0 + c, o = L / inner, t = L - o * inner;
    return o * (long long)m * inner + t;
  };
  auto slot = [&](int c, int p, int i) -> cx<double>& {
    return slots[((size_t)c * NP + p) * K + lp::sw(i)];
  };
  // item i of cv * count: (line, index), lines fastest on a strided axis
  auto split = [&](int i, int count, int& c, int& q) {
    if (cfast) {
      c = i & (cb - 1);
      q = i >> lcb;
    } else {
      c = i / count;
      q = i - c * count;
    }
  };
  const int items_m = cfast ? cb * m : cv * m;
  // kIO global accesses in flight per lane in the load and the scatter
  constexpr int kIO = 16;

  if (MODE == PASS_FWD || MODE == PASS_FUSED) {
    for (int i0 = tid; i0 < items_m; i0 += kIO * nthr) {
      double r[kIO];
#pragma unroll
      for (int u = 0; u < kIO; ++u) {
        int c, q;
        split(i0 + u * nthr, m, c, q);
        const bool ok = i0 + u * nthr < items_m && c < cv;
        r[u] = ok ? src[lbase(c) + (long long)q * inner] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kIO; ++u) {
        int c, q;
        split(i0 + u * nthr, m, c, q);
        if (!(i0 + u * nthr < items_m && c < cv)) continue;
        const int j = q / n, s = q - j * n;
        cx<double>& e = slot(c, s >> 1, j);
        if (s & 1) {
          e.y = r[u];
        } else {
          e.x = r[u];
          if (s == n - 1) e.y = 0.0;   // odd n: the last pair has one component
        }
      }
    }
  }
  __syncthreads();

  auto transforms = [&]() {   // K-point FFT of every pair, rounds of TPW tasks per wave
    const int ntask = cv * NP;
    for (int t0 = 0; t0 < ntask; t0 += nwaves * TPW) {
      const int task = t0 + wave * TPW + lane / G;
      if (task < ntask) {
        const int c = task / NP, p = task - c * NP;
        cx<double>* tb = slots + ((size_t)c * NP + p) * K;
        const int j = lane & (G - 1);
        cx<double> v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) v[t] = tb[lp::sw(j + G * t)];
        lp::wave_sync();
        lp::task_fft<double, LOG2K, 4>(v, tb, j, TW);
      }
    }
  };
  if (MODE == PASS_FWD || MODE == PASS_FUSED) {
    transforms();
    __syncthreads();
  }

  const double invK = 1.0 / K;
  const double sc = a.scale;
  constexpr int ne = N * N;
  // the n x n blocks of wave number k of lines c0 and (when two) c0 + 1:
  // each Bloch vector is read once for both lines
  auto block = [&](int c0, bool two, int k, const double (&dline)[2]) {
    const int kk = (K - k) & (K - 1);
    const int tre = k == 0 ? 0 : (2 * k == K ? K - 1 : 2 * k - 1);   // the real part's t
    const bool cplx = k != 0 && 2 * k != K;
    const cx<double>* __restrict__ wk = W + (size_t)(k >> 6) * ne * 64 + (k & 63);
    cx<double> X[2][2 * NP], U[2][N];
    if (MODE == PASS_FWD || MODE == PASS_FUSED) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int c = two ? c0 + v : c0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const cx<double> u = slot(c, p, k), w = slot(c, p, kk);
          X[v][2 * p] = {0.5 * (u.x + w.x), 0.5 * (u.y - w.y)};
          X[v][2 * p + 1] = {0.5 * (u.y + w.y), -0.5 * (u.x - w.x)};
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int s = 0; s < N; ++s) U[v][s] = {0.0, 0.0};
    const long long ob[2] = {MODE != PASS_FUSED ? lbase(c0) : 0,
                             MODE != PASS_FUSED && two ? lbase(c0 + 1) : 0};
    // one eigenvector per iteration (n complex entries in registers)
#pragma unroll 1
    for (int l = 0; l < N; ++l) {
      cx<double> wl[N];
#pragma unroll
      for (int s = 0; s < N; ++s) wl[s] = wk[(size_t)(l * N + s) * 64];
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        if (v == 1 && !two) break;
        double cr, ci;
        if (MODE == PASS_INV) {
          // (in place is safe: a workgroup reads only its own lines, all of
          // them before the barrier that precedes its stores)
          cr = src[ob[v] + ((long long)l * K + tre) * inner];
          ci = cplx ? src[ob[v] + ((long long)l * K + tre + 1) * inner] : 0.0;
        } else {
          cr = 0.0;
          ci = 0.0;
#pragma unroll
          for (int s = 0; s < N; ++s) {
            cr += wl[s].x * X[v][s].x + wl[s].y * X[v][s].y;   // conj(w) X
            ci += wl[s].x * X[v][s].y - wl[s].y * X[v][s].x;
          }
          cr *= invK;
          ci = cplx ? ci * invK : 0.0;
          if (MODE == PASS_FWD) {
            dst[ob[v] + ((long long)l * K + tre) * inner] = cr;
            if (cplx) dst[ob[v] + ((long long)l * K + tre + 1) * inner] = ci;
            continue;
          }
          const double den = dline[v] + sc * a.tab.lam[(size_t)l * K + tre];
          cr /= den;
          ci /= den;
        }
#pragma unroll
        for (int s = 0; s < N; ++s) {
          U[v][s].x += cr * wl[s].x - ci * wl[s].y;
          U[v][s].y += cr * wl[s].y + ci * wl[s].x;
        }
      }
    }
    if (MODE == PASS_FWD) return;
    // inverse-FFT input as conj(Z), Z = U_s + i U_{s+1}, at entries k and K - k
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      if (v == 1 && !two) break;
      const int c = c0 + v;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const cx<double> U0 = U[v][2 * p];
        const cx<double> U1 = 2 * p + 1 < N ? U[v][2 * p + 1] : cx<double>{0.0, 0.0};
        slot(c, p, k) = {U0.x - U1.y, -(U0.y + U1.x)};
        if (kk != k) slot(c, p, kk) = {U0.x + U1.y, U0.y - U1.x};
      }
    }
  };
  // denominator part of line c from the other axes (fused pass)
  auto line_den = [&](int c) -> double {
    double d = a.alpha;
    const long long t = (L0 + c) % inner;   // position among the other axes
    for (int i = 0; i < a.nother; ++i) d += a.oscale[i] * a.olam[i][(t / a.odiv[i]) % a.omod[i]];
    return d;
  };
  // one lane per (pair of lines, wave number k and its mirror K - k)
  const int npc = cb > 1 ? cb / 2 : 1, lnpc = __builtin_ctz(npc);
  const int items_k = (cfast ? npc : (cv + 1) / 2) * H;
  for (int i = tid; i < items_k; i += nthr) {
    int cp, k;
    if (cfast) {
      cp = i & (npc - 1);
      k = i >> lnpc;
    } else {
      cp = i / H;
      k = i - cp * H;
    }
    const int c0 = 2 * cp;
    if (c0 >= cv) continue;
    const bool two = c0 + 1 < cv;
    const double dline[2] = {MODE == PASS_FUSED ? line_den(c0) : 0.0,
                             MODE == PASS_FUSED && two ? line_den(c0 + 1) : 0.0};
    block(c0, two, k, dline);
    if (k == 0) block(c0, two, H, dline);   // the other self-conjugate wave number
  }
  if (MODE == PASS_FWD) return;
  __syncthreads();
  transforms();   // FFT of conj(Z) = conj of the inverse transform
  __syncthreads();
  for (int i0 = tid; i0 < items_m; i0 += kIO * nthr) {
    double r[kIO];
#pragma unroll
    for (int u = 0; u < kIO; ++u) {
      int c, q;
      split(i0 + u * nthr, m, c, q);
      r[u] = 0.0;
      if (i0 + u * nthr < items_m && c < cv) {
        const int j = q / n, s = q - j * n;
        const cx<double> e = slot(c, s >> 1, j);
        r[u] = (s & 1) ? -e.y : e.x;
      }
    }
#pragma unroll
    for (int u = 0; u < kIO; ++u) {
      int c, q;
      split(i0 + u * nthr, m, c, q);
      if (i0 + u * nthr < items_m && c < cv) dst[lbase(c) + (long long)q * inner] = r[u];
    }
  }
}

template <int N, int LOG2K, int MODE>
hipError_t launch_per_k(const PassArgs& a0, hipStream_t s) {
  constexpr int K = 1 << LOG2K;
  if (a0.tab.n != N || a0.tab.K != K || a0.tab.m != N * K) return hipErrorInvalidValue;
  const PerShape sh = per_shape(a0.tab.n, K, MODE, a0.nlines);
  if (sh.lds > 160 * 1024) return hipErrorInvalidValue;
  PassArgs a = a0;
  a.cb = sh.cb;
  auto fn = periodic_pass<N, LOG2K, MODE>;
  static bool raised = false;   // benign race: every caller sets the same value
  if (!raised) {
    const hipError_t e = hipFuncSetAttribute((const void*)fn,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    raised = true;
  }
  const long long blocks = (a.nlines + a.cb - 1) / a.cb;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(sh.threads), sh.lds, s, a);
  return hipGetLastError();
}

template <int N, int MODE>
hipError_t launch_per_nk(const PassArgs& a, hipStream_t s) {
  switch (a.tab.K) {
    case 2: return launch_per_k<N, 1, MODE>(a, s);
    case 4: return launch_per_k<N, 2, MODE>(a, s);
    case 8: return launch_per_k<N, 3, MODE>(a, s);
    case 16: return launch_per_k<N, 4, MODE>(a, s);
    case 32: return launch_per_k<N, 5, MODE>(a, s);
    case 64: return launch_per_k<N, 6, MODE>(a, s);
    case 128: return launch_per_k<N, 7, MODE>(a, s);
    case 256: return launch_per_k<N, 8, MODE>(a, s);
    case 512: return launch_per_k<N, 9, MODE>(a, s);
    case 1024: return launch_per_k<N, 10, MODE>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int MODE>
hipError_t launch_per_mode(const PassArgs& a, hipStream_t s) {
  switch (a.tab.n) {
    case 1: return launch_per_nk<1, MODE>(a, s);
    case 2: return launch_per_nk<2, MODE>(a, s);
    case 3: return launch_per_nk<3, MODE>(a, s);
    case 4: return launch_per_nk<4, MODE>(a, s);
    case 5: return launch_per_nk<5, MODE>(a, s);
    case 6: return launch_per_nk<6, MODE>(a, s);
    case 7: return launch_per_nk<7, MODE>(a, s);
    case 8: return launch_per_nk<8, MODE>(a, s);
    case 9: return launch_per_nk<9, MODE>(a, s);
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
