// Device kernels of the separable high-order FEM solve (gfx950).
//
// One pass streams a grid once along one axis.  A line of the axis holds
// the m = nK - 1 values of S_K^(n) (Section 2, paragraph 1) in physical order:
// node j at q = n j - 1, interior point s of element j at q = n (j-1) + s - 1.
// A workgroup owns `cb` whole lines and keeps them in LDS.
//
// Direct transform (transform theorem, item 2; input y = C w):
//   z_j = y_{j+1/2} + P y_{j-1/2}            (j = 1..K-1, n-1 components)
//   T0 = DST-I(y_nodes), Zh = DST-I(z)         (n sine transforms, length K-1)
//   w_{kl} = (T0_k + p_k^(l) . Zh_k) / ||s_k^(l)||^2     (k = 1..K-1)
//   w_{0l} = (sum_j (-P)^{j-1} y_{j-1/2}) . e^(l) / K
// Inverse transform (item 1):
//   W_k = sum_l w_{kl},  d_k = sum_l w_{kl} p_k^(l),  E0 = sum_l w_{0l} e^(l)
//   nodes = DST-I(W),  Z = DST-I(d) (Z_0 = Z_K = 0)
//   w_{j-1/2} = Z_{j-1} + P Z_j + (-P)^{j-1} E0
// (the paper's DST-III / DCT-III form of the interior values equals this
// DST-I form).  P reverses the order of the n-1 interior points.
//
// DST-I of length K-1, X_k = sum_j x_j sin(pi k j / K): two real sequences a,
// b are transformed together.  With y_j = sin(pi j/K)(x_j + x_{K-j}) +
// (x_j - x_{K-j})/2 (y_0 = 0) for each, W = FFT_K(y^a + i y^b); the even
// outputs are X_{2k} = -Im Y_k and the odd ones the running sums
// X_{2k+1} = X_{2k-1} + Re Y_k, X_1 = Re Y_0 / 2, where Y^a, Y^b are
// separated from W by conjugate symmetry.  The K-point complex FFT is a
// radix-4 (plus one radix-2) Stockham transform in LDS.
//
// LDS holds, per line, ceil(n/2) complex arrays of length K ("slots"); slot
// pair p carries sequences 2p (real part) and 2p+1 (imaginary part):
// sequence 0 is the node sequence, sequence s >= 1 the interior component s.
// The physical line is loaded into the same memory first; every phase that
// rewrites LDS in a different layout stages its values in registers across
// a barrier.

#include "kernels.h"

namespace hofem {
namespace {

constexpr int kThreads = 512;   // workgroup size of the line passes
constexpr int kMaxV = 16;       // complex values staged per thread
constexpr int kMaxCB = 64;      // lines per workgroup (upper bound)

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
  return {a.x - b.x, a.y - b.y};
}

// Wave-wide inclusive prefix sum of a complex value (64 lanes).
template <typename T>
__device__ __forceinline__ cx<T> wave_incl_scan(cx<T> v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T ux = __shfl_up(v.x, off, 64);
    T uy = __shfl_up(v.y, off, 64);
    if (lane >= off) {
      v.x += ux;
      v.y += uy;
    }
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Value x_j of sequence s (0 = nodes, s >= 1 = interior component s) of the
// forward pre-combine, read from a physical line in LDS; zero outside 1..K-1.
template <typename T>
__device__ __forceinline__ T fwd_seq(const T* ln, int n, int K, int s, int j) {
  if (j <= 0 || j >= K || s >= n) return T(0);
  if (s == 0) return ln[n * j - 1];
  return ln[n * j + s - 1] + ln[n * (j - 1) + (n - s) - 1];
}

// Value of sequence s at wave number j from a coefficient-ordered line in LDS
// after the inverse block (W_k at q = n k - 1, d_k component s at q = n k - 1 + s).
template <typename T>
__device__ __forceinline__ T inv_seq(const T* ln, int n, int K, int s, int j) {
  if (j <= 0 || j >= K || s >= n) return T(0);
  return ln[n * j - 1 + s];
}

// Sine-transform pre-processing of one pair at index j.
template <typename T>
__device__ __forceinline__ cx<T> dst_pre(cx<T> xj, cx<T> xkj, T snj, int j) {
  if (j == 0) return {T(0), T(0)};
  return {snj * (xj.x + xkj.x) + T(0.5) * (xj.x - xkj.x),
          snj * (xj.y + xkj.y) + T(0.5) * (xj.y - xkj.y)};
}

// In-place K-point forward complex FFT of `nf` arrays in LDS (Stockham
// autosort, natural order in and out).
template <typename T>
__device__ void lds_fft(cx<T>* data, int nf, int K, const cx<T>* __restrict__ tw) {
  const int tid = threadIdx.x;
  int Ns = 1;
  int log2K = 31 - __clz(K);
  if (log2K & 1) {
    // radix-2 stage (Ns = 1: no twiddles)
    const int half = K >> 1;
    const int nb = nf * half;
    cx<T> v[kMaxV / 2][2];
#pragma unroll
    for (int i = 0; i < kMaxV / 2; ++i) {
      int b = tid + i * kThreads;
      if (b < nb) {
        int f = b / half, j = b - f * half;
        v[i][0] = data[f * K + j];
        v[i][1] = data[f * K + j + half];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMaxV / 2; ++i) {
      int b = tid + i * kThreads;
      if (b < nb) {
        int f = b / half, j = b - f * half;
        cx<T> a0 = v[i][0], a1 = v[i][1];
        data[f * K + 2 * j] = cadd(a0, a1);
        data[f * K + 2 * j + 1] = csub(a0, a1);
      }
    }
    __syncthreads();
    Ns = 2;
  }
  const int quarter = K >> 2;
  const int nb = nf * quarter;
  while (Ns < K) {
    cx<T> v[kMaxV / 4][4];
#pragma unroll
    for (int i = 0; i < kMaxV / 4; ++i) {
      int b = tid + i * kThreads;
      if (b < nb) {
        int f = b / quarter, j = b - f * quarter;
        const cx<T>* src = data + f * K + j;
        v[i][0] = src[0];
        v[i][1] = src[quarter];
        v[i][2] = src[2 * quarter];
        v[i][3] = src[3 * quarter];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMaxV / 4; ++i) {
      int b = tid + i * kThreads;
      if (b < nb) {
        int f = b / quarter, j = b - f * quarter;
        int k1 = j & (Ns - 1);
        int step = K / (Ns * 4);
        cx<T> a0 = v[i][0], a1 = v[i][1], a2 = v[i][2], a3 = v[i][3];
        if (k1) {
          // forward twiddles exp(-2 pi i r k1 / (4 Ns))
          cx<T> w1 = tw[k1 * step], w2 = tw[2 * k1 * step], w3 = tw[3 * k1 * step];
          w1.y = -w1.y;
          w2.y = -w2.y;
          w3.y = -w3.y;
          a1 = cmul(a1, w1);
          a2 = cmul(a2, w2);
          a3 = cmul(a3, w3);
        }
        cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
        // X0 = t0 + t2, X2 = t0 - t2, X1 = t1 - i t3, X3 = t1 + i t3
        int d = (j - k1) * 4 + k1;
        cx<T>* dst = data + f * K + d;
        dst[0] = cadd(t0, t2);
        dst[Ns] = {t1.x + t3.y, t1.y - t3.x};
        dst[2 * Ns] = csub(t0, t2);
        dst[3 * Ns] = {t1.x - t3.y, t1.y + t3.x};
      }
    }
    __syncthreads();
    Ns *= 4;
  }
}

// After lds_fft: turn each slot array into the two sine transforms of its
// pair, stored as (X^a_k, X^b_k) at index k = 1..K-1 (index 0 set to zero).
template <typename T>
__device__ void dst_post(cx<T>* data, int nf, int K) {
  const int tid = threadIdx.x;
  const int half = K >> 1;
  const int items = nf * half;
  cx<T> ev[kMaxV / 2], rv[kMaxV / 2];
#pragma unroll
  for (int i = 0; i < kMaxV / 2; ++i) {
    int it = tid + i * kThreads;
    if (it < items) {
      int f = it / half, k = it - f * half;
      cx<T> a = data[f * K + k];
      cx<T> b = data[f * K + ((K - k) & (K - 1))];
      // Y^a_k = (W_k + conj W_{K-k}) / 2, Y^b_k = (W_k - conj W_{K-k}) / (2i)
      // even outputs X_{2k} = -Im Y_k; running-sum terms R_k = Re Y_k.
      ev[i] = {T(0.5) * (b.y - a.y), T(0.5) * (a.x - b.x)};
      rv[i] = {T(0.5) * (a.x + b.x), T(0.5) * (a.y + b.y)};
      if (k == 0) {
        ev[i] = {T(0), T(0)};
        rv[i] = {T(0.5) * a.x, T(0.5) * a.y};   // X_1 = Re Y_0 / 2
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kMaxV / 2; ++i) {
    int it = tid + i * kThreads;
    if (it < items) {
      int f = it / half, k = it - f * half;
      data[f * K + 2 * k] = ev[i];
      data[f * K + 2 * k + 1] = rv[i];
    }
  }
  __syncthreads();
  // Inclusive running sums over the odd indices, one wave per array.
  const int wave = tid >> 6, lane = tid & 63, nwaves = kThreads / 64;
  for (int f = wave; f < nf; f += nwaves) {
    cx<T>* odd = data + f * K + 1;   // odd[2k] = R_k
    if (half >= 64) {
      const int chunk = half / 64;
      cx<T> acc = {T(0), T(0)};
      for (int r = 0; r < chunk; ++r) {
        cx<T> v = odd[2 * (lane * chunk + r)];
        acc = cadd(acc, v);
      }
      cx<T> incl = wave_incl_scan(acc);
      cx<T> run = csub(incl, acc);
      for (int r = 0; r < chunk; ++r) {
        int idx = 2 * (lane * chunk + r);
        run = cadd(run, odd[idx]);
        odd[idx] = run;
      }
    } else {
      cx<T> v = {T(0), T(0)};
      if (lane < half) v = odd[2 * lane];
      cx<T> incl = wave_incl_scan(v);
      if (lane < half) odd[2 * lane] = incl;
    }
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T seq_of(const cx<T>* slots, int K, int c_np, int s, int k) {
  const cx<T> v = slots[(c_np + (s >> 1)) * K + k];
  return (s & 1) ? v.y : v.x;
}

template <typename T, int MODE, typename TIN, typename TOUT, int ACC>
__global__ __launch_bounds__(kThreads) void axis_pass(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int n = a.tab.n, K = a.tab.K, m = a.tab.m;
  const int NP = (n + 1) >> 1;
  const int LS = NP * K;                       // complex slots per line
  const long long inner = a.inner;
  const long long L0 = (long long)blockIdx.x * a.cb;
  const int cv = (int)min((long long)a.cb, a.nlines - L0);
  const bool cfast = inner != 1;

  cx<T>* slots = reinterpret_cast<cx<T>*>(smem);
  T* lines = reinterpret_cast<T*>(smem);       // line c at lines + c * 2 * LS
  T* s0 = reinterpret_cast<T*>(slots + (size_t)a.cb * LS);   // [cb][8]
  T* e0 = s0 + a.cb * 8;                                     // [cb][8]
  long long* base = reinterpret_cast<long long*>(e0 + a.cb * 8);   // [cb]
  double* denb = reinterpret_cast<double*>(base + a.cb);           // [cb]

  const T* __restrict__ P = static_cast<const T*>(a.tab.p);
  const T* __restrict__ IN = static_cast<const T*>(a.tab.inorm);
  const T* __restrict__ EV = static_cast<const T*>(a.tab.E);
  const cx<T>* __restrict__ TW = static_cast<const cx<T>*>(a.tab.tw);
  const T* __restrict__ SN = static_cast<const T*>(a.tab.sn);
  const TIN* __restrict__ src = static_cast<const TIN*>(a.in);
  TOUT* __restrict__ dst = static_cast<TOUT*>(a.out);

  if (tid < cv) {
    long long L = L0 + tid;
    long long o = L / inner, t = L - o * inner;
    base[tid] = o * (long long)m * inner + t;
    if (MODE == PASS_FUSED) {
      double d = a.alpha;
      for (int i = 0; i < a.nother; ++i) d += a.oscale[i] * a.olam[i][(t / a.odiv[i]) % a.omod[i]];
      denb[tid] = d;
    }
  }
  __syncthreads();

  // ---- load cv lines (physical or coefficient order) ---------------------
  {
    const int total = cv * m;
    for (int i = tid; i < total; i += kThreads) {
      int c, q;
      if (cfast) { q = i / cv; c = i - q * cv; }
      else { c = i / m; q = i - c * m; }
      lines[(size_t)c * 2 * LS + q] = (T)src[base[c] + (long long)q * inner];
    }
  }
  __syncthreads();

  const int nseq = cv * NP;   // slot arrays in use

  if (MODE == PASS_FWD || MODE == PASS_FUSED) {
    // ---- forward pre-combine and sine pre-processing into registers ------
    cx<T> reg[kMaxV];
    const int total = nseq * K;
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) {
      int i = tid + v * kThreads;
      if (i < total) {
        int f = i / K, j = i - f * K;
        int c = f / NP, p = f - c * NP;
        const T* ln = lines + (size_t)c * 2 * LS;
        cx<T> xj = {fwd_seq(ln, n, K, 2 * p, j), fwd_seq(ln, n, K, 2 * p + 1, j)};
        cx<T> xk = {fwd_seq(ln, n, K, 2 * p, K - j), fwd_seq(ln, n, K, 2 * p + 1, K - j)};
        reg[v] = dst_pre(xj, xk, SN[j], j);
      }
    }
    // S0_s = sum_{j=1..K} ((-P)^{j-1} y_{j-1/2})_s, one wave per (line, s).
    {
      const int wave = tid >> 6, lane = tid & 63, nwaves = kThreads / 64;
      for (int task = wave; task < cv * (n - 1); task += nwaves) {
        int c = task / (n - 1), s = task - c * (n - 1) + 1;
        const T* ln = lines + (size_t)c * 2 * LS;
        T acc = T(0);
        for (int j = 1 + lane; j <= K; j += 64)
          acc += (j & 1) ? ln[n * (j - 1) + s - 1] : -ln[n * (j - 1) + (n - s) - 1];
        acc = wave_sum(acc);
        if (lane == 0) s0[c * 8 + s - 1] = acc;
      }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) {
      int i = tid + v * kThreads;
      if (i < total) slots[i] = reg[v];
    }
    __syncthreads();

    lds_fft(slots, nseq, K, TW);
    dst_post(slots, nseq, K);

    if (MODE == PASS_FWD) {
      // ---- forward block, coefficients to global -------------------------
      const int items = cv * (K - 1);
      for (int i = tid; i < items; i += kThreads) {
        int c, k;
        if (cfast) { k = i / cv + 1; c = i - (k - 1) * cv; }
        else { c = i / (K - 1); k = i - c * (K - 1) + 1; }
        const int cnp = c * NP;
        T x[9];
#pragma unroll
        for (int s = 0; s < 9; ++s) x[s] = s < n ? seq_of(slots, K, cnp, s, k) : T(0);
        const long long ob = base[c];
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          if (l < n) {
            const T* pl = P + ((size_t)(k - 1) * n + l) * (n - 1);
            T acc = x[0];
#pragma unroll
            for (int s = 1; s < 9; ++s)
              if (s < n) acc += pl[s - 1] * x[s];
            acc *= IN[(k - 1) * n + l];
            long long q = (long long)n * k - 1 + l;
            if (ACC) dst[ob + q * inner] += (TOUT)acc;
            else dst[ob + q * inner] = (TOUT)acc;
          }
        }
      }
      // k = 0: w_{0l} = S0 . e^(l) / K
      const int items0 = cv * (n - 1);
      for (int i = tid; i < items0; i += kThreads) {
        int c = i / (n - 1), l = i - c * (n - 1);
        T acc = T(0);
        for (int s = 0; s < n - 1; ++s) acc += EV[s * (n - 1) + l] * s0[c * 8 + s];
        acc /= (T)K;
        if (ACC) dst[base[c] + (long long)l * inner] += (TOUT)acc;
        else dst[base[c] + (long long)l * inner] = (TOUT)acc;
      }
      return;
    }

    // ---- fused: forward block, spectral division, inverse block ----------
    {
      const double sc = a.scale;
      const double* __restrict__ lam = a.tab.lam;
      const int items = cv * (K - 1);
      for (int i = tid; i < items; i += kThreads) {
        int c = i / (K - 1), k = i - c * (K - 1) + 1;
        const int cnp = c * NP;
        T x[9], y[9];
#pragma unroll
        for (int s = 0; s < 9; ++s) {
          x[s] = s < n ? seq_of(slots, K, cnp, s, k) : T(0);
          y[s] = T(0);
        }
        const double db = denb[c];
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          if (l < n) {
            const T* pl = P + ((size_t)(k - 1) * n + l) * (n - 1);
            T pv[9];
            T acc = x[0];
#pragma unroll
            for (int s = 1; s < 9; ++s) {
              pv[s] = s < n ? pl[s - 1] : T(0);
              acc += pv[s] * x[s];
            }
            acc *= IN[(k - 1) * n + l];
            const double den = db + sc * lam[n * k - 1 + l];
            const T w = (T)((double)acc / den);
            y[0] += w;
#pragma unroll
            for (int s = 1; s < 9; ++s) y[s] += w * pv[s];
          }
        }
#pragma unroll
        for (int s = 0; s < 9; ++s) {
          if (s < n) {
            cx<T>& sl = slots[(cnp + (s >> 1)) * K + k];
            if (s & 1) sl.y = y[s]; else sl.x = y[s];
          }
        }
        if (n & 1) slots[(cnp + NP - 1) * K + k].y = T(0);
      }
      if (tid < cv) {
        const int c = tid;
        T w0[8];
#pragma unroll
        for (int l = 0; l < 8; ++l) {
          w0[l] = T(0);
          if (l < n - 1) {
            T acc = T(0);
            for (int s = 0; s < n - 1; ++s) acc += EV[s * (n - 1) + l] * s0[c * 8 + s];
            acc /= (T)K;
            const double den = denb[c] + sc * lam[l];
            w0[l] = (T)((double)acc / den);
          }
        }
        for (int s = 0; s < n - 1; ++s) {
          T acc = T(0);
#pragma unroll
          for (int l = 0; l < 8; ++l)
            if (l < n - 1) acc += EV[s * (n - 1) + l] * w0[l];
          e0[c * 8 + s] = acc;
        }
      }
      __syncthreads();
      // sine pre-processing of (W, d) in the slot layout, in place
      cx<T> reg2[kMaxV];
      const int total2 = nseq * K;
#pragma unroll
      for (int v = 0; v < kMaxV; ++v) {
        int i = tid + v * kThreads;
        if (i < total2) {
          int f = i / K, j = i - f * K;
          cx<T> xj = slots[f * K + j];
          cx<T> xk = slots[f * K + ((K - j) & (K - 1))];
          reg2[v] = dst_pre(xj, xk, SN[j], j);
        }
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < kMaxV; ++v) {
        int i = tid + v * kThreads;
        if (i < total2) slots[i] = reg2[v];
      }
      __syncthreads();
    }
  } else {
    // ---- inverse: block in place on the coefficient line -----------------
    const int items = cv * (K - 1);
    for (int i = tid; i < items; i += kThreads) {
      int c = i / (K - 1), k = i - c * (K - 1) + 1;
      T* ln = lines + (size_t)c * 2 * LS + (n * k - 1);
      T w[9], y[9];
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        w[s] = s < n ? ln[s] : T(0);
        y[s] = T(0);
      }
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        if (l < n) {
          const T* pl = P + ((size_t)(k - 1) * n + l) * (n - 1);
          y[0] += w[l];
#pragma unroll
          for (int s = 1; s < 9; ++s)
            if (s < n) y[s] += w[l] * pl[s - 1];
        }
      }
#pragma unroll
      for (int s = 0; s < 9; ++s)
        if (s < n) ln[s] = y[s];
    }
    if (tid < cv) {
      const int c = tid;
      const T* ln = lines + (size_t)c * 2 * LS;
      for (int s = 0; s < n - 1; ++s) {
        T acc = T(0);
        for (int l = 0; l < n - 1; ++l) acc += EV[s * (n - 1) + l] * ln[l];
        e0[c * 8 + s] = acc;
      }
    }
    __syncthreads();
    cx<T> reg[kMaxV];
    const int total = nseq * K;
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) {
      int i = tid + v * kThreads;
      if (i < total) {
        int f = i / K, j = i - f * K;
        int c = f / NP, p = f - c * NP;
        const T* ln = lines + (size_t)c * 2 * LS;
        cx<T> xj = {inv_seq(ln, n, K, 2 * p, j), inv_seq(ln, n, K, 2 * p + 1, j)};
        cx<T> xk = {inv_seq(ln, n, K, 2 * p, K - j), inv_seq(ln, n, K, 2 * p + 1, K - j)};
        reg[v] = dst_pre(xj, xk, SN[j], j);
      }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < kMaxV; ++v) {
      int i = tid + v * kThreads;
      if (i < total) slots[i] = reg[v];
    }
    __syncthreads();
  }

  // ---- inverse sine transforms and scatter to the physical line ----------
  lds_fft(slots, nseq, K, TW);
  dst_post(slots, nseq, K);
  {
    const int total = cv * m;
    for (int i = tid; i < total; i += kThreads) {
      int c, q;
      if (cfast) { q = i / cv; c = i - q * cv; }
      else { c = i / m; q = i - c * m; }
      const int cnp = c * NP;
      T v;
      const int g = q + 1;
      if (g % n == 0) {
        v = seq_of(slots, K, cnp, 0, g / n);
      } else {
        const int j = g / n + 1, s = g - (j - 1) * n;
        T zl = (j - 1 >= 1) ? seq_of(slots, K, cnp, s, j - 1) : T(0);
        T zr = (j <= K - 1) ? seq_of(slots, K, cnp, n - s, j) : T(0);
        T ee = (j & 1) ? e0[c * 8 + s - 1] : -e0[c * 8 + (n - s) - 1];
        v = zl + zr + ee;
      }
      const long long idx = base[c] + (long long)q * inner;
      if (ACC) dst[idx] += (TOUT)v;
      else dst[idx] = (TOUT)v;
    }
  }
}

template <typename T, int MODE, typename TIN, typename TOUT, int ACC>
hipError_t launch_t(const PassArgs& a, hipStream_t s) {
  const int NP = (a.tab.n + 1) / 2;
  size_t lds = (size_t)a.cb * NP * a.tab.K * sizeof(cx<T>) + (size_t)a.cb * 16 * sizeof(T) +
               (size_t)a.cb * (sizeof(long long) + sizeof(double));
  auto fn = axis_pass<T, MODE, TIN, TOUT, ACC>;
  static bool lds_raised = false;   // benign race: every caller sets the same value
  if (!lds_raised) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_raised = true;
  }
  long long blocks = (a.nlines + a.cb - 1) / a.cb;
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(int dt, const PassArgs& a, hipStream_t s) {
  switch (dt) {
    case 0: return launch_t<double, MODE, double, double, 0>(a, s);
    case 1: return launch_t<float, MODE, float, float, 0>(a, s);
    case 2: return launch_t<float, MODE, double, float, 0>(a, s);
    case 3: return launch_t<float, MODE, float, double, 0>(a, s);
    case 4: return launch_t<float, MODE, float, double, 1>(a, s);
    case 5: return launch_t<float, MODE, double, double, 0>(a, s);
    default: return hipErrorInvalidValue;
  }
}

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

void pass_shape(int n, int K, int is_f64, long long nlines, long long inner, int* cb,
                size_t* lds_bytes) {
  const int NP = (n + 1) / 2;
  const long long per_line = (long long)NP * K;          // complex slots
  const size_t cbytes = is_f64 ? 16 : 8;
  // Staging bound: every thread holds at most kMaxV complex values.
  long long c1 = (long long)kThreads * kMaxV / per_line;
  // LDS bound: about 64 KB per workgroup (two workgroups per CU), at least one line.
  long long c2 = (64 * 1024) / (long long)(per_line * cbytes);
  long long c = std::min(c1, c2);
  c = std::min<long long>(c, kMaxCB);
  c = std::min<long long>(c, nlines);
  if (c < 1) c = 1;
  (void)inner;
  *cb = (int)c;
  *lds_bytes = (size_t)c * per_line * cbytes + (size_t)c * 16 * (is_f64 ? 8 : 4) + (size_t)c * 16;
}

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

hipError_t launch_pass(int kind, int dt, const PassArgs& a, hipStream_t s) {
  switch (kind) {
    case PASS_FWD: return launch_mode<PASS_FWD>(dt, a, s);
    case PASS_INV: return launch_mode<PASS_INV>(dt, a, s);
    case PASS_FUSED: return launch_mode<PASS_FUSED>(dt, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hofem
