// Line passes of the separable high-order FEM solve (gfx950), templated on
// the element order N and on K = 2^LOG2K.  Included by linepass.hip, which is
// compiled once per order.
//
// One pass streams a grid once along one axis.  A line of the axis holds
// the m = NK - 1 values of S_K^(N) (Section 2, paragraph 1) in physical order:
// node j at q = N j - 1, interior point s of element j at q = N (j-1) + s - 1.
// A workgroup owns `cb` whole lines and keeps them in LDS.
//
// Direct transform (transform theorem, item 2; input y = C w):
//   z_j = y_{j+1/2} + P y_{j-1/2}            (j = 1..K-1, N-1 components)
//   T0 = DST-I(y_nodes), Zh = DST-I(z)         (N sine transforms, length K-1)
//   w_{kl} = (T0_k + p_k^(l) . Zh_k) / ||s_k^(l)||^2     (k = 1..K-1)
//   w_{0l} = (sum_j (-P)^{j-1} y_{j-1/2}) . e^(l) / K
// Inverse transform (item 1):
//   W_k = sum_l w_{kl},  d_k = sum_l w_{kl} p_k^(l),  E0 = sum_l w_{0l} e^(l)
//   nodes = DST-I(W),  Z = DST-I(d) (Z_0 = Z_K = 0)
//   w_{j-1/2} = Z_{j-1} + P Z_j + (-P)^{j-1} E0
// (the paper's DST-III / DCT-III form of the interior values equals this
// DST-I form).  P reverses the order of the N-1 interior points.
//
// DST-I of length K-1, X_k = sum_j x_j sin(pi k j / K): two real sequences a,
// b are transformed together.  With y_j = sin(pi j/K)(x_j + x_{K-j}) +
// (x_j - x_{K-j})/2 (y_0 = 0) for each, W = FFT_K(y^a + i y^b); the even
// outputs are X_{2k} = -Im Y_k and the odd ones the running sums
// X_{2k+1} = X_{2k-1} + Re Y_k, X_1 = Re Y_0 / 2, where Y^a, Y^b are
// separated from W by conjugate symmetry.
//
// FFT organisation.  One K-point transform ("task": one slot pair of one
// line) is owned by G = K / R lanes of one wavefront, each lane holding
// R = min(16, K) points in registers; a wave runs 64 / G tasks side by side.
// Stages are radix 16, 8, 4 or 2 Stockham steps on the registers; between
// stages the task's points go through its own K-entry LDS region with
// wavefront-level ordering only.  The running sums of the odd outputs are a
// lane-local scan plus a segmented wave scan.
//
// LDS holds, per line, ceil(N/2) complex arrays of length K ("slots") and
// one pad entry; slot pair p carries sequences 2p (real part) and 2p+1
// (imaginary part): sequence 0 is the node sequence, sequence s >= 1 the
// interior component s.  The physical line is loaded into the same memory
// first; the gather that reads it holds its values in registers across a
// workgroup barrier.
//
// Coefficients leave and enter a pass in the l-major coefficient order of
// AxisTab, so that lanes handling consecutive wave numbers touch consecutive
// addresses.
#pragma once

#include <algorithm>

#include "kernels.h"

namespace hofem {
namespace lp {

constexpr int kMaxCB = 64;         // lines per workgroup (upper bound)
// Workgroup size: 16 waves (up to 128 VGPRs per lane) in FP32, 8 waves (up
// to 256) in FP64, whose FFT registers do not fit in 128.  Every workgroup
// has the maximum size: the load, block and scatter phases use all lanes.
template <typename T>
constexpr int threads_for() { return 512; }
// global loads in flight per lane: one round for the workgroup's values
// (at most 64 KB of lines per workgroup unless a single line needs more)
template <typename T, int LOG2K>
constexpr int unroll_for() { return (sizeof(T) == 8 && LOG2K >= 10) ? 32 : 16; }
constexpr unsigned kXcds = 8;      // accelerator complex dies of an MI355X

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
// a * conj(w)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> w) {
  return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cmulk(cx<T> a, T c, T s) {   // a * (c + i s)
  return {a.x * c - a.y * s, a.x * s + a.y * c};
}

// Position of entry i of a task's K-entry LDS array: the low four bits are
// XOR-ed with the next four, so that strides of 16 entries (Stockham writes,
// the pair separation) spread over all LDS banks.
__device__ __forceinline__ int sw(int i) { return i ^ ((i >> 4) & 15); }

// Orders LDS traffic of the lanes of one wavefront (the lanes of a task).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- small forward DFTs in registers, X_k = sum_n x_n e^{-2 pi i n k / N} ----

template <typename T>
__device__ __forceinline__ void dft4(cx<T>& x0, cx<T>& x1, cx<T>& x2, cx<T>& x3) {
  const cx<T> t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), t3 = csub(x1, x3);
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = {t1.x + t3.y, t1.y - t3.x};   // t1 - i t3
  x3 = {t1.x - t3.y, t1.y + t3.x};   // t1 + i t3
}

template <typename T, int NR>
__device__ __forceinline__ void dft(cx<T> (&x)[NR]) {
  if constexpr (NR == 2) {
    const cx<T> a = x[0];
    x[0] = cadd(a, x[1]);
    x[1] = csub(a, x[1]);
  } else if constexpr (NR == 4) {
    dft4(x[0], x[1], x[2], x[3]);
  } else if constexpr (NR == 8) {
    // n = q + 2m, k = p + 4r: X[p + 4r] = sum_q W2^{qr} W8^{qp} DFT4_m(x[q + 2m])[p]
    const T h = T(0.70710678118654752440);
    cx<T> y0[4] = {x[0], x[2], x[4], x[6]};
    cx<T> y1[4] = {x[1], x[3], x[5], x[7]};
    dft4(y0[0], y0[1], y0[2], y0[3]);
    dft4(y1[0], y1[1], y1[2], y1[3]);
    y1[1] = cmulk(y1[1], h, -h);
    y1[2] = {y1[2].y, -y1[2].x};
    y1[3] = cmulk(y1[3], -h, -h);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      x[p] = cadd(y0[p], y1[p]);
      x[p + 4] = csub(y0[p], y1[p]);
    }
  } else if constexpr (NR == 16) {
    // n = q + 4m, k = p + 4r: X[p + 4r] = DFT4_q(W16^{qp} DFT4_m(x[q + 4m])[p])[r]
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173),
            h = T(0.70710678118654752440);
    cx<T> y[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      y[q][0] = x[q];
      y[q][1] = x[q + 4];
      y[q][2] = x[q + 8];
      y[q][3] = x[q + 12];
      dft4(y[q][0], y[q][1], y[q][2], y[q][3]);
    }
    // twiddles W16^e = cos(2 pi e/16) - i sin(2 pi e/16), e = q p
    y[1][1] = cmulk(y[1][1], c1, -s1);
    y[1][2] = cmulk(y[1][2], h, -h);
    y[1][3] = cmulk(y[1][3], s1, -c1);
    y[2][1] = cmulk(y[2][1], h, -h);
    y[2][2] = {y[2][2].y, -y[2][2].x};
    y[2][3] = cmulk(y[2][3], -h, -h);
    y[3][1] = cmulk(y[3][1], s1, -c1);
    y[3][2] = cmulk(y[3][2], -h, -h);
    y[3][3] = cmulk(y[3][3], -c1, s1);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      cx<T> a0 = y[0][p], a1 = y[1][p], a2 = y[2][p], a3 = y[3][p];
      dft4(a0, a1, a2, a3);
      x[p] = a0;
      x[p + 4] = a1;
      x[p + 8] = a2;
      x[p + 12] = a3;
    }
  }
}

// cos(pi t / 16), sin(pi t / 16), t = 0..15.
__device__ constexpr double kCos16[16] = {
    1.0, 0.980785280403230449126, 0.923879532511286756128, 0.831469612302545237079,
    0.707106781186547524401, 0.555570233019602224743, 0.382683432365089771728,
    0.195090322016128267848, 0.0, -0.195090322016128267848, -0.382683432365089771728,
    -0.555570233019602224743, -0.707106781186547524401, -0.831469612302545237079,
    -0.923879532511286756128, -0.980785280403230449126};
__device__ constexpr double kSin16[16] = {
    0.0, 0.195090322016128267848, 0.382683432365089771728, 0.555570233019602224743,
    0.707106781186547524401, 0.831469612302545237079, 0.923879532511286756128,
    0.980785280403230449126, 1.0, 0.980785280403230449126, 0.923879532511286756128,
    0.831469612302545237079, 0.707106781186547524401, 0.555570233019602224743,
    0.382683432365089771728, 0.195090322016128267848};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Number of table twiddles a radix-RHO butterfly loads: w, w^4, w^8, w^12
// (radix 16), w, w^4 (radix 8), w (radix 4, 2); the other powers are one
// complex product away from them.
template <int RHO>
struct TwBase {
  static constexpr int NBASE = RHO == 16 ? 4 : RHO == 8 ? 2 : 1;
};

// Base twiddles of the butterflies of lane j in a Stockham step of radix RHO
// with ns = 2^log2ns (table entry (r k1) K / (ns RHO) = e^{2 pi i r k1 / (ns RHO)}).
template <typename T, int K, int R, int RHO>
__device__ __forceinline__ void load_tw(cx<T> (&b)[R / RHO][TwBase<RHO>::NBASE], int j,
                                        int log2ns, const cx<T>* __restrict__ tw) {
  constexpr int G = K / R;
  constexpr int NB = R / RHO;
  constexpr int LOG2RHO = RHO == 16 ? 4 : RHO == 8 ? 3 : RHO == 4 ? 2 : 1;
  constexpr int LOG2K = __builtin_ctz(K);
  const int ns = 1 << log2ns;
  const int sh = LOG2K - log2ns - LOG2RHO;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int k1 = (j + G * i) & (ns - 1);
#pragma unroll
    for (int q = 0; q < TwBase<RHO>::NBASE; ++q) b[i][q] = tw[((q == 0 ? 1 : 4 * q) * k1) << sh];
  }
}

// All RHO powers w^r of one butterfly from its base twiddles.
template <typename T, int RHO>
__device__ __forceinline__ void tw_powers(const cx<T> (&b)[TwBase<RHO>::NBASE], cx<T> (&w)[RHO]) {
  w[0] = {T(1), T(0)};
  w[1] = b[0];
  if constexpr (RHO >= 4) {
    w[2] = cmul(b[0], b[0]);
    w[3] = cmul(w[2], b[0]);
  }
  if constexpr (RHO >= 8) {
    w[4] = b[1];
#pragma unroll
    for (int r = 1; r < 4; ++r) w[4 + r] = cmul(b[1], w[r]);
  }
  if constexpr (RHO == 16) {
    w[8] = b[2];
    w[12] = b[3];
#pragma unroll
    for (int r = 1; r < 4; ++r) {
      w[8 + r] = cmul(b[2], w[r]);
      w[12 + r] = cmul(b[3], w[r]);
    }
  }
}

// One Stockham step of radix RHO on the task's K points.  Lane j of the task
// holds the points j + G t (t = 0..R-1) in v; it performs R/RHO butterflies
// b = j + G i and writes their outputs to buf (natural Stockham positions).
// tb: the butterflies' base twiddles (unused in the first step).
template <typename T, int K, int R, int RHO>
__device__ __forceinline__ void fft_step(cx<T> (&v)[R], cx<T>* buf, int j, int log2ns,
                                         const cx<T> (&tb)[R / RHO][TwBase<RHO>::NBASE]) {
  constexpr int G = K / R;
  constexpr int NB = R / RHO;
  constexpr int LOG2RHO = RHO == 16 ? 4 : RHO == 8 ? 3 : RHO == 4 ? 2 : 1;
  const int ns = 1 << log2ns;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = j + G * i;
    const int k1 = b & (ns - 1);
    cx<T> x[RHO];
#pragma unroll
    for (int r = 0; r < RHO; ++r) x[r] = v[i + NB * r];
    if (log2ns > 0) {
      cx<T> w[RHO];
      tw_powers<T, RHO>(tb[i], w);
#pragma unroll
      for (int r = 1; r < RHO; ++r) x[r] = cmulc(x[r], w[r]);
    }
    dft<T, RHO>(x);
    const int d = ((b - k1) << LOG2RHO) + k1;
#pragma unroll
    for (int r = 0; r < RHO; ++r) buf[sw(d + r * ns)] = x[r];
  }
}

template <typename T, int K, int R>
__device__ __forceinline__ void load_canonical(cx<T> (&v)[R], const cx<T>* buf, int j) {
  constexpr int G = K / R;
#pragma unroll
  for (int t = 0; t < R; ++t) v[t] = buf[sw(j + G * t)];
}

// Points per lane: R = min(RMAX, K); a transform of K = 2^LOG2K points takes
// at most three radix-(<= R) steps.
template <int LOG2K, int LOG2RMAX = 4>
struct FftShape {
  static constexpr int K = 1 << LOG2K;
  static constexpr int LOG2R = LOG2K < LOG2RMAX ? LOG2K : LOG2RMAX;
  static constexpr int R = 1 << LOG2R;
  static constexpr int G = K / R;
};

// Forward K-point FFT of the task's points (in v, canonical distribution);
// result in natural order in buf.  The twiddles of the later steps are
// loaded before the first step, so that their latency overlaps it.
template <typename T, int LOG2K, int LOG2RMAX>
__device__ __forceinline__ void task_fft(cx<T> (&v)[(FftShape<LOG2K, LOG2RMAX>::R)], cx<T>* buf,
                                         int j, const cx<T>* __restrict__ tw) {
  using S = FftShape<LOG2K, LOG2RMAX>;
  constexpr int K = S::K, R = S::R, LR = S::LOG2R;
  constexpr int L1 = LOG2K - LR;                 // left after the first step
  constexpr int S2 = L1 >= LR ? LR : L1;         // log2 of the second radix
  constexpr int R2 = S2 > 0 ? (1 << S2) : 2;
  constexpr int D2 = LR;
  constexpr int L2 = L1 - S2;
  constexpr int R3 = L2 > 0 ? (1 << L2) : 2;
  constexpr int D3 = D2 + S2;
  static_assert(L2 <= LR, "at most three steps");
  cx<T> none[R / R][TwBase<R>::NBASE];
  cx<T> t2[R / R2][TwBase<R2>::NBASE];
  cx<T> t3[R / R3][TwBase<R3>::NBASE];
  if constexpr (L1 > 0) load_tw<T, K, R, R2>(t2, j, D2, tw);
  if constexpr (L2 > 0) load_tw<T, K, R, R3>(t3, j, D3, tw);
  fft_step<T, K, R, R>(v, buf, j, 0, none);
  if constexpr (L1 > 0) {
    wave_sync();
    load_canonical<T, K, R>(v, buf, j);
    wave_sync();
    fft_step<T, K, R, R2>(v, buf, j, D2, t2);
    if constexpr (L2 > 0) {
      wave_sync();
      load_canonical<T, K, R>(v, buf, j);
      wave_sync();
      fft_step<T, K, R, R3>(v, buf, j, D3, t3);
    }
  }
  wave_sync();
}

// sin(pi jj / K) for the task points jj = j + G t (t = 0..R-1) of lane j, from
// sin and cos of pi j / K (two table reads) and the constants of pi t / R.
template <typename T, int K, int R>
__device__ __forceinline__ void task_sines(const T* __restrict__ sn, int j, T (&out)[R]) {
  static_assert(R <= 16, "16 rotation constants");
  const T sa = sn[j], ca = sn[K / 2 - j];
#pragma unroll
  for (int t = 0; t < R; ++t)
    out[t] = sa * (T)kCos16[t * (16 / R)] + ca * (T)kSin16[t * (16 / R)];
}

// After task_fft: the two sine transforms of the pair, (X^a_k, X^b_k) at
// index k = 1..K-1 of buf (index 0 set to zero).  Lane j handles the wave
// numbers k in [j C, (j+1) C), C = K / (2 G).
template <typename T, int LOG2K, int LOG2RMAX>
__device__ __forceinline__ void task_post(cx<T>* buf, int j) {
  using S = FftShape<LOG2K, LOG2RMAX>;
  constexpr int K = S::K, G = S::G;
  constexpr int C = (K / 2) / G;
  // The running sums are carried in FP64 whatever T is: in FP32 their
  // rounding error would grow with K and vary smoothly along k.
  cx<T> ev[C];
  cx<double> rv[C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int k = j * C + i;
    const cx<T> a = buf[sw(k)];
    const cx<T> b = buf[sw((K - k) & (K - 1))];
    // Y^a_k = (W_k + conj W_{K-k}) / 2, Y^b_k = (W_k - conj W_{K-k}) / (2i):
    // even outputs X_{2k} = -Im Y_k, running-sum terms R_k = Re Y_k.
    ev[i] = {T(0.5) * (b.y - a.y), T(0.5) * (a.x - b.x)};
    rv[i] = {0.5 * ((double)a.x + (double)b.x), 0.5 * ((double)a.y + (double)b.y)};
    if (k == 0) {
      ev[i] = {T(0), T(0)};
      rv[i] = {0.5 * (double)a.x, 0.5 * (double)a.y};   // X_1 = Re Y_0 / 2
    }
  }
#pragma unroll
  for (int i = 1; i < C; ++i) rv[i] = cadd(rv[i], rv[i - 1]);
  // segmented inclusive scan of the lane totals over the G lanes of the task
  cx<double> incl = rv[C - 1];
  const cx<double> tot = incl;
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    const double ux = __shfl_up(incl.x, off, G);
    const double uy = __shfl_up(incl.y, off, G);
    if (j >= off) {
      incl.x += ux;
      incl.y += uy;
    }
  }
  const cx<double> excl = csub(incl, tot);
  wave_sync();
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int k = j * C + i;
    buf[sw(2 * k)] = ev[i];
    const cx<double> o = cadd(rv[i], excl);
    buf[sw(2 * k + 1)] = cx<T>{(T)o.x, (T)o.y};
  }
  wave_sync();
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Value x_j of sequence s (0 = nodes, s >= 1 = interior component s) of the
// forward pre-combine, read from a physical line in LDS; zero outside 1..K-1.
template <typename T, int N, int K>
__device__ __forceinline__ T fwd_seq(const T* ln, int s, int j) {
  if (j <= 0 || j >= K || s >= N) return T(0);
  if (s == 0) return ln[N * j - 1];
  return ln[N * j + s - 1] + ln[N * (j - 1) + (N - s) - 1];
}

// Value of sequence s at wave number j from a coefficient-ordered line in LDS
// after the inverse block (W_j at q = N-1 + j-1, d_j component s at
// q = N-1 + s (K-1) + j-1).
template <typename T, int N, int K>
__device__ __forceinline__ T inv_seq(const T* ln, int s, int j) {
  if (j <= 0 || j >= K || s >= N) return T(0);
  return ln[(N - 1) + s * (K - 1) + j - 1];
}

// Sine-transform pre-processing of one pair at index j.
template <typename T>
__device__ __forceinline__ cx<T> dst_pre(cx<T> xj, cx<T> xkj, T snj, int j) {
  if (j == 0) return {T(0), T(0)};
  return {snj * (xj.x + xkj.x) + T(0.5) * (xj.x - xkj.x),
          snj * (xj.y + xkj.y) + T(0.5) * (xj.y - xkj.y)};
}

// The N sine-transform outputs of one line (its slots) at wave number k.
template <typename T, int N, int K>
__device__ __forceinline__ void read_seqs(const cx<T>* ls, int k, T (&x)[N]) {
#pragma unroll
  for (int p = 0; p < (N + 1) / 2; ++p) {
    const cx<T> v = ls[p * K + sw(k)];
    x[2 * p] = v.x;
    if (2 * p + 1 < N) x[2 * p + 1] = v.y;
  }
}

// Entry e of the blocked table at wave number k (see AxisTab).
template <int N>
__device__ __forceinline__ size_t blk_base(int k) {
  constexpr int NE = N * (N - 1) + N;
  return (size_t)((k - 1) >> 6) * (NE * 64) + ((k - 1) & 63);
}

// Direct-transform coefficients at wave number k >= 1:
// acc[l] = (x_0 + sum_s p_k^(l)_s x_s) / ||s_k^(l)||^2.
template <typename T, int N>
__device__ __forceinline__ void fwd_block(const T* __restrict__ tb, const T (&x)[N],
                                          T (&acc)[N]) {
#pragma unroll
  for (int l = 0; l < N; ++l) {
    T s = x[0];
#pragma unroll
    for (int i = 1; i < N; ++i) s += tb[(l * (N - 1) + i - 1) * 64] * x[i];
    acc[l] = s * tb[(N * (N - 1) + l) * 64];
  }
}

// Inverse-transform combination at k >= 1: y_0 = sum_l w_l,
// y_s = sum_l w_l p_k^(l)_s.
template <typename T, int N>
__device__ __forceinline__ void inv_block(const T* __restrict__ tb, const T (&w)[N], T (&y)[N]) {
  constexpr int NP_ = N * (N - 1);
  T tab[NP_ > 0 ? NP_ : 1];
#pragma unroll
  for (int e = 0; e < NP_; ++e) tab[e] = tb[e * 64];
#pragma unroll
  for (int i = 0; i < N; ++i) y[i] = T(0);
#pragma unroll
  for (int l = 0; l < N; ++l) {
    y[0] += w[l];
#pragma unroll
    for (int i = 1; i < N; ++i) y[i] += w[l] * tab[l * (N - 1) + i - 1];
  }
}

// Fused pass at k >= 1: direct coefficients, division by the FP64
// denominators dbase + sc lamk[l], inverse combination.  The wave number's
// table entries are all loaded first (one read each, every load in flight at
// once) and then used for both products.
template <typename T, int N>
__device__ __forceinline__ void fused_block(const T* __restrict__ tb, const double* __restrict__ lk,
                                            int K, double dbase, double sc, const T (&x)[N],
                                            T (&y)[N]) {
  constexpr int NE = N * (N - 1) + N;
  T tab[NE];
  double lam[N];
#pragma unroll
  for (int e = 0; e < NE; ++e) tab[e] = tb[e * 64];
#pragma unroll
  for (int l = 0; l < N; ++l) lam[l] = lk[(size_t)l * (K - 1)];
#pragma unroll
  for (int i = 0; i < N; ++i) y[i] = T(0);
#pragma unroll
  for (int l = 0; l < N; ++l) {
    T s = x[0];
#pragma unroll
    for (int i = 1; i < N; ++i) s += tab[l * (N - 1) + i - 1] * x[i];
    s *= tab[N * (N - 1) + l];
    const T w = (T)((double)s / (dbase + sc * lam[l]));
    y[0] += w;
#pragma unroll
    for (int i = 1; i < N; ++i) y[i] += w * tab[l * (N - 1) + i - 1];
  }
}

// log2 of the points per lane: 8 in FP64 for K <= 512 (fewer registers, so
// that more workgroups share a CU), 16 otherwise.
template <typename T, int LOG2K>
constexpr int log2_rmax() { return (sizeof(T) == 8 && LOG2K <= 9) ? 3 : 4; }

// Register budget: four waves per SIMD (two 512-lane workgroups per CU, up
// to 128 VGPRs), except in FP64 for single-line passes and orders >= 7,
// whose per-wave-number tables alone take 2 n^2 registers (two waves).
template <typename T, int N, int LOG2K, int MODE>
constexpr int waves_per_simd() {
  if (sizeof(T) == 8) return (LOG2K <= 9 && N <= 6) ? 4 : 2;
  return 4;
}

template <typename T, int N, int LOG2K, int MODE, typename TIN, typename TOUT>
__global__ __launch_bounds__(threads_for<T>())
__attribute__((amdgpu_waves_per_eu(waves_per_simd<T, N, LOG2K, MODE>()))) void line_pass(PassArgs a) {
  constexpr int LRM = log2_rmax<T, LOG2K>();
  using S = FftShape<LOG2K, LRM>;
  constexpr int K = S::K, R = S::R, G = S::G;
  constexpr int TPW = 64 / G;          // tasks per wavefront
  constexpr int NP = (N + 1) / 2;      // slot pairs per line
  constexpr int M = N * K - 1;         // line length
  constexpr int KM = K - 1;
  constexpr int kUnroll = unroll_for<T, LOG2K>();
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int wave = tid >> 6, nwaves = nthr >> 6;
  const long long inner = a.inner;
  const int cb = a.cb;            // a power of two
  const int lcb = __builtin_ctz(cb);
  // One line per workgroup ("tight"): LDS holds the slots and nothing else,
  // so that two workgroups with the largest lines share a CU; the line's
  // address and denominator live in registers and the k = 0 quantities S0
  // and E0 in the index-0 entries of the slots, which no sine transform
  // output occupies.  Several lines: one pad entry per line (spreads the
  // lines over the LDS banks) and small arrays after the slots.
  const bool tight = cb == 1;
  const int lsp = tight ? NP * K : NP * K + 1;   // complex entries per line
  // Workgroups are dealt round-robin to the 8 XCDs (each with its own L2):
  // renumber them so that every XCD walks one contiguous range of lines, and
  // the lines that share cache lines (neighbouring columns of a strided
  // axis) meet in the same L2.
  const unsigned nb = gridDim.x, xcd = blockIdx.x % kXcds, per = nb / kXcds, rem = nb % kXcds;
  const unsigned wg = xcd * per + min(xcd, rem) + blockIdx.x / kXcds;
  const long long L0 = (long long)wg * cb;
  const int cv = (int)min((long long)cb, a.nlines - L0);
  const bool cfast = inner != 1;

  cx<T>* slots = reinterpret_cast<cx<T>*>(smem);
  T* lines = reinterpret_cast<T*>(smem);        // line c at lines + c * 2 * lsp
  T* s0 = reinterpret_cast<T*>(slots + (size_t)cb * lsp);   // [cb][8] (not tight)
  T* e0 = s0 + cb * 8;                                      // [cb][8] (not tight)
  long long* base = reinterpret_cast<long long*>(e0 + cb * 8);   // [cb] (not tight)
  double* denb = reinterpret_cast<double*>(base + cb);           // [cb] (not tight)
  // index-0 store of sequence-pair entries of line 0 (tight): value s < N-1
  auto i0 = [&](int s) -> T& { return lines[(size_t)(s >> 1) * 2 * K + (s & 1)]; };

  const T* __restrict__ BLK = static_cast<const T*>(a.tab.blk);
  const T* __restrict__ EV = static_cast<const T*>(a.tab.E);
  const cx<T>* __restrict__ TW = static_cast<const cx<T>*>(a.tab.tw);
  const T* __restrict__ SN = static_cast<const T*>(a.tab.sn);
  const TIN* __restrict__ src = static_cast<const TIN*>(a.in);
  TOUT* __restrict__ dst = static_cast<TOUT*>(a.out);

  // this lane's FFT task: (line tc, slot pair tp), lane j of G
  const int lane = tid & 63;
  const int task = wave * TPW + lane / G;
  const int j = lane & (G - 1);
  const bool task_ok = task < cb * NP;
  const int tc = task_ok ? task / NP : 0;
  const int tp = task - tc * NP;
  cx<T>* tbuf = slots + (size_t)tc * lsp + (size_t)tp * K;
  T snr[R];   // DST pre-weights sin(pi jj / K) of this lane's task points
  task_sines<T, K, R>(SN, j, snr);

  auto line_den = [&](long long t) -> double {
    double d = a.alpha;
    for (int i = 0; i < a.nother; ++i) d += a.oscale[i] * a.olam[i][(t / a.odiv[i]) % a.omod[i]];
    return d;
  };
  long long base1 = 0;
  double den1 = 0.0;
  if (tight) {
    const long long o = L0 / inner, t = L0 - o * inner;
    base1 = o * (long long)M * inner + t;
    if (MODE == PASS_FUSED) den1 = line_den(t);
  } else if (tid < cv) {
    const long long L = L0 + tid;
    const long long o = L / inner, t = L - o * inner;
    base[tid] = o * (long long)M * inner + t;
    if (MODE == PASS_FUSED) denb[tid] = line_den(t);
  }
  auto lbase = [&](int c) -> long long { return tight ? base1 : base[c]; };
  auto lden = [&](int c) -> double { return tight ? den1 : denb[c]; };
  auto s0v = [&](int c, int s) -> T { return tight ? i0(s) : s0[c * 8 + s]; };
  auto e0v = [&](int c, int s) -> T { return tight ? i0(s) : e0[c * 8 + s]; };

  // ---- load the cv lines (physical or coefficient order) ------------------
  // Contiguous axis: the cv lines are one contiguous range, swept by all
  // lanes.  Strided axis: lane (q, c) with c = tid mod cb, so adjacent lanes
  // read adjacent lines (adjacent in memory).  kUnroll loads in flight per
  // lane: one round for the longest lines.
  if (!cfast) {
    const TIN* sp = src + L0 * M;
    const int total = cv * M;
    for (int i00 = tid; i00 < total; i00 += kUnroll * nthr) {
      TIN r[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = i00 + u * nthr;
        r[u] = sp[i < total ? i : 0];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = i00 + u * nthr;
        if (i < total) {
          const int c = i / M, q = i - c * M;
          lines[(size_t)c * 2 * lsp + q] = (T)r[u];
        }
      }
    }
    __syncthreads();
  } else {
    __syncthreads();   // base[]
    const int c = tid & (cb - 1);
    const int qs = nthr >> lcb;
    if (c < cv) {
      const TIN* sp = src + lbase(c);
      T* d = lines + (size_t)c * 2 * lsp;
      for (int q0 = tid >> lcb; q0 < M; q0 += kUnroll * qs) {
        TIN r[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int q = q0 + u * qs;
          r[u] = sp[(long long)(q < M ? q : 0) * inner];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int q = q0 + u * qs;
          if (q < M) d[q] = (T)r[u];
        }
      }
    }
    __syncthreads();
  }

  cx<T> v[R];
  T e0r[N > 1 ? N - 1 : 1];   // tight: E0 of the line, in thread 0

  if (MODE == PASS_FWD || MODE == PASS_FUSED) {
    // ---- forward pre-combine + sine pre-processing, into registers -------
    if (task_ok) {
      const T* ln = lines + (size_t)tc * 2 * lsp;
      const bool live = tc < cv;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int jj = j + G * t;
        cx<T> xj = {fwd_seq<T, N, K>(ln, 2 * tp, jj), fwd_seq<T, N, K>(ln, 2 * tp + 1, jj)};
        cx<T> xk = {fwd_seq<T, N, K>(ln, 2 * tp, K - jj),
                    fwd_seq<T, N, K>(ln, 2 * tp + 1, K - jj)};
        v[t] = live ? dst_pre(xj, xk, snr[t], jj) : cx<T>{T(0), T(0)};
      }
    }
    // S0_s = sum_{j=1..K} ((-P)^{j-1} y_{j-1/2})_s, one wave per (line, s);
    // tight: a wave keeps its (at most two) sums in registers until the
    // slots' index-0 entries are free.
    T s0r[2] = {T(0), T(0)};
    if constexpr (N > 1) {
      int r = 0;
      for (int task0 = wave; task0 < cv * (N - 1); task0 += nwaves, ++r) {
        const int c = task0 / (N - 1), s = task0 - c * (N - 1) + 1;
        const T* ln = lines + (size_t)c * 2 * lsp;
        T acc = T(0);
        for (int jj = 1 + lane; jj <= K; jj += 64) {
          const bool odd = jj & 1;
          const T val = ln[N * (jj - 1) + (odd ? s : N - s) - 1];
          acc += odd ? val : -val;
        }
        acc = wave_sum(acc);
        if (tight) {
          if (r == 0) s0r[0] = acc; else s0r[1] = acc;
        } else if (lane == 0) {
          s0[c * 8 + s - 1] = acc;
        }
      }
    }
    __syncthreads();
    if (task_ok) {
      task_fft<T, LOG2K, LRM>(v, tbuf, j, TW);
      task_post<T, LOG2K, LRM>(tbuf, j);
    }
    __syncthreads();
    if constexpr (N > 1) {
      if (tight) {
        if (lane == 0) {
          if (wave < N - 1) i0(wave) = s0r[0];
          if (wave + nwaves < N - 1) i0(wave + nwaves) = s0r[1];
        }
        __syncthreads();
      }
    }

    if (MODE == PASS_FWD) {
      // ---- forward block, coefficients to global -------------------------
      // contiguous axis: k fastest over the lanes (l-major output order);
      // strided axis: line c fastest (adjacent lines adjacent in memory)
      const int items = cv * KM;
      for (int i = tid; i < (cfast ? cb * KM : items); i += nthr) {
        int c, k;
        if (cfast) {
          c = i & (cb - 1);
          k = (i >> lcb) + 1;
          if (c >= cv) continue;
        } else {
          c = i / KM;
          k = i - c * KM + 1;
        }
        T x[N], acc[N];
        read_seqs<T, N, K>(slots + (size_t)c * lsp, k, x);
        fwd_block<T, N>(BLK + blk_base<N>(k), x, acc);
        const long long ob = lbase(c) + ((long long)(N - 1) + (k - 1)) * inner;
#pragma unroll
        for (int l = 0; l < N; ++l) dst[ob + (long long)l * KM * inner] = (TOUT)acc[l];
      }
      // k = 0: w_{0l} = S0 . e^(l) / K
      if constexpr (N > 1) {
        const int items0 = cv * (N - 1);
        for (int i = tid; i < items0; i += nthr) {
          const int c = i / (N - 1), l = i - c * (N - 1);
          T acc = T(0);
#pragma unroll
          for (int s = 0; s < N - 1; ++s) acc += EV[s * (N - 1) + l] * s0v(c, s);
          dst[lbase(c) + (long long)l * inner] = (TOUT)(acc / (T)K);
        }
      }
      return;
    }

    // ---- fused: forward block, spectral division, inverse block ----------
    {
      const double sc = a.scale;
      const double* __restrict__ lam = a.tab.lam;
      const int items = cv * KM;
      for (int i = tid; i < items; i += nthr) {
        const int c = i / KM, k = i - c * KM + 1;
        cx<T>* ls = slots + (size_t)c * lsp;
        T x[N], y[N];
        read_seqs<T, N, K>(ls, k, x);
        fused_block<T, N>(BLK + blk_base<N>(k), lam + (N - 1) + (k - 1), K, lden(c), sc, x, y);
#pragma unroll
        for (int s = 0; s < N; ++s) {
          cx<T>& sl = ls[(s >> 1) * K + sw(k)];
          if (s & 1) sl.y = y[s]; else sl.x = y[s];
        }
        if (N & 1) ls[(NP - 1) * K + sw(k)].y = T(0);
      }
      if constexpr (N > 1) {
        if (tid < cv) {
          const int c = tid;
          T s0l[N - 1], w0[N - 1];
#pragma unroll
          for (int s = 0; s < N - 1; ++s) s0l[s] = s0v(c, s);
#pragma unroll
          for (int l = 0; l < N - 1; ++l) {
            T acc = T(0);
#pragma unroll
            for (int s = 0; s < N - 1; ++s) acc += EV[s * (N - 1) + l] * s0l[s];
            acc /= (T)K;
            const double den = lden(c) + sc * lam[l];
            w0[l] = (T)((double)acc / den);
          }
#pragma unroll
          for (int s = 0; s < N - 1; ++s) {
            T acc = T(0);
#pragma unroll
            for (int l = 0; l < N - 1; ++l) acc += EV[s * (N - 1) + l] * w0[l];
            if (tight) e0r[s] = acc; else e0[c * 8 + s] = acc;
          }
        }
      }
      __syncthreads();
      // sine pre-processing of the task's own (W, d) pair, in registers (the
      // weights are recomputed here rather than held across the block phase)
      task_sines<T, K, R>(SN, j, snr);
      if (task_ok) {
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int jj = j + G * t;
          v[t] = dst_pre(tbuf[sw(jj)], tbuf[sw((K - jj) & (K - 1))], snr[t], jj);
        }
        wave_sync();
      }
    }
  } else {
    // ---- inverse: block in place on the coefficient line -----------------
    // (thread of wave number k reads and writes the entries N-1 + l(K-1) + k-1)
    const int items = cv * KM;
    for (int i = tid; i < items; i += nthr) {
      const int c = i / KM, k = i - c * KM + 1;
      T* ln = lines + (size_t)c * 2 * lsp + (N - 1) + (k - 1);
      T w[N], y[N];
#pragma unroll
      for (int l = 0; l < N; ++l) w[l] = ln[l * KM];
      inv_block<T, N>(BLK + blk_base<N>(k), w, y);
#pragma unroll
      for (int s = 0; s < N; ++s) ln[s * KM] = y[s];
    }
    if constexpr (N > 1) {
      if (tid < cv) {
        const int c = tid;
        const T* ln = lines + (size_t)c * 2 * lsp;
#pragma unroll
        for (int s = 0; s < N - 1; ++s) {
          T acc = T(0);
#pragma unroll
          for (int l = 0; l < N - 1; ++l) acc += EV[s * (N - 1) + l] * ln[l];
          if (tight) e0r[s] = acc; else e0[c * 8 + s] = acc;
        }
      }
    }
    __syncthreads();
    if (task_ok) {
      const T* ln = lines + (size_t)tc * 2 * lsp;
      const bool live = tc < cv;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int jj = j + G * t;
        cx<T> xj = {inv_seq<T, N, K>(ln, 2 * tp, jj), inv_seq<T, N, K>(ln, 2 * tp + 1, jj)};
        cx<T> xk = {inv_seq<T, N, K>(ln, 2 * tp, K - jj),
                    inv_seq<T, N, K>(ln, 2 * tp + 1, K - jj)};
        v[t] = live ? dst_pre(xj, xk, snr[t], jj) : cx<T>{T(0), T(0)};
      }
    }
    __syncthreads();
  }

  // ---- inverse sine transforms and scatter to the physical line ----------
  if (task_ok) {
    task_fft<T, LOG2K, LRM>(v, tbuf, j, TW);
    task_post<T, LOG2K, LRM>(tbuf, j);
  }
  __syncthreads();
  if constexpr (N > 1) {
    if (tight) {
      if (tid == 0) {
#pragma unroll
        for (int s = 0; s < N - 1; ++s) i0(s) = e0r[s];
      }
      __syncthreads();
    }
  }
  {
    // value at position g = q + 1 = N jn + s of line c (s = 0: mesh node)
    auto value = [&](int c, int q) -> T {
      const int g = q + 1, jn = g / N, s = g - jn * N;
      const cx<T>* ls = slots + (size_t)c * lsp;
      auto seq = [&](int sq, int k) -> T {
        const cx<T> w = ls[(sq >> 1) * K + sw(k)];
        return (sq & 1) ? w.y : w.x;
      };
      if (s == 0) return seq(0, jn);
      const int je = jn + 1;   // element
      const T zl = (je - 1 >= 1) ? seq(s, je - 1) : T(0);
      const T zr = (je <= K - 1) ? seq(N - s, je) : T(0);
      const T ee = (je & 1) ? e0v(c, s - 1) : -e0v(c, (N - s) - 1);
      return zl + zr + ee;
    };
    if (!cfast) {
      TOUT* d = dst + L0 * M;
      const int total = cv * M;
      for (int i = tid; i < total; i += nthr) {
        const int c = i / M, q = i - c * M;
        d[i] = (TOUT)value(c, q);
      }
    } else {
      const int c = tid & (cb - 1);
      const int qs = nthr >> lcb;
      if (c < cv) {
        TOUT* d = dst + lbase(c);
        for (int q = tid >> lcb; q < M; q += qs) d[(long long)q * inner] = (TOUT)value(c, q);
      }
    }
  }
}

struct Shape {
  int cb, threads;
  size_t lds;
};

inline Shape shape_for(int n, int K, size_t cplx_bytes, long long nlines) {
  const int NP = (n + 1) / 2;
  const int rmax = (cplx_bytes == 16 && K <= 512) ? 8 : 16;   // as log2_rmax
  const int R = K < rmax ? K : rmax;
  const int G = K / R;
  const int TPW = 64 / G;
  const size_t per_line = ((size_t)NP * K + 1) * cplx_bytes;
  // LDS: about 64 KB per workgroup (two or more workgroups per CU); a line
  // that needs more gets a workgroup of its own.
  long long c = (long long)((64 * 1024) / per_line);
  const int threads = cplx_bytes == 16 ? threads_for<double>() : threads_for<float>();
  // every FFT task of the workgroup runs at once
  c = std::min<long long>(c, (long long)(threads / 64) * TPW / NP);
  c = std::min<long long>(c, kMaxCB);
  c = std::min<long long>(c, nlines);
  if (c < 1) c = 1;
  while (c & (c - 1)) c &= c - 1;   // round down to a power of two
  Shape s;
  s.cb = (int)c;
  s.threads = threads;
  if (c == 1)   // slots only (see line_pass)
    s.lds = (size_t)NP * K * cplx_bytes;
  else
    s.lds = (size_t)c * per_line + (size_t)c * 16 * (cplx_bytes / 2) + (size_t)c * 16;
  return s;
}

template <typename T, int N, int LOG2K, int MODE, typename TIN, typename TOUT>
hipError_t launch_k(const PassArgs& a, hipStream_t s) {
  const Shape sh = shape_for(N, 1 << LOG2K, sizeof(cx<T>), a.nlines);
  if (sh.cb != a.cb || a.tab.n != N || a.tab.K != (1 << LOG2K)) return hipErrorInvalidValue;
  auto fn = line_pass<T, N, LOG2K, MODE, TIN, TOUT>;
  static bool lds_raised = false;   // benign race: every caller sets the same value
  if (!lds_raised) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_raised = true;
  }
  const long long blocks = (a.nlines + a.cb - 1) / a.cb;
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(sh.threads), sh.lds, s, a);
  return hipGetLastError();
}

template <typename T, int N, int MODE, typename TIN, typename TOUT>
hipError_t launch_by_k(const PassArgs& a, hipStream_t s) {
  switch (a.tab.K) {
    case 2: return launch_k<T, N, 1, MODE, TIN, TOUT>(a, s);
    case 4: return launch_k<T, N, 2, MODE, TIN, TOUT>(a, s);
    case 8: return launch_k<T, N, 3, MODE, TIN, TOUT>(a, s);
    case 16: return launch_k<T, N, 4, MODE, TIN, TOUT>(a, s);
    case 32: return launch_k<T, N, 5, MODE, TIN, TOUT>(a, s);
    case 64: return launch_k<T, N, 6, MODE, TIN, TOUT>(a, s);
    case 128: return launch_k<T, N, 7, MODE, TIN, TOUT>(a, s);
    case 256: return launch_k<T, N, 8, MODE, TIN, TOUT>(a, s);
    case 512: return launch_k<T, N, 9, MODE, TIN, TOUT>(a, s);
    case 1024: return launch_k<T, N, 10, MODE, TIN, TOUT>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
hipError_t launch_order(int kind, int dt, const PassArgs& a, hipStream_t s) {
  // Instantiated combinations: kind x (compute, in, out) as the solver uses them.
  switch (kind) {
    case PASS_FWD:
      if (dt == 0) return launch_by_k<double, N, PASS_FWD, double, double>(a, s);
      if (dt == 1) return launch_by_k<float, N, PASS_FWD, float, float>(a, s);
      if (dt == 2) return launch_by_k<float, N, PASS_FWD, double, float>(a, s);
      break;
    case PASS_INV:
      if (dt == 0) return launch_by_k<double, N, PASS_INV, double, double>(a, s);
      if (dt == 1) return launch_by_k<float, N, PASS_INV, float, float>(a, s);
      if (dt == 3) return launch_by_k<float, N, PASS_INV, float, double>(a, s);
      break;
    case PASS_FUSED:
      if (dt == 0) return launch_by_k<double, N, PASS_FUSED, double, double>(a, s);
      if (dt == 1) return launch_by_k<float, N, PASS_FUSED, float, float>(a, s);
      if (dt == 5) return launch_by_k<float, N, PASS_FUSED, double, double>(a, s);
      break;
    default:
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace lp
}  // namespace hofem
