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
// LDS holds, per line, ceil(N/2) complex arrays of length K ("slot pairs"):
// interior component s and its mirror N - s share a pair, the node sequence
// takes the last one (layout at struct Seq below).  Each sine-transform task
// works on its own pair only, so a workgroup may run more tasks than it has
// wavefronts, in rounds.  The physical line is loaded straight into the
// entries of its sequences.
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
// Workgroup size: 8 waves (the register budget of waves_per_simd_of decides
// how many workgroups share a CU); the load, block and scatter phases use
// all lanes.  The one exception, set by shape_for: the inverse row pass of
// long FP64 lines runs 4 waves per line, two workgroups per CU.
template <typename T>
constexpr int threads_for() { return 512; }
// global loads in flight per lane: one round for the workgroup's values
// (at most 64 KB of lines per workgroup in the padded layout; the tight
// layout's two lines take ceil(2 (nK - 1) / 512) per lane, and so does one
// line on 256 lanes)
template <typename T, int N, int LOG2K, bool TIGHT>
constexpr int unroll_for() {
  return TIGHT ? (2 * (N * (1 << LOG2K) - 1) + 511) / 512 : (sizeof(T) == 8 && LOG2K >= 10) ? 32 : 16;
}
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

// 16 bytes of consecutive values, for vector loads and stores.
template <typename T>
struct alignas(16) vec16 {
  T v[16 / sizeof(T)];
};
// The values of two lines at one position of a row-pair interleaved block.
template <typename T>
struct alignas(2 * sizeof(T)) pair2 {
  T a, b;
};

// Elements of type T before the first 16-byte boundary at or after p.
template <typename T>
__device__ __forceinline__ int head16(const T* p) {
  return (int)(((16 - ((unsigned long long)p & 15)) & 15) / sizeof(T));
}

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

// cos(pi jj / K) for the same task points (cos(pi j / K) = sin(pi (K/2 - j) / K)).
template <typename T, int K, int R>
__device__ __forceinline__ void task_cosines(const T* __restrict__ sn, int j, T (&out)[R]) {
  static_assert(R <= 16, "16 rotation constants");
  const T sa = sn[j], ca = sn[K / 2 - j];
#pragma unroll
  for (int t = 0; t < R; ++t)
    out[t] = ca * (T)kCos16[t * (16 / R)] - sa * (T)kSin16[t * (16 / R)];
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

// Sine transforms of a pair without the running sums (FP32 inverse
// transforms).  The running sums add up K/2 rounded FFT outputs, so the odd
// outputs of an FP32 transform carry an error that grows like sqrt(k); on a
// smooth inverse transform that error alternates between odd and even nodes,
// i.e. it sits in the stiff high modes, and the next FP64 residual of a
// refinement step amplifies it by the condition number.  Here a second FFT
// of the cosine-weighted input y'_j = cos(pi j/K)(x_j + x_{K-j}) (an odd
// sequence, so its spectrum is imaginary: -Im Y'_k = X_{2k+1} + X_{2k-1})
// supplies the sums next to the differences R_k = Re Y_k = X_{2k+1} -
// X_{2k-1}, and X_{2k+1} = (R_k + Q_k) / 2 is formed directly.
// v: the sine-weighted input (as for task_fft), v2: the cosine-weighted one.
template <typename T, int LOG2K, int LOG2RMAX>
__device__ __forceinline__ void task_dst_direct(cx<T> (&v)[(FftShape<LOG2K, LOG2RMAX>::R)],
                                                cx<T> (&v2)[(FftShape<LOG2K, LOG2RMAX>::R)],
                                                cx<T>* buf, int j, const cx<T>* __restrict__ tw) {
  using S = FftShape<LOG2K, LOG2RMAX>;
  constexpr int K = S::K, G = S::G;
  constexpr int C = (K / 2) / G;
  task_fft<T, LOG2K, LOG2RMAX>(v, buf, j, tw);
  cx<T> ev[C], rv[C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int k = j * C + i;
    const cx<T> a = buf[sw(k)];
    const cx<T> b = buf[sw((K - k) & (K - 1))];
    ev[i] = k == 0 ? cx<T>{T(0), T(0)} : cx<T>{T(0.5) * (b.y - a.y), T(0.5) * (a.x - b.x)};
    rv[i] = {T(0.5) * (a.x + b.x), T(0.5) * (a.y + b.y)};   // R_k (R_0 = 2 X_1)
  }
  wave_sync();
  task_fft<T, LOG2K, LOG2RMAX>(v2, buf, j, tw);
  cx<T> od[C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int k = j * C + i;
    const cx<T> a = buf[sw(k)];
    const cx<T> b = buf[sw((K - k) & (K - 1))];
    // Q_k of both sequences (Q_0 = 0 exactly: a = b there)
    const cx<T> q = {T(0.5) * (b.y - a.y), T(0.5) * (a.x - b.x)};
    od[i] = {T(0.5) * (rv[i].x + q.x), T(0.5) * (rv[i].y + q.y)};
  }
  wave_sync();
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int k = j * C + i;
    buf[sw(2 * k)] = ev[i];
    buf[sw(2 * k + 1)] = od[i];
  }
  wave_sync();
}

// A value that is the same in every lane, moved to scalar registers (long
// lived per-line quantities then take no vector registers).
__device__ __forceinline__ long long uni(long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)x);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double x) {
  return __builtin_bit_cast(double, uni(__builtin_bit_cast(long long, x)));
}
__device__ __forceinline__ float uni(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(unsigned, x)));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---- line layout in LDS ------------------------------------------------------
//
// A line holds N sequences of K entries: sequence 0 the mesh nodes (entry j
// for node j = 1..K-1), sequence s >= 1 interior point s of the elements
// (entry e-1 for element e = 1..K).  The same entries hold in turn the
// physical values, the sine transforms, the coefficients of wave number k
// (entry k) and the inverse transforms; entry 0 of component s holds its
// k = 0 quantity (S0_s after the direct transforms, E0_s before the scatter).
// The sequences are stored as slot pairs of K complex entries: component s
// and its mirror N - s, which the reversal P couples, share a pair as real
// and imaginary part; the nodes take the last pair, together with the middle
// component N/2 when N is even.  The sine-transform task of a pair therefore
// reads and writes that pair only.
template <int N>
struct Seq {
  static constexpr int NP = (N + 1) / 2;
  __host__ __device__ static constexpr int pair(int s) {
    return (s == 0 || 2 * s == N) ? NP - 1 : (2 * s < N ? s - 1 : N - s - 1);
  }
  __host__ __device__ static constexpr int part(int s) { return (s == 0 || 2 * s < N) ? 0 : 1; }
};

// Entry i of sequence s of the line whose slots start at ls.
template <typename T, int N, int K>
__device__ __forceinline__ T& at(cx<T>* ls, int s, int i) {
  cx<T>& e = ls[Seq<N>::pair(s) * K + sw(i)];
  return Seq<N>::part(s) ? e.y : e.x;
}

// Input of the direct sine transforms of a pair at index j = 1..K-1, from
// its entries e = entry j and f = entry j-1.  Interior pair (s, N-s):
// z_j = y_{j+1/2} + P y_{j-1/2}, i.e. (y_s[j] + y_{N-s}[j-1], y_{N-s}[j] +
// y_s[j-1]); node pair: (node j, y_{N/2}[j] + y_{N/2}[j-1]) for even N,
// (node j, 0) for odd N.
template <typename T, int N>
__device__ __forceinline__ cx<T> fwd_in(bool interior, cx<T> e, cx<T> f) {
  // selects rather than branches: `interior` is uniform per task only
  const T re = e.x + (interior ? f.y : T(0));
  T im = e.y + (interior ? f.x : f.y);
  if constexpr (N % 2 == 1) im = interior ? im : T(0);
  return {re, im};
}

// Input of the inverse sine transforms of a pair (the imaginary part of the
// node pair carries no sequence for odd N).
template <typename T, int N>
__device__ __forceinline__ cx<T> inv_in(bool interior, cx<T> e) {
  if constexpr (N % 2 == 1) {
    if (!interior) return {e.x, T(0)};
  }
  return e;
}

// Sine-transform pre-processing of one pair at index j.
template <typename T>
__device__ __forceinline__ cx<T> dst_pre(cx<T> xj, cx<T> xkj, T snj, int j) {
  if (j == 0) return {T(0), T(0)};
  return {snj * (xj.x + xkj.x) + T(0.5) * (xj.x - xkj.x),
          snj * (xj.y + xkj.y) + T(0.5) * (xj.y - xkj.y)};
}

// The per-wave-number tables hold entries in 16-byte groups (see AxisTab):
// one load brings two FP64 or four FP32 entries.
template <typename T>
struct alignas(16) tgrp {
  T v[16 / sizeof(T)];
};

// Group 0 of wave number k's table; entry e is in group e / (16 / sizeof T).
template <int N, typename T>
__device__ __forceinline__ const tgrp<T>* blk_at(const tgrp<T>* blk, int k) {
  constexpr int GE = 16 / sizeof(T), NEG = (N * (N - 1) + N + GE - 1) / GE;
  return blk + (size_t)((k - 1) >> 6) * (NEG * 64) + ((k - 1) & 63);
}

template <typename T>
__device__ __forceinline__ T tab_e(const tgrp<T>* __restrict__ tb, int e) {
  constexpr int GE = 16 / sizeof(T);
  const tgrp<T> g = tb[(e / GE) * 64];
  return g.v[e % GE];
}

// The first NT entries of wave number k's table (all of them issued at once).
template <typename T, int NT>
__device__ __forceinline__ void load_tab(const tgrp<T>* __restrict__ tb, T (&tab)[NT]) {
#pragma unroll
  for (int e = 0; e < NT; ++e) tab[e] = tab_e(tb, e);
}

// Inverse-transform combination at k >= 1: y_0 = sum_l w_l,
// y_s = sum_l w_l p_k^(l)_s.
template <typename T, int N>
__device__ __forceinline__ void inv_apply(const T (&tab)[N * (N - 1) > 0 ? N * (N - 1) : 1],
                                          const T (&w)[N], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) y[i] = T(0);
#pragma unroll
  for (int l = 0; l < N; ++l) {
    y[0] += w[l];
#pragma unroll
    for (int i = 1; i < N; ++i) y[i] += w[l] * tab[l * (N - 1) + i - 1];
  }
}

// Direct-transform coefficients at wave number k >= 1 for NL lines,
// acc[u][l] = (x_0 + sum_s p_k^(l)_s x_s) / ||s_k^(l)||^2, and the fused
// form: division by the FP64 denominators dbase[u] + sc lam_k^(l), then the
// inverse combination y_0 = sum_l w_l, y_s = sum_l w_l p_k^(l)_s.  The row of
// eigenvector l (its N-1 entries, its norm and its eigenvalue) is read once
// per l and applied to every line.
template <typename T, int N, int NL>
__device__ __forceinline__ void fwd_lines(const tgrp<T>* __restrict__ tb, const T (&x)[NL][N],
                                          T (&acc)[NL][N]) {
#pragma unroll
  for (int l = 0; l < N; ++l) {
    T p[N > 1 ? N - 1 : 1];
#pragma unroll
    for (int i = 1; i < N; ++i) p[i - 1] = tab_e(tb, l * (N - 1) + i - 1);
    const T nrm = tab_e(tb, N * (N - 1) + l);
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      T s = x[u][0];
#pragma unroll
      for (int i = 1; i < N; ++i) s += p[i - 1] * x[u][i];
      acc[u][l] = s * nrm;
    }
  }
}

template <typename T, int N, int NL>
__device__ __forceinline__ void fused_lines(const tgrp<T>* __restrict__ tb, const double* __restrict__ lk,
                                            int lstride, const double (&dbase)[NL], double sc,
                                            const T (&x)[NL][N], T (&y)[NL][N]) {
#pragma unroll
  for (int u = 0; u < NL; ++u)
#pragma unroll
    for (int i = 0; i < N; ++i) y[u][i] = T(0);
#pragma unroll
  for (int l = 0; l < N; ++l) {
    T p[N > 1 ? N - 1 : 1];
#pragma unroll
    for (int i = 1; i < N; ++i) p[i - 1] = tab_e(tb, l * (N - 1) + i - 1);
    const T nrm = tab_e(tb, N * (N - 1) + l);
    const double lam = lk[(size_t)l * lstride];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      T s = x[u][0];
#pragma unroll
      for (int i = 1; i < N; ++i) s += p[i - 1] * x[u][i];
      s *= nrm;
      const T w = (T)((double)s / (dbase[u] + sc * lam));
      y[u][0] += w;
#pragma unroll
      for (int i = 1; i < N; ++i) y[u][i] += w * p[i - 1];
    }
  }
}

// log2 of the points per lane: 8 in FP64 for K <= 512 (fewer registers, so
// that more workgroups share a CU), 16 otherwise.
template <typename T, int LOG2K>
constexpr int log2_rmax() { return (sizeof(T) == 8 && LOG2K <= 9) ? 3 : 4; }

// Register budget: four waves per SIMD (two 512-lane workgroups per CU, up
// to 128 VGPRs), except in FP64 for K = 1024 and orders >= 7, whose
// per-wave-number tables alone take 2 n^2 registers (two waves).
constexpr int waves_per_simd_of(bool f64, int n, int log2K) {
  return f64 ? ((log2K <= 9 && n <= 6) ? 4 : 2) : 4;
}
// FP32 passes with inverse transforms of long lines of high order (two FFTs
// per slot pair, see task_dst_direct) spill at four waves: two waves per
// SIMD, one 512-lane workgroup per CU (FP32 large 2D solve 2.35 -> 1.97 ms).
template <typename T, int N, int LOG2K, int MODE>
constexpr int waves_per_simd() {
  return (sizeof(T) == 4 && MODE != PASS_FWD && LOG2K >= 6 && N >= 7)
             ? 2
             : waves_per_simd_of(sizeof(T) == 8, N, LOG2K);
}

// Lines per workgroup in the "tight" layout (at most).
constexpr int kTight = 2;

// Layout of a line of order n with K elements: padded when two or more fit
// in 64 KB (two or more workgroups per CU), tight (no padding, the per-line
// quantities in registers) otherwise.
constexpr bool tight_layout(int n, int K, int cplx_bytes) {
  return (64 * 1024) / (((n + 1) / 2 * K + 1) * cplx_bytes) < 2;
}

template <typename T, int N, int LOG2K, int MODE, typename TIN, typename TOUT>
__global__ __launch_bounds__(threads_for<T>())
__attribute__((amdgpu_waves_per_eu(waves_per_simd<T, N, LOG2K, MODE>()))) void line_pass(PassArgs a) {
  constexpr int LRM = log2_rmax<T, LOG2K>();
  using S = FftShape<LOG2K, LRM>;
  constexpr int K = S::K, R = S::R, G = S::G;
  constexpr int TPW = 64 / G;          // tasks per wavefront
  constexpr int NP = Seq<N>::NP;       // slot pairs per line
  constexpr int NE = N * (N - 1) + N;  // table entries per wave number
  constexpr int NPE = N * (N - 1) > 0 ? N * (N - 1) : 1;
  constexpr int M = N * K - 1;         // line length
  constexpr int KM = K - 1;
  constexpr bool tight = tight_layout(N, 1 << LOG2K, (int)sizeof(cx<T>));
  constexpr int kUnroll = unroll_for<T, N, LOG2K, tight>();
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int wave = tid >> 6, nwaves = nthr >> 6;
  const long long inner = a.inner;
  const int cb = a.cb;            // a power of two
  const int lcb = __builtin_ctz(cb);
  // Tight layout (lines too long for several per 64 KB): LDS holds the slots
  // and nothing else, the lines' addresses and denominators live in
  // registers.  Otherwise one pad entry per line (spreads the lines over the
  // LDS banks) and the per-line address and denominator after the slots.
  constexpr int NLB = kTight;   // lines per table read (tight)
  // S0 summed inside the transform tasks (tight FP64; FP32 has no registers
  // to spare for it)
  constexpr bool kS0In = tight && sizeof(T) == 8;
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
  long long* base = reinterpret_cast<long long*>(slots + (size_t)cb * lsp);   // [cb] (not tight)
  double* denb = reinterpret_cast<double*>(base + cb);                        // [cb] (not tight)
  T* e0a = reinterpret_cast<T*>(denb + cb);                                   // [cb][8] (not tight)
  auto lslots = [&](int c) -> cx<T>* { return slots + (size_t)c * lsp; };
  // Row-pair interleaved input / output (2D intermediate).  Along the rows:
  // the workgroup's two lines are one block, value q of line c at 2q + c.
  // Along the columns: value q of the line whose plain address is b moves
  // by ilv_shift.
  const bool pil_in = !cfast && a.ilv_in > 0 && cv == 2 && L0 + 1 < a.ilv_in;
  // one line of an interleaved pair: its values every other entry
  const bool sil_in = !cfast && a.ilv_in > 0 && cb == 1 && L0 < a.ilv_in;
  const bool pil_out = !cfast && a.ilv_out > 0 && cv == 2 && L0 + 1 < a.ilv_out;
  const long long MI = (long long)M * inner;
  // row L = o M + q of column t (plain address L inner + t) sits at
  // (L - (L & 1)) inner + 2t + (L & 1) when L < ilv
  auto ilv_shift = [&](long long ilv, long long orow, long long tcol, int q) -> long long {
    const long long L = orow + q;
    return L < ilv ? tcol - (L & 1) * (inner - 1) : 0;
  };

  const tgrp<T>* __restrict__ BLK = static_cast<const tgrp<T>*>(a.tab.blk);
  const T* __restrict__ EV = static_cast<const T*>(a.tab.E);
  const cx<T>* __restrict__ TW = static_cast<const cx<T>*>(a.tab.tw);
  const T* __restrict__ SN = static_cast<const T*>(a.tab.sn);
  const TIN* __restrict__ src = static_cast<const TIN*>(a.in);
  TOUT* __restrict__ dst = static_cast<TOUT*>(a.out);

  const int lane = tid & 63;
  const int j = lane & (G - 1);        // lane within the FFT task
  const int ntask = cv * NP;           // tasks: (line, slot pair)
  const int per_round = nwaves * TPW;

  auto line_den = [&](long long t) -> double {
    double d = a.alpha;
    for (int i = 0; i < a.nother; ++i) d += a.oscale[i] * a.olam[i][(t / a.odiv[i]) % a.omod[i]];
    return d;
  };
  // tight: every lane computes the lines' addresses and denominators, held
  // in scalar registers
  long long tbase[kTight];
  double tden[kTight];
  if constexpr (tight) {
#pragma unroll
    for (int u = 0; u < kTight; ++u) {
      const long long L = L0 + (u < cv ? u : 0);
      const long long o = L / inner, t = L - o * inner;
      tbase[u] = uni(o * (long long)M * inner + t);
      tden[u] = (MODE == PASS_FUSED) ? uni(line_den(t)) : 0.0;
    }
  } else if (tid < cv) {
    const long long L = L0 + tid;
    const long long o = L / inner, t = L - o * inner;
    base[tid] = o * (long long)M * inner + t;
    if (MODE == PASS_FUSED) denb[tid] = line_den(t);
  }
  auto lbase = [&](int c) -> long long {
    if (!tight) return base[c];
    long long b = tbase[0];
#pragma unroll
    for (int u = 1; u < kTight; ++u)
      if (c == u) b = tbase[u];
    return b;
  };
  auto lden = [&](int c) -> double {
    if (!tight) return denb[c];
    double d = tden[0];
#pragma unroll
    for (int u = 1; u < kTight; ++u)
      if (c == u) d = tden[u];
    return d;
  };
  // LDS entry of input value q of line c: physical order (node j at
  // q = N j - 1, interior point s of element e at q = N (e-1) + s - 1) or
  // coefficient order (inverse pass).
  auto in_entry = [&](int c, int q) -> T& {
    int s, i;
    if (MODE == PASS_INV || MODE == PASS_INV_ACC) {
      if (q < N - 1) {
        s = q;
        i = 0;
      } else {
        const int r = q - (N - 1);
        s = r / KM;
        i = r - s * KM + 1;
      }
    } else {
      const int g = q + 1;
      s = g % N;
      i = g / N;
    }
    return at<T, N, K>(lslots(c), s, i);
  };

  // ---- load the cv lines into their sequences ------------------------------
  // Contiguous axis: the cv lines are one contiguous range, swept by all
  // lanes.  Strided axis: lane (q, c) with c = tid mod cb, so adjacent lanes
  // read adjacent lines (adjacent in memory).  kUnroll loads in flight per
  // lane: one round for the longest lines.
  if (sil_in) {
    const TIN* sp = src + (L0 & ~1LL) * M + (L0 & 1);
    for (int q0 = tid; q0 < M; q0 += kUnroll * nthr) {
      TIN r[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int q = q0 + u * nthr < M ? q0 + u * nthr : 0;
        r[u] = sp[2 * q];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int q = q0 + u * nthr;
        if (q < M) in_entry(0, q) = (T)r[u];
      }
    }
    __syncthreads();
  } else if (!cfast) {
    // 16-byte loads from the first 16-byte boundary on; the elements before
    // it and the last few one by one
    const TIN* sp = src + L0 * M;
    const int total = cv * M;
    constexpr int VL = 16 / sizeof(TIN);
    constexpr int kUV = (kUnroll + VL - 1) / VL;
    const int h = min(head16(sp), total);
    const int nv = (total - h) / VL;
    const int tail0 = h + nv * VL;
    auto put = [&](int i, TIN v) {
      int c, q;
      if (pil_in) {
        c = i & 1;
        q = i >> 1;
      } else {
        c = i / M;
        q = i - c * M;
      }
      in_entry(c, q) = (T)v;
    };
    if (tid < h) put(tid, sp[tid]);
    if (tid < total - tail0) put(tail0 + tid, sp[tail0 + tid]);
    const vec16<TIN>* vp = reinterpret_cast<const vec16<TIN>*>(sp + h);
    for (int j00 = tid; j00 < nv; j00 += kUV * nthr) {
      vec16<TIN> r[kUV];
#pragma unroll
      for (int u = 0; u < kUV; ++u) {
        const int j = j00 + u * nthr;
        r[u] = vp[j < nv ? j : 0];
      }
#pragma unroll
      for (int u = 0; u < kUV; ++u) {
        const int j = j00 + u * nthr;
        if (j < nv) {
#pragma unroll
          for (int e = 0; e < VL; ++e) put(h + VL * j + e, r[u].v[e]);
        }
      }
    }
    __syncthreads();
  } else {
    __syncthreads();   // base[]
    const int c = tid & (cb - 1);
    const int qs = nthr >> lcb;
    if (c < cv) {
      const long long b = lbase(c);
      const TIN* sp = src + b;
      const long long ilv = a.ilv_in;
      long long orow = 0, tcol = 0;
      if (ilv > 0) {
        const long long o = b / MI;
        orow = o * M;
        tcol = b - o * MI;
      }
      // Row pairs of the interleaved input: one load brings both rows of the
      // column (16 bytes in FP64).  Pairs start at even grid rows; the rows
      // outside whole pairs (at most one at each end) go one by one.
      const bool pairs = ilv > 0 && ((reinterpret_cast<unsigned long long>(src) & (2 * sizeof(TIN) - 1)) == 0);
      const int qa = pairs ? (int)(orow & 1) : M;                     // first paired row
      const long long lim = min((long long)M, ilv - orow);             // rows below ilv
      const int npair = pairs && lim > qa ? (int)((lim - qa) / 2) : 0;
      const int qb = qa + 2 * npair;                                   // first row after them
      if (pairs) {
        const pair2<TIN>* pp = reinterpret_cast<const pair2<TIN>*>(src + (orow + qa) * inner + 2 * tcol);
        constexpr int KP = (kUnroll + 1) / 2;
        for (int p0 = tid >> lcb; p0 < npair; p0 += KP * qs) {
          pair2<TIN> r[KP];
#pragma unroll
          for (int u = 0; u < KP; ++u) {
            const int pi = p0 + u * qs < npair ? p0 + u * qs : 0;
            r[u] = pp[(long long)pi * inner];                          // rows 2 pi, 2 pi + 1 past qa
          }
#pragma unroll
          for (int u = 0; u < KP; ++u) {
            const int pi = p0 + u * qs;
            if (pi < npair) {
              in_entry(c, qa + 2 * pi) = (T)r[u].a;
              in_entry(c, qa + 2 * pi + 1) = (T)r[u].b;
            }
          }
        }
        // the rows before the first pair and after the last
        const int lt = tid >> lcb;
        const int q = lt < qa ? lt : qb + (lt - qa);
        if (lt < qa + (M - qb) && q < M) in_entry(c, q) = (T)sp[(long long)q * inner + ilv_shift(ilv, orow, tcol, q)];
      } else {
        for (int q0 = tid >> lcb; q0 < M; q0 += kUnroll * qs) {
          TIN r[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const int q = q0 + u * qs < M ? q0 + u * qs : 0;
            r[u] = sp[(long long)q * inner + ilv_shift(ilv, orow, tcol, q)];
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const int q = q0 + u * qs;
            if (q < M) in_entry(c, q) = (T)r[u];
          }
        }
      }
    }
    __syncthreads();
  }

  // E0 of the lines, from the k = 0 quantities at entry 0 of the sequences
  // (S0 in the fused pass, the coefficients w_{0l} in the inverse pass);
  // entry 0 is scratch space of the inverse transforms, so E0 waits in
  // scalar registers (tight) or in e0a (padded layout) until the scatter.
  T e0s[kTight][N > 1 ? N - 1 : 1];
  auto line_e0 = [&](int c, T (&e0)[N > 1 ? N - 1 : 1]) {
    if constexpr (N > 1) {
      cx<T>* ls = lslots(c);
      T w0[N - 1];
      if (MODE == PASS_FUSED) {
        // w_{0l} = S0 . e^(l) / K divided by its denominator
        T s0l[N - 1];
#pragma unroll
        for (int s = 0; s < N - 1; ++s) s0l[s] = at<T, N, K>(ls, s + 1, 0);
#pragma unroll
        for (int l = 0; l < N - 1; ++l) {
          T acc = T(0);
#pragma unroll
          for (int s = 0; s < N - 1; ++s) acc += EV[s * (N - 1) + l] * s0l[s];
          acc /= (T)K;
          const double den = lden(c) + a.scale * a.tab.lam[l];
          w0[l] = (T)((double)acc / den);
        }
      } else {
#pragma unroll
        for (int l = 0; l < N - 1; ++l) w0[l] = at<T, N, K>(ls, l, 0);
      }
#pragma unroll
      for (int s = 0; s < N - 1; ++s) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < N - 1; ++l) acc += EV[s * (N - 1) + l] * w0[l];
        e0[s] = acc;
      }
    }
  };
  auto keep_e0 = [&]() {
    if constexpr (N > 1) {
      if constexpr (tight) {
#pragma unroll
        for (int u = 0; u < kTight; ++u) {
          T e[N - 1];
          line_e0(u < cv ? u : 0, e);
#pragma unroll
          for (int s = 0; s < N - 1; ++s) e0s[u][s] = uni(e[s]);
        }
      } else if (tid < cv) {
        T e[N - 1];
        line_e0(tid, e);
#pragma unroll
        for (int s = 0; s < N - 1; ++s) e0a[tid * 8 + s] = e[s];
      }
    }
  };

  if (MODE == PASS_FWD || MODE == PASS_FUSED) {
    // ---- S0_s = sum_{e=1..K} ((-P)^(e-1) y_{e-1/2})_s ----------------------
    // = sum_e (-1)^(e-1) y_{e-1/2, s (e odd) or N-s (e even)}: one wave per
    // (line, component), read from the loaded entries before the transforms
    // overwrite them.  The sums wait in scalar registers (tight layout, at
    // most two per wave) or in e0a until the transforms have freed entry 0.
    T s0r[2] = {T(0), T(0)};
    auto s0_sums = [&]() {
      if constexpr (N > 1) {
        int r = 0;
        for (int w0 = wave; w0 < cv * (N - 1); w0 += nwaves, ++r) {
          const int c = w0 / (N - 1), s = w0 - c * (N - 1) + 1;
          cx<T>* ls = lslots(c);
          T acc = T(0);
#pragma unroll
          for (int e = 1 + lane; e <= K; e += 64) {
            const T val = at<T, N, K>(ls, (e & 1) ? s : N - s, e - 1);
            acc += (e & 1) ? val : -val;
          }
          acc = uni(wave_sum(acc));
          if constexpr (tight) {
            if (r == 0) s0r[0] = acc; else s0r[1] = acc;
          } else if (lane == 0) {
            e0a[c * 8 + s - 1] = acc;
          }
        }
      }
    };
    // Direct sine transforms, one task per (line, pair): a task reads its
    // pair into registers (forward pre-combine and sine pre-processing) and
    // transforms it in place.
    // (with S0IN, also the lane's terms of the pair's S0 sums: entry jj is
    // element jj + 1, sign (-1)^jj; the node pair of an even order carries
    // the middle component, its own mirror, in .y)
    auto fwd_read = [&](cx<T>* tb, bool interior, int j, cx<T> (&v)[R], T& sa, T& sb) {
      T snr[R];   // DST pre-weights sin(pi jj / K) of this lane's task points
      task_sines<T, K, R>(SN, j, snr);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int jj = j + G * t;
        const cx<T> e0 = tb[sw(jj)], e1 = tb[sw((jj - 1) & (K - 1))];
        const cx<T> m0 = tb[sw((K - jj) & (K - 1))], m1 = tb[sw((K - jj - 1) & (K - 1))];
        v[t] = dst_pre(fwd_in<T, N>(interior, e0, e1), fwd_in<T, N>(interior, m0, m1), snr[t], jj);
        if constexpr (kS0In) {
          const bool even = !(jj & 1);
          sa += interior ? (even ? e0.x : -e0.y) : T(0);
          sb += interior ? (even ? e0.y : -e0.x) : (N % 2 == 0 ? (even ? e0.y : -e0.y) : T(0));
        }
      }
    };
    if constexpr (tight) {
      // tasks in rounds: the sums first (FP32) or inside the tasks (FP64)
      if constexpr (!kS0In) {
        s0_sums();
        if constexpr (N > 1) __syncthreads();
      }
      for (int t0 = 0; t0 < ntask; t0 += per_round) {
        const int task = t0 + wave * TPW + lane / G;
        if (task < ntask) {
          const int tc = task / NP, tp = task - tc * NP;
          const bool interior = tp < NP - 1;
          cx<T>* tb = lslots(tc) + (size_t)tp * K;
          int j = lane & (G - 1);
          asm volatile("" : "+v"(j));   // keeps the lane's address arithmetic inside the loop
          cx<T> v[R];
          T sa = T(0), sb = T(0);
          fwd_read(tb, interior, j, v, sa, sb);
          wave_sync();
          task_fft<T, LOG2K, LRM>(v, tb, j, TW);
          task_post<T, LOG2K, LRM>(tb, j);
          if constexpr (kS0In && N > 1) {
            // the pair's S0 into its entry 0, free after the transform
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
              sa += __shfl_xor(sa, off, 64);
              sb += __shfl_xor(sb, off, 64);
            }
            if (j == 0) {
              if (interior) tb[sw(0)] = cx<T>{sa, sb};
              else if (N % 2 == 0) tb[sw(0)].y = sb;
            }
          }
        }
      }
    } else {
      // one round (the launch shape guarantees it): every task reads its
      // pair, the sums overlap those reads, then the transforms
      const int task = wave * TPW + lane / G;
      const int tc = task / NP, tp = task - tc * NP;
      cx<T>* tb = lslots(task < ntask ? tc : 0) + (size_t)tp * K;
      const int j = lane & (G - 1);
      cx<T> v[R];
      T sa = T(0), sb = T(0);
      if (task < ntask) fwd_read(tb, tp < NP - 1, j, v, sa, sb);
      s0_sums();
      __syncthreads();
      if (task < ntask) {
        task_fft<T, LOG2K, LRM>(v, tb, j, TW);
        task_post<T, LOG2K, LRM>(tb, j);
      }
    }
    __syncthreads();
    // S0 into entry 0 of its component (unless the tasks wrote it)
    if constexpr (N > 1 && !kS0In) {
      if constexpr (tight) {
        if (lane == 0) {
          int r = 0;
          for (int w0 = wave; w0 < cv * (N - 1); w0 += nwaves, ++r) {
            const int c = w0 / (N - 1), s = w0 - c * (N - 1) + 1;
            at<T, N, K>(lslots(c), s, 0) = r == 0 ? s0r[0] : s0r[1];
          }
        }
      } else {
        for (int i = tid; i < cv * (N - 1); i += nthr) {
          const int c = i / (N - 1), s = i - c * (N - 1) + 1;
          at<T, N, K>(lslots(c), s, 0) = e0a[c * 8 + s - 1];
        }
      }
      __syncthreads();
    }

    if (MODE == PASS_FWD) {
      // ---- forward block, coefficients to global -------------------------
      // output base and step of line c (row-pair interleaved: the pair's
      // block, step 2)
      const long long ostep = pil_out ? 2 : inner;
      auto obase = [&](int c) -> long long { return pil_out ? lbase(0) + c : lbase(c); };
      // interleaved pair: the two values of a coefficient are adjacent, one
      // store (when the output is aligned for it)
      static_assert(kTight == 2 && NLB == 2, "pair stores take two lines");
      const bool pst = pil_out && ((reinterpret_cast<unsigned long long>(dst) & (2 * sizeof(TOUT) - 1)) == 0);
      if (tight || pil_out) {
        // one wave number per lane; its table entries are read once for
        // all the lines
        for (int k = 1 + tid; k < K; k += nthr) {
#pragma unroll
          for (int u0 = 0; u0 < kTight; u0 += NLB) {
            if (u0 < cv) {
              T x[NLB][N], acc[NLB][N];
#pragma unroll
              for (int u = 0; u < NLB; ++u)
#pragma unroll
                for (int s = 0; s < N; ++s) x[u][s] = at<T, N, K>(lslots(u0 + u < cv ? u0 + u : 0), s, k);
              fwd_lines<T, N, NLB>(blk_at<N>(BLK, k), x, acc);
              if (pst) {
                const long long ob = lbase(0) + 2 * ((long long)(N - 1) + (k - 1));
#pragma unroll
                for (int l = 0; l < N; ++l) {
                  pair2<TOUT> v;
                  v.a = (TOUT)acc[0][l];
                  v.b = (TOUT)acc[1][l];
                  *reinterpret_cast<pair2<TOUT>*>(dst + ob + 2LL * l * KM) = v;
                }
              } else {
#pragma unroll
                for (int u = 0; u < NLB; ++u) {
                  if (u0 + u < cv) {
                    const long long ob = obase(u0 + u) + ((long long)(N - 1) + (k - 1)) * ostep;
#pragma unroll
                    for (int l = 0; l < N; ++l) dst[ob + (long long)l * KM * ostep] = (TOUT)acc[u][l];
                  }
                }
              }
            }
          }
        }
      } else {
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
          T x[1][N], acc[1][N];
#pragma unroll
          for (int s = 0; s < N; ++s) x[0][s] = at<T, N, K>(lslots(c), s, k);
          fwd_lines<T, N, 1>(blk_at<N>(BLK, k), x, acc);
          const long long ob = obase(c) + ((long long)(N - 1) + (k - 1)) * ostep;
#pragma unroll
          for (int l = 0; l < N; ++l) dst[ob + (long long)l * KM * ostep] = (TOUT)acc[0][l];
        }
      }
      // k = 0: w_{0l} = S0 . e^(l) / K
      if constexpr (N > 1) {
        const int items0 = cv * (N - 1);
        for (int i = tid; i < items0; i += nthr) {
          const int c = i / (N - 1), l = i - c * (N - 1);
          T acc = T(0);
#pragma unroll
          for (int s = 0; s < N - 1; ++s) acc += EV[s * (N - 1) + l] * at<T, N, K>(lslots(c), s + 1, 0);
          dst[obase(c) + (long long)l * ostep] = (TOUT)(acc / (T)K);
        }
      }
      return;
    }

    // ---- fused: forward block, spectral division, inverse block ----------
    {
      const double sc = a.scale;
      const double* __restrict__ lam = a.tab.lam;
      if constexpr (tight) {
        for (int k = 1 + tid; k < K; k += nthr) {
#pragma unroll
          for (int u0 = 0; u0 < kTight; u0 += NLB) {
            if (u0 < cv) {
              T x[NLB][N], y[NLB][N];
              double dn[NLB];
#pragma unroll
              for (int u = 0; u < NLB; ++u) {
                dn[u] = tden[u0 + u];
#pragma unroll
                for (int s = 0; s < N; ++s) x[u][s] = at<T, N, K>(lslots(u0 + u < cv ? u0 + u : 0), s, k);
              }
              fused_lines<T, N, NLB>(blk_at<N>(BLK, k), lam + (N - 1) + (k - 1), KM, dn, sc, x, y);
#pragma unroll
              for (int u = 0; u < NLB; ++u) {
                if (u0 + u < cv) {
#pragma unroll
                  for (int s = 0; s < N; ++s) at<T, N, K>(lslots(u0 + u), s, k) = y[u][s];
                }
              }
            }
          }
        }
      } else {
        const int items = cv * KM;
        for (int i = tid; i < items; i += nthr) {
          const int c = i / KM, k = i - c * KM + 1;
          cx<T>* ls = lslots(c);
          T x[1][N], y[1][N];
          const double dn[1] = {denb[c]};
#pragma unroll
          for (int s = 0; s < N; ++s) x[0][s] = at<T, N, K>(ls, s, k);
          fused_lines<T, N, 1>(blk_at<N>(BLK, k), lam + (N - 1) + (k - 1), KM, dn, sc, x, y);
#pragma unroll
          for (int s = 0; s < N; ++s) at<T, N, K>(ls, s, k) = y[0][s];
        }
      }
      keep_e0();
      __syncthreads();
    }
  } else {
    // ---- inverse: block in place on the coefficients ---------------------
    // (coefficient (l, k) is entry k of sequence l-1; the block at k turns
    // them into the entries k of the N sequences)
    if constexpr (tight) {
      for (int k = 1 + tid; k < K; k += nthr) {
        T tab[NPE];
        load_tab<T, NPE>(blk_at<N>(BLK, k), tab);
#pragma unroll
        for (int u = 0; u < kTight; ++u) {
          if (u < cv) {
            cx<T>* ls = lslots(u);
            T w[N], y[N];
#pragma unroll
            for (int l = 0; l < N; ++l) w[l] = at<T, N, K>(ls, l, k);
            inv_apply<T, N>(tab, w, y);
#pragma unroll
            for (int s = 0; s < N; ++s) at<T, N, K>(ls, s, k) = y[s];
          }
        }
      }
    } else {
      const int items = cv * KM;
      for (int i = tid; i < items; i += nthr) {
        const int c = i / KM, k = i - c * KM + 1;
        cx<T>* ls = lslots(c);
        T tab[NPE], w[N], y[N];
        load_tab<T, NPE>(blk_at<N>(BLK, k), tab);
#pragma unroll
        for (int l = 0; l < N; ++l) w[l] = at<T, N, K>(ls, l, k);
        inv_apply<T, N>(tab, w, y);
#pragma unroll
        for (int s = 0; s < N; ++s) at<T, N, K>(ls, s, k) = y[s];
      }
    }
    keep_e0();   // coefficient (l, 0) is entry 0 of sequence l-1
    __syncthreads();
  }

  // ---- inverse sine transforms, one task per (line, pair) ------------------
  auto inv_task = [&](int task, int j) {
    const int tc = task / NP, tp = task - tc * NP;
    const bool interior = tp < NP - 1;
    cx<T>* tb = lslots(tc) + (size_t)tp * K;
    T snr[R];
    task_sines<T, K, R>(SN, j, snr);
    cx<T> v[R];
    if constexpr (sizeof(T) == 4) {
      // FP32: both FFTs, no running sums (see task_dst_direct)
      T csr[R];
      task_cosines<T, K, R>(SN, j, csr);
      cx<T> v2[R];
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int jj = j + G * t;
        const cx<T> x0 = inv_in<T, N>(interior, tb[sw(jj)]);
        const cx<T> x1 = inv_in<T, N>(interior, tb[sw((K - jj) & (K - 1))]);
        v[t] = dst_pre(x0, x1, snr[t], jj);
        v2[t] = jj == 0 ? cx<T>{T(0), T(0)} : cx<T>{csr[t] * (x0.x + x1.x), csr[t] * (x0.y + x1.y)};
      }
      wave_sync();
      task_dst_direct<T, LOG2K, LRM>(v, v2, tb, j, TW);
    } else {
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int jj = j + G * t;
        v[t] = dst_pre(inv_in<T, N>(interior, tb[sw(jj)]),
                       inv_in<T, N>(interior, tb[sw((K - jj) & (K - 1))]), snr[t], jj);
      }
      wave_sync();
      task_fft<T, LOG2K, LRM>(v, tb, j, TW);
      task_post<T, LOG2K, LRM>(tb, j);
    }
  };
  if constexpr (tight) {
    for (int t0 = 0; t0 < ntask; t0 += per_round) {
      const int task = t0 + wave * TPW + lane / G;
      if (task < ntask) {
        int j = lane & (G - 1);
        asm volatile("" : "+v"(j));   // keeps the lane's address arithmetic inside the loop
        inv_task(task, j);
      }
    }
  } else {
    const int task = wave * TPW + lane / G;   // one round (launch shape)
    if (task < ntask) inv_task(task, lane & (G - 1));
  }
  __syncthreads();
  if constexpr (N > 1) {
    if (tid < cv) {
      cx<T>* ls = lslots(tid);
      if constexpr (tight) {
#pragma unroll
        for (int u = 0; u < kTight; ++u)
          if (tid == u) {
#pragma unroll
            for (int s = 1; s < N; ++s) at<T, N, K>(ls, s, 0) = e0s[u][s - 1];
          }
      } else {
#pragma unroll
        for (int s = 1; s < N; ++s) at<T, N, K>(ls, s, 0) = e0a[tid * 8 + s - 1];
      }
    }
    __syncthreads();
  }
  {
    // value at position g = q + 1 = N jn + s of line c (s = 0: mesh node):
    // node jn, or Z_s[e-1] + Z_{N-s}[e] + (-P)^(e-1) E0 for element e = jn + 1
    // (branch free: every read is in range and the unused terms are masked)
    auto value = [&](int c, int q) -> T {
      cx<T>* ls = lslots(c);
      const int g = q + 1, jn = g / N, s = g - jn * N;
      const bool inter = s != 0;
      const int je = jn + 1;
      const int s2 = inter ? N - s : 0;
      const T z1 = at<T, N, K>(ls, s, jn);                      // node jn, or Z_s[e-1]
      const T z2 = at<T, N, K>(ls, s2, je < K ? je : K - 1);    // Z_{N-s}[e]
      const T ee = at<T, N, K>(ls, (je & 1) ? s : s2, 0);        // E0_s or E0_{N-s}
      T v = jn >= 1 ? z1 : T(0);
      v += (inter && je <= K - 1) ? z2 : T(0);
      v += inter ? ((je & 1) ? ee : -ee) : T(0);
      return v;
    };
    constexpr int SU = 8;   // values gathered before their stores are issued
    // the inverse pass that adds its result to the output (refinement)
    constexpr bool kAcc = MODE == PASS_INV_ACC;
    auto store = [&](TOUT& o, T v) {
      if constexpr (kAcc) o += (TOUT)v; else o = (TOUT)v;
    };
    if (!cfast) {
      // 16-byte stores from the first 16-byte boundary on
      TOUT* d = dst + L0 * M;
      const int total = cv * M;
      constexpr int VS = 16 / sizeof(TOUT);
      constexpr int SUV = SU / VS > 0 ? SU / VS : 1;
      const int h = min(head16(d), total);
      const int nv = (total - h) / VS;
      const int tail0 = h + nv * VS;
      auto val_at = [&](int i) -> T {
        const int c = i / M, q = i - c * M;
        return value(c, q);
      };
      if (tid < h) store(d[tid], val_at(tid));
      if (tid < total - tail0) store(d[tail0 + tid], val_at(tail0 + tid));
      vec16<TOUT>* vd = reinterpret_cast<vec16<TOUT>*>(d + h);
      for (int j0 = tid; j0 < nv; j0 += SUV * nthr) {
        vec16<TOUT> val[SUV];
#pragma unroll
        for (int u = 0; u < SUV; ++u) {
          const int j = min(j0 + u * nthr, nv - 1);
#pragma unroll
          for (int e = 0; e < VS; ++e) val[u].v[e] = (TOUT)val_at(h + VS * j + e);
        }
#pragma unroll
        for (int u = 0; u < SUV; ++u) {
          const int j = j0 + u * nthr;
          if (j < nv) {
            if constexpr (kAcc) {
              vec16<TOUT> o = vd[j];
#pragma unroll
              for (int e = 0; e < VS; ++e) o.v[e] += val[u].v[e];
              vd[j] = o;
            } else {
              vd[j] = val[u];
            }
          }
        }
      }
    } else {
      const int c = tid & (cb - 1);
      const int qs = nthr >> lcb;
      if (c < cv) {
        const long long b = lbase(c);
        TOUT* d = dst + b;
        const long long ilv = a.ilv_out;
        long long orow = 0, tcol = 0;
        if (ilv > 0) {
          const long long o = b / MI;
          orow = o * M;
          tcol = b - o * MI;
        }
        // row pairs of the interleaved output: one store for both rows of
        // the column (as the column loads)
        const bool pairs = ilv > 0 && ((reinterpret_cast<unsigned long long>(dst) & (2 * sizeof(TOUT) - 1)) == 0);
        if (pairs) {
          const int qa = (int)(orow & 1);
          const long long lim = min((long long)M, ilv - orow);
          const int npair = lim > qa ? (int)((lim - qa) / 2) : 0;
          const int qb = qa + 2 * npair;
          pair2<TOUT>* pp = reinterpret_cast<pair2<TOUT>*>(dst + (orow + qa) * inner + 2 * tcol);
          constexpr int SUP = SU / 2;
          for (int p0 = tid >> lcb; p0 < npair; p0 += SUP * qs) {
            pair2<TOUT> v[SUP];
#pragma unroll
            for (int u = 0; u < SUP; ++u) {
              const int pi = min(p0 + u * qs, npair - 1);
              v[u].a = (TOUT)value(c, qa + 2 * pi);
              v[u].b = (TOUT)value(c, qa + 2 * pi + 1);
            }
#pragma unroll
            for (int u = 0; u < SUP; ++u) {
              const int pi = p0 + u * qs;
              if (pi < npair) {
                if constexpr (kAcc) {
                  pair2<TOUT> o = pp[(long long)pi * inner];
                  o.a += v[u].a;
                  o.b += v[u].b;
                  pp[(long long)pi * inner] = o;
                } else {
                  pp[(long long)pi * inner] = v[u];
                }
              }
            }
          }
          const int lt = tid >> lcb;
          const int q = lt < qa ? lt : qb + (lt - qa);
          if (lt < qa + (M - qb) && q < M) store(d[(long long)q * inner + ilv_shift(ilv, orow, tcol, q)], value(c, q));
        } else {
          for (int q0 = tid >> lcb; q0 < M; q0 += SU * qs) {
            T val[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) val[u] = value(c, min(q0 + u * qs, M - 1));
#pragma unroll
            for (int u = 0; u < SU; ++u) {
              const int q = q0 + u * qs;
              if (q < M) store(d[(long long)q * inner + ilv_shift(ilv, orow, tcol, q)], val[u]);
            }
          }
        }
      }
    }
  }
}

struct Shape {
  int cb, threads, tight;
  size_t lds;
};

// Lines per workgroup and LDS bytes.  Lines that fit two or more to 64 KB use
// the padded layout (80 KB per workgroup in FP64, 64 KB in FP32); longer lines use the
// tight one with as many lines (at most kTight) as the CU's LDS share of one
// workgroup holds: 160 KB divided by the workgroups per CU that the register
// budget allows.  one_line: the inverse pass along the rows in FP64, whose
// long lines then go one per 256-lane workgroup (two per CU, their phases
// overlapping).
inline Shape shape_for(int n, int K, size_t cplx_bytes, long long nlines, bool one_line = false) {
  const int NP = (n + 1) / 2;
  const bool f64 = cplx_bytes == 16;
  const int rmax = (f64 && K <= 512) ? 8 : 16;   // as log2_rmax
  const int R = K < rmax ? K : rmax;
  const int G = K / R;
  const int TPW = 64 / G;
  int threads = f64 ? threads_for<double>() : threads_for<float>();
  if (f64 && one_line && tight_layout(n, K, (int)cplx_bytes)) threads = 256;
  const size_t per_line = ((size_t)NP * K + 1) * cplx_bytes;
  Shape s;
  s.threads = threads;
  // padded layout: up to 80 KB per workgroup in FP64 (two workgroups fill
  // the CU's LDS; strided rows of n = 4, K = 128 lines then span whole cache
  // lines), 64 KB in FP32
  long long c = f64 ? (long long)((80 * 1024 - 64) / (per_line + 16 + 8 * (long long)(cplx_bytes / 2)))
                    : (long long)((64 * 1024) / per_line);
  if (!tight_layout(n, K, (int)cplx_bytes)) {
    // every FFT task of the workgroup in one round
    c = std::min<long long>(c, (long long)(threads / 64) * TPW / NP);
    c = std::min<long long>(c, kMaxCB);
    c = std::min<long long>(c, nlines);
    if (c < 1) c = 1;
    while (c & (c - 1)) c &= c - 1;   // round down to a power of two
    s.cb = (int)c;
    s.tight = 0;
    s.lds = (size_t)c * per_line + (size_t)c * 16 + (size_t)c * 8 * (cplx_bytes / 2);
    return s;
  }
  int log2K = 0;
  while ((1 << log2K) < K) ++log2K;
  const int wgs = std::max(1, waves_per_simd_of(f64, n, log2K) * 4 / (threads / 64));
  const size_t budget = (size_t)(160 * 1024) / wgs;
  const size_t tl = (size_t)NP * K * cplx_bytes;
  c = 1;
  while (c * 2 <= kTight && (size_t)(c * 2) * tl <= budget && c * 2 <= nlines) c *= 2;
  s.cb = (int)c;
  s.tight = 1;
  s.lds = (size_t)c * tl;
  return s;
}

// A requested shape (cb lines per workgroup of `threads` lanes): the
// layout is fixed by (n, K); the padded layout runs every transform task in
// one round, so cb pairs of tasks must fit the workgroup's waves; the tight
// layout holds at most kTight lines.  False when the kernel cannot run it.
inline bool shape_request(int n, int K, size_t cplx_bytes, long long nlines, int cb, int threads,
                          Shape* out) {
  if (threads != 256 && threads != 512) return false;
  if (cb < 1 || (cb & (cb - 1)) || cb > kMaxCB) return false;
  const int NP = (n + 1) / 2;
  const bool f64 = cplx_bytes == 16;
  const int rmax = (f64 && K <= 512) ? 8 : 16;
  const int R = K < rmax ? K : rmax;
  const int TPW = 64 / (K / R);
  Shape s;
  s.threads = threads;
  s.cb = cb;
  if (tight_layout(n, K, (int)cplx_bytes)) {
    if (cb > kTight) return false;
    // FP32 tight passes sum S0 in a separate phase, one wave per (line,
    // component), each wave keeping at most two sums
    if (!f64 && n > 1 && cb * (n - 1) > 2 * (threads / 64)) return false;
    s.tight = 1;
    s.lds = (size_t)cb * NP * K * cplx_bytes;
  } else {
    if (cb * NP > (threads / 64) * TPW) return false;
    s.tight = 0;
    const size_t per_line = ((size_t)NP * K + 1) * cplx_bytes;
    s.lds = (size_t)cb * per_line + (size_t)cb * 16 + (size_t)cb * 8 * (cplx_bytes / 2);
  }
  if (s.lds > 160 * 1024) return false;
  if ((long long)cb > 2 * nlines && cb > 1) return false;   // mostly idle workgroups
  *out = s;
  return true;
}

template <typename T, int N, int LOG2K, int MODE, typename TIN, typename TOUT>
hipError_t launch_k(const PassArgs& a0, hipStream_t s) {
  constexpr bool kInv = MODE == PASS_INV || MODE == PASS_INV_ACC;
  Shape sh = shape_for(N, 1 << LOG2K, sizeof(cx<T>), a0.nlines,
                       kInv && sizeof(T) == 8 && a0.inner == 1);
  if (a0.cb_req > 0 || a0.threads_req > 0) {
    if (!shape_request(N, 1 << LOG2K, sizeof(cx<T>), a0.nlines, a0.cb_req > 0 ? a0.cb_req : sh.cb,
                       a0.threads_req > 0 ? a0.threads_req : sh.threads, &sh))
      return hipErrorInvalidValue;
  }
  if (a0.tab.n != N || a0.tab.K != (1 << LOG2K)) return hipErrorInvalidValue;
  if (a0.ilv_in > 0 || a0.ilv_out > 0) {
    // the row-pair interleaved forms this kernel implements
    const bool rows = a0.inner == 1;
    if (rows && sh.cb != 2 && !(sh.cb == 1 && a0.ilv_out == 0)) return hipErrorInvalidValue;
    if (a0.ilv_out > 0 && (rows ? MODE != PASS_FWD : MODE == PASS_FWD)) return hipErrorInvalidValue;
    if ((a0.ilv_in | a0.ilv_out) & 1) return hipErrorInvalidValue;
  }
  PassArgs a = a0;
  a.cb = sh.cb;
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
    case PASS_INV_ACC:
      if (dt == 4) return launch_by_k<float, N, PASS_INV_ACC, float, double>(a, s);
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
