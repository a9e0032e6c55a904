// Line passes along Neumann axes (FP64).  A line holds the m = nK + 1 values
// of the axis, boundary nodes included: node j at q = n j (j = 0..K),
// interior point s of element e at q = n (e-1) + s.
//
// Eigenvectors (derivation in the plan builder): for k = 1..K-1 the cosine
// counterparts of Theorem 1's, node j: cos(pi k j / K), point s of element
// e: cos(pi k (e-1)/K) p_s + cos(pi k e/K) p_{n-s}, with the eigenvalue,
// p_k^(l) and norm of the Dirichlet wave number k; the other n + 1 are the
// band-edge cells (a, w) repeated along the axis with the factor +1
// (theta = 0) or (-1)^j (theta = pi), even under the reflection about a
// node: w_s = w_{n-s} at theta = 0, w_s = -w_{n-s} at theta = pi, normalised
// so that ||v||_C^2 = K.  With the DCT-I X_k = sum_{j=0}^{K} x_j cos(pi k j/K):
//   direct:  z^s_j = y_{j+1,s} + y_{j,n-s} (j = 0..K, missing elements count
//            zero), T0 = DCT-I(nodes), Z^s = DCT-I(z^s),
//            c_{k,l} = (T0_k + p_k^(l) . Z_k) / ||s_k^(l)||^2       (k = 1..K-1),
//            c_b = (a_b T0_k + 1/2 sum_s w_{b,s} Z^s_k) / K          (k = 0, K)
//   inverse: W_k = sum_l c_{kl}, d^s_k = sum_l c_{kl} p^(l)_{k,s}    (k = 1..K-1),
//            W_k = sum_b c_b a_b, d^s_k = 1/2 sum_b c_b w_{b,s}      (k = 0, K),
//            nodes = DCT-I(W), u_{e,s} = D^s_{e-1} + D^{n-s}_e with D^s = DCT-I(d^s).
// By the symmetries of w the band-edge blocks need only Z^s_0 + Z^{n-s}_0
// and Z^s_K - Z^{n-s}_K of a mirror pair, and give d^s_0 = d^{n-s}_0,
// d^s_K = -d^{n-s}_K.
//
// DCT-I of K+1 points by one K-point complex FFT for two real sequences
// (the cosine counterpart of the half-length sine method of the Dirichlet
// passes): y_j = (x_j + x_{K-j})/2 - sin(pi j/K)(x_j - x_{K-j}), j = 0..K-1,
// Y = FFT(y): X_{2k} = Re Y_k + (x_0 + x_K)/2 (k = 0..K/2) and the running
// sums X_{2k+1} = X_{2k-1} - Im Y_k from X_1 = sum_j x_j cos(pi j/K), which
// is formed from the inputs (the sums are FP64 like the Dirichlet FP64 ones).
//
// LDS per line: the slot pairs of the Dirichlet layout (component s and its
// mirror n-s share ceil(n/2) pairs of K complex entries; the nodes take the
// last pair, with the middle component for even n), element e's values at
// entry e-1, node j at entry j.  The values with no entry of their own —
// node K, and after a transform the k = 0 and k = K quantities — sit in
// entry 0 of each pair (interior pairs: (Z^s_0 + Z^{n-s}_0, Z^s_K -
// Z^{n-s}_K), node pair: (T0_0, T0_K)), node K at entry 0's free imaginary
// part for odd n, and in one extra double per line for even n (node K, the
// middle component's Z_0 and d_0, and the last node after the inverse).
#include "linepass.h"

namespace hofem {
namespace {

using lp::cx;

constexpr int kNeuMaxThreads = 512;
constexpr int kNeuMaxCB = 32;

struct NeuShape {
  int cb, threads;
  size_t lds;
};

// LDS bytes of cb lines: the slot pairs, then one double per line for even n.
inline size_t neu_lds(int n, int K, int cb) {
  const size_t slots = (size_t)cb * ((n + 1) / 2) * K * sizeof(cx<double>);
  return slots + (n % 2 == 0 ? (size_t)cb * sizeof(double) : 0);
}

// Lines per workgroup: as many as 160 KB of LDS holds (a power of two, at
// most kNeuMaxCB and the line count); 512 lanes when there are two or more.
inline NeuShape neu_shape(int n, int K, long long nlines) {
  long long cb = 1;
  while (cb * 2 <= kNeuMaxCB && neu_lds(n, K, (int)cb * 2) <= 160 * 1024 && cb * 2 <= nlines) cb *= 2;
  NeuShape s;
  s.cb = (int)cb;
  s.threads = cb >= 2 ? 512 : 256;
  s.lds = neu_lds(n, K, (int)cb);
  return s;
}

template <int N, int LOG2K, int MODE>
__global__ __launch_bounds__(kNeuMaxThreads) void neumann_pass(PassArgs a) {
  using S = lp::FftShape<LOG2K, 4>;
  constexpr int K = S::K, R = S::R, G = S::G;
  constexpr int C = (K / 2) / G;   // wave numbers per lane after the FFT
  constexpr int TPW = 64 / G;      // transform tasks per wavefront
  constexpr int NP = (N + 1) / 2;
  constexpr int m = N * K + 1;
  constexpr int NB0 = N / 2 + 1;   // band-edge vectors at theta = 0 (then (N+1)/2 at pi)
  constexpr bool kEven = N % 2 == 0;
  const int cb = a.cb, lcb = __builtin_ctz(cb);
  extern __shared__ __align__(16) unsigned char smem[];
  cx<double>* slots = reinterpret_cast<cx<double>*>(smem);                 // [cb][NP][K]
  double* side = reinterpret_cast<double*>(slots + (size_t)cb * NP * K);   // [cb], even N
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
  const lp::tgrp<double>* __restrict__ BLK = static_cast<const lp::tgrp<double>*>(a.tab.blk);
  const cx<double>* __restrict__ TW = static_cast<const cx<double>*>(a.tab.tw);
  const double* __restrict__ SN = static_cast<const double*>(a.tab.sn);
  const double* __restrict__ LAM = a.tab.lam;
  const double* __restrict__ BAND = a.tab.band;
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
  // the LDS place of physical value q of line c
  auto place = [&](int c, int q) -> double& {
    const int j = q / N, s = q - j * N;
    if (s == 0) {
      if (j < K) return slot(c, NP - 1, j).x;
      if constexpr (kEven) return side[c];
      else return slot(c, NP - 1, 0).y;
    }
    cx<double>& e = slot(c, lp::Seq<N>::pair(s), j);   // element j + 1
    return lp::Seq<N>::part(s) ? e.y : e.x;
  };
  const int items_m = cfast ? cb * m : cv * m;
  // kIO global accesses in flight per lane in the load and the scatter
  constexpr int kIO = 16;

  if (MODE != PASS_INV) {
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
        if (i0 + u * nthr < items_m && c < cv) place(c, q) = r[u];
      }
    }
  }
  __syncthreads();

  // DCT-I of the two sequences of pair p of line c, in place.  Forward: the
  // inputs are formed from the loaded values (z for interior pairs), entry 0
  // then receives the k = 0, K quantities.  Inverse: the inputs are the
  // synthesis coefficients (entry 0 as the blocks left it), the outputs are
  // combined into the element values u_{e,s} = D^s_{e-1} + D^{n-s}_e.
  auto dct_task = [&](int c, int p, bool inverse, int j) {
    cx<double>* tb = &slots[((size_t)c * NP + p) * K];
    const bool node = p == NP - 1;
    // (x^a_i, x^b_i) for i = 0..K
    cx<double> e0 = tb[lp::sw(0)];
    double sd = 0.0;
    if constexpr (kEven) sd = side[c];
    auto xin = [&](int i) -> cx<double> {
      if (!inverse) {
        const cx<double> e = i < K ? tb[lp::sw(i)] : cx<double>{0.0, 0.0};
        const cx<double> f = i > 0 ? tb[lp::sw(i - 1)] : cx<double>{0.0, 0.0};
        if (!node) return {e.x + f.y, e.y + f.x};   // (z^s_i, z^{n-s}_i)
        const double nd = i < K ? e.x : (kEven ? sd : e0.y);
        return {nd, kEven ? e.y + f.y : 0.0};         // (node i, z^{mid}_i)
      }
      if (i > 0 && i < K) {
        const cx<double> e = tb[lp::sw(i)];
        return {e.x, (node && !kEven) ? 0.0 : e.y};
      }
      if (!node) return i == 0 ? cx<double>{e0.x, e0.x} : cx<double>{e0.y, -e0.y};
      return i == 0 ? cx<double>{e0.x, kEven ? sd : 0.0} : cx<double>{e0.y, 0.0};
    };
    cx<double> v[R];
    cx<double> seed = {0.0, 0.0}, ch = {0.0, 0.0};
    const double sa = SN[j], ca = SN[K / 2 - j];   // sin, cos of pi j / K
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int jj = j + G * t;
      const double st = sa * lp::kCos16[t * (16 / R)] + ca * lp::kSin16[t * (16 / R)];   // sin(pi jj/K)
      const double ct = ca * lp::kCos16[t * (16 / R)] - sa * lp::kSin16[t * (16 / R)];   // cos(pi jj/K)
      const cx<double> xj = xin(jj), xk = xin(K - jj);
      v[t] = {0.5 * (xj.x + xk.x) - st * (xj.x - xk.x), 0.5 * (xj.y + xk.y) - st * (xj.y - xk.y)};
      seed.x += ct * xj.x;
      seed.y += ct * xj.y;
      if (jj == 0) {   // the i = K term of the seed (cos(pi) = -1) and (x_0 + x_K)/2
        seed.x -= xk.x;
        seed.y -= xk.y;
        ch = {0.5 * (xj.x + xk.x), 0.5 * (xj.y + xk.y)};
      }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      seed.x += __shfl_xor(seed.x, off, 64);
      seed.y += __shfl_xor(seed.y, off, 64);
      ch.x += __shfl_xor(ch.x, off, 64);
      ch.y += __shfl_xor(ch.y, off, 64);
    }
    lp::wave_sync();
    lp::task_fft<double, LOG2K, 4>(v, tb, j, TW);
    // even outputs and the odd outputs' increments of the wave numbers
    // k = jC..(j+1)C-1 of this lane
    cx<double> ev[C], rv[C];
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const int k = j * C + i;
      const cx<double> wa = tb[lp::sw(k)], wb = tb[lp::sw((K - k) & (K - 1))];
      // Y^a_k = (W_k + conj W_{K-k}) / 2, Y^b_k = (W_k - conj W_{K-k}) / (2i)
      ev[i] = {0.5 * (wa.x + wb.x) + ch.x, 0.5 * (wa.y + wb.y) + ch.y};
      rv[i] = {-0.5 * (wa.y - wb.y), 0.5 * (wa.x - wb.x)};
    }
    cx<double> xk = {0.0, 0.0};   // X_K of both sequences
    if (j == 0) {
      const cx<double> w = tb[lp::sw(K / 2)];
      xk = {w.x + ch.x, w.y + ch.y};
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      xk.x += __shfl_xor(xk.x, off, 64);
      xk.y += __shfl_xor(xk.y, off, 64);
    }
#pragma unroll
    for (int i = 1; i < C; ++i) rv[i] = lp::cadd(rv[i], rv[i - 1]);
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
    const cx<double> base = lp::cadd(seed, lp::csub(incl, tot));
    lp::wave_sync();
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const int k = j * C + i;
      tb[lp::sw(2 * k)] = ev[i];
      tb[lp::sw(2 * k + 1)] = lp::cadd(base, rv[i]);
    }
    lp::wave_sync();
    if (!inverse) {
      if (j == 0) {
        const cx<double> x0 = ev[0];   // k = 0 of lane 0
        if (!node) {
          tb[lp::sw(0)] = {x0.x + x0.y, xk.x - xk.y};
        } else {
          tb[lp::sw(0)] = {x0.x, xk.x};
          if constexpr (kEven) side[c] = x0.y;
        }
      }
      return;
    }
    // element values from the two transforms of the pair
    if (node && !kEven) {
      if (j == 0) tb[lp::sw(0)].y = xk.x;   // the last node
      return;
    }
    cx<double> cur[R], nxt[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int jj = j + G * t;
      cur[t] = tb[lp::sw(jj)];
      nxt[t] = jj + 1 < K ? tb[lp::sw(jj + 1)] : xk;
    }
    lp::wave_sync();
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int jj = j + G * t;
      if (!node) tb[lp::sw(jj)] = {cur[t].x + nxt[t].y, cur[t].y + nxt[t].x};
      else tb[lp::sw(jj)].y = cur[t].y + nxt[t].y;   // middle point; the node stays
    }
    if constexpr (kEven) {
      if (node && j == 0) side[c] = xk.x;   // the last node
    }
  };
  auto transforms = [&](bool inverse) {   // rounds of TPW tasks per wave
    const int ntask = cv * NP;
    for (int t0 = 0; t0 < ntask; t0 += nwaves * TPW) {
      const int task = t0 + wave * TPW + lane / G;
      if (task < ntask) {
        const int c = task / NP, p = task - c * NP;
        int j = lane & (G - 1);
        asm volatile("" : "+v"(j));   // keeps the lane's address arithmetic inside the loop
        dct_task(c, p, inverse, j);
      }
    }
  };
  if (MODE != PASS_INV) {
    transforms(false);
    __syncthreads();
  }

  // ---- blocks: k = 1..K-1 with the Dirichlet tables, k = 0 and K the band edges
  const double sc = a.scale;
  auto line_den = [&](int c) -> double {
    double d = a.alpha;
    const long long t = (L0 + c) % inner;   // position among the other axes
    for (int i = 0; i < a.nother; ++i) d += a.oscale[i] * a.olam[i][(t / a.odiv[i]) % a.omod[i]];
    return d;
  };
  auto comp = [&](int c, int s, int k) -> double& {
    cx<double>& e = slot(c, lp::Seq<N>::pair(s), k);
    return lp::Seq<N>::part(s) ? e.y : e.x;
  };
  // wave numbers k = 1..K-1: one lane per (pair of lines, k), the
  // eigenvector rows of k read once for both lines
  const int npc = cb > 1 ? cb / 2 : 1, lnpc = __builtin_ctz(npc);
  const int items_p = (cfast ? npc : (cv + 1) / 2) * (K - 1);
  for (int i = tid; i < items_p; i += nthr) {
    int cp, k;
    if (cfast) {
      cp = i & (npc - 1);
      k = (i >> lnpc) + 1;
    } else {
      cp = i / (K - 1);
      k = i - cp * (K - 1) + 1;
    }
    const int c0 = 2 * cp, c1 = c0 + 1;
    if (c0 >= cv) continue;
    const bool two = c1 < cv;
    const long long ob[2] = {lbase(c0), two ? lbase(c1) : 0};
    const lp::tgrp<double>* tb = lp::blk_at<N>(BLK, k);
    double x[2][N], y[2][N];
    if (MODE != PASS_INV) {
#pragma unroll
      for (int s = 0; s < N; ++s) {
        x[0][s] = comp(c0, s, k);
        x[1][s] = two ? comp(c1, s, k) : 0.0;
      }
    }
    if (MODE == PASS_FUSED) {
      const double dl[2] = {line_den(c0), two ? line_den(c1) : 1.0};
      lp::fused_lines<double, N, 2>(tb, LAM + (k - 1), K - 1, dl, sc, x, y);
    } else {
#pragma unroll
      for (int s = 0; s < N; ++s) y[0][s] = y[1][s] = 0.0;
#pragma unroll
      for (int l = 0; l < N; ++l) {
        double p[N > 1 ? N - 1 : 1];
#pragma unroll
        for (int s = 1; s < N; ++s) p[s - 1] = lp::tab_e(tb, l * (N - 1) + s - 1);
        const long long qo = ((long long)l * (K - 1) + (k - 1)) * inner;
        if (MODE == PASS_FWD) {
          const double nrm = lp::tab_e(tb, N * (N - 1) + l);
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            double acc = x[u][0];
#pragma unroll
            for (int s = 1; s < N; ++s) acc += p[s - 1] * x[u][s];
            if (u == 0 || two) dst[ob[u] + qo] = acc * nrm;
          }
        } else {
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const double w = (u == 0 || two) ? src[ob[u] + qo] : 0.0;
            y[u][0] += w;
#pragma unroll
            for (int s = 1; s < N; ++s) y[u][s] += w * p[s - 1];
          }
        }
      }
    }
    if (MODE != PASS_FWD) {
#pragma unroll
      for (int s = 0; s < N; ++s) {
        comp(c0, s, k) = y[0][s];
        if (two) comp(c1, s, k) = y[1][s];
      }
    }
  }
  // band edges: theta = 0 (k = 0, entry 0 .x) and theta = pi (k = K, .y),
  // one lane per (line, edge)
  const int items_b = (cfast ? cb : cv) * 2;
  for (int i = tid; i < items_b; i += nthr) {
    int c, e;
    split(i, 2, c, e);
    if (c >= cv) continue;
    const long long ob = lbase(c);
    const double dline = MODE == PASS_FUSED ? line_den(c) : 0.0;
    const bool hi = e == 1;
    const int b0 = hi ? NB0 : 0, b1 = hi ? N + 1 : NB0;
    cx<double>& nodee = slot(c, NP - 1, 0);
    const double t0 = hi ? nodee.y : nodee.x;
    double zp[NP > 1 ? NP - 1 : 1];   // Z^s_0 + Z^{n-s}_0 or Z^s_K - Z^{n-s}_K, s = p + 1
#pragma unroll
    for (int p = 0; p < NP - 1; ++p) zp[p] = hi ? slot(c, p, 0).y : slot(c, p, 0).x;
    const double zmid = (kEven && !hi) ? side[c] : 0.0;
    double wsum = 0.0, hp[NP > 1 ? NP - 1 : 1], hmid = 0.0;
#pragma unroll
    for (int p = 0; p < NP - 1; ++p) hp[p] = 0.0;
    for (int b = b0; b < b1; ++b) {
      const double* w = BAND + (size_t)b * N;
      const long long qa = ob + ((long long)N * (K - 1) + b) * inner;
      double cf;
      if (MODE == PASS_INV) {
        cf = src[qa];
      } else {
        double acc = w[0] * t0;
#pragma unroll
        for (int p = 0; p < NP - 1; ++p) acc += 0.5 * w[p + 1] * zp[p];
        if constexpr (kEven) acc += 0.5 * w[N / 2] * zmid;
        cf = acc / K;
        if (MODE == PASS_FWD) {
          dst[qa] = cf;
          continue;
        }
        cf /= dline + sc * LAM[(size_t)N * (K - 1) + b];
      }
      wsum += cf * w[0];
#pragma unroll
      for (int p = 0; p < NP - 1; ++p) hp[p] += 0.5 * cf * w[p + 1];
      if constexpr (kEven) hmid += 0.5 * cf * w[N / 2];
    }
    if (MODE != PASS_FWD) {
      if (hi) nodee.y = wsum; else nodee.x = wsum;
#pragma unroll
      for (int p = 0; p < NP - 1; ++p) {
        if (hi) slot(c, p, 0).y = hp[p]; else slot(c, p, 0).x = hp[p];
      }
      if constexpr (kEven) {
        if (!hi) side[c] = hmid;
      }
    }
  }
  if (MODE == PASS_FWD) return;
  __syncthreads();
  transforms(true);
  __syncthreads();
  for (int i0 = tid; i0 < items_m; i0 += kIO * nthr) {
    double r[kIO];
#pragma unroll
    for (int u = 0; u < kIO; ++u) {
      int c, q;
      split(i0 + u * nthr, m, c, q);
      r[u] = (i0 + u * nthr < items_m && c < cv) ? place(c, q) : 0.0;
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
hipError_t launch_neu_k(const PassArgs& a0, hipStream_t s) {
  constexpr int K = 1 << LOG2K;
  if (a0.tab.n != N || a0.tab.K != K || a0.tab.m != N * K + 1 || !a0.tab.band) return hipErrorInvalidValue;
  const NeuShape sh = neu_shape(N, K, a0.nlines);
  if (sh.lds > 160 * 1024) return hipErrorInvalidValue;
  PassArgs a = a0;
  a.cb = sh.cb;
  auto fn = neumann_pass<N, LOG2K, MODE>;
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
hipError_t launch_neu_nk(const PassArgs& a, hipStream_t s) {
  switch (a.tab.K) {
    case 2: return launch_neu_k<N, 1, MODE>(a, s);
    case 4: return launch_neu_k<N, 2, MODE>(a, s);
    case 8: return launch_neu_k<N, 3, MODE>(a, s);
    case 16: return launch_neu_k<N, 4, MODE>(a, s);
    case 32: return launch_neu_k<N, 5, MODE>(a, s);
    case 64: return launch_neu_k<N, 6, MODE>(a, s);
    case 128: return launch_neu_k<N, 7, MODE>(a, s);
    case 256: return launch_neu_k<N, 8, MODE>(a, s);
    case 512: return launch_neu_k<N, 9, MODE>(a, s);
    case 1024: return launch_neu_k<N, 10, MODE>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int MODE>
hipError_t launch_neu_mode(const PassArgs& a, hipStream_t s) {
  switch (a.tab.n) {
    case 1: return launch_neu_nk<1, MODE>(a, s);
    case 2: return launch_neu_nk<2, MODE>(a, s);
    case 3: return launch_neu_nk<3, MODE>(a, s);
    case 4: return launch_neu_nk<4, MODE>(a, s);
    case 5: return launch_neu_nk<5, MODE>(a, s);
    case 6: return launch_neu_nk<6, MODE>(a, s);
    case 7: return launch_neu_nk<7, MODE>(a, s);
    case 8: return launch_neu_nk<8, MODE>(a, s);
    case 9: return launch_neu_nk<9, MODE>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_neumann(int kind, const PassArgs& a, hipStream_t s) {
  if (a.nlines == 0) return hipSuccess;
  switch (kind) {
    case PASS_FWD: return launch_neu_mode<PASS_FWD>(a, s);
    case PASS_INV: return launch_neu_mode<PASS_INV>(a, s);
    case PASS_FUSED: return launch_neu_mode<PASS_FUSED>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hofem
