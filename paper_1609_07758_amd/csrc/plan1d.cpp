// Host precompute of the 1D eigen data of the nth-order FEM pencil, in
// binary128 (__float128, libquadmath), rounded once to FP64 and FP32.
//
// Route (Section 2, paragraphs 1-3 of the paper):
//   * local stiffness/mass on [-1, 1] (Lagrange basis on the equispaced nodes
//     -1 + 2k/n) by (n+1)-point Gauss-Legendre quadrature, which integrates
//     the degree-2n integrands exactly;
//   * the interior-node eigenproblem A~ e = lam C~ e of eq. (eig_elem) by a
//     Cholesky reduction and cyclic Jacobi, normalised C~ e . e = 1;
//   * for every wave number k = 1..K-1 the n roots of the secular equation
//     eq. (theta) at theta_k = cos(pi k / K), written with the expansion
//     coefficients a^(l), c^(l) of Lemma 2.  Its poles are the interior
//     eigenvalues lam_0^(l) and its n roots interlace with them (the roots are
//     the eigenvalues of a Hermitian pencil whose interior block is
//     (A~, C~)), one root in each of (0, lam_0^(1)), ..., (lam_0^(n-1), inf);
//   * p_k^(l) by the expansion formula of Lemma 2, and the norms
//     ||s_k^(l)||_C^2 = K (b0 + bn theta_k) of the transform theorem.
//
// Nothing here runs on the GPU; the tables are uploaded by the solver.

#include <quadmath.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "plan1d.h"

namespace hofem {
namespace {

typedef __float128 q128;

q128 qabs(q128 x) { return x < 0 ? -x : x; }

// Legendre polynomial P_npts(z) and its derivative by the three-term recurrence.
void legendre(int npts, q128 z, q128& p, q128& dp) {
  q128 p0 = 1, p1 = z;
  for (int k = 2; k <= npts; ++k) {
    q128 p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = npts * (z * p1 - p0) / (z * z - 1);
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton on P_npts (npts >= 2).
void gauss_legendre(int npts, std::vector<q128>& x, std::vector<q128>& w) {
  x.assign(npts, 0);
  w.assign(npts, 0);
  for (int i = 0; i < npts; ++i) {
    q128 z = cosq(M_PIq * (i + 0.75Q) / (npts + 0.5Q)), p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(npts, z, p, dp);
      q128 dz = p / dp;
      z -= dz;
      if (qabs(dz) < 1e-34Q) break;
    }
    legendre(npts, z, p, dp);
    // the initial guesses decrease with i: store in ascending order
    x[npts - 1 - i] = z;
    w[npts - 1 - i] = 2 / ((1 - z * z) * dp * dp);
  }
}

// Local matrices of the order-n Lagrange element on [-1, 1]; also returns the
// Gauss rule and the basis values / derivatives at its nodes.
void local_matrices(int n, std::vector<q128>& A, std::vector<q128>& C, std::vector<q128>& gx,
                    std::vector<q128>& gw, std::vector<q128>& Bq, std::vector<q128>& Dq) {
  const int nb = n + 1;
  std::vector<q128> xi(nb);
  for (int k = 0; k <= n; ++k) xi[k] = -1 + (q128)(2 * k) / n;
  gauss_legendre(n + 1, gx, gw);
  A.assign(nb * nb, 0);
  C.assign(nb * nb, 0);
  Bq.assign(nb * nb, 0);
  Dq.assign(nb * nb, 0);
  std::vector<q128> e(nb), de(nb);
  for (size_t g = 0; g < gx.size(); ++g) {
    const q128 x = gx[g];
    for (int l = 0; l <= n; ++l) {
      q128 v = 1;
      for (int m = 0; m <= n; ++m)
        if (m != l) v *= (x - xi[m]) / (xi[l] - xi[m]);
      e[l] = v;
      // derivative by the product rule, without dividing by (x - xi_m)
      q128 d = 0;
      for (int m = 0; m <= n; ++m) {
        if (m == l) continue;
        q128 t = 1 / (xi[l] - xi[m]);
        for (int r = 0; r <= n; ++r)
          if (r != l && r != m) t *= (x - xi[r]) / (xi[l] - xi[r]);
        d += t;
      }
      de[l] = d;
    }
    for (int r = 0; r <= n; ++r) {
      Bq[g * nb + r] = e[r];
      Dq[g * nb + r] = de[r];
      for (int s = 0; s <= n; ++s) {
        A[r * nb + s] += gw[g] * de[r] * de[s];
        C[r * nb + s] += gw[g] * e[r] * e[s];
      }
    }
  }
  // Symmetrise exactly (the quadrature is symmetric up to rounding).
  for (int r = 0; r <= n; ++r)
    for (int s = r + 1; s <= n; ++s) {
      q128 a = (A[r * nb + s] + A[s * nb + r]) / 2, c = (C[r * nb + s] + C[s * nb + r]) / 2;
      A[r * nb + s] = A[s * nb + r] = a;
      C[r * nb + s] = C[s * nb + r] = c;
    }
}

// Cyclic Jacobi eigen-decomposition of a symmetric d x d matrix (row major).
// On return B holds the eigenvalues on its diagonal and Q the eigenvectors
// (columns).
void jacobi(int d, std::vector<q128>& B, std::vector<q128>& Q) {
  Q.assign(d * d, 0);
  for (int i = 0; i < d; ++i) Q[i * d + i] = 1;
  for (int sweep = 0; sweep < 100; ++sweep) {
    q128 off = 0, tot = 0;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        q128 v = B[i * d + j] * B[i * d + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-70Q * tot) break;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) {
        q128 apq = B[p * d + q];
        if (apq == 0) continue;
        q128 app = B[p * d + p], aqq = B[q * d + q];
        q128 tau = (aqq - app) / (2 * apq);
        q128 t = (tau >= 0 ? 1 : -1) / (qabs(tau) + sqrtq(1 + tau * tau));
        q128 c = 1 / sqrtq(1 + t * t), s = t * c;
        for (int k = 0; k < d; ++k) {  // columns p, q
          q128 bkp = B[k * d + p], bkq = B[k * d + q];
          B[k * d + p] = c * bkp - s * bkq;
          B[k * d + q] = s * bkp + c * bkq;
        }
        for (int k = 0; k < d; ++k) {  // rows p, q
          q128 bpk = B[p * d + k], bqk = B[q * d + k];
          B[p * d + k] = c * bpk - s * bqk;
          B[q * d + k] = s * bpk + c * bqk;
        }
        for (int k = 0; k < d; ++k) {
          q128 qkp = Q[k * d + p], qkq = Q[k * d + q];
          Q[k * d + p] = c * qkp - s * qkq;
          Q[k * d + q] = s * qkp + c * qkq;
        }
      }
  }
}

// Interior pencil (At, Ct) of order d: eigenvalues ascending, C~-normalised
// eigenvectors as columns of E (row major d x d).
void interior_eigen(int d, const std::vector<q128>& At, const std::vector<q128>& Ct,
                    std::vector<q128>& lam0, std::vector<q128>& E) {
  lam0.assign(d, 0);
  E.assign(d * d, 0);
  if (d == 0) return;
  // Cholesky Ct = L L^T
  std::vector<q128> L(d * d, 0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j <= i; ++j) {
      q128 s = Ct[i * d + j];
      for (int k = 0; k < j; ++k) s -= L[i * d + k] * L[j * d + k];
      L[i * d + j] = (i == j) ? sqrtq(s) : s / L[j * d + j];
    }
  // Li = L^-1 (lower triangular)
  std::vector<q128> Li(d * d, 0);
  for (int col = 0; col < d; ++col) {
    for (int i = 0; i < d; ++i) {
      q128 s = (i == col) ? 1 : 0;
      for (int k = 0; k < i; ++k) s -= L[i * d + k] * Li[k * d + col];
      Li[i * d + col] = s / L[i * d + i];
    }
  }
  // B = Li At Li^T
  std::vector<q128> T(d * d, 0), B(d * d, 0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      q128 s = 0;
      for (int k = 0; k < d; ++k) s += Li[i * d + k] * At[k * d + j];
      T[i * d + j] = s;
    }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      q128 s = 0;
      for (int k = 0; k < d; ++k) s += T[i * d + k] * Li[j * d + k];
      B[i * d + j] = s;
    }
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j) B[i * d + j] = B[j * d + i] = (B[i * d + j] + B[j * d + i]) / 2;
  std::vector<q128> Q;
  jacobi(d, B, Q);
  std::vector<int> order(d);
  for (int i = 0; i < d; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return B[a * d + a] < B[b * d + b]; });
  for (int l = 0; l < d; ++l) {
    int o = order[l];
    lam0[l] = B[o * d + o];
    // e = Li^T y
    std::vector<q128> e(d, 0);
    for (int i = 0; i < d; ++i) {
      q128 s = 0;
      for (int k = 0; k < d; ++k) s += Li[k * d + i] * Q[k * d + o];
      e[i] = s;
    }
    // Sign: the lowest-index entry with |e_i| >= max|e| / 2 is positive.
    q128 mx = 0;
    for (int i = 0; i < d; ++i) mx = std::max(mx, qabs(e[i]));
    int lead = 0;
    while (qabs(e[lead]) < mx / 2) ++lead;
    q128 sg = e[lead] < 0 ? -1 : 1;
    for (int i = 0; i < d; ++i) E[i * d + l] = sg * e[i];
  }
}

struct Secular {
  int d;                       // n - 1
  q128 a0, c0, an, cn;
  std::vector<q128> al, cl, alc, clc, lam0;  // a^(l), c^(l), a-check^(l), c-check^(l)
  // F(lam) = (a0 - lam c0) + sum (a^(l) - lam c^(l))^2 / (lam - lam0_l)
  //        + theta [(an - lam cn) + sum (ac^(l) - lam cc^(l))(a^(l) - lam c^(l)) / (lam - lam0_l)]
  void eval(q128 lam, q128 th, q128& F, q128& dF) const {
    F = (a0 - lam * c0) + th * (an - lam * cn);
    dF = -c0 - th * cn;
    for (int l = 0; l < d; ++l) {
      q128 u = al[l] - lam * cl[l], v = alc[l] - lam * clc[l];
      q128 r = 1 / (lam - lam0[l]);
      q128 num = u * u + th * v * u;
      F += num * r;
      // d/dlam [num r] = num' r - num r^2
      q128 dnum = -2 * cl[l] * u + th * (-clc[l] * u - cl[l] * v);
      dF += dnum * r - num * r * r;
    }
  }
};

// One root of F in the open interval (lo, hi), with F > 0 just right of lo
// and F < 0 just left of hi: safeguarded Newton on bisection brackets.
q128 root_in(const Secular& S, q128 th, q128 lo, q128 hi) {
  q128 x = (lo + hi) / 2;
  for (int it = 0; it < 400; ++it) {
    q128 F, dF;
    S.eval(x, th, F, dF);
    if (F > 0) lo = x; else hi = x;
    if (F == 0) return x;
    q128 xn = x - F / dF;
    if (!(xn > lo && xn < hi) || dF == 0) xn = (lo + hi) / 2;
    if (qabs(xn - x) <= 1e-33Q * qabs(xn) || hi - lo <= 1e-33Q * qabs(x)) return xn;
    x = xn;
  }
  return x;
}

}  // namespace

int plan1d_build(int n, int K, Plan1DData* out) {
  if (n < 1 || n > 9 || K < 2 || K > 65536) return -1;
  const int nb = n + 1, d = n - 1, m = n * K - 1;
  std::vector<q128> A, C, gx, gw, Bq, Dq;
  local_matrices(n, A, C, gx, gw, Bq, Dq);
  auto Aat = [&](int r, int s) { return A[r * nb + s]; };
  auto Cat = [&](int r, int s) { return C[r * nb + s]; };
  std::vector<q128> At(d * d), Ct(d * d);
  for (int r = 0; r < d; ++r)
    for (int s = 0; s < d; ++s) {
      At[r * d + s] = Aat(r + 1, s + 1);
      Ct[r * d + s] = Cat(r + 1, s + 1);
    }
  std::vector<q128> lam0, E;
  interior_eigen(d, At, Ct, lam0, E);

  Secular S;
  S.d = d;
  S.a0 = Aat(0, 0); S.c0 = Cat(0, 0); S.an = Aat(0, n); S.cn = Cat(0, n);
  S.al.assign(d, 0); S.cl.assign(d, 0); S.alc.assign(d, 0); S.clc.assign(d, 0);
  S.lam0 = lam0;
  for (int l = 0; l < d; ++l)
    for (int i = 0; i < d; ++i) {
      q128 e = E[i * d + l];
      S.al[l] += Aat(i + 1, 0) * e;
      S.cl[l] += Cat(i + 1, 0) * e;
      S.alc[l] += Aat(i + 1, n) * e;
      S.clc[l] += Cat(i + 1, n) * e;
    }

  out->n = n;
  out->K = K;
  out->m = m;
  out->A.assign(nb * nb, 0);
  out->C.assign(nb * nb, 0);
  for (int i = 0; i < nb * nb; ++i) {
    out->A[i] = (double)A[i];
    out->C[i] = (double)C[i];
  }
  out->lam.assign(m, 0);
  out->p.assign((size_t)(K - 1) * n * std::max(d, 1), 0);
  out->inorm.assign((size_t)(K - 1) * n, 0);
  out->E.assign(std::max(d * d, 1), 0);
  out->lam0.assign(std::max(d, 1), 0);
  for (int i = 0; i < d * d; ++i) out->E[i] = (double)E[i];
  for (int l = 0; l < d; ++l) {
    out->lam0[l] = (double)lam0[l];
    out->lam[l] = (double)lam0[l];
  }

  std::vector<q128> lroots(n), p(d);
  for (int k = 1; k < K; ++k) {
    const q128 th = cosq(M_PIq * k / K);
    // brackets: (0, lam0_1), (lam0_1, lam0_2), ..., (lam0_{n-1}, hi)
    q128 top = d ? lam0[d - 1] : 0;
    q128 hi = 2 * top + 16;
    for (int it = 0; it < 200; ++it) {
      q128 F, dF;
      S.eval(hi, th, F, dF);
      if (F < 0) break;
      hi *= 2;
    }
    for (int l = 0; l < n; ++l) {
      q128 lo = (l == 0) ? 0 : lam0[l - 1];
      q128 up = (l == d) ? hi : lam0[l];
      lroots[l] = root_in(S, th, lo, up);
    }
    for (int l = 0; l < n; ++l) {
      const q128 lam = lroots[l];
      // Lemma 2: p = sum_m (a^(m) - lam c^(m)) / (lam - lam0_m) e^(m)
      for (int i = 0; i < d; ++i) p[i] = 0;
      for (int mm = 0; mm < d; ++mm) {
        q128 coef = (S.al[mm] - lam * S.cl[mm]) / (lam - lam0[mm]);
        for (int i = 0; i < d; ++i) p[i] += coef * E[i * d + mm];
      }
      // ||s||^2 = K (b0 + bn theta), b0 = c0 + (C~p + 2c).p, bn = cn + (C~p + 2c).Pp
      q128 b0 = S.c0, bn = S.cn;
      for (int i = 0; i < d; ++i) {
        q128 w = 2 * Cat(i + 1, 0);
        for (int j = 0; j < d; ++j) w += Ct[i * d + j] * p[j];
        b0 += w * p[i];
        bn += w * p[d - 1 - i];
      }
      q128 norm2 = K * (b0 + bn * th);
      size_t base = ((size_t)(k - 1) * n + l);
      out->inorm[base] = (double)(1 / norm2);
      for (int i = 0; i < d; ++i) out->p[base * d + i] = (double)p[i];
      out->lam[(size_t)(n - 1) + (size_t)l * (K - 1) + (k - 1)] = (double)lam;
    }
  }
  out->gx.assign(nb, 0);
  out->gw.assign(nb, 0);
  out->B.assign(nb * nb, 0);
  out->D.assign(nb * nb, 0);
  for (int i = 0; i < nb; ++i) {
    out->gx[i] = (double)gx[i];
    out->gw[i] = (double)gw[i];
  }
  for (int i = 0; i < nb * nb; ++i) {
    out->B[i] = (double)Bq[i];
    out->D[i] = (double)Dq[i];
  }
  // Barycentric differentiation matrix of the Gauss nodes: off the diagonal
  // (c_p / c_q) / (x_q - x_p) with c_j = 1 / prod_{m != j} (x_j - x_m); the
  // diagonal makes every row sum to zero.
  {
    std::vector<q128> c(nb, 1);
    for (int j = 0; j < nb; ++j) {
      for (int m = 0; m < nb; ++m)
        if (m != j) c[j] *= gx[j] - gx[m];
      c[j] = 1 / c[j];
    }
    out->Dh.assign(nb * nb, 0);
    for (int q = 0; q < nb; ++q) {
      q128 diag = 0;
      for (int p = 0; p < nb; ++p) {
        if (p == q) continue;
        const q128 v = (c[p] / c[q]) / (gx[q] - gx[p]);
        out->Dh[q * nb + p] = (double)v;
        diag -= v;
      }
      out->Dh[q * nb + q] = (double)diag;
    }
  }
  // FFT support: twiddles exp(2 pi i t / K) and sin(pi t / K), t = 0..K-1.
  out->tw.assign(2 * K, 0);
  out->sn.assign(K, 0);
  for (int t = 0; t < K; ++t) {
    out->tw[2 * t] = (double)cosq(2 * M_PIq * t / K);
    out->tw[2 * t + 1] = (double)sinq(2 * M_PIq * t / K);
    out->sn[t] = (double)sinq(M_PIq * t / K);
  }
  return 0;
}

// Periodic axis (Section 2's pencil on a periodic mesh; the paper's
// Bloch-type structure with phase 2 pi k / K).  A cell holds the n unknowns
// node j and the interior points of element j+1; element j+1 couples cell j
// with node j+1 of cell j+1, so the pencil is block circulant and its
// eigenvectors are Bloch waves v_j = w e^{i phi j}, phi = 2 pi k / K, where
// (lam, w) solve the n x n Hermitian pencil (T^H A T, T^H C T),
// T = [[I_n], [e^{i phi} e_0^T]] (local nodes 0..n-1 are the cell, local node
// n is node j+1).  The pencil is solved through its real 2n x 2n symmetric
// embedding [[X, -Y], [Y, X]] (every eigenvalue doubled) by Cholesky and
// Jacobi in binary128; w is normalised to w^H (T^H C T) w = 1 and rotated
// so that its largest entry is real and positive (real at k = 0, K/2).
int plan1d_build_periodic(int n, int K, Plan1DData* out) {
  if (K < 2) return -1;
  if (plan1d_build(n, K, out) != 0) return -1;   // local matrices, Gauss tables, twiddles
  const int nb = n + 1, d2 = 2 * n, m = n * K, nk = K / 2 + 1;
  std::vector<q128> A, C, gx, gw, Bq, Dq;
  local_matrices(n, A, C, gx, gw, Bq, Dq);
  out->bc = 1;
  out->m = m;
  out->p.clear();
  out->inorm.clear();
  out->lam.assign(m, 0);
  out->wr.assign((size_t)nk * n * n, 0);
  out->wi.assign((size_t)nk * n * n, 0);
  for (int k = 0; k < nk; ++k) {
    const q128 ph = 2 * M_PIq * k / K;
    const q128 cr = cosq(ph), ci = sinq(ph);
    // T^H M T for M = A, C: real part X, imaginary part Y (n x n)
    auto bloch = [&](const std::vector<q128>& M, std::vector<q128>& X, std::vector<q128>& Y) {
      X.assign(n * n, 0);
      Y.assign(n * n, 0);
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          // sum_{r,c} conj(T[r][a]) M[r][c] T[c][b]; T[r][a] = [r == a] (r < n),
          // T[n][a] = e^{i phi} [a == 0]
          q128 xr = M[a * nb + b], xi = 0;
          if (b == 0) {   // column c = n, T[n][0] = e^{i phi}
            xr += M[a * nb + n] * cr;
            xi += M[a * nb + n] * ci;
          }
          if (a == 0) {   // row r = n, conj(T[n][0]) = e^{-i phi}
            xr += M[n * nb + b] * cr;
            xi -= M[n * nb + b] * ci;
          }
          if (a == 0 && b == 0) xr += M[n * nb + n];
          X[a * n + b] = xr;
          Y[a * n + b] = xi;
        }
    };
    std::vector<q128> XA, YA, XC, YC;
    bloch(A, XA, YA);
    bloch(C, XC, YC);
    std::vector<q128> Ae(d2 * d2), Ce(d2 * d2);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        Ae[a * d2 + b] = XA[a * n + b];
        Ae[(a + n) * d2 + (b + n)] = XA[a * n + b];
        Ae[a * d2 + (b + n)] = -YA[a * n + b];
        Ae[(a + n) * d2 + b] = YA[a * n + b];
        Ce[a * d2 + b] = XC[a * n + b];
        Ce[(a + n) * d2 + (b + n)] = XC[a * n + b];
        Ce[a * d2 + (b + n)] = -YC[a * n + b];
        Ce[(a + n) * d2 + b] = YC[a * n + b];
      }
    std::vector<q128> lam2, V2;
    interior_eigen(d2, Ae, Ce, lam2, V2);   // ascending, pairs of equal eigenvalues
    for (int l = 0; l < n; ++l) {
      const int o = 2 * l;
      std::vector<q128> wr(n), wi(n);
      for (int s2 = 0; s2 < n; ++s2) {
        wr[s2] = V2[s2 * d2 + o];
        wi[s2] = V2[(s2 + n) * d2 + o];
      }
      // phase: largest entry real positive
      int big = 0;
      for (int s2 = 1; s2 < n; ++s2)
        if (wr[s2] * wr[s2] + wi[s2] * wi[s2] > wr[big] * wr[big] + wi[big] * wi[big]) big = s2;
      const q128 mag = sqrtq(wr[big] * wr[big] + wi[big] * wi[big]);
      const q128 pr = wr[big] / mag, pi = -wi[big] / mag;   // multiply by conj(w_big)/|w_big|
      for (int s2 = 0; s2 < n; ++s2) {
        const q128 a = wr[s2] * pr - wi[s2] * pi, b = wr[s2] * pi + wi[s2] * pr;
        wr[s2] = a;
        wi[s2] = b;
      }
      if (k == 0 || 2 * k == K)
        for (int s2 = 0; s2 < n; ++s2) wi[s2] = 0;
      // w^H C w = 1 with C = X_C + i Y_C
      q128 nrm = 0;
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          // conj(w_a) (X + iY)_ab w_b, real part
          const q128 mr = XC[a * n + b], mi = YC[a * n + b];
          const q128 tr = mr * wr[b] - mi * wi[b], ti = mr * wi[b] + mi * wr[b];
          nrm += wr[a] * tr + wi[a] * ti;
        }
      const q128 sc = 1 / sqrtq(nrm);
      for (int s2 = 0; s2 < n; ++s2) {
        out->wr[((size_t)k * n + l) * n + s2] = (double)(wr[s2] * sc);
        out->wi[((size_t)k * n + l) * n + s2] = (double)(wi[s2] * sc);
      }
      // the constants span the kernel of A: lambda = 0 exactly for k = 0, l = 0
      const double lv = k == 0 && l == 0 ? 0.0 : (double)lam2[o];
      if (k == 0) {
        out->lam[(size_t)l * K] = lv;
      } else if (2 * k == K) {
        out->lam[(size_t)l * K + K - 1] = lv;
      } else {
        out->lam[(size_t)l * K + 2 * k - 1] = lv;
        out->lam[(size_t)l * K + 2 * k] = lv;
      }
    }
  }
  return 0;
}

int plan1d_build_dense(Plan1DData* d) {
  const int n = d->n, K = d->K, m = d->m;
  if (m < 1 || m > kDenseMax) return -1;
  d->dense = 1;
  d->S.assign((size_t)m * m, 0.0);
  d->St.assign((size_t)m * m, 0.0);
  // sin and cos of pi x / K for an integer x, reduced modulo 2K first
  constexpr long double kPi = 3.14159265358979323846264338327950288L;
  auto red = [&](long long x) { return ((x % (2LL * K)) + 2LL * K) % (2LL * K); };
  auto sine = [&](long long x) -> long double { return sinl(kPi * (long double)red(x) / (long double)K); };
  auto cosine = [&](long long x) -> long double { return cosl(kPi * (long double)red(x) / (long double)K); };
  auto put = [&](int q, int c, long double v, double norm) {
    d->S[(size_t)q * m + c] = (double)v;
    d->St[(size_t)q * m + c] = (double)(v * norm);
  };
  if (d->bc == 1) {
    // periodic, column l K + t: the Bloch wave v = w_{k,l} e^{i 2 pi k j / K}
    // (cell j, component s at q = n j + s) as real vectors.  The passes'
    // coefficients are c = (1/K) v^H y stored as (Re c, Im c) at t = 2k-1, 2k
    // (0 < k < K/2) and the inverse is y = sum over all k of c v, the
    // conjugate wave numbers included; so S holds 2 Re v and -2 Im v there, St
    // Re v / K and -Im v / K, and v itself (real) and v / K at t = 0 (k = 0)
    // and t = K-1 (k = K/2, even K).
    const int ne = n * n;
    for (int k = 0; 2 * k <= K; ++k) {
      const bool self = k == 0 || 2 * k == K;
      const int t = k == 0 ? 0 : (2 * k == K ? K - 1 : 2 * k - 1);
      for (int l = 0; l < n; ++l) {
        const int c = l * K + t;
        for (int j = 0; j < K; ++j) {
          const long double ph = 2.0L * kPi * (long double)(((long long)k * j) % K) / (long double)K;
          const long double cr = cosl(ph), ci = sinl(ph);
          for (int s2 = 0; s2 < n; ++s2) {
            const long double wr = d->wr[(size_t)k * ne + (size_t)l * n + s2];
            const long double wi = d->wi[(size_t)k * ne + (size_t)l * n + s2];
            const long double vr = wr * cr - wi * ci, vi = wr * ci + wi * cr;
            const int q = n * j + s2;
            if (self) {
              put(q, c, vr, 1.0 / K);
            } else {
              d->S[(size_t)q * m + c] = (double)(2.0L * vr);
              d->St[(size_t)q * m + c] = (double)(vr / K);
              d->S[(size_t)q * m + c + 1] = (double)(-2.0L * vi);
              d->St[(size_t)q * m + c + 1] = (double)(-vi / K);
            }
          }
        }
      }
    }
    return 0;
  }
  if (d->bc == 2) {
    // Neumann: k = 1..K-1, l = 1..n (column (l-1)(K-1) + k-1): cos(pi k j / K)
    // at node j = 0..K (point n j), cos(pi k (e-1)/K) p_s + cos(pi k e/K) p_{n-s}
    // in element e; then the band-edge cells repeated with the factor 1 or
    // (-1)^j, norm K
    for (int k = 1; k < K; ++k)
      for (int l = 1; l <= n; ++l) {
        const int c = (l - 1) * (K - 1) + (k - 1);
        const double norm = d->inorm[(size_t)(k - 1) * n + (l - 1)];
        const double* p = d->p.data() + ((size_t)(k - 1) * n + (l - 1)) * (n - 1);
        for (int j = 0; j <= K; ++j) put(n * j, c, cosine((long long)k * j), norm);
        for (int e = 1; e <= K; ++e)
          for (int s = 1; s < n; ++s) {
            const long double v = cosine((long long)k * (e - 1)) * (long double)p[s - 1] +
                                  cosine((long long)k * e) * (long double)p[n - s - 1];
            put(n * (e - 1) + s, c, v, norm);
          }
      }
    const int nb0 = n / 2 + 1;
    for (int b = 0; b <= n; ++b) {
      const int c = n * (K - 1) + b;
      const long double sg = b < nb0 ? 1.0L : -1.0L;
      const double* w = d->band.data() + (size_t)b * n;
      long double f = 1.0L;   // sg^j
      for (int j = 0; j <= K; ++j, f *= sg) put(n * j, c, f * (long double)w[0], 1.0 / K);
      f = 1.0L;
      for (int e = 1; e <= K; ++e, f *= sg)
        for (int s = 1; s < n; ++s) put(n * (e - 1) + s, c, f * (long double)w[s], 1.0 / K);
    }
    return 0;
  }
  // k = 0, l = 1..n-1: zero at the nodes, ((-P)^(e-1) e^(l))_s in element e
  for (int l = 1; l < n; ++l) {
    const int c = l - 1;
    for (int e = 1; e <= K; ++e)
      for (int s = 1; s < n; ++s) {
        const int si = (e & 1) ? s : n - s;
        const long double v = (long double)d->E[(size_t)(si - 1) * (n - 1) + (l - 1)];
        put(n * (e - 1) + s - 1, c, (e & 1) ? v : -v, 1.0 / K);
      }
  }
  // k = 1..K-1, l = 1..n: sin(pi k j / K) at node j, and
  // sin(pi k (e-1) / K) p_s + sin(pi k e / K) p_(n-s) in element e
  for (int k = 1; k < K; ++k)
    for (int l = 1; l <= n; ++l) {
      const int c = (n - 1) + (l - 1) * (K - 1) + (k - 1);
      const double norm = d->inorm[(size_t)(k - 1) * n + (l - 1)];
      const double* p = d->p.data() + ((size_t)(k - 1) * n + (l - 1)) * (n - 1);
      for (int j = 1; j < K; ++j) put(n * j - 1, c, sine((long long)k * j), norm);
      for (int e = 1; e <= K; ++e)
        for (int s = 1; s < n; ++s) {
          const long double v = sine((long long)k * (e - 1)) * (long double)p[s - 1] +
                                sine((long long)k * e) * (long double)p[n - s - 1];
          put(n * (e - 1) + s - 1, c, v, norm);
        }
    }
  return 0;
}

int plan1d_build_neumann(int n, int K, Plan1DData* out) {
  if (K < 2 || K > 1024) return -1;
  // the Dirichlet tables of (n, K): p_k^(l), 1 / ||s_k^(l)||^2, the
  // eigenvalues of k = 1..K-1, twiddles, sines, local and Gauss tables
  if (plan1d_build(n, K, out) != 0) return -1;
  const int nb = n + 1, m = n * K + 1;
  std::vector<q128> A, C, gx, gw, Bq, Dq;
  local_matrices(n, A, C, gx, gw, Bq, Dq);
  std::vector<double> lam(m, 0.0);
  for (int l = 0; l < n; ++l)
    for (int k = 1; k < K; ++k)
      lam[(size_t)l * (K - 1) + (k - 1)] = out->lam[(size_t)(n - 1) + (size_t)l * (K - 1) + (k - 1)];
  // Band edges theta = 0 (sg = 1) and theta = pi (sg = -1): a cell
  // (node a, interior points w_1..w_{n-1}) repeated with the factor sg^j
  // maps to the element values (a, w, sg a); the Neumann vectors among them
  // are the even ones, w_s = sg w_{n-s} (the reflection about a node maps
  // point s of one element to point n-s of its neighbour).
  out->band.assign((size_t)(n + 1) * n, 0.0);
  int b = 0;
  for (int edge = 0; edge < 2; ++edge) {
    const int sg = edge == 0 ? 1 : -1;
    auto cell = [&](const std::vector<q128>& M) {
      std::vector<q128> X((size_t)n * n, 0);
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
          q128 v = M[r * nb + c];
          if (c == 0) v += sg * M[r * nb + n];
          if (r == 0) v += sg * M[n * nb + c];
          if (r == 0 && c == 0) v += M[n * nb + n];
          X[r * n + c] = v;
        }
      return X;
    };
    const std::vector<q128> Ac = cell(A), Cc = cell(C);
    // basis of the even cells: the node, then e_s + sg e_{n-s} (s < n-s),
    // then the middle point for even n at theta = 0
    std::vector<std::vector<q128>> basis;
    {
      std::vector<q128> e(n, 0);
      e[0] = 1;
      basis.push_back(e);
    }
    for (int s2 = 1; s2 < n; ++s2) {
      std::vector<q128> e(n, 0);
      if (2 * s2 < n) {
        e[s2] = 1;
        e[n - s2] = sg;
        basis.push_back(e);
      } else if (2 * s2 == n && sg == 1) {
        e[s2] = 1;
        basis.push_back(e);
      }
    }
    const int ne = (int)basis.size();
    std::vector<q128> Ar((size_t)ne * ne, 0), Cr((size_t)ne * ne, 0);
    for (int i = 0; i < ne; ++i)
      for (int j = 0; j < ne; ++j) {
        q128 sa = 0, sc = 0;
        for (int r = 0; r < n; ++r)
          for (int c = 0; c < n; ++c) {
            sa += basis[i][r] * Ac[r * n + c] * basis[j][c];
            sc += basis[i][r] * Cc[r * n + c] * basis[j][c];
          }
        Ar[i * ne + j] = sa;
        Cr[i * ne + j] = sc;
      }
    std::vector<q128> lr, Er;
    interior_eigen(ne, Ar, Cr, lr, Er);   // ascending, y^T Cr y = 1, so w^T Cc w = 1
    for (int col = 0; col < ne; ++col, ++b) {
      std::vector<q128> w(n, 0);
      for (int i = 0; i < ne; ++i)
        for (int s2 = 0; s2 < n; ++s2) w[s2] += basis[i][s2] * Er[i * ne + col];
      // sign: the lowest-index entry of at least half the largest magnitude is positive
      q128 big = 0;
      for (int s2 = 0; s2 < n; ++s2) big = fmaxq(big, fabsq(w[s2]));
      int at = 0;
      while (fabsq(w[at]) < big / 2) ++at;
      const q128 sgn = w[at] < 0 ? -1 : 1;
      for (int s2 = 0; s2 < n; ++s2) out->band[(size_t)b * n + s2] = (double)(sgn * w[s2]);
      // the constants span the kernel of A: lambda = 0 exactly
      lam[(size_t)n * (K - 1) + b] = edge == 0 && col == 0 ? 0.0 : (double)lr[col];
    }
    if (edge == 0) out->nb0 = ne;
  }
  out->lam = lam;
  out->bc = 2;
  out->m = m;
  return 0;
}

}  // namespace hofem
