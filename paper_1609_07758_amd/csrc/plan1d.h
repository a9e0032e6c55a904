// Internal interface of the binary128 host precompute (plan1d.cpp).
#pragma once

#include <vector>

namespace hofem {

// FP64 tables of the 1D eigen data for one (n, K), each value rounded once
// from binary128.  Coefficient index q of a line (length m = nK - 1):
//   k = 0, l = 1..n-1      ->  q = l - 1
//   k = 1..K-1, l = 1..n   ->  q = (n - 1) + (l - 1)(K - 1) + (k - 1)
struct Plan1DData {
  int bc = 0;                    // 0: Dirichlet, 1: periodic, 2: Neumann
  int n = 0, K = 0, m = 0;
  std::vector<double> A, C;      // local stiffness / mass on [-1,1], (n+1)^2 row major
  std::vector<double> lam;       // scaled eigenvalues in coefficient order (m)
  std::vector<double> p;         // p_k^(l): [(k-1) n + (l-1)] * (n-1) + i, i = 0..n-2
  std::vector<double> inorm;     // 1 / ||s_k^(l)||_C^2: [(k-1) n + (l-1)]
  std::vector<double> E;         // e^(l) as columns: E[i (n-1) + (l-1)]
  std::vector<double> lam0;      // interior eigenvalues (n-1)
  std::vector<double> tw;        // cos, sin of 2 pi t / K, t = 0..K-1 (interleaved)
  std::vector<double> sn;        // sin(pi t / K), t = 0..K-1
  // (n+1)-point Gauss-Legendre rule on [-1, 1] and the Lagrange basis there:
  std::vector<double> gx, gw;    // nodes, weights (n+1)
  std::vector<double> B, D;      // B[q (n+1) + r] = e_r(x_q), D[q (n+1) + r] = e_r'(x_q)
  // differentiation on the Gauss nodes: Dh[q (n+1) + p] = g_p'(x_q) for the
  // Lagrange basis g_p of the Gauss nodes (Dh = D B^-1; rows sum to zero)
  std::vector<double> Dh;

  // Dirichlet axes whose K is not a power of two (no FFT): the unnormalised
  // eigenvectors s_k^(l) of Theorem 1 as the columns of S (m x m, row q =
  // unknown, column c = coefficient index) and St = S diag(1 / ||s_c||_C^2)
  // (1/K for the k = 0 columns), so that the coefficients are St^T y and the
  // inverse transform S c
  int dense = 0;
  std::vector<double> S, St;

  // Neumann axes (m = nK + 1, lam in the Neumann coefficient order): the
  // n + 1 band-edge eigenvectors as cells (node value, interior points
  // 1..n-1), band[b n + s]; b < nb0 at theta = 0, the rest at theta = pi;
  // w^T C_cell w = 1, so that the axis vector has ||v||_C^2 = K
  std::vector<double> band;
  int nb0 = 0;

  // periodic axes: Bloch eigenvectors w_{k,l} (cell components s = 0..n-1:
  // node j, interior points of element j+1) for k = 0..K/2, index
  // (k n + l) n + s, real and imaginary parts; w^H C^(k) w = 1
  std::vector<double> wr, wi;
};

// Largest m of a dense (non-power-of-two K) axis: S and St take 2 m^2 doubles.
constexpr int kDenseMax = 4095;

// Returns 0 on success, -1 for unsupported (n, K).
int plan1d_build(int n, int K, Plan1DData* out);
// Fills S and St of a plan (m <= kDenseMax; columns in the plan's
// coefficient order, so that the coefficients are St^T y and the inverse
// S c); 0 on success.
int plan1d_build_dense(Plan1DData* d);
// Periodic axis (m = nK unknowns: node j at q = n j, interior point s of
// element j+1 at q = n j + s, j = 0..K-1): eigenvalues in the coefficient
// order q = l K + t (t = 0: k = 0; t = 2k-1, 2k: real and imaginary parts of
// wave number k = 1..K/2-1; t = K-1: k = K/2) and the Bloch eigenvectors.
// Returns 0 on success, -1 for unsupported (n, K).
int plan1d_build_periodic(int n, int K, Plan1DData* out);
// Neumann axis of K elements (m = nK + 1 unknowns, the points g h / n,
// g = 0..nK, boundary nodes included).  For k = 1..K-1 its eigenvectors are
// the cosine counterparts of Theorem 1's (node j: cos(pi k j / K); point s
// of element e: cos(pi k (e-1) / K) p_s + cos(pi k e / K) p_{n-s}) with the
// Dirichlet eigenvalues, p and norms of wave number k; the other n + 1 are
// the even band-edge cells at theta = 0 and pi.  Coefficient order:
// q = (l-1)(K-1) + (k-1) for k = 1..K-1, l = 1..n, then the band-edge
// vectors, q = n(K-1) + b.  Returns 0 on success, -1 for unsupported (n, K).
int plan1d_build_neumann(int n, int K, Plan1DData* out);

}  // namespace hofem
