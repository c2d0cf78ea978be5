// FP64 host linear algebra for the precomputation: one-sided Jacobi SVD
// (Hestenes rotations) and Householder QR for wide matrices.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

namespace kifmm {

namespace {

// One-sided Jacobi on the columns of G (m x n, column-major, m >= n).
// On return the columns of G are mutually orthogonal and V (n x n,
// column-major) holds the accumulated rotations.
bool jacobi_columns(std::vector<double>& G, int m, int n, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  const double eps = 2.220446049250313e-16;
  // columns whose squared norm falls below (eps ||A||_F)^2 are numerically
  // zero; rotating them against each other only stirs rounding noise
  double fro2 = 0;
  for (size_t i = 0; i < (size_t)m * n; ++i) fro2 += G[i] * G[i];
  const double negligible = eps * eps * fro2;
  // rotation threshold sqrt(m) eps (as in LAPACK's one-sided Jacobi); with
  // eps alone, rounding can flip one tiny rotation back and forth forever
  const double tol = std::sqrt((double)m) * eps;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p) {
      double* gp = &G[(size_t)p * m];
      for (int q = p + 1; q < n; ++q) {
        double* gq = &G[(size_t)q * m];
        double a = 0, b = 0, g = 0;
        for (int i = 0; i < m; ++i) {
          a += gp[i] * gp[i];
          b += gq[i] * gq[i];
          g += gp[i] * gq[i];
        }
        if (g == 0.0 || std::fabs(g) <= tol * std::sqrt(a * b)) continue;
        if (a < negligible || b < negligible) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t);
        const double s = c * t;
        for (int i = 0; i < m; ++i) {
          const double x = gp[i], y = gq[i];
          gp[i] = c * x - s * y;
          gq[i] = s * x + c * y;
        }
        double* vp = &V[(size_t)p * n];
        double* vq = &V[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    }
    if (!rotated) return true;
  }
  return false;
}

// SVD of a tall matrix given column-major (m x n, m >= n).
bool svd_tall_colmajor(std::vector<double> G, int m, int n, std::vector<double>& U,
                       std::vector<double>& s, std::vector<double>& V) {
  std::vector<double> W;
  if (!jacobi_columns(G, m, n, W)) return false;
  std::vector<double> norms(n);
  for (int j = 0; j < n; ++j) {
    double acc = 0;
    for (int i = 0; i < m; ++i) acc += G[(size_t)j * m + i] * G[(size_t)j * m + i];
    norms[j] = std::sqrt(acc);
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return norms[a] > norms[b]; });
  U.assign((size_t)m * n, 0.0);  // row-major m x n
  V.assign((size_t)n * n, 0.0);  // row-major n x n
  s.assign(n, 0.0);
  for (int jj = 0; jj < n; ++jj) {
    const int j = order[jj];
    s[jj] = norms[j];
    const double inv = norms[j] > 0 ? 1.0 / norms[j] : 0.0;
    for (int i = 0; i < m; ++i) U[(size_t)i * n + jj] = G[(size_t)j * m + i] * inv;
    for (int i = 0; i < n; ++i) V[(size_t)i * n + jj] = W[(size_t)j * n + i];
  }
  return true;
}

}  // namespace

bool svd(const double* A, int m, int n, std::vector<double>& U, std::vector<double>& s,
         std::vector<double>& V) {
  if (m >= n) {
    std::vector<double> G((size_t)m * n);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) G[(size_t)j * m + i] = A[(size_t)i * n + j];
    return svd_tall_colmajor(std::move(G), m, n, U, s, V);
  }
  // A^T = U' S V'^T  =>  A = V' S U'^T
  std::vector<double> G((size_t)n * m);  // A^T column-major (n x m) == A row-major
  std::copy(A, A + (size_t)m * n, G.begin());
  return svd_tall_colmajor(std::move(G), n, m, V, s, U);
}

bool svd_left_wide(const double* A, int m, int n, std::vector<double>& U, std::vector<double>& s) {
  if (n <= m) {
    std::vector<double> V;
    return svd(A, m, n, U, s, V);
  }
  // Householder QR of B = A^T (n x m).  B column-major equals A row-major.
  std::vector<double> B(A, A + (size_t)m * n);
  std::vector<double> v(n);
  for (int j = 0; j < m; ++j) {
    double* col = &B[(size_t)j * n];
    double nrm = 0;
    for (int i = j; i < n; ++i) nrm += col[i] * col[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double alpha = col[j] >= 0 ? -nrm : nrm;
    double vnorm2 = 0;
    for (int i = j; i < n; ++i) {
      v[i] = col[i];
      if (i == j) v[i] -= alpha;
      vnorm2 += v[i] * v[i];
    }
    if (vnorm2 == 0.0) continue;
    for (int k = j; k < m; ++k) {
      double* ck = &B[(size_t)k * n];
      double dot = 0;
      for (int i = j; i < n; ++i) dot += v[i] * ck[i];
      const double f = 2.0 * dot / vnorm2;
      for (int i = j; i < n; ++i) ck[i] -= f * v[i];
    }
  }
  // R (m x m, upper) sits in the top of B's columns; A = R^T Q^T.
  std::vector<double> Rt((size_t)m * m, 0.0);  // row-major R^T
  for (int k = 0; k < m; ++k)
    for (int i = 0; i <= k; ++i) Rt[(size_t)k * m + i] = B[(size_t)k * n + i];
  std::vector<double> V;
  return svd(Rt.data(), m, m, U, s, V);
}

}  // namespace kifmm
