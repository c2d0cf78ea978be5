// One-shot randomized SVD of K_fat on the device (Section 3.1, after Halko,
// Martinsson and Tropp): a Gaussian test matrix, oversampling, no power
// iterations.  The three products with the long dimension n = 316 n_s run
// on the FP64 MFMA GEMM of k_gemm.hip; the small factorizations stay on the
// host (Householder QR of the m x l sample, Jacobi SVD of the l x l Gram
// matrix).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace kifmm {

namespace {

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds of two
// 32 x 32 -> 64-bit products with multipliers 0xD2511F53 and 0xCD9E8D57,
// the key bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between
// rounds.
__device__ inline uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = uint4{(uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k.y,
              (uint32_t)p0};
  }
  return c;
}

// (0, 1]: 53 random bits, never zero (the logarithm below stays finite)
__device__ inline double unit_open0(uint32_t hi, uint32_t lo) {
  const uint64_t b = ((uint64_t)hi << 21) ^ (uint64_t)(lo >> 11);
  return ((double)(b & ((uint64_t(1) << 53) - 1)) + 1.0) * 0x1.0p-53;
}

// out[i], i < n: standard normal numbers, two per Philox call (Box-Muller),
// counter = pair index, key = seed.
__global__ void gaussian_kernel(double* __restrict__ out, int64_t n, uint64_t seed) {
  const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * pair >= n) return;
  const uint4 r = philox4x32_10(uint4{(uint32_t)pair, (uint32_t)(pair >> 32), 0u, 0u},
                                uint2{(uint32_t)seed, (uint32_t)(seed >> 32)});
  const double u1 = unit_open0(r.x, r.y), u2 = unit_open0(r.z, r.w);
  const double rad = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  out[2 * pair] = rad * c;
  if (2 * pair + 1 < n) out[2 * pair + 1] = rad * s;
}

// C[col][m] = sum_k A[m][k] B[col][k]: A (M x K, row stride lda), B (ncols x
// K, row stride ldb), C (ncols x M, row stride ldc)
hipError_t dense_gemm(const double* A, int M, int K, int lda, const double* B, int64_t ncols,
                      int ldb, double* C, int ldc, double* work, int64_t work_elems,
                      hipStream_t s) {
  Gemm64 g;
  g.A = A;
  g.M = M;
  g.K = K;
  g.lda = lda;
  g.alpha = 1.0;
  g.B = B;
  g.ks = K;
  g.nsegk = 1;
  g.bmap = nullptr;
  g.b_box = ldb;
  g.b_vec = 0;
  g.C = C;
  g.ms = M;
  g.nsegm = 1;
  g.cmap = nullptr;
  g.c_box = ldc;
  g.c_vec = 0;
  g.nbox = ncols;
  g.nvec = 1;
  g.accumulate = 0;
  g.work = work;
  g.work_elems = work_elems;
  return launch_gemm64(g, s);
}

// Thin Q (m x l, row-major, orthonormal columns) of Y (m x l, row-major),
// by Householder reflections.
void householder_q(const std::vector<double>& Y, int m, int l, std::vector<double>& Q) {
  std::vector<double> R(Y);  // reduced in place
  std::vector<std::vector<double>> vs((size_t)l);
  for (int j = 0; j < l; ++j) {
    double nrm = 0;
    for (int i = j; i < m; ++i) nrm += R[(size_t)i * l + j] * R[(size_t)i * l + j];
    nrm = std::sqrt(nrm);
    std::vector<double>& v = vs[(size_t)j];
    v.assign((size_t)m, 0.0);
    if (nrm == 0.0) continue;
    const double alpha = R[(size_t)j * l + j] >= 0 ? -nrm : nrm;
    double vn = 0;
    for (int i = j; i < m; ++i) {
      v[(size_t)i] = R[(size_t)i * l + j] - (i == j ? alpha : 0.0);
      vn += v[(size_t)i] * v[(size_t)i];
    }
    if (vn == 0.0) {
      v.assign((size_t)m, 0.0);
      continue;
    }
    const double sc = std::sqrt(2.0 / vn);
    for (int i = j; i < m; ++i) v[(size_t)i] *= sc;  // H = I - v v^T
    for (int c = j; c < l; ++c) {
      double dot = 0;
      for (int i = j; i < m; ++i) dot += v[(size_t)i] * R[(size_t)i * l + c];
      for (int i = j; i < m; ++i) R[(size_t)i * l + c] -= dot * v[(size_t)i];
    }
  }
  // Q = H_0 H_1 ... H_{l-1} applied to the first l columns of the identity
  Q.assign((size_t)m * l, 0.0);
  for (int j = 0; j < l; ++j) Q[(size_t)j * l + j] = 1.0;
  for (int j = l - 1; j >= 0; --j) {
    const std::vector<double>& v = vs[(size_t)j];
    for (int c = 0; c < l; ++c) {
      double dot = 0;
      for (int i = j; i < m; ++i) dot += v[(size_t)i] * Q[(size_t)i * l + c];
      for (int i = j; i < m; ++i) Q[(size_t)i * l + c] -= dot * v[(size_t)i];
    }
  }
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes); }
  double* d() const { return static_cast<double*>(p); }
};

}  // namespace

kifmm_status rsvd_left_device(const double* A, int m, int n, const SvdOptions& o,
                              std::vector<double>& U, std::vector<double>& s) {
  const int rank = std::max(1, std::min(m, o.rank > 0 ? o.rank : (m + 1) / 2));
  const int l = std::min(m, rank + o.oversample);
  // A^T, row-major n x m, for the product Q^T A
  std::vector<double> At((size_t)n * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) At[(size_t)j * m + i] = A[(size_t)i * n + j];
  if (hipSetDevice(o.device) != hipSuccess) return fail(KIFMM_EDEVICE, "hipSetDevice failed");
  const int64_t work_elems = (int64_t)8 << 20;
  DevBuf dA, dAt, dOm, dYt, dQt, dB, dG, dW;
  if (dA.alloc(sizeof(double) * (size_t)m * n) != hipSuccess ||
      dAt.alloc(sizeof(double) * (size_t)m * n) != hipSuccess ||
      dOm.alloc(sizeof(double) * (size_t)l * n) != hipSuccess ||
      dYt.alloc(sizeof(double) * (size_t)l * m) != hipSuccess ||
      dQt.alloc(sizeof(double) * (size_t)l * m) != hipSuccess ||
      dB.alloc(sizeof(double) * (size_t)l * n) != hipSuccess ||
      dG.alloc(sizeof(double) * (size_t)l * l) != hipSuccess ||
      dW.alloc(sizeof(double) * (size_t)work_elems) != hipSuccess)
    return fail(KIFMM_ENOMEM, "randomized SVD: device allocation failed");
  hipStream_t st = nullptr;  // the null stream: precompute is synchronous
  auto check = [](hipError_t e) { return e == hipSuccess; };
  bool ok = check(hipMemcpy(dA.p, A, sizeof(double) * (size_t)m * n, hipMemcpyHostToDevice)) &&
            check(hipMemcpy(dAt.p, At.data(), sizeof(double) * (size_t)m * n, hipMemcpyHostToDevice));
  // Omega^T (l x n): row c is the c-th test vector
  const int64_t total = (int64_t)l * n;
  if (ok) {
    gaussian_kernel<<<(unsigned)((total / 2 + 256) / 256), 256, 0, st>>>(dOm.d(), total, o.seed);
    ok = check(hipGetLastError());
  }
  // Y^T[c][i] = sum_k A[i][k] Omega[k][c]
  if (ok) ok = check(dense_gemm(dA.d(), m, n, n, dOm.d(), l, n, dYt.d(), m, dW.d(), work_elems, st));
  std::vector<double> Yt((size_t)l * m);
  if (ok) ok = check(hipMemcpy(Yt.data(), dYt.p, sizeof(double) * Yt.size(), hipMemcpyDeviceToHost));
  if (!ok) return fail(KIFMM_EDEVICE, "randomized SVD: sampling failed");
  std::vector<double> Y((size_t)m * l), Q;
  for (int c = 0; c < l; ++c)
    for (int i = 0; i < m; ++i) Y[(size_t)i * l + c] = Yt[(size_t)c * m + i];
  householder_q(Y, m, l, Q);
  std::vector<double> Qt((size_t)l * m);
  for (int i = 0; i < m; ++i)
    for (int c = 0; c < l; ++c) Qt[(size_t)c * m + i] = Q[(size_t)i * l + c];
  // B[c][k] = sum_i A^T[k][i] Q^T[c][i] (l x n), then G = B B^T (l x l)
  ok = check(hipMemcpy(dQt.p, Qt.data(), sizeof(double) * Qt.size(), hipMemcpyHostToDevice)) &&
       check(dense_gemm(dAt.d(), n, m, m, dQt.d(), l, m, dB.d(), n, dW.d(), work_elems, st)) &&
       check(dense_gemm(dB.d(), l, n, n, dB.d(), l, n, dG.d(), l, dW.d(), work_elems, st));
  std::vector<double> G((size_t)l * l);
  if (ok) ok = check(hipMemcpy(G.data(), dG.p, sizeof(double) * G.size(), hipMemcpyDeviceToHost));
  if (!ok) return fail(KIFMM_EDEVICE, "randomized SVD: projection failed");
  // G = W diag(sigma^2) W^T (symmetric positive semi-definite: its SVD is
  // its eigen-decomposition); U = Q W, keeping the leading `rank` columns
  for (int i = 0; i < l; ++i)
    for (int j = 0; j < i; ++j) G[(size_t)i * l + j] = G[(size_t)j * l + i] = 0.5 * (G[(size_t)i * l + j] + G[(size_t)j * l + i]);
  std::vector<double> W, s2, V;
  if (!svd(G.data(), l, l, W, s2, V)) return fail(KIFMM_ENUMERIC, "randomized SVD: Jacobi SVD did not converge");
  U.assign((size_t)m * rank, 0.0);
  s.assign((size_t)rank, 0.0);
  for (int j = 0; j < rank; ++j) s[(size_t)j] = std::sqrt(std::max(s2[(size_t)j], 0.0));
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < rank; ++j) {
      double acc = 0;
      for (int c = 0; c < l; ++c) acc += Q[(size_t)i * l + c] * W[(size_t)c * l + j];
      U[(size_t)i * rank + j] = acc;
    }
  return KIFMM_OK;
}

}  // namespace kifmm
