// FP64 GEMM with gathered / scattered columns for the kiFMM's small dense
// operators: the two pseudo-inverse factors (Section 2.1.1) and the M2M /
// L2L translations (Section 2.2).  FP64 vector arithmetic: on MI355X the
// FP64 vector and matrix rates are equal, so no MFMA is used here.
//
// Tile: 64 rows x 64 columns per 256-thread workgroup, K in steps of 16
// staged through LDS.  Lane (tm, tn) owns rows tm + 16 i and columns
// tn + 16 j; consecutive lanes own consecutive rows so that stores of a
// column (contiguous in memory) coalesce.
#include "kernels.h"

namespace kifmm {

namespace {

constexpr int kBM = 64, kBN = 64, kBK = 16;

__global__ __launch_bounds__(256) void gemm64_kernel(Gemm64 g) {
  __shared__ double As[kBK][kBM + 1];
  __shared__ double Bs[kBK][kBN + 1];
  const int tid = threadIdx.x;
  const int tm = tid % 16, tn = tid / 16;
  const int m0 = blockIdx.y * kBM;
  const int64_t n0 = (int64_t)blockIdx.x * kBN;
  const int64_t ncols = g.nbox * g.nvec;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int k0 = 0; k0 < g.K; k0 += kBK) {
    // A tile: As[kk][mm] = A[m0 + mm][k0 + kk]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kk = tid % kBK, mm = tid / kBK + 16 * r;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.lda + k] : 0.0;
    }
    // B tile: Bs[kk][nn] = B(k0 + kk, n0 + nn), gathered
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kk = tid % kBK, nn = tid / kBK + 16 * r;
      const int64_t col = n0 + nn;
      const int k = k0 + kk;
      double val = 0.0;
      if (col < ncols && k < g.K) {
        const int64_t b = col / g.nvec;
        const int v = (int)(col - b * g.nvec);
        const int seg = k / g.ks, kk2 = k - seg * g.ks;
        const int64_t bb = g.bmap ? (int64_t)g.bmap[b * g.nsegk + seg] : b;
        if (bb >= 0) val = g.B[bb * g.b_box + (int64_t)v * g.b_vec + kk2];
      }
      Bs[kk][nn] = val;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kBK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tm + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = n0 + tn + 16 * j;
    if (col >= ncols) continue;
    const int64_t b = col / g.nvec;
    const int v = (int)(col - b * g.nvec);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = m0 + tm + 16 * i;
      if (m >= g.M) continue;
      const int seg = m / g.ms, mm = m - seg * g.ms;
      const int64_t cb = g.cmap ? (int64_t)g.cmap[b * g.nsegm + seg] : b;
      if (cb < 0) continue;
      double* dst = &g.C[cb * g.c_box + (int64_t)v * g.c_vec + mm];
      const double val = g.alpha * acc[i][j];
      *dst = g.accumulate ? *dst + val : val;
    }
  }
}

}  // namespace

hipError_t launch_gemm64(const Gemm64& g, hipStream_t stream) {
  const int64_t ncols = g.nbox * g.nvec;
  if (ncols == 0 || g.M == 0) return hipSuccess;
  dim3 grid((unsigned)((ncols + kBN - 1) / kBN), (unsigned)((g.M + kBM - 1) / kBM));
  gemm64_kernel<<<grid, 256, 0, stream>>>(g);
  return hipGetLastError();
}

}  // namespace kifmm
