// FP64 GEMM with gathered / scattered columns for the kiFMM's small dense
// operators: the two pseudo-inverse factors (Section 2.1.1) and the M2M /
// L2L translations (Section 2.2).
//
// The operators have few rows (n_s = 152 at p = 6, or 8 n_s for L2L) and the
// data has many columns (boxes x charge vectors), so a workgroup owns 64
// data columns and a block of 80 operator rows: each of its four waves
// computes 16 data columns x 80 rows on v_mfma_f64_16x16x4f64 (five 16 x 16
// accumulator tiles), which leaves registers for four workgroups per CU.  The product runs in transposed form - data columns
// are the MFMA rows - so the sixteen lanes holding one accumulator row store
// sixteen consecutive entries of one output column.  K is staged through LDS
// sixteen at a time, with the next slice's global loads issued before the
// current slice's MFMAs.
//
// Coarse tree levels have few columns; there the K range is split over
// several workgroups that write partial products, and a second kernel sums
// the partials in a fixed order (deterministic) and applies the scatter.
#include <algorithm>

#include "group.h"
#include "kernels.h"

namespace kifmm {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kMT = 5;             // 16-row MFMA tiles per wave along the operator rows
constexpr int kBM = 16 * kMT;      // 80 operator rows per workgroup
constexpr int kBN = 64;            // data columns per workgroup (16 per wave)
constexpr int kBK = 16;
constexpr int64_t kSplitTarget = 512;  // split K below this many workgroups
constexpr int kALoads = kBK * kBM / 256;  // operator values per thread per K slice

// n / f.d and n % f.d for n < 2^32
__device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f, uint32_t& r) {
  uint32_t q = __umulhi(n, f.m);
  r = n - q * f.d;
  if (r >= f.d) {
    ++q;
    r -= f.d;
  }
  return q;
}

__device__ inline void col_split(int64_t col, int nvec, const FastDiv& fv, int64_t& b, int& v) {
  if (nvec == 1) {
    b = col;
    v = 0;
  } else {
    uint32_t r;
    b = (int64_t)fdiv((uint32_t)col, fv, r);
    v = (int)r;
  }
}

// Workgroup (bx, by, bz): data columns bx * 64.., operator rows by * 80..,
// K range [bz * kchunk, ..) of a split product; with `partial` set the raw
// sums go to partial[bz][col][m] (m < M) instead of C.
__device__ __forceinline__ void gemm64_body(const Gemm64& g, int kchunk, double* partial, int64_t bx,
                                            int by, int bz) {
  __shared__ double As[kBK][kBM + 2];  // operator, k-major
  __shared__ double Bs[kBK][kBN + 2];  // data columns, k-major
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int l16 = lane % 16, g4 = lane / 16;
  const int m0 = by * kBM;
  const int64_t n0 = bx * kBN;
  const int64_t ncols = g.nbox * g.nvec;
  const int kz0 = bz * kchunk;
  const int kz1 = min(g.K, kz0 + kchunk);
  v4d acc[kMT];
#pragma unroll
  for (int j = 0; j < kMT; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};

  // data loads: four consecutive k of one column per thread and K slice; the
  // column's (box, vector) split is computed once
  const int cs = tid >> 2, kq = (tid & 3) * 4;
  const int64_t mycol = n0 + cs;
  const bool col_ok = mycol < ncols;
  int64_t cb_box = 0;
  int cb_v = 0;
  if (col_ok) col_split(mycol, g.nvec, g.div_nvec, cb_box, cb_v);
  const int32_t* bmap_row = g.bmap ? g.bmap + cb_box * g.nsegk : nullptr;
  const double* bcol = g.B + (int64_t)cb_v * g.b_vec;
  const double* bdirect = g.B + cb_box * g.b_box + (int64_t)cb_v * g.b_vec;
  const bool single_seg = g.nsegk == 1 && bmap_row == nullptr;

  double ra[kALoads], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < kALoads; ++r) {
      const int idx = tid + 256 * r;
      const int kk = idx % kBK, mm = idx / kBK;
      const int m = m0 + mm, k = k0 + kk;
      ra[r] = (m < g.M && k < kz1) ? g.A[(int64_t)m * g.lda + k] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + kq + e;
      double val = 0.0;
      if (col_ok && k < kz1) {
        if (single_seg) {
          val = bdirect[k];
        } else {
          int seg = 0, kk2 = k;
          if (g.nsegk != 1) {
            uint32_t r;
            seg = (int)fdiv((uint32_t)k, g.div_ks, r);
            kk2 = (int)r;
          }
          const int64_t bb = bmap_row ? (int64_t)bmap_row[seg] : cb_box;
          if (bb >= 0) val = bcol[bb * g.b_box + kk2];
        }
      }
      rb[e] = val;
    }
  };

  fetch(kz0);
  for (int k0 = kz0; k0 < kz1; k0 += kBK) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kALoads; ++r) {
      const int idx = tid + 256 * r;
      As[idx % kBK][idx / kBK] = ra[r];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) Bs[kq + e][cs] = rb[e];
    __syncthreads();
    if (k0 + kBK < kz1) fetch(k0 + kBK);
#pragma unroll
    for (int ks = 0; ks < kBK; ks += 4) {
      const double a = Bs[ks + g4][wave * 16 + l16];
#pragma unroll
      for (int j = 0; j < kMT; ++j)
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, As[ks + g4][16 * j + l16], acc[j], 0, 0, 0);
    }
  }
  // lane holds data columns g4 + 4 e (of the wave's 16) and operator row l16
  // of each tile
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t col = n0 + wave * 16 + g4 + 4 * e;
    if (col >= ncols) continue;
    if (partial) {
      double* dst = partial + ((int64_t)bz * ncols + col) * g.M;
#pragma unroll
      for (int j = 0; j < kMT; ++j) {
        const int m = m0 + 16 * j + l16;
        if (m < g.M) dst[m] = acc[j][e];
      }
      continue;
    }
    int64_t b;
    int v;
    col_split(col, g.nvec, g.div_nvec, b, v);
    // destinations of the column's kMT entries first, then (accumulating)
    // all their old values in flight together, then the stores
    double* dst[kMT];
#pragma unroll
    for (int j = 0; j < kMT; ++j) {
      const int m = m0 + 16 * j + l16;
      dst[j] = nullptr;
      if (m >= g.M) continue;
      int seg = 0, mm = m;
      if (g.nsegm != 1) {
        uint32_t r;
        seg = (int)fdiv((uint32_t)m, g.div_ms, r);
        mm = (int)r;
      }
      const int64_t cb = g.cmap ? (int64_t)g.cmap[b * g.nsegm + seg] : b;
      if (cb >= 0) dst[j] = &g.C[cb * g.c_box + (int64_t)v * g.c_vec + mm];
    }
    double old[kMT];
#pragma unroll
    for (int j = 0; j < kMT; ++j) old[j] = (g.accumulate && dst[j]) ? *dst[j] : 0.0;
#pragma unroll
    for (int j = 0; j < kMT; ++j)
      if (dst[j]) *dst[j] = old[j] + g.alpha * acc[j][e];
  }
}

__global__ __launch_bounds__(256, 4) void gemm64_kernel(Gemm64 g, int kchunk, double* partial) {
  gemm64_body(g, kchunk, partial, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Grouped: workgroup b of job j (pre[j] <= b < pre[j + 1]) is workgroup
// b - pre[j] of that job's gx x gy x split grid (x fastest).
__global__ __launch_bounds__(256, 4) void gemm64_group_kernel(const GemmJob* __restrict__ jobs,
                                                              const int64_t* __restrict__ pre, int nj) {
  int64_t b;
  const GemmJob j = jobs[group_job(pre, nj, b)];
  const int64_t per_z = j.gx * j.gy;
  const int bz = (int)(b / per_z);
  const int64_t r = b - (int64_t)bz * per_z;
  const int by = (int)(r / j.gx);
  gemm64_body(j.g, j.kchunk, j.split > 1 ? j.g.work : nullptr, r - (int64_t)by * j.gx, by, bz);
}

// Sum the split-K partials in order z = 0, 1, ... and scatter like the GEMM.
__device__ __forceinline__ void gemm64_reduce_body(const Gemm64& g, int nsplit,
                                                   const double* __restrict__ partial, int64_t blk) {
  const int64_t ncols = g.nbox * g.nvec;
  const int64_t total = ncols * g.M;  // < 2^32 (checked by the launcher)
  const int64_t i = blk * 256 + threadIdx.x;
  if (i >= total) return;
  uint32_t mr;
  const int64_t col = fdiv((uint32_t)i, g.div_M, mr);
  const int m = (int)mr;
  // eight partials in flight at a time, summed in order z = 0, 1, ...
  double sum = 0.0;
  int z = 0;
  for (; z + 8 <= nsplit; z += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = partial[(int64_t)(z + u) * total + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += t[u];
  }
  for (; z < nsplit; ++z) sum += partial[(int64_t)z * total + i];
  int64_t b;
  int v;
  col_split(col, g.nvec, g.div_nvec, b, v);
  int seg = 0, mm = m;
  if (g.nsegm != 1) {
    uint32_t r;
    seg = (int)fdiv((uint32_t)m, g.div_ms, r);
    mm = (int)r;
  }
  const int64_t cb = g.cmap ? (int64_t)g.cmap[b * g.nsegm + seg] : b;
  if (cb < 0) return;
  double* dst = &g.C[cb * g.c_box + (int64_t)v * g.c_vec + mm];
  const double val = g.alpha * sum;
  *dst = g.accumulate ? *dst + val : val;
}

__global__ __launch_bounds__(256) void gemm64_reduce_kernel(Gemm64 g, int nsplit,
                                                            const double* __restrict__ partial) {
  gemm64_reduce_body(g, nsplit, partial, blockIdx.x);
}

// Grouped reduction: jobs with split > 1 only; ceil(M x columns / 256)
// workgroups each.
__global__ __launch_bounds__(256) void gemm64_reduce_group_kernel(const GemmJob* __restrict__ jobs,
                                                                  const int64_t* __restrict__ pre, int nj) {
  int64_t b;
  const GemmJob j = jobs[group_job(pre, nj, b)];
  gemm64_reduce_body(j.g, j.split, j.g.work, b);
}

FastDiv make_div(int d) {
  FastDiv f;
  f.d = (uint32_t)d;
  f.m = d == 1 ? 0xffffffffu : (uint32_t)((uint64_t(1) << 32) / (uint64_t)d);
  return f;
}

}  // namespace

int64_t gemm64_max_work_elems() { return 2 * kSplitTarget * kBN * kBM; }

hipError_t plan_gemm64(const Gemm64& g0, GemmJob& job) {
  Gemm64& g = job.g;
  g = g0;
  job.gx = job.gy = job.split = job.kchunk = 0;
  const int64_t ncols = g.nbox * g.nvec;
  if (ncols == 0 || g.M == 0) return hipSuccess;
  if (ncols >= ((int64_t)1 << 31) || g.ks < 1 || g.ms < 1 || g.nvec < 1) return hipErrorInvalidValue;
  g.div_ks = make_div(g.ks);
  g.div_ms = make_div(g.ms);
  g.div_nvec = make_div(g.nvec);
  g.div_M = make_div(g.M);
  const int64_t gx = (ncols + kBN - 1) / kBN, gy = (g.M + kBM - 1) / kBM;
  // split K when the grid cannot fill the chip, within the workspace
  const int64_t slices = (g.K + kBK - 1) / kBK;
  int64_t split = 1;
  const int64_t target = kSplitTarget;
  // (the reduction indexes (column, row) pairs in 32 bits)
  if (g.work && gx * gy < target && slices >= 4 && ncols * g.M < ((int64_t)1 << 32)) {
    split = std::min<int64_t>((target + gx * gy - 1) / (gx * gy), slices / 2);
    const int64_t cap = g.work_elems / (ncols * g.M);
    split = std::max<int64_t>(1, std::min(split, cap));
  }
  const int kchunk = (int)(((slices + split - 1) / split) * kBK);
  split = (g.K + kchunk - 1) / kchunk;
  job.gx = gx;
  job.gy = (int)gy;
  job.split = (int)split;
  job.kchunk = kchunk;
  return hipSuccess;
}

int64_t gemm64_job_blocks(const GemmJob& j) { return j.gx * j.gy * j.split; }
int64_t gemm64_reduce_blocks(const GemmJob& j) {
  return j.split > 1 ? (j.g.nbox * j.g.nvec * j.g.M + 255) / 256 : 0;
}

hipError_t launch_gemm64(const Gemm64& g0, hipStream_t stream) {
  GemmJob job;
  hipError_t e = plan_gemm64(g0, job);
  if (e != hipSuccess || job.split == 0) return e;
  const Gemm64& g = job.g;
  dim3 grid((unsigned)job.gx, (unsigned)job.gy, (unsigned)job.split);
  if (job.split == 1) {
    gemm64_kernel<<<grid, 256, 0, stream>>>(g, job.kchunk, nullptr);
    return hipGetLastError();
  }
  gemm64_kernel<<<grid, 256, 0, stream>>>(g, job.kchunk, g.work);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  gemm64_reduce_kernel<<<(unsigned)gemm64_reduce_blocks(job), 256, 0, stream>>>(g, job.split, g.work);
  return hipGetLastError();
}

hipError_t launch_gemm64_group(const GemmJob* jobs, const int64_t* pre, int nj, int64_t blocks,
                               bool reduce, hipStream_t stream) {
  if (blocks == 0) return hipSuccess;
  if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (reduce)
    gemm64_reduce_group_kernel<<<(unsigned)blocks, 256, 0, stream>>>(jobs, pre, nj);
  else
    gemm64_group_kernel<<<(unsigned)blocks, 256, 0, stream>>>(jobs, pre, nj);
  return hipGetLastError();
}

}  // namespace kifmm
