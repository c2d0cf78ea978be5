// Device-side re-setup for moving points: bin new positions into the
// current tree's leaves and sort them stably by leaf (Morton order of the
// leaves, then original index), the order the host tree build produces.
#include "kernels.h"

namespace kifmm {

namespace {

constexpr int kSortThreads = 256;  // one element per thread per sub-tile
constexpr int kSortTiles = 8;      // sub-tiles per workgroup
constexpr int kSortChunk = kSortThreads * kSortTiles;
constexpr int kScanThreads = 1024;

__device__ inline uint64_t morton(int64_t ax, int64_t ay, int64_t az, int level) {
  uint64_t m = 0;
  for (int b = 0; b < level; ++b) {
    m |= (uint64_t)((ax >> b) & 1) << (3 * b);
    m |= (uint64_t)((ay >> b) & 1) << (3 * b + 1);
    m |= (uint64_t)((az >> b) & 1) << (3 * b + 2);
  }
  return m | ((uint64_t)1 << (3 * level));
}

// leaf[i]: index of point i's leaf in the sorted keys, or -1 with *bad = 1
// (outside the domain cube, or a leaf the tree does not have)
__global__ void point_leaf_kernel(const double* __restrict__ pts, int64_t n,
                                  const uint64_t* __restrict__ keys, int64_t n_leaf, int depth,
                                  double ox, double oy, double oz, double w,
                                  int32_t* __restrict__ leaf, int32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double o[3] = {ox, oy, oz};
  const double scale = ldexp(1.0, depth);
  const int64_t top = ((int64_t)1 << depth) - 1;
  int64_t a[3];
  bool ok = true;
  for (int c = 0; c < 3; ++c) {
    const double u = (pts[3 * i + c] - o[c]) / w;
    ok = ok && (u >= 0.0 && u <= 1.0);
    const int64_t ai = ok ? (int64_t)floor(u * scale) : 0;
    a[c] = ai > top ? top : ai;
  }
  int32_t idx = -1;
  if (ok) {
    const uint64_t key = morton(a[0], a[1], a[2], depth);
    int64_t lo = 0, hi = n_leaf;  // first index with keys[idx] >= key
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    if (lo < n_leaf && keys[lo] == key) idx = (int32_t)lo;
  }
  leaf[i] = idx;
  if (idx < 0) *bad = 1;
}

__global__ void iota_kernel(int32_t* __restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int32_t)i;
}

__global__ void zero_kernel(int32_t* __restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = 0;
}

// digit histogram of one workgroup's chunk: hist[digit * nb + block]
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(
    const int32_t* __restrict__ key, int64_t n, int shift, int32_t* __restrict__ hist, int64_t nb) {
  __shared__ int32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int s = 0; s < kSortTiles; ++s) {
    const int64_t i = base + s * kSortThreads + tid;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)tid * nb + blockIdx.x] = h[tid];
}

// exclusive prefix sum of a[0, m) in place (one workgroup)
__global__ __launch_bounds__(kScanThreads) void scan_kernel(int32_t* __restrict__ a, int64_t m) {
  __shared__ int32_t part[kScanThreads];
  const int tid = threadIdx.x;
  const int64_t per = (m + kScanThreads - 1) / kScanThreads;
  const int64_t lo = min((int64_t)tid * per, m), hi = min(lo + per, m);
  int32_t sum = 0;
  for (int64_t i = lo; i < hi; ++i) sum += a[i];
  part[tid] = sum;
  __syncthreads();
  if (tid == 0) {
    int32_t run = 0;
    for (int k = 0; k < kScanThreads; ++k) {
      const int32_t v = part[k];
      part[k] = run;
      run += v;
    }
  }
  __syncthreads();
  int32_t run = part[tid];
  for (int64_t i = lo; i < hi; ++i) {
    const int32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

// stable scatter by one 8-bit digit: within a workgroup's chunk, elements
// keep their order (sub-tile, then wave, then lane); ranks among equal
// digits in a wave come from ballots, across waves from LDS counts
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const int32_t* __restrict__ key_in, const int32_t* __restrict__ val_in, int64_t n, int shift,
    const int32_t* __restrict__ offs, int64_t nb, int32_t* __restrict__ key_out,
    int32_t* __restrict__ val_out) {
  __shared__ int32_t cnt[256];
  __shared__ int32_t wc[kSortThreads / 64][256];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  cnt[tid] = offs[(int64_t)tid * nb + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  const uint64_t lt = (1ull << lane) - 1;
  for (int s = 0; s < kSortTiles; ++s) {
    for (int k = tid; k < (kSortThreads / 64) * 256; k += kSortThreads) (&wc[0][0])[k] = 0;
    __syncthreads();
    const int64_t i = base + s * kSortThreads + tid;
    const bool act = i < n;
    const int32_t kv = act ? key_in[i] : 0;
    const int dig = (kv >> shift) & 255;
    uint64_t m = __ballot(act);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1;
      const uint64_t bb = __ballot(act && bit);
      m &= bit ? bb : ~bb;
    }
    const int rank = __popcll(m & lt);
    if (act && rank == 0) wc[wave][dig] = __popcll(m);
    __syncthreads();
    if (act) {
      int pre = 0;
      for (int w2 = 0; w2 < wave; ++w2) pre += wc[w2][dig];
      const int32_t dst = cnt[dig] + pre + rank;
      key_out[dst] = kv;
      val_out[dst] = val_in[i];
    }
    __syncthreads();
    int32_t add = 0;
    for (int w2 = 0; w2 < kSortThreads / 64; ++w2) add += wc[w2][tid];
    cnt[tid] += add;
    __syncthreads();
  }
}

__global__ void leaf_count_kernel(const int32_t* __restrict__ leaf, int64_t n,
                                  int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&count[leaf[i]], 1);
}

__global__ void finish_kernel(const double* __restrict__ pts, const int32_t* __restrict__ order,
                              int64_t n, int64_t* __restrict__ perm, double* __restrict__ sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = order[i];
  perm[i] = j;
  for (int c = 0; c < 3; ++c) sorted[3 * i + c] = pts[3 * j + c];
}

__global__ void ranges_kernel(const int32_t* __restrict__ first, const int32_t* __restrict__ count,
                              int64_t n_leaf, int32_t* __restrict__ start, int32_t* __restrict__ end) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_leaf) return;
  start[i] = first[i];
  end[i] = first[i] + count[i];
}

unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_point_leaf(const double* pts, int64_t n, const uint64_t* leaf_keys,
                             int64_t n_leaf, int depth, const double origin[3], double width,
                             int32_t* leaf, int32_t* bad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  point_leaf_kernel<<<blocks(n, 256), 256, 0, s>>>(pts, n, leaf_keys, n_leaf, depth, origin[0],
                                                   origin[1], origin[2], width, leaf, bad);
  return hipGetLastError();
}

size_t sort_scratch_ints(int64_t n, int64_t n_leaf) {
  const int64_t nb = (n + kSortChunk - 1) / kSortChunk;
  return (size_t)(3 * n + 256 * nb + 2 * n_leaf);
}

hipError_t launch_sort_by_leaf(const double* pts, const int32_t* leaf, int64_t n, int64_t n_leaf,
                               int32_t* scratch, int64_t* perm, double* sorted, int32_t* start,
                               int32_t* end, hipStream_t s) {
  if (n <= 0 || n_leaf <= 0) return hipSuccess;
  if (n >= ((int64_t)1 << 31) || n_leaf >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int64_t nb = (n + kSortChunk - 1) / kSortChunk;
  int32_t* ka = scratch;            // keys (ping)
  int32_t* kb = ka + n;             // keys (pong)
  int32_t* va = kb + n;             // original indices (ping)
  int32_t* hist = va + n;           // [256][nb]
  int32_t* count = hist + 256 * nb; // [n_leaf]
  int32_t* first = count + n_leaf;  // [n_leaf]
  // the indices' pong buffer is perm's storage (room for 2 n int32)
  int32_t* vb = reinterpret_cast<int32_t*>(perm);
  int32_t* K[2] = {ka, kb};
  int32_t* V[2] = {va, vb};
  int bits = 1;
  while (((int64_t)1 << bits) < n_leaf) ++bits;
  const int passes = (bits + 7) / 8;
  hipError_t e = hipMemcpyAsync(ka, leaf, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  iota_kernel<<<blocks(n, 256), 256, 0, s>>>(va, n);
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p, in = p & 1, out = in ^ 1;
    radix_hist_kernel<<<(unsigned)nb, kSortThreads, 0, s>>>(K[in], n, shift, hist, nb);
    scan_kernel<<<1, kScanThreads, 0, s>>>(hist, 256 * nb);
    radix_scatter_kernel<<<(unsigned)nb, kSortThreads, 0, s>>>(K[in], V[in], n, shift, hist, nb,
                                                               K[out], V[out]);
  }
  // the sorted original indices; out of perm's storage before perm is written
  if (passes & 1) {
    e = hipMemcpyAsync(va, vb, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  const int32_t* order = va;
  finish_kernel<<<blocks(n, 256), 256, 0, s>>>(pts, order, n, perm, sorted);
  zero_kernel<<<blocks(n_leaf, 256), 256, 0, s>>>(count, n_leaf);
  leaf_count_kernel<<<blocks(n, 256), 256, 0, s>>>(leaf, n, count);
  e = hipMemcpyAsync(first, count, (size_t)n_leaf * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  scan_kernel<<<1, kScanThreads, 0, s>>>(first, n_leaf);
  ranges_kernel<<<blocks(n_leaf, 256), 256, 0, s>>>(first, count, n_leaf, start, end);
  return hipGetLastError();
}

}  // namespace kifmm
