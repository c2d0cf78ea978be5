// Device-side re-setup for moving points (the dynamic-particle setting of
// Section 5.1): the locational encoding of the points, their sort, the
// pruned box levels, the index pointers between leaves and points, the near
// and interaction lists, and the M2L maps (FFT-M2L source blocks and
// sibling-cluster halos, BLAS / dense target tiles with their transfer
// vectors).  Every structure equals the one the host tree build produces
// for the same points and domain, entry for entry.
//
// Codes are Morton codes without the sentinel bit (bit b of the x anchor at
// position 3b, of y at 3b + 1, of z at 3b + 2); level keys carry the
// sentinel at position 3l, as the host tree's keys do.
#include <algorithm>

#include "kernels.h"

namespace kifmm {

namespace {

constexpr int kSortThreads = 256;  // one element per thread per sub-tile
constexpr int kSortTiles = 8;      // sub-tiles per workgroup
constexpr int kSortChunk = kSortThreads * kSortTiles;
constexpr int kNumT = 316;         // transfer vectors of the M2L
constexpr int kThreads = 256;

unsigned blocks(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

__device__ inline uint64_t interleave(int64_t ax, int64_t ay, int64_t az, int level) {
  uint64_t m = 0;
  for (int b = 0; b < level; ++b) {
    m |= (uint64_t)((ax >> b) & 1) << (3 * b);
    m |= (uint64_t)((ay >> b) & 1) << (3 * b + 1);
    m |= (uint64_t)((az >> b) & 1) << (3 * b + 2);
  }
  return m;
}

__device__ inline uint64_t box_key(int64_t ax, int64_t ay, int64_t az, int level) {
  return interleave(ax, ay, az, level) | (uint64_t)1 << (3 * level);
}

// anchor of a code or key of the given level (bits at and above 3 level ignored)
__device__ inline void anchor_of(uint64_t key, int level, int a[3]) {
  a[0] = a[1] = a[2] = 0;
  for (int b = 0; b < level; ++b) {
    a[0] |= (int)((key >> (3 * b)) & 1) << b;
    a[1] |= (int)((key >> (3 * b + 1)) & 1) << b;
    a[2] |= (int)((key >> (3 * b + 2)) & 1) << b;
  }
}

// first index with k[idx] >= x
__device__ inline int64_t lower_bound(const uint64_t* __restrict__ k, int64_t n, uint64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (k[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// index of the box with anchor a at `level` among the sorted keys, or -1
__device__ inline int32_t find_box(const uint64_t* __restrict__ keys, int64_t n, int level,
                                   int64_t ax, int64_t ay, int64_t az) {
  const int64_t side = (int64_t)1 << level;
  if (ax < 0 || ay < 0 || az < 0 || ax >= side || ay >= side || az >= side) return -1;
  const uint64_t k = box_key(ax, ay, az, level);
  const int64_t i = lower_bound(keys, n, k);
  return i < n && keys[i] == k ? (int32_t)i : -1;
}

// ---- points: codes and a stable radix sort ------------------------------------

// code[i] = leaf code of point i, idx[i] = i; *bad = 1 for a point outside
// the domain cube.  The anchor rule is the host tree build's: u = (x - o) / w
// in [0, 1], a = min(floor(u 2^depth), 2^depth - 1).
__global__ void point_code_kernel(const double* __restrict__ pts, int64_t n, int depth, double ox,
                                  double oy, double oz, double w, uint64_t* __restrict__ code,
                                  int32_t* __restrict__ idx, int32_t* __restrict__ bad) {
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
  code[i] = ok ? interleave(a[0], a[1], a[2], depth) : 0;
  idx[i] = (int32_t)i;
  if (!ok) *bad = 1;
}

// digit histogram of one workgroup's chunk: hist[digit * nb + block]
template <typename K>
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(
    const K* __restrict__ key, int64_t n, int shift, int32_t* __restrict__ hist, int64_t nb) {
  __shared__ int32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int s = 0; s < kSortTiles; ++s) {
    const int64_t i = base + s * kSortThreads + tid;
    if (i < n) atomicAdd(&h[(int)((key[i] >> shift) & 255)], 1);
  }
  __syncthreads();
  hist[(int64_t)tid * nb + blockIdx.x] = h[tid];
}

// ---- exclusive prefix sums over the whole device ------------------------------
// a[0, m) in place, m = *mdev when given (at most m_cap), the sum to *total
// when given.  G <= kScanGroups workgroups each take a contiguous run of
// 1024-element tiles: per-workgroup sums (part[G]), one workgroup scans
// them, then each workgroup rescans its run with its offset.

constexpr int kScanTile = 4 * kThreads;  // 4 consecutive elements per thread
constexpr int kScanGroups = kTreeScanPart;

template <typename T>
__device__ inline T wave_inclusive(T x, int lane) {
  for (int d = 1; d < 64; d <<= 1) {
    const T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// exclusive prefix of x over the workgroup (kThreads threads) and the total
template <typename T>
__device__ inline T block_exclusive(T x, T* wsum, T& total) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T inc = wave_inclusive(x, lane);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  T pre = 0;
  total = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wave) pre += wsum[w];
    total += wsum[w];
  }
  __syncthreads();
  return pre + inc - x;
}

__device__ inline void scan_range(int64_t m, int G, int g, int64_t& t0, int64_t& t1) {
  const int64_t tiles = (m + kScanTile - 1) / kScanTile;
  const int64_t per = (tiles + G - 1) / G;
  t0 = min((int64_t)g * per, tiles);
  t1 = min(t0 + per, tiles);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const T* __restrict__ a, int64_t m_cap,
                                                               const int32_t* __restrict__ mdev,
                                                               T* __restrict__ part, int G) {
  __shared__ T wsum[kThreads / 64];
  const int64_t m = mdev ? min((int64_t)*mdev, m_cap) : m_cap;
  int64_t t0, t1;
  scan_range(m, G, blockIdx.x, t0, t1);
  T sum = 0;
  for (int64_t t = t0; t < t1; ++t)
    for (int k = 0; k < 4; ++k) {
      const int64_t i = t * kScanTile + k * kThreads + threadIdx.x;
      if (i < m) sum += a[i];
    }
  T total;
  (void)block_exclusive(sum, wsum, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kScanGroups) void scan_part_kernel(T* __restrict__ part, int G,
                                                                T* __restrict__ total) {
  __shared__ T wsum[kScanGroups / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T x = tid < G ? part[tid] : T(0);
  const T inc = wave_inclusive(x, lane);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  T pre = 0, all = 0;
  for (int w = 0; w < kScanGroups / 64; ++w) {
    if (w < wave) pre += wsum[w];
    all += wsum[w];
  }
  if (tid < G) part[tid] = pre + inc - x;
  if (tid == 0 && total) *total = all;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scan_apply_kernel(T* __restrict__ a, int64_t m_cap,
                                                              const int32_t* __restrict__ mdev,
                                                              const T* __restrict__ part, int G) {
  __shared__ T wsum[kThreads / 64];
  const int64_t m = mdev ? min((int64_t)*mdev, m_cap) : m_cap;
  int64_t t0, t1;
  scan_range(m, G, blockIdx.x, t0, t1);
  T carry = part[blockIdx.x];
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t base = t * kScanTile + 4 * (int64_t)threadIdx.x;
    T v[4];
    T sum = 0;
    for (int k = 0; k < 4; ++k) {
      v[k] = base + k < m ? a[base + k] : T(0);
      sum += v[k];
    }
    T total;
    T run = carry + block_exclusive(sum, wsum, total);
    for (int k = 0; k < 4; ++k) {
      if (base + k < m) a[base + k] = run;
      run += v[k];
    }
    carry += total;
  }
}

template <typename T>
void device_scan(T* a, int64_t m_cap, const int32_t* mdev, T* total, T* part, hipStream_t s) {
  const int64_t tiles = std::max<int64_t>(1, (m_cap + kScanTile - 1) / kScanTile);
  const int G = (int)std::min<int64_t>(kScanGroups, tiles);
  scan_reduce_kernel<T><<<G, kThreads, 0, s>>>(a, m_cap, mdev, part, G);
  scan_part_kernel<T><<<1, kScanGroups, 0, s>>>(part, G, total);
  scan_apply_kernel<T><<<G, kThreads, 0, s>>>(a, m_cap, mdev, part, G);
}

// stable scatter by one 8-bit digit: within a workgroup's chunk, elements
// keep their order (sub-tile, then wave, then lane); ranks among equal
// digits in a wave come from ballots, across waves from LDS counts
template <typename K>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const K* __restrict__ key_in, const int32_t* __restrict__ val_in, int64_t n, int shift,
    const int32_t* __restrict__ offs, int64_t nb, K* __restrict__ key_out,
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
    const K kv = act ? key_in[i] : K(0);
    const int dig = (int)((kv >> shift) & 255);
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

__global__ void init_counts_kernel(int32_t* __restrict__ cnt, int32_t n_src, int32_t n_tgt) {
  const int i = threadIdx.x;
  cnt[i] = i == 20 ? n_src : i == 21 ? n_tgt : 0;
}

// ---- unique codes, set union, levels --------------------------------------------

// flag[i] = 1 where code[i] >> shift starts a run (i < *n), else 0 (i < cap)
__global__ void head_kernel(const uint64_t* __restrict__ code, int64_t cap, const int32_t* __restrict__ n,
                            int shift, int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  const int64_t m = *n;
  flag[i] = i < m && (i == 0 || (code[i] >> shift) != (code[i - 1] >> shift)) ? 1 : 0;
}

// out[pos[i]] = code[i] >> shift at run heads; parent[i] = index of i's run
__global__ void compact_kernel(const uint64_t* __restrict__ code, int64_t cap, const int32_t* __restrict__ n,
                               int shift, const int32_t* __restrict__ pos, uint64_t* __restrict__ out,
                               int32_t* __restrict__ parent) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap || i >= *n) return;
  const bool head = i == 0 || (code[i] >> shift) != (code[i - 1] >> shift);
  if (head) out[pos[i]] = code[i] >> shift;
  if (parent) parent[i] = pos[i] + (head ? 1 : 0) - 1;
}

// flag[j] = 1 where b[j] (j < *nb) is not among a[0, *na)
__global__ void not_in_kernel(const uint64_t* __restrict__ b, int64_t cap, const int32_t* __restrict__ nb,
                              const uint64_t* __restrict__ a, const int32_t* __restrict__ na,
                              int32_t* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cap) return;
  int32_t f = 0;
  if (j < *nb) {
    const int64_t m = *na;
    const int64_t k = lower_bound(a, m, b[j]);
    f = (k < m && a[k] == b[j]) ? 0 : 1;
  }
  flag[j] = f;
}

__global__ void select_kernel(const uint64_t* __restrict__ b, int64_t cap, const int32_t* __restrict__ nb,
                              const uint64_t* __restrict__ a, const int32_t* __restrict__ na,
                              const int32_t* __restrict__ pos, uint64_t* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cap || j >= *nb) return;
  const int64_t m = *na;
  const int64_t k = lower_bound(a, m, b[j]);
  if (!(k < m && a[k] == b[j])) out[pos[j]] = b[j];
}

// union of the disjoint sorted sets a and b: an element's position is its
// own index plus the number of elements of the other set below it
__global__ void union_kernel(const uint64_t* __restrict__ a, const int32_t* __restrict__ na,
                             const uint64_t* __restrict__ b, const int32_t* __restrict__ nb,
                             int64_t cap, uint64_t* __restrict__ u, int32_t* __restrict__ nu) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ma = *na, mb = *nb;
  if (i == 0) *nu = (int32_t)(ma + mb);
  if (i >= cap) return;
  if (i < ma) u[i + lower_bound(b, mb, a[i])] = a[i];
  if (i < mb) u[i + lower_bound(a, ma, b[i])] = b[i];
}

// *differs = 1 unless the n_old sentinel keys equal the leaf codes u[0, *nu)
__global__ void same_kernel(const uint64_t* __restrict__ u, const int32_t* __restrict__ nu,
                            const uint64_t* __restrict__ old_keys, int64_t n_old, int depth,
                            int32_t* __restrict__ differs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && *nu != n_old) *differs = 1;
  if (i >= n_old || i >= *nu) return;
  if ((u[i] | (uint64_t)1 << (3 * depth)) != old_keys[i]) *differs = 1;
}

// ---- structures of the new tree (counts known on the host) -----------------------

__global__ void points_kernel(const double* __restrict__ pts, const int32_t* __restrict__ order,
                              int64_t n, int64_t* __restrict__ perm, double* __restrict__ sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = order[i];
  perm[i] = j;
  for (int c = 0; c < 3; ++c) sorted[3 * i + c] = pts[3 * j + c];
}

// [start, end) of each leaf's points among the sorted point codes
__global__ void ranges_kernel(const uint64_t* __restrict__ code, int64_t n,
                              const uint64_t* __restrict__ leaf, int64_t n_leaf,
                              int32_t* __restrict__ start, int32_t* __restrict__ end) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_leaf) return;
  start[i] = (int32_t)lower_bound(code, n, leaf[i]);
  end[i] = (int32_t)lower_bound(code, n, leaf[i] + 1);
}

__global__ void keys_kernel(const uint64_t* __restrict__ code, int64_t n, int level,
                            uint64_t* __restrict__ keys, int32_t* __restrict__ parent_out,
                            const int32_t* __restrict__ parent_in) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = code[i] | (uint64_t)1 << (3 * level);
  parent_out[i] = parent_in ? parent_in[i] : -1;
}

__global__ void fill_kernel(int32_t* __restrict__ v, int64_t n, int32_t x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = x;
}

// child_up[8 parent[i] + octant(i)] = i
__global__ void child_kernel(const uint64_t* __restrict__ keys, const int32_t* __restrict__ parent,
                             int64_t n, int32_t* __restrict__ child_up) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  child_up[8 * (int64_t)parent[i] + (int)(keys[i] & 7)] = (int32_t)i;
}

// leaf centres origin + (a + 1/2) w, rounded as the host computes them
__global__ void centers_kernel(const uint64_t* __restrict__ keys, int64_t n, int depth, double ox,
                               double oy, double oz, double w, double* __restrict__ c) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int a[3];
  anchor_of(keys[i], depth, a);
  const double o[3] = {ox, oy, oz};
  for (int k = 0; k < 3; ++k) {
    const double h = ((double)a[k] + 0.5) * w;
    c[3 * i + k] = o[k] + h;
  }
}

// halo[d][c]: the cluster (box of level lc) in direction d of cluster c,
// directions in lexicographic order of (dx, dy, dz) without 0; `empty`
// where absent
__global__ void halo_kernel(const uint64_t* __restrict__ keys, int64_t n, int level, int32_t empty,
                            int32_t* __restrict__ halo) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int a[3];
  anchor_of(keys[c], level, a);
  int d = 0;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        const int32_t s = find_box(keys, n, level, a[0] + dx, a[1] + dy, a[2] + dz);
        halo[(int64_t)d * n + c] = s >= 0 ? s : empty;
        ++d;
      }
}

// Interaction list of box i (level l >= 2): children of the parent's
// neighbours that are not adjacent to the box (Section 2, the M2L), in
// ascending source index - the parents' neighbours sorted by index, their
// children in octant order (children keys extend their parent's key and both
// levels are sorted, so child indices follow parent indices); count pass
// (tidx == nullptr) or fill pass.  A child's anchor is 2 (parent anchor) +
// octant bits, so no key is decoded per child.
__global__ void interactions_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                    const int32_t* __restrict__ parent,
                                    const uint64_t* __restrict__ keys_up, int64_t n_up,
                                    const int32_t* __restrict__ child_up, int level,
                                    const int16_t* __restrict__ tmap, int64_t* __restrict__ offs,
                                    int32_t* __restrict__ src, int16_t* __restrict__ tidx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int a[3];
  anchor_of(keys[i], level, a);
  const int pa[3] = {a[0] >> 1, a[1] >> 1, a[2] >> 1};
  // (index << 5 | direction) of the existing parent neighbours, ascending
  int64_t nb[27];
  int m = 0;
  for (int d = 0; d < 27; ++d) {
    const int dx = d / 9 - 1, dy = (d / 3) % 3 - 1, dz = d % 3 - 1;
    const int32_t s = find_box(keys_up, n_up, level - 1, pa[0] + dx, pa[1] + dy, pa[2] + dz);
    if (s < 0) continue;
    const int64_t v = (int64_t)s << 5 | d;
    int k = m++;
    while (k > 0 && nb[k - 1] > v) {
      nb[k] = nb[k - 1];
      --k;
    }
    nb[k] = v;
  }
  int64_t e = tidx ? offs[i] : 0;
  for (int k = 0; k < m; ++k) {
    const int32_t p = (int32_t)(nb[k] >> 5);
    const int d = (int)(nb[k] & 31);
    const int bx = 2 * (pa[0] + d / 9 - 1) - a[0], by = 2 * (pa[1] + (d / 3) % 3 - 1) - a[1],
              bz = 2 * (pa[2] + d % 3 - 1) - a[2];
    for (int o = 0; o < 8; ++o) {
      const int32_t s = child_up[8 * (int64_t)p + o];
      if (s < 0) continue;
      const int tx = bx + (o & 1), ty = by + ((o >> 1) & 1), tz = bz + ((o >> 2) & 1);
      if (max(abs(tx), max(abs(ty), abs(tz))) <= 1) continue;
      if (tidx) {
        src[e] = s;
        tidx[e] = tmap[(tx + 3) * 49 + (ty + 3) * 7 + (tz + 3)];
      }
      ++e;
    }
  }
  if (!tidx) offs[i] = e;
}

// near field of leaf i: leaves whose anchors differ by at most 1 per axis,
// itself included, ascending; count pass (src == nullptr) or fill pass
__global__ void near_kernel(const uint64_t* __restrict__ keys, int64_t n, int depth,
                            int64_t* __restrict__ offs, int32_t* __restrict__ src) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int a[3];
  anchor_of(keys[i], depth, a);
  int32_t row[27];
  int m = 0;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        const int32_t s = find_box(keys, n, depth, a[0] + dx, a[1] + dy, a[2] + dz);
        if (s < 0) continue;
        int k = m++;
        while (k > 0 && row[k - 1] > s) {
          row[k] = row[k - 1];
          --k;
        }
        row[k] = s;
      }
  if (!src) {
    offs[i] = m;
    return;
  }
  const int64_t e = offs[i];
  for (int k = 0; k < m; ++k) src[e + k] = row[k];
}

// total of an exclusive scan over m entries whose last count is cnt_last
__global__ void close_offsets_kernel(int64_t* __restrict__ offs, int64_t m, const int64_t* __restrict__ total) {
  offs[m] = *total;
}

// ---- FFT-M2L source blocks ---------------------------------------------------------

// shell slot of cluster c's own position within its aligned 4 x 4 x 4 cube
__device__ inline int own_slot(const int a[3]) {
  return ((a[0] & 3) + 1) + kHadShell * ((a[1] & 3) + 1) + kHadShell * kHadShell * ((a[2] & 3) + 1);
}

// block heads: clusters whose key >> 6 differs from the previous one's
__global__ void block_head_kernel(const uint64_t* __restrict__ keys, int64_t n, int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = i == 0 || (keys[i] >> 6) != (keys[i - 1] >> 6) ? 1 : 0;
}

__global__ void block_first_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                   const int32_t* __restrict__ pos, int32_t* __restrict__ tgt,
                                   int32_t* __restrict__ tbase, int level) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool head = i == 0 || (keys[i] >> 6) != (keys[i - 1] >> 6);
  if (head) tgt[pos[i]] = (int32_t)i;
  if (i == n - 1) tgt[pos[i] + (head ? 1 : 0)] = (int32_t)n;
  int a[3];
  anchor_of(keys[i], level, a);
  tbase[i] = (own_slot(a) - kHadSlotBias) * kHadRowBytes;
}

// One wave per block.  Slot (x, y, z) of the 6 x 6 x 6 shell is in the
// block's list when some member's 26 neighbour directions reach it: a member
// sits at inner position (x - 1 - dx, ...) for some direction d != 0.  Count
// pass (list == nullptr): cnt[b] = slots of block b; fill pass: the block's
// entries cluster << 8 | slot in ascending slot order, with the empty
// cluster n where no cluster sits at the slot.
__global__ __launch_bounds__(kThreads) void block_list_kernel(
    const uint64_t* __restrict__ keys, int64_t n, int level, const int32_t* __restrict__ tgt,
    int64_t nblk, int32_t* __restrict__ cnt, const int32_t* __restrict__ first,
    int32_t* __restrict__ list) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (b == 0 && lane == 0 && list) list[0] = (int32_t)((uint32_t)n << 8 | 255u);
  if (b >= nblk) return;
  const int32_t c0 = tgt[b], c1 = tgt[b + 1];
  // members on the 4 x 4 x 4 cube: bit x + 4 y + 16 z (at most 64 members)
  uint64_t mem = 0;
  if (c0 + lane < c1) {
    int a[3];
    anchor_of(keys[c0 + lane], level, a);
    mem = 1ull << ((a[0] & 3) + 4 * (a[1] & 3) + 16 * (a[2] & 3));
  }
  for (int sh = 1; sh < 64; sh <<= 1) mem |= __shfl_xor(mem, sh, 64);
  int a0[3];
  anchor_of(keys[c0], level, a0);
  const int bx = (a0[0] >> 2) * 4 - 1, by = (a0[1] >> 2) * 4 - 1, bz = (a0[2] >> 2) * 4 - 1;
  int64_t e = list ? first[b] : 0;
  for (int r = 0; r < (kHadSrcSlots + 63) / 64; ++r) {
    const int sl = r * 64 + lane;
    bool hit = false;
    if (sl < kHadSrcSlots) {
      const int x = sl % kHadShell, y = (sl / kHadShell) % kHadShell, z = sl / (kHadShell * kHadShell);
      for (int d = 0; d < 27 && !hit; ++d) {
        if (d == 13) continue;
        const int px = x - 1 - (d / 9 - 1), py = y - 1 - ((d / 3) % 3 - 1), pz = z - 1 - (d % 3 - 1);
        if (px < 0 || py < 0 || pz < 0 || px > 3 || py > 3 || pz > 3) continue;
        hit = (mem >> (px + 4 * py + 16 * pz)) & 1;
      }
    }
    const uint64_t bal = __ballot(hit);
    if (list && hit) {
      const int x = sl % kHadShell, y = (sl / kHadShell) % kHadShell, z = sl / (kHadShell * kHadShell);
      const int32_t c = find_box(keys, n, level, bx + x, by + y, bz + z);
      list[e + __popcll(bal & ((1ull << lane) - 1))] = (int32_t)((uint32_t)(c >= 0 ? c : (int32_t)n) << 8 | (uint32_t)sl);
    }
    e += __popcll(bal);
  }
  if (!list && lane == 0) cnt[b] = (int32_t)e;
}

// hb_src[b] = 1 + exclusive count (entry 0 is the empty cluster), and the end
__global__ void block_offsets_kernel(const int32_t* __restrict__ pos, int64_t nblk,
                                     const int32_t* __restrict__ total, int32_t* __restrict__ src) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nblk) src[b] = 1 + pos[b];
  if (b == 0) src[nblk] = 1 + *total;
}

// ---- BLAS / dense target tiles -------------------------------------------------------

__global__ void class_key_kernel(const uint64_t* __restrict__ keys, int64_t n, int32_t* __restrict__ cls,
                                 int32_t* __restrict__ idx, int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = (int)(keys[i] & 7);
  cls[i] = o;
  idx[i] = (int32_t)i;
  atomicAdd(&count[o], 1);
}

// the source box of target box i along transfer vector t (an index into
// the 316), or -1: the box at anchor + t exists and its parent is adjacent
// to box i's parent - the interaction-list condition, since |t| >= 2
__device__ inline int32_t source_along(const uint64_t* __restrict__ keys, int64_t n, int level,
                                       const int a[3], const int8_t* __restrict__ tvec, int t) {
  const int b[3] = {a[0] + tvec[3 * t], a[1] + tvec[3 * t + 1], a[2] + tvec[3 * t + 2]};
  for (int k = 0; k < 3; ++k) {
    if (b[k] < 0) return -1;
    if (abs((b[k] >> 1) - (a[k] >> 1)) > 1) return -1;
  }
  return find_box(keys, n, level, b[0], b[1], b[2]);
}

__global__ void tile_box_kernel(const int32_t* __restrict__ order, TileClasses tc, int TB,
                                int64_t ntiles, int32_t* __restrict__ tile_box,
                                int32_t* __restrict__ tile_class) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntiles * TB) return;
  const int64_t tile = e / TB;
  const int sl = (int)(e % TB);
  int o = 0;
  while (o < 7 && tile >= tc.first_tile[o + 1]) ++o;
  const int64_t r = (tile - tc.first_tile[o]) * TB + sl;
  tile_box[e] = r < tc.count[o] ? order[tc.start[o] + r] : -1;
  if (sl == 0) tile_class[tile] = o;
}

// present[tile * 316 + t] = 1 if some box of the tile has a source along t
__global__ void tile_present_kernel(const int32_t* __restrict__ tile_box, int64_t ntiles, int TB,
                                    const uint64_t* __restrict__ keys, int64_t n, int level,
                                    const int8_t* __restrict__ tvec, int64_t* __restrict__ present) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntiles * kNumT) return;
  const int64_t tile = e / kNumT;
  const int t = (int)(e % kNumT);
  int64_t any = 0;
  for (int sl = 0; sl < TB && !any; ++sl) {
    const int32_t bx = tile_box[tile * TB + sl];
    if (bx < 0) continue;
    int a[3];
    anchor_of(keys[bx], level, a);
    any = source_along(keys, n, level, a, tvec, t) >= 0;
  }
  present[e] = any;
}

// transfer vectors of each tile (ascending) with the source of every slot;
// the stacked form's [J][TB] sources per tile (class slot j of t) as well
__global__ void tile_fill_kernel(const int32_t* __restrict__ tile_box, const int32_t* __restrict__ tile_class,
                                 int64_t ntiles, int TB, const uint64_t* __restrict__ keys, int64_t n,
                                 int level, const int8_t* __restrict__ tvec,
                                 const int64_t* __restrict__ pos, int32_t* __restrict__ tl_t,
                                 int32_t* __restrict__ tl_src, int64_t* __restrict__ tl_offs,
                                 const int32_t* __restrict__ jof, int J, int32_t* __restrict__ tile_src) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntiles * kNumT) return;
  const int64_t tile = e / kNumT;
  const int t = (int)(e % kNumT);
  if (t == 0) tl_offs[tile] = pos[e];
  const bool present = pos[e + 1] != pos[e];
  const int o = tile_class[tile];
  const int j = tile_src ? jof[o * kNumT + t] : -1;
  if (!present) return;
  const int64_t q = pos[e];
  tl_t[q] = t;
  for (int sl = 0; sl < TB; ++sl) {
    const int32_t bx = tile_box[tile * TB + sl];
    int32_t s = -1;
    if (bx >= 0) {
      int a[3];
      anchor_of(keys[bx], level, a);
      s = source_along(keys, n, level, a, tvec, t);
    }
    tl_src[q * TB + sl] = s;
    if (j >= 0) tile_src[(tile * J + j) * TB + sl] = s;
  }
}

// scratch bump allocation, 256-byte aligned
struct Bump {
  char* p;
  template <typename T>
  T* take(int64_t count) {
    T* r = reinterpret_cast<T*>(p);
    p += ((size_t)count * sizeof(T) + 255) / 256 * 256;
    return r;
  }
};

int64_t level_cap(int64_t n, int l) { return l >= 21 ? n : std::min<int64_t>(n, (int64_t)1 << (3 * l)); }

// stable radix sort of (code, index) by the low `bits` bits of the code;
// the result is in whichever of the two buffer pairs the last pass wrote
hipError_t sort_codes(uint64_t* k0, int32_t* v0, uint64_t* k1, int32_t* v1, int32_t* hist, int64_t n,
                      int bits, uint64_t** k_out, int32_t** v_out, int32_t* part, hipStream_t s) {
  const int64_t nb = (n + kSortChunk - 1) / kSortChunk;
  uint64_t* K[2] = {k0, k1};
  int32_t* V[2] = {v0, v1};
  const int passes = std::max(1, (bits + 7) / 8);
  for (int p = 0; p < passes; ++p) {
    const int in = p & 1, out = in ^ 1;
    radix_hist_kernel<uint64_t><<<(unsigned)nb, kSortThreads, 0, s>>>(K[in], n, 8 * p, hist, nb);
    device_scan<int32_t>(hist, 256 * nb, nullptr, nullptr, part, s);
    radix_scatter_kernel<uint64_t><<<(unsigned)nb, kSortThreads, 0, s>>>(K[in], V[in], n, 8 * p, hist,
                                                                         nb, K[out], V[out]);
  }
  *k_out = K[passes & 1];
  *v_out = V[passes & 1];
  return hipGetLastError();
}

// unique codes of a sorted array of n (host-known) codes: out, *count
hipError_t unique_codes(const uint64_t* code, int64_t n, const int32_t* n_dev, int32_t* flag,
                        uint64_t* out, int32_t* count, int32_t* parent, int shift, int32_t* part,
                        hipStream_t s) {
  head_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(code, n, n_dev, shift, flag);
  device_scan<int32_t>(flag, n, n_dev, count, part, s);
  compact_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(code, n, n_dev, shift, flag, out, parent);
  return hipGetLastError();
}

}  // namespace

size_t tree_scratch_bytes(int64_t n_src, int64_t n_tgt, int depth) {
  const int64_t n = std::max(n_src, n_tgt), cap = n_src + n_tgt;
  const int64_t nb = (n + kSortChunk - 1) / kSortChunk;
  size_t b = 0;
  auto add = [&b](size_t bytes) { b += (bytes + 255) / 256 * 256; };
  for (int set = 0; set < 2; ++set) {
    const int64_t m = set == 0 ? n_src : n_tgt;
    add(m * 8); add(m * 8); add(m * 4); add(m * 4);  // codes and indices, ping and pong
  }
  add(256 * nb * 4);                                  // digit histograms
  add(cap * 4);                                       // flags / positions
  add(n_src * 8); add(n_tgt * 8); add(n_tgt * 8);     // unique source, target, target-only codes
  for (int l = 0; l <= depth; ++l) {
    add(level_cap(cap, l) * 8);                       // codes of level l
    add(level_cap(cap, l) * 4);                       // parents of level l
  }
  add(64 * 4);                                        // counts
  add(kScanGroups * 8);                               // scan partial sums
  return b;
}

hipError_t tree_sort_and_levels(const double* src, int64_t n_src, const double* tgt, int64_t n_tgt,
                                int depth, const double origin[3], double width,
                                const uint64_t* old_leaf_keys, int64_t n_old, void* scratch,
                                TreeBuild& out, hipStream_t s) {
  if (n_src <= 0 || n_tgt <= 0 || n_src + n_tgt >= ((int64_t)1 << 31) || depth < 1 || depth > 16)
    return hipErrorInvalidValue;
  const int64_t n = std::max(n_src, n_tgt), cap = n_src + n_tgt;
  const int64_t nb = (n + kSortChunk - 1) / kSortChunk;
  Bump m{static_cast<char*>(scratch)};
  uint64_t *ks[2][2];
  int32_t* vs[2][2];
  for (int set = 0; set < 2; ++set) {
    const int64_t c = set == 0 ? n_src : n_tgt;
    ks[set][0] = m.take<uint64_t>(c);
    ks[set][1] = m.take<uint64_t>(c);
    vs[set][0] = m.take<int32_t>(c);
    vs[set][1] = m.take<int32_t>(c);
  }
  int32_t* hist = m.take<int32_t>(256 * nb);
  int32_t* flag = m.take<int32_t>(cap);
  uint64_t* us = m.take<uint64_t>(n_src);
  uint64_t* ut = m.take<uint64_t>(n_tgt);
  uint64_t* uto = m.take<uint64_t>(n_tgt);
  uint64_t* code[17];
  int32_t* parent[17];
  for (int l = 0; l <= depth; ++l) {
    code[l] = m.take<uint64_t>(level_cap(cap, l));
    parent[l] = m.take<int32_t>(level_cap(cap, l));
  }
  int32_t* cnt = m.take<int32_t>(64);
  int64_t* part64 = m.take<int64_t>(kScanGroups);
  int32_t* part = reinterpret_cast<int32_t*>(part64);
  // cnt: [0] bad point, [1] leaf set differs, [2 + l] boxes of level l,
  // [20] point counts (src, tgt), [22] unique source / target / target-only
  init_counts_kernel<<<1, 64, 0, s>>>(cnt, (int32_t)n_src, (int32_t)n_tgt);
  hipError_t e = hipSuccess;
  const double* pts[2] = {src, tgt};
  for (int set = 0; set < 2; ++set) {
    const int64_t c = set == 0 ? n_src : n_tgt;
    point_code_kernel<<<blocks(c, kThreads), kThreads, 0, s>>>(pts[set], c, depth, origin[0], origin[1],
                                                                origin[2], width, ks[set][0], vs[set][0], cnt);
    uint64_t* ko;
    int32_t* vo;
    e = sort_codes(ks[set][0], vs[set][0], ks[set][1], vs[set][1], hist, c, 3 * depth, &ko, &vo, part, s);
    if (e != hipSuccess) return e;
    (set == 0 ? out.code_src : out.code_tgt) = ko;
    (set == 0 ? out.order_src : out.order_tgt) = vo;
  }
  // leaves: union of the non-empty source and target leaves
  e = unique_codes(out.code_src, n_src, cnt + 20, flag, us, cnt + 22, nullptr, 0, part, s);
  if (e != hipSuccess) return e;
  e = unique_codes(out.code_tgt, n_tgt, cnt + 21, flag, ut, cnt + 23, nullptr, 0, part, s);
  if (e != hipSuccess) return e;
  not_in_kernel<<<blocks(n_tgt, kThreads), kThreads, 0, s>>>(ut, n_tgt, cnt + 23, us, cnt + 22, flag);
  device_scan<int32_t>(flag, n_tgt, cnt + 23, cnt + 24, part, s);
  select_kernel<<<blocks(n_tgt, kThreads), kThreads, 0, s>>>(ut, n_tgt, cnt + 23, us, cnt + 22, flag, uto);
  union_kernel<<<blocks(std::max(n_src, n_tgt), kThreads), kThreads, 0, s>>>(
      us, cnt + 22, uto, cnt + 24, std::max(n_src, n_tgt), code[depth], cnt + 2 + depth);
  same_kernel<<<blocks(std::max<int64_t>(n_old, 1), kThreads), kThreads, 0, s>>>(
      code[depth], cnt + 2 + depth, old_leaf_keys, n_old, depth, cnt + 1);
  // ancestors level by level: parent code = code >> 3
  for (int l = depth; l >= 1; --l) {
    const int64_t c = level_cap(cap, l);
    e = unique_codes(code[l], c, cnt + 2 + l, flag, code[l - 1], cnt + 2 + l - 1, parent[l], 3, part, s);
    if (e != hipSuccess) return e;
  }
  for (int l = 0; l <= depth; ++l) {
    out.code[l] = code[l];
    out.parent[l] = parent[l];
  }
  out.counts = cnt;
  return hipGetLastError();
}

hipError_t tree_finish_points(const double* pts, const uint64_t* code, const int32_t* order, int64_t n,
                              const uint64_t* leaf_code, int64_t n_leaf, int64_t* perm, double* sorted,
                              int32_t* start, int32_t* end, hipStream_t s) {
  points_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(pts, order, n, perm, sorted);
  ranges_kernel<<<blocks(n_leaf, kThreads), kThreads, 0, s>>>(code, n, leaf_code, n_leaf, start, end);
  return hipGetLastError();
}

hipError_t tree_level(const uint64_t* code, const int32_t* parent, int64_t n, int level,
                      uint64_t* keys, int32_t* parent_out, int32_t* child_up, int64_t n_up,
                      hipStream_t s) {
  keys_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(code, n, level, keys, parent_out,
                                                        level > 0 ? parent : nullptr);
  if (child_up) {
    fill_kernel<<<blocks(8 * n_up + 8, kThreads), kThreads, 0, s>>>(child_up, 8 * n_up + 8, -1);
    child_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(keys, parent_out, n, child_up);
  }
  return hipGetLastError();
}

hipError_t tree_centers(const uint64_t* keys, int64_t n, int depth, const double origin[3], double w,
                        double* c, hipStream_t s) {
  centers_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(keys, n, depth, origin[0], origin[1],
                                                           origin[2], w, c);
  return hipGetLastError();
}

hipError_t tree_halo(const uint64_t* keys, int64_t n, int level, int32_t* halo, hipStream_t s) {
  halo_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(keys, n, level, (int32_t)n, halo);
  return hipGetLastError();
}

hipError_t tree_interactions(const uint64_t* keys, int64_t n, const int32_t* parent,
                             const uint64_t* keys_up, int64_t n_up, const int32_t* child_up, int level,
                             const int16_t* tmap, int64_t* offs, int64_t* total, int32_t* src,
                             int16_t* tidx, int64_t* part, hipStream_t s) {
  interactions_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(keys, n, parent, keys_up, n_up, child_up,
                                                                level, tmap, offs, src, tidx);
  if (!tidx) {
    device_scan<int64_t>(offs, n, nullptr, total, part, s);
    close_offsets_kernel<<<1, 1, 0, s>>>(offs, n, total);
  }
  return hipGetLastError();
}

hipError_t tree_near(const uint64_t* keys, int64_t n, int depth, int64_t* offs, int64_t* total,
                     int32_t* src, int64_t* part, hipStream_t s) {
  near_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(keys, n, depth, offs, src);
  if (!src) {
    device_scan<int64_t>(offs, n, nullptr, total, part, s);
    close_offsets_kernel<<<1, 1, 0, s>>>(offs, n, total);
  }
  return hipGetLastError();
}

hipError_t tree_blocks(const uint64_t* keys, int64_t n, int level, int32_t* flag, int32_t* tgt,
                       int32_t* tbase, int32_t* counts, int64_t* part, hipStream_t s) {
  block_head_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(keys, n, flag);
  device_scan<int32_t>(flag, n, nullptr, counts, reinterpret_cast<int32_t*>(part), s);
  block_first_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(keys, n, flag, tgt, tbase, level);
  return hipGetLastError();
}

hipError_t tree_block_lists(const uint64_t* keys, int64_t n, int level, const int32_t* tgt, int64_t nblk,
                            int32_t* cnt, int32_t* src, int32_t* total, int32_t* list, int64_t* part,
                            hipStream_t s) {
  if (!list) {
    block_list_kernel<<<blocks(nblk * 64, kThreads), kThreads, 0, s>>>(keys, n, level, tgt, nblk, cnt,
                                                                        nullptr, nullptr);
    device_scan<int32_t>(cnt, nblk, nullptr, total, reinterpret_cast<int32_t*>(part), s);
    block_offsets_kernel<<<blocks(nblk, kThreads), kThreads, 0, s>>>(cnt, nblk, total, src);
    return hipGetLastError();
  }
  block_list_kernel<<<blocks(nblk * 64, kThreads), kThreads, 0, s>>>(keys, n, level, tgt, nblk, nullptr,
                                                                      src, list);
  return hipGetLastError();
}

hipError_t tree_classes(const uint64_t* keys, int64_t n, int32_t* scratch, int32_t* order,
                        int32_t* counts, int64_t* part, hipStream_t s) {
  // stable order of the boxes by octant class: one radix pass on the class
  const int64_t nb = (n + kSortChunk - 1) / kSortChunk;
  int32_t* cls = scratch;
  int32_t* idx = cls + n;
  int32_t* cls2 = idx + n;
  int32_t* hist = cls2 + n;
  fill_kernel<<<1, 64, 0, s>>>(counts, 8, 0);
  class_key_kernel<<<blocks(n, kThreads), kThreads, 0, s>>>(keys, n, cls, idx, counts);
  radix_hist_kernel<int32_t><<<(unsigned)nb, kSortThreads, 0, s>>>(cls, n, 0, hist, nb);
  device_scan<int32_t>(hist, 256 * nb, nullptr, nullptr, reinterpret_cast<int32_t*>(part), s);
  radix_scatter_kernel<int32_t><<<(unsigned)nb, kSortThreads, 0, s>>>(cls, idx, n, 0, hist, nb, cls2,
                                                                      order);
  return hipGetLastError();
}

size_t tree_classes_scratch_ints(int64_t n) {
  return (size_t)(3 * n + 256 * ((n + kSortChunk - 1) / kSortChunk));
}

hipError_t tree_tiles(const uint64_t* keys, int64_t n, int level, const int32_t* order,
                      const TileClasses& tc, int TB, int64_t ntiles, const int8_t* tvec,
                      int32_t* tile_box, int32_t* tile_class, int64_t* present, int64_t* total,
                      int64_t* part, hipStream_t s) {
  tile_box_kernel<<<blocks(ntiles * TB, kThreads), kThreads, 0, s>>>(order, tc, TB, ntiles, tile_box,
                                                                      tile_class);
  tile_present_kernel<<<blocks(ntiles * kNumT, kThreads), kThreads, 0, s>>>(tile_box, ntiles, TB, keys, n,
                                                                             level, tvec, present);
  device_scan<int64_t>(present, ntiles * kNumT, nullptr, total, part, s);
  close_offsets_kernel<<<1, 1, 0, s>>>(present, ntiles * kNumT, total);
  return hipGetLastError();
}

hipError_t tree_tiles_fill(const uint64_t* keys, int64_t n, int level, const int32_t* tile_box,
                           const int32_t* tile_class, int64_t ntiles, int TB, const int8_t* tvec,
                           const int64_t* pos, int32_t* tl_t, int32_t* tl_src, int64_t* tl_offs,
                           const int32_t* jof, int J, int32_t* tile_src, hipStream_t s) {
  if (tile_src)
    fill_kernel<<<blocks(ntiles * J * TB, kThreads), kThreads, 0, s>>>(tile_src, ntiles * J * TB, -1);
  tile_fill_kernel<<<blocks(ntiles * kNumT, kThreads), kThreads, 0, s>>>(
      tile_box, tile_class, ntiles, TB, keys, n, level, tvec, pos, tl_t, tl_src, tl_offs, jof, J, tile_src);
  close_offsets_kernel<<<1, 1, 0, s>>>(tl_offs, ntiles, pos + ntiles * kNumT);
  return hipGetLastError();
}

}  // namespace kifmm
