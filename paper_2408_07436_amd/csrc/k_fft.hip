// FFT-M2L on gfx950 (Appendix A.1-A.2 of arXiv 2408.07436).
//
// 1. fft_forward: the upward-equivalent densities of each box sit on the
//    (2p-1)^3 convolution grid at their lattice positions (zeros elsewhere;
//    2p - 1 points per axis are enough for the convolution not to wrap).  A
//    real-to-complex 3D DFT that skips the zero planes gives (2p-1)^2 p
//    coefficients per box, written in frequency order [f][cluster, v][child]
//    so that the eight siblings of a cluster are contiguous per frequency.
// 2. hadamard: for every frequency f and target cluster, the 8 x 8 complex
//    products against the kernel spectra of the 26 source clusters of its
//    halo, summed.  Per frequency this is a real GEMM
//       [rows = (cluster, v)] x [K = 26 dirs x 8 sources x (re, im)]
//         x [N = 8 targets x (re, im)],
//    with the A operand gathered through the halo table; it runs on
//    v_mfma_f32_16x16x4f32 (FP32) or v_mfma_f64_16x16x4f64 (FP64).
// 3. fft_inverse: complex inverse DFTs along x and y, then the c2r step along
//    z (odd length: no Nyquist term), evaluated only at the check-surface
//    lattice points.
#include "kernels.h"

namespace kifmm {

namespace {

template <typename T> struct C2T;
template <> struct C2T<float> { using type = float2; };
template <> struct C2T<double> { using type = double2; };

template <typename C2>
__device__ inline C2 cmul(C2 a, C2 b) {
  C2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// a * conj(b)
template <typename C2>
__device__ inline C2 cmulc(C2 a, C2 b) {
  C2 r;
  r.x = a.x * b.x + a.y * b.y;
  r.y = a.y * b.x - a.x * b.y;
  return r;
}

constexpr int kFftThreads = 256;

template <typename T, int P, int ITEMS>
__global__ __launch_bounds__(kFftThreads) void fft_forward_kernel(
    const double* __restrict__ M, const int32_t* __restrict__ child, int64_t n_rows, int nvec,
    const int16_t* __restrict__ lat2surf, const typename C2T<T>::type* __restrict__ tw,
    typename C2T<T>::type* __restrict__ Qhat) {
  using C2 = typename C2T<T>::type;
  constexpr int N = 2 * P - 1, H = P, NS = 6 * (P - 1) * (P - 1) + 2;
  __shared__ C2 w[N];
  __shared__ int16_t l2s[P * P * P];
  __shared__ T sv[ITEMS][NS];
  __shared__ C2 a1[ITEMS][P][P][H];
  const int tid = threadIdx.x;
  const int64_t g0 = (int64_t)blockIdx.x * ITEMS;  // first (row, child) item
  for (int t = tid; t < N; t += kFftThreads) w[t] = tw[t];
  for (int t = tid; t < P * P * P; t += kFftThreads) l2s[t] = lat2surf[t];
  for (int idx = tid; idx < ITEMS * NS; idx += kFftThreads) {
    const int it = idx / NS, s = idx % NS;
    const int64_t g = g0 + it, row = g / 8;
    double val = 0.0;
    if (row < n_rows) {
      const int64_t c = row / nvec;
      const int v = (int)(row - c * nvec);
      const int32_t box = child[c * 8 + (g % 8)];
      if (box >= 0) val = M[((int64_t)box * nvec + v) * NS + s];
    }
    sv[it][s] = (T)val;
  }
  __syncthreads();
  // z: real -> complex, kz in [0, p)
  for (int idx = tid; idx < ITEMS * P * P * H; idx += kFftThreads) {
    const int it = idx / (P * P * H);
    const int rem = idx % (P * P * H);
    const int x = rem / (P * H), y = (rem / H) % P, kz = rem % H;
    C2 acc;
    acc.x = T(0);
    acc.y = T(0);
#pragma unroll
    for (int z = 0; z < P; ++z) {
      const int s = l2s[(x * P + y) * P + z];
      if (s >= 0) {
        const T d = sv[it][s];
        const C2 wz = w[(kz * z) % N];
        acc.x += d * wz.x;
        acc.y += d * wz.y;
      }
    }
    a1[it][x][y][kz] = acc;
  }
  __syncthreads();
  // y then x; each task owns one (ky, kz) column of one item
  for (int idx = tid; idx < ITEMS * N * H; idx += kFftThreads) {
    const int it = idx % ITEMS, col = idx / ITEMS;
    const int ky = col / H, kz = col % H;
    const int64_t g = g0 + it, row = g / 8;
    if (row >= n_rows) continue;
    C2 cx[P];
#pragma unroll
    for (int x = 0; x < P; ++x) {
      C2 acc;
      acc.x = T(0);
      acc.y = T(0);
#pragma unroll
      for (int y = 0; y < P; ++y) {
        const C2 t = cmul(a1[it][x][y][kz], w[(ky * y) % N]);
        acc.x += t.x;
        acc.y += t.y;
      }
      cx[x] = acc;
    }
#pragma unroll
    for (int kx = 0; kx < N; ++kx) {
      C2 acc;
      acc.x = T(0);
      acc.y = T(0);
#pragma unroll
      for (int x = 0; x < P; ++x) {
        const C2 t = cmul(cx[x], w[(kx * x) % N]);
        acc.x += t.x;
        acc.y += t.y;
      }
      const int64_t f = ((int64_t)kx * N + ky) * H + kz;
      Qhat[(f * n_rows + row) * 8 + (g % 8)] = acc;
    }
  }
}

template <typename T, int P, int ITEMS>
__global__ __launch_bounds__(kFftThreads) void fft_inverse_kernel(
    const typename C2T<T>::type* __restrict__ Phat, const int32_t* __restrict__ child,
    int64_t n_rows, int nvec, const int16_t* __restrict__ surf_lat,
    const typename C2T<T>::type* __restrict__ tw, double scale, double* __restrict__ out) {
  using C2 = typename C2T<T>::type;
  constexpr int N = 2 * P - 1, H = P, NS = 6 * (P - 1) * (P - 1) + 2;
  __shared__ C2 w[N];
  __shared__ C2 b2[ITEMS][P][N][H];
  __shared__ C2 b1[ITEMS][P][P][H];
  const int tid = threadIdx.x;
  const int64_t g0 = (int64_t)blockIdx.x * ITEMS;
  for (int t = tid; t < N; t += kFftThreads) w[t] = tw[t];
  __syncthreads();
  // x: complex inverse, only x in [0, p) is kept
  for (int idx = tid; idx < ITEMS * N * H; idx += kFftThreads) {
    const int it = idx % ITEMS, col = idx / ITEMS;
    const int ky = col / H, kz = col % H;
    const int64_t g = g0 + it, row = g / 8;
    C2 v[N];
#pragma unroll
    for (int kx = 0; kx < N; ++kx) {
      const int64_t f = ((int64_t)kx * N + ky) * H + kz;
      if (row < n_rows) {
        v[kx] = Phat[(f * n_rows + row) * 8 + (g % 8)];
      } else {
        v[kx].x = T(0);
        v[kx].y = T(0);
      }
    }
#pragma unroll
    for (int x = 0; x < P; ++x) {
      C2 acc;
      acc.x = T(0);
      acc.y = T(0);
#pragma unroll
      for (int kx = 0; kx < N; ++kx) {
        const C2 t = cmulc(v[kx], w[(kx * x) % N]);
        acc.x += t.x;
        acc.y += t.y;
      }
      b2[it][x][ky][kz] = acc;
    }
  }
  __syncthreads();
  // y: complex inverse, y in [0, p)
  for (int idx = tid; idx < ITEMS * P * P * H; idx += kFftThreads) {
    const int it = idx / (P * P * H);
    const int rem = idx % (P * P * H);
    const int x = rem / (P * H), y = (rem / H) % P, kz = rem % H;
    C2 acc;
    acc.x = T(0);
    acc.y = T(0);
#pragma unroll
    for (int ky = 0; ky < N; ++ky) {
      const C2 t = cmulc(b2[it][x][ky][kz], w[(ky * y) % N]);
      acc.x += t.x;
      acc.y += t.y;
    }
    b1[it][x][y][kz] = acc;
  }
  __syncthreads();
  // z: complex -> real on the check-surface points only
  for (int idx = tid; idx < ITEMS * NS; idx += kFftThreads) {
    const int it = idx / NS, s = idx % NS;
    const int64_t g = g0 + it, row = g / 8;
    if (row >= n_rows) continue;
    const int64_t c = row / nvec;
    const int v = (int)(row - c * nvec);
    const int32_t box = child[c * 8 + (g % 8)];
    if (box < 0) continue;
    const int x = surf_lat[3 * s], y = surf_lat[3 * s + 1], z = surf_lat[3 * s + 2];
    T val = b1[it][x][y][0].x;
    T acc = T(0);
#pragma unroll
    for (int kz = 1; kz < H; ++kz) acc += cmulc(b1[it][x][y][kz], w[(kz * z) % N]).x;
    val += T(2) * acc;
    out[((int64_t)box * nvec + v) * NS + s] = scale * (double)val;
  }
}

// ---- Hadamard products on MFMA ---------------------------------------------

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// accumulator row of element i of lane group g (measured lane layouts)
__device__ inline int out_row(float, int g, int i) { return 4 * g + i; }
__device__ inline int out_row(double, int g, int i) { return g + 4 * i; }

template <typename T> struct V4T;
template <> struct V4T<float> { using type = v4f; };
template <> struct V4T<double> { using type = v4d; };

constexpr int kHadThreads = 256;

template <typename T> struct Vec4T;
template <> struct Vec4T<float> { using type = float4; };
template <> struct Vec4T<double> { using type = double4; };

// directions handled per batch of loads in the gather form: all 26 in
// FP32, 13 in FP64 to stay within the register file
template <typename T> struct HadChunk { static constexpr int value = 26; };
template <> struct HadChunk<double> { static constexpr int value = 13; };

__device__ inline float4 load4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ inline double4 load4(const double* p) {
  const double2 lo = *reinterpret_cast<const double2*>(p);
  const double2 hi = *reinterpret_cast<const double2*>(p + 2);
  return double4{lo.x, lo.y, hi.x, hi.y};
}

// Gather form (FP64).  Workgroup = one frequency x a chunk of 16-row tiles;
// four waves share the
// frequency's B operand (the 416 x 16 real form of its 26 x 8 x 8
// complex kernel coefficients), staged in LDS in the lanes' operand order.
// The
// source spectra are gathered through the halo table with 32-bit offsets
// from the frequency's base; absent neighbours point at the empty cluster,
// so the gather needs no masking and the VALU work per MFMA stays small
// (on gfx950 the VALU does not co-issue with the MFMA of the same wave).
template <typename T>
__global__ __launch_bounds__(kHadThreads) void hadamard_gather_kernel(
    const typename C2T<T>::type* __restrict__ Khat, const T* __restrict__ Qhat,
    const int32_t* __restrict__ halo, int64_t n_c, int nvec, int64_t n_rows, int n_chunks,
    int tiles_per_wave, int64_t total_blocks, T* __restrict__ Phat) {
  using C2 = typename C2T<T>::type;
  using V4 = typename V4T<T>::type;
  using T4 = typename Vec4T<T>::type;
  constexpr int DC = HadChunk<T>::value;
  __shared__ T4 Bl[26][64];
  const int64_t b = blockIdx.x;
  const int64_t per_xcd = (total_blocks + 7) / 8;
  const int64_t logical = (b % 8) * per_xcd + b / 8;  // consecutive work per XCD
  if (logical >= total_blocks) return;
  const int64_t f = logical / n_chunks;
  const int chunk = (int)(logical % n_chunks);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 26 * 64; idx += kHadThreads) {
    const int d = idx / 64, lane = idx % 64;
    const int n = lane % 16, g = lane / 16;
    const int i = n / 2, cout = n % 2;
    T val[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int j = 2 * g + s / 2, cin = s % 2;
      const C2 K = Khat[((f * 26 + d) * 8 + i) * 8 + j];
      if (cin == 0)
        val[s] = cout == 0 ? K.x : K.y;
      else
        val[s] = cout == 0 ? -K.y : K.x;
    }
    Bl[d][lane] = T4{val[0], val[1], val[2], val[3]};
  }
  __syncthreads();
  const int wave = tid / 64, lane = tid % 64;
  const int rl = lane % 16, g = lane / 16;
  // this frequency's spectra (n_rows + nvec rows: the empty cluster last)
  // and products; lanes address them with 32-bit byte offsets
  const char* qf = reinterpret_cast<const char*>(Qhat + f * (n_rows + nvec) * 16);
  T* pf = Phat + f * n_rows * 16;
  for (int t = 0; t < tiles_per_wave; ++t) {
    const int64_t tile = ((int64_t)chunk * tiles_per_wave + t) * 4 + wave;
    const int64_t row0 = tile * 16;
    if (row0 >= n_rows) break;
    // rows past the end repeat the last row; their results are not stored
    const uint32_t row = (uint32_t)min(row0 + rl, n_rows - 1);
    const uint32_t c = row / (uint32_t)nvec;
    const uint32_t lane_off = ((row - c * (uint32_t)nvec) * 16 + 4 * g) * (uint32_t)sizeof(T);
    // two accumulators (even / odd directions) so consecutive MFMAs are
    // independent
    V4 acc0, acc1;
    acc0[0] = acc0[1] = acc0[2] = acc0[3] = T(0);
    acc1 = acc0;
#pragma unroll
    for (int d0 = 0; d0 < 26; d0 += DC) {
      T4 a[DC];
#pragma unroll
      for (int dd = 0; dd < DC; ++dd) {
        const int32_t* hd = halo + (int64_t)(d0 + dd) * n_c;
        const uint32_t nb = (uint32_t)hd[c];
        const uint32_t off = __umul24(nb, (uint32_t)nvec) * (16 * (uint32_t)sizeof(T)) + lane_off;
        a[dd] = load4(reinterpret_cast<const T*>(qf + off));
      }
#pragma unroll
      for (int dd = 0; dd < DC; ++dd) {
        const T4 bv = Bl[d0 + dd][lane];
        V4& acc = ((d0 + dd) & 1) ? acc1 : acc0;
        acc = mfma16(a[dd].x, bv.x, acc);
        acc = mfma16(a[dd].y, bv.y, acc);
        acc = mfma16(a[dd].z, bv.z, acc);
        acc = mfma16(a[dd].w, bv.w, acc);
      }
    }
    V4 acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = acc0[i] + acc1[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = row0 + out_row(T(0), g, i);
      if (r < n_rows) pf[r * 16 + rl] = acc[i];
    }
  }
}

constexpr int kHadSrcMax = 216;  // source slots of one 4 x 4 x 4 block: its 6 x 6 x 6 shell
constexpr int kHadStage = (kHadSrcMax * 4 + kHadThreads - 1) / kHadThreads;

// Block form (FP32).  Workgroup = one frequency x a run of (block, charge
// vector) items.  Each lane holds the frequency's B operand for all 26
// directions in registers (the 416 x 16 real form of the 26 x 8 x 8 complex
// kernel coefficients, in its operand order).  Per item the spectra of the
// block's source clusters (at most 216 rows of 16 reals) are staged in LDS
// - the next item's rows are loaded into registers while the current one
// computes - and each wave takes one 16-cluster tile of the block's (at
// most 64) target clusters, reading its A operands at the slots of the
// clusters' 26 neighbours.  A source slot is 8 x rank + the parity class of
// the source's position, so the eight clusters of an aligned 2 x 2 x 2 cube
// (eight consecutive lanes) always read distinct LDS banks.  Every source
// spectrum crosses the cache hierarchy once per block, and the VALU work per
// MFMA stays small (on gfx950 the VALU does not co-issue with the MFMA of the
// same wave).
__global__ __launch_bounds__(kHadThreads, 3) void hadamard_block_kernel(
    const float2* __restrict__ Khat, const float* __restrict__ Qhat,
    const int32_t* __restrict__ blk_tgt, const int32_t* __restrict__ blk_src,
    const int32_t* __restrict__ blk_list, const uint32_t* __restrict__ slots, int64_t n_items,
    int nvec, int64_t n_rows, int items_per_wg, int n_groups, int64_t total_wgs,
    float* __restrict__ Phat) {
  constexpr int kRow = 5;  // LDS row stride in float4: 16 reals + padding
  __shared__ float4 As[2][kHadSrcMax * kRow + 1];  // + one discard entry
  const int64_t b = blockIdx.x;
  const int64_t per_xcd = (total_wgs + 7) / 8;
  const int64_t logical = (b % 8) * per_xcd + b / 8;  // consecutive work per XCD
  if (logical >= total_wgs) return;
  const int64_t f = logical / n_groups;
  const int64_t item0 = (logical % n_groups) * items_per_wg;
  const int64_t item1 = min(item0 + items_per_wg, n_items);
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int rl = lane % 16, g = lane / 16;
  // B operand: lane (n, g) multiplies inputs 2g, 2g + 1 (real, imaginary
  // parts) into output n / 2, real part for even n and imaginary for odd n
  float4 B[26];
#pragma unroll
  for (int d = 0; d < 26; ++d) {
    const float4 k =
        *reinterpret_cast<const float4*>(&Khat[((f * 26 + d) * 8 + rl / 2) * 8 + 2 * g]);
    B[d] = (rl & 1) ? float4{k.y, k.x, k.w, k.z} : float4{k.x, -k.y, k.z, -k.w};
  }
  // this frequency's spectra (n_rows + nvec rows: the empty cluster last)
  const char* qf = reinterpret_cast<const char*>(Qhat + f * (n_rows + nvec) * 16);
  float* pf = Phat + f * n_rows * 16;
  const int tr0 = wave * 16;  // this wave's tile of the block's targets
  // staging registers: four 16-byte pieces per thread (216 rows x 4 pieces
  // over 256 threads), named rather than an array so they stay in VGPRs
  static_assert(kHadStage == 4, "staging pieces per thread");
  float4 stg0, stg1, stg2, stg3;
  int sl0 = 0, sl1 = 0, sl2 = 0, sl3 = 0;
  uint32_t w[7], wn[7];
  int buf = 0;
  // iteration `it` issues the loads of item it (into registers) and then
  // computes item it - 1, whose rows the previous iteration loaded
  for (int64_t it = item0; it <= item1; ++it) {
    if (it > item0) {
      As[buf][sl0] = stg0;
      As[buf][sl1] = stg1;
      As[buf][sl2] = stg2;
      As[buf][sl3] = stg3;
#pragma unroll
      for (int k = 0; k < 7; ++k) w[k] = wn[k];
      __syncthreads();  // As[buf] complete; As[buf ^ 1] free for the next item
    }
    if (it < item1) {
      const int64_t blk = it / nvec;
      const uint32_t v = (uint32_t)(it - blk * nvec);
      const int s0 = blk_src[blk], ns = blk_src[blk + 1] - s0;
      const int t0 = blk_tgt[blk], nt = blk_tgt[blk + 1] - t0;
      // piece k of this thread: row (tid + 256 k) / 4, quarter tid % 4;
      // threads past the list read its first entry into the discard entry
      auto piece = [&](int k, float4& st, int& slot) __attribute__((always_inline)) {
        const int idx = tid + kHadThreads * k, r = idx >> 2, part = idx & 3;
        const int32_t e = blk_list[s0 + (r < ns ? r : 0)];
        const uint32_t src = (uint32_t)e >> 8;
        const uint32_t off = ((src * (uint32_t)nvec + v) * 16 + 4 * part) * 4u;
        st = *reinterpret_cast<const float4*>(qf + off);
        slot = r < ns ? (e & 255) * kRow + part : kHadSrcMax * kRow;
      };
      piece(0, stg0, sl0);
      piece(1, stg1, sl1);
      piece(2, stg2, sl2);
      piece(3, stg3, sl3);
      const int tr = min(tr0 + rl, nt - 1);
#pragma unroll
      for (int k = 0; k < 7; ++k) wn[k] = slots[(int64_t)(t0 + tr) * 7 + k];
    }
    if (it == item0) continue;
    const int64_t item = it - 1;
    const int64_t blk = item / nvec;
    const int v = (int)(item - blk * nvec);
    const int t0 = blk_tgt[blk], nt = blk_tgt[blk + 1] - t0;
    const int cur = buf;
    buf ^= 1;
    if (tr0 >= nt) continue;
    // two accumulators (even / odd directions) so consecutive MFMAs are
    // independent
    v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
    for (int d = 0; d < 26; ++d) {
      const uint32_t slot = (w[d / 4] >> (8 * (d % 4))) & 0xffu;
      const float4 a = As[cur][slot * kRow + g];
      v4f& acc = (d & 1) ? acc1 : acc0;
      acc = mfma16(a.x, B[d].x, acc);
      acc = mfma16(a.y, B[d].y, acc);
      acc = mfma16(a.z, B[d].z, acc);
      acc = mfma16(a.w, B[d].w, acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int to = tr0 + out_row(0.f, g, i);
      if (to < nt) pf[((int64_t)(t0 + to) * nvec + v) * 16 + rl] = acc0[i] + acc1[i];
    }
  }
}

template <typename T, int P, int ITEMS>
hipError_t fwd_launch(const double* M, const int32_t* child, int64_t n_rows, int nvec,
                      const int16_t* lat2surf, const void* tw, void* Qhat, hipStream_t s) {
  using C2 = typename C2T<T>::type;
  const int64_t items = n_rows * 8;
  const unsigned grid = (unsigned)((items + ITEMS - 1) / ITEMS);
  fft_forward_kernel<T, P, ITEMS><<<grid, kFftThreads, 0, s>>>(M, child, n_rows, nvec, lat2surf,
                                                             (const C2*)tw, (C2*)Qhat);
  return hipGetLastError();
}

template <typename T, int P, int ITEMS>
hipError_t inv_launch(const void* Phat, const int32_t* child, int64_t n_rows, int nvec,
                      const int16_t* surf_lat, const void* tw, double scale, double* out,
                      hipStream_t s) {
  using C2 = typename C2T<T>::type;
  const int64_t items = n_rows * 8;
  const unsigned grid = (unsigned)((items + ITEMS - 1) / ITEMS);
  fft_inverse_kernel<T, P, ITEMS><<<grid, kFftThreads, 0, s>>>((const C2*)Phat, child, n_rows, nvec,
                                                             surf_lat, (const C2*)tw, scale, out);
  return hipGetLastError();
}

// items per workgroup, sized so the LDS stays within 64 KiB
template <typename T, int P> struct Items {
  static constexpr int bytes = sizeof(T) * 2;
  static constexpr int per = P * (2 * P - 1) * P * bytes + P * P * P * bytes;  // inverse
  static constexpr int raw = 49152 / per;
  static constexpr int value = raw >= 16 ? 16 : raw >= 8 ? 8 : raw >= 4 ? 4 : raw >= 2 ? 2 : 1;
};

template <typename T>
hipError_t fwd_dispatch(int p, const double* M, const int32_t* child, int64_t n_rows, int nvec,
                        const int16_t* l2s, const void* tw, void* Q, hipStream_t s) {
  switch (p) {
#define KIFMM_FWD(PP) \
  case PP: return fwd_launch<T, PP, Items<T, PP>::value>(M, child, n_rows, nvec, l2s, tw, Q, s);
    KIFMM_FWD(2) KIFMM_FWD(3) KIFMM_FWD(4) KIFMM_FWD(5) KIFMM_FWD(6) KIFMM_FWD(7) KIFMM_FWD(8)
#undef KIFMM_FWD
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t inv_dispatch(int p, const void* Ph, const int32_t* child, int64_t n_rows, int nvec,
                        const int16_t* sl, const void* tw, double scale, double* out, hipStream_t s) {
  switch (p) {
#define KIFMM_INV(PP) \
  case PP: return inv_launch<T, PP, Items<T, PP>::value>(Ph, child, n_rows, nvec, sl, tw, scale, out, s);
    KIFMM_INV(2) KIFMM_INV(3) KIFMM_INV(4) KIFMM_INV(5) KIFMM_INV(6) KIFMM_INV(7) KIFMM_INV(8)
#undef KIFMM_INV
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fft_forward(int p, bool fp64, const double* M, const int32_t* child,
                              int64_t n_clusters, int nvec, const int16_t* lat2surf,
                              const void* twiddle, void* Qhat, hipStream_t stream) {
  const int64_t n_rows = n_clusters * nvec;
  if (n_rows == 0) return hipSuccess;
  return fp64 ? fwd_dispatch<double>(p, M, child, n_rows, nvec, lat2surf, twiddle, Qhat, stream)
              : fwd_dispatch<float>(p, M, child, n_rows, nvec, lat2surf, twiddle, Qhat, stream);
}

hipError_t launch_fft_inverse(int p, bool fp64, const void* Phat, const int32_t* child,
                              int64_t n_clusters, int nvec, const int16_t* surf_lat,
                              const void* twiddle, double scale, double* out, hipStream_t stream) {
  const int64_t n_rows = n_clusters * nvec;
  if (n_rows == 0) return hipSuccess;
  return fp64 ? inv_dispatch<double>(p, Phat, child, n_rows, nvec, surf_lat, twiddle, scale, out, stream)
              : inv_dispatch<float>(p, Phat, child, n_rows, nvec, surf_lat, twiddle, scale, out, stream);
}

hipError_t launch_hadamard(bool fp64, int F, const void* Khat, const void* Qhat,
                           const int32_t* halo, int64_t n_blocks, const int32_t* blk_tgt,
                           const int32_t* blk_src, const int32_t* blk_list, const uint32_t* slots,
                           int64_t n_clusters, int nvec, void* Phat, hipStream_t stream) {
  const int64_t n_rows = n_clusters * nvec;
  if (n_rows == 0) return hipSuccess;
  // 24-bit cluster indices and 32-bit byte offsets within one frequency
  if (n_clusters + 1 >= (int64_t(1) << 23) ||
      (n_clusters + 1) * nvec * 16 * (fp64 ? 8 : 4) >= (int64_t(1) << 32))
    return hipErrorInvalidValue;
  if (fp64) {
    const int64_t tiles = (n_rows + 15) / 16;
    const int tpw = tiles >= 256 ? 8 : tiles >= 64 ? 4 : 1;
    const int n_chunks = (int)((tiles + 4 * tpw - 1) / (4 * tpw));
    const int64_t total = (int64_t)F * n_chunks;
    const unsigned grid = (unsigned)(8 * ((total + 7) / 8));
    hadamard_gather_kernel<double><<<grid, kHadThreads, 0, stream>>>(
        (const double2*)Khat, (const double*)Qhat, halo, n_clusters, nvec, n_rows, n_chunks, tpw,
        total, (double*)Phat);
    return hipGetLastError();
  }
  const int64_t n_items = n_blocks * nvec;
  const int ipw = n_items >= 64 ? 8 : n_items >= 16 ? 4 : 1;
  const int n_groups = (int)((n_items + ipw - 1) / ipw);
  const int64_t total = (int64_t)F * n_groups;
  const unsigned grid = (unsigned)(8 * ((total + 7) / 8));
  hadamard_block_kernel<<<grid, kHadThreads, 0, stream>>>(
      (const float2*)Khat, (const float*)Qhat, blk_tgt, blk_src, blk_list, slots, n_items, nvec,
      n_rows, ipw, n_groups, total, (float*)Phat);
  return hipGetLastError();
}

}  // namespace kifmm
