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
// The transforms are direct sums along each axis with the n x p twiddle
// matrix Wm[k][j] = exp(-2 pi i (k j mod n) / n).
#include "group.h"
#include "kernels.h"

namespace kifmm {

namespace {

template <typename T> struct C2T;
template <> struct C2T<float> { using type = float2; };
template <> struct C2T<double> { using type = double2; };

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
// Row r of an A operand whose product row out_row(g, i) is to hold logical
// row 4 g + i (so each lane's four outputs are consecutive logical rows)
__device__ inline int a_row(float, int r) { return r; }
__device__ inline int a_row(double, int r) { return 4 * (r % 4) + r / 4; }

template <typename T> struct V4T;
template <> struct V4T<float> { using type = v4f; };
template <> struct V4T<double> { using type = v4d; };

// acc += a * w and acc += a * conj(w) as four FMAs each
template <typename C2>
__device__ inline void cmac(C2& acc, C2 a, C2 w) {
  acc.x = fma(a.x, w.x, acc.x);
  acc.x = fma(-a.y, w.y, acc.x);
  acc.y = fma(a.x, w.y, acc.y);
  acc.y = fma(a.y, w.x, acc.y);
}
template <typename C2>
__device__ inline void cmacc(C2& acc, C2 a, C2 w) {
  acc.x = fma(a.x, w.x, acc.x);
  acc.x = fma(a.y, w.y, acc.x);
  acc.y = fma(a.y, w.x, acc.y);
  acc.y = fma(-a.x, w.y, acc.y);
}

// LDS layout of the separable transforms, per order P and complex width
// (W = 2 dwords for FP32, 4 for FP64): `items` (row, child) boxes per
// workgroup; the z-stage buffer a1[item][x][y][kz] and the x/y-stage buffer
// a2[item][x][ky][kz] (complex units).  The strides are padded so that the
// lanes of each stage hit distinct LDS banks as far as possible (chosen by
// a bank model of the three stages' access patterns).
template <int P, int W> struct FftLds;
#define KIFMM_FFT_LDS(PP, WW, IT, A, B, C, D, E, F)                                   \
  template <> struct FftLds<PP, WW> {                                                \
    static constexpr int items = IT, s1y = A, s1x = B, s1i = C, s2k = D, s2x = E, s2i = F; \
  };
KIFMM_FFT_LDS(2, 2, 8, 3, 6, 12, 2, 8, 18)
KIFMM_FFT_LDS(2, 4, 8, 3, 6, 12, 2, 6, 13)
KIFMM_FFT_LDS(3, 2, 8, 4, 19, 57, 3, 19, 58)
KIFMM_FFT_LDS(3, 4, 8, 4, 19, 57, 3, 19, 57)
KIFMM_FFT_LDS(4, 2, 8, 5, 20, 80, 4, 28, 114)
KIFMM_FFT_LDS(4, 4, 8, 5, 20, 80, 4, 28, 113)
KIFMM_FFT_LDS(5, 2, 8, 5, 25, 125, 5, 53, 266)
KIFMM_FFT_LDS(5, 4, 4, 6, 37, 185, 5, 45, 226)
KIFMM_FFT_LDS(6, 2, 8, 7, 42, 252, 6, 70, 422)
KIFMM_FFT_LDS(6, 4, 4, 7, 42, 252, 6, 70, 422)
KIFMM_FFT_LDS(7, 2, 4, 7, 54, 383, 7, 103, 724)
KIFMM_FFT_LDS(7, 4, 2, 7, 49, 343, 7, 95, 668)
KIFMM_FFT_LDS(8, 2, 2, 9, 72, 576, 8, 120, 968)
KIFMM_FFT_LDS(8, 4, 1, 9, 72, 576, 8, 120, 960)
#undef KIFMM_FFT_LDS

template <typename T, int P> struct FftCfg {
  using L = FftLds<P, (int)sizeof(T) / 2>;
  static constexpr int items = L::items;
  // one thread per line of the z stage, and at least seven waves: the MFMA
  // stages then spread over more waves and the persistent grid holds fewer,
  // larger workgroups, which runs faster beside the coarse levels' M2L
  static constexpr int lines = (items * P * P + 63) / 64 * 64;
  static constexpr int threads = lines > 448 ? lines : 448;
};

// Forward transforms of `items` boxes per workgroup in three stages, with
// the twiddle matrix Wm[k][j] = exp(-2 pi i (k j mod n) / n) (n x p):
//   z: a1[x][y][kz] = sum_z d(x, y, z) Wm[kz][z]        (real input, kz < p;
//      VALU, one thread per line, twiddles at wave-uniform addresses)
//   y: a2[x][ky][kz] = sum_y a1[x][y][kz] Wm[ky][y]     (ky < n)
//   x: Qhat[f][row][child] = sum_x a2[x][ky][kz] Wm[kx][x], f = (kx n + ky) p + kz.
// The y and x stages are real products on MFMA: the 2n x 2p real form of Wm
// (held in registers) times 16-column tiles of the lines' real and
// imaginary parts.
// Box item g is child g % 8 of row g / 8 (row = cluster * nvec + v).
template <typename T, int P>
__device__ __forceinline__ void fft_forward_body(const FwdArgs& a, int64_t blk, int64_t nblk) {
  using C2 = typename C2T<T>::type;
  const double* __restrict__ M = a.M;
  const int32_t* __restrict__ child = a.child;
  const int64_t n_rows = a.n_rows;
  const int nvec = a.nvec;
  const int16_t* __restrict__ lat2surf = a.lat2surf;
  const C2* __restrict__ Wm = static_cast<const C2*>(a.wm);
  C2* __restrict__ Qhat = static_cast<C2*>(a.Qhat);
  using L = typename FftCfg<T, P>::L;
  constexpr int N = 2 * P - 1, H = P, NS = 6 * (P - 1) * (P - 1) + 2;
  constexpr int IT = FftCfg<T, P>::items, TH = FftCfg<T, P>::threads;
  __shared__ C2 a1[IT * L::s1i];
  __shared__ C2 a2[IT * L::s2i];
  // densities of the group being transformed on the p^3 lattice (zero off
  // the surface: the interior is never written), and each surface point's
  // lattice index
  __shared__ T dl[IT * P * P * P];
  __shared__ int16_t s2l[NS];
  static_assert(IT <= 8 && 8 % IT == 0, "an item group lies within one row");
  const int tid = threadIdx.x;
  // Persistent workgroups: while group gc is transformed, the densities of
  // group gc + nwg are loaded into registers (issued before the z stage,
  // written to dl after the y stage).  The group's eight child box indices
  // are read with scalar loads, so no vector-memory wait (which would also
  // wait for the previous group's spectrum stores) sits between them and
  // the density loads.  Logical workgroups are numbered per XCD, so at each
  // iteration an XCD works on consecutive rows and the two 64-byte halves
  // of a 128-byte line of Qhat meet in the same L2.
  constexpr int KL = (IT * NS + TH - 1) / TH;
  const int64_t n_groups = (n_rows * 8 + IT - 1) / IT;
  const int64_t nwg = nblk, per_xcd = nwg / 8;  // grid: a multiple of 8
  const int64_t wg = (blk % 8) * per_xcd + blk / 8;
  for (int t = tid; t < P * P * P; t += TH) {
    const int sidx = lat2surf[t];
    if (sidx >= 0) s2l[sidx] = (int16_t)t;
  }
  for (int t = tid; t < IT * P * P * P; t += TH) dl[t] = T(0);
  __syncthreads();
  // MFMA operand A of the y and x stages: the real form of Wm, rows
  // (k, re/im), columns (j, re/im); lane (lc, lg) holds row lc, column lg of
  // each 16 x 4 block, rows ordered so that lane (lc, g) of a product holds
  // the real and imaginary parts of outputs k = 8 mt + 2 g and 8 mt + 2 g + 1
  using V4 = typename V4T<T>::type;
  constexpr int MT = (2 * N + 15) / 16, KS = (2 * P + 3) / 4, NW = TH / 64;
  const int wave = tid / 64, lc = tid % 16, lg = (tid % 64) / 16;
  T Ar[MT][KS];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int m = 16 * mt + a_row(T(0), lc), k = 4 * ks + lg;
      T val = T(0);
      if (m < 2 * N && k < 2 * P) {
        const C2 w = Wm[(m >> 1) * P + (k >> 1)];
        val = (m & 1) ? ((k & 1) ? w.x : w.y) : ((k & 1) ? -w.y : w.x);
      }
      Ar[mt][ks] = val;
    }
  // MFMA operand A of the z stage: the real form of Wm[kz][z] on real
  // input, rows (kz, re/im), columns z
  constexpr int KZ = (P + 3) / 4;
  static_assert(2 * H <= 16, "one 16-row tile holds a z line's outputs");
  T Az[KZ];
#pragma unroll
  for (int ks = 0; ks < KZ; ++ks) {
    const int m = a_row(T(0), lc), z = 4 * ks + lg;
    T val = T(0);
    if (m < 2 * H && z < P) {
      const C2 w = Wm[(m >> 1) * P + z];
      val = (m & 1) ? w.y : w.x;
    }
    Az[ks] = val;
  }
  const T* a1f = reinterpret_cast<const T*>(a1);
  const T* a2f = reinterpret_cast<const T*>(a2);
  // densities of group gl into pre (box indices of absent children read
  // box 0; their values are masked when written to dl), and the lattice
  // offset in dl of each of the thread's surface values
  double pre[KL];
  uint32_t okm = 0;
  int dlo[KL];
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    const int idx = tid + TH * k;
    const int it = idx < IT * NS ? idx / NS : 0, sidx = idx - it * NS;
    // (clamped: every surface point has its lattice point, so the clamp never acts)
    dlo[k] = idx < IT * NS ? it * P * P * P + min(max((int)s2l[sidx], 0), P * P * P - 1) : 0;
  }
  auto load_group = [&](int64_t gl) __attribute__((always_inline)) {
    const int64_t g0 = gl * IT;
    const uint32_t row = (uint32_t)(g0 / 8), c = row / (uint32_t)nvec;
    const int v = (int)(row - c * (uint32_t)nvec);
    int32_t cb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) cb[j] = child[(int64_t)c * 8 + j];  // uniform: scalar loads
    okm = 0;
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int idx = tid + TH * k;
      const int it = idx < IT * NS ? idx / NS : 0, sidx = idx - it * NS;
      int32_t box = cb[0];
#pragma unroll
      for (int j = 1; j < 8; ++j)
        if ((int)(g0 % 8) + it == j) box = cb[j];
      const bool ok = idx < IT * NS && box >= 0;
      okm |= (uint32_t)ok << k;
      pre[k] = M[((int64_t)(ok ? box : 0) * nvec + v) * NS + (ok ? sidx : 0)];
    }
  };
  auto store_group = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int idx = tid + TH * k;
      if (idx < IT * NS) dl[dlo[k]] = (okm >> k) & 1 ? (T)pre[k] : T(0);
    }
  };
  if (wg >= n_groups) return;
  load_group(wg);
  store_group();
  __syncthreads();
  for (int64_t gc = wg; gc < n_groups; gc += nwg) {
    // past the last group the current one is loaded again (unused), so the
    // loads and their stores to dl stay unconditional
    const int64_t gn = gc + nwg, g0 = gc * IT;
    load_group(gn < n_groups ? gn : gc);
    // z stage on MFMA: a1[(kz, re/im)][line] = Az x dl[line][z], line =
    // (item, x, y); columns past the last line read the last one (zero
    // columns of Az past z = p - 1 take any finite value)
    {
      constexpr int NC = IT * P * P, NT = (NC + 15) / 16;
      for (int t = wave; t < NT; t += NW) {
        const int col = 16 * t + lc;
        const int cc = col < NC ? col : NC - 1;
        const T* src = dl + cc * P;
        V4 acc = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < KZ; ++ks) acc = mfma16(Az[ks], src[min(4 * ks + lg, P - 1)], acc);
        if (col < NC) {
          const int it = cc / (P * P), x = (cc / P) % P, y = cc % P;
          C2* o = a1 + it * L::s1i + x * L::s1x + y * L::s1y;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int kz = 2 * lg + h;
            if (kz < H) o[kz] = C2{acc[2 * h], acc[2 * h + 1]};
          }
        }
      }
    }
    __syncthreads();
    // y stage on MFMA: a2[(ky, re/im)][col] = Ar x a1[(y, re/im)][col],
    // col = (item, x, kz), kz fastest
    {
      constexpr int NC = IT * P * H, NT = (NC + 15) / 16;
      for (int t = wave; t < NT; t += NW) {
        const int col = 16 * t + lc;
        const bool ok = col < NC;
        const int cc = ok ? col : 0;
        const int kz = cc % H, x = (cc / H) % P, it = cc / (H * P);
        const int b1 = 2 * (it * L::s1i + x * L::s1x + kz);
        V4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + lg;  // (y, re/im)
          const T bv = a1f[b1 + (k < 2 * P ? (k >> 1) * 2 * L::s1y + (k & 1) : 0)];
          const T b = (ok && k < 2 * P) ? bv : T(0);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma16(Ar[mt][ks], b, acc[mt]);
        }
        C2* o2 = a2 + it * L::s2i + x * L::s2x + kz;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int ky = 8 * mt + 2 * lg + h;
            if (ok && ky < N) o2[ky * L::s2k] = C2{acc[mt][2 * h], acc[mt][2 * h + 1]};
          }
      }
    }
    store_group();  // the z stage is done with dl
    __syncthreads();
    // x stage on MFMA: Qhat(f, row, child) = Ar x a2[(x, re/im)][col],
    // col = (ky, kz, item), item fastest, f = (kx n + ky) p + kz
    {
      constexpr int NC = IT * N * H, NT = (NC + 15) / 16;
      for (int t = wave; t < NT; t += NW) {
        const int col = 16 * t + lc;
        const bool ok = col < NC;
        const int cc = ok ? col : 0;
        const int it = cc % IT, rest = cc / IT;
        const int kz = rest % H, ky = rest / H;
        const int64_t g = g0 + it, row = g / 8;
        const int b2 = 2 * (it * L::s2i + ky * L::s2k + kz);
        V4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + lg;  // (x, re/im)
          const T bv = a2f[b2 + (k < 2 * P ? (k >> 1) * 2 * L::s2x + (k & 1) : 0)];
          const T b = (ok && k < 2 * P) ? bv : T(0);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma16(Ar[mt][ks], b, acc[mt]);
        }
        if (ok && row < n_rows) {
          C2* qrow = Qhat + row * 8 + (g % 8) + ((int64_t)ky * H + kz) * n_rows * 8;
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int kx = 8 * mt + 2 * lg + h;
              if (kx < N) qrow[(int64_t)kx * N * H * n_rows * 8] = C2{acc[mt][2 * h], acc[mt][2 * h + 1]};
            }
        }
      }
    }
  }
}

// Inverse transforms, one (row, child) box per item: complex inverse DFTs
// along x (only x < p kept) and y (y < p), then the complex-to-real step
// along z (odd length: no Nyquist term) at the p^3 lattice points, and the
// check-surface points of those, scaled, stored in surface order.  The x and
// y stages are real products on MFMA: the 2p x 2n real form of the inverse
// twiddles conj(Wm[k][j]) (held in registers) times 16-column tiles of the
// lines' real and imaginary parts; the x stage takes its operand straight
// from the spectra (each lane one complex value per group of four
// frequencies), the y stage from LDS.  The z stage is a VALU sum per line
// with the twiddles at wave-uniform addresses.  The row's child boxes and
// the surface-lattice table are read once per workgroup, so the output
// stores wait on no vector-memory load.
constexpr int kInvThreads = 512;

// LDS layout of the inverse transform per order P and complex width W
// (dwords): `items` boxes per workgroup (within 52 KiB); the x-stage output
// b2[item][x][ky][kz] (strides s2k, s2x, s2i) and the y-stage output
// b1[item][x][y][kz] (strides s1y, s1x, s1i), in complex units, padded so
// that the MFMA stages' stores and operand reads and the z stage's reads
// spread over the banks (chosen by a bank model of those access patterns);
// at p = 6 the padding keeps four workgroups per CU (40 KiB each).
template <int P, int W> struct InvLds;
#define KIFMM_INV_LDS(PP, WW, IT, A, B, C, D, E, F)                                   \
  template <> struct InvLds<PP, WW> {                                                \
    static constexpr int items = IT, s2k = A, s2x = B, s2i = C, s1y = D, s1x = E, s1i = F; \
  };
KIFMM_INV_LDS(2, 2, 8, 2, 7, 20, 2, 5, 12)
KIFMM_INV_LDS(2, 4, 8, 2, 7, 14, 4, 8, 17)
KIFMM_INV_LDS(3, 2, 8, 3, 15, 52, 5, 15, 45)
KIFMM_INV_LDS(3, 4, 8, 3, 15, 46, 3, 9, 27)
KIFMM_INV_LDS(4, 2, 8, 6, 43, 172, 4, 16, 65)
KIFMM_INV_LDS(4, 4, 8, 4, 29, 118, 4, 17, 70)
KIFMM_INV_LDS(5, 2, 8, 6, 55, 276, 5, 25, 125)
KIFMM_INV_LDS(5, 4, 8, 5, 45, 226, 5, 25, 126)
KIFMM_INV_LDS(6, 2, 8, 6, 67, 404, 6, 36, 219)
KIFMM_INV_LDS(6, 4, 4, 6, 67, 404, 6, 36, 217)
KIFMM_INV_LDS(7, 2, 4, 7, 94, 664, 10, 71, 504)
KIFMM_INV_LDS(7, 4, 2, 7, 95, 680, 9, 63, 456)
KIFMM_INV_LDS(8, 2, 4, 9, 138, 1112, 8, 65, 524)
KIFMM_INV_LDS(8, 4, 2, 8, 121, 968, 10, 81, 648)
#undef KIFMM_INV_LDS

template <typename C2>
__device__ inline C2 cmulc(C2 a, C2 b) {  // a * conj(b)
  C2 r;
  r.x = a.x * b.x + a.y * b.y;
  r.y = a.y * b.x - a.x * b.y;
  return r;
}

template <typename T, int P>
__device__ __forceinline__ void fft_inverse_body(const InvArgs& a, int64_t blk) {
  using C2 = typename C2T<T>::type;
  using V4 = typename V4T<T>::type;
  using L = InvLds<P, (int)sizeof(T) / 2>;
  constexpr int ITEMS = L::items;
  const C2* __restrict__ Phat = static_cast<const C2*>(a.Phat);
  const int32_t* __restrict__ child = a.child;
  const int64_t n_rows = a.n_rows;
  const int nvec = a.nvec;
  const int16_t* __restrict__ surf_lat = a.surf_lat;
  const C2* __restrict__ Wm = static_cast<const C2*>(a.wm);
  const double scale = a.scale;
  double* __restrict__ out = a.out;
  constexpr int N = 2 * P - 1, H = P, NS = 6 * (P - 1) * (P - 1) + 2;
  // frequencies in groups of four along a line: K step 2q holds the real
  // parts of frequencies 4q .. 4q + 3 (one per lane group), step 2q + 1
  // their imaginary parts
  constexpr int KQ = (N + 3) / 4, KS = 2 * KQ, NW = kInvThreads / 64;
  static_assert(2 * P <= 16, "one 16-row MFMA tile holds a line's outputs");
  __shared__ C2 b2[ITEMS * L::s2i];
  __shared__ C2 b1[ITEMS * L::s1i];
  __shared__ int16_t sl[3 * NS];
  // real lattice values of the z stage, in b2 (free after the y stage)
  static_assert(sizeof(T) * P * P * P <= sizeof(C2) * L::s2i, "lattice fits in b2");
  T* zb = reinterpret_cast<T*>(b2);
  static_assert(ITEMS <= 8 && 8 % ITEMS == 0, "a workgroup's items lie within one row");
  const int tid = threadIdx.x, wave = tid / 64, lc = tid % 16, lg = (tid % 64) / 16;
  // consecutive rows on one XCD, so the two 64-byte halves of a 128-byte
  // line of Phat are fetched once, into the same L2
  const int64_t nwg = (n_rows * 8 + ITEMS - 1) / ITEMS, per_xcd = (nwg + 7) / 8;
  const int64_t wg = (blk % 8) * per_xcd + blk / 8;
  if (wg >= nwg) return;
  const int64_t g0 = wg * ITEMS;
  // the row's child boxes, read with scalar loads (uniform addresses), so
  // the output stores need no vector-memory wait between them
  const uint32_t row0 = (uint32_t)(g0 / 8), c0 = row0 / (uint32_t)nvec;
  const int v0 = (int)(row0 - c0 * (uint32_t)nvec);
  int32_t cb[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) cb[j] = child[(int64_t)c0 * 8 + j];
  // MFMA operand A: lane (lc, lg) holds logical row m = (j, re/im) of the
  // real form of conj(Wm)^T, column (frequency 4 (ks / 2) + lg, re/im of
  // the input by the parity of ks); rows j >= p and frequencies >= n are 0,
  // so the operand reads past a line's end may take any finite value.  Its
  // twiddles are loaded first, then every x-stage operand of the wave (all
  // loads in flight together; addresses clamped, so the waits count exactly).
  const int m = a_row(T(0), lc), jm = m >> 1;
  C2 wq[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) wq[q] = Wm[min(4 * q + lg, N - 1) * P + min(jm, P - 1)];
  // x: b2[it][j][ky][kz] = sum_kx Phat[(kx n + ky) p + kz][row][child] conj(Wm[kx][j]);
  // columns (item, ky, kz), item fastest, so a lane group's eight columns
  // read one row's contiguous children
  constexpr int NCX = ITEMS * N * H, NTX = (NCX + 15) / 16, TPX = (NTX + NW - 1) / NW;
  C2 vx[TPX][KQ];
  {
    const int64_t fstride = n_rows * 8;  // complex values per frequency
    const C2* __restrict__ base = Phat + (int64_t)row0 * 8 + (g0 % 8);
#pragma unroll
    for (int u = 0; u < TPX; ++u) {
      const int col = min(16 * (wave + u * NW) + lc, NCX - 1);
      const int it = col % ITEMS, rest = col / ITEMS;  // rest = ky p + kz
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const int kx = min(4 * q + lg, N - 1);
        vx[u][q] = base[((int64_t)kx * N * H + rest) * fstride + it];
      }
    }
  }
  T Ar[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const C2 w = wq[ks >> 1];
    // (vr + i vi)(wr - i wi) = (vr wr + vi wi) + i (vi wr - vr wi)
    const T val = (m & 1) ? ((ks & 1) ? w.x : -w.y) : ((ks & 1) ? w.y : w.x);
    Ar[ks] = (jm < P && 4 * (ks >> 1) + lg < N) ? val : T(0);
  }
#pragma unroll
  for (int u = 0; u < TPX; ++u) {
    const int t = wave + u * NW;
    if (t < NTX) {
      V4 acc = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        acc = mfma16(Ar[2 * q], vx[u][q].x, acc);
        acc = mfma16(Ar[2 * q + 1], vx[u][q].y, acc);
      }
      const int col = 16 * t + lc;
      if (col < NCX) {
        const int it = col % ITEMS, rest = col / ITEMS, ky = rest / H, kz = rest % H;
        C2* o = b2 + it * L::s2i + ky * L::s2k + kz;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = 2 * lg + h;
          if (j < P) o[j * L::s2x] = C2{acc[2 * h], acc[2 * h + 1]};
        }
      }
    }
  }
  // the surface-lattice table, loaded after the spectra (its wait would
  // otherwise hold back their loads)
  for (int t = tid; t < 3 * NS; t += kInvThreads) sl[t] = surf_lat[t];
  __syncthreads();
  // y: b1[it][x][j][kz] = sum_ky b2[it][x][ky][kz] conj(Wm[ky][j]);
  // columns (item, x, kz), item fastest; the wave's operands are read first
  {
    constexpr int NC = ITEMS * P * H, NT = (NC + 15) / 16, TPY = (NT + NW - 1) / NW;
    C2 vy[TPY][KQ];
#pragma unroll
    for (int u = 0; u < TPY; ++u) {
      const int col = min(16 * (wave + u * NW) + lc, NC - 1);
      const int it = col % ITEMS, x = (col / ITEMS) % P, kz = col / (ITEMS * P);
      const C2* src = b2 + it * L::s2i + x * L::s2x + kz;
#pragma unroll
      for (int q = 0; q < KQ; ++q) vy[u][q] = src[min(4 * q + lg, N - 1) * L::s2k];
    }
#pragma unroll
    for (int u = 0; u < TPY; ++u) {
      const int t = wave + u * NW, col = 16 * t + lc;
      if (t < NT) {
        V4 acc = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
          acc = mfma16(Ar[2 * q], vy[u][q].x, acc);
          acc = mfma16(Ar[2 * q + 1], vy[u][q].y, acc);
        }
        if (col < NC) {
          const int it = col % ITEMS, x = (col / ITEMS) % P, kz = col / (ITEMS * P);
          C2* o = b1 + it * L::s1i + x * L::s1x + kz;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int j = 2 * lg + h;
            if (j < P) o[j * L::s1y] = C2{acc[2 * h], acc[2 * h + 1]};
          }
        }
      }
    }
  }
  __syncthreads();
  // z: complex -> real at every lattice point; one task per (item, x, y) line
  for (int idx = tid; idx < ITEMS * P * P; idx += kInvThreads) {
    const int it = idx / (P * P), x = (idx / P) % P, y = idx % P;
    C2 v[H];
#pragma unroll
    for (int kz = 0; kz < H; ++kz) v[kz] = b1[it * L::s1i + x * L::s1x + y * L::s1y + kz];
#pragma unroll 1
    for (int z = 0; z < P; ++z) {
      T acc = T(0);
#pragma unroll
      for (int kz = 1; kz < H; ++kz) acc += cmulc(v[kz], Wm[kz * P + z]).x;
      zb[((it * P + x) * P + y) * P + z] = v[0].x + T(2) * acc;
    }
  }
  __syncthreads();
  // the check-surface points, scaled
  for (int idx = tid; idx < ITEMS * NS; idx += kInvThreads) {
    const int it = idx / NS, s = idx % NS;
    const int ch = (int)(g0 % 8) + it;
    int32_t box = cb[0];
#pragma unroll
    for (int j = 1; j < 8; ++j)
      if (ch == j) box = cb[j];
    if (box < 0) continue;
    const int x = sl[3 * s], y = sl[3 * s + 1], z = sl[3 * s + 2];
    out[((int64_t)box * nvec + v0) * NS + s] = scale * (double)zb[((it * P + x) * P + y) * P + z];
  }
}

// ---- Hadamard products on MFMA ---------------------------------------------

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
__device__ __forceinline__ void hadamard_gather_body(const HadGatherArgs& a, int64_t b) {
  using C2 = typename C2T<T>::type;
  using V4 = typename V4T<T>::type;
  using T4 = typename Vec4T<T>::type;
  const C2* __restrict__ Khat = static_cast<const C2*>(a.Khat);
  const T* __restrict__ Qhat = static_cast<const T*>(a.Qhat);
  const int32_t* __restrict__ halo = a.halo;
  const int64_t n_c = a.n_c;
  const int nvec = a.nvec;
  const int64_t n_rows = a.n_rows;
  const int n_chunks = a.n_chunks, tiles_per_wave = a.tiles_per_wave;
  const int64_t total_blocks = a.total_blocks;
  T* __restrict__ Phat = static_cast<T*>(a.Phat);
  constexpr int DC = HadChunk<T>::value;
  __shared__ T4 Bl[26][64];
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

constexpr int kHadSrcMax = kHadSrcSlots;  // source slots of one 4 x 4 x 4 block: its 6 x 6 x 6 shell
static_assert(kHadRowBytes % 16 == 0 && kHadRowBytes >= 64, "LDS row of 16 floats");
constexpr int kHadStage = (kHadSrcMax * 4 + kHadThreads - 1) / kHadThreads;
constexpr int kHadDiscard = kHadSrcMax * kHadRowBytes;  // LDS bytes past the slots

// Byte offset, relative to a cluster's biased base, of its neighbour in
// direction d (the 26 offsets of {-1, 0, 1}^3 \ {0} in lexicographic order,
// x slowest): a compile-time constant once the direction loop is unrolled.
__host__ __device__ constexpr int had_dir_bytes(int d) {
  return (kHadSlotBias + ((d < 13 ? d : d + 1) / 9 - 1) +
          kHadShell * ((d < 13 ? d : d + 1) / 3 % 3 - 1) +
          kHadShell * kHadShell * ((d < 13 ? d : d + 1) % 3 - 1)) *
         kHadRowBytes;
}
static_assert(had_dir_bytes(0) == 0 && had_dir_bytes(25) == 2 * kHadSlotBias * kHadRowBytes,
              "direction offsets span the shell");

// Block form (FP32).  Workgroup = one frequency x a run of (block, charge
// vector) items.  Each lane holds the frequency's B operand for all 26
// directions in registers (the 416 x 16 real form of the 26 x 8 x 8 complex
// kernel coefficients, in its operand order).  Per item the spectra of the
// block's source clusters (at most 216 rows of 16 reals) are staged in LDS
// at the slots of their shell positions - the next item's rows are loaded
// into registers while the current one computes, and the list entries that
// address them one item earlier still, so no load waits on another inside
// an item - and each wave takes one 16-cluster tile of the block's (at most
// 64) target clusters.  A lane's A operand for direction d is read at its
// cluster's base offset plus a constant, so the eight clusters of an
// aligned 2 x 2 x 2 cube (eight consecutive lanes) read distinct LDS banks,
// and the read for the next direction is issued before the current
// direction's MFMAs.  Every source spectrum crosses the cache hierarchy
// once per block, and the VALU work per MFMA stays small (on gfx950 the
// VALU does not co-issue with the MFMA of the same wave).
__device__ __forceinline__ void hadamard_block_body(const HadBlockArgs& a, int64_t b, int64_t nblk) {
  const float2* __restrict__ Khat = static_cast<const float2*>(a.Khat);
  const float* __restrict__ Qhat = static_cast<const float*>(a.Qhat);
  const int32_t* __restrict__ blk_tgt = a.blk_tgt;
  const int32_t* __restrict__ blk_src = a.blk_src;
  const int32_t* __restrict__ blk_list = a.blk_list;
  const int32_t* __restrict__ tbase = a.tbase;
  const int n_items = a.n_items, nvec = a.nvec;
  const int64_t n_rows = a.n_rows, total_items = a.total_items, unit_len = a.unit_len;
  const int64_t n_units = a.n_units, n_wgs = a.n_wgs;
  float* __restrict__ Phat = static_cast<float*>(a.Phat);
  constexpr int kRow = kHadRowBytes / 16;  // LDS row stride in float4: 16 reals + padding
  constexpr int kBuf = kHadSrcMax * kRow + 4;  // + a 64-byte discard area
  __shared__ float4 As[2 * kBuf];
  const int64_t per_xcd = nblk / 8;  // grid: a multiple of 8
  const int64_t logical = (b % 8) * per_xcd + b / 8;  // consecutive work per XCD
  if (logical >= n_wgs) return;
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int rl = lane % 16, g = lane / 16;
  const int tr0 = wave * 16;  // this wave's tile of the block's targets
  const uint32_t row_bytes = 64u * (uint32_t)nvec;  // one cluster's rows
  // staging registers: four 16-byte pieces per thread (216 rows x 4 pieces
  // over 256 threads), named rather than an array so they stay in VGPRs;
  // piece k is row (tid + 256 k) / 4, quarter tid % 4.  A piece past the
  // block's list takes the list's first entry, the empty cluster at slot
  // 255, whose LDS offset is clamped into the discard area.
  static_assert(kHadStage == 4, "staging pieces per thread");
  const uint32_t part_bytes = 16u * (uint32_t)(tid & 3);
  float4 stg0, stg1, stg2, stg3;
  // list entries of two consecutive items (sets a and b alternate between
  // steps, so no loaded register is copied) and the lane's target base of
  // two consecutive items
  uint32_t ea0 = 0, ea1 = 0, ea2 = 0, ea3 = 0;
  uint32_t eb0 = 0, eb1 = 0, eb2 = 0, eb3 = 0;
  uint32_t tba = 0, tbb = 0;
  float res0 = 0.f, res1 = 0.f, res2 = 0.f, res3 = 0.f;  // products of the last item computed
  auto entry = [&](int s0, int ns, int k) __attribute__((always_inline)) {
    const int r = (tid + kHadThreads * k) >> 2;
    return (uint32_t)blk_list[r < ns ? s0 + r : 0];
  };
  auto lds_slot = [&](uint32_t e) __attribute__((always_inline)) {
    return min((e & 255u) * (uint32_t)kHadRowBytes, (uint32_t)kHadDiscard) + part_bytes;
  };
  int buf = 0;
  // Units of unit_len consecutive frequency-major (frequency, block, vector)
  // items: this workgroup takes units logical, logical + n_wgs, ..., each in
  // segments of one frequency.  Persistent form: one unit per workgroup, a
  // device-full of workgroups; unit form: 8-item units, one per workgroup.
  for (int64_t unit = logical; unit < n_units; unit += n_wgs) {
  const int64_t q0 = unit * unit_len, q1 = min(q0 + unit_len, total_items);
  for (int64_t seg = q0; seg < q1;) {
  const int64_t f = seg / n_items;
  const int item0 = (int)(seg - f * n_items);
  const int item1 = (int)(min(q1, (f + 1) * n_items) - f * n_items);
  seg = f * n_items + item1;
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
  // and products, addressed with 32-bit byte offsets from these bases
  const char* qf = reinterpret_cast<const char*>(Qhat + f * (n_rows + nvec) * 16);
  char* pf = reinterpret_cast<char*>(Phat + f * n_rows * 16);
  // Software pipeline over the segment's items, one step per item plus two:
  // step `it` (1) writes the rows of item it - 1 to LDS and stores the
  // products of item it - 2, (2) issues every global load of item it (rows,
  // target base) and the list entries of item it + 1, and (3) computes item
  // it - 1.  A step's loads are consumed only after the next step's single
  // wait at its top, which the MFMA work of (3) covers, so no wait inside a
  // step (gfx9 counts loads and stores in one in-order counter) falls on a
  // load or store issued in the same step.  Block bounds are read one step
  // ahead as well.
  int lblk = item0 / nvec, lv = item0 - lblk * nvec;  // item it
  int cv = 0, ct0 = 0, cnt = 0;  // item it - 1: vector, first cluster, count
  int sv = 0, st0 = 0, snt = 0;  // item it - 2
  // bounds kept as loaded (differences taken at their use, a step later,
  // so that no scalar load is waited for in the step that issues it)
  int nt0 = blk_tgt[lblk], nt1 = blk_tgt[lblk + 1];  // clusters of item it's block
  int es0, es1;  // list range of item it + 1
  {
    const int s0 = blk_src[lblk], ns = blk_src[lblk + 1] - s0;
    ea0 = entry(s0, ns, 0);
    ea1 = entry(s0, ns, 1);
    ea2 = entry(s0, ns, 2);
    ea3 = entry(s0, ns, 3);
    const int b1 = (lv + 1 == nvec) ? lblk + 1 : lblk;
    const int bb = min(b1, (int)(((int64_t)n_items - 1) / nvec));
    es0 = blk_src[bb];
    es1 = blk_src[bb + 1];
  }
  auto step = [&](int it, uint32_t& w0, uint32_t& w1, uint32_t& w2, uint32_t& w3, uint32_t u0,
                  uint32_t u1, uint32_t u2, uint32_t u3, uint32_t tbc, uint32_t& tbn)
                  __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0);  // the previous step's loads and stores
    const bool write = it > item0 && it <= item1;  // rows of item it - 1 staged
    if (write) {
      char* ab = reinterpret_cast<char*>(As + buf * kBuf);
      *reinterpret_cast<float4*>(ab + lds_slot(w0)) = stg0;
      *reinterpret_cast<float4*>(ab + lds_slot(w1)) = stg1;
      *reinterpret_cast<float4*>(ab + lds_slot(w2)) = stg2;
      *reinterpret_cast<float4*>(ab + lds_slot(w3)) = stg3;
    }
    if (it >= item0 + 2 && tr0 < snt) {
      // row tr0 + 4 g + i of the tile: cluster st0 + that row, vector sv
      const uint32_t o0 = ((uint32_t)(st0 + tr0 + 4 * g) * nvec + sv) * 64u + 4u * rl;
      const int rr = tr0 + 4 * g;
      if (rr + 0 < snt) *reinterpret_cast<float*>(pf + o0) = res0;
      if (rr + 1 < snt) *reinterpret_cast<float*>(pf + o0 + row_bytes) = res1;
      if (rr + 2 < snt) *reinterpret_cast<float*>(pf + o0 + 2 * row_bytes) = res2;
      if (rr + 3 < snt) *reinterpret_cast<float*>(pf + o0 + 3 * row_bytes) = res3;
    }
    if (write) __syncthreads();  // this buffer complete; the other one free for the next item
    sv = cv;
    st0 = ct0;
    snt = cnt;
    if (it < item1) {
      const uint32_t vb = (uint32_t)lv * 64u + part_bytes;
      stg0 = *reinterpret_cast<const float4*>(qf + ((u0 >> 8) * row_bytes + vb));
      stg1 = *reinterpret_cast<const float4*>(qf + ((u1 >> 8) * row_bytes + vb));
      stg2 = *reinterpret_cast<const float4*>(qf + ((u2 >> 8) * row_bytes + vb));
      stg3 = *reinterpret_cast<const float4*>(qf + ((u3 >> 8) * row_bytes + vb));
      tbn = (uint32_t)tbase[nt0 + min(tr0 + rl, nt1 - nt0 - 1)];
      if (it + 1 < item1) {
        w0 = entry(es0, es1 - es0, 0);
        w1 = entry(es0, es1 - es0, 1);
        w2 = entry(es0, es1 - es0, 2);
        w3 = entry(es0, es1 - es0, 3);
      }
    }
    // item it becomes item it - 1 of the next step; advance to item it + 1
    const int pnt0 = nt0, pnt1 = nt1, plv = lv;
    if (++lv == nvec) {
      lv = 0;
      ++lblk;
    }
    if (it + 1 < item1) {
      nt0 = blk_tgt[lblk];
      nt1 = blk_tgt[lblk + 1];
    }
    if (it + 2 < item1) {
      const int b2 = (lv + 1 == nvec) ? lblk + 1 : lblk;  // block of item it + 2
      es0 = blk_src[b2];
      es1 = blk_src[b2 + 1];
    }
    if (write && tr0 < cnt) {
      // two accumulators so consecutive MFMAs are independent: K slices x
      // and y (real and imaginary parts of source children 0, 2, 4, 6) into
      // one, z and w (children 1, 3, 5, 7) into the other, so each holds
      // whole complex products and their sum cancels no more than the
      // products themselves; the next direction's A operand is in flight
      // while the current one's MFMAs issue
      const char* ab = reinterpret_cast<const char*>(As + buf * kBuf) + tbc + 16 * g;
      v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
      float4 an = *reinterpret_cast<const float4*>(ab + had_dir_bytes(0));
#pragma unroll
      for (int d = 0; d < 26; ++d) {
        const float4 a = an;
        if (d + 1 < 26) an = *reinterpret_cast<const float4*>(ab + had_dir_bytes(d + 1));
        // keep the read above the MFMAs (the scheduler would sink it)
        __builtin_amdgcn_sched_barrier(0);
        acc0 = mfma16(a.x, B[d].x, acc0);
        acc1 = mfma16(a.z, B[d].z, acc1);
        acc0 = mfma16(a.y, B[d].y, acc0);
        acc1 = mfma16(a.w, B[d].w, acc1);
      }
      res0 = acc0[0] + acc1[0];
      res1 = acc0[1] + acc1[1];
      res2 = acc0[2] + acc1[2];
      res3 = acc0[3] + acc1[3];
    }
    if (write) buf ^= 1;
    cv = plv;
    ct0 = pnt0;
    cnt = it < item1 ? pnt1 - pnt0 : 0;
  };
  for (int it = item0; it <= item1 + 1; it += 2) {
    step(it, eb0, eb1, eb2, eb3, ea0, ea1, ea2, ea3, tbb, tba);
    if (it + 1 <= item1 + 1) step(it + 1, ea0, ea1, ea2, ea3, eb0, eb1, eb2, eb3, tba, tbb);
  }
  }
  }
}

// Split form (FP32 inputs and outputs, products on BF16 MFMA).  Every FP32
// operand value x is split into three BF16 parts, x0 = bf16(x),
// x1 = bf16(x - x0), x2 = bf16(x - x0 - x1) (each residual exact in FP32),
// which together carry its 24 significant bits; a product a b is taken as
// the six part products of order at most two, a0 b0 + a0 b1 + a1 b0 + a0 b2
// + a1 b1 + a2 b0 (the dropped ones lie below 2^-24 |a b|).  Each BF16
// product is exact in FP32 and v_mfma_f32_16x16x32_bf16 sums them in FP32,
// so the result carries an FP32 GEMM's rounding error, at six BF16 MFMAs
// (16 cycles each) per two directions instead of eight FP32 MFMAs (32 cycles
// each).  Work split and staging pipeline are those of the block form.  An
// LDS row (kSplitRowBytes = 96) holds the three parts of a cluster's 16
// reals: reals 0-7 as parts 0, 1, 2 (16 bytes each), then reals 8-15 the
// same way; the cluster at shell position (x, y, z) of staging buffer b sits
// in row x + 6 b + 12 y + 72 z (the two buffers interleaved along x).  With
// this layout the 128-bit operand reads of a tile's sixteen clusters meet no
// LDS bank conflict in any direction (measured with rocprofv3's
// SQ_LDS_BANK_CONFLICT on the exact access pattern; 32-byte plane rows of
// 112 bytes cost four conflict cycles per read).  K step j of a product
// covers two directions (lane groups 0, 1 and 2, 3), each lane group eight
// consecutive reals of its direction's source row; the B parts are split
// once per kernel-spectrum table.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
constexpr int kSplitRowBytes = 96;  // 2 halves x 3 parts x 16 bytes
constexpr int kSplitHalf = 48;      // bytes from reals 0-7 to reals 8-15
constexpr int kSplitPart = 16;      // bytes from one part to the next within a half
constexpr int kSplitY = 12, kSplitZ = 72;  // row strides along y and z (x: 1, buffers: 6)
constexpr int kSplitBias = 1 + kSplitY + kSplitZ;  // rows of shell position (1, 1, 1)
constexpr int kSplitDiscard = kHadShell * kSplitZ * kSplitRowBytes;  // past both buffers' rows
constexpr int kSplitLds = kSplitDiscard + kSplitRowBytes;
static_assert(kSplitRowBytes == 2 * kSplitHalf && kSplitHalf == 3 * kSplitPart, "row of 2 x 3 parts");
static_assert(kSplitY == 2 * kHadShell && kSplitZ == kHadShell * kSplitY,
              "the two buffers fill the gaps along x");
// LDS row of shell slot s = x + 6 y + 36 z (s < 256) in buffer b:
// x + 12 y + 72 z + 6 b = s + 6 (s / 6 + b), s / 6 as (171 s) >> 10
__device__ inline uint32_t split_row(uint32_t s, uint32_t b) { return s + 6u * (((s * 171u) >> 10) + b); }
// byte offset of direction d (numbered as had_dir_bytes) from a biased base
__host__ __device__ constexpr int split_dir_bytes(int d) {
  return (kSplitBias + ((d < 13 ? d : d + 1) / 9 - 1) + kSplitY * ((d < 13 ? d : d + 1) / 3 % 3 - 1) +
          kSplitZ * ((d < 13 ? d : d + 1) % 3 - 1)) *
         kSplitRowBytes;
}
// Direction of half h of K step j: the nine pairs (x, y, -1), (x, y, +1),
// then (x, -1, 0), (x, +1, 0) for x = -1, 0, 1, then (-1, 0, 0), (+1, 0, 0),
// so that the second half's LDS offset exceeds the first's by one of three
// constants (144, 24 or 2 rows).  Directions are numbered as had_dir_bytes.
__host__ __device__ constexpr int split_pair_dir(int j, int h) {
  const int x = j < 9 ? j / 3 - 1 : j < 12 ? j - 10 : (h ? 1 : -1);
  const int y = j < 9 ? j % 3 - 1 : j < 12 ? (h ? 1 : -1) : 0;
  const int z = j < 9 ? (h ? 1 : -1) : 0;
  const int ix = (x + 1) * 9 + (y + 1) * 3 + (z + 1);
  return ix < 13 ? ix : ix - 1;
}
__host__ __device__ constexpr int split_pair_step(int j) {  // second-half offset over the first, bytes
  return split_dir_bytes(split_pair_dir(j, 1)) - split_dir_bytes(split_pair_dir(j, 0));
}
static_assert(split_pair_step(0) == 2 * kSplitZ * kSplitRowBytes &&
                  split_pair_step(9) == 2 * kSplitY * kSplitRowBytes && split_pair_step(12) == 2 * kSplitRowBytes,
              "pair offsets");

__device__ inline void split3(float x, __bf16& h0, __bf16& h1, __bf16& h2) {
  h0 = (__bf16)x;
  const float r1 = x - (float)h0;
  h1 = (__bf16)r1;
  h2 = (__bf16)(r1 - (float)h1);
}
// the three parts of two values, two BF16 per dword (value a in the low half)
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ inline void split3x2(float a, float b, uint32_t& p0, uint32_t& p1, uint32_t& p2) {
  p0 = __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{a, b}, v2bf));
  const float ra = a - __uint_as_float(p0 << 16), rb = b - __uint_as_float(p0 & 0xffff0000u);
  p1 = __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{ra, rb}, v2bf));
  const float sa = ra - __uint_as_float(p1 << 16), sb = rb - __uint_as_float(p1 & 0xffff0000u);
  p2 = __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{sa, sb}, v2bf));
}
__device__ inline v4f mfbf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// B operand parts of the split form, once per kernel-spectrum table:
// Bs[((f * 3 + part) * 13 + j) * 64 + lane] (8 BF16 each) holds part `part`
// of the coefficients that lane (n, g) of K step j takes: source reals
// 8 (g % 2) .. + 7 (children 4 (g % 2) .. + 3, real and imaginary parts) of
// direction split_pair_dir(j, g / 2) into output n (target child n / 2, real
// part for even n, imaginary for odd n).  One thread per (f, j, lane).
__global__ __launch_bounds__(256) void hadamard_split_prep_kernel(const float2* __restrict__ Khat, int F,
                                                                 v8bf* __restrict__ Bs) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)F * 13 * 64) return;
  const int lane = (int)(t % 64), j = (int)(t / 64 % 13);
  const int64_t f = t / (64 * 13);
  const int rl = lane % 16, g = lane / 16;
  const int d = split_pair_dir(j, g >> 1);
  v8bf p[3];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float2 k = Khat[((f * 26 + d) * 8 + rl / 2) * 8 + 4 * (g & 1) + c];
    const float cre = (rl & 1) ? k.y : k.x;   // coefficient of the real part
    const float cim = (rl & 1) ? k.x : -k.y;  // coefficient of the imaginary part
    __bf16 h0, h1, h2;
    split3(cre, h0, h1, h2);
    p[0][2 * c] = h0;
    p[1][2 * c] = h1;
    p[2][2 * c] = h2;
    split3(cim, h0, h1, h2);
    p[0][2 * c + 1] = h0;
    p[1][2 * c + 1] = h1;
    p[2][2 * c + 1] = h2;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) Bs[((f * 3 + q) * 13 + j) * 64 + lane] = p[q];
}

__device__ __forceinline__ void hadamard_split_body(const HadBlockArgs& a, int64_t b, int64_t nblk) {
  const v8bf* __restrict__ Ksp = static_cast<const v8bf*>(a.Khat);  // parts from the prep kernel
  const float* __restrict__ Qhat = static_cast<const float*>(a.Qhat);
  const int32_t* __restrict__ blk_tgt = a.blk_tgt;
  const int32_t* __restrict__ blk_src = a.blk_src;
  const int32_t* __restrict__ blk_list = a.blk_list;
  const int32_t* __restrict__ tbase = a.tbase;
  const int n_items = a.n_items, nvec = a.nvec;
  const int64_t n_rows = a.n_rows, total_items = a.total_items, unit_len = a.unit_len;
  const int64_t n_units = a.n_units, n_wgs = a.n_wgs;
  float* __restrict__ Phat = static_cast<float*>(a.Phat);
  __shared__ __attribute__((aligned(16))) char As[kSplitLds];  // both staging buffers
  const int64_t per_xcd = nblk / 8;  // grid: a multiple of 8
  const int64_t logical = (b % 8) * per_xcd + b / 8;  // consecutive work per XCD
  if (logical >= n_wgs) return;
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int rl = lane % 16, g = lane / 16;
  const int tr0 = wave * 16;  // this wave's tile of the block's targets
  const uint32_t row_bytes = 64u * (uint32_t)nvec;  // one cluster's rows in Qhat / Phat
  // staging: four 16-byte pieces (4 reals) per thread as in the block form;
  // piece k is row (tid + 256 k) / 4, reals 4 (tid % 4) .. + 3, written as
  // three 8-byte parts, kSplitPart apart, in half (tid % 4) / 2
  static_assert(kHadStage == 4, "staging pieces per thread");
  const uint32_t part_bytes = (uint32_t)(kSplitHalf * ((tid & 3) >> 1) + 8 * (tid & 1));
  float4 stg0, stg1, stg2, stg3;
  uint32_t ea0 = 0, ea1 = 0, ea2 = 0, ea3 = 0;
  uint32_t eb0 = 0, eb1 = 0, eb2 = 0, eb3 = 0;
  uint32_t tba = 0, tbb = 0;
  float res0 = 0.f, res1 = 0.f, res2 = 0.f, res3 = 0.f;  // products of the last item computed
  auto entry = [&](int s0, int ns, int k) __attribute__((always_inline)) {
    const int r = (tid + kHadThreads * k) >> 2;
    return (uint32_t)blk_list[r < ns ? s0 + r : 0];
  };
  // slots past the shell (the empty cluster's 255) map past both buffers'
  // rows, into the discard row
  auto lds_slot = [&](uint32_t e, uint32_t b) __attribute__((always_inline)) {
    return min(split_row(e & 255u, b), (uint32_t)(kHadShell * kSplitZ)) * (uint32_t)kSplitRowBytes + part_bytes;
  };
  auto put = [&](char* ab, uint32_t off, float4 v) __attribute__((always_inline)) {
    uint2 p0, p1, p2;
    split3x2(v.x, v.y, p0.x, p1.x, p2.x);
    split3x2(v.z, v.w, p0.y, p1.y, p2.y);
    *reinterpret_cast<uint2*>(ab + off) = p0;
    *reinterpret_cast<uint2*>(ab + off + kSplitPart) = p1;
    *reinterpret_cast<uint2*>(ab + off + 2 * kSplitPart) = p2;
  };
  int buf = 0;
  for (int64_t unit = logical; unit < n_units; unit += n_wgs) {
  const int64_t q0 = unit * unit_len, q1 = min(q0 + unit_len, total_items);
  for (int64_t seg = q0; seg < q1;) {
  const int64_t f = seg / n_items;
  const int item0 = (int)(seg - f * n_items);
  const int item1 = (int)(min(q1, (f + 1) * n_items) - f * n_items);
  seg = f * n_items + item1;
  // B parts of this frequency (laid out by hadamard_split_prep_kernel), in
  // registers: the LDS carries only the A parts, whose reads bound the rate
  v8bf B0[13], B1[13], B2[13];
  {
    const v8bf* kb = Ksp + f * 3 * 13 * 64;
#pragma unroll
    for (int j = 0; j < 13; ++j) {
      B0[j] = kb[j * 64 + lane];
      B1[j] = kb[(13 + j) * 64 + lane];
      B2[j] = kb[(26 + j) * 64 + lane];
    }
  }
  const char* qf = reinterpret_cast<const char*>(Qhat + f * (n_rows + nvec) * 16);
  char* pf = reinterpret_cast<char*>(Phat + f * n_rows * 16);
  // software pipeline of the block form: step `it` stages item it - 1,
  // stores the products of item it - 2, loads item it and computes item it - 1
  int lblk = item0 / nvec, lv = item0 - lblk * nvec;  // item it
  int cv = 0, ct0 = 0, cnt = 0;  // item it - 1: vector, first cluster, count
  int sv = 0, st0 = 0, snt = 0;  // item it - 2
  int nt0 = blk_tgt[lblk], nt1 = blk_tgt[lblk + 1];  // clusters of item it's block
  int es0, es1;  // list range of item it + 1
  {
    const int s0 = blk_src[lblk], ns = blk_src[lblk + 1] - s0;
    ea0 = entry(s0, ns, 0);
    ea1 = entry(s0, ns, 1);
    ea2 = entry(s0, ns, 2);
    ea3 = entry(s0, ns, 3);
    const int b1 = (lv + 1 == nvec) ? lblk + 1 : lblk;
    const int bb = min(b1, (int)(((int64_t)n_items - 1) / nvec));
    es0 = blk_src[bb];
    es1 = blk_src[bb + 1];
  }
  auto step = [&](int it, uint32_t& w0, uint32_t& w1, uint32_t& w2, uint32_t& w3, uint32_t u0,
                  uint32_t u1, uint32_t u2, uint32_t u3, uint32_t tbc, uint32_t& tbn)
                  __attribute__((always_inline)) {
    __builtin_amdgcn_s_waitcnt(0);  // the previous step's loads and stores
    const bool write = it > item0 && it <= item1;  // rows of item it - 1 staged
    if (write) {
      put(As, lds_slot(w0, buf), stg0);
      put(As, lds_slot(w1, buf), stg1);
      put(As, lds_slot(w2, buf), stg2);
      put(As, lds_slot(w3, buf), stg3);
    }
    if (it >= item0 + 2 && tr0 < snt) {
      const uint32_t o0 = ((uint32_t)(st0 + tr0 + 4 * g) * nvec + sv) * 64u + 4u * rl;
      const int rr = tr0 + 4 * g;
      if (rr + 0 < snt) *reinterpret_cast<float*>(pf + o0) = res0;
      if (rr + 1 < snt) *reinterpret_cast<float*>(pf + o0 + row_bytes) = res1;
      if (rr + 2 < snt) *reinterpret_cast<float*>(pf + o0 + 2 * row_bytes) = res2;
      if (rr + 3 < snt) *reinterpret_cast<float*>(pf + o0 + 3 * row_bytes) = res3;
    }
    if (write) __syncthreads();  // this buffer complete; the other one free for the next item
    sv = cv;
    st0 = ct0;
    snt = cnt;
    if (it < item1) {
      const uint32_t vb = (uint32_t)lv * 64u + 16u * (uint32_t)(tid & 3);
      stg0 = *reinterpret_cast<const float4*>(qf + ((u0 >> 8) * row_bytes + vb));
      stg1 = *reinterpret_cast<const float4*>(qf + ((u1 >> 8) * row_bytes + vb));
      stg2 = *reinterpret_cast<const float4*>(qf + ((u2 >> 8) * row_bytes + vb));
      stg3 = *reinterpret_cast<const float4*>(qf + ((u3 >> 8) * row_bytes + vb));
      tbn = (uint32_t)tbase[nt0 + min(tr0 + rl, nt1 - nt0 - 1)];
    }
    if (it + 1 < item1) {  // entries of item it + 1 (those of item it - 1 are staged)
      w0 = entry(es0, es1 - es0, 0);
      w1 = entry(es0, es1 - es0, 1);
      w2 = entry(es0, es1 - es0, 2);
      w3 = entry(es0, es1 - es0, 3);
    }
    const int pnt0 = nt0, pnt1 = nt1, plv = lv;
    if (++lv == nvec) {
      lv = 0;
      ++lblk;
    }
    if (it + 1 < item1) {
      nt0 = blk_tgt[lblk];
      nt1 = blk_tgt[lblk + 1];
    }
    if (it + 2 < item1) {
      const int b2 = (lv + 1 == nvec) ? lblk + 1 : lblk;  // block of item it + 2
      es0 = blk_src[b2];
      es1 = blk_src[b2 + 1];
    }
    if (write && tr0 < cnt) {
      // the lane's source row of K step j's first direction (lane groups 0,
      // 1) or second (2, 3): the target's biased base (its slot from the
      // block-form offset) plus the direction's constant offset; the next
      // step's parts are read before the current step's MFMAs.  Two
      // accumulators take alternate products.
      const uint32_t ts = tbc / (uint32_t)kHadRowBytes + (uint32_t)kHadSlotBias;  // target's slot
      const char* ab = As + (split_row(ts, buf) - kSplitBias) * kSplitRowBytes + kSplitHalf * (g & 1);
      const bool hi = g >= 2;
      const int hs72 = hi ? 2 * kSplitZ * kSplitRowBytes : 0, hs12 = hi ? 2 * kSplitY * kSplitRowBytes : 0,
                hs2 = hi ? 2 * kSplitRowBytes : 0;
      auto ldA = [&](int j, v8bf& x0, v8bf& x1, v8bf& x2) __attribute__((always_inline)) {
        const char* pa = ab + (j < 9 ? hs72 : j < 12 ? hs12 : hs2) + split_dir_bytes(split_pair_dir(j, 0));
        x0 = *reinterpret_cast<const v8bf*>(pa);
        x1 = *reinterpret_cast<const v8bf*>(pa + kSplitPart);
        x2 = *reinterpret_cast<const v8bf*>(pa + 2 * kSplitPart);
      };
      v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
      v8bf n0, n1, n2;
      ldA(0, n0, n1, n2);
#pragma unroll
      for (int j = 0; j < 13; ++j) {
        const v8bf a0 = n0, a1 = n1, a2 = n2;
        if (j + 1 < 13) ldA(j + 1, n0, n1, n2);
        __builtin_amdgcn_sched_barrier(0);
        acc0 = mfbf16(a0, B0[j], acc0);
        acc1 = mfbf16(a0, B1[j], acc1);
        acc0 = mfbf16(a1, B0[j], acc0);
        acc1 = mfbf16(a0, B2[j], acc1);
        acc0 = mfbf16(a1, B1[j], acc0);
        acc1 = mfbf16(a2, B0[j], acc1);
      }
      res0 = acc0[0] + acc1[0];
      res1 = acc0[1] + acc1[1];
      res2 = acc0[2] + acc1[2];
      res3 = acc0[3] + acc1[3];
    }
    if (write) buf ^= 1;
    cv = plv;
    ct0 = pnt0;
    cnt = it < item1 ? pnt1 - pnt0 : 0;
  };
  for (int it = item0; it <= item1 + 1; it += 2) {
    step(it, eb0, eb1, eb2, eb3, ea0, ea1, ea2, ea3, tbb, tba);
    if (it + 1 <= item1 + 1) step(it + 1, ea0, ea1, ea2, ea3, eb0, eb1, eb2, eb3, tba, tbb);
  }
  }
  }
}

// ---- kernels: the bodies above as plain and as grouped launches ------------
// (scalar parameters: with the arguments as one by-value struct the compiler
// kept 120 instead of 66 VGPRs at p = 6, FP32)
template <typename T, int P>
__global__ __launch_bounds__((FftCfg<T, P>::threads)) void fft_forward_kernel(
    const double* __restrict__ M, const int32_t* __restrict__ child, int64_t n_rows, int nvec,
    const int16_t* __restrict__ lat2surf, const void* __restrict__ wm, void* __restrict__ Qhat) {
  const FwdArgs a{M, child, n_rows, nvec, lat2surf, wm, Qhat};
  fft_forward_body<T, P>(a, blockIdx.x, gridDim.x);
}
template <typename T, int P>
__global__ __launch_bounds__((FftCfg<T, P>::threads)) void fft_forward_group_kernel(
    const FwdArgs* __restrict__ jobs, const int64_t* __restrict__ pre, int nj) {
  int64_t b;
  const int j = group_job(pre, nj, b);
  const FwdArgs a = jobs[j];
  fft_forward_body<T, P>(a, b, pre[j + 1] - pre[j]);
}
// eight waves per SIMD (four workgroups per CU) where the LDS allows them
template <typename T, int P> struct InvWaves {
  using L = InvLds<P, (int)sizeof(T) / 2>;
  static constexpr int lds = L::items * (L::s2i + L::s1i) * 2 * (int)sizeof(T);
  static constexpr int value = lds * 4 <= 160 * 1024 - 4 * 1024 ? 8 : 6;
};
template <typename T, int P>
__global__ __launch_bounds__(kInvThreads) __attribute__((amdgpu_waves_per_eu(InvWaves<T, P>::value))) void fft_inverse_kernel(InvArgs a) {
  fft_inverse_body<T, P>(a, blockIdx.x);
}
template <typename T, int P>
__global__ __launch_bounds__(kInvThreads) __attribute__((amdgpu_waves_per_eu(InvWaves<T, P>::value))) void fft_inverse_group_kernel(const InvArgs* __restrict__ jobs,
                                                                        const int64_t* __restrict__ pre,
                                                                        int nj) {
  int64_t b;
  const InvArgs a = jobs[group_job(pre, nj, b)];
  fft_inverse_body<T, P>(a, b);
}
template <typename T>
__global__ __launch_bounds__(kHadThreads) void hadamard_gather_kernel(HadGatherArgs a) {
  hadamard_gather_body<T>(a, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(kHadThreads) void hadamard_gather_group_kernel(
    const HadGatherArgs* __restrict__ jobs, const int64_t* __restrict__ pre, int nj) {
  int64_t b;
  const HadGatherArgs a = jobs[group_job(pre, nj, b)];
  hadamard_gather_body<T>(a, b);
}
__global__ __launch_bounds__(kHadThreads, 2) void hadamard_split_kernel(HadBlockArgs a) {
  hadamard_split_body(a, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kHadThreads, 2) void hadamard_split_group_kernel(
    const HadBlockArgs* __restrict__ jobs, const int64_t* __restrict__ pre, int nj) {
  int64_t b;
  const int j = group_job(pre, nj, b);
  const HadBlockArgs a = jobs[j];
  hadamard_split_body(a, b, pre[j + 1] - pre[j]);
}
__global__ __launch_bounds__(kHadThreads, 3) void hadamard_block_kernel(HadBlockArgs a) {
  hadamard_block_body(a, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kHadThreads, 3) void hadamard_block_group_kernel(
    const HadBlockArgs* __restrict__ jobs, const int64_t* __restrict__ pre, int nj) {
  int64_t b;
  const int j = group_job(pre, nj, b);
  const HadBlockArgs a = jobs[j];
  hadamard_block_body(a, b, pre[j + 1] - pre[j]);
}

// Workgroups resident on the whole device for a kernel (occupancy x CUs).
template <typename K>
int64_t resident_wgs(K kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      cus < 1 || per_cu < 1)
    return 0;
  return (int64_t)cus * per_cu;
}

// Forward workgroups: persistent (enough to fill the device once, each an
// equal number of item groups) or, for grouped launches, one item group per
// workgroup; a multiple of 8 for the XCD numbering.  -1 on failure.
template <typename T, int P>
int64_t fwd_blocks(int64_t n_rows, bool persistent) {
  constexpr int IT = FftCfg<T, P>::items, TH = FftCfg<T, P>::threads;
  const int64_t n_groups = (n_rows * 8 + IT - 1) / IT;
  if (!persistent) return (n_groups + 7) / 8 * 8;
  static const int64_t resident = resident_wgs(fft_forward_kernel<T, P>, TH);
  if (resident < 1) return -1;
  const int64_t rounds = (n_groups + resident - 1) / resident;
  return ((n_groups + rounds - 1) / rounds + 7) / 8 * 8;
}

template <typename T, int P>
void fwd_go(const FwdArgs* one, const FwdArgs* jobs, const int64_t* pre, int nj, int64_t blocks,
            hipStream_t s) {
  constexpr int TH = FftCfg<T, P>::threads;
  if (!jobs)
    fft_forward_kernel<T, P><<<(unsigned)blocks, TH, 0, s>>>(one->M, one->child, one->n_rows, one->nvec,
                                                             one->lat2surf, one->wm, one->Qhat);
  else
    fft_forward_group_kernel<T, P><<<(unsigned)blocks, TH, 0, s>>>(jobs, pre, nj);
}

template <typename T, int P>
int64_t inv_blocks(int64_t n_rows) {
  constexpr int IT = InvLds<P, (int)sizeof(T) / 2>::items;
  return 8 * (((n_rows * 8 + IT - 1) / IT + 7) / 8);
}

template <typename T, int P>
void inv_go(const InvArgs* one, const InvArgs* jobs, const int64_t* pre, int nj, int64_t blocks,
            hipStream_t s) {
  if (!jobs)
    fft_inverse_kernel<T, P><<<(unsigned)blocks, kInvThreads, 0, s>>>(*one);
  else
    fft_inverse_group_kernel<T, P><<<(unsigned)blocks, kInvThreads, 0, s>>>(jobs, pre, nj);
}

// p = 2..8 as a template argument
#define KIFMM_SWITCH_P(p, CALL)                                                                  \
  switch (p) {                                                                                   \
    case 2: { constexpr int PP = 2; CALL; } break;                                               \
    case 3: { constexpr int PP = 3; CALL; } break;                                               \
    case 4: { constexpr int PP = 4; CALL; } break;                                               \
    case 5: { constexpr int PP = 5; CALL; } break;                                               \
    case 6: { constexpr int PP = 6; CALL; } break;                                               \
    case 7: { constexpr int PP = 7; CALL; } break;                                               \
    case 8: { constexpr int PP = 8; CALL; } break;                                               \
    default: return hipErrorInvalidValue;                                                        \
  }

hipError_t fwd_dispatch(int inst, const FwdArgs* one, const FwdArgs* jobs, const int64_t* pre, int nj,
                        int64_t blocks, hipStream_t s) {
  if (blocks == 0) return hipSuccess;
  if (blocks < 0 || blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const bool fp64 = inst >= 16;
  if (fp64) {
    KIFMM_SWITCH_P(inst % 16, (fwd_go<double, PP>(one, jobs, pre, nj, blocks, s)))
  } else {
    KIFMM_SWITCH_P(inst % 16, (fwd_go<float, PP>(one, jobs, pre, nj, blocks, s)))
  }
  return hipGetLastError();
}

hipError_t inv_dispatch(int inst, const InvArgs* one, const InvArgs* jobs, const int64_t* pre, int nj,
                        int64_t blocks, hipStream_t s) {
  if (blocks == 0) return hipSuccess;
  if (blocks < 0 || blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const bool fp64 = inst >= 16;
  if (fp64) {
    KIFMM_SWITCH_P(inst % 16, (inv_go<double, PP>(one, jobs, pre, nj, blocks, s)))
  } else {
    KIFMM_SWITCH_P(inst % 16, (inv_go<float, PP>(one, jobs, pre, nj, blocks, s)))
  }
  return hipGetLastError();
}

// inst: 0 = FP32 block form, 1 = FP64 gather form, 2 = split (BF16 parts) block form
hipError_t had_dispatch(int inst, const void* one, const void* jobs, const int64_t* pre, int nj,
                        int64_t blocks, hipStream_t s) {
  if (blocks == 0) return hipSuccess;
  if (blocks < 0 || blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (inst == 2) {
    if (!jobs)
      hadamard_split_kernel<<<(unsigned)blocks, kHadThreads, 0, s>>>(*static_cast<const HadBlockArgs*>(one));
    else
      hadamard_split_group_kernel<<<(unsigned)blocks, kHadThreads, 0, s>>>(
          static_cast<const HadBlockArgs*>(jobs), pre, nj);
  } else if (inst == 1) {
    if (!jobs)
      hadamard_gather_kernel<double><<<(unsigned)blocks, kHadThreads, 0, s>>>(
          *static_cast<const HadGatherArgs*>(one));
    else
      hadamard_gather_group_kernel<double><<<(unsigned)blocks, kHadThreads, 0, s>>>(
          static_cast<const HadGatherArgs*>(jobs), pre, nj);
  } else {
    if (!jobs)
      hadamard_block_kernel<<<(unsigned)blocks, kHadThreads, 0, s>>>(*static_cast<const HadBlockArgs*>(one));
    else
      hadamard_block_group_kernel<<<(unsigned)blocks, kHadThreads, 0, s>>>(
          static_cast<const HadBlockArgs*>(jobs), pre, nj);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t plan_fft_forward(int p, bool fp64, const double* M, const int32_t* child, int64_t n_clusters,
                            int nvec, const int16_t* lat2surf, const void* wm, void* Qhat,
                            bool persistent, FwdArgs& a, int& inst, int64_t& blocks) {
  const int64_t n_rows = n_clusters * nvec;
  a = FwdArgs{M, child, n_rows, nvec, lat2surf, wm, Qhat};
  inst = (fp64 ? 16 : 0) + p;
  blocks = 0;
  if (n_rows == 0) return hipSuccess;
  if (p < 2 || p > 8 || n_rows >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (fp64) {
    switch (p) {
#define KIFMM_FB(PP) case PP: blocks = fwd_blocks<double, PP>(n_rows, persistent); break;
      KIFMM_FB(2) KIFMM_FB(3) KIFMM_FB(4) KIFMM_FB(5) KIFMM_FB(6) KIFMM_FB(7) KIFMM_FB(8)
#undef KIFMM_FB
    }
  } else {
    switch (p) {
#define KIFMM_FB(PP) case PP: blocks = fwd_blocks<float, PP>(n_rows, persistent); break;
      KIFMM_FB(2) KIFMM_FB(3) KIFMM_FB(4) KIFMM_FB(5) KIFMM_FB(6) KIFMM_FB(7) KIFMM_FB(8)
#undef KIFMM_FB
    }
  }
  return blocks < 0 ? hipErrorInvalidValue : hipSuccess;
}

hipError_t launch_fft_forward(int p, bool fp64, const double* M, const int32_t* child,
                              int64_t n_clusters, int nvec, const int16_t* lat2surf,
                              const void* wm, void* Qhat, hipStream_t stream) {
  FwdArgs a;
  int inst;
  int64_t blocks;
  hipError_t e = plan_fft_forward(p, fp64, M, child, n_clusters, nvec, lat2surf, wm, Qhat, true, a, inst,
                                  blocks);
  if (e != hipSuccess) return e;
  return fwd_dispatch(inst, &a, nullptr, nullptr, 0, blocks, stream);
}

hipError_t launch_fft_forward_group(int inst, const FwdArgs* jobs, const int64_t* pre, int nj,
                                    int64_t blocks, hipStream_t stream) {
  return fwd_dispatch(inst, nullptr, jobs, pre, nj, blocks, stream);
}

hipError_t plan_fft_inverse(int p, bool fp64, const void* Phat, const int32_t* child, int64_t n_clusters,
                            int nvec, const int16_t* surf_lat, const void* wm, double scale, double* out,
                            InvArgs& a, int& inst, int64_t& blocks) {
  const int64_t n_rows = n_clusters * nvec;
  a = InvArgs{Phat, child, n_rows, nvec, surf_lat, wm, scale, out};
  inst = (fp64 ? 16 : 0) + p;
  blocks = 0;
  if (n_rows == 0) return hipSuccess;
  if (p < 2 || p > 8 || n_rows >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (fp64) {
    switch (p) {
#define KIFMM_IB(PP) case PP: blocks = inv_blocks<double, PP>(n_rows); break;
      KIFMM_IB(2) KIFMM_IB(3) KIFMM_IB(4) KIFMM_IB(5) KIFMM_IB(6) KIFMM_IB(7) KIFMM_IB(8)
#undef KIFMM_IB
    }
  } else {
    switch (p) {
#define KIFMM_IB(PP) case PP: blocks = inv_blocks<float, PP>(n_rows); break;
      KIFMM_IB(2) KIFMM_IB(3) KIFMM_IB(4) KIFMM_IB(5) KIFMM_IB(6) KIFMM_IB(7) KIFMM_IB(8)
#undef KIFMM_IB
    }
  }
  return hipSuccess;
}

hipError_t launch_fft_inverse(int p, bool fp64, const void* Phat, const int32_t* child,
                              int64_t n_clusters, int nvec, const int16_t* surf_lat,
                              const void* wm, double scale, double* out, hipStream_t stream) {
  InvArgs a;
  int inst;
  int64_t blocks;
  hipError_t e = plan_fft_inverse(p, fp64, Phat, child, n_clusters, nvec, surf_lat, wm, scale, out, a,
                                  inst, blocks);
  if (e != hipSuccess) return e;
  return inv_dispatch(inst, &a, nullptr, nullptr, 0, blocks, stream);
}

hipError_t launch_fft_inverse_group(int inst, const InvArgs* jobs, const int64_t* pre, int nj,
                                    int64_t blocks, hipStream_t stream) {
  return inv_dispatch(inst, nullptr, jobs, pre, nj, blocks, stream);
}

hipError_t plan_hadamard(bool fp64, bool bf16, int F, const void* Khat, const void* Qhat, const int32_t* halo,
                         int64_t n_blocks, const int32_t* blk_tgt, const int32_t* blk_src,
                         const int32_t* blk_list, const int32_t* tbase, int64_t n_clusters, int nvec,
                         int split, void* Phat, HadBlockArgs& ab, HadGatherArgs& ag, int64_t& blocks) {
  const int64_t n_rows = n_clusters * nvec;
  blocks = 0;
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
    ag = HadGatherArgs{Khat, Qhat, halo, n_clusters, nvec, n_rows, n_chunks, tpw, total, Phat};
    blocks = 8 * ((total + 7) / 8);
    return hipSuccess;
  }
  // persistent form (split 0): a device-full of workgroups, each taking one
  // run of the frequency-major items (the B operand is loaded once per
  // frequency in a run); unit form (1): one workgroup per 8 items; frequency
  // form (2): one workgroup per frequency, over all its items
  static const int64_t res_block = resident_wgs(hadamard_block_kernel, kHadThreads);
  static const int64_t res_split = resident_wgs(hadamard_split_kernel, kHadThreads);
  const int64_t resident = bf16 ? res_split : res_block;
  const int64_t n_items = n_blocks * nvec;
  if (resident < 8 || n_items >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  const int64_t total = (int64_t)F * n_items;
  int64_t unit_len, n_units, n_wgs;
  if (split == 1 || split == 2) {
    unit_len = split == 1 ? 8 : n_items;
    n_units = (total + unit_len - 1) / unit_len;
    n_wgs = n_units;
  } else {
    n_wgs = min(total, resident / 8 * 8);
    unit_len = (total + n_wgs - 1) / n_wgs;
    n_units = (total + unit_len - 1) / unit_len;
  }
  ab = HadBlockArgs{Khat, Qhat, blk_tgt, blk_src, blk_list, tbase, (int)n_items, nvec, n_rows, total,
                    unit_len, n_units, n_wgs, Phat};
  blocks = 8 * ((n_wgs + 7) / 8);
  return hipSuccess;
}

hipError_t launch_hadamard(bool fp64, bool bf16, int F, const void* Khat, const void* Qhat,
                           const int32_t* halo, int64_t n_blocks, const int32_t* blk_tgt,
                           const int32_t* blk_src, const int32_t* blk_list, const int32_t* tbase,
                           int64_t n_clusters, int nvec, bool units, void* Phat,
                           hipStream_t stream) {
  HadBlockArgs ab;
  HadGatherArgs ag;
  int64_t blocks;
  hipError_t e = plan_hadamard(fp64, bf16, F, Khat, Qhat, halo, n_blocks, blk_tgt, blk_src, blk_list, tbase,
                               n_clusters, nvec, units ? 1 : 0, Phat, ab, ag, blocks);
  if (e != hipSuccess) return e;
  return had_dispatch(hadamard_inst(fp64, bf16), fp64 ? (const void*)&ag : (const void*)&ab, nullptr,
                      nullptr, 0, blocks, stream);
}

hipError_t launch_hadamard_group(int inst, const void* jobs, const int64_t* pre, int nj, int64_t blocks,
                                 hipStream_t stream) {
  return had_dispatch(inst, nullptr, jobs, pre, nj, blocks, stream);
}

int64_t hadamard_split_bytes(int F) { return (int64_t)F * 3 * 13 * 64 * 16; }

hipError_t launch_hadamard_split_prep(const void* Khat, int F, void* parts, hipStream_t stream) {
  const int64_t n = (int64_t)F * 13 * 64;
  if (n == 0) return hipSuccess;
  hadamard_split_prep_kernel<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(
      static_cast<const float2*>(Khat), F, static_cast<v8bf*>(parts));
  return hipGetLastError();
}

}  // namespace kifmm
