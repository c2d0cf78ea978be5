// BLAS-M2L on gfx950 (Section 3.2 of arXiv 2408.07436, steps 3-5 fused).
//
// For every level the compressed check potential of a target box is
//     phi~_tau = sum_t  Ubar_t (Vbar'_t^T q~_{tau + t})           (two-stage)
// or  phi~_tau = sum_t  C_t q~_{tau + t}                             (single)
// over the transfer vectors of its interaction list.  The paper gathers the
// compressed multipoles of each t into a buffer (step 3), runs two GEMMs
// per t (step 4) and accumulates per target (step 5); here a workgroup owns a
// tile of target boxes of one octant class (so they share their transfer
// vectors) times all charge vectors, keeps the accumulators in registers over
// the whole t loop, gathers the source columns straight into MFMA operands,
// and passes the intermediate Xi = Vbar'^T q~ from the first product to the
// second in registers: the first product's accumulator layout is the second
// product's B-operand layout, with the K order of the second product permuted
// accordingly (operators are packed in that order on the host).
//
// Three arithmetic modes: FP64 (v_mfma_f64_16x16x4f64), FP32
// (v_mfma_f32_16x16x4f32) and BF16x3 (v_mfma_f32_16x16x32_bf16 with both
// operands split a = hi + lo in bf16, products hi*hi + hi*lo + lo*hi,
// FP32 accumulation).  Accumulation order over t is fixed (ascending t).
#include <type_traits>

#include "kernels.h"

namespace kifmm {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kMaxRB = 10;  // accumulator row blocks of 16: k_pad <= 160

__device__ inline v4f mf32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline v4d mf64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfbf(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline v4f ld4(const float* p) { return *reinterpret_cast<const v4f*>(p); }
__device__ inline v4d ld4(const double* p) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  return v4d{a.x, a.y, b.x, b.y};
}
__device__ inline v8bf ld8bf(const __bf16* p) { return *reinterpret_cast<const v8bf*>(p); }

// x = hi + lo, both round-to-nearest-even bf16
__device__ inline void split8(const float* x, v8bf& hi, v8bf& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    lo[e] = (__bf16)(x[e] - (float)h);
  }
}

// Tiles in consecutive runs per XCD: workgroup b runs on XCD b % 8, and
// neighbouring tiles (consecutive boxes of one octant class) gather many of
// the same source columns, which then meet in that XCD's L2.  The grid is a
// multiple of 8; -1 past the last tile.
__device__ inline int xcd_tile(int64_t ntiles) {
  const int64_t b = blockIdx.x, per_xcd = gridDim.x / 8;
  const int64_t t = (b % 8) * per_xcd + b / 8;
  return t < ntiles ? (int)t : -1;
}

struct ColInfo {
  int slot[2], v[2];
  bool ok[2];
};

__device__ inline ColInfo columns(const BlasM2L& a, int wave, int l16) {
  ColInfo c;
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int col = (wave * 2 + ct) * 16 + l16;
    c.ok[ct] = col < a.C;
    c.slot[ct] = c.ok[ct] ? col / a.nvec : 0;
    c.v[ct] = c.ok[ct] ? col - c.slot[ct] * a.nvec : 0;
  }
  return c;
}

// ---- FP32 / FP64 -----------------------------------------------------------
// RB / KB: accumulator row blocks (k_pad / 16) and Xi row blocks (k_t pad
// / 16) the instance holds registers for; the launcher takes the smallest
// instance that covers the operators, so FP64 fits two waves per SIMD.
template <typename T, bool TWO, int RB, int KB>
__global__ __launch_bounds__(256, (sizeof(T) == 8 ? (RB > 8 ? 1 : 2) : (RB > 8 ? 2 : 3))) void blas_m2l_kernel(BlasM2L a) {
  using V4 = typename std::conditional<sizeof(T) == 4, v4f, v4d>::type;
  constexpr int kMaxKB = KB;
  const int tile = xcd_tile(a.ntiles);
  if (tile < 0) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int l16 = lane % 16, g4 = lane / 16;
  const int nrb = a.kp / 16;
  const T* q = static_cast<const T*>(a.q);
  const T* ops = static_cast<const T*>(a.op_hi);
  const ColInfo ci = columns(a, wave, l16);
  V4 acc[RB][2];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rb][ct] = V4{T(0), T(0), T(0), T(0)};

  const int64_t e0 = a.tl_offs[tile], e1 = a.tl_offs[tile + 1];
  for (int64_t e = e0; e < e1; ++e) {
    const int t = a.tl_t[e];
    const T* Vt = ops + a.op_off[t];
    const T* qp[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int sb = ci.ok[ct] ? a.tl_src[e * a.TB + ci.slot[ct]] : -1;
      qp[ct] = sb >= 0 ? q + ((int64_t)sb * a.nvec + ci.v[ct]) * a.kp : nullptr;
    }
    if constexpr (TWO) {
      const int ktp = a.ktp[t];
      const int nkb = ktp / 16;
      const int nq = a.ktq[t];  // second-product K steps that hold Xi rows
      const T* Ub = Vt + (int64_t)ktp * a.kp;
      V4 xi[kMaxKB][2];
#pragma unroll
      for (int rx = 0; rx < kMaxKB; ++rx)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) xi[rx][ct] = V4{T(0), T(0), T(0), T(0)};
      for (int kb = 0; kb < a.kp; kb += 16) {
        V4 bq[2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          bq[ct] = qp[ct] ? ld4(qp[ct] + kb + 4 * g4) : V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int rx = 0; rx < kMaxKB; ++rx) {
          if (rx < nkb) {
            const V4 av = ld4(Vt + (int64_t)(rx * 16 + l16) * a.kp + kb + 4 * g4);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                if constexpr (sizeof(T) == 4)
                  xi[rx][ct] = mf32(av[s], bq[ct][s], xi[rx][ct]);
                else
                  xi[rx][ct] = mf64(av[s], bq[ct][s], xi[rx][ct]);
              }
          }
        }
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb < nrb) {
#pragma unroll
          for (int rx = 0; rx < kMaxKB; ++rx) {
            if (rx < nkb) {
              const V4 au = ld4(Ub + (int64_t)(rb * 16 + l16) * ktp + rx * 16 + 4 * g4);
              if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                  if (4 * rx + s >= nq) continue;  // only zero Xi rows
#pragma unroll
                  for (int ct = 0; ct < 2; ++ct) acc[rb][ct] = mf32(au[s], xi[rx][ct][s], acc[rb][ct]);
                }
              } else {
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                  for (int s = 0; s < 4; ++s) acc[rb][ct] = mf64(au[s], xi[rx][ct][s], acc[rb][ct]);
              }
            }
          }
        }
      }
    } else {
      for (int kb = 0; kb < a.kp; kb += 16) {
        V4 bq[2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          bq[ct] = qp[ct] ? ld4(qp[ct] + kb + 4 * g4) : V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb < nrb) {
            const V4 ac = ld4(Vt + (int64_t)(rb * 16 + l16) * a.kp + kb + 4 * g4);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                if constexpr (sizeof(T) == 4)
                  acc[rb][ct] = mf32(ac[s], bq[ct][s], acc[rb][ct]);
                else
                  acc[rb][ct] = mf64(ac[s], bq[ct][s], acc[rb][ct]);
              }
          }
        }
      }
    }
  }
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    if (!ci.ok[ct]) continue;
    const int box = a.tile_box[tile * a.TB + ci.slot[ct]];
    if (box < 0) continue;
    double* dst = a.out + ((int64_t)box * a.nvec + ci.v[ct]) * a.k;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if (rb < nrb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // FP32 accumulator rows are 4 g4 + i, FP64 rows g4 + 4 i
          const int row = rb * 16 + (sizeof(T) == 4 ? 4 * g4 + i : g4 + 4 * i);
          if (row < a.k) dst[row] = a.scale * (double)acc[rb][ct][i];
        }
      }
    }
  }
}

// ---- BF16 x 3 ----------------------------------------------------------------
template <bool TWO>
__global__ __launch_bounds__(256) void blas_m2l_bf16_kernel(BlasM2L a) {
  constexpr int RB = kMaxRB;
  constexpr int kMaxKB = 4;  // Xi row blocks: k_t pad <= 64
  const int tile = xcd_tile(a.ntiles);
  if (tile < 0) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int l16 = lane % 16, g4 = lane / 16;
  const int nrb = a.kp / 16;
  const float* q = static_cast<const float*>(a.q);
  const __bf16* oph = static_cast<const __bf16*>(a.op_hi);
  const __bf16* opl = static_cast<const __bf16*>(a.op_lo);
  const ColInfo ci = columns(a, wave, l16);
  v4f acc[RB][2];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rb][ct] = v4f{0.f, 0.f, 0.f, 0.f};

  const int64_t e0 = a.tl_offs[tile], e1 = a.tl_offs[tile + 1];
  for (int64_t e = e0; e < e1; ++e) {
    const int t = a.tl_t[e];
    const int64_t off = a.op_off[t];
    const float* qp[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int sb = ci.ok[ct] ? a.tl_src[e * a.TB + ci.slot[ct]] : -1;
      qp[ct] = sb >= 0 ? q + ((int64_t)sb * a.nvec + ci.v[ct]) * a.kp : nullptr;
    }
    if constexpr (TWO) {
      const int ktp = a.ktp[t];
      const int nkb = ktp / 16;
      const int64_t uoff = off + (int64_t)ktp * a.kp;
      v4f xi[kMaxKB][2];
#pragma unroll
      for (int rx = 0; rx < kMaxKB; ++rx)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) xi[rx][ct] = v4f{0.f, 0.f, 0.f, 0.f};
      for (int kb = 0; kb < a.kp; kb += 32) {
        v8bf bh[2], bl[2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          float x[8];
          if (qp[ct]) {
            const v4f u = ld4(qp[ct] + kb + 8 * g4), w = ld4(qp[ct] + kb + 8 * g4 + 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              x[i] = u[i];
              x[4 + i] = w[i];
            }
          } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = 0.f;
          }
          split8(x, bh[ct], bl[ct]);
        }
#pragma unroll
        for (int rx = 0; rx < kMaxKB; ++rx) {
          if (rx < nkb) {
            const int64_t o = off + (int64_t)(rx * 16 + l16) * a.kp + kb + 8 * g4;
            const v8bf ah = ld8bf(oph + o), al = ld8bf(opl + o);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
              xi[rx][ct] = mfbf(ah, bh[ct], xi[rx][ct]);
              xi[rx][ct] = mfbf(ah, bl[ct], xi[rx][ct]);
              xi[rx][ct] = mfbf(al, bh[ct], xi[rx][ct]);
            }
          }
        }
      }
      // second product: K' steps of 32 take Xi row blocks (2j, 2j+1); lane
      // element e < 4 is row 4 g4 + e of block 2j, e >= 4 row 4 g4 + e - 4 of
      // block 2j + 1 (Ubar's columns are packed in that order)
      v8bf xh[kMaxKB / 2][2], xl[kMaxKB / 2][2];
#pragma unroll
      for (int j = 0; j < kMaxKB / 2; ++j)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          float x[8];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            x[i] = xi[2 * j][ct][i];
            x[4 + i] = xi[2 * j + 1][ct][i];
          }
          split8(x, xh[j][ct], xl[j][ct]);
        }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb < nrb) {
#pragma unroll
          for (int j = 0; j < kMaxKB / 2; ++j) {
            if (2 * j < nkb) {
              const int64_t o = uoff + (int64_t)(rb * 16 + l16) * ktp + 32 * j + 8 * g4;
              const v8bf ah = ld8bf(oph + o), al = ld8bf(opl + o);
#pragma unroll
              for (int ct = 0; ct < 2; ++ct) {
                acc[rb][ct] = mfbf(ah, xh[j][ct], acc[rb][ct]);
                acc[rb][ct] = mfbf(ah, xl[j][ct], acc[rb][ct]);
                acc[rb][ct] = mfbf(al, xh[j][ct], acc[rb][ct]);
              }
            }
          }
        }
      }
    } else {
      for (int kb = 0; kb < a.kp; kb += 32) {
        v8bf bh[2], bl[2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          float x[8];
          if (qp[ct]) {
            const v4f u = ld4(qp[ct] + kb + 8 * g4), w = ld4(qp[ct] + kb + 8 * g4 + 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              x[i] = u[i];
              x[4 + i] = w[i];
            }
          } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = 0.f;
          }
          split8(x, bh[ct], bl[ct]);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (rb < nrb) {
            const int64_t o = off + (int64_t)(rb * 16 + l16) * a.kp + kb + 8 * g4;
            const v8bf ah = ld8bf(oph + o), al = ld8bf(opl + o);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
              acc[rb][ct] = mfbf(ah, bh[ct], acc[rb][ct]);
              acc[rb][ct] = mfbf(ah, bl[ct], acc[rb][ct]);
              acc[rb][ct] = mfbf(al, bh[ct], acc[rb][ct]);
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    if (!ci.ok[ct]) continue;
    const int box = a.tile_box[tile * a.TB + ci.slot[ct]];
    if (box < 0) continue;
    double* dst = a.out + ((int64_t)box * a.nvec + ci.v[ct]) * a.k;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if (rb < nrb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = rb * 16 + 4 * g4 + i;
          if (row < a.k) dst[row] = a.scale * (double)acc[rb][ct][i];
        }
      }
    }
  }
}

// q~ (FP64, [box][v][k]) -> padded [box][v][kp] in T
template <typename T>
__global__ void pad_convert_kernel(const double* __restrict__ in, int k, int64_t ncols, int kp,
                                   T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= ncols * kp) return;
  const int64_t col = i / kp;
  const int r = (int)(i - col * kp);
  out[i] = r < k ? (T)in[col * k + r] : T(0);
}

}  // namespace

hipError_t launch_blas_m2l(const BlasM2L& a, int mode, bool two_stage, hipStream_t stream) {
  if (a.ntiles == 0) return hipSuccess;
  if (a.kp > 16 * kMaxRB || a.C > 128) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(8 * ((a.ntiles + 7) / 8))), block(256);
  if (mode == 0 || mode == 1) {
    if (two_stage && a.ktp_max > 48) return hipErrorInvalidValue;
    const int nrb = a.kp / 16;
    const int rb = nrb <= 4 ? 4 : nrb <= 8 ? 8 : 10;
    const int kb = two_stage ? (a.ktp_max <= 16 ? 1 : a.ktp_max <= 32 ? 2 : 3) : 1;
#define KIFMM_BLAS(TT, TW, RR, KK) blas_m2l_kernel<TT, TW, RR, KK><<<grid, block, 0, stream>>>(a)
#define KIFMM_BLAS_KB(TT, RR)                 \
  if (!two_stage) KIFMM_BLAS(TT, false, RR, 1); \
  else if (kb == 1) KIFMM_BLAS(TT, true, RR, 1); \
  else if (kb == 2) KIFMM_BLAS(TT, true, RR, 2); \
  else KIFMM_BLAS(TT, true, RR, 3);
#define KIFMM_BLAS_RB(TT)                     \
  if (rb == 4) { KIFMM_BLAS_KB(TT, 4) }       \
  else if (rb == 8) { KIFMM_BLAS_KB(TT, 8) }  \
  else { KIFMM_BLAS_KB(TT, 10) }
    if (mode == 0) {
      KIFMM_BLAS_RB(double)
    } else {
      KIFMM_BLAS_RB(float)
    }
#undef KIFMM_BLAS_RB
#undef KIFMM_BLAS_KB
#undef KIFMM_BLAS
  } else {
    if (two_stage) blas_m2l_bf16_kernel<true><<<grid, block, 0, stream>>>(a);
    else blas_m2l_bf16_kernel<false><<<grid, block, 0, stream>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_pad_convert(const double* in, int k, int64_t ncols, int kp, bool fp64, void* out,
                              hipStream_t stream) {
  const int64_t n = ncols * kp;
  if (n == 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (fp64)
    pad_convert_kernel<double><<<grid, 256, 0, stream>>>(in, k, ncols, kp, (double*)out);
  else
    pad_convert_kernel<float><<<grid, 256, 0, stream>>>(in, k, ncols, kp, (float*)out);
  return hipGetLastError();
}

}  // namespace kifmm
