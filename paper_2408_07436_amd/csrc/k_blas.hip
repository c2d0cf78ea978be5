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

// ---- stacked form (two-stage operators) -------------------------------------
// Column c of a tile (TB boxes x nvec vectors, c < C): slot c / nvec, vector
// c % nvec; wave w takes columns 32 w .. 32 w + 31 as two MFMA column tiles.
struct StackCols {
  int slot[2], v[2];
  bool ok[2];
};
__device__ inline StackCols stack_columns(const BlasStack& a, int wave, int l16) {
  StackCols c;
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int col = (wave * 2 + ct) * 16 + l16;
    c.ok[ct] = col < a.C;
    c.slot[ct] = c.ok[ct] ? col / a.nvec : 0;
    c.v[ct] = c.ok[ct] ? col - c.slot[ct] * a.nvec : 0;
  }
  return c;
}

// Work item w of a grid that is a multiple of 8, consecutive items on one
// XCD (workgroup b runs on XCD b % 8): tiles are ordered by class, so an
// XCD's L2 holds the operators of about one class.
__device__ inline int64_t xcd_item() {
  const int64_t b = blockIdx.x, per_xcd = gridDim.x / 8;
  return (b % 8) * per_xcd + b / 8;
}

// Stage A, FP32 / FP64: one workgroup per (tile, rpw consecutive 128-row
// blocks of the class's stacked operator), the blocks' K slabs as one
// pipeline; xi[box][row][v] for rows < Rs.
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 2 : 3) void stack_a_kernel(BlasStack a, int rpw) {
  using V4 = typename std::conditional<sizeof(T) == 4, v4f, v4d>::type;
  const int nmb = a.Rpad / 128, nparts = (nmb + rpw - 1) / rpw;
  const int64_t w = xcd_item();
  if (w >= a.ntiles * nparts) return;
  const int64_t tile = w / nparts;
  const int mb0 = (int)(w - tile * nparts) * rpw;
  const int nrb = min(rpw, nmb - mb0);
  const int nsl = a.kp / 16;  // K slabs per row block
  const int cls = a.tile_class[tile];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int l16 = lane % 16, g4 = lane / 16;
  const T* q = static_cast<const T*>(a.q_hi);
  const T* A = static_cast<const T*>(a.A_hi) + (int64_t)cls * a.Rpad * a.kp;
  const StackCols cc = stack_columns(a, wave, l16);
  int box[2];
  const T* qp[2];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    box[ct] = cc.ok[ct] ? a.tile_box[tile * a.TB + cc.slot[ct]] : -1;
    qp[ct] = box[ct] >= 0 ? q + ((int64_t)box[ct] * a.nvec + cc.v[ct]) * a.kp : nullptr;
  }
  V4 acc[8][2];
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rb][ct] = V4{T(0), T(0), T(0), T(0)};
  // The workgroup's 128 operator rows are shared by its four waves: each K
  // slab of 16 is staged once in LDS (double-buffered; rows padded to RS
  // elements so that a quarter-wave's 16 row reads fall in distinct banks),
  // the next slab's operator and multipole values are loaded from global
  // memory before the current slab's MFMAs, and each row block's LDS read is
  // issued one block ahead.
  constexpr int RS = sizeof(T) == 8 ? 18 : 20;
  __shared__ __attribute__((aligned(16))) T lds[2][128 * RS];
  const V4 zero4 = V4{T(0), T(0), T(0), T(0)};
  const int srow = threadIdx.x >> 1, shalf = threadIdx.x & 1;
  V4 st0, st1;  // 8 staged operator values of this thread
  // slab s of the pipeline: row block mb0 + s / nsl, K from 16 (s % nsl)
  auto gload = [&](int s) {
    const T* src = A + ((int64_t)(mb0 + s / nsl) * 128 + srow) * a.kp + shalf * 8 + 16 * (s % nsl);
    st0 = ld4(src);
    st1 = ld4(src + 4);
  };
  auto swrite = [&](int buf) {
    T* d = &lds[buf][srow * RS + shalf * 8];
    if constexpr (sizeof(T) == 8) {
      reinterpret_cast<double2*>(d)[0] = double2{st0[0], st0[1]};
      reinterpret_cast<double2*>(d)[1] = double2{st0[2], st0[3]};
      reinterpret_cast<double2*>(d)[2] = double2{st1[0], st1[1]};
      reinterpret_cast<double2*>(d)[3] = double2{st1[2], st1[3]};
    } else {
      reinterpret_cast<v4f*>(d)[0] = st0;
      reinterpret_cast<v4f*>(d)[1] = st1;
    }
  };
  // loads without branches (a column without a box reads box 0's values and
  // discards them; the last slab reloads itself), so that the compiler can
  // count the loads in flight and wait only for the current slab's
  const T* qs[2];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) qs[ct] = qp[ct] ? qp[ct] : q;
  auto load_q = [&](int kb, V4 (&bq)[2]) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const V4 v = ld4(qs[ct] + kb + 4 * g4);
      bq[ct] = qp[ct] ? v : zero4;
    }
  };
  T* xi = static_cast<T*>(a.xi_hi);
  // row block mb's results.  FP32 accumulator rows are 4 g4 + i, FP64 rows
  // g4 + 4 i; Rs is a multiple of 4, so an FP32 lane's four rows exist
  // together and an FP64 row block's rows g4 + 4 i exist for i below a bound
  // that is the same for every lane
  auto store_block = [&](int mb) {
    const int rows_left = a.Rs - mb * 128;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      if (box[ct] < 0) continue;
      T* dst = xi + ((int64_t)box[ct] * a.Rs + mb * 128 + (sizeof(T) == 4 ? 4 * g4 : g4)) * a.nvec + cc.v[ct];
#pragma unroll
      for (int rb = 0; rb < 8; ++rb) {
        if (16 * rb >= rows_left) break;
        T* d = dst + (int64_t)16 * rb * a.nvec;
        if constexpr (sizeof(T) == 4) {
          if (16 * rb + 4 * g4 < rows_left) {
#pragma unroll
            for (int i = 0; i < 4; ++i) d[(int64_t)i * a.nvec] = acc[rb][ct][i];
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (16 * rb + 4 * i < rows_left) d[(int64_t)4 * i * a.nvec] = acc[rb][ct][i];
        }
      }
    }
  };
  const int nst = nrb * nsl;
  gload(0);
  swrite(0);
  V4 bq[2];
  load_q(0, bq);
  __syncthreads();
  int buf = 0;
  for (int st = 0; st < nst; ++st, buf ^= 1) {
    const bool more = st + 1 < nst;
    const int sn = more ? st + 1 : st;
    V4 nbq[2];
    gload(sn);
    load_q(16 * (sn % nsl), nbq);
    // keep the next slab's loads ahead of this slab's MFMAs
    __builtin_amdgcn_sched_barrier(0);
    const T* L = &lds[buf][l16 * RS + 4 * g4];
    V4 av = ld4(L);
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) {
      const V4 nav = rb < 7 ? ld4(L + (rb + 1) * 16 * RS) : zero4;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          if constexpr (sizeof(T) == 4)
            acc[rb][ct] = mf32(av[s], bq[ct][s], acc[rb][ct]);
          else
            acc[rb][ct] = mf64(av[s], bq[ct][s], acc[rb][ct]);
        }
      av = nav;
    }
    if (more) swrite(buf ^ 1);
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) bq[ct] = nbq[ct];
    // FP32: a row block's results out after its last slab; FP64 (whose
    // accumulators fill the registers) runs one row block per workgroup
    if constexpr (sizeof(T) == 4) {
      if (st % nsl == nsl - 1) {
        store_block(mb0 + st / nsl);
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) acc[rb][ct] = zero4;
      }
    }
  }
  if constexpr (sizeof(T) == 8) store_block(mb0);
}

// Stage B, FP32 / FP64: one workgroup per target tile; K step n covers rows
// 4n .. 4n + 3 of the class's stacked K (one transfer vector j, whose xi
// rows start at info[n].y).  The operator, the same for the four waves, is
// staged in LDS a chunk of steps at a time (double-buffered; each lane's
// values padded to a 16-byte multiple off 64 bytes so that 16-byte reads of
// consecutive lanes spread over the banks), the next chunk loaded from
// global memory while the current one is used.  The other loads run ahead
// of the MFMAs: the table entry three steps, the source box two steps, xi
// and the operator (from LDS) one step.
// Work item of Stage B: (tile, part of its K steps), consecutive items per
// XCD; the part's steps [n0, n1).
struct StackPart {
  int64_t tile;
  int part, n0, n1;
};
__device__ inline bool stack_part(const BlasStack& a, int nst, StackPart& p) {
  const int64_t w = xcd_item();
  if (w >= a.ntiles * a.ksplit) return false;
  p.tile = w / a.ksplit;
  p.part = (int)(w - p.tile * a.ksplit);
  p.n0 = (int)((int64_t)nst * p.part / a.ksplit);
  p.n1 = (int)((int64_t)nst * (p.part + 1) / a.ksplit);
  return true;
}

// Stage B's result for one column: the scaled sum (one part), or the raw
// partial sum of this part (several parts; the reduction scales).
__device__ inline double* stack_dst(const BlasStack& a, const StackPart& p, int box, int v) {
  if (a.ksplit == 1) return a.out + ((int64_t)box * a.nvec + v) * a.k;
  return a.partial + (((int64_t)p.part * a.n_boxes + box) * a.nvec + v) * a.k;
}

template <typename T, int RBO>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 2 : 3) void stack_b_kernel(BlasStack a) {
  using V4 = typename std::conditional<sizeof(T) == 4, v4f, v4d>::type;
  // steps per staged chunk: 4 in FP64 where that keeps 16-byte staging (two
  // workgroups' double buffers fit a CU's LDS), else kStackChunk
  constexpr int C = sizeof(T) == 8 && RBO % 4 == 0 ? 4 : kStackChunk;
  // padded values per lane in LDS (16-byte aligned lanes; at RBO = 8 the
  // lanes of a quarter wave start in distinct bank groups)
  constexpr int LS = sizeof(T) == 8 ? RBO + 2 : (RBO + 3) / 4 * 4 + 4;
  constexpr int PT = C * RBO / 4;  // staged values per thread (a multiple of 4: RBO is even)
  static_assert(RBO % 2 == 0 && PT % 4 == 0, "staging in 16-byte loads and pairs");
  __shared__ __attribute__((aligned(16))) T ops[2][C * 64 * LS];
  StackPart sp;
  if (!stack_part(a, a.nsteps, sp)) return;
  const int64_t tile = sp.tile;
  const int cls = a.tile_class[tile];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int l16 = lane % 16, g4 = lane / 16;
  const StackCols cc = stack_columns(a, wave, l16);
  const int32_t* src = a.tile_src + (int64_t)tile * a.J * a.TB;
  const int2* info = reinterpret_cast<const int2*>(a.info) + (int64_t)cls * a.nsteps;
  const T* Bcls = static_cast<const T*>(a.B_hi) + (int64_t)cls * a.nsteps * 64 * RBO;
  const T* xi = static_cast<const T*>(a.xi_hi);
  const int64_t rs = a.Rs;
  const int nb = sp.n0, nst = sp.n1;  // steps of this part
  V4 acc[RBO][2];
#pragma unroll
  for (int rb = 0; rb < RBO; ++rb)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rb][ct] = V4{T(0), T(0), T(0), T(0)};
  if (nb >= nst) return;
  // staging: thread t holds values [t PT, (t + 1) PT) of a chunk (two lanes'
  // worth in step order), written to LDS at the lanes' padded slots
  V4 stg[PT / 4];
  auto gload = [&](int n) {
    const T* p = Bcls + (int64_t)n * 64 * RBO + threadIdx.x * PT;
#pragma unroll
    for (int i = 0; i < PT / 4; ++i) stg[i] = ld4(p + 4 * i);
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PT / 4; ++i)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // pairs never straddle two lanes' values (RBO is even)
        const int e = threadIdx.x * PT + 4 * i + 2 * h;  // value index within the chunk
        T* d = &ops[buf][(e / RBO) * LS + e % RBO];
        if constexpr (sizeof(T) == 8)
          *reinterpret_cast<double2*>(d) = double2{stg[i][2 * h], stg[i][2 * h + 1]};
        else
          *reinterpret_cast<float2*>(d) = float2{stg[i][2 * h], stg[i][2 * h + 1]};
      }
  };
  auto oread = [&](int buf, int j, T (&o)[RBO]) {
    const T* s = &ops[buf][(j * 64 + lane) * LS];
#pragma unroll
    for (int rb = 0; rb < RBO; rb += 4) {
      const V4 v = ld4(s + rb);
#pragma unroll
      for (int i = 0; i < 4 && rb + i < RBO; ++i) o[rb + i] = v[i];
    }
  };
  // Loads without branches (clamped addresses); a loaded value is masked
  // where it is used, so the compiler waits for it only then.  The chunk's
  // steps are unrolled, so every iteration issues the same loads and the
  // waits count exactly.  Pipeline depth: the xi values of step n are loaded
  // at step n - D, their source boxes at n - D - 1, the table entries at
  // n - D - 2.
  constexpr int D = sizeof(T) == 8 ? 2 : 3;
  const int sl[2] = {cc.ok[0] ? cc.slot[0] : 0, cc.ok[1] ? cc.slot[1] : 0};
  auto entry = [&](int n) -> int2 {
    const int2 e = info[min(n, nst - 1)];
    return n < nst ? e : make_int2(-1, 0);
  };
  auto src_raw = [&](int2 in, int ct) -> int { return src[max(in.x, 0) * a.TB + sl[ct]]; };
  auto x_raw = [&](int sb, int row, int ct) -> T {
    return xi[((int64_t)max(sb, 0) * rs + row + g4) * a.nvec + cc.v[ct]];
  };
  // pipeline registers: eD / eD1 = table entries of steps n + D and n + D + 1;
  // sD / svD = raw source boxes of step n + D and their validity; xr[i] /
  // xv[i] = raw xi values of step n + i and their validity; o0 = operator
  // values of step n
  int2 eD = entry(nb + D), eD1 = entry(nb + D + 1);
  int sD[2];
  bool svD[2];
  T xr[D][2];
  bool xv[D][2];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const int2 e = entry(nb + i);
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int sb = src_raw(e, ct);
      xv[i][ct] = cc.ok[ct] && e.x >= 0 && sb >= 0;
      xr[i][ct] = x_raw(xv[i][ct] ? sb : 0, e.y, ct);
    }
  }
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    sD[ct] = src_raw(eD, ct);
    svD[ct] = cc.ok[ct] && eD.x >= 0;
  }
  T o0[RBO];
  int buf = 0;
  gload(nb);
  swrite(0);
  __syncthreads();
  oread(0, 0, o0);
  for (int c0 = nb; c0 < nst; c0 += C) {
    // the next chunk's operator (the padded buffer keeps the last one in bounds)
    gload(c0 + C);
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int n = c0 + j;
      // loads of later steps
      const int2 eD2 = entry(n + D + 2);
      int sD1[2];
      bool svD1[2], xvD[2];
      T xrD[2];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        sD1[ct] = src_raw(eD1, ct);
        svD1[ct] = cc.ok[ct] && eD1.x >= 0;
        xvD[ct] = svD[ct] && sD[ct] >= 0;
        xrD[ct] = x_raw(xvD[ct] ? sD[ct] : 0, eD.y, ct);
      }
      // products of step n (none past the part's end)
      T o1[RBO];
      if (n < nst) {
        T x0[2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) x0[ct] = xv[0][ct] ? xr[0][ct] : T(0);
#pragma unroll
        for (int rb = 0; rb < RBO; ++rb)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) {
            if constexpr (sizeof(T) == 4)
              acc[rb][ct] = mf32(o0[rb], x0[ct], acc[rb][ct]);
            else
              acc[rb][ct] = mf64(o0[rb], x0[ct], acc[rb][ct]);
          }
      }
      // the next step's operator values, read while the MFMAs run
      if (j + 1 < C) oread(buf, j + 1, o1);
      // roll
#pragma unroll
      for (int i = 0; i + 1 < D; ++i)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          xr[i][ct] = xr[i + 1][ct];
          xv[i][ct] = xv[i + 1][ct];
        }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        xr[D - 1][ct] = xrD[ct];
        xv[D - 1][ct] = xvD[ct];
        sD[ct] = sD1[ct];
        svD[ct] = svD1[ct];
      }
      eD = eD1;
      eD1 = eD2;
      if (j + 1 < C) {
#pragma unroll
        for (int rb = 0; rb < RBO; ++rb) o0[rb] = o1[rb];
      }
    }
    // end of a chunk: the next one into the other buffer (its last reader
    // passed the previous barrier)
    swrite(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    oread(buf, 0, o0);
  }
  const double scale = a.ksplit == 1 ? a.scale : 1.0;
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    if (!cc.ok[ct]) continue;
    const int box = a.tile_box[tile * a.TB + cc.slot[ct]];
    if (box < 0) continue;
    double* dst = stack_dst(a, sp, box, cc.v[ct]);
#pragma unroll
    for (int rb = 0; rb < RBO; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb * 16 + (sizeof(T) == 4 ? 4 * g4 + i : g4 + 4 * i);
        if (row < a.k) dst[row] = scale * (double)acc[rb][ct][i];
      }
  }
}

// out = scale * (sum of the ksplit partial sums, in order)
__global__ void stack_reduce_kernel(BlasStack a) {
  const int64_t total = a.n_boxes * a.nvec * a.k;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  double sum = 0.0;
  for (int p = 0; p < a.ksplit; ++p) sum += a.partial[(int64_t)p * total + i];
  a.out[i] = a.scale * sum;
}

// Stage A, BF16 parts: operands split into NP = 2 parts (BF16x3: hi + lo,
// three products) or NP = 3 (BF16x6: x0 + x1 + x2, the six products of
// order at most two, FP32-class), FP32 accumulation; xi stored split,
// [box][Rs / 8][v][8] so that eight consecutive rows of one column are one
// 16-byte load in Stage B.
// The NP bf16 parts (round to nearest even; each residual exact in FP32) of
// two values, packed two per dword (value x in the low half) into word w of
// each part's uint2.
template <int NP>
__device__ __forceinline__ void split_pairs(float x, float y, uint2 (&p)[NP], int w) {
  typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
  typedef float v2f __attribute__((ext_vector_type(2)));
  float rx = x, ry = y;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{rx, ry}, v2bf));
    if (w == 0) p[q].x = h; else p[q].y = h;
    rx -= __uint_as_float(h << 16);
    ry -= __uint_as_float(h & 0xffff0000u);
  }
}
template <int NP>
__device__ __forceinline__ void parts_mfma(v4f& acc, const v8bf (&a)[NP], const v8bf (&b)[NP]) {
  acc = mfbf(a[0], b[0], acc);
  acc = mfbf(a[0], b[1], acc);
  acc = mfbf(a[1], b[0], acc);
  if (NP == 3) {
    acc = mfbf(a[0], b[NP - 1], acc);
    acc = mfbf(a[1], b[1], acc);
    acc = mfbf(a[NP - 1], b[0], acc);
  }
}
// A workgroup takes rpw consecutive 128-row blocks of one tile (fewer in the
// class's last part) as one pipeline of K slabs, so that only its first slab
// waits for loads with nothing in flight.
template <int NP>
__global__ __launch_bounds__(256, 2) void stack_a_bf16_kernel(BlasStack a, int rpw) {
  const int nmb = a.Rpad / 128, nparts = (nmb + rpw - 1) / rpw;
  const int64_t w = xcd_item();
  if (w >= a.ntiles * nparts) return;
  const int64_t tile = w / nparts;
  const int mb0 = (int)(w - tile * nparts) * rpw;
  const int nrb = min(rpw, nmb - mb0);
  const int nsl = a.kp / 32;  // K slabs per row block
  const int cls = a.tile_class[tile];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int l16 = lane % 16, g4 = lane / 16;
  const __bf16* qp[3] = {static_cast<const __bf16*>(a.q_hi), static_cast<const __bf16*>(a.q_lo),
                         static_cast<const __bf16*>(a.q_p2)};
  const int64_t aoff = (int64_t)cls * a.Rpad * a.kp;
  const __bf16* Ap[3] = {static_cast<const __bf16*>(a.A_hi) + aoff, static_cast<const __bf16*>(a.A_lo) + aoff,
                         NP == 3 ? static_cast<const __bf16*>(a.A_p2) + aoff : nullptr};
  const StackCols cc = stack_columns(a, wave, l16);
  int box[2];
  int64_t qo[2];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    box[ct] = cc.ok[ct] ? a.tile_box[tile * a.TB + cc.slot[ct]] : -1;
    qo[ct] = box[ct] >= 0 ? ((int64_t)box[ct] * a.nvec + cc.v[ct]) * a.kp : -1;
  }
  v4f acc[8][2];
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rb][ct] = v4f{0.f, 0.f, 0.f, 0.f};
  const v8bf zero8 = {};
  // As in the FP32 / FP64 Stage A: each K slab (32) of the workgroup's 128
  // operator rows, every part, staged once in LDS (double-buffered, rows
  // padded to 80 bytes for conflict-free 16-byte reads), the next slab's
  // operator and multipole loads issued branch-free ahead of the current
  // slab's MFMAs.
  constexpr int RS = 40;  // bf16 values per LDS row
  __shared__ __attribute__((aligned(16))) __bf16 lds[2][NP][128 * RS];
  const int srow = threadIdx.x >> 1, shalf = threadIdx.x & 1;
  v8bf sg[NP][2];  // 16 staged values of each part of this thread
  // slab s of the pipeline: row block mb0 + s / nsl, K from 32 (s % nsl)
  auto gload = [&](int s) {
    const int64_t o = ((int64_t)(mb0 + s / nsl) * 128 + srow) * a.kp + shalf * 16 + 32 * (s % nsl);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      sg[q][0] = ld8bf(Ap[q] + o);
      sg[q][1] = ld8bf(Ap[q] + o + 8);
    }
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      __bf16* dq = &lds[buf][q][srow * RS + shalf * 16];
      reinterpret_cast<v8bf*>(dq)[0] = sg[q][0];
      reinterpret_cast<v8bf*>(dq)[1] = sg[q][1];
    }
  };
  const int64_t qs[2] = {qo[0] >= 0 ? qo[0] : 0, qo[1] >= 0 ? qo[1] : 0};
  auto load_q = [&](int kb, v8bf (&bq)[2][NP]) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const v8bf v = ld8bf(qp[q] + qs[ct] + kb + 8 * g4);
        bq[ct][q] = qo[ct] >= 0 ? v : zero8;
      }
  };
  __bf16* xp[3] = {static_cast<__bf16*>(a.xi_hi), static_cast<__bf16*>(a.xi_lo),
                   static_cast<__bf16*>(a.xi_p2)};
  const int64_t rb_step = (int64_t)16 * a.nvec;
  // row block mb's results: rows mb 128 + 16 rb + 4 g4 .. + 3 of this lane,
  // half g4 % 2 of eight-row group 16 mb + 2 rb + g4 / 2, so one column
  // tile's stores step by 16 nvec values per row block (Rs is a multiple of
  // 8: the four rows exist together)
  auto store_block = [&](int mb) {
    const int rows_left = a.Rs - mb * 128 - 4 * g4;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      if (box[ct] < 0) continue;
      const int64_t o = (((int64_t)box[ct] * (a.Rs / 8) + 16 * mb + (g4 >> 1)) * a.nvec + cc.v[ct]) * 8 + 4 * (g4 & 1);
#pragma unroll
      for (int rb = 0; rb < 8; ++rb) {
        if (16 * rb >= rows_left) break;
        uint2 pv[NP];
        split_pairs<NP>(acc[rb][ct][0], acc[rb][ct][1], pv, 0);
        split_pairs<NP>(acc[rb][ct][2], acc[rb][ct][3], pv, 1);
#pragma unroll
        for (int q = 0; q < NP; ++q) *reinterpret_cast<uint2*>(xp[q] + o + rb * rb_step) = pv[q];
      }
    }
  };
  const int nst = nrb * nsl;
  gload(0);
  swrite(0);
  v8bf bq[2][NP];
  load_q(0, bq);
  __syncthreads();
  int buf = 0;
  for (int st = 0; st < nst; ++st, buf ^= 1) {
    const bool more = st + 1 < nst;
    const int sn = more ? st + 1 : st;
    v8bf nbq[2][NP];
    gload(sn);
    load_q(32 * (sn % nsl), nbq);
    // keep the next slab's loads ahead of this slab's MFMAs
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) {
      v8bf ap[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) ap[q] = ld8bf(&lds[buf][q][l16 * RS + 8 * g4] + rb * 16 * RS);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) parts_mfma<NP>(acc[rb][ct], ap, bq[ct]);
    }
    if (more) swrite(buf ^ 1);
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int q = 0; q < NP; ++q) bq[ct][q] = nbq[ct][q];
    if (st % nsl == nsl - 1) {  // the row block's last slab: its results out
      store_block(mb0 + st / nsl);
#pragma unroll
      for (int rb = 0; rb < 8; ++rb)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[rb][ct] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  }
}

// Stage B, BF16 parts (NP = 2 or 3, as Stage A): K steps of 32 rows; lane
// group g4 takes the eight rows of row group 4n + g4 (info per group),
// possibly of another transfer vector than its neighbours.  Operators
// [8][nsteps][64 lanes][RBO][8] per part.
template <int RBO, int NP>
__global__ __launch_bounds__(256, 2) void stack_b_bf16_kernel(BlasStack a) {
  StackPart sp;
  if (!stack_part(a, a.nsteps, sp)) return;
  const int64_t tile = sp.tile;
  const int cls = a.tile_class[tile];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int l16 = lane % 16, g4 = lane / 16;
  const StackCols cc = stack_columns(a, wave, l16);
  const int32_t* src = a.tile_src + (int64_t)tile * a.J * a.TB;
  const int2* info = reinterpret_cast<const int2*>(a.info) + (int64_t)cls * a.nsteps * 4;
  const int64_t coff = (int64_t)cls * a.nsteps * 64 * RBO * 8;
  const __bf16* Bp[3] = {static_cast<const __bf16*>(a.B_hi) + coff, static_cast<const __bf16*>(a.B_lo) + coff,
                         NP == 3 ? static_cast<const __bf16*>(a.B_p2) + coff : nullptr};
  const __bf16* xq[3] = {static_cast<const __bf16*>(a.xi_hi), static_cast<const __bf16*>(a.xi_lo),
                         static_cast<const __bf16*>(a.xi_p2)};
  const int64_t rb8 = a.Rs / 8;
  const int nb = sp.n0, nst = sp.n1;  // steps of this part
  v4f acc[RBO][2];
#pragma unroll
  for (int rb = 0; rb < RBO; ++rb)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rb][ct] = v4f{0.f, 0.f, 0.f, 0.f};
  const v8bf zero8 = {};
  if (nb >= nst) return;
  // The step's operator (every part, the same for the four waves)
  // staged in LDS one step ahead (double-buffered; each lane's values padded
  // by 16 bytes so that a quarter wave's 16-byte reads spread over the
  // banks).  Loads without branches, masked where used: the table entries
  // three steps ahead, the source boxes two, the xi values one.
  constexpr int LS = RBO * 8 + 8;                  // bf16 values per lane in LDS
  constexpr int U = RBO % 4 == 0 ? 8 : 4;          // staging unit (bf16 values)
  constexpr int PU = 2 * RBO / U;                  // units per thread and part
  typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
  using SV = typename std::conditional<U == 8, v8bf, v4bf>::type;
  __shared__ __attribute__((aligned(16))) __bf16 ops[2][NP][64 * LS];
  // thread t stages values [2 RBO t, 2 RBO (t + 1)) of the step's 8 RBO x 64
  const int st_lane = threadIdx.x / 4, st_off = (threadIdx.x % 4) * 2 * RBO;
  SV sg[NP][PU];
  auto gload = [&](int n) {
    const int64_t o = (int64_t)n * 64 * RBO * 8 + (int64_t)threadIdx.x * 2 * RBO;
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int u = 0; u < PU; ++u) sg[q][u] = *reinterpret_cast<const SV*>(Bp[q] + o + u * U);
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int u = 0; u < PU; ++u) *reinterpret_cast<SV*>(&ops[buf][q][st_lane * LS + st_off + u * U]) = sg[q][u];
  };
  const int sl[2] = {cc.ok[0] ? cc.slot[0] : 0, cc.ok[1] ? cc.slot[1] : 0};
  auto entry = [&](int n) -> int2 {
    const int2 e = info[4 * min(n, nst - 1) + g4];
    return n < nst ? e : make_int2(-1, 0);
  };
  auto src_raw = [&](int2 e, int ct) -> int { return src[max(e.x, 0) * a.TB + sl[ct]]; };
  auto xoff = [&](int sb, int2 e, int ct) -> int64_t {
    return (((int64_t)max(sb, 0) * rb8 + e.y / 8) * a.nvec + cc.v[ct]) * 8;
  };
  // pipeline registers: e1 / e2 = table entries of steps n + 1, n + 2;
  // s1 / sv1 = raw source boxes of step n + 1 and their validity; x0 / xv0 =
  // raw xi parts of step n and their validity
  const int2 e0 = entry(nb);
  int2 e1 = entry(nb + 1), e2 = entry(nb + 2);
  int s1[2];
  bool sv1[2], xv0[2];
  v8bf x0[2][NP];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int s0 = src_raw(e0, ct);
    xv0[ct] = cc.ok[ct] && e0.x >= 0 && s0 >= 0;
    const int64_t o = xoff(xv0[ct] ? s0 : 0, e0, ct);
#pragma unroll
    for (int q = 0; q < NP; ++q) x0[ct][q] = ld8bf(xq[q] + o);
    s1[ct] = src_raw(e1, ct);
    sv1[ct] = cc.ok[ct] && e1.x >= 0;
  }
  int buf = 0;
  gload(nb);
  swrite(0);
  __syncthreads();
  for (int n = nb; n < nst; ++n) {
    // loads of later steps (the padded operator keeps step n + 1 in bounds)
    const int2 e3 = entry(n + 3);
    int s2[2];
    bool sv2[2], xv1[2];
    v8bf x1[2][NP];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      s2[ct] = src_raw(e2, ct);
      sv2[ct] = cc.ok[ct] && e2.x >= 0;
      xv1[ct] = sv1[ct] && s1[ct] >= 0;
      const int64_t o = xoff(xv1[ct] ? s1[ct] : 0, e1, ct);
#pragma unroll
      for (int q = 0; q < NP; ++q) x1[ct][q] = ld8bf(xq[q] + o);
    }
    gload(n + 1);
    // products of step n
    v8bf bq[2][NP];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int q = 0; q < NP; ++q) bq[ct][q] = xv0[ct] ? x0[ct][q] : zero8;
#pragma unroll
    for (int rb = 0; rb < RBO; ++rb) {
      v8bf ap[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) ap[q] = ld8bf(&ops[buf][q][lane * LS] + rb * 8);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) parts_mfma<NP>(acc[rb][ct], ap, bq[ct]);
    }
    // the next step's operator into the other buffer (its last reader
    // passed the previous barrier)
    swrite(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    // roll
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
#pragma unroll
      for (int q = 0; q < NP; ++q) x0[ct][q] = x1[ct][q];
      xv0[ct] = xv1[ct];
      s1[ct] = s2[ct];
      sv1[ct] = sv2[ct];
    }
    e1 = e2;
    e2 = e3;
  }
  const double scale = a.ksplit == 1 ? a.scale : 1.0;
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    if (!cc.ok[ct]) continue;
    const int box = a.tile_box[tile * a.TB + cc.slot[ct]];
    if (box < 0) continue;
    double* dst = stack_dst(a, sp, box, cc.v[ct]);
#pragma unroll
    for (int rb = 0; rb < RBO; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rb * 16 + 4 * g4 + i;
        if (row < a.k) dst[row] = scale * (double)acc[rb][ct][i];
      }
  }
}

// q~ (FP64, [box][v][k]) -> padded [box][v][kp] bf16 parts: high and low
// (p2 null), or three parts x0, x1, x2
__global__ void pad_split_kernel(const double* __restrict__ in, int k, int64_t ncols, int kp,
                                 __bf16* __restrict__ hi, __bf16* __restrict__ lo, __bf16* __restrict__ p2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= ncols * kp) return;
  const int64_t col = i / kp;
  const int r = (int)(i - col * kp);
  const float x = r < k ? (float)in[col * k + r] : 0.f;
  const __bf16 h = (__bf16)x;
  const float r1 = x - (float)h;
  const __bf16 l = (__bf16)r1;
  hi[i] = h;
  lo[i] = l;
  if (p2) p2[i] = (__bf16)(r1 - (float)l);
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

hipError_t launch_blas_stacked(const BlasStack& a, hipStream_t stream) {
  if (a.ntiles == 0) return hipSuccess;
  const bool parts = a.mode >= 2;  // BF16 parts: 2 (BF16x3) or 3 (BF16x6)
  if (a.C > 128 || a.Rpad % 128 != 0 || a.Rs > a.Rpad || a.kp % (parts ? 32 : 16) != 0 ||
      a.rbo * 16 < a.kp || a.kp < a.k || a.Rs % (parts ? 8 : 4) != 0 || a.mode > 3 ||
      (a.mode == 3 && (!a.A_p2 || !a.B_p2 || !a.q_p2 || !a.xi_p2)))
    return hipErrorInvalidValue;
  if (a.ksplit < 1 || (a.ksplit > 1 && !a.partial)) return hipErrorInvalidValue;
  const int64_t nb_items = a.ntiles * a.ksplit;
  const dim3 grid_b((unsigned)(8 * ((nb_items + 7) / 8)));
  // Stage A: up to five row blocks per workgroup (FP64: one) where the grid
  // stays above 16,384 workgroups
  const int nmb = a.Rpad / 128;
  int rpw = 1;
  for (int r = a.mode == 0 ? 1 : 5; r > 1; --r)
    if (a.ntiles * ((nmb + r - 1) / r) >= 16384) {
      rpw = r;
      break;
    }
  const int64_t nwork_a = a.ntiles * ((nmb + rpw - 1) / rpw);
  const dim3 grid_a((unsigned)(8 * ((nwork_a + 7) / 8)));
  const dim3 block(256);
  if (a.mode == 0) stack_a_kernel<double><<<grid_a, block, 0, stream>>>(a, rpw);
  else if (a.mode == 1) stack_a_kernel<float><<<grid_a, block, 0, stream>>>(a, rpw);
  else if (a.mode == 2) stack_a_bf16_kernel<2><<<grid_a, block, 0, stream>>>(a, rpw);
  else stack_a_bf16_kernel<3><<<grid_a, block, 0, stream>>>(a, rpw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define KIFMM_STACK_B(RR)                                                        \
  if (a.mode == 0) stack_b_kernel<double, RR><<<grid_b, block, 0, stream>>>(a);  \
  else if (a.mode == 1) stack_b_kernel<float, RR><<<grid_b, block, 0, stream>>>(a); \
  else if (a.mode == 2) stack_b_bf16_kernel<RR, 2><<<grid_b, block, 0, stream>>>(a); \
  else stack_b_bf16_kernel<RR, 3><<<grid_b, block, 0, stream>>>(a);
  switch (a.rbo) {
    case 2: KIFMM_STACK_B(2) break;
    case 4: KIFMM_STACK_B(4) break;
    case 6: KIFMM_STACK_B(6) break;
    case 8: KIFMM_STACK_B(8) break;
    case 10: KIFMM_STACK_B(10) break;
    default: return hipErrorInvalidValue;
  }
#undef KIFMM_STACK_B
  if (a.ksplit > 1) {
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = a.n_boxes * a.nvec * a.k;
    stack_reduce_kernel<<<(unsigned)((total + 255) / 256), 256, 0, stream>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_pad_split(const double* in, int k, int64_t ncols, int kp, void* hi, void* lo, void* p2,
                            hipStream_t stream) {
  const int64_t n = ncols * kp;
  if (n == 0) return hipSuccess;
  pad_split_kernel<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(in, k, ncols, kp, (__bf16*)hi,
                                                                    (__bf16*)lo, (__bf16*)p2);
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
