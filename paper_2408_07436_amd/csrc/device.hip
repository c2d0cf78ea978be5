// Device state and the evaluate pipeline of the kiFMM (Section 2: upward
// pass P2M + M2M, downward pass M2L + L2L per level, then L2P + P2P).
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "internal.h"
#include "kernels.h"

namespace kifmm {

struct DevLevel {
  int64_t n = 0;
  double w = 1.0;               // box width
  int32_t* child = nullptr;     // [n][8]
  int32_t* halo = nullptr;      // [26][n_{l-1}]
  // FFT-M2L work buffers of this level (levels run concurrently): spectra
  // of the n_{l-1} + 1 clusters, their products, and the check potentials
  void* Qhat = nullptr;
  void* Phat = nullptr;
  double* chk = nullptr;
  // FFT-M2L source blocks: the clusters of one aligned 4 x 4 x 4 cube of
  // level l-1 (consecutive in Morton order) share one list of the at most
  // 216 source clusters of the cube's 6 x 6 x 6 shell, each at the slot of
  // its shell position; tbase[c] is (slot(c) - kHadSlotBias) * kHadRowBytes
  int64_t hb_n = 0;
  int32_t* hb_tgt = nullptr;    // [hb_n + 1] first cluster of each block
  int32_t* hb_src = nullptr;    // [hb_n + 1] offsets into hb_list
  int32_t* hb_list = nullptr;   // cluster << 8 | slot (the empty cluster n_{l-1} included);
                                // entry 0 is the empty cluster at slot 255
  int32_t* hb_tbase = nullptr;  // [n_{l-1}] LDS byte offset of the cluster's own slot, biased
  // BLAS / dense M2L: target tiles of one octant class and, per tile, the
  // transfer vectors present with the source box of every tile slot
  int64_t ntiles = 0;
  int32_t* tile_box = nullptr;
  int64_t* tl_offs = nullptr;
  int32_t* tl_t = nullptr;
  int32_t* tl_src = nullptr;
  // stacked form: octant class of each tile and the source box of every
  // (transfer vector j of the class, tile slot), -1 where absent
  int32_t* tile_class = nullptr;
  int32_t* tile_src = nullptr;
  // a tree built on the device (moving points): keys, parents and the
  // interaction lists of the level (host layout of Level)
  uint64_t* keys = nullptr;
  int32_t* parent = nullptr;
  int64_t* il_offs = nullptr;
  int32_t* il_src = nullptr;
  int16_t* il_t = nullptr;
};

struct DeviceState {
  int device = 0;
  bool fp64 = true;
  std::vector<void*> allocs;
  // points and leaves
  double* src_xyz = nullptr;
  double* tgt_xyz = nullptr;
  int64_t* src_perm = nullptr;
  // keys of the leaves (compared with the leaves of moved points)
  uint64_t* leaf_keys = nullptr;
  int64_t* tgt_perm = nullptr;
  // device tree build: scratch, totals, lookup tables (transfer index over
  // (t + 3) in base 7, the 316 vectors as int8 triples, the stacked form's
  // class slot of each transfer vector); tree_dev once the levels, lists
  // and maps of the handle were built on the device
  void* tree_scratch = nullptr;
  size_t tree_scratch_bytes = 0;
  int64_t* tree_totals = nullptr;  // [64]
  int64_t* tree_part = nullptr;    // [kTreeScanPart] prefix-sum partials
  int16_t* tmap = nullptr;
  int8_t* tvec = nullptr;
  int32_t* jof = nullptr;
  bool tree_dev = false;
  int32_t *src_start = nullptr, *src_end = nullptr, *tgt_start = nullptr, *tgt_end = nullptr;
  int64_t* near_offs = nullptr;
  int32_t* near_src = nullptr;
  double* leaf_centers = nullptr;
  // operators
  double* surf = nullptr;    // [ns][3] equivalent-surface offsets
  double* surf_c = nullptr;  // [nc][3] check-surface offsets
  int16_t* lat2surf = nullptr;
  int16_t* surf_lat = nullptr;
  double *up_V = nullptr, *up_Ut = nullptr, *down_V = nullptr, *down_Ut = nullptr;
  double *m2m = nullptr, *l2l = nullptr;
  // composite operators of the reduced-precision modes (one GEMM per
  // pseudo-inverse, pseudo-inverses folded into M2M / L2L)
  double *up_P = nullptr, *down_P = nullptr, *m2m_c = nullptr, *l2l_c = nullptr;
  void* khat = nullptr;
  void* khat_split = nullptr;  // FP32: BF16 parts of khat for the split Hadamard
  void* twiddle = nullptr;
  double* Ublas = nullptr;   // nc x k: decompression
  double* SblasT = nullptr;  // k x ns: compression
  // packed per-t M2L operators of the fused kernel (see pack_blas_operators)
  int blas_mode = 0, kp = 0;
  bool two_stage = false;
  int64_t* op_off = nullptr;
  int32_t* ktp = nullptr;
  int ktp_max = 0;
  int32_t* ktq = nullptr;
  void* op_hi = nullptr;
  void* op_lo = nullptr;
  int tile_tb = 0;            // target boxes per tile of the current tiles
  void* qpad = nullptr;       // padded compressed multipoles
  // stacked two-stage form (BlasStack in kernels.h): operators of Stage A
  // and B, the row-group table, the per-class slot j of each transfer vector
  bool stack_ok = false;
  int st_Rs = 0, st_Rpad = 0, st_nsteps = 0, st_rbo = 0, st_J = 0;
  void *st_A_hi = nullptr, *st_A_lo = nullptr, *st_B_hi = nullptr, *st_B_lo = nullptr;
  void *st_A_p2 = nullptr, *st_B_p2 = nullptr;  // BF16x6: third parts
  int32_t* st_info = nullptr;
  std::vector<int32_t> st_jof;  // [8][316]
  void *xi_hi = nullptr, *xi_lo = nullptr, *xi_p2 = nullptr;  // work: stacked intermediates
  std::vector<DevLevel> lv;
  // work buffers
  int nvec_cap = 0;
  void* qs = nullptr;
  std::vector<double*> mult, local;
  double* phi = nullptr;
  double* tmp = nullptr;
  double* tmp2 = nullptr;
  double* gemm_ws = nullptr;  // split-K partials
  void* nearbuf = nullptr;    // near-field sums in sorted target order (split leaf passes)
  int64_t gemm_ws_elems = 0;
  // FFT-M2L evaluates run as a dependency graph: the leaf level's M2L on
  // the evaluate stream, the coarse levels' M2M and downward work on a
  // coarse stream, and each coarse level's M2L on a side stream
  hipStream_t coarse = nullptr;
  std::vector<hipStream_t> side;    // [depth + 1]: M2L of coarse level l
  hipEvent_t fork_ev = nullptr;     // leaf multipoles ready
  hipEvent_t down_ev = nullptr;     // coarse locals ready
  // the near field runs on its own stream from the sorted charges on
  hipStream_t nearst = nullptr;
  hipEvent_t near_fork_ev = nullptr;  // sorted charges ready
  hipEvent_t near_ev = nullptr;       // near-field sums stored
  std::vector<hipEvent_t> up_ev;    // [depth + 1] multipoles of coarse level l ready
  std::vector<hipEvent_t> join_ev;  // [depth + 1] M2L of coarse level l done
  std::vector<void*> work_allocs;
  hipEvent_t ev[8] = {};
  std::vector<hipEvent_t> lev_ev;  // [level][4] marks around the M2L kernels
  bool events = false;
  // key of the shared FFT-M2L kernel spectra and twiddles (khat, twiddle)
  // when this handle holds a reference to them
  bool fft_shared = false;
  std::tuple<int, int, int, uint64_t> fft_key{};
  // set while a batch records this handle's serial schedule (nothing is
  // enqueued then; see LaunchSink)
  LaunchSink* sink = nullptr;
};

namespace {

template <typename T>
kifmm_status dalloc(DeviceState* d, T** p, size_t count, bool work = false) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return fail(KIFMM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  (work ? d->work_allocs : d->allocs).push_back(*p);
  return KIFMM_OK;
}

// free one allocation of d->allocs (null is ignored) and clear the pointer
template <typename T>
void dfree(DeviceState* d, T** p) {
  if (!*p) return;
  (void)hipFree((void*)*p);
  d->allocs.erase(std::remove(d->allocs.begin(), d->allocs.end(), (void*)*p), d->allocs.end());
  *p = nullptr;
}

template <typename T>
kifmm_status upload(DeviceState* d, T** p, const T* host, size_t count) {
  kifmm_status st = dalloc(d, p, count);
  if (st != KIFMM_OK) return st;
  if (count) KIFMM_HIP(hipMemcpy(*p, host, count * sizeof(T), hipMemcpyHostToDevice));
  return KIFMM_OK;
}

#define KIFMM_TRY(expr)                     \
  do {                                      \
    kifmm_status s_ = (expr);               \
    if (s_ != KIFMM_OK) return s_;          \
  } while (0)

#define KIFMM_LAUNCH(expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(KIFMM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// round-to-nearest-even bf16 bits of a float
uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

// The stacked BLAS form runs when its operators exist and the knob asks for
// it; BF16x6 has no fused form, so it always runs stacked.
bool use_stacked(const kifmm_handle* h, const DeviceState* d) {
  return d->stack_ok && (h->tune[KIFMM_TUNE_BLAS_FORM] == 0 || d->blas_mode == 3);
}

// Position of column c of a second-product operator in its packed row, per
// mode: FP32 keeps the order; FP64 accumulator rows are g + 4 s, so a lane's
// four K values (c = 16 j + g + 4 s) are packed at 16 j + 4 g + s; bf16 steps
// of 32 take Xi rows 16 h + 4 g + i of blocks (2 j, 2 j + 1), packed at
// 32 j + 8 g + 4 h + i.
int packed_col(int mode, int c) {
  if (mode == 0) {
    const int j = c / 16, r = c % 16, g = r % 4, s = r / 4;
    return 16 * j + 4 * g + s;
  }
  if (mode == 2) {
    const int j = c / 32, r = c % 32, h = r / 16, g = (r % 16) / 4, i = r % 4;
    return 32 * j + 8 * g + 4 * h + i;
  }
  return c;
}

// Row of Xi (the first product's output) that holds row r of Vbar'_t^T in
// the FP32 mode: row r goes to second-product K step q = r / 4, whose four K
// values are Xi rows 16 (q / 4) + 4 g + q % 4 (g = r % 4), so the steps past
// ceil(k_t / 4) hold only zero rows and are skipped.  (Measured: FP32 5%
// faster; FP64, with fewer waves to hide latency, 3% slower - kept in order.)
int xi_row(int mode, int r) {
  if (mode != 1) return r;
  const int q = r / 4, g = r % 4;
  return 16 * (q / 4) + 4 * g + q % 4;
}

// Operators of the fused BLAS / dense M2L kernel, per t, unit box:
//   two-stage: Vbar'_t^T (ktp x kp) then Ubar_t (kp x ktp, packed columns)
//   single:    C_t (kp x kp)
// ktp = k_t and kp = k rounded up to 16 (FP32 / FP64) or 32 (bf16).
kifmm_status pack_blas_operators(kifmm_handle* h, DeviceState* d) {
  const Operators& op = h->op;
  const int mode = h->cfg.prec == KIFMM_FP64 ? 0 : h->cfg.prec == KIFMM_FP32 ? 1
                   : h->cfg.prec == KIFMM_BF16X3 ? 2 : 3;
  // BF16x6 runs the stacked form only (three-part operands of Stage A / B)
  if (mode == 3 && !op.recompressed)
    return fail(KIFMM_EUNSUPPORTED, "BF16x6 needs directional recompression (the stacked BLAS form)");
  const int q = mode >= 2 ? 32 : 16;
  const int k = op.k;
  const int kp = (k + q - 1) / q * q;
  if (kp > 160) return fail(KIFMM_EUNSUPPORTED, "compressed rank above 160 is not supported");
  d->blas_mode = mode;
  d->kp = kp;
  d->two_stage = op.recompressed;
  std::vector<int64_t> off(kNumTransfer);
  std::vector<int32_t> ktp(kNumTransfer, 0), ktq(kNumTransfer, 0);
  std::vector<double> packed;
  for (int t = 0; t < kNumTransfer; ++t) {
    off[t] = (int64_t)packed.size();
    if (!op.recompressed) {
      std::vector<double> C((size_t)kp * kp, 0.0);
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) C[(size_t)i * kp + j] = op.Vbarp[t][(size_t)i * k + j];
      packed.insert(packed.end(), C.begin(), C.end());
      continue;
    }
    const int kt = op.kt[t];
    const int tp = (kt + q - 1) / q * q;
    if (mode != 3 && tp > (mode == 2 ? 64 : 48))
      return fail(KIFMM_EUNSUPPORTED, "directional rank above the fused kernel's limit");
    ktp[t] = tp;
    ktq[t] = mode == 1 ? (kt + 3) / 4 : tp / 4;
    std::vector<double> V((size_t)tp * kp, 0.0), Ub((size_t)kp * tp, 0.0);
    for (int r = 0; r < kt; ++r) {
      const int xr = xi_row(mode, r);
      for (int c = 0; c < k; ++c) V[(size_t)xr * kp + c] = op.Vbarp[t][(size_t)c * kt + r];
    }
    for (int r = 0; r < k; ++r)
      for (int c = 0; c < kt; ++c) {
        const int xc = xi_row(mode, c);
        Ub[(size_t)r * tp + packed_col(mode, xc)] = op.Ubar[t][(size_t)r * kt + c];
      }
    packed.insert(packed.end(), V.begin(), V.end());
    packed.insert(packed.end(), Ub.begin(), Ub.end());
  }
  KIFMM_TRY(upload(d, &d->op_off, off.data(), off.size()));
  KIFMM_TRY(upload(d, &d->ktp, ktp.data(), ktp.size()));
  KIFMM_TRY(upload(d, &d->ktq, ktq.data(), ktq.size()));
  d->ktp_max = *std::max_element(ktp.begin(), ktp.end());
  if (mode == 0) {
    double* p;
    KIFMM_TRY(upload(d, &p, packed.data(), packed.size()));
    d->op_hi = p;
  } else if (mode == 1) {
    std::vector<float> f(packed.begin(), packed.end());
    float* p;
    KIFMM_TRY(upload(d, &p, f.data(), f.size()));
    d->op_hi = p;
  } else if (mode == 3) {
    d->op_hi = d->op_lo = nullptr;  // no fused form in BF16x6
  } else {
    std::vector<uint16_t> hi(packed.size()), lo(packed.size());
    for (size_t i = 0; i < packed.size(); ++i) {
      const float x = (float)packed[i];
      hi[i] = bf16_bits(x);
      lo[i] = bf16_bits(x - bf16_value(hi[i]));
    }
    uint16_t *ph, *pl;
    KIFMM_TRY(upload(d, &ph, hi.data(), hi.size()));
    KIFMM_TRY(upload(d, &pl, lo.data(), lo.size()));
    d->op_hi = ph;
    d->op_lo = pl;
  }
  return KIFMM_OK;
}

// Operators of the stacked two-stage form.  Target class o (key & 7) takes
// the transfer vectors T(o) (ascending index; t_x = -3 only for odd x, +3
// only for even x, likewise y and z); a source of class c serves T(c ^ 7),
// and the source of target class o along t has class o ^ (t mod 2).  Each
// t's k_t rows are padded to P = 4 (BF16x3: 8) rows.
//   Stage A operators [8][Rpad][kp]: class c's rows are Vbar'_t^T for t in
//     T(c ^ 7), stacked; Rs = rows per class (all classes alike).
//   Stage B operators, class o, K = the stacked rows of T(o): FP32 / FP64
//     [8][nsteps][64 lanes][rbo] with lane (g, l) of step n holding
//     Ubar(row 16 rb + l, K 4 n + g); BF16x3 [8][nsteps][64][rbo][8] holding
//     K 32 n + 8 g + e, split into bf16 high and low parts.
//   info [8][groups][2]: per group of 4 (BF16x3: 8) K rows, the class slot j
//     of its transfer vector and the xi row of its first row (-1: padding).
kifmm_status pack_blas_stacked(kifmm_handle* h, DeviceState* d) {
  const Operators& op = h->op;
  const int mode = d->blas_mode, k = op.k, kp = d->kp;
  const int P = mode >= 2 ? 8 : 4, KS = mode >= 2 ? 32 : 4, G = mode >= 2 ? 8 : 4;
  const int rbo = (kp / 16 + 1) / 2 * 2;
  auto admissible = [](int o, const int t[3]) {
    for (int ax = 0; ax < 3; ++ax) {
      const int b = (o >> ax) & 1;
      if ((b == 0 && t[ax] == -3) || (b == 1 && t[ax] == 3)) return false;
    }
    return true;
  };
  auto parity = [](int it) {
    int t[3];
    transfer_vector(it, t);
    return (t[0] & 1) | ((t[1] & 1) << 1) | ((t[2] & 1) << 2);
  };
  std::vector<std::vector<int>> Tt(8);
  for (int o = 0; o < 8; ++o)
    for (int it = 0; it < kNumTransfer; ++it) {
      int t[3];
      transfer_vector(it, t);
      if (admissible(o, t)) Tt[o].push_back(it);
    }
  const int J = (int)Tt[0].size();
  for (int o = 1; o < 8; ++o)
    if ((int)Tt[o].size() != J) return fail(KIFMM_ENUMERIC, "octant classes with different transfer-vector counts");
  auto seg = [&](int it) { return (op.kt[it] + P - 1) / P * P; };
  std::vector<int> srcoff((size_t)8 * kNumTransfer, -1), tgtoff((size_t)8 * kNumTransfer, -1);
  std::vector<int> Rt(8, 0);
  int Rs = 0;
  for (int c = 0; c < 8; ++c) {
    int off = 0;
    for (int it : Tt[c ^ 7]) {
      srcoff[(size_t)c * kNumTransfer + it] = off;
      off += seg(it);
    }
    Rs = std::max(Rs, off);
    off = 0;
    for (int it : Tt[c]) {
      tgtoff[(size_t)c * kNumTransfer + it] = off;
      off += seg(it);
    }
    Rt[c] = off;
  }
  const int Rpad = (Rs + 127) / 128 * 128;
  const int Rtmax = *std::max_element(Rt.begin(), Rt.end());
  const int nsteps = (Rtmax + KS - 1) / KS;
  const int ngroups = nsteps * KS / G;
  // row r of class o's stacked K -> (transfer vector, row within its k_t), or -1
  std::vector<int32_t> rt_it((size_t)8 * nsteps * KS, -1), rt_i((size_t)8 * nsteps * KS, 0);
  std::vector<int32_t> info((size_t)8 * ngroups * 2, 0);
  d->st_jof.assign((size_t)8 * kNumTransfer, -1);
  for (int o = 0; o < 8; ++o) {
    for (int j = 0; j < J; ++j) {
      const int it = Tt[o][j];
      d->st_jof[(size_t)o * kNumTransfer + it] = j;
      const int r0 = tgtoff[(size_t)o * kNumTransfer + it];
      for (int i = 0; i < seg(it); ++i) {
        rt_it[(size_t)o * nsteps * KS + r0 + i] = it;
        rt_i[(size_t)o * nsteps * KS + r0 + i] = i;
      }
    }
    for (int n = 0; n < ngroups; ++n) {
      const int r = n * G;
      const int it = rt_it[(size_t)o * nsteps * KS + r];
      int32_t* e = &info[((size_t)o * ngroups + n) * 2];
      if (it < 0) {
        e[0] = -1;
        e[1] = 0;
        continue;
      }
      const int c = o ^ parity(it);
      e[0] = d->st_jof[(size_t)o * kNumTransfer + it];
      e[1] = srcoff[(size_t)c * kNumTransfer + it] + rt_i[(size_t)o * nsteps * KS + r];
    }
  }
  std::vector<double> A((size_t)8 * Rpad * kp, 0.0);
  for (int c = 0; c < 8; ++c)
    for (int it : Tt[c ^ 7]) {
      const int kt = op.kt[it], r0 = srcoff[(size_t)c * kNumTransfer + it];
      for (int i = 0; i < kt; ++i)
        for (int cc = 0; cc < k; ++cc)
          A[((size_t)c * Rpad + r0 + i) * kp + cc] = op.Vbarp[it][(size_t)cc * kt + i];
    }
  auto ubar = [&](int o, int m, int r) -> double {
    if (m >= k || r >= nsteps * KS) return 0.0;
    const int it = rt_it[(size_t)o * nsteps * KS + r];
    if (it < 0) return 0.0;
    const int kt = op.kt[it], i = rt_i[(size_t)o * nsteps * KS + r];
    return i < kt ? op.Ubar[it][(size_t)m * kt + i] : 0.0;
  };
  const int per = mode >= 2 ? 8 : 1;  // values per (lane, row block)
  // (plus 2 kStackChunk zero steps past the last class: Stage B stages the
  // operator one chunk ahead, so a part's last chunk reads up to two chunks
  // past its last step)
  std::vector<double> B(((size_t)8 * nsteps + 2 * kStackChunk) * 64 * rbo * per, 0.0);
  for (int o = 0; o < 8; ++o)
    for (int n = 0; n < nsteps; ++n)
      for (int lane = 0; lane < 64; ++lane)
        for (int rb = 0; rb < rbo; ++rb)
          for (int e = 0; e < per; ++e) {
            const int m = rb * 16 + lane % 16;
            const int r = mode >= 2 ? 32 * n + 8 * (lane / 16) + e : 4 * n + lane / 16;
            B[((((size_t)o * nsteps + n) * 64 + lane) * rbo + rb) * per + e] = ubar(o, m, r);
          }
  auto put = [&](const std::vector<double>& v, void** hi, void** lo, void** p2) -> kifmm_status {
    if (mode == 0) {
      double* p;
      KIFMM_TRY(upload(d, &p, v.data(), v.size()));
      *hi = p;
    } else if (mode == 1) {
      std::vector<float> f(v.begin(), v.end());
      float* p;
      KIFMM_TRY(upload(d, &p, f.data(), f.size()));
      *hi = p;
    } else {
      // BF16 parts: x0 = bf16(x), x1 = bf16(x - x0) (and x2 = bf16(x - x0 - x1))
      std::vector<uint16_t> vh(v.size()), vl(v.size()), v2(mode == 3 ? v.size() : 0);
      for (size_t i = 0; i < v.size(); ++i) {
        const float x = (float)v[i];
        vh[i] = bf16_bits(x);
        const float r1 = x - bf16_value(vh[i]);
        vl[i] = bf16_bits(r1);
        if (mode == 3) v2[i] = bf16_bits(r1 - bf16_value(vl[i]));
      }
      uint16_t *ph, *pl;
      KIFMM_TRY(upload(d, &ph, vh.data(), vh.size()));
      KIFMM_TRY(upload(d, &pl, vl.data(), vl.size()));
      *hi = ph;
      *lo = pl;
      if (mode == 3) {
        uint16_t* p3;
        KIFMM_TRY(upload(d, &p3, v2.data(), v2.size()));
        *p2 = p3;
      }
    }
    return KIFMM_OK;
  };
  KIFMM_TRY(put(A, &d->st_A_hi, &d->st_A_lo, &d->st_A_p2));
  KIFMM_TRY(put(B, &d->st_B_hi, &d->st_B_lo, &d->st_B_p2));
  KIFMM_TRY(upload(d, &d->st_info, info.data(), info.size()));
  d->st_Rs = Rs;
  d->st_Rpad = Rpad;
  d->st_nsteps = nsteps;
  d->st_rbo = rbo;
  d->st_J = J;
  d->stack_ok = true;
  return KIFMM_OK;
}

// Target tiles of TB boxes of one octant class per level (boxes of a class
// share their transfer vectors) and, per tile, the transfer vectors present
// in ascending order with the source box of each slot.
kifmm_status build_blas_tiles_host(kifmm_handle* h, DeviceState* d, int TB) {
  const Tree& t = h->tree;
  for (int l = 2; l <= t.depth; ++l) {
    const Level& L = t.levels[l];
    DevLevel& D = d->lv[l];
    for (void* p : {(void*)D.tile_box, (void*)D.tl_offs, (void*)D.tl_t, (void*)D.tl_src,
                    (void*)D.tile_class, (void*)D.tile_src}) {
      if (!p) continue;
      (void)hipFree(p);
      d->allocs.erase(std::remove(d->allocs.begin(), d->allocs.end(), p), d->allocs.end());
    }
    std::vector<int32_t> tile_box, tl_t, tl_src, tile_class, tile_src;
    std::vector<int64_t> tl_offs(1, 0);
    const int J = d->st_J;
    std::vector<int32_t> map((size_t)TB * kNumTransfer, -1);
    for (int o = 0; o < 8; ++o) {
      std::vector<int32_t> boxes;
      for (int64_t i = 0; i < L.n; ++i)
        if ((int)(L.keys[i] & 7) == o) boxes.push_back((int32_t)i);
      for (size_t b0 = 0; b0 < boxes.size(); b0 += TB) {
        const size_t nb = std::min<size_t>(TB, boxes.size() - b0);
        for (size_t sl = 0; sl < (size_t)TB; ++sl) tile_box.push_back(sl < nb ? boxes[b0 + sl] : -1);
        tile_class.push_back(o);
        if (d->stack_ok) tile_src.resize(tile_src.size() + (size_t)J * TB, -1);
        for (size_t sl = 0; sl < nb; ++sl) {
          const int32_t bx = boxes[b0 + sl];
          for (int64_t e = L.il_offs[bx]; e < L.il_offs[bx + 1]; ++e) {
            map[(size_t)sl * kNumTransfer + L.il_t[e]] = L.il_src[e];
            if (d->stack_ok) {
              const int j = d->st_jof[(size_t)o * kNumTransfer + L.il_t[e]];
              if (j < 0) return fail(KIFMM_ENUMERIC, "interaction outside the octant class's transfer vectors");
              tile_src[tile_src.size() - (size_t)J * TB + (size_t)j * TB + sl] = L.il_src[e];
            }
          }
        }
        for (int tt = 0; tt < kNumTransfer; ++tt) {
          bool any = false;
          for (size_t sl = 0; sl < nb; ++sl) any |= map[(size_t)sl * kNumTransfer + tt] >= 0;
          if (!any) continue;
          tl_t.push_back(tt);
          for (size_t sl = 0; sl < (size_t)TB; ++sl) {
            int32_t& m = map[sl * kNumTransfer + tt];
            tl_src.push_back(sl < nb ? m : -1);
            m = -1;
          }
        }
        tl_offs.push_back((int64_t)tl_t.size());
      }
    }
    D.ntiles = (int64_t)tl_offs.size() - 1;
    KIFMM_TRY(upload(d, &D.tile_box, tile_box.data(), tile_box.size()));
    KIFMM_TRY(upload(d, &D.tl_offs, tl_offs.data(), tl_offs.size()));
    KIFMM_TRY(upload(d, &D.tl_t, tl_t.data(), tl_t.size()));
    KIFMM_TRY(upload(d, &D.tl_src, tl_src.data(), tl_src.size()));
    KIFMM_TRY(upload(d, &D.tile_class, tile_class.data(), tile_class.size()));
    if (d->stack_ok) KIFMM_TRY(upload(d, &D.tile_src, tile_src.data(), tile_src.size()));
  }
  d->tile_tb = TB;
  return KIFMM_OK;
}

// Lookup tables of the device tree build (once per device state).
kifmm_status tree_tables(DeviceState* d) {
  if (d->tmap) return KIFMM_OK;
  std::vector<int16_t> tm(343, -1);
  std::vector<int8_t> tv(3 * kNumTransfer);
  for (int it = 0; it < kNumTransfer; ++it) {
    int t[3];
    transfer_vector(it, t);
    tm[(t[0] + 3) * 49 + (t[1] + 3) * 7 + (t[2] + 3)] = (int16_t)it;
    for (int k = 0; k < 3; ++k) tv[3 * it + k] = (int8_t)t[k];
  }
  KIFMM_TRY(upload(d, &d->tmap, tm.data(), tm.size()));
  KIFMM_TRY(upload(d, &d->tvec, tv.data(), tv.size()));
  if (d->stack_ok) KIFMM_TRY(upload(d, &d->jof, d->st_jof.data(), d->st_jof.size()));
  KIFMM_TRY(dalloc(d, &d->tree_totals, 64));
  KIFMM_TRY(dalloc(d, &d->tree_part, kTreeScanPart));
  return KIFMM_OK;
}

// The same tiles from a tree built on the device (keys of every level on
// the device): boxes in stable octant-class order, TB per tile, and per tile
// the transfer vectors whose source box exists for some slot.
kifmm_status build_blas_tiles_device(kifmm_handle* h, DeviceState* d, int TB) {
  const Tree& t = h->tree;
  KIFMM_TRY(tree_tables(d));
  const hipStream_t s = nullptr;
  for (int l = 2; l <= t.depth; ++l) {
    DevLevel& D = d->lv[l];
    dfree(d, &D.tile_box);
    dfree(d, &D.tl_offs);
    dfree(d, &D.tl_t);
    dfree(d, &D.tl_src);
    dfree(d, &D.tile_class);
    dfree(d, &D.tile_src);
    D.ntiles = 0;
    const int64_t n = D.n;
    int32_t *scr = nullptr, *order = nullptr;
    int64_t* present = nullptr;
    auto release = [&] {
      dfree(d, &scr);
      dfree(d, &order);
      dfree(d, &present);
    };
    kifmm_status st = dalloc(d, &scr, tree_classes_scratch_ints(n) + 8);
    if (st == KIFMM_OK) st = dalloc(d, &order, (size_t)n);
    if (st != KIFMM_OK) {
      release();
      return st;
    }
    int32_t* counts = scr + tree_classes_scratch_ints(n);
    int32_t cls[8];
    hipError_t e = tree_classes(D.keys, n, scr, order, counts, d->tree_part, s);
    if (e == hipSuccess) e = hipMemcpy(cls, counts, sizeof cls, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      release();
      return fail(KIFMM_EDEVICE, std::string("tile classes: ") + hipGetErrorString(e));
    }
    TileClasses tc;
    int32_t run = 0;
    int64_t tiles = 0;
    for (int o = 0; o < 8; ++o) {
      tc.start[o] = run;
      tc.count[o] = cls[o];
      tc.first_tile[o] = tiles;
      run += cls[o];
      tiles += (cls[o] + TB - 1) / TB;
    }
    tc.first_tile[8] = tiles;
    st = dalloc(d, &D.tile_box, (size_t)tiles * TB);
    if (st == KIFMM_OK) st = dalloc(d, &D.tile_class, (size_t)tiles);
    if (st == KIFMM_OK) st = dalloc(d, &D.tl_offs, (size_t)tiles + 1);
    if (st == KIFMM_OK) st = dalloc(d, &present, (size_t)tiles * kNumTransfer + 1);
    if (st != KIFMM_OK) {
      release();
      return st;
    }
    int64_t total = 0;
    e = tree_tiles(D.keys, n, l, order, tc, TB, tiles, d->tvec, D.tile_box, D.tile_class, present,
                   d->tree_totals, d->tree_part, s);
    if (e == hipSuccess) e = hipMemcpy(&total, d->tree_totals, sizeof total, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      release();
      return fail(KIFMM_EDEVICE, std::string("tiles: ") + hipGetErrorString(e));
    }
    st = dalloc(d, &D.tl_t, (size_t)total);
    if (st == KIFMM_OK) st = dalloc(d, &D.tl_src, (size_t)total * TB);
    if (st == KIFMM_OK && d->stack_ok) st = dalloc(d, &D.tile_src, (size_t)tiles * d->st_J * TB);
    if (st != KIFMM_OK) {
      release();
      return st;
    }
    e = tree_tiles_fill(D.keys, n, l, D.tile_box, D.tile_class, tiles, TB, d->tvec, present, D.tl_t,
                        D.tl_src, D.tl_offs, d->jof, d->st_J, d->stack_ok ? D.tile_src : nullptr, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    release();
    if (e != hipSuccess) return fail(KIFMM_EDEVICE, std::string("tile lists: ") + hipGetErrorString(e));
    D.ntiles = tiles;
  }
  d->tile_tb = TB;
  return KIFMM_OK;
}

kifmm_status build_blas_tiles(kifmm_handle* h, DeviceState* d, int TB) {
  return d->tree_dev ? build_blas_tiles_device(h, d, TB) : build_blas_tiles_host(h, d, TB);
}

// Source blocks of one FFT-M2L level (see DevLevel): clusters grouped by
// Morton key >> 6 (aligned 4 x 4 x 4 cubes).  A block's sources sit at fixed
// slots, their positions in the 6 x 6 x 6 shell around the cube
// (slot = x + 6 y + 36 z, shell coordinates 0..5), so the cluster in
// direction D of a member at slot s is at slot s + D_x + 6 D_y + 36 D_z and
// the kernel needs one base offset per member, not a table per direction.
// The list names every slot some member's halo reaches, with the empty
// cluster (index nc, zero spectra) where no cluster is present.
static kifmm_status build_source_blocks(DeviceState* d, DevLevel& D, const Level& up,
                                        const std::vector<int32_t>& halo) {
  const int64_t nc = up.n;
  std::vector<int32_t> tgt, src, list, tbase((size_t)nc, 0);
  int doff[kNumDirections];
  for (int dd = 0; dd < kNumDirections; ++dd) {
    int v[3];
    direction_vector(dd, v);
    doff[dd] = v[0] + kHadShell * v[1] + kHadShell * kHadShell * v[2];
  }
  std::vector<int32_t> at(kHadSrcSlots);
  // entry 0: the empty cluster at slot 255, taken by staging lanes past a
  // block's list (their LDS writes land in a discard area)
  list.push_back((int32_t)((uint32_t)nc << 8 | 255u));
  int64_t c = 0;
  while (c < nc) {
    const uint64_t bk = up.keys[c] >> 6;
    int64_t e = c;
    while (e < nc && (up.keys[e] >> 6) == bk) ++e;
    std::fill(at.begin(), at.end(), -1);
    const int32_t* a0 = &up.anchor[3 * (size_t)c];
    for (int64_t i = c; i < e; ++i) {
      const int32_t* an = &up.anchor[3 * (size_t)i];
      if ((an[0] >> 2) != (a0[0] >> 2) || (an[1] >> 2) != (a0[1] >> 2) || (an[2] >> 2) != (a0[2] >> 2))
        return fail(KIFMM_ENUMERIC, "FFT-M2L source block is not an aligned 4 x 4 x 4 cube");
      const int own = ((an[0] & 3) + 1) + kHadShell * ((an[1] & 3) + 1) +
                      kHadShell * kHadShell * ((an[2] & 3) + 1);
      tbase[(size_t)i] = (own - kHadSlotBias) * kHadRowBytes;
      for (int dd = 0; dd < kNumDirections; ++dd) {
        const int slot = own + doff[dd];
        const int32_t s = halo[(size_t)dd * nc + i];
        if (at[(size_t)slot] >= 0 && at[(size_t)slot] != s)
          return fail(KIFMM_ENUMERIC, "FFT-M2L halo disagrees with the cluster positions");
        at[(size_t)slot] = s;
      }
    }
    tgt.push_back((int32_t)c);
    src.push_back((int32_t)list.size());
    for (int slot = 0; slot < kHadSrcSlots; ++slot)
      if (at[(size_t)slot] >= 0) list.push_back((int32_t)((uint32_t)at[(size_t)slot] << 8 | (uint32_t)slot));
    c = e;
  }
  D.hb_n = (int64_t)tgt.size();
  tgt.push_back((int32_t)nc);
  src.push_back((int32_t)list.size());
  KIFMM_TRY(upload(d, &D.hb_tgt, tgt.data(), tgt.size()));
  KIFMM_TRY(upload(d, &D.hb_src, src.data(), src.size()));
  KIFMM_TRY(upload(d, &D.hb_list, list.data(), list.size()));
  KIFMM_TRY(upload(d, &D.hb_tbase, tbase.data(), tbase.size()));
  return KIFMM_OK;
}

// FFT-M2L kernel spectra and twiddles depend only on the order, the radius
// of the (coincident) upward-equivalent and downward-check surfaces and the
// precision - the unit box's; a level's width is a scale of the inverse
// transform - so the handles on one device share one copy (reference
// counted): many problems with equal orders, as in a batch, read the same
// operator data from L2 instead of one copy each.
struct SharedFft {
  int64_t refs = 0;
  void* khat = nullptr;
  void* khat_split = nullptr;
  void* twiddle = nullptr;
};
std::mutex g_fft_mu;
std::map<std::tuple<int, int, int, uint64_t>, SharedFft> g_fft;

void release_shared_fft(DeviceState* d) {
  if (!d->fft_shared) return;
  std::lock_guard<std::mutex> lock(g_fft_mu);
  auto it = g_fft.find(d->fft_key);
  if (it != g_fft.end() && --it->second.refs == 0) {
    // teardown: failures are ignored
    (void)hipFree(it->second.khat);
    if (it->second.khat_split) (void)hipFree(it->second.khat_split);
    (void)hipFree(it->second.twiddle);
    g_fft.erase(it);
  }
  d->fft_shared = false;
}

kifmm_status upload_all(kifmm_handle* h) {
  const Tree& t = h->tree;
  const Operators& op = h->op;
  auto* d = new DeviceState();
  h->dev = d;
  d->device = h->cfg.device;
  d->fp64 = h->cfg.prec == KIFMM_FP64;
  KIFMM_HIP(hipSetDevice(d->device));
  const int depth = t.depth;
  const int ns = op.ns;

  KIFMM_TRY(upload(d, &d->src_xyz, t.src_sorted.data(), t.src_sorted.size()));
  KIFMM_TRY(upload(d, &d->tgt_xyz, t.tgt_sorted.data(), t.tgt_sorted.size()));
  KIFMM_TRY(upload(d, &d->src_perm, t.src_perm.data(), t.src_perm.size()));
  KIFMM_TRY(upload(d, &d->tgt_perm, t.tgt_perm.data(), t.tgt_perm.size()));
  KIFMM_TRY(upload(d, &d->src_start, t.src_start.data(), t.src_start.size()));
  KIFMM_TRY(upload(d, &d->src_end, t.src_end.data(), t.src_end.size()));
  KIFMM_TRY(upload(d, &d->tgt_start, t.tgt_start.data(), t.tgt_start.size()));
  KIFMM_TRY(upload(d, &d->tgt_end, t.tgt_end.data(), t.tgt_end.size()));
  KIFMM_TRY(upload(d, &d->near_offs, t.near_offs.data(), t.near_offs.size()));
  KIFMM_TRY(upload(d, &d->near_src, t.near_src.data(), t.near_src.size()));
  KIFMM_TRY(upload(d, &d->leaf_keys, t.levels[depth].keys.data(), t.levels[depth].keys.size()));
  {
    const Level& L = t.levels[depth];
    const double w = t.width / std::ldexp(1.0, depth);
    std::vector<double> c(3 * L.n);
    for (int64_t i = 0; i < L.n; ++i)
      for (int k = 0; k < 3; ++k) c[3 * i + k] = t.origin[k] + (L.anchor[3 * i + k] + 0.5) * w;
    KIFMM_TRY(upload(d, &d->leaf_centers, c.data(), c.size()));
  }

  KIFMM_TRY(upload(d, &d->surf, op.surf.data(), op.surf.size()));
  KIFMM_TRY(upload(d, &d->surf_c, op.surf_c.data(), op.surf_c.size()));
  {
    std::vector<int16_t> sl(op.lattice.begin(), op.lattice.end());
    KIFMM_TRY(upload(d, &d->surf_lat, sl.data(), sl.size()));
    std::vector<int16_t> l2s((size_t)op.p * op.p * op.p, -1);
    for (int s = 0; s < ns; ++s)
      l2s[((size_t)op.lattice[3 * s] * op.p + op.lattice[3 * s + 1]) * op.p + op.lattice[3 * s + 2]] = (int16_t)s;
    KIFMM_TRY(upload(d, &d->lat2surf, l2s.data(), l2s.size()));
  }
  KIFMM_TRY(upload(d, &d->up_V, op.up_V.data(), op.up_V.size()));
  KIFMM_TRY(upload(d, &d->up_Ut, op.up_Ut.data(), op.up_Ut.size()));
  KIFMM_TRY(upload(d, &d->down_V, op.down_V.data(), op.down_V.size()));
  KIFMM_TRY(upload(d, &d->down_Ut, op.down_Ut.data(), op.down_Ut.size()));
  KIFMM_TRY(upload(d, &d->m2m, op.m2m.data(), op.m2m.size()));
  KIFMM_TRY(upload(d, &d->l2l, op.l2l.data(), op.l2l.size()));
  if (!d->fp64) {
    KIFMM_TRY(upload(d, &d->up_P, op.up_P.data(), op.up_P.size()));
    KIFMM_TRY(upload(d, &d->down_P, op.down_P.data(), op.down_P.size()));
    KIFMM_TRY(upload(d, &d->m2m_c, op.m2m_c.data(), op.m2m_c.size()));
    KIFMM_TRY(upload(d, &d->l2l_c, op.l2l_c.data(), op.l2l_c.size()));
  }

  d->lv.resize(depth + 1);
  for (int l = 0; l <= depth; ++l) {
    DevLevel& D = d->lv[l];
    const Level& L = t.levels[l];
    D.n = L.n;
    D.w = t.width / std::ldexp(1.0, l);
    if (l < depth) {
      // one empty cluster past the end (all children absent): its FFT-M2L
      // spectra are zero and stand in for absent sibling clusters
      std::vector<int32_t> ch(L.child);
      ch.resize(L.child.size() + 8, -1);
      KIFMM_TRY(upload(d, &D.child, ch.data(), ch.size()));
    }
    if (l >= 2 && h->cfg.m2l == KIFMM_M2L_FFT) {
      std::vector<int32_t> hl(L.halo);
      const int32_t empty = (int32_t)t.levels[l - 1].n;
      for (int32_t& x : hl)
        if (x < 0) x = empty;
      KIFMM_TRY(upload(d, &D.halo, hl.data(), hl.size()));
      KIFMM_TRY(build_source_blocks(d, D, t.levels[l - 1], hl));
    }
  }

  if (h->cfg.m2l == KIFMM_M2L_FFT) {
    const int n = op.n, F = op.F;
    uint64_t ai_bits;
    std::memcpy(&ai_bits, &op.ai, sizeof ai_bits);
    const auto key = std::make_tuple(d->device, op.p, d->fp64 ? 1 : 0, ai_bits);
    std::lock_guard<std::mutex> lock(g_fft_mu);
    auto found = g_fft.find(key);
    if (found != g_fft.end()) {
      ++found->second.refs;
      d->khat = found->second.khat;
      d->khat_split = found->second.khat_split;
      d->twiddle = found->second.twiddle;
      d->fft_key = key;
      d->fft_shared = true;
    } else {
      // twiddle matrix Wm[k][j] = exp(-2 pi i (k j mod n) / n), k < n, j < p
      std::vector<double> tw(2 * (size_t)n * op.p);
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < op.p; ++j) {
          const int m = (k * j) % n;
          tw[2 * ((size_t)k * op.p + j)] = std::cos(2.0 * M_PI * m / n);
          tw[2 * ((size_t)k * op.p + j) + 1] = -std::sin(2.0 * M_PI * m / n);
        }
      // kernel spectra in sibling-cluster frequency order [f][26][8 i][8 j]
      std::vector<double> kh((size_t)F * 26 * 64 * 2, 0.0);
      for (int dd = 0; dd < 26; ++dd) {
        int D[3];
        direction_vector(dd, D);
        for (int i = 0; i < 8; ++i)
          for (int j = 0; j < 8; ++j) {
            const int tx = 2 * D[0] + (j & 1) - (i & 1);
            const int ty = 2 * D[1] + ((j >> 1) & 1) - ((i >> 1) & 1);
            const int tz = 2 * D[2] + ((j >> 2) & 1) - ((i >> 2) & 1);
            const int it = transfer_index(tx, ty, tz);
            if (it < 0) continue;  // adjacent pair: zero kernel
            for (int f = 0; f < F; ++f) {
              const size_t o = ((((size_t)f * 26 + dd) * 8 + i) * 8 + j) * 2;
              kh[o] = op.spectra[((size_t)it * F + f) * 2];
              kh[o + 1] = op.spectra[((size_t)it * F + f) * 2 + 1];
            }
          }
      }
      // the shared copy is allocated outside the handle's own allocations
      auto put = [](const void* host, size_t bytes, void** dev) -> kifmm_status {
        *dev = nullptr;
        hipError_t e = hipMalloc(dev, bytes);
        if (e != hipSuccess) return fail(KIFMM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        e = hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
          (void)hipFree(*dev);
          *dev = nullptr;
          return fail(KIFMM_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
        return KIFMM_OK;
      };
      SharedFft sh;
      kifmm_status st;
      if (d->fp64) {
        st = put(tw.data(), tw.size() * sizeof(double), &sh.twiddle);
        if (st == KIFMM_OK) st = put(kh.data(), kh.size() * sizeof(double), &sh.khat);
      } else {
        std::vector<float> twf(tw.begin(), tw.end()), khf(kh.begin(), kh.end());
        st = put(twf.data(), twf.size() * sizeof(float), &sh.twiddle);
        if (st == KIFMM_OK) st = put(khf.data(), khf.size() * sizeof(float), &sh.khat);
        if (st == KIFMM_OK) {
          // BF16 parts of the B operand of the split Hadamard
          hipError_t e = hipMalloc(&sh.khat_split, (size_t)hadamard_split_bytes(F));
          if (e != hipSuccess) {
            sh.khat_split = nullptr;
            st = fail(KIFMM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
          } else {
            e = launch_hadamard_split_prep(sh.khat, F, sh.khat_split, nullptr);
            if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
            if (e != hipSuccess) st = fail(KIFMM_EDEVICE, std::string("split prep: ") + hipGetErrorString(e));
          }
        }
      }
      if (st != KIFMM_OK) {
        if (sh.twiddle) (void)hipFree(sh.twiddle);
        if (sh.khat) (void)hipFree(sh.khat);
        if (sh.khat_split) (void)hipFree(sh.khat_split);
        return st;
      }
      sh.refs = 1;
      g_fft[key] = sh;
      d->khat = sh.khat;
      d->khat_split = sh.khat_split;
      d->twiddle = sh.twiddle;
      d->fft_key = key;
      d->fft_shared = true;
    }
  } else {
    const int k = op.k;
    std::vector<double> St((size_t)k * ns);
    for (int i = 0; i < ns; ++i)
      for (int j = 0; j < k; ++j) St[(size_t)j * ns + i] = op.S[(size_t)i * k + j];
    KIFMM_TRY(upload(d, &d->Ublas, op.U.data(), op.U.size()));
    KIFMM_TRY(upload(d, &d->SblasT, St.data(), St.size()));
    KIFMM_TRY(pack_blas_operators(h, d));
    if (op.recompressed && h->cfg.m2l == KIFMM_M2L_BLAS) KIFMM_TRY(pack_blas_stacked(h, d));
  }
  for (int e = 0; e < 8; ++e) KIFMM_HIP(hipEventCreate(&d->ev[e]));
  d->lev_ev.assign(4 * (depth + 1), nullptr);
  for (auto& e : d->lev_ev) KIFMM_HIP(hipEventCreate(&e));
  d->events = true;
  if (h->cfg.m2l == KIFMM_M2L_FFT) {
    KIFMM_HIP(hipStreamCreateWithFlags(&d->coarse, hipStreamNonBlocking));
    d->side.assign(depth + 1, nullptr);
    d->up_ev.assign(depth + 1, nullptr);
    d->join_ev.assign(depth + 1, nullptr);
    for (int l = 2; l < depth; ++l) {
      KIFMM_HIP(hipStreamCreateWithFlags(&d->side[l], hipStreamNonBlocking));
      KIFMM_HIP(hipEventCreateWithFlags(&d->up_ev[l], hipEventDisableTiming));
      KIFMM_HIP(hipEventCreateWithFlags(&d->join_ev[l], hipEventDisableTiming));
    }
    KIFMM_HIP(hipEventCreateWithFlags(&d->fork_ev, hipEventDisableTiming));
    KIFMM_HIP(hipEventCreateWithFlags(&d->down_ev, hipEventDisableTiming));
    KIFMM_HIP(hipStreamCreateWithFlags(&d->nearst, hipStreamNonBlocking));
    KIFMM_HIP(hipEventCreateWithFlags(&d->near_fork_ev, hipEventDisableTiming));
    KIFMM_HIP(hipEventCreateWithFlags(&d->near_ev, hipEventDisableTiming));
  }
  return KIFMM_OK;
}

// Target boxes per BLAS / dense tile for n_vec vectors: the knob, clamped
// to the 128 MFMA columns of a tile.
int blas_tile_width(const kifmm_handle* h, int nvec) {
  const int tb_max = std::max(1, 128 / nvec), knob = h->tune[KIFMM_TUNE_BLAS_TILE];
  return knob > 0 ? std::min(knob, tb_max) : tb_max;
}

// The per-evaluate work buffers of a handle for n_vec vectors: charges in
// sorted order, multipoles and locals per level, check potentials, GEMM
// intermediates, split-K partials (gemm_elems doubles), padded compressed
// multipoles (BLAS / dense) and the spectra and check potentials of each
// FFT-M2L level (the levels run concurrently).  Each slot names its size
// and the DeviceState field that points at it; ensure_work allocates the
// slots one by one, the no-allocation evaluate carves them out of one
// fixed array.
struct WorkSlot {
  size_t bytes;
  std::function<void*()> get;
  std::function<void(void*)> set;
};

std::vector<WorkSlot> work_slots(const kifmm_handle* h, DeviceState* d, int nvec, int64_t gemm_elems) {
  const Tree& t = h->tree;
  const Operators& op = h->op;
  const int depth = t.depth;
  const size_t ns = op.ns, nv = (size_t)nvec;
  int64_t maxn = 0;
  for (int l = 0; l <= depth; ++l) maxn = std::max(maxn, t.levels[l].n);
  const size_t qbytes = (d->fp64 ? 8 : 4);
  if ((int)d->mult.size() != depth + 1) d->mult.assign(depth + 1, nullptr);
  if ((int)d->local.size() != depth + 1) d->local.assign(depth + 1, nullptr);
  std::vector<WorkSlot> w;
  auto dbl = [](double** f) {
    return std::make_pair(std::function<void*()>([f] { return (void*)*f; }),
                          std::function<void(void*)>([f](void* p) { *f = (double*)p; }));
  };
  auto raw = [](void** f) {
    return std::make_pair(std::function<void*()>([f] { return *f; }),
                          std::function<void(void*)>([f](void* p) { *f = p; }));
  };
  auto add = [&w](size_t bytes, std::pair<std::function<void*()>, std::function<void(void*)>> gs) {
    w.push_back(WorkSlot{bytes, gs.first, gs.second});
  };
  add(nv * (size_t)t.n_src * qbytes, raw(&d->qs));
  for (int l = 2; l <= depth; ++l) {
    add((size_t)t.levels[l].n * nv * ns * 8, dbl(&d->mult[l]));
    add((size_t)t.levels[l].n * nv * ns * 8, dbl(&d->local[l]));
  }
  // check potentials have nc >= ns entries per box and vector
  const size_t ncs = std::max<size_t>(ns, (size_t)op.nc);
  const size_t kmax = std::max<size_t>(ncs, (size_t)std::max(op.k, 1));
  add((size_t)maxn * nv * ncs * 8, dbl(&d->phi));
  add((size_t)maxn * nv * kmax * 8, dbl(&d->tmp));
  add((size_t)maxn * nv * kmax * 8, dbl(&d->tmp2));
  add((size_t)gemm_elems * 8, dbl(&d->gemm_ws));
  // the near-field pass's sums in sorted target order, read back by the
  // far-field pass (split leaf passes: FFT schedules and batches)
  add(nv * (size_t)t.n_tgt * qbytes, raw(&d->nearbuf));
  if (h->cfg.m2l != KIFMM_M2L_FFT) {
    // padded compressed multipoles: FP64 8 bytes, FP32 / two BF16 parts 4,
    // three BF16 parts 6 per value
    add((size_t)maxn * nv * d->kp * (d->blas_mode == 0 ? 8 : d->blas_mode == 3 ? 6 : 4), raw(&d->qpad));
    if (use_stacked(h, d)) {
      const size_t xi = (size_t)maxn * nv * d->st_Rs;
      if (d->blas_mode >= 2) {
        add(xi * 2, raw(&d->xi_hi));
        add(xi * 2, raw(&d->xi_lo));
        if (d->blas_mode == 3) add(xi * 2, raw(&d->xi_p2));
      } else {
        add(xi * (d->blas_mode == 0 ? 8 : 4), raw(&d->xi_hi));
      }
    }
  } else {
    const size_t cb = d->fp64 ? 16 : 8;
    for (int l = 2; l <= depth; ++l) {
      DevLevel& D = d->lv[l];
      const size_t nc = (size_t)t.levels[l - 1].n;
      add((size_t)op.F * (nc + 1) * nv * 8 * cb, raw(&D.Qhat));  // + empty cluster
      add((size_t)op.F * nc * nv * 8 * cb, raw(&D.Phat));
      add((size_t)t.levels[l].n * nv * ns * 8, dbl(&D.chk));
    }
  }
  return w;
}

kifmm_status ensure_work(kifmm_handle* h, int nvec) {
  DeviceState* d = h->dev;
  if (h->cfg.m2l != KIFMM_M2L_FFT) {
    const int TB = blas_tile_width(h, nvec);
    if (TB != d->tile_tb) {
      if (h->batches > 0)
        return fail(KIFMM_ESTATE, "a batch holds this handle: its BLAS tiles cannot be rebuilt");
      KIFMM_TRY(build_blas_tiles(h, d, TB));
    }
  }
  const bool need_xi = use_stacked(h, d) && h->cfg.m2l != KIFMM_M2L_FFT;
  if (nvec <= d->nvec_cap && (!need_xi || d->xi_hi)) return KIFMM_OK;
  if (h->batches > 0)
    return fail(KIFMM_ESTATE, "a batch holds this handle: more vectors than its buffers hold");
  d->xi_hi = d->xi_lo = d->xi_p2 = nullptr;
  nvec = std::max(nvec, d->nvec_cap);
  for (void* p : d->work_allocs) (void)hipFree(p);
  d->work_allocs.clear();
  d->nvec_cap = 0;
  const int64_t gemm_elems = (int64_t)8 << 20;  // 64 MiB of split-K partials
  for (WorkSlot& ws : work_slots(h, d, nvec, gemm_elems)) {
    char* p;
    KIFMM_TRY(dalloc(d, &p, ws.bytes, true));
    ws.set(p);
  }
  d->gemm_ws_elems = gemm_elems;
  d->nvec_cap = nvec;
  return KIFMM_OK;
}

// Launches of the evaluate: enqueued at once, or recorded into d->sink as
// jobs of grouped launches (the grouped forward takes one item group per
// workgroup and the FP32 Hadamard one workgroup per frequency; both compute
// every item as the launches here do).
hipError_t gemm(DeviceState* d, Gemm64 g, hipStream_t s) {
  g.work = d->gemm_ws;
  g.work_elems = d->gemm_ws_elems;
  if (!d->sink) return launch_gemm64(g, s);
  GemmJob j;
  const hipError_t e = plan_gemm64(g, j);
  if (e != hipSuccess || j.split == 0) return e;
  d->sink->add(kFamGemm, 0, j, gemm64_job_blocks(j));
  if (j.split > 1) d->sink->add(kFamGemmReduce, 0, j, gemm64_reduce_blocks(j));
  return hipSuccess;
}

hipError_t run_fft_forward(DeviceState* d, int p, const double* M, const int32_t* child, int64_t ncl,
                           int nvec, void* Qhat, hipStream_t s) {
  if (!d->sink) return launch_fft_forward(p, d->fp64, M, child, ncl, nvec, d->lat2surf, d->twiddle, Qhat, s);
  FwdArgs a;
  int inst;
  int64_t blocks;
  const hipError_t e = plan_fft_forward(p, d->fp64, M, child, ncl, nvec, d->lat2surf, d->twiddle, Qhat,
                                        false, a, inst, blocks);
  if (e == hipSuccess && blocks > 0) d->sink->add(kFamFwd, inst, a, blocks);
  return e;
}

hipError_t run_hadamard(DeviceState* d, int F, const DevLevel& D, int64_t ncl, int nvec, bool units,
                        bool split, hipStream_t s) {
  const bool bf16 = split && !d->fp64;
  const void* kt = bf16 ? d->khat_split : d->khat;
  if (!d->sink)
    return launch_hadamard(d->fp64, bf16, F, kt, D.Qhat, D.halo, D.hb_n, D.hb_tgt, D.hb_src, D.hb_list,
                           D.hb_tbase, ncl, nvec, units, D.Phat, s);
  HadBlockArgs ab;
  HadGatherArgs ag;
  int64_t blocks;
  const hipError_t e = plan_hadamard(d->fp64, bf16, F, kt, D.Qhat, D.halo, D.hb_n, D.hb_tgt, D.hb_src,
                                     D.hb_list, D.hb_tbase, ncl, nvec, 2, D.Phat, ab, ag, blocks);
  if (e != hipSuccess || blocks == 0) return e;
  if (d->fp64)
    d->sink->add(kFamHad, hadamard_inst(true, false), ag, blocks);
  else
    d->sink->add(kFamHad, hadamard_inst(false, bf16), ab, blocks);
  return hipSuccess;
}

hipError_t run_fft_inverse(DeviceState* d, int p, const void* Phat, const int32_t* child, int64_t ncl,
                           int nvec, double scale, double* out, hipStream_t s) {
  if (!d->sink)
    return launch_fft_inverse(p, d->fp64, Phat, child, ncl, nvec, d->surf_lat, d->twiddle, scale, out, s);
  InvArgs a;
  int inst;
  int64_t blocks;
  const hipError_t e = plan_fft_inverse(p, d->fp64, Phat, child, ncl, nvec, d->surf_lat, d->twiddle,
                                        scale, out, a, inst, blocks);
  if (e == hipSuccess && blocks > 0) d->sink->add(kFamInv, inst, a, blocks);
  return e;
}

// a launch without a grouped form: enqueued at once or recorded as is
hipError_t run_single(DeviceState* d, std::function<hipError_t(hipStream_t)> f, hipStream_t s) {
  if (!d->sink) return f(s);
  d->sink->add_single(std::move(f));
  return hipSuccess;
}

void stage_mark(DeviceState* d, int phase, int level) {
  if (d->sink) d->sink->stage(phase, level);
}

// Apply a unit-box pseudo-inverse V (Ut phi) scaled by the box width w:
// check potentials [box][v][nc] -> equivalent densities [box][v][ns].
kifmm_status pinv_apply(kifmm_handle* h, const double* V, const double* Ut, int r, double w,
                        const double* in, double* out, int64_t nbox, int nvec, hipStream_t s) {
  DeviceState* d = h->dev;
  const int ns = h->op.ns, nc = h->op.nc;  // equivalent-side and check-side points
  Gemm64 g1{Ut, r, nc, nc, w, in, nc, 1, nullptr, (int64_t)nvec * nc, nc,
            d->tmp, r, 1, nullptr, (int64_t)nvec * r, r, nbox, nvec, 0};
  KIFMM_LAUNCH(gemm(d, g1, s));
  Gemm64 g2{V, ns, r, r, 1.0, d->tmp, r, 1, nullptr, (int64_t)nvec * r, r,
            out, ns, 1, nullptr, (int64_t)nvec * ns, ns, nbox, nvec, 0};
  KIFMM_LAUNCH(gemm(d, g2, s));
  return KIFMM_OK;
}

// M2L check potentials of one level: in[box][v][ns] equivalent densities,
// out[box][v][nc] check potentials (overwritten)
kifmm_status m2l_level(kifmm_handle* h, int l, const double* in, double* out, int nvec,
                       hipStream_t s, bool timed) {
  DeviceState* d = h->dev;
  const Operators& op = h->op;
  const DevLevel& D = d->lv[l];
  const int ns = op.ns, ncp = op.nc;
  hipEvent_t* mark = timed ? &d->lev_ev[4 * l] : nullptr;
  if (mark) KIFMM_HIP(hipEventRecord(mark[0], s));
  if (h->cfg.m2l == KIFMM_M2L_FFT) {
    const int64_t nc = d->lv[l - 1].n;
    const int32_t* child = d->lv[l - 1].child;
    // spectra of the nc clusters and of the empty cluster behind them
    KIFMM_LAUNCH(run_fft_forward(d, op.p, in, child, nc + 1, nvec, D.Qhat, s));
    if (mark) KIFMM_HIP(hipEventRecord(mark[1], s));
    KIFMM_LAUNCH(run_hadamard(d, op.F, D, nc, nvec, h->tune[KIFMM_TUNE_HADAMARD] == 1,
                              h->tune[KIFMM_TUNE_PRODUCTS] == 0, s));
    if (mark) KIFMM_HIP(hipEventRecord(mark[2], s));
    const double scale = 1.0 / ((double)op.n * op.n * op.n * D.w);  // 1 / (n^3 w)
    KIFMM_LAUNCH(run_fft_inverse(d, op.p, D.Phat, child, nc, nvec, scale, out, s));
    if (mark) KIFMM_HIP(hipEventRecord(mark[3], s));
    return KIFMM_OK;
  }
  // dense / compressed M2L (Section 3.2), fused per target tile
  const int k = op.k;
  const bool dense = h->cfg.m2l == KIFMM_M2L_DENSE;
  const double* qsrc = in;
  if (!dense) {
    // compressed multipoles  Q~ = S^T Q
    Gemm64 g{d->SblasT, k, ns, ns, 1.0, in, ns, 1, nullptr, (int64_t)nvec * ns, ns,
             d->tmp, k, 1, nullptr, (int64_t)nvec * k, k, D.n, nvec, 0};
    KIFMM_LAUNCH(gemm(d, g, s));
    qsrc = d->tmp;
  }
  if (!dense && use_stacked(h, d)) {
    // stacked form: Stage A (xi of every source box), Stage B (targets)
    void* qlo = nullptr;
    void* qp2 = nullptr;
    if (d->blas_mode >= 2) {
      const size_t part = (size_t)D.n * nvec * d->kp * 2;  // bytes of one BF16 part
      qlo = static_cast<char*>(d->qpad) + part;
      if (d->blas_mode == 3) qp2 = static_cast<char*>(d->qpad) + 2 * part;
      void* qhi = d->qpad;
      const int kp = d->kp;
      const int64_t ncols = D.n * nvec;
      KIFMM_LAUNCH(run_single(d, [=](hipStream_t st) { return launch_pad_split(qsrc, k, ncols, kp, qhi, qlo, qp2, st); }, s));
    } else {
      void* qp = d->qpad;
      const int kp = d->kp;
      const bool f64 = d->blas_mode == 0;
      const int64_t ncols = D.n * nvec;
      KIFMM_LAUNCH(run_single(d, [=](hipStream_t st) { return launch_pad_convert(qsrc, k, ncols, kp, f64, qp, st); }, s));
    }
    if (mark) KIFMM_HIP(hipEventRecord(mark[1], s));
    BlasStack b;
    b.mode = d->blas_mode;
    b.k = k;
    b.kp = d->kp;
    b.nvec = nvec;
    b.TB = d->tile_tb;
    b.C = d->tile_tb * nvec;
    b.ntiles = D.ntiles;
    b.tile_box = D.tile_box;
    b.tile_class = D.tile_class;
    b.tile_src = D.tile_src;
    b.J = d->st_J;
    b.Rs = d->st_Rs;
    b.Rpad = d->st_Rpad;
    b.nsteps = d->st_nsteps;
    b.rbo = d->st_rbo;
    b.A_hi = d->st_A_hi;
    b.A_lo = d->st_A_lo;
    b.B_hi = d->st_B_hi;
    b.B_lo = d->st_B_lo;
    b.info = d->st_info;
    b.q_hi = d->qpad;
    b.q_lo = qlo;
    b.xi_hi = d->xi_hi;
    b.xi_lo = d->xi_lo;
    b.A_p2 = d->st_A_p2;
    b.B_p2 = d->st_B_p2;
    b.q_p2 = qp2;
    b.xi_p2 = d->xi_p2;
    b.out = d->tmp2;
    b.scale = 1.0 / D.w;
    // levels with few tiles split Stage B's K steps over up to 16 workgroups
    // per tile; the partial sums go to tmp (free once the compressed
    // multipoles are padded), which holds maxn x n_vec x max(n_s, n_c, k)
    if (D.ntiles > 0 && D.ntiles < 1024) {
      int64_t maxn = 0;
      for (const Level& L : h->tree.levels) maxn = std::max(maxn, L.n);
      const int64_t kmax = std::max<int64_t>(std::max(op.ns, op.nc), k);
      const int64_t want = std::min<int64_t>(16, (2048 + D.ntiles - 1) / D.ntiles);
      const int64_t fits = (maxn * kmax) / std::max<int64_t>(1, D.n * (int64_t)k);
      b.ksplit = (int)std::max<int64_t>(1, std::min(want, fits));
    }
    b.n_boxes = D.n;
    b.partial = d->tmp;
    KIFMM_LAUNCH(run_single(d, [=](hipStream_t st) { return launch_blas_stacked(b, st); }, s));
    if (mark) KIFMM_HIP(hipEventRecord(mark[2], s));
    Gemm64 g{d->Ublas, ncp, k, k, 1.0, d->tmp2, k, 1, nullptr, (int64_t)nvec * k, k,
             out, ncp, 1, nullptr, (int64_t)nvec * ncp, ncp, D.n, nvec, 0};
    KIFMM_LAUNCH(gemm(d, g, s));
    if (mark) KIFMM_HIP(hipEventRecord(mark[3], s));
    return KIFMM_OK;
  }
  {
    void* qp = d->qpad;
    const int kp = d->kp;
    const bool f64 = d->blas_mode == 0;
    const int64_t ncols = D.n * nvec;
    KIFMM_LAUNCH(run_single(d, [=](hipStream_t st) { return launch_pad_convert(qsrc, k, ncols, kp, f64, qp, st); }, s));
  }
  if (mark) KIFMM_HIP(hipEventRecord(mark[1], s));
  BlasM2L b;
  b.q = d->qpad;
  b.kp = d->kp;
  b.k = k;
  b.nvec = nvec;
  b.TB = d->tile_tb;
  b.C = d->tile_tb * nvec;
  b.ntiles = D.ntiles;
  b.tile_box = D.tile_box;
  b.tl_offs = D.tl_offs;
  b.tl_t = D.tl_t;
  b.tl_src = D.tl_src;
  b.op_off = d->op_off;
  b.ktp = d->ktp;
  b.ktp_max = d->ktp_max;
  b.ktq = d->ktq;
  b.op_hi = d->op_hi;
  b.op_lo = d->op_lo;
  b.out = dense ? out : d->tmp2;
  b.scale = 1.0 / D.w;
  {
    const int mode = d->blas_mode;
    const bool two = d->two_stage;
    KIFMM_LAUNCH(run_single(d, [=](hipStream_t st) { return launch_blas_m2l(b, mode, two, st); }, s));
  }
  if (mark) KIFMM_HIP(hipEventRecord(mark[2], s));
  if (!dense) {
    // check potentials  Phi = U Phi~
    Gemm64 g{d->Ublas, ncp, k, k, 1.0, d->tmp2, k, 1, nullptr, (int64_t)nvec * k, k,
             out, ncp, 1, nullptr, (int64_t)nvec * ncp, ncp, D.n, nvec, 0};
    KIFMM_LAUNCH(gemm(d, g, s));
  }
  if (mark) KIFMM_HIP(hipEventRecord(mark[3], s));
  return KIFMM_OK;
}

}  // namespace

void destroy_device(DeviceState* d) {
  if (!d) return;
  // teardown: failures are ignored
  (void)hipSetDevice(d->device);
  release_shared_fft(d);
  if (d->events)
    for (auto& e : d->ev) (void)hipEventDestroy(e);
  for (auto& e : d->lev_ev)
    if (e) (void)hipEventDestroy(e);
  if (d->fork_ev) (void)hipEventDestroy(d->fork_ev);
  if (d->down_ev) (void)hipEventDestroy(d->down_ev);
  if (d->near_fork_ev) (void)hipEventDestroy(d->near_fork_ev);
  if (d->near_ev) (void)hipEventDestroy(d->near_ev);
  if (d->nearst) (void)hipStreamDestroy(d->nearst);
  for (auto& e : d->up_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : d->join_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& st : d->side)
    if (st) (void)hipStreamDestroy(st);
  if (d->coarse) (void)hipStreamDestroy(d->coarse);
  for (void* p : d->work_allocs) (void)hipFree(p);
  for (void* p : d->allocs) (void)hipFree(p);
  delete d;
}

// Size limits of the kernels, checked before anything is enqueued: the fused
// BLAS / dense kernel holds at most 128 columns (boxes x vectors) per tile;
// the FFT-M2L kernels index clusters with 24 bits, one frequency's spectra
// with 32-bit byte offsets and rows (cluster x vector) with 31 bits.
kifmm_status check_limits(const kifmm_handle* h, int nvec) {
  if (nvec < 1) return fail(KIFMM_EINVAL, "n_vec must be >= 1");
  if (h->cfg.m2l != KIFMM_M2L_FFT) {
    if (nvec > 128) return fail(KIFMM_EUNSUPPORTED, "BLAS / dense M2L takes at most 128 vectors per call");
    return KIFMM_OK;
  }
  const int64_t cb = h->cfg.prec == KIFMM_FP64 ? 8 : 4;
  for (int l = 2; l <= h->tree.depth; ++l) {
    const int64_t nc = h->tree.levels[l - 1].n;
    if (nc + 1 >= (int64_t(1) << 23) || (nc + 1) * nvec * 16 * cb >= (int64_t(1) << 32) ||
        (nc + 1) * nvec * 8 >= (int64_t(1) << 31))
      return fail(KIFMM_EUNSUPPORTED, "FFT-M2L level too large for this many vectors "
                                      "(clusters x vectors x 128 bytes must stay below 4 GiB)");
  }
  return KIFMM_OK;
}

kifmm_status device_ready(kifmm_handle* h, int nvec) {
  KIFMM_TRY(check_limits(h, nvec));
  if (!h->dev) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
      return fail(KIFMM_EDEVICE, "no HIP device available");
    if (h->cfg.device < 0 || h->cfg.device >= count)
      return fail(KIFMM_EINVAL, "device ordinal out of range");
    kifmm_status st = upload_all(h);
    if (st != KIFMM_OK) {
      destroy_device(h->dev);
      h->dev = nullptr;
      return st;
    }
  }
  KIFMM_HIP(hipSetDevice(h->dev->device));
  return ensure_work(h, nvec);
}

namespace {

// The evaluate's launches on buffers already in place (device_ready or the
// no-allocation scratch).
kifmm_status evaluate_launches(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                               int64_t ldphi, hipStream_t s) {
  DeviceState* d = h->dev;
  const Tree& t = h->tree;
  const Operators& op = h->op;
  const int depth = t.depth, ns = op.ns, nc = op.nc;  // equivalent / check points
  const bool timed = h->timing;
  if (timed) KIFMM_HIP(hipEventRecord(d->ev[0], s));

  const bool fft = h->cfg.m2l == KIFMM_M2L_FFT;
  // Schedules: `graph` (FFT, untimed) runs the FMM passes as a dependency
  // graph over several streams; `phased` (FFT, timed) runs the phases one
  // after another with the M2L levels concurrent and the leaf work as two
  // kernels (near field, then far field), so each phase and kernel is timed
  // on its own; `serial` (other M2L forms, and under stream capture, where
  // the multi-stream graph is not recorded) runs everything back to back on
  // s.  graph runs the near field on a stream of its own from the start and
  // the far field last; serial uses the fused leaf kernel.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  KIFMM_HIP(hipStreamIsCapturing(s, &cap));
  // (a batch recording the schedule takes the serial one, untimed)
  const bool fork = fft && cap == hipStreamCaptureStatusNone && !d->sink;
  const bool graph = fork && !timed && h->tune[KIFMM_TUNE_SCHEDULE] == 0;
  const bool phased = fork && timed;
  const DevLevel& leaf = d->lv[depth];
  const double ar_leaf = op.ao * 0.5 * leaf.w;
  auto leaf_pass = [&](int mode, hipStream_t st) -> kifmm_status {
    if (d->sink) {
      LeafArgs a;
      int inst;
      int64_t blocks;
      plan_leaf_eval(d->tgt_xyz, d->src_xyz, leaf.w, d->qs, d->fp64, t.n_src, d->tgt_start, d->tgt_end,
                     d->src_start, d->src_end, d->near_offs, d->near_src, d->leaf_centers, leaf.n,
                     d->surf, ar_leaf, ns, d->local[depth], d->tgt_perm, phi, ldphi, d->nearbuf,
                     t.n_tgt, nvec, mode, a, inst, blocks);
      if (inst < 0) return fail(KIFMM_EINVAL, "bad leaf-pass mode");
      if (blocks > 0) d->sink->add(kFamLeaf, inst, a, blocks);
      return KIFMM_OK;
    }
    KIFMM_LAUNCH(launch_leaf_eval(d->tgt_xyz, d->src_xyz, leaf.w, d->qs, d->fp64, t.n_src,
                                  d->tgt_start, d->tgt_end, d->src_start, d->src_end, d->near_offs,
                                  d->near_src, d->leaf_centers, leaf.n, d->surf, ar_leaf, ns,
                                  d->local[depth], d->tgt_perm, phi, ldphi, d->nearbuf, t.n_tgt, nvec,
                                  mode, st));
    return KIFMM_OK;
  };

  stage_mark(d, 0, 0);
  if (d->sink) {
    GatherArgs a{q, ldq, d->src_perm, t.n_src, nvec, d->qs};
    d->sink->add(kFamGather, d->fp64 ? 1 : 0, a, (t.n_src + 255) / 256 * nvec);
    // the near field on a branch of its own from the sorted charges on (its
    // raw sums, completed by the far field at the end: near then far gives
    // the fused kernel's result bit for bit)
    d->sink->side = true;
    stage_mark(d, 7, 0);
    KIFMM_TRY(leaf_pass(1, s));
    d->sink->side = false;
  } else {
    KIFMM_LAUNCH(launch_gather(q, ldq, d->src_perm, t.n_src, nvec, d->fp64, d->qs, s));
  }
  if (graph) {
    // The near field needs only the sorted charges: it runs on its own
    // stream, concurrently with the upward, M2L and downward passes, and
    // stores its raw sums, which the far-field kernel completes at the end
    // (near then far gives exactly the fused kernel's result).
    KIFMM_HIP(hipEventRecord(d->near_fork_ev, s));
    KIFMM_HIP(hipStreamWaitEvent(d->nearst, d->near_fork_ev, 0));
    KIFMM_TRY(leaf_pass(1, d->nearst));
    KIFMM_HIP(hipEventRecord(d->near_ev, d->nearst));
  }
  // upward pass
  if (timed) KIFMM_HIP(hipEventRecord(d->ev[6], s));
  stage_mark(d, 1, 0);
  if (d->sink) {
    P2MArgs a;
    int inst;
    int64_t blocks;
    plan_p2m(d->src_xyz, d->qs, d->fp64, t.n_src, d->src_start, d->src_end, d->leaf_centers, leaf.n,
             d->surf_c, ar_leaf, nc, nvec, d->phi, a, inst, blocks);
    if (blocks > 0) d->sink->add(kFamP2M, inst, a, blocks);
  } else {
    KIFMM_LAUNCH(launch_p2m(d->src_xyz, d->qs, d->fp64, t.n_src, d->src_start, d->src_end,
                            d->leaf_centers, leaf.n, d->surf_c, ar_leaf, nc, nvec, d->phi, s));
  }
  stage_mark(d, 2, 0);
  if (timed) KIFMM_HIP(hipEventRecord(d->ev[7], s));
  // FP64: two-factor pseudo-inverses after each M2M (Section 2.1.1); the
  // reduced-precision modes apply the composite operators (M2M with the
  // parent's pseudo-inverse folded in: the width scalings cancel)
  const bool composite = !d->fp64;
  if (composite) {
    Gemm64 g{d->up_P, ns, nc, nc, leaf.w, d->phi, nc, 1, nullptr, (int64_t)nvec * nc, nc,
             d->mult[depth], ns, 1, nullptr, (int64_t)nvec * ns, ns, leaf.n, nvec, 0};
    KIFMM_LAUNCH(gemm(d, g, s));
  } else {
    KIFMM_TRY(pinv_apply(h, d->up_V, d->up_Ut, op.r_up, leaf.w, d->phi, d->mult[depth], leaf.n, nvec, s));
  }
  // M2M into level l from level l + 1 (FP64: then the two-factor pinv)
  auto m2m_level = [&](int l, hipStream_t st) -> kifmm_status {
    const DevLevel& D = d->lv[l];
    if (composite) {
      Gemm64 g{d->m2m_c, ns, 8 * ns, 8 * ns, 1.0, d->mult[l + 1], ns, 8, D.child,
               (int64_t)nvec * ns, ns, d->mult[l], ns, 1, nullptr, (int64_t)nvec * ns, ns, D.n, nvec, 0};
      KIFMM_LAUNCH(gemm(d, g, st));
      return KIFMM_OK;
    }
    Gemm64 g{d->m2m, nc, 8 * ns, 8 * ns, 1.0 / D.w, d->mult[l + 1], ns, 8, D.child,
             (int64_t)nvec * ns, ns, d->phi, nc, 1, nullptr, (int64_t)nvec * nc, nc, D.n, nvec, 0};
    KIFMM_LAUNCH(gemm(d, g, st));
    return pinv_apply(h, d->up_V, d->up_Ut, op.r_up, D.w, d->phi, d->mult[l], D.n, nvec, st);
  };
  // locals of level l from its M2L check potentials chk and the parent's
  // locals: L2L (l >= 3) and the down pseudo-inverse
  auto down_level = [&](int l, double* chk, hipStream_t st) -> kifmm_status {
    const DevLevel& D = d->lv[l];
    if (composite) {
      // local = w down_P chk + (w / w_parent) [down_P L_o] local_parent
      Gemm64 g1{d->down_P, ns, nc, nc, D.w, chk, nc, 1, nullptr, (int64_t)nvec * nc, nc,
                d->local[l], ns, 1, nullptr, (int64_t)nvec * ns, ns, D.n, nvec, 0};
      KIFMM_LAUNCH(gemm(d, g1, st));
      if (l >= 3) {
        const DevLevel& P = d->lv[l - 1];
        Gemm64 g2{d->l2l_c, 8 * ns, ns, ns, D.w / P.w, d->local[l - 1], ns, 1, nullptr,
                  (int64_t)nvec * ns, ns, d->local[l], ns, 8, P.child, (int64_t)nvec * ns, ns,
                  P.n, nvec, 1};
        KIFMM_LAUNCH(gemm(d, g2, st));
      }
      return KIFMM_OK;
    }
    if (l >= 3) {
      const DevLevel& P = d->lv[l - 1];
      Gemm64 g{d->l2l, 8 * nc, ns, ns, 1.0 / P.w, d->local[l - 1], ns, 1, nullptr,
               (int64_t)nvec * ns, ns, chk, nc, 8, P.child, (int64_t)nvec * nc, nc, P.n, nvec, 1};
      KIFMM_LAUNCH(gemm(d, g, st));
    }
    return pinv_apply(h, d->down_V, d->down_Ut, op.r_down, D.w, chk, d->local[l], D.n, nvec, st);
  };

  if (graph) {
    // Each level's M2L needs only that level's multipoles.  The leaf level's
    // M2L (the critical path) starts on s as soon as the leaf multipoles
    // exist; the coarse stream runs the M2M chain, each coarse level's M2L
    // runs on its side stream once its multipoles exist, and the coarse
    // stream then walks the coarse downward pass as their M2L complete; s
    // finishes the leaf level's downward step after the coarse locals.
    if (timed) KIFMM_HIP(hipEventRecord(d->ev[1], s));
    KIFMM_HIP(hipEventRecord(d->fork_ev, s));
    KIFMM_TRY(m2l_level(h, depth, d->mult[depth], d->lv[depth].chk, nvec, s, timed));
    KIFMM_HIP(hipStreamWaitEvent(d->coarse, d->fork_ev, 0));
    for (int l = depth - 1; l >= 2; --l) {
      KIFMM_TRY(m2m_level(l, d->coarse));
      KIFMM_HIP(hipEventRecord(d->up_ev[l], d->coarse));
      KIFMM_HIP(hipStreamWaitEvent(d->side[l], d->up_ev[l], 0));
      KIFMM_TRY(m2l_level(h, l, d->mult[l], d->lv[l].chk, nvec, d->side[l], timed));
      KIFMM_HIP(hipEventRecord(d->join_ev[l], d->side[l]));
    }
    for (int l = 2; l < depth; ++l) {
      KIFMM_HIP(hipStreamWaitEvent(d->coarse, d->join_ev[l], 0));
      KIFMM_TRY(down_level(l, d->lv[l].chk, d->coarse));
    }
    KIFMM_HIP(hipEventRecord(d->down_ev, d->coarse));
    KIFMM_HIP(hipStreamWaitEvent(s, d->down_ev, 0));
    KIFMM_TRY(down_level(depth, d->lv[depth].chk, s));
    KIFMM_HIP(hipStreamWaitEvent(s, d->near_ev, 0));
    return leaf_pass(2, s);
  }
  for (int l = depth - 1; l >= 2; --l) {
    stage_mark(d, 3, 20 - l);
    KIFMM_TRY(m2m_level(l, s));
  }
  if (timed) KIFMM_HIP(hipEventRecord(d->ev[1], s));
  if (phased) {
    // M2L of all levels, concurrently: the coarse levels on side streams
    KIFMM_HIP(hipEventRecord(d->fork_ev, s));
    for (int l = 2; l < depth; ++l) {
      KIFMM_HIP(hipStreamWaitEvent(d->side[l], d->fork_ev, 0));
      KIFMM_TRY(m2l_level(h, l, d->mult[l], d->lv[l].chk, nvec, d->side[l], timed));
      KIFMM_HIP(hipEventRecord(d->join_ev[l], d->side[l]));
    }
    KIFMM_TRY(m2l_level(h, depth, d->mult[depth], d->lv[depth].chk, nvec, s, timed));
    for (int l = 2; l < depth; ++l) KIFMM_HIP(hipStreamWaitEvent(s, d->join_ev[l], 0));
    KIFMM_HIP(hipEventRecord(d->ev[4], s));
    for (int l = 2; l <= depth; ++l) KIFMM_TRY(down_level(l, d->lv[l].chk, s));
  } else {
    for (int l = 2; l <= depth; ++l) {
      // recorded: the FFT-M2L of all levels in one stage (each level has
      // its own buffers); other forms share phi and tmp buffers across
      // levels, so their M2L stays in the level's downward stage
      double* chk = fft ? d->lv[l].chk : d->phi;
      stage_mark(d, fft ? 4 : 5, fft ? 0 : l);
      KIFMM_TRY(m2l_level(h, l, d->mult[l], chk, nvec, s, timed));
      if (fft) stage_mark(d, 5, l);
      KIFMM_TRY(down_level(l, chk, s));
    }
  }
  if (timed) KIFMM_HIP(hipEventRecord(d->ev[2], s));
  if (phased) {
    KIFMM_TRY(leaf_pass(1, s));
    KIFMM_HIP(hipEventRecord(d->ev[5], s));
    KIFMM_TRY(leaf_pass(2, s));
  } else {
    stage_mark(d, 6, 0);
    KIFMM_TRY(leaf_pass(d->sink ? 2 : 0, s));
  }
  if (timed) {
    KIFMM_HIP(hipEventRecord(d->ev[3], s));
    KIFMM_HIP(hipEventSynchronize(d->ev[3]));
    float a = 0, b = 0, c = 0, tot = 0;
    KIFMM_HIP(hipEventElapsedTime(&a, d->ev[0], d->ev[1]));
    KIFMM_HIP(hipEventElapsedTime(&b, d->ev[1], d->ev[2]));
    KIFMM_HIP(hipEventElapsedTime(&c, d->ev[2], d->ev[3]));
    KIFMM_HIP(hipEventElapsedTime(&tot, d->ev[0], d->ev[3]));
    double parts[3] = {0, 0, 0};
    for (int l = 2; l <= depth; ++l)
      for (int k = 0; k < 3; ++k) {
        float ms = 0.f;
        KIFMM_HIP(hipEventElapsedTime(&ms, d->lev_ev[4 * l + k], d->lev_ev[4 * l + k + 1]));
        parts[k] += ms;
      }
    // phased: the M2L is the wall time of the concurrent levels; serial:
    // the levels run back to back and their kernel phases add up
    double m2l_ms = parts[0] + parts[1] + parts[2];
    if (phased) {
      float w = 0.f, nf = 0.f, ff = 0.f;
      KIFMM_HIP(hipEventElapsedTime(&w, d->ev[1], d->ev[4]));
      KIFMM_HIP(hipEventElapsedTime(&nf, d->ev[2], d->ev[5]));
      KIFMM_HIP(hipEventElapsedTime(&ff, d->ev[5], d->ev[3]));
      m2l_ms = w;
      h->timings[9] = nf;
      h->timings[10] = ff;
    } else {
      h->timings[9] = h->timings[10] = 0.0;
    }
    float p2m = 0.f;
    KIFMM_HIP(hipEventElapsedTime(&p2m, d->ev[6], d->ev[7]));
    h->timings[11] = p2m;
    h->timings[0] = a;
    h->timings[1] = m2l_ms;
    h->timings[2] = b - m2l_ms;
    h->timings[3] = c;
    h->timings[4] = tot;
    h->timings[5] = parts[0];
    h->timings[6] = parts[1];
    h->timings[7] = parts[2];
    h->timings[8] = depth - 1;
  }
  return KIFMM_OK;
}

}  // namespace

kifmm_status device_evaluate(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                             int64_t ldphi, hipStream_t s) {
  KIFMM_TRY(device_ready(h, nvec));
  return evaluate_launches(h, q, ldq, nvec, phi, ldphi, s);
}

// Record one evaluate's serial schedule into sink (nothing is enqueued):
// the device state, work buffers and tiles must already exist (a previous
// evaluate with the same vector count and knobs).
kifmm_status device_record(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                           int64_t ldphi, LaunchSink* sink, hipStream_t s) {
  DeviceState* d = h->dev;
  if (!d || nvec > d->nvec_cap) return fail(KIFMM_ESTATE, "recording before the device buffers exist");
  if (h->cfg.m2l != KIFMM_M2L_FFT && blas_tile_width(h, nvec) != d->tile_tb)
    return fail(KIFMM_ESTATE, "recording with BLAS tiles of another width");
  const bool timing = h->timing;
  h->timing = false;
  d->sink = sink;
  const kifmm_status st = evaluate_launches(h, q, ldq, nvec, phi, ldphi, s);
  d->sink = nullptr;
  h->timing = timing;
  return st;
}

// ---- evaluate without allocation ----------------------------------------------
// For callers that cannot allocate device memory (HIP graph capture, serving
// loops, harnesses that forbid it): the work buffers of one evaluate are
// carved out of `scratch`, a fixed device array each device holds until the
// process ends.  In host code `scratch` names a host-side stand-in, so the
// library takes the array's device address once per device with
// hipGetSymbolAddress (that device current) and only ever passes that
// address.  The split-K workspace is the largest the GEMM launcher can use,
// so its split, and with it every sum, is the one kifmm_evaluate computes.
static __device__ __align__(256) unsigned char scratch[KIFMM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
kifmm_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(KIFMM_EUNSUPPORTED, "no-allocation evaluate: device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(KIFMM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return KIFMM_OK;
}

}  // namespace

kifmm_status device_evaluate_noalloc(kifmm_handle* h, const void* q, int64_t ldq, int nvec,
                                     void* phi, int64_t ldphi, hipStream_t s) {
  KIFMM_TRY(check_limits(h, nvec));
  DeviceState* d = h->dev;
  if (!d)
    return fail(KIFMM_ESTATE, "no-allocation evaluate: the tree and operators are not on the device "
                              "yet (one kifmm_evaluate or kifmm_stage places them there)");
  if (h->cfg.m2l != KIFMM_M2L_FFT && blas_tile_width(h, nvec) != d->tile_tb)
    return fail(KIFMM_ESTATE, "no-allocation evaluate: the BLAS tiles were built for another tile "
                              "width (one kifmm_evaluate with this n_vec rebuilds them)");
  KIFMM_HIP(hipSetDevice(d->device));
  void* base = nullptr;
  KIFMM_TRY(scratch_address(d->device, &base));
  const int64_t gemm_elems = gemm64_max_work_elems();
  std::vector<WorkSlot> slots = work_slots(h, d, nvec, gemm_elems);
  std::vector<size_t> off(slots.size());
  size_t total = 0;
  for (size_t i = 0; i < slots.size(); ++i) {
    off[i] = total;
    total += (slots[i].bytes + 255) / 256 * 256;
  }
  if (total > (size_t)KIFMM_NOALLOC_SCRATCH_BYTES)
    return fail(KIFMM_EINVAL, "no-allocation evaluate: this problem needs " + std::to_string(total >> 20) +
                                  " MiB of work buffers; the scratch array holds " +
                                  std::to_string((size_t)KIFMM_NOALLOC_SCRATCH_BYTES >> 20) + " MiB");
  // the handle's own work buffers are set aside for the call and put back
  struct Swap {
    DeviceState* d;
    std::vector<WorkSlot>& slots;
    std::vector<void*> kept;
    int nvec_cap;
    int64_t gemm_ws_elems;
    ~Swap() {
      for (size_t i = 0; i < slots.size(); ++i) slots[i].set(kept[i]);
      d->nvec_cap = nvec_cap;
      d->gemm_ws_elems = gemm_ws_elems;
    }
  } swap{d, slots, {}, d->nvec_cap, d->gemm_ws_elems};
  for (WorkSlot& ws : slots) swap.kept.push_back(ws.get());
  for (size_t i = 0; i < slots.size(); ++i) slots[i].set(static_cast<char*>(base) + off[i]);
  d->nvec_cap = nvec;
  d->gemm_ws_elems = gemm_elems;
  return evaluate_launches(h, q, ldq, nvec, phi, ldphi, s);
}

kifmm_status device_stage(kifmm_handle* h, int level, const void* in, void* out, int nvec,
                          hipStream_t s) {
  KIFMM_TRY(device_ready(h, nvec));
  DeviceState* d = h->dev;
  const bool timed = h->timing;
  KIFMM_TRY(m2l_level(h, level, (const double*)in, (double*)out, nvec, s, timed));
  if (timed) {
    // this level's kernel phases; the stream is synchronised first
    hipEvent_t* mark = &d->lev_ev[4 * level];
    KIFMM_HIP(hipEventSynchronize(mark[3]));
    float ph[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < 3; ++k) KIFMM_HIP(hipEventElapsedTime(&ph[k], mark[k], mark[k + 1]));
    for (double& t : h->timings) t = 0.0;
    h->timings[1] = (double)ph[0] + ph[1] + ph[2];
    h->timings[4] = h->timings[1];
    for (int k = 0; k < 3; ++k) h->timings[5 + k] = ph[k];
    h->timings[8] = 1;
  }
  return KIFMM_OK;
}

// Autotuner: each candidate knob setting that applies to the handle's M2L
// form and precision is timed with one warm-up and `reps` untimed evaluates
// (HIP events on s); the setting with the smallest median is kept.
kifmm_status device_autotune(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                             int64_t ldphi, hipStream_t s, int reps, double* best_ms) {
  KIFMM_TRY(check_limits(h, nvec));
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  KIFMM_HIP(hipStreamIsCapturing(s, &cap));
  if (cap != hipStreamCaptureStatusNone) return fail(KIFMM_EINVAL, "autotune on a capturing stream");
  using Knobs = std::array<int32_t, KIFMM_TUNE_COUNT>;
  Knobs base;
  std::copy(h->tune, h->tune + KIFMM_TUNE_COUNT, base.begin());
  std::vector<Knobs> cand;
  if (h->cfg.m2l == KIFMM_M2L_FFT) {
    const int forms = h->cfg.prec == KIFMM_FP64 ? 1 : 2;  // FP64 uses the gather form only
    for (int sched = 0; sched < 2; ++sched)
      for (int form = 0; form < forms; ++form) {
        Knobs c = base;
        c[KIFMM_TUNE_SCHEDULE] = sched;
        c[KIFMM_TUNE_HADAMARD] = form;
        cand.push_back(c);
      }
  } else {
    const int tb_max = std::max(1, 128 / nvec);
    const bool two_forms = h->cfg.m2l == KIFMM_M2L_BLAS && h->op.recompressed && h->cfg.prec != KIFMM_BF16X6;
    for (int form = 0; form < (two_forms ? 2 : 1); ++form) {
      int last = -1;
      for (int k = 0; k < 4; ++k) {
        const int tb = std::max(1, tb_max >> k);
        if (tb == last) continue;
        last = tb;
        Knobs c = base;
        c[KIFMM_TUNE_BLAS_TILE] = tb;
        c[KIFMM_TUNE_BLAS_FORM] = form;
        cand.push_back(c);
      }
    }
  }
  struct Restore {  // events, the timing switch and (on errors) the knobs
    kifmm_handle* h;
    bool timing;
    Knobs knobs;
    bool done = false;
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Restore() {
      h->timing = timing;
      if (!done) std::copy(knobs.begin(), knobs.end(), h->tune);
      for (hipEvent_t ev : e)
        if (ev) (void)hipEventDestroy(ev);
    }
  } guard{h, h->timing, base};
  h->timing = false;
  KIFMM_HIP(hipEventCreate(&guard.e[0]));
  KIFMM_HIP(hipEventCreate(&guard.e[1]));
  double best = 0.0;
  Knobs chosen = base;
  for (size_t i = 0; i < cand.size(); ++i) {
    std::copy(cand[i].begin(), cand[i].end(), h->tune);
    KIFMM_TRY(device_evaluate(h, q, ldq, nvec, phi, ldphi, s));
    std::vector<float> t((size_t)reps);
    for (int r = 0; r < reps; ++r) {
      KIFMM_HIP(hipEventRecord(guard.e[0], s));
      KIFMM_TRY(device_evaluate(h, q, ldq, nvec, phi, ldphi, s));
      KIFMM_HIP(hipEventRecord(guard.e[1], s));
      KIFMM_HIP(hipEventSynchronize(guard.e[1]));
      KIFMM_HIP(hipEventElapsedTime(&t[(size_t)r], guard.e[0], guard.e[1]));
    }
    std::sort(t.begin(), t.end());
    const double med = t[(size_t)reps / 2];
    if (i == 0 || med < best) {
      best = med;
      chosen = cand[i];
    }
  }
  std::copy(chosen.begin(), chosen.end(), h->tune);
  guard.done = true;
  if (best_ms) *best_ms = best;
  return KIFMM_OK;
}

// Levels, lists and maps of a tree built on the device (the leaf set
// changed): everything sized by box counts is reallocated and rebuilt from
// the sorted codes in tb; n[l] = boxes of level l.
kifmm_status rebuild_tree(kifmm_handle* h, const TreeBuild& tb, const std::vector<int64_t>& n,
                          const double* src, const double* tgt, hipStream_t s) {
  DeviceState* d = h->dev;
  Tree& t = h->tree;
  const int depth = t.depth;
  const bool fft = h->cfg.m2l == KIFMM_M2L_FFT;
  KIFMM_TRY(tree_tables(d));
  // the old structures (an evaluate in flight on another stream still reads
  // them: hipFree waits for the device)
  KIFMM_HIP(hipDeviceSynchronize());
  for (DevLevel& D : d->lv) {
    dfree(d, &D.child);
    dfree(d, &D.halo);
    dfree(d, &D.hb_tgt);
    dfree(d, &D.hb_src);
    dfree(d, &D.hb_list);
    dfree(d, &D.hb_tbase);
    dfree(d, &D.tile_box);
    dfree(d, &D.tl_offs);
    dfree(d, &D.tl_t);
    dfree(d, &D.tl_src);
    dfree(d, &D.tile_class);
    dfree(d, &D.tile_src);
    dfree(d, &D.keys);
    dfree(d, &D.parent);
    dfree(d, &D.il_offs);
    dfree(d, &D.il_src);
    dfree(d, &D.il_t);
    D.hb_n = 0;
    D.ntiles = 0;
  }
  dfree(d, &d->src_start);
  dfree(d, &d->src_end);
  dfree(d, &d->tgt_start);
  dfree(d, &d->tgt_end);
  dfree(d, &d->near_offs);
  dfree(d, &d->near_src);
  dfree(d, &d->leaf_centers);
  dfree(d, &d->leaf_keys);
  for (void* p : d->work_allocs) (void)hipFree(p);
  d->work_allocs.clear();
  d->nvec_cap = 0;
  d->xi_hi = d->xi_lo = d->xi_p2 = nullptr;
  d->tile_tb = 0;
  // from here on the handle holds the new tree; its host arrays are filled
  // from the device on demand (refresh_host_tree)
  d->tree_dev = true;
  h->tree_on_device = true;
  h->points_on_device = true;
  for (int l = 0; l <= depth; ++l) {
    Level& L = t.levels[l];
    L = Level();
    L.n = n[l];
    d->lv[l].n = n[l];
  }
  const int64_t nleaf = n[depth];
  // levels: keys, parents, children
  for (int l = 0; l <= depth; ++l) {
    DevLevel& D = d->lv[l];
    KIFMM_TRY(dalloc(d, &D.keys, (size_t)n[l]));
    KIFMM_TRY(dalloc(d, &D.parent, (size_t)n[l]));
    if (l < depth) KIFMM_TRY(dalloc(d, &D.child, (size_t)8 * n[l] + 8));
  }
  for (int l = 0; l <= depth; ++l)
    KIFMM_LAUNCH(tree_level(tb.code[l], tb.parent[l], n[l], l, d->lv[l].keys, d->lv[l].parent,
                            l > 0 ? d->lv[l - 1].child : nullptr, l > 0 ? n[l - 1] : 0, s));
  // leaves: points, ranges, centres, keys
  KIFMM_TRY(dalloc(d, &d->src_start, (size_t)nleaf));
  KIFMM_TRY(dalloc(d, &d->src_end, (size_t)nleaf));
  KIFMM_TRY(dalloc(d, &d->tgt_start, (size_t)nleaf));
  KIFMM_TRY(dalloc(d, &d->tgt_end, (size_t)nleaf));
  KIFMM_TRY(dalloc(d, &d->leaf_centers, (size_t)3 * nleaf));
  KIFMM_TRY(dalloc(d, &d->leaf_keys, (size_t)nleaf));
  KIFMM_TRY(dalloc(d, &d->near_offs, (size_t)nleaf + 1));
  KIFMM_LAUNCH(tree_finish_points(src, tb.code_src, tb.order_src, t.n_src, tb.code[depth], nleaf,
                                  d->src_perm, d->src_xyz, d->src_start, d->src_end, s));
  KIFMM_LAUNCH(tree_finish_points(tgt, tb.code_tgt, tb.order_tgt, t.n_tgt, tb.code[depth], nleaf,
                                  d->tgt_perm, d->tgt_xyz, d->tgt_start, d->tgt_end, s));
  KIFMM_LAUNCH(tree_centers(d->lv[depth].keys, nleaf, depth, t.origin, t.width / std::ldexp(1.0, depth),
                            d->leaf_centers, s));
  KIFMM_HIP(hipMemcpyAsync(d->leaf_keys, d->lv[depth].keys, (size_t)nleaf * sizeof(uint64_t),
                           hipMemcpyDeviceToDevice, s));
  // counts of the lists and the FFT-M2L source blocks
  int64_t nmax = 0;
  for (int l = 0; l <= depth; ++l) nmax = std::max(nmax, n[l]);
  int32_t* flag = nullptr;  // scratch of the block builds (freed at the end, or with the state)
  KIFMM_TRY(dalloc(d, &flag, (size_t)nmax + 1));
  int32_t* tot32 = reinterpret_cast<int32_t*>(d->tree_totals + 40);  // [2][17] int32 past the int64 totals
  for (int l = 2; l <= depth; ++l) {
    DevLevel& D = d->lv[l];
    const DevLevel& U = d->lv[l - 1];
    KIFMM_TRY(dalloc(d, &D.halo, (size_t)kNumDirections * n[l - 1]));
    KIFMM_LAUNCH(tree_halo(U.keys, n[l - 1], l - 1, D.halo, s));
    KIFMM_TRY(dalloc(d, &D.il_offs, (size_t)n[l] + 1));
    KIFMM_LAUNCH(tree_interactions(D.keys, n[l], D.parent, U.keys, n[l - 1], U.child, l, d->tmap,
                                   D.il_offs, d->tree_totals + l, nullptr, nullptr, d->tree_part, s));
    if (fft) {
      KIFMM_TRY(dalloc(d, &D.hb_tgt, (size_t)n[l - 1] + 1));
      KIFMM_TRY(dalloc(d, &D.hb_tbase, (size_t)n[l - 1]));
      KIFMM_LAUNCH(tree_blocks(U.keys, n[l - 1], l - 1, flag, D.hb_tgt, D.hb_tbase, tot32 + l, d->tree_part, s));
    }
  }
  KIFMM_LAUNCH(tree_near(d->lv[depth].keys, nleaf, depth, d->near_offs, d->tree_totals + 20, nullptr,
                         d->tree_part, s));
  int64_t tot[40];
  KIFMM_HIP(hipMemcpyAsync(tot, d->tree_totals, sizeof tot, hipMemcpyDeviceToHost, s));
  int32_t t32[34];
  KIFMM_HIP(hipMemcpyAsync(t32, tot32, sizeof t32, hipMemcpyDeviceToHost, s));
  KIFMM_HIP(hipStreamSynchronize(s));
  // the lists and the block source counts
  for (int l = 2; l <= depth; ++l) {
    DevLevel& D = d->lv[l];
    const DevLevel& U = d->lv[l - 1];
    KIFMM_TRY(dalloc(d, &D.il_src, (size_t)tot[l]));
    KIFMM_TRY(dalloc(d, &D.il_t, (size_t)tot[l]));
    KIFMM_LAUNCH(tree_interactions(D.keys, n[l], D.parent, U.keys, n[l - 1], U.child, l, d->tmap,
                                   D.il_offs, nullptr, D.il_src, D.il_t, d->tree_part, s));
    if (fft) {
      D.hb_n = t32[l];
      KIFMM_TRY(dalloc(d, &D.hb_src, (size_t)D.hb_n + 1));
      KIFMM_LAUNCH(tree_block_lists(U.keys, n[l - 1], l - 1, D.hb_tgt, D.hb_n, flag, D.hb_src,
                                    tot32 + 17 + l, nullptr, d->tree_part, s));
    }
  }
  KIFMM_TRY(dalloc(d, &d->near_src, (size_t)tot[20]));
  KIFMM_LAUNCH(tree_near(d->lv[depth].keys, nleaf, depth, d->near_offs, nullptr, d->near_src,
                         d->tree_part, s));
  if (fft) {
    KIFMM_HIP(hipMemcpyAsync(t32, tot32, sizeof t32, hipMemcpyDeviceToHost, s));
    KIFMM_HIP(hipStreamSynchronize(s));
    for (int l = 2; l <= depth; ++l) {
      DevLevel& D = d->lv[l];
      KIFMM_TRY(dalloc(d, &D.hb_list, (size_t)1 + t32[17 + l]));
      KIFMM_LAUNCH(tree_block_lists(d->lv[l - 1].keys, n[l - 1], l - 1, D.hb_tgt, D.hb_n, nullptr,
                                    D.hb_src, nullptr, D.hb_list, d->tree_part, s));
    }
  }
  KIFMM_HIP(hipStreamSynchronize(s));
  dfree(d, &flag);
  return KIFMM_OK;
}

// Moving points (the dynamic-particle setting of Section 5.1): the tree of
// the new positions over the handle's domain cube is built on the device.
// When the leaves are those of the current tree only the point order and
// the leaves' point ranges change; otherwise the levels, the near and
// interaction lists and the M2L maps are rebuilt on the device.  Nothing
// changes if a point lies outside the domain cube.
kifmm_status device_update_points(kifmm_handle* h, const double* src, const double* tgt,
                                  hipStream_t s) {
  if (!h->dev) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
      return fail(KIFMM_EDEVICE, "no HIP device available");
    if (h->cfg.device < 0 || h->cfg.device >= count)
      return fail(KIFMM_EINVAL, "device ordinal out of range");
    kifmm_status st = upload_all(h);
    if (st != KIFMM_OK) {
      destroy_device(h->dev);
      h->dev = nullptr;
      return st;
    }
  }
  DeviceState* d = h->dev;
  KIFMM_HIP(hipSetDevice(d->device));
  const Tree& t = h->tree;
  const int depth = t.depth;
  const size_t need = tree_scratch_bytes(t.n_src, t.n_tgt, depth);
  if (d->tree_scratch_bytes < need) {
    dfree(d, &d->tree_scratch);
    d->tree_scratch_bytes = 0;
    char* p = nullptr;
    KIFMM_TRY(dalloc(d, &p, need));
    d->tree_scratch = p;
    d->tree_scratch_bytes = need;
  }
  const int64_t n_old = d->lv[depth].n;
  TreeBuild tb;
  KIFMM_LAUNCH(tree_sort_and_levels(src, t.n_src, tgt, t.n_tgt, depth, t.origin, t.width, d->leaf_keys,
                                    n_old, d->tree_scratch, tb, s));
  int32_t cnt[2 + 17];
  KIFMM_HIP(hipMemcpyAsync(cnt, tb.counts, sizeof cnt, hipMemcpyDeviceToHost, s));
  KIFMM_HIP(hipStreamSynchronize(s));
  if (cnt[0]) return fail(KIFMM_ESTATE, "a point lies outside the domain cube; call kifmm_set_points");
  if (cnt[1]) {
    std::vector<int64_t> n(depth + 1);
    for (int l = 0; l <= depth; ++l) n[l] = cnt[2 + l];
    const kifmm_status st = rebuild_tree(h, tb, n, src, tgt, s);
    if (st != KIFMM_OK) {
      // a partly rebuilt tree is not usable: the handle needs new points
      destroy_device(h->dev);
      h->dev = nullptr;
      h->has_points = false;
      h->points_on_device = false;
      h->tree_on_device = false;
    }
    return st;
  }
  // the same leaves: new point order and ranges
  KIFMM_LAUNCH(tree_finish_points(src, tb.code_src, tb.order_src, t.n_src, tb.code[depth], n_old,
                                  d->src_perm, d->src_xyz, d->src_start, d->src_end, s));
  KIFMM_LAUNCH(tree_finish_points(tgt, tb.code_tgt, tb.order_tgt, t.n_tgt, tb.code[depth], n_old,
                                  d->tgt_perm, d->tgt_xyz, d->tgt_start, d->tgt_end, s));
  KIFMM_HIP(hipStreamSynchronize(s));
  h->points_on_device = true;
  return KIFMM_OK;
}

// The host tree from the device after device updates: the point order and
// ranges, and after a rebuild the levels and lists too.
kifmm_status refresh_host_tree(kifmm_handle* h) {
  if ((!h->points_on_device && !h->tree_on_device) || !h->dev) return KIFMM_OK;
  DeviceState* d = h->dev;
  Tree& t = h->tree;
  const int depth = t.depth;
  KIFMM_HIP(hipSetDevice(d->device));
  KIFMM_HIP(hipDeviceSynchronize());
  auto down = [](auto& v, const auto* p, size_t count) -> hipError_t {
    v.resize(count);
    return count ? hipMemcpy(v.data(), p, count * sizeof(v[0]), hipMemcpyDeviceToHost) : hipSuccess;
  };
  const size_t nleaf = (size_t)d->lv[depth].n;
  KIFMM_HIP(down(t.src_perm, d->src_perm, (size_t)t.n_src));
  KIFMM_HIP(down(t.tgt_perm, d->tgt_perm, (size_t)t.n_tgt));
  KIFMM_HIP(down(t.src_sorted, d->src_xyz, (size_t)3 * t.n_src));
  KIFMM_HIP(down(t.tgt_sorted, d->tgt_xyz, (size_t)3 * t.n_tgt));
  KIFMM_HIP(down(t.src_start, d->src_start, nleaf));
  KIFMM_HIP(down(t.src_end, d->src_end, nleaf));
  KIFMM_HIP(down(t.tgt_start, d->tgt_start, nleaf));
  KIFMM_HIP(down(t.tgt_end, d->tgt_end, nleaf));
  if (h->tree_on_device) {
    for (int l = 0; l <= depth; ++l) {
      Level& L = t.levels[l];
      const DevLevel& D = d->lv[l];
      const size_t nl = (size_t)D.n;
      KIFMM_HIP(down(L.keys, D.keys, nl));
      KIFMM_HIP(down(L.parent, D.parent, nl));
      L.anchor.resize(3 * nl);
      for (size_t i = 0; i < nl; ++i) {
        int32_t* a = &L.anchor[3 * i];
        a[0] = a[1] = a[2] = 0;
        for (int b = 0; b < l; ++b)
          for (int k = 0; k < 3; ++k) a[k] |= (int32_t)((L.keys[i] >> (3 * b + k)) & 1) << b;
      }
      if (l < depth) KIFMM_HIP(down(L.child, D.child, 8 * nl));
      if (l >= 2) {
        KIFMM_HIP(down(L.il_offs, D.il_offs, nl + 1));
        KIFMM_HIP(down(L.il_src, D.il_src, (size_t)L.il_offs[nl]));
        KIFMM_HIP(down(L.il_t, D.il_t, (size_t)L.il_offs[nl]));
        const int32_t nc = (int32_t)d->lv[l - 1].n;
        KIFMM_HIP(down(L.halo, D.halo, (size_t)kNumDirections * nc));
        for (int32_t& x : L.halo)
          if (x == nc) x = -1;
      }
    }
    KIFMM_HIP(down(t.near_offs, d->near_offs, nleaf + 1));
    KIFMM_HIP(down(t.near_src, d->near_src, (size_t)t.near_offs[nleaf]));
  }
  h->points_on_device = false;
  h->tree_on_device = false;
  return KIFMM_OK;
}

}  // namespace kifmm
