// Internal declarations of the kiFMM library (host side and kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/kifmm.h"

namespace kifmm {

// ---- error plumbing ------------------------------------------------------
struct Error {
  kifmm_status code;
  std::string msg;
};
void set_error(const std::string& msg);
kifmm_status fail(kifmm_status code, const std::string& msg);

#define KIFMM_HIP(expr)                                                               \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::kifmm::fail(KIFMM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kNumTransfer = 316;   // offsets in [-3,3]^3 with max |t_i| >= 2
constexpr int kNumDirections = 26;  // neighbour directions of a sibling cluster

// ---- tree ---------------------------------------------------------------
struct Level {
  int64_t n = 0;
  std::vector<uint64_t> keys;     // sorted Morton keys
  std::vector<int32_t> anchor;    // [n][3]
  std::vector<int32_t> parent;    // index at level-1 (-1 at level 0)
  std::vector<int32_t> child;     // [n][8] index at level+1 or -1 (empty at the leaf level)
  // interaction lists (level >= 2), CSR over targets
  std::vector<int64_t> il_offs;
  std::vector<int32_t> il_src;
  std::vector<int16_t> il_t;
  // FFT sibling clusters of this level are the boxes of level-1; halo[d][c]
  // is the cluster in direction d of cluster c (or -1)
  std::vector<int32_t> halo;      // [26][n_{level-1}]
};

struct Tree {
  int depth = 0;
  double origin[3] = {0, 0, 0};
  double width = 1.0;
  int64_t n_src = 0, n_tgt = 0;
  std::vector<double> src_sorted, tgt_sorted;  // [n][3] in sorted order
  std::vector<int64_t> src_perm, tgt_perm;     // sorted position -> original index
  std::vector<Level> levels;                   // 0..depth
  std::vector<int32_t> src_start, src_end, tgt_start, tgt_end;  // per leaf
  std::vector<int64_t> near_offs;              // per leaf CSR
  std::vector<int32_t> near_src;
};

// Builds the tree; returns KIFMM_OK or an error (sets message).
kifmm_status build_tree(Tree& t, int depth, const double origin[3], double width, const double* src,
                        int64_t n_src, const double* tgt, int64_t n_tgt);

// Transfer-vector helpers.
int transfer_index(int tx, int ty, int tz);  // -1 if not one of the 316
void transfer_vector(int idx, int t[3]);
void direction_vector(int d, int D[3]);      // 26 directions, lexicographic, 0 skipped

// ---- dense linear algebra (host, FP64) -----------------------------------
// A = U diag(s) V^T for A (m x n) row-major; U (m x r), s (r), V (n x r) with
// r = min(m, n), singular values descending.  One-sided Jacobi.
bool svd(const double* A, int m, int n, std::vector<double>& U, std::vector<double>& s,
         std::vector<double>& V);
// Left singular vectors and values of a wide matrix A (m x n, m << n):
// QR of A^T then an SVD of the small factor.
bool svd_left_wide(const double* A, int m, int n, std::vector<double>& U, std::vector<double>& s);

// ---- operators ------------------------------------------------------------
struct Operators {
  // equivalent surfaces of order p (ns = n_e points), check surfaces of order
  // pc >= p (nc = n_c points; pc = p except for BLAS-M2L with a finer check
  // surface); spectrum length and grid size 2p-1 of the FFT form
  int p = 0, ns = 0, F = 0, n = 0;
  int pc = 0, nc = 0;
  double ai = 1.05, ao = 2.95;
  std::vector<double> surf;         // [ns][3] unit offsets -1 + 2 i/(p-1)
  std::vector<int32_t> lattice;     // [ns][3] integer positions
  std::vector<double> surf_c;       // [nc][3] check-surface offsets -1 + 2 i/(pc-1)
  // pseudo-inverses of K(check, equivalent) of the unit box (width 1),
  // V (ns x r) and Ut (r x nc)
  int r_up = 0, r_down = 0;
  std::vector<double> up_V, up_Ut, down_V, down_Ut;
  // M2M: [nc] x [8 ns] = [K_0 .. K_7] for a parent of width 1
  std::vector<double> m2m;
  // L2L: [8 nc] x [ns] = [L_0; ..; L_7] for a parent of width 1
  std::vector<double> l2l;
  // composite forms for the reduced-precision modes: up_P = up_V up_Ut,
  // down_P = down_V down_Ut (ns x nc), m2m_c = up_P m2m (ns x 8 ns),
  // l2l_c = [down_P L_0; ..; down_P L_7] (8 ns x ns)
  std::vector<double> up_P, down_P, m2m_c, l2l_c;
  // FFT: kernel spectra of the unit box, [316][F] complex (re, im)
  std::vector<double> spectra;
  // BLAS / dense M2L of the unit box: K_t ~ U C_t S^T
  int k = 0;                         // compressed rank (= ns for dense)
  std::vector<double> U;             // nc x k (row-major): decompression
  std::vector<double> S;             // ns x k (row-major): compression (= U when nc = ns)
  std::vector<int> kt;               // per t rank (k when not recompressed)
  std::vector<std::vector<double>> Ubar, Vbarp;  // per t: k x kt (row-major)
  bool recompressed = false;
  bool ready = false;
};

// Compression of K_fat for BLAS-M2L (Section 3.1): the deterministic host
// SVD or the one-shot randomized SVD on the device (kifmm_set_svd).
struct SvdOptions {
  int mode = KIFMM_SVD_DETERMINISTIC;
  int rank = 0;  // target rank; 0 = ceil(ns / 2)
  int oversample = 10;
  uint64_t seed = 0;
  int device = 0;
};
// Leading left singular vectors U (m x r, row-major, r = the target rank)
// and values s of A (m x n, row-major) by a one-shot randomized SVD: the
// products with the long dimension on the device, the small
// factorizations on the host.
kifmm_status rsvd_left_device(const double* A, int m, int n, const SvdOptions& o,
                              std::vector<double>& U, std::vector<double>& s);

kifmm_status precompute_operators(Operators& op, const kifmm_config& cfg, const SvdOptions& svd);

// ---- recorded launches -----------------------------------------------------
// A batch (batch.hip) runs the serial evaluate schedule of many problems as
// grouped launches (kernels.h): with a sink set, the evaluate records every
// launch instead of enqueuing it, with a stage key that orders the launches
// of one problem; launches of several problems with equal keys, kernel
// family and instance are independent and become one grouped launch.
enum LaunchFamily {
  kFamGather = 0, kFamP2M, kFamGemm, kFamGemmReduce, kFamFwd, kFamHad, kFamInv, kFamLeaf,
  kFamSingle  // no grouped form: the recorded launch itself
};
struct LaunchRec {
  int64_t key = 0;
  int family = 0, inst = 0, problem = 0;
  bool side = false;                              // on the near-field branch
  int64_t blocks = 0;
  std::vector<uint8_t> args;                      // the job's argument struct
  std::function<hipError_t(hipStream_t)> single;  // kFamSingle
};
struct LaunchSink {
  std::vector<LaunchRec> recs;
  int problem = 0;
  int64_t phase = 0, level = 0, step = 0;
  // launches recorded while set form a branch beside the others (the near
  // field, which needs only the sorted charges: stage 0 before it, the far
  // field of stage 6 after it)
  bool side = false;
  // stages: 0 charge gather, 1 P2M, 2 leaf pseudo-inverse, 3 M2M (level
  // key 20 - l), 4 FFT-M2L of every level, 5 M2L of other forms and the
  // downward step of level l, 6 leaf evaluation; steps count launches
  void stage(int64_t ph, int64_t lv) {
    phase = ph;
    level = lv;
    step = 0;
  }
  int64_t next_key() { return (phase * 64 + level) * 4096 + step++; }
  template <typename A>
  void add(int family, int inst, const A& a, int64_t blocks) {
    LaunchRec r;
    r.key = next_key();
    r.family = family;
    r.inst = inst;
    r.problem = problem;
    r.side = side;
    r.blocks = blocks;
    r.args.resize(sizeof(A));
    std::memcpy(r.args.data(), &a, sizeof(A));
    recs.push_back(std::move(r));
  }
  void add_single(std::function<hipError_t(hipStream_t)> f) {
    LaunchRec r;
    r.key = next_key();
    r.family = kFamSingle;
    r.problem = problem;
    r.side = side;
    r.single = std::move(f);
    recs.push_back(std::move(r));
  }
};

// ---- device side -------------------------------------------------------------
struct DeviceState;  // defined in device.hip
void destroy_device(DeviceState* d);

}  // namespace kifmm

struct kifmm_handle {
  kifmm_config cfg;
  kifmm::Tree tree;
  kifmm::Operators op;
  bool has_points = false;
  kifmm::DeviceState* dev = nullptr;
  bool timing = false;
  double timings[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  int32_t tune[KIFMM_TUNE_COUNT] = {0, 0, 0, 0, 0};  // autotuning knobs (kifmm.h)
  bool points_on_device = false;  // host copies of the point order are stale
  bool tree_on_device = false;    // host copies of the levels and lists are stale
  kifmm::SvdOptions svd;          // K_fat compression (BLAS-M2L)
  // batches alive that hold this handle: their launches read the handle's
  // device buffers by address, so nothing may free or rebuild them meanwhile
  int32_t batches = 0;
};
