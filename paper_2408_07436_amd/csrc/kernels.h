// Launchers of the gfx950 kernels.  All pointers are device pointers; every
// launcher enqueues on `stream` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kifmm {

// qs[v][i] = q[v * ldq + perm[i]] (gather of charges into sorted order)
hipError_t launch_gather(const void* q, int64_t ldq, const int64_t* perm, int64_t n, int nvec,
                         bool fp64, void* qs, hipStream_t stream);

// P2M check potentials at the leaves (Section 2.1.1):
// phi[leaf][v][i] = sum_{y in leaf} K(c + ar s_i, y) q_y,v  (FP64 result)
hipError_t launch_p2m(const double* src_xyz, const void* qs, bool q_fp64, int64_t n_src,
                      const int32_t* start, const int32_t* end, const double* centers, int64_t n_leaf,
                      const double* surf, double ar, int ns, int nvec, double* phi,
                      hipStream_t stream);

// Leaf evaluation: L2P (FP64) + P2P over the near field (precision of the
// charges), written to the caller's target order.  mode 0: both; mode 1:
// the near field only, phi receives its raw sums (no 1/(4 pi)); mode 2: the
// far field added to the raw sums in phi, finished - 1 then 2 equals 0.
// src_xyz: sorted sources (FP64); leaf_w: the leaf width (the FP32 near
// field refines pairs closer than leaf_w / 16).
hipError_t launch_leaf_eval(const double* tgt_xyz, const double* src_xyz, double leaf_w,
                            const void* qs, bool fp64, int64_t n_src, const int32_t* tstart,
                            const int32_t* tend, const int32_t* sstart, const int32_t* send,
                            const int64_t* near_offs, const int32_t* near_src,
                            const double* centers, int64_t n_leaf, const double* surf, double ar,
                            int ns, const double* local, const int64_t* tgt_perm, void* phi,
                            int64_t ldphi, void* near, int64_t ldnear, int nvec, int mode,
                            hipStream_t stream);

// Grouped forms of the point kernels (see "grouped launches" below).
struct GatherArgs {  // ceil(n / 256) x nvec workgroups
  const void* q; int64_t ldq; const int64_t* perm; int64_t n; int nvec; void* qs;
};
hipError_t launch_gather_group(bool fp64, const GatherArgs* jobs, const int64_t* pre, int nj,
                               int64_t blocks, hipStream_t stream);
struct P2MArgs {  // one workgroup per leaf
  const double* xyz; const void* qs; int64_t n_src; const int32_t* start; const int32_t* end;
  const double* centers; const double* surf; double ar; int ns; int nvec; double* phi;
  int64_t n_leaf;
};
// arguments, kernel instance (element type, check points per lane, vector
// block) and workgroups of launch_p2m
void plan_p2m(const double* src_xyz, const void* qs, bool q_fp64, int64_t n_src, const int32_t* start,
              const int32_t* end, const double* centers, int64_t n_leaf, const double* surf, double ar,
              int ns, int nvec, double* phi, P2MArgs& a, int& inst, int64_t& blocks);
hipError_t launch_p2m_group(int inst, const P2MArgs* jobs, const int64_t* pre, int nj, int64_t blocks,
                            hipStream_t stream);
struct LeafArgs {  // 8 ceil(n_leaf / 8) workgroups (leaves placed by XCD)
  const double* txyz; const double* sxyz; const void* qs; int64_t n_src; const int32_t* tstart;
  const int32_t* tend; const int32_t* sstart; const int32_t* send; const int64_t* near_offs;
  const int32_t* near_src; const double* centers; const double* surf; double ar; int ns;
  const double* local; const int64_t* tgt_perm; void* phi; int64_t ldphi; int nvec; int64_t n_leaf;
  double tau2;
  void* near; int64_t ldnear;  // near-field sums in sorted target order (modes 1 and 2)
};
void plan_leaf_eval(const double* tgt_xyz, const double* src_xyz, double leaf_w, const void* qs,
                    bool fp64, int64_t n_src, const int32_t* tstart, const int32_t* tend,
                    const int32_t* sstart, const int32_t* send, const int64_t* near_offs,
                    const int32_t* near_src, const double* centers, int64_t n_leaf,
                    const double* surf, double ar, int ns, const double* local,
                    const int64_t* tgt_perm, void* phi, int64_t ldphi, void* near, int64_t ldnear,
                    int nvec, int mode, LeafArgs& a, int& inst, int64_t& blocks);
hipError_t launch_leaf_eval_group(int inst, const LeafArgs* jobs, const int64_t* pre, int nj,
                                  int64_t blocks, hipStream_t stream);

// ---- device re-setup for moving points (k_setup.hip) ------------------------
// Codes are Morton codes without the sentinel bit; level keys carry it at
// bit 3 l (the host tree's keys).  Every launcher enqueues on s.  `part`
// is device scratch of kTreeScanPart int64 for the prefix sums (calls on
// one stream may share it).
constexpr int kTreeScanPart = 1024;

// Device results of tree_sort_and_levels (pointers into the scratch):
// sorted leaf codes of the points with the original index of each sorted
// position, the codes of every level's boxes and each box's parent index,
// and counts[]: [0] 1 if a point lies outside the domain cube, [1] 1 if the
// leaf set differs from the given old one, [2 + l] boxes of level l.
struct TreeBuild {
  const uint64_t* code_src = nullptr;
  const int32_t* order_src = nullptr;
  const uint64_t* code_tgt = nullptr;
  const int32_t* order_tgt = nullptr;
  const uint64_t* code[17] = {};
  const int32_t* parent[17] = {};
  int32_t* counts = nullptr;
};
// Bytes of scratch tree_sort_and_levels needs.
size_t tree_scratch_bytes(int64_t n_src, int64_t n_tgt, int depth);
// Leaf codes of the points (domain cube [origin, origin + width]^3, depth
// levels), a stable sort by code (ties keep the input order), the leaves
// (union of the source and target leaves) and their ancestors.
hipError_t tree_sort_and_levels(const double* src, int64_t n_src, const double* tgt, int64_t n_tgt,
                                int depth, const double origin[3], double width,
                                const uint64_t* old_leaf_keys, int64_t n_old, void* scratch,
                                TreeBuild& out, hipStream_t s);
// perm / sorted points in code order and each leaf's range [start, end).
hipError_t tree_finish_points(const double* pts, const uint64_t* code, const int32_t* order, int64_t n,
                              const uint64_t* leaf_code, int64_t n_leaf, int64_t* perm, double* sorted,
                              int32_t* start, int32_t* end, hipStream_t s);
// Keys and parents of level `level` (n boxes) and, when child_up is given,
// the children [8 n_up + 8] of level - 1 (an empty cluster past the end).
hipError_t tree_level(const uint64_t* code, const int32_t* parent, int64_t n, int level,
                      uint64_t* keys, int32_t* parent_out, int32_t* child_up, int64_t n_up,
                      hipStream_t s);
// Leaf centres origin + (anchor + 1/2) w.
hipError_t tree_centers(const uint64_t* keys, int64_t n, int depth, const double origin[3], double w,
                        double* c, hipStream_t s);
// Sibling-cluster halos [26][n] of the boxes of `level` (n where absent).
hipError_t tree_halo(const uint64_t* keys, int64_t n, int level, int32_t* halo, hipStream_t s);
// Interaction lists of level `level` >= 2: with tidx == nullptr, offs[n + 1]
// and *total; else src / tidx (transfer index, tmap over (t + 3) in base 7).
hipError_t tree_interactions(const uint64_t* keys, int64_t n, const int32_t* parent,
                             const uint64_t* keys_up, int64_t n_up, const int32_t* child_up, int level,
                             const int16_t* tmap, int64_t* offs, int64_t* total, int32_t* src,
                             int16_t* tidx, int64_t* part, hipStream_t s);
// Near fields of the leaves: with src == nullptr offs[n + 1] and *total, else src.
hipError_t tree_near(const uint64_t* keys, int64_t n, int depth, int64_t* offs, int64_t* total,
                     int32_t* src, int64_t* part, hipStream_t s);
// FFT-M2L source blocks over the clusters (boxes of `level`): block firsts
// tgt[nblk + 1], tbase[n], counts[0] = nblk (flag: n ints of scratch).
hipError_t tree_blocks(const uint64_t* keys, int64_t n, int level, int32_t* flag, int32_t* tgt,
                       int32_t* tbase, int32_t* counts, int64_t* part, hipStream_t s);
// Block source lists: with list == nullptr src[nblk + 1] and *total (cnt:
// nblk ints of scratch), else list[1 + total].
hipError_t tree_block_lists(const uint64_t* keys, int64_t n, int level, const int32_t* tgt, int64_t nblk,
                            int32_t* cnt, int32_t* src, int32_t* total, int32_t* list, int64_t* part,
                            hipStream_t s);
// Boxes in stable octant-class order (order[n]) and counts[8] per class.
size_t tree_classes_scratch_ints(int64_t n);
hipError_t tree_classes(const uint64_t* keys, int64_t n, int32_t* scratch, int32_t* order,
                        int32_t* counts, int64_t* part, hipStream_t s);
struct TileClasses {
  int32_t start[8];       // first position of class o in the class order
  int32_t count[8];       // boxes of class o
  int64_t first_tile[9];  // first tile of class o; [8] = number of tiles
};
// BLAS / dense target tiles of TB boxes per class: tile_box, tile_class and
// the offsets of the transfer vectors present (present[ntiles * 316 + 1],
// exclusive positions, *total), tvec = the 316 vectors as int8 triples.
hipError_t tree_tiles(const uint64_t* keys, int64_t n, int level, const int32_t* order,
                      const TileClasses& tc, int TB, int64_t ntiles, const int8_t* tvec,
                      int32_t* tile_box, int32_t* tile_class, int64_t* present, int64_t* total,
                      int64_t* part, hipStream_t s);
hipError_t tree_tiles_fill(const uint64_t* keys, int64_t n, int level, const int32_t* tile_box,
                           const int32_t* tile_class, int64_t ntiles, int TB, const int8_t* tvec,
                           const int64_t* pos, int32_t* tl_t, int32_t* tl_src, int64_t* tl_offs,
                           const int32_t* jof, int J, int32_t* tile_src, hipStream_t s);

// FP64 GEMM with gathered columns: C(:, col) = alpha * A * B(:, col) (+ C).
// Columns are (box, v) pairs, col = box * nvec + v.  B's row k of column
// (b, v) lives at B[bb * b_box + v * b_vec + k % ks] with
// bb = bmap ? bmap[b * nsegk + k / ks] : b  (bb < 0 reads zero); C's row m
// of column (b, v) at C[cb * c_box + v * c_vec + m % ms] with
// cb = cmap ? cmap[b * nsegm + m / ms] : b  (cb < 0 is skipped).
// Small grids split K over workgroups when a workspace is given: partials
// of work_elems doubles at most, summed in a fixed order.
// Division by a fixed divisor d >= 1 of numerators below 2^32: multiply-high
// by floor(2^32 / d) and one correction step (set by the launcher).
struct FastDiv {
  uint32_t d = 1, m = 0xffffffffu;
};
struct Gemm64 {
  const double* A; int M; int K; int lda; double alpha;
  const double* B; int ks; int nsegk; const int32_t* bmap; int64_t b_box; int b_vec;
  double* C; int ms; int nsegm; const int32_t* cmap; int64_t c_box; int c_vec;
  int64_t nbox; int nvec; int accumulate;
  double* work = nullptr; int64_t work_elems = 0;
  FastDiv div_ks, div_ms, div_nvec, div_M;  // filled by launch_gemm64
};
hipError_t launch_gemm64(const Gemm64& g, hipStream_t stream);

// ---- grouped launches -------------------------------------------------------
// One launch runs the same kernel for many independent jobs (the problems of
// a batch): job j owns workgroups pre[j] .. pre[j + 1] - 1 of the grid (pre
// is an exclusive prefix sum of the jobs' workgroup counts, in device
// memory, as is the job array), and each workgroup runs exactly what the
// job's own launch would have run in its place, so results are those of
// separate launches.  Jobs whose kernels place work by XCD take multiples
// of 8 workgroups.

// A planned FP64 GEMM: the launch shape launch_gemm64 would use (gx column
// blocks, gy row blocks, split K parts of kchunk each; split == 0: nothing to
// do); the split-K partials go to g.work when split > 1.
struct GemmJob {
  Gemm64 g;
  int64_t gx = 0;
  int gy = 0, split = 0, kchunk = 0;
};
hipError_t plan_gemm64(const Gemm64& g, GemmJob& job);
int64_t gemm64_job_blocks(const GemmJob& j);    // gx * gy * split
int64_t gemm64_reduce_blocks(const GemmJob& j);  // 0 unless split > 1
// reduce = false: the products; true: the split-K sums (jobs with split > 1)
hipError_t launch_gemm64_group(const GemmJob* jobs, const int64_t* pre, int nj, int64_t blocks,
                               bool reduce, hipStream_t stream);
// Largest split-K workspace (doubles) launch_gemm64 uses for any shape:
// only grids of fewer than 512 workgroups are split, into at most
// ceil(512 / workgroups) parts, so parts x columns x rows stays below
// 2 x 512 workgroups x 64 columns x 80 rows.  A workspace of this size
// never limits the split, so the partial sums do not depend on it.
int64_t gemm64_max_work_elems();

// ---- FFT-M2L (Appendix A.1) ----------------------------------------------
// FP32 block-form Hadamard: a block's sources are staged in LDS at the slots
// of their positions in the 6 x 6 x 6 shell around the block's aligned
// 4 x 4 x 4 cube (slot = x + 6 y + 36 z); an LDS row is 16 floats + 16
// bytes of padding, so eight clusters of an aligned 2 x 2 x 2 cube (slots
// congruent to 0, 1, 6, 7, 36, 37, 42, 43 plus a constant) fall on distinct
// 16-byte bank groups modulo 128 bytes.  Member slots run from 43 (shell
// position (1, 1, 1)) to 172, and the per-cluster base offsets are biased
// by kHadSlotBias slots so that every direction's offset is non-negative.
constexpr int kHadRowBytes = 80;
constexpr int kHadShell = 6;
constexpr int kHadSrcSlots = kHadShell * kHadShell * kHadShell;
constexpr int kHadSlotBias = 1 + kHadShell + kHadShell * kHadShell;
// Forward: densities M[box][v][ns] (FP64) of the children of each cluster
// -> spectra Qhat[f][row][8] (complex, T), row = cluster * nvec + v.
// lat2surf[(x p + y) p + z] is the surface index of a lattice point or -1;
// wm is the twiddle matrix Wm[k][j] = exp(-2 pi i (k j mod n) / n), n x p
// complex T.
hipError_t launch_fft_forward(int p, bool fp64, const double* M, const int32_t* child,
                              int64_t n_clusters, int nvec, const int16_t* lat2surf,
                              const void* wm, void* Qhat, hipStream_t stream);
// Hadamard products by sibling cluster: Phat[f][row][i] = sum_d sum_j
// Khat[f][d][i][j] Qhat[f][halo[d][c] * nvec + v][j], row = c * nvec + v.
// Qhat holds n_clusters + 1 clusters per frequency, the last one zero;
// absent neighbours name it.  FP64 gathers through halo; FP32 stages
// source blocks: block b covers clusters [blk_tgt[b], blk_tgt[b + 1]), its
// sources are blk_list[blk_src[b] ...] packed as cluster << 8 | slot
// (blk_list[0] = n_clusters << 8 | 255, the empty cluster at a discard slot), and
// tbase[c] = (slot(c) - kHadSlotBias) * kHadRowBytes, so the neighbour in
// direction D of cluster c sits at byte tbase[c] + (kHadSlotBias + D_x +
// 6 D_y + 36 D_z) * kHadRowBytes.  FP32 work split: units = false gives persistent
// workgroups over contiguous runs of the frequency-major (frequency, block,
// vector) items, true one workgroup per unit of 8 items.
hipError_t launch_hadamard(bool fp64, bool bf16, int F, const void* Khat, const void* Qhat,
                           const int32_t* halo, int64_t n_blocks, const int32_t* blk_tgt,
                           const int32_t* blk_src, const int32_t* blk_list, const int32_t* tbase,
                           int64_t n_clusters, int nvec, bool units, void* Phat,
                           hipStream_t stream);
// Inverse: spectra -> check potentials out[box][v][s] = scale * phi (FP64).
// surf_lat[3 s + k] is lattice coordinate k of surface point s.
hipError_t launch_fft_inverse(int p, bool fp64, const void* Phat, const int32_t* child,
                              int64_t n_clusters, int nvec, const int16_t* surf_lat,
                              const void* wm, double scale, double* out, hipStream_t stream);

// Grouped forms of the FFT-M2L kernels: arguments, kernel instance
// ((fp64 ? 16 : 0) + p) and workgroups of one launch.  A grouped forward
// takes one item group per workgroup (persistent = false); the FP32
// Hadamard of a grouped launch takes one workgroup per frequency (split 2).
struct FwdArgs {
  const double* M; const int32_t* child; int64_t n_rows; int nvec; const int16_t* lat2surf;
  const void* wm; void* Qhat;
};
struct InvArgs {
  const void* Phat; const int32_t* child; int64_t n_rows; int nvec; const int16_t* surf_lat;
  const void* wm; double scale; double* out;
};
struct HadGatherArgs {  // FP64
  const void* Khat; const void* Qhat; const int32_t* halo; int64_t n_c; int nvec; int64_t n_rows;
  int n_chunks; int tiles_per_wave; int64_t total_blocks; void* Phat;
};
struct HadBlockArgs {  // FP32
  const void* Khat; const void* Qhat; const int32_t* blk_tgt; const int32_t* blk_src;
  const int32_t* blk_list; const int32_t* tbase; int n_items; int nvec; int64_t n_rows;
  int64_t total_items; int64_t unit_len; int64_t n_units; int64_t n_wgs; void* Phat;
};
hipError_t plan_fft_forward(int p, bool fp64, const double* M, const int32_t* child, int64_t n_clusters,
                            int nvec, const int16_t* lat2surf, const void* wm, void* Qhat,
                            bool persistent, FwdArgs& a, int& inst, int64_t& blocks);
hipError_t launch_fft_forward_group(int inst, const FwdArgs* jobs, const int64_t* pre, int nj,
                                    int64_t blocks, hipStream_t stream);
hipError_t plan_fft_inverse(int p, bool fp64, const void* Phat, const int32_t* child, int64_t n_clusters,
                            int nvec, const int16_t* surf_lat, const void* wm, double scale, double* out,
                            InvArgs& a, int& inst, int64_t& blocks);
hipError_t launch_fft_inverse_group(int inst, const InvArgs* jobs, const int64_t* pre, int nj,
                                    int64_t blocks, hipStream_t stream);
// fills ab (FP32) or ag (FP64); FP32 work split: 0 persistent runs, 1
// 8-item units, 2 one workgroup per frequency (all its items)
hipError_t plan_hadamard(bool fp64, bool bf16, int F, const void* Khat, const void* Qhat, const int32_t* halo,
                         int64_t n_blocks, const int32_t* blk_tgt, const int32_t* blk_src,
                         const int32_t* blk_list, const int32_t* tbase, int64_t n_clusters, int nvec,
                         int split, void* Phat, HadBlockArgs& ab, HadGatherArgs& ag, int64_t& blocks);
// Kernel instance of a Hadamard launch: 0 = FP32 block form, 1 = FP64
// gather form, 2 = split form (FP32 block form whose products run as BF16
// parts on BF16 MFMA; Khat is then the parts table written by
// launch_hadamard_split_prep).  jobs: HadGatherArgs (1) or HadBlockArgs.
inline int hadamard_inst(bool fp64, bool bf16) { return fp64 ? 1 : bf16 ? 2 : 0; }
hipError_t launch_hadamard_group(int inst, const void* jobs, const int64_t* pre, int nj, int64_t blocks,
                                 hipStream_t stream);
// Split form's B-operand parts of an FP32 kernel-spectrum table Khat
// (F x 26 x 8 x 8 complex): hadamard_split_bytes(F) bytes of BF16 parts.
int64_t hadamard_split_bytes(int F);
hipError_t launch_hadamard_split_prep(const void* Khat, int F, void* parts, hipStream_t stream);

// ---- BLAS-M2L (Section 3.2) -----------------------------------------------
// Fused per-level compressed M2L: out[box][v][0:k] = scale * sum over the
// tile's transfer vectors t of (Ubar_t Vbar'_t^T | C_t) q[src][v][0:kp].
// Tiles hold TB target boxes of one octant class; columns C = TB * nvec
// <= 128.  Operators are packed per t at op_off[t] (see device.hip).
struct BlasM2L {
  const void* q; int kp; int k; int nvec; int TB; int C; int64_t ntiles;
  const int32_t* tile_box;  // [ntiles][TB], -1 padded
  const int64_t* tl_offs;   // [ntiles + 1]
  const int32_t* tl_t;      // [E] transfer-vector index, ascending per tile
  const int32_t* tl_src;    // [E][TB] source box per slot, -1 if none
  const int64_t* op_off;    // [316] element offset of t's operators
  const int32_t* ktp;       // [316] padded rank (two-stage)
  int ktp_max;              // largest ktp (two-stage)
  const int32_t* ktq;       // [316] second-product K steps of 4 to run (FP64 / FP32)
  const void* op_hi;        // FP64 / FP32 operators, or bf16 high parts
  const void* op_lo;        // bf16 low parts
  double* out;
  double scale;
};
// mode 0 FP64, 1 FP32, 2 BF16x3
hipError_t launch_blas_m2l(const BlasM2L& a, int mode, bool two_stage, hipStream_t stream);
// Stacked form of the two-stage BLAS-M2L (Section 3.2 with the per-t
// products regrouped around the boxes).  Boxes are grouped by octant class
// (key & 7); a class serves the same 189 transfer vectors as target and as
// source.  Stage A, per source box sigma of class c:
//     xi[sigma] = [Vbar'_t^T for the 189 t sigma serves, stacked] q~[sigma]
// (Rs rows per box and vector, each t's k_t rows padded to 4 (8 for
// BF16x3)), one GEMM per class over all its boxes.  Stage B, per target box
// tau of class c:
//     out[tau] = [Ubar_t for the 189 t of tau, side by side] . xi-rows of
// the sources tau + t (gathered), one GEMM per class with K = the class's
// stacked rows.  Each (sigma, t) block of xi is read by exactly one target.
// Stage B stages its operator in LDS at most kStackChunk K steps at a time.
constexpr int kStackChunk = 8;
struct BlasStack {
  int mode;                   // 0 FP64, 1 FP32, 2 BF16x3, 3 BF16x6 (three BF16 parts)
  int k, kp;                  // compressed rank; padded (K of Stage A, M of Stage B)
  int nvec, TB, C;            // vectors, boxes per tile, columns per tile (TB * nvec <= 128)
  int64_t ntiles;
  const int32_t* tile_box;    // [ntiles][TB], -1 padded
  const int32_t* tile_class;  // [ntiles] octant class of the tile's boxes
  const int32_t* tile_src;    // [ntiles][J][TB] source box of transfer vector j, -1 if none
  int J;                      // transfer vectors per class (189)
  int Rs;                     // xi rows per (box, vector)
  int Rpad;                   // Stage A operator rows per class (Rs rounded up to 128)
  int nsteps;                 // Stage B K steps per class (4 rows; 32 for BF16x3)
  int rbo;                    // Stage B operator row blocks of 16 (kp / 16)
  const void* A_hi;           // Stage A operators [8][Rpad][kp] (BF16 parts: first)
  const void* A_lo;           //   BF16 parts: second
  const void* B_hi;           // Stage B operators in MFMA lane order (see device.hip)
  const void* B_lo;
  const int32_t* info;        // [8][groups][2]: (j, first xi row) per row group of Stage B's K
  const void* q_hi;           // padded compressed multipoles [box][v][kp] (BF16 parts: first)
  const void* q_lo;           //   BF16 parts: second
  void* xi_hi;                // [box][Rs][v] (BF16 parts: [box][Rs / 8][v][8], first)
  void* xi_lo;                //   BF16 parts: second
  const void* A_p2 = nullptr;  // BF16x6: third parts of A, B, q and xi
  const void* B_p2 = nullptr;
  const void* q_p2 = nullptr;
  void* xi_p2 = nullptr;
  double* out;                // [box][v][k]
  double scale;
  // Stage B's K steps split over ksplit workgroups per tile (levels with
  // few tiles): each writes its raw sums to partial[part][box][v][k], and a
  // reduction adds the parts in order, scales and writes out
  int ksplit = 1;
  int64_t n_boxes = 0;        // boxes of the level (partial's box extent)
  double* partial = nullptr;
};
hipError_t launch_blas_stacked(const BlasStack& a, hipStream_t stream);
// q~ [col][k] FP64 -> [col][kp] zero-padded bf16 parts: high and low (p2
// null), or the three parts of the BF16x6 mode
hipError_t launch_pad_split(const double* in, int k, int64_t ncols, int kp, void* hi, void* lo, void* p2,
                            hipStream_t stream);
// q~ [col][k] FP64 -> [col][kp] zero-padded, FP64 or FP32
hipError_t launch_pad_convert(const double* in, int k, int64_t ncols, int kp, bool fp64, void* out,
                              hipStream_t stream);

}  // namespace kifmm
