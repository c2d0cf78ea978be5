/*
 * kifmm.h - C ABI of the MI355X (gfx950) kernel-independent FMM library.
 *
 * The library evaluates potentials phi_i = sum_j K(x_i, y_j) q_j of the 3D
 * Laplace kernel K(x, y) = 1 / (4 pi |x - y|) (the N-body sum and kernel of
 * Section 1 of arXiv 2408.07436) with the kernel-independent FMM on a pruned
 * uniform octree (Section 2), and applies the multipole-to-local (M2L)
 * translation in one of three forms:
 *   KIFMM_M2L_DENSE - the uncompressed M2L matvec of Section 2.2,
 *   KIFMM_M2L_FFT   - the convolution form (Appendix A.1-A.2) on a grid of
 *                     2P-1 points per axis, Hadamard products grouped by
 *                     sibling cluster,
 *   KIFMM_M2L_BLAS  - SVD-compressed operators with directional
 *                     recompression (Section 3.1-3.2).
 *
 * Workflow (the paper's setup / runtime split, Section 4 and Section 5.1):
 *   kifmm_create -> kifmm_set_points -> kifmm_precompute -> kifmm_evaluate*
 *   -> kifmm_destroy.
 * create, set_points, precompute and the introspection calls run on the host
 * only (no GPU is touched).  The first evaluate or stage call uploads the
 * tree and operators to the device selected in the config.
 *
 * Conventions (fixed here because the paper leaves them open):
 *   - Domain: cube [origin, origin + width]^3; width <= 0 selects the
 *     tightest cube around all points, centred on their bounding box.
 *     A point x lies in the leaf with anchor
 *     a = min(floor((x - origin) / width * 2^depth), 2^depth - 1) per axis.
 *   - Morton key of a box with anchor a at level l: bit b of a_x at bit 3b,
 *     of a_y at 3b+1, of a_z at 3b+2, plus a sentinel bit 3l.  parent =
 *     key >> 3, octant = key & 7.  Points are ordered by (leaf key, index).
 *   - Boxes at a level are the ancestors of non-empty leaves, ascending key.
 *   - Interaction list of a box at level l >= 2: boxes of the level whose
 *     parent is adjacent to (or is) the box's parent, minus the box's own
 *     3x3x3 neighbourhood; ascending source key.  Transfer vector
 *     t = anchor(source) - anchor(target), index = rank of t in
 *     lexicographic (tx, ty, tz) order over the 316 offsets of [-3,3]^3
 *     with max |t_i| >= 2 (Section 3.1).
 *   - Surfaces of order p: c + alpha r (-1 + 2 i/(p-1)), i in [0,p-1]^3 on
 *     the lattice boundary, i_x slowest; 6(p-1)^2 + 2 points (Appendix A.3).
 *     Upward-equivalent and downward-check surfaces use alpha_inner,
 *     upward-check and downward-equivalent surfaces alpha_outer.
 *   - Self term (the paper takes sources equal to targets, Section 4, and
 *     does not say what K is at r = 0): K(x, y) = 0 for coincident points.
 *     The kernels zero a pair when |x - y|^2, formed in the working
 *     precision, is below that precision's smallest normal number; bitwise-
 *     equal points always are.  Distinct points are zeroed only when their
 *     separation is below what the working precision resolves: about
 *     1.5e-154 in FP64, and in the FP32 near field (which forms separations
 *     from FP64 offsets to the target leaf's centre) about 1e-16 times the
 *     domain width.
 *   - Pseudo-inverses keep singular values > max(M,N) * 2^-52 * sigma_0 and
 *     are applied as two FP64 factors V (Sigma^-1 U^T) (Section 2.1.1).
 *   - The M2L and L2L check potentials of a box are summed before its
 *     check-to-equivalent pseudo-inverse is applied once.
 *
 * Errors: every call returns a kifmm_status and never aborts; the message
 * of the last failure on the calling thread is kifmm_last_error().
 * A handle is not thread-safe; use one handle per host thread.
 */
#ifndef KIFMM_H
#define KIFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kifmm_handle kifmm_handle;

typedef enum {
  KIFMM_OK = 0,
  KIFMM_EINVAL = 1,       /* bad argument: null pointer, bad size, point outside domain */
  KIFMM_ESTATE = 2,       /* call out of order (e.g. evaluate before precompute) */
  KIFMM_ENOMEM = 3,       /* host or device allocation failed */
  KIFMM_EDEVICE = 4,      /* HIP runtime error (no device, launch failure) */
  KIFMM_EUNSUPPORTED = 5, /* valid but unsupported combination */
  KIFMM_ENUMERIC = 6      /* SVD failed to converge */
} kifmm_status;

typedef enum { KIFMM_M2L_DENSE = 0, KIFMM_M2L_FFT = 1, KIFMM_M2L_BLAS = 2 } kifmm_m2l;

/* Arithmetic of the M2L step.  P2M, M2M, L2L, the pseudo-inverses, L2P and
 * the accumulation of check potentials and local expansions are FP64 in
 * every mode; P2P runs in the precision of the charges.
 *   KIFMM_FP64   - charges/potentials double; M2L in FP64.
 *   KIFMM_FP32   - charges/potentials float; M2L in FP32 (FFT: FP32 complex
 *                  transforms and Hadamard products - by default as three
 *                  BF16 parts per FP32 value on BF16 MFMA, FP32-class
 *                  rounding, see KIFMM_TUNE_PRODUCTS; BLAS/DENSE: FP32 GEMMs).
 *   KIFMM_BF16X3 - charges/potentials float; BLAS/DENSE M2L GEMMs on bf16
 *                  MFMA with hi+lo split operands (a = hi + lo, products
 *                  hi*hi + hi*lo + lo*hi, FP32 accumulation); FFT M2L as FP32.
 *   KIFMM_BF16X6 - charges/potentials float; BLAS-M2L with directional
 *                  recompression (Section 3.2's two products per transfer
 *                  vector, stacked form) on bf16 MFMA with three-part split
 *                  operands (a = a0 + a1 + a2, the six products of order at
 *                  most two, FP32 accumulation): FP32-class rounding.  Other
 *                  M2L forms, and BLAS-M2L without recompression, are
 *                  refused (EUNSUPPORTED at kifmm_create / kifmm_precompute). */
typedef enum { KIFMM_FP64 = 0, KIFMM_FP32 = 1, KIFMM_BF16X3 = 2, KIFMM_BF16X6 = 3 } kifmm_prec;

typedef struct {
  uint32_t size;            /* sizeof(kifmm_config), for ABI versioning */
  int32_t order;            /* expansion order p >= 2 (points per surface edge) */
  int32_t depth;            /* uniform leaf depth, 2..16 */
  int32_t m2l;              /* kifmm_m2l */
  int32_t prec;             /* kifmm_prec */
  int32_t device;           /* HIP device ordinal used by evaluate */
  double svd_rel_tol;       /* BLAS: keep sigma_i(K_fat) > tol * sigma_0; 0 = full rank */
  double svd_rel_tol_dir;   /* BLAS: keep sigma_i(C_t) > tol * sigma_0(C_t); < 0 = no recompression */
  double alpha_inner;       /* 0 selects 1.05 */
  double alpha_outer;       /* 0 selects 2.95 */
  double origin[3];         /* lower corner of the domain cube */
  double width;             /* side of the domain cube; <= 0 selects the tight cube */
  int32_t check_order;      /* P_c, order of both check surfaces; 0 = order.  Above order
                               (more check than equivalent points, Section 5.1; the P_e and
                               P_c columns of Section 4's BLAS-M2L parameter table) for
                               KIFMM_M2L_BLAS only: the convolution form needs equal
                               orders.  Check-side arrays then have n_c = 6 (P_c - 1)^2 + 2
                               points, equivalent-side ones n_s = 6 (P_e - 1)^2 + 2, and the
                               compressed rank k is at most n_s. */
} kifmm_config;

/* Fill *cfg with defaults: p = 6, depth = 4, FFT, FP64, tolerances 0 / -1,
 * alpha 1.05 / 2.95, origin 0, width 1, device 0.  The parameters are those
 * of the paper's runtime tables (expansion order P, tree depth, M2L form,
 * precision; Section 4). */
void kifmm_config_default(kifmm_config* cfg);

/* Create a handle for one FMM configuration: the parameters of Section 4's
 * setup (order, depth, M2L form of Section 2.2 / 3 / Appendix A, precision),
 * nothing computed yet.  Validates the config (EINVAL: order < 2, depth
 * outside 2..16, unknown m2l/prec, 0 < check_order < order; EUNSUPPORTED:
 * BF16X3 with FFT, FFT with order > 8, check_order > order without
 * BLAS-M2L).  *out receives the handle, owned by the caller until
 * kifmm_destroy. */
kifmm_status kifmm_create(const kifmm_config* cfg, kifmm_handle** out);

/* Build the tree and all lists from host positions src[n_src][3] and
 * tgt[n_tgt][3] (row-major doubles; copied): the uniform octree with
 * empty branches pruned, near fields and interaction lists of Section 2
 * and the transfer-vector index of Section 3.1.  tgt may equal src.
 * EINVAL: null pointers, n <= 0, or a point outside the domain cube.
 * ESTATE: a batch holds the handle. */
kifmm_status kifmm_set_points(kifmm_handle* h, const double* src, int64_t n_src,
                              const double* tgt, int64_t n_tgt);

/* Compute all operators in FP64 on the host: pseudo-inverse factors, M2M
 * and L2L kernel matrices, and the M2L operators of the selected form.
 * Depends only on the configuration (Section 5.1): pseudo-inverses of
 * Section 2.1.1, kernel spectra of Appendix A.1 or the compressed
 * operators of Section 3.1.  Idempotent.
 * ENUMERIC: an SVD did not converge; ESTATE: a batch holds the handle. */
kifmm_status kifmm_precompute(kifmm_handle* h);

/* Compression of K_fat = [K_1 .. K_316] (n_s x 316 n_s) for BLAS-M2L
 * (Section 3.1).
 *   KIFMM_SVD_DETERMINISTIC (default) - host SVD: Householder QR of K_fat^T,
 *     then a Jacobi SVD of the triangular factor.
 *   KIFMM_SVD_RANDOMIZED - the one-shot randomized SVD the paper uses for
 *     setup (Section 3.1, after Halko, Martinsson and Tropp): no power
 *     iterations, only oversampling and a rank estimate.  With l = rank +
 *     oversample (at most n_s): Omega (316 n_s x l) of standard normal
 *     numbers (Philox4x32-10 keyed by `seed`, counter = pair index,
 *     Box-Muller), Y = K_fat Omega, Q an orthonormal basis of Y, B = Q^T
 *     K_fat, the SVD of B from the eigen-decomposition of B B^T, and the
 *     left vectors Q times those of B.  The three products with the long
 *     dimension run on the handle's device (FP64 MFMA); the factorizations of
 *     the small matrices on the host.  The basis keeps at most `rank`
 *     vectors (those above svd_rel_tol, as in the deterministic mode); rank
 *     0 selects ceil(n_s / 2), the paper's rank estimate for the Laplace
 *     kernel.  Forming B B^T squares the singular values, so those below
 *     about 1e-8 sigma_0 are not resolved.
 * Applies to BLAS-M2L only (other forms ignore it).  Call before
 * kifmm_precompute.  Operators are cached per configuration and SVD setting.
 * EINVAL: null handle, unknown mode, rank < 0 or oversample < 0.
 * ESTATE: after kifmm_precompute.  At precompute: ENOMEM / EDEVICE if the
 * device buffers (about 4 x 8 n_s x 316 n_s bytes + 64 MiB) or products fail. */
typedef enum { KIFMM_SVD_DETERMINISTIC = 0, KIFMM_SVD_RANDOMIZED = 1 } kifmm_svd;
kifmm_status kifmm_set_svd(kifmm_handle* h, int32_t mode, int32_t rank, int32_t oversample,
                           uint64_t seed);

/* Evaluate potentials phi_i = sum_j K(x_i, y_j) q_j (Section 1) with the
 * FMM passes of Section 2 (upward P2M / M2M, downward M2L / L2L, leaf L2P
 * and P2P), for n_vec charge vectors through the same launches (the
 * multiple right-hand sides of Section 3.2), asynchronously on hip_stream
 * (a hipStream_t; NULL = default stream).  q_dev holds n_vec charge vectors,
 * column-major [n_vec][ldq] in the caller's source order; phi_dev receives
 * [n_vec][ldphi] in the caller's target order (overwritten).  Element type
 * is double for KIFMM_FP64 and float otherwise; both are device pointers
 * owned by the caller.  ldq >= n_src, ldphi >= n_tgt, n_vec >= 1.
 * ESTATE: called before set_points / precompute, or a batch holds the
 * handle and this call needs more vectors than the batch's (or other knobs).
 * EUNSUPPORTED: n_vec above a kernel limit (BLAS / dense: 128; FFT: the
 * spectra of a level, clusters x n_vec x 128 bytes, must stay below 4 GiB),
 * checked before anything is enqueued.  EDEVICE: HIP error. */
kifmm_status kifmm_evaluate(kifmm_handle* h, const void* q_dev, int64_t ldq, int32_t n_vec,
                            void* phi_dev, int64_t ldphi, void* hip_stream);

/* Size in bytes of the device array kifmm_evaluate_noalloc takes its work
 * buffers from (256 MiB), held on each device the library runs on until the
 * process ends. */
#define KIFMM_NOALLOC_SCRATCH_BYTES (256LL << 20)

/* kifmm_evaluate without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, serving loops and harnesses that
 * forbid hipMalloc.  Arguments, layouts, results and errors as
 * kifmm_evaluate: the same kernels in the same schedule on the same inputs,
 * so the potentials are those kifmm_evaluate returns.  The per-evaluate work
 * buffers (sorted charges, multipoles and locals per level, check
 * potentials, GEMM intermediates and split-K partials, FFT spectra, padded
 * compressed multipoles) come from one fixed device array of
 * KIFMM_NOALLOC_SCRATCH_BYTES per device instead of buffers the handle
 * allocates; the call calls no hipMalloc, hipFree or allocating library
 * routine.  Every call on one device shares that device's array, which keeps
 * the last call's contents; the evaluate writes every entry before it reads
 * it, so nothing needs to start at zero.  Calls that overlap on one device
 * (several streams or host threads, or a captured graph replayed while
 * another call runs) race on the array: the caller serialises them.
 * ESTATE (nothing enqueued): the handle's tree and operators are not on the
 * device yet - one kifmm_evaluate, kifmm_stage or kifmm_update_points places
 * them there - or, for BLAS / dense M2L, the target tiles were last built
 * for another tile width (128 / n_vec or the tuning knob; one kifmm_evaluate
 * with this n_vec rebuilds them).  EINVAL: as kifmm_evaluate, or this
 * problem's work buffers (40 MiB of split-K partials included) exceed the
 * array; the message gives both sizes.  At p = 6 in FP32 an FFT-M2L problem
 * of about 1e5 points at depth 4 with one vector fits. */
kifmm_status kifmm_evaluate_noalloc(kifmm_handle* h, const void* q_dev, int64_t ldq,
                                    int32_t n_vec, void* phi_dev, int64_t ldphi,
                                    void* hip_stream);

/* Release the handle and all device memory it owns: what the setup of
 * Section 5.1 built (tree, buffers and index pointers, maps, precomputed
 * operators).  NULL is accepted.  ESTATE (nothing released): a batch holds
 * the handle. */
kifmm_status kifmm_destroy(kifmm_handle* h);

/* Message of the last failed call on this thread ("" if none); the
 * library's own error report, not a passage of the paper. */
const char* kifmm_last_error(void);

/* ---- introspection (host only, valid after set_points) ----------------
 * The tree and lists of Section 2 (boxes, near fields, interaction lists)
 * and the operators of Sections 2.1.1, 3.1 and Appendix A.1, for checks. */

/* Number of boxes at a level (0..depth). */
kifmm_status kifmm_num_boxes(const kifmm_handle* h, int32_t level, int64_t* n);
/* Sorted Morton keys of the boxes of a level; cap = capacity of keys. */
kifmm_status kifmm_box_keys(const kifmm_handle* h, int32_t level, uint64_t* keys, int64_t cap);
/* Sorting permutation: sorted position i holds original point perm[i].
 * which = 0 for sources, 1 for targets. */
kifmm_status kifmm_point_perm(const kifmm_handle* h, int32_t which, int64_t* perm, int64_t cap);
/* Interaction lists of level >= 2 in CSR form: offs[n_boxes + 1], source box
 * indices src[offs[n]] and transfer-vector indices tidx[offs[n]].  Passing
 * NULL arrays returns only the total count in *n_pairs. */
kifmm_status kifmm_interactions(const kifmm_handle* h, int32_t level, int64_t* offs,
                                int64_t* src, int32_t* tidx, int64_t cap, int64_t* n_pairs);
/* Near-field (P2P) lists of the leaves in CSR form, like kifmm_interactions. */
kifmm_status kifmm_near(const kifmm_handle* h, int64_t* offs, int64_t* src, int64_t cap,
                        int64_t* n_pairs);

/* Host FP64 operators (valid after precompute), for checks.  which:
 *   0 KIFMM_OP_UP_PINV_V, 1 KIFMM_OP_UP_PINV_UT, 2 KIFMM_OP_DOWN_PINV_V,
 *   3 KIFMM_OP_DOWN_PINV_UT (unit box, level scale applied by the library),
 *   4 KIFMM_OP_FFT_SPECTRA: kernel spectra of the unit box, [316][F] complex
 *     as interleaved (re, im) doubles with F = n^2 (n/2 + 1), n = 2p - 1,
 *     ordered [kx][ky][kz], kz fastest.  Convolution grid (Appendix A.1):
 *     n = 2p - 1 points per axis (enough for the circular convolution not
 *     to wrap; the paper pads to 2p), kernel value K(c_tau - c_sigma + h m)
 *     at index m mod n for m in [-(p-1), p-1]^3, densities at their lattice
 *     positions;
 *   5 KIFMM_OP_BLAS_U: U (n_c x k, row-major), 6 KIFMM_OP_BLAS_RANKS: k then
 *     k_t for the 316 transfer vectors (as doubles), 7 KIFMM_OP_BLAS_APPLIED:
 *     the applied operator U Ubar_t Vbar'_t^T S^T of every t, [316][n_c][n_s],
 *     for the unit box (n_c = n_s unless check_order > order).  The pseudo-
 *     inverse factors are V (n_s x r) and Ut (r x n_c).
 * *n receives the element count; out may be NULL to query it. */
kifmm_status kifmm_operator(const kifmm_handle* h, int32_t which, double* out, int64_t cap,
                            int64_t* n);

/* ---- stages and timings (device) ---------------------------------------- */

/* The M2L of one level (Section 2.2: check potentials of every target box
 * from the multipoles of its interaction list; in the configured form,
 * Appendix A.1 or Section 3.2) on caller device buffers, asynchronously:
 * in_dev = upward-equivalent densities [n_boxes(level)][n_vec][n_s] (double,
 * boxes in key order), out_dev = M2L check potentials
 * [n_boxes(level)][n_vec][n_c] (double, overwritten; n_c = n_s unless
 * check_order > order).  Uses the configured M2L form and precision.  stage must be
 * KIFMM_STAGE_M2L (0).  The buffers must hold every box of the level
 * (kifmm_num_boxes); the call cannot check their size.  EINVAL: level
 * outside 2..depth, null buffers; EUNSUPPORTED: as kifmm_evaluate. */
kifmm_status kifmm_stage(kifmm_handle* h, int32_t stage, int32_t level, const void* in_dev,
                         void* out_dev, int32_t n_vec, void* hip_stream);

/* Enable (1) or disable (0) timing of evaluate and stage with HIP events
 * recorded between kernels (the per-phase times T_FMM, T_M2L, T_P2P the
 * paper reports in Section 4's runtime tables).  A timed call synchronises
 * before it returns. */
kifmm_status kifmm_set_timing(kifmm_handle* h, int32_t on);
/* Milliseconds of the last timed evaluate or stage (cap >= 5; more entries
 * are filled when cap allows, up to 12).  An untimed FFT-M2L evaluate runs
 * as a dependency graph over several streams (near field beside the FMM
 * passes, coarse levels beside the leaf level); a timed one runs the
 * phases one after another (the M2L levels still concurrently) so that each
 * phase is measured on its own: [0] upward (P2M + M2M), [1] M2L (all
 * levels; FFT: wall time of the concurrent levels), [2] rest of the
 * downward pass (L2L + pseudo-inverses), [3] leaves (L2P + P2P), [4] total,
 * [5] M2L first kernel summed over levels (FFT: forward transform;
 * BLAS/dense: compression), [6] M2L main kernel (FFT: Hadamard; BLAS/dense:
 * per-transfer-vector products), [7] M2L last kernel (FFT: inverse
 * transform; BLAS: decompression), [8] number of M2L levels, [9] near-field
 * pass (P2P) and [10] far-field pass (L2P) of FFT evaluates (0 otherwise),
 * [11] the P2M kernel (leaf check potentials, part of [0]).
 * [5..7] are each kernel's own start-to-end times and overlap when levels
 * run concurrently.  After a timed stage: [1] = [4] = the level's M2L,
 * [5..7] its three kernels, [8] = 1, the rest 0. */
kifmm_status kifmm_timings(const kifmm_handle* h, double* ms, int32_t cap);

/* Work counts of one M2L level (>= 2; the M2L pairs of Section 2.2 and the
 * sibling-cluster pairs of Appendix A.2), valid after set_points: [0] target
 * boxes, [1] M2L box pairs, [2] sibling clusters (boxes of level-1),
 * [3] (target cluster, existing source cluster) pairs over the 26-cluster
 * halos.  cap >= 4. */
kifmm_status kifmm_m2l_counts(const kifmm_handle* h, int32_t level, int64_t* counts, int32_t cap);

/* ---- moving points --------------------------------------------------------- */

/* Re-setup for points that move between evaluates (the dynamic-particle
 * setting of Section 5.1, where the locational encoding, the index pointers
 * and the M2L maps are rebuilt each step; Tables 5-6 list that setup cost
 * as Tree and Map Creation), on the device: the new positions
 * src_dev[n_src][3] and tgt_dev[n_tgt][3] (device memory, FP64, row-major,
 * the counts of kifmm_set_points; tgt_dev may equal src_dev; they must not
 * be buffers the library returned) get their leaf codes in the handle's
 * domain cube and are sorted on the GPU, stably by leaf (Morton order) and
 * then by index.  If the leaves are those of the current tree, only the
 * point order and the leaves' point ranges change.  Otherwise the tree is
 * rebuilt on the device: the levels (ancestors of the non-empty leaves),
 * parents and children, the near lists, the interaction lists with their
 * transfer vectors (Section 2), the sibling-cluster halos and source blocks
 * of FFT-M2L (Appendix A) and, at the next evaluate, the target tiles of
 * BLAS / dense M2L with the transfer vectors present (Section 3.2, Step 1);
 * the work buffers sized by box counts are reallocated.  Every structure,
 * and so the potentials, equals that of kifmm_set_points with the same
 * positions and the handle's domain cube (origin and width as resolved at
 * set_points); box_keys, interactions, near and point_perm read the
 * device's tree.  The operators are kept.  The buffers are read on
 * hip_stream; the call synchronises the device.  ESTATE: no points or
 * operators yet, a batch holds the handle, or some point lies outside the
 * domain cube (then nothing has changed).  EINVAL: null arguments.
 * ENOMEM / EDEVICE during a rebuild leave the handle without points
 * (kifmm_set_points is needed). */
kifmm_status kifmm_update_points(kifmm_handle* h, const void* src_dev, const void* tgt_dev,
                                 void* hip_stream);

/* ---- autotuning ---------------------------------------------------------- */

/* Knobs of the evaluate's schedule and tile shapes (int32; 0 = built-in
 * default).  The paper tunes its CPU kernels by hand (the batch size of
 * Appendix A.2, the parameter search of Section 4); these knobs are this
 * library's own launch shapes.  Settings of the first three knobs give
 * bit-identical potentials; the two BLAS-M2L forms sum the same products in
 * different orders (results agree to rounding).
 *   [KIFMM_TUNE_BLAS_TILE] BLAS / dense M2L: target boxes per tile.  A tile's
 *       MFMA columns are its boxes x n_vec, at most 128; larger values are
 *       clamped to 128 / n_vec.  0 = 128 / n_vec.  Range 0..128.
 *   [KIFMM_TUNE_SCHEDULE] FFT-M2L evaluates that are not timed and not under
 *       stream capture: 0 = the FMM passes as a dependency graph over several
 *       streams (the M2L of each level beside the others), 1 = every pass
 *       back to back on the caller's stream.
 *   [KIFMM_TUNE_HADAMARD] FP32 FFT-M2L Hadamard: 0 = persistent workgroups,
 *       one device-full, each over one contiguous run of the frequency-major
 *       (frequency, block, vector) items; 1 = one workgroup per unit of 8
 *       consecutive items.
 *   [KIFMM_TUNE_BLAS_FORM] BLAS-M2L with directional recompression (Section
 *       3.1-3.2: phi~ = sum_t Ubar_t Vbar'_t^T q~): 0 = stacked, two GEMM
 *       kernels per level over octant classes - Stage A forms Vbar'_t^T q~
 *       of every source box for all 189 transfer vectors its class serves
 *       (kept in device memory, about 4 sum_t k_t bytes per box and vector
 *       in FP32, twice that in FP64), Stage B sums Ubar_t times those blocks
 *       per target box; 1 = fused, one kernel per level that gathers q~ per
 *       target tile and transfer vector and keeps Vbar'_t^T q~ in registers
 *       (no intermediate in memory).  Other M2L forms ignore it.
 *   [KIFMM_TUNE_PRODUCTS] FP32 FFT-M2L Hadamard products (Appendix A.2's
 *       complex multiply-adds in single precision): 0 = every FP32 operand
 *       value split into three BF16 parts (x0 = bf16(x), x1 = bf16(x - x0),
 *       x2 = bf16(x - x0 - x1)) and each product taken as the six part
 *       products of order at most two, summed in FP32 on BF16 MFMA (the
 *       dropped terms lie below 2^-24 of the product, so the sums carry an
 *       FP32 product's rounding error); 1 = FP32 MFMA.  The two agree to
 *       FP32 rounding, not bit for bit. */
enum {
  KIFMM_TUNE_BLAS_TILE = 0,
  KIFMM_TUNE_SCHEDULE = 1,
  KIFMM_TUNE_HADAMARD = 2,
  KIFMM_TUNE_BLAS_FORM = 3,
  KIFMM_TUNE_PRODUCTS = 4,
  KIFMM_TUNE_COUNT = 5
};
/* Current knob values into knobs[0 .. KIFMM_TUNE_COUNT); cap >= KIFMM_TUNE_COUNT.
 * Host only. */
/* Current knobs (KIFMM_TUNE_COUNT values; cap >= KIFMM_TUNE_COUNT): the
 * launch-shape counterparts of the CPU parameters the paper tunes (the
 * batch size of Appendix A.2, Section 4's parameter search). */
kifmm_status kifmm_get_tuning(const kifmm_handle* h, int32_t* knobs, int32_t cap);
/* Set the first n knobs (n <= KIFMM_TUNE_COUNT); EINVAL (nothing changed) if a
 * value is out of range; ESTATE if a batch holds the handle and a value
 * changes.  Host only; takes effect at the next evaluate. */
kifmm_status kifmm_set_tuning(kifmm_handle* h, const int32_t* knobs, int32_t n);
/* Autotuner: times every candidate setting that applies to the handle's M2L
 * form and precision (FFT: schedule x Hadamard form for FP32, schedule for
 * FP64; BLAS / dense: four tile widths, times the two forms for BLAS-M2L
 * with directional recompression) with one warm-up and `reps` (1..100)
 * evaluates of the given charges (arguments as in kifmm_evaluate), keeps
 * the setting with the smallest median evaluate time, and writes that time
 * to *best_ms (if not NULL).  phi_dev holds the last evaluate's potentials.
 * Runs untimed whatever kifmm_set_timing says; synchronises hip_stream.
 * On an error the knobs are left as they were.
 * EINVAL: bad arguments or a capturing stream; ESTATE: as evaluate, or a
 * batch holds the handle. */
kifmm_status kifmm_autotune(kifmm_handle* h, const void* q_dev, int64_t ldq, int32_t n_vec,
                            void* phi_dev, int64_t ldphi, void* hip_stream, int32_t reps,
                            double* best_ms);

/* ---- batches of independent problems ------------------------------------ */

/* A batch evaluates n independent, precomputed handles (many problems of
 * uneven sizes, orders, depths and vector counts, served together; the
 * multiple right-hand sides of Section 3.2 within each) with one graph
 * launch of grouped launches.  kifmm_batch_create runs every evaluate once
 * eagerly on hip_stream (which finishes all lazy device setup), records each
 * problem's serial schedule (charge gather, P2M, pseudo-inverses, M2M by
 * level, M2L of every level, downward steps by level, leaf evaluation), and
 * merges the launches of equal stage, kernel and instance across the
 * problems into one launch each: workgroup b of such a launch runs the part
 * of one problem's kernel that workgroup b - offset of that problem's own
 * launch would run, so every problem's potentials are those of its own
 * serial evaluate (the FP32 FFT-M2L Hadamard step of a grouped launch runs
 * one workgroup per frequency over all its items; every work split gives
 * the same potentials).  The grouped launches, a few dozen
 * for a batch of any size, are captured into one HIP graph.  The device
 * buffers q_dev[i] / phi_dev[i] (layout and types as in kifmm_evaluate,
 * n_vec[i] vectors, leading dimensions ldq[i] / ldphi[i]) are the ones
 * kifmm_batch_launch uses; kifmm_batch_evaluate takes others per launch.
 * A handle may appear at most once.  While a batch holds a handle, calls
 * that would free or rebuild its device buffers (more vectors, other tile
 * knobs, set_points, precompute, update_points, destroy) return ESTATE.
 * EINVAL: bad arguments or a repeated handle; ESTATE: a handle without
 * points or operators; ENOMEM / EDEVICE: the job buffer or the capture. */
typedef struct kifmm_batch kifmm_batch;
kifmm_status kifmm_batch_create(kifmm_handle* const* handles, int32_t n, const void* const* q_dev,
                                const int64_t* ldq, const int32_t* n_vec, void* const* phi_dev,
                                const int64_t* ldphi, void* hip_stream, kifmm_batch** out);
/* Autotuned batch: for each candidate knob setting that applies to the
 * batch's handles (BLAS / dense: tile widths (128 / n_vec[i]) >> k,
 * k = 0..3, times the two BLAS-M2L forms where directional recompression
 * is on; a batch of FFT-M2L problems has one setting, since the schedule
 * and Hadamard knobs do not apply to grouped launches), sets the knobs of every handle,
 * builds the batch as kifmm_batch_create does, times one warm-up and `reps`
 * (1..100) launches on hip_stream, and destroys it; then builds the batch
 * with the fastest setting into *out, leaves that setting in the handles and
 * writes its median launch time to *best_ms (if not NULL).  Arguments and
 * errors as kifmm_batch_create; EINVAL also for reps out of range.  On an
 * error every handle's knobs are restored. */
kifmm_status kifmm_batch_autotune(kifmm_handle* const* handles, int32_t n,
                                  const void* const* q_dev, const int64_t* ldq,
                                  const int32_t* n_vec, void* const* phi_dev,
                                  const int64_t* ldphi, void* hip_stream, int32_t reps,
                                  kifmm_batch** out, double* best_ms);
/* Launch the recorded graph on hip_stream (asynchronous), with the charge
 * and potential buffers given at creation (their current contents): every
 * problem's FMM passes (Section 2) with its vectors through the same
 * launches (Section 3.2's multiple right-hand sides). */
kifmm_status kifmm_batch_launch(kifmm_batch* batch, void* hip_stream);
/* Launch the graph (the passes of Section 2 for every problem, as
 * kifmm_batch_launch) on hip_stream with other buffers: q_dev[i] / phi_dev[i]
 * replace problem i's charge and potential buffers (same types, vector
 * counts and leading dimensions as at creation; device pointers owned by
 * the caller).  The buffer addresses are copied into the batch's device
 * job table on hip_stream, ordered after earlier launches on that stream:
 * launches of one batch on several streams at once race.  EINVAL: null
 * arguments. */
kifmm_status kifmm_batch_evaluate(kifmm_batch* batch, const void* const* q_dev,
                                  void* const* phi_dev, void* hip_stream);
/* Shape of the batch's launch schedule (a property of this library's
 * grouped launches, not of the paper's method): info[0] problems, info[1]
 * launches per replay, info[2] of which grouped
 * (the rest are kernels without a grouped form, such as the BLAS-M2L
 * kernels, one per problem and stage).  cap >= 3. */
kifmm_status kifmm_batch_info(const kifmm_batch* batch, int64_t* info, int32_t cap);
/* Destroy the graph and its capture streams (not the handles, whose setup
 * of Section 5.1 stays for their own evaluates). */
kifmm_status kifmm_batch_destroy(kifmm_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* KIFMM_H */
