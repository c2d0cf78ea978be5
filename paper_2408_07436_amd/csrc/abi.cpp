// extern "C" entry points of libkifmm (declared in include/kifmm.h).
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>

#include "internal.h"

namespace kifmm {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

kifmm_status fail(kifmm_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

kifmm_status device_evaluate(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                             int64_t ldphi, hipStream_t s);
kifmm_status device_evaluate_noalloc(kifmm_handle* h, const void* q, int64_t ldq, int nvec,
                                     void* phi, int64_t ldphi, hipStream_t s);
kifmm_status device_stage(kifmm_handle* h, int level, const void* in, void* out, int nvec,
                          hipStream_t s);
kifmm_status device_autotune(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                             int64_t ldphi, hipStream_t s, int reps, double* best_ms);
kifmm_status device_update_points(kifmm_handle* h, const double* src, const double* tgt,
                                  hipStream_t s);
kifmm_status refresh_host_tree(kifmm_handle* h);

}  // namespace kifmm

using kifmm::fail;

extern "C" {

void kifmm_config_default(kifmm_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->size = sizeof(kifmm_config);
  cfg->order = 6;
  cfg->depth = 4;
  cfg->m2l = KIFMM_M2L_FFT;
  cfg->prec = KIFMM_FP64;
  cfg->device = 0;
  cfg->svd_rel_tol = 0.0;
  cfg->svd_rel_tol_dir = -1.0;
  cfg->alpha_inner = 1.05;
  cfg->alpha_outer = 2.95;
  cfg->width = 1.0;
  cfg->check_order = 0;
}

const char* kifmm_last_error(void) { return kifmm::g_last_error.c_str(); }

kifmm_status kifmm_create(const kifmm_config* cfg, kifmm_handle** out) {
  if (!cfg || !out) return fail(KIFMM_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->size != sizeof(kifmm_config)) return fail(KIFMM_EINVAL, "kifmm_config.size mismatch");
  if (cfg->order < 2) return fail(KIFMM_EINVAL, "order must be >= 2");
  if (cfg->depth < 2 || cfg->depth > 16) return fail(KIFMM_EINVAL, "depth must be in 2..16");
  if (cfg->m2l < KIFMM_M2L_DENSE || cfg->m2l > KIFMM_M2L_BLAS)
    return fail(KIFMM_EINVAL, "unknown m2l form");
  if (cfg->prec < KIFMM_FP64 || cfg->prec > KIFMM_BF16X6)
    return fail(KIFMM_EINVAL, "unknown precision");
  if (cfg->m2l == KIFMM_M2L_FFT && cfg->order > 8)
    return fail(KIFMM_EUNSUPPORTED, "FFT M2L is built for orders 2..8");
  if (cfg->m2l == KIFMM_M2L_FFT && cfg->prec == KIFMM_BF16X3)
    return fail(KIFMM_EUNSUPPORTED, "bf16 split precision applies to the BLAS and dense M2L only");
  if (cfg->prec == KIFMM_BF16X6 && cfg->m2l != KIFMM_M2L_BLAS)
    return fail(KIFMM_EUNSUPPORTED, "BF16x6 applies to the stacked BLAS M2L only");
  if (cfg->check_order != 0 && cfg->check_order < cfg->order)
    return fail(KIFMM_EINVAL, "check_order must be 0 or >= order");
  if (cfg->check_order > cfg->order && cfg->m2l != KIFMM_M2L_BLAS)
    return fail(KIFMM_EUNSUPPORTED, "a check order above the expansion order needs BLAS-M2L");
  auto* h = new (std::nothrow) kifmm_handle();
  if (!h) return fail(KIFMM_ENOMEM, "out of host memory");
  h->cfg = *cfg;
  if (h->cfg.alpha_inner <= 0) h->cfg.alpha_inner = 1.05;
  if (h->cfg.alpha_outer <= 0) h->cfg.alpha_outer = 2.95;
  *out = h;
  return KIFMM_OK;
}

kifmm_status kifmm_set_points(kifmm_handle* h, const double* src, int64_t n_src, const double* tgt,
                              int64_t n_tgt) {
  if (!h || !src || !tgt) return fail(KIFMM_EINVAL, "null argument");
  if (n_src <= 0 || n_tgt <= 0) return fail(KIFMM_EINVAL, "point counts must be positive");
  if (n_src > INT32_MAX || n_tgt > INT32_MAX) return fail(KIFMM_EINVAL, "too many points");
  if (h->batches > 0) return fail(KIFMM_ESTATE, "a batch holds this handle");
  if (h->dev) {
    kifmm::destroy_device(h->dev);
    h->dev = nullptr;
  }
  h->has_points = false;
  h->points_on_device = false;
  h->tree_on_device = false;
  kifmm_status st = kifmm::build_tree(h->tree, h->cfg.depth, h->cfg.origin, h->cfg.width, src, n_src,
                                      tgt, n_tgt);
  if (st != KIFMM_OK) return st;
  h->has_points = true;
  return KIFMM_OK;
}

kifmm_status kifmm_precompute(kifmm_handle* h) {
  if (!h) return fail(KIFMM_EINVAL, "null handle");
  if (h->op.ready) return KIFMM_OK;
  if (h->batches > 0) return fail(KIFMM_ESTATE, "a batch holds this handle");
  if (h->dev) {
    kifmm::destroy_device(h->dev);
    h->dev = nullptr;
  }
  // operators depend only on the configuration (Section 5.1): one FP64
  // precomputation per distinct configuration and process
  using Key = std::tuple<int, int, double, double, double, double, int, int, int, uint64_t>;
  static std::mutex mu;
  static std::map<Key, kifmm::Operators> cache;
  const kifmm_config& c = h->cfg;
  const bool blas = c.m2l == KIFMM_M2L_BLAS;
  const bool rnd = blas && h->svd.mode == KIFMM_SVD_RANDOMIZED;
  const int pc = c.check_order > 0 ? c.check_order : c.order;
  const Key key{c.order * 64 + pc, c.m2l, blas ? c.svd_rel_tol : 0.0, blas ? c.svd_rel_tol_dir : 0.0,
                c.alpha_inner, c.alpha_outer, rnd ? 1 : 0, rnd ? h->svd.rank : 0,
                rnd ? h->svd.oversample : 0, rnd ? h->svd.seed : 0};
  // BF16x6 runs only the stacked form, which needs the second compression
  auto usable = [h]() -> kifmm_status {
    if (h->cfg.prec == KIFMM_BF16X6 && !h->op.recompressed) {
      h->op = kifmm::Operators{};
      return fail(KIFMM_EUNSUPPORTED, "BF16x6 needs directional recompression (svd_rel_tol_dir >= 0)");
    }
    return KIFMM_OK;
  };
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      h->op = it->second;
      return usable();
    }
  }
  kifmm::SvdOptions svd = h->svd;
  svd.device = c.device;
  kifmm_status st = kifmm::precompute_operators(h->op, h->cfg, svd);
  if (st != KIFMM_OK) return st;
  std::lock_guard<std::mutex> lock(mu);
  cache.emplace(key, h->op);
  return usable();
}

kifmm_status kifmm_set_svd(kifmm_handle* h, int32_t mode, int32_t rank, int32_t oversample,
                           uint64_t seed) {
  if (!h) return fail(KIFMM_EINVAL, "null handle");
  if (mode != KIFMM_SVD_DETERMINISTIC && mode != KIFMM_SVD_RANDOMIZED)
    return fail(KIFMM_EINVAL, "unknown SVD mode");
  if (rank < 0 || oversample < 0) return fail(KIFMM_EINVAL, "negative rank or oversampling");
  if (h->op.ready) return fail(KIFMM_ESTATE, "the SVD is chosen before kifmm_precompute");
  if (h->batches > 0) return fail(KIFMM_ESTATE, "a batch holds this handle");
  h->svd.mode = mode;
  h->svd.rank = rank;
  h->svd.oversample = oversample;
  h->svd.seed = seed;
  return KIFMM_OK;
}

kifmm_status kifmm_evaluate(kifmm_handle* h, const void* q_dev, int64_t ldq, int32_t n_vec,
                            void* phi_dev, int64_t ldphi, void* hip_stream) {
  if (!h) return fail(KIFMM_EINVAL, "null handle");
  if (!h->has_points) return fail(KIFMM_ESTATE, "evaluate before set_points");
  if (!h->op.ready) return fail(KIFMM_ESTATE, "evaluate before precompute");
  if (!q_dev || !phi_dev) return fail(KIFMM_EINVAL, "null buffer");
  if (n_vec < 1 || ldq < h->tree.n_src || ldphi < h->tree.n_tgt)
    return fail(KIFMM_EINVAL, "bad n_vec or leading dimension");
  return kifmm::device_evaluate(h, q_dev, ldq, n_vec, phi_dev, ldphi, (hipStream_t)hip_stream);
}

kifmm_status kifmm_evaluate_noalloc(kifmm_handle* h, const void* q_dev, int64_t ldq, int32_t n_vec,
                                    void* phi_dev, int64_t ldphi, void* hip_stream) {
  if (!h) return fail(KIFMM_EINVAL, "null handle");
  if (!h->has_points) return fail(KIFMM_ESTATE, "evaluate before set_points");
  if (!h->op.ready) return fail(KIFMM_ESTATE, "evaluate before precompute");
  if (!q_dev || !phi_dev) return fail(KIFMM_EINVAL, "null buffer");
  if (n_vec < 1 || ldq < h->tree.n_src || ldphi < h->tree.n_tgt)
    return fail(KIFMM_EINVAL, "bad n_vec or leading dimension");
  return kifmm::device_evaluate_noalloc(h, q_dev, ldq, n_vec, phi_dev, ldphi, (hipStream_t)hip_stream);
}

kifmm_status kifmm_destroy(kifmm_handle* h) {
  if (!h) return KIFMM_OK;
  if (h->batches > 0) return fail(KIFMM_ESTATE, "a batch holds this handle; destroy the batch first");
  kifmm::destroy_device(h->dev);
  delete h;
  return KIFMM_OK;
}

kifmm_status kifmm_num_boxes(const kifmm_handle* h, int32_t level, int64_t* n) {
  if (!h || !n) return fail(KIFMM_EINVAL, "null argument");
  if (!h->has_points) return fail(KIFMM_ESTATE, "no points set");
  if (level < 0 || level > h->tree.depth) return fail(KIFMM_EINVAL, "level out of range");
  *n = h->tree.levels[level].n;
  return KIFMM_OK;
}

kifmm_status kifmm_box_keys(const kifmm_handle* h, int32_t level, uint64_t* keys, int64_t cap) {
  if (!h || !keys) return fail(KIFMM_EINVAL, "null argument");
  if (!h->has_points) return fail(KIFMM_ESTATE, "no points set");
  if (level < 0 || level > h->tree.depth) return fail(KIFMM_EINVAL, "level out of range");
  kifmm_status st = kifmm::refresh_host_tree(const_cast<kifmm_handle*>(h));
  if (st != KIFMM_OK) return st;
  const auto& k = h->tree.levels[level].keys;
  if (cap < (int64_t)k.size()) return fail(KIFMM_EINVAL, "capacity too small");
  std::memcpy(keys, k.data(), k.size() * sizeof(uint64_t));
  return KIFMM_OK;
}

kifmm_status kifmm_point_perm(const kifmm_handle* h, int32_t which, int64_t* perm, int64_t cap) {
  if (!h || !perm) return fail(KIFMM_EINVAL, "null argument");
  if (!h->has_points) return fail(KIFMM_ESTATE, "no points set");
  if (which != 0 && which != 1) return fail(KIFMM_EINVAL, "which must be 0 or 1");
  // after device updates the host copy is refreshed from the device
  kifmm_status st = kifmm::refresh_host_tree(const_cast<kifmm_handle*>(h));
  if (st != KIFMM_OK) return st;
  const auto& p = which == 0 ? h->tree.src_perm : h->tree.tgt_perm;
  if (cap < (int64_t)p.size()) return fail(KIFMM_EINVAL, "capacity too small");
  std::memcpy(perm, p.data(), p.size() * sizeof(int64_t));
  return KIFMM_OK;
}

kifmm_status kifmm_interactions(const kifmm_handle* h, int32_t level, int64_t* offs, int64_t* src,
                                int32_t* tidx, int64_t cap, int64_t* n_pairs) {
  if (!h || !n_pairs) return fail(KIFMM_EINVAL, "null argument");
  if (!h->has_points) return fail(KIFMM_ESTATE, "no points set");
  if (level < 2 || level > h->tree.depth) return fail(KIFMM_EINVAL, "level out of range");
  kifmm_status st = kifmm::refresh_host_tree(const_cast<kifmm_handle*>(h));
  if (st != KIFMM_OK) return st;
  const auto& L = h->tree.levels[level];
  *n_pairs = (int64_t)L.il_src.size();
  if (!offs && !src && !tidx) return KIFMM_OK;
  if (!offs || !src || !tidx) return fail(KIFMM_EINVAL, "null array");
  if (cap < *n_pairs) return fail(KIFMM_EINVAL, "capacity too small");
  std::memcpy(offs, L.il_offs.data(), L.il_offs.size() * sizeof(int64_t));
  for (size_t e = 0; e < L.il_src.size(); ++e) {
    src[e] = L.il_src[e];
    tidx[e] = L.il_t[e];
  }
  return KIFMM_OK;
}

kifmm_status kifmm_near(const kifmm_handle* h, int64_t* offs, int64_t* src, int64_t cap,
                        int64_t* n_pairs) {
  if (!h || !n_pairs) return fail(KIFMM_EINVAL, "null argument");
  if (!h->has_points) return fail(KIFMM_ESTATE, "no points set");
  kifmm_status st = kifmm::refresh_host_tree(const_cast<kifmm_handle*>(h));
  if (st != KIFMM_OK) return st;
  *n_pairs = (int64_t)h->tree.near_src.size();
  if (!offs && !src) return KIFMM_OK;
  if (!offs || !src) return fail(KIFMM_EINVAL, "null array");
  if (cap < *n_pairs) return fail(KIFMM_EINVAL, "capacity too small");
  std::memcpy(offs, h->tree.near_offs.data(), h->tree.near_offs.size() * sizeof(int64_t));
  for (size_t e = 0; e < h->tree.near_src.size(); ++e) src[e] = h->tree.near_src[e];
  return KIFMM_OK;
}

kifmm_status kifmm_operator(const kifmm_handle* h, int32_t which, double* out, int64_t cap,
                            int64_t* n) {
  if (!h || !n) return fail(KIFMM_EINVAL, "null argument");
  if (!h->op.ready) return fail(KIFMM_ESTATE, "operators not precomputed");
  const kifmm::Operators& op = h->op;
  std::vector<double> buf;
  const std::vector<double>* src = nullptr;
  switch (which) {
    case 0: src = &op.up_V; break;
    case 1: src = &op.up_Ut; break;
    case 2: src = &op.down_V; break;
    case 3: src = &op.down_Ut; break;
    case 4:
      if (h->cfg.m2l != KIFMM_M2L_FFT) return fail(KIFMM_EINVAL, "no FFT spectra in this mode");
      src = &op.spectra;
      break;
    case 5:
      if (h->cfg.m2l == KIFMM_M2L_FFT) return fail(KIFMM_EINVAL, "no BLAS operators in this mode");
      src = &op.U;
      break;
    case 6:
      if (h->cfg.m2l == KIFMM_M2L_FFT) return fail(KIFMM_EINVAL, "no BLAS operators in this mode");
      buf.push_back(op.k);
      for (int r : op.kt) buf.push_back(r);
      src = &buf;
      break;
    case 7: {
      if (h->cfg.m2l == KIFMM_M2L_FFT) return fail(KIFMM_EINVAL, "no BLAS operators in this mode");
      const int ns = op.ns, nc = op.nc, k = op.k;
      buf.assign((size_t)kifmm::kNumTransfer * nc * ns, 0.0);
      std::vector<double> C((size_t)k * k), UC((size_t)nc * k);
      for (int it = 0; it < kifmm::kNumTransfer; ++it) {
        if (!op.recompressed) {
          C = op.Vbarp[it];
        } else {
          const int r = op.kt[it];
          for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
              double acc = 0;
              for (int l = 0; l < r; ++l)
                acc += op.Ubar[it][(size_t)i * r + l] * op.Vbarp[it][(size_t)j * r + l];
              C[(size_t)i * k + j] = acc;
            }
        }
        for (int i = 0; i < nc; ++i)
          for (int j = 0; j < k; ++j) {
            double acc = 0;
            for (int l = 0; l < k; ++l) acc += op.U[(size_t)i * k + l] * C[(size_t)l * k + j];
            UC[(size_t)i * k + j] = acc;
          }
        double* dst = &buf[(size_t)it * nc * ns];
        for (int i = 0; i < nc; ++i)
          for (int j = 0; j < ns; ++j) {
            double acc = 0;
            for (int l = 0; l < k; ++l) acc += UC[(size_t)i * k + l] * op.S[(size_t)j * k + l];
            dst[(size_t)i * ns + j] = acc;
          }
      }
      src = &buf;
      break;
    }
    default:
      return fail(KIFMM_EINVAL, "unknown operator id");
  }
  *n = (int64_t)src->size();
  if (!out) return KIFMM_OK;
  if (cap < *n) return fail(KIFMM_EINVAL, "capacity too small");
  std::memcpy(out, src->data(), src->size() * sizeof(double));
  return KIFMM_OK;
}

kifmm_status kifmm_stage(kifmm_handle* h, int32_t stage, int32_t level, const void* in_dev,
                         void* out_dev, int32_t n_vec, void* hip_stream) {
  if (!h) return fail(KIFMM_EINVAL, "null handle");
  if (stage != 0) return fail(KIFMM_EINVAL, "unknown stage");
  if (!h->has_points || !h->op.ready) return fail(KIFMM_ESTATE, "stage before set_points / precompute");
  if (level < 2 || level > h->tree.depth) return fail(KIFMM_EINVAL, "level out of range");
  if (!in_dev || !out_dev || n_vec < 1) return fail(KIFMM_EINVAL, "bad buffers or n_vec");
  return kifmm::device_stage(h, level, in_dev, out_dev, n_vec, (hipStream_t)hip_stream);
}

kifmm_status kifmm_set_timing(kifmm_handle* h, int32_t on) {
  if (!h) return fail(KIFMM_EINVAL, "null handle");
  h->timing = on != 0;
  return KIFMM_OK;
}

kifmm_status kifmm_timings(const kifmm_handle* h, double* ms, int32_t cap) {
  if (!h || !ms) return fail(KIFMM_EINVAL, "null argument");
  if (cap < 5) return fail(KIFMM_EINVAL, "capacity too small");
  for (int i = 0; i < cap && i < 12; ++i) ms[i] = h->timings[i];
  return KIFMM_OK;
}

kifmm_status kifmm_update_points(kifmm_handle* h, const void* src_dev, const void* tgt_dev,
                                 void* hip_stream) {
  if (!h || !src_dev || !tgt_dev) return fail(KIFMM_EINVAL, "null argument");
  if (!h->has_points) return fail(KIFMM_ESTATE, "update_points before set_points");
  if (!h->op.ready) return fail(KIFMM_ESTATE, "update_points before precompute");
  if (h->batches > 0) return fail(KIFMM_ESTATE, "a batch holds this handle");
  return kifmm::device_update_points(h, (const double*)src_dev, (const double*)tgt_dev,
                                     (hipStream_t)hip_stream);
}

kifmm_status kifmm_get_tuning(const kifmm_handle* h, int32_t* knobs, int32_t cap) {
  if (!h || !knobs) return fail(KIFMM_EINVAL, "null argument");
  if (cap < KIFMM_TUNE_COUNT) return fail(KIFMM_EINVAL, "capacity too small");
  for (int i = 0; i < KIFMM_TUNE_COUNT; ++i) knobs[i] = h->tune[i];
  return KIFMM_OK;
}

kifmm_status kifmm_set_tuning(kifmm_handle* h, const int32_t* knobs, int32_t n) {
  if (!h || !knobs) return fail(KIFMM_EINVAL, "null argument");
  if (n < 0 || n > KIFMM_TUNE_COUNT) return fail(KIFMM_EINVAL, "bad knob count");
  static const int32_t hi[KIFMM_TUNE_COUNT] = {128, 1, 1, 1, 1};
  for (int i = 0; i < n; ++i)
    if (knobs[i] < 0 || knobs[i] > hi[i]) return fail(KIFMM_EINVAL, "knob value out of range");
  if (h->batches > 0)
    for (int i = 0; i < n; ++i)
      if (knobs[i] != h->tune[i]) return fail(KIFMM_ESTATE, "a batch holds this handle");
  for (int i = 0; i < n; ++i) h->tune[i] = knobs[i];
  return KIFMM_OK;
}

kifmm_status kifmm_autotune(kifmm_handle* h, const void* q_dev, int64_t ldq, int32_t n_vec,
                            void* phi_dev, int64_t ldphi, void* hip_stream, int32_t reps,
                            double* best_ms) {
  if (!h) return fail(KIFMM_EINVAL, "null handle");
  if (!h->has_points) return fail(KIFMM_ESTATE, "autotune before set_points");
  if (!h->op.ready) return fail(KIFMM_ESTATE, "autotune before precompute");
  if (!q_dev || !phi_dev) return fail(KIFMM_EINVAL, "null buffer");
  if (n_vec < 1 || ldq < h->tree.n_src || ldphi < h->tree.n_tgt)
    return fail(KIFMM_EINVAL, "bad n_vec or leading dimension");
  if (reps < 1 || reps > 100) return fail(KIFMM_EINVAL, "reps out of range");
  if (h->batches > 0) return fail(KIFMM_ESTATE, "a batch holds this handle");
  return kifmm::device_autotune(h, q_dev, ldq, n_vec, phi_dev, ldphi, (hipStream_t)hip_stream,
                                reps, best_ms);
}

kifmm_status kifmm_m2l_counts(const kifmm_handle* h, int32_t level, int64_t* counts, int32_t cap) {
  if (!h || !counts) return fail(KIFMM_EINVAL, "null argument");
  if (!h->has_points) return fail(KIFMM_ESTATE, "no points set");
  if (level < 2 || level > h->tree.depth) return fail(KIFMM_EINVAL, "level out of range");
  if (cap < 4) return fail(KIFMM_EINVAL, "capacity too small");
  kifmm_status st = kifmm::refresh_host_tree(const_cast<kifmm_handle*>(h));
  if (st != KIFMM_OK) return st;
  const auto& L = h->tree.levels[level];
  counts[0] = L.n;
  counts[1] = (int64_t)L.il_src.size();
  counts[2] = h->tree.levels[level - 1].n;
  int64_t cp = 0;
  for (int32_t v : L.halo) cp += v >= 0;
  counts[3] = cp;
  return KIFMM_OK;
}

}  // extern "C"
