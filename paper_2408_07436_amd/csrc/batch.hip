// Batches of independent kiFMM problems replayed as one HIP graph.
#include <algorithm>
#include <array>
#include <set>
#include <vector>

#include "internal.h"

namespace kifmm {
kifmm_status device_evaluate(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                             int64_t ldphi, hipStream_t s);
}  // namespace kifmm

using kifmm::fail;

struct kifmm_batch {
  std::vector<kifmm_handle*> handles;  // each holds one count in handle->batches
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

namespace {

void release(kifmm_batch* b) {
  if (!b) return;
  for (kifmm_handle* h : b->handles) --h->batches;
  // teardown: nothing to do about a failure here
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto e : b->events) (void)hipEventDestroy(e);
  for (auto s : b->streams) (void)hipStreamDestroy(s);
  delete b;
}

}  // namespace

extern "C" {

kifmm_status kifmm_batch_create(kifmm_handle* const* handles, int32_t n, const void* const* q_dev,
                                const int64_t* ldq, const int32_t* n_vec, void* const* phi_dev,
                                const int64_t* ldphi, void* hip_stream, kifmm_batch** out) {
  if (!handles || !q_dev || !ldq || !n_vec || !phi_dev || !ldphi || !out || n < 1)
    return fail(KIFMM_EINVAL, "bad batch arguments");
  *out = nullptr;
  std::set<kifmm_handle*> seen;
  for (int i = 0; i < n; ++i) {
    kifmm_handle* h = handles[i];
    if (!h || !q_dev[i] || !phi_dev[i] || n_vec[i] < 1) return fail(KIFMM_EINVAL, "bad batch entry");
    if (!seen.insert(h).second) return fail(KIFMM_EINVAL, "a handle appears twice in the batch");
    if (!h->has_points || !h->op.ready) return fail(KIFMM_ESTATE, "batch handle not precomputed");
    if (ldq[i] < h->tree.n_src || ldphi[i] < h->tree.n_tgt)
      return fail(KIFMM_EINVAL, "bad leading dimension in batch");
    if (h->cfg.device != handles[0]->cfg.device) return fail(KIFMM_EINVAL, "batch spans devices");
  }
  hipStream_t s0 = (hipStream_t)hip_stream;
  const int device = handles[0]->cfg.device;
  KIFMM_HIP(hipSetDevice(device));
  // eager pass: uploads, work buffers and tiles exist before capture
  for (int i = 0; i < n; ++i) {
    kifmm_handle* h = handles[i];
    const bool timing = h->timing;
    h->timing = false;
    kifmm_status st = kifmm::device_evaluate(h, q_dev[i], ldq[i], n_vec[i], phi_dev[i], ldphi[i], s0);
    h->timing = timing;
    if (st != KIFMM_OK) return st;
  }
  KIFMM_HIP(hipStreamSynchronize(s0));

  auto* b = new kifmm_batch();
  b->device = device;
  // capture on a private origin stream; one forked stream per problem
  hipStream_t origin;
  if (hipStreamCreate(&origin) != hipSuccess) {
    release(b);
    return fail(KIFMM_EDEVICE, "hipStreamCreate failed");
  }
  b->streams.push_back(origin);
  for (int i = 0; i < n; ++i) {
    hipStream_t s;
    hipEvent_t e;
    if (hipStreamCreate(&s) != hipSuccess || hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      release(b);
      return fail(KIFMM_EDEVICE, "stream or event creation failed");
    }
    b->streams.push_back(s);
    b->events.push_back(e);
  }
  hipEvent_t fork;
  if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
    release(b);
    return fail(KIFMM_EDEVICE, "event creation failed");
  }
  b->events.push_back(fork);
  kifmm_status st = KIFMM_OK;
  hipError_t e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) e = hipEventRecord(fork, origin);
  for (int i = 0; i < n && e == hipSuccess && st == KIFMM_OK; ++i) {
    hipStream_t si = b->streams[i + 1];
    e = hipStreamWaitEvent(si, fork, 0);
    if (e != hipSuccess) break;
    kifmm_handle* h = handles[i];
    const bool timing = h->timing;
    h->timing = false;
    st = kifmm::device_evaluate(h, q_dev[i], ldq[i], n_vec[i], phi_dev[i], ldphi[i], si);
    h->timing = timing;
    if (st != KIFMM_OK) break;
    e = hipEventRecord(b->events[i], si);
    if (e == hipSuccess) e = hipStreamWaitEvent(origin, b->events[i], 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(origin, &graph);
  b->graph = graph;
  if (st != KIFMM_OK) {
    release(b);
    return st;
  }
  if (e != hipSuccess || e_end != hipSuccess) {
    release(b);
    return fail(KIFMM_EDEVICE, std::string("graph capture failed: ") +
                                   hipGetErrorString(e != hipSuccess ? e : e_end));
  }
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    release(b);
    return fail(KIFMM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  b->handles.assign(handles, handles + n);
  for (kifmm_handle* h : b->handles) ++h->batches;
  *out = b;
  return KIFMM_OK;
}

kifmm_status kifmm_batch_autotune(kifmm_handle* const* handles, int32_t n,
                                  const void* const* q_dev, const int64_t* ldq,
                                  const int32_t* n_vec, void* const* phi_dev,
                                  const int64_t* ldphi, void* hip_stream, int32_t reps,
                                  kifmm_batch** out, double* best_ms) {
  if (!handles || !n_vec || !out || n < 1) return fail(KIFMM_EINVAL, "bad batch arguments");
  if (reps < 1 || reps > 100) return fail(KIFMM_EINVAL, "reps out of range");
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (!handles[i] || n_vec[i] < 1) return fail(KIFMM_EINVAL, "bad batch entry");
  for (int i = 0; i < n; ++i)
    if (handles[i]->batches > 0) return fail(KIFMM_ESTATE, "a batch already holds a handle");
  bool fft32 = false, tiled = false;
  for (int i = 0; i < n; ++i) {
    const kifmm_config& c = handles[i]->cfg;
    if (c.m2l == KIFMM_M2L_FFT && c.prec != KIFMM_FP64) fft32 = true;
    if (c.m2l != KIFMM_M2L_FFT) tiled = true;
  }
  // candidates: (Hadamard form, BLAS tile shift): the tile width of problem
  // i is (128 / n_vec[i]) >> shift; the schedule knob does not apply under
  // capture
  std::vector<std::array<int, 2>> cand;
  for (int form = 0; form < (fft32 ? 2 : 1); ++form)
    for (int shift = 0; shift < (tiled ? 4 : 1); ++shift) cand.push_back({form, shift});
  using Knobs = std::array<int32_t, KIFMM_TUNE_COUNT>;
  std::vector<Knobs> saved((size_t)n);
  for (int i = 0; i < n; ++i) std::copy(handles[i]->tune, handles[i]->tune + KIFMM_TUNE_COUNT, saved[i].begin());
  auto apply = [&](const std::array<int, 2>& c) {
    for (int i = 0; i < n; ++i) {
      kifmm_handle* h = handles[i];
      std::copy(saved[i].begin(), saved[i].end(), h->tune);
      if (h->cfg.m2l == KIFMM_M2L_FFT) {
        if (h->cfg.prec != KIFMM_FP64) h->tune[KIFMM_TUNE_HADAMARD] = c[0];
      } else {
        h->tune[KIFMM_TUNE_BLAS_TILE] = std::max(1, (128 / n_vec[i]) >> c[1]);
      }
    }
  };
  auto restore = [&]() {
    for (int i = 0; i < n; ++i) std::copy(saved[i].begin(), saved[i].end(), handles[i]->tune);
  };
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t ev[2] = {nullptr, nullptr};
  auto cleanup = [&]() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
    cleanup();
    return fail(KIFMM_EDEVICE, "event creation failed");
  }
  double best = 0.0;
  size_t chosen = 0;
  for (size_t k = 0; k < cand.size(); ++k) {
    apply(cand[k]);
    kifmm_batch* b = nullptr;
    kifmm_status st = kifmm_batch_create(handles, n, q_dev, ldq, n_vec, phi_dev, ldphi, hip_stream, &b);
    std::vector<float> t((size_t)reps);
    hipError_t e = hipSuccess;
    if (st == KIFMM_OK) {
      e = hipGraphLaunch(b->exec, s);  // warm-up
      for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(ev[0], s);
        if (e == hipSuccess) e = hipGraphLaunch(b->exec, s);
        if (e == hipSuccess) e = hipEventRecord(ev[1], s);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&t[(size_t)r], ev[0], ev[1]);
      }
      kifmm_batch_destroy(b);
    }
    if (st != KIFMM_OK || e != hipSuccess) {
      restore();
      cleanup();
      return st != KIFMM_OK ? st : fail(KIFMM_EDEVICE, std::string("batch autotune: ") + hipGetErrorString(e));
    }
    std::sort(t.begin(), t.end());
    const double med = t[(size_t)reps / 2];
    if (k == 0 || med < best) {
      best = med;
      chosen = k;
    }
  }
  cleanup();
  apply(cand[chosen]);
  const kifmm_status st = kifmm_batch_create(handles, n, q_dev, ldq, n_vec, phi_dev, ldphi, hip_stream, out);
  if (st != KIFMM_OK) {
    restore();
    return st;
  }
  if (best_ms) *best_ms = best;
  return KIFMM_OK;
}

kifmm_status kifmm_batch_launch(kifmm_batch* b, void* hip_stream) {
  if (!b || !b->exec) return fail(KIFMM_EINVAL, "null batch");
  KIFMM_HIP(hipSetDevice(b->device));
  KIFMM_HIP(hipGraphLaunch(b->exec, (hipStream_t)hip_stream));
  return KIFMM_OK;
}

kifmm_status kifmm_batch_destroy(kifmm_batch* b) {
  if (!b) return KIFMM_OK;
  (void)hipSetDevice(b->device);
  release(b);
  return KIFMM_OK;
}

}  // extern "C"
