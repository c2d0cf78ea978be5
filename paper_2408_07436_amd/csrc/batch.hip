// Batches of independent kiFMM problems replayed as one HIP graph.
#include <set>
#include <vector>

#include "internal.h"

namespace kifmm {
kifmm_status device_evaluate(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                             int64_t ldphi, hipStream_t s);
}  // namespace kifmm

using kifmm::fail;

struct kifmm_batch {
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

namespace {

void release(kifmm_batch* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (auto e : b->events) hipEventDestroy(e);
  for (auto s : b->streams) hipStreamDestroy(s);
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
  *out = b;
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
  hipSetDevice(b->device);
  release(b);
  return KIFMM_OK;
}

}  // extern "C"
