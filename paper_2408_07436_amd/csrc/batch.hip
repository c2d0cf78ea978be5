// Batches of independent kiFMM problems (uneven sizes, orders, depths and
// vector counts) run as one graph of grouped launches: every problem's
// serial evaluate schedule is recorded (device.hip), launches of equal
// stage, kernel and instance across the problems are merged into one
// grouped launch (kernels.h), and the few dozen grouped launches are
// captured into one HIP graph.  The multiple right-hand sides of Section
// 3.2 go through each problem's launches as in a single evaluate.
#include <algorithm>
#include <array>
#include <cstddef>
#include <set>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace kifmm {
kifmm_status device_evaluate(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                             int64_t ldphi, hipStream_t s);
kifmm_status device_record(kifmm_handle* h, const void* q, int64_t ldq, int nvec, void* phi,
                           int64_t ldphi, LaunchSink* sink, hipStream_t s);
}  // namespace kifmm

using kifmm::fail;

namespace {

// One launch of a replay: a grouped launch over jobs [args_off, ..) with the
// prefix sums at pre_off (byte offsets into the batch's job buffer), or a
// recorded launch without a grouped form.
struct GroupLaunch {
  int64_t key = 0;
  int family = 0, inst = 0, nj = 0;
  int64_t blocks = 0;
  size_t args_off = 0, pre_off = 0;
  std::function<hipError_t(hipStream_t)> single;
};

}  // namespace

struct kifmm_batch {
  std::vector<kifmm_handle*> handles;  // each holds one count in handle->batches
  std::vector<int64_t> ldq, ldphi;
  std::vector<int32_t> nvec;
  std::vector<GroupLaunch> launches;   // main branch, in order
  std::vector<GroupLaunch> side;       // near-field branch, in order
  std::vector<uint8_t> host_jobs;      // host copy of the job buffer
  void* dev_jobs = nullptr;            // job arguments and prefix sums of every grouped launch
  // per problem: byte offsets of its charge pointer and of its potential
  // pointers (near and far field)
  std::vector<size_t> q_at;
  std::vector<std::vector<size_t>> phi_at;
  hipStream_t origin = nullptr, branch = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
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
  if (b->origin) (void)hipStreamDestroy(b->origin);
  if (b->branch) (void)hipStreamDestroy(b->branch);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->dev_jobs) (void)hipFree(b->dev_jobs);
  delete b;
}

hipError_t run_group(const GroupLaunch& g, const uint8_t* base, hipStream_t s) {
  using namespace kifmm;
  const void* jobs = base + g.args_off;
  const int64_t* pre = reinterpret_cast<const int64_t*>(base + g.pre_off);
  switch (g.family) {
    case kFamGather:
      return launch_gather_group(g.inst == 1, static_cast<const GatherArgs*>(jobs), pre, g.nj, g.blocks, s);
    case kFamP2M:
      return launch_p2m_group(g.inst, static_cast<const P2MArgs*>(jobs), pre, g.nj, g.blocks, s);
    case kFamGemm:
      return launch_gemm64_group(static_cast<const GemmJob*>(jobs), pre, g.nj, g.blocks, false, s);
    case kFamGemmReduce:
      return launch_gemm64_group(static_cast<const GemmJob*>(jobs), pre, g.nj, g.blocks, true, s);
    case kFamFwd:
      return launch_fft_forward_group(g.inst, static_cast<const FwdArgs*>(jobs), pre, g.nj, g.blocks, s);
    case kFamHad:
      return launch_hadamard_group(g.inst, jobs, pre, g.nj, g.blocks, s);
    case kFamInv:
      return launch_fft_inverse_group(g.inst, static_cast<const InvArgs*>(jobs), pre, g.nj, g.blocks, s);
    case kFamLeaf:
      return launch_leaf_eval_group(g.inst, static_cast<const LeafArgs*>(jobs), pre, g.nj, g.blocks, s);
    case kFamSingle:
      return g.single(s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

extern "C" {

kifmm_status kifmm_batch_create(kifmm_handle* const* handles, int32_t n, const void* const* q_dev,
                                const int64_t* ldq, const int32_t* n_vec, void* const* phi_dev,
                                const int64_t* ldphi, void* hip_stream, kifmm_batch** out) {
  using namespace kifmm;
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
  // eager pass: uploads, work buffers and tiles exist before recording
  for (int i = 0; i < n; ++i) {
    kifmm_handle* h = handles[i];
    const bool timing = h->timing;
    h->timing = false;
    kifmm_status st = device_evaluate(h, q_dev[i], ldq[i], n_vec[i], phi_dev[i], ldphi[i], s0);
    h->timing = timing;
    if (st != KIFMM_OK) return st;
  }
  KIFMM_HIP(hipStreamSynchronize(s0));

  // record every problem's serial schedule
  LaunchSink sink;
  for (int i = 0; i < n; ++i) {
    sink.problem = i;
    const kifmm_status st = device_record(handles[i], q_dev[i], ldq[i], n_vec[i], phi_dev[i], ldphi[i],
                                          &sink, s0);
    if (st != KIFMM_OK) return st;
  }
  std::vector<LaunchRec>& recs = sink.recs;
  std::stable_sort(recs.begin(), recs.end(), [](const LaunchRec& a, const LaunchRec& b) {
    if (a.side != b.side) return !a.side;
    if (a.key != b.key) return a.key < b.key;
    if (a.family != b.family) return a.family < b.family;
    return a.inst < b.inst;
  });

  auto* b = new kifmm_batch();
  b->device = device;
  b->q_at.assign((size_t)n, SIZE_MAX);
  b->phi_at.assign((size_t)n, {});
  auto align = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t r = 0;
  while (r < recs.size()) {
    std::vector<GroupLaunch>& dst = recs[r].side ? b->side : b->launches;
    GroupLaunch g;
    g.family = recs[r].family;
    g.inst = recs[r].inst;
    g.key = recs[r].key;
    if (g.family == kFamSingle) {
      g.single = recs[r].single;
      dst.push_back(std::move(g));
      ++r;
      continue;
    }
    size_t e = r;
    while (e < recs.size() && recs[e].side == recs[r].side && recs[e].key == recs[r].key &&
           recs[e].family == g.family && recs[e].inst == g.inst)
      ++e;
    g.nj = (int)(e - r);
    const size_t asz = recs[r].args.size();
    g.args_off = align(b->host_jobs.size());
    g.pre_off = align(g.args_off + asz * g.nj);
    b->host_jobs.resize(g.pre_off + sizeof(int64_t) * (g.nj + 1), 0);
    int64_t acc = 0;
    for (size_t k = r; k < e; ++k) {
      const size_t at = g.args_off + asz * (k - r);
      std::memcpy(b->host_jobs.data() + at, recs[k].args.data(), asz);
      const int64_t pv = acc;
      std::memcpy(b->host_jobs.data() + g.pre_off + sizeof(int64_t) * (k - r), &pv, sizeof(int64_t));
      acc += recs[k].blocks;
      if (g.family == kFamGather) b->q_at[(size_t)recs[k].problem] = at + offsetof(GatherArgs, q);
      if (g.family == kFamLeaf) b->phi_at[(size_t)recs[k].problem].push_back(at + offsetof(LeafArgs, phi));
    }
    std::memcpy(b->host_jobs.data() + g.pre_off + sizeof(int64_t) * g.nj, &acc, sizeof(int64_t));
    g.blocks = acc;
    dst.push_back(std::move(g));
    r = e;
  }
  for (int i = 0; i < n; ++i)
    if (b->q_at[(size_t)i] == SIZE_MAX || b->phi_at[(size_t)i].empty()) {
      release(b);
      return fail(KIFMM_ENUMERIC, "batch: a problem without charge gather or leaf evaluation");
    }
  hipError_t e = hipMalloc(&b->dev_jobs, std::max<size_t>(b->host_jobs.size(), 256));
  if (e == hipSuccess)
    e = hipMemcpy(b->dev_jobs, b->host_jobs.data(), b->host_jobs.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->branch, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
  if (e != hipSuccess) {
    release(b);
    return fail(KIFMM_ENOMEM, std::string("batch job buffer: ") + hipGetErrorString(e));
  }
  // capture the grouped launches in order on one stream, the near-field
  // branch forked after the charge gathers (stage 0) and joined before the
  // far field (stage 6)
  const int64_t after_gather = (int64_t)1 * 64 * 4096, far_field = (int64_t)6 * 64 * 4096;
  e = hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal);
  const uint8_t* base = static_cast<const uint8_t*>(b->dev_jobs);
  hipError_t le = hipSuccess;
  bool forked = b->side.empty(), joined = b->side.empty();
  auto fork_branch = [&]() -> hipError_t {
    hipError_t x = hipEventRecord(b->fork, b->origin);
    if (x == hipSuccess) x = hipStreamWaitEvent(b->branch, b->fork, 0);
    for (size_t k = 0; k < b->side.size() && x == hipSuccess; ++k) x = run_group(b->side[k], base, b->branch);
    if (x == hipSuccess) x = hipEventRecord(b->join, b->branch);
    forked = true;
    return x;
  };
  for (size_t k = 0; k < b->launches.size() && e == hipSuccess && le == hipSuccess; ++k) {
    const GroupLaunch& g = b->launches[k];
    if (!forked && g.key >= after_gather) le = fork_branch();
    if (le == hipSuccess && !joined && g.key >= far_field) {
      le = hipStreamWaitEvent(b->origin, b->join, 0);
      joined = true;
    }
    if (le == hipSuccess) le = run_group(g, base, b->origin);
  }
  if (e == hipSuccess && le == hipSuccess && !forked) le = fork_branch();
  if (e == hipSuccess && le == hipSuccess && !joined) le = hipStreamWaitEvent(b->origin, b->join, 0);
  hipGraph_t graph = nullptr;
  const hipError_t e_end = e == hipSuccess ? hipStreamEndCapture(b->origin, &graph) : e;
  b->graph = graph;
  if (e != hipSuccess || le != hipSuccess || e_end != hipSuccess) {
    const hipError_t bad = e != hipSuccess ? e : (le != hipSuccess ? le : e_end);
    release(b);
    return fail(KIFMM_EDEVICE, std::string("batch graph capture: ") + hipGetErrorString(bad));
  }
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    release(b);
    return fail(KIFMM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  b->handles.assign(handles, handles + n);
  b->ldq.assign(ldq, ldq + n);
  b->ldphi.assign(ldphi, ldphi + n);
  b->nvec.assign(n_vec, n_vec + n);
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
  bool tiled = false, stacked = false;
  for (int i = 0; i < n; ++i) {
    const kifmm_config& c = handles[i]->cfg;
    if (c.m2l != KIFMM_M2L_FFT) tiled = true;
    // the form knob chooses between two forms (BF16x6 has the stacked one only)
    if (c.m2l == KIFMM_M2L_BLAS && handles[i]->op.recompressed && c.prec != KIFMM_BF16X6) stacked = true;
  }
  // candidates: (BLAS form, BLAS tile shift): the tile width of problem i is
  // (128 / n_vec[i]) >> shift.  The FFT schedule and Hadamard work split do
  // not apply: a batch runs the serial schedule as grouped launches.
  std::vector<std::array<int, 2>> cand;
  for (int form = 0; form < (stacked ? 2 : 1); ++form)
    for (int shift = 0; shift < (tiled ? 4 : 1); ++shift) cand.push_back({form, shift});
  using Knobs = std::array<int32_t, KIFMM_TUNE_COUNT>;
  std::vector<Knobs> saved((size_t)n);
  for (int i = 0; i < n; ++i) std::copy(handles[i]->tune, handles[i]->tune + KIFMM_TUNE_COUNT, saved[i].begin());
  auto apply = [&](const std::array<int, 2>& c) {
    for (int i = 0; i < n; ++i) {
      kifmm_handle* h = handles[i];
      std::copy(saved[i].begin(), saved[i].end(), h->tune);
      if (h->cfg.m2l != KIFMM_M2L_FFT) {
        h->tune[KIFMM_TUNE_BLAS_TILE] = std::max(1, (128 / n_vec[i]) >> c[1]);
        if (h->cfg.m2l == KIFMM_M2L_BLAS) h->tune[KIFMM_TUNE_BLAS_FORM] = c[0];
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

kifmm_status kifmm_batch_evaluate(kifmm_batch* b, const void* const* q_dev, void* const* phi_dev,
                                  void* hip_stream) {
  if (!b || !b->exec || !q_dev || !phi_dev) return fail(KIFMM_EINVAL, "bad batch arguments");
  const size_t n = b->handles.size();
  for (size_t i = 0; i < n; ++i)
    if (!q_dev[i] || !phi_dev[i]) return fail(KIFMM_EINVAL, "null buffer in batch");
  for (size_t i = 0; i < n; ++i) {
    std::memcpy(b->host_jobs.data() + b->q_at[i], &q_dev[i], sizeof(void*));
    for (size_t at : b->phi_at[i]) std::memcpy(b->host_jobs.data() + at, &phi_dev[i], sizeof(void*));
  }
  hipStream_t s = (hipStream_t)hip_stream;
  KIFMM_HIP(hipSetDevice(b->device));
  // ordered on s after every earlier replay on s, before this one
  KIFMM_HIP(hipMemcpyAsync(b->dev_jobs, b->host_jobs.data(), b->host_jobs.size(), hipMemcpyHostToDevice, s));
  KIFMM_HIP(hipGraphLaunch(b->exec, s));
  return KIFMM_OK;
}

kifmm_status kifmm_batch_info(const kifmm_batch* b, int64_t* info, int32_t cap) {
  if (!b || !info || cap < 3) return fail(KIFMM_EINVAL, "bad batch info arguments");
  int64_t grouped = 0;
  for (const GroupLaunch& g : b->launches) grouped += g.family != kifmm::kFamSingle;
  for (const GroupLaunch& g : b->side) grouped += g.family != kifmm::kFamSingle;
  info[0] = (int64_t)b->handles.size();
  info[1] = (int64_t)(b->launches.size() + b->side.size());
  info[2] = grouped;
  return KIFMM_OK;
}

kifmm_status kifmm_batch_destroy(kifmm_batch* b) {
  if (!b) return KIFMM_OK;
  (void)hipSetDevice(b->device);
  release(b);
  return KIFMM_OK;
}

}  // extern "C"
