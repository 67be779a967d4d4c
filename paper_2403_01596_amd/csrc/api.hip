// C ABI entry points of libp2p: argument validation, plan lifetime, dispatch.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>

#include "mrhs.h"

namespace p2p {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

p2p_status fail(p2p_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

p2p_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? P2P_ERR_NOMEM : P2P_ERR_HIP;
}

namespace {
std::mutex g_handles_mu;
std::unordered_set<const void*>* g_handles = nullptr;  // never freed: handles may outlive static destruction
}  // namespace

void handle_add(const void* h) {
  std::lock_guard<std::mutex> lk(g_handles_mu);
  if (!g_handles) g_handles = new std::unordered_set<const void*>();
  g_handles->insert(h);
}

void handle_remove(const void* h) {
  std::lock_guard<std::mutex> lk(g_handles_mu);
  if (g_handles) g_handles->erase(h);
}

bool handle_live(const void* h) {
  std::lock_guard<std::mutex> lk(g_handles_mu);
  return g_handles && g_handles->count(h) != 0;
}

bool record_use(hipEvent_t ev, hipStream_t s) {
  if (!ev) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (cs != hipStreamCaptureStatusNone) return false;
  if (hipEventRecord(ev, s) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

p2p_status wait_built(p2p_plan_s* P, hipStream_t s, bool force) {
  if (P->built || !P->ready || (!force && s == P->build_stream)) return P2P_OK;
  P2P_HIP(hipEventSynchronize(P->ready));
  P->built = true;
  return P2P_OK;
}

static p2p_status check_plan(p2p_plan_s* P) {
  if (!P || !handle_live(P) || P->magic != kPlanMagic) return fail(P2P_ERR_STATE, "invalid plan handle");
  return P2P_OK;
}

SweepTimer::SweepTimer(p2p_plan_s* plan, hipStream_t st) : P(plan), s(st) {}

void SweepTimer::start() {
  if (!P->timing) return;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    e0 = e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, s);
}

void SweepTimer::stop() {
  if (!P->timing || !e0) return;
  (void)hipEventRecord(e1, s);
  P->timed->emplace_back(e0, e1);
}

static void drop_events(p2p_plan_s* P) {
  if (!P->timed) return;
  for (auto& pr : *P->timed) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  P->timed->clear();
}

// Releases everything.  The device memory goes back to the cache behind the
// plan's last recorded work (the build, or its last call: calls on a plan are
// ordered, so that covers every earlier one), without a host wait.
static p2p_status free_plan(p2p_plan_s* P) {
  p2p_status rc = P2P_OK;
  handle_remove(P);
  int cur = P->device;
  (void)hipGetDevice(&cur);
  if (cur != P->device) (void)hipSetDevice(P->device);
  if (P->self_batch) batch_free(P->self_batch);
  drop_events(P);
  delete P->timed;
  // the event recorded last (the last call's, or the build's) goes to the cache,
  // which owns it from here
  hipEvent_t rel = P->used ? P->last_use : P->ready, other = P->used ? P->ready : P->last_use;
  void* blocks[2] = {P->arena, P->arena2};
  dmem_free_after(blocks, 2, rel);
  if (other) (void)hipEventDestroy(other);
  if (cur != P->device) (void)hipSetDevice(cur);
  P->magic = 0;
  delete P;
  return rc;
}

}  // namespace p2p

using namespace p2p;

extern "C" {

const char* p2p_status_str(p2p_status s) {
  switch (s) {
    case P2P_OK: return "ok";
    case P2P_ERR_ARG: return "invalid argument";
    case P2P_ERR_RANGE: return "value out of range";
    case P2P_ERR_DTYPE: return "dtype does not match the plan";
    case P2P_ERR_NOMEM: return "out of device memory";
    case P2P_ERR_HIP: return "HIP runtime error";
    case P2P_ERR_STATE: return "invalid plan";
  }
  return "unknown status";
}

const char* p2p_last_error(void) { return g_last_error.c_str(); }

p2p_status p2p_box_ids(const double* xyz, int64_t n, const double* origin, double h, int32_t* box_ijk,
                       void* stream) {
  if (n < 0) return fail(P2P_ERR_ARG, "n < 0");
  if (!origin) return fail(P2P_ERR_ARG, "origin is NULL");
  if (n > 0 && (!xyz || !box_ijk)) return fail(P2P_ERR_ARG, "xyz or box_ijk is NULL");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(P2P_ERR_RANGE, "h must be finite and > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(origin[a])) return fail(P2P_ERR_RANGE, "origin must be finite");
  return box_ids(xyz, n, origin, h, box_ijk, (hipStream_t)stream);
}

p2p_status p2p_leaf_level(const double* xyz, int64_t n, const double* origin, double size, int32_t ct,
                          int32_t min_level, int32_t* level, double* h, int32_t* t_max, void* stream) {
  if (n < 0) return fail(P2P_ERR_ARG, "n < 0");
  if (!origin || !level || !h || !t_max) return fail(P2P_ERR_ARG, "origin, level, h or t_max is NULL");
  if (n > 0 && !xyz) return fail(P2P_ERR_ARG, "xyz is NULL");
  if (n > kMaxPoints) return fail(P2P_ERR_RANGE, "n exceeds 79,536,431 points");
  if (!(size > 0.0) || !std::isfinite(size)) return fail(P2P_ERR_RANGE, "size must be finite and > 0");
  if (ct < 1) return fail(P2P_ERR_RANGE, "ct must be >= 1");
  if (min_level < 1 || min_level > 22) return fail(P2P_ERR_RANGE, "min_level must be in [1, 22]");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(origin[a])) return fail(P2P_ERR_RANGE, "origin must be finite");
  return leaf_level(xyz, n, origin, size, ct, min_level, level, h, t_max, (hipStream_t)stream);
}

p2p_status p2p_box_ids_noalloc(const double* xyz, int64_t n, const double* origin, double h, int32_t* box_ijk,
                               void* stream) {
  if (n < 0) return fail(P2P_ERR_ARG, "n < 0");
  if (n > kMaxPoints) return fail(P2P_ERR_RANGE, "n exceeds 79,536,431 points");
  if (!origin) return fail(P2P_ERR_ARG, "origin is NULL");
  if (n > 0 && (!xyz || !box_ijk)) return fail(P2P_ERR_ARG, "xyz or box_ijk is NULL");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(P2P_ERR_RANGE, "h must be finite and > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(origin[a])) return fail(P2P_ERR_RANGE, "origin must be finite");
  return box_ids_noalloc(xyz, n, origin, h, box_ijk, (hipStream_t)stream);
}

namespace {

// Common to the create calls: ids from box_ijk, or (box_ijk null) from gspec.
// n_targets >= 0: distinct sets, the first n_targets points are the targets.
p2p_status create_plan(const double* xyz, const int32_t* box_ijk, const p2p::GridSpec* gspec, int64_t n, double k,
                       const p2p_opts* opts, void* stream, p2p_plan* out, int64_t n_targets = -1) {
  if (!out) return fail(P2P_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n < 0) return fail(P2P_ERR_ARG, "n < 0");
  if (n > 0 && (!xyz || (!box_ijk && !gspec))) return fail(P2P_ERR_ARG, "xyz or box_ijk is NULL");
  if (n > kMaxPoints) return fail(P2P_ERR_RANGE, "n exceeds 79,536,431 points");
  if (!std::isfinite(k) || k < 0) return fail(P2P_ERR_RANGE, "k must be finite and >= 0");
  p2p_opts o{P2P_C64, P2P_LAYOUT_TILES, 1, 0u, nullptr};
  if (opts) o = *opts;
  if (o.precision != P2P_C64 && o.precision != P2P_C128) return fail(P2P_ERR_ARG, "unknown precision");
  if (o.layout != P2P_LAYOUT_TILES && o.layout != P2P_LAYOUT_CSR) return fail(P2P_ERR_ARG, "unknown layout");
  if (o.max_rhs < 1 || o.max_rhs > 4096) return fail(P2P_ERR_ARG, "max_rhs must be in [1, 4096]");
  if (o.flags != 0u) return fail(P2P_ERR_ARG, "flags must be 0");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(P2P_ERR_HIP, "no HIP device");
  p2p_plan_s* P = new (std::nothrow) p2p_plan_s();
  if (!P) return fail(P2P_ERR_NOMEM, "host allocation failed");
  std::memset(P, 0, sizeof(*P));
  P->magic = kPlanMagic;
  P->device = dev;
  P->n = n;
  P->k = k;
  P->precision = o.precision;
  P->layout = o.layout;
  P->max_rhs = o.max_rhs;
  P->distinct_sets = n_targets >= 0;
  P->n_targets = P->distinct_sets ? n_targets : n;
  P->n_pairs = -1;
  P->n_zero = -1;
  P->n_close = -1;
  P->n_near = -1;
  P->timed = new (std::nothrow) std::vector<std::pair<hipEvent_t, hipEvent_t>>();
  if (!P->timed) {
    delete P;
    return fail(P2P_ERR_NOMEM, "host allocation failed");
  }
  handle_add(P);
  p2p_status rc = P2P_OK;
  const hipStream_t s = (hipStream_t)stream;
  P->build_stream = s;
  if (hipEventCreateWithFlags(&P->last_use, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P->ready, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    rc = fail(P2P_ERR_HIP, "hipEventCreateWithFlags failed");
  }
  if (rc == P2P_OK) {
    rc = build_plan(P, xyz, box_ijk, box_ijk ? nullptr : gspec, s);
    // the build returns once its work is enqueued: the event marks its end, for
    // calls on other streams and, until the plan is used, for the release of its
    // memory
    if (hipEventRecord(P->ready, s) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(s);
      P->built = true;
      (void)hipEventDestroy(P->ready);
      P->ready = nullptr;
    }
  }
  if (rc == P2P_OK && P->precision == P2P_C64 && P->max_rhs >= kMrhsMin && !P->distinct_sets) {
    rc = wait_built(P, nullptr, true);  // the batch tables are made from the plan's arrays on the host
    if (rc == P2P_OK) rc = batch_create(&P, 1, P->max_rhs, &P->self_batch);
    if (rc == P2P_OK && o.tune_cache) batch_use_cache(P->self_batch, o.tune_cache);
  }
  if (rc != P2P_OK) {
    std::string msg = g_last_error;
    free_plan(P);
    set_error(msg);
    return rc;
  }
  *out = P;
  return P2P_OK;
}

}  // namespace

p2p_status p2p_plan_create(const double* xyz, const int32_t* box_ijk, int64_t n, double k, const p2p_opts* opts,
                           void* stream, p2p_plan* out) {
  if (n > 0 && !box_ijk) {
    if (out) *out = nullptr;
    return fail(P2P_ERR_ARG, "xyz or box_ijk is NULL");
  }
  return create_plan(xyz, box_ijk, nullptr, n, k, opts, stream, out);
}

p2p_status p2p_plan_create_st(const double* targets, int64_t n_targets, const double* sources, int64_t n_sources,
                              const double* origin, double h, double k, const p2p_opts* opts, void* stream,
                              p2p_plan* out) {
  if (out) *out = nullptr;
  if (!out) return fail(P2P_ERR_ARG, "out is NULL");
  if (n_targets < 0 || n_sources < 0) return fail(P2P_ERR_ARG, "n_targets or n_sources < 0");
  if ((n_targets > 0 && !targets) || (n_sources > 0 && !sources)) return fail(P2P_ERR_ARG, "targets or sources is NULL");
  if (!origin) return fail(P2P_ERR_ARG, "origin is NULL");
  if (n_targets + n_sources > kMaxPoints) return fail(P2P_ERR_RANGE, "more than 79,536,431 points in all");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(P2P_ERR_RANGE, "h must be finite and > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(origin[a])) return fail(P2P_ERR_RANGE, "origin must be finite");
  const int64_t n = n_targets + n_sources;
  const hipStream_t s = (hipStream_t)stream;
  // one point array, targets first: the plan's boxes then list each box's targets
  // before its sources
  void* both = nullptr;
  if (n > 0) {
    both = dmem_alloc(sizeof(double) * 3 * (size_t)n);
    if (!both) return fail(P2P_ERR_NOMEM, "device allocation failed");
    hipError_t e = hipSuccess;
    if (n_targets > 0) e = hipMemcpyAsync(both, targets, sizeof(double) * 3 * n_targets, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && n_sources > 0)
      e = hipMemcpyAsync((double*)both + 3 * n_targets, sources, sizeof(double) * 3 * n_sources,
                         hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);
      dmem_free(both);
      return hip_fail(e, "hipMemcpyAsync");
    }
  }
  const p2p::GridSpec g{{origin[0], origin[1], origin[2]}, h};
  const p2p_status rc = create_plan((const double*)both, nullptr, &g, n, k, opts, stream, out, n_targets);
  dmem_free_on(&both, 1, s);  // behind the build, which has copied what it needs
  return rc;
}

p2p_status p2p_plan_create_grid(const double* xyz, int64_t n, const double* origin, double h, double k,
                                const p2p_opts* opts, void* stream, p2p_plan* out) {
  if (!origin) {
    if (out) *out = nullptr;
    return fail(P2P_ERR_ARG, "origin is NULL");
  }
  if (!(h > 0.0) || !std::isfinite(h)) {
    if (out) *out = nullptr;
    return fail(P2P_ERR_RANGE, "h must be finite and > 0");
  }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(origin[a])) {
      if (out) *out = nullptr;
      return fail(P2P_ERR_RANGE, "origin must be finite");
    }
  const p2p::GridSpec g{{origin[0], origin[1], origin[2]}, h};
  return create_plan(xyz, nullptr, &g, n, k, opts, stream, out);
}

p2p_status p2p_plan_info(p2p_plan plan, p2p_info* out) {
  p2p_status rc = check_plan(plan);
  if (rc != P2P_OK) return rc;
  if (!out) return fail(P2P_ERR_ARG, "out is NULL");
  rc = wait_built(plan, nullptr, true);
  if (rc == P2P_OK) rc = count_pairs(plan, nullptr);
  if (rc != P2P_OK) return rc;
  out->n_points = plan->n;
  out->n_boxes = plan->B;
  out->n_nbr = plan->nnz;
  out->n_slots = plan->n_slots;
  out->n_pairs = plan->n_pairs;
  out->n_zero_pairs = plan->n_zero;
  out->tile_entries = plan->tile_len;
  out->device_bytes = (int64_t)plan->device_bytes;
  out->t_max = plan->t_max;
  out->quantum_exp = plan->precision == P2P_C64 ? plan->qexp : 0;
  out->d_mean = plan->B ? (double)plan->n / (double)plan->B : 0.0;
  out->max_sep = plan->max_sep;
  out->n_close_pairs = plan->n_close;
  out->n_targets = plan->n_targets;
  out->n_near_boxes = plan->n_near;
  return P2P_OK;
}

p2p_status p2p_plan_export(p2p_plan plan, uint64_t* box_key, int32_t* box_start, int32_t* perm, int32_t* nbr_start,
                           int32_t* nbr_idx) {
  p2p_status rc = check_plan(plan);
  if (rc != P2P_OK) return rc;
  const int64_t B = plan->B, n = plan->n;
  rc = wait_built(plan, nullptr, true);
  if (rc != P2P_OK) return rc;
  if (box_key && B) P2P_HIP(hipMemcpy(box_key, plan->box_key, sizeof(uint64_t) * B, hipMemcpyDeviceToHost));
  if (box_start) P2P_HIP(hipMemcpy(box_start, plan->box_start, sizeof(int32_t) * (B + 1), hipMemcpyDeviceToHost));
  if (perm && n) P2P_HIP(hipMemcpy(perm, plan->perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  if (nbr_start) P2P_HIP(hipMemcpy(nbr_start, plan->nbr_start, sizeof(int32_t) * (B + 1), hipMemcpyDeviceToHost));
  if (nbr_idx && plan->nnz)
    P2P_HIP(hipMemcpy(nbr_idx, plan->nbr_idx, sizeof(int32_t) * plan->nnz, hipMemcpyDeviceToHost));
  return P2P_OK;
}

static p2p_status check_call(p2p_plan plan, int32_t nrhs, p2p_dtype dtype) {
  p2p_status rc = check_plan(plan);
  if (rc != P2P_OK) return rc;
  if (dtype != P2P_C64 && dtype != P2P_C128) return fail(P2P_ERR_DTYPE, "unknown dtype");
  if (dtype != plan->precision) return fail(P2P_ERR_DTYPE, "dtype differs from the plan's precision");
  if (nrhs < 1 || nrhs > plan->max_rhs) return fail(P2P_ERR_ARG, "nrhs must be in [1, max_rhs]");
  return P2P_OK;
}

p2p_status p2p_apply(p2p_plan plan, const void* q, void* y, int32_t nrhs, p2p_dtype dtype, void* stream) {
  p2p_status rc = check_call(plan, nrhs, dtype);
  if (rc != P2P_OK) return rc;
  if ((plan->n - (plan->distinct_sets ? plan->n_targets : 0) > 0 && !q) || (plan->n_targets > 0 && !y))
    return fail(P2P_ERR_ARG, "q or y is NULL");
  rc = wait_built(plan, (hipStream_t)stream);
  if (rc != P2P_OK) return rc;
  if (plan->self_batch && nrhs >= kMrhsMin) {
    void* yy = y;
    rc = batch_apply(plan->self_batch, &q, &yy, nrhs, (hipStream_t)stream, plan->timing, plan->timed);
  } else {
    rc = launch_apply(plan, q, y, nrhs, (hipStream_t)stream);
  }
  if (rc == P2P_OK && record_use(plan->last_use, (hipStream_t)stream)) plan->used = true;
  return rc;
}

p2p_status p2p_apply_backward(p2p_plan plan, const void* q, const void* grad_y, void* grad_q, double* grad_xyz,
                              int32_t nrhs, p2p_dtype dtype, void* stream) {
  p2p_status rc = check_call(plan, nrhs, dtype);
  if (rc != P2P_OK) return rc;
  if (plan->distinct_sets) return fail(P2P_ERR_ARG, "no reverse pass for plans of distinct target and source sets");
  if (plan->n > 0 && (!q || !grad_y)) return fail(P2P_ERR_ARG, "q or grad_y is NULL");
  rc = wait_built(plan, (hipStream_t)stream);
  if (rc != P2P_OK) return rc;
  rc = launch_backward(plan, q, grad_y, grad_q, grad_xyz, nrhs, (hipStream_t)stream);
  if (rc == P2P_OK && record_use(plan->last_use, (hipStream_t)stream)) plan->used = true;
  return rc;
}

p2p_status p2p_plan_timing(p2p_plan plan, int enable) {
  p2p_status rc = check_plan(plan);
  if (rc != P2P_OK) return rc;
  plan->timing = enable != 0;
  return P2P_OK;
}

p2p_status p2p_plan_timing_read(p2p_plan plan, double* ms, int64_t* calls) {
  p2p_status rc = check_plan(plan);
  if (rc != P2P_OK) return rc;
  if (!ms || !calls) return fail(P2P_ERR_ARG, "ms or calls is NULL");
  double total = 0.0;
  for (auto& pr : *plan->timed) {
    float t = 0.0f;
    P2P_HIP(hipEventSynchronize(pr.second));
    P2P_HIP(hipEventElapsedTime(&t, pr.first, pr.second));
    total += t;
  }
  *ms = total;
  *calls = (int64_t)plan->timed->size();
  drop_events(plan);
  return P2P_OK;
}

p2p_status p2p_plan_destroy(p2p_plan plan) {
  if (!plan) return P2P_OK;
  p2p_status rc = check_plan(plan);
  if (rc != P2P_OK) return rc;
  return free_plan(plan);
}

}  // extern "C"
