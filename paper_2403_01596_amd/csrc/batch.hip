// Batches of plans for the multi-right-hand-side product, and its autotuner.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "mrhs.h"

struct p2p_batch_s {
  uint64_t magic;
  int device;
  int count, m;
  std::vector<p2p_plan_s*> plans;
  void* mem;                   // device: descriptors and both item lists
  p2p::MrhsSetup set64, set32, set16;  // items for 64, 32 and 16 right-hand sides per item
  int width, wpb;              // launch shape
  hipEvent_t last_use;         // recorded after each apply: destroy waits for it
  bool timing;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
};

namespace p2p {

constexpr uint64_t kBatchMagic = 0x7032705f62617463ull;

static p2p_status check_batch(p2p_batch_s* b) {
  if (!b || !handle_live(b) || b->magic != kBatchMagic) return fail(P2P_ERR_STATE, "invalid batch handle");
  return P2P_OK;
}

// Waits for the batch's last recorded launch, then releases it.
void batch_free(p2p_batch_s* b) {
  handle_remove(b);
  if (b->last_use) {
    (void)hipEventSynchronize(b->last_use);
    (void)hipEventDestroy(b->last_use);
  }
  for (auto& pr : b->timed) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  dmem_free(b->mem);
  b->magic = 0;
  delete b;
}

p2p_status batch_create(p2p_plan_s* const* plans, int count, int m, p2p_batch_s** out) {
  *out = nullptr;
  if (count < 1 || count > kMaxBatch) return fail(P2P_ERR_ARG, "count must be in [1, 32]");
  if (m < 1) return fail(P2P_ERR_ARG, "nrhs must be >= 1");
  for (int i = 0; i < count; ++i) {
    const p2p_plan_s* P = plans[i];
    if (!P || P->magic != kPlanMagic) return fail(P2P_ERR_STATE, "invalid plan handle in batch");
    if (P->distinct_sets) return fail(P2P_ERR_ARG, "batches take plans of one point set");
    if (P->precision != P2P_C64) return fail(P2P_ERR_DTYPE, "batches serve complex64 plans");
    if (P->layout != plans[0]->layout) return fail(P2P_ERR_ARG, "all plans of a batch need one layout");
    if (P->max_rhs < m) return fail(P2P_ERR_ARG, "a plan's max_rhs is below nrhs");
    if (P->device != plans[0]->device) return fail(P2P_ERR_ARG, "all plans of a batch need one device");
  }
  for (int i = 0; i < count; ++i) {  // the tables below are made from the plans' arrays on the host
    const p2p_status rc = wait_built(plans[i], nullptr, true);
    if (rc != P2P_OK) return rc;
  }
  p2p_batch_s* b = new (std::nothrow) p2p_batch_s();
  if (!b) return fail(P2P_ERR_NOMEM, "host allocation failed");
  b->magic = kBatchMagic;
  b->device = plans[0]->device;
  b->count = count;
  b->m = m;
  b->plans.assign(plans, plans + count);
  b->mem = nullptr;
  b->width = 64;
  b->wpb = 4;
  b->timing = false;
  b->last_use = nullptr;
  handle_add(b);
  if (hipEventCreateWithFlags(&b->last_use, hipEventDisableTiming) != hipSuccess) {
    b->last_use = nullptr;
    batch_free(b);
    return fail(P2P_ERR_HIP, "hipEventCreateWithFlags failed");
  }
  std::vector<InstDesc> desc(count);
  bool helm = false;
  for (int i = 0; i < count; ++i) {
    desc[i] = make_desc(plans[i]);
    helm = helm || plans[i]->k != 0.0;
  }
  std::vector<int4> it64, it32, it16;
  XcdSplit sp64, sp32, sp16;
  p2p_status rc = build_items(b->plans, m, 64, it64, sp64);
  if (rc == P2P_OK) rc = build_items(b->plans, m, 32, it32, sp32);
  if (rc == P2P_OK) rc = build_items(b->plans, m, 16, it16, sp16);
  if (rc != P2P_OK) {
    batch_free(b);
    return rc;
  }
  const size_t bd = sizeof(InstDesc) * count, b64 = sizeof(int4) * it64.size(), b32 = sizeof(int4) * it32.size(),
               b16 = sizeof(int4) * it16.size();
  const size_t off64 = (bd + 255) & ~size_t(255), off32 = (off64 + b64 + 255) & ~size_t(255),
               off16 = (off32 + b32 + 255) & ~size_t(255);
  b->mem = dmem_alloc(off16 + b16 + 16);
  if (!b->mem) {
    batch_free(b);
    return fail(P2P_ERR_NOMEM, "device allocation for the batch failed");
  }
  char* base = (char*)b->mem;
  hipError_t e = hipMemcpy(base, desc.data(), bd, hipMemcpyHostToDevice);
  if (e == hipSuccess && b64) e = hipMemcpy(base + off64, it64.data(), b64, hipMemcpyHostToDevice);
  if (e == hipSuccess && b32) e = hipMemcpy(base + off32, it32.data(), b32, hipMemcpyHostToDevice);
  if (e == hipSuccess && b16) e = hipMemcpy(base + off16, it16.data(), b16, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "hipMemcpy (batch tables)");
  }
  const bool csr = plans[0]->layout == P2P_LAYOUT_CSR;
  bool small = true;  // every instance's strengths within 32-bit byte offsets
  for (int i = 0; i < count; ++i) small = small && plans[i]->n * (int64_t)m * 8 < (int64_t(1) << 32);
  b->set64 = MrhsSetup{(InstDesc*)base, (int4*)(base + off64), (int64_t)it64.size(), sp64, helm, csr, small};
  b->set32 = MrhsSetup{(InstDesc*)base, (int4*)(base + off32), (int64_t)it32.size(), sp32, helm, csr, small};
  b->set16 = MrhsSetup{(InstDesc*)base, (int4*)(base + off16), (int64_t)it16.size(), sp16, helm, csr, small};
  *out = b;
  return P2P_OK;
}

static BatchIO make_io(const p2p_batch_s* b, const void* const* q, void* const* y, int m) {
  BatchIO io;
  std::memset(&io, 0, sizeof(io));
  io.count = b->count;
  io.m = m;
  for (int i = 0; i < b->count; ++i) {
    io.q[i] = (const float2*)q[i];
    io.y[i] = (float2*)y[i];
  }
  return io;
}

static p2p_status run(p2p_batch_s* b, const BatchIO& io, int width, int wpb, hipStream_t s,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  return launch_mrhs(width == 64 ? b->set64 : (width == 32 ? b->set32 : b->set16), io, width, wpb, s, e0, e1);
}

p2p_status batch_apply(p2p_batch_s* b, const void* const* q, void* const* y, int m, hipStream_t s, bool timing,
                       std::vector<std::pair<hipEvent_t, hipEvent_t>>* sink) {
  if (m < 1 || m > b->m) return fail(P2P_ERR_ARG, "nrhs must be in [1, the batch's nrhs]");
  for (int i = 0; i < b->count; ++i)
    if (b->plans[i]->n > 0 && (!q[i] || !y[i])) return fail(P2P_ERR_ARG, "q or y is NULL");
  const BatchIO io = make_io(b, q, y, m);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timing && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
    (void)hipGetLastError();
    e0 = e1 = nullptr;
  }
  // a call with at most 16 (32) right-hand sides fills 16-column (32-column) items
  // and would leave at least half of every wider item idle
  p2p_status rc = run(b, io, m <= 16 ? 16 : (m <= 32 ? 32 : b->width), b->wpb, s, e0, e1);
  if (e0) sink->emplace_back(e0, e1);
  if (rc == P2P_OK) record_use(b->last_use, s);
  return rc;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
static std::string tune_key(const p2p_batch_s* b) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) arch = prop.gcnArchName;
  int64_t n = 0, B = 0;
  for (auto* P : b->plans) {
    n += P->n;
    B += P->B;
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "arch=%s count=%d n=%lld m=%d layout=%s d=%.1f k=%s", arch.c_str(), b->count,
                (long long)n, b->m, b->plans[0]->layout == P2P_LAYOUT_CSR ? "csr" : "tiles",
                B ? (double)n / (double)B : 0.0, b->set64.helm ? "helmholtz" : "laplace");
  return buf;
}

static bool cache_lookup(const char* path, const std::string& key, int* width, int* wpb) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t tab = line.find('\t');
    if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != key.size()) continue;
    std::istringstream rest(line.substr(tab + 1));
    int w = 0, p = 0;
    if (rest >> w >> p && (w == 16 || w == 32 || w == 64) && (p == 1 || p == 2 || p == 4)) {
      *width = w;
      *wpb = p;
      return true;
    }
  }
  return false;
}

void batch_use_cache(p2p_batch_s* b, const char* path) {
  int width = b->width, wpb = b->wpb;
  if (cache_lookup(path, tune_key(b), &width, &wpb)) {
    b->width = width;
    b->wpb = wpb;
  }
}

p2p_status batch_tune(p2p_batch_s* b, const void* const* q, void* const* y, const char* path, hipStream_t s,
                      int32_t* chosen) {
  const std::string key = tune_key(b);
  int width = 64, wpb = 4;
  if (!cache_lookup(path, key, &width, &wpb)) {
    const BatchIO io = make_io(b, q, y, b->m);
    // item widths worth timing: up to 16 (32) right-hand sides fill only 16-column
    // (32-column) items, which is also what every call of that size uses
    const int widths[2] = {b->m <= 16 ? 16 : (b->m <= 32 ? 32 : 64), 32}, wpbs[3] = {4, 2, 1};
    const int nwidths = b->m <= 32 ? 1 : 2;
    float best = 1e30f;
    hipEvent_t e0, e1;
    P2P_HIP(hipEventCreate(&e0));
    P2P_HIP(hipEventCreate(&e1));
    for (int wi = 0; wi < nwidths; ++wi)
      for (int pi = 0; pi < 3; ++pi) {
        p2p_status rc = run(b, io, widths[wi], wpbs[pi], s);  // warm-up
        if (rc != P2P_OK) return rc;
        P2P_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) {
          rc = run(b, io, widths[wi], wpbs[pi], s);
          if (rc != P2P_OK) return rc;
        }
        P2P_HIP(hipEventRecord(e1, s));
        P2P_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        P2P_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          width = widths[wi];
          wpb = wpbs[pi];
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (path) {
      std::ofstream f(path, std::ios::app);
      f << key << '\t' << width << '\t' << wpb << '\t' << best / 3.0f << '\n';
    }
  }
  b->width = width;
  b->wpb = wpb;
  if (chosen) {
    chosen[0] = width;
    chosen[1] = wpb;
  }
  P2P_HIP(hipStreamSynchronize(s));
  return P2P_OK;
}

}  // namespace p2p

using namespace p2p;

extern "C" {

p2p_status p2p_batch_create(const p2p_plan* plans, int32_t count, int32_t nrhs, p2p_batch* out) {
  if (!out) return fail(P2P_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!plans) return fail(P2P_ERR_ARG, "plans is NULL");
  return batch_create(plans, count, nrhs, out);
}

p2p_status p2p_batch_apply(p2p_batch batch, const void* const* q, void* const* y, void* stream) {
  p2p_status rc = check_batch(batch);
  if (rc != P2P_OK) return rc;
  if (!q || !y) return fail(P2P_ERR_ARG, "q or y is NULL");
  return batch_apply(batch, q, y, batch->m, (hipStream_t)stream, batch->timing, &batch->timed);
}

p2p_status p2p_batch_tune(p2p_batch batch, const void* const* q, void* const* y, const char* cache_path,
                          void* stream, int32_t* chosen) {
  p2p_status rc = check_batch(batch);
  if (rc != P2P_OK) return rc;
  if (!q || !y) return fail(P2P_ERR_ARG, "q or y is NULL");
  return batch_tune(batch, q, y, cache_path, (hipStream_t)stream, chosen);
}

p2p_status p2p_batch_timing(p2p_batch batch, int enable) {
  p2p_status rc = check_batch(batch);
  if (rc != P2P_OK) return rc;
  batch->timing = enable != 0;
  return P2P_OK;
}

p2p_status p2p_batch_timing_read(p2p_batch batch, double* ms, int64_t* calls) {
  p2p_status rc = check_batch(batch);
  if (rc != P2P_OK) return rc;
  if (!ms || !calls) return fail(P2P_ERR_ARG, "ms or calls is NULL");
  double total = 0.0;
  for (auto& pr : batch->timed) {
    float t = 0.f;
    P2P_HIP(hipEventSynchronize(pr.second));
    P2P_HIP(hipEventElapsedTime(&t, pr.first, pr.second));
    total += t;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  *ms = total;
  *calls = (int64_t)batch->timed.size();
  batch->timed.clear();
  return P2P_OK;
}

p2p_status p2p_batch_destroy(p2p_batch batch) {
  if (!batch) return P2P_OK;
  p2p_status rc = check_batch(batch);
  if (rc != P2P_OK) return rc;
  batch_free(batch);
  return P2P_OK;
}

}  // extern "C"
