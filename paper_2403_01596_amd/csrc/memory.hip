// Device memory cache and pinned staging for the plan build.
//
// Plans are built and released often (one per geometry, and every benchmark
// step), and the driver's allocation calls cost tens to hundreds of
// microseconds each.  Blocks released by the library are kept per device and
// handed out again for requests they fit; readbacks of the plan build's small
// status block go through one pinned host buffer per device.
//
// Releases are stream-ordered: a block whose last work may still be in flight
// waits, with an event recorded behind that work, on a pending list, and joins
// the free blocks when a later allocation finds the event complete.  No release
// waits on the host.
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace p2p {

namespace {

constexpr size_t kGranule = size_t(2) << 20;          // 2 MiB
constexpr size_t kCacheCap = size_t(64) << 30;        // cached bytes kept per device at most
constexpr int kMaxDevices = 64;

// Blocks released behind work that may still be running, with the event
// recorded after that work.
struct Pending {
  void* p[2];
  int count;
  hipEvent_t ev;
};

struct DeviceCache {
  std::multimap<size_t, void*> free_blocks;   // size -> block
  std::unordered_map<void*, size_t> size_of;  // every block handed out or cached
  size_t cached = 0;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> spare_events;  // completed events, recorded again by later releases
  void* staging = nullptr;
  size_t staging_bytes = 0;
  std::mutex staging_mu;
};

std::mutex g_mu;
DeviceCache g_dev[kMaxDevices];

int current_device() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kMaxDevices) return -1;
  return d;
}

void release_cached(DeviceCache& c) {
  for (auto& kv : c.free_blocks) {
    (void)hipFree(kv.second);
    c.size_of.erase(kv.second);
  }
  c.free_blocks.clear();
  c.cached = 0;
}

// (lock held) a block whose work is done joins the free blocks, or goes back to
// the driver when the cache is full
void cache_block(DeviceCache& c, void* p) {
  auto it = c.size_of.find(p);
  if (it == c.size_of.end()) return;
  if (c.cached + it->second > kCacheCap) {
    c.size_of.erase(it);
    (void)hipFree(p);
    return;
  }
  c.free_blocks.emplace(it->second, p);
  c.cached += it->second;
}

constexpr size_t kSpareEvents = 64;

// (lock held) pending blocks whose event has completed join the free blocks;
// wait: every pending event is waited for first (out-of-memory retry)
void reap(DeviceCache& c, bool wait) {
  size_t i = 0;
  while (i < c.pending.size()) {
    Pending& q = c.pending[i];
    const hipError_t e = wait ? hipEventSynchronize(q.ev) : hipEventQuery(q.ev);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // not ready: no error of the caller's
      if (!wait) {
        ++i;
        continue;
      }
    }
    for (int k = 0; k < q.count; ++k) cache_block(c, q.p[k]);
    if (c.spare_events.size() < kSpareEvents) c.spare_events.push_back(q.ev);
    else (void)hipEventDestroy(q.ev);
    q = c.pending.back();
    c.pending.pop_back();
  }
}

// P2P_TEST_FAIL_ALLOC=n: the n-th allocation after the variable is set (or given a
// new value) fails.  Tests drive the out-of-memory paths with it.
bool injected_failure() {
  static std::string armed;
  static long long seen = 0;
  const char* v = std::getenv("P2P_TEST_FAIL_ALLOC");
  if (!v || !*v) {
    armed.clear();
    return false;
  }
  if (armed != v) {
    armed = v;
    seen = 0;
  }
  return ++seen == std::atoll(v);
}

}  // namespace

void* dmem_alloc(size_t bytes) {
  const int d = current_device();
  if (d < 0) return nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (injected_failure()) return nullptr;
  }
  const size_t want = (std::max<size_t>(bytes, 1) + kGranule - 1) / kGranule * kGranule;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCache& c = g_dev[d];
  if (!c.pending.empty()) reap(c, false);
  // the smallest cached block that fits and wastes at most half of itself
  auto it = c.free_blocks.lower_bound(want);
  if (it != c.free_blocks.end() && it->first <= 2 * want) {
    void* p = it->second;
    c.cached -= it->first;
    c.free_blocks.erase(it);
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess || !p) {
    (void)hipGetLastError();
    reap(c, true);  // wait for the pending blocks, give the cache back to the driver, try once more
    release_cached(c);
    p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  c.size_of[p] = want;
  return p;
}

void dmem_free(void* p) {
  if (!p) return;
  const int d = current_device();
  std::lock_guard<std::mutex> lk(g_mu);
  if (d < 0) return;
  cache_block(g_dev[d], p);
}

void dmem_free_after(void* const* blocks, int count, hipEvent_t ev) {
  const int d = current_device();
  std::lock_guard<std::mutex> lk(g_mu);
  if (d < 0) return;
  DeviceCache& c = g_dev[d];
  Pending q{{nullptr, nullptr}, 0, ev};
  for (int k = 0; k < count && k < 2; ++k)
    if (blocks[k]) q.p[q.count++] = blocks[k];
  if (!ev) {
    for (int k = 0; k < q.count; ++k) cache_block(c, q.p[k]);
    return;
  }
  c.pending.push_back(q);
}

void dmem_free_on(void* const* blocks, int count, hipStream_t s) {
  bool any = false;
  for (int k = 0; k < count && k < 2; ++k) any = any || blocks[k];
  if (!any) return;
  hipEvent_t ev = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const int d = current_device();
    if (d >= 0 && !g_dev[d].spare_events.empty()) {
      ev = g_dev[d].spare_events.back();
      g_dev[d].spare_events.pop_back();
    }
  }
  if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
  if (!ev || hipEventRecord(ev, s) != hipSuccess) {  // no event: wait on the host instead
    (void)hipGetLastError();
    if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamSynchronize(s);
    for (int k = 0; k < count && k < 2; ++k) dmem_free(blocks[k]);
    return;
  }
  dmem_free_after(blocks, count, ev);
}

StagingLock staging(size_t bytes) {
  StagingLock s;
  const int d = current_device();
  if (d < 0) return s;
  DeviceCache& c = g_dev[d];
  s.lock = std::unique_lock<std::mutex>(c.staging_mu);
  if (c.staging_bytes < bytes) {
    if (c.staging) (void)hipHostFree(c.staging);
    c.staging = nullptr;
    c.staging_bytes = 0;
    const size_t want = std::max<size_t>(bytes, 4096);
    if (hipHostMalloc(&c.staging, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      c.staging = nullptr;
      return s;
    }
    c.staging_bytes = want;
  }
  s.host = c.staging;
  return s;
}

}  // namespace p2p
