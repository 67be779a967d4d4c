// Internal declarations shared by the HIP sources of libp2p (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/p2p.h"

namespace p2p {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kIdBits = 21;      // box ids per axis live in [0, 2^21)
constexpr int kBlock = 256;      // threads per workgroup for the streaming kernels
// largest point count: neighbour-list entries (at most 27 n) are 32-bit offsets
constexpr int64_t kMaxPoints = 0x7fffffff / 27;
// FP32 plans: near pairs whose fixed-point difference is shorter than this many
// quanta get their kernel value from the FP64 coordinates (see p2p_plan_s).
// Every other pair is at least 2^20 quanta apart, so the rounding of its
// coordinates (at most one quantum per axis) perturbs its term by at most
// sqrt(3) 2^-20 relative.
constexpr int kCloseBits = 20;
constexpr int32_t kCloseQuanta = 1 << kCloseBits;

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
p2p_status fail(p2p_status s, const std::string& msg);
p2p_status hip_fail(hipError_t e, const char* what);

#define P2P_HIP(call)                                                   \
  do {                                                                  \
    hipError_t e_ = (call);                                             \
    if (e_ != hipSuccess) return ::p2p::hip_fail(e_, #call);            \
  } while (0)

}  // namespace p2p

struct p2p_batch_s;

struct p2p_plan_s {
  uint64_t magic;
  int device;
  int64_t n, B, nnz, tile_len, n_slots;
  int64_t n_pairs, n_zero;  // -1 until counted
  int32_t t_max;
  double k;
  p2p_dtype precision;
  p2p_layout layout;
  int32_t max_rhs;
  int32_t qexp;      // quantum exponent: FP32 coordinates are integers in units of 2^qexp
  double max_sep;    // largest per-axis difference of a near pair
  bool may_coincide; // bounding boxes of two distinct neighbour boxes intersect
  double max_turns;  // largest k r / (2 pi) over near pairs (bound)
  size_t device_bytes;
  void* arena;       // first allocation: arrays sized by n
  void* arena2;      // second allocation: neighbour lists and replicated lists

  // sorted-order tables
  int32_t* perm;       // [n]   sorted position -> original index
  uint64_t* box_key;   // [B]
  int32_t* box_start;  // [B+1]
  int32_t* nbr_start;  // [B+1]
  int32_t* nbr_idx;    // [nnz]
  int32_t* work;       // [B]   boxes in processing order (largest pair count first)
  // geometry, sorted order
  double* sx64;        // [3][n] FP64 coordinates (SoA)
  int32_t* sx32;       // [3][n] fixed-point coordinates, low 32 bits (FP32 plans)
  // replicated per-box source lists (TILES); the offsets are kept for both layouts
  // (CSR sweeps take each box's list length from them)
  int32_t* tile_start; // [B+1]
  int32_t* tile_src;   // [tile_len] sorted position of the source
  double* tile_x64;    // [3][tile_len] (FP64 plans)
  int32_t* tile_x32;   // [3][tile_len] (FP32 plans)
  // FP32 plans: per box, nonzero if the bounding box of some other neighbour box
  // comes within kCloseQuanta + 2 quanta of the box's own on every axis, or if two
  // of the box's own points are within kCloseQuanta quanta of each other on every
  // axis.  Only such boxes can hold a pair whose fixed-point difference is shorter
  // than kCloseQuanta quanta; the kernels take those pairs' differences from the
  // FP64 coordinates.
  int32_t* near;       // [B]
  // Plans of distinct target and source sets: the plan's points are the targets
  // [0, n_targets) followed by the sources; each box lists its targets first, and
  // its sources start at src_start[T].  Null for one set.
  bool distinct_sets;
  int64_t n_targets;
  int32_t* src_start;  // [B + 1]
  int64_t n_close;     // ordered near pairs closer than kCloseQuanta quanta, -1 until counted
  int64_t n_near;      // boxes marked near (FP32 plans), counted with n_close
  // scratch for apply/backward: strengths and upstream gradients in sorted order
  void* q_sorted;      // [n * max_rhs] complex
  void* g_sorted;      // [n * max_rhs] complex
  // complex64 plans with max_rhs >= 16: the matrix-core path for many right-hand sides
  p2p_batch_s* self_batch;
  hipEvent_t last_use;  // recorded after each call's work (used: at least once)
  hipEvent_t ready;     // recorded after the build
  hipStream_t build_stream;
  bool built;           // the build is known to be complete
  bool used;            // destroy releases the plan's memory behind last_use, else ready
  // diagnostics: event pairs around the sweep kernels
  bool timing;
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* timed;
};

namespace p2p {

// Box T's sources are the sorted positions [src_begin[T], box_start[T + 1]) and its
// targets [box_start[T], tgt_end[T]): all its points for one set.
inline const int32_t* src_begin(const p2p_plan_s* P) { return P->src_start ? P->src_start : P->box_start; }
inline const int32_t* tgt_end(const p2p_plan_s* P) { return P->src_start ? P->src_start : P->box_start + 1; }

constexpr uint64_t kPlanMagic = 0x7032705f706c616eull;

// Live handles (plans and batches).  A handle is looked up here before it is
// dereferenced, so a destroyed or foreign pointer is reported as an invalid
// handle instead of being read.
void handle_add(const void* h);
void handle_remove(const void* h);
bool handle_live(const void* h);

// Records ev on stream s unless s is being captured into a graph (a recorded
// event there would only be reached by replays): the last call a destroy has to
// wait for.
bool record_use(hipEvent_t ev, hipStream_t s);  // true: recorded

// Before work on plan P that runs on stream s: when s is not the stream the plan
// was built on, waits for the build on the host (once; later calls find it
// complete).  Host reads of the plan's arrays pass s = nullptr with force.
p2p_status wait_built(p2p_plan_s* P, hipStream_t s, bool force = false);

// device memory cache and pinned staging (memory.hip)
// P2P_TEST_FAIL_ALLOC=n (test hook): the n-th allocation after the variable is set
// (or changed) fails as if the device were out of memory.
void* dmem_alloc(size_t bytes);  // current device; nullptr when out of memory
void dmem_free(void* p);         // the caller guarantees no pending work uses p
// Stream-ordered releases (no host wait): the blocks are handed out again once the
// work before event ev has completed; the cache takes ownership of ev (null: no
// pending work, released at once).  At most two blocks per call.
void dmem_free_after(void* const* blocks, int count, hipEvent_t ev);
// The blocks (at most two; null entries skipped) are handed out again once the
// work enqueued on s so far has completed: one event for all of them.
void dmem_free_on(void* const* blocks, int count, hipStream_t s);
struct StagingLock {
  void* host = nullptr;  // pinned host buffer, valid while the lock is held
  std::unique_lock<std::mutex> lock;
};
StagingLock staging(size_t bytes);

// plan build (plan.hip)
// Leaf grid of the positions: id = floor((x - o) / h) per axis.
struct GridSpec {
  double o[3];
  double h;
};

// ids null: computed from xyz with gspec.
p2p_status build_plan(p2p_plan_s* P, const double* xyz, const int32_t* ids, const GridSpec* gspec, hipStream_t s);
p2p_status count_pairs(p2p_plan_s* P, hipStream_t s);
// The leaf height for a clustering threshold (p2p_leaf_level).
p2p_status leaf_level(const double* xyz, int64_t n, const double* origin, double size, int32_t ct, int32_t lmin,
                      int32_t* level, double* h, int32_t* t_max, hipStream_t s);
p2p_status box_ids(const double* xyz, int64_t n, const double* origin, double h, int32_t* ids, hipStream_t s);
// The same without allocation: the status word in a static device array.
p2p_status box_ids_noalloc(const double* xyz, int64_t n, const double* origin, double h, int32_t* ids,
                           hipStream_t s);

// diagnostics (api.hip): events around the sweep kernels of one call
struct SweepTimer {
  p2p_plan_s* P;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SweepTimer(p2p_plan_s* plan, hipStream_t st);
  void start();
  void stop();
};

// apply / backward (apply.hip, backward.hip)
p2p_status launch_apply(p2p_plan_s* P, const void* q, void* y, int nrhs, hipStream_t s);
p2p_status launch_backward(p2p_plan_s* P, const void* q, const void* gy, void* gq, double* gx, int nrhs,
                           hipStream_t s);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

template <typename T>
__device__ __forceinline__ T uniform(T v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// Load through the constant address space: with a wave-uniform address this is a
// scalar load.  Only for data the running kernel does not write.
template <typename T>
__device__ __forceinline__ T ld_uniform(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}

// Load through the global address space (a vector memory load that waits on the
// vector counter only), for pointers the compiler sees as generic.
template <typename T>
__device__ __forceinline__ T ld_global(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// Sum over the 64 lanes of a wavefront, valid in lane 63 only; every lane must be
// active.  Quad butterflies, then row shifts by 4 and 8 (lane 15 of each row holds
// the row's sum), then the row broadcasts 15 and 31 (lane 63 gathers the four
// rows).  Every step reads 0 where its source lane does not exist, and the values
// the broadcasts leave in rows 0-2 never flow into lane 63, so all masks stay full
// and each step is a single DPP add.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// Reductions to lane 63 for max / or: out-of-range sources return the lane's own
// value, so no identity element is needed.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_keep_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_keep_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)rhi << 32) | (uint32_t)rlo);
}
__device__ __forceinline__ uint32_t wave_max63(uint32_t v) {
  v = max(v, dpp_keep_u32<0xb1>(v));
  v = max(v, dpp_keep_u32<0x4e>(v));
  v = max(v, dpp_keep_u32<0x114>(v));
  v = max(v, dpp_keep_u32<0x118>(v));
  v = max(v, dpp_keep_u32<0x142>(v));
  v = max(v, dpp_keep_u32<0x143>(v));
  return v;
}
__device__ __forceinline__ uint32_t wave_or63(uint32_t v) {
  v |= dpp_keep_u32<0xb1>(v);
  v |= dpp_keep_u32<0x4e>(v);
  v |= dpp_keep_u32<0x114>(v);
  v |= dpp_keep_u32<0x118>(v);
  v |= dpp_keep_u32<0x142>(v);
  v |= dpp_keep_u32<0x143>(v);
  return v;
}
__device__ __forceinline__ double wave_max63(double v) {
  v = fmax(v, dpp_keep_f64<0xb1>(v));
  v = fmax(v, dpp_keep_f64<0x4e>(v));
  v = fmax(v, dpp_keep_f64<0x114>(v));
  v = fmax(v, dpp_keep_f64<0x118>(v));
  v = fmax(v, dpp_keep_f64<0x142>(v));
  v = fmax(v, dpp_keep_f64<0x143>(v));
  return v;
}
// 32-bit integer sum to lane 63 (out-of-range sources read 0).
__device__ __forceinline__ uint32_t wave_add63(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xf, 0xf, true);
  return v;
}

// The same reductions over each half of the wavefront separately (lanes 0-31 and
// 32-63), for code that works on two items per wavefront: the first five steps
// only.  Lane 31 then holds the lower half's result and lane 63 the upper half's:
// row broadcast 15 combines row 0 into row 1 and row 2 into row 3, and what it
// carries from row 1 into row 2 reaches neither lane.
__device__ __forceinline__ uint32_t half_add(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xf, 0xf, true);
  return v;
}
__device__ __forceinline__ uint32_t half_or(uint32_t v) {
  v |= dpp_keep_u32<0xb1>(v);
  v |= dpp_keep_u32<0x4e>(v);
  v |= dpp_keep_u32<0x114>(v);
  v |= dpp_keep_u32<0x118>(v);
  v |= dpp_keep_u32<0x142>(v);
  return v;
}
__device__ __forceinline__ double half_max(double v) {
  v = fmax(v, dpp_keep_f64<0xb1>(v));
  v = fmax(v, dpp_keep_f64<0x4e>(v));
  v = fmax(v, dpp_keep_f64<0x114>(v));
  v = fmax(v, dpp_keep_f64<0x118>(v));
  v = fmax(v, dpp_keep_f64<0x142>(v));
  return v;
}
// Lane 31's value (wave-uniform).
__device__ __forceinline__ uint32_t lane31(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 31); }
__device__ __forceinline__ uint64_t lane31(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 31);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 31);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double lane31(double v) {
  return __builtin_bit_cast(double, lane31(__builtin_bit_cast(uint64_t, v)));
}

__device__ __forceinline__ float wave_sum63(float v) {
  v += dpp_f32<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f32<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_f32<0x114>(v);  // row_shr:4
  v += dpp_f32<0x118>(v);  // row_shr:8
  v += dpp_f32<0x142>(v);  // row_bcast:15
  v += dpp_f32<0x143>(v);  // row_bcast:31
  return v;
}
// Sums over the 64 lanes of two values at once: lane 31 receives the sum of a,
// lane 63 the sum of b.  Exchanging lanes 32-63 of a with lanes 0-31 of b puts
// the halves of a in lanes 0-31 and those of b in lanes 32-63, so one add and the
// first five steps above (which leave each half's total in its last lane) serve
// both values.
__device__ __forceinline__ float wave_sum_pair(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                                  false, false);
  float v = __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
  v += dpp_f32<0xb1>(v);
  v += dpp_f32<0x4e>(v);
  v += dpp_f32<0x114>(v);
  v += dpp_f32<0x118>(v);
  v += dpp_f32<0x142>(v);
  return v;
}
__device__ __forceinline__ double wave_sum63(double v) {
  v += dpp_f64<0xb1>(v);
  v += dpp_f64<0x4e>(v);
  v += dpp_f64<0x114>(v);
  v += dpp_f64<0x118>(v);
  v += dpp_f64<0x142>(v);
  v += dpp_f64<0x143>(v);
  return v;
}

// The same for doubles: both 32-bit halves take the same lane exchange.
__device__ __forceinline__ double wave_sum_pair(double a, double b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  const double x = __builtin_bit_cast(double, ((uint64_t)(unsigned)hi[0] << 32) | (unsigned)lo[0]);
  const double y = __builtin_bit_cast(double, ((uint64_t)(unsigned)hi[1] << 32) | (unsigned)lo[1]);
  double v = x + y;
  v += dpp_f64<0xb1>(v);
  v += dpp_f64<0x4e>(v);
  v += dpp_f64<0x114>(v);
  v += dpp_f64<0x118>(v);
  v += dpp_f64<0x142>(v);
  return v;
}

// Morton key of box ids: bit 3b <- bit b of x, 3b+1 <- y, 3b+2 <- z.
__host__ __device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}
__host__ __device__ __forceinline__ uint64_t morton3(uint32_t ix, uint32_t iy, uint32_t iz) {
  return spread3(ix) | (spread3(iy) << 1) | (spread3(iz) << 2);
}

// Inverse of spread3: bits 0, 3, 6, ... of x back into a 21-bit integer.
__host__ __device__ __forceinline__ uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x | (x >> 4)) & 0x100f00f00f00f00full;
  x = (x | (x >> 8)) & 0x001f0000ff0000ffull;
  x = (x | (x >> 16)) & 0x001f00000000ffffull;
  x = (x | (x >> 32)) & 0x00000000001fffffull;
  return (uint32_t)x;
}

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace p2p
