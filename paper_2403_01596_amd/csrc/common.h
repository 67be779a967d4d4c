// Internal declarations shared by the HIP sources of libp2p (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/p2p.h"

namespace p2p {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kIdBits = 21;      // box ids per axis live in [0, 2^21)
constexpr int kBlock = 256;      // threads per workgroup for the streaming kernels

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

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct DeviceArena {
  // Device memory from the stream-ordered pool; released in one go.
  void* base = nullptr;
  size_t bytes = 0;
};

}  // namespace p2p

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
  // replicated per-box source lists (TILES)
  int32_t* tile_start; // [B+1]
  int32_t* tile_src;   // [tile_len] sorted position of the source
  double* tile_x64;    // [3][tile_len] (FP64 plans)
  int32_t* tile_x32;   // [3][tile_len] (FP32 plans)
  // scratch for apply/backward: strengths and upstream gradients in sorted order
  void* q_sorted;      // [n * max_rhs] complex
  void* g_sorted;      // [n * max_rhs] complex
  // diagnostics: event pairs around the sweep kernels
  bool timing;
  std::vector<std::pair<hipEvent_t, hipEvent_t>>* timed;
};

namespace p2p {

constexpr uint64_t kPlanMagic = 0x7032705f706c616eull;

// plan build (plan.hip)
p2p_status build_plan(p2p_plan_s* P, const double* xyz, const int32_t* ids, hipStream_t s);
p2p_status count_pairs(p2p_plan_s* P, hipStream_t s);
p2p_status box_ids(const double* xyz, int64_t n, const double* origin, double h, int32_t* ids, hipStream_t s);

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

// Sum over the 64 lanes of a wavefront; every lane must be active.  The total
// ends up in lane 63 and is returned to all lanes.  Row-local butterflies
// (quad permutes, row shifts), then the row broadcasts 15 and 31.
__device__ __forceinline__ float wave_sum(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xb1, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4e, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x114, 0xf, 0xe, true));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x118, 0xf, 0xc, true));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xa, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xc, 0xf, false));
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
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

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace p2p
