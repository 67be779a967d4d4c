// Multi-right-hand-side apply on the matrix cores and batches of instances
// (internal to libp2p).
#pragma once

#include <vector>

#include "common.h"

namespace p2p {

constexpr int kMaxBatch = 32;  // instances per batch (their pointers travel as kernel arguments)
constexpr int kMrhsMin = 6;   // right-hand sides from which p2p_apply uses the matrix cores

// Geometry of one instance, in device memory, read by the batched kernels.
struct InstDesc {
  int64_t n, tl;
  const int32_t* perm;
  const int32_t* box_start;
  const int32_t* nbr_start;
  const int32_t* nbr_idx;
  const int32_t* tile_start;
  const int32_t* tsrc;
  const int32_t* tx32;
  const int32_t* sx32;
  float kturns;      // k * 2^qexp / (2 pi)
  float scale;       // 2^-qexp / (4 pi)
  int32_t may_coincide;  // points of distinct boxes may coincide
  // close pairs, as in p2p_plan_s: per-box near flags, and the FP64 coordinates
  // their differences come from
  const int32_t* near;
  const double* sx64;    // [3][n] FP64 coordinates, sorted order
  double qinv;           // 2^-qexp
};

// Per-call pointers, passed by value (so that a captured graph holds them).
struct BatchIO {
  const float2* q[kMaxBatch];
  float2* y[kMaxBatch];
  int count;
  int m;
};

// Item ranges of the eight XCDs.
struct XcdSplit {
  int64_t start[9];
};

struct MrhsSetup {
  InstDesc* desc;  // device [count]
  int4* items;     // device [nitems]
  int64_t nitems;
  XcdSplit split;
  bool helm, csr;
  bool off32;      // every instance's strengths span less than 4 GiB (32-bit byte offsets)
};

// Launch variant for m right-hand sides: the fast form needs 32-bit offsets and
// every item's columns inside [0, m).
inline bool mrhs_fast(const MrhsSetup& S, int m, int width) { return S.off32 && m % width == 0; }

InstDesc make_desc(const p2p_plan_s* P);
p2p_status build_items(const std::vector<p2p_plan_s*>& plans, int m, int width, std::vector<int4>& items,
                       XcdSplit& split);
unsigned mrhs_grid(const XcdSplit& split, int wpb);
p2p_status launch_mrhs(const MrhsSetup& S, const BatchIO& io, int width, int wpb, hipStream_t s,
                       hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// batches (batch.hip)
p2p_status batch_create(p2p_plan_s* const* plans, int count, int m, p2p_batch_s** out);
p2p_status batch_apply(p2p_batch_s* b, const void* const* q, void* const* y, int m, hipStream_t s, bool timing,
                       std::vector<std::pair<hipEvent_t, hipEvent_t>>* sink);
void batch_free(p2p_batch_s* b);
// The launch shape recorded for this batch's workload key in an autotuner cache
// file, if there is one (no timing).
void batch_use_cache(p2p_batch_s* b, const char* path);

}  // namespace p2p
