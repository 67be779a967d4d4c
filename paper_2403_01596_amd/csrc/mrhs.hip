// Near-field apply for many right-hand sides on the matrix cores, and batches of
// uneven instances served by one launch.
//
// For a target box T and its neighbourhood S(T), Y_T += G_TS Q_S with G_TS the
// n_T x n_S matrix of kernel values (paper, sections 3.2-3.3: the same pairs as
// the single-RHS sweep) and Q_S the n_S x m block of strengths.  Work item = (one
// instance, one box, 16 targets, up to W right-hand sides).  Per step of 4
// sources, lane l evaluates G(target l % 16, source l / 16) in FP32 -- exactly
// the A-operand layout of v_mfma_f32_16x16x4_f32 -- and loads the strengths of
// its source for columns l % 16 + 16 t, the B-operand layout.  The complex
// product takes three real MFMAs per 16-column tile (the 3-multiplication form,
// one product fewer than the schoolbook four):
//   P1 += Gr Qr,  P2 += Gi Qi,  P3 += (Gr + Gi)(Qr + Qi),
//   Re Y = P1 - P2,  Im Y = P3 - P1 - P2.
// G never leaves registers; the accumulators hold D[i][j] at lane j + 16 (i / 4),
// register i % 4.  The loads of the next 4 sources are in flight while the
// matrix cores work on the current ones.
//
// Items are ordered instance by instance, boxes in Morton order, and cut into
// eight ranges of equal cost, one per XCD: workgroup w runs on XCD w % 8 and takes
// its items from that XCD's range, so neighbouring boxes, which share most of
// their sources, meet in the same L2.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mrhs.h"
#include "sweep.h"

namespace p2p {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kXcds = 8;
constexpr int kStepSrc = 4;      // sources per MFMA step (the K of 16x16x4)
constexpr int kGroupSrc = 512;   // neighbourhood entries staged in LDS at a time

// A group's neighbourhood entries {x, y, z, caller's row} into the wavefront's LDS,
// entries [sg, ge) of box T's list: CSR walks the box's own points first, then
// its neighbour boxes; TILES copies the box's replicated list.
template <bool CSR>
__device__ __forceinline__ void stage_group(int32_t T, int32_t sg, int32_t ge, const InstDesc& D, int64_t n,
                                            int4* ent, int lane) {
  if (CSR) {
    int32_t off = 0;
    const int32_t j0 = ld_uniform(D.nbr_start + T), j1 = ld_uniform(D.nbr_start + T + 1);
    for (int32_t j = j0 - 1; j < j1 && off < ge; ++j) {
      const int32_t S = j < j0 ? T : ld_uniform(D.nbr_idx + j);
      if (j >= j0 && S == T) continue;
      const int32_t a = ld_uniform(D.box_start + S), len = ld_uniform(D.box_start + S + 1) - a;
      const int32_t lo = max(off, sg), hi = min(off + len, ge);
      for (int32_t e = lo + lane; e < hi; e += kWave) {
        const int32_t p = a + (e - off);
        ent[e - sg] = make_int4(ld_global(D.sx32 + p), ld_global(D.sx32 + n + p), ld_global(D.sx32 + 2 * n + p),
                                ld_global(D.perm + p));
      }
      off += len;
    }
  } else {
    const int64_t tl = D.tl;
    for (int32_t e = sg + lane; e < ge; e += kWave)
      ent[e - sg] = make_int4(ld_global(D.tx32 + e), ld_global(D.tx32 + tl + e), ld_global(D.tx32 + 2 * tl + e),
                              ld_global(D.perm + ld_global(D.tsrc + e)));
  }
  wave_lds_sync();
}

// One step's operands for a lane: its source (coordinates and caller's row) and
// that source's strengths in the lane's column of every 16-column tile.
template <int TILES16>
struct StepSrc {
  int4 src;
  f2 q[TILES16];
};

// Strengths of the source in s.src, read straight from the caller's array: with
// 32-bit byte offsets from a wave-uniform base when the array spans < 4 GiB.
template <int TILES16, bool OFF32>
__device__ __forceinline__ void load_q(StepSrc<TILES16>& s, const float2* qb, int m, const uint32_t (&colb)[TILES16]) {
  if (OFF32) {
    const uint32_t rb = (uint32_t)s.src.w * (uint32_t)m * 8u;
    const char* base = reinterpret_cast<const char*>(qb);
#pragma unroll
    for (int q = 0; q < TILES16; ++q) s.q[q] = ld_global(reinterpret_cast<const f2*>(base + (rb + colb[q])));
  } else {
    const f2* row = reinterpret_cast<const f2*>(qb) + (int64_t)s.src.w * m;
#pragma unroll
    for (int q = 0; q < TILES16; ++q) s.q[q] = ld_global(row + colb[q] / 8u);
  }
}

// Marks a step's operands as produced here.  Applied to the group's first load,
// it keeps the compiler from merging that load with the in-loop prefetch into
// one load at the loop head, which would put the whole memory latency back in
// front of every step's products.
template <int TILES16>
__device__ __forceinline__ void pin_step(StepSrc<TILES16>& s) {
  asm volatile("" : "+v"(s.src.x), "+v"(s.src.y), "+v"(s.src.z), "+v"(s.src.w));
#pragma unroll
  for (int q = 0; q < TILES16; ++q) asm volatile("" : "+v"(s.q[q]));
}

// One step: the lane's kernel value, then three products per column tile.
template <int TILES16, bool HELM>
__device__ __forceinline__ void mfma_step(const StepSrc<TILES16>& s, bool valid, int32_t tx, int32_t ty, int32_t tz,
                                          float kturns, f4 (&p1)[TILES16], f4 (&p2)[TILES16],
                                          f4 (&p3)[TILES16]) {
  const F32::Geo g = F32::template geo<HELM, true>(tx, ty, tz, s.src.x, s.src.y, s.src.z, kturns);
  const float w = valid ? g.rinv : 0.0f;
  const float gr = g.c * w, gi = g.s * w;
  const float gs = gr + gi;
#pragma unroll
  for (int q = 0; q < TILES16; ++q) {
    const float qs = s.q[q].x + s.q[q].y;
    p1[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(gr, s.q[q].x, p1[q], 0, 0, 0);
    p2[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(gi, s.q[q].y, p2[q], 0, 0, 0);
    p3[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(gs, qs, p3[q], 0, 0, 0);
  }
}

template <int TILES16, bool HELM, bool CSR, bool OFF32>
__global__ void __launch_bounds__(kBlock) k_mrhs(BatchIO io, const InstDesc* __restrict__ desc,
                                              const int4* __restrict__ items, XcdSplit split, int wpb) {
  __shared__ int4 lds_ent[kWavesPerBlock][kGroupSrc];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  if (wv >= wpb) return;
  // XCD-aware item selection
  const int xcd = blockIdx.x % kXcds;
  const int64_t u = (int64_t)(blockIdx.x / kXcds) * wpb + wv;
  const int64_t it = split.start[xcd] + u;
  if (it >= split.start[xcd + 1]) return;
  const int4 item = items[it];
  const int inst = uniform(item.x);
  const int32_t T = uniform(item.y);
  const InstDesc& D = desc[inst];
  const int m = io.m;
  const int32_t bt0 = ld_uniform(D.box_start + T), bt1 = ld_uniform(D.box_start + T + 1);
  const int32_t t_first = bt0 + 16 * item.z;
  const int nt = min(16, bt1 - t_first);
  const int rg = item.w * 16 * TILES16;  // first right-hand side of this item
  if (rg >= m) return;  // items built for more right-hand sides than this call has
  // the neighbourhood's entries
  int32_t s0 = 0, s1 = 0;
  if (CSR) {
    const int32_t j1 = ld_uniform(D.nbr_start + T + 1);
    for (int32_t j = ld_uniform(D.nbr_start + T); j < j1; ++j) {
      const int32_t S = ld_uniform(D.nbr_idx + j);
      s1 += ld_uniform(D.box_start + S + 1) - ld_uniform(D.box_start + S);
    }
  } else {
    s0 = ld_uniform(D.tile_start + T);
    s1 = ld_uniform(D.tile_start + T + 1);
  }
  const int64_t n = D.n;
  const int i = lane & 15;    // target row of A, column of B
  const int kk = lane >> 4;   // source of the step
  const bool tvalid = i < nt;
  const int32_t t = t_first + (tvalid ? i : 0);
  const int32_t tx = ld_global(D.sx32 + t), ty = ld_global(D.sx32 + n + t), tz = ld_global(D.sx32 + 2 * n + t);
  const float kturns = D.kturns;
  const float2* qb = io.q[inst];
  // byte offsets of the lane's columns; columns past the call's last one read that
  // last column, and their sums are never stored
  uint32_t colb[TILES16];
#pragma unroll
  for (int q = 0; q < TILES16; ++q) colb[q] = 8u * (uint32_t)min(rg + i + 16 * q, m - 1);

  // 3-multiplication complex product: with P1 = Gr Qr, P2 = Gi Qi and
  // P3 = (Gr + Gi)(Qr + Qi), Re Y = P1 - P2 and Im Y = P3 - P1 - P2.
  f4 p1[TILES16], p2[TILES16], p3[TILES16];
#pragma unroll
  for (int q = 0; q < TILES16; ++q) {
    p1[q] = f4{0.f, 0.f, 0.f, 0.f};
    p2[q] = f4{0.f, 0.f, 0.f, 0.f};
    p3[q] = f4{0.f, 0.f, 0.f, 0.f};
  }
  int4* ent = lds_ent[wv];
  for (int32_t sg = s0; sg < s1; sg += kGroupSrc) {
    const int32_t cnt = min(s1 - sg, kGroupSrc);
    stage_group<CSR>(T, sg, sg + cnt, D, n, ent, lane);
    // Two operand sets in flight: the loads of the next step are issued before
    // the products of the current one.  Entries past the group's end reload its
    // first entry and are given a zero kernel value.
    StepSrc<TILES16> a, b;
    a.src = ent[kk < cnt ? kk : 0];
    load_q<TILES16, OFF32>(a, qb, m, colb);
    pin_step<TILES16>(a);
    for (int32_t e0 = 0; e0 < cnt; e0 += 2 * kStepSrc) {
      const int32_t e1 = e0 + kStepSrc + kk, e2 = e0 + 2 * kStepSrc + kk;
      b.src = ent[e1 < cnt ? e1 : 0];
      load_q<TILES16, OFF32>(b, qb, m, colb);
      mfma_step<TILES16, HELM>(a, tvalid && e0 + kk < cnt, tx, ty, tz, kturns, p1, p2, p3);
      a.src = ent[e2 < cnt ? e2 : 0];
      load_q<TILES16, OFF32>(a, qb, m, colb);
      mfma_step<TILES16, HELM>(b, tvalid && e1 < cnt, tx, ty, tz, kturns, p1, p2, p3);
    }
    wave_lds_sync();
  }
  // D[row][col]: lane j + 16 (row / 4), register row % 4
  float2* y = io.y[inst];
  const float sc = D.scale;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * kk + r;
    if (row < nt) {
      const int64_t yi = (int64_t)D.perm[t_first + row] * m;
#pragma unroll
      for (int q = 0; q < TILES16; ++q) {
        const int c = rg + i + 16 * q;
        const float re = p1[q][r] - p2[q][r];
        const float im = p3[q][r] - p1[q][r] - p2[q][r];
        if (c < m) y[yi + c] = make_float2(re * sc, im * sc);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
InstDesc make_desc(const p2p_plan_s* P) {
  InstDesc d;
  std::memset(&d, 0, sizeof(d));
  d.n = P->n;
  d.tl = P->tile_len;
  d.perm = P->perm;
  d.box_start = P->box_start;
  d.nbr_start = P->nbr_start;
  d.nbr_idx = P->nbr_idx;
  d.tile_start = P->tile_start;
  d.tsrc = P->tile_src;
  d.tx32 = P->tile_x32;
  d.sx32 = P->sx32;
  d.kturns = (float)(P->k * std::ldexp(1.0, P->qexp) / (2.0 * M_PI));
  d.scale = (float)(std::ldexp(1.0, -P->qexp) / (4.0 * M_PI));
  return d;
}

// Items of every instance: per box, ceil(n_T / 16) target tiles times the
// right-hand-side groups; cost = neighbourhood size.  Cut into eight ranges of
// equal cost (one per XCD).
p2p_status build_items(const std::vector<p2p_plan_s*>& plans, int m, int width, std::vector<int4>& items,
                       XcdSplit& split) {
  items.clear();
  std::vector<double> cost;
  const int groups = (m + width - 1) / width;
  for (size_t in = 0; in < plans.size(); ++in) {
    const p2p_plan_s* P = plans[in];
    if (P->B == 0) continue;
    std::vector<int32_t> bs(P->B + 1), ts(P->B + 1);
    P2P_HIP(hipMemcpy(bs.data(), P->box_start, sizeof(int32_t) * (P->B + 1), hipMemcpyDeviceToHost));
    P2P_HIP(hipMemcpy(ts.data(), P->tile_start, sizeof(int32_t) * (P->B + 1), hipMemcpyDeviceToHost));
    for (int64_t T = 0; T < P->B; ++T) {
      const int nT = bs[T + 1] - bs[T];
      const int nS = ts[T + 1] - ts[T];
      for (int mt = 0; mt * 16 < nT; ++mt)
        for (int g = 0; g < groups; ++g) {
          items.push_back(int4{(int)in, (int)T, mt, g});
          cost.push_back((double)nS + 8.0);
        }
    }
  }
  double total = 0;
  for (double c : cost) total += c;
  split.start[0] = 0;
  double acc = 0;
  int x = 1;
  for (size_t k = 0; k < items.size() && x < kXcds; ++k) {
    acc += cost[k];
    while (x < kXcds && acc >= total * x / kXcds) split.start[x++] = (int64_t)k + 1;
  }
  while (x <= kXcds) split.start[x++] = (int64_t)items.size();
  return P2P_OK;
}

unsigned mrhs_grid(const XcdSplit& split, int wpb) {
  int64_t most = 0;
  for (int x = 0; x < kXcds; ++x) most = std::max<int64_t>(most, split.start[x + 1] - split.start[x]);
  const int64_t per = (most + wpb - 1) / wpb;
  return (unsigned)std::max<int64_t>(1, per * kXcds);
}

p2p_status launch_mrhs(const MrhsSetup& S, const BatchIO& io, int width, int wpb, hipStream_t s, hipEvent_t e0,
                       hipEvent_t e1) {
  if (S.nitems == 0) return P2P_OK;
  if (e0) P2P_HIP(hipEventRecord(e0, s));
  const unsigned g = mrhs_grid(S.split, wpb);
#define P2P_MRHS(TL, H, C, O) \
  hipLaunchKernelGGL((k_mrhs<TL, H, C, O>), dim3(g), dim3(kBlock), 0, s, io, S.desc, S.items, S.split, wpb)
#define P2P_MRHS_O(TL, H, C) \
  do {                       \
    if (S.off32)             \
      P2P_MRHS(TL, H, C, true); \
    else                     \
      P2P_MRHS(TL, H, C, false); \
  } while (0)
#define P2P_MRHS_C(TL, H) \
  do {                    \
    if (S.csr)            \
      P2P_MRHS_O(TL, H, true); \
    else                  \
      P2P_MRHS_O(TL, H, false); \
  } while (0)
  if (width == 64) {
    if (S.helm) P2P_MRHS_C(4, true); else P2P_MRHS_C(4, false);
  } else {
    if (S.helm) P2P_MRHS_C(2, true); else P2P_MRHS_C(2, false);
  }
#undef P2P_MRHS_C
#undef P2P_MRHS_O
#undef P2P_MRHS
  P2P_HIP(hipGetLastError());
  if (e1) P2P_HIP(hipEventRecord(e1, s));
  return P2P_OK;
}

}  // namespace p2p
