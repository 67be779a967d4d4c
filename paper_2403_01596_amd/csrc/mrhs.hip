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
constexpr int kGroupSrc = 512;   // LDS slots per wavefront for staged neighbourhood entries
constexpr int kGroupCap = kGroupSrc - 2 * kStepSrc;  // real entries per group (the rest: padding)

// A group's neighbourhood entries into the wavefront's LDS: {x, y, z, r} with r the
// source's row in the caller's array (FAST: its byte offset, row * m * 8), and in
// pos the source's sorted position (read only for close pairs).  Entries
// [sg, ge) of box T's list: CSR walks the box's own points first, then its
// neighbour boxes; TILES copies the box's replicated list.  The slots from ge - sg
// to 8 past the next multiple of 8 repeat the first entry, so that steps and the
// prefetch of the step after the last never read a slot that was not written.
template <bool CSR, bool FAST>
__device__ __forceinline__ void stage_group(int32_t T, int32_t sg, int32_t ge, const InstDesc& D, int64_t n, int m,
                                            int4* ent, int32_t* pos, int lane) {
  const uint32_t rs = FAST ? 8u * (uint32_t)m : 1u;
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
                                (int32_t)((uint32_t)ld_global(D.perm + p) * rs));
        pos[e - sg] = p;
      }
      off += len;
    }
  } else {
    const int64_t tl = D.tl;
    for (int32_t e = sg + lane; e < ge; e += kWave) {
      const int32_t p = ld_global(D.tsrc + e);
      ent[e - sg] = make_int4(ld_global(D.tx32 + e), ld_global(D.tx32 + tl + e), ld_global(D.tx32 + 2 * tl + e),
                              (int32_t)((uint32_t)ld_global(D.perm + p) * rs));
      pos[e - sg] = p;
    }
  }
  wave_lds_sync();
  const int32_t cnt = ge - sg, padded = ((cnt + 2 * kStepSrc - 1) & ~(2 * kStepSrc - 1)) + 2 * kStepSrc;
  if (lane < padded - cnt) {
    ent[cnt + lane] = ent[0];
    pos[cnt + lane] = pos[0];
  }
  wave_lds_sync();
}

// One step's operands for a lane: its source (coordinates and row) and that
// source's strengths in the lane's column of every 16-column tile.
template <int TILES16>
struct StepSrc {
  int4 src;
  f2 q[TILES16];
};

// Strengths of the source in s.src, read straight from the caller's array.  FAST:
// one 32-bit byte offset from a wave-uniform base, the tiles 128 bytes apart
// (immediate offsets).  Otherwise 64-bit addressing and clamped columns.
template <int TILES16, bool FAST>
__device__ __forceinline__ void load_q(StepSrc<TILES16>& s, const float2* qb, int m, uint32_t lcol,
                                       const int32_t (&col)[TILES16]) {
  if (FAST) {
    const char* base = reinterpret_cast<const char*>(qb) + ((uint32_t)s.src.w + lcol);
#pragma unroll
    for (int q = 0; q < TILES16; ++q) s.q[q] = ld_global(reinterpret_cast<const f2*>(base + 128 * q));
  } else {
    const f2* row = reinterpret_cast<const f2*>(qb) + (int64_t)s.src.w * m;
#pragma unroll
    for (int q = 0; q < TILES16; ++q) s.q[q] = ld_global(row + col[q]);
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

// The lane's target: its fixed-point coordinates, its sorted position t, and its
// own entry's index within the current group (its self pair).
struct StepTgt {
  int32_t x, y, z, t, self_e;
};

// One step: the lane's kernel value, then three products per column tile.  The
// lane's source is entry ei of the group (cnt real entries).  MASK: the pair may be
// at distance zero, closer than kCloseQuanta quanta (then its difference comes
// from the FP64 coordinates, as in the single-column sweep) or past the list's end
// (then the kernel value is zero).
template <int TILES16, bool HELM, bool MASK>
__device__ __forceinline__ void mfma_step(const StepSrc<TILES16>& s, int32_t ei, int32_t cnt, const StepTgt& tg,
                                          const int32_t* pos, const ExactCtx& E, float kturns, f4 (&p1)[TILES16],
                                          f4 (&p2)[TILES16], f4 (&p3)[TILES16]) {
  F32::Geo g = F32::template geo<HELM, MASK>(tg.x, tg.y, tg.z, s.src.x, s.src.y, s.src.z, kturns);
  bool valid = true;
  if (MASK) {
    valid = ei < cnt;
    const bool close = valid && g.r2 < kCloseR2 && ei != tg.self_e;
    if (__ballot(close)) {
      if (close) g = exact_geo<HELM>(E, tg.t, pos[ei], kturns);
    }
  }
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

// Operands and accumulators of one wavefront's item.
template <int TILES16>
struct MrhsState {
  StepSrc<TILES16> a, b;
  f4 p1[TILES16], p2[TILES16], p3[TILES16];
};

// Two steps (8 entries from e0): the loads of each step are issued one step ahead.
template <int TILES16, bool HELM, bool FAST, bool MASK>
__device__ __forceinline__ void mrhs_block(MrhsState<TILES16>& S, const int4* ent, const int32_t* pos, int32_t e0,
                                           int32_t cnt, int kk, const float2* qb, int m, uint32_t lcol,
                                           const int32_t (&col)[TILES16], const StepTgt& tg, const ExactCtx& E,
                                           float kturns) {
  S.b.src = ent[e0 + kStepSrc + kk];
  load_q<TILES16, FAST>(S.b, qb, m, lcol, col);
  mfma_step<TILES16, HELM, MASK>(S.a, e0 + kk, cnt, tg, pos, E, kturns, S.p1, S.p2, S.p3);
  S.a.src = ent[e0 + 2 * kStepSrc + kk];
  load_q<TILES16, FAST>(S.a, qb, m, lcol, col);
  mfma_step<TILES16, HELM, MASK>(S.b, e0 + kStepSrc + kk, cnt, tg, pos, E, kturns, S.p1, S.p2, S.p3);
}

template <int TILES16, bool HELM, bool CSR, bool FAST>
__global__ void __launch_bounds__(kBlock) k_mrhs(BatchIO io, const InstDesc* __restrict__ desc,
                                              const int4* __restrict__ items, XcdSplit split, int wpb) {
  __shared__ int4 lds_ent[kWavesPerBlock][kGroupSrc];
  __shared__ int32_t lds_pos[kWavesPerBlock][kGroupSrc];
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
  // entries [s0, s_self) are the box's own points (listed first); a zero distance
  // or a close pair can only occur there, unless points of distinct boxes may
  // coincide or the box is marked near
  const bool near_box = D.near != nullptr && ld_uniform(D.near + T) != 0;
  const int32_t s_self = (D.may_coincide || near_box) ? s1 : s0 + (bt1 - bt0);
  const int64_t n = D.n;
  const int i = lane & 15;    // target row of A, column of B
  const int kk = lane >> 4;   // source of the step
  // rows past the tile's last target repeat its first; their sums are never stored
  const int32_t t = t_first + (i < nt ? i : 0);
  StepTgt tg{ld_global(D.sx32 + t), ld_global(D.sx32 + n + t), ld_global(D.sx32 + 2 * n + t), t, 0};
  const ExactCtx E{D.sx64, n, D.qinv};
  const float kturns = D.kturns;
  const float2* qb = io.q[inst];
  const uint32_t lcol = 8u * (uint32_t)(rg + i);
  // general form: columns past the call's last one read that last column; their
  // sums are never stored
  int32_t col[TILES16];
#pragma unroll
  for (int q = 0; q < TILES16; ++q) col[q] = min(rg + i + 16 * q, m - 1);

  // 3-multiplication complex product: with P1 = Gr Qr, P2 = Gi Qi and
  // P3 = (Gr + Gi)(Qr + Qi), Re Y = P1 - P2 and Im Y = P3 - P1 - P2.
  MrhsState<TILES16> S;
#pragma unroll
  for (int q = 0; q < TILES16; ++q) {
    S.p1[q] = f4{0.f, 0.f, 0.f, 0.f};
    S.p2[q] = f4{0.f, 0.f, 0.f, 0.f};
    S.p3[q] = f4{0.f, 0.f, 0.f, 0.f};
  }
  int4* ent = lds_ent[wv];
  int32_t* pos = lds_pos[wv];
  for (int32_t sg = s0; sg < s1; sg += kGroupCap) {
    const int32_t cnt = min(s1 - sg, kGroupCap);
    stage_group<CSR, FAST>(T, sg, sg + cnt, D, n, m, ent, pos, lane);
    tg.self_e = (t - bt0) + (s0 - sg);  // own points are listed first
    S.a.src = ent[kk];
    load_q<TILES16, FAST>(S.a, qb, m, lcol, col);
    pin_step<TILES16>(S.a);
    // Blocks that may meet a zero distance (the box's own points), then the plain
    // blocks, then the block that reaches the padding: the first and last take the
    // masked form.
    const int32_t plain_from = max(0, s_self - sg);
    int32_t e0 = 0;
    for (; e0 < cnt && e0 < plain_from; e0 += 2 * kStepSrc)
      mrhs_block<TILES16, HELM, FAST, true>(S, ent, pos, e0, cnt, kk, qb, m, lcol, col, tg, E, kturns);
    for (; e0 + 2 * kStepSrc <= cnt; e0 += 2 * kStepSrc)
      mrhs_block<TILES16, HELM, FAST, false>(S, ent, pos, e0, cnt, kk, qb, m, lcol, col, tg, E, kturns);
    if (e0 < cnt) mrhs_block<TILES16, HELM, FAST, true>(S, ent, pos, e0, cnt, kk, qb, m, lcol, col, tg, E, kturns);
    wave_lds_sync();
  }
  // D[row][col]: lane j + 16 (row / 4), register row % 4
  float re[4][TILES16], im[4][TILES16];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < TILES16; ++q) {
      re[r][q] = S.p1[q][r] - S.p2[q][r];
      im[r][q] = S.p3[q][r] - S.p1[q][r] - S.p2[q][r];
    }
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
        if (c < m) y[yi + c] = make_float2(re[r][q] * sc, im[r][q] * sc);
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
  d.may_coincide = P->may_coincide ? 1 : 0;
  d.near = P->near;
  d.sx64 = P->sx64;
  d.qinv = std::ldexp(1.0, -P->qexp);
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
  const bool fast = mrhs_fast(S, io.m, width);
#define P2P_MRHS_O(TL, H, C) \
  do {                       \
    if (fast)                \
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
  } else if (width == 32) {
    if (S.helm) P2P_MRHS_C(2, true); else P2P_MRHS_C(2, false);
  } else {
    if (S.helm) P2P_MRHS_C(1, true); else P2P_MRHS_C(1, false);
  }
#undef P2P_MRHS_C
#undef P2P_MRHS_O
#undef P2P_MRHS
  P2P_HIP(hipGetLastError());
  if (e1) P2P_HIP(hipEventRecord(e1, s));
  return P2P_OK;
}

}  // namespace p2p
