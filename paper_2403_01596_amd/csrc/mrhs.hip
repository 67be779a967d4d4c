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
// product runs as four real MFMAs per 16-column tile:
//   Re Y += Gr Qr - Gi Qi,  Im Y += Gr Qi + Gi Qr.
// G never leaves registers; the accumulators hold D[i][j] at lane j + 16 (i / 4),
// register i % 4.
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

constexpr int kXcds = 8;
constexpr int kStepSrc = 4;      // sources per MFMA step (the K of 16x16x4)
constexpr int kGroupSrc = 256;   // sources whose indices are staged in LDS at a time (CSR)

// q rows of every instance (caller's order) -> the instance's sorted scratch
__global__ void __launch_bounds__(kBlock) k_gather_batch(BatchIO io, const InstDesc* __restrict__ desc) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= io.prefix[io.count]) return;
  int inst = 0;
  while (inst + 1 < io.count && io.prefix[inst + 1] <= e) ++inst;
  const InstDesc& D = desc[inst];
  const int m = io.m;
  const int64_t loc = e - io.prefix[inst];
  const int64_t p = loc / m;
  const int c = (int)(loc - p * m);
  D.q_sorted[loc] = io.q[inst][(int64_t)D.perm[p] * m + c];
}

template <int TILES16, bool HELM, bool CSR>
__global__ void __launch_bounds__(kBlock) k_mrhs(BatchIO io, const InstDesc* __restrict__ desc,
                                              const int4* __restrict__ items, XcdSplit split, int wpb) {
  __shared__ int32_t lds_idx[kWavesPerBlock][CSR ? kGroupSrc : 1];
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
  const int64_t n = D.n, tl = D.tl;
  const int i = lane & 15;    // target row of A, column of B
  const int kk = lane >> 4;   // source of the step
  const bool tvalid = i < nt;
  const int32_t t = t_first + (tvalid ? i : 0);
  const int32_t tx = D.sx32[t], ty = D.sx32[n + t], tz = D.sx32[2 * n + t];
  const float kturns = D.kturns;

  f4 accR[TILES16], accI[TILES16];
#pragma unroll
  for (int q = 0; q < TILES16; ++q) {
    accR[q] = f4{0.f, 0.f, 0.f, 0.f};
    accI[q] = f4{0.f, 0.f, 0.f, 0.f};
  }
  for (int32_t sg = s0; sg < s1; sg += kGroupSrc) {
    const int32_t ge = min(s1, sg + kGroupSrc);
    if (CSR) csr_indices(T, sg, kGroupSrc, D.box_start, D.nbr_start, D.nbr_idx, lds_idx[wv], lane);
    for (int32_t e0 = sg; e0 < ge; e0 += kStepSrc) {
      const int32_t e = e0 + kk;
      const bool svalid = e < ge;
      int32_t p, sx, sy, sz;
      if (CSR) {
        p = lds_idx[wv][svalid ? e - sg : 0];
        sx = D.sx32[p];
        sy = D.sx32[n + p];
        sz = D.sx32[2 * n + p];
      } else {
        const int32_t e2 = svalid ? e : sg;
        p = D.tsrc[e2];
        sx = D.tx32[e2];
        sy = D.tx32[tl + e2];
        sz = D.tx32[2 * tl + e2];
      }
      const F32::Geo g = F32::template geo<HELM, true>(tx, ty, tz, sx, sy, sz, kturns);
      const float w = (svalid && tvalid) ? g.rinv : 0.0f;
      const float gr = g.c * w, gi = g.s * w;
      const float2* qrow = D.q_sorted + (int64_t)p * m;
#pragma unroll
      for (int q = 0; q < TILES16; ++q) {
        const int col = rg + i + 16 * q;
        float2 qv = make_float2(0.f, 0.f);
        if (svalid && col < m) qv = qrow[col];
        accR[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(gr, qv.x, accR[q], 0, 0, 0);
        accR[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(gi, -qv.y, accR[q], 0, 0, 0);
        accI[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(gr, qv.y, accI[q], 0, 0, 0);
        accI[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(gi, qv.x, accI[q], 0, 0, 0);
      }
    }
    if (CSR) wave_lds_sync();
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
        const int col = rg + i + 16 * q;
        if (col < m) y[yi + col] = make_float2(accR[q][r] * sc, accI[q][r] * sc);
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
  d.q_sorted = (float2*)P->q_sorted;
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
  if (S.nitems == 0 || io.prefix[io.count] == 0) return P2P_OK;
  hipLaunchKernelGGL(k_gather_batch, dim3(grid_for(io.prefix[io.count])), dim3(kBlock), 0, s, io, S.desc);
  if (e0) P2P_HIP(hipEventRecord(e0, s));
  const unsigned g = mrhs_grid(S.split, wpb);
  const bool helm = S.helm, csr = S.csr;
#define P2P_MRHS(TL, H, C) \
  hipLaunchKernelGGL((k_mrhs<TL, H, C>), dim3(g), dim3(kBlock), 0, s, io, S.desc, S.items, S.split, wpb)
  if (width == 64) {
    if (helm) {
      if (csr) P2P_MRHS(4, true, true); else P2P_MRHS(4, true, false);
    } else {
      if (csr) P2P_MRHS(4, false, true); else P2P_MRHS(4, false, false);
    }
  } else {
    if (helm) {
      if (csr) P2P_MRHS(2, true, true); else P2P_MRHS(2, true, false);
    } else {
      if (csr) P2P_MRHS(2, false, true); else P2P_MRHS(2, false, false);
    }
  }
#undef P2P_MRHS
  P2P_HIP(hipGetLastError());
  if (e1) P2P_HIP(hipEventRecord(e1, s));
  return P2P_OK;
}

}  // namespace p2p
