// The near-field sweep shared by the forward and reverse kernels.
//
// Paper, sections 3.2 and 3.3: every target loops over the sources of its own and
// the adjacent boxes and evaluates the pair kernel.  Mapping on CDNA:
//  - one wavefront per target box (boxes taken from a work list, largest first);
//  - the 64 lanes hold 64 different sources of the box's neighbourhood, up to
//    K chunks of 64 in registers at a time (K chosen by the operation);
//  - the box's targets are walked one at a time, wave-uniform, with their
//    coordinates and payload in scalar registers;
//  - every lane accumulates its sources' terms for the current target, and one
//    wavefront reduction per target (DPP row operations) yields the target's sum,
//    which the lane owning that target keeps; outputs are written once, by one
//    lane, so results do not depend on scheduling and need no atomics.
// Source layouts (both list a box's own points first, then its other neighbours):
//  - TILES: the box's neighbourhood sources replicated into one contiguous list
//    (the redundant layout of section 3.3, kept per box instead of per target);
//  - CSR: no replicated geometry; the wavefront writes the sorted positions of
//    its neighbour boxes' points into LDS (the indexed layout of section 3.2) and
//    gathers coordinates through them.
#pragma once

#include <cmath>
#include <type_traits>

#include "common.h"

namespace p2p {

constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------------------
// arithmetic traits
// ---------------------------------------------------------------------------
// Pair geometry: given the target and source coordinates, the reciprocal distance
// (zero when the distance is zero: the pair is skipped), and for the Helmholtz
// kernel cos and sin of k r.
struct F32 {
  using coord = int32_t;  // fixed point, units of 2^qexp, low 32 bits
  using real = float;
  using cplx = float2;
  static constexpr int K = 8, K1 = 8;  // chunks of 64 sources per group (K1: one column)
  struct Geo {
    float dx, dy, dz, r2, rinv, c, s;
  };
  // k_turns: k * 2^qexp / (2 pi), the phase in turns per quantum of distance.
  // MASK: the pair may be at distance zero (then rinv = 0 and the term vanishes).
  template <bool HELM, bool MASK>
  __device__ static __forceinline__ Geo geo(int32_t tx, int32_t ty, int32_t tz, int32_t sx, int32_t sy, int32_t sz,
                                            float k_turns, float floor_r2 = 0.0f) {
    // x_target - x_source: exact modulo 2^32, exact as an integer for near pairs
    return from_d<HELM, MASK>((float)(int32_t)((uint32_t)tx - (uint32_t)sx),
                              (float)(int32_t)((uint32_t)ty - (uint32_t)sy),
                              (float)(int32_t)((uint32_t)tz - (uint32_t)sz), k_turns, floor_r2);
  }
  // The same from a difference already in FP32 (quantum units).  MASK: pairs with
  // r2 <= floor_r2 get rinv = 0 (with the default floor, the pairs at distance
  // zero; with a positive one, the sweep adds those terms separately).
  template <bool HELM, bool MASK>
  __device__ static __forceinline__ Geo from_d(float dx, float dy, float dz, float k_turns, float floor_r2 = 0.0f) {
    Geo g;
    g.dx = dx;
    g.dy = dy;
    g.dz = dz;
    const float r2 = __builtin_fmaf(g.dz, g.dz, __builtin_fmaf(g.dy, g.dy, g.dx * g.dx));
    const float ri = __builtin_amdgcn_rsqf(r2);
    g.r2 = r2;
    g.rinv = MASK ? ((r2 > floor_r2) ? ri : 0.0f) : ri;
    if (HELM) {
      const float turns = (r2 * g.rinv) * k_turns;
      g.c = __builtin_amdgcn_cosf(turns);
      g.s = __builtin_amdgcn_sinf(turns);
    } else {
      g.c = 1.0f;
      g.s = 0.0f;
    }
    return g;
  }
};

// a * b + c written as one three-operand v_fma_f64.  Given a loop-invariant c,
// the compiler otherwise picks the two-operand v_fmac_f64, whose addend is also its
// destination, and copies c into a fresh register pair before every use.
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// sin(2 pi x) and cos(2 pi x) for |x| <= 1/4 from their Taylor series in x:
// coefficients (2 pi)^n / n! with alternating signs, each correctly rounded to
// double.  The first omitted terms are below 1.3e-18 (sin, x^23) and 1.9e-17 (cos,
// x^22) in magnitude on that interval.
constexpr double kSinTurn[11] = {0x1.921fb54442d18p+2,  -0x1.4abbce625be53p+5, 0x1.466bc6775aae2p+6,
                                 -0x1.32d2cce62bd86p+6, 0x1.50783487ee782p+5,  -0x1.e3074fde8871fp+3,
                                 0x1.e8f434d018d63p+1,  -0x1.6fadb9f155744p-1, 0x1.aaec32af93359p-4,
                                 -0x1.8a404211f9547p-7, 0x1.2877020d52cf0p-10};
constexpr double kCosTurn[11] = {0x1.0000000000000p+0,  -0x1.3bd3cc9be45dep+4, 0x1.03c1f081b5ac4p+6,
                                 -0x1.55d3c7e3cbffap+6, 0x1.e1f506891babbp+5,  -0x1.a6d1f2a204a8cp+4,
                                 0x1.f9d38a3763cc3p+2,  -0x1.b6e24f44b128fp+0, 0x1.20c62c2f2d7f5p-2,
                                 -0x1.2a0c591af8314p-5, 0x1.ef6e308d6d1c4p-9};

struct F64 {
  using coord = double;
  using real = double;
  using cplx = double2;
  static constexpr int K = 4, K1 = 8;  // chunks of 64 sources per group (K1: one column)
  struct Geo {
    double dx, dy, dz, rinv, c, s;
  };
  // kt: k / (2 pi), the phase in turns per unit of distance.  Coordinates are the
  // caller's FP64 values, and the difference is formed exactly as in the
  // definition, x_target - x_source.
  template <bool HELM, bool MASK>
  __device__ static __forceinline__ Geo geo(double tx, double ty, double tz, double sx, double sy, double sz,
                                            double kt) {
    Geo g;
    g.dx = tx - sx;
    g.dy = ty - sy;
    g.dz = tz - sz;
    const double r2 = __builtin_fma(g.dz, g.dz, __builtin_fma(g.dy, g.dy, g.dx * g.dx));
    // 1/r: the hardware estimate y refined by one third-order step,
    // y (1 + e/2 + 3e^2/8) with e = 1 - r2 y^2 (the series of (1 - e)^(-1/2)).
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2 * y, y, 1.0);
    const double ri = __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
    g.rinv = MASK ? ((r2 > 0.0) ? ri : 0.0) : ri;
    if (HELM) {
      // phase t in turns; t = h/2 + x with h the nearest whole number of half
      // turns (so x = t - h/2 is exact and |x| <= 1/4), and an odd h flips the
      // signs of both sin and cos
      const double t = kt * (r2 * g.rinv);
      const double h = __builtin_rint(t + t);
      const double x = __builtin_fma(-0.5, h, t);
      const double x2 = x * x;
      // Estrin's scheme (pairs of terms in x2, then x4 and x8): two multiplications
      // more than Horner's rule, and much shorter dependency chains
      const double x4 = x2 * x2, x8 = x4 * x4;
      const double s01 = fma3(kSinTurn[1], x2, kSinTurn[0]);
      const double s23 = fma3(kSinTurn[3], x2, kSinTurn[2]);
      const double s45 = fma3(kSinTurn[5], x2, kSinTurn[4]);
      const double s67 = fma3(kSinTurn[7], x2, kSinTurn[6]);
      const double s89 = fma3(kSinTurn[9], x2, kSinTurn[8]);
      const double s0_3 = __builtin_fma(s23, x4, s01);
      const double s4_7 = __builtin_fma(s67, x4, s45);
      const double s8_10 = fma3(kSinTurn[10], x4, s89);
      const double ps = __builtin_fma(__builtin_fma(s8_10, x8, s4_7), x8, s0_3);
      const double c01 = fma3(kCosTurn[1], x2, kCosTurn[0]);
      const double c23 = fma3(kCosTurn[3], x2, kCosTurn[2]);
      const double c45 = fma3(kCosTurn[5], x2, kCosTurn[4]);
      const double c67 = fma3(kCosTurn[7], x2, kCosTurn[6]);
      const double c89 = fma3(kCosTurn[9], x2, kCosTurn[8]);
      const double c0_3 = __builtin_fma(c23, x4, c01);
      const double c4_7 = __builtin_fma(c67, x4, c45);
      const double c8_10 = fma3(kCosTurn[10], x4, c89);
      const double pc = __builtin_fma(__builtin_fma(c8_10, x8, c4_7), x8, c0_3);
      const double hh = 0.5 * h;
      const double sg = __builtin_fma(-4.0, hh - __builtin_floor(hh), 1.0);  // (-1)^h
      g.s = (sg * x) * ps;
      g.c = sg * pc;
    } else {
      g.c = 1.0;
      g.s = 0.0;
    }
    return g;
  }
};

// FP32 plans: a pair whose fixed-point difference is shorter than kCloseQuanta
// quanta (r2 below kCloseR2 in quantum units) takes its coordinate difference from
// the FP64 coordinates instead -- the difference of the definition, exact for such
// a pair, rounded once to FP32 -- and the rest of its geometry as any other pair.
// The rounding of fixed-point coordinates (half a quantum per axis) would move
// its term by up to a quantum over its distance; for every other pair, at least
// 2^20 quanta apart, by at most 2^-20 relative.  A pair at FP64 distance zero
// gets rinv = 0, as the definition skips it.
constexpr float kCloseR2 = (float)kCloseQuanta * (float)kCloseQuanta;

struct ExactCtx {
  const double* x;  // [3][n] FP64 coordinates, sorted order
  int64_t n;
  double qinv;      // 2^-qexp: length to quanta
};

template <bool HELM>
__device__ __forceinline__ F32::Geo exact_geo(const ExactCtx& E, int32_t t, int32_t p, float k_turns) {
  float d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d[a] = (float)((E.x[a * E.n + t] - E.x[a * E.n + p]) * E.qinv);
    // one axis at a time: this runs beside the sweep's live registers, and only
    // one pair of FP64 temporaries fits there
    asm volatile("" : "+v"(d[a])::"memory");
  }
  return F32::from_d<HELM, true>(d[0], d[1], d[2], k_turns);
}

// The paper's two-dimensional potential, G(r) = -ln(r) / (2 pi) = -ln(r^2) / (4 pi),
// in FP64 on points of a plane (z equal for all points, so dz = 0).  geo() leaves
// ln(r^2) in l (zero for a masked pair at distance zero); the operation scales.
struct L2D {
  using coord = double;
  using real = double;
  using cplx = double2;
  static constexpr int K = 4, K1 = 8;
  struct Geo {
    double dx, dy, dz, l;
  };
  template <bool HELM, bool MASK>
  __device__ static __forceinline__ Geo geo(double tx, double ty, double tz, double sx, double sy, double sz,
                                            double) {
    Geo g;
    g.dx = tx - sx;
    g.dy = ty - sy;
    g.dz = tz - sz;
    const double r2 = __builtin_fma(g.dz, g.dz, __builtin_fma(g.dy, g.dy, g.dx * g.dx));
    g.l = MASK ? ((r2 > 0.0) ? log(r2) : 0.0) : log(r2);
    return g;
  }
};

// ---------------------------------------------------------------------------
// geometry arguments common to every sweep
// ---------------------------------------------------------------------------
template <class Tr>
struct SweepGeom {
  const int32_t* work;
  int32_t nb;
  const int32_t* box_start;
  // Box T's targets are the sorted positions [box_start[T], tgt_end[T]), its sources
  // [src_begin[T], box_start[T + 1]).  One point set: both are all its points
  // (src_begin = box_start, tgt_end = box_start + 1).  Distinct sets (st): targets
  // first, then sources, and no target is also a source.
  const int32_t* src_begin;
  const int32_t* tgt_end;
  bool st;
  const int32_t* tile_start;
  const int32_t* tsrc;
  const typename Tr::coord* tx;  // [3][tl]
  int64_t tl;
  const int32_t* nbr_start;
  const int32_t* nbr_idx;
  const typename Tr::coord* sx;  // [3][n]
  int64_t n;
  const int32_t* perm;
  typename Tr::real kparam;      // F32: turns per quantum; F64: turns per unit length
  typename Tr::coord far;        // x offset of padding entries: farther than any near pair
  bool may_coincide;             // points of distinct boxes may coincide: mask every chunk
  // FP32 plans: per box, nonzero if a neighbour box's bounding box comes within
  // kCloseQuanta + 2 quanta of the box's own on every axis (only then can a pair
  // of distinct boxes be close; see exact_geo); and the FP64 coordinates for those
  // pairs
  const int32_t* near;
  ExactCtx exact;
};

template <class Tr>
inline SweepGeom<Tr> make_geom(const p2p_plan_s* P) {
  SweepGeom<Tr> G;
  G.work = P->work;
  G.nb = (int32_t)P->B;
  G.box_start = P->box_start;
  G.src_begin = src_begin(P);
  G.tgt_end = tgt_end(P);
  G.st = P->src_start != nullptr;
  G.tile_start = P->tile_start;
  G.tsrc = P->tile_src;
  G.tl = P->tile_len;
  G.nbr_start = P->nbr_start;
  G.nbr_idx = P->nbr_idx;
  G.n = P->n;
  G.perm = P->perm;
  G.may_coincide = P->may_coincide;
  G.near = std::is_same<Tr, F32>::value ? P->near : nullptr;
  G.exact = ExactCtx{P->sx64, P->n, std::ldexp(1.0, -P->qexp)};
  if constexpr (std::is_same<Tr, F32>::value) {
    G.tx = P->tile_x32;
    G.sx = P->sx32;
    G.kparam = (float)(P->k * std::ldexp(1.0, P->qexp) / (2.0 * M_PI));
    G.far = 1 << 30;  // near-pair differences stay below 2^30 quanta
  } else {
    G.tx = P->tile_x64;
    G.sx = P->sx64;
    G.kparam = P->k / (2.0 * M_PI);
    G.far = 2.0 * P->max_sep + 1.0;  // near-pair differences stay below max_sep
  }
  return G;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sorted positions of neighbourhood entries [sg, sg + cap) of box T, into idx.  The
// neighbourhood is ordered as the replicated lists are: the box's own sources first,
// then the other neighbour boxes' in list order; box S's sources are the sorted
// positions [src_begin[S], box_start[S + 1]).
__device__ __forceinline__ void csr_indices(int32_t T, int32_t sg, int32_t cap, const int32_t* __restrict__ box_start,
                                            const int32_t* __restrict__ src_begin,
                                            const int32_t* __restrict__ nbr_start,
                                            const int32_t* __restrict__ nbr_idx, int32_t* idx, int lane) {
  int32_t off = 0;
  const int32_t j0 = ld_uniform(nbr_start + T), j1 = ld_uniform(nbr_start + T + 1);
  for (int32_t j = j0 - 1; j < j1; ++j) {
    const int32_t S = j < j0 ? T : ld_uniform(nbr_idx + j);
    if (j >= j0 && S == T) continue;
    const int32_t a = ld_uniform(src_begin + S), len = ld_uniform(box_start + S + 1) - a;
    const int32_t lo = max(off, sg), hi = min(off + len, sg + cap);
    for (int32_t e = lo + lane; e < hi; e += kWave) idx[e - sg] = a + (e - off);
    off += len;
    if (off >= sg + cap) break;
  }
  wave_lds_sync();
}

// Per-wavefront LDS of a sweep: the target sums of the current block of 64
// targets and, for the CSR layout, the source indices of the current group.
template <class Tr, class Op, bool CSR>
struct SweepLds {
  typename Tr::real sums[Op::NA][kWave];
  int32_t idx[CSR ? kWave * Op::K : 1];
  // FP32: the current target's close sources, as entries of the group (0 = sg)
  int32_t close[std::is_same<Tr, F32>::value ? kWave * Op::K : 1];
};

// Which chunks of a group take the zero-distance mask: every chunk, the first
// only (the group holds the box's own points, at most 64, in its first chunk), or
// none.  Three straight-line forms of the target loop, chosen per group: a branch
// per chunk between a masked and a plain form made the compiler copy the
// accumulators at every join.
enum SweepMask { kMaskAll, kMaskFirst, kMaskNone };

// Entries of the close-pair queue: the target (offset from the block's first)
// and the source (entry of the group) of one close pair.
__device__ __forceinline__ int32_t close_entry(int32_t t_off, int32_t e_off) { return (t_off << 16) | e_off; }
constexpr int32_t kNoMiss = 0x7fffffff;
// self_off of plans whose targets are not sources: no entry is a target's own
constexpr int32_t kNoSelf = -(1 << 30);

// The close pairs of target t in chunk c of a group: lanes whose fixed-point r2 is
// at most kCloseR2 (so that the FP32 geometry gave them no term; far: the others),
// except the self pair and entries past the group's end.
__device__ __forceinline__ uint64_t close_mask(uint64_t far, int32_t t, int32_t self_off, int32_t sg, int32_t s1,
                                               int c) {
  uint64_t cm = ~far;
  const int32_t sl = t + self_off - sg - c * kWave;
  if (sl >= 0 && sl < kWave) cm &= ~(1ull << sl);
  const int32_t nv = s1 - sg - c * kWave;
  if (nv < kWave) cm &= nv > 0 ? (1ull << nv) - 1ull : 0ull;
  return cm;
}

// Appends the lanes of cm to the close-pair queue for target t, unless the queue
// is stopped or cannot take them; then it is stopped and target t's entries are
// dropped, to be found again by close_rescan from t_miss on.
template <class LdsT>
__device__ __forceinline__ void close_push(LdsT& L, uint64_t cm, int32_t t_off, int c, int32_t cap, int32_t nq_t,
                                           int32_t t, int32_t& nq, int32_t& t_miss) {
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t k = __popcll(cm);
  if (t_miss == kNoMiss && nq + k <= cap) {
    if ((cm >> lane) & 1ull) L.close[nq + __popcll(cm & ((1ull << lane) - 1ull))] = close_entry(t_off, c * kWave + lane);
    nq += k;
  } else if (t_miss == kNoMiss) {
    nq = nq_t;
    t_miss = t;
  }
}

// Targets [tb, te) against the group's chunks in registers.  The group holds
// entries [sg, s1) of the box's neighbourhood list; a target's own entry (its
// self pair) is entry t + self_off of that list.  FP32: the close pairs met are
// queued in L.close (nq entries); t_miss is the first target whose pairs did not
// fit, or kNoMiss.  CLOSE: the box is marked near (FP32), so its masked chunks
// may hold close pairs; other boxes' masked chunks only skip zero distances.
template <class Tr, class Op, bool HELM, bool CSR, int MODE, bool CLOSE, class LdsT>
__device__ __forceinline__ void sweep_targets(const SweepGeom<Tr>& G, const Op& op, LdsT& L,
                                              const typename Tr::coord (&X)[Op::K],
                                              const typename Tr::coord (&Y)[Op::K],
                                              const typename Tr::coord (&Z)[Op::K],
                                              const typename Tr::real (&P)[Op::K][Op::NP > 0 ? Op::NP : 1], int nch,
                                              int32_t tb, int32_t te, bool first_group, int32_t sg, int32_t s1,
                                              int32_t self_off, int32_t& nq, int32_t& t_miss) {
  using real = typename Tr::real;
  using coord = typename Tr::coord;
  constexpr int K = Op::K;
  constexpr int NT = Op::NT, NA = Op::NA;
  constexpr int32_t kCap = kWave * K;  // one target's pairs of a group always fit
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t n = G.n;
  // target coordinates are fetched one target ahead
  coord nx = ld_uniform(G.sx + tb), ny = ld_uniform(G.sx + n + tb), nz = ld_uniform(G.sx + 2 * n + tb);
  for (int32_t t = tb; t < te; ++t) {
    const coord px = nx, py = ny, pz = nz;
    if (t + 1 < te) {
      nx = ld_uniform(G.sx + t + 1);
      ny = ld_uniform(G.sx + n + t + 1);
      nz = ld_uniform(G.sx + 2 * n + t + 1);
    }
    real tp[NT > 0 ? NT : 1];
    op.load_tgt(t, tp);
    real acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = real(0);
    const int32_t nq_t = nq;  // the queue before target t
#pragma unroll
    for (int c = 0; c < K; ++c)
      if (c < nch) {
        // c is a constant in each unrolled copy, so this choice costs no branch
        const bool masked = MODE == kMaskAll || (MODE == kMaskFirst && c == 0);
        if (masked) {
          if constexpr (std::is_same<Tr, F32>::value && CLOSE) {
            // Pairs under kCloseQuanta quanta get no term here (rinv = 0); the
            // close ones among them (the self pair and padding entries are not)
            // are queued and taken from the FP64 coordinates after the group.
            const typename Tr::Geo g = Tr::template geo<HELM, true>(px, py, pz, X[c], Y[c], Z[c], G.kparam, kCloseR2);
            const uint64_t cm = close_mask(__ballot(g.r2 > kCloseR2), t, self_off, sg, s1, c);
            if (cm) close_push(L, cm, t - tb, c, kCap, nq_t, t, nq, t_miss);
            op.template pair<HELM>(g, P[c], tp, acc);
          } else {
            const typename Tr::Geo g = Tr::template geo<HELM, true>(px, py, pz, X[c], Y[c], Z[c], G.kparam);
            op.template pair<HELM>(g, P[c], tp, acc);
          }
        } else {
          const typename Tr::Geo g = Tr::template geo<HELM, false>(px, py, pz, X[c], Y[c], Z[c], G.kparam);
          op.template pair<HELM>(g, P[c], tp, acc);
        }
      }
    // accumulators in pairs: the even one's sum lands in lane 31, the odd one's
    // (and a last unpaired one's) in lane 63
#pragma unroll
    for (int a = 0; a + 1 < NA; a += 2) acc[a] = acc[a + 1] = wave_sum_pair(acc[a], acc[a + 1]);
    if (NA % 2) acc[NA - 1] = wave_sum63(acc[NA - 1]);
    if (lane == 31 || lane == kWave - 1) {
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const bool in63 = (a & 1) || a == NA - 1;
        if ((lane == kWave - 1) == in63)
          L.sums[a][t - tb] = first_group ? acc[a] : L.sums[a][t - tb] + acc[a];
      }
    }
  }
}

// FP32, after the queue filled up: the close pairs of targets [tf, te) found
// again, with the sweep's own test on the group's coordinates (chunks in the
// masked form only), into the emptied queue.  Returns the first target whose pairs
// did not fit, or kNoMiss; the first target always fits.
template <class Op, bool CSR, int MODE, class LdsT>
__device__ __forceinline__ int32_t close_rescan(const SweepGeom<F32>& G, LdsT& L, const int32_t (&X)[Op::K],
                                                const int32_t (&Y)[Op::K], const int32_t (&Z)[Op::K], int nch,
                                                int32_t tb, int32_t tf, int32_t te, int32_t sg, int32_t s1,
                                                int32_t self_off, int32_t& nq) {
  constexpr int K = Op::K;
  constexpr int32_t kCap = kWave * K;
  const int64_t n = G.n;
  int32_t t_miss = kNoMiss;
  for (int32_t t = tf; t < te && t_miss == kNoMiss; ++t) {
    const int32_t px = ld_uniform(G.sx + t), py = ld_uniform(G.sx + n + t), pz = ld_uniform(G.sx + 2 * n + t);
    const int32_t nq_t = nq;
#pragma unroll
    for (int c = 0; c < K; ++c)
      if (c < nch && (MODE == kMaskAll || (MODE == kMaskFirst && c == 0))) {
        const F32::Geo g = F32::template geo<false, false>(px, py, pz, X[c], Y[c], Z[c], 0.0f);
        const uint64_t cm = close_mask(__ballot(g.r2 > kCloseR2), t, self_off, sg, s1, c);
        if (cm) close_push(L, cm, t - tb, c, kCap, nq_t, t, nq, t_miss);
      }
  }
  return t_miss;
}

// FP32: the queued close pairs of a group, one at a time (wave-uniform): the
// difference from the FP64 coordinates, the pair arithmetic, and the term added
// to its target's sums, which the group has already written.
template <class Tr, class Op, bool HELM, bool CSR, class LdsT>
__device__ __forceinline__ void close_terms(const SweepGeom<Tr>& G, const Op& op, LdsT& L, int32_t tb, int32_t sg,
                                            int32_t nq) {
  using real = typename Tr::real;
  constexpr int NT = Op::NT, NP = Op::NP, NA = Op::NA;
  const int lane = threadIdx.x & (kWave - 1);
  wave_lds_sync();
  for (int32_t j = 0; j < nq; ++j) {
    const int32_t ent = uniform(L.close[j]);
    const int32_t t = tb + (ent >> 16), off = ent & 0xffff;
    int32_t p;
    if constexpr (CSR) p = uniform(L.idx[off]);
    else p = ld_uniform(G.tsrc + sg + off);
    real tp[NT > 0 ? NT : 1], sp[NP > 0 ? NP : 1], a[NA];
    op.load_tgt(t, tp);
    op.load_src(p, sp);
#pragma unroll
    for (int i = 0; i < NA; ++i) a[i] = real(0);
    op.template pair<HELM>(exact_geo<HELM>(G.exact, t, p, G.kparam), sp, tp, a);
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < NA; ++i) L.sums[i][t - tb] += a[i];
    }
    wave_lds_sync();
  }
}

// The sweep.  Op supplies:
//   K                     chunks of 64 sources held in registers per group
//   NP, NT, NA            payload reals per source, per target, accumulators
//   load_src(p, pay)      payload of the source at sorted position p
//   load_tgt(t, pay)      payload of the target at sorted position t (uniform)
//   pair<HELM>(geo, spay, tpay, acc)
//   store(t, acc)         final values of target t (sorted position), by its lane
template <class Tr, class Op, bool HELM, bool CSR>
__device__ __forceinline__ void sweep(const SweepGeom<Tr>& G, const Op& op, SweepLds<Tr, Op, CSR>& L) {
  using real = typename Tr::real;
  using coord = typename Tr::coord;
  constexpr int K = Op::K;
  constexpr int NP = Op::NP, NA = Op::NA;
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t w = uniform((int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave));
  if (w >= G.nb) return;
  const int32_t T = ld_uniform(G.work + w);
  const int32_t t0 = ld_uniform(G.box_start + T), t1 = ld_uniform(G.tgt_end + T);
  // the box's own sources, first in its neighbourhood list; a target's own entry
  // (its self pair) is entry t + so of the list, with one point set only
  const int32_t n_own = ld_uniform(G.box_start + T + 1) - ld_uniform(G.src_begin + T);
  // the box's neighbourhood list: entries [s0, s1) of the replicated lists (TILES),
  // or [0, s1) numbered from the box's own sources on (CSR; the plan keeps the
  // offsets of the replicated lists for both layouts)
  int32_t s0 = ld_uniform(G.tile_start + T), s1 = ld_uniform(G.tile_start + T + 1);
  if (CSR) {
    s1 -= s0;
    s0 = 0;
  }
  const int64_t n = G.n, tl = G.tl;
  const bool near_box = G.near != nullptr && ld_uniform(G.near + T) != 0;
  for (int32_t tb = t0; tb < t1; tb += kWave) {
    const int32_t te = min(tb + kWave, t1);
    if (s1 == s0) {  // no sources near the box (distinct sets only): zero sums
      real zero[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) zero[a] = real(0);
      if (tb + lane < te) op.store(tb + lane, zero);
      continue;
    }
    for (int32_t sg = s0; sg < s1; sg += kWave * K) {
      const int nch = min(K, (s1 - sg + kWave - 1) / kWave);
      if (CSR) csr_indices(T, sg, kWave * K, G.box_start, G.src_begin, G.nbr_start, G.nbr_idx, L.idx, lane);
      const bool first_group = sg == s0;
      // A zero distance can only occur among the box's own points, entries
      // [s0, s0 + n_T), unless points of distinct boxes may coincide; a close pair
      // (FP32) only in a box marked near, whose chunks all take the masked form
      // with the close-pair test.  Padding entries sit far away.  The first-chunk
      // form needs all own points in the first chunk of the first group.
      const bool own_here = sg < s0 + n_own;
      const int32_t so = G.st ? kNoSelf : s0 - t0;
      const int mode = (G.may_coincide || (own_here && !(first_group && n_own <= kWave)))
                           ? kMaskAll
                           : (first_group ? kMaskFirst : kMaskNone);
      coord X[K], Y[K], Z[K];
      real P[K][NP > 0 ? NP : 1];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        // Entries past the end take the group's first source moved G.far along x,
        // with a zero payload: a finite term (the distance is never zero) that adds
        // exactly zero.
        const int32_t e = sg + c * kWave + lane;
        const bool ok = e < s1;
        X[c] = Y[c] = Z[c] = coord(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) P[c][a] = real(0);
        if (c < nch) {
          int32_t p;
          if (CSR) {
            p = L.idx[ok ? e - sg : 0];
            X[c] = G.sx[p];
            Y[c] = G.sx[n + p];
            Z[c] = G.sx[2 * n + p];
          } else {
            const int32_t e2 = ok ? e : sg;
            p = G.tsrc[e2];
            X[c] = G.tx[e2];
            Y[c] = G.tx[tl + e2];
            Z[c] = G.tx[2 * tl + e2];
          }
          if (ok) op.load_src(p, P[c]);
          if (!ok) {
            if constexpr (std::is_same<coord, int32_t>::value)
              X[c] = (int32_t)((uint32_t)X[c] + (uint32_t)G.far);  // modulo 2^32, like every difference
            else
              X[c] += G.far;
          }
        }
      }
      int32_t nq = 0, t_miss = kNoMiss;
      if (std::is_same<Tr, F32>::value && near_box)
        sweep_targets<Tr, Op, HELM, CSR, kMaskAll, true>(G, op, L, X, Y, Z, P, nch, tb, te, first_group, sg, s1,
                                                         so, nq, t_miss);
      else if (mode == kMaskAll)
        sweep_targets<Tr, Op, HELM, CSR, kMaskAll, false>(G, op, L, X, Y, Z, P, nch, tb, te, first_group, sg, s1,
                                                          so, nq, t_miss);
      else if (mode == kMaskFirst)
        sweep_targets<Tr, Op, HELM, CSR, kMaskFirst, false>(G, op, L, X, Y, Z, P, nch, tb, te, first_group, sg, s1,
                                                            so, nq, t_miss);
      else
        sweep_targets<Tr, Op, HELM, CSR, kMaskNone, false>(G, op, L, X, Y, Z, P, nch, tb, te, first_group, sg, s1,
                                                           so, nq, t_miss);
      if constexpr (std::is_same<Tr, F32>::value) {
        // close pairs (marked boxes only, rare): their terms, then, if the queue
        // filled up, the pairs it could not take, found again
        while (nq) {
          close_terms<Tr, Op, HELM, CSR>(G, op, L, tb, sg, nq);
          nq = 0;
          if (t_miss == kNoMiss) break;
          const int32_t tf = t_miss;
          t_miss = close_rescan<Op, CSR, kMaskAll>(G, L, X, Y, Z, nch, tb, tf, te, sg, s1, so, nq);
        }
      }
      if (CSR) wave_lds_sync();  // the index buffer is refilled for the next group
    }
    wave_lds_sync();
    real mine[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) mine[a] = L.sums[a][lane];
    if (tb + lane < te) op.store(tb + lane, mine);
    wave_lds_sync();  // the sums are rewritten by the next block of targets
  }
}

}  // namespace p2p
