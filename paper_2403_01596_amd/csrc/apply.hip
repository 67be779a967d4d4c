// Forward near-field apply y = A_near q (paper, sections 3.2 and 3.3: each target
// sums, over the sources of its own and the adjacent boxes, the kernel value
// times the source strength).  The sweep itself (one wavefront per target box,
// lanes over sources, one reduction per target) lives in sweep.h.
//
// FP32 path: coordinates are integers in units of 2^qexp, so a coordinate
// difference is one exact integer subtraction rounded once to FP32; the phase is
// computed in turns and fed to the hardware sine and cosine, which take turns and
// reduce the range exactly.  Terms are accumulated in quantum units and scaled
// once per target by 2^-qexp / (4 pi).
// FP64 path: the same sum in double precision from the caller's coordinates.
#include "sweep.h"

namespace p2p {

// y[i, col + c] = scale * sum_j G(r_ij) q[j, col + c] for the M columns c < M of
// one launch: the kernel value is evaluated once per pair and serves all M.
// Chunks per group: the precision's one-column count for one column, its count up
// to 4 columns, half of it for 8 (measured on the 2M sphere: fewer chunks leave
// the 2M per-target sums of a group to too few pairs, more cost occupancy).
template <class Tr, int M = 1>
struct FwdOp {
  using real = typename Tr::real;
  using cplx = typename Tr::cplx;
  static constexpr int K = M == 1 ? Tr::K1 : (M <= 4 ? Tr::K : Tr::K / 2), NP = 2 * M, NT = 0, NA = 2 * M;
  const cplx* __restrict__ qs;
  int m, col;
  const int32_t* __restrict__ perm;
  cplx* __restrict__ y;
  real scale;

  __device__ __forceinline__ void load_src(int32_t p, real* pay) const {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const cplx q = qs[(int64_t)p * m + col + c];
      pay[2 * c] = q.x;
      pay[2 * c + 1] = q.y;
    }
  }
  __device__ __forceinline__ void load_tgt(int32_t, real*) const {}
  template <bool HELM>
  __device__ __forceinline__ void pair(const typename Tr::Geo& g, const real* sp, const real*, real* acc) const {
    if (HELM) {
      const real gr = g.c * g.rinv, gi = g.s * g.rinv;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        acc[2 * c] = fma(gr, sp[2 * c], acc[2 * c]);
        acc[2 * c] = fma(-gi, sp[2 * c + 1], acc[2 * c]);
        acc[2 * c + 1] = fma(gr, sp[2 * c + 1], acc[2 * c + 1]);
        acc[2 * c + 1] = fma(gi, sp[2 * c], acc[2 * c + 1]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        acc[2 * c] = fma(g.rinv, sp[2 * c], acc[2 * c]);
        acc[2 * c + 1] = fma(g.rinv, sp[2 * c + 1], acc[2 * c + 1]);
      }
    }
  }
  __device__ __forceinline__ void store(int32_t t, const real* a) const {
    const int64_t i = perm[t];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      cplx v;
      v.x = a[2 * c] * scale;
      v.y = a[2 * c + 1] * scale;
      y[i * m + col + c] = v;
    }
  }
};

template <class Tr, bool HELM, bool CSR>
__global__ void __launch_bounds__(kBlock) k_apply(SweepGeom<Tr> G, FwdOp<Tr> op) {
  __shared__ SweepLds<Tr, FwdOp<Tr>, CSR> lds[kWavesPerBlock];
  sweep<Tr, FwdOp<Tr>, HELM, CSR>(G, op, lds[threadIdx.x / kWave]);
}

// M columns per launch (M = 2, 4 or 8)
template <class Tr, bool HELM, bool CSR, int M>
__global__ void __launch_bounds__(kBlock) k_apply_cols(SweepGeom<Tr> G, FwdOp<Tr, M> op) {
  __shared__ SweepLds<Tr, FwdOp<Tr, M>, CSR> lds[kWavesPerBlock];
  sweep<Tr, FwdOp<Tr, M>, HELM, CSR>(G, op, lds[threadIdx.x / kWave]);
}

// rows of q (original order) -> rows of qs (sorted order).  Plans of distinct sets:
// q holds the sources only (points n_targets on), and targets' rows are zero.
template <typename C>
__global__ void __launch_bounds__(kBlock) k_gather_rows(const C* __restrict__ q, const int32_t* __restrict__ perm,
                                                     int64_t n, int m, int64_t n_targets, C* __restrict__ qs) {
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * m) return;
  int64_t p = e / m;
  int c = (int)(e - p * m);
  const int64_t row = (int64_t)perm[p] - n_targets;
  qs[e] = row >= 0 ? q[row * m + c] : C{};
}

// 1 / (4 pi) times the unit conversion of the accumulated terms (FP32: quanta)
template <class Tr>
double fwd_scale(const p2p_plan_s* P) {
  return (P->precision == P2P_C64 ? std::ldexp(1.0, -P->qexp) : 1.0) / (4.0 * M_PI);
}

template <class Tr, int M>
static void launch_cols(const SweepGeom<Tr>& G, const FwdOp<Tr, M>& op, bool helm, bool csr, dim3 grid,
                        hipStream_t s) {
  auto kern = helm ? (csr ? k_apply_cols<Tr, true, true, M> : k_apply_cols<Tr, true, false, M>)
                   : (csr ? k_apply_cols<Tr, false, true, M> : k_apply_cols<Tr, false, false, M>);
  hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, G, op);
}

template <class Tr>
static p2p_status run_apply(p2p_plan_s* P, const void* q, void* y, int m, hipStream_t s) {
  using cplx = typename Tr::cplx;
  using real = typename Tr::real;
  const int64_t n = P->n;
  hipLaunchKernelGGL(k_gather_rows<cplx>, dim3(grid_for(n * m)), dim3(kBlock), 0, s, (const cplx*)q, P->perm, n, m,
                     P->distinct_sets ? P->n_targets : (int64_t)0, (cplx*)P->q_sorted);
  SweepGeom<Tr> G = make_geom<Tr>(P);
  const bool helm = P->k != 0.0, csr = P->layout == P2P_LAYOUT_CSR;
  auto kern = helm ? (csr ? k_apply<Tr, true, true> : k_apply<Tr, true, false>)
                   : (csr ? k_apply<Tr, false, true> : k_apply<Tr, false, false>);
  const real sc = (real)fwd_scale<Tr>(P);
  SweepTimer timer(P, s);
  timer.start();
  // columns in blocks of 8 (FP64 only: complex64 plans serve that many columns on
  // the matrix cores), 4, 2 and 1, one launch per block
  const dim3 grid(grid_for(G.nb, kWavesPerBlock)), block(kBlock);
  constexpr bool kBlocks8 = std::is_same<Tr, F64>::value;
  for (int c = 0; c < m;) {
    const int left = m - c;
    if constexpr (kBlocks8) {
      if (left >= 8) {
        launch_cols<Tr, 8>(G, FwdOp<Tr, 8>{(const cplx*)P->q_sorted, m, c, P->perm, (cplx*)y, sc}, helm, csr, grid,
                           s);
        c += 8;
        continue;
      }
    }
    if (left >= 4) {
      launch_cols<Tr, 4>(G, FwdOp<Tr, 4>{(const cplx*)P->q_sorted, m, c, P->perm, (cplx*)y, sc}, helm, csr, grid, s);
      c += 4;
    } else if (left >= 2) {
      launch_cols<Tr, 2>(G, FwdOp<Tr, 2>{(const cplx*)P->q_sorted, m, c, P->perm, (cplx*)y, sc}, helm, csr, grid, s);
      c += 2;
    } else {
      FwdOp<Tr> op{(const cplx*)P->q_sorted, m, c, P->perm, (cplx*)y, sc};
      hipLaunchKernelGGL(kern, grid, block, 0, s, G, op);
      c += 1;
    }
  }
  timer.stop();
  P2P_HIP(hipGetLastError());
  return P2P_OK;
}

p2p_status launch_apply(p2p_plan_s* P, const void* q, void* y, int m, hipStream_t s) {
  if (P->n == 0) return P2P_OK;
  return P->precision == P2P_C64 ? run_apply<F32>(P, q, y, m, s) : run_apply<F64>(P, q, y, m, s);
}

}  // namespace p2p
