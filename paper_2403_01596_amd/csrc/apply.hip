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

// y[i] = scale * sum_j G(r_ij) q_j
template <class Tr>
struct FwdOp {
  using real = typename Tr::real;
  using cplx = typename Tr::cplx;
  static constexpr int K = Tr::K, NP = 2, NT = 0, NA = 2;
  const cplx* __restrict__ qs;
  int m, col;
  const int32_t* __restrict__ perm;
  cplx* __restrict__ y;
  real scale;

  __device__ __forceinline__ void load_src(int32_t p, real* pay) const {
    const cplx q = qs[(int64_t)p * m + col];
    pay[0] = q.x;
    pay[1] = q.y;
  }
  __device__ __forceinline__ void load_tgt(int32_t, real*) const {}
  template <bool HELM>
  __device__ __forceinline__ void pair(const typename Tr::Geo& g, const real* sp, const real*, real* acc) const {
    if (HELM) {
      const real gr = g.c * g.rinv, gi = g.s * g.rinv;
      acc[0] = fma(gr, sp[0], acc[0]);
      acc[0] = fma(-gi, sp[1], acc[0]);
      acc[1] = fma(gr, sp[1], acc[1]);
      acc[1] = fma(gi, sp[0], acc[1]);
    } else {
      acc[0] = fma(g.rinv, sp[0], acc[0]);
      acc[1] = fma(g.rinv, sp[1], acc[1]);
    }
  }
  __device__ __forceinline__ void store(int32_t t, const real* a) const {
    const int64_t i = perm[t];
    cplx v;
    v.x = a[0] * scale;
    v.y = a[1] * scale;
    y[i * m + col] = v;
  }
};

template <class Tr, bool HELM, bool CSR>
__global__ void __launch_bounds__(kBlock) k_apply(SweepGeom<Tr> G, FwdOp<Tr> op) {
  __shared__ SweepLds<Tr, FwdOp<Tr>, CSR> lds[kWavesPerBlock];
  sweep<Tr, FwdOp<Tr>, HELM, CSR>(G, op, lds[threadIdx.x / kWave]);
}

// rows of q (original order) -> rows of qs (sorted order)
template <typename C>
__global__ void __launch_bounds__(kBlock) k_gather_rows(const C* __restrict__ q, const int32_t* __restrict__ perm,
                                                     int64_t n, int m, C* __restrict__ qs) {
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * m) return;
  int64_t p = e / m;
  int c = (int)(e - p * m);
  qs[e] = q[(int64_t)perm[p] * m + c];
}

// 1 / (4 pi) times the unit conversion of the accumulated terms (FP32: quanta)
template <class Tr>
double fwd_scale(const p2p_plan_s* P) {
  return (P->precision == P2P_C64 ? std::ldexp(1.0, -P->qexp) : 1.0) / (4.0 * M_PI);
}

template <class Tr>
static p2p_status run_apply(p2p_plan_s* P, const void* q, void* y, int m, hipStream_t s) {
  using cplx = typename Tr::cplx;
  using real = typename Tr::real;
  const int64_t n = P->n;
  hipLaunchKernelGGL(k_gather_rows<cplx>, dim3(grid_for(n * m)), dim3(kBlock), 0, s, (const cplx*)q, P->perm, n, m,
                     (cplx*)P->q_sorted);
  SweepGeom<Tr> G = make_geom<Tr>(P);
  const bool helm = P->k != 0.0, csr = P->layout == P2P_LAYOUT_CSR;
  auto kern = helm ? (csr ? k_apply<Tr, true, true> : k_apply<Tr, true, false>)
                   : (csr ? k_apply<Tr, false, true> : k_apply<Tr, false, false>);
  const real sc = (real)fwd_scale<Tr>(P);
  SweepTimer timer(P, s);
  timer.start();
  for (int c = 0; c < m; ++c) {
    FwdOp<Tr> op{(const cplx*)P->q_sorted, m, c, P->perm, (cplx*)y, sc};
    hipLaunchKernelGGL(kern, dim3(grid_for(G.nb, kWavesPerBlock)), dim3(kBlock), 0, s, G, op);
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
