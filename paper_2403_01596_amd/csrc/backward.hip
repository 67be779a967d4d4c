// Reverse pass of the near-field apply, for a real loss L(y) with upstream
// g = dL/dRe y + i dL/dIm y (the paper has no gradients; this is the adjoint of
// the operator it computes):
//   grad_q[i] = conj( sum_j G(r_ij) conj(g_j) ) = sum_j conj(G(r_ij)) g_j
//   grad_x[i] = sum_j Re( G'(r_ij) (conj(g_i) q_j + conj(g_j) q_i) ) (x_i - x_j) / r_ij
//   G'(r)     = exp(i k r) (i k r - 1) / (4 pi r^2)
// Both come out of one sweep over the same pairs as the forward apply (sweep.h):
// because the near relation is symmetric, every target box can form its own
// grad_x from its own neighbourhood, and no output is written by two lanes.
#include "sweep.h"

namespace p2p {

template <class Tr, bool DQ, bool DX>
struct BwdOp {
  using real = typename Tr::real;
  using cplx = typename Tr::cplx;
  static constexpr int K = Tr::K;
  static constexpr int NP = 4, NT = DX ? 4 : 0, NA = (DQ ? 2 : 0) + (DX ? 3 : 0);
  static constexpr int OX = DQ ? 2 : 0;  // first dx accumulator
  const cplx* __restrict__ qs;
  const cplx* __restrict__ gs;
  int m, col;
  const int32_t* __restrict__ perm;
  cplx* __restrict__ gq;
  double* __restrict__ gx;
  real q_scale;
  double x_scale;
  real kw;  // the wavenumber in the geometry's units (FP32: radians per quantum)

  __device__ __forceinline__ void load_src(int32_t p, real* pay) const {
    const cplx q = qs[(int64_t)p * m + col], g = gs[(int64_t)p * m + col];
    pay[0] = q.x;
    pay[1] = q.y;
    pay[2] = g.x;
    pay[3] = g.y;
  }
  __device__ __forceinline__ void load_tgt(int32_t t, real* tp) const {
    if (DX) {
      const real* q = reinterpret_cast<const real*>(qs + (int64_t)t * m + col);
      const real* g = reinterpret_cast<const real*>(gs + (int64_t)t * m + col);
      tp[0] = ld_uniform(q);
      tp[1] = ld_uniform(q + 1);
      tp[2] = ld_uniform(g);
      tp[3] = ld_uniform(g + 1);
    }
  }
  template <bool HELM>
  __device__ __forceinline__ void pair(const typename Tr::Geo& G, const real* sp, const real* tp, real* acc) const {
    // G = (c + i s) rinv
    const real gr = G.c * G.rinv, gi = G.s * G.rinv;
    if (DQ) {
      // conj(G) g_j
      acc[0] = fma(gr, sp[2], acc[0]);
      acc[0] = fma(gi, sp[3], acc[0]);
      acc[1] = fma(gr, sp[3], acc[1]);
      acc[1] = fma(-gi, sp[2], acc[1]);
    }
    if (DX) {
      // u = conj(g_i) q_j + conj(g_j) q_i
      real ur = tp[2] * sp[0];
      ur = fma(tp[3], sp[1], ur);
      ur = fma(sp[2], tp[0], ur);
      ur = fma(sp[3], tp[1], ur);
      real ui = tp[2] * sp[1];
      ui = fma(-tp[3], sp[0], ui);
      ui = fma(sp[2], tp[1], ui);
      ui = fma(-sp[3], tp[0], ui);
      // 4 pi r G' = (c + i s)(i k r - 1) / r = (c + i s)(i k - rinv): since r rinv = 1,
      // its parts are -(gr + s k) and c k - gi, with no product k r per pair
      real w;
      if (HELM) {
        const real dr = -fma(G.s, kw, gr);
        const real di = fma(G.c, kw, -gi);
        w = fma(dr, ur, -(di * ui));
      } else {
        w = -gr * ur;
      }
      w *= G.rinv * G.rinv;  // Re(G' u) / r, up to the scale
      acc[OX + 0] = fma(w, G.dx, acc[OX + 0]);
      acc[OX + 1] = fma(w, G.dy, acc[OX + 1]);
      acc[OX + 2] = fma(w, G.dz, acc[OX + 2]);
    }
  }
  __device__ __forceinline__ void store(int32_t t, const real* a) const {
    const int64_t i = perm[t];
    if (DQ) {
      cplx v;
      v.x = a[0] * q_scale;
      v.y = a[1] * q_scale;
      gq[i * m + col] = v;
    }
    if (DX) {
      for (int d = 0; d < 3; ++d) {
        const double v = (double)a[OX + d] * x_scale;
        gx[3 * i + d] = (col == 0) ? v : gx[3 * i + d] + v;
      }
    }
  }
};

template <class Tr, bool HELM, bool CSR, bool DQ, bool DX>
__global__ void __launch_bounds__(kBlock) k_backward(SweepGeom<Tr> G, BwdOp<Tr, DQ, DX> op) {
  __shared__ SweepLds<Tr, BwdOp<Tr, DQ, DX>, CSR> lds[kWavesPerBlock];
  sweep<Tr, BwdOp<Tr, DQ, DX>, HELM, CSR>(G, op, lds[threadIdx.x / kWave]);
}

template <typename C>
__global__ void __launch_bounds__(kBlock) k_gather_rows2(const C* __restrict__ q, const C* __restrict__ g,
                                                      const int32_t* __restrict__ perm, int64_t n, int m,
                                                      C* __restrict__ qs, C* __restrict__ gs) {
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * m) return;
  int64_t p = e / m;
  int c = (int)(e - p * m);
  int64_t src = (int64_t)perm[p] * m + c;
  qs[e] = q[src];
  gs[e] = g[src];
}

template <class Tr, bool DQ, bool DX>
static void launch_cols(p2p_plan_s* P, const SweepGeom<Tr>& G, void* gq, double* gx, int m, hipStream_t s) {
  using real = typename Tr::real;
  using cplx = typename Tr::cplx;
  const bool helm = P->k != 0.0, csr = P->layout == P2P_LAYOUT_CSR;
  auto kern = helm ? (csr ? k_backward<Tr, true, true, DQ, DX> : k_backward<Tr, true, false, DQ, DX>)
                   : (csr ? k_backward<Tr, false, true, DQ, DX> : k_backward<Tr, false, false, DQ, DX>);
  const bool f32 = P->precision == P2P_C64;
  const double unit = f32 ? std::ldexp(1.0, -P->qexp) : 1.0;  // quantum -> length
  const real qsc = (real)(unit / (4.0 * M_PI));
  const double xsc = unit * unit / (4.0 * M_PI);
  const real kw = (real)(P->k / unit);
  for (int c = 0; c < m; ++c) {
    BwdOp<Tr, DQ, DX> op{(const cplx*)P->q_sorted, (const cplx*)P->g_sorted, m, c, P->perm, (cplx*)gq, gx, qsc, xsc,
                         kw};
    hipLaunchKernelGGL(kern, dim3(grid_for(G.nb, kWavesPerBlock)), dim3(kBlock), 0, s, G, op);
  }
}

template <class Tr>
static p2p_status run_backward(p2p_plan_s* P, const void* q, const void* gy, void* gq, double* gx, int m,
                               hipStream_t s) {
  using cplx = typename Tr::cplx;
  const int64_t n = P->n;
  hipLaunchKernelGGL(k_gather_rows2<cplx>, dim3(grid_for(n * m)), dim3(kBlock), 0, s, (const cplx*)q,
                     (const cplx*)gy, P->perm, n, m, (cplx*)P->q_sorted, (cplx*)P->g_sorted);
  SweepGeom<Tr> G = make_geom<Tr>(P);
  SweepTimer timer(P, s);
  timer.start();
  if (gq && gx) launch_cols<Tr, true, true>(P, G, gq, gx, m, s);
  else if (gq) launch_cols<Tr, true, false>(P, G, gq, gx, m, s);
  else if (gx) launch_cols<Tr, false, true>(P, G, gq, gx, m, s);
  timer.stop();
  P2P_HIP(hipGetLastError());
  return P2P_OK;
}

p2p_status launch_backward(p2p_plan_s* P, const void* q, const void* gy, void* gq, double* gx, int m, hipStream_t s) {
  if (P->n == 0 || (!gq && !gx)) return P2P_OK;
  return P->precision == P2P_C64 ? run_backward<F32>(P, q, gy, gq, gx, m, s)
                                 : run_backward<F64>(P, q, gy, gq, gx, m, s);
}

}  // namespace p2p
