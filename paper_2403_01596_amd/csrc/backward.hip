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

// M columns per launch: the kernel value, G' and the geometry are formed once per
// pair and serve every column; dx sums over the columns in one accumulator set.
// Chunks per group: the precision's one-column count for one column, its count up
// to 2 columns, half of it for 4 (measured on the 500k cube).
template <class Tr, bool DQ, bool DX, int M = 1>
struct BwdOp {
  using real = typename Tr::real;
  using cplx = typename Tr::cplx;
  static constexpr int K = M == 1 ? Tr::K1 : (M <= 2 ? Tr::K : Tr::K / 2);
  static constexpr int NP = 4 * M, NT = DX ? 4 * M : 0, NA = (DQ ? 2 * M : 0) + (DX ? 3 : 0);
  static constexpr int OX = DQ ? 2 * M : 0;  // first dx accumulator
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
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const cplx q = qs[(int64_t)p * m + col + c], g = gs[(int64_t)p * m + col + c];
      pay[4 * c] = q.x;
      pay[4 * c + 1] = q.y;
      pay[4 * c + 2] = g.x;
      pay[4 * c + 3] = g.y;
    }
  }
  __device__ __forceinline__ void load_tgt(int32_t t, real* tp) const {
    if (DX) {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const real* q = reinterpret_cast<const real*>(qs + (int64_t)t * m + col + c);
        const real* g = reinterpret_cast<const real*>(gs + (int64_t)t * m + col + c);
        tp[4 * c] = ld_uniform(q);
        tp[4 * c + 1] = ld_uniform(q + 1);
        tp[4 * c + 2] = ld_uniform(g);
        tp[4 * c + 3] = ld_uniform(g + 1);
      }
    }
  }
  template <bool HELM>
  __device__ __forceinline__ void pair(const typename Tr::Geo& G, const real* sp, const real* tp, real* acc) const {
    // G = (c + i s) rinv
    const real gr = G.c * G.rinv, gi = G.s * G.rinv;
    if (DQ) {
      // conj(G) g_j
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const real* p = sp + 4 * c;
        acc[2 * c] = fma(gr, p[2], acc[2 * c]);
        acc[2 * c] = fma(gi, p[3], acc[2 * c]);
        acc[2 * c + 1] = fma(gr, p[3], acc[2 * c + 1]);
        acc[2 * c + 1] = fma(-gi, p[2], acc[2 * c + 1]);
      }
    }
    if (DX) {
      // 4 pi r G' = (c + i s)(i k r - 1) / r = (c + i s)(i k - rinv): since r rinv = 1,
      // its parts are -(gr + s k) and c k - gi, with no product k r per pair
      real dr, di;
      if (HELM) {
        dr = -fma(G.s, kw, gr);
        di = fma(G.c, kw, -gi);
      } else {
        dr = -gr;
        di = real(0);
      }
      real w = real(0);
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const real *p = sp + 4 * c, *t = tp + 4 * c;
        // u = conj(g_i) q_j + conj(g_j) q_i
        real ur = t[2] * p[0];
        ur = fma(t[3], p[1], ur);
        ur = fma(p[2], t[0], ur);
        ur = fma(p[3], t[1], ur);
        real ui = t[2] * p[1];
        ui = fma(-t[3], p[0], ui);
        ui = fma(p[2], t[1], ui);
        ui = fma(-p[3], t[0], ui);
        w = fma(dr, ur, w);
        if (HELM) w = fma(-di, ui, w);
      }
      w *= G.rinv * G.rinv;  // sum over the columns of Re(G' u) / r, up to the scale
      acc[OX + 0] = fma(w, G.dx, acc[OX + 0]);
      acc[OX + 1] = fma(w, G.dy, acc[OX + 1]);
      acc[OX + 2] = fma(w, G.dz, acc[OX + 2]);
    }
  }
  __device__ __forceinline__ void store(int32_t t, const real* a) const {
    const int64_t i = perm[t];
    if (DQ) {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        cplx v;
        v.x = a[2 * c] * q_scale;
        v.y = a[2 * c + 1] * q_scale;
        gq[i * m + col + c] = v;
      }
    }
    if (DX) {
      for (int d = 0; d < 3; ++d) {
        const double v = (double)a[OX + d] * x_scale;
        gx[3 * i + d] = (col == 0) ? v : gx[3 * i + d] + v;
      }
    }
  }
};

template <class Tr, bool HELM, bool CSR, bool DQ, bool DX, int M = 1>
__global__ void __launch_bounds__(kBlock) k_backward(SweepGeom<Tr> G, BwdOp<Tr, DQ, DX, M> op) {
  __shared__ SweepLds<Tr, BwdOp<Tr, DQ, DX, M>, CSR> lds[kWavesPerBlock];
  sweep<Tr, BwdOp<Tr, DQ, DX, M>, HELM, CSR>(G, op, lds[threadIdx.x / kWave]);
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

template <class Tr, bool DQ, bool DX, int M>
static void launch_block(p2p_plan_s* P, const SweepGeom<Tr>& G, void* gq, double* gx, int m, int col,
                         hipStream_t s) {
  using real = typename Tr::real;
  using cplx = typename Tr::cplx;
  const bool helm = P->k != 0.0, csr = P->layout == P2P_LAYOUT_CSR;
  auto kern = helm ? (csr ? k_backward<Tr, true, true, DQ, DX, M> : k_backward<Tr, true, false, DQ, DX, M>)
                   : (csr ? k_backward<Tr, false, true, DQ, DX, M> : k_backward<Tr, false, false, DQ, DX, M>);
  const bool f32 = P->precision == P2P_C64;
  const double unit = f32 ? std::ldexp(1.0, -P->qexp) : 1.0;  // quantum -> length
  const real qsc = (real)(unit / (4.0 * M_PI));
  const double xsc = unit * unit / (4.0 * M_PI);
  const real kw = (real)(P->k / unit);
  BwdOp<Tr, DQ, DX, M> op{(const cplx*)P->q_sorted, (const cplx*)P->g_sorted, m, col, P->perm, (cplx*)gq, gx, qsc,
                          xsc, kw};
  hipLaunchKernelGGL(kern, dim3(grid_for(G.nb, kWavesPerBlock)), dim3(kBlock), 0, s, G, op);
}

// columns in launches of 4, 2 and 1
template <class Tr, bool DQ, bool DX>
static void launch_cols(p2p_plan_s* P, const SweepGeom<Tr>& G, void* gq, double* gx, int m, hipStream_t s) {
  for (int c = 0; c < m;) {
    const int left = m - c;
    if (left >= 4) {
      launch_block<Tr, DQ, DX, 4>(P, G, gq, gx, m, c, s);
      c += 4;
    } else if (left >= 2) {
      launch_block<Tr, DQ, DX, 2>(P, G, gq, gx, m, c, s);
      c += 2;
    } else {
      launch_block<Tr, DQ, DX, 1>(P, G, gq, gx, m, c, s);
      c += 1;
    }
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
