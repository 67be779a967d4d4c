// FP64 CPU oracle for the near-field P2P operator.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
// this file: only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark use it.  It shares no source, header, table or helper with the HIP
// library; the two meet only through arrays produced by the seeded generators.
//
// What it computes (paper: section 1 splits the MLFMA product into a near and a
// far field and names the near-field operator P2P; section 3.1 puts the points
// into the boxes of the last tree level; sections 3.2-3.3 sum, for each target,
// over the sources of the adjacent boxes, the box included; section 4.1's CPU
// baseline walks the boxes in Morton order and, for each target, loops over the
// sources of its neighbourhood):
//
//   y[i,c] = sum over j with  max_a |b_i[a] - b_j[a]| <= 1  and  x_i != x_j  of
//            G(|x_i - x_j|) q[j,c],          G(r) = exp(i k r) / (4 pi r)
//
// The three-dimensional Helmholtz kernel and the 27-box neighbourhood lift the
// paper's two-dimensional, nine-box setting (section 3.2 counts nine adjacent
// boxes in 2-D).  The self term and any coincident pair are skipped; the paper is
// silent on them.
//
// Plain loops in a fixed order, libm sqrt/cos/sin, compiled without FMA
// contraction.  OpenMP splits target boxes over threads; each output element is
// written by exactly one thread, so results do not depend on the thread count.
//
// Parity pins: every function here is checked in tests/ against brute force,
// closed forms and invariants (see tests/test_oracle_*.py).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const int kAxisBits = 21;
const int32_t kIdLimit = 1 << kAxisBits;
const double kPi = 3.14159265358979323846;

// Morton key (section 3.2 keeps boxes "in the order of the box's morton index"):
// bit 3b of the key is bit b of the x id, bit 3b+1 bit b of y, bit 3b+2 bit b of z.
uint64_t morton_key(int32_t ix, int32_t iy, int32_t iz) {
  uint64_t key = 0;
  for (int b = 0; b < kAxisBits; ++b) {
    key |= (uint64_t)((ix >> b) & 1) << (3 * b);
    key |= (uint64_t)((iy >> b) & 1) << (3 * b + 1);
    key |= (uint64_t)((iz >> b) & 1) << (3 * b + 2);
  }
  return key;
}

struct Plan {
  int64_t n = 0;
  std::vector<uint64_t> key;        // per point
  std::vector<int32_t> perm;        // sorted position -> original index
  std::vector<uint64_t> box_key;    // per non-empty box, ascending
  std::vector<int32_t> box_start;   // [B+1] offsets into perm
  std::vector<int32_t> nbr_start;   // [B+1] offsets into nbr_idx
  std::vector<int32_t> nbr_idx;     // neighbour boxes (self included), ascending
  std::vector<int32_t> box_of;      // sorted position -> box
};

// Contribution of source j to target i, for every right-hand side.
inline void accumulate(const double* xi, const double* xj, double k, const double* qj, int m, double* acc) {
  double dx = xi[0] - xj[0];
  double dy = xi[1] - xj[1];
  double dz = xi[2] - xj[2];
  if (dx == 0.0 && dy == 0.0 && dz == 0.0) return;  // r = 0: skipped
  double r = std::sqrt(dx * dx + dy * dy + dz * dz);
  double th = k * r;
  double gr = std::cos(th) / (4.0 * kPi * r);
  double gi = std::sin(th) / (4.0 * kPi * r);
  for (int c = 0; c < m; ++c) {
    double qr = qj[2 * c], qi = qj[2 * c + 1];
    acc[2 * c] += gr * qr - gi * qi;
    acc[2 * c + 1] += gr * qi + gi * qr;
  }
}

// Target-side rows: y for the target at sorted position p.
void row(const Plan& P, const double* xyz, double k, const double* q, int m, int64_t p, double* out) {
  for (int c = 0; c < 2 * m; ++c) out[c] = 0.0;
  int32_t i = P.perm[p];
  int32_t T = P.box_of[p];
  for (int32_t e = P.nbr_start[T]; e < P.nbr_start[T + 1]; ++e) {
    int32_t S = P.nbr_idx[e];
    for (int32_t s = P.box_start[S]; s < P.box_start[S + 1]; ++s) {
      int32_t j = P.perm[s];
      accumulate(xyz + 3 * (int64_t)i, xyz + 3 * (int64_t)j, k, q + 2 * (int64_t)m * j, m, out);
    }
  }
}

void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

// Small forward-mode dual number: value plus one derivative.
struct Dual {
  double v, d;
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual dsqrt(Dual a) {
  double s = std::sqrt(a.v);
  return {s, a.d / (2.0 * s)};
}
inline Dual dcos(Dual a) { return {std::cos(a.v), -std::sin(a.v) * a.d}; }
inline Dual dsin(Dual a) { return {std::sin(a.v), std::cos(a.v) * a.d}; }

}  // namespace

extern "C" {

// Status codes mirror the meaning of the library's, but are defined here on their own.
enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_RANGE = 2 };

int orc_box_ids(const double* xyz, int64_t n, const double* origin, double h, int32_t* ids) {
  if (n < 0 || (n > 0 && (!xyz || !ids)) || !origin) return ORC_ERR_ARG;
  if (!(h > 0.0) || !std::isfinite(h)) return ORC_ERR_RANGE;
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      double v = std::floor((xyz[3 * i + a] - origin[a]) / h);
      if (!(v >= 0.0 && v < (double)kIdLimit)) return ORC_ERR_RANGE;
    }
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) ids[3 * i + a] = (int32_t)std::floor((xyz[3 * i + a] - origin[a]) / h);
  return ORC_OK;
}

uint64_t orc_morton(int32_t ix, int32_t iy, int32_t iz) { return morton_key(ix, iy, iz); }

int orc_plan_build(const int32_t* ids, int64_t n, void** out) {
  if (!out || n < 0 || (n > 0 && !ids) || n >= (int64_t)INT32_MAX) return ORC_ERR_ARG;
  for (int64_t i = 0; i < 3 * n; ++i)
    if (ids[i] < 0 || ids[i] >= kIdLimit) return ORC_ERR_RANGE;
  Plan* P = new Plan();
  P->n = n;
  P->key.resize(n);
  for (int64_t i = 0; i < n; ++i) P->key[i] = morton_key(ids[3 * i], ids[3 * i + 1], ids[3 * i + 2]);
  // Points in key order; ties keep the original order.
  P->perm.resize(n);
  std::iota(P->perm.begin(), P->perm.end(), 0);
  std::stable_sort(P->perm.begin(), P->perm.end(),
                   [&](int32_t a, int32_t b) { return P->key[a] < P->key[b]; });
  // Runs of equal keys are the non-empty boxes.
  P->box_of.resize(n);
  for (int64_t p = 0; p < n; ++p) {
    uint64_t kk = P->key[P->perm[p]];
    if (p == 0 || kk != P->box_key.back()) {
      P->box_key.push_back(kk);
      P->box_start.push_back((int32_t)p);
    }
    P->box_of[p] = (int32_t)P->box_key.size() - 1;
  }
  P->box_start.push_back((int32_t)n);
  // Neighbour boxes: every non-empty box whose ids differ by at most one on each
  // axis (no wrap-around), the box itself included, in ascending key order.
  int64_t B = (int64_t)P->box_key.size();
  P->nbr_start.push_back(0);
  for (int64_t T = 0; T < B; ++T) {
    int32_t i0 = P->perm[P->box_start[T]];
    int32_t bx = ids[3 * i0], by = ids[3 * i0 + 1], bz = ids[3 * i0 + 2];
    std::vector<int32_t> hits;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int32_t x = bx + dx, y = by + dy, z = bz + dz;
          if (x < 0 || y < 0 || z < 0 || x >= kIdLimit || y >= kIdLimit || z >= kIdLimit) continue;
          uint64_t kk = morton_key(x, y, z);
          auto it = std::lower_bound(P->box_key.begin(), P->box_key.end(), kk);
          if (it != P->box_key.end() && *it == kk) hits.push_back((int32_t)(it - P->box_key.begin()));
        }
    std::sort(hits.begin(), hits.end());
    P->nbr_idx.insert(P->nbr_idx.end(), hits.begin(), hits.end());
    P->nbr_start.push_back((int32_t)P->nbr_idx.size());
  }
  *out = P;
  return ORC_OK;
}

void orc_plan_free(void* h) { delete (Plan*)h; }
int64_t orc_plan_nboxes(const void* h) { return (int64_t)((const Plan*)h)->box_key.size(); }
int64_t orc_plan_nnbr(const void* h) { return (int64_t)((const Plan*)h)->nbr_idx.size(); }

void orc_plan_export(const void* h, uint64_t* box_key, int32_t* box_start, int32_t* perm, int32_t* nbr_start,
                     int32_t* nbr_idx) {
  const Plan* P = (const Plan*)h;
  if (box_key) std::copy(P->box_key.begin(), P->box_key.end(), box_key);
  if (box_start) std::copy(P->box_start.begin(), P->box_start.end(), box_start);
  if (perm) std::copy(P->perm.begin(), P->perm.end(), perm);
  if (nbr_start) std::copy(P->nbr_start.begin(), P->nbr_start.end(), nbr_start);
  if (nbr_idx) std::copy(P->nbr_idx.begin(), P->nbr_idx.end(), nbr_idx);
}

// Pair statistics: ordered near pairs with r != 0, pairs skipped for r == 0
// (self pairs included), and the largest box occupancy t.
void orc_plan_stats(const void* h, const double* xyz, int64_t* n_pairs, int64_t* n_zero, int32_t* t_max) {
  const Plan* P = (const Plan*)h;
  int64_t B = (int64_t)P->box_key.size();
  int64_t pairs = 0, zero = 0;
  int32_t tm = 0;
  for (int64_t T = 0; T < B; ++T) {
    int32_t nT = P->box_start[T + 1] - P->box_start[T];
    tm = std::max(tm, nT);
    for (int32_t p = P->box_start[T]; p < P->box_start[T + 1]; ++p) {
      const double* xi = xyz + 3 * (int64_t)P->perm[p];
      for (int32_t e = P->nbr_start[T]; e < P->nbr_start[T + 1]; ++e) {
        int32_t S = P->nbr_idx[e];
        for (int32_t s = P->box_start[S]; s < P->box_start[S + 1]; ++s) {
          const double* xj = xyz + 3 * (int64_t)P->perm[s];
          if (xi[0] == xj[0] && xi[1] == xj[1] && xi[2] == xj[2]) ++zero;
          else ++pairs;
        }
      }
    }
  }
  *n_pairs = pairs;
  *n_zero = zero;
  *t_max = tm;
}

// y = A_near q for all points.  q, y: complex128 interleaved, [n, m] row-major,
// original point order.
int orc_apply(const void* h, const double* xyz, double k, const double* q, int m, double* y, int nthreads) {
  const Plan* P = (const Plan*)h;
  if (m < 1 || !std::isfinite(k) || k < 0) return ORC_ERR_ARG;
  set_threads(nthreads);
  int64_t n = P->n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < n; ++p) row(*P, xyz, k, q, m, p, y + 2 * (int64_t)m * P->perm[p]);
  return ORC_OK;
}

// y for the listed targets only (original indices), written to y_rows[nrows, m].
int orc_apply_rows(const void* h, const double* xyz, double k, const double* q, int m, const int64_t* rows,
                   int64_t nrows, double* y_rows, int nthreads) {
  const Plan* P = (const Plan*)h;
  if (m < 1 || !std::isfinite(k) || k < 0) return ORC_ERR_ARG;
  std::vector<int64_t> pos(P->n);
  for (int64_t p = 0; p < P->n; ++p) pos[P->perm[p]] = p;
  for (int64_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= P->n) return ORC_ERR_RANGE;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nrows; ++r) row(*P, xyz, k, q, m, pos[rows[r]], y_rows + 2 * (int64_t)m * r);
  return ORC_OK;
}

// Reverse mode for a real loss L(y) with upstream g = dL/dRe y + i dL/dIm y:
//   dq = conj(A conj(g))     (A is complex symmetric)
//   dx_i = sum_j Re( G'(r_ij) (conj(g_i) q_j + conj(g_j) q_i) ) (x_i - x_j) / r_ij,
//   G'(r) = exp(i k r) (i k r - 1) / (4 pi r^2),  summed over right-hand sides.
// dq or dx may be null.
int orc_backward(const void* h, const double* xyz, double k, const double* q, const double* g, int m, double* dq,
                 double* dx, int nthreads) {
  const Plan* P = (const Plan*)h;
  if (m < 1 || !std::isfinite(k) || k < 0) return ORC_ERR_ARG;
  set_threads(nthreads);
  int64_t n = P->n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < n; ++p) {
    int32_t i = P->perm[p];
    int32_t T = P->box_of[p];
    const double* xi = xyz + 3 * (int64_t)i;
    const double* qi = q + 2 * (int64_t)m * i;
    const double* gi = g + 2 * (int64_t)m * i;
    std::vector<double> accq(2 * m, 0.0);
    double ax = 0, ay = 0, az = 0;
    for (int32_t e = P->nbr_start[T]; e < P->nbr_start[T + 1]; ++e) {
      int32_t S = P->nbr_idx[e];
      for (int32_t s = P->box_start[S]; s < P->box_start[S + 1]; ++s) {
        int32_t j = P->perm[s];
        const double* xj = xyz + 3 * (int64_t)j;
        double ddx = xi[0] - xj[0], ddy = xi[1] - xj[1], ddz = xi[2] - xj[2];
        if (ddx == 0.0 && ddy == 0.0 && ddz == 0.0) continue;
        double r = std::sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
        double th = k * r;
        double c = std::cos(th), sn = std::sin(th);
        double gr = c / (4.0 * kPi * r), gim = sn / (4.0 * kPi * r);
        const double* qj = q + 2 * (int64_t)m * j;
        const double* gj = g + 2 * (int64_t)m * j;
        // G' = (c + i s)(i k r - 1) / (4 pi r^2) = (-(c + s k r) + i (c k r - s)) / (4 pi r^2)
        double dr = -(c + sn * k * r) / (4.0 * kPi * r * r);
        double di = (c * k * r - sn) / (4.0 * kPi * r * r);
        double w = 0.0;
        for (int cc = 0; cc < m; ++cc) {
          // conj(A conj g): accumulate G * conj(g_j), conjugate at the end
          double gjr = gj[2 * cc], gji = -gj[2 * cc + 1];
          accq[2 * cc] += gr * gjr - gim * gji;
          accq[2 * cc + 1] += gr * gji + gim * gjr;
          // u = conj(g_i) q_j + conj(g_j) q_i
          double ur = gi[2 * cc] * qj[2 * cc] + gi[2 * cc + 1] * qj[2 * cc + 1] + gj[2 * cc] * qi[2 * cc] +
                      gj[2 * cc + 1] * qi[2 * cc + 1];
          double ui = gi[2 * cc] * qj[2 * cc + 1] - gi[2 * cc + 1] * qj[2 * cc] + gj[2 * cc] * qi[2 * cc + 1] -
                      gj[2 * cc + 1] * qi[2 * cc];
          w += dr * ur - di * ui;  // Re(G' u)
        }
        ax += w * ddx / r;
        ay += w * ddy / r;
        az += w * ddz / r;
      }
    }
    if (dq)
      for (int cc = 0; cc < m; ++cc) {
        dq[2 * (int64_t)m * i + 2 * cc] = accq[2 * cc];
        dq[2 * (int64_t)m * i + 2 * cc + 1] = -accq[2 * cc + 1];
      }
    if (dx) {
      dx[3 * (int64_t)i] = ax;
      dx[3 * (int64_t)i + 1] = ay;
      dx[3 * (int64_t)i + 2] = az;
    }
  }
  return ORC_OK;
}

// Forward-mode derivative of L = sum |y|^2 with respect to coordinate a of point
// i, by dual numbers through the forward sum.  Only the rows whose value depends
// on x_i (i itself and its near points) are differentiated.  Independent of the
// closed-form reverse pass above.
int orc_dual_dx(const void* h, const double* xyz, double k, const double* q, int m, int64_t i, int a, double* dL) {
  const Plan* P = (const Plan*)h;
  if (i < 0 || i >= P->n || a < 0 || a > 2 || m < 1) return ORC_ERR_ARG;
  std::vector<int64_t> pos(P->n);
  for (int64_t p = 0; p < P->n; ++p) pos[P->perm[p]] = p;
  int32_t Ti = P->box_of[pos[i]];
  // Rows that depend on x_i: every point of every box adjacent to i's box.
  std::vector<int32_t> rows;
  for (int32_t e = P->nbr_start[Ti]; e < P->nbr_start[Ti + 1]; ++e) {
    int32_t S = P->nbr_idx[e];
    for (int32_t s = P->box_start[S]; s < P->box_start[S + 1]; ++s) rows.push_back(P->perm[s]);
  }
  double total = 0.0;
  for (int32_t r : rows) {
    int32_t T = P->box_of[pos[r]];
    std::vector<Dual> yr(m, Dual{0, 0}), yi(m, Dual{0, 0});
    Dual xr[3];
    for (int b = 0; b < 3; ++b) xr[b] = Dual{xyz[3 * (int64_t)r + b], (r == i && b == a) ? 1.0 : 0.0};
    for (int32_t e = P->nbr_start[T]; e < P->nbr_start[T + 1]; ++e) {
      int32_t S = P->nbr_idx[e];
      for (int32_t s = P->box_start[S]; s < P->box_start[S + 1]; ++s) {
        int32_t j = P->perm[s];
        Dual xj[3];
        for (int b = 0; b < 3; ++b) xj[b] = Dual{xyz[3 * (int64_t)j + b], (j == i && b == a) ? 1.0 : 0.0};
        Dual d0 = xr[0] - xj[0], d1 = xr[1] - xj[1], d2 = xr[2] - xj[2];
        if (d0.v == 0.0 && d1.v == 0.0 && d2.v == 0.0) continue;
        Dual rr = dsqrt(d0 * d0 + d1 * d1 + d2 * d2);
        Dual th = Dual{k, 0.0} * rr;
        Dual den = Dual{4.0 * kPi, 0.0} * rr;
        Dual gr = dcos(th) / den, gim = dsin(th) / den;
        for (int c = 0; c < m; ++c) {
          Dual qr{q[2 * (int64_t)m * j + 2 * c], 0.0}, qi{q[2 * (int64_t)m * j + 2 * c + 1], 0.0};
          yr[c] = yr[c] + (gr * qr - gim * qi);
          yi[c] = yi[c] + (gr * qi + gim * qr);
        }
      }
    }
    for (int c = 0; c < m; ++c) total += 2.0 * (yr[c].v * yr[c].d + yi[c].v * yi[c].d);
  }
  *dL = total;
  return ORC_OK;
}

// ---------------------------------------------------------------------------
// The paper's own two-dimensional setting (section 3.1: a quadtree of height L,
// branching factor 4, whose 4^(L-1) leaf boxes cover the plate; sections 3.2 and
// 3.3: nine neighbour boxes in 2-D, the box itself included; section 4: random
// points on a square plate, one real potential per source).  The plate is the
// unit square, leaf box (bx, by) = (floor(x 2^(L-1)), floor(y 2^(L-1))).  The
// paper names its kernel only as the electric potential in two dimensions; the
// reading taken here is the 2-D free-space potential G(r) = -ln(r) / (2 pi).
// Boxes in Morton order with bit 2b of the key from bit b of bx and bit 2b+1 from
// bit b of by: the 3-D key of ids (bx, by, 0) orders boxes the same way, so the
// quadtree plan is the 3-D plan of those ids (its 27 offsets find the same nine
// boxes, the other layers being empty).
// ---------------------------------------------------------------------------

// Leaf-box ids (bx, by, 0) of points of the unit square for a quadtree of height L.
int quad_ids(const double* xy, int64_t n, int32_t level, std::vector<int32_t>& ids) {
  if (level < 1 || level > kAxisBits + 1) return ORC_ERR_RANGE;
  const double side = std::ldexp(1.0, level - 1);  // boxes per axis
  ids.assign(3 * (size_t)n, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 2; ++a) {
      double x = xy[2 * i + a];
      if (!(x >= 0.0 && x < 1.0)) return ORC_ERR_RANGE;
      ids[3 * i + a] = (int32_t)std::floor(x * side);
    }
  return ORC_OK;
}

// y_i = sum over j in the nine boxes around i's box, x_j != x_i, of -ln|x_i - x_j| / (2 pi) q_j.
// xy: [n, 2]; q, y: [n] real, original point order.
int orc2d_apply(const double* xy, const double* q, int64_t n, int32_t level, double* y, int nthreads) {
  if (n < 0 || (n > 0 && (!xy || !q || !y))) return ORC_ERR_ARG;
  std::vector<int32_t> ids;
  int rc = quad_ids(xy, n, level, ids);
  if (rc != ORC_OK) return rc;
  void* h = nullptr;
  rc = orc_plan_build(ids.data(), n, &h);
  if (rc != ORC_OK) return rc;
  const Plan* P = (const Plan*)h;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < n; ++p) {
    const int32_t i = P->perm[p];
    const int32_t T = P->box_of[p];
    double acc = 0.0;
    for (int32_t e = P->nbr_start[T]; e < P->nbr_start[T + 1]; ++e) {
      const int32_t S = P->nbr_idx[e];
      for (int32_t s = P->box_start[S]; s < P->box_start[S + 1]; ++s) {
        const int32_t j = P->perm[s];
        const double dx = xy[2 * (int64_t)i] - xy[2 * (int64_t)j], dy = xy[2 * (int64_t)i + 1] - xy[2 * (int64_t)j + 1];
        if (dx == 0.0 && dy == 0.0) continue;  // r = 0: skipped
        const double r = std::sqrt(dx * dx + dy * dy);
        acc += -std::log(r) / (2.0 * kPi) * q[j];
      }
    }
    y[i] = acc;
  }
  orc_plan_free(h);
  return ORC_OK;
}

// Near pairs (ordered, r != 0), skipped pairs (r == 0, self pairs included), the
// largest box occupancy t and the number of non-empty boxes of the quadtree.
int orc2d_stats(const double* xy, int64_t n, int32_t level, int64_t* n_pairs, int64_t* n_zero, int32_t* t_max,
                int64_t* n_boxes) {
  std::vector<int32_t> ids;
  int rc = quad_ids(xy, n, level, ids);
  if (rc != ORC_OK) return rc;
  std::vector<double> xyz(3 * (size_t)n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    xyz[3 * i] = xy[2 * i];
    xyz[3 * i + 1] = xy[2 * i + 1];
  }
  void* h = nullptr;
  rc = orc_plan_build(ids.data(), n, &h);
  if (rc != ORC_OK) return rc;
  orc_plan_stats(h, xyz.data(), n_pairs, n_zero, t_max);
  *n_boxes = orc_plan_nboxes(h);
  orc_plan_free(h);
  return ORC_OK;
}

}  // extern "C"
