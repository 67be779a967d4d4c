// The paper's own experiment: points on a square plate, a quadtree of height L,
// nine neighbour boxes, one real potential per source and the 2-D potential
// G(r) = -ln(r) / (2 pi), computed by the paper's two GPU layouts and by this
// library's sweep.
//
// Section 3.1: the 4^(L-1) leaf boxes of a quadtree over the plate (here the unit
// square), box (floor(x 2^(L-1)), floor(y 2^(L-1))).  Section 3.2, the Indexing
// method: the host collects seven arrays (target and source coordinates, the
// targets of every box in Morton order with their box offsets, the neighbour
// sources of every box with their offsets, the source potentials), stored one
// after the other; the device runs one thread per box, which loops over its
// targets and, for each, over the box's neighbour sources.  Section 3.3, the
// Repetition method: the host writes one record per target, [x, y, count, then
// (x, y, q) of every neighbour source], each record padded to the same length so
// that a thread finds its own from its index alone; the device runs one thread
// per target.  Both layouts are collected on the host and copied to the device
// for every run, as in the paper, so the three phases (collection, transfer,
// kernel) are timed separately.  The paper adds nothing to either design
// (section 3: no shared memory, prefetching or overlap); neither is tuned here.
//
// This library's own route to the same result is the plan of the points with
// ids (bx, by, 0) -- the quadtree's boxes in the same Morton order -- built on
// the device, and the wavefront-per-box sweep of sweep.h with the 2-D kernel
// (p2p_apply_log2d).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "sweep.h"

struct p2p2d_s {
  uint64_t magic;
  p2p2d_method method;
  int64_t n;
  int32_t level, ct;
  int64_t boxes;        // 4^(L-1): every leaf box, empty ones included
  int64_t n_src;        // Indexing: neighbour-source entries over all boxes
  int32_t t_max;        // largest box occupancy
  int32_t rec;          // Repetition: record length in doubles
  int64_t n_slots;      // ordered near pairs, self pairs included
  std::vector<char> host;  // the collected layout
  void* dev;            // its device copy (after p2p2d_transfer)
  size_t dev_bytes;
  double collect_ms, transfer_ms;
  hipEvent_t last_use;  // recorded after each run: destroy waits for it
  // offsets of the arrays within the layout
  size_t o_txy, o_sxy, o_tidx, o_tstart, o_sidx, o_sstart, o_q, o_rec, o_perm;
};

namespace p2p {

constexpr uint64_t k2dMagic = 0x7032705f71756164ull;

static p2p_status check2d(p2p2d_s* h) {
  if (!h || !handle_live(h) || h->magic != k2dMagic) return fail(P2P_ERR_STATE, "invalid 2-D handle");
  return P2P_OK;
}

// Morton key of a quadtree box: bit 2b from bit b of bx, bit 2b+1 from bit b of by.
static inline uint64_t quad_key(uint32_t bx, uint32_t by) {
  uint64_t k = 0;
  for (int b = 0; b < 32; ++b) {
    k |= (uint64_t)((bx >> b) & 1u) << (2 * b);
    k |= (uint64_t)((by >> b) & 1u) << (2 * b + 1);
  }
  return k;
}
static inline uint32_t quad_x(uint64_t k) {
  uint32_t v = 0;
  for (int b = 0; b < 32; ++b) v |= (uint32_t)((k >> (2 * b)) & 1u) << b;
  return v;
}
static inline uint32_t quad_y(uint64_t k) { return quad_x(k >> 1); }

// The pair term of both layouts' kernels: ln(r^2) q, the scale -1/(4 pi) applied once.
__device__ __forceinline__ double log_term(double dx, double dy, double q) {
  const double r2 = dx * dx + dy * dy;
  return r2 > 0.0 ? log(r2) * q : 0.0;
}

// Indexing (section 3.2): one thread per box, every box of the tree.
__global__ void __launch_bounds__(kBlock) k_indexing(const double* __restrict__ txy, const double* __restrict__ sxy,
                                                  const int32_t* __restrict__ tidx,
                                                  const int32_t* __restrict__ tstart,
                                                  const int32_t* __restrict__ sidx,
                                                  const int32_t* __restrict__ sstart,
                                                  const double* __restrict__ q, int64_t boxes,
                                                  double* __restrict__ y) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= boxes) return;
  const int32_t s0 = sstart[b], s1 = sstart[b + 1];
  for (int32_t k = tstart[b]; k < tstart[b + 1]; ++k) {
    const int32_t i = tidx[k];
    const double xi = txy[2 * (int64_t)i], yi = txy[2 * (int64_t)i + 1];
    double acc = 0.0;
    for (int32_t e = s0; e < s1; ++e) {
      const int32_t j = sidx[e];
      acc += log_term(xi - sxy[2 * (int64_t)j], yi - sxy[2 * (int64_t)j + 1], q[j]);
    }
    y[i] = acc * (-1.0 / (4.0 * M_PI));
  }
}

// Repetition (section 3.3): one thread per target, its record at index * rec.
__global__ void __launch_bounds__(kBlock) k_repetition(const double* __restrict__ recs, int32_t rec,
                                                    const int32_t* __restrict__ perm, int64_t n,
                                                    double* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const double* r = recs + t * rec;
  const double xi = r[0], yi = r[1];
  const int32_t cnt = (int32_t)r[2];  // the count travels as a double
  double acc = 0.0;
  for (int32_t c = 0; c < cnt; ++c) acc += log_term(xi - r[3 + 3 * c], yi - r[4 + 3 * c], r[5 + 3 * c]);
  y[perm[t]] = acc * (-1.0 / (4.0 * M_PI));
}

// ---------------------------------------------------------------------------
// the library's sweep on the same problem
// ---------------------------------------------------------------------------
struct LogOp {
  static constexpr int K = L2D::K1, NP = 1, NT = 0, NA = 1;
  const double* __restrict__ qs;
  const int32_t* __restrict__ perm;
  double* __restrict__ y;
  __device__ __forceinline__ void load_src(int32_t p, double* pay) const { pay[0] = qs[p]; }
  __device__ __forceinline__ void load_tgt(int32_t, double*) const {}
  template <bool HELM>
  __device__ __forceinline__ void pair(const L2D::Geo& g, const double* sp, const double*, double* acc) const {
    acc[0] = fma(g.l, sp[0], acc[0]);
  }
  __device__ __forceinline__ void store(int32_t t, const double* a) const {
    y[perm[t]] = a[0] * (-1.0 / (4.0 * M_PI));
  }
};

template <bool CSR>
__global__ void __launch_bounds__(kBlock) k_log2d(SweepGeom<L2D> G, LogOp op) {
  __shared__ SweepLds<L2D, LogOp, CSR> lds[kWavesPerBlock];
  sweep<L2D, LogOp, false, CSR>(G, op, lds[threadIdx.x / kWave]);
}

__global__ void __launch_bounds__(kBlock) k_gather_real(const double* __restrict__ q, const int32_t* __restrict__ perm,
                                                     int64_t n, double* __restrict__ qs) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < n) qs[p] = q[perm[p]];
}

// ---------------------------------------------------------------------------
// host collection (single-threaded, as the paper's data collection)
// ---------------------------------------------------------------------------
namespace {

struct Boxes {
  std::vector<int32_t> tidx;    // points box by box (Morton order), input order inside a box
  std::vector<int32_t> tstart;  // [boxes + 1]
  int32_t t_max = 0;
};

p2p_status quad_boxes(const double* xy, int64_t n, int32_t level, Boxes& bx) {
  const double side = std::ldexp(1.0, level - 1);
  const int64_t boxes = (int64_t)1 << (2 * (level - 1));
  std::vector<int64_t> key(n);
  for (int64_t i = 0; i < n; ++i) {
    const double x = xy[2 * i], y = xy[2 * i + 1];
    if (!(x >= 0.0 && x < 1.0 && y >= 0.0 && y < 1.0)) return fail(P2P_ERR_RANGE, "a point lies outside the unit square");
    key[i] = (int64_t)quad_key((uint32_t)std::floor(x * side), (uint32_t)std::floor(y * side));
  }
  // counting sort by box (stable)
  bx.tstart.assign(boxes + 1, 0);
  for (int64_t i = 0; i < n; ++i) ++bx.tstart[key[i] + 1];
  for (int64_t b = 0; b < boxes; ++b) {
    bx.t_max = std::max(bx.t_max, bx.tstart[b + 1]);
    bx.tstart[b + 1] += bx.tstart[b];
  }
  bx.tidx.resize(n);
  std::vector<int32_t> fill(bx.tstart.begin(), bx.tstart.end() - 1);
  for (int64_t i = 0; i < n; ++i) bx.tidx[fill[key[i]]++] = (int32_t)i;
  return P2P_OK;
}

// The nine boxes around b (b included, those inside the tree), ascending by key.
int neighbours(uint64_t b, int32_t level, uint64_t* out) {
  const int64_t side = (int64_t)1 << (level - 1);
  const int64_t x = quad_x(b), y = quad_y(b);
  int c = 0;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const int64_t nx = x + dx, ny = y + dy;
      if (nx < 0 || ny < 0 || nx >= side || ny >= side) continue;
      out[c++] = quad_key((uint32_t)nx, (uint32_t)ny);
    }
  std::sort(out, out + c);
  return c;
}

template <typename T>
T* at(std::vector<char>& v, size_t off) {
  return reinterpret_cast<T*>(v.data() + off);
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

static p2p_status collect(p2p2d_s* h, const double* xy, const double* q) {
  const int64_t n = h->n;
  Boxes bx;
  p2p_status rc = quad_boxes(xy, n, h->level, bx);
  if (rc != P2P_OK) return rc;
  h->t_max = bx.t_max;
  uint64_t nb[9];
  try {
    if (h->method == P2P2D_INDEXING) {
      // neighbour-source offsets first (sizes), then the seven arrays back to back
      std::vector<int32_t> sstart(h->boxes + 1, 0);
      int64_t total = 0, pairs = 0;
      for (int64_t b = 0; b < h->boxes; ++b) {
        const int c = neighbours((uint64_t)b, h->level, nb);
        int64_t ns = 0;
        for (int e = 0; e < c; ++e) ns += bx.tstart[nb[e] + 1] - bx.tstart[nb[e]];
        total += ns;
        pairs += ns * (bx.tstart[b + 1] - bx.tstart[b]);
        if (total > 0x7fffffffll) return fail(P2P_ERR_RANGE, "more than 2^31 neighbour-source entries");
        sstart[b + 1] = (int32_t)total;
      }
      h->n_src = total;
      h->n_slots = pairs;
      size_t o = 0;
      h->o_txy = o;
      o = align256(o + 16 * (size_t)n);
      h->o_sxy = o;
      o = align256(o + 16 * (size_t)n);
      h->o_tidx = o;
      o = align256(o + 4 * (size_t)n);
      h->o_tstart = o;
      o = align256(o + 4 * (size_t)(h->boxes + 1));
      h->o_sidx = o;
      o = align256(o + 4 * (size_t)total);
      h->o_sstart = o;
      o = align256(o + 4 * (size_t)(h->boxes + 1));
      h->o_q = o;
      o = align256(o + 8 * (size_t)n);
      h->host.resize(o);
      std::memcpy(at<double>(h->host, h->o_txy), xy, 16 * (size_t)n);
      std::memcpy(at<double>(h->host, h->o_sxy), xy, 16 * (size_t)n);
      std::memcpy(at<int32_t>(h->host, h->o_tidx), bx.tidx.data(), 4 * (size_t)n);
      std::memcpy(at<int32_t>(h->host, h->o_tstart), bx.tstart.data(), 4 * (size_t)(h->boxes + 1));
      std::memcpy(at<int32_t>(h->host, h->o_sstart), sstart.data(), 4 * (size_t)(h->boxes + 1));
      std::memcpy(at<double>(h->host, h->o_q), q, 8 * (size_t)n);
      int32_t* sidx = at<int32_t>(h->host, h->o_sidx);
      for (int64_t b = 0; b < h->boxes; ++b) {
        const int c = neighbours((uint64_t)b, h->level, nb);
        int32_t w = sstart[b];
        for (int e = 0; e < c; ++e)
          for (int32_t k = bx.tstart[nb[e]]; k < bx.tstart[nb[e] + 1]; ++k) sidx[w++] = bx.tidx[k];
      }
    } else {
      // record length: 3 + 3 * the neighbourhood bound 9 CT (section 3.3), or the
      // largest neighbourhood when boxes hold more than CT points
      int64_t smax = 9 * (int64_t)h->ct, pairs = 0;
      for (int64_t b = 0; b < h->boxes; ++b) {
        if (bx.tstart[b + 1] == bx.tstart[b]) continue;
        const int c = neighbours((uint64_t)b, h->level, nb);
        int64_t ns = 0;
        for (int e = 0; e < c; ++e) ns += bx.tstart[nb[e] + 1] - bx.tstart[nb[e]];
        smax = std::max(smax, ns);
        pairs += ns * (bx.tstart[b + 1] - bx.tstart[b]);
      }
      if (3 + 3 * smax > 0x7fffffffll) return fail(P2P_ERR_RANGE, "record too long");
      h->rec = (int32_t)(3 + 3 * smax);
      h->n_slots = pairs;
      h->o_rec = 0;
      h->o_perm = align256(8 * (size_t)n * (size_t)h->rec);
      h->host.assign(h->o_perm + 4 * (size_t)n, 0);
      double* recs = at<double>(h->host, h->o_rec);
      int32_t* perm = at<int32_t>(h->host, h->o_perm);
      int64_t t = 0;
      for (int64_t b = 0; b < h->boxes; ++b) {
        if (bx.tstart[b + 1] == bx.tstart[b]) continue;
        const int c = neighbours((uint64_t)b, h->level, nb);
        for (int32_t k = bx.tstart[b]; k < bx.tstart[b + 1]; ++k, ++t) {
          const int32_t i = bx.tidx[k];
          double* r = recs + t * h->rec;
          r[0] = xy[2 * (int64_t)i];
          r[1] = xy[2 * (int64_t)i + 1];
          int64_t cnt = 0;
          for (int e = 0; e < c; ++e)
            for (int32_t kk = bx.tstart[nb[e]]; kk < bx.tstart[nb[e] + 1]; ++kk, ++cnt) {
              const int32_t j = bx.tidx[kk];
              r[3 + 3 * cnt] = xy[2 * (int64_t)j];
              r[4 + 3 * cnt] = xy[2 * (int64_t)j + 1];
              r[5 + 3 * cnt] = q[j];
            }
          r[2] = (double)cnt;
          perm[t] = i;
        }
      }
    }
  } catch (const std::bad_alloc&) {
    return fail(P2P_ERR_NOMEM, "host allocation for the collected layout failed");
  }
  return P2P_OK;
}

}  // namespace p2p

using namespace p2p;

extern "C" {

p2p_status p2p2d_collect(p2p2d_method method, const double* xy, const double* q, int64_t n, int32_t level,
                         int32_t ct, p2p2d* out) {
  if (!out) return fail(P2P_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (method != P2P2D_INDEXING && method != P2P2D_REPETITION) return fail(P2P_ERR_ARG, "unknown method");
  if (n < 0 || (n > 0 && (!xy || !q))) return fail(P2P_ERR_ARG, "n < 0 or NULL arrays");
  if (n > 0x7fffffffll) return fail(P2P_ERR_RANGE, "n exceeds 2^31 - 1");
  if (level < 1 || level > 15) return fail(P2P_ERR_RANGE, "level must be in [1, 15]");
  if (ct < 1) return fail(P2P_ERR_ARG, "ct must be >= 1");
  p2p2d_s* h = new (std::nothrow) p2p2d_s();
  if (!h) return fail(P2P_ERR_NOMEM, "host allocation failed");
  h->magic = k2dMagic;
  h->method = method;
  h->n = n;
  h->level = level;
  h->ct = ct;
  h->boxes = (int64_t)1 << (2 * (level - 1));
  h->dev = nullptr;
  h->last_use = nullptr;  // created by the first transfer: collection needs no device
  handle_add(h);
  const auto t0 = std::chrono::steady_clock::now();
  p2p_status rc = collect(h, xy, q);
  h->collect_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rc != P2P_OK) {
    handle_remove(h);
    delete h;
    return rc;
  }
  *out = h;
  return P2P_OK;
}

p2p_status p2p2d_transfer(p2p2d h, void* stream) {
  p2p_status rc = check2d(h);
  if (rc != P2P_OK) return rc;
  const hipStream_t s = (hipStream_t)stream;
  if (!h->last_use && hipEventCreateWithFlags(&h->last_use, hipEventDisableTiming) != hipSuccess) {
    h->last_use = nullptr;
    return fail(P2P_ERR_HIP, "hipEventCreateWithFlags failed");
  }
  const auto t0 = std::chrono::steady_clock::now();
  if (!h->dev || h->dev_bytes < h->host.size()) {
    if (h->dev) {
      P2P_HIP(hipStreamSynchronize(s));
      dmem_free(h->dev);
    }
    h->dev = dmem_alloc(h->host.size());
    if (!h->dev) return fail(P2P_ERR_NOMEM, "device allocation for the collected layout failed");
    h->dev_bytes = h->host.size();
  }
  if (!h->host.empty()) P2P_HIP(hipMemcpyAsync(h->dev, h->host.data(), h->host.size(), hipMemcpyHostToDevice, s));
  P2P_HIP(hipStreamSynchronize(s));
  h->transfer_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return P2P_OK;
}

p2p_status p2p2d_run(p2p2d h, double* y, void* stream) {
  p2p_status rc = check2d(h);
  if (rc != P2P_OK) return rc;
  if (h->n > 0 && !y) return fail(P2P_ERR_ARG, "y is NULL");
  if (h->n > 0 && !h->dev) return fail(P2P_ERR_STATE, "the layout has not been transferred");
  if (h->n == 0) return P2P_OK;
  const hipStream_t s = (hipStream_t)stream;
  char* d = (char*)h->dev;
  if (h->method == P2P2D_INDEXING) {
    hipLaunchKernelGGL(k_indexing, dim3(grid_for(h->boxes)), dim3(kBlock), 0, s, (const double*)(d + h->o_txy),
                       (const double*)(d + h->o_sxy), (const int32_t*)(d + h->o_tidx),
                       (const int32_t*)(d + h->o_tstart), (const int32_t*)(d + h->o_sidx),
                       (const int32_t*)(d + h->o_sstart), (const double*)(d + h->o_q), h->boxes, y);
  } else {
    hipLaunchKernelGGL(k_repetition, dim3(grid_for(h->n)), dim3(kBlock), 0, s, (const double*)(d + h->o_rec),
                       h->rec, (const int32_t*)(d + h->o_perm), h->n, y);
  }
  P2P_HIP(hipGetLastError());
  record_use(h->last_use, s);
  return P2P_OK;
}

p2p_status p2p2d_info(p2p2d h, p2p2d_info_t* out) {
  p2p_status rc = check2d(h);
  if (rc != P2P_OK) return rc;
  if (!out) return fail(P2P_ERR_ARG, "out is NULL");
  out->n_points = h->n;
  out->n_boxes = h->boxes;
  out->layout_bytes = (int64_t)h->host.size();
  out->n_slots = h->n_slots;
  out->n_src_entries = h->n_src;
  out->t_max = h->t_max;
  out->record_len = h->rec;
  out->collect_ms = h->collect_ms;
  out->transfer_ms = h->transfer_ms;
  return P2P_OK;
}

p2p_status p2p2d_layout(p2p2d h, const void** data, int64_t* bytes, int64_t* offsets) {
  p2p_status rc = check2d(h);
  if (rc != P2P_OK) return rc;
  if (!data || !bytes || !offsets) return fail(P2P_ERR_ARG, "NULL output");
  *data = h->host.data();
  *bytes = (int64_t)h->host.size();
  const size_t o[9] = {h->o_txy, h->o_sxy, h->o_tidx, h->o_tstart, h->o_sidx, h->o_sstart, h->o_q, h->o_rec, h->o_perm};
  for (int i = 0; i < 9; ++i) offsets[i] = (int64_t)o[i];
  return P2P_OK;
}

p2p_status p2p2d_destroy(p2p2d h) {
  if (!h) return P2P_OK;
  p2p_status rc = check2d(h);
  if (rc != P2P_OK) return rc;
  handle_remove(h);
  if (h->last_use) {
    (void)hipEventSynchronize(h->last_use);
    (void)hipEventDestroy(h->last_use);
  }
  dmem_free(h->dev);
  h->magic = 0;
  delete h;
  return P2P_OK;
}

p2p_status p2p_apply_log2d(p2p_plan plan, const double* q, double* y, void* stream) {
  if (!plan || !handle_live(plan) || plan->magic != kPlanMagic) return fail(P2P_ERR_STATE, "invalid plan handle");
  if (plan->precision != P2P_C128) return fail(P2P_ERR_DTYPE, "the 2-D kernel runs on FP64 (complex128) plans");
  if (plan->distinct_sets) return fail(P2P_ERR_ARG, "the 2-D kernel runs on plans of one point set");
  if (plan->n > 0 && (!q || !y)) return fail(P2P_ERR_ARG, "q or y is NULL");
  if (plan->n == 0) return P2P_OK;
  const hipStream_t s = (hipStream_t)stream;
  const p2p_status rc = wait_built(plan, s);
  if (rc != P2P_OK) return rc;
  hipLaunchKernelGGL(k_gather_real, dim3(grid_for(plan->n)), dim3(kBlock), 0, s, q, plan->perm, plan->n,
                     (double*)plan->q_sorted);
  const SweepGeom<L2D> G = make_geom<L2D>(plan);
  const LogOp op{(const double*)plan->q_sorted, plan->perm, y};
  SweepTimer timer(plan, s);
  timer.start();
  if (plan->layout == P2P_LAYOUT_CSR)
    hipLaunchKernelGGL(k_log2d<true>, dim3(grid_for(G.nb, kWavesPerBlock)), dim3(kBlock), 0, s, G, op);
  else
    hipLaunchKernelGGL(k_log2d<false>, dim3(grid_for(G.nb, kWavesPerBlock)), dim3(kBlock), 0, s, G, op);
  timer.stop();
  P2P_HIP(hipGetLastError());
  if (record_use(plan->last_use, s)) plan->used = true;
  return P2P_OK;
}

}  // extern "C"
