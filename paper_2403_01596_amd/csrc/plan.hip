// Plan build on the device: leaf-box ids, Morton keys, stable radix sort, box
// table, neighbour lists, fixed-point coordinates and the replicated per-box
// source lists.
//
// Paper, section 3.1: the points go into the boxes of the last tree level.
// Section 3.2: boxes are kept in Morton order; for each box, the indices of its
// targets and of the sources in its neighbour boxes, with offset arrays.
// Section 3.3: the redundant layout, in which every consumer owns a contiguous
// copy of all the sources it reads.  The paper builds these on the host and
// copies them to the device on every run; here they are built once per point
// set, on the device, and stay resident.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace p2p {

// ---------------------------------------------------------------------------
// device scan (exclusive prefix sum), three passes: tile sums, scan of the tile
// sums in one workgroup, tile scans plus offsets.
// ---------------------------------------------------------------------------
constexpr int kWavesPerBlockPlan = kBlock / kWave;
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T* lds, T* total) {
  // lds: kBlock / kWave entries
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  T incl = v;
  for (int off = 1; off < kWave; off <<= 1) {
    T o = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += o;
  }
  if (lane == kWave - 1) lds[wave] = incl;
  __syncthreads();
  T base = 0, sum = 0;
  for (int w = 0; w < kBlock / kWave; ++w) {
    if (w < wave) base += lds[w];
    sum += lds[w];
  }
  __syncthreads();
  *total = sum;
  return base + incl - v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_reduce(const T* __restrict__ in, int64_t n, T* __restrict__ part) {
  __shared__ T lds[kBlock / kWave];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = 0;
  for (int r = 0; r < kScanItems; ++r) {
    int64_t e = base + (int64_t)r * kBlock + threadIdx.x;
    if (e < n) s += in[e];
  }
  T tot;
  block_exclusive_scan<T>(s, lds, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_partials(T* __restrict__ part, int64_t g, T* __restrict__ total_out) {
  __shared__ T lds[kBlock / kWave];
  T carry = 0;
  for (int64_t c = 0; c < g; c += kBlock) {
    int64_t e = c + threadIdx.x;
    T v = e < g ? part[e] : T(0);
    T tot;
    T ex = block_exclusive_scan<T>(v, lds, &tot);
    if (e < g) part[e] = ex + carry;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_apply(const T* __restrict__ in, int64_t n, const T* __restrict__ part,
                                                    T* __restrict__ out) {
  // each thread owns kScanItems consecutive elements of the tile
  __shared__ T lds[kBlock / kWave];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
  for (int r = 0; r < kScanItems; ++r) {
    int64_t e = base + r;
    v[r] = e < n ? in[e] : T(0);
    s += v[r];
  }
  T tot;
  T ex = block_exclusive_scan<T>(s, lds, &tot) + part[blockIdx.x];
  for (int r = 0; r < kScanItems; ++r) {
    int64_t e = base + r;
    if (e < n) out[e] = ex;
    ex += v[r];
  }
}

// out[0..n) = exclusive prefix of in; *total = sum (device pointer, may be null).
// part: workspace of at least grid_for(n, kScanTile) elements.  in == out allowed.
template <typename T>
static p2p_status scan(const T* in, T* out, int64_t n, T* part, T* total, hipStream_t s) {
  if (n <= 0) {
    if (total) P2P_HIP(hipMemsetAsync(total, 0, sizeof(T), s));
    return P2P_OK;
  }
  unsigned g = grid_for(n, kScanTile);
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(g), dim3(kBlock), 0, s, in, n, part);
  hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(kBlock), 0, s, part, (int64_t)g, total);
  hipLaunchKernelGGL(k_scan_apply<T>, dim3(g), dim3(kBlock), 0, s, in, n, part, out);
  P2P_HIP(hipGetLastError());
  return P2P_OK;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (u64 key, i32 value), 8 bits per pass
// ---------------------------------------------------------------------------
constexpr int kRsItems = 16;
constexpr int kRsTile = kBlock * kRsItems;

__global__ void __launch_bounds__(kBlock) k_rs_hist(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                 uint32_t* __restrict__ hist, int g) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    int64_t e = base + (int64_t)r * kBlock + threadIdx.x;
    if (e < n) atomicAdd(&h[(key[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * g + blockIdx.x] = h[threadIdx.x];
}

// Scatter one tile in input order.  Within a round of 256 elements the rank of
// an element among equal digits comes from wave ballots (lanes below it with the
// same digit) plus the counts of the waves before it; rounds are processed in
// order, so equal digits keep their input order (stability).
__global__ void __launch_bounds__(kBlock) k_rs_scatter(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                    uint64_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t n,
                                                    int shift, const uint32_t* __restrict__ offs, int g) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kBlock / kWave][256];
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid & (kWave - 1);
  run[tid] = offs[(int64_t)tid * g + blockIdx.x];
  for (int w = 0; w < kBlock / kWave; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsItems; ++r) {
    int64_t e = base + (int64_t)r * kBlock + tid;
    bool valid = e < n;
    uint64_t k = valid ? kin[e] : 0ull;
    uint32_t d = (uint32_t)(k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      uint64_t bb = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    uint32_t rank = __popcll(peers & below);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = k;
      vout[pos] = vin[e];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      add += wcnt[w][tid];
      wcnt[w][tid] = 0;
    }
    run[tid] += add;
    __syncthreads();
  }
}

// Sorts (k0, v0) by the low `bits` bits of the key.  Result is in (k0, v0) or
// (k1, v1); *in_second tells which.  hist: 256 * grid entries, part: scan workspace.
static p2p_status radix_sort(uint64_t* k0, int32_t* v0, uint64_t* k1, int32_t* v1, int64_t n, int bits,
                             uint32_t* hist, uint32_t* part, bool* in_second, hipStream_t s) {
  *in_second = false;
  if (n <= 1 || bits <= 0) return P2P_OK;
  int g = (int)grid_for(n, kRsTile);
  uint64_t* ka = k0;
  int32_t* va = v0;
  uint64_t* kb = k1;
  int32_t* vb = v1;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(g), dim3(kBlock), 0, s, ka, n, shift, hist, g);
    p2p_status st = scan<uint32_t>(hist, hist, (int64_t)256 * g, part, nullptr, s);
    if (st != P2P_OK) return st;
    hipLaunchKernelGGL(k_rs_scatter, dim3(g), dim3(kBlock), 0, s, ka, va, kb, vb, n, shift, hist, g);
    P2P_HIP(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
    *in_second = !*in_second;
  }
  return P2P_OK;
}

// ---------------------------------------------------------------------------
// plan kernels
// ---------------------------------------------------------------------------
// 32-bit status words written by the device and read back by the host.  Minima
// are kept as maxima of (2^21 - 1 - v), so every word starts at zero.
enum {
  ST_BAD_ID = 0, ST_BAD_X, ST_ID_OR, ST_TMAX, ST_LO_X, ST_LO_Y, ST_LO_Z, ST_HI_X, ST_HI_Y, ST_HI_Z, ST_OVERLAP,
  ST_COUNT
};
// 64-bit scalars: pair slots, list entries, near-pair separation bound and the
// largest |coordinate| (the last two as the bits of non-negative doubles).
enum { S64_SLOTS = 0, S64_SRCSUM, S64_MAXSEP, S64_MAXABS, S64_COUNT };

constexpr uint32_t kIdMask = (1u << kIdBits) - 1;
constexpr int kGridStride = 2048;  // workgroups of the grid-stride kernels

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  for (int off = 32; off >= 1; off >>= 1) {
    T o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off, kWave);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_add(T v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Raises *p to at least v; reads first so that most callers skip the atomic.
__device__ __forceinline__ void raise_u32(uint32_t* p, uint32_t v) {
  if (v > __atomic_load_n(p, __ATOMIC_RELAXED)) atomicMax(p, v);
}
__device__ __forceinline__ void raise_u64(uint64_t* p, uint64_t v) {
  if (v > __atomic_load_n(p, __ATOMIC_RELAXED)) atomicMax((unsigned long long*)p, (unsigned long long)v);
}
__device__ __forceinline__ void or_u32(uint32_t* p, uint32_t v) {
  if ((v | __atomic_load_n(p, __ATOMIC_RELAXED)) != __atomic_load_n(p, __ATOMIC_RELAXED)) atomicOr(p, v);
}

// Morton keys, identity values, validation, and the bit width and range of the ids.
__global__ void __launch_bounds__(kBlock) k_keys(const double* __restrict__ xyz, const int32_t* __restrict__ ids,
                                              int64_t n, uint64_t* __restrict__ key, int32_t* __restrict__ idx,
                                              uint32_t* __restrict__ st) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t bad_id = 0, bad_x = 0, orv = 0, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  if (i < n) {
    const int32_t a = ids[3 * i], b = ids[3 * i + 1], c = ids[3 * i + 2];
    const uint32_t lim = 1u << kIdBits;
    bad_id = ((uint32_t)a >= lim) | ((uint32_t)b >= lim) | ((uint32_t)c >= lim);
    const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    bad_x = !(isfinite(x) && isfinite(y) && isfinite(z));
    const uint32_t u[3] = {(uint32_t)a & kIdMask, (uint32_t)b & kIdMask, (uint32_t)c & kIdMask};
    orv = u[0] | u[1] | u[2];
    for (int d = 0; d < 3; ++d) {
      lo[d] = kIdMask - u[d];
      hi[d] = u[d];
    }
    key[i] = morton3(u[0], u[1], u[2]);
    idx[i] = (int32_t)i;
  }
  bad_id = wave_or(bad_id);
  bad_x = wave_or(bad_x);
  orv = wave_or(orv);
  for (int d = 0; d < 3; ++d) {
    lo[d] = wave_max(lo[d]);
    hi[d] = wave_max(hi[d]);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (bad_id) atomicOr(&st[ST_BAD_ID], 1u);
    if (bad_x) atomicOr(&st[ST_BAD_X], 1u);
    or_u32(&st[ST_ID_OR], orv);
    for (int d = 0; d < 3; ++d) {
      raise_u32(&st[ST_LO_X + d], lo[d]);
      raise_u32(&st[ST_HI_X + d], hi[d]);
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_box_flags(const uint64_t* __restrict__ key, int64_t n,
                                                   int32_t* __restrict__ flag) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < n) flag[p] = (p == 0 || key[p] != key[p - 1]) ? 1 : 0;
}

// Dense cell table over the occupied id range plus a one-cell halo of empty
// cells, so that the 27 lookups of a box need no range checks.
struct CellGrid {
  int32_t* table;  // null: look boxes up by binary search instead
  int32_t x0, y0, z0;
  int64_t gx, gy;  // extents including the halo
  __device__ __forceinline__ int64_t cell(int32_t x, int32_t y, int32_t z) const {
    return ((int64_t)(z - z0 + 1) * gy + (y - y0 + 1)) * gx + (x - x0 + 1);
  }
};

// excl holds the exclusive scan of the run-start flags: the box of a run start p is excl[p].
__global__ void __launch_bounds__(kBlock) k_box_write(const uint64_t* __restrict__ key, int64_t n,
                                                   const int32_t* __restrict__ excl, const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ ids, uint64_t* __restrict__ box_key,
                                                   int32_t* __restrict__ box_start, const int32_t* __restrict__ nbox,
                                                   CellGrid grid) {
  int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  if (p == 0 || key[p] != key[p - 1]) {
    const int32_t b = excl[p];
    box_key[b] = key[p];
    box_start[b] = (int32_t)p;
    if (grid.table) {
      const int64_t i = perm[p];
      grid.table[grid.cell(ids[3 * i], ids[3 * i + 1], ids[3 * i + 2])] = b;
    }
  }
  if (p == n - 1) box_start[*nbox] = (int32_t)n;
}

// One wavefront per box (grid-stride): sorted FP64 coordinates (SoA), the box's
// bounding box, the largest occupancy and the largest |coordinate|.
__global__ void __launch_bounds__(kBlock) k_box_geom(const double* __restrict__ xyz, const int32_t* __restrict__ perm,
                                                  int64_t n, const int32_t* __restrict__ box_start,
                                                  const int32_t* __restrict__ nbox, double* __restrict__ sx,
                                                  double* __restrict__ bb, uint32_t* __restrict__ st,
                                                  uint64_t* __restrict__ s64) {
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t nb = *nbox;
  uint32_t tmax = 0;
  double amax = 0.0;
  for (int32_t T = blockIdx.x * kWavesPerBlockPlan + threadIdx.x / kWave; T < nb;
       T += gridDim.x * kWavesPerBlockPlan) {
    const int32_t p0 = box_start[T], p1 = box_start[T + 1];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t p = p0 + lane; p < p1; p += kWave) {
      const int64_t i = perm[p];
      for (int d = 0; d < 3; ++d) {
        const double v = xyz[3 * i + d];
        sx[d * n + p] = v;
        lo[d] = fmin(lo[d], v);
        hi[d] = fmax(hi[d], v);
      }
    }
    for (int d = 0; d < 3; ++d) {
      lo[d] = -wave_max(-lo[d]);
      hi[d] = wave_max(hi[d]);
      amax = fmax(amax, fmax(fabs(lo[d]), fabs(hi[d])));
    }
    if (lane == 0)
      for (int d = 0; d < 3; ++d) {
        bb[6 * (int64_t)T + d] = lo[d];
        bb[6 * (int64_t)T + 3 + d] = hi[d];
      }
    tmax = max(tmax, (uint32_t)(p1 - p0));
  }
  if (lane == 0) {
    raise_u32(&st[ST_TMAX], tmax);
    raise_u64(&s64[S64_MAXABS], (uint64_t)__double_as_longlong(amax));
  }
}

__device__ inline int32_t find_box(const uint64_t* __restrict__ box_key, int32_t nb, uint64_t k) {
  int32_t lo = 0, hi = nb;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (box_key[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return (lo < nb && box_key[lo] == k) ? lo : -1;
}

// Neighbour boxes of the box holding point i0 (itself included), ascending.
__device__ inline int neighbours(const uint64_t* __restrict__ box_key, int32_t nb, const CellGrid& grid,
                                 const int32_t* __restrict__ ids, int32_t i0, int32_t out[27]) {
  const int32_t bx = ids[3 * (int64_t)i0], by = ids[3 * (int64_t)i0 + 1], bz = ids[3 * (int64_t)i0 + 2];
  const int32_t lim = 1 << kIdBits;
  int cnt = 0;
  const int64_t c0 = grid.table ? grid.cell(bx, by, bz) : 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int32_t S;
        if (grid.table) {
          S = grid.table[c0 + ((int64_t)dz * grid.gy + dy) * grid.gx + dx];
        } else {
          const int32_t x = bx + dx, y = by + dy, z = bz + dz;
          if (x < 0 || y < 0 || z < 0 || x >= lim || y >= lim || z >= lim) continue;
          S = find_box(box_key, nb, morton3(x, y, z));
        }
        if (S >= 0) {
          int j = cnt++;
          while (j > 0 && out[j - 1] > S) {
            out[j] = out[j - 1];
            --j;
          }
          out[j] = S;
        }
      }
  return cnt;
}

// Per box (grid-stride): neighbour count, the neighbourhood's source count, the
// pair slots (targets x sources) and the largest per-axis coordinate difference
// to any neighbour, from the bounding boxes.
__global__ void __launch_bounds__(kBlock) k_nbr_count(const uint64_t* __restrict__ box_key,
                                                   const int32_t* __restrict__ box_start,
                                                   const int32_t* __restrict__ perm, const int32_t* __restrict__ ids,
                                                   const double* __restrict__ bb, const int32_t* __restrict__ nbox,
                                                   CellGrid grid, int32_t* __restrict__ cnt, int32_t* __restrict__ src,
                                                   uint64_t* __restrict__ s64, uint32_t* __restrict__ st) {
  const int32_t nb = *nbox;
  double msep = 0.0;
  uint32_t overlap = 0;
  uint64_t sl = 0, ss = 0;
  const int32_t stride = gridDim.x * kBlock;
  const int32_t first = blockIdx.x * kBlock + threadIdx.x;
  // every lane runs the same number of rounds so that the wave reductions see all lanes
  const int32_t rounds = (nb + stride - 1) / stride;
  for (int32_t r = 0; r < rounds; ++r) {
    const int32_t T = first + r * stride;
    if (T < nb) {
      int32_t nbr[27];
      const int c = neighbours(box_key, nb, grid, ids, perm[box_start[T]], nbr);
      int64_t ssum = 0;
      for (int e = 0; e < c; ++e) {
        const int32_t S = nbr[e];
        ssum += box_start[S + 1] - box_start[S];
        bool meet = S != T;
        for (int a = 0; a < 3; ++a) {
          const double up = bb[6 * (int64_t)S + 3 + a] - bb[6 * (int64_t)T + a];
          const double dn = bb[6 * (int64_t)T + 3 + a] - bb[6 * (int64_t)S + a];
          msep = fmax(msep, fmax(up, dn));
          meet = meet && up >= 0.0 && dn >= 0.0;
        }
        // two boxes whose bounding boxes intersect may hold coincident points
        overlap |= meet ? 1u : 0u;
      }
      cnt[T] = c;
      src[T] = (int32_t)(ssum < 0x7fffffff ? ssum : 0x7fffffff);
      ss += (uint64_t)ssum;
      sl += (uint64_t)ssum * (uint64_t)(box_start[T + 1] - box_start[T]);
    }
  }
  sl = wave_add(sl);
  ss = wave_add(ss);
  msep = wave_max(msep);
  overlap = wave_or(overlap);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (overlap) atomicOr(&st[ST_OVERLAP], 1u);
    if (sl) atomicAdd((unsigned long long*)&s64[S64_SLOTS], (unsigned long long)sl);
    if (ss) atomicAdd((unsigned long long*)&s64[S64_SRCSUM], (unsigned long long)ss);
    raise_u64(&s64[S64_MAXSEP], (uint64_t)__double_as_longlong(msep));
  }
}

__global__ void __launch_bounds__(kBlock) k_nbr_fill(const uint64_t* __restrict__ box_key,
                                                  const int32_t* __restrict__ box_start,
                                                  const int32_t* __restrict__ perm, const int32_t* __restrict__ ids,
                                                  const int32_t* __restrict__ nbr_start, int32_t nb, CellGrid grid,
                                                  int32_t* __restrict__ nbr_idx) {
  const int64_t T = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (T >= nb) return;
  int32_t nbr[27];
  const int c = neighbours(box_key, nb, grid, ids, perm[box_start[T]], nbr);
  const int32_t o = nbr_start[T];
  for (int e = 0; e < c; ++e) nbr_idx[o + e] = nbr[e];
}

// Fixed-point coordinates: X = rint(x * 2^-qexp), kept modulo 2^32.  Differences of
// two such values taken modulo 2^32 are exact whenever the true difference is
// below 2^31 in magnitude, which the choice of qexp guarantees for near pairs.
__global__ void __launch_bounds__(kBlock) k_fixed(const double* __restrict__ sx, int64_t n3, int qexp,
                                               int32_t* __restrict__ fx) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n3) return;
  const double v = rint(ldexp(sx[p], -qexp));
  fx[p] = (int32_t)(uint32_t)(uint64_t)(int64_t)v;
}

// Replicated source lists: one wavefront per target box copies the points of its
// neighbourhood into the box's contiguous list, its own points first.
template <bool F64>
__global__ void __launch_bounds__(kBlock) k_tile_fill(const int32_t* __restrict__ box_start,
                                                   const int32_t* __restrict__ nbr_start,
                                                   const int32_t* __restrict__ nbr_idx,
                                                   const int32_t* __restrict__ tile_start, int32_t nb, int64_t n,
                                                   int64_t tl, const double* __restrict__ sx64,
                                                   const int32_t* __restrict__ sx32, int32_t* __restrict__ tsrc,
                                                   double* __restrict__ t64, int32_t* __restrict__ t32) {
  const int32_t T = uniform((int32_t)(blockIdx.x * kWavesPerBlockPlan + threadIdx.x / kWave));
  if (T >= nb) return;
  const int lane = threadIdx.x & (kWave - 1);
  int64_t o = tile_start[T];
  // the box's own points first, then the other neighbours in list order
  for (int32_t e = nbr_start[T] - 1; e < nbr_start[T + 1]; ++e) {
    const int32_t S = e < nbr_start[T] ? T : nbr_idx[e];
    if (e >= nbr_start[T] && S == T) continue;
    const int32_t p0 = box_start[S], ns = box_start[S + 1] - p0;
    for (int32_t j = lane; j < ns; j += kWave) {
      const int64_t p = p0 + j, d = o + j;
      tsrc[d] = (int32_t)p;
      if (F64) {
        t64[d] = sx64[p];
        t64[tl + d] = sx64[n + p];
        t64[2 * tl + d] = sx64[2 * n + p];
      } else {
        t32[d] = sx32[p];
        t32[tl + d] = sx32[n + p];
        t32[2 * tl + d] = sx32[2 * n + p];
      }
    }
    o += ns;
  }
}

// Processing order of the sweep: boxes in decreasing order of their pair slots,
// bucketed on a log scale (8 buckets per octave), Morton order inside a bucket.
__global__ void __launch_bounds__(kBlock) k_cost_keys(const int32_t* __restrict__ box_start,
                                                   const int32_t* __restrict__ src, int32_t nb,
                                                   uint64_t* __restrict__ key, int32_t* __restrict__ idx) {
  const int64_t T = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (T >= nb) return;
  const double c = (double)(box_start[T + 1] - box_start[T]) * (double)src[T];
  const int b = (int)fmin(255.0, floor(log2(c + 1.0) * 8.0));
  key[T] = (uint64_t)(255 - b);
  idx[T] = (int32_t)T;
}

// Zero-distance pairs (self pairs included), FP64 coordinates.
__global__ void __launch_bounds__(kBlock) k_count_zero(const double* __restrict__ sx, int64_t n,
                                                    const int32_t* __restrict__ box_start,
                                                    const int32_t* __restrict__ nbr_start,
                                                    const int32_t* __restrict__ nbr_idx, int32_t nb,
                                                    unsigned long long* __restrict__ zero) {
  const int64_t T = (int64_t)blockIdx.x * kWavesPerBlockPlan + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long z = 0;
  if (T < nb) {
    for (int32_t t = box_start[T]; t < box_start[T + 1]; ++t) {
      const double x = sx[t], y = sx[n + t], w = sx[2 * n + t];
      for (int32_t e = nbr_start[T]; e < nbr_start[T + 1]; ++e) {
        const int32_t S = nbr_idx[e];
        for (int32_t p = box_start[S] + lane; p < box_start[S + 1]; p += kWave)
          z += (sx[p] == x && sx[n + p] == y && sx[2 * n + p] == w) ? 1 : 0;
      }
    }
  }
  z = wave_add(z);
  if (lane == 0 && z) atomicAdd(zero, z);
}

__global__ void __launch_bounds__(kBlock) k_box_ids(const double* __restrict__ xyz, int64_t n3, double ox, double oy,
                                                 double oz, double h, int32_t* __restrict__ ids,
                                                 uint32_t* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n3) return;
  const int a = (int)(e % 3);
  const double o = a == 0 ? ox : (a == 1 ? oy : oz);
  double v = floor((xyz[e] - o) / h);
  if (!(v >= 0.0 && v < (double)(1 << kIdBits))) {
    atomicOr(bad, 1u);
    v = 0.0;
  }
  ids[e] = (int32_t)v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

struct Bump {
  // Carves aligned sub-arrays out of one allocation.
  char* base;
  size_t off, cap;
  template <typename T>
  T* take(int64_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += sizeof(T) * (size_t)(count > 0 ? count : 0);
    return p;
  }
};

template <typename F>
size_t measure(F&& f) {
  Bump b{nullptr, 0, 0};
  f(b);
  return (b.off + 255) & ~size_t(255);
}

p2p_status dev_alloc(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (bytes == 0) return P2P_OK;
  hipError_t e = hipMallocAsync(p, bytes, s);
  if (e != hipSuccess || !*p) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(P2P_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return P2P_OK;
}

int bit_length(uint32_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

// Largest dense cell table, in cells: 32 bytes per point or 64 MB, whichever is larger.
int64_t table_cell_limit(int64_t n) { return std::max<int64_t>(16ll << 20, 8 * n); }

}  // namespace

p2p_status box_ids(const double* xyz, int64_t n, const double* origin, double h, int32_t* ids, hipStream_t s) {
  if (n == 0) return P2P_OK;
  uint32_t* bad = nullptr;
  p2p_status st = dev_alloc((void**)&bad, sizeof(uint32_t), s);
  if (st != P2P_OK) return st;
  P2P_HIP(hipMemsetAsync(bad, 0, sizeof(uint32_t), s));
  hipLaunchKernelGGL(k_box_ids, dim3(grid_for(3 * n)), dim3(kBlock), 0, s, xyz, 3 * n, origin[0], origin[1], origin[2],
                     h, ids, bad);
  uint32_t hb = 0;
  P2P_HIP(hipGetLastError());
  P2P_HIP(hipMemcpyAsync(&hb, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  P2P_HIP(hipFreeAsync(bad, s));
  P2P_HIP(hipStreamSynchronize(s));
  if (hb) return fail(P2P_ERR_RANGE, "a coordinate is not finite or its box id falls outside [0, 2^21)");
  return P2P_OK;
}

p2p_status build_plan(p2p_plan_s* P, const double* xyz, const int32_t* ids, hipStream_t s) {
  const int64_t n = P->n;
  const bool f64 = P->precision == P2P_C128;
  const bool tiles = P->layout == P2P_LAYOUT_TILES;
  const size_t cbytes = f64 ? 16 : 8;

  // ---- persistent arrays whose size depends on n only (first allocation)
  auto carve1 = [&](Bump& b) {
    P->perm = b.take<int32_t>(n);
    P->box_key = b.take<uint64_t>(n);
    P->box_start = b.take<int32_t>(n + 1);
    P->nbr_start = b.take<int32_t>(n + 1);
    P->tile_start = b.take<int32_t>(n + 1);
    P->work = b.take<int32_t>(n);
    P->sx64 = b.take<double>(3 * n);
    P->sx32 = f64 ? nullptr : b.take<int32_t>(3 * n);
    P->q_sorted = b.take<char>((int64_t)(n * (int64_t)P->max_rhs * cbytes));
    P->g_sorted = b.take<char>((int64_t)(n * (int64_t)P->max_rhs * cbytes));
  };
  size_t bytes1 = measure(carve1);
  p2p_status rc = dev_alloc(&P->arena, bytes1, s);
  if (rc != P2P_OK) return rc;
  P->device_bytes = bytes1;
  {
    Bump b{(char*)P->arena, 0, bytes1};
    carve1(b);
  }
  if (n == 0) {
    P2P_HIP(hipMemsetAsync(P->box_start, 0, sizeof(int32_t), s));
    P2P_HIP(hipMemsetAsync(P->nbr_start, 0, sizeof(int32_t), s));
    P2P_HIP(hipMemsetAsync(P->tile_start, 0, sizeof(int32_t), s));
    P->qexp = -30;
    P2P_HIP(hipStreamSynchronize(s));
    return P2P_OK;
  }

  // ---- temporaries, freed before returning
  const int64_t g_rs = grid_for(n, kRsTile);
  const int64_t scan_parts = grid_for(std::max<int64_t>(256 * g_rs, n + 1), kScanTile);
  uint64_t *k0, *k1, *s64;
  int32_t *v1, *flag, *cnt, *src, *part32, *tot;
  uint32_t *hist, *partu, *st;
  double* bb;
  auto carvet = [&](Bump& b) {
    k0 = b.take<uint64_t>(n);
    k1 = b.take<uint64_t>(n);
    v1 = b.take<int32_t>(n);
    flag = b.take<int32_t>(n + 1);
    cnt = b.take<int32_t>(n + 1);
    src = b.take<int32_t>(n + 1);
    hist = b.take<uint32_t>(256 * g_rs);
    partu = b.take<uint32_t>(scan_parts);
    part32 = b.take<int32_t>(scan_parts);
    bb = b.take<double>(6 * n);
    st = b.take<uint32_t>(ST_COUNT);
    s64 = b.take<uint64_t>(S64_COUNT);
    tot = b.take<int32_t>(2);
  };
  size_t bytest = measure(carvet);
  void* tmp = nullptr;
  rc = dev_alloc(&tmp, bytest, s);
  if (rc != P2P_OK) return rc;
  struct TmpGuard {
    void* p;
    hipStream_t s;
    ~TmpGuard() {
      if (p) (void)hipFreeAsync(p, s);
    }
  } guard{tmp, s}, guard_table{nullptr, s};
  {
    Bump b{(char*)tmp, 0, bytest};
    carvet(b);
  }
  P2P_HIP(hipMemsetAsync(st, 0, sizeof(uint32_t) * ST_COUNT, s));
  P2P_HIP(hipMemsetAsync(s64, 0, sizeof(uint64_t) * S64_COUNT, s));
  P2P_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (n + 1), s));
  P2P_HIP(hipMemsetAsync(src, 0, sizeof(int32_t) * (n + 1), s));

  // ---- 1. Morton keys and validation (first readback)
  hipLaunchKernelGGL(k_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, xyz, ids, n, k0, P->perm, st);
  P2P_HIP(hipGetLastError());
  uint32_t hst[ST_COUNT];
  P2P_HIP(hipMemcpyAsync(hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
  P2P_HIP(hipStreamSynchronize(s));
  if (hst[ST_BAD_ID]) return fail(P2P_ERR_RANGE, "a box id falls outside [0, 2^21)");
  if (hst[ST_BAD_X]) return fail(P2P_ERR_RANGE, "a coordinate is not finite");

  // dense cell table when the occupied id range is small enough
  CellGrid grid{nullptr, 0, 0, 0, 0, 0};
  {
    const int32_t lo[3] = {(int32_t)(kIdMask - hst[ST_LO_X]), (int32_t)(kIdMask - hst[ST_LO_Y]),
                           (int32_t)(kIdMask - hst[ST_LO_Z])};
    const int64_t ext[3] = {(int64_t)hst[ST_HI_X] - lo[0] + 3, (int64_t)hst[ST_HI_Y] - lo[1] + 3,
                            (int64_t)hst[ST_HI_Z] - lo[2] + 3};
    const double cells = (double)ext[0] * (double)ext[1] * (double)ext[2];
    if (cells <= (double)table_cell_limit(n)) {
      void* tp = nullptr;
      rc = dev_alloc(&tp, sizeof(int32_t) * (size_t)cells, s);
      if (rc == P2P_OK) {
        guard_table.p = tp;
        P2P_HIP(hipMemsetAsync(tp, 0xff, sizeof(int32_t) * (size_t)cells, s));  // -1: no box
        grid = CellGrid{(int32_t*)tp, lo[0], lo[1], lo[2], ext[0], ext[1]};
      } else {
        set_error("");  // no room for the table: fall back to binary search
      }
    }
  }

  // ---- 2. stable sort of the points by key, over the key bits in use
  const int bits = 3 * bit_length(hst[ST_ID_OR]);
  bool second = false;
  rc = radix_sort(k0, P->perm, k1, v1, n, bits, hist, partu, &second, s);
  if (rc != P2P_OK) return rc;
  const uint64_t* skey = second ? k1 : k0;
  if (second) P2P_HIP(hipMemcpyAsync(P->perm, v1, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));

  // ---- 3. box table: runs of equal keys
  int32_t* dnb = flag + n;  // scan total = number of boxes
  hipLaunchKernelGGL(k_box_flags, dim3(grid_for(n)), dim3(kBlock), 0, s, skey, n, flag);
  rc = scan<int32_t>(flag, flag, n, part32, dnb, s);
  if (rc != P2P_OK) return rc;
  hipLaunchKernelGGL(k_box_write, dim3(grid_for(n)), dim3(kBlock), 0, s, skey, n, flag, P->perm, ids, P->box_key,
                     P->box_start, dnb, grid);
  const unsigned gs = (unsigned)std::min<int64_t>(kGridStride, grid_for(n, kWavesPerBlockPlan));
  hipLaunchKernelGGL(k_box_geom, dim3(gs), dim3(kBlock), 0, s, xyz, P->perm, n, P->box_start, dnb, P->sx64, bb, st,
                     s64);

  // ---- 4. neighbour counts, neighbourhood source counts, separation bound.
  //         Entries past the last box stay zero, so scanning n entries gives the
  //         offsets of the B boxes and, at index B, the totals.
  const unsigned gt = (unsigned)std::min<int64_t>(kGridStride, grid_for(n));
  hipLaunchKernelGGL(k_nbr_count, dim3(gt), dim3(kBlock), 0, s, P->box_key, P->box_start, P->perm, ids, bb, dnb, grid,
                     cnt, src, s64, st);
  P2P_HIP(hipGetLastError());
  rc = scan<int32_t>(cnt, P->nbr_start, n + 1, part32, tot, s);  // tot[0] = list entries
  if (rc != P2P_OK) return rc;
  rc = scan<int32_t>(src, P->tile_start, n + 1, part32, nullptr, s);
  if (rc != P2P_OK) return rc;

  // second readback: sizes of the lists and the geometry bounds
  int32_t hB = 0, hnnz = 0;
  uint64_t h64[S64_COUNT];
  P2P_HIP(hipMemcpyAsync(&hB, dnb, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  P2P_HIP(hipMemcpyAsync(&hnnz, tot, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  P2P_HIP(hipMemcpyAsync(h64, s64, sizeof(h64), hipMemcpyDeviceToHost, s));
  P2P_HIP(hipMemcpyAsync(hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
  P2P_HIP(hipStreamSynchronize(s));
  const int32_t B = hB;
  P->B = B;
  P->nnz = hnnz;
  P->n_slots = (int64_t)h64[S64_SLOTS];
  P->t_max = (int32_t)hst[ST_TMAX];
  P->may_coincide = hst[ST_OVERLAP] != 0;
  const int64_t srclen = (int64_t)h64[S64_SRCSUM];
  double sep, xabs;
  std::memcpy(&sep, &h64[S64_MAXSEP], sizeof(double));
  std::memcpy(&xabs, &h64[S64_MAXABS], sizeof(double));
  P->max_sep = sep;
  if (srclen > 0x7fffffffll) return fail(P2P_ERR_RANGE, "the per-box source lists exceed 2^31 entries");
  P->tile_len = tiles ? srclen : 0;
  P->max_turns = P->k * std::sqrt(3.0) * sep / (2.0 * M_PI);

  // ---- 5. quantum of the FP32 coordinates: 2^qexp with sep < 2^(qexp + 30), so a
  //         near-pair difference plus one quantum of rounding stays below 2^31.
  if (sep > 0) {
    int e = 0;
    std::frexp(sep, &e);  // sep < 2^e
    P->qexp = e - 30;
  } else {
    P->qexp = -30;
  }
  if (!f64 && xabs > std::ldexp(1.0, P->qexp + 62))
    return fail(P2P_ERR_RANGE, "coordinates are too far from the origin for the FP32 fixed-point grid");

  // ---- 6. second allocation: neighbour lists and replicated source lists
  auto carve2 = [&](Bump& b) {
    P->nbr_idx = b.take<int32_t>(P->nnz);
    P->tile_src = tiles ? b.take<int32_t>(P->tile_len) : nullptr;
    P->tile_x64 = (tiles && f64) ? b.take<double>(3 * P->tile_len) : nullptr;
    P->tile_x32 = (tiles && !f64) ? b.take<int32_t>(3 * P->tile_len) : nullptr;
  };
  size_t bytes2 = measure(carve2);
  rc = dev_alloc(&P->arena2, bytes2, s);
  if (rc != P2P_OK) return rc;
  P->device_bytes += bytes2;
  {
    Bump b{(char*)P->arena2, 0, bytes2};
    carve2(b);
  }
  hipLaunchKernelGGL(k_nbr_fill, dim3(grid_for(B)), dim3(kBlock), 0, s, P->box_key, P->box_start, P->perm, ids,
                     P->nbr_start, B, grid, P->nbr_idx);
  if (!f64) hipLaunchKernelGGL(k_fixed, dim3(grid_for(3 * n)), dim3(kBlock), 0, s, P->sx64, 3 * n, P->qexp, P->sx32);
  if (tiles) {
    const unsigned g = grid_for(B, kWavesPerBlockPlan);
    if (f64)
      hipLaunchKernelGGL(k_tile_fill<true>, dim3(g), dim3(kBlock), 0, s, P->box_start, P->nbr_start, P->nbr_idx,
                         P->tile_start, B, n, P->tile_len, P->sx64, P->sx32, P->tile_src, P->tile_x64, P->tile_x32);
    else
      hipLaunchKernelGGL(k_tile_fill<false>, dim3(g), dim3(kBlock), 0, s, P->box_start, P->nbr_start, P->nbr_idx,
                         P->tile_start, B, n, P->tile_len, P->sx64, P->sx32, P->tile_src, P->tile_x64, P->tile_x32);
  }
  // processing order: most pair slots first (one 8-bit radix pass, stable)
  hipLaunchKernelGGL(k_cost_keys, dim3(grid_for(B)), dim3(kBlock), 0, s, P->box_start, src, B, k0, P->work);
  P2P_HIP(hipGetLastError());
  rc = radix_sort(k0, P->work, k1, v1, B, 8, hist, partu, &second, s);
  if (rc != P2P_OK) return rc;
  if (second) P2P_HIP(hipMemcpyAsync(P->work, v1, sizeof(int32_t) * B, hipMemcpyDeviceToDevice, s));
  P2P_HIP(hipGetLastError());
  P2P_HIP(hipStreamSynchronize(s));
  return P2P_OK;
}

p2p_status count_pairs(p2p_plan_s* P, hipStream_t s) {
  if (P->n_pairs >= 0) return P2P_OK;
  unsigned long long* z = nullptr;
  p2p_status rc = dev_alloc((void**)&z, sizeof(unsigned long long), s);
  if (rc != P2P_OK) return rc;
  P2P_HIP(hipMemsetAsync(z, 0, sizeof(unsigned long long), s));
  if (P->B > 0)
    hipLaunchKernelGGL(k_count_zero, dim3(grid_for(P->B, kWavesPerBlockPlan)), dim3(kBlock), 0, s, P->sx64, P->n,
                       P->box_start, P->nbr_start, P->nbr_idx, (int32_t)P->B, z);
  unsigned long long hz = 0;
  P2P_HIP(hipGetLastError());
  P2P_HIP(hipMemcpyAsync(&hz, z, sizeof(hz), hipMemcpyDeviceToHost, s));
  P2P_HIP(hipFreeAsync(z, s));
  P2P_HIP(hipStreamSynchronize(s));
  P->n_zero = (int64_t)hz;
  P->n_pairs = P->n_slots - P->n_zero;
  return P2P_OK;
}

}  // namespace p2p
