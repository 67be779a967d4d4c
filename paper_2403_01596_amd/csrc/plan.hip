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
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"
#include "sweep.h"

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

// lim (optional, device): only the first *lim + 1 entries are live; the rest are
// zero and need not be read or written.
__device__ __forceinline__ int64_t live(int64_t n, const int32_t* lim) {
  return lim ? min(n, (int64_t)*lim + 1) : n;
}

// One or two arrays of the same length scanned by the same launches; array y is
// handled by the workgroups with blockIdx.y == y.
template <typename T>
struct ScanIO {
  const T* in[2];
  T* out[2];
  T* part[2];   // workspace: one entry per tile
  T* total[2];  // sum of the array (device), or null
};

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_reduce(ScanIO<T> io, int64_t n, const int32_t* __restrict__ lim) {
  __shared__ T lds[kBlock / kWave];
  const int y = blockIdx.y;
  const T* __restrict__ in = io.in[y];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  n = live(n, lim);
  if (base >= n) {
    if (threadIdx.x == 0) io.part[y][blockIdx.x] = T(0);
    return;
  }
  T s = 0;
  for (int r = 0; r < kScanItems; ++r) {
    int64_t e = base + (int64_t)r * kBlock + threadIdx.x;
    if (e < n) s += in[e];
  }
  T tot;
  block_exclusive_scan<T>(s, lds, &tot);
  if (threadIdx.x == 0) io.part[y][blockIdx.x] = tot;
}

// One workgroup per array: the exclusive prefix sums of its g partial sums, each
// thread taking kScanItems consecutive ones per round (a round's loads all in
// flight at once; up to kScanTile partials, 2^22 scanned elements, take one round).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_partials(ScanIO<T> io, int64_t g) {
  __shared__ T lds[kBlock / kWave];
  const int y = blockIdx.y;
  T* __restrict__ part = io.part[y];
  T carry = 0;
  for (int64_t c = 0; c < g; c += kScanTile) {
    const int64_t base = c + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems], sum = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
      v[r] = base + r < g ? part[base + r] : T(0);
      sum += v[r];
    }
    T tot;
    T ex = block_exclusive_scan<T>(sum, lds, &tot) + carry;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
      if (base + r < g) part[base + r] = ex;
      ex += v[r];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && io.total[y]) *io.total[y] = carry;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_apply(ScanIO<T> io, int64_t n, const int32_t* __restrict__ lim) {
  // each thread owns kScanItems consecutive elements of the tile
  __shared__ T lds[kBlock / kWave];
  const int y = blockIdx.y;
  const T* in = io.in[y];
  T* out = io.out[y];
  n = live(n, lim);
  if ((int64_t)blockIdx.x * kScanTile >= n) return;
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
  for (int r = 0; r < kScanItems; ++r) {
    int64_t e = base + r;
    v[r] = e < n ? in[e] : T(0);
    s += v[r];
  }
  T tot;
  T ex = block_exclusive_scan<T>(s, lds, &tot) + io.part[y][blockIdx.x];
  for (int r = 0; r < kScanItems; ++r) {
    int64_t e = base + r;
    if (e < n) out[e] = ex;
    ex += v[r];
  }
}

template <typename T>
__global__ void k_zero_one(T* p) {
  if (threadIdx.x == 0) *p = T(0);
}

// Exclusive prefix sums of io's first `arrays` arrays, each n long (in == out
// allowed); totals where io.total is set.  lim: see live().
template <typename T>
static p2p_status scan_arrays(const ScanIO<T>& io, int arrays, int64_t n, hipStream_t s,
                              const int32_t* lim = nullptr) {
  if (n <= 0) {
    for (int y = 0; y < arrays; ++y)
      if (io.total[y]) hipLaunchKernelGGL(k_zero_one<T>, dim3(1), dim3(kWave), 0, s, io.total[y]);
    P2P_HIP(hipGetLastError());
    return P2P_OK;
  }
  const unsigned g = grid_for(n, kScanTile);
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(g, arrays), dim3(kBlock), 0, s, io, n, lim);
  hipLaunchKernelGGL(k_scan_partials<T>, dim3(1, arrays), dim3(kBlock), 0, s, io, (int64_t)g);
  hipLaunchKernelGGL(k_scan_apply<T>, dim3(g, arrays), dim3(kBlock), 0, s, io, n, lim);
  P2P_HIP(hipGetLastError());
  return P2P_OK;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, i32 value), 8 bits per pass.  Per pass: digit
// counts per tile, a scan of each digit's row of tile counts (one workgroup per
// digit, which also writes the digit's total), then the scatter, which turns
// the 256 totals into the digits' start slots itself.  Keys are
// narrowed to 32 bits by the first pass when the key bits in use allow it, and
// the first pass makes the identity values itself.
// ---------------------------------------------------------------------------
constexpr int kRsItems = 16;
constexpr int kRsTile = kBlock * kRsItems;
constexpr int kRsWaveItems = kRsItems * kWave;  // keys of one wavefront's part of a tile

template <typename KI>
__global__ void __launch_bounds__(kBlock) k_rs_hist(const KI* __restrict__ key, int64_t n,
                                                 const int32_t* __restrict__ lim, int shift,
                                                 uint32_t* __restrict__ hist, int g) {
  __shared__ uint32_t h[256];
  if (lim) n = min(n, (int64_t)*lim);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  KI k[kRsItems];
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {  // every load in flight before the first count
    const int64_t e = base + (int64_t)r * kBlock + threadIdx.x;
    k[r] = e < n ? key[e] : KI(0);
  }
#pragma unroll
  for (int r = 0; r < kRsItems; ++r)
    if (base + (int64_t)r * kBlock + threadIdx.x < n) atomicAdd(&h[(uint32_t)(k[r] >> shift) & 255u], 1u);
  __syncthreads();
  hist[(int64_t)threadIdx.x * g + blockIdx.x] = h[threadIdx.x];
}

// hist is [digit][tile]; row d (workgroup d) becomes its exclusive prefix sums,
// each thread scanning kScanItems consecutive tiles; total[d] gets the row's sum.
__global__ void __launch_bounds__(kBlock) k_rs_rows(uint32_t* __restrict__ hist, int g, uint32_t* __restrict__ total) {
  __shared__ uint32_t lds[kBlock / kWave];
  uint32_t* __restrict__ row = hist + (int64_t)blockIdx.x * g;
  uint32_t carry = 0;
  for (int c = 0; c < g; c += kScanTile) {
    const int base = c + threadIdx.x * kScanItems;
    uint32_t v[kScanItems], sum = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
      v[r] = base + r < g ? row[base + r] : 0u;
      sum += v[r];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<uint32_t>(sum, lds, &tot) + carry;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
      if (base + r < g) row[base + r] = ex;
      ex += v[r];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) total[blockIdx.x] = carry;
}

// Scatter one tile.  Wavefront w ranks the w-th quarter of the tile on its own, in
// input order: the rank of a key among equal digits is the count of that digit in
// the wavefront's earlier rounds (an LDS counter per digit) plus the lanes below
// it with the same digit (wave ballots).  The quarters are stacked in order under
// each digit's start, so equal digits keep their input order (stability).  The
// tile is first laid out sorted in LDS and then written with consecutive threads
// on consecutive slots, so each digit's run goes out as whole lines rather than
// one scattered element per lane.  vin null: the values are the input positions.
template <typename KI, typename KO>
__global__ void __launch_bounds__(kBlock) k_rs_scatter(const KI* __restrict__ kin, const int32_t* __restrict__ vin,
                                                    KO* __restrict__ kout, int32_t* __restrict__ vout, int64_t n,
                                                    const int32_t* __restrict__ lim, int shift,
                                                    const uint32_t* __restrict__ offs,
                                                    const uint32_t* __restrict__ dtotal, int g) {
  __shared__ uint32_t cnt[kBlock / kWave][256];
  __shared__ uint64_t lds[kBlock / kWave];
  __shared__ uint32_t delta[256];
  __shared__ KO sk[kRsTile];
  __shared__ int32_t sv[kRsTile];
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid & (kWave - 1);
  if (lim) n = min(n, (int64_t)*lim);
  for (int d = lane; d < 256; d += kWave) cnt[wave][d] = 0;
  // thread tid: digit tid's count over all tiles, and this tile's start within it
  const uint32_t dtot = dtotal[tid];
  const uint32_t doff = offs[(int64_t)tid * g + blockIdx.x];
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile0 = (int64_t)blockIdx.x * kRsTile;
  const int64_t base = tile0 + (int64_t)wave * kRsWaveItems;
  // every load of the wavefront's quarter in flight before the ranking
  KI k[kRsItems];
  int32_t v[kRsItems];
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    const int64_t e = base + (int64_t)r * kWave + lane;
    k[r] = e < n ? kin[e] : KI(0);
    v[r] = e < n ? (vin ? vin[e] : (int32_t)e) : 0;
  }
  // LDS accesses of one wavefront take effect in program order, so a round's
  // counter reads see the previous round's writes without a barrier
  uint32_t pos[kRsItems];
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    const int64_t e = base + (int64_t)r * kWave + lane;
    const bool valid = e < n;
    const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = __popcll(peers & below);
    const uint32_t before = cnt[wave][d];
    pos[r] = before + rank;
    if (valid && rank == 0) cnt[wave][d] = before + __popcll(peers);
  }
  __syncthreads();
  // thread tid, digit tid: its count in each quarter; one scan gives both the
  // digit's start among all keys (high half) and within the tile (low half)
  uint32_t c[kBlock / kWave], tcount = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    c[w] = cnt[w][tid];
    tcount += c[w];
  }
  uint64_t all;
  const uint64_t both = block_exclusive_scan<uint64_t>(((uint64_t)dtot << 32) | tcount, lds, &all);
  const uint32_t lstart = (uint32_t)both;
  delta[tid] = (uint32_t)(both >> 32) + doff - lstart;
  uint32_t run = lstart;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    cnt[w][tid] = run;  // the quarter's first slot of this digit within the tile
    run += c[w];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    if (base + (int64_t)r * kWave + lane < n) {
      const uint32_t at = cnt[wave][(uint32_t)(k[r] >> shift) & 255u] + pos[r];
      sk[at] = (KO)k[r];
      sv[at] = v[r];
    }
  }
  __syncthreads();
  const int live = (int)min<int64_t>(kRsTile, n - tile0);
#pragma unroll
  for (int r = 0; r < kRsItems; ++r) {
    const int i = r * kBlock + tid;
    if (i < live) {
      const KO kk = sk[i];
      const uint32_t at = delta[(uint32_t)(kk >> shift) & 255u] + (uint32_t)i;
      kout[at] = kk;
      vout[at] = sv[i];
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_iota(int32_t* __restrict__ v, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) v[e] = (int32_t)e;
}

// One pass of the sort over the digit at `shift`: keys kin -> kout, values vin
// (null: the input positions) -> vout.  lim as for radix_sort below.
template <typename KI, typename KO>
static p2p_status radix_pass(const KI* kin, const int32_t* vin, KO* kout, int32_t* vout, int64_t n, int shift,
                             uint32_t* hist, uint32_t* part, hipStream_t s, const int32_t* lim = nullptr) {
  const int g = (int)grid_for(n, kRsTile);
  hipLaunchKernelGGL(k_rs_hist<KI>, dim3(g), dim3(kBlock), 0, s, kin, n, lim, shift, hist, g);
  hipLaunchKernelGGL(k_rs_rows, dim3(256), dim3(kBlock), 0, s, hist, g, part);
  hipLaunchKernelGGL((k_rs_scatter<KI, KO>), dim3(g), dim3(kBlock), 0, s, kin, vin, kout, vout, n, lim, shift, hist,
                     part, g);
  P2P_HIP(hipGetLastError());
  return P2P_OK;
}

// Sorts the keys k0[0..n) by their low `bits` bits; the stable order of the
// positions lands in vals.  Workspace: kx (n u64), vx (n i32), hist (256 per tile
// of kRsTile keys), part (256 digit totals).  lim (optional, device): the count of
// keys actually sorted is min(n, *lim); n sizes the launches.  Returns in *sorted
// the sorted keys: 32-bit (in kx's storage) when bits <= 32, else 64-bit (k0 or kx).
struct SortedKeys {
  const uint32_t* k32;
  const uint64_t* k64;
};

static p2p_status radix_sort(uint64_t* k0, int32_t* vals, uint64_t* kx, int32_t* vx, int64_t n, int bits,
                             uint32_t* hist, uint32_t* part, SortedKeys* sorted, hipStream_t s,
                             const int32_t* lim = nullptr) {
  const int passes = bits <= 0 ? 0 : (bits + 7) / 8;
  const bool narrow = bits <= 32;
  sorted->k32 = nullptr;
  sorted->k64 = k0;
  if (n <= 0) return P2P_OK;
  const int g = (int)grid_for(n, kRsTile);
  if (passes == 0) {  // every key equal: the identity order
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(kBlock), 0, s, vals, n);
    P2P_HIP(hipGetLastError());
    return P2P_OK;
  }
  uint32_t* a32 = reinterpret_cast<uint32_t*>(kx);
  uint32_t* b32 = a32 + n;
  const uint64_t* cur64 = k0;
  const uint32_t* cur32 = nullptr;
  const int32_t* vcur = nullptr;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    // the last pass writes vals, the ones before alternate backwards from it
    int32_t* vout = ((passes - 1 - p) % 2 == 0) ? vals : vx;
    if (cur32)
      hipLaunchKernelGGL(k_rs_hist<uint32_t>, dim3(g), dim3(kBlock), 0, s, cur32, n, lim, shift, hist, g);
    else
      hipLaunchKernelGGL(k_rs_hist<uint64_t>, dim3(g), dim3(kBlock), 0, s, cur64, n, lim, shift, hist, g);
    hipLaunchKernelGGL(k_rs_rows, dim3(256), dim3(kBlock), 0, s, hist, g, part);
    if (narrow) {
      uint32_t* kout = (p % 2 == 0) ? a32 : b32;
      if (cur32)
        hipLaunchKernelGGL((k_rs_scatter<uint32_t, uint32_t>), dim3(g), dim3(kBlock), 0, s, cur32, vcur, kout, vout, n,
                           lim, shift, hist, part, g);
      else
        hipLaunchKernelGGL((k_rs_scatter<uint64_t, uint32_t>), dim3(g), dim3(kBlock), 0, s, cur64, vcur, kout, vout, n,
                           lim, shift, hist, part, g);
      cur32 = kout;
    } else {
      uint64_t* kout = (p % 2 == 0) ? kx : k0;
      hipLaunchKernelGGL((k_rs_scatter<uint64_t, uint64_t>), dim3(g), dim3(kBlock), 0, s, cur64, vcur, kout, vout, n,
                         lim, shift, hist, part, g);
      cur64 = kout;
    }
    P2P_HIP(hipGetLastError());
    vcur = vout;
  }
  sorted->k32 = cur32;
  sorted->k64 = cur32 ? nullptr : cur64;
  return P2P_OK;
}

// ---------------------------------------------------------------------------
// plan kernels
// ---------------------------------------------------------------------------
// Status block written by the device and read back by the host in one copy.
// Minima of the ids are kept as maxima of (2^21 - 1 - v), so everything starts
// at zero.
enum {
  ST_BAD_ID = 0, ST_BAD_X, ST_ID_OR, ST_TMAX, ST_LO_X, ST_LO_Y, ST_LO_Z, ST_HI_X, ST_HI_Y, ST_HI_Z, ST_OVERLAP,
  ST_COUNT
};
struct DevStatus {
  uint32_t st[16];
  int32_t nbox;        // boxes (scan total of the run starts)
  int32_t nnz;         // neighbour-list entries (scan total)
  uint64_t slots;      // sum over boxes of targets x neighbourhood sources
  uint64_t srcsum;     // sum over boxes of neighbourhood sources (list length)
  uint64_t maxsep;     // bits of the largest per-axis near-pair difference (>= 0)
  uint64_t maxabs;     // bits of the largest |coordinate|
  uint64_t zero;       // zero-distance pairs (statistics only)
  uint64_t ncp;        // FP32 plans: close pairs (statistics only)
  uint64_t nnear;      // FP32 plans: boxes marked near (statistics only)
};

constexpr uint32_t kIdMask = (1u << kIdBits) - 1;
constexpr int kGridStride = 2048;  // workgroups of the grid-stride kernels

// Per-workgroup partial results of the reductions over points and boxes.  Each
// workgroup of a grid-stride kernel writes its own row (no atomics: on a chip of
// eight dies, same-address atomics from thousands of wavefronts serialise); one
// small kernel folds the rows into the status block before each readback.
struct Partial {
  uint32_t bad;     // bit 0: id out of range, bit 1: coordinate not finite
  uint32_t id_or;
  uint32_t lo[3];   // kIdMask - smallest id per axis
  uint32_t hi[3];   // largest id per axis
  uint32_t tmax;
  uint32_t overlap;
  uint64_t slots, srcsum;
  double maxsep, maxabs;
};

__device__ __forceinline__ void fold_into(Partial& a, const Partial& p) {
  a.bad |= p.bad;
  a.id_or |= p.id_or;
  for (int d = 0; d < 3; ++d) {
    a.lo[d] = max(a.lo[d], p.lo[d]);
    a.hi[d] = max(a.hi[d], p.hi[d]);
  }
  a.tmax = max(a.tmax, p.tmax);
  a.overlap |= p.overlap;
  a.slots += p.slots;
  a.srcsum += p.srcsum;
  a.maxsep = fmax(a.maxsep, p.maxsep);
  a.maxabs = fmax(a.maxabs, p.maxabs);
}

// One workgroup folds the kGridStride partial rows: every thread kFoldRows of them,
// all loaded before the first fold (one after another, each load's latency had
// been the kernel's time), then a tree over the threads.
constexpr int kFoldRows = kGridStride / kBlock;
static_assert(kFoldRows * kBlock == kGridStride, "partial rows must fill the fold's threads");
__global__ void __launch_bounds__(kBlock) k_fold(const Partial* __restrict__ part, DevStatus* __restrict__ status) {
  __shared__ Partial acc[kBlock];
  Partial b[kFoldRows];
#pragma unroll
  for (int i = 0; i < kFoldRows; ++i) b[i] = part[i * kBlock + threadIdx.x];
  Partial a = b[0];
#pragma unroll
  for (int i = 1; i < kFoldRows; ++i) fold_into(a, b[i]);
  acc[threadIdx.x] = a;
  __syncthreads();
  for (int half = kBlock / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half) fold_into(acc[threadIdx.x], acc[threadIdx.x + half]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const Partial& t = acc[0];
    status->st[ST_BAD_ID] = t.bad & 1u;
    status->st[ST_BAD_X] = (t.bad >> 1) & 1u;
    status->st[ST_ID_OR] = t.id_or;
    for (int d = 0; d < 3; ++d) {
      status->st[ST_LO_X + d] = t.lo[d];
      status->st[ST_HI_X + d] = t.hi[d];
    }
    status->st[ST_TMAX] = t.tmax;
    status->st[ST_OVERLAP] = t.overlap;
    status->slots = t.slots;
    status->srcsum = t.srcsum;
    status->maxsep = (uint64_t)__double_as_longlong(t.maxsep);
    status->maxabs = (uint64_t)__double_as_longlong(t.maxabs);
  }
}

// Lane 63 of every wavefront holds its wavefront's value; the first wavefront of
// the workgroup combines the four through LDS.
template <typename T, typename F>
__device__ __forceinline__ T block_combine63(T v, T* lds, F op) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  if (lane == kWave - 1) lds[wv] = v;
  __syncthreads();
  T r = lds[0];
  for (int w = 1; w < kWavesPerBlockPlan; ++w) r = op(r, lds[w]);
  __syncthreads();
  return r;
}

// Zeroes `words` 32-bit words at `zero` (status block and partial rows) and two
// counter arrays of n1 entries, and marks every cell of the dense table empty (-1).
__global__ void __launch_bounds__(kBlock) k_init(uint32_t* __restrict__ zero, int64_t words, int32_t* __restrict__ cnt,
                                              int32_t* __restrict__ src, int64_t n1, int32_t* __restrict__ table,
                                              int64_t cells) {
  const int64_t end = max(max(n1, cells), words);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < end; i += stride) {
    if (i < n1) {
      cnt[i] = 0;
      src[i] = 0;
    }
    if (i < cells) table[i] = -1;
    if (i < words) zero[i] = 0;
  }
}

// Morton keys, validation of the ids, and their bit width and range (grid-stride;
// one partial row per workgroup).  The coordinates are checked later, where the
// geometry pass reads them.
// Leaf-box id of one coordinate: floor((x - o) / h) in FP64 (correctly rounded
// subtraction and division), -1 when it is not an id (out of range or not finite).
__device__ __forceinline__ int32_t grid_id(double x, double o, double h) {
  const double v = floor((x - o) / h);
  return (v >= 0.0 && v < (double)(1 << kIdBits)) ? (int32_t)v : -1;
}

// GRID: the ids are computed from the positions, the origin and the box size
// (ids unused); else read from ids.
template <bool GRID>
__global__ void __launch_bounds__(kBlock) k_keys(const int32_t* __restrict__ ids, const double* __restrict__ xyz,
                                              GridSpec gs, int64_t n, uint64_t* __restrict__ key,
                                              Partial* __restrict__ part) {
  __shared__ uint32_t lds[kWavesPerBlockPlan];
  uint32_t bad = 0, orv = 0, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  const uint32_t lim = 1u << kIdBits;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    int32_t a, b, c;
    if (GRID) {
      a = grid_id(xyz[3 * i], gs.o[0], gs.h);
      b = grid_id(xyz[3 * i + 1], gs.o[1], gs.h);
      c = grid_id(xyz[3 * i + 2], gs.o[2], gs.h);
    } else {
      a = ids[3 * i];
      b = ids[3 * i + 1];
      c = ids[3 * i + 2];
    }
    const bool bad_id = ((uint32_t)a >= lim) | ((uint32_t)b >= lim) | ((uint32_t)c >= lim);
    bad |= bad_id ? 1u : 0u;
    const uint32_t u[3] = {(uint32_t)a & kIdMask, (uint32_t)b & kIdMask, (uint32_t)c & kIdMask};
    orv |= u[0] | u[1] | u[2];
    for (int d = 0; d < 3; ++d) {
      lo[d] = max(lo[d], kIdMask - u[d]);
      hi[d] = max(hi[d], u[d]);
    }
    key[i] = morton3(u[0], u[1], u[2]);
  }
  auto vor = [](uint32_t x, uint32_t y) { return x | y; };
  auto vmax = [](uint32_t x, uint32_t y) { return x > y ? x : y; };
  bad = block_combine63(wave_or63(bad), lds, vor);
  orv = block_combine63(wave_or63(orv), lds, vor);
  for (int d = 0; d < 3; ++d) {
    lo[d] = block_combine63(wave_max63(lo[d]), lds, vmax);
    hi[d] = block_combine63(wave_max63(hi[d]), lds, vmax);
  }
  if (threadIdx.x == 0) {
    Partial& p = part[blockIdx.x];
    p.bad = bad;
    p.id_or = orv;
    for (int d = 0; d < 3; ++d) {
      p.lo[d] = lo[d];
      p.hi[d] = hi[d];
    }
  }
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

// Box table from the sorted keys, over tiles of kScanTile keys (each thread owns
// kScanItems consecutive ones): a run of equal keys is a box, and a key that
// differs from the one before it starts a run.  First pass: run starts per tile;
// after those counts are scanned, the second pass numbers each tile's run starts
// in order and writes the box's key, its first point and its cell of the table.
template <typename K>
__device__ __forceinline__ int32_t run_starts(const K* __restrict__ key, int64_t n, int64_t base, uint32_t& mask) {
  K prev = base > 0 && base - 1 < n ? key[base - 1] : K(0);
  int32_t c = 0;
  mask = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t e = base + r;
    if (e < n) {
      const K k = key[e];
      if (e == 0 || k != prev) {
        mask |= 1u << r;
        ++c;
      }
      prev = k;
    }
  }
  return c;
}

// Also marks every cell of the dense cell table empty (table may be null), ahead of
// k_runs_write, which enters the boxes.
template <typename K>
__global__ void __launch_bounds__(kBlock) k_runs_count(const K* __restrict__ key, int64_t n,
                                                    int32_t* __restrict__ part, int32_t* __restrict__ table,
                                                    int64_t cells) {
  __shared__ int32_t lds[kBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t mask;
  const int32_t c = run_starts(key, n, base, mask);
  int32_t tot;
  block_exclusive_scan<int32_t>(c, lds, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < cells; i += (int64_t)gridDim.x * kBlock)
    table[i] = -1;
}

// part: the tile counts, scanned; status->nbox: the number of boxes.
template <typename K>
__global__ void __launch_bounds__(kBlock) k_runs_write(const K* __restrict__ key, int64_t n,
                                                    const int32_t* __restrict__ part, uint64_t* __restrict__ box_key,
                                                    int32_t* __restrict__ box_start,
                                                    const DevStatus* __restrict__ status, CellGrid grid) {
  __shared__ int32_t lds[kBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t mask;
  const int32_t c = run_starts(key, n, base, mask);
  int32_t tot;
  int32_t b = block_exclusive_scan<int32_t>(c, lds, &tot) + part[blockIdx.x];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    if (mask & (1u << r)) {
      const int64_t e = base + r;
      const uint64_t k = key[e];
      box_key[b] = k;
      box_start[b] = (int32_t)e;
      if (grid.table) grid.table[grid.cell(compact3(k), compact3(k >> 1), compact3(k >> 2))] = b;
      ++b;
    }
    if (base + r == n - 1) box_start[status->nbox] = (int32_t)n;
  }
}

// Plans of distinct sets: the first source of each box.  A box lists its points
// in input order, targets (indices below n_targets) first, so its first source is
// found by binary search over perm.  Entry nbox is n.
__global__ void __launch_bounds__(kBlock) k_src_start(const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ box_start,
                                                   const DevStatus* __restrict__ status, int64_t n,
                                                   int64_t n_targets, int32_t* __restrict__ src_start) {
  const int64_t T = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int32_t nb = status->nbox;
  if (T > nb) return;
  if (T == nb) {
    src_start[T] = (int32_t)n;
    return;
  }
  int32_t lo = box_start[T], hi = box_start[T + 1];
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (perm[mid] < n_targets) lo = mid + 1;
    else hi = mid;
  }
  src_start[T] = lo;
}

// One box per half wavefront (grid-stride): sorted FP64 coordinates (SoA), the
// box's bounding box, the largest occupancy and the largest |coordinate|.
__global__ void __launch_bounds__(kBlock) k_box_geom(const double* __restrict__ xyz, const int32_t* __restrict__ perm,
                                                  int64_t n, const int32_t* __restrict__ box_start,
                                                  const DevStatus* __restrict__ status, double* __restrict__ sx,
                                                  double* __restrict__ bb, Partial* __restrict__ part) {
  __shared__ double ldsd[kWavesPerBlockPlan];
  __shared__ uint32_t ldsu[kWavesPerBlockPlan];
  const int lane = threadIdx.x & (kWave - 1), half = lane >> 5, h = lane & 31;
  const int32_t nb = status->nbox;
  uint32_t tmax = 0;
  bool bad_x = false;
  double amax = 0.0;
  for (int32_t T0 = 2 * (blockIdx.x * kWavesPerBlockPlan + threadIdx.x / kWave); T0 < nb;
       T0 += 2 * gridDim.x * kWavesPerBlockPlan) {
    const int32_t T = T0 + half;
    const bool live = T < nb;
    const int32_t p0 = live ? box_start[T] : 0, p1 = live ? box_start[T + 1] : 0;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = INFINITY;
      hi[d] = -INFINITY;
    }
    for (int32_t p = p0 + h; p < p1; p += 32) {
      const int64_t i = perm[p];
      for (int d = 0; d < 3; ++d) {
        const double v = xyz[3 * i + d];
        bad_x |= !isfinite(v);
        sx[d * n + p] = v;
        lo[d] = fmin(lo[d], v);
        hi[d] = fmax(hi[d], v);
      }
    }
    for (int d = 0; d < 3; ++d) {
      lo[d] = -half_max(-lo[d]);
      hi[d] = half_max(hi[d]);
    }
    if (h == 31 && live) {
      for (int d = 0; d < 3; ++d) {
        bb[6 * (int64_t)T + d] = lo[d];
        bb[6 * (int64_t)T + 3 + d] = hi[d];
        amax = fmax(amax, fmax(fabs(lo[d]), fabs(hi[d])));
      }
      tmax = max(tmax, (uint32_t)(p1 - p0));
    }
  }
  // lanes 31 and 63 hold the two halves' results; lane 63 takes both
  tmax = max(tmax, lane31(tmax));
  amax = fmax(amax, lane31(amax));
  tmax = block_combine63(tmax, ldsu, [](uint32_t x, uint32_t y) { return x > y ? x : y; });
  amax = block_combine63(amax, ldsd, [](double x, double y) { return fmax(x, y); });
  const uint32_t bx = block_combine63(wave_or63(bad_x ? 2u : 0u), ldsu, [](uint32_t x, uint32_t y) { return x | y; });
  if (threadIdx.x == 0) {
    part[blockIdx.x].tmax = tmax;
    part[blockIdx.x].maxabs = amax;
    part[blockIdx.x].bad |= bx;
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

// Lane l < 27 of a wavefront: the neighbour of box T at offset
// (l % 3 - 1, l / 3 % 3 - 1, l / 9 - 1), or -1 if that box is empty or off the grid.
__device__ __forceinline__ int32_t neighbour_lane(const uint64_t* __restrict__ box_key, int32_t nb,
                                                  const CellGrid& grid, uint64_t kT, int lane) {
  if (lane >= 27) return -1;
  const int32_t x = (int32_t)compact3(kT) + lane % 3 - 1;
  const int32_t y = (int32_t)compact3(kT >> 1) + lane / 3 % 3 - 1;
  const int32_t z = (int32_t)compact3(kT >> 2) + lane / 9 - 1;
  if (grid.table) return grid.table[grid.cell(x, y, z)];
  const int32_t lim = 1 << kIdBits;
  if (x < 0 || y < 0 || z < 0 || x >= lim || y >= lim || z >= lim) return -1;
  return find_box(box_key, nb, morton3(x, y, z));
}

// One wavefront per box (grid-stride), one lane per neighbour offset.  Counting
// pass: the number of neighbours, the neighbourhood's source count, the pair
// slots and, from the bounding boxes, the largest per-axis coordinate difference
// to any neighbour and whether two distinct boxes' bounding boxes intersect.
// Filling pass: the neighbour indices in ascending order.
// Fixed-point coordinate: X = rint(x * 2^-qexp), kept modulo 2^32.  Differences of
// two such values taken modulo 2^32 are exact whenever the true difference is below
// 2^31 in magnitude, which the choice of qexp guarantees for near pairs.
__device__ __forceinline__ int32_t fixed_point(double x, int qexp) {
  const double v = rint(ldexp(x, -qexp));
  return (int32_t)(uint32_t)(uint64_t)(int64_t)v;
}

// Lane l of each 32-lane half reads lane l ^ J of the same half (swizzle, bit-mask
// mode: and-mask 31, xor-mask J).  (DPP row rotations would spare the LDS
// crossbar, but folded by the compiler into the integer subtraction that uses
// them they were measured on gfx950 to read the lane's own value, and kept as
// moves of their own they cost more instructions than the swizzles.)
template <int J>
__device__ __forceinline__ uint32_t swizzle_xor(int32_t v) {
  return (uint32_t)__builtin_amdgcn_ds_swizzle(v, 0x1f | (J << 10));
}

// Whether lane h's point (u = its fixed-point coordinates plus kCloseQuanta) lies
// within kCloseQuanta quanta, on every axis, of the point y held by lane h ^ J of
// its half, for one of the partners J = OFF + j; lanes h ^ J at or beyond ns hold
// no point.  All lanes take part in every swizzle (no short-circuit).
template <int OFF, int... j>
__device__ __forceinline__ bool close_partners(const uint32_t (&u)[3], const int32_t (&y)[3], int h, int32_t ns,
                                               std::integer_sequence<int, j...>) {
  constexpr uint32_t kTwoQ = 2u * (uint32_t)kCloseQuanta;
  bool hit = false;
  ((hit = hit | (((h ^ (OFF + j)) < ns) &
                 (max(max(u[0] - swizzle_xor<OFF + j>(y[0]), u[1] - swizzle_xor<OFF + j>(y[1])),
                      u[2] - swizzle_xor<OFF + j>(y[2])) <= kTwoQ))),
   ...);
  return hit;
}

// FILL false: neighbour counts, neighbourhood sizes and the geometry bounds.  FILL
// true: the lists themselves and, when sx32 is given (FP32 plans), the fixed-point
// coordinates of the box's own points and the box's near flag: whether two of its
// own points lie within kCloseQuanta quanta of each other on every axis, or the
// bounding box of another neighbour comes within reach of the box's own on every
// axis; either way every pair whose fixed-point r2 is at most kCloseR2 lies in a
// box marked near.  Each half of a wavefront takes one box (27 of its 32 lanes
// look up the neighbours), so a wavefront has two boxes' lookups in flight.
template <bool FILL>
__global__ void __launch_bounds__(kBlock) k_nbr(const uint64_t* __restrict__ box_key,
                                             const int32_t* __restrict__ box_start, const double* __restrict__ bb,
                                             const DevStatus* __restrict__ status, CellGrid grid,
                                             int32_t* __restrict__ cnt, int32_t* __restrict__ src,
                                             const int32_t* __restrict__ nbr_start, int32_t* __restrict__ nbr_idx,
                                             Partial* __restrict__ part, const double* __restrict__ sx64,
                                             int32_t* __restrict__ sx32, int64_t n, int qexp,
                                             int32_t* __restrict__ near, double reach,
                                             const int32_t* __restrict__ src_begin,
                                             const int32_t* __restrict__ tgt_end) {
  __shared__ uint64_t ldsl[kWavesPerBlockPlan];
  __shared__ double ldsd[kWavesPerBlockPlan];
  __shared__ uint32_t ldsu[kWavesPerBlockPlan];
  const int lane = threadIdx.x & (kWave - 1), half = lane >> 5, h = lane & 31;
  const uint64_t hmask = half ? 0xffffffff00000000ull : 0x00000000ffffffffull;
  const int32_t nb = status->nbox;
  uint64_t slots = 0, srcsum = 0;
  double msep = 0.0;
  uint32_t overlap = 0;
  if (!FILL && blockIdx.x == 0 && threadIdx.x == 0) {  // the scans' last entry
    cnt[nb] = 0;
    src[nb] = 0;
  }
  for (int32_t T0 = 2 * (blockIdx.x * kWavesPerBlockPlan + threadIdx.x / kWave); T0 < nb;
       T0 += 2 * gridDim.x * kWavesPerBlockPlan) {
    const int32_t T = T0 + half;
    const bool live = T < nb;
    const uint64_t kT = live ? box_key[T] : 0;
    const int32_t S = live ? neighbour_lane(box_key, nb, grid, kT, h) : -1;
    const bool found = S >= 0;
    if (FILL) {
      // rank among the found neighbours of the same box by box index (= by key)
      int32_t rank = 0;
      for (int j = 0; j < 27; ++j) {
        const int32_t a = __builtin_amdgcn_readlane(S, j), b = __builtin_amdgcn_readlane(S, 32 + j);
        const int32_t Sj = half ? b : a;
        rank += (Sj >= 0 && Sj < S) ? 1 : 0;
      }
      if (found) nbr_idx[nbr_start[T] + rank] = S;
      if (sx32) {
        // the box's own points in chunks of 32 per half: their fixed-point
        // coordinates, and whether two of them lie within kCloseQuanta quanta of each
        // other on every axis (coincident points included), each chunk tested
        // against itself and against the box's earlier chunks
        const int32_t b0 = live ? box_start[T] : 0, b1 = live ? box_start[T + 1] : 0;
        const int32_t nc = (b1 - b0 + 31) >> 5;
        const int32_t ncw = max(__builtin_amdgcn_readlane(nc, 0), __builtin_amdgcn_readlane(nc, 32));
        bool own = false;
        for (int32_t ci = 0; ci < ncw; ++ci) {
          const int32_t pt = b0 + 32 * ci + h;
          const bool vt = pt < b1;
          int32_t X[3] = {0, 0, 0};
          if (vt)
            for (int d = 0; d < 3; ++d) {
              X[d] = fixed_point(sx64[d * n + pt], qexp);
              sx32[d * n + pt] = X[d];
            }
          const uint32_t U[3] = {(uint32_t)X[0] + kCloseQuanta, (uint32_t)X[1] + kCloseQuanta,
                                 (uint32_t)X[2] + kCloseQuanta};
          own = own | (vt & close_partners<1>(U, X, h, b1 - b0 - 32 * ci, std::make_integer_sequence<int, 31>{}));
          for (int32_t cj = 0; cj < ci; ++cj) {
            const int32_t ps = b0 + 32 * cj + h;
            int32_t Y[3] = {0, 0, 0};
            if (ps < b1)
              for (int d = 0; d < 3; ++d) Y[d] = fixed_point(sx64[d * n + ps], qexp);
            own = own | (vt & close_partners<0>(U, Y, h, b1 - b0 - 32 * cj, std::make_integer_sequence<int, 32>{}));
          }
        }
        uint32_t close = own ? 1u : 0u;
        if (found && S != T) {
          bool within = true;
          for (int a = 0; a < 3; ++a) {
            const double gap = fmax(bb[6 * (int64_t)S + a] - bb[6 * (int64_t)T + 3 + a],
                                    bb[6 * (int64_t)T + a] - bb[6 * (int64_t)S + 3 + a]);
            within = within && gap < reach;
          }
          close |= within ? 1u : 0u;
        }
        close = half_or(close);
        if (h == 31 && live) near[T] = (int32_t)close;
      }
    } else {
      uint32_t ns = 0;
      double sep = 0.0;
      uint32_t meet = 0;
      if (found) {
        ns = (uint32_t)(box_start[S + 1] - src_begin[S]);
        bool inter = S != T;
        for (int a = 0; a < 3; ++a) {
          const double up = bb[6 * (int64_t)S + 3 + a] - bb[6 * (int64_t)T + a];
          const double dn = bb[6 * (int64_t)T + 3 + a] - bb[6 * (int64_t)S + a];
          sep = fmax(sep, fmax(up, dn));
          inter = inter && up >= 0.0 && dn >= 0.0;
        }
        meet = inter ? 1u : 0u;
      }
      const uint32_t c = (uint32_t)__popcll(__ballot(found) & hmask);
      ns = half_add(ns);
      sep = half_max(sep);
      meet = half_or(meet);
      if (h == 31 && live) {
        const int32_t nT = tgt_end[T] - box_start[T];
        cnt[T] = (int32_t)c;
        src[T] = (int32_t)ns;
        srcsum += ns;
        slots += (uint64_t)ns * (uint64_t)nT;
        msep = fmax(msep, sep);
        overlap |= meet;
      }
    }
  }
  if (!FILL) {
    // lanes 31 and 63 hold the two halves' sums; lane 63 takes both
    slots += lane31(slots);
    srcsum += lane31(srcsum);
    msep = fmax(msep, lane31(msep));
    overlap |= lane31(overlap);
    auto add = [](uint64_t x, uint64_t y) { return x + y; };
    slots = block_combine63(slots, ldsl, add);
    srcsum = block_combine63(srcsum, ldsl, add);
    msep = block_combine63(msep, ldsd, [](double x, double y) { return fmax(x, y); });
    overlap = block_combine63(overlap, ldsu, [](uint32_t x, uint32_t y) { return x | y; });
    if (threadIdx.x == 0) {
      Partial& p = part[blockIdx.x];
      p.slots = slots;
      p.srcsum = srcsum;
      p.maxsep = msep;
      p.overlap = overlap;
    }
  }
}

// Replicated source lists: one wavefront per target box copies the points of its
// neighbourhood into the box's contiguous list, its own points first.
template <bool F64>
__global__ void __launch_bounds__(kBlock) k_tile_fill(const int32_t* __restrict__ box_start,
                                                   const int32_t* __restrict__ src_begin,
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
    const int32_t p0 = src_begin[S], ns = box_start[S + 1] - p0;
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
                                                   const int32_t* __restrict__ tgt_end,
                                                   const int32_t* __restrict__ src,
                                                   const DevStatus* __restrict__ status,
                                                   uint64_t* __restrict__ key) {
  const int64_t T = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (T >= status->nbox) return;
  const double c = (double)(tgt_end[T] - box_start[T]) * (double)src[T];
  const int b = (int)fmin(255.0, floor(log2(c + 1.0) * 8.0));
  key[T] = (uint64_t)(255 - b);
}

// Lane j's value of a double (wave-uniform j).
__device__ __forceinline__ double lane_read(double v, int j) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), j);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Zero-distance pairs (self pairs included), FP64 coordinates, one wavefront per
// box; one partial sum per workgroup.  self_only: points of distinct boxes cannot
// coincide (their bounding boxes do not meet), so only the box's own points are
// compared.
__global__ void __launch_bounds__(kBlock) k_count_zero(const double* __restrict__ sx, int64_t n,
                                                    const int32_t* __restrict__ box_start,
                                                    const int32_t* __restrict__ src_begin,
                                                    const int32_t* __restrict__ tgt_end,
                                                    const int32_t* __restrict__ nbr_start,
                                                    const int32_t* __restrict__ nbr_idx, int32_t nb, bool self_only,
                                                    uint64_t* __restrict__ part) {
  __shared__ uint64_t lds[kWavesPerBlockPlan];
  const int64_t T = (int64_t)blockIdx.x * kWavesPerBlockPlan + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t z = 0;
  if (T < nb) {
    // up to 64 targets and 64 sources in registers at a time, lane l holding one of
    // each; the targets are walked with lane reads, so the inner loop touches no
    // memory.  Lanes past a chunk's end hold NaN, which equals nothing.
    const int32_t e0 = self_only ? 0 : nbr_start[T], e1 = self_only ? 1 : nbr_start[T + 1];
    const int32_t b0 = box_start[T], b1 = tgt_end[T];
    for (int32_t tb = b0; tb < b1; tb += kWave) {
      const int nt = min(kWave, b1 - tb);
      const bool tl = lane < nt;
      const double tx = tl ? sx[tb + lane] : NAN, ty = tl ? sx[n + tb + lane] : NAN,
                   tz = tl ? sx[2 * n + tb + lane] : NAN;
      for (int32_t e = e0; e < e1; ++e) {
        const int32_t S = self_only ? (int32_t)T : nbr_idx[e];
        const int32_t s0 = src_begin[S], s1 = box_start[S + 1];
        for (int32_t sb = s0; sb < s1; sb += kWave) {
          const bool sl = lane < s1 - sb;
          const double qx = sl ? sx[sb + lane] : NAN, qy = sl ? sx[n + sb + lane] : NAN,
                       qz = sl ? sx[2 * n + sb + lane] : NAN;
          for (int j = 0; j < nt; ++j)
            z += (qx == lane_read(tx, j) && qy == lane_read(ty, j) && qz == lane_read(tz, j)) ? 1 : 0;
        }
      }
    }
  }
  const uint64_t zb = block_combine63((uint64_t)wave_add63(z), lds, [](uint64_t a, uint64_t b) { return a + b; });
  if (threadIdx.x == 0) part[blockIdx.x] = zb;
}

// Statistics of FP32 plans: ordered near pairs whose fixed-point difference is
// shorter than kCloseQuanta quanta and whose FP64 distance is not zero -- the pairs
// whose geometry the kernels take from the FP64 coordinates.  As k_count_zero: one
// wavefront per box, targets and sources in registers; the neighbour boxes are
// visited only for boxes marked near (no other box holds such a pair with them).
__global__ void __launch_bounds__(kBlock) k_count_close(const int32_t* __restrict__ sx32,
                                                     const double* __restrict__ sx, int64_t n,
                                                     const int32_t* __restrict__ box_start,
                                                     const int32_t* __restrict__ src_begin,
                                                     const int32_t* __restrict__ tgt_end,
                                                     const int32_t* __restrict__ nbr_start,
                                                     const int32_t* __restrict__ nbr_idx,
                                                     const int32_t* __restrict__ near, int32_t nb,
                                                     uint64_t* __restrict__ part) {
  __shared__ uint64_t lds[kWavesPerBlockPlan];
  const int64_t T = (int64_t)blockIdx.x * kWavesPerBlockPlan + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  constexpr uint64_t lim = (uint64_t)kCloseQuanta * (uint64_t)kCloseQuanta;
  uint32_t c = 0;
  if (T < nb) {
    const bool all = near[T] != 0;
    const int32_t e0 = all ? nbr_start[T] : 0, e1 = all ? nbr_start[T + 1] : 1;
    const int32_t b0 = box_start[T], b1 = tgt_end[T];
    for (int32_t tb = b0; tb < b1; tb += kWave) {
      const int nt = min(kWave, b1 - tb);
      const int32_t ti = tb + min(lane, nt - 1);
      const int32_t tx = sx32[ti], ty = sx32[n + ti], tz = sx32[2 * n + ti];
      const double fx = sx[ti], fy = sx[n + ti], fz = sx[2 * n + ti];
      for (int32_t e = e0; e < e1; ++e) {
        const int32_t S = all ? nbr_idx[e] : (int32_t)T;
        const int32_t s0 = src_begin[S], s1 = box_start[S + 1];
        for (int32_t sb = s0; sb < s1; sb += kWave) {
          const bool sl = lane < s1 - sb;
          const int32_t si = sl ? sb + lane : s0;
          const int32_t qx = sx32[si], qy = sx32[n + si], qz = sx32[2 * n + si];
          const double gx = sx[si], gy = sx[n + si], gz = sx[2 * n + si];
          for (int j = 0; j < nt; ++j) {
            const int64_t dx = (int32_t)((uint32_t)__builtin_amdgcn_readlane(tx, j) - (uint32_t)qx);
            const int64_t dy = (int32_t)((uint32_t)__builtin_amdgcn_readlane(ty, j) - (uint32_t)qy);
            const int64_t dz = (int32_t)((uint32_t)__builtin_amdgcn_readlane(tz, j) - (uint32_t)qz);
            const uint64_t d2 = (uint64_t)(dx * dx) + (uint64_t)(dy * dy) + (uint64_t)(dz * dz);
            const bool same = gx == lane_read(fx, j) && gy == lane_read(fy, j) && gz == lane_read(fz, j);
            c += (sl && d2 < lim && !same) ? 1u : 0u;
          }
        }
      }
    }
  }
  const uint64_t cb = block_combine63((uint64_t)wave_add63(c), lds, [](uint64_t a, uint64_t b) { return a + b; });
  if (threadIdx.x == 0) part[blockIdx.x] = cb;
}

// out = sum of a[0..n), one workgroup: per-thread sums, then a tree in LDS.
__global__ void __launch_bounds__(kBlock) k_sum_u64(const uint64_t* __restrict__ a, int64_t n,
                                                 uint64_t* __restrict__ out) {
  __shared__ uint64_t lds[kBlock];
  uint64_t v = 0;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) v += a[i];
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int half = kBlock / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half) lds[threadIdx.x] += lds[threadIdx.x + half];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = lds[0];
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
  size_t off;
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
  Bump b{nullptr, 0};
  f(b);
  return (b.off + 255) & ~size_t(255);
}

p2p_status dev_alloc(void** p, size_t bytes) {
  *p = dmem_alloc(bytes);
  if (!*p) return fail(P2P_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  return P2P_OK;
}

// Scratch that goes back to the cache when the scope ends, behind the work
// enqueued on the stream so far (no host wait).
struct ScopedBlock {
  void* p = nullptr;
  hipStream_t s;
  explicit ScopedBlock(hipStream_t st) : s(st) {}
  ~ScopedBlock() { dmem_free_on(&p, 1, s); }
};

// Two such blocks released behind one event.
struct ScopedBlocks2 {
  void* p[2] = {nullptr, nullptr};
  hipStream_t s;
  explicit ScopedBlocks2(hipStream_t st) : s(st) {}
  ~ScopedBlocks2() { dmem_free_on(p, 2, s); }
};

// Copies the device status block to the host (one copy through pinned memory)
// and waits for it.
p2p_status read_status(const DevStatus* dev, DevStatus* host, hipStream_t s) {
  StagingLock st = staging(sizeof(DevStatus));
  if (st.host) {
    P2P_HIP(hipMemcpyAsync(st.host, dev, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    P2P_HIP(hipStreamSynchronize(s));
    std::memcpy(host, st.host, sizeof(DevStatus));
  } else {
    P2P_HIP(hipMemcpyAsync(host, dev, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    P2P_HIP(hipStreamSynchronize(s));
  }
  return P2P_OK;
}

// A status copy to the host that the host waits for through an event, so that
// work enqueued after the copy overlaps the wait.
struct StatusCopy {
  StagingLock st;
  hipEvent_t ev = nullptr;
  DevStatus pageable;  // target when no pinned staging buffer could be had
  ~StatusCopy() {
    if (ev) (void)hipEventDestroy(ev);
  }
  p2p_status start(const DevStatus* dev, hipStream_t s) {
    st = staging(sizeof(DevStatus));
    P2P_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    P2P_HIP(hipMemcpyAsync(st.host ? st.host : (void*)&pageable, dev, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    P2P_HIP(hipEventRecord(ev, s));
    return P2P_OK;
  }
  p2p_status finish(DevStatus* host) {
    P2P_HIP(hipEventSynchronize(ev));
    std::memcpy(host, st.host ? st.host : (void*)&pageable, sizeof(DevStatus));
    return P2P_OK;
  }
};

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
  ScopedBlock blk(s);
  p2p_status rc = dev_alloc(&blk.p, sizeof(DevStatus));
  if (rc != P2P_OK) return rc;
  DevStatus* status = (DevStatus*)blk.p;
  hipLaunchKernelGGL(k_init, dim3(1), dim3(kBlock), 0, s, (uint32_t*)status,
                     (int64_t)(sizeof(DevStatus) / sizeof(uint32_t)), nullptr, nullptr, (int64_t)0, nullptr, (int64_t)0);
  hipLaunchKernelGGL(k_box_ids, dim3(grid_for(3 * n)), dim3(kBlock), 0, s, xyz, 3 * n, origin[0], origin[1], origin[2],
                     h, ids, &status->st[ST_BAD_ID]);
  P2P_HIP(hipGetLastError());
  DevStatus hs;
  rc = read_status(status, &hs, s);
  if (rc != P2P_OK) return rc;
  if (hs.st[ST_BAD_ID]) return fail(P2P_ERR_RANGE, "a coordinate is not finite or its box id falls outside [0, 2^21)");
  return P2P_OK;
}

// ---------------------------------------------------------------------------
// Box ids without allocation (p2p_box_ids_noalloc).  The status word that
// k_box_ids raises lives in this file-scope device array rather than in a block
// from the allocator, and the host reads it into a stack variable.  Each device
// holds its own copy; its address is looked up once per device.  Calls that
// overlap on one device share the word and race.
// ---------------------------------------------------------------------------
constexpr int kScratchWords = 64;  // 256 bytes per device: word 0 is the status
static __device__ __align__(256) uint32_t scratch[kScratchWords];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch[kScratchDevices] = {};

// The current device's copy of scratch (its device address).
p2p_status scratch_ptr(uint32_t** out) {
  int d = 0;
  P2P_HIP(hipGetDevice(&d));
  if (d < 0 || d >= kScratchDevices) return fail(P2P_ERR_HIP, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[d]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    g_scratch[d] = (uint32_t*)p;
  }
  *out = g_scratch[d];
  return P2P_OK;
}
}  // namespace

__global__ void __launch_bounds__(kWave) k_zero_words(uint32_t* __restrict__ p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

p2p_status box_ids_noalloc(const double* xyz, int64_t n, const double* origin, double h, int32_t* ids,
                           hipStream_t s) {
  uint32_t* word = nullptr;
  p2p_status rc = scratch_ptr(&word);
  if (rc != P2P_OK) return rc;
  if (n == 0) return P2P_OK;
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(kWave), 0, s, word, 1);
  hipLaunchKernelGGL(k_box_ids, dim3(grid_for(3 * n)), dim3(kBlock), 0, s, xyz, 3 * n, origin[0], origin[1], origin[2],
                     h, ids, word);
  P2P_HIP(hipGetLastError());
  uint32_t bad = 0;
  P2P_HIP(hipMemcpyAsync(&bad, word, sizeof(bad), hipMemcpyDeviceToHost, s));
  P2P_HIP(hipStreamSynchronize(s));
  if (bad) return fail(P2P_ERR_RANGE, "a coordinate is not finite or its box id falls outside [0, 2^21)");
  return P2P_OK;
}

// ---------------------------------------------------------------------------
// Leaf level from the clustering threshold (paper, section 3.1: the tree height is
// raised until no leaf box holds more than CT points).  Height L has 2^(L-1) boxes
// per axis over the cube [origin, origin + size)^3, box size h = size 2^(1-L).  The
// points' keys on the finest grid (2^21 per axis, height 22) are sorted once; the
// boxes of height L are then the runs of equal key >> 3 (22 - L).  A point's id at
// height L, floor((x - o) / h), equals its finest id shifted right by 22 - L (h is
// size times a power of two), so the ids p2p_box_ids gives for the returned h have
// exactly the occupancy found here.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_fine_keys(const double* __restrict__ xyz, int64_t n, double ox, double oy,
                                                   double oz, double size, uint64_t* __restrict__ key,
                                                   uint32_t* __restrict__ bad) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const double o[3] = {ox, oy, oz};
  uint32_t id[3];
  bool out = false;
  for (int a = 0; a < 3; ++a) {
    const double v = (xyz[3 * p + a] - o[a]) / size;
    out = out || !(v >= 0.0 && v < 1.0);
    id[a] = out ? 0u : (uint32_t)floor(ldexp(v, kIdBits));
  }
  if (out) atomicOr(bad, 1u);
  key[p] = morton3(id[0], id[1], id[2]);
}

// Largest run of sorted keys equal after >> shift: every run start finds its run's
// end by binary search; the maximum over the launch lands in *tmax.
__global__ void __launch_bounds__(kBlock) k_level_tmax(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                    uint32_t* __restrict__ tmax) {
  __shared__ uint32_t lds[kBlock / kWave];
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t len = 0;
  if (p < n) {
    const uint64_t pre = key[p] >> shift;
    if (p == 0 || (key[p - 1] >> shift) != pre) {
      const uint64_t end_key = (pre + 1) << shift;  // first key of the next box (at most 2^63)
      int64_t lo = p + 1, hi = n;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] < end_key) lo = mid + 1;
        else hi = mid;
      }
      len = (uint32_t)std::min<int64_t>(lo - p, 0xffffffffll);
    }
  }
  const uint32_t m = block_combine63(wave_max63(len), lds, [](uint32_t x, uint32_t y) { return x > y ? x : y; });
  if (threadIdx.x == 0 && m) atomicMax(tmax, m);
}

p2p_status leaf_level(const double* xyz, int64_t n, const double* origin, double size, int32_t ct, int32_t lmin,
                      int32_t* level, double* h, int32_t* t_max, hipStream_t s) {
  constexpr int kTop = kIdBits + 1;  // height of the finest grid
  *level = lmin;
  *h = std::ldexp(size, 1 - lmin);
  *t_max = 0;
  if (n == 0) return P2P_OK;
  const int64_t g_rs = grid_for(n, kRsTile);
  const int64_t scan_parts = grid_for(std::max<int64_t>(256 * g_rs, n + 1), kScanTile);
  uint64_t *k0 = nullptr, *kx = nullptr;
  int32_t *v0 = nullptr, *vx = nullptr;
  uint32_t *hist = nullptr, *part = nullptr, *word = nullptr;
  auto carve = [&](Bump& b) {
    word = b.take<uint32_t>(64);
    k0 = b.take<uint64_t>(n);
    kx = b.take<uint64_t>(n);
    v0 = b.take<int32_t>(n);
    vx = b.take<int32_t>(n);
    hist = b.take<uint32_t>(256 * g_rs);
    part = b.take<uint32_t>(std::max<int64_t>(scan_parts, 256));
  };
  ScopedBlock blk(s);
  p2p_status rc = dev_alloc(&blk.p, measure(carve));
  if (rc != P2P_OK) return rc;
  {
    Bump b{(char*)blk.p, 0};
    carve(b);
  }
  hipLaunchKernelGGL(k_init, dim3(1), dim3(kBlock), 0, s, word, (int64_t)64, nullptr, nullptr, (int64_t)0, nullptr,
                     (int64_t)0);
  hipLaunchKernelGGL(k_fine_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, xyz, n, origin[0], origin[1], origin[2],
                     size, k0, word);
  SortedKeys sk;
  rc = radix_sort(k0, v0, kx, vx, n, 3 * kIdBits, hist, part, &sk, s);
  if (rc != P2P_OK) return rc;
  uint32_t host[kTop + 2] = {};
  for (int L = lmin; L <= kTop; ++L)
    hipLaunchKernelGGL(k_level_tmax, dim3(grid_for(n)), dim3(kBlock), 0, s, sk.k64, n, 3 * (kTop - L), word + L);
  P2P_HIP(hipGetLastError());
  P2P_HIP(hipMemcpyAsync(host, word, sizeof(host), hipMemcpyDeviceToHost, s));
  P2P_HIP(hipStreamSynchronize(s));
  if (host[0]) return fail(P2P_ERR_RANGE, "a point lies outside [origin, origin + size) or is not finite");
  for (int L = lmin; L <= kTop; ++L) {
    *level = L;
    *h = std::ldexp(size, 1 - L);
    *t_max = (int32_t)host[L];
    if ((int64_t)host[L] <= ct) return P2P_OK;
  }
  return fail(P2P_ERR_RANGE, "more than ct points share one box of the finest grid (coincident points)");
}

p2p_status build_plan(p2p_plan_s* P, const double* xyz, const int32_t* ids, const GridSpec* gspec, hipStream_t s) {
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
    P->src_start = P->distinct_sets ? b.take<int32_t>(n + 1) : nullptr;
    P->q_sorted = b.take<char>((int64_t)(n * (int64_t)P->max_rhs * cbytes));
    P->g_sorted = b.take<char>((int64_t)(n * (int64_t)P->max_rhs * cbytes));
  };
  const size_t bytes1 = measure(carve1);
  p2p_status rc = dev_alloc(&P->arena, bytes1);
  if (rc != P2P_OK) return rc;
  P->device_bytes = bytes1;
  {
    Bump b{(char*)P->arena, 0};
    carve1(b);
  }

  // ---- the id range decides between the dense cell table and binary search;
  //      it is known only after the first kernel, so the table is sized from the
  //      first readback and allocated then.
  const int64_t g_rs = grid_for(n, kRsTile);
  const int64_t scan_parts = grid_for(std::max<int64_t>(256 * g_rs, n + 1), kScanTile);
  uint64_t *k0 = nullptr, *k1 = nullptr;
  int32_t *v1 = nullptr, *cnt = nullptr, *src = nullptr, *part32 = nullptr;
  uint32_t *hist = nullptr, *partu = nullptr;
  double* bb = nullptr;
  DevStatus* status = nullptr;
  Partial* part = nullptr;
  auto carvet = [&](Bump& b) {
    status = b.take<DevStatus>(1);
    part = b.take<Partial>(kGridStride);
    k0 = b.take<uint64_t>(n);
    k1 = b.take<uint64_t>(n);
    v1 = b.take<int32_t>(n);
    cnt = b.take<int32_t>(n + 1);
    src = b.take<int32_t>(n + 1);
    hist = b.take<uint32_t>(256 * g_rs);
    partu = b.take<uint32_t>(std::max<int64_t>(scan_parts, 256));
    part32 = b.take<int32_t>(scan_parts);
    bb = b.take<double>(6 * std::max<int64_t>(n, 1));
  };
  ScopedBlocks2 tmp(s);  // p[0]: this scratch, p[1]: the dense cell table
  rc = dev_alloc(&tmp.p[0], measure(carvet));
  if (rc != P2P_OK) return rc;
  {
    Bump b{(char*)tmp.p[0], 0};
    carvet(b);
  }
  // status block and partial rows are contiguous in the scratch block
  const int64_t zero_words = (int64_t)(((char*)(part + kGridStride) - (char*)status) / sizeof(uint32_t));
  hipLaunchKernelGGL(k_init, dim3((unsigned)std::min<int64_t>(kGridStride, grid_for(n + 1))), dim3(kBlock), 0, s,
                     (uint32_t*)status, zero_words, nullptr, nullptr, (int64_t)0, nullptr, (int64_t)0);
  if (n == 0) {  // offsets of an empty plan: box_start = nbr_start = tile_start = {0}
    hipLaunchKernelGGL(k_init, dim3(1), dim3(kBlock), 0, s, nullptr, (int64_t)0, P->box_start, P->nbr_start,
                       (int64_t)1, nullptr, (int64_t)0);
    hipLaunchKernelGGL(k_init, dim3(1), dim3(kBlock), 0, s, nullptr, (int64_t)0, P->tile_start, P->tile_start,
                       (int64_t)1, nullptr, (int64_t)0);
    P->qexp = -30;
    P2P_HIP(hipGetLastError());
    P2P_HIP(hipStreamSynchronize(s));
    return P2P_OK;
  }

  // ---- 1. Morton keys and validation (first readback)
  const unsigned gk = (unsigned)std::min<int64_t>(kGridStride, grid_for(n));
  if (gspec)
    hipLaunchKernelGGL(k_keys<true>, dim3(gk), dim3(kBlock), 0, s, nullptr, xyz, *gspec, n, k0, part);
  else
    hipLaunchKernelGGL(k_keys<false>, dim3(gk), dim3(kBlock), 0, s, ids, nullptr, GridSpec{{0, 0, 0}, 1.0}, n, k0,
                       part);
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(kBlock), 0, s, part, status);
  P2P_HIP(hipGetLastError());
  // The first radix pass does not depend on what the copy reports, so it is
  // enqueued behind it and runs while the host waits: it assumes keys of at most
  // 32 bits (narrowed on the way) and an odd number of passes (values into perm),
  // which holds for 17-24 key bits; the other cases are put right below.
  uint32_t* a32 = reinterpret_cast<uint32_t*>(k1);
  uint32_t* b32 = a32 + n;
  DevStatus hs;
  {
    StatusCopy copy;
    rc = copy.start(status, s);
    if (rc != P2P_OK) return rc;
    rc = radix_pass<uint64_t, uint32_t>(k0, nullptr, a32, P->perm, n, 0, hist, partu, s);
    if (rc != P2P_OK) return rc;
    rc = copy.finish(&hs);
    if (rc != P2P_OK) return rc;
  }
  if (hs.st[ST_BAD_ID])
    return fail(P2P_ERR_RANGE, gspec ? "a coordinate is not finite or its box id falls outside [0, 2^21)"
                                     : "a box id falls outside [0, 2^21)");
  if (hs.st[ST_BAD_X]) return fail(P2P_ERR_RANGE, "a coordinate is not finite");

  // dense cell table when the occupied id range is small enough
  CellGrid grid{nullptr, 0, 0, 0, 0, 0};
  int64_t table_cells = 0;
  {
    const int32_t lo[3] = {(int32_t)(kIdMask - hs.st[ST_LO_X]), (int32_t)(kIdMask - hs.st[ST_LO_Y]),
                           (int32_t)(kIdMask - hs.st[ST_LO_Z])};
    const int64_t ext[3] = {(int64_t)hs.st[ST_HI_X] - lo[0] + 3, (int64_t)hs.st[ST_HI_Y] - lo[1] + 3,
                            (int64_t)hs.st[ST_HI_Z] - lo[2] + 3};
    const double cells = (double)ext[0] * (double)ext[1] * (double)ext[2];
    if (cells <= (double)table_cell_limit(n)) {
      tmp.p[1] = dmem_alloc(sizeof(int32_t) * (size_t)cells);  // no room: fall back to binary search
      if (tmp.p[1]) {
        grid = CellGrid{(int32_t*)tmp.p[1], lo[0], lo[1], lo[2], ext[0], ext[1]};
        table_cells = (int64_t)cells;  // marked empty by the box-table pass
      }
    }
  }

  // ---- 2. stable sort of the points by key, over the key bits in use (8 per pass;
  //         with no bits in use the first pass alone gives the identity order)
  const int bits = 3 * bit_length(hs.st[ST_ID_OR]);
  SortedKeys sk;
  if (bits <= 32) {
    const int passes = std::max(1, (bits + 7) / 8);
    uint32_t *kc = a32, *ko = b32;
    int32_t *vc = P->perm, *vo = v1;
    for (int p = 1; p < passes; ++p) {
      rc = radix_pass<uint32_t, uint32_t>(kc, vc, ko, vo, n, 8 * p, hist, partu, s);
      if (rc != P2P_OK) return rc;
      std::swap(kc, ko);
      std::swap(vc, vo);
    }
    if (vc != P->perm) P2P_HIP(hipMemcpyAsync(P->perm, vc, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    sk.k32 = kc;
    sk.k64 = nullptr;
  } else {  // 64-bit keys: the speculative pass is discarded and the sort starts over
    rc = radix_sort(k0, P->perm, k1, v1, n, bits, hist, partu, &sk, s);
    if (rc != P2P_OK) return rc;
  }

  // ---- 3. box table: runs of equal keys
  {
    const unsigned gt = grid_for(n, kScanTile);
    if (sk.k32)
      hipLaunchKernelGGL(k_runs_count<uint32_t>, dim3(gt), dim3(kBlock), 0, s, sk.k32, n, part32, grid.table,
                         table_cells);
    else
      hipLaunchKernelGGL(k_runs_count<uint64_t>, dim3(gt), dim3(kBlock), 0, s, sk.k64, n, part32, grid.table,
                         table_cells);
    const ScanIO<int32_t> io{{nullptr, nullptr}, {nullptr, nullptr}, {part32, nullptr}, {&status->nbox, nullptr}};
    hipLaunchKernelGGL(k_scan_partials<int32_t>, dim3(1, 1), dim3(kBlock), 0, s, io, (int64_t)gt);
    if (sk.k32)
      hipLaunchKernelGGL(k_runs_write<uint32_t>, dim3(gt), dim3(kBlock), 0, s, sk.k32, n, part32, P->box_key,
                         P->box_start, status, grid);
    else
      hipLaunchKernelGGL(k_runs_write<uint64_t>, dim3(gt), dim3(kBlock), 0, s, sk.k64, n, part32, P->box_key,
                         P->box_start, status, grid);
    P2P_HIP(hipGetLastError());
  }
  if (P->src_start)
    hipLaunchKernelGGL(k_src_start, dim3(grid_for(n + 1)), dim3(kBlock), 0, s, P->perm, P->box_start, status, n,
                       P->n_targets, P->src_start);
  const unsigned gs = (unsigned)std::min<int64_t>(kGridStride, grid_for(n, kWavesPerBlockPlan));
  hipLaunchKernelGGL(k_box_geom, dim3(gs), dim3(kBlock), 0, s, xyz, P->perm, n, P->box_start, status, P->sx64, bb,
                     part);

  // ---- 4. neighbour counts, neighbourhood source counts, separation bound.
  //         The counting pass also zeroes entry B, so scanning B + 1 entries gives
  //         the offsets of the B boxes and, at index B, the totals.
  hipLaunchKernelGGL(k_nbr<false>, dim3(gs), dim3(kBlock), 0, s, P->box_key, P->box_start, bb, status, grid, cnt, src,
                     nullptr, nullptr, part, nullptr, nullptr, n, 0, nullptr, 0.0, src_begin(P), tgt_end(P));
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(kBlock), 0, s, part, status);
  P2P_HIP(hipGetLastError());
  {  // both box-indexed arrays in one set of launches (partu is free once the sort is done)
    const ScanIO<int32_t> io{{cnt, src}, {P->nbr_start, P->tile_start}, {part32, (int32_t*)partu},
                             {&status->nnz, nullptr}};
    rc = scan_arrays<int32_t>(io, 2, n + 1, s, &status->nbox);
  }
  if (rc != P2P_OK) return rc;

  // second readback: sizes of the lists and the geometry bounds.  The processing
  // order of the sweep (boxes with the most pair slots first: one stable 8-bit
  // radix pass over cost keys, with the box count read on the device) is enqueued
  // behind the copy and runs while the host waits for it.
  {
    StatusCopy copy;
    rc = copy.start(status, s);
    if (rc != P2P_OK) return rc;
    hipLaunchKernelGGL(k_cost_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, P->box_start, tgt_end(P), src, status, k0);
    P2P_HIP(hipGetLastError());
    rc = radix_sort(k0, P->work, k1, v1, n, 8, hist, partu, &sk, s, &status->nbox);
    if (rc != P2P_OK) return rc;
    rc = copy.finish(&hs);
    if (rc != P2P_OK) return rc;
  }
  if (hs.st[ST_BAD_X]) return fail(P2P_ERR_RANGE, "a coordinate is not finite");
  const int32_t B = hs.nbox;
  P->B = B;
  P->nnz = hs.nnz;
  P->n_slots = (int64_t)hs.slots;
  P->t_max = (int32_t)hs.st[ST_TMAX];
  P->may_coincide = hs.st[ST_OVERLAP] != 0;
  double sep, xabs;
  std::memcpy(&sep, &hs.maxsep, sizeof(double));
  std::memcpy(&xabs, &hs.maxabs, sizeof(double));
  P->max_sep = sep;
  if ((int64_t)hs.srcsum > 0x7fffffffll) return fail(P2P_ERR_RANGE, "the per-box source lists exceed 2^31 entries");
  P->tile_len = tiles ? (int64_t)hs.srcsum : 0;
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

  // ---- 6. second allocation: neighbour lists, replicated source lists and, for
  //         FP32 plans, the near flags
  auto carve2 = [&](Bump& b) {
    P->nbr_idx = b.take<int32_t>(P->nnz);
    P->tile_src = tiles ? b.take<int32_t>(P->tile_len) : nullptr;
    P->tile_x64 = (tiles && f64) ? b.take<double>(3 * P->tile_len) : nullptr;
    P->tile_x32 = (tiles && !f64) ? b.take<int32_t>(3 * P->tile_len) : nullptr;
    P->near = f64 ? nullptr : b.take<int32_t>(B);
  };
  const size_t bytes2 = measure(carve2);
  rc = dev_alloc(&P->arena2, bytes2);
  if (rc != P2P_OK) return rc;
  P->device_bytes += bytes2;
  {
    Bump b{(char*)P->arena2, 0};
    carve2(b);
  }
  // two boxes whose bounding boxes are at least kCloseQuanta + 2 quanta apart on
  // some axis hold no pair closer than kCloseQuanta quanta in fixed point (each
  // coordinate rounds by at most half a quantum; the bounding boxes' FP64
  // differences by far less than the second quantum of margin)
  const double reach = std::ldexp((double)kCloseQuanta + 2.0, P->qexp);
  // the filling pass writes no partial rows: one wavefront per two boxes
  hipLaunchKernelGGL(k_nbr<true>, dim3((unsigned)grid_for(B, 2 * kWavesPerBlockPlan)),
                     dim3(kBlock), 0, s, P->box_key, P->box_start, bb, status, grid, cnt, src, P->nbr_start,
                     P->nbr_idx, part, P->sx64, f64 ? nullptr : P->sx32, n, P->qexp, P->near, reach, src_begin(P),
                     tgt_end(P));
  if (tiles) {
    const unsigned g = grid_for(B, kWavesPerBlockPlan);
    if (f64)
      hipLaunchKernelGGL(k_tile_fill<true>, dim3(g), dim3(kBlock), 0, s, P->box_start, src_begin(P), P->nbr_start,
                         P->nbr_idx,
                         P->tile_start, B, n, P->tile_len, P->sx64, P->sx32, P->tile_src, P->tile_x64, P->tile_x32);
    else
      hipLaunchKernelGGL(k_tile_fill<false>, dim3(g), dim3(kBlock), 0, s, P->box_start, src_begin(P), P->nbr_start,
                         P->nbr_idx,
                         P->tile_start, B, n, P->tile_len, P->sx64, P->sx32, P->tile_src, P->tile_x64, P->tile_x32);
  }
  P2P_HIP(hipGetLastError());
  return P2P_OK;
}

// The number of nonzero entries of a[0..n), added to *out (one atomic per
// workgroup).
__global__ void __launch_bounds__(kBlock) k_count_nonzero(const int32_t* __restrict__ a, int64_t n,
                                                       unsigned long long* __restrict__ out) {
  __shared__ uint64_t lds[kWavesPerBlockPlan];
  uint64_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    c += a[i] != 0 ? 1u : 0u;
  c = block_combine63((uint64_t)wave_add63(c), lds, [](uint64_t x, uint64_t y) { return x + y; });
  if (threadIdx.x == 0 && c) atomicAdd(out, (unsigned long long)c);
}

p2p_status count_pairs(p2p_plan_s* P, hipStream_t s) {
  if (P->n_pairs >= 0) return P2P_OK;
  ScopedBlock blk(s);
  const unsigned g = grid_for(std::max<int64_t>(P->B, 1), kWavesPerBlockPlan);
  p2p_status rc = dev_alloc(&blk.p, sizeof(DevStatus) + sizeof(uint64_t) * g);
  if (rc != P2P_OK) return rc;
  DevStatus* status = (DevStatus*)blk.p;
  uint64_t* part = (uint64_t*)((char*)blk.p + sizeof(DevStatus));
  hipLaunchKernelGGL(k_init, dim3(1), dim3(kBlock), 0, s, (uint32_t*)status,
                     (int64_t)(sizeof(DevStatus) / sizeof(uint32_t)), nullptr, nullptr, (int64_t)0, nullptr, (int64_t)0);
  if (P->B > 0) {
    hipLaunchKernelGGL(k_count_zero, dim3(g), dim3(kBlock), 0, s, P->sx64, P->n, P->box_start, src_begin(P),
                       tgt_end(P), P->nbr_start,
                       P->nbr_idx, (int32_t)P->B, !P->may_coincide, part);
    hipLaunchKernelGGL(k_sum_u64, dim3(1), dim3(kBlock), 0, s, part, (int64_t)g, &status->zero);
    if (P->near) {
      hipLaunchKernelGGL(k_count_close, dim3(g), dim3(kBlock), 0, s, P->sx32, P->sx64, P->n, P->box_start,
                         src_begin(P), tgt_end(P), P->nbr_start, P->nbr_idx, P->near, (int32_t)P->B, part);
      hipLaunchKernelGGL(k_sum_u64, dim3(1), dim3(kBlock), 0, s, part, (int64_t)g, &status->ncp);
      hipLaunchKernelGGL(k_count_nonzero, dim3((unsigned)std::min<int64_t>(256, grid_for(P->B))), dim3(kBlock), 0, s,
                         P->near, (int64_t)P->B, (unsigned long long*)&status->nnear);
    }
  }
  P2P_HIP(hipGetLastError());
  DevStatus hs;
  rc = read_status(status, &hs, s);
  if (rc != P2P_OK) return rc;
  P->n_zero = (int64_t)hs.zero;
  P->n_pairs = P->n_slots - P->n_zero;
  P->n_close = (int64_t)hs.ncp;
  P->n_near = (int64_t)hs.nnear;
  return P2P_OK;
}

}  // namespace p2p
