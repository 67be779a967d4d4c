/*
 * p2p.h - C ABI of the MI355X near-field P2P operator.
 *
 * The operator is the near-field part of the MLFMA matrix-vector product (the
 * paper's section 1 splits the product into a directly computed near field, the
 * P2P operator, and a hierarchical far field).  Points are grouped into the
 * boxes of the last tree level (section 3.1); every target receives, from every
 * source in its own and the adjacent boxes (sections 3.2 and 3.3; 27 boxes in
 * three dimensions), the kernel value times the source strength:
 *
 *     y[i,c] = sum_{j ~ i, x_j != x_i}  G(|x_i - x_j|) q[j,c],
 *     G(r)   = exp(i k r) / (4 pi r)        (k = 0: the Laplace kernel),
 *     i ~ j  <=>  max_a |b_i[a] - b_j[a]| <= 1  for the integer leaf-box ids b.
 *
 * The near relation is defined by the ids, not by the positions.  Pairs at
 * distance zero (the self pair and coincident points) are skipped.
 *
 * Conventions for every entry point:
 *  - Array arguments are HIP device pointers, except p2p_plan_export's outputs
 *    and p2p_box_ids' origin, which are host memory.
 *  - xyz is [n,3] row-major float64.  box_ijk is [n,3] row-major int32, each id
 *    in [0, 2^21).  q, y and gradients are [n, nrhs] row-major complex numbers
 *    with interleaved (re, im) parts, complex64 (P2P_C64) or complex128
 *    (P2P_C128), in the caller's original point order.
 *  - The caller owns every array it passes.  A plan owns the device memory it
 *    allocates and frees it in p2p_plan_destroy.
 *  - stream is a hipStream_t (NULL: the legacy default stream).  Work is
 *    enqueued on it, and calls return as soon as their work is enqueued.  The
 *    p2p_plan_create calls wait on the host only for two small readbacks of
 *    their own work, mid-build; the rest of the build may still be running when
 *    they return.  Later calls on the build's stream are ordered after it by the
 *    stream; the first call on any other stream (and every call that reads the
 *    plan on the host: p2p_plan_info, p2p_plan_export, p2p_batch_create) waits
 *    for the build on the host first.
 *  - A call returns a status and never aborts.  On error no output is written
 *    (for asynchronous calls: no work is enqueued) and p2p_last_error() returns
 *    a message for the calling thread.
 *  - p2p_apply and p2p_apply_backward allocate nothing and do not synchronise,
 *    so they may be captured in a HIP graph.  They use scratch memory owned by
 *    the plan: calls on one plan must be ordered (one stream at a time).
 */
#ifndef P2P_H
#define P2P_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct p2p_plan_s* p2p_plan;

typedef enum {
  P2P_OK = 0,
  P2P_ERR_ARG = 1,   /* null pointer, negative size, bad option value            */
  P2P_ERR_RANGE = 2, /* id outside [0, 2^21), non-finite coordinate, bad k or h  */
  P2P_ERR_DTYPE = 3, /* complex type differs from the plan's precision            */
  P2P_ERR_NOMEM = 4, /* device allocation failed                                  */
  P2P_ERR_HIP = 5,   /* a HIP runtime call failed                                 */
  P2P_ERR_STATE = 6  /* plan handle invalid (null or destroyed)                   */
} p2p_status;

typedef enum {
  P2P_C64 = 1,  /* complex64 strengths, FP32 arithmetic (fixed-point differences) */
  P2P_C128 = 2  /* complex128 strengths, FP64 arithmetic                          */
} p2p_dtype;

typedef enum {
  /* Per target box, one contiguous SoA list holding every source of its
   * neighbourhood (the redundant layout of the paper's section 3.3, kept per box). */
  P2P_LAYOUT_TILES = 0,
  /* No replicated sources: each box walks its neighbour boxes' ranges of the
   * sorted point arrays (the non-redundant, indexed layout of section 3.2).     */
  P2P_LAYOUT_CSR = 1
} p2p_layout;

typedef struct {
  p2p_dtype precision; /* arithmetic of p2p_apply / p2p_apply_backward             */
  p2p_layout layout;
  int32_t max_rhs;     /* largest nrhs accepted by apply and backward (>= 1)        */
  uint32_t flags;      /* reserved, must be 0                                      */
  const char* tune_cache; /* NULL, or an autotuner cache file (p2p_batch_tune): a
                             complex64 plan with max_rhs >= 6 serves many right-hand
                             sides with the launch shape recorded there for its
                             workload, if any (read at creation, never timed)      */
} p2p_opts;

typedef struct {
  int64_t n_points;
  int64_t n_boxes;      /* non-empty leaf boxes B                                  */
  int64_t n_nbr;        /* entries of the neighbour lists, sum over boxes          */
  int64_t n_slots;      /* sum over targets of the neighbourhood's source count    */
  int64_t n_pairs;      /* ordered near pairs with r != 0 (interactions per RHS)   */
  int64_t n_zero_pairs; /* near pairs skipped because r == 0 (self pairs included) */
  int64_t tile_entries; /* length of the replicated source lists (TILES), else 0   */
  int64_t device_bytes; /* device memory held by the plan                          */
  int32_t t_max;        /* largest box occupancy t                                 */
  int32_t quantum_exp;  /* FP32 plans: coordinates are integers in units of 2^e    */
  double d_mean;        /* n_points / n_boxes                                      */
  double max_sep;       /* largest per-axis coordinate difference of a near pair   */
  int64_t n_close_pairs; /* FP32 plans: ordered near pairs closer than 2^20 quanta
                            (r != 0), whose kernel values the kernels take from the
                            FP64 coordinates; 0 for FP64 plans                     */
  int64_t n_targets;    /* plans of distinct sets (p2p_plan_create_st): targets, the
                           first n_targets of n_points; otherwise n_points         */
  int64_t n_near_boxes; /* FP32 plans: boxes whose sweep checks every pair for the
                           close-pair path (two own points within 2^20 quanta, or
                           a neighbour's bounding box within reach); 0 for FP64  */
} p2p_info;

/* Leaf-box ids from positions: box_ijk[i][a] = floor((xyz[i][a] - origin[a]) / h),
 * evaluated in FP64 with a correctly rounded subtraction and division (paper
 * section 3.1: the points are assigned to the boxes of the last level).
 * origin: host double[3].  Returns P2P_ERR_RANGE (and writes nothing) if a
 * coordinate is not finite or an id falls outside [0, 2^21).  Synchronises stream. */
p2p_status p2p_box_ids(const double* xyz, int64_t n, const double* origin, double h, int32_t* box_ijk,
                       void* stream);

/* The leaf level for a clustering threshold (paper section 3.1: the tree height is
 * raised, from a starting value, until no leaf box holds more than CT points).
 * Height L divides the cube [origin, origin + size)^3 into 2^(L-1) boxes per axis,
 * box size h = size 2^(1-L), L in [1, 22].  Returns in *level the smallest
 * L >= min_level whose boxes hold at most ct points each, in *h its box size and
 * in *t_max its largest occupancy; p2p_box_ids with (origin, *h) then gives ids of
 * exactly that occupancy.  origin: host double[3]; level, h, t_max: host.
 * P2P_ERR_RANGE if a point lies outside the cube or is not finite, or if even
 * height 22 leaves more than ct points in one box (coincident points; *level, *h
 * and *t_max then describe height 22).  Synchronises stream. */
p2p_status p2p_leaf_level(const double* xyz, int64_t n, const double* origin, double size, int32_t ct,
                          int32_t min_level, int32_t* level, double* h, int32_t* t_max, void* stream);

/* p2p_box_ids for callers that cannot allocate memory (harnesses that forbid
 * hipMalloc, loops that must not allocate): the same ids and errors, but the
 * status word the kernel raises lives in a static 256-byte device array of the
 * library (one per device, kept until the process ends) instead of a block from
 * the library's allocator, and is read back into host stack memory.  Calls no
 * allocating routine.  Calls that overlap on one device share that array and
 * race; order them.  n above 79,536,431 (the largest plan) gives P2P_ERR_RANGE.
 * Synchronises stream. */
p2p_status p2p_box_ids_noalloc(const double* xyz, int64_t n, const double* origin, double h, int32_t* box_ijk,
                               void* stream);

/* Builds the plan of one point set (paper sections 3.1-3.3: boxes in Morton order,
 * neighbour lists, and the per-box source lists): Morton keys of the ids, a stable
 * sort of the points by key, the table of non-empty boxes, the 27-neighbour lists
 * (each sorted by key) and, for P2P_LAYOUT_TILES, the replicated per-box source
 * lists.  Morton key: bit 3b is bit b of the x id, 3b+1 of y, 3b+2 of z.
 * n = 0 gives a valid empty plan.  k must be finite and >= 0.  opts may be NULL
 * (complex64, tiles, max_rhs 1).  Copies what it needs from xyz and box_ijk.
 * Synchronises stream.  On success *out holds the plan. */
p2p_status p2p_plan_create(const double* xyz, const int32_t* box_ijk, int64_t n, double k, const p2p_opts* opts,
                           void* stream, p2p_plan* out);

/* The same plan with the ids computed inside the build from the positions and a
 * uniform leaf grid: box_ijk[i][a] = floor((xyz[i][a] - origin[a]) / h), evaluated
 * exactly as p2p_box_ids does (paper section 3.1), without writing or reading an
 * id array and without p2p_box_ids' own synchronisation.  origin: host double[3];
 * h finite and > 0.  Returns P2P_ERR_RANGE if a coordinate is not finite or an id
 * falls outside [0, 2^21).  Otherwise as p2p_plan_create. */
p2p_status p2p_plan_create_grid(const double* xyz, int64_t n, const double* origin, double h, double k,
                                const p2p_opts* opts, void* stream, p2p_plan* out);

/* A plan whose targets and sources are distinct point sets (the paper keeps the
 * two in separate arrays, section 3.1):
 *     y[i,c] = sum over sources j in the 27 boxes around target i's box, with
 *              t_i != s_j, of G(|t_i - s_j|) q[j,c].
 * targets [n_targets,3], sources [n_sources,3] float64, device; both on the leaf
 * grid (origin, h) as in p2p_plan_create_grid.  p2p_apply on such a plan takes q
 * [n_sources, nrhs] (source order) and writes y [n_targets, nrhs] (target order),
 * through the single-column sweep for any nrhs; p2p_apply_backward, batches and
 * p2p_apply_log2d refuse it (P2P_ERR_ARG).  p2p_plan_export gives the tables of the
 * combined set, targets first (perm entries below n_targets are targets).
 * Otherwise as p2p_plan_create_grid. */
p2p_status p2p_plan_create_st(const double* targets, int64_t n_targets, const double* sources, int64_t n_sources,
                              const double* origin, double h, double k, const p2p_opts* opts, void* stream,
                              p2p_plan* out);

/* Plan statistics (paper section 3.2: t, the largest box occupancy; section 3.4.1:
 * D, the mean number of points per box).  n_pairs, n_zero_pairs and n_close_pairs
 * are counted on the device the first time they are asked for (synchronously). */
p2p_status p2p_plan_info(p2p_plan plan, p2p_info* out);

/* Copies the plan's tables to host memory (any pointer may be NULL): the boxes in
 * Morton order with their points, and each box's neighbour boxes (paper section
 * 3.2: targets and neighbour sources of every box, with their offset arrays):
 * box_key u64[B], box_start i32[B+1], perm i32[n] (sorted position -> original
 * index), nbr_start i32[B+1], nbr_idx i32[n_nbr].  Synchronous: waits for the
 * plan's build, not for other work on the device. */
p2p_status p2p_plan_export(p2p_plan plan, uint64_t* box_key, int32_t* box_start, int32_t* perm, int32_t* nbr_start,
                           int32_t* nbr_idx);

/* y = A_near q for nrhs right-hand sides (paper sections 3.2 and 3.3: every target
 * sums, over the sources of its own and the adjacent boxes, the kernel value times
 * the source's strength; section 1 names this the P2P operator of the near field).
 * q and y: [n, nrhs] in the caller's point order.  dtype must equal the plan's
 * precision; 1 <= nrhs <= max_rhs.  y is overwritten.  FP32 plans: the kernel
 * value of every near pair closer than 2^20 quanta comes from the FP64
 * coordinates (p2p_info.n_close_pairs), the others from fixed-point differences.
 * Asynchronous on stream. */
p2p_status p2p_apply(p2p_plan plan, const void* q, void* y, int32_t nrhs, p2p_dtype dtype, void* stream);

/* Reverse pass of p2p_apply (the adjoint of the operator of paper sections 3.2 and
 * 3.3; the paper itself has no gradients) for a real loss L(y), given
 * grad_y = dL/dRe y + i dL/dIm y:
 *   grad_q = conj(A conj(grad_y))      (A is complex symmetric),
 *   grad_xyz[i] = sum_j sum_c Re( G'(r_ij) (conj(gy_ic) q_jc + conj(gy_jc) q_ic) ) (x_i - x_j) / r_ij,
 *   G'(r) = exp(i k r) (i k r - 1) / (4 pi r^2),
 * with the ids (and so the pair set) held fixed.  q, grad_y, grad_q: [n, nrhs] in
 * the caller's point order; grad_xyz: float64 [n,3].  grad_q or grad_xyz may be
 * NULL (not computed).  The same pairs as p2p_apply (close pairs of FP32 plans
 * included).  Asynchronous on stream. */
p2p_status p2p_apply_backward(p2p_plan plan, const void* q, const void* grad_y, void* grad_q, double* grad_xyz,
                              int32_t nrhs, p2p_dtype dtype, void* stream);

/* Diagnostics.  While enabled, p2p_apply and p2p_apply_backward record a pair of
 * HIP events on their stream around the near-field sweep kernels (the strength
 * gathers are outside the pair).  p2p_plan_timing_read waits for the recorded
 * events, returns the summed sweep time in milliseconds and the number of calls
 * timed, and clears them.  Event creation allocates host objects, so timing must
 * be off for calls that are captured into a HIP graph. */
p2p_status p2p_plan_timing(p2p_plan plan, int enable);
p2p_status p2p_plan_timing_read(p2p_plan plan, double* ms, int64_t* calls);

/* Batches: several complex64 plans (same layout, FP32) served together for nrhs
 * right-hand sides: for every plan y = A_near q as in p2p_apply (paper sections
 * 3.2-3.3, the same near pairs and kernel), each box's block of the product on the
 * matrix cores.  Every plan must have been created with max_rhs >= nrhs, and
 * count <= 32.  The plans stay owned by the caller and must outlive the batch.
 * p2p_batch_apply(q, y): host arrays of count device pointers, q[i] and y[i] are
 * [n_i, nrhs] complex64 in plan i's point order; one kernel launch that reads the
 * strengths in that order, no allocation, no scratch memory and no
 * synchronisation (capturable in a HIP graph, replayable with the same pointers).
 * Plans created with max_rhs >= 6 use the same path from p2p_apply when
 * nrhs >= 6.  A call with nrhs <= 16 (<= 32) uses 16 (32) columns per work item,
 * whatever the autotuner chose.  Errors: P2P_ERR_STATE for a plan or batch handle
 * that is not live, P2P_ERR_ARG for null arrays or count/nrhs out of range,
 * P2P_ERR_DTYPE for a complex128 plan, P2P_ERR_NOMEM when the batch's tables do
 * not fit. */
typedef struct p2p_batch_s* p2p_batch;
p2p_status p2p_batch_create(const p2p_plan* plans, int32_t count, int32_t nrhs, p2p_batch* out);
p2p_status p2p_batch_apply(p2p_batch batch, const void* const* q, void* const* y, void* stream);

/* Autotuner: times each launch shape of the product kernel (right-hand sides per
 * work item: 32 or 64, or only 16 (32) when the batch has at most 16 (32);
 * wavefronts per workgroup: 1, 2 or 4) on the given inputs,
 * keeps the fastest for the batch, and records it in the text file cache_path
 * (one line per workload key; NULL: no file).  A shape found in the file for the
 * same key is taken without timing.  Synchronises stream.  chosen: NULL or
 * int32[2] receiving (right-hand sides per item, wavefronts per workgroup). */
p2p_status p2p_batch_tune(p2p_batch batch, const void* const* q, void* const* y, const char* cache_path,
                          void* stream, int32_t* chosen);
/* Diagnostics as p2p_plan_timing / p2p_plan_timing_read, around the product kernel. */
p2p_status p2p_batch_timing(p2p_batch batch, int enable);
p2p_status p2p_batch_timing_read(p2p_batch batch, double* ms, int64_t* calls);
/* Frees the batch (not its plans) after its last p2p_batch_apply outside graph
 * capture has finished.  NULL is a no-op; a handle that is not a live batch gives
 * P2P_ERR_STATE and is not read. */
p2p_status p2p_batch_destroy(p2p_batch batch);

/* Frees the plan without waiting: its device memory goes back to the library's
 * cache, to be handed out again only once the plan's build and its last
 * p2p_apply or p2p_apply_backward call outside graph capture have completed on
 * the device (calls on one plan are ordered, so that covers every earlier one);
 * graphs that captured the plan's work must not be replayed after this.  NULL is a no-op; a handle that is not a live plan
 * (destroyed already, or never created) gives P2P_ERR_STATE and is not read.
 * Plan creation fails with P2P_ERR_NOMEM when device memory runs out; the
 * environment variable P2P_TEST_FAIL_ALLOC=n makes the library's n-th device
 * allocation after the variable is set (or changed) fail that way, for tests. */
p2p_status p2p_plan_destroy(p2p_plan plan);

/* ---- The paper's own experiment in two dimensions (sections 3.1-3.3, 4.6) ----
 * Points of the unit square (the paper's plate), a quadtree of height L whose
 * 4^(L-1) leaf boxes are (floor(x 2^(L-1)), floor(y 2^(L-1))), the nine neighbour
 * boxes (the box itself included), one real potential per source, and the 2-D
 * potential G(r) = -ln(r) / (2 pi), the reading taken of the kernel the paper
 * names without writing it:
 *     y_i = sum over j in the nine boxes around i's box, x_j != x_i, of G(|x_i - x_j|) q_j.
 * The paper's two GPU layouts, each collected on the host, copied to the device
 * and swept by its own kernel, with the three phases timed separately:
 *   P2P2D_INDEXING   (section 3.2): seven arrays stored one after the other --
 *                    target and source coordinates, the targets of every box in
 *                    Morton order and their box offsets, the neighbour sources of
 *                    every box and their offsets, the source potentials; one
 *                    thread per box, every box of the tree (empty ones included);
 *   P2P2D_REPETITION (section 3.3): one record per target, [x, y, count, then x,
 *                    y and potential of each neighbour source], all records of
 *                    one length, 3 + 27 CT doubles (eq. 8), or 3 + 3 times the
 *                    largest neighbourhood when boxes hold more than CT points;
 *                    one thread per target.  A target-index array (one int per
 *                    target) maps records to output rows.
 * Morton key of a box: bit 2b from bit b of its x index, 2b+1 from its y index.
 * Host arrays: xy [n, 2] float64, q [n] float64; y: device [n] float64, in the
 * caller's point order.  A point outside [0, 1)^2 gives P2P_ERR_RANGE. */
typedef enum { P2P2D_INDEXING = 0, P2P2D_REPETITION = 1 } p2p2d_method;
typedef struct p2p2d_s* p2p2d;
typedef struct {
  int64_t n_points;
  int64_t n_boxes;        /* 4^(L-1), empty boxes included                          */
  int64_t layout_bytes;   /* the collected layout                                   */
  int64_t n_slots;        /* ordered near pairs, self pairs included                */
  int64_t n_src_entries;  /* Indexing: neighbour-source entries over all boxes      */
  int32_t t_max;          /* largest box occupancy                                  */
  int32_t record_len;     /* Repetition: doubles per record                         */
  double collect_ms;      /* host collection (p2p2d_collect)                        */
  double transfer_ms;     /* host-to-device copy (last p2p2d_transfer)              */
} p2p2d_info_t;
/* Host collection of the method's layout (single-threaded, as the paper's). level
 * in [1, 15]; ct >= 1 (the clustering threshold of section 3.1, which sizes the
 * Repetition records). */
p2p_status p2p2d_collect(p2p2d_method method, const double* xy, const double* q, int64_t n, int32_t level,
                         int32_t ct, p2p2d* out);
/* Copies the layout to the device (allocating device memory on first use) and
 * waits for the copy. */
p2p_status p2p2d_transfer(p2p2d h, void* stream);
/* The method's kernel: y = the near-field potentials.  Asynchronous on stream. */
p2p_status p2p2d_run(p2p2d h, double* y, void* stream);
p2p_status p2p2d_info(p2p2d h, p2p2d_info_t* out);
/* Diagnostics: the collected host layout (valid until p2p2d_destroy) and the byte
 * offsets within it of, in order: target coordinates, source coordinates, target
 * indices, their box offsets, neighbour-source indices, their box offsets, source
 * potentials (Indexing), records, record target indices (Repetition); offsets of
 * the other method's arrays are 0.  Host only. */
p2p_status p2p2d_layout(p2p2d h, const void** data, int64_t* bytes, int64_t* offsets);
/* Frees the handle after its last run has finished; NULL is a no-op, a handle
 * that is not live gives P2P_ERR_STATE. */
p2p_status p2p2d_destroy(p2p2d h);

/* The same 2-D near field by this library's own route: a complex128 (FP64) plan
 * of the points (x, y, 0) with ids (floor(x 2^(L-1)), floor(y 2^(L-1)), 0) -- for
 * instance p2p_plan_create_grid with origin 0 and h = 2^(1-L) -- whose boxes are
 * the quadtree's in the same Morton order, swept one wavefront per box with the
 * kernel -ln(r) / (2 pi).  q, y: device [n] float64 in the caller's order.  The
 * plan's own (Helmholtz) k is not used.  Asynchronous on stream. */
p2p_status p2p_apply_log2d(p2p_plan plan, const double* q, double* y, void* stream);

const char* p2p_status_str(p2p_status s);
const char* p2p_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* P2P_H */
