/*
 * ghn.h - C ABI of libghn, a gfx950 (MI355X) implementation of Grid Hashing
 * Neighborhood KNN (Tchaye-Kondi, Zhai, Zhu, arXiv 2004.02290).
 *
 * The method (Section III):
 *   build   - "cell sampling": every training point is hashed to the cell of a
 *             virtual grid given by Eq. 1 (cell id = point // cell measurement,
 *             per dimension) and the points are grouped by cell (Algorithm 1);
 *             only non-empty cells are kept.
 *   predict - "exploration": each query is hashed to its central cell; cells are
 *             then visited layer by layer outward (layer l = the cells whose
 *             index differs from the central cell's by at most l in every
 *             dimension and by exactly l in one), keeping the k nearest points
 *             seen so far, until a stop rule fires; the k neighbours then give a
 *             majority vote or a mean (Section I, Section III-D).
 *
 * Conventions shared by every entry point:
 *   - All array arguments are DEVICE pointers owned by the caller unless marked
 *     HOST.  Arrays are dense and row-major: points are n x f, queries m x f,
 *     neighbour outputs m x k.  Pointers must be aligned to their element size.
 *   - `stream` is a hipStream_t (NULL = the default stream).  The library
 *     never synchronises a stream except where stated (ghn_build).
 *   - Every function returns a ghn_status; no exception crosses the ABI.  On
 *     failure ghn_last_error() returns a message for the calling thread.
 *   - Argument errors are detected on the host before anything is launched.
 *     An asynchronous HIP error from earlier work on the device is reported
 *     as GHN_E_HIP by the next call that checks.
 *   - Distances are squared Euclidean.  Neighbours are ordered by
 *     (d, original row index), d being the FP64 value
 *       d = (...((q0-x0)^2 + (q1-x1)^2) + ...) + (q_{f-1}-x_{f-1})^2
 *     with every difference, square and sum rounded to FP64 in that order (no
 *     fused multiply-add).  Ties in d go to the smaller row index.
 *   - Cell ids are the exact floor of (x_j - o_j) / a_j, where x_j - o_j is
 *     rounded to FP64 first (exact whenever o = 0, the grid of Eq. 1).  Query
 *     cell ids are exact up to 2^40 in magnitude and saturate at +-2^40 beyond;
 *     reported stop layers saturate at INT32_MAX.  A query more than 2^28 cells
 *     outside the occupied box of some dimension is walked with the same layers
 *     (same cells, same order, same layer numbers); under GHN_STOP_EXACT its walk
 *     may run to a later layer than the ring bound of its true layer box would
 *     allow (its neighbours are still exact).
 */
#ifndef GHN_H
#define GHN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GHN_K_MAX 64 /* largest k a predict call accepts */
#define GHN_F_MAX 32 /* largest number of features */

typedef enum {
    GHN_OK = 0,
    GHN_E_INVALID_ARG = -1,  /* bad size, null pointer, bad enum, width <= 0 or not finite */
    GHN_E_UNSUPPORTED = -2,  /* valid request this library cannot serve */
    GHN_E_K_GT_N = -3,       /* k larger than the number of training points */
    GHN_E_NONFINITE = -4,    /* a training point has a NaN or infinite coordinate */
    GHN_E_KEY_OVERFLOW = -5, /* cell ids span more than the key can hold */
    GHN_E_WORKSPACE = -6,    /* workspace missing or smaller than required */
    GHN_E_HIP = -7,          /* a HIP runtime call failed */
    GHN_E_NOMEM = -8         /* device allocation failed */
} ghn_status;

typedef enum { GHN_F32 = 0, GHN_BF16 = 1 } ghn_dtype;        /* storage of training points */
typedef enum { GHN_CLASSIFY = 0, GHN_REGRESS = 1 } ghn_task; /* int32 labels | float32 targets */

/* Stop rule of the exploration (Section III-B).
 * GHN_STOP_PAPER: stop after a layer that changed none of the k buffered
 *   neighbours while the buffer is full (the rule as the paper states it; it
 *   can miss a true neighbour, which the paper acknowledges).
 * GHN_STOP_EXACT: stop after layer l once the buffer is full and its k-th
 *   distance is below the squared distance from the query to the outside of
 *   the box of layers 0..l; the result then equals brute-force KNN.
 * Both rules also stop once every occupied cell has been visited. */
typedef enum { GHN_STOP_EXACT = 0, GHN_STOP_PAPER = 1 } ghn_stop;

/* Distance arithmetic of the candidate screen.  The selected neighbours are
 * the same in both: candidates near the k-th distance are re-scored in FP64.
 * GHN_PREC_FP32: per-query FP32 distances on the vector ALUs.
 * GHN_PREC_BF16_MFMA: queries grouped by central cell; |q|^2 + |x|^2 - 2 q.x
 *   on bf16 matrix cores with FP32 accumulation. */
typedef enum { GHN_PREC_FP32 = 0, GHN_PREC_BF16_MFMA = 1 } ghn_prec;

/* predict flags */
#define GHN_FLAG_NO_PRUNE 1u /* visit every cell of a layer, even those that provably
                                cannot hold a closer point (same result, slower) */
#define GHN_FLAG_NO_SORT 2u  /* do not reorder queries by central cell before the walk */
#define GHN_FLAG_RING_GROW 8u /* GHN_STOP_EXACT, FP32 screen: while a query's buffer holds fewer than k
                                entries, each step of its walk covers twice the layers of the step
                                before (from ghn_predict_opts.ring_step, at most 64; back to it once
                                the buffer is full); same result */
#define GHN_FLAG_MEDIAN 4u   /* regression index: predict the median of the k targets instead of
                                their mean (the paper names both, Sections I and IV): the middle
                                target in IEEE total order, or for even k the FP64 mean of the two
                                middle targets rounded to FP32 */

typedef struct ghn_index ghn_index; /* opaque HOST handle; owns its device memory, except an
                                       index built into caller storage (ghn_build_into) */

typedef struct {
    int64_t n;               /* training points */
    int32_t f;               /* features */
    int32_t dtype;           /* ghn_dtype */
    int32_t task;            /* ghn_task */
    int32_t lookup;          /* GHN_LOOKUP_DENSE, GHN_LOOKUP_TREE or GHN_LOOKUP_HASH */
    int64_t num_cells;       /* non-empty cells (never more than n, Section III-C) */
    int64_t box_cells;       /* cells in the bounding box of the occupied cells */
    int64_t max_occupancy;   /* points in the fullest cell */
    int32_t cell_min[GHN_F_MAX]; /* per-dimension range of occupied cell ids */
    int32_t cell_max[GHN_F_MAX];
    float cell_width[GHN_F_MAX];
    float origin[GHN_F_MAX];
    size_t device_bytes;     /* device memory held by the index */
} ghn_index_info;

/* Cell sampling (Eq. 1, Algorithm 1).
 *   points      n x f, float32 (dtype GHN_F32) or bfloat16 bits (GHN_BF16)
 *   targets     n int32 class labels (GHN_CLASSIFY) or n float32 values (GHN_REGRESS)
 *   cell_width  HOST, n_width floats: one width for every dimension (n_width = 1)
 *               or one per dimension (n_width = f); each finite and > 0
 *   origin      HOST, f floats or NULL (NULL = 0, the grid of Eq. 1)
 *   out         receives the handle
 * The index copies what it needs (points in cell order, targets), so the
 * caller's arrays may be freed afterwards.  Allocates device memory and
 * synchronises `stream` once (to learn the cell range and check the data).
 * Errors: GHN_E_INVALID_ARG, GHN_E_NONFINITE, GHN_E_KEY_OVERFLOW (cell ids of
 * one dimension span 2^28 or more, or the packed key needs more than 64 bits),
 * GHN_E_NOMEM, GHN_E_HIP.  On error *out is NULL and nothing is leaked. */
ghn_status ghn_build(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets,
                     int32_t task, const float* cell_width, int32_t n_width, const float* origin,
                     void* stream, ghn_index** out);

/* Cell lookup structures (ghn_build_opts.lookup, ghn_index_info.lookup).
 * GHN_LOOKUP_DENSE: an offset table over every cell of the bounding box of the
 *   occupied cells, points in row-major cell order; a run of cells along the
 *   last dimension is one run of points.  For low dimensions.
 * GHN_LOOKUP_TREE: only the occupied cells, in Morton order, under a 64-ary
 *   tree of bounding boxes; for many dimensions, where the box (and the number
 *   of cells per layer, Eq. 2) grows exponentially.
 * GHN_LOOKUP_HASH: only the occupied cells, in row-major order of a 64-bit
 *   key over the box (the cell's "unique identifier", Section III-A), in an
 *   open-addressing hash table (linear probing, load at most 1/2).  A layer is
 *   enumerated as generated cell ids (rows of the layer box with runs along the
 *   last dimension) and every generated cell is looked up, so a layer costs
 *   about its cell count (Eq. 2) in probes: for low dimensions when the box is
 *   too large for the dense table.  The key must fit 62 bits (the box holds at
 *   most 2^62 cells), else GHN_E_KEY_OVERFLOW.  Only on request: AUTO never
 *   picks it.  Grouped bf16 walks and batches walk a hash index with its tree
 *   (every index also holds the occupied-cell tree).
 * GHN_LOOKUP_AUTO: dense when the box holds at most max(16 n, 2^24) cells,
 *   otherwise the tree. */
#define GHN_LOOKUP_AUTO (-1)
#define GHN_LOOKUP_DENSE 0
#define GHN_LOOKUP_TREE 1
#define GHN_LOOKUP_HASH 2

typedef struct {
    int32_t lookup; /* GHN_LOOKUP_* */
} ghn_build_opts;

/* ghn_build with options (HOST, may be NULL = GHN_LOOKUP_AUTO).  A dense table
 * larger than the limit above is refused with GHN_E_UNSUPPORTED; the tree needs
 * the Morton code of the cell ids (sum over dimensions of the bits of each
 * dimension's id range) to fit 64 bits, else GHN_E_KEY_OVERFLOW. */
ghn_status ghn_build_ex(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets,
                        int32_t task, const float* cell_width, int32_t n_width, const float* origin,
                        const ghn_build_opts* opts, void* stream, ghn_index** out);

/* ---- the build into caller-owned device memory ---------------------------------------
 * The same build (Eq. 1, Algorithm 1) with every byte of device memory supplied by
 * the caller, e.g. as torch tensors: `index_storage` receives the index (points in
 * cell order, targets, cell list and lookup; the handle points into it, so the
 * storage must outlive the handle and is never freed by the library), `ws` holds
 * the build's temporaries (free again when the call returns).  Both are DEVICE
 * buffers aligned to 256 bytes.  Nothing is allocated on the device.
 *
 * ghn_build_workspace_bytes: bytes of `ws` for n points (any data).
 * ghn_index_bytes: bytes of `index_storage` enough for any n points of f features
 *   with any lookup; the dense table is counted at its largest size (max(16 n, 2^24)
 *   cells), so it is at least 64 MiB.
 * ghn_index_bytes_for: bytes of `index_storage` for these points and widths with the
 *   lookup the build will choose (the dense table at its actual size; the cell
 *   list, tree and hash table bounded by num_cells <= n).  It runs the cell-range
 *   pass of the build in `ws` (ghn_build_workspace_bytes(n, f) bytes) and
 *   synchronises `stream`.  targets are not read.
 * ghn_build_into: arguments as ghn_build_ex, plus the two buffers.  Synchronises
 *   `stream` (as ghn_build).  Errors: ghn_build's, and GHN_E_WORKSPACE when a
 *   buffer is missing or smaller than stated above.  ghn_index_get_info reports
 *   the bytes of the storage in use as device_bytes.  ghn_destroy frees only the
 *   host handle.  ghn_insert refuses such an index (GHN_E_UNSUPPORTED): build the
 *   enlarged index with ghn_build_into. */
size_t ghn_build_workspace_bytes(int64_t n, int32_t f);
size_t ghn_index_bytes(int64_t n, int32_t f, int32_t dtype, int32_t task);
ghn_status ghn_index_bytes_for(const void* points, int64_t n, int32_t f, int32_t dtype, int32_t task,
                               const float* cell_width, int32_t n_width, const float* origin,
                               const ghn_build_opts* opts, void* ws, size_t ws_bytes, void* stream,
                               size_t* out_bytes);
ghn_status ghn_build_into(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets,
                          int32_t task, const float* cell_width, int32_t n_width, const float* origin,
                          const ghn_build_opts* opts, void* index_storage, size_t index_bytes, void* ws,
                          size_t ws_bytes, void* stream, ghn_index** out);

/* Describe a built index.  `out` is HOST memory. */
ghn_status ghn_index_get_info(const ghn_index* index, ghn_index_info* out);

/* The cells of Eq. 1 as the build grouped the points (Algorithm 1): for each of the
 * index's num_cells occupied cells, in the index's cell order, its ids (out_ids,
 * num_cells x f int32) and point count (out_counts, num_cells int64), and for every
 * training point, in original row order, the position of its cell in that list
 * (out_point_cell, n int32).  DEVICE arrays; any may be NULL.  Asynchronous on
 * `stream`.  Errors: GHN_E_INVALID_ARG, GHN_E_HIP. */
ghn_status ghn_index_cells(const ghn_index* index, int32_t* out_ids, int64_t* out_counts, int32_t* out_point_cell,
                           void* stream);

/* Release the index and its device memory (only the handle for an index built
 * into caller storage).  NULL is ignored. */
void ghn_destroy(ghn_index* index);

typedef struct {
    int32_t stop;            /* ghn_stop */
    int32_t prec;            /* ghn_prec */
    uint32_t flags;          /* GHN_FLAG_* */
    int32_t* out_stop_layer; /* optional, m int32: layer at which each walk stopped */
    int64_t* out_cands;      /* optional, m int64: candidate points scored per query */
    int64_t* out_probes;     /* optional, m int64: cell-table entries read per query */
    const uint32_t* order;   /* optional, m uint32: order in which to walk the queries (a
                                permutation of 0..m-1, e.g. from ghn_query_order); when set,
                                no sort is done and no workspace is needed (FP32 screen) */
    int32_t group_levels;    /* bf16 screen, EXACT rule: queries whose central cells agree
                                after dropping the lowest group_levels bits of every cell id
                                (blocks of 2^group_levels cells per dimension) are walked
                                together, up to 16 per group; -1 = automatic (3 with 12 or
                                more dimensions, else 1).  The PAPER
                                rule always groups by identical central cell. */
    void* walk_event_begin;  /* optional hipEvent_t: recorded on the stream right before the walk
                                kernel (the exploration launch, after any query sort/grouping) */
    void* walk_event_end;    /* optional hipEvent_t: recorded right after the walk kernel */
    int64_t* out_rerank;     /* optional, m int64: candidates re-scored in FP64 per query (those the
                                FP32 or bf16 screen could not rule out: the re-rank band) */
    int32_t ring_step;       /* GHN_STOP_EXACT, FP32 screen: the walk's ring schedule, layers visited
                                per step before the stop test (0 or 1: one, the paper's layer by layer;
                                at most 64).  Every step's stop test uses the EXACT bound of its last
                                layer, so the neighbours do not depend on it; the reported stop layer
                                is the last layer of the final step.  Must be 0 or 1 under
                                GHN_STOP_PAPER (and without GHN_FLAG_RING_GROW) */
    int32_t group_size;      /* bf16 screen: most queries per group, 1..16 (0 = 16, a full matrix tile of
                                query rows; smaller groups leave rows empty but share fewer cells) */
    int32_t tile_width;      /* bf16 screen: candidates per screened tile, 32 or 64 (0 = 64): two or four
                                16 x 16 result blocks per admission check.  A narrower tile updates the
                                thresholds sooner and wastes less at the end of a layer's candidate
                                list; a wider one spreads the per-tile work over more candidates.  The
                                neighbours do not depend on it */
} ghn_predict_opts;

/* Bytes of device workspace ghn_predict needs for these arguments (the bf16
 * screen always needs one: it sorts and groups the queries). */
size_t ghn_predict_workspace_bytes(const ghn_index* index, int64_t m, int32_t k, const ghn_predict_opts* opts);

/* Exploration + prediction for m queries (Section III-B, III-D).
 *   queries   m x f float32
 *   k         1 <= k <= min(n, GHN_K_MAX)
 *   opts      HOST, may be NULL (= EXACT stop, FP32 screen, no flags)
 *   out_idx   m x k int64: original row ids of the neighbours, ascending (d, id)
 *   out_d2    m x k double, may be NULL: the FP64 distances d defined above
 *   out_pred  m int32 majority label (ties -> smallest label), or m float32
 *             mean (FP64 sum over the neighbours in order, / k, rounded to FP32)
 *   ws        device workspace of at least ghn_predict_workspace_bytes() bytes,
 *             256-byte aligned (may be NULL when that is 0).  Batches of 4096
 *             queries or more are walked in a spatial order (a sort by the
 *             Morton code of the central cell) unless GHN_FLAG_NO_SORT is set;
 *             the sort needs the workspace.
 * Asynchronous on `stream`; allocates nothing and launches only kernels (no
 * memset, copy or host synchronisation), so a call can be captured in a graph
 * and replayed.  m = 0 is a no-op; m must be below 2^32.  A query
 * with a non-finite coordinate gets ids -1, distances NaN and prediction -1
 * (classification) or NaN (regression), stop layer -1 (see ghn_walk_faults for
 * the same row with stop layer -2).
 * Errors: GHN_E_INVALID_ARG, GHN_E_K_GT_N, GHN_E_WORKSPACE, GHN_E_UNSUPPORTED,
 * GHN_E_HIP. */
ghn_status ghn_predict(const ghn_index* index, const float* queries, int64_t m, int32_t k,
                       const ghn_predict_opts* opts, int64_t* out_idx, double* out_d2, void* out_pred,
                       void* ws, size_t ws_bytes, void* stream);

/* ghn_predict for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments, kernels and results as ghn_predict, with the workspace taken from
 * an array the library holds on each GPU (GHN_NOALLOC_WS_BYTES bytes, a static
 * device array that every GPU the library runs on keeps until the process ends)
 * instead of a caller workspace.  The caller still passes inputs and outputs.
 * A call whose workspace (ghn_predict_workspace_bytes) exceeds the array fails
 * with GHN_E_WORKSPACE before anything is launched: above about 1.85 million
 * queries for the bf16 screen, 2.76 million for the FP32 screen's spatial sort
 * (the FP32 screen with GHN_FLAG_NO_SORT or a given order needs none).  No hipMalloc,
 * hipFree or other allocation happens.  The first call on a GPU looks up that
 * GPU's array (the device current at the call is used).  Every call on a GPU
 * shares that GPU's array and its contents from the last call (nothing in it
 * needs to start at zero: the kernels write what they read): calls that overlap
 * on one GPU (several streams or threads) race, so the caller must serialise
 * them.  Errors: those of ghn_predict. */
#define GHN_NOALLOC_WS_BYTES ((size_t)64 << 20)
ghn_status ghn_predict_noalloc(const ghn_index* index, const float* queries, int64_t m, int32_t k,
                               const ghn_predict_opts* opts, int64_t* out_idx, double* out_d2, void* out_pred,
                               void* stream);

/* Exhaustive KNN (the plain definition, Section I; the paper's comparison
 * method in Table 2) on the same index: every training point is screened for
 * every query with the bf16 matrix-core screen and the exact FP64 re-rank of
 * ghn_predict's GHN_PREC_BF16_MFMA path, without the grid walk.  The result is
 * the k smallest (d, id) over all points, bit-identical to ghn_predict with
 * GHN_STOP_EXACT.  Arguments, outputs, workspace (that of GHN_PREC_BF16_MFMA)
 * and errors as ghn_predict; of opts only flags (GHN_FLAG_MEDIAN), the
 * diagnostics outputs and the walk events are used.  Stop layers are reported
 * as 0. */
ghn_status ghn_bruteforce(const ghn_index* index, const float* queries, int64_t m, int32_t k,
                          const ghn_predict_opts* opts, int64_t* out_idx, double* out_d2, void* out_pred,
                          void* ws, size_t ws_bytes, void* stream);

/* Spatial walk order of a query batch: the permutation of 0..m-1 that sorts
 * the queries by the Morton code of their central cell (Eq. 1) clamped to the
 * occupied box.  Neighbouring queries then share cells, which keeps the
 * gathered cells in cache.  Only the order of work depends on it.
 *   queries   m x f float32;  out_order  m uint32 (device)
 *   ws        device workspace of ghn_query_order_workspace_bytes(m) bytes,
 *             256-byte aligned
 * Asynchronous on `stream`; allocates nothing.
 * Errors: GHN_E_INVALID_ARG, GHN_E_WORKSPACE, GHN_E_HIP. */
size_t ghn_query_order_workspace_bytes(int64_t m);
ghn_status ghn_query_order(const ghn_index* index, const float* queries, int64_t m, uint32_t* out_order, void* ws,
                           size_t ws_bytes, void* stream);

/* ---- many independent indexes in one launch -------------------------------------
 * A batch is a list of (index, queries, k, outputs) items answered by ONE
 * persistent kernel launch: waves take queries of all items from a shared work
 * counter, so items of very different size and depth balance across the GPU.
 * ghn_batch_prepare validates the items, uploads their descriptors into the
 * caller's device workspace (synchronising `stream`) and returns a HOST handle;
 * ghn_predict_batched then only launches kernels that read device memory, so
 * the call can be captured into a graph (hipStreamBeginCapture) and replayed.
 * Results equal those of ghn_predict on each item with the same options.  All
 * items must share f.
 * With the FP32 screen the waves take single queries, from 8 ranges of the
 * batch's queries (one per XCD, stealing from the others once empty), in spatial
 * order (all items' queries sorted by (item, Morton code of the central cell))
 * unless GHN_FLAG_NO_SORT is set or the batch holds fewer than 4096 queries; the
 * environment variable GHN_BATCH_BLOCKS, read by ghn_batch_prepare, fixes the
 * launch's grid size (results do not depend on it).  With GHN_PREC_BF16_MFMA
 * all items' queries are sorted together by (item, Morton code of the central
 * cell) and cut into groups (one item, one cell or, under GHN_STOP_EXACT, one
 * block of 2^group_levels cells per dimension), and one persistent launch walks
 * every group of every item with the grouped matrix-core screen (as ghn_predict's
 * GHN_PREC_BF16_MFMA path). */
typedef struct {
    const ghn_index* index;
    const float* queries;  /* m x f float32 */
    int64_t m;
    int32_t k;
    int64_t* out_idx;      /* m x k */
    double* out_d2;        /* m x k or NULL */
    void* out_pred;        /* m */
} ghn_batch_item;

typedef struct ghn_batch ghn_batch;

/* Workspace of a batch: ghn_batch_workspace_bytes covers the FP32 screen without
 * the spatial order (item descriptors and the work counters);
 * ghn_batch_workspace_bytes_for covers the given items and options (HOST),
 * including the sort (and for the bf16 screen the groups) of all their queries,
 * about 36 bytes per query. */
size_t ghn_batch_workspace_bytes(int32_t n_items);
size_t ghn_batch_workspace_bytes_for(const ghn_batch_item* items, int32_t n_items, const ghn_predict_opts* opts);
/* items and opts are HOST memory; opts may be NULL (EXACT, FP32).  Of opts the stop
 * rule, the screen (prec), the flags and group_levels are used.  The workspace
 * and every item's arrays must stay valid until the batch is destroyed.
 * Errors: GHN_E_INVALID_ARG, GHN_E_K_GT_N, GHN_E_WORKSPACE, GHN_E_UNSUPPORTED,
 * GHN_E_HIP. */
ghn_status ghn_batch_prepare(const ghn_batch_item* items, int32_t n_items, const ghn_predict_opts* opts, void* ws,
                             size_t ws_bytes, void* stream, ghn_batch** out);
/* Asynchronous on `stream`; allocates nothing.  Batches sharing a workspace
 * must not run concurrently. */
ghn_status ghn_predict_batched(const ghn_batch* batch, void* stream);
void ghn_batch_destroy(ghn_batch* batch);

/* ---- autotuning ---------------------------------------------------------------------
 * Times ghn_predict on a sample of queries for every candidate setting and
 * returns the fastest: the scalar cell width (each candidate builds an index),
 * the screen (FP32 per query, in input order or in spatial order, and under
 * GHN_STOP_EXACT with the ring schedules ring_step 2, GHN_FLAG_RING_GROW from 1
 * and from 2; grouped bf16 with 2^s-cell groups, s = 0 .. 3, of at most 16 or 8
 * queries) and the lookup: the one the build chooses,
 * and, where that is the tree in at most 6 dimensions, also the hash lookup
 * (FP32 settings; build the index with the returned lookup).  Under
 * GHN_STOP_EXACT every width gives the same (brute-force) neighbours, so widths
 * are tuned: `widths` (HOST) lists the candidates, or NULL for six widths
 * 2^-3 .. 2^2 times the width that puts 8 points in a cell of the points'
 * bounding box on average.  Under GHN_STOP_PAPER the width is part of the
 * method: exactly one width must be given and only the execution settings are
 * tuned.  `trials` (HOST, optional) receives up to max_trials measurements.
 * Synchronises `stream`; allocates and frees device memory.
 * Errors: as ghn_build and ghn_predict; GHN_E_UNSUPPORTED if no candidate builds. */
typedef struct {
    float cell_width;
    int32_t lookup;        /* GHN_LOOKUP_DENSE, GHN_LOOKUP_TREE or GHN_LOOKUP_HASH */
    int32_t prec;          /* ghn_prec */
    int32_t group_levels;  /* bf16: ghn_predict_opts.group_levels */
    uint32_t flags;        /* GHN_FLAG_* to pass to ghn_predict */
    int32_t ring_step;     /* ghn_predict_opts.ring_step (FP32 screen, GHN_STOP_EXACT) */
    int32_t group_size;    /* ghn_predict_opts.group_size (bf16 screen) */
    int32_t tile_width;    /* ghn_predict_opts.tile_width (bf16 screen) */
    double ms;             /* time of one predict call over the sample, or -1 if the setting failed */
} ghn_tune_trial;

ghn_status ghn_autotune(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets, int32_t task,
                        const float* queries, int64_t m, int32_t k, int32_t stop, const float* widths,
                        int32_t n_widths, ghn_tune_trial* best, ghn_tune_trial* trials, int32_t max_trials,
                        int32_t* n_trials, void* stream);

/* The paper's cell measurement rule (Section III-A, Fig. 3).  For every
 * dimension j, the range [mn_j, mx_j] covered by the points is cut into s equal
 * splits of width w = fl32((mx_j - mn_j) / s); a point x lies in split
 * min(floor((x_j - mn_j) / w), s - 1) (exact floor; the last split is closed at
 * mx_j).  The result is the largest s that leaves no split empty: out_splits[j]
 * = s, out_width[j] = w, out_origin[j] = mn_j.  Passing width and origin to
 * ghn_build makes the cells of Eq. 1 the splits (a point equal to mx_j may land
 * one cell past the last split).  A dimension whose points all coincide gets
 * s = 1 and width 1.
 *   points   n x f float32 or bf16 bits (DEVICE)
 *   out_*    f entries each (HOST)
 * Synchronises `stream`; allocates and frees temporary device memory (about
 * 24 n bytes) and copies each dimension's sorted keys (8 n bytes) to the host.
 * Errors: GHN_E_INVALID_ARG, GHN_E_NONFINITE, GHN_E_NOMEM, GHN_E_HIP. */
ghn_status ghn_cell_measure(const void* points, int64_t n, int32_t f, int32_t dtype, float* out_width,
                            float* out_origin, int64_t* out_splits, void* stream);

/* Diagnostic of the GHN_PREC_BF16_MFMA screen: for every query (DEVICE, m x f
 * float32), its screen value s = |q'|^2 + |x'|^2 - 2 q'.x' (the screen's bf16
 * operands and matrix instruction) against the exact FP64 distance d, over
 * min(sample, n) points spread evenly over the index.  out_abs[q] = max |s - d|,
 * out_rel[q] = max |s - d| / (|q'|^2 + |x'|^2) (DEVICE, m float32 each; NaN for
 * a query with a non-finite coordinate).  The screen admits with a margin of
 * 2^-12 (|q'|^2 + |x'|^2); its proven error is below 2^-13.8 of that norm sum.
 * Asynchronous on `stream`.  Errors: GHN_E_INVALID_ARG, GHN_E_HIP. */
ghn_status ghn_screen_error(const ghn_index* index, const float* queries, int64_t m, int64_t sample,
                            float* out_abs, float* out_rel, void* stream);

/* ---- persistence and insertion ---------------------------------------------------
 * The model of the method is the training data plus the grid parameters (Section
 * III-A, Algorithm 1); the grid itself is rebuilt from them, deterministically.
 *
 * ghn_index_save writes an index into HOST memory (ghn_index_save_bytes(index)
 * bytes): a versioned header (cell widths, origin, task, lookup, dtype), the
 * points in their original row order as float32 (bf16 points widen exactly) and
 * the targets.  ghn_index_load rebuilds the index from such a buffer (HOST);
 * predictions of the loaded index equal those of the saved one.  Both
 * synchronise `stream`.  Errors: GHN_E_INVALID_ARG (NULL, bad magic, version or
 * size), GHN_E_WORKSPACE (save buffer too small), GHN_E_NOMEM, GHN_E_HIP, and
 * ghn_build's errors on load. */
size_t ghn_index_save_bytes(const ghn_index* index);
ghn_status ghn_index_save(const ghn_index* index, void* buffer, size_t bytes, void* stream);
ghn_status ghn_index_load(const void* buffer, size_t bytes, void* stream, ghn_index** out);

/* Insert n_new training points (DEVICE, n_new x f, float32 or bf16 bits) and their
 * targets (DEVICE, int32 labels or float32 values as the index's task) into an
 * index: Algorithm 1 appends every point to its cell.  The new points get row
 * ids n .. n + n_new - 1.  A dense-table or hash index sorts only the new points
 * and merges them into its cell order (each after the points already in its
 * cell), then rebuilds its cell tables from that order; a tree index (Morton
 * order), or one whose enlarged box needs the tree, is rebuilt from all points.
 * Either way the index keeps its cell widths, origin and lookup choice
 * (GHN_LOOKUP_AUTO may pick the other lookup if the occupied box grew) and
 * equals ghn_build on all points.  The handle stays valid (its device memory is replaced:
 * batches prepared with it must be prepared again); on error the index is
 * unchanged.  Synchronises `stream`.  Errors: as ghn_build. */
ghn_status ghn_insert(ghn_index* index, const void* points, int64_t n_new, int32_t dtype, const void* targets,
                      void* stream);

/* Walk faults (Section III-B: a walk returns k rows of the index).  Every walk ends
 * with k neighbours by construction; if one ever ends with fewer, or with an entry
 * that is not a row of the index, its query gets the "no answer" row of a
 * non-finite query (ids -1, distances NaN, prediction -1 or NaN) with stop layer
 * -2, and the GPU raises GHN_WALK_SHORT in a fault word the library keeps on each
 * device.  ghn_walk_faults waits for `stream`, then writes that word of the current
 * device to *out_flags (HOST) and, if `clear` is nonzero, resets it to 0.  The word
 * collects faults of every ghn_predict, ghn_predict_noalloc, ghn_bruteforce and
 * batched launch on the device since it was last cleared.  Errors:
 * GHN_E_INVALID_ARG, GHN_E_HIP. */
#define GHN_WALK_SHORT 1u
ghn_status ghn_walk_faults(uint32_t* out_flags, int clear, void* stream);

/* Last error message of the calling thread ("" if none).  Valid until the
 * thread's next failing call. */
const char* ghn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GHN_H */
