/*
 * bdl.h -- C ABI of the MI355X BDL-tree library.
 *
 * The BDL-tree ("Parallel Batch-Dynamic kd-trees", Yesantharao, Wang,
 * Dhulipala, Shun) keeps a set of points as a buffer of fewer than X points
 * plus static kd-trees whose capacities are 2^i * X (Section III-C, the
 * logarithmic method).  Batch insertion rebuilds the minimum set of trees
 * (Insert_L, Alg. 3), batch deletion erases from every tree and rebuilds
 * trees that fall below half capacity (Erase_L, Alg. 4), and batched k-NN
 * visits every non-empty tree with one k-NN state per query (kNN_L, Alg. 5).
 * Each tree is built with the spatial median (Section V-C; the object median
 * with BDL_FLAG_OBJECT_MEDIAN) in van Emde Boas order (BuildvEB, Alg. 1).
 *
 * All work runs in HIP kernels on one gfx950 GPU.  Points are float32 of a
 * fixed dimension d (1..16) with caller-chosen uint32 ids.
 *
 * Conventions shared by every entry point:
 *  - Return value: 0 on success, a negative BDL_E* code on failure; the
 *    calling thread's message is then available from bdl_last_error().
 *  - Argument errors are found before any GPU work is enqueued and leave the
 *    tree unchanged.  BDL_ENOMEM also leaves the tree unchanged: new device
 *    memory is obtained before anything old is released.
 *  - Device pointers are plain HIP device addresses (for example a torch
 *    tensor's data_ptr()).  The caller owns every input and output buffer;
 *    the library copies inserted points into its own device memory.
 *  - Every call is ordered on the stream given to bdl_create.  A handle is
 *    not thread-safe.
 *  - n = 0 and nq = 0 are valid no-ops.
 */
#ifndef BDL_H
#define BDL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BDL_OK 0
#define BDL_EINVAL (-1) /* invalid argument or precondition */
#define BDL_ENOMEM (-2) /* device allocation failed or memory budget exceeded */
#define BDL_EHIP (-3)   /* a HIP runtime call failed */

#define BDL_MAX_DIM 16
#define BDL_MAX_K 64
#define BDL_INVALID_ID 0xFFFFFFFFu /* padding id; never a valid point id */

/* bdl_config.flags */
#define BDL_FLAG_CHECK_INPUTS 1u /* validate ids and coordinates on the GPU
                                    before each insert (costs one sync) */
#define BDL_FLAG_PROFILE 2u      /* time each phase with HIP events on the
                                    tree's stream (see bdl_profile) */
#define BDL_FLAG_OBJECT_MEDIAN 4u /* build every tree with the object median
                                     of Section V-C instead of the spatial
                                     median: a node splits at its coordinate
                                     of rank floor(count/2) in the split
                                     dimension (0-based, ascending; the
                                     maximum if that equals the minimum), so
                                     distinct coordinates halve exactly.
                                     Results of kNN_L are unchanged. */
/* The two baselines of Section III-B instead of the BDL-tree; both keep one
 * kd-tree (reported as static tree 0, F = 1 while it holds points) and no
 * buffer, and exclude each other. */
#define BDL_FLAG_REBUILD_ALL 8u   /* B1: every insert and every erase that
                                     removes a point rebuilds the tree over
                                     the live points (old slot order, then
                                     the batch) */
#define BDL_FLAG_NO_REBUILD 16u   /* B2: the first insert builds the tree;
                                     later inserts follow its splits into
                                     its leaves (boxes grow to contain the
                                     new points, leaves keep their points
                                     first) and erases leave tombstones; no
                                     split ever changes */

/* Phases timed under BDL_FLAG_PROFILE. */
#define BDL_PH_GATHER 0    /* Insert_L: gather of the points of new trees */
#define BDL_PH_PASSES 1    /* Insert_L: per-depth split/partition passes */
#define BDL_PH_FINISH 2    /* Insert_L: LDS subtree finisher */
#define BDL_PH_LAYOUT 3    /* Insert_L: vEB ordering and node write-out */
#define BDL_PH_ERASE 4     /* Erase_L: locate and tombstone */
#define BDL_PH_ORDER 5     /* kNN_L: Hilbert-curve ordering of the queries
                              (bdl_knn_graph: its group list) */
#define BDL_PH_TRAVERSE 6  /* kNN_L: the traversal kernel */
#define BDL_NPHASES 8

typedef struct bdl_tree bdl_tree; /* opaque, owned by the library */

typedef struct {
  int32_t dim;          /* d, 1..16 */
  int32_t leaf_size;    /* points per leaf, >= 1 (Section V-D uses 16) */
  int32_t buffer_size;  /* X, >= 1 (Section V-D uses 1024) */
  uint32_t id_capacity; /* every id must be < id_capacity (sizes the id map) */
  uint64_t mem_budget;  /* device bytes the library may hold; 0 = unlimited */
  uint32_t flags;       /* BDL_FLAG_* */
} bdl_config;

/* Create an empty tree whose work is ordered on `stream` (a hipStream_t;
 * NULL is the null stream).  *out receives the handle. */
int bdl_create(const bdl_config* cfg, void* stream, bdl_tree** out);

/* Insert_L (Alg. 3).  pts: device, row-major [n][dim] float32; ids: device
 * [n] uint32.  Preconditions: coordinates finite, ids < id_capacity and not
 * live (not currently in the tree, not repeated in the batch).  With
 * BDL_FLAG_CHECK_INPUTS a violation of the first two and of "not live" is
 * reported as BDL_EINVAL with the tree unchanged (the check waits for the
 * stream once); otherwise violating inputs give undefined results (never
 * out-of-bounds accesses).  Asynchronous: the whole insert, including the
 * build of every new tree for as many depths as its data needs, is enqueued
 * on the tree's stream without waiting for it (on a device without
 * cooperative launch the host waits once per budget of build depths), so
 * the inputs must stay unchanged until the stream has passed the call.
 * The build's device-side consistency checks (scratch overflow, a build
 * that does not end; never expected) are reported by the next bdl_sync or
 * bdl_erase as BDL_EHIP. */
int bdl_insert(bdl_tree* t, const float* pts, const uint32_t* ids, int64_t n);

/* Erase_L (Alg. 4).  A pair (pts[i], ids[i]) erases the live point with
 * that id if its stored coordinates are bitwise equal to pts[i]; otherwise
 * it is a no-op.  A repeated id erases once.  Afterwards every static tree
 * whose live count is below half of its capacity 2^i X is rebuilt through
 * Insert_L.  Synchronises the stream once to read the per-tree live counts.
 * n_erased (host, may be NULL) receives the number of points erased.
 * Memory: BDL_ENOMEM before the erase step leaves the tree unchanged; if the
 * rebuild cannot get memory (a static tree's first arena), the erase has
 * still taken effect, the trees below half stay as they are (a later erase
 * rebuilds them) and BDL_ENOMEM is returned. */
int bdl_erase(bdl_tree* t, const float* pts, const uint32_t* ids, int64_t n,
              int64_t* n_erased);

/* kNN_L (Alg. 5).  q: device [nq][dim] float32; out_ids: device [nq][k]
 * uint32; out_d2: device [nq][k] float32.  Row i holds the k live points
 * nearest to q[i], ascending by (squared distance, id), where the squared
 * distance is the float32 sum over dimensions, in order, of fmaf(t, t, acc)
 * with t = q[j] - p[j].  Rows with fewer than k live points are padded with
 * (BDL_INVALID_ID, +inf).  A query equal to a live point returns it at 0.
 * 1 <= k <= BDL_MAX_K.  Asynchronous. */
int bdl_knn(bdl_tree* t, const float* q, int64_t nq, int32_t k, uint32_t* out_ids,
            float* out_d2);

/* kNN_L without device allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Arguments, results, ordering and errors are those of
 * bdl_knn; the call is asynchronous.  The scratch it needs (the Hilbert-curve
 * ordering of the queries) is a static device array of about 17.8 MB that
 * each GPU holds until the process ends, shared by every tree on that GPU:
 * calls on one GPU whose work overlaps in time (different streams, or
 * different host threads) race on it, so callers must order them.
 * BDL_EINVAL for nq > 1048576 (the array's capacity), BDL_EHIP if the
 * runtime could not resolve the array's address on the tree's GPU. */
int bdl_knn_noalloc(bdl_tree* t, const float* q, int64_t nq, int32_t k, uint32_t* out_ids,
                    float* out_d2);

/* The k-NN graph of the live points: kNN_L (Alg. 5) with every live point
 * as a query (BDL_PARAM_GRAPH_START chooses between presorted queries
 * searched from the roots and the leaf-based search of Section II).  Row
 * `id` of out_ids
 * and out_d2 (device, [id_capacity][k] row-major, caller-owned) receives the
 * k nearest live points of live point `id`, sorted by (squared distance, id)
 * and padded as bdl_knn: exactly the row bdl_knn returns for that point as
 * a query (the point itself comes first at 0 unless another live point has
 * the same coordinates and a smaller id).  Rows of ids that are not live are
 * not written.  Asynchronous; the outputs must stay allocated until the
 * stream passes the call.  Allocates scratch on first use (BDL_ENOMEM if it
 * cannot): 4(d + 1) + 8k bytes per stored point for presorted queries,
 * about 40 bytes per stored point for the leaf-based search.  BDL_EINVAL for
 * k outside 1..64 or a null output. */
int bdl_knn_graph(bdl_tree* t, int32_t k, uint32_t* out_ids, float* out_d2);

/* Tuning parameters (bdl_set_param).  They change speed, never results. */
#define BDL_PARAM_KNN_KERNEL 1 /* 0: one lane per query; 1: one wavefront per
                                  64 neighbouring queries; 3: one wavefront
                                  per query; 2 (default): 3 for launches of
                                  at most BDL_PARAM_QUERY_MAX queries and for
                                  every launch when dim >= 5, 1 when a launch
                                  has at least 65536 queries and half as many
                                  as live points, else 0.  3 needs every tree
                                  below 2^26 nodes, else 0 runs; a tree of
                                  2^25 slots or more whose build is still
                                  running makes the call wait for that build
                                  to learn its node count */
#define BDL_PARAM_SORT_MIN 2   /* query batches of at least this many queries
                                  are visited in Hilbert-curve order (default 4096) */
#define BDL_PARAM_KNN_BLOCK 3  /* k-NN workgroup size: 64, 128 or 256 (default) */
#define BDL_PARAM_USE_GRAPHS 4 /* 1 (default): bdl_knn_batch replays captured
                                  hipGraphs; 0: it launches eagerly */
#define BDL_PARAM_PERSISTENT 5 /* 1: a k-NN batch larger than the device holds at
                                  once runs on a resident grid that draws groups
                                  of queries (64, or 128 for two per lane) from
                                  per-XCD work counters;
                                  0: one wavefront per group; 2 (default): 1 for
                                  the wavefront kernel, 0 for the lane kernel */
#define BDL_PARAM_QUERY_MAX 6  /* launches of at most this many queries use one
                                  wavefront per query under kernel 2 (default
                                  131072; 0 disables) */
#define BDL_PARAM_QUERY_STACK 7 /* pending-node entries per wavefront of kernel
                                   3, at least 130 (default and maximum 1536);
                                   a smaller stack walks more subtrees through
                                   parent links instead */
#define BDL_PARAM_ERASE_ROUTE 8 /* how bdl_erase finds a point.  0 (default):
                                   through the id map, one lookup per pair.
                                   1: as Erase_S (Alg. 2) with the Bloom
                                   filters of Section V-A: every tree whose
                                   filter may hold the pair is descended
                                   along its splits to one leaf, which is
                                   searched; each tree's filter (16 bits per
                                   point, 4 bits in one 64-bit word) is built
                                   at the first such erase after the tree
                                   changed, the buffer's at every such
                                   erase.  Same results either way. */
#define BDL_PARAM_GRAPH_START 9 /* how bdl_knn_graph searches.  0 (default):
                                   every live point becomes a query, the
                                   queries are ordered along the Hilbert
                                   curve and searched from the roots as by
                                   bdl_knn, and each row is moved to the row
                                   of its id.  1: the leaf-based search of
                                   Section II: one wavefront per subtree of
                                   at most 64 points, starting in that
                                   subtree and climbing through parent links.
                                   Same results either way. */
int bdl_set_param(bdl_tree* t, int32_t param, int64_t value);

/* One row of a launch-shape table for kNN_L (bdl_knn and bdl_knn_batch).  A
 * launch whose largest k lies in [k_lo, k_hi] and whose query count lies in
 * [nq_lo, nq_hi] uses this row's kernel, workgroup size, persistence and
 * Hilbert-curve ordering; the first matching row wins and a launch
 * no row matches uses the values of bdl_set_param.  Rows come from an
 * autotuner that times the candidates on the device.  Shapes change speed,
 * never results. */
typedef struct {
  int32_t k_lo, k_hi;   /* 1..64 */
  int64_t nq_lo, nq_hi; /* query counts, inclusive */
  int32_t kernel;       /* 0 lane, 1 wave, 3 wavefront per query (as
                           BDL_PARAM_KNN_KERNEL) */
  int32_t block;        /* 64, 128 or 256 */
  int32_t persistent;   /* 0 or 1 */
  int32_t sort;         /* 0 or 1: order the queries along the Hilbert curve
                           first (by default: for the wavefront-per-group
                           kernel, and for the lane kernel from
                           BDL_PARAM_SORT_MIN queries on) */
} bdl_knn_shape;

#define BDL_MAX_SHAPES 256

/* Install a copy of rows[0..n) (n <= BDL_MAX_SHAPES) as the tree's shape
 * table, replacing the previous one; n = 0 removes it.  BDL_EINVAL on a row
 * with a value out of range (the table is then unchanged). */
int bdl_set_knn_shapes(bdl_tree* t, const bdl_knn_shape* rows, int32_t n);

/* Remove every point.  Device memory stays allocated for reuse; the tree
 * is then as if just created.  Asynchronous. */
int bdl_clear(bdl_tree* t);

/* Device time accumulated per phase since creation or the last reset
 * (milliseconds, from HIP events recorded on the tree's stream around the
 * phase's kernels) and the number of times each phase ran.  Synchronises the
 * stream.  All zero unless the tree was created with BDL_FLAG_PROFILE. */
typedef struct {
  double ms[BDL_NPHASES];
  int64_t calls[BDL_NPHASES];
  /* k-NN work summed over queries: nodes entered, leaves scanned and point
   * distances evaluated (with the wavefront kernel a lane does the work of
   * every node its wave enters) */
  int64_t knn_nodes, knn_leaves, knn_points;
} bdl_profile_t;
int bdl_profile(bdl_tree* t, bdl_profile_t* out, int reset);

/* One request of a batched k-NN call (device pointers, as in bdl_knn). */
typedef struct {
  const float* q;     /* [nq][dim] */
  int64_t nq;
  int32_t k;          /* 1..BDL_MAX_K */
  int32_t pad_;
  uint32_t* out_ids;  /* [nq][k] */
  float* out_d2;      /* [nq][k] */
} bdl_knn_request;

/* Batched form of kNN_L: the requests' results are those bdl_knn would give
 * for each request in turn (no update runs in between), but all requests run
 * in one launch sequence: their queries are concatenated, ordered jointly,
 * and traversed by one kernel in which every query carries its own k and
 * output location.  With BDL_PARAM_USE_GRAPHS (default on) the sequence is
 * captured once per size bucket (a power of two of at least 4096 queries)
 * and replayed as a hipGraph.  Asynchronous; reqs is a host array that may
 * be reused once the call returns. */
int bdl_knn_batch(bdl_tree* t, const bdl_knn_request* reqs, int32_t nreq);

/* Block until all work enqueued on the tree's stream has finished.  Returns
 * BDL_EHIP if a k-NN traversal since the last call met an out-of-range tree
 * index, or a build reported a device-side error (a corrupt tree or an
 * undersized scratch; never expected). */
int bdl_sync(bdl_tree* t);

/* Number of times the library has blocked the calling thread on the tree's
 * stream since bdl_create (stream and event waits: bdl_erase's readback,
 * bdl_sync, inspection calls, input checks, scratch growth).  A sequence of
 * inserts into a tree whose scratch is already large enough adds none. */
int bdl_host_waits(const bdl_tree* t, int64_t* waits);

void bdl_destroy(bdl_tree* t);

/* Number of live points. */
int64_t bdl_size(const bdl_tree* t);

/* Host arrays of at least 64 entries: live and capacity of static tree i
 * for i < *nlev (live 0 for an empty tree); *buf_live receives the buffer's
 * point count, *F the bitmask of non-empty trees.  Any pointer may be NULL. */
int bdl_level_info(const bdl_tree* t, int32_t* nlev, int64_t* live, int64_t* cap,
                   int64_t* buf_live, uint64_t* F);

/* Host arrays of at least 64 entries: slots (points at build time) and
 * node count of static tree i for i < *nlev; the buffer tree's node count in
 * *buf_nodes.  Any pointer may be NULL. */
int bdl_level_sizes(const bdl_tree* t, int32_t* nlev, int64_t* n_slots, int64_t* n_nodes,
                    int64_t* buf_nodes);

/* Cumulative counters: points written by static-tree builds and points
 * moved by Erase_L's half-capacity rebuilds.  Any pointer may be NULL. */
int bdl_counters(const bdl_tree* t, int64_t* rebuilt_points, int64_t* reinserted_points);

/* Node layout of bdl_debug_export_level (host memory, one per node). */
typedef struct {
  float lo[BDL_MAX_DIM];   /* tight bounding box of the subtree's points */
  float hi[BDL_MAX_DIM];
  float split;             /* internal: left child holds x[dim] < split */
  int32_t dim;             /* split dimension, -1 for a leaf */
  int32_t left, right;     /* child node indices, -1 for a leaf */
  int32_t parent;          /* -1 for the root */
  int32_t begin, count;    /* slot range of the subtree */
  int32_t depth;
  int32_t pad_;
  uint64_t path;           /* left/right moves from the root, first move in
                              the most significant of `depth` bits */
} bdl_node;

/* Copy static tree `level` (0..63) or, for level == -1, the buffer's tree,
 * to host memory: ids[n_slots] (BDL_INVALID_ID for an erased slot),
 * pts[n_slots][dim] in slot order, and nodes[n_nodes] in vEB order.  Any
 * output pointer may be NULL; *n_slots / *n_nodes always receive the sizes.
 * Synchronises the stream.  Returns BDL_EINVAL for an empty tree. */
int bdl_debug_export_level(bdl_tree* t, int32_t level, uint32_t* ids, float* pts,
                           bdl_node* nodes, int64_t* n_slots, int64_t* n_nodes);

/* The buffer's points in arrival order (host outputs, may be NULL). */
int bdl_debug_export_buffer(bdl_tree* t, uint32_t* ids, float* pts, int64_t* n);

/* Message for the last failing call on this thread ("" if none). */
const char* bdl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BDL_H */
