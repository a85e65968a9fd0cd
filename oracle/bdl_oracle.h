/*
 * Serial CPU oracle for the BDL-tree ("Parallel Batch-Dynamic kd-trees",
 * Yesantharao, Wang, Dhulipala, Shun).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously correct
 * reimplementation of what the GPU library computes.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * GPU library never links, includes or calls anything here, and nothing here
 * includes the GPU library's headers.
 *
 * Everything is single-threaded.  Floating point is float32 exactly as the
 * method fixes it (no fast-math, no contraction: build with
 * -ffp-contract=off); distances use the canonical squared distance
 *     acc = 0; for j: t = q[j] - p[j]; acc = fmaf(t, t, acc)
 * so that results are bit-reproducible.
 *
 * Parity status per function (see the comments at each definition):
 *   orc_bruteforce_knn  pinned (scipy kd-tree on float64, exact integer lattice)
 *   orc_tree_*          pinned (Fig. 1 split example, hand-derived
 *                       spatial- and object-median split values of
 *                       Section V-C, exact halving by the object median,
 *                       Fig. 3 vEB example, structural invariants checked
 *                       outside the oracle)
 *   orc_insert          pinned (Fig. 4 sequence, binary-counter closed form;
 *                       baselines: B1 equals one fresh build, B2 keeps its
 *                       splits and places points by them)
 *   orc_erase           pinned (live-set bookkeeping, half-capacity invariant)
 *   orc_knn             pinned (against the brute force definition)
 */
#ifndef BDL_ORACLE_H
#define BDL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXD 16
#define ORC_MAX_DEPTH 63
#define ORC_MAXLEV 48
#define ORC_TOMB 0xFFFFFFFFu
/* the structure: the BDL-tree, or one of the baselines of Section III-B */
#define ORC_MODE_BDL 0          /* log structure of static trees + buffer */
#define ORC_MODE_REBUILD_ALL 1  /* B1: one tree, rebuilt after every update */
#define ORC_MODE_NO_REBUILD 2   /* B2: one tree, updated in place, never rebuilt */
/* split heuristics of Section V-C */
#define ORC_SPLIT_SPATIAL 0 /* midpoint of the node's tight extent */
#define ORC_SPLIT_OBJECT 1  /* median of the node's coordinates */

/* Node of a static kd-tree, in the tree's vEB order (index 0 = root). */
typedef struct {
  float lo[ORC_MAXD];   /* tight bounding box of the node's points */
  float hi[ORC_MAXD];
  float split;          /* internal: left = {x[dim] < split}; leaf: 0 */
  int32_t dim;          /* split dimension, -1 for a leaf */
  int32_t left, right;  /* child indices, -1 for a leaf */
  int32_t parent;       /* -1 for the root */
  int32_t begin, count; /* slot range covered by the subtree */
  int32_t depth;
  int32_t pad_;
  uint64_t path;        /* moves from the root, first move most significant */
} orc_node;

typedef struct {
  int64_t node_visits;  /* nodes entered by the traversal */
  int64_t dist_evals;   /* point distances computed */
} orc_counters;

typedef struct orc_bdl orc_bdl;

/* --- BDL-tree log structure (Section IV-B) ----------------------------- */
orc_bdl* orc_create(int dim, int leaf_size, int buffer_size);
void orc_destroy(orc_bdl* t);
/* Split heuristic of every tree built from now on (ORC_SPLIT_*); only on an
 * empty structure.  Returns 0, or -1 if the rule is unknown or the structure
 * holds points.  The default is the spatial median. */
int orc_set_split_rule(orc_bdl* t, int rule);
/* Structure (ORC_MODE_*); only on an empty structure.  Returns 0 or -1.  The
 * baselines keep one tree as static tree 0 (F = 1 while it holds slots) and
 * no buffer. */
int orc_set_mode(orc_bdl* t, int mode);
/* Insert_L (Alg. 3).  Returns 0. */
int orc_insert(orc_bdl* t, const float* pts, const uint32_t* ids, int64_t n);
/* Erase_L (Alg. 4).  Returns the number of points erased. */
int64_t orc_erase(orc_bdl* t, const float* pts, const uint32_t* ids, int64_t n);
/* kNN_L (Alg. 5): rows of k (id, squared distance), ascending by (d2, id),
 * padded with (ORC_TOMB, +inf). */
void orc_knn(orc_bdl* t, const float* q, int64_t nq, int k, uint32_t* out_ids,
             float* out_d2, orc_counters* cnt);
/* The same rows with the queries spread over host threads (OpenMP, for the
 * all-cores CPU baseline); returns the number of threads used. */
int orc_knn_parallel(orc_bdl* t, const float* q, int64_t nq, int k, uint32_t* out_ids,
                     float* out_d2, orc_counters* cnt);
int64_t orc_size(const orc_bdl* t);
/* Per-level state: live[i], cap[i] for i < *nlev, buffer live count, the
 * bitmask F and the cumulative rebuild/reinsert counters. */
void orc_level_info(const orc_bdl* t, int32_t* nlev, int64_t* live, int64_t* cap,
                    int64_t* n_slots, int64_t* buf_live, uint64_t* F,
                    int64_t* rebuilt_points, int64_t* reinserted_points);
/* Copy level `level` (or the buffer tree for level == -1) out: slots in slot
 * order (ids ORC_TOMB for erased slots), nodes in vEB order.  Any pointer
 * may be NULL to query sizes only.  Returns 0, or -1 if the level is empty. */
int orc_export_level(const orc_bdl* t, int32_t level, uint32_t* ids, float* pts,
                     orc_node* nodes, int64_t* n_slots, int64_t* n_nodes);
/* The buffer's arrival-order pool. */
int orc_export_buffer_pool(const orc_bdl* t, uint32_t* ids, float* pts, int64_t* n);

/* --- single static tree (Section IV-A) --------------------------------- */
/* BuildvEB with the spatial median over n points: permutes pts/ids in place
 * into slot order and writes nodes in vEB order (at most 2n-1).  Returns the
 * node count. */
int64_t orc_tree_build(int dim, int leaf_size, float* pts, uint32_t* ids, int64_t n,
                       orc_node* nodes_out, int32_t* height_out);
/* The same with either heuristic of Section V-C (ORC_SPLIT_*). */
int64_t orc_tree_build_rule(int dim, int leaf_size, int rule, float* pts, uint32_t* ids,
                            int64_t n, orc_node* nodes_out, int32_t* height_out);

/* --- definition of the result ------------------------------------------- */
void orc_bruteforce_knn(int dim, const float* pts, const uint32_t* ids, int64_t n,
                        const float* q, int64_t nq, int k, uint32_t* out_ids,
                        float* out_d2);
/* Canonical squared distance. */
float orc_dist2(int dim, const float* a, const float* b);

/* sizeof(orc_node), for bindings that mirror the struct. */
int32_t orc_sizeof_node(void);

#ifdef __cplusplus
}
#endif
#endif
