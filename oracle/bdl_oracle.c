/*
 * Serial CPU oracle for the BDL-tree -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain single-threaded C written from "Parallel Batch-Dynamic kd-trees"
 * (Yesantharao, Wang, Dhulipala, Shun).  Each function cites the passage it
 * follows.  It shares no code, header or table with the GPU library; the
 * test suite, the smoke check and the benchmark's CPU-baseline leg are its
 * only users.  Build with -O3 -ffp-contract=off and without fast-math
 * (-fopenmp for the all-cores k-NN baseline).
 *
 * Readings of passages that the paper leaves open are listed at the point
 * where they are used and are marked "reading".
 */
#include "bdl_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */

static void* xmalloc(size_t n) {
  void* p = malloc(n ? n : 1);
  if (!p) {
    fprintf(stderr, "bdl_oracle: out of memory (%zu bytes)\n", n);
    abort();
  }
  return p;
}

/* Canonical squared distance: coordinate differences accumulated with a
 * fused multiply-add in dimension order, in float32. */
float orc_dist2(int dim, const float* a, const float* b) {
  float acc = 0.0f;
  for (int j = 0; j < dim; ++j) {
    float t = a[j] - b[j];
    acc = fmaf(t, t, acc);
  }
  return acc;
}

/* (squared distance, id) packed so that unsigned order is lexicographic
 * order; squared distances are never negative, so their bit patterns order
 * like the values. */
static uint64_t mkkey(float d2, uint32_t id) {
  uint32_t b;
  memcpy(&b, &d2, 4);
  return ((uint64_t)b << 32) | id;
}

static float key_d2(uint64_t key) {
  uint32_t b = (uint32_t)(key >> 32);
  float f;
  memcpy(&f, &b, 4);
  return f;
}

static uint32_t key_id(uint64_t key) { return (uint32_t)(key & 0xFFFFFFFFu); }

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

/* Bounding boxes hold +0.0 for a zero coordinate of either sign (reading:
 * the paper's boxes are sets of reals, where -0 and +0 are one value). */
static float box_val(float x) { return x == 0.0f ? 0.0f : x; }

static int64_t level_cap(const orc_bdl* t, int i);

/* ------------------------------------------------------------------------ */
/* Result definition: brute force k-NN (Section III-A.1: the k nearest       */
/* points of q).  Ties in squared distance are broken by the smaller id      */
/* (reading: the paper is silent).  Rows are padded with (ORC_TOMB, +inf).   */
/* ------------------------------------------------------------------------ */

void orc_bruteforce_knn(int dim, const float* pts, const uint32_t* ids, int64_t n,
                        const float* q, int64_t nq, int k, uint32_t* out_ids,
                        float* out_d2) {
  uint64_t pad = mkkey(INFINITY, ORC_TOMB);
  uint64_t* best = (uint64_t*)xmalloc(sizeof(uint64_t) * (size_t)k);
  for (int64_t qi = 0; qi < nq; ++qi) {
    const float* qq = q + qi * dim;
    for (int j = 0; j < k; ++j) best[j] = pad;
    for (int64_t i = 0; i < n; ++i) {
      if (ids[i] == ORC_TOMB) continue;
      uint64_t key = mkkey(orc_dist2(dim, qq, pts + i * dim), ids[i]);
      if (key >= best[k - 1]) continue;
      int j = k - 1;
      while (j > 0 && best[j - 1] > key) {
        best[j] = best[j - 1];
        --j;
      }
      best[j] = key;
    }
    for (int j = 0; j < k; ++j) {
      out_ids[qi * k + j] = key_id(best[j]);
      out_d2[qi * k + j] = key_d2(best[j]);
    }
  }
  free(best);
}

/* ------------------------------------------------------------------------ */
/* Static kd-tree construction (Section IV-A.1, Alg. 1, with the spatial     */
/* median of Section V-C and the leaf coarsening of Section V-D).            */
/* ------------------------------------------------------------------------ */

typedef struct {
  int dim, leaf;
  int rule;          /* ORC_SPLIT_SPATIAL or ORC_SPLIT_OBJECT */
  float* sortbuf;    /* n coordinates, for the object median */
  float* pts;
  uint32_t* ids;
  float* tmp_pts;
  uint32_t* tmp_ids;
  orc_node* nodes;  /* build order; re-laid out afterwards */
  int64_t nn;
  int32_t height;
} build_ctx;

static int cmp_f32(const void* a, const void* b) {
  float x = *(const float*)a, y = *(const float*)b;
  return (x > y) - (x < y);
}

/* Recursive build.  A node is a leaf when it holds at most leaf_size
 * points, when all its points coincide, or at depth ORC_MAX_DEPTH (reading:
 * coarsened leaves of Section V-D; the depth cap bounds the tree height for
 * inputs with near-coincident points).  Otherwise the split dimension is
 * depth mod d, moved forward to the first dimension with non-zero extent
 * (reading of the dimension rotation in Alg. 1), the split value comes from
 * one of the two heuristics of Section V-C, and the node's points are
 * partitioned stably into {x < split} then {x >= split} (the partition
 * primitive of Section III-D).
 *  - spatial median: the midpoint of the tight extent in that dimension;
 *  - object median: the true median of the node's coordinates in that
 *    dimension, found by sorting them (the paper sorts).  Reading: for
 *    count points the median is the coordinate of rank floor(count/2)
 *    (0-based, ascending), so that distinct coordinates split into
 *    floor(count/2) points below it and the rest at or above it.
 * Either way, a split that would leave the left side empty (the value equals
 * the minimum: adjacent floats for the midpoint, or more than half of the
 * points sharing the minimum for the median) or an overflowing midpoint is
 * replaced by the maximum, and a zero split is stored as +0 (like boxes). */
static int32_t build_rec(build_ctx* b, int64_t begin, int64_t count, int depth,
                         uint64_t path, int32_t parent) {
  const int d = b->dim;
  int32_t me = (int32_t)b->nn++;
  orc_node* nd = &b->nodes[me];
  memset(nd, 0, sizeof(*nd));
  nd->depth = depth;
  nd->path = path;
  nd->parent = parent;
  nd->begin = (int32_t)begin;
  nd->count = (int32_t)count;
  nd->left = nd->right = -1;
  nd->dim = -1;
  if (depth + 1 > b->height) b->height = depth + 1;

  /* tight bounding box */
  for (int j = 0; j < d; ++j) {
    nd->lo[j] = box_val(b->pts[begin * d + j]);
    nd->hi[j] = nd->lo[j];
  }
  for (int64_t i = begin + 1; i < begin + count; ++i) {
    for (int j = 0; j < d; ++j) {
      float x = box_val(b->pts[i * d + j]);
      if (x < nd->lo[j]) nd->lo[j] = x;
      if (x > nd->hi[j]) nd->hi[j] = x;
    }
  }
  int degenerate = 1;
  for (int j = 0; j < d; ++j)
    if (nd->hi[j] > nd->lo[j]) degenerate = 0;
  if (count <= b->leaf || degenerate || depth >= ORC_MAX_DEPTH) return me;

  int c = depth % d;
  while (!(nd->hi[c] > nd->lo[c])) c = (c + 1) % d;
  float mn = nd->lo[c], mx = nd->hi[c];
  float split;
  if (b->rule == ORC_SPLIT_OBJECT) {
    for (int64_t i = 0; i < count; ++i) b->sortbuf[i] = b->pts[(begin + i) * d + c];
    qsort(b->sortbuf, (size_t)count, sizeof(float), cmp_f32);
    split = box_val(b->sortbuf[count / 2]);
  } else {
    split = (mn + mx) * 0.5f;
  }
  /* reading: if the split is not above mn (adjacent floats, or more than
   * half of the points at the minimum) or the midpoint overflows, split at
   * mx so that neither side is empty */
  if (!(split > mn) || split > mx) split = mx;
  nd->dim = c;
  nd->split = split;

  /* stable partition of [begin, begin+count) */
  int64_t nl = 0;
  for (int64_t i = begin; i < begin + count; ++i) {
    if (b->pts[i * d + c] < split) {
      memcpy(b->tmp_pts + nl * d, b->pts + i * d, sizeof(float) * d);
      b->tmp_ids[nl] = b->ids[i];
      ++nl;
    }
  }
  int64_t w = nl;
  for (int64_t i = begin; i < begin + count; ++i) {
    if (!(b->pts[i * d + c] < split)) {
      memcpy(b->tmp_pts + w * d, b->pts + i * d, sizeof(float) * d);
      b->tmp_ids[w] = b->ids[i];
      ++w;
    }
  }
  memcpy(b->pts + begin * d, b->tmp_pts, sizeof(float) * d * count);
  memcpy(b->ids + begin, b->tmp_ids, sizeof(uint32_t) * count);

  int32_t l = build_rec(b, begin, nl, depth + 1, path << 1, me);
  int32_t r = build_rec(b, begin + nl, count - nl, depth + 1, (path << 1) | 1u, me);
  b->nodes[me].left = l;
  b->nodes[me].right = r;
  return me;
}

/* vEB layout (Section IV-A.1, Alg. 1): a tree of l levels is stored as its
 * top l_t levels (recursively laid out) followed by the subtrees rooted at
 * depth l_t, left to right, each laid out recursively with l_b levels.
 * Reading of the garbled formula: l_b = hyperceiling(floor((l+1)/2)) and
 * l_t = l - l_b, which reproduces the worked example of Fig. 3 (l = 4 gives
 * l_b = l_t = 2).  A spatial-median tree is not complete; the recursion is
 * applied to the tree's height and simply skips absent nodes, so nodes keep
 * the relative order they would have in the complete tree. */
static int hyperceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

typedef struct {
  const orc_node* nodes;
  int32_t* order;
  int64_t no;
} veb_ctx;

static void veb_place(veb_ctx* v, int32_t r, int l);

static void veb_bottoms(veb_ctx* v, int32_t s, int rel, int lt, int lb) {
  if (rel == lt) {
    veb_place(v, s, lb);
    return;
  }
  if (v->nodes[s].dim < 0) return;
  veb_bottoms(v, v->nodes[s].left, rel + 1, lt, lb);
  veb_bottoms(v, v->nodes[s].right, rel + 1, lt, lb);
}

static void veb_place(veb_ctx* v, int32_t r, int l) {
  if (l == 1) {
    v->order[v->no++] = r;
    return;
  }
  int lb = hyperceil((l + 1) / 2);
  int lt = l - lb;
  veb_place(v, r, lt);
  veb_bottoms(v, r, 0, lt, lb);
}

int64_t orc_tree_build(int dim, int leaf_size, float* pts, uint32_t* ids, int64_t n,
                       orc_node* nodes_out, int32_t* height_out) {
  return orc_tree_build_rule(dim, leaf_size, ORC_SPLIT_SPATIAL, pts, ids, n, nodes_out,
                             height_out);
}

int64_t orc_tree_build_rule(int dim, int leaf_size, int rule, float* pts, uint32_t* ids,
                            int64_t n, orc_node* nodes_out, int32_t* height_out) {
  if (height_out) *height_out = 0;
  if (n <= 0) return 0;
  build_ctx b;
  b.dim = dim;
  b.leaf = leaf_size;
  b.rule = rule;
  b.sortbuf = rule == ORC_SPLIT_OBJECT ? (float*)xmalloc(sizeof(float) * (size_t)n) : NULL;
  b.pts = pts;
  b.ids = ids;
  b.tmp_pts = (float*)xmalloc(sizeof(float) * (size_t)(n * dim));
  b.tmp_ids = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)n);
  b.nodes = (orc_node*)xmalloc(sizeof(orc_node) * (size_t)(2 * n - 1));
  b.nn = 0;
  b.height = 0;
  build_rec(&b, 0, n, 0, 0, -1);

  veb_ctx v;
  v.nodes = b.nodes;
  v.order = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)b.nn);
  v.no = 0;
  veb_place(&v, 0, b.height);
  if (v.no != b.nn) {
    fprintf(stderr, "bdl_oracle: vEB layout placed %lld of %lld nodes\n",
            (long long)v.no, (long long)b.nn);
    abort();
  }
  int32_t* pos = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)b.nn);
  for (int64_t i = 0; i < b.nn; ++i) pos[v.order[i]] = (int32_t)i;
  for (int64_t i = 0; i < b.nn; ++i) {
    orc_node nd = b.nodes[v.order[i]];
    if (nd.left >= 0) nd.left = pos[nd.left];
    if (nd.right >= 0) nd.right = pos[nd.right];
    if (nd.parent >= 0) nd.parent = pos[nd.parent];
    nodes_out[i] = nd;
  }
  if (height_out) *height_out = b.height;
  int64_t nn = b.nn;
  free(pos);
  free(v.order);
  free(b.nodes);
  free(b.tmp_pts);
  free(b.tmp_ids);
  free(b.sortbuf);
  return nn;
}

/* ------------------------------------------------------------------------ */
/* The log structure (Section III-C, Section IV-B)                           */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t n;       /* slots (points at build time) */
  int64_t live;    /* slots whose id is not ORC_TOMB */
  float* pts;      /* n * dim, slot order */
  uint32_t* ids;   /* n */
  orc_node* nodes; /* vEB order */
  int64_t n_nodes;
  int32_t height;
} orc_tree;

struct orc_bdl {
  int dim, leaf, X;
  int rule;                /* split heuristic of every tree */
  int mode;                /* ORC_MODE_*: the BDL-tree or a baseline */
  uint64_t F;              /* bit i set iff static tree i is non-empty */
  orc_tree lev[ORC_MAXLEV];
  /* buffer region: arrival-order pool of fewer than X points and a kd-tree
   * over it */
  float* bpts;
  uint32_t* bids;
  int64_t bn;
  orc_tree btree;
  int64_t rebuilt;         /* points passed to static-tree builds */
  int64_t reinserted;      /* points moved by Erase_L rebalancing */
};

static void tree_free(orc_tree* tr) {
  free(tr->pts);
  free(tr->ids);
  free(tr->nodes);
  memset(tr, 0, sizeof(*tr));
}

/* Takes ownership of pts/ids (n points in gather order) and builds. */
static void tree_make(const orc_bdl* t, orc_tree* tr, float* pts, uint32_t* ids,
                      int64_t n) {
  tree_free(tr);
  tr->n = n;
  tr->live = n;
  tr->pts = pts;
  tr->ids = ids;
  if (n > 0) {
    tr->nodes = (orc_node*)xmalloc(sizeof(orc_node) * (size_t)(2 * n - 1));
    tr->n_nodes = orc_tree_build_rule(t->dim, t->leaf, t->rule, pts, ids, n, tr->nodes,
                                      &tr->height);
  }
}

static int64_t level_cap(const orc_bdl* t, int i) { return ((int64_t)1 << i) * t->X; }

orc_bdl* orc_create(int dim, int leaf_size, int buffer_size) {
  if (dim < 1 || dim > ORC_MAXD || leaf_size < 1 || buffer_size < 1) return NULL;
  orc_bdl* t = (orc_bdl*)xmalloc(sizeof(orc_bdl));
  memset(t, 0, sizeof(*t));
  t->dim = dim;
  t->leaf = leaf_size;
  t->X = buffer_size;
  t->rule = ORC_SPLIT_SPATIAL;
  t->mode = ORC_MODE_BDL;
  return t;
}

int orc_set_mode(orc_bdl* t, int mode) {
  if (mode != ORC_MODE_BDL && mode != ORC_MODE_REBUILD_ALL && mode != ORC_MODE_NO_REBUILD)
    return -1;
  if (t->F || t->bn) return -1;
  t->mode = mode;
  return 0;
}

int orc_set_split_rule(orc_bdl* t, int rule) {
  if (rule != ORC_SPLIT_SPATIAL && rule != ORC_SPLIT_OBJECT) return -1;
  if (t->F || t->bn) return -1;
  t->rule = rule;
  return 0;
}

void orc_destroy(orc_bdl* t) {
  if (!t) return;
  for (int i = 0; i < ORC_MAXLEV; ++i) tree_free(&t->lev[i]);
  tree_free(&t->btree);
  free(t->bpts);
  free(t->bids);
  free(t);
}

static void rebuild_buffer_tree(orc_bdl* t) {
  const int d = t->dim;
  float* p = (float*)xmalloc(sizeof(float) * (size_t)(t->bn * d));
  uint32_t* ids = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)t->bn);
  memcpy(p, t->bpts, sizeof(float) * (size_t)(t->bn * d));
  memcpy(ids, t->bids, sizeof(uint32_t) * (size_t)t->bn);
  tree_make(t, &t->btree, p, ids, t->bn);
}

/* ------------------------------------------------------------------------ */
/* The two baselines of Section III-B (B1 and B2 of Section VI): one kd-tree  */
/* over all live points, kept as static tree 0 (F = 1 while it holds slots);  */
/* no buffer.                                                                */
/* ------------------------------------------------------------------------ */

/* Copies of the live points of tree 0 in slot order followed by pts/ids. */
static int64_t gather_live_plus(const orc_bdl* t, const float* pts, const uint32_t* ids,
                                int64_t n, float** out_p, uint32_t** out_i) {
  const int d = t->dim;
  const orc_tree* tr = &t->lev[0];
  int64_t tot = n + ((t->F & 1u) ? tr->live : 0);
  float* p = (float*)xmalloc(sizeof(float) * (size_t)(tot * d));
  uint32_t* id = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)tot);
  int64_t w = 0;
  if (t->F & 1u) {
    for (int64_t s = 0; s < tr->n; ++s) {
      if (tr->ids[s] == ORC_TOMB) continue;
      memcpy(p + w * d, tr->pts + s * d, sizeof(float) * d);
      id[w++] = tr->ids[s];
    }
  }
  if (n > 0) {
    memcpy(p + w * d, pts, sizeof(float) * (size_t)(n * d));
    memcpy(id + w, ids, sizeof(uint32_t) * (size_t)n);
  }
  *out_p = p;
  *out_i = id;
  return tot;
}

/* B1: the tree is rebuilt after every batch update (Section III-B).  Reading:
 * the rebuild takes the old tree's live points in slot order followed by the
 * batch in input order. */
static void b1_rebuild(orc_bdl* t, const float* pts, const uint32_t* ids, int64_t n) {
  float* p;
  uint32_t* id;
  int64_t tot = gather_live_plus(t, pts, ids, n, &p, &id);
  if (tot == 0) {
    free(p);
    free(id);
    tree_free(&t->lev[0]);
    t->F = 0;
    return;
  }
  tree_make(t, &t->lev[0], p, id, tot);
  t->F = 1;
  t->rebuilt += tot;
}

/* B2: the tree keeps the spatial partition of its first build; a batch is
 * inserted into the existing structure (Section III-B).  Each new point
 * follows the splits (x[dim] < split goes left) to a leaf, which takes it
 * after its own points (input order among the new ones); the boxes on its
 * path grow to contain it, so every box still bounds its subtree.  The slots
 * are then laid out again, leaves in their order.  Erased points stay as
 * tombstones (nothing is ever rebuilt). */
typedef struct {
  int64_t* cnt;    /* new points per node (leaves only) */
  int64_t* start;  /* first index into the bucket array per leaf */
  int64_t* bucket; /* new point indices grouped by leaf, input order */
  float* np;
  uint32_t* ni;
  int64_t w;
} b2_ctx;

static void b2_layout(const orc_bdl* t, orc_tree* tr, b2_ctx* c, const float* pts,
                      const uint32_t* ids, int32_t v) {
  const int d = t->dim;
  orc_node* nd = &tr->nodes[v];
  if (nd->dim < 0) {
    const int64_t b = c->w;
    for (int64_t s = nd->begin; s < (int64_t)nd->begin + nd->count; ++s) {
      memcpy(c->np + c->w * d, tr->pts + s * d, sizeof(float) * d);
      c->ni[c->w++] = tr->ids[s];
    }
    for (int64_t k = 0; k < c->cnt[v]; ++k) {
      const int64_t i = c->bucket[c->start[v] + k];
      memcpy(c->np + c->w * d, pts + i * d, sizeof(float) * d);
      c->ni[c->w++] = ids[i];
    }
    nd->begin = (int32_t)b;
    nd->count = (int32_t)(c->w - b);
    return;
  }
  b2_layout(t, tr, c, pts, ids, nd->left);
  b2_layout(t, tr, c, pts, ids, nd->right);
  nd->begin = tr->nodes[nd->left].begin;
  nd->count = tr->nodes[nd->left].count + tr->nodes[nd->right].count;
}

static void b2_insert(orc_bdl* t, const float* pts, const uint32_t* ids, int64_t n) {
  const int d = t->dim;
  if (n <= 0) return;
  if (!(t->F & 1u)) {
    b1_rebuild(t, pts, ids, n);  /* the first batch builds the tree */
    return;
  }
  orc_tree* tr = &t->lev[0];
  int64_t* leaf = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)n);
  b2_ctx c;
  c.cnt = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)tr->n_nodes);
  c.start = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)tr->n_nodes);
  memset(c.cnt, 0, sizeof(int64_t) * (size_t)tr->n_nodes);
  for (int64_t i = 0; i < n; ++i) {
    const float* p = pts + i * d;
    int32_t v = 0;
    while (1) {
      orc_node* nd = &tr->nodes[v];
      for (int j = 0; j < d; ++j) {
        float x = box_val(p[j]);
        if (x < nd->lo[j]) nd->lo[j] = x;
        if (x > nd->hi[j]) nd->hi[j] = x;
      }
      if (nd->dim < 0) break;
      v = p[nd->dim] < nd->split ? nd->left : nd->right;
    }
    leaf[i] = v;
    c.cnt[v]++;
  }
  int64_t run = 0;
  for (int64_t v = 0; v < tr->n_nodes; ++v) {
    c.start[v] = run;
    run += c.cnt[v];
  }
  c.bucket = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)n);
  int64_t* fill = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)tr->n_nodes);
  memset(fill, 0, sizeof(int64_t) * (size_t)tr->n_nodes);
  for (int64_t i = 0; i < n; ++i) c.bucket[c.start[leaf[i]] + fill[leaf[i]]++] = i;
  c.np = (float*)xmalloc(sizeof(float) * (size_t)((tr->n + n) * d));
  c.ni = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)(tr->n + n));
  c.w = 0;
  b2_layout(t, tr, &c, pts, ids, 0);
  free(tr->pts);
  free(tr->ids);
  tr->pts = c.np;
  tr->ids = c.ni;
  tr->n += n;
  tr->live += n;
  free(leaf);
  free(fill);
  free(c.cnt);
  free(c.start);
  free(c.bucket);
}

/* Insert_L (Alg. 3 and the text that follows it).
 * Readings of what the paper leaves open:
 *  - the pool is the buffer's points in arrival order followed by P in input
 *    order; floor(|pool|/X) whole chunks go to static trees and the last
 *    |pool| mod X points stay in the buffer (this reproduces Fig. 4);
 *  - F_new = F + floor(|pool|/X); new trees J = F_new \ F, cleared C = F \ F_new;
 *  - the highest new tree takes every live point of the cleared trees (in
 *    ascending tree, then slot order) followed by the leading pool slice that
 *    fills its nominal capacity 2^j X; the other new trees, highest first, take
 *    the following pool slices of 2^j X points each. */
int orc_insert(orc_bdl* t, const float* pts, const uint32_t* ids, int64_t n) {
  if (t->mode == ORC_MODE_REBUILD_ALL) {
    if (n > 0) b1_rebuild(t, pts, ids, n);
    return 0;
  }
  if (t->mode == ORC_MODE_NO_REBUILD) {
    b2_insert(t, pts, ids, n);
    return 0;
  }
  const int d = t->dim;
  const int64_t X = t->X;
  int64_t pn = t->bn + n;
  float* pool = (float*)xmalloc(sizeof(float) * (size_t)(pn * d));
  uint32_t* pid = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)pn);
  memcpy(pool, t->bpts, sizeof(float) * (size_t)(t->bn * d));
  memcpy(pid, t->bids, sizeof(uint32_t) * (size_t)t->bn);
  if (n > 0) {
    memcpy(pool + t->bn * d, pts, sizeof(float) * (size_t)(n * d));
    memcpy(pid + t->bn, ids, sizeof(uint32_t) * (size_t)n);
  }
  uint64_t m = (uint64_t)(pn / X);
  uint64_t Fn = t->F + m;
  uint64_t J = Fn & ~t->F;
  uint64_t C = t->F & ~Fn;
  int64_t off = 0;
  if (J) {
    int js = 63;
    while (!((J >> js) & 1u)) --js;
    /* highest new tree: gathered live points of cleared trees + pool slice */
    int64_t ccap = 0, clive = 0;
    for (int i = 0; i < ORC_MAXLEV; ++i)
      if ((C >> i) & 1u) {
        ccap += level_cap(t, i);
        clive += t->lev[i].live;
      }
    int64_t slice = level_cap(t, js) - ccap;
    int64_t tot = clive + slice;
    float* np_ = (float*)xmalloc(sizeof(float) * (size_t)(tot * d));
    uint32_t* ni = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)tot);
    int64_t w = 0;
    for (int i = 0; i < ORC_MAXLEV; ++i) {
      if (!((C >> i) & 1u)) continue;
      orc_tree* tr = &t->lev[i];
      for (int64_t s = 0; s < tr->n; ++s) {
        if (tr->ids[s] == ORC_TOMB) continue;
        memcpy(np_ + w * d, tr->pts + s * d, sizeof(float) * d);
        ni[w] = tr->ids[s];
        ++w;
      }
      tree_free(tr);
    }
    memcpy(np_ + w * d, pool + off * d, sizeof(float) * (size_t)(slice * d));
    memcpy(ni + w, pid + off, sizeof(uint32_t) * (size_t)slice);
    off += slice;
    tree_make(t, &t->lev[js], np_, ni, tot);
    t->rebuilt += tot;
    for (int j = js - 1; j >= 0; --j) {
      if (!((J >> j) & 1u)) continue;
      int64_t c = level_cap(t, j);
      float* p2 = (float*)xmalloc(sizeof(float) * (size_t)(c * d));
      uint32_t* i2 = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)c);
      memcpy(p2, pool + off * d, sizeof(float) * (size_t)(c * d));
      memcpy(i2, pid + off, sizeof(uint32_t) * (size_t)c);
      off += c;
      tree_make(t, &t->lev[j], p2, i2, c);
      t->rebuilt += c;
    }
  }
  /* the remaining pool tail becomes the buffer */
  int64_t bn = pn - off;
  float* bp = (float*)xmalloc(sizeof(float) * (size_t)(bn * d));
  uint32_t* bi = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)bn);
  memcpy(bp, pool + off * d, sizeof(float) * (size_t)(bn * d));
  memcpy(bi, pid + off, sizeof(uint32_t) * (size_t)bn);
  free(t->bpts);
  free(t->bids);
  t->bpts = bp;
  t->bids = bi;
  t->bn = bn;
  rebuild_buffer_tree(t);
  t->F = Fn;
  free(pool);
  free(pid);
  return 0;
}

/* Erase_S for one point (Alg. 2): route the point down the tree by the split
 * at each node (a stored point p sits in the left subtree iff
 * p[dim] < split), then mark a matching slot in the leaf as deleted.  A
 * match needs the same id and bitwise-equal coordinates (reading: points are
 * identified by caller ids).  Nodes are left in place (reading: splicing out
 * emptied nodes changes no result). */
static int erase_in_tree(const orc_bdl* t, orc_tree* tr, const float* p, uint32_t id) {
  if (tr->n_nodes == 0) return 0;
  const int d = t->dim;
  int32_t ni = 0;
  while (tr->nodes[ni].dim >= 0) {
    const orc_node* nd = &tr->nodes[ni];
    ni = (p[nd->dim] < nd->split) ? nd->left : nd->right;
  }
  const orc_node* lf = &tr->nodes[ni];
  for (int64_t s = lf->begin; s < (int64_t)lf->begin + lf->count; ++s) {
    if (tr->ids[s] == id && memcmp(tr->pts + s * d, p, sizeof(float) * d) == 0) {
      tr->ids[s] = ORC_TOMB;
      tr->live -= 1;
      return 1;
    }
  }
  return 0;
}

/* Erase_L (Alg. 4): erase from every non-empty tree and from the buffer,
 * then gather every static tree whose live count fell strictly below half of
 * its nominal capacity 2^i X (reading of "below half of their original
 * capacity") into R, in ascending tree then slot order, clear those trees,
 * and Insert_L(R).  The buffer has no half rule; it keeps its arrival order
 * and shrinks. */
int64_t orc_erase(orc_bdl* t, const float* pts, const uint32_t* ids, int64_t n) {
  const int d = t->dim;
  int64_t erased = 0;
  if (t->mode != ORC_MODE_BDL) {
    /* baselines: tombstone in the one tree; B1 then rebuilds from the
     * survivors (if anything was erased), B2 never does */
    for (int64_t e = 0; e < n; ++e)
      if (ids[e] != ORC_TOMB && (t->F & 1u))
        erased += erase_in_tree(t, &t->lev[0], pts + e * d, ids[e]);
    if (t->mode == ORC_MODE_REBUILD_ALL && erased > 0) b1_rebuild(t, NULL, NULL, 0);
    return erased;
  }
  int buffer_hit = 0;
  for (int64_t e = 0; e < n; ++e) {
    const float* p = pts + e * d;
    uint32_t id = ids[e];
    if (id == ORC_TOMB) continue;
    int done = 0;
    for (int i = 0; i < ORC_MAXLEV && !done; ++i)
      if ((t->F >> i) & 1u) done = erase_in_tree(t, &t->lev[i], p, id);
    if (!done) {
      for (int64_t s = 0; s < t->bn; ++s) {
        if (t->bids[s] == id && memcmp(t->bpts + s * d, p, sizeof(float) * d) == 0) {
          t->bids[s] = ORC_TOMB;
          done = 1;
          buffer_hit = 1;
          break;
        }
      }
    }
    erased += done;
  }
  if (buffer_hit) {
    int64_t w = 0;
    for (int64_t s = 0; s < t->bn; ++s) {
      if (t->bids[s] == ORC_TOMB) continue;
      memmove(t->bpts + w * d, t->bpts + s * d, sizeof(float) * d);
      t->bids[w] = t->bids[s];
      ++w;
    }
    t->bn = w;
    rebuild_buffer_tree(t);
  }
  int64_t rn = 0;
  for (int i = 0; i < ORC_MAXLEV; ++i)
    if (((t->F >> i) & 1u) && 2 * t->lev[i].live < level_cap(t, i)) rn += t->lev[i].live;
  float* rp = (float*)xmalloc(sizeof(float) * (size_t)(rn * d));
  uint32_t* ri = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)rn);
  int64_t w = 0;
  for (int i = 0; i < ORC_MAXLEV; ++i) {
    if (!(((t->F >> i) & 1u) && 2 * t->lev[i].live < level_cap(t, i))) continue;
    orc_tree* tr = &t->lev[i];
    for (int64_t s = 0; s < tr->n; ++s) {
      if (tr->ids[s] == ORC_TOMB) continue;
      memcpy(rp + w * d, tr->pts + s * d, sizeof(float) * d);
      ri[w] = tr->ids[s];
      ++w;
    }
    tree_free(tr);
    t->F &= ~((uint64_t)1 << i);
  }
  if (rn > 0) {
    orc_insert(t, rp, ri, rn);
    t->reinserted += rn;
  }
  free(rp);
  free(ri);
  return erased;
}

/* ------------------------------------------------------------------------ */
/* k-NN (Section IV-A.3 for one tree, Alg. 5 over the log structure)         */
/* ------------------------------------------------------------------------ */

/* The k-NN buffer of Section IV-A.3: 2k slots, appends, and when full a
 * selection keeps the k smallest keys.  The selection here is a sort. */
typedef struct {
  uint64_t* key;
  int n, k;
} kbuf;

static void kb_compact(kbuf* b) {
  qsort(b->key, (size_t)b->n, sizeof(uint64_t), cmp_u64);
  if (b->n > b->k) b->n = b->k;
}

static void kb_add(kbuf* b, uint64_t key) {
  b->key[b->n++] = key;
  if (b->n == 2 * b->k) kb_compact(b);
}

static int kb_full(const kbuf* b) { return b->n >= b->k; }

static float kb_worst_d2(kbuf* b) {
  kb_compact(b);
  return key_d2(b->key[b->k - 1]);
}

typedef struct {
  int dim;
  const float* q;
  const orc_tree* tr;
  kbuf* kb;
  orc_counters* cnt;
} kctx;

static float mindist2(int d, const float* q, const orc_node* nd) {
  float acc = 0.0f;
  for (int j = 0; j < d; ++j) {
    float a = nd->lo[j] - q[j];
    float b = q[j] - nd->hi[j];
    float t = a > 0.0f ? a : (b > 0.0f ? b : 0.0f);
    acc = fmaf(t, t, acc);
  }
  return acc;
}

static float maxdist2(int d, const float* q, const orc_node* nd) {
  float acc = 0.0f;
  for (int j = 0; j < d; ++j) {
    float a = fabsf(q[j] - nd->lo[j]);
    float b = fabsf(q[j] - nd->hi[j]);
    float t = a > b ? a : b;
    acc = fmaf(t, t, acc);
  }
  return acc;
}

/* every live point in the subtree's contiguous slot range */
static void add_all(kctx* x, const orc_node* nd) {
  const int d = x->dim;
  for (int64_t s = nd->begin; s < (int64_t)nd->begin + nd->count; ++s) {
    uint32_t id = x->tr->ids[s];
    if (id == ORC_TOMB) continue;
    x->cnt->dist_evals++;
    kb_add(x->kb, mkkey(orc_dist2(d, x->q, x->tr->pts + s * d), id));
  }
}

/* kNN_S for one query (Section IV-A.3): descend to the leaf that q falls in
 * and add its points; while unwinding, if the buffer holds fewer than k
 * points add every point of the sibling subtree; otherwise prune the sibling
 * if its box lies entirely outside the current k-th distance, add all of it
 * if the box lies entirely inside, and recurse into it if they intersect.
 * Reading: "outside" is the strict test mindist^2 > worst^2, so a point tied
 * at the k-th distance with a smaller id is never pruned. */
static void knn_rec(kctx* x, int32_t ni) {
  const orc_node* nd = &x->tr->nodes[ni];
  x->cnt->node_visits++;
  if (nd->dim < 0) {
    add_all(x, nd);
    return;
  }
  int32_t near_ = (x->q[nd->dim] < nd->split) ? nd->left : nd->right;
  int32_t far_ = (near_ == nd->left) ? nd->right : nd->left;
  knn_rec(x, near_);
  const orc_node* fn = &x->tr->nodes[far_];
  if (!kb_full(x->kb)) {
    x->cnt->node_visits++;
    add_all(x, fn);
    return;
  }
  float w = kb_worst_d2(x->kb);
  if (mindist2(x->dim, x->q, fn) > w) return;
  if (maxdist2(x->dim, x->q, fn) <= w) {
    x->cnt->node_visits++;
    add_all(x, fn);
    return;
  }
  knn_rec(x, far_);
}

/* kNN_L (Alg. 5) for one query: one k-NN buffer shared by every non-empty
 * tree; trees are visited one after another from the largest to the smallest
 * (Section V-B), then the buffer tree.  Writes the row of k (id, d2). */
static void knn_one(const orc_bdl* t, const float* qrow, int k, kbuf* kb, orc_counters* cnt,
                    uint32_t* out_ids, float* out_d2) {
  const uint64_t pad = mkkey(INFINITY, ORC_TOMB);
  kb->n = 0;
  kctx x;
  x.dim = t->dim;
  x.q = qrow;
  x.kb = kb;
  x.cnt = cnt;
  for (int i = ORC_MAXLEV - 1; i >= 0; --i) {
    if (!((t->F >> i) & 1u) || t->lev[i].n_nodes == 0) continue;
    x.tr = &t->lev[i];
    knn_rec(&x, 0);
  }
  if (t->btree.n_nodes > 0) {
    x.tr = &t->btree;
    knn_rec(&x, 0);
  }
  kb_compact(kb);
  for (int j = 0; j < k; ++j) {
    uint64_t key = j < kb->n ? kb->key[j] : pad;
    out_ids[j] = key_id(key);
    out_d2[j] = key_d2(key);
  }
}

/* kNN_L (Alg. 5) over a batch of queries, one after another. */
void orc_knn(orc_bdl* t, const float* q, int64_t nq, int k, uint32_t* out_ids,
             float* out_d2, orc_counters* cnt) {
  orc_counters local = {0, 0};
  if (!cnt) cnt = &local;
  kbuf kb;
  kb.key = (uint64_t*)xmalloc(sizeof(uint64_t) * (size_t)(2 * k));
  kb.k = k;
  for (int64_t qi = 0; qi < nq; ++qi)
    knn_one(t, q + qi * t->dim, k, &kb, cnt, out_ids + qi * k, out_d2 + qi * k);
  free(kb.key);
}

/* The same batch with the queries spread over host threads (OpenMP): the
 * data-parallel k-NN of Section IV-A.3 runs each query's search serially and
 * parallelizes across queries.  Each thread has its own k-NN buffer and
 * counters; rows are those of orc_knn.  Returns the number of threads used. */
int orc_knn_parallel(orc_bdl* t, const float* q, int64_t nq, int k, uint32_t* out_ids,
                     float* out_d2, orc_counters* cnt) {
  int used = 1;
  int64_t nodes = 0, evals = 0;
#pragma omp parallel reduction(+ : nodes, evals)
  {
    orc_counters c = {0, 0};
    kbuf kb;
    kb.key = (uint64_t*)xmalloc(sizeof(uint64_t) * (size_t)(2 * k));
    kb.k = k;
#ifdef _OPENMP
#pragma omp single
    used = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 256)
    for (int64_t qi = 0; qi < nq; ++qi)
      knn_one(t, q + qi * t->dim, k, &kb, &c, out_ids + qi * k, out_d2 + qi * k);
    free(kb.key);
    nodes += c.node_visits;
    evals += c.dist_evals;
  }
  if (cnt) {
    cnt->node_visits += nodes;
    cnt->dist_evals += evals;
  }
  return used;
}

/* ------------------------------------------------------------------------ */
/* inspection                                                                */
/* ------------------------------------------------------------------------ */

int64_t orc_size(const orc_bdl* t) {
  int64_t s = t->bn;
  for (int i = 0; i < ORC_MAXLEV; ++i)
    if ((t->F >> i) & 1u) s += t->lev[i].live;
  return s;
}

void orc_level_info(const orc_bdl* t, int32_t* nlev, int64_t* live, int64_t* cap,
                    int64_t* n_slots, int64_t* buf_live, uint64_t* F,
                    int64_t* rebuilt_points, int64_t* reinserted_points) {
  int top = 0;
  for (int i = 0; i < ORC_MAXLEV; ++i)
    if ((t->F >> i) & 1u) top = i + 1;
  if (nlev) *nlev = top;
  for (int i = 0; i < top; ++i) {
    int on = (int)((t->F >> i) & 1u);
    if (live) live[i] = on ? t->lev[i].live : 0;
    if (cap) cap[i] = level_cap(t, i);
    if (n_slots) n_slots[i] = on ? t->lev[i].n : 0;
  }
  if (buf_live) *buf_live = t->bn;
  if (F) *F = t->F;
  if (rebuilt_points) *rebuilt_points = t->rebuilt;
  if (reinserted_points) *reinserted_points = t->reinserted;
}

int orc_export_level(const orc_bdl* t, int32_t level, uint32_t* ids, float* pts,
                     orc_node* nodes, int64_t* n_slots, int64_t* n_nodes) {
  const orc_tree* tr;
  if (level == -1) {
    tr = &t->btree;
  } else {
    if (level < 0 || level >= ORC_MAXLEV || !((t->F >> level) & 1u)) {
      if (n_slots) *n_slots = 0;
      if (n_nodes) *n_nodes = 0;
      return -1;
    }
    tr = &t->lev[level];
  }
  if (n_slots) *n_slots = tr->n;
  if (n_nodes) *n_nodes = tr->n_nodes;
  if (ids) memcpy(ids, tr->ids, sizeof(uint32_t) * (size_t)tr->n);
  if (pts) memcpy(pts, tr->pts, sizeof(float) * (size_t)(tr->n * t->dim));
  if (nodes) memcpy(nodes, tr->nodes, sizeof(orc_node) * (size_t)tr->n_nodes);
  return 0;
}

int32_t orc_sizeof_node(void) { return (int32_t)sizeof(orc_node); }

int orc_export_buffer_pool(const orc_bdl* t, uint32_t* ids, float* pts, int64_t* n) {
  if (n) *n = t->bn;
  if (ids) memcpy(ids, t->bids, sizeof(uint32_t) * (size_t)t->bn);
  if (pts) memcpy(pts, t->bpts, sizeof(float) * (size_t)(t->bn * t->dim));
  return 0;
}
