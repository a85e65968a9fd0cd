// Host launchers of the batched k-NN query (kNN_L, Alg. 5).
#pragma once

#include "bdl_common.hpp"

namespace bdl {

// Scratch for ordering a query batch spatially (Hilbert-curve order).
struct QueryScratch {
  uint64_t cap = 0;
  uint32_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint32_t* tmp = nullptr;
  uint32_t* box = nullptr;  // 2 * kMaxDim ordered-u32 bounds
};

size_t query_scratch_bytes(uint64_t cap);

// Batches of at least this many queries are visited in Hilbert-curve order.
constexpr uint64_t kSortQueriesMin = 4096;

// Traversal variants: one lane per query, or one wavefront per group of 64
// neighbouring queries (128 with two per lane, for d <= 3, k <= 5 and large
// batches).
constexpr int kKnnLane = 0;
constexpr int kKnnWave = 1;
constexpr int kKnnAuto = 2;  // chosen per launch from the query density
constexpr int kKnnQuery = 3;  // one wavefront per query (small batches)
// a tree with this many nodes or more cannot be searched by kKnnQuery
constexpr uint64_t kKnnQueryMaxNodes = 1ull << 26;

// One k-NN request as the kernels see it: its queries, k and outputs, and
// the position of its first query in the concatenated query array.
struct KnnReqDev {
  const float* q;
  uint32_t* out_ids;
  float* out_d2;
  uint64_t qoff;
  uint32_t nq;
  int32_t k;
};

// A set of queries: q holds all of them contiguously ([nq][d]).  When qreq
// is null every query belongs to `one`; otherwise qreq[i] indexes reqs.  The
// count is read from nq_dev when it is not null (graph replays).
struct KnnQueries {
  const float* q;
  const uint64_t* nq_dev;
  uint64_t nq;
  const uint32_t* qreq;
  const KnnReqDev* reqs;
  KnnReqDev one;
};

// Kernel choice and workgroup size (64, 128 or 256).  With `persistent` set
// and a queue given (kKnnQueueWords words of device memory owned by the
// caller, not in use by another launch on another stream), a batch larger
// than the device holds at once runs on a resident grid whose waves draw
// groups of queries from per-XCD counters.  dry_run only prepares the
// launch (occupancy lookups), so that a later launch under stream capture
// makes no such query.
struct KnnLaunch {
  int mode = kKnnWave;
  int block = 256;
  int persistent = 0;
  uint32_t* queue = nullptr;
  bool dry_run = false;
  int qstack = 1 << 30;  // kKnnQuery: pending-node entries per wave (clamped)
};

constexpr int kKnnQueueStride = 64;  // words between the per-XCD counters
constexpr int kKnnQueueWords = 8 * kKnnQueueStride;

// kNN_L over the trees listed in `views` (device memory, visited in order).
// grid_q bounds the number of queries (sizes the grid); order may be null
// (queries in array order).  err (device) receives a nonzero bit if a tree
// index is out of range; stats (device, may be null) accumulates, per query,
// nodes entered, leaves scanned and points evaluated.
int launch_knn(const KnnLaunch& L, int d, int kmax, const KnnQueries& Q, uint64_t grid_q,
               const uint32_t* order, const LevelViews* views, uint32_t* err,
               unsigned long long* stats, hipStream_t s);

// Hilbert-curve order of queries [0, nq) of q, sorting cap >= nq keys (positions
// from nq on sort last).  Returns the device array holding the permutation.
const uint32_t* spatial_order(int d, const float* q, const uint64_t* nq_dev, uint64_t nq_host,
                             uint64_t cap, QueryScratch& qs, hipStream_t s);

// One wavefront's share of a k-NN graph launch: at most 64 consecutive slots
// [begin, begin + count) of tree `view` (an index into LevelViews), all in
// the subtree of node `node` of that tree.
struct GraphGroup {
  uint32_t view, node, begin, count;
};

// Groups a k-NN graph launch needs at most for a tree of n slots: one per
// subtree (at most one per leaf) plus one per further 64 slots.
inline uint64_t graph_group_bound(uint64_t n) { return n + n / 64 + 1; }

// Scratch of a k-NN graph launch for at most `cap` groups: the group list
// and its Hilbert-curve order (sort keys and values, two buffers each, and
// 65536 words of sort scratch).
struct GraphScratch {
  uint64_t cap = 0;
  GraphGroup* groups = nullptr;
  uint64_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint32_t* tmp = nullptr;
};
size_t graph_scratch_bytes(uint64_t cap);

// Orders the *ngroups groups along the Hilbert curve of their first points
// (cells of the largest tree's root box): afterwards vals[*sel] (sel and
// width: one device word each) lists the groups in that order, so that
// neighbouring wavefronts, and each XCD's range of them, work on
// neighbouring regions.
void launch_graph_order(int d, const LevelViews* views, GraphScratch& gs, const uint32_t* ngroups,
                        uint32_t* width, uint32_t* sel, hipStream_t s);

// Appends the groups of tree `view` of `views` (device) to groups (capacity
// cap entries, count in *ngroups, device).  A group's subtree is the highest
// one that holds at most 64 points by the nodes' point counts (or a leaf
// that holds more); its slots are cut into runs of at most 64.  Slots per
// tree at most n_slots (host bound for the grid).  err bit 64 on an
// inconsistent tree or a full list.
void launch_graph_groups(const LevelViews* views, int view, int d, uint64_t n_slots,
                         GraphGroup* groups, uint64_t cap, uint32_t* ngroups, uint32_t* err,
                         hipStream_t s);

// The k-NN graph of the live points of the trees in `views` (device): row
// `id` of out_ids/out_d2 ([idcap][k]) receives the k nearest live points of
// live point `id`, by (squared distance, id), exactly the row kNN_L returns
// for that point as a query; other rows are not written.  The group list
// comes from launch_graph_groups, in the order launch_graph_order left in
// gs.vals[*sel].  queue: kKnnQueueWords words (zeroed here).  stats as
// launch_knn.
int launch_knn_graph(int d, int k, const LevelViews* views, const GraphScratch& gs,
                     const uint32_t* ngroups, const uint32_t* sel, uint32_t* out_ids,
                     float* out_d2, uint32_t idcap, uint32_t* err, unsigned long long* stats,
                     uint32_t* queue, hipStream_t s);

// The other way to the k-NN graph: every live point gathered as a query
// (coordinates [cap][d], ids), ordered along the Hilbert curve and searched
// from the roots by the kNN_L kernels into rows [cap][k], which are then
// moved to row `id` of the caller's outputs.  count: one 64-bit device word.
struct GraphQueries {
  uint64_t cap = 0;      // queries (live points) at most
  uint64_t row_cap = 0;  // result words per array (cap * k for the largest k so far)
  float* q = nullptr;
  uint32_t* ids = nullptr;
  uint32_t* rid = nullptr;
  float* rd2 = nullptr;
  unsigned long long* count = nullptr;
};

// Appends the live points of tree `view` (at most n_slots, host bound) to
// gq.q / gq.ids at positions taken from *gq.count.  err bit 64 if more than
// gq.cap arrive.
void launch_graph_gather(const LevelViews* views, int view, int d, uint64_t n_slots,
                         GraphQueries& gq, uint32_t* err, hipStream_t s);

// Rows [*gq.count][k] of gq.rid / gq.rd2 to rows ids[r] of out ([idcap][k]).
void launch_graph_scatter(const GraphQueries& gq, int k, uint32_t* out_ids, float* out_d2,
                          uint32_t idcap, hipStream_t s);

// Concatenate the queries of counts[1] requests (offsets in reqs[i].qoff,
// counts[0] <= cap queries in all; device memory) into qall and record each
// query's request in qreq.
void launch_gather_queries(const KnnReqDev* reqs, const uint64_t* counts, uint64_t cap, int d,
                           float* qall, uint32_t* qreq, hipStream_t s);

}  // namespace bdl
