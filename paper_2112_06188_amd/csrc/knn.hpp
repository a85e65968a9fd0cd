// Host launchers of the batched k-NN query (kNN_L, Alg. 5).
#pragma once

#include "bdl_common.hpp"

namespace bdl {

// Scratch for ordering a query batch spatially (Morton order).
struct QueryScratch {
  uint64_t cap = 0;
  uint32_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint32_t* tmp = nullptr;
  uint32_t* box = nullptr;  // 2 * kMaxDim ordered-u32 bounds
};

size_t query_scratch_bytes(uint64_t cap);

// Batches of at least this many queries are visited in Morton order.
constexpr uint64_t kSortQueriesMin = 4096;

// kNN_L over the given trees (visited in the given order).  order may be
// null (queries in input order).  Returns 0 or a BDL_E* code.
// Traversal variants: one lane per query, or one wavefront per group of 64
// neighbouring queries.
constexpr int kKnnLane = 0;
constexpr int kKnnWave = 1;

// err (device) receives a nonzero bit if a tree index is out of range.
// stats (device, may be null) accumulates, per query, nodes entered, leaves
// scanned and points whose distance was evaluated.
int launch_knn(int mode, int d, int k, const float* q, uint64_t nq, const LevelViews& views,
               const uint32_t* order, uint32_t* out_ids, float* out_d2, uint32_t* err,
               unsigned long long* stats, hipStream_t s);

// Compute a Morton order of the queries; returns the device array holding
// the permutation (inside qs).
const uint32_t* morton_order(int d, const float* q, uint64_t nq, QueryScratch& qs,
                             hipStream_t s);

}  // namespace bdl
