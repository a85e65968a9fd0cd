// Host launchers of Erase_L's locate-and-tombstone step and of the optional
// input validation of Insert_L.
#pragma once

#include "bdl_common.hpp"

namespace bdl {

// Where each map entry's (level, slot) points.
struct EraseTable {
  float* rec[kMaxLevels];
  uint32_t nslots[kMaxLevels];
  float* pool;     // the buffer's records in arrival order
  uint32_t bn;
  uint32_t pad_;
};

// What the coordinate-routed erase reads besides the records: each static
// tree's nodes and Bloom filter (2^bloom_log2 words of 64 bits, null for an
// empty tree), the buffer's filter, and the trees' node counts on the
// device (level_nodes[level]).
struct RouteTable {
  const float* nodes[kMaxLevels];
  const uint64_t* bloom[kMaxLevels];
  uint8_t bloom_log2[kMaxLevels];
  const uint64_t* pool_bloom;
  const uint32_t* level_nodes;
  uint32_t pool_bloom_log2;
  uint32_t pad_;
};

// ectr[0] += points erased, ectr[1] += points erased from the buffer,
// live[level] -= points erased from each static tree.
void launch_erase(const float* pts, const uint32_t* ids, uint64_t n, int d, uint64_t* map,
                  uint32_t idcap, const EraseTable& et, uint32_t* live, uint32_t* ectr,
                  hipStream_t s);

// Blocked Bloom filter of the live records [0, n) of a record array: every
// (id, coordinates) sets four bits of one 64-bit word of bloom
// (2^log2 words, cleared first here).
void launch_bloom_build(const float* rec, uint64_t n, int d, uint64_t* bloom, int log2,
                        hipStream_t s);

// Erase_S (Alg. 2) with Bloom prefilters (Section V-A): each pair is tested
// against every static tree's filter, routed from the root of each tree that
// may hold it along the splits to a leaf, and tombstoned there if the leaf
// holds the same id with bitwise-equal coordinates (a compare-and-swap on the
// id, so a repeated id erases once); pairs found in no tree are looked up in
// the buffer (filter, then a scan of its fewer than X records).  The id map
// entry of every erased point is cleared.  Counters as launch_erase.
void launch_erase_routed(const float* pts, const uint32_t* ids, uint64_t n, int d,
                         uint64_t* map, uint32_t idcap, const EraseTable& et,
                         const RouteTable& rt, uint32_t* live, uint32_t* ectr, hipStream_t s);

// errs[0]: ids >= idcap, errs[1]: ids already live, errs[2]: non-finite
// coordinates.
void launch_validate(const float* pts, const uint32_t* ids, uint64_t n, int d,
                     const uint64_t* map, uint32_t idcap, uint32_t* errs, hipStream_t s);

}  // namespace bdl
