// Host launchers of the in-place insert of baseline B2 (Section III-B): a
// kd-tree that keeps the partition of its first build and takes new points
// into its existing leaves.
#pragma once

#include "bdl_common.hpp"

namespace bdl {

// Scratch of one B2 insert of n points into a tree of nn nodes.
struct B2Scratch {
  uint32_t* keys[2];  // old slot begin of each point's leaf (sorted in place)
  uint32_t* vals[2];  // point index
  uint32_t* obox;     // nn * 2d ordered-u32 bounds
  uint32_t* tmp;      // radix sort scratch (radix_tmp_words(n) words)
};

// Route the n points (caller rows [n][d], ids) down the tree's splits (x < split
// goes left): keys[0][i] = the slot begin of the leaf that takes point i,
// vals[0][i] = i; every box on the path grows to contain the point (nodes'
// boxes are rewritten).  Then the points are sorted by leaf (stable) and the
// records re-laid out into rec_out: each leaf's old records (slot order,
// tombstones included) followed by its new points in input order.  Leaves'
// slot ranges and the id map entries of every record are updated.  A child
// index out of range (a corrupt tree) sets bit 64 of *err (device).  Returns
// 0 or a BDL_E* code (launch failure).
int b2_insert(const float* pts, const uint32_t* ids, uint64_t n, int d, float* nodes,
              uint32_t nn, const float* rec_in, uint32_t n_slots, float* rec_out,
              uint64_t* map, uint32_t idcap, uint32_t level, uint32_t* err, B2Scratch& sc,
              hipStream_t s);

}  // namespace bdl
