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

// ectr[0] += points erased, ectr[1] += points erased from the buffer,
// live[level] -= points erased from each static tree.
void launch_erase(const float* pts, const uint32_t* ids, uint64_t n, int d, uint64_t* map,
                  uint32_t idcap, const EraseTable& et, uint32_t* live, uint32_t* ectr,
                  hipStream_t s);

// errs[0]: ids >= idcap, errs[1]: ids already live, errs[2]: non-finite
// coordinates.
void launch_validate(const float* pts, const uint32_t* ids, uint64_t n, int d,
                     const uint64_t* map, uint32_t idcap, uint32_t* errs, hipStream_t s);

}  // namespace bdl
