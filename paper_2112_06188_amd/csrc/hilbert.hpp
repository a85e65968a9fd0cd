// Hilbert-curve keys of grid cells (used to order queries and k-NN graph
// groups spatially).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdl {

// Position along the Hilbert curve of the cell x[0..D) (BITS per
// coordinate), by Skilling's transform of the axes into the curve's
// "transposed" index (J. Skilling, Programming the Hilbert curve, AIP Conf.
// Proc. 707, 2004) followed by bit interleaving.  Unlike Morton order the
// curve has no jumps: consecutive keys are neighbouring cells, so a group of
// consecutive queries covers a compact region.  x is overwritten.  D and
// BITS are compile-time, so the transform is straight-line code.
template <int D, int BITS>
__device__ inline uint32_t hilbert_key(uint32_t (&x)[D]) {
  constexpr uint32_t top = 1u << (BITS - 1);
#pragma unroll
  for (uint32_t q = top; q > 1; q >>= 1) {
    const uint32_t low = q - 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const uint32_t t = (x[0] ^ x[j]) & low;
      const bool set = (x[j] & q) != 0u;
      // bit q of x[j] set: invert the low bits of x[0]; else exchange them
      // between x[0] and x[j]
      const uint32_t x0 = set ? (x[0] ^ low) : (x[0] ^ t);
      const uint32_t xj = set ? x[j] : (x[j] ^ t);
      x[0] = x0;
      if (j != 0) x[j] = xj;
    }
  }
#pragma unroll
  for (int j = 1; j < D; ++j) x[j] ^= x[j - 1];
  uint32_t t = 0;
#pragma unroll
  for (uint32_t q = top; q > 1; q >>= 1)
    if (x[D - 1] & q) t ^= q - 1;
#pragma unroll
  for (int j = 0; j < D; ++j) x[j] ^= t;
  uint32_t key = 0;
#pragma unroll
  for (int b = BITS - 1; b >= 0; --b)
#pragma unroll
    for (int j = 0; j < D; ++j) key = (key << 1) | ((x[j] >> b) & 1u);
  return key;
}

}  // namespace bdl
