// Device-wide primitives used by the build and the query paths: exclusive
// prefix sums (the prefix-sum primitive of Section III-D) and a stable LSD
// radix sort of (key, uint32 value) pairs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdl {

// Cross-lane moves of the 64-lane wavefront by DPP (VALU operand routing, no
// LDS traffic): row_shr:k moves within rows of 16 lanes, row_bcast:15 and
// row_bcast:31 carry a row's last lane into the following rows.  A lane
// whose source lies outside its row, or whose row is not in ROW_MASK,
// receives `old`.  Six such steps form a scan over the whole wavefront.
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142;  // rows 1 and 3 (row mask 0xA)
constexpr int kDppRowBcast31 = 0x143;  // rows 2 and 3 (row mask 0xC)

template <int CTRL, int ROW_MASK>
__device__ inline uint32_t dpp_move(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// Inclusive/exclusive scans inside a 64-lane wavefront and a workgroup.
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  v += dpp_move<kDppRowShr1, 0xF>(0u, v);
  v += dpp_move<kDppRowShr2, 0xF>(0u, v);
  v += dpp_move<kDppRowShr4, 0xF>(0u, v);
  v += dpp_move<kDppRowShr8, 0xF>(0u, v);
  v += dpp_move<kDppRowBcast15, 0xA>(0u, v);
  v += dpp_move<kDppRowBcast31, 0xC>(0u, v);
  return v;
}

// Exclusive scan over the workgroup (blockDim.x a multiple of 64, <= 1024).
// `wsum` is LDS scratch of at least 17 words.  Returns the exclusive prefix;
// *total receives the workgroup sum.  Contains __syncthreads.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int i = 0; i < nw; ++i) {
      uint32_t t = wsum[i];
      wsum[i] = run;
      run += t;
    }
    wsum[16] = run;
  }
  __syncthreads();
  uint32_t r = wsum[w] + inc - v;
  if (total) *total = wsum[16];
  __syncthreads();
  return r;
}

// Scratch (uint32 words) needed by scan_exclusive_u32 for n elements.
size_t scan_tmp_words(uint64_t n);
// out[i] = sum(in[0..i)); in == out is allowed.  If total != nullptr the sum
// of all n elements is written there (device).
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total,
                        uint32_t* tmp, hipStream_t s);

// Scratch (uint32 words) needed by the radix sorts for n elements.
size_t radix_tmp_words(uint64_t n);
// Stable sort of n pairs by key bits [begin_bit, end_bit).  Returns 0 when
// the sorted pairs are in (keys, vals), 1 when they are in (keys_alt,
// vals_alt).
int radix_sort_pairs_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                         uint32_t* vals_alt, uint64_t n, int begin_bit, int end_bit,
                         uint32_t* tmp, hipStream_t s);
int radix_sort_pairs_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                         uint32_t* vals_alt, uint64_t n, int begin_bit, int end_bit,
                         uint32_t* tmp, hipStream_t s);
// Stable sort of *n_dev (device, at most n_cap) pairs from (keys[0], vals[0])
// by key bits [0, *width_dev) (device, at most max_bits): passes of 8 bits
// on a fixed grid whose workgroups own contiguous chunks, and a pass whose
// first bit is at or above the width does nothing, so no host readback is
// needed.  *sel_dev (device) receives the index of the buffer pair that
// holds the result.  tmp: 65536 words.
void radix_sort_pairs_u64_dev(uint64_t* keys[2], uint32_t* vals[2], const uint32_t* n_dev,
                              uint64_t n_cap, const uint32_t* width_dev, int max_bits,
                              uint32_t* sel_dev, uint32_t* tmp, hipStream_t s);

}  // namespace bdl
