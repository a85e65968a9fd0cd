// Device-wide exclusive scan and stable LSD radix sort for gfx950.
#include "primitives.hpp"

namespace bdl {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kRadixThreads * kRadixItems;

__device__ inline int pidx(int i) { return i + (i >> 5); }  // LDS bank padding

__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(const uint32_t* __restrict__ in, uint64_t n, uint32_t* __restrict__ bsum) {
  __shared__ uint32_t wsum[17];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    uint64_t i = base + (uint64_t)r * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_excl_scan(s, wsum, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024)
k_scan_top(uint32_t* __restrict__ bsum, uint32_t nb, uint32_t* __restrict__ total) {
  __shared__ uint32_t wsum[17];
  uint32_t carry = 0;
  for (uint32_t c = 0; c < nb; c += blockDim.x) {
    uint32_t i = c + threadIdx.x;
    uint32_t v = i < nb ? bsum[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_excl_scan(v, wsum, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(const uint32_t* in, uint32_t* out, uint64_t n, const uint32_t* __restrict__ bsum) {
  __shared__ uint32_t tile[kScanTile + kScanTile / 32];
  __shared__ uint32_t wsum[17];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    int li = r * kScanThreads + threadIdx.x;
    uint64_t i = base + li;
    tile[pidx(li)] = i < n ? in[i] : 0u;
  }
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) s += tile[pidx(threadIdx.x * kScanItems + j)];
  uint32_t run = block_excl_scan(s, wsum, nullptr) + bsum[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int li = pidx(threadIdx.x * kScanItems + j);
    uint32_t v = tile[li];
    tile[li] = run;
    run += v;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    int li = r * kScanThreads + threadIdx.x;
    uint64_t i = base + li;
    if (i < n) out[i] = tile[pidx(li)];
  }
}

// The whole scan in one workgroup of 1024 threads, for short arrays (one
// launch instead of three): rounds of kSingleTile elements staged in LDS.
constexpr int kSingleThreads = 1024;
constexpr int kSingleTile = kSingleThreads * kScanItems;
constexpr uint64_t kSingleMax = 2 * kSingleTile;

__device__ __forceinline__ void scan_single_body(const uint32_t* in, uint32_t* out, uint64_t n,
                                                 uint32_t* __restrict__ total) {
  __shared__ uint32_t tile[kSingleTile + kSingleTile / 32];
  __shared__ uint32_t wsum[17];
  uint32_t carry = 0;
  for (uint64_t base = 0; base < n; base += kSingleTile) {
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
      const int li = r * kSingleThreads + threadIdx.x;
      const uint64_t i = base + li;
      tile[pidx(li)] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s += tile[pidx(threadIdx.x * kScanItems + j)];
    uint32_t tot;
    uint32_t run = block_excl_scan(s, wsum, &tot) + carry;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int li = pidx(threadIdx.x * kScanItems + j);
      const uint32_t v = tile[li];
      tile[li] = run;
      run += v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
      const int li = r * kSingleThreads + threadIdx.x;
      const uint64_t i = base + li;
      if (i < n) out[i] = tile[pidx(li)];
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void __launch_bounds__(kSingleThreads)
k_scan_single(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* __restrict__ total) {
  scan_single_body(in, out, n, total);
}

// Lanes of the wavefront whose digit equals this lane's, found with one
// ballot per digit bit; only meaningful for valid lanes.
__device__ inline uint64_t digit_peers(uint32_t dig, bool valid, int bits) {
  uint64_t m = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const bool bit = (dig >> b) & 1u;
    const uint64_t bb = __ballot(valid && bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ inline uint64_t lanes_below() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// Digit counts of one tile; one LDS add per distinct digit of a wavefront.
template <typename K>
__device__ __forceinline__ void radix_hist_tile(const K* __restrict__ keys, uint64_t n, int shift,
                                                int bits, uint32_t* __restrict__ hist,
                                                uint32_t nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t mask = (1u << bits) - 1u;
  const uint64_t below = lanes_below();
  const uint64_t base = (uint64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const uint64_t i = base + (uint64_t)r * kRadixThreads + threadIdx.x;
    const bool valid = i < n;
    const uint32_t dig = valid ? (uint32_t)(keys[i] >> shift) & mask : 0u;
    const uint64_t m = digit_peers(dig, valid, bits);
    if (valid && (m & below) == 0) atomicAdd(&h[dig], (uint32_t)__popcll(m));
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

template <typename K>
__global__ void __launch_bounds__(kRadixThreads)
k_radix_hist(const K* __restrict__ keys, uint64_t n, int shift, int bits,
             uint32_t* __restrict__ hist, uint32_t nb) {
  radix_hist_tile<K>(keys, n, shift, bits, hist, nb);
}

template <typename K>
__device__ __forceinline__ void radix_scatter_tile(const K* __restrict__ kin,
                                                   const uint32_t* __restrict__ vin,
                                                   K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                   uint64_t n, int shift, int bits,
                                                   const uint32_t* __restrict__ hscan,
                                                   uint32_t nb) {
  constexpr int kWaves = kRadixThreads / 64;
  constexpr int kRounds = kRadixTile / kRadixThreads;  // rounds of 64 per wavefront
  static_assert(kRadixThreads == 256, "one thread per digit");
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t gofs[256];
  __shared__ uint32_t wsum[17];
  __shared__ K skey[kRadixTile];
  __shared__ uint32_t sval[kRadixTile];
  const int tid = threadIdx.x;
  const int lane = __lane_id();
  const int w = tid >> 6;
  const uint32_t mask = (1u << bits) - 1u;
  const uint64_t below = lanes_below();
#pragma unroll
  for (int v = 0; v < kWaves; ++v) wcnt[v][tid] = 0;
  gofs[tid] = hscan[(uint64_t)tid * nb + blockIdx.x];
  __syncthreads();
  const uint64_t tbase = (uint64_t)blockIdx.x * kRadixTile;
  const uint64_t wbase = tbase + (uint64_t)w * (kRounds * 64);
  K key[kRounds];
  uint32_t val[kRounds];
  uint32_t rank[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t i = wbase + (uint64_t)r * 64 + lane;
    key[r] = i < n ? kin[i] : (K)0;
    val[r] = i < n ? vin[i] : 0u;
  }
  // rank among the equal digits of this wavefront's earlier elements; the
  // counters are private to the wavefront, whose LDS accesses stay in order
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool valid = wbase + (uint64_t)r * 64 + lane < n;
    const uint32_t dig = (uint32_t)(key[r] >> shift) & mask;
    const uint64_t m = digit_peers(dig, valid, bits);
    const uint32_t lower = (uint32_t)__popcll(m & below);
    const uint32_t seen = valid ? wcnt[w][dig] : 0u;
    rank[r] = seen + lower;
    if (valid && lower == 0) wcnt[w][dig] = seen + (uint32_t)__popcll(m);
  }
  __syncthreads();
  // thread tid owns digit tid: wavefront prefixes, then the tile's digit starts
  uint32_t tot = 0;
#pragma unroll
  for (int v = 0; v < kWaves; ++v) {
    const uint32_t c = wcnt[v][tid];
    wcnt[v][tid] = tot;
    tot += c;
  }
  dstart[tid] = block_excl_scan(tot, wsum, nullptr);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    if (wbase + (uint64_t)r * 64 + lane < n) {
      const uint32_t dig = (uint32_t)(key[r] >> shift) & mask;
      const uint32_t lp = dstart[dig] + wcnt[w][dig] + rank[r];
      skey[lp] = key[r];
      sval[lp] = val[r];
    }
  }
  __syncthreads();
  const uint64_t left = n - tbase;
  const uint32_t tcount = left < (uint64_t)kRadixTile ? (uint32_t)left : (uint32_t)kRadixTile;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t li = (uint32_t)(r * kRadixThreads + tid);
    if (li < tcount) {
      const K k = skey[li];
      const uint32_t dig = (uint32_t)(k >> shift) & mask;
      const uint64_t dst = (uint64_t)gofs[dig] + (li - dstart[dig]);
      kout[dst] = k;
      vout[dst] = sval[li];
    }
  }
}

template <typename K>
__global__ void __launch_bounds__(kRadixThreads)
k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                K* __restrict__ kout, uint32_t* __restrict__ vout, uint64_t n, int shift,
                int bits, const uint32_t* __restrict__ hscan, uint32_t nb) {
  radix_scatter_tile<K>(kin, vin, kout, vout, n, shift, bits, hscan, nb);
}

// ---- sorts whose element count and key width are read on the device ----
//
// A fixed grid of kChunkBlocks workgroups: workgroup b owns the contiguous
// chunk [b * chunk, (b + 1) * chunk) of the n elements (chunk a multiple of
// the tile), so the digit counts have a fixed shape (256 x kChunkBlocks) and
// the work follows n, not a host bound.  A pass whose first bit is at or
// above the width does nothing; passes that run form a prefix, so the
// result lies in buffer pair (passes run) & 1.
constexpr uint32_t kChunkBlocks = 256;

__device__ inline void chunk_of(uint64_t n, uint64_t* b0, uint64_t* b1) {
  uint64_t chunk = (n + kChunkBlocks - 1) / kChunkBlocks;
  chunk = (chunk + kRadixTile - 1) / kRadixTile * kRadixTile;
  *b0 = (uint64_t)blockIdx.x * chunk;
  *b1 = *b0 + chunk < n ? *b0 + chunk : n;
}

template <typename K>
__global__ void __launch_bounds__(kRadixThreads)
k_radix_hist_chunk(const K* __restrict__ keys, const uint32_t* n_dev, const uint32_t* width_dev,
                   int shift, uint32_t* __restrict__ hist) {
  if ((uint32_t)shift >= *width_dev) return;
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint64_t b0, b1;
  chunk_of(*n_dev, &b0, &b1);
  const uint64_t below = lanes_below();
  for (uint64_t i0 = b0; i0 < b1; i0 += kRadixThreads) {
    const uint64_t i = i0 + threadIdx.x;
    const bool valid = i < b1;
    const uint32_t dig = valid ? (uint32_t)(keys[i] >> shift) & 255u : 0u;
    const uint64_t m = digit_peers(dig, valid, 8);
    if (valid && (m & below) == 0) atomicAdd(&h[dig], (uint32_t)__popcll(m));
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * kChunkBlocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the 256 x kChunkBlocks digit counts in one workgroup.
__global__ void __launch_bounds__(kSingleThreads)
k_radix_scan_chunk(uint32_t* hist, const uint32_t* width_dev, int shift) {
  if ((uint32_t)shift >= *width_dev) return;
  scan_single_body(hist, hist, 256ull * kChunkBlocks, nullptr);
}

// Stable scatter of a chunk, tile by tile in order: every tile is ranked by
// digit as in the tiled pass, and each digit's write position advances by
// the tile's count of that digit.
template <typename K>
__global__ void __launch_bounds__(kRadixThreads)
k_radix_scatter_chunk(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                      K* __restrict__ kout, uint32_t* __restrict__ vout, const uint32_t* n_dev,
                      const uint32_t* width_dev, int shift, const uint32_t* __restrict__ hscan) {
  if ((uint32_t)shift >= *width_dev) return;
  constexpr int kWaves = kRadixThreads / 64;
  constexpr int kRounds = kRadixTile / kRadixThreads;
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t gofs[256];
  __shared__ uint32_t wsum[17];
  __shared__ K skey[kRadixTile];
  __shared__ uint32_t sval[kRadixTile];
  uint64_t b0, b1;
  chunk_of(*n_dev, &b0, &b1);
  if (b0 >= b1) return;
  const int tid = threadIdx.x;
  const int lane = __lane_id();
  const int w = tid >> 6;
  const uint64_t below = lanes_below();
  gofs[tid] = hscan[(uint64_t)tid * kChunkBlocks + blockIdx.x];
  for (uint64_t tbase = b0; tbase < b1; tbase += kRadixTile) {
#pragma unroll
    for (int v = 0; v < kWaves; ++v) wcnt[v][tid] = 0;
    __syncthreads();
    const uint64_t wbase = tbase + (uint64_t)w * (kRounds * 64);
    K key[kRounds];
    uint32_t val[kRounds];
    uint32_t rank[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint64_t i = wbase + (uint64_t)r * 64 + lane;
      key[r] = i < b1 ? kin[i] : (K)0;
      val[r] = i < b1 ? vin[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const bool valid = wbase + (uint64_t)r * 64 + lane < b1;
      const uint32_t dig = (uint32_t)(key[r] >> shift) & 255u;
      const uint64_t m = digit_peers(dig, valid, 8);
      const uint32_t lower = (uint32_t)__popcll(m & below);
      const uint32_t seen = valid ? wcnt[w][dig] : 0u;
      rank[r] = seen + lower;
      if (valid && lower == 0) wcnt[w][dig] = seen + (uint32_t)__popcll(m);
    }
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int v = 0; v < kWaves; ++v) {
      const uint32_t c = wcnt[v][tid];
      wcnt[v][tid] = tot;
      tot += c;
    }
    dstart[tid] = block_excl_scan(tot, wsum, nullptr);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      if (wbase + (uint64_t)r * 64 + lane < b1) {
        const uint32_t dig = (uint32_t)(key[r] >> shift) & 255u;
        const uint32_t lp = dstart[dig] + wcnt[w][dig] + rank[r];
        skey[lp] = key[r];
        sval[lp] = val[r];
      }
    }
    __syncthreads();
    const uint64_t left = b1 - tbase;
    const uint32_t tcount = left < (uint64_t)kRadixTile ? (uint32_t)left : (uint32_t)kRadixTile;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint32_t li = (uint32_t)(r * kRadixThreads + tid);
      if (li < tcount) {
        const K k = skey[li];
        const uint32_t dig = (uint32_t)(k >> shift) & 255u;
        const uint64_t dst = (uint64_t)gofs[dig] + (li - dstart[dig]);
        kout[dst] = k;
        vout[dst] = sval[li];
      }
    }
    __syncthreads();
    gofs[tid] += tot;  // this tile's count of digit tid
  }
}

// Index of the buffer holding the result: one flip per pass that ran.
__global__ void k_radix_sel(const uint32_t* width_dev, uint32_t* sel) {
  if (threadIdx.x == 0) sel[0] = ((*width_dev + 7u) / 8u) & 1u;
}

template <typename K>
int radix_sort_pairs(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, uint64_t n,
                     int begin_bit, int end_bit, uint32_t* tmp, hipStream_t s) {
  if (n == 0 || begin_bit >= end_bit) return 0;
  const uint32_t nb = (uint32_t)((n + kRadixTile - 1) / kRadixTile);
  uint32_t* hist = tmp;
  uint32_t* stmp = tmp + (size_t)256 * nb;
  K* kb[2] = {keys, keys_alt};
  uint32_t* vb[2] = {vals, vals_alt};
  int cur = 0;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    int bits = end_bit - shift < 8 ? end_bit - shift : 8;
    hipLaunchKernelGGL(k_radix_hist<K>, dim3(nb), dim3(kRadixThreads), 0, s, kb[cur], n, shift,
                       bits, hist, nb);
    scan_exclusive_u32(hist, hist, (uint64_t)256 * nb, nullptr, stmp, s);
    hipLaunchKernelGGL(k_radix_scatter<K>, dim3(nb), dim3(kRadixThreads), 0, s, kb[cur], vb[cur],
                       kb[cur ^ 1], vb[cur ^ 1], n, shift, bits, hist, nb);
    cur ^= 1;
  }
  return cur;
}

}  // namespace

size_t scan_tmp_words(uint64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 2; }

void radix_sort_pairs_u64_dev(uint64_t* keys[2], uint32_t* vals[2], const uint32_t* n_dev,
                              uint64_t n_cap, const uint32_t* width_dev, int max_bits,
                              uint32_t* sel_dev, uint32_t* tmp, hipStream_t s) {
  (void)n_cap;
  uint32_t* hist = tmp;
  int p = 0;
  for (int shift = 0; shift < max_bits; shift += 8, ++p) {
    const int cur = p & 1;
    hipLaunchKernelGGL(k_radix_hist_chunk<uint64_t>, dim3(kChunkBlocks), dim3(kRadixThreads), 0,
                       s, keys[cur], n_dev, width_dev, shift, hist);
    hipLaunchKernelGGL(k_radix_scan_chunk, dim3(1), dim3(kSingleThreads), 0, s, hist, width_dev,
                       shift);
    hipLaunchKernelGGL(k_radix_scatter_chunk<uint64_t>, dim3(kChunkBlocks), dim3(kRadixThreads),
                       0, s, keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_dev,
                       width_dev, shift, hist);
  }
  hipLaunchKernelGGL(k_radix_sel, dim3(1), dim3(64), 0, s, width_dev, sel_dev);
}

void scan_exclusive_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total,
                        uint32_t* tmp, hipStream_t s) {
  if (n == 0) {
    if (total) hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, 0u, total);
    return;
  }
  if (n <= kSingleMax) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kSingleThreads), 0, s, in, out, n, total);
    return;
  }
  const uint32_t nb = (uint32_t)((n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, nb, total);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, s, in, out, n, tmp);
}

size_t radix_tmp_words(uint64_t n) {
  uint64_t nb = (n + kRadixTile - 1) / kRadixTile;
  return (size_t)(256 * nb + scan_tmp_words(256 * nb));
}

int radix_sort_pairs_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                         uint32_t* vals_alt, uint64_t n, int begin_bit, int end_bit,
                         uint32_t* tmp, hipStream_t s) {
  return radix_sort_pairs<uint64_t>(keys, vals, keys_alt, vals_alt, n, begin_bit, end_bit, tmp, s);
}

int radix_sort_pairs_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                         uint32_t* vals_alt, uint64_t n, int begin_bit, int end_bit,
                         uint32_t* tmp, hipStream_t s) {
  return radix_sort_pairs<uint32_t>(keys, vals, keys_alt, vals_alt, n, begin_bit, end_bit, tmp, s);
}

}  // namespace bdl
