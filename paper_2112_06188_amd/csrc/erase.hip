// Erase_L's erase step (Alg. 4, first line) on gfx950.
//
// The paper routes each erased point down every tree (Erase_S, Alg. 2), with
// a Bloom filter per tree to skip the trees that cannot hold it (Section
// V-A); k_erase_routed does that.  By default every live id has a map entry
// (tree, slot) written when its tree was built, so a point is located in
// O(1) instead (k_erase): the entry is checked against the stored
// coordinates (bitwise) and the slot is tombstoned.  A compare-and-swap on
// the map entry (or, routed, on the record's id) makes a repeated id in one
// batch erase once.  Per-tree live counts are reduced per workgroup before
// one atomic per tree.
#include "erase.hpp"

namespace bdl {

namespace {

__global__ void __launch_bounds__(256)
k_erase(const float* __restrict__ pts, const uint32_t* __restrict__ ids, uint64_t n, int d,
        uint64_t* map, uint32_t idcap, EraseTable et, uint32_t* live, uint32_t* ectr) {
  __shared__ uint32_t dec[kMaxLevels + 1];
  for (int i = threadIdx.x; i <= kMaxLevels; i += blockDim.x) dec[i] = 0;
  __syncthreads();
  const int S = rec_stride(d);
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t id = ids[e];
    if (id >= idcap) continue;
    const uint64_t m = map[id];
    if (m == kMapInvalid) continue;
    const uint32_t level = (uint32_t)(m >> 32);
    const uint32_t slot = (uint32_t)m;
    float* r;
    int bucket;
    if (level == kBufferLevel) {
      if (slot >= et.bn || !et.pool) continue;
      r = et.pool + (uint64_t)slot * S;
      bucket = kMaxLevels;
    } else if (level < (uint32_t)kMaxLevels && et.rec[level] && slot < et.nslots[level]) {
      r = et.rec[level] + (uint64_t)slot * S;
      bucket = (int)level;
    } else {
      continue;
    }
    bool eq = __float_as_uint(r[d]) == id;
    for (int j = 0; j < d; ++j)
      eq = eq && (__float_as_uint(r[j]) == __float_as_uint(pts[e * d + j]));
    if (!eq) continue;
    if (atomicCAS(reinterpret_cast<unsigned long long*>(map + id), (unsigned long long)m,
                  (unsigned long long)kMapInvalid) != (unsigned long long)m)
      continue;
    r[d] = __uint_as_float(kTomb);
    atomicAdd(&dec[bucket], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int l = 0; l <= kMaxLevels; ++l) {
      const uint32_t c = dec[l];
      if (!c) continue;
      tot += c;
      if (l < kMaxLevels) atomicSub(&live[l], c);
      else atomicAdd(&ectr[1], c);
    }
    if (tot) atomicAdd(&ectr[0], tot);
  }
}

// SplitMix64 finalizer (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", 2014): a bijective 64-bit mix.
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Hash of a point's identity: its id and the bit patterns of its coordinates.
__device__ inline uint64_t point_hash(const float* p, int d, uint32_t id) {
  uint64_t h = mix64(id);
  for (int j = 0; j < d; ++j) h = mix64(h ^ __float_as_uint(p[j]));
  return h;
}

// Word and the four bits (from the hash's upper 24 bits) of a blocked filter.
__device__ inline uint64_t bloom_bits(uint64_t h) {
  return (1ull << ((h >> 40) & 63)) | (1ull << ((h >> 46) & 63)) | (1ull << ((h >> 52) & 63)) |
         (1ull << ((h >> 58) & 63));
}

__global__ void k_bloom_build(const float* rec, uint64_t n, int d, uint64_t* bloom, uint64_t mask) {
  const int S = rec_stride(d);
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (uint64_t)gridDim.x * blockDim.x) {
    const float* r = rec + s * S;
    const uint32_t id = __float_as_uint(r[d]);
    if (id == kTomb) continue;
    const uint64_t h = point_hash(r, d, id);
    atomicOr(reinterpret_cast<unsigned long long*>(&bloom[h & mask]),
             (unsigned long long)bloom_bits(h));
  }
}

__global__ void k_fill64(uint64_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Tombstones the record of `p` (same id, bitwise-equal coordinates) in slots
// [a, a+b) by swapping its id; false if none is there or another lane took
// it first.
__device__ inline bool take_in(float* rec, int S, uint32_t a, uint32_t b, const float* p, int d,
                               uint32_t id) {
  for (uint32_t sl = a; sl < a + b; ++sl) {
    float* r = rec + (uint64_t)sl * S;
    if (__float_as_uint(r[d]) != id) continue;
    bool eq = true;
    for (int j = 0; j < d; ++j) eq = eq && __float_as_uint(r[j]) == __float_as_uint(p[j]);
    if (!eq) continue;
    if (atomicCAS(reinterpret_cast<unsigned*>(r + d), id, kTomb) == id) return true;
  }
  return false;
}

__global__ void __launch_bounds__(256)
k_erase_routed(const float* __restrict__ pts, const uint32_t* __restrict__ ids, uint64_t n,
               int d, uint64_t* map, uint32_t idcap, EraseTable et, RouteTable rt,
               uint32_t* live, uint32_t* ectr) {
  __shared__ uint32_t dec[kMaxLevels + 1];
  for (int i = threadIdx.x; i <= kMaxLevels; i += blockDim.x) dec[i] = 0;
  __syncthreads();
  const int S = rec_stride(d);
  const int NS = node_stride(d);
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t id = ids[e];
    if (id >= idcap) continue;  // never inserted (as k_erase)
    const float* p = pts + e * d;
    const uint64_t h = point_hash(p, d, id);
    const uint64_t m = bloom_bits(h);
    int bucket = -1;
    for (int l = 0; l < kMaxLevels && bucket < 0; ++l) {
      if (!et.rec[l] || !rt.bloom[l]) continue;
      const uint64_t w = rt.bloom[l][h & ((1ull << rt.bloom_log2[l]) - 1ull)];
      if ((w & m) != m) continue;  // certainly not in this tree
      const float* nodes = rt.nodes[l];
      const uint32_t nn = rt.level_nodes[l];
      uint32_t v = 0;
      for (int depth = 0; depth <= kMaxDepth && v < nn; ++depth) {
        const float* f = nodes + (uint64_t)v * NS;
        const int dim = __float_as_int(f[NF_DIM]);
        const uint32_t a = (uint32_t)__float_as_int(f[NF_A]);
        const uint32_t b = (uint32_t)__float_as_int(f[NF_B]);
        if (dim < 0) {
          if (a <= et.nslots[l] && b <= et.nslots[l] - a && take_in(et.rec[l], S, a, b, p, d, id))
            bucket = l;
          break;
        }
        v = p[dim] < f[NF_SPLIT] ? a : b;
      }
    }
    if (bucket < 0 && et.bn && et.pool && rt.pool_bloom) {
      const uint64_t w = rt.pool_bloom[h & ((1ull << rt.pool_bloom_log2) - 1ull)];
      if ((w & m) == m && take_in(et.pool, S, 0u, et.bn, p, d, id)) bucket = kMaxLevels;
    }
    if (bucket < 0) continue;
    map[id] = kMapInvalid;
    atomicAdd(&dec[bucket], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int l = 0; l <= kMaxLevels; ++l) {
      const uint32_t c = dec[l];
      if (!c) continue;
      tot += c;
      if (l < kMaxLevels) atomicSub(&live[l], c);
      else atomicAdd(&ectr[1], c);
    }
    if (tot) atomicAdd(&ectr[0], tot);
  }
}

__global__ void __launch_bounds__(256)
k_validate(const float* pts, const uint32_t* ids, uint64_t n, int d, const uint64_t* map,
           uint32_t idcap, uint32_t* errs) {
  uint32_t e0 = 0, e1 = 0, e2 = 0;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t id = ids[e];
    if (id >= idcap) ++e0;
    else if (map[id] != kMapInvalid) ++e1;
    for (int j = 0; j < d; ++j) {
      const uint32_t b = __float_as_uint(pts[e * d + j]);
      if ((b & 0x7F800000u) == 0x7F800000u) {
        ++e2;
        break;
      }
    }
  }
  if (e0) atomicAdd(&errs[0], e0);
  if (e1) atomicAdd(&errs[1], e1);
  if (e2) atomicAdd(&errs[2], e2);
}

inline unsigned grid_for(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 2048) g = 2048;
  return (unsigned)g;
}

}  // namespace

void launch_erase(const float* pts, const uint32_t* ids, uint64_t n, int d, uint64_t* map,
                  uint32_t idcap, const EraseTable& et, uint32_t* live, uint32_t* ectr,
                  hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_erase, dim3(grid_for(n)), dim3(256), 0, s, pts, ids, n, d, map, idcap,
                     et, live, ectr);
}

void launch_bloom_build(const float* rec, uint64_t n, int d, uint64_t* bloom, int log2,
                        hipStream_t s) {
  const uint64_t words = 1ull << log2;
  hipLaunchKernelGGL(k_fill64, dim3(grid_for(words)), dim3(256), 0, s, bloom, words);
  if (!n) return;
  hipLaunchKernelGGL(k_bloom_build, dim3(grid_for(n)), dim3(256), 0, s, rec, n, d, bloom,
                     words - 1);
}

void launch_erase_routed(const float* pts, const uint32_t* ids, uint64_t n, int d,
                         uint64_t* map, uint32_t idcap, const EraseTable& et,
                         const RouteTable& rt, uint32_t* live, uint32_t* ectr, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_erase_routed, dim3(grid_for(n)), dim3(256), 0, s, pts, ids, n, d, map,
                     idcap, et, rt, live, ectr);
}

void launch_validate(const float* pts, const uint32_t* ids, uint64_t n, int d,
                     const uint64_t* map, uint32_t idcap, uint32_t* errs, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(n)), dim3(256), 0, s, pts, ids, n, d, map, idcap,
                     errs);
}

}  // namespace bdl
