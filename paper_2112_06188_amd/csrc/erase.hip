// Erase_L's erase step (Alg. 4, first line) on gfx950.
//
// The paper routes each erased point down every tree (Erase_S, Alg. 2, with
// bloom filters to skip trees, Section V-A).  Here every live id has a map
// entry (tree, slot) written when its tree was built, so a point is located
// in O(1): the entry is checked against the stored coordinates (bitwise) and
// the slot is tombstoned.  A compare-and-swap on the map entry makes a
// repeated id in one batch erase once.  Per-tree live counts are reduced per
// workgroup before one atomic per tree.
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

void launch_validate(const float* pts, const uint32_t* ids, uint64_t n, int d,
                     const uint64_t* map, uint32_t idcap, uint32_t* errs, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(n)), dim3(256), 0, s, pts, ids, n, d, map, idcap,
                     errs);
}

}  // namespace bdl
