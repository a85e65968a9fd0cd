// Baseline B2 of Section III-B on the GPU: a batch is inserted into the
// existing kd-tree without recomputing any split.  Each new point follows
// the splits to a leaf, the boxes on its way grow to contain it, and the
// records are laid out again with every leaf's new points after its own.
#include "baseline.hpp"
#include "bdl.h"
#include "primitives.hpp"

namespace bdl {

namespace {

// Node boxes as ordered-u32 bounds, so that they can grow by integer atomics.
__global__ void k_b2_box_in(const float* nodes, uint32_t nn, int d, uint32_t* obox) {
  const int NS = node_stride(d);
  const uint64_t total = (uint64_t)nn * 2 * d;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t v = e / (2 * d);
    const int j = (int)(e % (2 * d));
    obox[e] = f2o(nodes[v * NS + NF_BOX + j]);
  }
}

__global__ void k_b2_box_out(float* nodes, uint32_t nn, int d, const uint32_t* obox) {
  const int NS = node_stride(d);
  const uint64_t total = (uint64_t)nn * 2 * d;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t v = e / (2 * d);
    const int j = (int)(e % (2 * d));
    nodes[v * NS + NF_BOX + j] = o2f(obox[e]);
  }
}

// One lane per new point: descend by the splits (x[dim] < split goes left),
// growing each box on the way; the key is the slot begin of the leaf
// reached.  A bound is only written when the point lies outside it (bounds
// only move outwards, so a stale read can only cause an extra atomic).
__global__ void k_b2_route(const float* pts, uint64_t n, int d, const float* nodes, uint32_t nn,
                           uint32_t* obox, uint32_t* keys, uint32_t* vals, uint32_t* err) {
  const int NS = node_stride(d);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const float* p = pts + i * d;
    uint32_t v = 0;
    for (int depth = 0;; ++depth) {
      const float* f = nodes + (uint64_t)v * NS;
      uint32_t* ob = obox + (uint64_t)v * 2 * d;
      for (int j = 0; j < d; ++j) {
        const uint32_t o = f2o(p[j]);
        if (o < ob[j]) atomicMin(&ob[j], o);
        if (o > ob[d + j]) atomicMax(&ob[d + j], o);
      }
      const int dim = __float_as_int(f[NF_DIM]);
      if (dim < 0) break;
      const uint32_t next = (uint32_t)__float_as_int(p[dim] < f[NF_SPLIT] ? f[NF_A] : f[NF_B]);
      if (next >= nn || depth > kMaxDepth) {
        atomicOr(err, 64u);
        break;
      }
      v = next;
    }
    keys[i] = (uint32_t)__float_as_int(nodes[(uint64_t)v * NS + NF_A]);
    vals[i] = (uint32_t)i;
  }
}

__device__ inline uint64_t lower_bound_u32(const uint32_t* a, uint64_t n, uint32_t x) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// One wavefront per leaf: the leaf's old records move to its new begin (old
// begin + new points of the leaves before it), its new points follow in
// input order (the sorted range of its key), and the id map follows every
// live record.
__global__ void k_b2_layout(float* nodes, uint32_t nn, int d, const float* rec_in,
                            float* rec_out, const uint32_t* skeys, const uint32_t* svals,
                            uint64_t n, const float* pts, const uint32_t* ids, uint64_t* map,
                            uint32_t idcap, uint32_t level) {
  const int NS = node_stride(d);
  const int S = rec_stride(d);
  const int lane = __lane_id();
  const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t v = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); v < nn;
       v += nw) {
    float* f = nodes + v * NS;
    if (__float_as_int(f[NF_DIM]) >= 0) continue;
    const uint32_t ob = (uint32_t)__float_as_int(f[NF_A]);
    const uint32_t oc = (uint32_t)__float_as_int(f[NF_B]);
    const uint64_t lb = lower_bound_u32(skeys, n, ob);
    const uint64_t ub = lower_bound_u32(skeys, n, ob + 1u);
    const uint64_t nb = ob + lb;
    for (uint32_t i = lane; i < oc; i += 64) {
      const float* src = rec_in + (uint64_t)(ob + i) * S;
      float* dst = rec_out + (nb + i) * S;
      for (int j = 0; j < S; ++j) dst[j] = src[j];
      const uint32_t id = __float_as_uint(src[d]);
      if (id != kTomb && id < idcap) map[id] = ((uint64_t)level << 32) | (nb + i);
    }
    for (uint64_t r = lb + lane; r < ub; r += 64) {
      const uint64_t p = svals[r];
      const uint64_t slot = nb + oc + (r - lb);
      float* dst = rec_out + slot * S;
      for (int j = 0; j < d; ++j) dst[j] = pts[p * d + j];
      const uint32_t id = ids[p];
      dst[d] = __uint_as_float(id);
      for (int j = d + 1; j < S; ++j) dst[j] = 0.0f;
      if (id < idcap) map[id] = ((uint64_t)level << 32) | slot;
    }
    if (lane == 0) {
      f[NF_A] = __int_as_float((int)nb);
      f[NF_B] = __int_as_float((int)(oc + (ub - lb)));
    }
  }
}

unsigned grid_of(uint64_t n, unsigned threads, unsigned cap) {
  uint64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

}  // namespace

int b2_insert(const float* pts, const uint32_t* ids, uint64_t n, int d, float* nodes,
              uint32_t nn, const float* rec_in, uint32_t n_slots, float* rec_out,
              uint64_t* map, uint32_t idcap, uint32_t level, uint32_t* err, B2Scratch& sc,
              hipStream_t s) {
  if (n == 0) return 0;
  const uint64_t nbox = (uint64_t)nn * 2 * d;
  hipLaunchKernelGGL(k_b2_box_in, dim3(grid_of(nbox, 256, 4096)), dim3(256), 0, s, nodes, nn, d,
                     sc.obox);
  hipLaunchKernelGGL(k_b2_route, dim3(grid_of(n, 256, 8192)), dim3(256), 0, s, pts, n, d, nodes,
                     nn, sc.obox, sc.keys[0], sc.vals[0], err);
  hipLaunchKernelGGL(k_b2_box_out, dim3(grid_of(nbox, 256, 4096)), dim3(256), 0, s, nodes, nn,
                     d, sc.obox);
  int bits = 1;
  while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)n_slots) ++bits;
  const int w = radix_sort_pairs_u32(sc.keys[0], sc.vals[0], sc.keys[1], sc.vals[1], n, 0, bits,
                                     sc.tmp, s);
  hipLaunchKernelGGL(k_b2_layout, dim3(grid_of((uint64_t)nn * 64, 256, 8192)), dim3(256), 0, s,
                     nodes, nn, d, rec_in, rec_out, sc.keys[w], sc.vals[w], n, pts, ids, map,
                     idcap, level);
  return hipGetLastError() == hipSuccess ? 0 : BDL_EHIP;
}

}  // namespace bdl
