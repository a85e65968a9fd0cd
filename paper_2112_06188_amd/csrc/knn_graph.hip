// Host side of the k-NN graph launch (kNN_L over every live point, started
// from the leaves): the group list and the dispatch by dimension.
#include "bdl.h"
#include "hilbert.hpp"
#include "knn_graph.hpp"
#include "primitives.hpp"

namespace bdl {

namespace knn_detail {
template <int D>
void launch_graph_d(const LevelViews*, const GraphScratch&, const uint32_t*, const uint32_t*, int,
                    uint32_t*, float*, uint32_t, uint32_t*, unsigned long long*, uint32_t*,
                    hipStream_t);
}  // namespace knn_detail

namespace {

constexpr uint32_t kGroupPoints = 64;

__device__ inline uint32_t node_count(const float* nodes, int NS, uint32_t v) {
  return __float_as_uint(nodes[(uint64_t)v * NS + NS - 1]);
}

// One thread per node of one tree: a node starts a group when it is a leaf
// or holds at most 64 points, and its parent (if any) holds more.  Counts
// only grow towards the root, so every leaf lies under exactly one such
// node.  The group's slots run from its leftmost leaf's begin to its
// rightmost leaf's end (a subtree's slots are contiguous).
__global__ void k_graph_groups(const LevelViews* views, int view, int d, GraphGroup* groups,
                               uint64_t cap, uint32_t* ngroups, uint32_t* err) {
  const LevelView V = views->v[view];
  const int NS = node_stride(d);
  const uint32_t nn = V.n_nodes;
  const float* nodes = V.nodes;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nn;
       u += gridDim.x * blockDim.x) {
    const float* f = nodes + (uint64_t)u * NS;
    const bool leaf = __float_as_int(f[NF_DIM]) < 0;
    if (!leaf && node_count(nodes, NS, u) > kGroupPoints) continue;
    const int parent = __float_as_int(f[NF_PARENT]);
    if (parent >= 0) {
      if ((uint32_t)parent >= nn) {
        atomicOr(err, 64u);
        continue;
      }
      if (node_count(nodes, NS, (uint32_t)parent) <= kGroupPoints) continue;
    }
    uint32_t x = u, y = u;
    bool ok = true;
    for (int step = 0; step <= kMaxDepth + 1 && ok; ++step) {
      const float* fx = nodes + (uint64_t)x * NS;
      if (__float_as_int(fx[NF_DIM]) < 0) break;
      x = (uint32_t)__float_as_int(fx[NF_A]);
      ok = x < nn && step <= kMaxDepth;
    }
    for (int step = 0; step <= kMaxDepth + 1 && ok; ++step) {
      const float* fy = nodes + (uint64_t)y * NS;
      if (__float_as_int(fy[NF_DIM]) < 0) break;
      y = (uint32_t)__float_as_int(fy[NF_B]);
      ok = y < nn && step <= kMaxDepth;
    }
    if (!ok) {
      atomicOr(err, 64u);
      continue;
    }
    const uint32_t begin = (uint32_t)__float_as_int(nodes[(uint64_t)x * NS + NF_A]);
    const uint32_t yb = (uint32_t)__float_as_int(nodes[(uint64_t)y * NS + NF_A]);
    const uint32_t yc = (uint32_t)__float_as_int(nodes[(uint64_t)y * NS + NF_B]);
    if (yb > V.n_slots || yc > V.n_slots - yb || yb + yc < begin) {
      atomicOr(err, 64u);
      continue;
    }
    const uint32_t end = yb + yc;
    const uint32_t runs = (end - begin + kGroupPoints - 1) / kGroupPoints;
    if (runs == 0) continue;
    const uint32_t base = atomicAdd(ngroups, runs);
    if ((uint64_t)base + runs > cap) {
      atomicOr(err, 64u);
      continue;
    }
    for (uint32_t r = 0; r < runs; ++r) {
      const uint32_t b = begin + r * kGroupPoints;
      const uint32_t c = end - b < kGroupPoints ? end - b : kGroupPoints;
      groups[base + r] = GraphGroup{(uint32_t)view, u, b, c};
    }
  }
}

// Sort key of every group: the Hilbert-curve cell of its first point in the
// root box of the first (largest) tree, floor(30 / D) bits per dimension
// (points outside the box take the nearest cell).  Above it, the key puts
// the groups of the smaller trees first within each eighth of the curve:
// their points are spread out, so their wavefronts run longest, and the
// grid's per-XCD ranges (about one eighth of the curve each) should start
// them early rather than leave them for the end of the launch.
template <int D>
__global__ void k_graph_keys(const LevelViews* views, const GraphGroup* groups,
                             const uint32_t* ngroups, uint64_t* keys, uint32_t* vals,
                             uint32_t* width) {
  constexpr int kBits = 30 / D > 0 ? 30 / D : 1;
  constexpr int kKeyBits = kBits * D;
  constexpr int S = (D + 1 + 3) & ~3;
  const uint32_t n = *ngroups;
  if (blockIdx.x == 0 && threadIdx.x == 0) *width = (uint32_t)(kKeyBits + 4);
  const float* root = views->v[0].nodes;
  const float cells = (float)(1u << kBits);
  float lo[D], ext[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    lo[j] = root[NF_BOX + j];
    ext[j] = root[NF_BOX + D + j] - lo[j];
  }
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
    const GraphGroup G = groups[g];
    const float* r = views->v[G.view].rec + (uint64_t)G.begin * S;
    uint32_t cell[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const float u = ext[j] > 0.0f ? (r[j] - lo[j]) / ext[j] : 0.0f;
      int c = (int)(u * cells);
      c = c < 0 ? 0 : (c >= (1 << kBits) ? (1 << kBits) - 1 : c);
      cell[j] = (uint32_t)c;
    }
    const uint64_t h = hilbert_key<D, kBits>(cell);
    const uint64_t eighth = kKeyBits >= 3 ? h >> (kKeyBits - 3) : h;
    const uint64_t big = G.view == 0 ? 1u : 0u;
    keys[g] = (eighth << (kKeyBits + 1)) | (big << kKeyBits) | h;
    vals[g] = g;
  }
}

// One thread per slot of one tree; the live ones take consecutive positions
// per wavefront (one atomic per wavefront), in no particular order overall.
__global__ void k_graph_gather(const LevelViews* views, int view, int d, float* q, uint32_t* ids,
                               unsigned long long* count, uint64_t cap, uint32_t* err) {
  const LevelView V = views->v[view];
  const int S = rec_stride(d);
  const uint64_t ns = V.n_slots;
  const int lane = __lane_id();
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < ns; base += stride) {
    const uint64_t i = base + threadIdx.x;
    const float* r = V.rec + i * S;
    const uint32_t id = i < ns ? __float_as_uint(r[d]) : kTomb;
    const bool live = id != kTomb;
    const uint64_t m = __ballot(live);
    if (m == 0ull) continue;
    unsigned long long first = 0;
    if (lane == __builtin_ctzll(m)) first = atomicAdd(count, (unsigned long long)__popcll(m));
    first = __shfl(first, __builtin_ctzll(m), 64);
    if (!live) continue;
    const uint64_t pos = first + (uint64_t)__popcll(m & below);
    if (pos >= cap) {
      atomicOr(err, 64u);
      continue;
    }
    for (int j = 0; j < d; ++j) q[pos * d + j] = r[j];
    ids[pos] = id;
  }
}

// One thread per result word: row r goes to row ids[r] of the outputs.
__global__ void k_graph_scatter(const uint32_t* rid, const float* rd2, const uint32_t* ids,
                                const unsigned long long* count, int k, uint32_t* out_ids,
                                float* out_d2, uint32_t idcap) {
  const uint64_t n = (uint64_t)*count * (uint64_t)k;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = e / (uint64_t)k;
    const uint32_t id = ids[r];
    if (id >= idcap) continue;
    const uint64_t o = (uint64_t)id * (uint64_t)k + (e - r * (uint64_t)k);
    out_ids[o] = rid[e];
    out_d2[o] = rd2[e];
  }
}

}  // namespace

void launch_graph_gather(const LevelViews* views, int view, int d, uint64_t n_slots,
                         GraphQueries& gq, uint32_t* err, hipStream_t s) {
  uint64_t g = (n_slots + 255) / 256;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_graph_gather, dim3((unsigned)g), dim3(256), 0, s, views, view, d, gq.q,
                     gq.ids, gq.count, gq.cap, err);
}

void launch_graph_scatter(const GraphQueries& gq, int k, uint32_t* out_ids, float* out_d2,
                          uint32_t idcap, hipStream_t s) {
  uint64_t g = (gq.cap * (uint64_t)k + 255) / 256;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_graph_scatter, dim3((unsigned)g), dim3(256), 0, s, gq.rid, gq.rd2, gq.ids,
                     gq.count, k, out_ids, out_d2, idcap);
}

size_t graph_scratch_bytes(uint64_t cap) {
  return (size_t)cap * (sizeof(GraphGroup) + 2 * 8 + 2 * 4) + 65536 * 4;
}

void launch_graph_order(int d, const LevelViews* views, GraphScratch& gs, const uint32_t* ngroups,
                        uint32_t* width, uint32_t* sel, hipStream_t s) {
  uint64_t g = (gs.cap + 255) / 256;
  if (g > 4096) g = 4096;
  switch (d) {
#define BDL_GKEY_CASE(DD)                                                                       \
  case DD:                                                                                      \
    hipLaunchKernelGGL(k_graph_keys<DD>, dim3((unsigned)g), dim3(256), 0, s, views, gs.groups,  \
                       ngroups, gs.keys[0], gs.vals[0], width);                                 \
    break;
    BDL_GKEY_CASE(1) BDL_GKEY_CASE(2) BDL_GKEY_CASE(3) BDL_GKEY_CASE(4)
    BDL_GKEY_CASE(5) BDL_GKEY_CASE(6) BDL_GKEY_CASE(7) BDL_GKEY_CASE(8)
    BDL_GKEY_CASE(9) BDL_GKEY_CASE(10) BDL_GKEY_CASE(11) BDL_GKEY_CASE(12)
    BDL_GKEY_CASE(13) BDL_GKEY_CASE(14) BDL_GKEY_CASE(15) BDL_GKEY_CASE(16)
#undef BDL_GKEY_CASE
    default:
      return;
  }
  radix_sort_pairs_u64_dev(gs.keys, gs.vals, ngroups, gs.cap, width, 40, sel, gs.tmp, s);
}

void launch_graph_groups(const LevelViews* views, int view, int d, uint64_t n_slots,
                         GraphGroup* groups, uint64_t cap, uint32_t* ngroups, uint32_t* err,
                         hipStream_t s) {
  const uint64_t bound = 2 * n_slots + 1;  // nodes of a tree of n_slots points
  uint64_t g = (bound + 255) / 256;
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_graph_groups, dim3((unsigned)g), dim3(256), 0, s, views, view, d, groups,
                     cap, ngroups, err);
}

int launch_knn_graph(int d, int k, const LevelViews* views, const GraphScratch& gs,
                     const uint32_t* ngroups, const uint32_t* sel, uint32_t* out_ids,
                     float* out_d2, uint32_t idcap, uint32_t* err, unsigned long long* stats,
                     uint32_t* queue, hipStream_t s) {
  if (k < 1 || k > BDL_MAX_K || d < 1 || d > kMaxDim) return BDL_EINVAL;
  switch (d) {
#define BDL_GRAPH_CASE(DD)                                                                  \
  case DD:                                                                                  \
    knn_detail::launch_graph_d<DD>(views, gs, ngroups, sel, k, out_ids, out_d2, idcap, err, \
                                   stats, queue, s);                                        \
    break;
    BDL_GRAPH_CASE(1) BDL_GRAPH_CASE(2) BDL_GRAPH_CASE(3) BDL_GRAPH_CASE(4)
    BDL_GRAPH_CASE(5) BDL_GRAPH_CASE(6) BDL_GRAPH_CASE(7) BDL_GRAPH_CASE(8)
    BDL_GRAPH_CASE(9) BDL_GRAPH_CASE(10) BDL_GRAPH_CASE(11) BDL_GRAPH_CASE(12)
    BDL_GRAPH_CASE(13) BDL_GRAPH_CASE(14) BDL_GRAPH_CASE(15) BDL_GRAPH_CASE(16)
#undef BDL_GRAPH_CASE
    default:
      return BDL_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? 0 : BDL_EHIP;
}

}  // namespace bdl
