// k-NN graph of the live points: kNN_L (Alg. 5) with every live point as a
// query, started from the leaves (the leaf-based search discussed in
// Section II) instead of the root.
//
// The query points are the trees' own records.  Each tree is cut into
// groups: a group is the subtree of a node holding at most 64 points whose
// parent holds more (or a larger leaf), split into runs of at most 64
// consecutive slots.  A subtree's slots are contiguous and its box is a
// kd-tree cell, so a group's points are close together and reading them is
// one coalesced load per lane.  The groups themselves are taken in the
// Hilbert-curve order of their first points.
//
// One wavefront takes a group, one lane per point, and searches:
//  1. its own tree from the group's node: first that subtree (which holds
//     every lane's own leaf, so each lane gets its k best nearby at once),
//     then, going up through parent links, the other child of each
//     ancestor, entered depth first like the wavefront kernel of kNN_L
//     (a ballot over the lanes' strict prune tests, near side first);
//  2. every other tree from its root, as that kernel does.
// The order of the visits changes only the work, never the result: each
// lane ends with the exact k nearest live points by (squared distance, id),
// the row kNN_L returns for that point as a query.
#pragma once

#include "knn_traverse.hpp"

namespace bdl {
namespace knn_detail {

template <int D, int KMAX>
__device__ __forceinline__ void knn_graph_group(const LevelViews* __restrict__ views,
                                                const GraphGroup G, int k,
                                                uint32_t* __restrict__ out_ids,
                                                float* __restrict__ out_d2, uint32_t idcap,
                                                uint32_t* __restrict__ err,
                                                unsigned long long* __restrict__ stats) {
  constexpr int S = (D + 1 + 3) & ~3;
  constexpr int NS = (5 + 2 * D + 3) & ~3;
  constexpr int SV = S / 4;
  constexpr int NV = NS / 4;
  const int lane = __lane_id();
  const int nviews = views->n;
  if (G.view >= (uint32_t)nviews) {
    if (lane == 0) atomicOr(err, 64u);
    return;
  }
  const LevelView Vq = views->v[G.view];
  if (G.count > 64u || G.begin > Vq.n_slots || G.count > Vq.n_slots - G.begin) {
    if (lane == 0) atomicOr(err, 64u);
    return;
  }
  // the lane's query: the record at slot begin + lane of its own tree
  float qq[D];
  uint32_t qid = kTomb;
  if ((uint32_t)lane < G.count) {
    const float4* rp = reinterpret_cast<const float4*>(Vq.rec) + (uint64_t)(G.begin + lane) * SV;
    float r[S];
#pragma unroll
    for (int u = 0; u < SV; ++u) {
      const float4 x = rp[u];
      r[4 * u + 0] = x.x;
      r[4 * u + 1] = x.y;
      r[4 * u + 2] = x.z;
      r[4 * u + 3] = x.w;
    }
#pragma unroll
    for (int j = 0; j < D; ++j) qq[j] = r[j];
    qid = __float_as_uint(r[D]);
  } else {
#pragma unroll
    for (int j = 0; j < D; ++j) qq[j] = 0.0f;
  }
  const bool valid = qid != kTomb;
  const int skip = KMAX - k;
  uint64_t key[KMAX];
  // a lane without a live point asks for no node (its keys are all 0)
#pragma unroll
  for (int j = 0; j < KMAX; ++j) key[j] = (j < skip || !valid) ? 0ull : kPadKey;
  const uint64_t vmask = __ballot(valid);
  const int nvalid = __popcll(vmask);
  if (nvalid == 0) return;
  uint32_t c_nodes = 0, c_leaves = 0, c_points = 0;

  // (lanes without a point are masked out after the ballot, so that the
  // test runs without a branch)
  auto wanted = [&](const float (&f)[NS]) -> bool {
    const float worst = __uint_as_float((uint32_t)(key[KMAX - 1] >> 32));
    return (__ballot(!(box_dist2<D>(qq, f + NF_BOX) > worst)) & vmask) != 0ull;
  };

  bool bad = false;
  for (int it = -1; it < nviews && !bad; ++it) {
    const int v = it < 0 ? (int)G.view : it;
    if (it >= 0 && v == (int)G.view) continue;
    const LevelView V = views->v[v];
    const cvf4_ptr nodes = as_cvf4(V.nodes);
    const cvf4_ptr rec = as_cvf4(V.rec);
    const uint32_t nn = V.n_nodes;
    const uint32_t ns = V.n_slots;
    if (nn == 0) continue;
    const uint32_t start = it < 0 ? G.node : 0u;
    if (start >= nn) {
      bad = true;
      break;
    }
    int stk = 0;  // lane i holds stack entry i
    int sp = 0;
    float cur[NS];
    load_node<NV>(nodes, (int)start, cur);
    ++c_nodes;
    // `up` is the root of the part of the tree searched so far; its parent
    // is where the search continues once that part is done
    uint32_t up = start;
    int up_parent = __float_as_int(cur[NF_PARENT]);
    bool have = wanted(cur);
    uint32_t steps_left = 2u * nn + 80u;
    while (true) {
      if (--steps_left == 0) {
        bad = true;
        break;
      }
      if (have) {
        // node fields are the same on every lane: kept in scalar registers
        const int dim = wave_uniform(__float_as_int(cur[NF_DIM]));
        const int a = wave_uniform(__float_as_int(cur[NF_A]));
        const int b = wave_uniform(__float_as_int(cur[NF_B]));
        if (dim < 0) {
          if ((uint32_t)a > ns || (uint32_t)b > ns - (uint32_t)a) {
            bad = true;
            break;
          }
          ++c_leaves;
          c_points += (uint32_t)b;
          // records four at a time at wave-uniform addresses; the arrays
          // carry spare records, so reading up to three past the end stays
          // in bounds, and such records are skipped (as are erased ones); a
          // record enters the insertion where its distance is at most the
          // lane's k-th
          const int end = a + b;
          for (int sl = a; sl < end; sl += 4) {
            float r[4][S];
            const cvf4_ptr rp = rec + (uint64_t)sl * SV;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
              for (int u = 0; u < SV; ++u) {
                const vf4 x = rp[i * SV + u];
                r[i][4 * u + 0] = x.x;
                r[i][4 * u + 1] = x.y;
                r[i][4 * u + 2] = x.z;
                r[i][4 * u + 3] = x.w;
              }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const uint32_t id = __float_as_uint(r[i][D]);
              if (sl + i >= end || id == kTomb) continue;
              float acc = 0.0f;
#pragma unroll
              for (int j = 0; j < D; ++j) {
                const float tt = qq[j] - r[i][j];
                acc = __builtin_fmaf(tt, tt, acc);
              }
              const float worst = __uint_as_float((uint32_t)(key[KMAX - 1] >> 32));
              if (acc <= worst)
                topk_insert<KMAX>(key, ((uint64_t)__float_as_uint(acc) << 32) | id);
            }
          }
          have = false;
        } else {
          if ((uint32_t)a >= nn || (uint32_t)b >= nn) {
            bad = true;
            break;
          }
          // near child first: the side of the split where at least half of
          // the lanes' points lie
          const uint64_t lv =
              __ballot(select_dim_uniform<D>(qq, dim) < wave_uniform(cur[NF_SPLIT])) & vmask;
          const bool left_first = 2 * __popcll(lv) >= nvalid;
          float fa[NS], fb[NS];
          load_node<NV>(nodes, a, fa);
          load_node<NV>(nodes, b, fb);
          c_nodes += 2;
          const bool wa = wanted(fa);
          const bool wb = wanted(fb);
          const bool wn = left_first ? wa : wb;
          const bool wf = left_first ? wb : wa;
          if (wn && wf) {
            if (sp >= 64) {
              bad = true;
              break;
            }
            stk = lane == sp ? (left_first ? b : a) : stk;
            ++sp;
          }
          if (wn || wf) {
#pragma unroll
            for (int u = 0; u < NS; ++u) cur[u] = wave_uniform((left_first == wn) ? fa[u] : fb[u]);
            have = true;
          } else {
            have = false;
          }
        }
      } else if (sp > 0) {
        --sp;
        const int n = __builtin_amdgcn_readlane(stk, sp);
        if ((uint32_t)n >= nn) {
          bad = true;
          break;
        }
        load_node<NV>(nodes, n, cur);
        ++c_nodes;
        have = wanted(cur);
      } else {
        // the part under `up` is done: go on with its parent's other child
        if (up_parent < 0) break;
        const uint32_t p = (uint32_t)up_parent;
        if (p >= nn) {
          bad = true;
          break;
        }
        float pf[NS];
        load_node<NV>(nodes, (int)p, pf);
        const uint32_t pa = (uint32_t)__float_as_int(pf[NF_A]);
        const uint32_t pb = (uint32_t)__float_as_int(pf[NF_B]);
        if (__float_as_int(pf[NF_DIM]) < 0 || (pa != up && pb != up) || pa >= nn || pb >= nn) {
          bad = true;
          break;
        }
        const uint32_t sib = pa == up ? pb : pa;
        up = p;
        up_parent = __float_as_int(pf[NF_PARENT]);
        load_node<NV>(nodes, (int)sib, cur);
        c_nodes += 2;
        have = wanted(cur);
      }
    }
  }
  if (bad) {
    if (lane == 0) atomicOr(err, 64u);
    return;
  }
  if (stats && lane == 0) {
    atomicAdd(&stats[0], (unsigned long long)c_nodes * nvalid);
    atomicAdd(&stats[1], (unsigned long long)c_leaves * nvalid);
    atomicAdd(&stats[2], (unsigned long long)c_points * nvalid);
  }
  if (!valid || qid >= idcap) return;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j >= skip) {
      const uint64_t o = (uint64_t)qid * (uint64_t)k + (uint64_t)(j - skip);
      out_ids[o] = (uint32_t)key[j];
      out_d2[o] = __uint_as_float((uint32_t)(key[j] >> 32));
    }
  }
}

// A resident grid whose wavefronts draw groups, in Hilbert-curve order,
// from per-XCD ranges, so that each XCD's L2 serves one region of space.
template <int D, int KMAX>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(wave_kernel_min_waves<D, KMAX>())))
k_knn_graph(const LevelViews* __restrict__ views, const GraphGroup* __restrict__ groups,
            const uint32_t* __restrict__ order0, const uint32_t* __restrict__ order1,
            const uint32_t* __restrict__ sel, const uint32_t* __restrict__ ngroups, int k,
            uint32_t* __restrict__ out_ids, float* __restrict__ out_d2, uint32_t idcap,
            uint32_t* __restrict__ err, unsigned long long* __restrict__ stats,
            uint32_t* __restrict__ queue) {
  const uint32_t n = *ngroups;
  const uint32_t* order = *sel ? order1 : order0;
  GroupSched gs = make_sched(queue, (uint64_t)n * 64u);
  uint32_t g;
  while (gs.next(g)) {
    // the group is the same for the whole wavefront: keep it in scalar
    // registers, so that the tree it names is read with scalar loads
    const uint32_t o = __builtin_amdgcn_readfirstlane(order[g]);
    if (o >= n) {
      if (__lane_id() == 0) atomicOr(err, 64u);
      continue;
    }
    const GraphGroup* gp = groups + o;
    GraphGroup G;
    G.view = __builtin_amdgcn_readfirstlane(gp->view);
    G.node = __builtin_amdgcn_readfirstlane(gp->node);
    G.begin = __builtin_amdgcn_readfirstlane(gp->begin);
    G.count = __builtin_amdgcn_readfirstlane(gp->count);
    knn_graph_group<D, KMAX>(views, G, k, out_ids, out_d2, idcap, err, stats);
  }
}

template <int D, int KMAX>
void launch_graph_one(const LevelViews* views, const GraphScratch& G, const uint32_t* ngroups,
                      const uint32_t* sel, int k, uint32_t* out_ids, float* out_d2,
                      uint32_t idcap, uint32_t* err, unsigned long long* stats, uint32_t* queue,
                      hipStream_t s) {
  const void* kern = reinterpret_cast<const void*>(&k_knn_graph<D, KMAX>);
  uint64_t nb = resident_blocks(kern, 256);
  if (nb == 0) nb = 2048;
  zero_queue(queue, s);
  hipLaunchKernelGGL((k_knn_graph<D, KMAX>), dim3((unsigned)nb), dim3(256), 0, s, views,
                     G.groups, G.vals[0], G.vals[1], sel, ngroups, k, out_ids, out_d2, idcap,
                     err, stats, queue);
}

template <int D>
void launch_graph_d(const LevelViews* views, const GraphScratch& G, const uint32_t* ngroups,
                    const uint32_t* sel, int k, uint32_t* out_ids, float* out_d2,
                    uint32_t idcap, uint32_t* err, unsigned long long* stats, uint32_t* queue,
                    hipStream_t s) {
#define BDL_GRAPH_K(KK)                                                                       \
  return launch_graph_one<D, KK>(views, G, ngroups, sel, k, out_ids, out_d2, idcap, err, stats, \
                                 queue, s)
  if (k <= 4) BDL_GRAPH_K(4);
  if (k == 5) BDL_GRAPH_K(5);
  if (k <= 8) BDL_GRAPH_K(8);
  if (k == 10) BDL_GRAPH_K(10);
  if (k <= 16) BDL_GRAPH_K(16);
  if (k <= 32) BDL_GRAPH_K(32);
  BDL_GRAPH_K(64);
#undef BDL_GRAPH_K
}

#define BDL_KNN_GRAPH_D(DD)                                                                \
  template void launch_graph_d<DD>(const LevelViews*, const GraphScratch&, const uint32_t*, \
                                   const uint32_t*, int, uint32_t*, float*, uint32_t,       \
                                   uint32_t*, unsigned long long*, uint32_t*, hipStream_t);

}  // namespace knn_detail
}  // namespace bdl
