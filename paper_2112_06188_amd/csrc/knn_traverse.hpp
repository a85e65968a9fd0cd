// Traversal kernels of the batched k-NN query (kNN_L, Alg. 5) on gfx950.
//
// One lane per query.  Every lane keeps its k best (squared distance, id)
// keys in registers and visits the trees one after another, largest first
// (Section V-B), then the buffer's tree.  Inside a tree it follows kNN_S
// (Section IV-A.3): descend towards the leaf that holds the query, then
// unwind through parent links; on the way up the sibling subtree is entered
// unless its tight box lies strictly farther than the current k-th distance.
// Parent links make the traversal stackless.  Which order subtrees are
// visited in does not change the result: it is the exact k nearest by
// (squared distance, id), because the box distance is a float32 lower bound
// of every point distance inside the box and pruning is strict.
//
// The kernels are templates over the dimension and the register top-k size;
// knn_dN_M.hip instantiate them for a range of dimensions each, so that the
// instantiations compile in parallel.
#pragma once

#include <map>
#include <mutex>
#include <tuple>

#include "bdl.h"
#include "knn.hpp"

namespace bdl {
namespace knn_detail {

// Workgroups of `bs` threads of kernel `kern` that fit on the device at once
// (a multiple of 8, so that every XCD gets as many), cached per device.
uint64_t resident_blocks(const void* kern, int bs);

// Zero the work counters of a persistent launch (a kernel, so that the step
// may be captured into a graph).
void zero_queue(uint32_t* queue, hipStream_t s);


constexpr uint64_t kPadKey = (0x7F800000ull << 32) | 0xFFFFFFFFull;

template <int D>
__device__ inline float select_dim(const float (&qq)[D], int dim) {
  float v = qq[0];
#pragma unroll
  for (int j = 1; j < D; ++j) v = dim == j ? qq[j] : v;
  return v;
}

// qq[dim] for a dim that may differ per lane, by masks (a chain of selects here would be
// turned into an indexed load from private memory)
template <int D>
__device__ __forceinline__ float select_dim_masked(const float (&qq)[D], int dim) {
  uint32_t r = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) r |= (dim == j ? 0xFFFFFFFFu : 0u) & __float_as_uint(qq[j]);
  return __uint_as_float(r);
}

// qq[dim] for a dim the whole wavefront holds alike (0 <= dim < D): one
// bitwise select (v_bfi) per dimension above the first, with the bit mask
// made by the scalar unit as the sign of (dim ^ j) - 1.  (A chain of selects
// on dim == j is turned by the compiler into an indexed access to memory.)
template <int D>
__device__ __forceinline__ float select_dim_uniform(const float (&qq)[D], int dim) {
  uint32_t v = __float_as_uint(qq[0]);
#pragma unroll
  for (int j = 1; j < D; ++j) {
    const uint32_t m = (uint32_t)(((dim ^ j) - 1) >> 31);
    v = (m & __float_as_uint(qq[j])) | (~m & v);
  }
  return __uint_as_float(v);
}

// mindist^2 from the query to a box lo[0..D), hi[0..D): per dimension the
// gap max(lo - q, 0, q - hi), accumulated like a point distance.
template <int D>
__device__ inline float box_dist2(const float (&qq)[D], const float* box) {
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    // lo <= hi in every box, so at most one of the two gaps is positive
    const float t = fmaxf(fmaxf(box[j] - qq[j], qq[j] - box[D + j]), 0.0f);
    acc = __builtin_fmaf(t, t, acc);
  }
  return acc;
}

// Insert c into the ascending array a (c < a[KMAX-1], keys distinct); the
// largest key falls off the end.  With g[j] = (a[j] > c), which is false
// below the insertion point and true from it on:
//   new a[j] = g[j-1] ? a[j-1] : (g[j] ? c : a[j]),  new a[0] = g[0] ? c : a[0].
// All comparisons use the old values, so they issue back to back.  Each
// g[j] goes through the wave's compare mask (a ballot of the lanes' compares
// and its inverse), which keeps the compiler from rewriting the selects as
// a minimum and a maximum per position with a 64-bit compare each.  If c is
// not below a[KMAX-1], every g[j] is false and a is left as it is.
template <int KMAX>
__device__ inline void topk_insert(uint64_t (&a)[KMAX], uint64_t c) {
  bool g[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j)
    g[j] = __builtin_amdgcn_inverse_ballot_w64(__builtin_amdgcn_uicmpl(a[j], c, 34 /* ugt */));
#pragma unroll
  for (int j = KMAX - 1; j > 0; --j) a[j] = g[j - 1] ? a[j - 1] : (g[j] ? c : a[j]);
  a[0] = g[0] ? c : a[0];
}

// XCD-aware block order: gfx950 hands consecutive workgroups to its 8 XCDs
// round robin, each with its own L2.  Remap so that XCD x runs one contiguous
// range of the (Hilbert-ordered) query blocks; neighbouring waves then share
// tree nodes in the same L2.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t x = b & 7u;
  const uint32_t q = nb >> 3, r = nb & 7u;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Work distribution in groups of `group` (64 unless stated) consecutive
// (Hilbert-ordered) queries, one group per wavefront at a time.
//
// Without a queue, wave w of the launch takes group w once (blocks remapped
// with xcd_block).  With a queue the grid is persistent: the groups are split
// into eight contiguous ranges, one per XCD, each with its own counter (64
// words apart, zeroed before the launch).  A wave draws groups from the range
// of its own XCD (workgroup index mod 8) and, once that is drained, from the
// other ranges in turn; every counter is bumped at most once per wave after
// its range is drained, so each wave leaves after at most eight misses.
constexpr int kQueueStride = kKnnQueueStride;

struct GroupSched {
  uint32_t* queue;
  uint32_t ngroups;
  uint32_t home;   // this workgroup's XCD
  uint32_t sweep;  // ranges drained so far (queue), or groups handed out (no queue)
  uint32_t fixed;  // the one group of this wave (no queue)

  __device__ bool next(uint32_t& g) {
    if (!queue) {
      if (sweep) return false;
      sweep = 1;
      g = fixed;
      return g < ngroups;
    }
    while (sweep < 8) {
      const uint32_t r = (home + sweep) & 7u;
      const uint32_t lo = (uint32_t)(((uint64_t)ngroups * r) >> 3);
      const uint32_t hi = (uint32_t)(((uint64_t)ngroups * (r + 1)) >> 3);
      uint32_t v = 0;
      if (__lane_id() == 0) v = atomicAdd(&queue[r * kQueueStride], 1u);
      v = __builtin_amdgcn_readlane(v, 0);
      if (v < hi - lo) {
        g = lo + v;
        return true;
      }
      ++sweep;
    }
    return false;
  }
};

__device__ inline GroupSched make_sched(uint32_t* queue, uint64_t nq, uint32_t group = 64) {
  GroupSched gs;
  gs.queue = queue;
  gs.ngroups = (uint32_t)((nq + group - 1) / group);
  gs.home = blockIdx.x & 7u;
  gs.sweep = 0;
  gs.fixed = xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  return gs;
}

template <int D, int KMAX>
__device__ __forceinline__ void knn_lane_query(const KnnQueries& Q, const uint32_t* __restrict__ order,
                                               const LevelViews* __restrict__ views,
                                               uint32_t* __restrict__ err,
                                               unsigned long long* __restrict__ stats, uint64_t t) {
  constexpr int S = (D + 1 + 3) & ~3;
  constexpr int NS = (5 + 2 * D + 3) & ~3;
  constexpr int SV = S / 4;
  constexpr int NV = NS / 4;
  const uint64_t gi = order ? (uint64_t)order[t] : t;
  // the request's output location is read after the traversal
  const uint32_t rq = Q.qreq ? Q.qreq[gi] : 0u;
  const int k = Q.qreq ? Q.reqs[rq].k : Q.one.k;
  float qq[D];
#pragma unroll
  for (int j = 0; j < D; ++j) qq[j] = Q.q[gi * D + j];
  const int skip = KMAX - k;
  uint64_t key[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) key[j] = j < skip ? 0ull : kPadKey;

  uint32_t c_nodes = 0, c_leaves = 0, c_points = 0;
  const int nviews = views->n;
  for (int v = 0; v < nviews; ++v) {
    const LevelView V = views->v[v];
    const float4* __restrict__ nodes = reinterpret_cast<const float4*>(V.nodes);
    const float4* __restrict__ rec = reinterpret_cast<const float4*>(V.rec);
    const uint32_t nn = V.n_nodes;
    const uint32_t ns = V.n_slots;
    int n = 0;
    bool up = false;
    // every node is entered once and left once; a longer walk means corrupt
    // parent links, so stop instead of looping
    uint64_t steps_left = 4ull * nn + 16;
    while (true) {
      if (--steps_left == 0) {
        atomicOr(err, 8u);
        break;
      }
      if (!up) {
        if ((uint32_t)n >= nn) {
          atomicOr(err, 1u);
          break;
        }
        float f[NS];
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          float4 x = nodes[(uint64_t)n * NV + u];
          f[4 * u + 0] = x.x;
          f[4 * u + 1] = x.y;
          f[4 * u + 2] = x.z;
          f[4 * u + 3] = x.w;
        }
        const float worst = __uint_as_float((uint32_t)(key[KMAX - 1] >> 32));
        ++c_nodes;
        if (box_dist2<D>(qq, f + NF_BOX) > worst) {
          up = true;
          continue;
        }
        const int dim = __float_as_int(f[NF_DIM]);
        const int a = __float_as_int(f[NF_A]);
        const int b = __float_as_int(f[NF_B]);
        if (dim < 0) {
          if ((uint32_t)a > ns || (uint32_t)b > ns - (uint32_t)a) {
            atomicOr(err, 2u);
            break;
          }
          ++c_leaves;
          c_points += (uint32_t)b;
          for (int sl = a; sl < a + b; ++sl) {
            float r[S];
#pragma unroll
            for (int u = 0; u < SV; ++u) {
              float4 x = rec[(uint64_t)sl * SV + u];
              r[4 * u + 0] = x.x;
              r[4 * u + 1] = x.y;
              r[4 * u + 2] = x.z;
              r[4 * u + 3] = x.w;
            }
            const uint32_t id = __float_as_uint(r[D]);
            if (id == kTomb) continue;
            float acc = 0.0f;
#pragma unroll
            for (int j = 0; j < D; ++j) {
              float tt = qq[j] - r[j];
              acc = __builtin_fmaf(tt, tt, acc);
            }
            const uint64_t ck = ((uint64_t)__float_as_uint(acc) << 32) | id;
            if (ck < key[KMAX - 1]) topk_insert<KMAX>(key, ck);
          }
          up = true;
          continue;
        }
        n = select_dim<D>(qq, dim) < f[NF_SPLIT] ? a : b;
      } else {
        if (n == 0) break;
        const int p = __float_as_int(nodes[(uint64_t)n * NV + 1].x);
        if ((uint32_t)p >= nn) {
          atomicOr(err, 4u);
          break;
        }
        const float4 h = nodes[(uint64_t)p * NV];
        const int dim = __float_as_int(h.y);
        const int a = __float_as_int(h.z);
        const int b = __float_as_int(h.w);
        const int nearc = select_dim<D>(qq, dim) < h.x ? a : b;
        if (n == nearc) {
          n = nearc == a ? b : a;
          up = false;
        } else {
          n = p;
        }
      }
    }
  }
  if (stats) {
    atomicAdd(&stats[0], (unsigned long long)c_nodes);
    atomicAdd(&stats[1], (unsigned long long)c_leaves);
    atomicAdd(&stats[2], (unsigned long long)c_points);
  }
  const KnnReqDev R = Q.qreq ? Q.reqs[rq] : Q.one;
  const uint64_t qi = gi - R.qoff;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j >= skip) {
      const uint64_t o = qi * (uint64_t)k + (uint64_t)(j - skip);
      R.out_ids[o] = (uint32_t)key[j];
      R.out_d2[o] = __uint_as_float((uint32_t)(key[j] >> 32));
    }
  }
}


// PERSIST selects the work-queue loop; without it every wave takes its one
// group and the kernel holds no scheduling state (fewer SGPRs, which keeps
// more waves resident).
template <int D, int KMAX, bool PERSIST>
__global__ void __launch_bounds__(256)
k_knn(KnnQueries Q, const uint32_t* __restrict__ order, const LevelViews* __restrict__ views,
      uint32_t* __restrict__ err, unsigned long long* __restrict__ stats,
      uint32_t* __restrict__ queue) {
  const uint64_t nq = Q.nq_dev ? *Q.nq_dev : Q.nq;
  GroupSched gs = make_sched(PERSIST ? queue : nullptr, nq);
  uint32_t g;
  while (gs.next(g)) {
    const uint64_t t = (uint64_t)g * 64 + __lane_id();
    if (t < nq) knn_lane_query<D, KMAX>(Q, order, views, err, stats, t);
  }
}

// A pointer into the constant address space.  The tree does not change
// during a k-NN launch, so its nodes and records may be read through such a
// pointer; a load at a wave-uniform address through it is a scalar load whose
// result lands in SGPRs.
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) vf4* cvf4_ptr;

__device__ inline cvf4_ptr as_cvf4(const float* p) { return (cvf4_ptr)(p); }

// A value the whole wavefront holds alike, kept in a scalar register: the
// compiler otherwise moves node fields that pass through selects and loop
// merges into vector registers, and a per-lane split dimension then turns
// the choice of the query's coordinate into an indexed access to memory.
__device__ __forceinline__ float wave_uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

template <int NV>
__device__ inline void load_node(cvf4_ptr nodes, int n, float (&f)[4 * NV]) {
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const vf4 x = nodes[(uint64_t)n * NV + u];
    f[4 * u + 0] = x.x;
    f[4 * u + 1] = x.y;
    f[4 * u + 2] = x.z;
    f[4 * u + 3] = x.w;
  }
}

// Wavefront-cooperative variant: the 64 lanes of a wave hold 64 * QPL queries
// that are neighbours in Hilbert-curve order (lane l holds queries l, l + 64,
// ... of its group) and walk each tree together, depth first.  At an internal
// node both children are read at once.  The near child (the side of the split
// where the majority of the wave's queries lie) is entered first, without a
// prune test when every tree is balanced (kViewBalanced); the far child, and
// the near one otherwise, is tested by a ballot over the strict prune tests
// of all the wave's queries (it is entered when ANY query may still find a
// neighbour in it), pushed on a wave-uniform stack kept in one VGPR (entry i
// in lane i) and tested again when popped.  Node and leaf data are read at
// wave-uniform addresses (scalar loads into SGPRs); every query keeps its own
// k best keys.  Entering extra nodes never changes a query's result.
//
// The kernel is bound by instruction issue: every lane takes part in every
// node and record any query of its wave needs.  With QPL queries per lane a
// wave's path serves more queries, and the path of 64 * QPL neighbouring
// queries grows more slowly than their number (the boundary of the region
// they cover grows more slowly than its volume), so the work per query
// drops; each lane pays with QPL sets of registers.
template <int D, int KMAX, int QPL, bool NEAR_FREE>
__device__ __forceinline__ void knn_wave_group(const KnnQueries& Q, const uint32_t* __restrict__ order,
                                               const LevelViews* __restrict__ views,
                                               uint32_t* __restrict__ err,
                                               unsigned long long* __restrict__ stats, uint64_t t0,
                                               uint64_t nq) {
  constexpr int S = (D + 1 + 3) & ~3;
  constexpr int NS = (5 + 2 * D + 3) & ~3;
  constexpr int SV = S / 4;
  constexpr int NV = NS / 4;
  const int lane = __lane_id();
  float qq[QPL][D];
  uint64_t key[QPL][KMAX];
  uint64_t vm[QPL];
  int nvalid = 0;
#pragma unroll
  for (int u = 0; u < QPL; ++u) {
    const uint64_t t = t0 + 64u * u;
    const bool valid = t < nq;
    const uint64_t gi = valid ? (order ? (uint64_t)order[t] : t) : 0;
    // only k is needed during the traversal; the request's output location
    // is read afterwards, so that it does not occupy registers meanwhile
    const int k = !valid ? KMAX : (Q.qreq ? Q.reqs[Q.qreq[gi]].k : Q.one.k);
#pragma unroll
    for (int j = 0; j < D; ++j) qq[u][j] = valid ? Q.q[gi * D + j] : 0.0f;
    // a lane without a query never asks for a node or a record: its keys are
    // all 0, so no distance is below its k-th; keys below KMAX - k are 0 too
#pragma unroll
    for (int j = 0; j < KMAX; ++j) key[u][j] = (j < KMAX - k || !valid) ? 0ull : kPadKey;
    vm[u] = __ballot(valid);
    nvalid += __popcll(vm[u]);
  }
  if (nvalid == 0) return;
  uint32_t c_nodes = 0, c_leaves = 0, c_points = 0;

  // (the lanes without a query are masked out after the ballot, so that the
  // test itself runs without a branch)
  auto wanted = [&](const float (&f)[NS]) -> bool {
    uint64_t any = 0;
#pragma unroll
    for (int u = 0; u < QPL; ++u) {
      const float worst = __uint_as_float((uint32_t)(key[u][KMAX - 1] >> 32));
      any |= __ballot(!(box_dist2<D>(qq[u], f + NF_BOX) > worst)) & vm[u];
    }
    return any != 0ull;
  };

  const int nviews = views->n;
  for (int v = 0; v < nviews; ++v) {
    const LevelView V = views->v[v];
    const cvf4_ptr nodes = as_cvf4(V.nodes);
    const cvf4_ptr rec = as_cvf4(V.rec);
    const uint32_t nn = V.n_nodes;
    const uint32_t ns = V.n_slots;
    if (nn == 0) continue;
    int stk = 0;  // lane i holds stack entry i
    int sp = 0;
    float cur[NS];
    load_node<NV>(nodes, 0, cur);
    ++c_nodes;
    bool have = wanted(cur);
    uint32_t steps_left = 2u * nn + 8u;
    while (true) {
      if (have) {
        if (--steps_left == 0) {
          if (lane == 0) atomicOr(err, 8u);
          break;
        }
        const int dim = wave_uniform(__float_as_int(cur[NF_DIM]));
        const int a = wave_uniform(__float_as_int(cur[NF_A]));
        const int b = wave_uniform(__float_as_int(cur[NF_B]));
        if (dim < 0) {
          if ((uint32_t)a > ns || (uint32_t)b > ns - (uint32_t)a) {
            if (lane == 0) atomicOr(err, 2u);
            break;
          }
          ++c_leaves;
          c_points += (uint32_t)b;
          // the leaf's records are read four at a time at wave-uniform
          // addresses (scalar loads into SGPRs).  Record arrays carry
          // kRecPad spare records, so reading up to three past the leaf's end
          // stays in bounds; records past the end and erased ones are
          // skipped by wave-uniform branches.  A record enters the insertion
          // only where its distance is at most the query's k-th (a superset
          // of the keys below the k-th key; the insertion leaves the keys as
          // they are for the others).
          const int end = a + b;
          for (int sl = a; sl < end; sl += 4) {
            float r[4][S];
            const cvf4_ptr rp = rec + (uint64_t)sl * SV;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
              for (int w = 0; w < SV; ++w) {
                const vf4 x = rp[i * SV + w];
                r[i][4 * w + 0] = x.x;
                r[i][4 * w + 1] = x.y;
                r[i][4 * w + 2] = x.z;
                r[i][4 * w + 3] = x.w;
              }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const uint32_t id = __float_as_uint(r[i][D]);
              if (sl + i >= end || id == kTomb) continue;
#pragma unroll
              for (int u = 0; u < QPL; ++u) {
                float acc = 0.0f;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                  const float tt = qq[u][j] - r[i][j];
                  acc = __builtin_fmaf(tt, tt, acc);
                }
                const float worst = __uint_as_float((uint32_t)(key[u][KMAX - 1] >> 32));
                if (acc <= worst)
                  topk_insert<KMAX>(key[u], ((uint64_t)__float_as_uint(acc) << 32) | id);
              }
            }
          }
          have = false;
        } else {
          if ((uint32_t)a >= nn || (uint32_t)b >= nn) {
            if (lane == 0) atomicOr(err, 1u);
            break;
          }
          float fa[NS], fb[NS];
          load_node<NV>(nodes, a, fa);
          load_node<NV>(nodes, b, fb);
          c_nodes += 2;
          // the near child (the side of the split where at least half of
          // the wave's queries lie) is entered without a test when every
          // tree is balanced: at least one query almost always needs it
          // there, and a box test costs about as much as scanning two
          // records.  In a deep, skewed tree (clustered points under
          // spatial-median splits) an untested near child leads down long
          // chains of splits no query needs, and it is tested; the far
          // child always is.
          const float split = wave_uniform(cur[NF_SPLIT]);
          int nleft = 0;
#pragma unroll
          for (int u = 0; u < QPL; ++u)
            nleft += __popcll(__ballot(select_dim_uniform<D>(qq[u], dim) < split) & vm[u]);
          const bool left_first = 2 * nleft >= nvalid;
          const bool wf = left_first ? wanted(fb) : wanted(fa);
          const bool wn = NEAR_FREE || (left_first ? wanted(fa) : wanted(fb));
          if (wn && wf) {
            if (sp >= 64) {
              if (lane == 0) atomicOr(err, 16u);
              break;
            }
            stk = lane == sp ? (left_first ? b : a) : stk;
            ++sp;
          }
          if (wn || wf) {
#pragma unroll
            for (int w = 0; w < NS; ++w) cur[w] = wave_uniform((left_first == wn) ? fa[w] : fb[w]);
            have = true;
          } else {
            have = false;
          }
        }
      } else {
        if (sp == 0) break;
        --sp;
        const int n = __builtin_amdgcn_readlane(stk, sp);
        if ((uint32_t)n >= nn) {
          if (lane == 0) atomicOr(err, 4u);
          break;
        }
        load_node<NV>(nodes, n, cur);
        ++c_nodes;
        have = wanted(cur);
      }
    }
  }
  // counts per query: wave-level work times the queries of the wave
  if (stats && lane == 0) {
    atomicAdd(&stats[0], (unsigned long long)c_nodes * nvalid);
    atomicAdd(&stats[1], (unsigned long long)c_leaves * nvalid);
    atomicAdd(&stats[2], (unsigned long long)c_points * nvalid);
  }
#pragma unroll
  for (int u = 0; u < QPL; ++u) {
    const uint64_t t = t0 + 64u * u;
    if (t >= nq) continue;
    const uint64_t gi = order ? (uint64_t)order[t] : t;
    const KnnReqDev R = Q.qreq ? Q.reqs[Q.qreq[gi]] : Q.one;
    const int k = R.k;
    const uint64_t qi = gi - R.qoff;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j >= KMAX - k) {
        const uint64_t o = qi * (uint64_t)k + (uint64_t)(j - (KMAX - k));
        R.out_ids[o] = (uint32_t)key[u][j];
        R.out_d2[o] = __uint_as_float((uint32_t)(key[u][j] >> 32));
      }
    }
  }
}

// Occupancy: for small d and k the kernel is held to eight wavefronts per
// SIMD (64 VGPRs), which measured faster than seven; larger instances keep
// the compiler's choice (a minimum of one).
template <int D, int KMAX>
constexpr int wave_kernel_min_waves() {
  return (D <= 3 && KMAX <= 5) ? 8 : 1;
}

// Queries per lane of the wavefront-per-group kernel: up to two where the
// registers allow it (small d and k), else one.  Two are used only for
// batches of at least kWaveQpl2Queries queries: below that, 128-query groups
// would give each resident wavefront fewer than two groups, and the launch
// would lose the wavefronts that hide its load latency (1M queries on the
// clustered 2D workload: slower with two per lane).
template <int D, int KMAX>
constexpr int wave_kernel_max_qpl() {
  return (D <= 3 && KMAX <= 5) ? 2 : 1;
}
constexpr uint64_t kWaveQpl2Queries = 1ull << 21;

template <int D, int KMAX, bool PERSIST, int QPL>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(wave_kernel_min_waves<D, KMAX>())))
k_knn_wave(KnnQueries Q, const uint32_t* __restrict__ order,
           const LevelViews* __restrict__ views, uint32_t* __restrict__ err,
           unsigned long long* __restrict__ stats, uint32_t* __restrict__ queue) {
  const uint64_t nq = Q.nq_dev ? *Q.nq_dev : Q.nq;
  // every tree balanced: the near child is entered without a test
  const bool near_free = (views->flags & kViewBalanced) != 0u;
  GroupSched gs = make_sched(PERSIST ? queue : nullptr, nq, 64 * QPL);
  uint32_t g;
  while (gs.next(g)) {
    const uint64_t t0 = (uint64_t)g * (64 * QPL) + __lane_id();
    if (near_free)
      knn_wave_group<D, KMAX, QPL, true>(Q, order, views, err, stats, t0, nq);
    else
      knn_wave_group<D, KMAX, QPL, false>(Q, order, views, err, stats, t0, nq);
  }
}

// ---------------------------------------------------------------------------
// One wavefront per query, for small batches where one lane per query
// leaves the device idle and a query's own chain of dependent node reads
// sets the latency.
//
// The 64 lanes search every tree of the query at once.  The query's k best
// keys are spread over the lanes (lane i holds the i-th best; a candidate is
// placed with one ballot and one shuffle), so the prune bound is one
// wave-uniform value.  The search:
//  1. descends the largest tree along the query's side of each split and
//     scans the leaf it reaches, which gives a first bound;
//  2. repeatedly pops up to 64 pending nodes (all trees' roots to begin
//     with) from a stack in LDS, one per lane; a node whose box lies
//     strictly farther than the bound is dropped, an internal node pushes
//     its far and then its near child, and the leaves' records are scanned
//     by the whole wave;
//  3. if the stack is close to full (`cap` entries are usable, at most
//     kQStack), the top pending subtree is walked by
//     the whole wave without a stack, through parent links (descend,
//     unwind, enter the far side when its box may hold a better point).
// A key already held is not inserted again, so a leaf met twice is
// harmless.  Any visiting order gives the exact k nearest, as in the other
// kernels.
constexpr int kQStack = 1536;        // pending nodes per wave (LDS)
constexpr int kQLeaves = 4;          // small leaves scanned together
constexpr int kQViewShift = 26;      // stack entry: view << 26 | node
constexpr uint32_t kQNodeMask = (1u << kQViewShift) - 1u;

__device__ inline uint64_t lanemask_lt64() {
  const int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ inline uint64_t shfl_up64(uint64_t v, int d) {
  const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, d, 64);
  const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), d, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// The wave's k best keys, lane i holding the i-th (lanes >= k hold keys that
// never decide a position below k).
struct WaveTopK {
  uint64_t key;
  uint64_t worst;  // the k-th best key (wave-uniform)
  int k;

  __device__ __forceinline__ void init(int kk) {
    k = kk;
    key = kPadKey;
    worst = kPadKey;
  }
  // c: wave-uniform candidate
  __device__ __forceinline__ void insert(uint64_t c) {
    if (!(c < worst)) return;
    if (__ballot(key == c)) return;  // held already
    const uint64_t gt = __ballot(key > c);
    const int p = gt ? __builtin_ctzll(gt) : 64;
    if (p >= k) return;
    const uint64_t up = shfl_up64(key, 1);
    const int lane = __lane_id();
    key = lane == p ? c : (lane > p ? up : key);
    worst = readlane64(key, k - 1);
  }
};

template <int D>
__device__ __forceinline__ void scan_leaf_wave(const float (&qq)[D], const float* __restrict__ rec,
                                      uint32_t a, uint32_t b, WaveTopK& T) {
  constexpr int S = (D + 1 + 3) & ~3;
  const int lane = __lane_id();
  for (uint32_t base = a; base < a + b; base += 64) {
    const uint32_t idx = base + (uint32_t)lane;
    uint64_t cand = kPadKey;
    if (idx < a + b) {
      const float* r = rec + (uint64_t)idx * S;
      const uint32_t id = __float_as_uint(r[D]);
      if (id != kTomb) {
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const float tt = qq[j] - r[j];
          acc = __builtin_fmaf(tt, tt, acc);
        }
        cand = ((uint64_t)__float_as_uint(acc) << 32) | id;
      }
    }
    uint64_t m = __ballot(cand < T.worst);
    while (m) {
      const int l = __builtin_ctzll(m);
      m &= m - 1;
      T.insert(readlane64(cand, l));
    }
  }
}

// Up to NL leaves of at most 16 records each at once: lane group g (64 / NL
// lanes) takes leaf g, and each of its lanes NL / 4 of the leaf's records,
// so that the leaves' records are read by NL / 4 loads per lane instead of
// one round trip to memory per leaf.  recs/la/lb/cnt are the same on every
// lane.
template <int D, int NL>
__device__ __forceinline__ void scan_leaves_wave(const float (&qq)[D],
                                                 const float* const (&recs)[NL],
                                                 const uint32_t (&la)[NL],
                                                 const uint32_t (&lb)[NL], int cnt,
                                                 WaveTopK& T) {
  constexpr int S = (D + 1 + 3) & ~3;
  constexpr int LPL = 64 / NL;  // lanes per leaf
  constexpr int RPL = 16 / LPL;  // records per lane
  static_assert(LPL * NL == 64 && RPL * LPL == 16, "leaves of 16 records over 64 lanes");
  const int lane = __lane_id();
  const int g = lane / LPL;
  const uint32_t r0 = (uint32_t)(lane % LPL);
  // the lane's leaf by bitwise selects on masks (-1 where g == h), which
  // the compiler does not turn into an indexed access to memory
  uint64_t rpv = (uint64_t)recs[0];
  uint32_t a = la[0], b = lb[0];
#pragma unroll
  for (int h = 1; h < NL; ++h) {
    const uint32_t mk = (uint32_t)(((g ^ h) - 1) >> 31);
    const uint64_t mk2 = ((uint64_t)mk << 32) | mk;
    rpv = (mk2 & (uint64_t)recs[h]) | (~mk2 & rpv);
    a = (mk & la[h]) | (~mk & a);
    b = (mk & lb[h]) | (~mk & b);
  }
  const float* rp = (const float*)rpv;
  // every record is loaded before any is used
  float x[RPL][D];
  uint32_t id[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const uint32_t r = r0 + (uint32_t)(u * LPL);
    id[u] = kTomb;
    if (g < cnt && r < b) {
      const float* xp = rp + (uint64_t)(a + r) * S;
#pragma unroll
      for (int j = 0; j < D; ++j) x[u][j] = xp[j];
      id[u] = __float_as_uint(xp[D]);
    } else {
#pragma unroll
      for (int j = 0; j < D; ++j) x[u][j] = 0.0f;
    }
  }
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    uint64_t cand = kPadKey;
    if (id[u] != kTomb) {
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const float tt = qq[j] - x[u][j];
        acc = __builtin_fmaf(tt, tt, acc);
      }
      cand = ((uint64_t)__float_as_uint(acc) << 32) | id[u];
    }
    uint64_t m = __ballot(cand < T.worst);
    while (m) {
      const int l = __builtin_ctzll(m);
      m &= m - 1;
      T.insert(readlane64(cand, l));
    }
  }
}

template <int D>
__global__ void __launch_bounds__(256)
k_knn_query(KnnQueries Q, const uint32_t* __restrict__ order, const LevelViews* __restrict__ views,
            uint32_t* __restrict__ err, unsigned long long* __restrict__ stats, int cap) {
  constexpr int NS = (5 + 2 * D + 3) & ~3;
  constexpr int NV = NS / 4;
  __shared__ uint32_t stack_all[4][kQStack];
  // the tree table in LDS: a popped node's tree is read from there, one
  // dependent trip to memory less per round
  __shared__ LevelView s_views[kMaxViews];
  for (int i = threadIdx.x; i < kMaxViews; i += blockDim.x) s_views[i] = views->v[i];
  __syncthreads();
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  uint32_t* stk = stack_all[w];
  const uint64_t nq = Q.nq_dev ? *Q.nq_dev : Q.nq;
  const uint64_t t = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (uint64_t)w;
  if (t >= nq) return;  // the whole wave
  const uint64_t gi = order ? (uint64_t)order[t] : t;
  const uint32_t rq = Q.qreq ? Q.qreq[gi] : 0u;
  const int k = Q.qreq ? Q.reqs[rq].k : Q.one.k;
  float qq[D];
#pragma unroll
  for (int j = 0; j < D; ++j) qq[j] = Q.q[gi * D + j];
  WaveTopK T;
  T.init(k);
  const int nviews = views->n;
  uint64_t c_nodes = 0, c_leaves = 0, c_points = 0;
  bool bad = false;

  // 1. seed: the largest tree, along the query's side of every split
  if (nviews > 0 && views->v[0].n_nodes > 0) {
    const LevelView V = views->v[0];
    const cvf4_ptr nodes = as_cvf4(V.nodes);
    uint32_t n = 0;
    for (int depth = 0; depth <= kMaxDepth + 1; ++depth) {
      float f[NS];
      load_node<NV>(nodes, (int)n, f);
      ++c_nodes;
      const int dim = __float_as_int(f[NF_DIM]);
      const uint32_t a = (uint32_t)__float_as_int(f[NF_A]);
      const uint32_t b = (uint32_t)__float_as_int(f[NF_B]);
      if (dim < 0) {
        if (a > V.n_slots || b > V.n_slots - a) {
          bad = true;
          break;
        }
        ++c_leaves;
        c_points += b;
        scan_leaf_wave<D>(qq, V.rec, a, b, T);
        break;
      }
      n = select_dim_masked<D>(qq, dim) < f[NF_SPLIT] ? a : b;
      if (n >= V.n_nodes) {
        bad = true;
        break;
      }
    }
  }

  // 2. wide search over every tree
  int size = 0;
  for (int v = 0; v < nviews; ++v)
    if (views->v[v].n_nodes > 0 && size < cap) {
      if (lane == 0) stk[size] = (uint32_t)v << kQViewShift;
      ++size;
    }
  uint64_t rounds_left = 1;
  for (int v = 0; v < nviews; ++v) rounds_left += 4ull * views->v[v].n_nodes + 16;
  while (size > 0 && !bad) {
    if (--rounds_left == 0) {
      bad = true;
      break;
    }
    __builtin_amdgcn_wave_barrier();
    if (cap - size < 128) {
      // 3. stack nearly full: walk the top pending subtree without a stack
      --size;
      const uint32_t e = stk[size];
      const int v = (int)(e >> kQViewShift);
      const uint32_t root = e & kQNodeMask;
      const LevelView V = views->v[v];
      const cvf4_ptr nodes = as_cvf4(V.nodes);
      uint32_t n = root;
      bool up = false;
      uint64_t steps = 4ull * V.n_nodes + 16;
      while (true) {
        if (--steps == 0 || n >= V.n_nodes) {
          bad = true;
          break;
        }
        if (!up) {
          float f[NS];
          load_node<NV>(nodes, (int)n, f);
          ++c_nodes;
          if (box_dist2<D>(qq, f + NF_BOX) > __uint_as_float((uint32_t)(T.worst >> 32))) {
            up = true;
            continue;
          }
          const int dim = __float_as_int(f[NF_DIM]);
          const uint32_t a = (uint32_t)__float_as_int(f[NF_A]);
          const uint32_t b = (uint32_t)__float_as_int(f[NF_B]);
          if (dim < 0) {
            if (a > V.n_slots || b > V.n_slots - a) {
              bad = true;
              break;
            }
            ++c_leaves;
            c_points += b;
            scan_leaf_wave<D>(qq, V.rec, a, b, T);
            up = true;
            continue;
          }
          n = select_dim_masked<D>(qq, dim) < f[NF_SPLIT] ? a : b;
        } else {
          if (n == root) break;
          const uint32_t p = (uint32_t)__float_as_int(nodes[(uint64_t)n * NV + 1].x);
          if (p >= V.n_nodes) {
            bad = true;
            break;
          }
          const vf4 h = nodes[(uint64_t)p * NV];
          const int dim = __float_as_int(h.y);
          const uint32_t a = (uint32_t)__float_as_int(h.z);
          const uint32_t b = (uint32_t)__float_as_int(h.w);
          const uint32_t nearc = select_dim_masked<D>(qq, dim) < h.x ? a : b;
          if (n == nearc) {
            n = nearc == a ? b : a;
            up = false;
          } else {
            n = p;
          }
        }
      }
      continue;
    }
    // pop up to 64 pending nodes, one per lane
    const int m = size < 64 ? size : 64;
    const bool act0 = lane < m;
    const uint32_t e = act0 ? stk[size - 1 - lane] : 0u;
    size -= m;
    __builtin_amdgcn_wave_barrier();
    const int v = (int)(e >> kQViewShift);
    const uint32_t n = e & kQNodeMask;
    const LevelView* Vp = &s_views[v < kMaxViews ? v : 0];
    const uint32_t nn = act0 ? Vp->n_nodes : 0u;
    const uint32_t ns = act0 ? Vp->n_slots : 0u;
    bool act = act0 && n < nn;
    if (__ballot(act0 && !act)) bad = true;
    float f[NS];
    if (act) {
      const float4* np = reinterpret_cast<const float4*>(Vp->nodes) + (uint64_t)n * NV;
#pragma unroll
      for (int u = 0; u < NV; ++u) {
        const float4 x = np[u];
        f[4 * u + 0] = x.x;
        f[4 * u + 1] = x.y;
        f[4 * u + 2] = x.z;
        f[4 * u + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int u = 0; u < NS; ++u) f[u] = 0.0f;
    }
    c_nodes += (uint64_t)__popcll(__ballot(act));
    const float worst = __uint_as_float((uint32_t)(T.worst >> 32));
    act = act && !(box_dist2<D>(qq, f + NF_BOX) > worst);
    const int dim = __float_as_int(f[NF_DIM]);
    const uint32_t a = (uint32_t)__float_as_int(f[NF_A]);
    const uint32_t b = (uint32_t)__float_as_int(f[NF_B]);
    const bool inner = act && dim >= 0;
    const bool leafn = act && dim < 0;
    if (__ballot(inner && (a >= nn || b >= nn))) bad = true;
    if (__ballot(leafn && (a > ns || b > ns - a))) bad = true;
    if (bad) break;
    // push the children of inner nodes: far first, near on top
    const uint64_t im = __ballot(inner);
    if (inner) {
      const uint32_t nearc = select_dim_masked<D>(qq, dim) < f[NF_SPLIT] ? a : b;
      const uint32_t farc = nearc == a ? b : a;
      const int pos = size + 2 * (int)__popcll(im & lanemask_lt64());
      const uint32_t tag = (uint32_t)v << kQViewShift;
      stk[pos] = tag | farc;
      stk[pos + 1] = tag | nearc;
    }
    size += 2 * (int)__popcll(im);
    // scan the leaves with the whole wave: those of at most 16 records
    // kQLeaves at a time (one memory round trip for them all), larger ones
    // one after another
    uint64_t sm = __ballot(leafn && b <= 16u);
    uint64_t lm = __ballot(leafn) & ~sm;
    while (sm) {
      const float* recs[kQLeaves];
      uint32_t la[kQLeaves], lb[kQLeaves];
      int cnt = 0;
#pragma unroll
      for (int h = 0; h < kQLeaves; ++h) {
        recs[h] = nullptr;
        la[h] = 0u;
        lb[h] = 0u;
        if (sm) {
          const int l = __builtin_ctzll(sm);
          sm &= sm - 1;
          const int lv = __builtin_amdgcn_readlane(v, l);
          recs[h] = views->v[lv].rec;
          la[h] = (uint32_t)__builtin_amdgcn_readlane((int)a, l);
          lb[h] = (uint32_t)__builtin_amdgcn_readlane((int)b, l);
          ++cnt;
          ++c_leaves;
          c_points += lb[h];
        }
      }
      scan_leaves_wave<D, kQLeaves>(qq, recs, la, lb, cnt, T);
    }
    while (lm) {
      const int l = __builtin_ctzll(lm);
      lm &= lm - 1;
      const int lv = __builtin_amdgcn_readlane(v, l);
      const uint32_t la = (uint32_t)__builtin_amdgcn_readlane((int)a, l);
      const uint32_t lb = (uint32_t)__builtin_amdgcn_readlane((int)b, l);
      ++c_leaves;
      c_points += lb;
      scan_leaf_wave<D>(qq, views->v[lv].rec, la, lb, T);
    }
  }
  if (bad && lane == 0) atomicOr(err, 32u);
  if (stats && lane == 0) {
    atomicAdd(&stats[0], (unsigned long long)c_nodes);
    atomicAdd(&stats[1], (unsigned long long)c_leaves);
    atomicAdd(&stats[2], (unsigned long long)c_points);
  }
  const KnnReqDev R = Q.qreq ? Q.reqs[rq] : Q.one;
  const uint64_t qi = gi - R.qoff;
  if (lane < k) {
    const uint64_t o = qi * (uint64_t)k + (uint64_t)lane;
    R.out_ids[o] = (uint32_t)T.key;
    R.out_d2[o] = __uint_as_float((uint32_t)(T.key >> 32));
  }
}

template <int D, int KMAX>
void launch_one(const KnnLaunch& L, const KnnQueries& Q, uint64_t grid_q, const uint32_t* order,
                const LevelViews* views, uint32_t* err, unsigned long long* stats,
                hipStream_t s) {
  const int bs = L.block;
  // queries per thread: the group kernel's lanes may hold two
  constexpr int QMAX = wave_kernel_max_qpl<D, KMAX>();
  const bool two = L.mode == kKnnWave && QMAX == 2 && grid_q >= kWaveQpl2Queries;
  const void* kern = L.mode != kKnnWave
                         ? reinterpret_cast<const void*>(&k_knn<D, KMAX, true>)
                         : (two ? reinterpret_cast<const void*>(&k_knn_wave<D, KMAX, true, QMAX>)
                                : reinterpret_cast<const void*>(&k_knn_wave<D, KMAX, true, 1>));
  const uint64_t per = two ? 2u : 1u;
  uint64_t nb = (grid_q + bs * per - 1) / (bs * per);
  bool persist = false;
  if (L.persistent && L.queue) {
    const uint64_t res = resident_blocks(kern, bs);
    if (L.dry_run) return;
    if (res && nb > res) {
      nb = res;
      persist = true;
      zero_queue(L.queue, s);
    }
  }
  if (L.dry_run) return;
  const unsigned g = (unsigned)nb;
  if (L.mode == kKnnWave && two) {
    if (persist)
      hipLaunchKernelGGL((k_knn_wave<D, KMAX, true, QMAX>), dim3(g), dim3(bs), 0, s, Q, order,
                         views, err, stats, L.queue);
    else
      hipLaunchKernelGGL((k_knn_wave<D, KMAX, false, QMAX>), dim3(g), dim3(bs), 0, s, Q, order,
                         views, err, stats, nullptr);
  } else if (L.mode == kKnnWave) {
    if (persist)
      hipLaunchKernelGGL((k_knn_wave<D, KMAX, true, 1>), dim3(g), dim3(bs), 0, s, Q, order,
                         views, err, stats, L.queue);
    else
      hipLaunchKernelGGL((k_knn_wave<D, KMAX, false, 1>), dim3(g), dim3(bs), 0, s, Q, order,
                         views, err, stats, nullptr);
  } else {
    if (persist)
      hipLaunchKernelGGL((k_knn<D, KMAX, true>), dim3(g), dim3(bs), 0, s, Q, order, views, err,
                         stats, L.queue);
    else
      hipLaunchKernelGGL((k_knn<D, KMAX, false>), dim3(g), dim3(bs), 0, s, Q, order, views, err,
                         stats, nullptr);
  }
}

template <int D>
void launch_d(const KnnLaunch& L, int kmax, const KnnQueries& Q, uint64_t grid_q,
              const uint32_t* order, const LevelViews* views, uint32_t* err,
              unsigned long long* st, hipStream_t s) {
  if (L.mode == kKnnQuery) {
    if (L.dry_run) return;
    const unsigned g = (unsigned)((grid_q + 3) / 4);
    const int cap = L.qstack < 130 ? 130 : (L.qstack > kQStack ? kQStack : L.qstack);
    hipLaunchKernelGGL((k_knn_query<D>), dim3(g), dim3(256), 0, s, Q, order, views, err, st, cap);
    return;
  }
  if (L.mode == kKnnWave) {
    // register arrays sized to the common k exactly (no sentinel slots)
    if (kmax == 1) return launch_one<D, 1>(L, Q, grid_q, order, views, err, st, s);
    if (kmax == 2) return launch_one<D, 2>(L, Q, grid_q, order, views, err, st, s);
    if (kmax == 5) return launch_one<D, 5>(L, Q, grid_q, order, views, err, st, s);
    if (kmax == 10) return launch_one<D, 10>(L, Q, grid_q, order, views, err, st, s);
  }
  if (kmax <= 4) launch_one<D, 4>(L, Q, grid_q, order, views, err, st, s);
  else if (kmax <= 8) launch_one<D, 8>(L, Q, grid_q, order, views, err, st, s);
  else if (kmax <= 16) launch_one<D, 16>(L, Q, grid_q, order, views, err, st, s);
  else if (kmax <= 32) launch_one<D, 32>(L, Q, grid_q, order, views, err, st, s);
  else launch_one<D, 64>(L, Q, grid_q, order, views, err, st, s);
}

#define BDL_KNN_LAUNCH_D(DD)                                                                \
  template void launch_d<DD>(const KnnLaunch&, int, const KnnQueries&, uint64_t,             \
                             const uint32_t*, const LevelViews*, uint32_t*, unsigned long long*, \
                             hipStream_t);

}  // namespace knn_detail
}  // namespace bdl
