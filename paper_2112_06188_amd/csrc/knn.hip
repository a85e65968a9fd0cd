// Batched k-NN over the log structure (kNN_L, Alg. 5) on gfx950.
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
#include "bdl.h"
#include "knn.hpp"
#include "primitives.hpp"

namespace bdl {

namespace {

constexpr uint64_t kPadKey = (0x7F800000ull << 32) | 0xFFFFFFFFull;

template <int D>
__device__ inline float select_dim(const float (&qq)[D], int dim) {
  float v = qq[0];
#pragma unroll
  for (int j = 1; j < D; ++j) v = dim == j ? qq[j] : v;
  return v;
}

// mindist^2 from the query to a box lo[0..D), hi[0..D): per dimension the
// gap max(lo - q, 0, q - hi), accumulated like a point distance.
template <int D>
__device__ inline float box_dist2(const float (&qq)[D], const float* box) {
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    float a = box[j] - qq[j];
    float b = qq[j] - box[D + j];
    float t = a > 0.0f ? a : (b > 0.0f ? b : 0.0f);
    acc = __builtin_fmaf(t, t, acc);
  }
  return acc;
}

// Insert c into the ascending array a (c < a[KMAX-1], keys distinct); the
// largest key falls off the end.  With g[j] = (a[j] > c), which is false
// below the insertion point and true from it on:
//   new a[j] = g[j-1] ? a[j-1] : (g[j] ? c : a[j]),  new a[0] = g[0] ? c : a[0].
// All comparisons use the old values, so they issue back to back.
template <int KMAX>
__device__ inline void topk_insert(uint64_t (&a)[KMAX], uint64_t c) {
  bool g[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) g[j] = a[j] > c;
#pragma unroll
  for (int j = KMAX - 1; j > 0; --j) a[j] = g[j - 1] ? a[j - 1] : (g[j] ? c : a[j]);
  a[0] = g[0] ? c : a[0];
}

template <int D, int KMAX>
__global__ void __launch_bounds__(256)
k_knn(KnnQueries Q, const uint32_t* __restrict__ order, const LevelViews* __restrict__ views,
      uint32_t* __restrict__ err, unsigned long long* __restrict__ stats) {
  constexpr int S = (D + 1 + 3) & ~3;
  constexpr int NS = (5 + 2 * D + 3) & ~3;
  constexpr int SV = S / 4;
  constexpr int NV = NS / 4;
  const uint64_t nq = Q.nq_dev ? *Q.nq_dev : Q.nq;
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nq) return;
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

// XCD-aware block order: gfx950 hands consecutive workgroups to its 8 XCDs
// round robin, each with its own L2.  Remap so that XCD x runs one contiguous
// range of the (Morton-ordered) query blocks; neighbouring waves then share
// tree nodes in the same L2.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t x = b & 7u;
  const uint32_t q = nb >> 3, r = nb & 7u;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// A pointer into the constant address space.  The tree does not change
// during a k-NN launch, so its nodes and records may be read through such a
// pointer; a load at a wave-uniform address through it is a scalar load whose
// result lands in SGPRs.
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) vf4* cvf4_ptr;

__device__ inline cvf4_ptr as_cvf4(const float* p) { return (cvf4_ptr)(p); }

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

// Wavefront-cooperative variant: the 64 lanes of a wave hold 64 queries that
// are neighbours in Morton order and walk each tree together, depth first.
// At an internal node both children are read at once and each is tested by a
// ballot over the lanes' strict prune tests: a child is entered when ANY lane
// may still find a neighbour in it.  The near child (the side of the split
// where the majority of the wave's queries lie) is entered first; the far one
// is pushed on a wave-uniform stack kept in one VGPR (entry i in lane i) and
// tested again when popped.  Node and leaf data are read at wave-uniform
// addresses (scalar loads for nodes, one coalesced load per leaf broadcast
// with v_readlane); every lane keeps its own k best keys.  Entering extra
// nodes never changes a lane's result.
template <int D, int KMAX>
__global__ void __launch_bounds__(256)
k_knn_wave(KnnQueries Q, const uint32_t* __restrict__ order,
           const LevelViews* __restrict__ views, uint32_t* __restrict__ err,
           unsigned long long* __restrict__ stats) {
  constexpr int S = (D + 1 + 3) & ~3;
  constexpr int NS = (5 + 2 * D + 3) & ~3;
  constexpr int SV = S / 4;
  constexpr int NV = NS / 4;
  const uint64_t nq = Q.nq_dev ? *Q.nq_dev : Q.nq;
  const uint64_t t = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool valid = t < nq;
  const int lane = __lane_id();
  const uint64_t gi = valid ? (order ? (uint64_t)order[t] : t) : 0;
  // only k is needed during the traversal; the request's output location is
  // read afterwards, so that it does not occupy registers meanwhile
  const uint32_t rq = (valid && Q.qreq) ? Q.qreq[gi] : 0u;
  const int k = !valid ? KMAX : (Q.qreq ? Q.reqs[rq].k : Q.one.k);
  float qq[D];
#pragma unroll
  for (int j = 0; j < D; ++j) qq[j] = valid ? Q.q[gi * D + j] : 0.0f;
  const int skip = KMAX - k;
  uint64_t key[KMAX];
  // a lane without a query never asks for a node: its keys are all 0, so no
  // box distance is ever within its k-th distance
#pragma unroll
  for (int j = 0; j < KMAX; ++j) key[j] = (j < skip || !valid) ? 0ull : kPadKey;
  const uint64_t vmask = __ballot(valid);
  const int nvalid = __popcll(vmask);
  if (nvalid == 0) return;
  uint32_t c_nodes = 0, c_leaves = 0, c_points = 0;

  auto wanted = [&](const float (&f)[NS]) -> bool {
    const float worst = __uint_as_float((uint32_t)(key[KMAX - 1] >> 32));
    return __ballot(valid && !(box_dist2<D>(qq, f + NF_BOX) > worst)) != 0ull;
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
        const int dim = __float_as_int(cur[NF_DIM]);
        const int a = __float_as_int(cur[NF_A]);
        const int b = __float_as_int(cur[NF_B]);
        if (dim < 0) {
          if ((uint32_t)a > ns || (uint32_t)b > ns - (uint32_t)a) {
            if (lane == 0) atomicOr(err, 2u);
            break;
          }
          ++c_leaves;
          c_points += (uint32_t)b;
          // the leaf's records are read at wave-uniform addresses (scalar
          // loads, four records per step) and used straight from SGPRs
          const int end = a + b;
          for (int sl = a; sl < end; sl += 4) {
            float r[4][S];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int si = sl + i < end ? sl + i : sl;
#pragma unroll
              for (int u = 0; u < SV; ++u) {
                const vf4 x = rec[(uint64_t)si * SV + u];
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
                float tt = qq[j] - r[i][j];
                acc = __builtin_fmaf(tt, tt, acc);
              }
              const uint64_t ck = ((uint64_t)__float_as_uint(acc) << 32) | id;
              if (ck < key[KMAX - 1]) topk_insert<KMAX>(key, ck);
            }
          }
          have = false;
        } else {
          if ((uint32_t)a >= nn || (uint32_t)b >= nn) {
            if (lane == 0) atomicOr(err, 1u);
            break;
          }
          const uint64_t lv = __ballot(valid && select_dim<D>(qq, dim) < cur[NF_SPLIT]);
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
              if (lane == 0) atomicOr(err, 16u);
              break;
            }
            stk = lane == sp ? (left_first ? b : a) : stk;
            ++sp;
          }
          if (wn || wf) {
#pragma unroll
            for (int u = 0; u < NS; ++u) cur[u] = (left_first == wn) ? fa[u] : fb[u];
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
  // counts per lane with a query: wave-level work times the active lanes
  if (stats && lane == 0) {
    atomicAdd(&stats[0], (unsigned long long)c_nodes * nvalid);
    atomicAdd(&stats[1], (unsigned long long)c_leaves * nvalid);
    atomicAdd(&stats[2], (unsigned long long)c_points * nvalid);
  }
  if (!valid) return;
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

__global__ void k_query_box_init(uint32_t* box) {
  const int t = threadIdx.x;
  if (t < kMaxDim) {
    box[t] = 0xFFFFFFFFu;
    box[kMaxDim + t] = 0u;
  }
}

__global__ void __launch_bounds__(256)
k_query_box(const float* q, const uint64_t* nq_dev, uint64_t nq_host, int d, uint32_t* box) {
  __shared__ uint32_t red[8];
  const uint64_t nq = nq_dev ? *nq_dev : nq_host;
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  for (int j = 0; j < d; ++j) {
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
         i += (uint64_t)gridDim.x * blockDim.x) {
      uint32_t o = f2o(q[i * d + j]);
      mn = o < mn ? o : mn;
      mx = o > mx ? o : mx;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      uint32_t a = __shfl_xor(mn, o, 64);
      uint32_t b = __shfl_xor(mx, o, 64);
      mn = a < mn ? a : mn;
      mx = b > mx ? b : mx;
    }
    if (lane == 0) {
      red[w] = mn;
      red[4 + w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int v = 1; v < 4; ++v) {
        mn = red[v] < mn ? red[v] : mn;
        mx = red[4 + v] > mx ? red[4 + v] : mx;
      }
      atomicMin(&box[j], mn);
      atomicMax(&box[kMaxDim + j], mx);
    }
    __syncthreads();
  }
}

// Morton key with bits = floor(30 / d) bits per dimension; positions from nq
// up to cap get the key 0xFFFFFFFF, which sorts after every real key.
__global__ void k_morton(const float* q, const uint64_t* nq_dev, uint64_t nq_host, uint64_t cap,
                         int d, const uint32_t* box, uint32_t* keys, uint32_t* vals) {
  const uint64_t nq = nq_dev ? *nq_dev : nq_host;
  const int bits = 30 / d > 0 ? 30 / d : 1;
  const float cells = (float)(1u << bits);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
       i += (uint64_t)gridDim.x * blockDim.x) {
    vals[i] = (uint32_t)i;
    if (i >= nq) {
      keys[i] = 0xFFFFFFFFu;
      continue;
    }
    uint32_t cell[kMaxDim];
    for (int j = 0; j < d; ++j) {
      float lo = o2f(box[j]), hi = o2f(box[kMaxDim + j]);
      float ext = hi - lo;
      float u = ext > 0.0f ? (q[i * d + j] - lo) / ext : 0.0f;
      int c = (int)(u * cells);
      c = c < 0 ? 0 : (c >= (int)(1u << bits) ? (int)(1u << bits) - 1 : c);
      cell[j] = (uint32_t)c;
    }
    uint32_t key = 0;
    for (int b = bits - 1; b >= 0; --b)
      for (int j = 0; j < d; ++j) key = (key << 1) | ((cell[j] >> b) & 1u);
    keys[i] = key;
  }
}

// Concatenate the queries of a request table into one array and record the
// request of every query (binary search over the requests' offsets).
__global__ void k_gather_queries(const KnnReqDev* reqs, const uint64_t* counts, int d,
                                 float* qall, uint32_t* qreq) {
  const uint64_t nq = counts[0];
  const uint32_t nreq = (uint32_t)counts[1];
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = nreq - 1;
    while (lo < hi) {
      uint32_t mid = (lo + hi + 1) >> 1;
      if (reqs[mid].qoff <= i) lo = mid; else hi = mid - 1;
    }
    const KnnReqDev& R = reqs[lo];
    const uint64_t li = i - R.qoff;
    for (int j = 0; j < d; ++j) qall[i * d + j] = R.q[li * d + j];
    qreq[i] = lo;
  }
}

template <int D, int KMAX>
void launch_one(const KnnLaunch& L, const KnnQueries& Q, uint64_t grid_q, const uint32_t* order,
                const LevelViews* views, uint32_t* err, unsigned long long* stats,
                hipStream_t s) {
  const int bs = L.block;
  const unsigned g = (unsigned)((grid_q + bs - 1) / bs);
  if (L.mode == kKnnWave)
    hipLaunchKernelGGL((k_knn_wave<D, KMAX>), dim3(g), dim3(bs), 0, s, Q, order, views, err,
                       stats);
  else
    hipLaunchKernelGGL((k_knn<D, KMAX>), dim3(g), dim3(bs), 0, s, Q, order, views, err, stats);
}

template <int D>
void launch_d(const KnnLaunch& L, int kmax, const KnnQueries& Q, uint64_t grid_q,
              const uint32_t* order, const LevelViews* views, uint32_t* err,
              unsigned long long* st, hipStream_t s) {
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

}  // namespace

size_t query_scratch_bytes(uint64_t cap) {
  return 4 * (size_t)cap * 4 + radix_tmp_words(cap) * 4 + 2 * kMaxDim * 4;
}

const uint32_t* morton_order(int d, const float* q, const uint64_t* nq_dev, uint64_t nq_host,
                             uint64_t cap, QueryScratch& qs, hipStream_t s) {
  hipLaunchKernelGGL(k_query_box_init, dim3(1), dim3(64), 0, s, qs.box);
  unsigned g = (unsigned)((cap + 255) / 256);
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(k_query_box, dim3(g), dim3(256), 0, s, q, nq_dev, nq_host, d, qs.box);
  unsigned g2 = (unsigned)((cap + 255) / 256);
  if (g2 > 4096) g2 = 4096;
  hipLaunchKernelGGL(k_morton, dim3(g2), dim3(256), 0, s, q, nq_dev, nq_host, cap, d, qs.box,
                     qs.keys[0], qs.vals[0]);
  const int bits = (30 / d > 0 ? 30 / d : 1) * d;
  int which = radix_sort_pairs_u32(qs.keys[0], qs.vals[0], qs.keys[1], qs.vals[1], cap, 0, bits,
                                   qs.tmp, s);
  return qs.vals[which];
}

void launch_gather_queries(const KnnReqDev* reqs, const uint64_t* counts, uint64_t cap, int d,
                           float* qall, uint32_t* qreq, hipStream_t s) {
  unsigned g = (unsigned)((cap + 255) / 256);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_gather_queries, dim3(g), dim3(256), 0, s, reqs, counts, d, qall, qreq);
}

int launch_knn(const KnnLaunch& L, int d, int kmax, const KnnQueries& Q, uint64_t grid_q,
               const uint32_t* order, const LevelViews* views, uint32_t* err,
               unsigned long long* stats, hipStream_t s) {
  switch (d) {
#define BDL_KNN_CASE(DD) \
  case DD:               \
    launch_d<DD>(L, kmax, Q, grid_q, order, views, err, stats, s); \
    break;
    BDL_KNN_CASE(1) BDL_KNN_CASE(2) BDL_KNN_CASE(3) BDL_KNN_CASE(4)
    BDL_KNN_CASE(5) BDL_KNN_CASE(6) BDL_KNN_CASE(7) BDL_KNN_CASE(8)
    BDL_KNN_CASE(9) BDL_KNN_CASE(10) BDL_KNN_CASE(11) BDL_KNN_CASE(12)
    BDL_KNN_CASE(13) BDL_KNN_CASE(14) BDL_KNN_CASE(15) BDL_KNN_CASE(16)
#undef BDL_KNN_CASE
    default:
      return BDL_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? 0 : BDL_EHIP;
}

}  // namespace bdl
