// Static kd-tree construction for Insert_L on gfx950.
//
// BuildvEB (Alg. 1) with the spatial median (Section V-C), data-parallel
// over every tree an Insert_L call builds:
//  1. gather: the points of each new tree go to a contiguous range of a
//     structure-of-arrays build buffer (Insert_L's "deconstruct and gather");
//  2. global passes, one depth per pass, for nodes with more points than the
//     LDS finisher holds: split choice per node, a count of left points per
//     2048-point tile, a prefix sum over tiles and a stable scatter into the
//     other build buffer that also accumulates the children's tight boxes;
//  3. the LDS finisher: one workgroup builds a whole small subtree in LDS and
//     writes its points as records in final slot order;
//  4. layout: every node emitted above is keyed by its position in the van
//     Emde Boas order of the tree's height, sorted, and written out with
//     child and parent indices.
// The result is identical to a serial recursive build: splits depend only on
// a node's point set, and every partition is stable.
#include "bdl.h"
#include "build.hpp"
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "primitives.hpp"

namespace bdl {

namespace {

constexpr uint16_t kFrozen = 0xFFFF;

__device__ inline const uint32_t* soa_ids(const float* soa, int d, uint64_t cap) {
  return reinterpret_cast<const uint32_t*>(soa + (uint64_t)d * cap);
}
__device__ inline uint32_t* soa_ids_w(float* soa, int d, uint64_t cap) {
  return reinterpret_cast<uint32_t*>(soa + (uint64_t)d * cap);
}

__device__ inline uint64_t lanemask_lt() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// Spatial-median split of a node with ordered-u32 box lo[j] / hi[j]
// (Section V-C): dimension depth mod d moved forward to the first dimension
// with non-zero extent, value = midpoint of the tight extent; if rounding
// puts the midpoint on the lower bound (or the sum overflows), the upper
// bound is used so that both sides are non-empty.
__device__ inline int choose_dim(const uint32_t* lo, const uint32_t* hi, int d, int depth) {
  int c = depth % d;
  for (int it = 0; it < d && !(hi[c] > lo[c]); ++it) c = (c + 1 == d) ? 0 : c + 1;
  return c;
}

__device__ inline void choose_split(const uint32_t* lo, const uint32_t* hi, int d, int depth,
                                    int* dim_out, float* split_out) {
  const int c = choose_dim(lo, hi, d, depth);
  float mn = o2f(lo[c]);
  float mx = o2f(hi[c]);
  float split = (mn + mx) * 0.5f;
  if (!(split > mn) || split > mx) split = mx;
  *dim_out = c;
  *split_out = split;
}

// Object-median split (Section V-C) from the ordered-u32 key of the
// coordinate of rank floor(count/2) in dimension c: that coordinate (+0 for
// a zero), or the upper bound if it equals the lower bound (more than half of
// the points at the minimum), so that both sides are non-empty.
__device__ inline float object_split(const uint32_t* lo, const uint32_t* hi, int c,
                                     uint32_t key) {
  return key > lo[c] ? o2f(key) : o2f(hi[c]);
}

// A build counter written by other workgroups earlier in the same launch (the
// cooperative depth loop): read at the device's coherence point, so that
// every workgroup sees the same value after a grid barrier.
__device__ inline uint32_t ld_ctr(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lanes of the wavefront whose 8-bit digit equals this lane's (one ballot per
// digit bit); meaningful for valid lanes only.
__device__ inline uint64_t digit_peers8(uint32_t dig, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (dig >> b) & 1u;
    const uint64_t bb = __ballot(valid && bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ inline void write_emit(uint32_t* emit, int es, uint32_t idx, uint64_t path,
                                  uint32_t depth, uint32_t job, uint32_t parent, uint32_t side,
                                  uint32_t begin, uint32_t count, float split, int dim,
                                  const uint32_t* lo, const uint32_t* hi, int d) {
  // a record starts 8-byte aligned (es is even) and its fields pair up, so
  // it is written with 8-byte stores
  uint2* e = reinterpret_cast<uint2*>(emit + (uint64_t)idx * es);
  static_assert(EF_PATH_LO == 0 && EF_DEPTH == 2 && EF_PARENT == 4 && EF_BEGIN == 6 &&
                    EF_SPLIT == 8 && EF_BOX == 10,
                "emit fields pair up");
  e[0] = make_uint2((uint32_t)path, (uint32_t)(path >> 32));
  e[1] = make_uint2(depth, job);
  e[2] = make_uint2(parent, side);
  e[3] = make_uint2(begin, count);
  e[4] = make_uint2(__float_as_uint(split), (uint32_t)dim);
  // box words lo[0..d) then hi[0..d), two at a time (2d is even)
  for (int w = 0; w < 2 * d; w += 2) {
    const uint32_t a = w < d ? o2f_bits(lo[w]) : o2f_bits(hi[w - d]);
    const uint32_t b = w + 1 < d ? o2f_bits(lo[w + 1]) : o2f_bits(hi[w + 1 - d]);
    e[5 + w / 2] = make_uint2(a, b);
  }
}

// Slots from an LDS counter for the lanes that want one, with one atomic per
// wavefront (atomics on one LDS address serialize lane by lane).  Every lane
// of the wavefront calls it; lanes that want no slot get an unspecified value.
__device__ inline uint32_t wave_alloc(uint32_t* counter, bool want) {
  const uint64_t m = __ballot(want);
  if (m == 0) return 0u;
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (__lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = (uint32_t)__shfl((int)base, leader, 64);
  return base + (uint32_t)__popcll(m & lanemask_lt());
}

// Lanes of the wavefront with the same job as this one (jobs < kMaxJobs = 64,
// one ballot per bit of the job index); meaningful for valid lanes only.
__device__ inline uint64_t job_peers(uint32_t job, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    const bool bit = (job >> b) & 1u;
    const uint64_t bb = __ballot(valid && bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ inline void wave_minmax(uint32_t& mn, uint32_t& mx) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    uint32_t a = __shfl_xor(mn, o, 64);
    uint32_t b = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
}

__device__ inline uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------------
// gather
// ------------------------------------------------------------------------

__global__ void k_pool_to_soa(PoolSrc src, int d, uint64_t p0, uint64_t cnt, float* soa,
                              uint64_t cap, uint64_t dst) {
  const int S = rec_stride(d);
  uint32_t* ids = soa_ids_w(soa, d, cap);
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt;
       e += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t i = p0 + e;
    uint64_t o = dst + e;
    uint32_t id;
    const float* r;
    if (i < src.bn) {
      r = src.bufrec + i * S;
      id = __float_as_uint(r[d]);
    } else {
      uint64_t b = i - src.bn;
      if (src.batch_ids) {
        r = src.batch + b * d;
        id = src.batch_ids[b];
      } else {
        r = src.batch + b * S;
        id = __float_as_uint(r[d]);
      }
    }
    for (int j = 0; j < d; ++j) soa[(uint64_t)j * cap + o] = r[j];
    ids[o] = id;
  }
}

__global__ void k_pool_to_records(PoolSrc src, int d, uint64_t p0, uint64_t cnt, float* out,
                                  uint64_t* map, uint32_t idcap) {
  const int S = rec_stride(d);
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt;
       e += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t i = p0 + e;
    uint32_t id;
    const float* r;
    if (i < src.bn) {
      r = src.bufrec + i * S;
      id = __float_as_uint(r[d]);
    } else {
      uint64_t b = i - src.bn;
      if (src.batch_ids) {
        r = src.batch + b * d;
        id = src.batch_ids[b];
      } else {
        r = src.batch + b * S;
        id = __float_as_uint(r[d]);
      }
    }
    float* w = out + e * S;
    for (int j = 0; j < d; ++j) w[j] = r[j];
    w[d] = __uint_as_float(id);
    for (int j = d + 1; j < S; ++j) w[j] = 0.0f;
    if (map && id < idcap) map[id] = ((uint64_t)kBufferLevel << 32) | (uint64_t)e;
  }
}

__global__ void k_records_to_soa(const float* rec, int d, uint64_t n, float* soa, uint64_t cap,
                                 uint64_t dst) {
  const int S = rec_stride(d);
  uint32_t* ids = soa_ids_w(soa, d, cap);
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const float* r = rec + e * S;
    for (int j = 0; j < d; ++j) soa[(uint64_t)j * cap + dst + e] = r[j];
    ids[dst + e] = __float_as_uint(r[d]);
  }
}

__global__ void __launch_bounds__(kPassThreads)
k_count_live(const float* rec, int d, uint64_t n, uint32_t* tile_cnt) {
  __shared__ uint32_t red[4];
  const int S = rec_stride(d);
  const uint64_t t0 = (uint64_t)blockIdx.x * kTile;
  uint32_t c = 0;
  for (int r = 0; r < kItems; ++r) {
    uint64_t i = t0 + (uint64_t)r * kPassThreads + threadIdx.x;
    if (i < n && __float_as_uint(rec[i * S + d]) != kTomb) ++c;
  }
  c = wave_sum(c);
  if (__lane_id() == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Stable compaction of the live records of one tile to out positions
// tile_off[tile] + rank, either into build buffers (soa) or into records.
__global__ void __launch_bounds__(kPassThreads)
k_compact_live(const float* rec, int d, uint64_t n, const uint32_t* tile_off, float* soa,
               uint64_t cap, uint64_t dst, float* out_rec) {
  __shared__ uint32_t lt[kItems][4];
  const int S = rec_stride(d);
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  const uint64_t t0 = (uint64_t)blockIdx.x * kTile;
  uint64_t m[kItems];
  uint32_t fl = 0;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    uint64_t i = t0 + (uint64_t)r * kPassThreads + threadIdx.x;
    bool f = i < n && __float_as_uint(rec[i * S + d]) != kTomb;
    fl |= (uint32_t)f << r;
    m[r] = __ballot(f);
  }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < kItems; ++r) lt[r][w] = (uint32_t)__popcll(m[r]);
  }
  __syncthreads();
  const uint64_t ltm = lanemask_lt();
  uint32_t run = 0;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    uint32_t before = 0, row = 0;
    for (int v = 0; v < 4; ++v) {
      uint32_t x = lt[r][v];
      before += v < w ? x : 0u;
      row += x;
    }
    if ((fl >> r) & 1u) {
      uint64_t i = t0 + (uint64_t)r * kPassThreads + threadIdx.x;
      uint64_t o = (uint64_t)tile_off[blockIdx.x] + run + before + (uint32_t)__popcll(m[r] & ltm);
      const float* src = rec + i * S;
      if (out_rec) {
        float* wr = out_rec + o * S;
        for (int j = 0; j < S; ++j) wr[j] = src[j];
      } else {
        for (int j = 0; j < d; ++j) soa[(uint64_t)j * cap + dst + o] = src[j];
        soa_ids_w(soa, d, cap)[dst + o] = __float_as_uint(src[d]);
      }
    }
    run += row;
  }
}

// ------------------------------------------------------------------------
// build setup
// ------------------------------------------------------------------------

__global__ void k_reset_counters(BuildCounters* c, JobTable jt, Job* jobs_dev) {
  const int t = threadIdx.x;
  if (t == 0) {
    c->nseg[0] = c->nseg[1] = 0;
    c->ntiles[0] = c->ntiles[1] = c->ebase[0] = c->ebase[1] = 0;
    c->nfin = c->nemit = c->err = 0;
    c->fin_next = c->retry = 0;
    c->par_final = 0;
    c->deepest = 0;
  }
  if (t < kMaxJobs) {
    c->job_nodes[t] = 0;
    c->job_height[t] = 0;
    c->job_node_off[t] = 0;
    for (int j = 0; j < kMaxDim; ++j) {
      c->job_box[t][j] = 0xFFFFFFFFu;
      c->job_box[t][kMaxDim + j] = 0u;
    }
    if (t < jt.n) jobs_dev[t] = jt.jobs[t];
  }
}

// Tight box of every job's points.  A bounded number of workgroups per job
// stride over its tiles and combine their bounds in registers, so that each
// workgroup adds only one pair of device atomics per dimension.
__global__ void k_clear_retry(BuildCounters* c) {
  if (threadIdx.x == 0) c->retry = 0u;
}

__global__ void __launch_bounds__(kPassThreads)
k_root_box(const float* soa, uint64_t cap, int d, const Job* jobs, BuildCounters* c) {
  __shared__ uint32_t red[8];
  const Job J = jobs[blockIdx.y];
  // the workgroup's first element lies beyond the job: nothing to add
  if ((uint64_t)blockIdx.x * kPassThreads >= J.count) return;
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  for (int j = 0; j < d; ++j) {
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
    const float* x = soa + (uint64_t)j * cap + J.base;
    // eight independent loads per step (indices clamped into the job; a
    // repeated element does not change a bound)
    const uint64_t stride = (uint64_t)gridDim.x * kPassThreads;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kPassThreads + threadIdx.x; i0 < J.count;
         i0 += 8 * stride) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint64_t i = i0 + (uint64_t)u * stride;
        v[u] = x[i < J.count ? i : i0];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t o = f2o(v[u]);
        mn = o < mn ? o : mn;
        mx = o > mx ? o : mx;
      }
    }
    wave_minmax(mn, mx);
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
      atomicMin(&c->job_box[blockIdx.y][j], mn);
      atomicMax(&c->job_box[blockIdx.y][kMaxDim + j], mx);
    }
    __syncthreads();
  }
}

// Root of every job: one lane per job (kMaxJobs is one wavefront); jobs above
// the finisher threshold start the global passes, the others go straight to
// the finisher.  List order is job order.  The roots' tiles are numbered here
// (the list kernel numbers those of every later depth), and the roots' nodes
// take emit indices [0, roots).
__global__ void k_init_lists(const Job* jobs, int njobs, BuildCounters* c, Seg* cur, Fin* fin,
                             uint32_t* tile_seg, uint32_t T, uint64_t max_seg, uint64_t max_fin,
                             uint64_t max_tiles) {
  static_assert(kMaxJobs == 64, "one lane per job");
  const int jb = threadIdx.x;
  uint32_t cnt = 0, base = 0;
  if (jb < njobs) {
    cnt = jobs[jb].count;
    base = jobs[jb].base;
  }
  const bool is_seg = cnt > T;
  const bool is_fin = cnt > 0 && cnt <= T;
  const uint64_t below = lanemask_lt();
  const uint64_t ms = __ballot(is_seg), mf = __ballot(is_fin);
  const uint32_t nroot = (uint32_t)__popcll(ms);
  // tiles of the roots, numbered in list order
  const uint32_t ntl = is_seg ? (cnt + kTile - 1) / kTile : 0u;
  const uint32_t tinc = wave_incl_scan(ntl);
  const uint32_t ttot = (uint32_t)__shfl((int)tinc, 63, 64);
  const bool over = nroot > max_seg || ttot > max_tiles;
  if (jb == 0) {
    c->nseg[0] = over ? 0u : nroot;
    c->ntiles[0] = over ? 0u : ttot;
    c->nfin = (uint32_t)__popcll(mf);
    c->ebase[0] = 0;
    c->nemit = over ? 0u : nroot;
    if (over) atomicOr(&c->err, nroot > max_seg ? 1u : 256u);
  }
  if (is_seg && !over) {
    const uint32_t k = (uint32_t)__popcll(ms & below);
    Seg& g = cur[k];
    g.begin = base;
    g.count = cnt;
    g.job = (uint32_t)jb;
    g.depth = 0;
    g.path = 0;
    g.parent_emit = kNone;
    g.side = 0;
    g.tile_begin = tinc - ntl;
    g.ntiles = ntl;
    for (int j = 0; j < 2 * kMaxDim; ++j) g.box[j] = c->job_box[jb][j];
    atomicAdd(&c->job_nodes[jb], 1u);
    atomicMax(&c->job_height[jb], 1u);
  } else if (is_fin) {
    const uint32_t f = (uint32_t)__popcll(mf & below);
    if (f >= max_fin) {
      atomicOr(&c->err, 2u);
    } else {
      Fin& F = fin[f];
      F.begin = base;
      F.count = cnt;
      F.job = (uint32_t)jb;
      F.depth = 0;
      F.path = 0;
      F.parent_emit = kNone;
      F.side = 0;
      F.bufsel = 0;
    }
  }
  if (over) return;
  // segment of every root tile, the wavefront filling one root's run at a time
  uint64_t rest = ms;
  while (rest) {
    const int l = __ffsll((unsigned long long)rest) - 1;
    rest &= rest - 1;
    const uint32_t k = (uint32_t)__popcll(ms & ((1ull << l) - 1ull));
    const uint32_t tb = (uint32_t)__shfl((int)(tinc - ntl), l, 64);
    const uint32_t tn = (uint32_t)__shfl((int)ntl, l, 64);
    for (uint32_t i = jb; i < tn; i += 64) tile_seg[tb + i] = k;
  }
}

// ------------------------------------------------------------------------
// global passes (one depth per pass)
// ------------------------------------------------------------------------

constexpr uint32_t kListLds = 4096;  // list entries whose tile starts stay in LDS

// Left points of a tile before each of its quarters (eight rows of 64): the
// counts before quarters 1, 2 and 3 (at most 512, 1024 and 1536) in 10, 11
// and 11 bits, so that the scatter can hand each quarter to its own
// wavefront.
__device__ inline uint32_t pack_quarters(uint32_t l1, uint32_t l2, uint32_t l3) {
  return l1 | (l2 << 10) | (l3 << 21);
}
__device__ inline uint32_t left_before_quarter(uint32_t packed, uint32_t q) {
  return q == 0 ? 0u : q == 1 ? (packed & 0x3FFu) : q == 2 ? ((packed >> 10) & 0x7FFu)
                                                           : (packed >> 21);
}
static_assert(kTile == 2048, "quarter counts are packed for tiles of 2048 points");

// Left count of every tile: one wavefront per tile (ballots, no barriers),
// so that all of a tile's loads are in flight at once.  Every wavefront of a
// segment takes the segment's decision itself (leaf, or split dimension and
// value from its box); the wavefront of its first tile emits the node and
// records the decision for the list and scatter kernels.
// Wavefront wv of nwv takes tiles wv, wv + nwv, ...
__device__ __forceinline__ void count_tiles(Seg* cur, const uint32_t* tile_seg, BuildCounters* c,
                                            int par, const Job* jobs, uint32_t* emit, int es,
                                            int d, uint32_t leaf, const float* src, uint64_t cap,
                                            uint32_t* tile_left, uint32_t* tile_q, int rule,
                                            uint32_t wv, uint32_t nwv) {
  const uint32_t nt = ld_ctr(&c->ntiles[par]);
  const uint32_t ebase = ld_ctr(&c->ebase[par]);
  const int lane = __lane_id();
  for (uint32_t t = wv; t < nt; t += nwv) {
    const uint32_t s = tile_seg[t];
    Seg& g = cur[s];
    const uint32_t* lo = g.box;
    const uint32_t* hi = g.box + kMaxDim;
    bool degenerate = true;
    for (int j = 0; j < d; ++j) degenerate = degenerate && (lo[j] == hi[j]);
    const bool isleaf = g.count <= leaf || degenerate || g.depth >= (uint32_t)kMaxDepth;
    int dim = -1;
    float split = 0.0f;
    if (!isleaf) choose_split(lo, hi, d, (int)g.depth, &dim, &split);
    if (!isleaf && rule == kSplitObject) split = object_split(lo, hi, dim, g.sel_key);
    if (t == g.tile_begin && lane == 0) {
      const uint32_t eidx = ebase + s;
      write_emit(emit, es, eidx, g.path, g.depth, g.job, g.parent_emit, g.side,
                 g.begin - jobs[g.job].base, g.count, split, dim, lo, hi, d);
      g.emit = eidx;
      g.dim = dim;
      g.split = split;
    }
    if (dim < 0) {
      if (lane == 0) {
        tile_left[t] = 0;
        tile_q[t] = 0;
      }
      continue;
    }
    const uint64_t tstart = (uint64_t)g.begin + (uint64_t)(t - g.tile_begin) * kTile;
    const uint64_t tend = min((uint64_t)g.begin + g.count, tstart + kTile);
    const float* x = src + (uint64_t)dim * cap;
    // loads at a clamped index (always in the tile) so that none waits on
    // a branch and all of them can be in flight together; counts per
    // quarter of the tile (eight rows each)
    uint32_t cq[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int r = 0; r < kTile / 64; ++r) {
      const uint64_t i = tstart + (uint64_t)r * 64 + lane;
      const float xv = x[i < tend ? i : tend - 1];
      cq[r / (kTile / 256)] += (uint32_t)__popcll(__ballot((i < tend) & (xv < split)));
    }
    if (lane == 0) {
      tile_left[t] = cq[0] + cq[1] + cq[2] + cq[3];
      tile_q[t] = pack_quarters(cq[0], cq[0] + cq[1], cq[0] + cq[1] + cq[2]);
    }
  }
}

__global__ void __launch_bounds__(kPassThreads)
k_count(Seg* cur, const uint32_t* tile_seg, BuildCounters* c, int par, const Job* jobs,
        uint32_t* emit, int es, int d, uint32_t leaf, const float* src, uint64_t cap,
        uint32_t* tile_left, uint32_t* tile_q, int rule) {
  constexpr int kWaves = kPassThreads / 64;
  count_tiles(cur, tile_seg, c, par, jobs, emit, es, d, leaf, src, cap, tile_left, tile_q, rule,
              blockIdx.x * kWaves + (threadIdx.x >> 6), gridDim.x * kWaves);
}

// Object median of the global passes: a radix select per segment over the
// ordered-u32 keys of its coordinates in the split dimension, four rounds of
// 8-bit digits from the most significant.  In round r a tile counts, per
// digit, its keys whose higher digits equal the segment's digits selected so
// far (all keys in round 0); the pick kernel then finds the digit holding
// the sought rank (floor(count/2) in round 0) and narrows the rank to it.
// After four rounds sel_key is the key of that rank.  One wavefront per tile,
// as in the count; the workgroup's wavefronts merge their counts per segment
// before the device atomics.
template <int kWaves>
__device__ __forceinline__ void sel_hist_tiles(const Seg* cur, const uint32_t* tile_seg,
                                               const BuildCounters* c, int par, int d,
                                               uint32_t leaf, const float* src, uint64_t cap,
                                               uint32_t* hist, int round, uint32_t blk,
                                               uint32_t nblk) {
  static_assert(kWaves * 64 >= 256, "one thread per digit in the merge");
  __shared__ uint32_t h[kWaves][256];
  __shared__ uint32_t hs[kWaves];
  const uint32_t nt = ld_ctr(&c->ntiles[par]);
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  const uint64_t below = lanemask_lt();
  const int shift = 24 - 8 * round;
  const uint32_t nw = nblk * kWaves;
  // every wavefront of the workgroup runs the same rounds (barriers inside)
  for (uint32_t t0 = blk * kWaves; t0 < nt; t0 += nw) {
    const uint32_t t = t0 + w;
    for (int i = lane; i < 256; i += 64) h[w][i] = 0u;
    uint32_t s = kNone;
    if (t < nt) {
      s = tile_seg[t];
      const Seg& g = cur[s];
      const uint32_t* lo = g.box;
      const uint32_t* hi = g.box + kMaxDim;
      bool degenerate = true;
      for (int j = 0; j < d; ++j) degenerate = degenerate && (lo[j] == hi[j]);
      if (g.count <= leaf || degenerate || g.depth >= (uint32_t)kMaxDepth) {
        s = kNone;
      } else {
        const int dim = choose_dim(lo, hi, d, (int)g.depth);
        const uint32_t pref = round == 0 ? 0u : g.sel_key;
        const uint64_t tstart = (uint64_t)g.begin + (uint64_t)(t - g.tile_begin) * kTile;
        const uint64_t tend = min((uint64_t)g.begin + g.count, tstart + kTile);
        const float* x = src + (uint64_t)dim * cap;
        for (uint64_t i0 = tstart; i0 < tend; i0 += 64) {
          const uint64_t i = i0 + lane;
          const bool in = i < tend;
          const uint32_t key = in ? f2o(x[i]) : 0u;
          // higher digits equal those selected so far (64-bit shifts: in
          // round 0 there are none and both sides are 0)
          const bool match =
              in && ((uint64_t)key >> (shift + 8)) == ((uint64_t)pref >> (shift + 8));
          const uint32_t dig = (key >> shift) & 255u;
          const uint64_t m = digit_peers8(dig, match);
          if (match && (m & below) == 0) atomicAdd(&h[w][dig], (uint32_t)__popcll(m));
        }
      }
    }
    if (lane == 0) hs[w] = s;
    __syncthreads();
    // thread b owns digit b: each segment among the wavefronts adds its sum once
    const int b = threadIdx.x;
    for (int v = 0; v < kWaves && b < 256; ++v) {
      const uint32_t sv = hs[v];
      bool first = sv != kNone;
      for (int u = 0; u < v; ++u) first = first && hs[u] != sv;
      if (!first) continue;
      uint32_t sum = 0;
      for (int u = v; u < kWaves; ++u) sum += hs[u] == sv ? h[u][b] : 0u;
      if (sum) atomicAdd(&hist[(uint64_t)sv * 256 + b], sum);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kPassThreads)
k_sel_hist(const Seg* cur, const uint32_t* tile_seg, const BuildCounters* c, int par, int d,
           uint32_t leaf, const float* src, uint64_t cap, uint32_t* hist, int round) {
  sel_hist_tiles<kPassThreads / 64>(cur, tile_seg, c, par, d, leaf, src, cap, hist, round,
                                    blockIdx.x, gridDim.x);
}

// One wavefront per segment: the digit of round r that holds the sought rank;
// clears the segment's counts for the next round.
__device__ __forceinline__ void sel_pick_segs(Seg* cur, const BuildCounters* c, int par,
                                              uint32_t* hist, int round, uint32_t wv,
                                              uint32_t nwv) {
  const uint32_t ns = ld_ctr(&c->nseg[par]);
  const int lane = __lane_id();
  const int shift = 24 - 8 * round;
  for (uint32_t s = wv; s < ns; s += nwv) {
    Seg& g = cur[s];
    uint32_t* hr = hist + (uint64_t)s * 256;
    const uint4 hv = reinterpret_cast<const uint4*>(hr)[lane];
    reinterpret_cast<uint4*>(hr)[lane] = make_uint4(0u, 0u, 0u, 0u);
    const uint32_t hb[4] = {hv.x, hv.y, hv.z, hv.w};
    const uint32_t own = hb[0] + hb[1] + hb[2] + hb[3];
    const uint32_t incl = wave_incl_scan(own);
    // a leaf segment counted nothing: no lane holds the rank
    const uint32_t rank = round == 0 ? g.count / 2u : g.sel_rank;
    const uint32_t pref = round == 0 ? 0u : g.sel_key;
    const uint32_t excl = incl - own;
    if (excl <= rank && rank < incl) {
      uint32_t cum = excl;
      int q = 0;
      while (q < 3 && rank >= cum + hb[q]) cum += hb[q++];
      g.sel_key = pref | ((uint32_t)(lane * 4 + q) << shift);
      g.sel_rank = rank - cum;
    }
  }
}

__global__ void __launch_bounds__(kPassThreads)
k_sel_pick(Seg* cur, const BuildCounters* c, int par, uint32_t* hist, int round) {
  constexpr int kWaves = kPassThreads / 64;
  sel_pick_segs(cur, c, par, hist, round, blockIdx.x * kWaves + (threadIdx.x >> 6),
                gridDim.x * kWaves);
}

// Prefix sum of the tiles' left counts; create the children of every split
// segment: large ones go to the next depth's list, small ones to the
// finisher.
// One workgroup of any multiple of 64 threads up to 1024.
__device__ __forceinline__ void tilescan_block(Seg* cur, Seg* nxt, BuildCounters* c, int par,
                                               const uint32_t* tile_left, uint32_t* tile_off,
                                               Fin* fin, uint32_t T, uint64_t max_seg,
                                               uint64_t max_fin, int d, uint32_t* segtb,
                                               uint32_t* tile_seg_next, uint64_t max_tiles,
                                               uint64_t max_emit) {
  const int d4 = (d + 3) & ~3;
  __shared__ uint32_t wsum[17];
  // list sizes are counted in LDS (this is the only workgroup) and stored once
  __shared__ uint32_t s_nseg, s_nfin, s_n;
  // per-job node counts and heights of the next depth
  __shared__ uint32_t s_jn[kMaxJobs], s_jh[kMaxJobs];
  __shared__ uint32_t s_tb[kListLds];
  const uint32_t nt = ld_ctr(&c->ntiles[par]);
  const uint32_t ns = ld_ctr(&c->nseg[par]);
  if (threadIdx.x == 0) {
    s_nseg = 0;
    s_nfin = ld_ctr(&c->nfin);
  }
  if (threadIdx.x < kMaxJobs) {
    s_jn[threadIdx.x] = 0;
    s_jh[threadIdx.x] = 0;
  }
  __syncthreads();
  uint32_t carry = 0;
  for (uint32_t ch = 0; ch < nt; ch += blockDim.x) {
    uint32_t t = ch + threadIdx.x;
    uint32_t v = t < nt ? tile_left[t] : 0u;
    uint32_t tot;
    uint32_t ex = block_excl_scan(v, wsum, &tot);
    if (t < nt) tile_off[t] = carry + ex;
    carry += tot;
  }
  __syncthreads();
  // every thread runs the same number of rounds, so that list slots can be
  // taken with one LDS atomic per wavefront
  for (uint32_t s0 = 0; s0 < ns; s0 += blockDim.x) {
    const uint32_t s = s0 + threadIdx.x;
    const bool split = s < ns && cur[s].dim >= 0;
    if (s < ns && !split) cur[s].child[0] = cur[s].child[1] = kNone;
    uint32_t nl = 0, gbegin = 0, gcount = 0;
    if (split) {
      Seg& g = cur[s];
      const uint32_t last = g.tile_begin + g.ntiles;
      const uint32_t g0 = tile_off[g.tile_begin];
      const uint32_t g1 = last < nt ? tile_off[last] : carry;
      nl = g1 - g0;
      g.nleft = nl;
      gbegin = g.begin;
      gcount = g.count;
    }
    for (int side = 0; side < 2; ++side) {
      const uint32_t cb = side ? gbegin + nl : gbegin;
      const uint32_t cc = side ? gcount - nl : nl;
      const bool to_seg = split && cc > T;
      const bool to_fin = split && !(cc > T);
      const uint32_t k = wave_alloc(&s_nseg, to_seg);
      const uint32_t f = wave_alloc(&s_nfin, to_fin);
      {
        // the next depth's nodes per job: one LDS update per job and wavefront
        const uint32_t cj = split ? cur[s].job : 0u;
        const uint64_t m = job_peers(cj, to_seg);
        if (to_seg && (m & lanemask_lt()) == 0) {
          atomicAdd(&s_jn[cj], (uint32_t)__popcll(m));
          atomicMax(&s_jh[cj], cur[s].depth + 2u);
        }
      }
      if (!split) continue;
      Seg& g = cur[s];
      const uint64_t cpath = (g.path << 1) | (uint64_t)side;
      if (to_seg) {
        if (k >= max_seg) {
          atomicOr(&c->err, 8u);
          g.child[side] = kNone;
          continue;
        }
        Seg& h = nxt[k];
        h.begin = cb;
        h.count = cc;
        h.job = g.job;
        h.depth = g.depth + 1;
        h.path = cpath;
        h.parent_emit = g.emit;
        h.side = (uint32_t)side;
        // neutral bounds for the first d dimensions (the only ones used),
        // four at a time
        for (int j = 0; j < d4; j += 4) {
          *reinterpret_cast<uint4*>(&h.box[j]) =
              make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
          *reinterpret_cast<uint4*>(&h.box[kMaxDim + j]) = make_uint4(0u, 0u, 0u, 0u);
        }
        g.child[side] = k;
      } else {
        g.child[side] = kNone;
        if (f >= max_fin) {
          atomicOr(&c->err, 16u);
          continue;
        }
        Fin& F = fin[f];
        F.begin = cb;
        F.count = cc;
        F.job = g.job;
        F.depth = g.depth + 1;
        F.path = cpath;
        F.parent_emit = g.emit;
        F.side = (uint32_t)side;
        F.bufsel = (uint32_t)(par ^ 1);
      }
    }
  }
  __syncthreads();
  // the next depth's list: emit range, overflow checks, tile numbering
  if (threadIdx.x == 0) {
    c->nfin = s_nfin;
    uint32_t nn = s_nseg;
    if (nn > max_seg || ld_ctr(&c->err)) {
      // an overflow was flagged: stop working on these trees
      if (nn > max_seg) atomicOr(&c->err, 8u);
      nn = 0;
    }
    const uint32_t base = ld_ctr(&c->nemit);
    if ((uint64_t)base + nn > max_emit) {
      atomicOr(&c->err, 4u);
      nn = 0;
    }
    c->ebase[par ^ 1] = base;
    c->nemit = base + nn;
    s_n = nn;
  }
  __syncthreads();
  const uint32_t n = s_n;
  if (threadIdx.x < kMaxJobs && s_jn[threadIdx.x] && n) {
    atomicAdd(&c->job_nodes[threadIdx.x], s_jn[threadIdx.x]);
    atomicMax(&c->job_height[threadIdx.x], s_jh[threadIdx.x]);
  }
  carry = 0;
  for (uint32_t k0 = 0; k0 < n; k0 += blockDim.x) {
    const uint32_t k = k0 + threadIdx.x;
    const uint32_t ntl = k < n ? (nxt[k].count + kTile - 1) / kTile : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(ntl, wsum, &tot);
    if (k < n) {
      nxt[k].tile_begin = carry + ex;
      nxt[k].ntiles = ntl;
      segtb[k] = carry + ex;
      if (k < kListLds) s_tb[k] = carry + ex;
    }
    carry += tot;
  }
  const bool over = carry > max_tiles;
  if (threadIdx.x == 0) {
    if (over) atomicOr(&c->err, 256u);
    c->nseg[par ^ 1] = over ? 0u : n;
    c->ntiles[par ^ 1] = over ? 0u : carry;
    // the next depth's list is non-empty: the passes run at least to it
    if (n) c->deepest = nxt[0].depth + 1u > c->deepest ? nxt[0].depth + 1u : c->deepest;
  }
  if (over || n == 0) return;
  __syncthreads();
  // segment of every tile of the next depth: the largest k with tile start <= t
  const uint32_t* tb = n <= kListLds ? s_tb : segtb;
  for (uint32_t t = threadIdx.x; t < carry; t += blockDim.x) {
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (tb[mid] <= t) lo = mid; else hi = mid - 1;
    }
    tile_seg_next[t] = lo;
  }
}

__global__ void __launch_bounds__(1024)
k_tilescan(Seg* cur, Seg* nxt, BuildCounters* c, int par, const uint32_t* tile_left,
           uint32_t* tile_off, Fin* fin, uint32_t T, uint64_t max_seg, uint64_t max_fin, int d,
           uint32_t* segtb, uint32_t* tile_seg_next, uint64_t max_tiles, uint64_t max_emit) {
  tilescan_block(cur, nxt, c, par, tile_left, tile_off, fin, T, max_seg, max_fin, d, segtb,
                 tile_seg_next, max_tiles, max_emit);
}

// Add one bound of a child's box to the device copy.  A side with no point
// keeps the neutral value (0xFFFFFFFF for a minimum, 0 for a maximum), which
// no finite coordinate maps to; it is skipped, as is a missing child.
__device__ inline void add_bound(Seg* nxt, uint32_t ch, int j, bool is_max, uint32_t v) {
  if (ch == kNone) return;
  if (is_max) {
    if (v != 0u) atomicMax(&nxt[ch].box[kMaxDim + j], v);
  } else {
    if (v != 0xFFFFFFFFu) atomicMin(&nxt[ch].box[j], v);
  }
}

// Lane 4j+q adds bound q (left min, left max, right min, right max) of
// dimension j of a tile's children.
template <int D>
__device__ inline void add_child_boxes(Seg* nxt, uint32_t c0, uint32_t c1,
                                       const uint32_t (&bx)[D][4], int lane) {
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (lane == 4 * j + q) add_bound(nxt, q < 2 ? c0 : c1, j, q & 1, bx[j][q]);
}

// Stable partition of every tile into the other build buffer; accumulates
// the tight boxes of children that stay in the global passes; leaves that
// are too large for the finisher (coincident points) are copied out whole.
// One wavefront per tile walks its rows of 64 points in order: a ballot per
// row gives every point its rank among the tile's left (or right) points,
// with the running count held wave-uniform, so no LDS or barrier is needed.
// D is the dimension: all columns of a row are read once, and the children's
// boxes are kept in registers for all dimensions.  A wavefront's last tile
// does not add its boxes to the device right away: the workgroup's
// wavefronts hold consecutive tiles, mostly of one segment near the root,
// and merge their boxes first, so that the device atomics on a child's box
// (all of which meet at one address) are fewer by the wavefront count.
constexpr int kScatterThreads = 512;

template <int D, int kWaves>
__device__ __forceinline__ void scatter_tiles(const Seg* cur, const uint32_t* tile_seg, Seg* nxt,
                                              const BuildCounters* c, int par,
                                              const float* __restrict__ src,
                                              float* __restrict__ dst, uint64_t cap,
                                              const uint32_t* tile_off,
                                              const uint32_t* tile_q, const Job* jobs,
                                              uint64_t* map, uint32_t idcap, uint32_t blk,
                                              uint32_t nblk) {
  __shared__ uint32_t s_ch[kWaves][2];
  __shared__ uint32_t s_bx[kWaves][4 * D];
  const uint32_t nt = ld_ctr(&c->ntiles[par]);
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  const uint64_t below = lanemask_lt();
  const uint32_t* sid = soa_ids(src, D, cap);
  uint32_t* did = soa_ids_w(dst, D, cap);
  const uint32_t nw = nblk * kWaves;
  // this wavefront's slot of the workgroup merge: its last tile's children
  // and boxes (empty until then)
  if (lane < 2) s_ch[w][lane] = kNone;
  if (lane < 4 * D) s_bx[w][lane] = (lane & 1) ? 0u : 0xFFFFFFFFu;
  // work units are quarter tiles (eight rows), unit un = 4 * tile + quarter
  const uint32_t nu = nt * 4u;
  for (uint32_t un = blk * kWaves + w; un < nu; un += nw) {
    const uint32_t t = un >> 2, qt = un & 3u;
    const uint32_t s = tile_seg[t];
    const Seg& g = cur[s];
    const uint64_t gbegin = g.begin;
    const uint64_t tstart = gbegin + (uint64_t)(t - g.tile_begin) * kTile;
    const uint64_t tend = min(gbegin + g.count, tstart + kTile);
    const uint32_t tcnt = (uint32_t)(tend - tstart);
    // this unit's points: tile positions [i0, i1)
    const uint32_t i0 = qt * (kTile / 4);
    const uint32_t i1 = min(tcnt, i0 + (uint32_t)(kTile / 4));
    if (i0 >= i1) continue;
    const int dim = g.dim;
    if (dim < 0) {
      const Job J = jobs[g.job];
      constexpr int S = (D + 1 + 3) & ~3;
      for (uint32_t i = i0 + lane; i < i1; i += 64) {
        const uint64_t p = tstart + i;
        const uint64_t slot = p - J.base;
        float* rr = J.rec + slot * S;
#pragma unroll
        for (int j = 0; j < D; ++j) rr[j] = src[(uint64_t)j * cap + p];
        const uint32_t id = sid[p];
        rr[D] = __uint_as_float(id);
#pragma unroll
        for (int j = D + 1; j < S; ++j) rr[j] = 0.0f;
        if (J.write_map && id < idcap) map[id] = ((uint64_t)J.level << 32) | slot;
      }
      continue;
    }
    const float split = g.split;
    const uint32_t tloff = tile_off[t] - tile_off[g.tile_begin];
    const uint64_t lbase = gbegin + tloff;
    const uint64_t rbase = gbegin + g.nleft + ((tstart - gbegin) - tloff);
    uint32_t bx[D][4];  // left min, left max, right min, right max (ordered u32)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      bx[j][0] = 0xFFFFFFFFu;
      bx[j][1] = 0u;
      bx[j][2] = 0xFFFFFFFFu;
      bx[j][3] = 0u;
    }
    // left points in earlier rows of the tile (earlier quarters from the count)
    uint32_t lrun = left_before_quarter(tile_q[t], qt);
    // groups of kRows rows: all loads of a group are issued before its
    // stores (indices are clamped into the unit, so no load waits on a branch)
    constexpr int kRows = 4;
    for (uint32_t r0 = i0 / 64; r0 * 64 < i1; r0 += kRows) {
      float v[kRows][D];
      uint32_t idv[kRows];
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        const uint32_t i = (r0 + u) * 64 + lane;
        const uint64_t p = tstart + (i < i1 ? i : i1 - 1);
#pragma unroll
        for (int j = 0; j < D; ++j) v[u][j] = src[(uint64_t)j * cap + p];
        idv[u] = sid[p];
      }
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        const uint32_t i = (r0 + u) * 64 + lane;
        const bool in = i < i1;
        float vd = 0.0f;
#pragma unroll
        for (int j = 0; j < D; ++j) vd = j == dim ? v[u][j] : vd;
        const bool f = in && vd < split;
        const uint64_t m = __ballot(f);
        const uint32_t lr = lrun + (uint32_t)__popcll(m & below);
        lrun += (uint32_t)__popcll(m);
        if (in) {
          const uint64_t dp = f ? lbase + lr : rbase + (i - lr);
#pragma unroll
          for (int j = 0; j < D; ++j) {
            dst[(uint64_t)j * cap + dp] = v[u][j];
            const uint32_t o = f2o(v[u][j]);
            const int q = f ? 0 : 2;
            bx[j][q] = o < bx[j][q] ? o : bx[j][q];
            bx[j][q + 1] = o > bx[j][q + 1] ? o : bx[j][q + 1];
          }
          did[dp] = idv[u];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
      wave_minmax(bx[j][0], bx[j][1]);
      wave_minmax(bx[j][2], bx[j][3]);
    }
    const uint32_t c0 = g.child[0], c1 = g.child[1];
    if (un + nw < nu) {
      add_child_boxes<D>(nxt, c0, c1, bx, lane);
    } else {
      if (lane == 0) {
        s_ch[w][0] = c0;
        s_ch[w][1] = c1;
      }
#pragma unroll
      for (int j = 0; j < D; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (lane == 4 * j + q) s_bx[w][4 * j + q] = bx[j][q];
    }
  }
  // workgroup merge: runs of wavefronts with the same child combine their
  // bounds before one device atomic per run
  __syncthreads();
  if (w == 0 && lane < 4 * D) {
    const int j = lane >> 2, q = lane & 3;
    const bool is_max = q & 1;
    const uint32_t neutral = is_max ? 0u : 0xFFFFFFFFu;
    uint32_t run_ch = kNone, acc = neutral;
    for (int v = 0; v < kWaves; ++v) {
      const uint32_t ch = s_ch[v][q >> 1];
      const uint32_t x = s_bx[v][lane];
      if (ch != run_ch) {
        add_bound(nxt, run_ch, j, is_max, acc);
        run_ch = ch;
        acc = x;
      } else {
        acc = is_max ? (x > acc ? x : acc) : (x < acc ? x : acc);
      }
    }
    add_bound(nxt, run_ch, j, is_max, acc);
  }
}

template <int D>
__global__ void __launch_bounds__(kScatterThreads)
__attribute__((amdgpu_waves_per_eu(D <= 3 ? 8 : 1)))  // d <= 3 fits 64 VGPRs without spills
k_scatter(const Seg* cur, const uint32_t* tile_seg, Seg* nxt, const BuildCounters* c, int par,
          const float* __restrict__ src, float* __restrict__ dst, uint64_t cap,
          const uint32_t* tile_off, const uint32_t* tile_q, const Job* jobs, uint64_t* map,
          uint32_t idcap) {
  scatter_tiles<D, kScatterThreads / 64>(cur, tile_seg, nxt, c, par, src, dst, cap, tile_off,
                                         tile_q, jobs, map, idcap, blockIdx.x, gridDim.x);
}

// Arguments of the depth loop (every buffer of the global passes).
struct PassArgs {
  Seg* seg[2];
  uint32_t* tile_seg[2];
  uint32_t* segtb[2];
  float* soa[2];
  BuildCounters* c;
  const Job* jobs;
  uint32_t* emit;
  uint32_t* tile_left;
  uint32_t* tile_q;
  uint32_t* tile_off;
  Fin* fin;
  uint64_t* map;
  uint32_t* sel_hist;
  uint64_t cap, max_seg, max_fin, max_tiles, max_emit;
  uint32_t T, leaf, idcap;
  int es, d, rule, par0, depth0;
};

// All remaining depths of the global passes in one cooperative launch: the
// workgroups run count, list and scatter (and the object median's select
// rounds) of a depth with a grid-wide barrier between the steps, and stop
// when the depth's list is empty (every segment went to the finisher or was
// a leaf), when an error is flagged, or past the depth cap.  The stop test
// reads the counters at the coherence point after a barrier, so every
// workgroup takes the same decision.  The parity of the last list is left in
// par_final for the finisher.
template <int D>
__global__ void __launch_bounds__(kScatterThreads) k_passes(PassArgs A) {
  constexpr int KW = kScatterThreads / 64;
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const uint32_t wv = blockIdx.x * KW + (threadIdx.x >> 6);
  const uint32_t nwv = gridDim.x * KW;
  int par = A.par0;
  for (int depth = A.depth0; depth <= kMaxDepth + 1; ++depth) {
    if (ld_ctr(&A.c->nseg[par]) == 0u || ld_ctr(&A.c->err) != 0u) break;
    if (A.rule == kSplitObject) {
      for (int r = 0; r < 4; ++r) {
        sel_hist_tiles<KW>(A.seg[par], A.tile_seg[par], A.c, par, A.d, A.leaf, A.soa[par],
                           A.cap, A.sel_hist, r, blockIdx.x, gridDim.x);
        grid.sync();
        sel_pick_segs(A.seg[par], A.c, par, A.sel_hist, r, wv, nwv);
        grid.sync();
      }
    }
    count_tiles(A.seg[par], A.tile_seg[par], A.c, par, A.jobs, A.emit, A.es, A.d, A.leaf,
                A.soa[par], A.cap, A.tile_left, A.tile_q, A.rule, wv, nwv);
    grid.sync();
    if (blockIdx.x == 0)
      tilescan_block(A.seg[par], A.seg[par ^ 1], A.c, par, A.tile_left, A.tile_off, A.fin, A.T,
                     A.max_seg, A.max_fin, A.d, A.segtb[par ^ 1], A.tile_seg[par ^ 1],
                     A.max_tiles, A.max_emit);
    grid.sync();
    scatter_tiles<D, KW>(A.seg[par], A.tile_seg[par], A.seg[par ^ 1], A.c, par, A.soa[par],
                         A.soa[par ^ 1], A.cap, A.tile_off, A.tile_q, A.jobs, A.map, A.idcap,
                         blockIdx.x,
                         gridDim.x);
    grid.sync();
    par ^= 1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) A.c->par_final = (uint32_t)par;
}

__global__ void k_set_par_final(BuildCounters* c, int par) {
  if (threadIdx.x == 0) c->par_final = (uint32_t)par;
}

// ------------------------------------------------------------------------
// LDS finisher: one workgroup builds a whole subtree of at most TCAP points
// ------------------------------------------------------------------------

struct Act {
  uint16_t begin, count;
  int8_t dim;
  uint8_t depth;
  float split;
  uint32_t emit;
  uint64_t path;
};

// OBJ selects the object median (Section V-C): after a depth's internal
// nodes are classified, a radix select over 4-bit digits (eight rounds, LDS
// counts per node) finds each node's coordinate of rank floor(count/2) in its
// split dimension, which replaces the spatial split in the node and its
// emitted record.
template <int DMAX, int TCAP, int MAXACT, int NT, bool OBJ>
__global__ void __launch_bounds__(NT)
k_finish(const Fin* fin, const float* soa0, const float* soa1, uint64_t cap, int d,
         uint32_t leaf, const Job* jobs, uint32_t* emit, int es, BuildCounters* c,
         uint64_t* map, uint32_t idcap, uint64_t max_emit) {
  constexpr int PT = (TCAP + NT - 1) / NT;
  constexpr int MAXCH = 2 * MAXACT;
  static_assert(MAXCH <= NT, "one child per thread");
  __shared__ float xs[DMAX][TCAP];
  __shared__ uint32_t ids[TCAP];
  __shared__ uint16_t pos[2][TCAP];
  __shared__ uint16_t sidv[2][TCAP];
  __shared__ uint16_t L[TCAP + 2];
  __shared__ Act act[2][MAXACT];
  __shared__ uint32_t cbox[MAXCH][2 * DMAX];
  __shared__ uint16_t remap[MAXCH];
  __shared__ uint32_t wsum[17];
  __shared__ uint32_t s_nact, s_base, s_maxdepth, s_fi;
  // object median, per internal node of the depth: digits selected so far,
  // rank still sought, box bounds in the split dimension, digit counts
  constexpr int OA = OBJ ? MAXACT : 1;
  __shared__ uint32_t o_key[OA], o_rank[OA], o_lo[OA], o_hi[OA];
  __shared__ uint32_t o_hist[OA][16];

  const int tid = threadIdx.x;
  const int lane = __lane_id();
  const int S = rec_stride(d);

  // The launch follows the global passes without a readback in between:
  // if a segment is still above the threshold (or an error was flagged) the
  // lists are incomplete, so nothing is done and the host is asked for more
  // passes and a new launch.
  __shared__ uint32_t s_go;
  if (tid == 0) {
    const uint32_t par_end = c->par_final & 1u;
    const uint32_t e = c->err;
    const bool stop = e != 0u || c->nseg[par_end] != 0u;
    if (stop && e == 0u && blockIdx.x == 0) c->retry = 1u;
    s_go = stop ? 0u : 1u;
  }
  __syncthreads();
  if (!s_go) return;
  const uint32_t nfin = c->nfin;
  // entries are taken from a counter, so that the grid can be one
  // resident wave of workgroups whatever the list size
  while (true) {
    if (tid == 0) s_fi = atomicAdd(&c->fin_next, 1u);
    __syncthreads();
    const uint32_t fi = s_fi;
    __syncthreads();
    if (fi >= nfin) break;
    const Fin F = fin[fi];
    const uint32_t n = F.count;
    if (n > TCAP || n == 0) {
      if (tid == 0) atomicOr(&c->err, 32u);
      continue;
    }
    // Every child of a depth is emitted, so a depth emits exactly nch nodes
    // and its emit range can be reserved one depth ahead: thread 0 keeps the
    // reservation in flight in a register while the depth's boxes and
    // classification are computed.
    uint32_t ebase_next = 0;
    if (tid == 0) ebase_next = atomicAdd(&c->nemit, 1u);
    const float* src = F.bufsel ? soa1 : soa0;
    const uint32_t* srcid = soa_ids(src, d, cap);
    const Job J = jobs[F.job];
    for (uint32_t i = tid; i < n; i += NT) {
      for (int j = 0; j < d; ++j) xs[j][i] = src[(uint64_t)j * cap + F.begin + i];
      ids[i] = srcid[F.begin + i];
      pos[0][i] = (uint16_t)i;
      sidv[0][i] = 0;
    }
    if (tid < 2 * DMAX) cbox[0][tid] = tid < DMAX ? 0xFFFFFFFFu : 0u;
    if (tid == 0) {
      s_maxdepth = 0;
      s_nact = 0;
    }
    int cur = 0;    // pos/sid buffer holding the current order
    int ca = 0;     // act table of the current depth
    uint32_t nch = 1;
    bool root = true;
    __syncthreads();

    // child boxes by a segmented min/max over positions (children are
    // contiguous runs of equal sid, so a child occurs as one run in a
    // wavefront and equal keys mean the same run): a segmented inclusive
    // scan by DPP steps, whose result at the run's last lane is added to
    // the child's box
    auto child_boxes = [&](int buf) {
      constexpr uint32_t kNoKey = 0xFFFFFFFEu;  // no child has this key
      for (uint32_t b0 = 0; b0 < n; b0 += NT) {
        const uint32_t i = b0 + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? (uint32_t)sidv[buf][i] : (uint32_t)kFrozen;
        const uint32_t p = valid ? (uint32_t)pos[buf][i] : 0u;
        bool same[6];
        same[0] = dpp_move<kDppRowShr1, 0xF>(kNoKey, key) == key;
        same[1] = dpp_move<kDppRowShr2, 0xF>(kNoKey, key) == key;
        same[2] = dpp_move<kDppRowShr4, 0xF>(kNoKey, key) == key;
        same[3] = dpp_move<kDppRowShr8, 0xF>(kNoKey, key) == key;
        same[4] = dpp_move<kDppRowBcast15, 0xA>(kNoKey, key) == key;
        same[5] = dpp_move<kDppRowBcast31, 0xC>(kNoKey, key) == key;
        const uint32_t kn = (uint32_t)__shfl_down((int)key, 1, 64);
        const bool last = key != kFrozen && (lane == 63 || kn != key);
        for (int j = 0; j < d; ++j) {
          uint32_t lo = valid ? f2o(xs[j][p]) : 0u;
          uint32_t hi = lo;
          auto step = [&](bool sm, uint32_t olo, uint32_t ohi) {
            if (sm) {
              lo = olo < lo ? olo : lo;
              hi = ohi > hi ? ohi : hi;
            }
          };
          step(same[0], dpp_move<kDppRowShr1, 0xF>(lo, lo), dpp_move<kDppRowShr1, 0xF>(hi, hi));
          step(same[1], dpp_move<kDppRowShr2, 0xF>(lo, lo), dpp_move<kDppRowShr2, 0xF>(hi, hi));
          step(same[2], dpp_move<kDppRowShr4, 0xF>(lo, lo), dpp_move<kDppRowShr4, 0xF>(hi, hi));
          step(same[3], dpp_move<kDppRowShr8, 0xF>(lo, lo), dpp_move<kDppRowShr8, 0xF>(hi, hi));
          step(same[4], dpp_move<kDppRowBcast15, 0xA>(lo, lo),
               dpp_move<kDppRowBcast15, 0xA>(hi, hi));
          step(same[5], dpp_move<kDppRowBcast31, 0xC>(lo, lo),
               dpp_move<kDppRowBcast31, 0xC>(hi, hi));
          if (last) {
            atomicMin(&cbox[key][j], lo);
            atomicMax(&cbox[key][DMAX + j], hi);
          }
        }
      }
    };

    child_boxes(cur);
    __syncthreads();

    // Per depth: classify the children of the previous depth (their sizes
    // come from the previous depth's left-count prefix L), emit them, flag
    // every point's side with a block scan, scatter.  A child's table entry
    // is found through remap[], so positions are not renumbered in a pass of
    // their own.
    while (true) {
      // ---- classify the children of the previous depth (or the root) ----
      const int na = ca ^ 1;  // table that receives this depth's internal nodes
      uint32_t cbegin = 0, ccount = 0, cdepth = 0, cparent = kNone, cside = 0, le = 0;
      uint32_t ai = kNone;
      uint64_t cpath = 0;
      int cdim = -1;
      float csplit = 0.0f;
      const bool have = (uint32_t)tid < nch;
      bool want_act = false;
      if (have) {
        const uint32_t ch = (uint32_t)tid;
        if (root) {
          cbegin = 0;
          ccount = n;
          cdepth = F.depth;
          cpath = F.path;
          cparent = F.parent_emit;
          cside = F.side;
        } else {
          const Act& A = act[ca][ch >> 1];
          const uint32_t nl = (uint32_t)L[A.begin + A.count] - (uint32_t)L[A.begin];
          cside = ch & 1u;
          cbegin = cside ? A.begin + nl : A.begin;
          ccount = cside ? A.count - nl : nl;
          cdepth = A.depth + 1u;
          cpath = (A.path << 1) | (uint64_t)cside;
          cparent = A.emit;
        }
        const uint32_t* lo = cbox[ch];
        const uint32_t* hi = cbox[ch] + DMAX;
        bool degenerate = true;
        for (int j = 0; j < d; ++j) degenerate = degenerate && lo[j] == hi[j];
        const bool isleaf = ccount <= leaf || degenerate || cdepth >= (uint32_t)kMaxDepth;
        if (!isleaf) choose_split(lo, hi, d, (int)cdepth, &cdim, &csplit);
        le = ch;
        want_act = !isleaf;
      }
      // internal children get act-table slots, one LDS atomic per wavefront
      {
        const uint32_t slot = wave_alloc(&s_nact, want_act);
        if (want_act) {
          ai = slot;
          if (ai >= (uint32_t)MAXACT) {
            atomicOr(&c->err, 64u);
            ai = kNone;
          }
        }
      }
      if (have) remap[tid] = ai == kNone ? kFrozen : (uint16_t)ai;
      // all children of a depth have the same depth
      if (tid == 0) s_maxdepth = cdepth > s_maxdepth ? cdepth : s_maxdepth;
      if (tid == 0) {
        uint32_t base = ebase_next;
        if ((uint64_t)base + nch > max_emit) {
          atomicOr(&c->err, 128u);
          base = 0xFFFFFFFFu;
        } else {
          atomicAdd(&c->job_nodes[F.job], nch);
        }
        s_base = base;
      }
      __syncthreads();
      if (have && s_base != 0xFFFFFFFFu) {
        const uint32_t eidx = s_base + le;
        write_emit(emit, es, eidx, cpath, cdepth, F.job, cparent, cside,
                   F.begin + cbegin - J.base, ccount, csplit, cdim, cbox[tid], cbox[tid] + DMAX, d);
        if (ai != kNone) {
          Act& A = act[na][ai];
          A.begin = (uint16_t)cbegin;
          A.count = (uint16_t)ccount;
          A.dim = (int8_t)cdim;
          A.depth = (uint8_t)cdepth;
          A.split = csplit;
          A.emit = eidx;
          A.path = cpath;
          if constexpr (OBJ) {
            o_lo[ai] = cbox[tid][cdim];
            o_hi[ai] = cbox[tid][DMAX + cdim];
          }
        }
      }
      root = false;
      __syncthreads();
      const uint32_t nact =
          (s_base == 0xFFFFFFFFu || s_nact > (uint32_t)MAXACT) ? 0u : s_nact;
      if (nact == 0) break;
      ca = na;
      if constexpr (OBJ) {
        // ---- object median: radix select of rank floor(count/2) per node ----
        for (uint32_t a = tid; a < nact; a += NT) {
          o_key[a] = 0u;
          o_rank[a] = (uint32_t)act[ca][a].count / 2u;
        }
        for (int r = 0; r < 8; ++r) {
          const int shift = 28 - 4 * r;
          for (uint32_t e = tid; e < nact * 16u; e += NT) o_hist[e >> 4][e & 15u] = 0u;
          __syncthreads();
          for (uint32_t i = tid; i < n; i += NT) {
            const uint16_t s0 = sidv[cur][i];
            const uint16_t sx = s0 == kFrozen ? kFrozen : remap[s0];
            if (sx == kFrozen) continue;
            const uint32_t key = f2o(xs[act[ca][sx].dim][pos[cur][i]]);
            // higher digits equal those selected so far (none in round 0)
            if (((uint64_t)key >> (shift + 4)) == ((uint64_t)o_key[sx] >> (shift + 4)))
              atomicAdd(&o_hist[sx][(key >> shift) & 15u], 1u);
          }
          __syncthreads();
          for (uint32_t a = tid; a < nact; a += NT) {
            const uint32_t rank = o_rank[a];
            uint32_t cum = 0;
            int g = 0;
            while (g < 15 && rank >= cum + o_hist[a][g]) cum += o_hist[a][g++];
            o_key[a] |= (uint32_t)g << shift;
            o_rank[a] = rank - cum;
          }
          __syncthreads();
        }
        for (uint32_t a = tid; a < nact; a += NT) {
          Act& A = act[ca][a];
          const float sp = o_key[a] > o_lo[a] ? o2f(o_key[a]) : o2f(o_hi[a]);
          A.split = sp;
          emit[(uint64_t)A.emit * es + EF_SPLIT] = __float_as_uint(sp);
        }
        __syncthreads();
      }
      // ---- flags and block-wide exclusive scan (blocked positions) ----
      uint32_t fl = 0, cnt = 0;
#pragma unroll
      for (int q = 0; q < PT; ++q) {
        const uint32_t i = (uint32_t)tid * PT + q;
        if (i < n) {
          const uint16_t s0 = sidv[cur][i];
          const uint16_t s = s0 == kFrozen ? kFrozen : remap[s0];
          if (s != kFrozen) {
            const Act& A = act[ca][s];
            const bool f = xs[A.dim][pos[cur][i]] < A.split;
            fl |= (uint32_t)f << q;
            cnt += f;
          }
        }
      }
      uint32_t tot;
      uint32_t run = block_excl_scan(cnt, wsum, &tot);
#pragma unroll
      for (int q = 0; q < PT; ++q) {
        const uint32_t i = (uint32_t)tid * PT + q;
        if (i < n) L[i] = (uint16_t)run;
        run += (fl >> q) & 1u;
      }
      if (tid == 0) L[n] = (uint16_t)tot;
      __syncthreads();
      nch = 2 * nact;
      if (tid == 0) ebase_next = atomicAdd(&c->nemit, nch);
      // ---- stable scatter into the other position buffer ----
      if (tid == 0) s_nact = 0;
      for (uint32_t i = tid; i < n; i += NT) {
        const uint16_t s0 = sidv[cur][i];
        const uint16_t s = s0 == kFrozen ? kFrozen : remap[s0];
        const uint16_t p = pos[cur][i];
        if (s == kFrozen) {
          pos[cur ^ 1][i] = p;
          sidv[cur ^ 1][i] = kFrozen;
        } else {
          const Act& A = act[ca][s];
          const uint32_t nl = (uint32_t)L[A.begin + A.count] - (uint32_t)L[A.begin];
          const uint32_t lr = (uint32_t)L[i] - (uint32_t)L[A.begin];
          const bool f = L[i + 1] != L[i];
          const uint32_t np =
              f ? A.begin + lr : A.begin + nl + (i - A.begin - lr);
          pos[cur ^ 1][np] = p;
          sidv[cur ^ 1][np] = (uint16_t)(2u * s + (f ? 0u : 1u));
        }
      }
      for (uint32_t e = tid; e < nch * 2 * DMAX; e += NT) {
        const uint32_t j = e % (2 * DMAX);
        cbox[e / (2 * DMAX)][j] = j < (uint32_t)DMAX ? 0xFFFFFFFFu : 0u;
      }
      cur ^= 1;
      __syncthreads();
      child_boxes(cur);
      __syncthreads();
    }
    // ---- write the subtree's points in final slot order ----
    for (uint32_t i = tid; i < n; i += NT) {
      const uint16_t p = pos[cur][i];
      const uint64_t slot = (uint64_t)F.begin + i - J.base;
      float* rr = J.rec + slot * S;
      for (int j = 0; j < d; ++j) rr[j] = xs[j][p];
      const uint32_t id = ids[p];
      rr[d] = __uint_as_float(id);
      for (int j = d + 1; j < S; ++j) rr[j] = 0.0f;
      if (J.write_map && id < idcap) map[id] = ((uint64_t)J.level << 32) | slot;
    }
    if (tid == 0) atomicMax(&c->job_height[F.job], s_maxdepth + 1u);
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// layout
// ------------------------------------------------------------------------

__global__ void k_job_offsets(BuildCounters* c, int njobs, int jobbits) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0, h = 0;
  for (int j = 0; j < njobs; ++j) {
    c->job_node_off[j] = run;
    run += c->job_nodes[j];
    h = c->job_height[j] > h ? c->job_height[j] : h;
  }
  c->max_height = h;
  c->job_bits = (uint32_t)jobbits;
}

// vEB key of every emitted node (its job's height decides the layout); the
// count comes from the device, so no readback precedes the layout.
__global__ void k_layout_keys(const uint32_t* emit, int es, const BuildCounters* c,
                              int job_shift, uint64_t* keys, uint32_t* vals) {
  const uint32_t n = c->nemit;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const uint32_t* r = emit + (uint64_t)e * es;
    const uint64_t path = (uint64_t)r[EF_PATH_LO] | ((uint64_t)r[EF_PATH_HI] << 32);
    const uint32_t job = r[EF_JOB];
    uint64_t key = veb_key((int)c->job_height[job], (int)r[EF_DEPTH], path);
    if (job_shift >= 0) key |= (uint64_t)job << job_shift;
    keys[e] = key;
    vals[e] = e;
  }
}

// After the sort by vEB key: the job of every node, in that order, into the
// first buffer pair (for a stable sort by job that keeps the vEB order
// within each job).
__global__ void k_layout_jobkeys(const uint32_t* emit, int es, const BuildCounters* c,
                                 uint32_t* vals0, const uint32_t* vals1, uint64_t* keys0) {
  const uint32_t n = c->nemit;
  const uint32_t* vin = c->sort_sel ? vals1 : vals0;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const uint32_t e = vin[r];
    keys0[r] = emit[(uint64_t)e * es + EF_JOB];
    vals0[r] = e;
  }
}

__global__ void k_layout_rank(const uint32_t* vals0, const uint32_t* vals1, const uint32_t* emit,
                              int es, const BuildCounters* c, uint32_t* final_of) {
  const uint32_t n = c->nemit;
  const uint32_t* vals = c->sort_sel ? vals1 : vals0;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const uint32_t e = vals[r];
    const uint32_t job = emit[(uint64_t)e * es + EF_JOB];
    final_of[e] = r - c->job_node_off[job];
  }
}

// Write every node at its place in the vEB order.  Nodes are visited in that
// order (order[r] is the emitted node of rank r), so the rows a wavefront
// writes are adjacent.  An internal node's child links are written by its
// children; the node itself leaves those two words alone.
__global__ void k_layout_write(const uint32_t* emit, int es, const BuildCounters* c,
                               const uint32_t* order0, const uint32_t* order1,
                               const uint32_t* final_of, const Job* jobs, int d, uint32_t* err) {
  const int NS = node_stride(d);
  const uint32_t n = c->nemit;
  const uint32_t* order = c->sort_sel ? order1 : order0;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const uint32_t e = order[q];
    const uint32_t* r = emit + (uint64_t)e * es;
    const Job& J = jobs[r[EF_JOB]];
    const uint32_t f = final_of[e];
    const uint32_t parent = r[EF_PARENT];
    const uint32_t fp = parent == kNone ? 0u : final_of[parent];
    if (f >= J.node_cap || (parent != kNone && fp >= J.node_cap)) {
      atomicOr(err, 512u);
      continue;
    }
    float* nd = J.nodes + (uint64_t)f * NS;
    const int dim = (int)r[EF_DIM];
    *reinterpret_cast<float2*>(nd + NF_SPLIT) =
        make_float2(__uint_as_float(r[EF_SPLIT]), __int_as_float(dim));
    if (dim < 0)
      *reinterpret_cast<float2*>(nd + NF_A) =
          make_float2(__uint_as_float(r[EF_BEGIN]), __uint_as_float(r[EF_COUNT]));
    // words NF_PARENT.. (parent, box, zero padding, point count) in 16-byte
    // stores
    const int nbox = 2 * d;
    for (int q4 = NF_PARENT; q4 < NS; q4 += 4) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = q4 + u;
        v[u] = j == NF_PARENT ? __int_as_float(parent == kNone ? -1 : (int)fp)
             : j == NS - 1    ? __uint_as_float(r[EF_COUNT])
             : (j - NF_BOX < nbox ? __uint_as_float(r[EF_BOX + (j - NF_BOX)]) : 0.0f);
      }
      *reinterpret_cast<float4*>(nd + q4) = make_float4(v[0], v[1], v[2], v[3]);
    }
    if (parent != kNone) {
      float* pn = J.nodes + (uint64_t)fp * NS;
      pn[r[EF_SIDE] ? NF_B : NF_A] = __uint_as_float(f);
    }
  }
}

// End of a build: publish every job's node count for its tree (slot
// kMaxLevels is the buffer's tree) and keep any error for the next check on
// the host (a segment left above the finisher's size counts as one).
__global__ void k_build_done(BuildCounters* c, const Job* jobs, int njobs, uint32_t* level_nodes,
                             uint32_t* sticky_err) {
  const int j = threadIdx.x;
  if (j < njobs) {
    const uint32_t lv = jobs[j].level;
    const uint32_t at = lv == kBufferLevel ? (uint32_t)kMaxLevels : lv;
    level_nodes[at] = c->job_nodes[j];
    level_nodes[kLevelHeightBase + at] = c->job_height[j];
  }
  if (j == 0) {
    const uint32_t e = c->err | (c->retry ? 1024u : 0u);
    if (e) atomicOr(sticky_err, e);
    level_nodes[kMaxLevels + 1] = c->deepest;
  }
}

// Node counts of the trees k-NN visits, from the builds' published counts,
// and their kViewBalanced flags from the published heights.
__global__ void k_patch_views(LevelViews* v, const uint32_t* level_nodes, uint32_t leaf,
                              int balanced_ok) {
  const int i = threadIdx.x;
  if (i < v->n) {
    const uint32_t lv = v->v[i].level;
    v->v[i].n_nodes = level_nodes[lv];
    const uint32_t h = level_nodes[kLevelHeightBase + lv];
    // ceil(log2(ceil(slots / leaf)))
    const uint32_t leaves = (v->v[i].n_slots + leaf - 1) / leaf;
    const uint32_t lg = leaves <= 1u ? 0u : 32u - (uint32_t)__clz((int)(leaves - 1u));
    v->v[i].flags = (balanced_ok && h <= lg + (uint32_t)kBalancedMargin) ? kViewBalanced : 0u;
  }
  const bool skewed = i < v->n && !(v->v[i].flags & kViewBalanced);
  if (__ballot(skewed) == 0ull && i == 0) v->flags = kViewBalanced;
  else if (i == 0) v->flags = 0u;
}

struct U32x64 {
  uint32_t v[64];
};

__global__ void k_store_vals(uint32_t* dst, U32x64 vals, int n) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = vals.v[threadIdx.x];
}

__global__ void k_store_views(LevelViews* dst, LevelViews v) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&v);
  uint32_t* out = reinterpret_cast<uint32_t*>(dst);
  for (uint32_t i = threadIdx.x; i < sizeof(LevelViews) / 4; i += blockDim.x) out[i] = src[i];
}

__global__ void k_fill(uint32_t* dst, uint32_t v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

inline unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 4096) {
  uint64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

template <int D>
void launch_scatter_d(unsigned grid, const BuildScratch& sc, int par, uint64_t* map,
                      uint32_t idcap, hipStream_t s) {
  hipLaunchKernelGGL((k_scatter<D>), dim3(grid), dim3(kScatterThreads), 0, s, sc.seg[par],
                     sc.tile_seg[par], sc.seg[par ^ 1], sc.ctr, par, sc.soa[par], sc.soa[par ^ 1],
                     sc.cap, sc.tile_off, sc.tile_left + sc.max_tiles, sc.jobs, map, idcap);
}

void launch_scatter(int d, unsigned grid, const BuildScratch& sc, int par, uint64_t* map,
                    uint32_t idcap, hipStream_t s) {
  switch (d) {
#define BDL_SCATTER_CASE(DD) \
  case DD:                   \
    return launch_scatter_d<DD>(grid, sc, par, map, idcap, s);
    BDL_SCATTER_CASE(1) BDL_SCATTER_CASE(2) BDL_SCATTER_CASE(3) BDL_SCATTER_CASE(4)
    BDL_SCATTER_CASE(5) BDL_SCATTER_CASE(6) BDL_SCATTER_CASE(7) BDL_SCATTER_CASE(8)
    BDL_SCATTER_CASE(9) BDL_SCATTER_CASE(10) BDL_SCATTER_CASE(11) BDL_SCATTER_CASE(12)
    BDL_SCATTER_CASE(13) BDL_SCATTER_CASE(14) BDL_SCATTER_CASE(15) BDL_SCATTER_CASE(16)
#undef BDL_SCATTER_CASE
    default:
      return;
  }
}

// Cooperative launch of the depth loop on one resident wave of workgroups.
template <int D>
hipError_t launch_passes_d(const PassArgs& A, hipStream_t s) {
  static const unsigned g = [] {
    int dev = 0, cus = 0, per = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void*>(&k_passes<D>), kScatterThreads, 0) !=
            hipSuccess ||
        !coop || cus <= 0 || per <= 0)
      return 0u;
    // one workgroup per compute unit: a grid barrier costs more with more
    // workgroups, and this launch only finishes the depths left over
    return (unsigned)cus;
  }();
  if (g == 0) return hipErrorNotSupported;
  PassArgs a = A;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_passes<D>), dim3(g),
                                    dim3(kScatterThreads), args, 0, s);
}

hipError_t launch_passes(int d, const PassArgs& A, hipStream_t s) {
  switch (d) {
#define BDL_PASSES_CASE(DD) \
  case DD:                  \
    return launch_passes_d<DD>(A, s);
    BDL_PASSES_CASE(1) BDL_PASSES_CASE(2) BDL_PASSES_CASE(3) BDL_PASSES_CASE(4)
    BDL_PASSES_CASE(5) BDL_PASSES_CASE(6) BDL_PASSES_CASE(7) BDL_PASSES_CASE(8)
    BDL_PASSES_CASE(9) BDL_PASSES_CASE(10) BDL_PASSES_CASE(11) BDL_PASSES_CASE(12)
    BDL_PASSES_CASE(13) BDL_PASSES_CASE(14) BDL_PASSES_CASE(15) BDL_PASSES_CASE(16)
#undef BDL_PASSES_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <int DMAX, int TCAP, int MAXACT, int NT, bool OBJ>
void launch_finish(const BuildScratch& sc, int d, uint32_t leaf, uint64_t* map, uint32_t idcap,
                   hipStream_t s) {
  // one resident wave of workgroups (computed once; every device here is
  // the same kind)
  static const unsigned g = [] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void*>(&k_finish<DMAX, TCAP, MAXACT, NT, OBJ>), NT, 0) !=
            hipSuccess ||
        cus <= 0 || per <= 0)
      return 512u;
    return (unsigned)(cus * per);
  }();
  hipLaunchKernelGGL((k_finish<DMAX, TCAP, MAXACT, NT, OBJ>), dim3(g), dim3(NT), 0, s, sc.fin,
                     sc.soa[0], sc.soa[1], sc.cap, d, leaf, sc.jobs, sc.emit, emit_stride(d),
                     sc.ctr, map, idcap, sc.max_emit);
}

void launch_finisher(bool obj, const BuildScratch& sc, int d, uint32_t leaf, uint64_t* map,
                     uint32_t idcap, hipStream_t s) {
  if (obj) {
    if (d <= 3) launch_finish<3, 2304, 144, 768, true>(sc, d, leaf, map, idcap, s);
    else if (d <= 8) launch_finish<8, 1024, 64, 256, true>(sc, d, leaf, map, idcap, s);
    else launch_finish<16, 512, 32, 256, true>(sc, d, leaf, map, idcap, s);
  } else {
    if (d <= 3) launch_finish<3, 2304, 144, 768, false>(sc, d, leaf, map, idcap, s);
    else if (d <= 8) launch_finish<8, 1024, 64, 256, false>(sc, d, leaf, map, idcap, s);
    else launch_finish<16, 512, 32, 256, false>(sc, d, leaf, map, idcap, s);
  }
}

}  // namespace

// Finisher configurations: (max dim, LDS point capacity, max internal nodes
// per depth, threads).  The threshold also guarantees that one depth of a
// finisher subtree has at most MAXACT internal nodes (each holds > leaf
// points).  For d <= 3 a workgroup takes 74 KB of LDS, so two share a CU
// (12 waves each); the finisher is bound by LDS latency and barriers, and
// measured faster this way than with one larger workgroup per CU.
uint32_t finisher_threshold(int d, int leaf_size) {
  uint32_t tcap, maxact;
  if (d <= 3) { tcap = 2304; maxact = 144; }
  else if (d <= 8) { tcap = 1024; maxact = 64; }
  else { tcap = 512; maxact = 32; }
  uint64_t t = (uint64_t)maxact * (uint64_t)(leaf_size + 1);
  return (uint32_t)(t < tcap ? t : tcap);
}

size_t build_scratch_bytes(uint64_t cap, int d, uint32_t T) {
  uint64_t max_seg = cap / T + kMaxJobs + 8;
  uint64_t max_tiles = cap / kTile + max_seg + 8;
  uint64_t max_fin = 2 * (uint64_t)(kMaxDepth + 1) * (cap / T + 1) + 2 * kMaxJobs;
  uint64_t max_emit = 2 * cap + kMaxJobs;
  size_t b = 0;
  b += 2 * (size_t)(d + 1) * cap * 4;
  b += 2 * max_seg * (sizeof(Seg) + 4);
  b += 4 * max_tiles * 4;
  b += max_fin * sizeof(Fin);
  b += max_emit * (size_t)emit_stride(d) * 4;
  b += 2 * max_emit * 12 + max_emit * 4;
  b += (radix_tmp_words(max_emit) + scan_tmp_words(cap) + 16) * 4;
  b += (cap / kTile + 2) * 4;
  return b;
}

void launch_pool_to_soa(const PoolSrc& src, int d, uint64_t p0, uint64_t cnt, float* soa,
                        uint64_t cap, uint64_t dst, hipStream_t s) {
  if (!cnt) return;
  hipLaunchKernelGGL(k_pool_to_soa, dim3(grid_for(cnt, 256)), dim3(256), 0, s, src, d, p0, cnt,
                     soa, cap, dst);
}

void launch_pool_to_records(const PoolSrc& src, int d, uint64_t p0, uint64_t cnt, float* rec,
                            uint64_t* map, uint32_t idcap, hipStream_t s) {
  if (!cnt) return;
  hipLaunchKernelGGL(k_pool_to_records, dim3(grid_for(cnt, 256)), dim3(256), 0, s, src, d, p0,
                     cnt, rec, map, idcap);
}

void launch_records_to_soa(const float* rec, int d, uint64_t n, float* soa, uint64_t cap,
                           uint64_t dst, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_records_to_soa, dim3(grid_for(n, 256)), dim3(256), 0, s, rec, d, n, soa,
                     cap, dst);
}

void launch_compact_live(const float* rec, int d, uint64_t n, float* soa, uint64_t cap,
                         uint64_t dst, float* out_rec, uint32_t* tile_cnt, uint32_t* tmp,
                         hipStream_t s) {
  if (!n) return;
  const uint32_t nt = (uint32_t)((n + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_count_live, dim3(nt), dim3(kPassThreads), 0, s, rec, d, n, tile_cnt);
  scan_exclusive_u32(tile_cnt, tile_cnt, nt, nullptr, tmp, s);
  hipLaunchKernelGGL(k_compact_live, dim3(nt), dim3(kPassThreads), 0, s, rec, d, n, tile_cnt,
                     soa, cap, dst, out_rec);
}

void launch_store_u32(uint32_t* dst, const uint32_t* vals, int n, hipStream_t s) {
  U32x64 v;
  for (int i = 0; i < 64; ++i) v.v[i] = i < n ? vals[i] : 0u;
  hipLaunchKernelGGL(k_store_vals, dim3(1), dim3(64), 0, s, dst, v, n);
}

void launch_patch_views(LevelViews* views, const uint32_t* level_nodes, uint32_t leaf,
                        bool balanced_ok, hipStream_t s) {
  static_assert(kMaxViews <= 64, "one lane per view");
  hipLaunchKernelGGL(k_patch_views, dim3(1), dim3(64), 0, s, views, level_nodes, leaf,
                     balanced_ok ? 1 : 0);
}

void launch_store_views(LevelViews* dst, const LevelViews& v, hipStream_t s) {
  hipLaunchKernelGGL(k_store_views, dim3(1), dim3(256), 0, s, dst, v);
}

void launch_fill_u32(uint32_t* dst, uint32_t v, uint64_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, v, n);
}

static int hip_fail(const char** err, const char* what) {
  *err = what;
  return BDL_EHIP;
}

int run_build(const JobTable& jt, BuildScratch& sc, int d, uint32_t leaf, uint32_t T,
              int rule, float depth_ratio, uint64_t* map, uint32_t idcap, hipStream_t s,
              uint32_t* level_nodes, uint32_t* sticky_err, int* base_depths,
              int64_t* host_waits, const char** err, const PhaseTimer& pt) {
  if (base_depths) *base_depths = 0;
  const bool obj = rule == kSplitObject;
  const int njobs = jt.n;
  uint64_t R = 0, maxcount = 0;
  for (int j = 0; j < njobs; ++j) {
    R += jt.jobs[j].count;
    if (jt.jobs[j].count > maxcount) maxcount = jt.jobs[j].count;
  }
  if (R == 0) return 0;
  const int es = emit_stride(d);
  pt.begin(BDL_PH_PASSES);
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(kMaxJobs), 0, s, sc.ctr, jt, sc.jobs);
  {
    dim3 g(grid_for(maxcount, kTile, 256), (unsigned)njobs);
    hipLaunchKernelGGL(k_root_box, g, dim3(kPassThreads), 0, s, sc.soa[0], sc.cap, d, sc.jobs,
                       sc.ctr);
  }
  hipLaunchKernelGGL(k_init_lists, dim3(1), dim3(64), 0, s, sc.jobs, njobs, sc.ctr, sc.seg[0],
                     sc.fin, sc.tile_seg[0], T, sc.max_seg, sc.max_fin, sc.max_tiles);
  // Global passes.  The host launches a budget of depths: the base
  // log2(n / T) + 1, scaled by the ratio of needed to base depths that the
  // tree's recent builds showed (clustered points need two to three times
  // the base); each depth's kernels do nothing once its list is empty.  A cooperative
  // kernel then runs whatever depths are left, on the device, so the host
  // never waits for the build.  Without cooperative launch the host asks the
  // finisher whether more depths are needed (one wait per budget).
  const unsigned pass_grid = grid_for(R, kTile, 2048);
  // one wavefront per segment of a depth (at most max_seg)
  const unsigned sel_grid = grid_for(sc.max_seg, kPassThreads / 64, 1024);
  // four wavefronts of the scatter (one per quarter tile) per tile of R
  // points (a depth has at most R / kTile + segments tiles)
  const unsigned scatter_grid = grid_for(R, kTile * (kScatterThreads / 256), 2048);
  auto launch_depths = [&](int from, int count) {
    for (int depth = from; depth < from + count; ++depth) {
      const int par = depth & 1;
      if (obj) {
        for (int r = 0; r < 4; ++r) {
          hipLaunchKernelGGL(k_sel_hist, dim3(pass_grid), dim3(kPassThreads), 0, s, sc.seg[par],
                             sc.tile_seg[par], sc.ctr, par, d, leaf, sc.soa[par], sc.cap,
                             sc.sel_hist, r);
          hipLaunchKernelGGL(k_sel_pick, dim3(sel_grid), dim3(kPassThreads), 0, s, sc.seg[par],
                             sc.ctr, par, sc.sel_hist, r);
        }
      }
      hipLaunchKernelGGL(k_count, dim3(pass_grid), dim3(kPassThreads), 0, s, sc.seg[par],
                         sc.tile_seg[par], sc.ctr, par, sc.jobs, sc.emit, es, d, leaf,
                         sc.soa[par], sc.cap, sc.tile_left, sc.tile_left + sc.max_tiles, rule);
      hipLaunchKernelGGL(k_tilescan, dim3(1), dim3(1024), 0, s, sc.seg[par], sc.seg[par ^ 1],
                         sc.ctr, par, sc.tile_left, sc.tile_off, sc.fin, T, sc.max_seg,
                         sc.max_fin, d, sc.segtb[par ^ 1], sc.tile_seg[par ^ 1], sc.max_tiles,
                         sc.max_emit);
      launch_scatter(d, scatter_grid, sc, par, map, idcap, s);
    }
  };
  int depth = 0;
  bool host_loop = false;
  if (maxcount > T) {
    int base = 1;
    while (((uint64_t)T << base) < maxcount && base < 40) ++base;
    base += 1;
    if (base_depths) *base_depths = base;
    int budget = (int)ceilf((depth_ratio > 1.0f ? depth_ratio : 1.0f) * (float)base);
    if (budget > kMaxDepth + 1) budget = kMaxDepth + 1;
    launch_depths(0, budget);
    depth = budget;
    PassArgs A;
    for (int i = 0; i < 2; ++i) {
      A.seg[i] = sc.seg[i];
      A.tile_seg[i] = sc.tile_seg[i];
      A.segtb[i] = sc.segtb[i];
      A.soa[i] = sc.soa[i];
    }
    A.c = sc.ctr;
    A.jobs = sc.jobs;
    A.emit = sc.emit;
    A.tile_left = sc.tile_left;
    A.tile_q = sc.tile_left + sc.max_tiles;
    A.tile_off = sc.tile_off;
    A.fin = sc.fin;
    A.map = map;
    A.sel_hist = sc.sel_hist;
    A.cap = sc.cap;
    A.max_seg = sc.max_seg;
    A.max_fin = sc.max_fin;
    A.max_tiles = sc.max_tiles;
    A.max_emit = sc.max_emit;
    A.T = T;
    A.leaf = leaf;
    A.idcap = idcap;
    A.es = es;
    A.d = d;
    A.rule = rule;
    A.par0 = depth & 1;
    A.depth0 = depth;
    if (launch_passes(d, A, s) != hipSuccess) {
      (void)hipGetLastError();
      host_loop = true;
    }
  }
  if (!host_loop) {
    pt.end(BDL_PH_PASSES);
    pt.begin(BDL_PH_FINISH);
    launch_finisher(obj, sc, d, leaf, map, idcap, s);
    pt.end(BDL_PH_FINISH);
  } else {
    while (true) {
      pt.end(BDL_PH_PASSES);
      pt.begin(BDL_PH_FINISH);
      hipLaunchKernelGGL(k_set_par_final, dim3(1), dim3(64), 0, s, sc.ctr, depth & 1);
      launch_finisher(obj, sc, d, leaf, map, idcap, s);
      pt.end(BDL_PH_FINISH);
      if (hipMemcpyAsync(sc.host_ctr, sc.ctr, sizeof(BuildCounters), hipMemcpyDeviceToHost,
                         s) != hipSuccess)
        return hip_fail(err, "counter readback failed");
      if (host_waits) ++*host_waits;
      if (hipStreamSynchronize(s) != hipSuccess) return hip_fail(err, "build passes failed");
      const uint32_t e = sc.host_ctr->err;
      if (e) {
        *err = (e & (32u | 64u | 128u)) ? "build scratch overflow in the finisher"
                                         : "build scratch overflow in the global passes";
        return BDL_EHIP;
      }
      if (!sc.host_ctr->retry) break;
      if (depth > kMaxDepth + 2) {
        *err = "build did not terminate";
        return BDL_EHIP;
      }
      hipLaunchKernelGGL(k_clear_retry, dim3(1), dim3(64), 0, s, sc.ctr);
      pt.begin(BDL_PH_PASSES);
      launch_depths(depth, 4);
      depth += 4;
    }
  }
  // vEB layout: sort the emitted nodes by (job, vEB key) with the node count
  // and the key width read on the device, then write every node at its rank
  int jobbits = 0;
  while ((1 << jobbits) < njobs) ++jobbits;
  pt.begin(BDL_PH_LAYOUT);
  hipLaunchKernelGGL(k_job_offsets, dim3(1), dim3(64), 0, s, sc.ctr, njobs, jobbits);
  // a build of R points emits at most 2R - 1 nodes per job
  const uint64_t ncap = std::min<uint64_t>(sc.max_emit, 2 * R + (uint64_t)njobs);
  const unsigned g = grid_for(ncap, 256);
  hipLaunchKernelGGL(k_layout_keys, dim3(g), dim3(256), 0, s, sc.emit, es, sc.ctr, -1, sc.keys[0],
                     sc.vals[0]);
  radix_sort_pairs_u64_dev(sc.keys, sc.vals, &sc.ctr->nemit, ncap, &sc.ctr->max_height, 64,
                           &sc.ctr->sort_sel, sc.tmp, s);
  if (jobbits > 0) {
    hipLaunchKernelGGL(k_layout_jobkeys, dim3(g), dim3(256), 0, s, sc.emit, es, sc.ctr,
                       sc.vals[0], sc.vals[1], sc.keys[0]);
    radix_sort_pairs_u64_dev(sc.keys, sc.vals, &sc.ctr->nemit, ncap, &sc.ctr->job_bits, 8,
                             &sc.ctr->sort_sel, sc.tmp, s);
  }
  hipLaunchKernelGGL(k_layout_rank, dim3(g), dim3(256), 0, s, sc.vals[0], sc.vals[1], sc.emit,
                     es, sc.ctr, sc.final_of);
  hipLaunchKernelGGL(k_layout_write, dim3(g), dim3(256), 0, s, sc.emit, es, sc.ctr, sc.vals[0],
                     sc.vals[1], sc.final_of, sc.jobs, d, &sc.ctr->err);
  hipLaunchKernelGGL(k_build_done, dim3(1), dim3(kMaxJobs), 0, s, sc.ctr, sc.jobs, njobs,
                     level_nodes, sticky_err);
  pt.end(BDL_PH_LAYOUT);
  if (hipGetLastError() != hipSuccess) return hip_fail(err, "build kernel launch failed");
  return 0;
}

}  // namespace bdl
