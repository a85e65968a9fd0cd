// Host controller of the BDL-tree and the C ABI declared in bdl.h.
//
// The controller only decides: it mirrors F (the bitmask of non-empty static
// trees, Section III-C), every tree's slot and live counts and the buffer's
// size, plans each Insert_L (which trees are built, which are cleared, which
// pool slice goes where) and owns the device memory.  All work on points is
// done by the kernels in build.hip, erase.hip and knn.hip, enqueued on the
// tree's stream.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "baseline.hpp"
#include "bdl.h"
#include "bdl_common.hpp"
#include "build.hpp"
#include "erase.hpp"
#include "knn.hpp"
#include "primitives.hpp"
#include "tree_access.hpp"

using namespace bdl;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Device scratch of bdl_knn_noalloc: the Hilbert-ordering keys and values
// (two ping-pong pairs), the radix sort's partial counts and the query box,
// for at most kNoAllocMaxQueries queries.  Each GPU the library runs on
// holds its own copy until the process ends.  In host code the array's name
// is only a stand-in: host code uses the address that hipGetSymbolAddress
// returns for the current device (scratch_on), never the name itself.
constexpr uint64_t kNoAllocMaxQueries = 1ull << 20;
constexpr uint64_t kNoAllocTmpWords = 1ull << 18;
constexpr uint64_t kNoAllocWords = 4 * kNoAllocMaxQueries + kNoAllocTmpWords + 2 * kMaxDim;
static __device__ __align__(256) uint32_t scratch[kNoAllocWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// Address of `scratch` on device `dev`, which must be current; resolved once
// per device.  Null if the runtime cannot resolve it.
uint32_t* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_tried[dev]) {
    g_scratch_tried[dev] = true;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) {
      g_scratch_ptr[dev] = (uint32_t*)p;
    } else {
      (void)hipGetLastError();
    }
  }
  return g_scratch_ptr[dev];
}

constexpr int kModeBdl = 0;
constexpr int kModeRebuildAll = 1;
constexpr int kModeNoRebuild = 2;

struct LevelState {
  float* rec = nullptr;
  float* nodes = nullptr;
  int64_t cap = 0;
  int64_t n_slots = 0;
  int64_t live = 0;
  int64_t n_nodes = 0;
  bool on = false;
  // Bloom filter of the tree's points for the routed erase, built at the
  // first such erase after the tree changed (2^bloom_log2 words in use)
  uint64_t* bloom = nullptr;
  int64_t bloom_words = 0;
  int bloom_log2 = 0;
  bool bloom_ok = false;
};

}  // namespace

struct bdl_tree {
  bdl_config cfg;
  hipStream_t s = nullptr;
  int dev = 0;
  int rule = kSplitSpatial;  // split heuristic of every tree (BDL_FLAG_OBJECT_MEDIAN)
  // the structure: the BDL-tree, or one of the baselines of Section III-B,
  // which keep one tree as static tree 0 and no buffer
  int mode = 0;              // kModeBdl, kModeRebuildAll (B1), kModeNoRebuild (B2)
  float* b2_alt = nullptr;   // B2: spare record arena the next insert lays out into
  int64_t b2_alt_cap = 0;
  B2Scratch b2{};            // B2: scratch of one insert
  uint64_t b2_pts_cap = 0, b2_box_words = 0, b2_tmp_words = 0;
  uint32_t* noalloc_scratch = nullptr;  // this device's `scratch` (bdl_knn_noalloc)
  int d = 0, S = 0, NS = 0;
  uint32_t T = 0;
  uint64_t F = 0;
  LevelState lev[kMaxLevels];
  // buffer: arrival-order pool (two arrays, ping-pong) and its tree
  float* pool[2] = {nullptr, nullptr};
  int pcur = 0;
  int64_t bn = 0;
  uint64_t* pool_bloom = nullptr;  // the pool's filter (routed erase), rebuilt per erase
  int64_t pool_bloom_words = 0;
  int erase_route = 0;             // BDL_PARAM_ERASE_ROUTE
  GraphScratch graph;              // group list of bdl_knn_graph and its order
  GraphQueries gq;                 // bdl_knn_graph from presorted queries
  int graph_start = 0;             // BDL_PARAM_GRAPH_START
  float* brec = nullptr;
  float* bnodes = nullptr;
  int64_t b_nodes = 0;
  uint64_t* map = nullptr;
  // node counts of the trees, published by the builds on the device
  // (kMaxLevels + 1 words, the last for the buffer's tree); the host learns
  // them from a pinned copy once the builds that wrote them are done
  uint32_t* d_level_nodes = nullptr;
  uint32_t* h_level_nodes = nullptr;  // pinned copy, valid once ev_nodes completes
  hipEvent_t ev_nodes = nullptr;
  bool nodes_pending = false;         // some n_nodes (< 0) wait for that copy
  // ratio of the global-pass depths recent builds needed to their base
  // budget log2(n / T) + 1; the host launches that many depths up front and
  // the device finishes any left
  float depth_ratio = 1.0f;
  int pub_base = 0;                   // base budget of the build last published
  int64_t host_waits = 0;             // times the library blocked on the stream
  uint32_t* d_live = nullptr;   // kMaxLevels
  uint32_t* d_misc = nullptr;   // erase counters [0..1], validation [4..6], error words
                                // [8..9], k-NN graph group count, sort width and buffer [10..12]
  unsigned long long* d_stats = nullptr;  // k-NN work counters (profiling)
  uint32_t* h_pin = nullptr;    // pinned staging, kMaxLevels + 16 words
  BuildScratch sc;
  QueryScratch qs;
  float* rbuf = nullptr;        // Erase_L's gathered points R (records)
  int64_t rbuf_cap = 0;
  int64_t rebuilt = 0, reinserted = 0;
  int knn_mode = kKnnAuto;
  int knn_block = 256;
  int use_graphs = 1;
  int persistent = 2;  // 2: on for the wavefront kernel
  uint64_t query_max = 131072;  // auto: batches up to this size use one wave per query
  int query_stack = 1 << 30;  // pending-node entries per wave of that kernel
  uint64_t sort_min = kSortQueriesMin;
  std::vector<bdl_knn_shape> shapes;  // launch-shape table (autotuned)
  uint32_t* d_queue = nullptr;        // work counters of persistent k-NN launches
  LevelViews* d_views = nullptr;   // the trees kNN_L visits, in device memory
  // batched kNN_L (bdl_knn_batch)
  QueryScratch bqs;                // ordering scratch sized for bcap queries
  uint64_t bcap = 0;
  float* bq = nullptr;             // concatenated queries [bcap][d]
  uint32_t* bqreq = nullptr;       // request of each query
  KnnReqDev* breqs = nullptr;      // request table (kMaxBatchReqs)
  uint64_t* bcount = nullptr;      // [0] total queries, [1] request count
  KnnReqDev* h_breqs[2] = {nullptr, nullptr};  // pinned staging ring
  uint64_t* h_bcount[2] = {nullptr, nullptr};
  hipEvent_t bslot_ev[2] = {nullptr, nullptr};
  int bslot = 0;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  std::map<std::tuple<uint64_t, int, int, int, int>, hipGraphExec_t> graphs;
  size_t held = 0;
  std::unordered_map<void*, size_t> sizes;
  // phase timing (BDL_FLAG_PROFILE)
  PhaseTimer pt;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  hipEvent_t ev_open[BDL_NPHASES] = {};
  double prof_ms[BDL_NPHASES] = {};
  int64_t prof_calls[BDL_NPHASES] = {};
};

namespace {

void* dmalloc(bdl_tree* t, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (t->cfg.mem_budget && t->held + bytes > t->cfg.mem_budget) return nullptr;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  t->held += bytes;
  t->sizes[p] = bytes;
  return p;
}

void dfree(bdl_tree* t, void* p) {
  if (!p) return;
  auto it = t->sizes.find(p);
  if (it != t->sizes.end()) {
    t->held -= it->second;
    t->sizes.erase(it);
  }
  (void)hipFree(p);
}

hipEvent_t take_event(bdl_tree* t) {
  if (!t->ev_free.empty()) {
    hipEvent_t e = t->ev_free.back();
    t->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void phase_mark(void* ctx, int ph, int is_end) {
  bdl_tree* t = (bdl_tree*)ctx;
  if (!is_end) {
    hipEvent_t e = take_event(t);
    if (e && hipEventRecord(e, t->s) == hipSuccess) t->ev_open[ph] = e;
    return;
  }
  hipEvent_t a = t->ev_open[ph];
  t->ev_open[ph] = nullptr;
  if (!a) return;
  hipEvent_t b = take_event(t);
  if (!b || hipEventRecord(b, t->s) != hipSuccess) {
    t->ev_free.push_back(a);
    return;
  }
  t->ev_pending.push_back({ph, {a, b}});
}

// Fold completed event pairs into the per-phase totals.
void resolve_events(bdl_tree* t) {
  for (auto& pe : t->ev_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(pe.second.second) == hipSuccess &&
        hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      t->prof_ms[pe.first] += ms;
      t->prof_calls[pe.first] += 1;
    }
    t->ev_free.push_back(pe.second.first);
    t->ev_free.push_back(pe.second.second);
  }
  t->ev_pending.clear();
}

int64_t level_cap(const bdl_tree* t, int i) { return ((int64_t)1 << i) * t->cfg.buffer_size; }

// Block until the tree's stream is idle (counted in host_waits).
hipError_t wait_stream(bdl_tree* t) {
  ++t->host_waits;
  return hipStreamSynchronize(t->s);
}

// Host copies of the node counts the builds published.  With block, wait for
// the copy; otherwise use it only if it has already arrived.
void resolve_nodes(bdl_tree* t, bool block) {
  if (!t->nodes_pending) return;
  if (block) {
    ++t->host_waits;
    if (hipEventSynchronize(t->ev_nodes) != hipSuccess) return;
  } else if (hipEventQuery(t->ev_nodes) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  for (int i = 0; i < kMaxLevels; ++i)
    if (t->lev[i].on && t->lev[i].n_nodes < 0) t->lev[i].n_nodes = t->h_level_nodes[i];
  if (t->b_nodes < 0) t->b_nodes = t->h_level_nodes[kMaxLevels];
  t->nodes_pending = false;
  // learn how many depths beyond the base budget the last build needed;
  // forget slowly, so that one shallow build does not cost the next deep one
  // a round on the device's leftover path
  if (t->pub_base > 0) {
    const float seen = (float)t->h_level_nodes[kMaxLevels + 1] / (float)t->pub_base;
    const float decayed = t->depth_ratio * 0.9f;
    t->depth_ratio = seen > decayed ? seen : decayed;
    if (t->depth_ratio < 1.0f) t->depth_ratio = 1.0f;
    if (t->depth_ratio > 8.0f) t->depth_ratio = 8.0f;
    t->pub_base = 0;
  }
}

// After a build: bring its node counts to the host when the stream gets
// there (no wait now).
void publish_nodes(bdl_tree* t, int base_depths) {
  t->nodes_pending = true;
  t->pub_base = base_depths;
  if (hipMemcpyAsync(t->h_level_nodes, t->d_level_nodes, (kMaxLevels + 2) * 4,
                     hipMemcpyDeviceToHost, t->s) != hipSuccess ||
      hipEventRecord(t->ev_nodes, t->s) != hipSuccess)
    (void)hipGetLastError();
}

void free_build_scratch(bdl_tree* t) {
  BuildScratch& sc = t->sc;
  for (int i = 0; i < 2; ++i) {
    dfree(t, sc.soa[i]);
    dfree(t, sc.seg[i]);
    dfree(t, sc.segtb[i]);
    dfree(t, sc.keys[i]);
    dfree(t, sc.vals[i]);
  }
  dfree(t, sc.tile_left);
  dfree(t, sc.tile_seg[0]);
  dfree(t, sc.tile_seg[1]);
  dfree(t, sc.tile_off);
  dfree(t, sc.fin);
  dfree(t, sc.emit);
  dfree(t, sc.final_of);
  dfree(t, sc.tmp);
  dfree(t, sc.tile_cnt);
  dfree(t, sc.sel_hist);
  BuildCounters* hc = sc.host_ctr;
  BuildCounters* dc = sc.ctr;
  Job* jb = sc.jobs;
  sc = BuildScratch();
  sc.host_ctr = hc;
  sc.ctr = dc;
  sc.jobs = jb;
}

// Grow the build scratch to hold `need` points.  Returns false on ENOMEM
// (the old scratch is kept).
bool ensure_build_scratch(bdl_tree* t, uint64_t need) {
  if (need <= t->sc.cap) return true;
  uint64_t cap = t->sc.cap ? t->sc.cap : 4096;
  while (cap < need) cap *= 2;
  if (cap > (1ull << 31)) cap = need;
  const int d = t->d;
  BuildScratch n;
  n.cap = cap;
  n.max_seg = cap / t->T + kMaxJobs + 8;
  n.max_tiles = cap / kTile + n.max_seg + 8;
  n.max_fin = 2 * (uint64_t)(kMaxDepth + 1) * (cap / t->T + 1) + 2 * kMaxJobs;
  n.max_emit = 2 * cap + kMaxJobs;
  n.tmp_words = radix_tmp_words(n.max_emit);
  uint64_t st = scan_tmp_words(cap) + 16;
  if (st > n.tmp_words) n.tmp_words = st;
  // the layout's sort keeps 256 digit counts for each of its 256 chunks
  if (n.tmp_words < 256 * 256 + 16) n.tmp_words = 256 * 256 + 16;
  bool ok = true;
  auto A = [&](size_t bytes) -> void* {
    void* p = ok ? dmalloc(t, bytes) : nullptr;
    if (!p) ok = false;
    return p;
  };
  for (int i = 0; i < 2; ++i) {
    n.soa[i] = (float*)A((size_t)(d + 1) * cap * 4);
    n.seg[i] = (Seg*)A(n.max_seg * sizeof(Seg));
    n.segtb[i] = (uint32_t*)A(n.max_seg * 4);
    n.keys[i] = (uint64_t*)A(n.max_emit * 8);
    n.vals[i] = (uint32_t*)A(n.max_emit * 4);
  }
  n.tile_left = (uint32_t*)A(n.max_tiles * 8);  // left counts, then quarter prefixes
  n.tile_seg[0] = (uint32_t*)A(n.max_tiles * 4);
  n.tile_seg[1] = (uint32_t*)A(n.max_tiles * 4);
  n.tile_off = (uint32_t*)A(n.max_tiles * 4);
  n.fin = (Fin*)A(n.max_fin * sizeof(Fin));
  n.emit = (uint32_t*)A(n.max_emit * (size_t)emit_stride(d) * 4);
  n.final_of = (uint32_t*)A(n.max_emit * 4);
  n.tmp = (uint32_t*)A(n.tmp_words * 4);
  n.tile_cnt = (uint32_t*)A((cap / kTile + 2) * 4 + (2ull << 20));
  if (t->rule == kSplitObject) n.sel_hist = (uint32_t*)A(n.max_seg * 256 * 4);
  if (!ok) {
    void* ps[] = {n.soa[0], n.soa[1], n.seg[0], n.seg[1], n.segtb[0], n.segtb[1], n.keys[0],
                  n.keys[1], n.vals[0], n.vals[1], n.tile_left, n.tile_seg[0], n.tile_seg[1],
                  n.tile_off, n.fin,
                  n.emit,
                  n.final_of, n.tmp, n.tile_cnt, n.sel_hist};
    for (void* p : ps) dfree(t, p);
    return false;
  }
  // the select kernels expect zero counts and clear them after each use
  if (n.sel_hist) launch_fill_u32(n.sel_hist, 0u, n.max_seg * 256, t->s);
  (void)wait_stream(t);
  free_build_scratch(t);
  n.host_ctr = t->sc.host_ctr;
  n.ctr = t->sc.ctr;
  n.jobs = t->sc.jobs;
  t->sc = n;
  return true;
}

bool ensure_query_scratch(bdl_tree* t, uint64_t need) {
  if (need <= t->qs.cap) return true;
  uint64_t cap = t->qs.cap ? t->qs.cap : 65536;
  while (cap < need) cap *= 2;
  QueryScratch n;
  n.cap = cap;
  bool ok = true;
  auto A = [&](size_t bytes) -> void* {
    void* p = ok ? dmalloc(t, bytes) : nullptr;
    if (!p) ok = false;
    return p;
  };
  for (int i = 0; i < 2; ++i) {
    n.keys[i] = (uint32_t*)A(cap * 4);
    n.vals[i] = (uint32_t*)A(cap * 4);
  }
  n.tmp = (uint32_t*)A(radix_tmp_words(cap) * 4);
  n.box = (uint32_t*)A(2 * kMaxDim * 4);
  if (!ok) {
    void* ps[] = {n.keys[0], n.keys[1], n.vals[0], n.vals[1], n.tmp, n.box};
    for (void* p : ps) dfree(t, p);
    return false;
  }
  (void)wait_stream(t);
  void* old[] = {t->qs.keys[0], t->qs.keys[1], t->qs.vals[0], t->qs.vals[1], t->qs.tmp,
                 t->qs.box};
  for (void* p : old) dfree(t, p);
  t->qs = n;
  return true;
}

// Filter size for n records: 16 bits per record, rounded up to a power of
// two of 64-bit words (a false-positive rate of a few per thousand with four
// bits per key in one word).
int bloom_log2_for(int64_t n) {
  int lg = 0;
  while ((1ll << lg) * 4 < n) ++lg;
  return lg;
}

// Grows a device array of 64-bit words to at least `need` words (contents
// not kept).
bool ensure_words(bdl_tree* t, uint64_t*& p, int64_t& have, int64_t need) {
  if (p && have >= need) return true;
  uint64_t* q = (uint64_t*)dmalloc(t, (size_t)need * 8);
  if (!q) return false;
  if (p) {
    (void)wait_stream(t);
    dfree(t, p);
  }
  p = q;
  have = need;
  return true;
}

bool ensure_level(bdl_tree* t, int j) {
  LevelState& L = t->lev[j];
  if (L.rec) return true;
  const int64_t cap = level_cap(t, j);
  float* rec = (float*)dmalloc(t, (size_t)(cap + kRecPad) * t->S * 4);
  if (!rec) return false;
  float* nodes = (float*)dmalloc(t, (size_t)(2 * cap) * t->NS * 4);
  if (!nodes) {
    dfree(t, rec);
    return false;
  }
  L.rec = rec;
  L.nodes = nodes;
  L.cap = cap;
  return true;
}

void upload_live(bdl_tree* t) {
  uint32_t v[kMaxLevels];
  for (int i = 0; i < kMaxLevels; ++i) v[i] = t->lev[i].on ? (uint32_t)t->lev[i].live : 0u;
  launch_store_u32(t->d_live, v, kMaxLevels, t->s);
}

LevelViews make_views(const bdl_tree* t);

// Refresh the device copy of the trees kNN_L visits (after every change of
// the structure; stream-ordered before any later k-NN launch or replay).
void upload_views(bdl_tree* t) {
  LevelViews v = make_views(t);
  launch_store_views(t->d_views, v, t->s);
  launch_patch_views(t->d_views, t->d_level_nodes, (uint32_t)t->cfg.leaf_size,
                     t->mode != kModeNoRebuild, t->s);
}

// Insert_L (Alg. 3) over the pool = buffer (arrival order) ++ batch.  The
// batch is either caller rows [n][d] with ids, or records (batch_ids null).
// Readings of what the paper leaves open:
//  - floor(|pool| / X) whole chunks of X points leave the pool; its last
//    |pool| mod X points form the new buffer (this reproduces Fig. 4);
//  - F_new = F + floor(|pool| / X); new trees J = F_new \ F; cleared trees
//    C = F \ F_new (all below the highest new tree j*);
//  - j* takes the live points of the cleared trees (ascending tree, then
//    slot order) followed by the leading pool slice that fills its nominal
//    capacity 2^j* X; each other new tree, highest first, takes the next
//    pool slice of 2^j X points.
// Insert_L of n points (caller rows with ids, or records when batch_ids is
// null).  Trees in pre_clear are taken out first (Erase_L's half rule: their
// live points are in the batch); they stay untouched unless the insert
// succeeds, so that BDL_ENOMEM leaves the trees as they were.
int insert_single(bdl_tree* t, const float* batch, const uint32_t* batch_ids, int64_t n,
                  uint64_t pre_clear);

int insert_impl(bdl_tree* t, const float* batch, const uint32_t* batch_ids, int64_t n,
                uint64_t pre_clear = 0) {
  resolve_nodes(t, false);  // learn from builds that have finished (no wait)
  if (t->mode != kModeBdl) return insert_single(t, batch, batch_ids, n, pre_clear);
  const int64_t X = t->cfg.buffer_size;
  const int64_t pn = t->bn + n;
  const uint64_t m = (uint64_t)(pn / X);
  const uint64_t F0 = t->F & ~pre_clear;
  const uint64_t Fn = F0 + m;
  if (Fn >> (kMaxLevels - 1)) return fail(BDL_EINVAL, "too many points for the level table");
  const uint64_t J = Fn & ~F0;
  const uint64_t C = F0 & ~Fn;
  struct Src {
    int kind;  // 0 whole level, 1 live records of a level, 2 pool range
    int level;
    uint64_t p0, cnt, dst;
  };
  std::vector<Src> srcs;
  JobTable jt;
  std::memset(&jt, 0, sizeof(jt));
  uint64_t base = 0;
  int64_t off = 0;
  std::vector<int> job_level;
  if (J) {
    const int js = 63 - __builtin_clzll(J);
    int64_t ccap = 0, clive = 0;
    for (int i = 0; i < kMaxLevels; ++i)
      if ((C >> i) & 1u) {
        ccap += level_cap(t, i);
        clive += t->lev[i].live;
      }
    const int64_t slice = level_cap(t, js) - ccap;
    if (slice < 0 || slice > pn) return fail(BDL_EINVAL, "inconsistent insert plan");
    uint64_t acc = base;
    for (int i = 0; i < kMaxLevels; ++i) {
      if (!((C >> i) & 1u)) continue;
      const LevelState& L = t->lev[i];
      srcs.push_back({L.live == L.n_slots ? 0 : 1, i, 0, (uint64_t)L.n_slots, acc});
      acc += (uint64_t)L.live;
    }
    srcs.push_back({2, -1, 0, (uint64_t)slice, acc});
    Job jb{};
    jb.base = (uint32_t)base;
    jb.count = (uint32_t)(clive + slice);
    jb.level = (uint32_t)js;
    jb.write_map = 1;
    jt.jobs[jt.n++] = jb;
    job_level.push_back(js);
    base += (uint64_t)(clive + slice);
    off = slice;
    for (int j = js - 1; j >= 0; --j) {
      if (!((J >> j) & 1u)) continue;
      const int64_t c = level_cap(t, j);
      srcs.push_back({2, -1, (uint64_t)off, (uint64_t)c, base});
      Job jj{};
      jj.base = (uint32_t)base;
      jj.count = (uint32_t)c;
      jj.level = (uint32_t)j;
      jj.write_map = 1;
      jt.jobs[jt.n++] = jj;
      job_level.push_back(j);
      base += (uint64_t)c;
      off += c;
    }
  }
  const int64_t bn_new = pn - off;
  if (bn_new < 0 || bn_new >= X) return fail(BDL_EINVAL, "inconsistent buffer plan");
  if (bn_new > 0) {
    srcs.push_back({2, -1, (uint64_t)off, (uint64_t)bn_new, base});
    Job jb{};
    jb.base = (uint32_t)base;
    jb.count = (uint32_t)bn_new;
    jb.level = kBufferLevel;
    jb.write_map = 0;
    jt.jobs[jt.n++] = jb;
    job_level.push_back(-1);
    base += (uint64_t)bn_new;
  }
  const uint64_t R = base;
  if (R >= (1ull << 31)) return fail(BDL_EINVAL, "insert rebuilds too many points at once");
  // ---- memory first: nothing has been enqueued yet ----
  for (int i = 0; i < jt.n; ++i)
    if (job_level[i] >= 0 && !ensure_level(t, job_level[i]))
      return fail(BDL_ENOMEM, "cannot allocate a static tree");
  if (!t->pool[0]) {
    t->pool[0] = (float*)dmalloc(t, (size_t)X * t->S * 4);
    t->pool[1] = (float*)dmalloc(t, (size_t)X * t->S * 4);
    t->brec = (float*)dmalloc(t, (size_t)(X + kRecPad) * t->S * 4);
    t->bnodes = (float*)dmalloc(t, (size_t)(2 * X) * t->NS * 4);
    if (!t->pool[0] || !t->pool[1] || !t->brec || !t->bnodes) {
      dfree(t, t->pool[0]);
      dfree(t, t->pool[1]);
      dfree(t, t->brec);
      dfree(t, t->bnodes);
      t->pool[0] = t->pool[1] = t->brec = t->bnodes = nullptr;
      return fail(BDL_ENOMEM, "cannot allocate the buffer");
    }
  }
  if (R && !ensure_build_scratch(t, R)) return fail(BDL_ENOMEM, "cannot allocate build scratch");
  for (int i = 0; i < jt.n; ++i) {
    if (job_level[i] >= 0) {
      jt.jobs[i].rec = t->lev[job_level[i]].rec;
      jt.jobs[i].nodes = t->lev[job_level[i]].nodes;
      jt.jobs[i].node_cap = (uint32_t)(2 * t->lev[job_level[i]].cap);
    } else {
      jt.jobs[i].rec = t->brec;
      jt.jobs[i].nodes = t->bnodes;
      jt.jobs[i].node_cap = (uint32_t)(2 * X);
    }
  }
  // ---- gather ----
  t->pt.begin(BDL_PH_GATHER);
  PoolSrc ps;
  ps.bufrec = t->pool[t->pcur];
  ps.bn = (uint64_t)t->bn;
  ps.batch = batch;
  ps.batch_ids = batch_ids;
  ps.n = (uint64_t)n;
  BuildScratch& sc = t->sc;
  for (const Src& sr : srcs) {
    if (sr.kind == 0) {
      launch_records_to_soa(t->lev[sr.level].rec, t->d, sr.cnt, sc.soa[0], sc.cap, sr.dst, t->s);
    } else if (sr.kind == 1) {
      launch_compact_live(t->lev[sr.level].rec, t->d, sr.cnt, sc.soa[0], sc.cap, sr.dst, nullptr,
                          sc.tile_cnt, sc.tmp, t->s);
    } else {
      launch_pool_to_soa(ps, t->d, sr.p0, sr.cnt, sc.soa[0], sc.cap, sr.dst, t->s);
    }
  }
  launch_pool_to_records(ps, t->d, (uint64_t)off, (uint64_t)bn_new, t->pool[t->pcur ^ 1], t->map,
                         t->cfg.id_capacity, t->s);
  t->pt.end(BDL_PH_GATHER);
  // ---- build ----
  const char* err = nullptr;
  int base_depths = 0;
  int rc = run_build(jt, sc, t->d, (uint32_t)t->cfg.leaf_size, t->T, t->rule, t->depth_ratio,
                     t->map, t->cfg.id_capacity, t->s, t->d_level_nodes, t->d_misc + 9,
                     &base_depths, &t->host_waits, &err, t->pt);
  if (rc) return fail(rc, err ? err : "build failed");
  // ---- commit ----
  for (int i = 0; i < kMaxLevels; ++i) {
    if (!(((C | pre_clear) >> i) & 1u)) continue;
    LevelState& L = t->lev[i];
    L.on = false;
    L.n_slots = L.live = L.n_nodes = 0;
    L.bloom_ok = false;
  }
  t->b_nodes = 0;
  for (int i = 0; i < jt.n; ++i) {
    if (job_level[i] >= 0) {
      LevelState& L = t->lev[job_level[i]];
      L.on = true;
      L.n_slots = L.live = jt.jobs[i].count;
      L.n_nodes = -1;  // on the device until publish_nodes' copy arrives
      L.bloom_ok = false;
      t->rebuilt += jt.jobs[i].count;
    } else {
      t->b_nodes = -1;
    }
  }
  if (jt.n) publish_nodes(t, base_depths);
  t->pcur ^= 1;
  t->bn = bn_new;
  t->F = Fn;
  upload_live(t);
  upload_views(t);
  if (hipGetLastError() != hipSuccess) return fail(BDL_EHIP, "kernel launch failed in insert");
  return 0;
}

// B2's in-place insert (Section III-B): the batch goes into the existing
// tree's leaves along its splits, and the records are laid out again into
// the spare arena, which then becomes the tree's.
int insert_b2(bdl_tree* t, const float* pts, const uint32_t* ids, int64_t n) {
  LevelState& L = t->lev[0];
  resolve_nodes(t, true);  // the kernels walk the tree's nodes
  if (L.n_nodes <= 0) return fail(BDL_EHIP, "tree without nodes");
  const int64_t total = L.n_slots + n;
  if (total >= (1ll << 31)) return fail(BDL_EINVAL, "tree too large");
  // ---- memory first ----
  if (t->b2_alt_cap < total) {
    int64_t cap = t->b2_alt_cap > L.cap ? t->b2_alt_cap : L.cap;
    while (cap < total) cap *= 2;
    float* alt = (float*)dmalloc(t, (size_t)(cap + kRecPad) * t->S * 4);
    if (!alt) return fail(BDL_ENOMEM, "cannot allocate the record arena");
    (void)wait_stream(t);
    dfree(t, t->b2_alt);
    t->b2_alt = alt;
    t->b2_alt_cap = cap;
  }
  const uint64_t nbox = (uint64_t)L.n_nodes * 2 * t->d;
  const uint64_t ntmp = radix_tmp_words((uint64_t)n);
  if ((uint64_t)n > t->b2_pts_cap || nbox > t->b2_box_words || ntmp > t->b2_tmp_words) {
    uint64_t pc = t->b2_pts_cap > (uint64_t)n ? t->b2_pts_cap : (uint64_t)n;
    uint64_t bw = t->b2_box_words > nbox ? t->b2_box_words : nbox;
    uint64_t tw = radix_tmp_words(pc);
    B2Scratch b{};
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i) {
      b.keys[i] = (uint32_t*)dmalloc(t, pc * 4);
      b.vals[i] = (uint32_t*)dmalloc(t, pc * 4);
      ok = b.keys[i] && b.vals[i];
    }
    b.obox = ok ? (uint32_t*)dmalloc(t, bw * 4) : nullptr;
    b.tmp = ok && b.obox ? (uint32_t*)dmalloc(t, tw * 4) : nullptr;
    if (!b.tmp) {
      void* ps[] = {b.keys[0], b.keys[1], b.vals[0], b.vals[1], b.obox};
      for (void* q : ps) dfree(t, q);
      return fail(BDL_ENOMEM, "cannot allocate insert scratch");
    }
    (void)wait_stream(t);
    void* old[] = {t->b2.keys[0], t->b2.keys[1], t->b2.vals[0], t->b2.vals[1], t->b2.obox,
                   t->b2.tmp};
    for (void* q : old) dfree(t, q);
    t->b2 = b;
    t->b2_pts_cap = pc;
    t->b2_box_words = bw;
    t->b2_tmp_words = tw;
  }
  t->pt.begin(BDL_PH_GATHER);
  int rc = b2_insert(pts, ids, (uint64_t)n, t->d, L.nodes, (uint32_t)L.n_nodes, L.rec,
                     (uint32_t)L.n_slots, t->b2_alt, t->map, t->cfg.id_capacity, 0u,
                     t->d_misc + 8, t->b2, t->s);
  t->pt.end(BDL_PH_GATHER);
  if (rc) return fail(rc, "in-place insert failed to launch");
  std::swap(L.rec, t->b2_alt);
  std::swap(L.cap, t->b2_alt_cap);
  L.n_slots = total;
  L.live += n;
  L.bloom_ok = false;
  upload_live(t);
  upload_views(t);
  return 0;
}

// The baselines' insert.  B1 (and B2's first batch): one build over the live
// points of tree 0, in slot order (none if pre_clear takes the tree out),
// followed by the batch (caller rows with ids, or records when batch_ids is
// null).  B2 afterwards inserts in place.  Tree 0's arenas grow as needed.
int insert_single(bdl_tree* t, const float* batch, const uint32_t* batch_ids, int64_t n,
                  uint64_t pre_clear) {
  LevelState& L = t->lev[0];
  const bool have = L.on && !(pre_clear & 1u);
  if (t->mode == kModeNoRebuild && have && L.n_slots > 0) {
    if (n == 0) return 0;
    if (!batch_ids) return fail(BDL_EINVAL, "in-place insert takes caller rows");
    return insert_b2(t, batch, batch_ids, n);
  }
  const int64_t keep = have ? L.live : 0;
  const int64_t total = keep + n;
  if (total >= (1ll << 31)) return fail(BDL_EINVAL, "tree too large");
  if (total == 0) {
    L.on = false;
    L.n_slots = L.live = L.n_nodes = 0;
    L.bloom_ok = false;
    t->F = 0;
    upload_live(t);
    upload_views(t);
    return 0;
  }
  // ---- memory first: nothing has been enqueued yet ----
  float* rec = L.rec;
  float* nodes = L.nodes;
  int64_t cap = L.cap;
  const bool grow = !L.rec || L.cap < total;
  if (grow) {
    cap = L.cap > t->cfg.buffer_size ? L.cap : t->cfg.buffer_size;
    while (cap < total) cap *= 2;
    rec = (float*)dmalloc(t, (size_t)(cap + kRecPad) * t->S * 4);
    nodes = rec ? (float*)dmalloc(t, (size_t)(2 * cap) * t->NS * 4) : nullptr;
    if (!nodes) {
      dfree(t, rec);
      return fail(BDL_ENOMEM, "cannot allocate the tree");
    }
  }
  if (!ensure_build_scratch(t, (uint64_t)total)) {
    if (grow) {
      dfree(t, rec);
      dfree(t, nodes);
    }
    return fail(BDL_ENOMEM, "cannot allocate build scratch");
  }
  BuildScratch& sc = t->sc;
  JobTable jt;
  std::memset(&jt, 0, sizeof(jt));
  jt.n = 1;
  jt.jobs[0].base = 0;
  jt.jobs[0].count = (uint32_t)total;
  jt.jobs[0].level = 0;
  jt.jobs[0].write_map = 1;
  jt.jobs[0].rec = rec;
  jt.jobs[0].nodes = nodes;
  jt.jobs[0].node_cap = (uint32_t)(2 * cap);
  // ---- gather (every source is read into the build buffers before the
  // build writes the tree, so the tree may be rebuilt in its own arena) ----
  t->pt.begin(BDL_PH_GATHER);
  if (keep) {
    if (L.live == L.n_slots)
      launch_records_to_soa(L.rec, t->d, (uint64_t)L.n_slots, sc.soa[0], sc.cap, 0, t->s);
    else
      launch_compact_live(L.rec, t->d, (uint64_t)L.n_slots, sc.soa[0], sc.cap, 0, nullptr,
                          sc.tile_cnt, sc.tmp, t->s);
  }
  if (n) {
    PoolSrc ps;
    ps.bufrec = nullptr;
    ps.bn = 0;
    ps.batch = batch;
    ps.batch_ids = batch_ids;
    ps.n = (uint64_t)n;
    launch_pool_to_soa(ps, t->d, 0, (uint64_t)n, sc.soa[0], sc.cap, (uint64_t)keep, t->s);
  }
  t->pt.end(BDL_PH_GATHER);
  const char* err = nullptr;
  int base_depths = 0;
  int rc = run_build(jt, sc, t->d, (uint32_t)t->cfg.leaf_size, t->T, t->rule, t->depth_ratio,
                     t->map, t->cfg.id_capacity, t->s, t->d_level_nodes, t->d_misc + 9,
                     &base_depths, &t->host_waits, &err, t->pt);
  if (rc) {
    if (grow) {
      (void)wait_stream(t);
      dfree(t, rec);
      dfree(t, nodes);
    }
    return fail(rc, err ? err : "build failed");
  }
  if (grow && L.rec) {
    (void)wait_stream(t);
    dfree(t, L.rec);
    dfree(t, L.nodes);
  }
  L.rec = rec;
  L.nodes = nodes;
  L.cap = cap;
  L.on = true;
  L.n_slots = L.live = total;
  L.n_nodes = -1;
  L.bloom_ok = false;
  publish_nodes(t, base_depths);
  t->F = 1;
  t->rebuilt += total;
  upload_live(t);
  upload_views(t);
  if (hipGetLastError() != hipSuccess) return fail(BDL_EHIP, "kernel launch failed in insert");
  return 0;
}

LevelViews make_views(const bdl_tree* t) {
  LevelViews v;
  std::memset(&v, 0, sizeof(v));
  for (int i = kMaxLevels - 1; i >= 0; --i) {
    const LevelState& L = t->lev[i];
    if (!L.on || L.n_slots == 0) continue;
    v.v[v.n].rec = L.rec;
    v.v[v.n].nodes = L.nodes;
    v.v[v.n].n_slots = (uint32_t)L.n_slots;
    v.v[v.n].n_nodes = 0;  // set on the device from the published counts
    v.v[v.n].level = (uint32_t)i;
    ++v.n;
  }
  if (t->bn > 0) {
    v.v[v.n].rec = t->brec;
    v.v[v.n].nodes = t->bnodes;
    v.v[v.n].n_slots = (uint32_t)t->bn;
    v.v[v.n].n_nodes = 0;
    v.v[v.n].level = (uint32_t)kMaxLevels;
    ++v.n;
  }
  return v;
}

void destroy_graphs(bdl_tree* t) {
  for (auto& kv : t->graphs) (void)hipGraphExecDestroy(kv.second);
  t->graphs.clear();
}

// Scratch of the batched path for cap queries; growing it invalidates the
// captured graphs (they hold its addresses).
bool ensure_batch_scratch(bdl_tree* t, uint64_t cap) {
  if (cap <= t->bcap) return true;
  QueryScratch n;
  n.cap = cap;
  bool ok = true;
  auto A = [&](size_t bytes) -> void* {
    void* p = ok ? dmalloc(t, bytes) : nullptr;
    if (!p) ok = false;
    return p;
  };
  float* bq = (float*)A((size_t)cap * t->d * 4);
  uint32_t* bqreq = (uint32_t*)A((size_t)cap * 4);
  for (int i = 0; i < 2; ++i) {
    n.keys[i] = (uint32_t*)A(cap * 4);
    n.vals[i] = (uint32_t*)A(cap * 4);
  }
  n.tmp = (uint32_t*)A(radix_tmp_words(cap) * 4);
  n.box = (uint32_t*)A(2 * kMaxDim * 4);
  if (!ok) {
    void* ps[] = {bq, bqreq, n.keys[0], n.keys[1], n.vals[0], n.vals[1], n.tmp, n.box};
    for (void* p : ps) dfree(t, p);
    return false;
  }
  (void)wait_stream(t);
  destroy_graphs(t);
  void* old[] = {t->bq, t->bqreq, t->bqs.keys[0], t->bqs.keys[1], t->bqs.vals[0],
                 t->bqs.vals[1], t->bqs.tmp, t->bqs.box};
  for (void* p : old) dfree(t, p);
  t->bq = bq;
  t->bqreq = bqreq;
  t->bqs = n;
  t->bcap = cap;
  return true;
}

// Kernel template bucket of the register array for the largest k.
int kmax_bucket(int mode, int kmax) {
  if (mode == kKnnQuery) return kmax;
  if (mode == kKnnWave && (kmax == 1 || kmax == 2 || kmax == 5 || kmax == 10)) return kmax;
  if (kmax <= 4) return 4;
  if (kmax <= 8) return 8;
  if (kmax <= 16) return 16;
  if (kmax <= 32) return 32;
  return 64;
}

// The batched sequence: gather the requests' queries, order them, traverse.
// Every size it uses is fixed by cap, every count is read from device
// memory, so the same sequence is valid for any batch that fits cap.
// Launch shape of a k-NN launch with largest k `kmax` over nq queries: the
// first matching row of the shape table, else the tree's parameters.  *sort
// (may be null) tells whether a bdl_knn call orders its queries.
KnnLaunch choose_launch(const bdl_tree* t, int kmax, uint64_t nq, bool* sort) {
  KnnLaunch L;
  L.mode = t->knn_mode;
  // the wavefront-per-query kernel keeps node indices in 26 bits
  bdl_tree* tw = const_cast<bdl_tree*>(t);
  resolve_nodes(tw, false);
  // a count still on the device is bounded by 2 slots - 1
  auto nodes_of = [](int64_t nn, int64_t slots) -> uint64_t {
    return nn >= 0 ? (uint64_t)nn : (uint64_t)(2 * slots);
  };
  auto max_nodes_of = [&]() -> uint64_t {
    uint64_t m = t->bn ? nodes_of(t->b_nodes, t->bn) : 0;
    for (int i = 0; i < kMaxLevels; ++i)
      if (t->lev[i].on) {
        const uint64_t x = nodes_of(t->lev[i].n_nodes, t->lev[i].n_slots);
        if (x > m) m = x;
      }
    return m;
  };
  uint64_t max_nodes = max_nodes_of();
  // a tree of 2^25 slots or more only passes with its exact count: wait for
  // the build that publishes it (the launch would wait for it on the
  // stream anyway), rather than fall back to a slower kernel
  if (max_nodes >= kKnnQueryMaxNodes && t->nodes_pending) {
    resolve_nodes(tw, true);
    max_nodes = max_nodes_of();
  }
  const bool query_ok = max_nodes < kKnnQueryMaxNodes;
  if (L.mode == kKnnAuto) {
    // a small batch leaves the device idle with one lane per query: one
    // wavefront searches each query; the wavefront-per-group kernel pays
    // off when the queries are dense among the points (queries adjacent on
    // the Hilbert curve then share most of their paths); otherwise sparse
    // queries take one lane each
    // In five or more dimensions the 64 queries of a group no longer share
    // their paths (a Hilbert cell of the group spans little of each
    // dimension), and one wavefront per query wins at every batch size
    // (7D clustered, 9M queries: 1.15 s against 2.56 s for the group kernel
    // and 1.73 s for one lane per query).
    const int64_t live = bdl_size(t);
    if ((nq <= t->query_max || t->d >= 5) && query_ok)
      L.mode = kKnnQuery;
    else
      L.mode = (nq >= 65536 && (int64_t)nq * 2 >= live) ? kKnnWave : kKnnLane;
  }
  L.block = t->knn_block;
  L.persistent = t->persistent == 2 ? (L.mode == kKnnWave ? 1 : 0) : t->persistent;
  L.queue = t->d_queue;
  L.qstack = t->query_stack;
  // the Hilbert order gives neighbouring queries to neighbouring lanes and
  // waves: the wavefront-per-group kernel needs it, the lane kernel gains
  // from it on large batches, one wavefront per query does not use it
  bool srt = L.mode == kKnnWave || (L.mode == kKnnLane && nq >= t->sort_min);
  for (const bdl_knn_shape& r : t->shapes) {
    if (kmax < r.k_lo || kmax > r.k_hi || (int64_t)nq < r.nq_lo || (int64_t)nq > r.nq_hi)
      continue;
    if (r.kernel == kKnnQuery && !query_ok) continue;
    L.mode = r.kernel;
    L.block = r.block;
    L.persistent = r.persistent;
    srt = r.sort != 0;
    break;
  }
  if (L.mode == kKnnQuery && !query_ok) L.mode = kKnnLane;
  if (sort) *sort = srt;
  return L;
}

int enqueue_batch(bdl_tree* t, hipStream_t s, uint64_t cap, int kt, const KnnLaunch& L,
                  bool sort) {
  launch_gather_queries(t->breqs, t->bcount, cap, t->d, t->bq, t->bqreq, s);
  const uint32_t* order =
      sort ? spatial_order(t->d, t->bq, t->bcount, 0, cap, t->bqs, s) : nullptr;
  KnnQueries Q;
  std::memset(&Q, 0, sizeof(Q));
  Q.q = t->bq;
  Q.nq_dev = t->bcount;
  Q.qreq = t->bqreq;
  Q.reqs = t->breqs;
  return launch_knn(L, t->d, kt, Q, cap, order, t->d_views, t->d_misc + 8,
                    t->pt.mark ? t->d_stats : nullptr, s);
}

int run_batch(bdl_tree* t, const bdl_knn_request* reqs, int nreq) {
  const int slot = t->bslot;
  // the staging slot is free once its previous copy has executed
  if (hipEventSynchronize(t->bslot_ev[slot]) != hipSuccess)
    return fail(BDL_EHIP, "staging wait failed");
  KnnReqDev* h = t->h_breqs[slot];
  uint64_t total = 0, largest = 0;
  int kmax = 0, m = 0;
  for (int i = 0; i < nreq; ++i) {
    const bdl_knn_request& r = reqs[i];
    if (r.nq == 0) continue;
    if ((uint64_t)r.nq > largest) largest = (uint64_t)r.nq;
    h[m].q = r.q;
    h[m].out_ids = r.out_ids;
    h[m].out_d2 = r.out_d2;
    h[m].qoff = total;
    h[m].nq = (uint32_t)r.nq;
    h[m].k = r.k;
    total += (uint64_t)r.nq;
    if (r.k > kmax) kmax = r.k;
    ++m;
  }
  if (m == 0) return 0;
  uint64_t cap = 4096;
  while (cap < total) cap <<= 1;
  if (!ensure_batch_scratch(t, cap)) return fail(BDL_ENOMEM, "batch scratch");
  t->h_bcount[slot][0] = total;
  t->h_bcount[slot][1] = (uint64_t)m;
  if (hipMemcpyAsync(t->breqs, h, sizeof(KnnReqDev) * m, hipMemcpyHostToDevice, t->s) !=
          hipSuccess ||
      hipMemcpyAsync(t->bcount, t->h_bcount[slot], 2 * sizeof(uint64_t), hipMemcpyHostToDevice,
                     t->s) != hipSuccess ||
      hipEventRecord(t->bslot_ev[slot], t->s) != hipSuccess)
    return fail(BDL_EHIP, "request table copy failed");
  t->bslot ^= 1;
  // the shape is the one a plain call of the largest request would get
  // (rounded up to a power of two, so that one graph serves every batch
  // whose largest request falls in the same bucket): merged requests fill
  // the device better, but their queries are no denser among the points
  bool sort = true;
  uint64_t shape_nq = 1;
  while (shape_nq < largest) shape_nq <<= 1;
  const KnnLaunch L = choose_launch(t, kmax, shape_nq, &sort);
  const int kt = kmax_bucket(L.mode, kmax);
  t->pt.begin(BDL_PH_TRAVERSE);
  if (t->use_graphs) {
    const auto key = std::make_tuple(cap, kt, L.mode, L.block, L.persistent * 2 + (sort ? 1 : 0));
    auto it = t->graphs.find(key);
    if (it == t->graphs.end()) {
      hipGraph_t g = nullptr;
      hipGraphExec_t ex = nullptr;
      KnnLaunch dry = L;
      dry.dry_run = true;
      (void)launch_knn(dry, t->d, kt, KnnQueries{}, cap, nullptr, nullptr, nullptr, nullptr,
                       t->cap_stream);
      if (hipStreamBeginCapture(t->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(BDL_EHIP, "graph capture failed to start");
      int rc = enqueue_batch(t, t->cap_stream, cap, kt, L, sort);
      hipError_t e = hipStreamEndCapture(t->cap_stream, &g);
      if (rc || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return fail(BDL_EHIP, "graph capture failed");
      }
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(BDL_EHIP, "graph instantiation failed");
      it = t->graphs.emplace(key, ex).first;
    }
    if (hipGraphLaunch(it->second, t->s) != hipSuccess)
      return fail(BDL_EHIP, "graph launch failed");
  } else {
    int rc = enqueue_batch(t, t->s, cap, kt, L, sort);
    if (rc) return fail(rc, "batched k-NN launch failed");
  }
  t->pt.end(BDL_PH_TRAVERSE);
  return 0;
}

// bdl_knn_graph by kNN_L over the live points: they are gathered as
// queries, ordered along the Hilbert curve with the other queries' machinery
// and searched from the roots, and each row is moved to the row of its id.
int knn_graph_presorted(bdl_tree* t, const LevelViews& v, int k, uint32_t* out_ids,
                        float* out_d2) {
  uint64_t cap = 0;
  for (int i = 0; i < v.n; ++i) cap += v.v[i].n_slots;
  const uint64_t rows = cap * (uint64_t)k;
  if (!ensure_query_scratch(t, cap)) return fail(BDL_ENOMEM, "query scratch");
  GraphQueries& g = t->gq;
  if (cap > g.cap || rows > g.row_cap) {
    GraphQueries n;
    n.cap = cap > g.cap ? cap : g.cap;
    n.row_cap = rows > g.row_cap ? rows : g.row_cap;
    bool ok = true;
    auto A = [&](size_t bytes) -> void* {
      void* p = ok ? dmalloc(t, bytes) : nullptr;
      if (!p) ok = false;
      return p;
    };
    n.q = (float*)A((size_t)n.cap * t->d * 4);
    n.ids = (uint32_t*)A((size_t)n.cap * 4);
    n.rid = (uint32_t*)A((size_t)n.row_cap * 4);
    n.rd2 = (float*)A((size_t)n.row_cap * 4);
    n.count = (unsigned long long*)A(8);
    void* fresh[] = {n.q, n.ids, n.rid, n.rd2, n.count};
    if (!ok) {
      for (void* p : fresh) dfree(t, p);
      return fail(BDL_ENOMEM, "cannot allocate the k-NN graph's queries");
    }
    void* old[] = {g.q, g.ids, g.rid, g.rd2, g.count};
    if (g.q) (void)wait_stream(t);
    for (void* p : old) dfree(t, p);
    g = n;
  }
  launch_fill_u32((uint32_t*)g.count, 0u, 2, t->s);
  t->pt.begin(BDL_PH_ORDER);
  for (int i = 0; i < v.n; ++i)
    launch_graph_gather(t->d_views, i, t->d, v.v[i].n_slots, g, t->d_misc + 8, t->s);
  const uint64_t* nq_dev = reinterpret_cast<const uint64_t*>(g.count);
  const uint32_t* order = spatial_order(t->d, g.q, nq_dev, 0, cap, t->qs, t->s);
  t->pt.end(BDL_PH_ORDER);
  bool sort = false;
  const KnnLaunch L = choose_launch(t, k, cap, &sort);
  KnnQueries Q;
  std::memset(&Q, 0, sizeof(Q));
  Q.q = g.q;
  Q.nq_dev = nq_dev;
  Q.nq = cap;
  Q.one.q = g.q;
  Q.one.out_ids = g.rid;
  Q.one.out_d2 = g.rd2;
  Q.one.qoff = 0;
  Q.one.nq = (uint32_t)cap;
  Q.one.k = k;
  t->pt.begin(BDL_PH_TRAVERSE);
  int rc = launch_knn(L, t->d, k, Q, cap, order, t->d_views, t->d_misc + 8,
                      t->pt.mark ? t->d_stats : nullptr, t->s);
  t->pt.end(BDL_PH_TRAVERSE);
  if (rc) return fail(rc, "k-NN graph launch failed");
  launch_graph_scatter(g, k, out_ids, out_d2, t->cfg.id_capacity, t->s);
  if (hipGetLastError() != hipSuccess) return fail(BDL_EHIP, "k-NN graph launch failed");
  return 0;
}

}  // namespace

namespace bdl {
hipStream_t tree_stream(const bdl_tree* t) { return t->s; }
int tree_dim(const bdl_tree* t) { return t->d; }
int tree_fail(int code, const char* msg) { return fail(code, msg); }
}  // namespace bdl

extern "C" {

const char* bdl_last_error(void) { return g_err.c_str(); }

int bdl_knn_batch(bdl_tree* t, const bdl_knn_request* reqs, int32_t nreq) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (nreq < 0) return fail(BDL_EINVAL, "negative request count");
  if (nreq == 0) return 0;
  if (!reqs) return fail(BDL_EINVAL, "null request array");
  for (int i = 0; i < nreq; ++i) {
    const bdl_knn_request& r = reqs[i];
    if (r.k < 1 || r.k > BDL_MAX_K) return fail(BDL_EINVAL, "k must be in 1..64");
    if (r.nq < 0 || r.nq >= (1ll << 31)) return fail(BDL_EINVAL, "bad query count");
    if (r.nq > 0 && (!r.q || !r.out_ids || !r.out_d2))
      return fail(BDL_EINVAL, "null query or output");
  }
  // launches of at most kMaxBatchReqs requests and 2^31 queries each
  int i = 0;
  while (i < nreq) {
    int j = i;
    uint64_t tot = 0;
    while (j < nreq && j - i < kMaxBatchReqs && tot + (uint64_t)reqs[j].nq < (1ull << 31)) {
      tot += (uint64_t)reqs[j].nq;
      ++j;
    }
    int rc = run_batch(t, reqs + i, j - i);
    if (rc) return rc;
    i = j;
  }
  return 0;
}

int bdl_create(const bdl_config* cfg, void* stream, bdl_tree** out) {
  if (!cfg || !out) return fail(BDL_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->dim < 1 || cfg->dim > BDL_MAX_DIM) return fail(BDL_EINVAL, "dim must be in 1..16");
  if (cfg->leaf_size < 1) return fail(BDL_EINVAL, "leaf_size must be >= 1");
  if (cfg->buffer_size < 1 || cfg->buffer_size > (1 << 24))
    return fail(BDL_EINVAL, "buffer_size must be in 1..2^24");
  if (cfg->id_capacity < 1) return fail(BDL_EINVAL, "id_capacity must be >= 1");
  if ((cfg->flags & BDL_FLAG_REBUILD_ALL) && (cfg->flags & BDL_FLAG_NO_REBUILD))
    return fail(BDL_EINVAL, "BDL_FLAG_REBUILD_ALL and BDL_FLAG_NO_REBUILD exclude each other");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BDL_EHIP, "no HIP device");
  bdl_tree* t = new bdl_tree();
  t->cfg = *cfg;
  t->s = (hipStream_t)stream;
  t->dev = dev;
  t->noalloc_scratch = scratch_on(dev);
  t->rule = (cfg->flags & BDL_FLAG_OBJECT_MEDIAN) ? kSplitObject : kSplitSpatial;
  t->mode = (cfg->flags & BDL_FLAG_REBUILD_ALL)  ? kModeRebuildAll
            : (cfg->flags & BDL_FLAG_NO_REBUILD) ? kModeNoRebuild
                                                 : kModeBdl;
  t->d = cfg->dim;
  t->S = rec_stride(cfg->dim);
  t->NS = node_stride(cfg->dim);
  t->T = finisher_threshold(cfg->dim, cfg->leaf_size);
  if (cfg->flags & BDL_FLAG_PROFILE) {
    t->pt.ctx = t;
    t->pt.mark = phase_mark;
  }
  t->map = (uint64_t*)dmalloc(t, (size_t)cfg->id_capacity * 8);
  t->d_level_nodes = (uint32_t*)dmalloc(t, kLevelPubWords * 4);
  t->d_live = (uint32_t*)dmalloc(t, kMaxLevels * 4);
  t->d_misc = (uint32_t*)dmalloc(t, 16 * 4);
  t->d_stats = (unsigned long long*)dmalloc(t, 8 * 8);
  t->d_views = (LevelViews*)dmalloc(t, sizeof(LevelViews));
  t->d_queue = (uint32_t*)dmalloc(t, kKnnQueueWords * 4);
  t->breqs = (KnnReqDev*)dmalloc(t, sizeof(KnnReqDev) * kMaxBatchReqs);
  t->bcount = (uint64_t*)dmalloc(t, 2 * sizeof(uint64_t));
  t->sc.ctr = (BuildCounters*)dmalloc(t, sizeof(BuildCounters));
  t->sc.jobs = (Job*)dmalloc(t, sizeof(Job) * kMaxJobs);
  bool ok = t->map && t->d_level_nodes && t->d_live && t->d_misc && t->d_stats && t->d_views &&
            t->d_queue && t->breqs && t->bcount && t->sc.ctr && t->sc.jobs;
  for (int i = 0; ok && i < 2; ++i) {
    if (hipHostMalloc((void**)&t->h_breqs[i], sizeof(KnnReqDev) * kMaxBatchReqs,
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&t->h_bcount[i], 2 * sizeof(uint64_t), hipHostMallocDefault) !=
            hipSuccess ||
        hipEventCreateWithFlags(&t->bslot_ev[i], hipEventDisableTiming) != hipSuccess)
      ok = false;
  }
  if (ok && hipStreamCreateWithFlags(&t->cap_stream, hipStreamNonBlocking) != hipSuccess)
    ok = false;
  if (ok && hipHostMalloc((void**)&t->h_pin, (kMaxLevels + 16) * 4, hipHostMallocDefault) !=
                hipSuccess)
    ok = false;
  if (ok && hipHostMalloc((void**)&t->sc.host_ctr, sizeof(BuildCounters), hipHostMallocDefault) !=
                hipSuccess)
    ok = false;
  if (ok && hipHostMalloc((void**)&t->h_level_nodes, (kMaxLevels + 2) * 4,
                          hipHostMallocDefault) != hipSuccess)
    ok = false;
  if (ok && hipEventCreateWithFlags(&t->ev_nodes, hipEventDisableTiming) != hipSuccess) ok = false;
  if (!ok) {
    bdl_destroy(t);
    return fail(BDL_ENOMEM, "cannot allocate the tree");
  }
  launch_fill_u32((uint32_t*)t->map, 0xFFFFFFFFu, (uint64_t)cfg->id_capacity * 2, t->s);
  launch_fill_u32(t->d_live, 0u, kMaxLevels, t->s);
  launch_fill_u32(t->d_level_nodes, 0u, kLevelPubWords, t->s);
  launch_fill_u32(t->d_misc, 0u, 16, t->s);
  launch_fill_u32((uint32_t*)t->d_stats, 0u, 16, t->s);
  if (ok) upload_views(t);
  if (wait_stream(t) != hipSuccess) {
    bdl_destroy(t);
    return fail(BDL_EHIP, "stream synchronisation failed");
  }
  *out = t;
  return 0;
}

void bdl_destroy(bdl_tree* t) {
  if (!t) return;
  (void)wait_stream(t);
  std::vector<void*> ps;
  for (auto& kv : t->sizes) ps.push_back(kv.first);
  for (void* p : ps) dfree(t, p);
  resolve_events(t);
  destroy_graphs(t);
  for (int i = 0; i < 2; ++i) {
    if (t->h_breqs[i]) (void)hipHostFree(t->h_breqs[i]);
    if (t->h_bcount[i]) (void)hipHostFree(t->h_bcount[i]);
    if (t->bslot_ev[i]) (void)hipEventDestroy(t->bslot_ev[i]);
  }
  if (t->cap_stream) (void)hipStreamDestroy(t->cap_stream);
  for (hipEvent_t e : t->ev_free) (void)hipEventDestroy(e);
  for (hipEvent_t e : t->ev_open)
    if (e) (void)hipEventDestroy(e);
  if (t->h_pin) (void)hipHostFree(t->h_pin);
  if (t->sc.host_ctr) (void)hipHostFree(t->sc.host_ctr);
  if (t->h_level_nodes) (void)hipHostFree(t->h_level_nodes);
  if (t->ev_nodes) (void)hipEventDestroy(t->ev_nodes);
  delete t;
}

int bdl_set_param(bdl_tree* t, int32_t param, int64_t value) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  switch (param) {
    case BDL_PARAM_KNN_KERNEL:
      if (value != kKnnLane && value != kKnnWave && value != kKnnAuto && value != kKnnQuery)
        return fail(BDL_EINVAL, "unknown k-NN kernel");
      t->knn_mode = (int)value;
      return 0;
    case BDL_PARAM_SORT_MIN:
      if (value < 1) return fail(BDL_EINVAL, "sort threshold must be >= 1");
      t->sort_min = (uint64_t)value;
      return 0;
    case BDL_PARAM_KNN_BLOCK:
      if (value != 64 && value != 128 && value != 256)
        return fail(BDL_EINVAL, "k-NN workgroup size must be 64, 128 or 256");
      t->knn_block = (int)value;
      return 0;
    case BDL_PARAM_USE_GRAPHS:
      if (value != 0 && value != 1) return fail(BDL_EINVAL, "use_graphs is 0 or 1");
      t->use_graphs = (int)value;
      return 0;
    case BDL_PARAM_QUERY_STACK:
      if (value < 130 || value > (1 << 30)) return fail(BDL_EINVAL, "query stack out of range");
      t->query_stack = (int)value;
      destroy_graphs(t);
      return 0;
    case BDL_PARAM_QUERY_MAX:
      if (value < 0) return fail(BDL_EINVAL, "query_max must be >= 0");
      t->query_max = (uint64_t)value;
      return 0;
    case BDL_PARAM_GRAPH_START:
      if (value != 0 && value != 1) return fail(BDL_EINVAL, "graph_start is 0 or 1");
      t->graph_start = (int)value;
      return 0;
    case BDL_PARAM_ERASE_ROUTE:
      if (value != 0 && value != 1) return fail(BDL_EINVAL, "erase_route is 0 or 1");
      t->erase_route = (int)value;
      return 0;
    case BDL_PARAM_PERSISTENT:
      if (value < 0 || value > 2) return fail(BDL_EINVAL, "persistent is 0, 1 or 2");
      t->persistent = (int)value;
      return 0;
    default:
      return fail(BDL_EINVAL, "unknown parameter");
  }
}
int bdl_set_knn_shapes(bdl_tree* t, const bdl_knn_shape* rows, int32_t n) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (n < 0 || n > BDL_MAX_SHAPES) return fail(BDL_EINVAL, "shape table size out of range");
  if (n > 0 && !rows) return fail(BDL_EINVAL, "null shape table");
  for (int32_t i = 0; i < n; ++i) {
    const bdl_knn_shape& r = rows[i];
    if (r.k_lo < 1 || r.k_hi > BDL_MAX_K || r.k_lo > r.k_hi || r.nq_lo < 0 || r.nq_lo > r.nq_hi ||
        (r.kernel != kKnnLane && r.kernel != kKnnWave && r.kernel != kKnnQuery) ||
        (r.block != 64 && r.block != 128 && r.block != 256) || (r.persistent & ~1) ||
        (r.sort & ~1))
      return fail(BDL_EINVAL, "shape row " + std::to_string(i) + " out of range");
  }
  t->shapes.assign(rows, rows + n);
  return 0;
}

int bdl_clear(bdl_tree* t) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  for (int i = 0; i < kMaxLevels; ++i) {
    LevelState& L = t->lev[i];
    L.on = false;
    L.n_slots = L.live = L.n_nodes = 0;
    L.bloom_ok = false;
  }
  t->F = 0;
  t->bn = 0;
  t->b_nodes = 0;
  t->rebuilt = t->reinserted = 0;
  launch_fill_u32((uint32_t*)t->map, 0xFFFFFFFFu, (uint64_t)t->cfg.id_capacity * 2, t->s);
  launch_fill_u32(t->d_live, 0u, kMaxLevels, t->s);
  upload_views(t);
  if (hipGetLastError() != hipSuccess) return fail(BDL_EHIP, "clear failed");
  return 0;
}

int bdl_profile(bdl_tree* t, bdl_profile_t* out, int reset) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (wait_stream(t) != hipSuccess) return fail(BDL_EHIP, "stream error");
  resolve_events(t);
  unsigned long long st[3] = {0, 0, 0};
  if (hipMemcpy(st, t->d_stats, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(BDL_EHIP, "counter readback failed");
  if (out) {
    for (int i = 0; i < BDL_NPHASES; ++i) {
      out->ms[i] = t->prof_ms[i];
      out->calls[i] = t->prof_calls[i];
    }
    out->knn_nodes = (int64_t)st[0];
    out->knn_leaves = (int64_t)st[1];
    out->knn_points = (int64_t)st[2];
  }
  if (reset) {
    for (int i = 0; i < BDL_NPHASES; ++i) {
      t->prof_ms[i] = 0.0;
      t->prof_calls[i] = 0;
    }
    launch_fill_u32((uint32_t*)t->d_stats, 0u, 16, t->s);
    (void)wait_stream(t);
  }
  return 0;
}

// Device-side error words: [8] k-NN traversal (an out-of-range tree index,
// or a route past the tree in B2's insert), [9] builds (scratch overflow, a
// build that did not end).  Read by the calls that wait anyway; a word that
// is set is cleared and reported.
int check_device_errors(bdl_tree* t) {
  const uint32_t knn = t->h_pin[kMaxLevels + 8], build = t->h_pin[kMaxLevels + 9];
  if (!knn && !build) return 0;
  launch_fill_u32(t->d_misc + 8, 0u, 2, t->s);
  (void)wait_stream(t);
  if (build)
    return fail(BDL_EHIP, (build & 1024u) ? "a build did not end (a node stayed above the LDS size)"
                                          : "build scratch overflow");
  if (knn & 64u)
    return fail(BDL_EHIP, "an in-place insert or a k-NN graph launch met an inconsistent tree");
  return fail(BDL_EHIP, "k-NN traversal met an out-of-range tree index");
}

int bdl_sync(bdl_tree* t) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (hipMemcpyAsync(t->h_pin + kMaxLevels + 8, t->d_misc + 8, 8, hipMemcpyDeviceToHost, t->s) !=
          hipSuccess ||
      wait_stream(t) != hipSuccess)
    return fail(BDL_EHIP, "stream error");
  resolve_nodes(t, false);
  return check_device_errors(t);
}

int bdl_host_waits(const bdl_tree* t, int64_t* waits) {
  if (!t || !waits) return fail(BDL_EINVAL, "null argument");
  *waits = t->host_waits;
  return 0;
}

int bdl_insert(bdl_tree* t, const float* pts, const uint32_t* ids, int64_t n) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (n < 0) return fail(BDL_EINVAL, "negative n");
  if (n == 0) return 0;
  if (!pts || !ids) return fail(BDL_EINVAL, "null points or ids");
  if (n >= (1ll << 31)) return fail(BDL_EINVAL, "batch too large");
  if (t->cfg.flags & BDL_FLAG_CHECK_INPUTS) {
    launch_fill_u32(t->d_misc + 4, 0u, 3, t->s);
    launch_validate(pts, ids, (uint64_t)n, t->d, t->map, t->cfg.id_capacity, t->d_misc + 4, t->s);
    if (hipMemcpyAsync(t->h_pin, t->d_misc + 4, 12, hipMemcpyDeviceToHost, t->s) != hipSuccess ||
        wait_stream(t) != hipSuccess)
      return fail(BDL_EHIP, "input validation failed to run");
    if (t->h_pin[0]) return fail(BDL_EINVAL, "ids must be < id_capacity");
    if (t->h_pin[1]) return fail(BDL_EINVAL, "an inserted id is already live");
    if (t->h_pin[2]) return fail(BDL_EINVAL, "coordinates must be finite");
  }
  return insert_impl(t, pts, ids, n);
}

int bdl_erase(bdl_tree* t, const float* pts, const uint32_t* ids, int64_t n, int64_t* n_erased) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (n_erased) *n_erased = 0;
  if (n < 0) return fail(BDL_EINVAL, "negative n");
  if (n == 0) return 0;
  if (!pts || !ids) return fail(BDL_EINVAL, "null points or ids");
  // Erase_L's R holds at most half of the static trees' capacity; reserve it
  // before anything changes so that ENOMEM leaves the tree unchanged.
  int64_t half = 0;
  for (int i = 0; i < kMaxLevels && t->mode == kModeBdl; ++i)
    if (t->lev[i].on) half += t->lev[i].cap / 2;
  if (half > t->rbuf_cap) {
    int64_t cap = t->rbuf_cap ? t->rbuf_cap : 4096;
    while (cap < half) cap *= 2;
    float* nb = (float*)dmalloc(t, (size_t)cap * t->S * 4);
    if (!nb) return fail(BDL_ENOMEM, "cannot allocate the rebuild buffer");
    (void)wait_stream(t);
    dfree(t, t->rbuf);
    t->rbuf = nb;
    t->rbuf_cap = cap;
  }
  if (!ensure_build_scratch(t, (uint64_t)bdl_size(t) + t->cfg.buffer_size))
    return fail(BDL_ENOMEM, "cannot allocate build scratch");
  EraseTable et;
  std::memset(&et, 0, sizeof(et));
  for (int i = 0; i < kMaxLevels; ++i)
    if (t->lev[i].on) {
      et.rec[i] = t->lev[i].rec;
      et.nslots[i] = (uint32_t)t->lev[i].n_slots;
    }
  et.pool = t->pool[t->pcur];
  et.bn = (uint32_t)t->bn;
  RouteTable rt;
  std::memset(&rt, 0, sizeof(rt));
  if (t->erase_route) {
    // filters first: ENOMEM here leaves the tree unchanged
    for (int i = 0; i < kMaxLevels; ++i) {
      LevelState& L = t->lev[i];
      if (!L.on || L.n_slots == 0 || L.bloom_ok) continue;
      const int lg = bloom_log2_for(L.n_slots);
      if (!ensure_words(t, L.bloom, L.bloom_words, 1ll << lg))
        return fail(BDL_ENOMEM, "cannot allocate a Bloom filter");
    }
    if (t->bn > 0 &&
        !ensure_words(t, t->pool_bloom, t->pool_bloom_words, 1ll << bloom_log2_for(t->bn)))
      return fail(BDL_ENOMEM, "cannot allocate a Bloom filter");
  }
  launch_fill_u32(t->d_misc, 0u, 2, t->s);
  t->pt.begin(BDL_PH_ERASE);
  if (t->erase_route) {
    for (int i = 0; i < kMaxLevels; ++i) {
      LevelState& L = t->lev[i];
      if (!L.on || L.n_slots == 0) continue;
      if (!L.bloom_ok) {
        L.bloom_log2 = bloom_log2_for(L.n_slots);
        launch_bloom_build(L.rec, (uint64_t)L.n_slots, t->d, L.bloom, L.bloom_log2, t->s);
        L.bloom_ok = true;
      }
      rt.nodes[i] = L.nodes;
      rt.bloom[i] = L.bloom;
      rt.bloom_log2[i] = (uint8_t)L.bloom_log2;
    }
    if (t->bn > 0) {
      rt.pool_bloom_log2 = (uint32_t)bloom_log2_for(t->bn);
      launch_bloom_build(et.pool, (uint64_t)t->bn, t->d, t->pool_bloom, (int)rt.pool_bloom_log2,
                         t->s);
      rt.pool_bloom = t->pool_bloom;
    }
    rt.level_nodes = t->d_level_nodes;
    launch_erase_routed(pts, ids, (uint64_t)n, t->d, t->map, t->cfg.id_capacity, et, rt,
                        t->d_live, t->d_misc, t->s);
  } else {
    launch_erase(pts, ids, (uint64_t)n, t->d, t->map, t->cfg.id_capacity, et, t->d_live,
                 t->d_misc, t->s);
  }
  t->pt.end(BDL_PH_ERASE);
  if (hipMemcpyAsync(t->h_pin, t->d_live, kMaxLevels * 4, hipMemcpyDeviceToHost, t->s) !=
          hipSuccess ||
      hipMemcpyAsync(t->h_pin + kMaxLevels, t->d_misc, 10 * 4, hipMemcpyDeviceToHost, t->s) !=
          hipSuccess ||
      wait_stream(t) != hipSuccess)
    return fail(BDL_EHIP, "erase failed");
  resolve_nodes(t, false);  // every build's copy has arrived
  if (int rc = check_device_errors(t)) return rc;
  const uint32_t erased = t->h_pin[kMaxLevels];
  const uint32_t bufhits = t->h_pin[kMaxLevels + 1];
  for (int i = 0; i < kMaxLevels; ++i)
    if (t->lev[i].on) t->lev[i].live = t->h_pin[i];
  if (n_erased) *n_erased = erased;
  if (t->mode != kModeBdl) {
    // the baselines: B1 rebuilds its tree from the survivors after every
    // erase that hit; B2 keeps the tombstones (no buffer in either)
    if (t->mode == kModeRebuildAll && erased > 0) {
      int rc = insert_single(t, nullptr, nullptr, 0, 0);
      if (rc) return rc;
    } else {
      upload_live(t);
      upload_views(t);
    }
    if (hipGetLastError() != hipSuccess) return fail(BDL_EHIP, "kernel launch failed in erase");
    return 0;
  }
  if (bufhits) {
    // the buffer keeps its arrival order and shrinks (no half rule)
    launch_compact_live(t->pool[t->pcur], t->d, (uint64_t)t->bn, nullptr, 0, 0,
                        t->pool[t->pcur ^ 1], t->sc.tile_cnt, t->sc.tmp, t->s);
    t->pcur ^= 1;
    t->bn -= bufhits;
  }
  // half-capacity rule (Alg. 4): gather trees with 2 * live < 2^i X into R;
  // the trees are taken out by the insert of R, only if it succeeds
  int64_t rn = 0;
  uint64_t below = 0;
  for (int i = 0; i < kMaxLevels; ++i) {
    LevelState& L = t->lev[i];
    if (!L.on || 2 * L.live >= L.cap) continue;
    if (L.live > 0)
      launch_compact_live(L.rec, t->d, (uint64_t)L.n_slots, nullptr, 0, 0, t->rbuf + rn * t->S,
                          t->sc.tile_cnt, t->sc.tmp, t->s);
    rn += L.live;
    below |= 1ull << i;
  }
  if (rn > 0 || below || bufhits) {
    int rc = insert_impl(t, t->rbuf, nullptr, rn, below);
    if (rc) {
      // the erase took effect; the rebuild did not (the trees below half
      // stay).  The buffer's tree still holds erased buffer points: rebuild
      // it alone, which needs no new memory.
      const std::string msg = g_err;
      if (bufhits) (void)insert_impl(t, nullptr, nullptr, 0, 0);
      upload_live(t);
      upload_views(t);
      return fail(rc, msg);
    }
    t->reinserted += rn;
  } else {
    upload_live(t);
    upload_views(t);
  }
  if (hipGetLastError() != hipSuccess) return fail(BDL_EHIP, "kernel launch failed in erase");
  return 0;
}

int bdl_knn(bdl_tree* t, const float* q, int64_t nq, int32_t k, uint32_t* out_ids, float* out_d2) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (k < 1 || k > BDL_MAX_K) return fail(BDL_EINVAL, "k must be in 1..64");
  if (nq < 0) return fail(BDL_EINVAL, "negative nq");
  if (nq == 0) return 0;
  if (!q || !out_ids || !out_d2) return fail(BDL_EINVAL, "null query or output");
  if (nq >= (1ll << 32)) return fail(BDL_EINVAL, "query batch too large");
  bool sort = false;
  const KnnLaunch L = choose_launch(t, k, (uint64_t)nq, &sort);
  const uint32_t* order = nullptr;
  if (sort) {
    if (!ensure_query_scratch(t, (uint64_t)nq)) return fail(BDL_ENOMEM, "query scratch");
    t->pt.begin(BDL_PH_ORDER);
    order = spatial_order(t->d, q, nullptr, (uint64_t)nq, (uint64_t)nq, t->qs, t->s);
    t->pt.end(BDL_PH_ORDER);
  }
  KnnQueries Q;
  std::memset(&Q, 0, sizeof(Q));
  Q.q = q;
  Q.nq = (uint64_t)nq;
  Q.one.q = q;
  Q.one.out_ids = out_ids;
  Q.one.out_d2 = out_d2;
  Q.one.qoff = 0;
  Q.one.nq = (uint32_t)nq;
  Q.one.k = k;
  t->pt.begin(BDL_PH_TRAVERSE);
  int rc = launch_knn(L, t->d, k, Q, (uint64_t)nq, order, t->d_views, t->d_misc + 8,
                      t->pt.mark ? t->d_stats : nullptr, t->s);
  t->pt.end(BDL_PH_TRAVERSE);
  if (rc) return fail(rc, "k-NN launch failed");
  return 0;
}

int bdl_knn_graph(bdl_tree* t, int32_t k, uint32_t* out_ids, float* out_d2) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (k < 1 || k > BDL_MAX_K) return fail(BDL_EINVAL, "k must be in 1..64");
  if (!out_ids || !out_d2) return fail(BDL_EINVAL, "null output");
  const LevelViews v = make_views(t);
  if (v.n == 0) return 0;
  if (t->graph_start == 0) return knn_graph_presorted(t, v, k, out_ids, out_d2);
  uint64_t cap = 0;
  for (int i = 0; i < v.n; ++i) cap += graph_group_bound(v.v[i].n_slots);
  if (cap > t->graph.cap) {
    GraphScratch g;
    g.cap = cap;
    bool ok = true;
    auto A = [&](size_t bytes) -> void* {
      void* p = ok ? dmalloc(t, bytes) : nullptr;
      if (!p) ok = false;
      return p;
    };
    g.groups = (GraphGroup*)A((size_t)cap * sizeof(GraphGroup));
    for (int i = 0; i < 2; ++i) {
      g.keys[i] = (uint64_t*)A((size_t)cap * 8);
      g.vals[i] = (uint32_t*)A((size_t)cap * 4);
    }
    g.tmp = (uint32_t*)A(65536 * 4);
    void* fresh[] = {g.groups, g.keys[0], g.keys[1], g.vals[0], g.vals[1], g.tmp};
    if (!ok) {
      for (void* p : fresh) dfree(t, p);
      return fail(BDL_ENOMEM, "cannot allocate the k-NN graph's group list");
    }
    void* old[] = {t->graph.groups, t->graph.keys[0], t->graph.keys[1], t->graph.vals[0],
                   t->graph.vals[1], t->graph.tmp};
    if (t->graph.groups) (void)wait_stream(t);
    for (void* p : old) dfree(t, p);
    t->graph = g;
  }
  uint32_t* ngroups = t->d_misc + 10;
  launch_fill_u32(ngroups, 0u, 1, t->s);
  t->pt.begin(BDL_PH_ORDER);
  for (int i = 0; i < v.n; ++i)
    launch_graph_groups(t->d_views, i, t->d, v.v[i].n_slots, t->graph.groups, t->graph.cap,
                        ngroups, t->d_misc + 8, t->s);
  launch_graph_order(t->d, t->d_views, t->graph, ngroups, t->d_misc + 11, t->d_misc + 12, t->s);
  t->pt.end(BDL_PH_ORDER);
  t->pt.begin(BDL_PH_TRAVERSE);
  const int rc = launch_knn_graph(t->d, k, t->d_views, t->graph, ngroups, t->d_misc + 12,
                                  out_ids, out_d2, t->cfg.id_capacity, t->d_misc + 8,
                                  t->pt.mark ? t->d_stats : nullptr, t->d_queue, t->s);
  t->pt.end(BDL_PH_TRAVERSE);
  if (rc) return fail(rc, "k-NN graph launch failed");
  return 0;
}

int bdl_knn_noalloc(bdl_tree* t, const float* q, int64_t nq, int32_t k, uint32_t* out_ids,
                    float* out_d2) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (k < 1 || k > BDL_MAX_K) return fail(BDL_EINVAL, "k must be in 1..64");
  if (nq < 0) return fail(BDL_EINVAL, "negative nq");
  if (nq == 0) return 0;
  if (!q || !out_ids || !out_d2) return fail(BDL_EINVAL, "null query or output");
  if ((uint64_t)nq > kNoAllocMaxQueries)
    return fail(BDL_EINVAL, "bdl_knn_noalloc takes at most 1048576 queries per call");
  if (!t->noalloc_scratch)
    return fail(BDL_EHIP, "the device scratch of bdl_knn_noalloc has no address on this GPU");
  if (radix_tmp_words((uint64_t)nq) > kNoAllocTmpWords)
    return fail(BDL_EINVAL, "query batch exceeds the no-allocation scratch");
  bool sort = false;
  const KnnLaunch L = choose_launch(t, k, (uint64_t)nq, &sort);
  const uint32_t* order = nullptr;
  if (sort) {
    // the same ordering as bdl_knn, in the device's static scratch instead of
    // the tree's growable scratch; every word it reads is written first
    uint32_t* base = t->noalloc_scratch;
    QueryScratch qs;
    qs.cap = (uint64_t)nq;
    qs.keys[0] = base;
    qs.keys[1] = base + kNoAllocMaxQueries;
    qs.vals[0] = base + 2 * kNoAllocMaxQueries;
    qs.vals[1] = base + 3 * kNoAllocMaxQueries;
    qs.tmp = base + 4 * kNoAllocMaxQueries;
    qs.box = base + 4 * kNoAllocMaxQueries + kNoAllocTmpWords;
    order = spatial_order(t->d, q, nullptr, (uint64_t)nq, (uint64_t)nq, qs, t->s);
  }
  KnnQueries Q;
  std::memset(&Q, 0, sizeof(Q));
  Q.q = q;
  Q.nq = (uint64_t)nq;
  Q.one.q = q;
  Q.one.out_ids = out_ids;
  Q.one.out_d2 = out_d2;
  Q.one.qoff = 0;
  Q.one.nq = (uint32_t)nq;
  Q.one.k = k;
  int rc = launch_knn(L, t->d, k, Q, (uint64_t)nq, order, t->d_views, t->d_misc + 8, nullptr,
                      t->s);
  if (rc) return fail(rc, "k-NN launch failed");
  return 0;
}

int64_t bdl_size(const bdl_tree* t) {
  if (!t) return 0;
  int64_t s = t->bn;
  for (int i = 0; i < kMaxLevels; ++i)
    if (t->lev[i].on) s += t->lev[i].live;
  return s;
}

int bdl_level_info(const bdl_tree* t, int32_t* nlev, int64_t* live, int64_t* cap,
                   int64_t* buf_live, uint64_t* F) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  int top = 0;
  for (int i = 0; i < kMaxLevels; ++i)
    if (t->lev[i].on) top = i + 1;
  if (nlev) *nlev = top;
  for (int i = 0; i < top; ++i) {
    if (live) live[i] = t->lev[i].on ? t->lev[i].live : 0;
    if (cap) cap[i] = t->mode == kModeBdl ? level_cap(t, i) : t->lev[i].cap;
  }
  if (buf_live) *buf_live = t->bn;
  if (F) *F = t->F;
  return 0;
}

int bdl_level_sizes(const bdl_tree* t, int32_t* nlev, int64_t* n_slots, int64_t* n_nodes,
                    int64_t* buf_nodes) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  resolve_nodes(const_cast<bdl_tree*>(t), true);
  int top = 0;
  for (int i = 0; i < kMaxLevels; ++i)
    if (t->lev[i].on) top = i + 1;
  if (nlev) *nlev = top;
  for (int i = 0; i < top; ++i) {
    if (n_slots) n_slots[i] = t->lev[i].on ? t->lev[i].n_slots : 0;
    if (n_nodes) n_nodes[i] = t->lev[i].on ? t->lev[i].n_nodes : 0;
  }
  if (buf_nodes) *buf_nodes = t->bn ? t->b_nodes : 0;
  return 0;
}

int bdl_counters(const bdl_tree* t, int64_t* rebuilt_points, int64_t* reinserted_points) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (rebuilt_points) *rebuilt_points = t->rebuilt;
  if (reinserted_points) *reinserted_points = t->reinserted;
  return 0;
}

int bdl_debug_export_level(bdl_tree* t, int32_t level, uint32_t* ids, float* pts,
                           bdl_node* nodes, int64_t* n_slots, int64_t* n_nodes) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  resolve_nodes(t, true);
  const float* rec;
  const float* nd;
  int64_t ns, nn;
  if (level == -1) {
    rec = t->brec;
    nd = t->bnodes;
    ns = t->bn;
    nn = t->b_nodes;
  } else {
    if (level < 0 || level >= kMaxLevels || !t->lev[level].on)
      return fail(BDL_EINVAL, "empty tree");
    rec = t->lev[level].rec;
    nd = t->lev[level].nodes;
    ns = t->lev[level].n_slots;
    nn = t->lev[level].n_nodes;
  }
  if (n_slots) *n_slots = ns;
  if (n_nodes) *n_nodes = nn;
  if (ns == 0) return level == -1 ? 0 : fail(BDL_EINVAL, "empty tree");
  const int d = t->d, S = t->S, NS = t->NS;
  std::vector<float> hr((size_t)ns * S), hn((size_t)nn * NS);
  if (wait_stream(t) != hipSuccess ||
      hipMemcpy(hr.data(), rec, hr.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      (nn && hipMemcpy(hn.data(), nd, hn.size() * 4, hipMemcpyDeviceToHost) != hipSuccess))
    return fail(BDL_EHIP, "export copy failed");
  for (int64_t i = 0; i < ns; ++i) {
    if (ids) std::memcpy(&ids[i], &hr[(size_t)i * S + d], 4);
    if (pts)
      for (int j = 0; j < d; ++j) pts[(size_t)i * d + j] = hr[(size_t)i * S + j];
  }
  if (nodes && nn) {
    auto I = [&](int64_t i, int f) {
      int32_t v;
      std::memcpy(&v, &hn[(size_t)i * NS + f], 4);
      return v;
    };
    for (int64_t i = 0; i < nn; ++i) {
      bdl_node& o = nodes[i];
      std::memset(&o, 0, sizeof(o));
      o.split = hn[(size_t)i * NS + NF_SPLIT];
      o.dim = I(i, NF_DIM);
      o.parent = I(i, NF_PARENT);
      for (int j = 0; j < d; ++j) {
        o.lo[j] = hn[(size_t)i * NS + NF_BOX + j];
        o.hi[j] = hn[(size_t)i * NS + NF_BOX + d + j];
      }
      if (o.dim < 0) {
        o.split = 0.0f;
        o.left = o.right = -1;
        o.begin = I(i, NF_A);
        o.count = I(i, NF_B);
      } else {
        o.left = I(i, NF_A);
        o.right = I(i, NF_B);
      }
    }
    // depth, path and subtree slot ranges from the root down / leaves up
    std::vector<int64_t> order;
    order.reserve(nn);
    order.push_back(0);
    nodes[0].depth = 0;
    nodes[0].path = 0;
    for (size_t h = 0; h < order.size(); ++h) {
      bdl_node& p = nodes[order[h]];
      if (p.dim < 0) continue;
      for (int side = 0; side < 2; ++side) {
        int32_t c = side ? p.right : p.left;
        if (c < 0 || c >= nn) return fail(BDL_EHIP, "corrupt node array");
        nodes[c].depth = p.depth + 1;
        nodes[c].path = (p.path << 1) | (uint64_t)side;
        order.push_back(c);
      }
    }
    for (size_t h = order.size(); h-- > 0;) {
      bdl_node& p = nodes[order[h]];
      if (p.dim < 0) continue;
      p.begin = nodes[p.left].begin;
      p.count = nodes[p.left].count + nodes[p.right].count;
    }
  }
  return 0;
}

int bdl_debug_export_buffer(bdl_tree* t, uint32_t* ids, float* pts, int64_t* n) {
  if (!t) return fail(BDL_EINVAL, "null tree");
  if (n) *n = t->bn;
  if (t->bn == 0) return 0;
  const int d = t->d, S = t->S;
  std::vector<float> hr((size_t)t->bn * S);
  if (wait_stream(t) != hipSuccess ||
      hipMemcpy(hr.data(), t->pool[t->pcur], hr.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(BDL_EHIP, "export copy failed");
  for (int64_t i = 0; i < t->bn; ++i) {
    if (ids) std::memcpy(&ids[i], &hr[(size_t)i * S + d], 4);
    if (pts)
      for (int j = 0; j < d; ++j) pts[(size_t)i * d + j] = hr[(size_t)i * S + j];
  }
  return 0;
}

}  // extern "C"
