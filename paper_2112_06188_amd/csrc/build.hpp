// Host launchers of the static-tree build (BuildvEB with the spatial median)
// and of the gather steps of Insert_L.
#pragma once

#include "bdl_common.hpp"

namespace bdl {

// Device scratch of one Insert_L build, sized for up to `cap` points.
struct BuildScratch {
  uint64_t cap = 0;        // points
  uint64_t max_seg = 0;    // per depth list capacity
  uint64_t max_fin = 0;
  uint64_t max_emit = 0;
  float* soa[2] = {nullptr, nullptr};  // ping-pong build buffers, (d+1) * cap
  Seg* seg[2] = {nullptr, nullptr};
  uint32_t* segtb[2] = {nullptr, nullptr};
  uint32_t* tile_left = nullptr;  // 2 * max_tiles: left count per tile, then its quarter prefixes
  uint32_t* tile_seg[2] = {nullptr, nullptr};  // segment of each tile, by depth parity
  uint32_t* tile_off = nullptr;
  uint64_t max_tiles = 0;
  Fin* fin = nullptr;
  uint32_t* emit = nullptr;      // max_emit * emit_stride(d) words
  uint64_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint32_t* final_of = nullptr;
  uint32_t* tmp = nullptr;       // scan / sort scratch
  uint64_t tmp_words = 0;
  uint32_t* tile_cnt = nullptr;  // compaction per-tile counts (tiles of kTile)
  uint32_t* sel_hist = nullptr;  // object median: 256 digit counts per segment (max_seg rows)
  BuildCounters* ctr = nullptr;
  BuildCounters* host_ctr = nullptr;  // pinned mirror
  Job* jobs = nullptr;           // device copy of the job table
};

// Sizes (bytes) of the scratch needed for `cap` points of dimension d.
size_t build_scratch_bytes(uint64_t cap, int d, uint32_t T);

// Finisher threshold: subtrees of at most this many points are built in LDS.
uint32_t finisher_threshold(int d, int leaf_size);

// --- gather kernels ---
// pool elements [p0, p0 + cnt) -> build buffer positions [dst, dst + cnt)
void launch_pool_to_soa(const PoolSrc& src, int d, uint64_t p0, uint64_t cnt, float* soa,
                        uint64_t cap, uint64_t dst, hipStream_t s);
// pool elements [p0, p0 + cnt) -> records (the new buffer pool), map entries
void launch_pool_to_records(const PoolSrc& src, int d, uint64_t p0, uint64_t cnt, float* rec,
                            uint64_t* map, uint32_t idcap, hipStream_t s);
// records [0, n) all live -> build buffer positions [dst, dst + n)
void launch_records_to_soa(const float* rec, int d, uint64_t n, float* soa, uint64_t cap,
                           uint64_t dst, hipStream_t s);
// stable compaction of live records [0, n) (id != tomb) into build buffer
// positions starting at dst (to_soa) or into records out (!to_soa).
void launch_compact_live(const float* rec, int d, uint64_t n, float* soa, uint64_t cap,
                         uint64_t dst, float* out_rec, uint32_t* tile_cnt, uint32_t* tmp,
                         hipStream_t s);

// Build every job of the table from build buffer 0 with split heuristic
// `rule` (kSplitSpatial or kSplitObject).  Writes records (slot order),
// nodes (vEB order) and, where requested, the id map, all on stream s with
// no host wait: each job's node count is stored on the device in
// level_nodes[level] (level_nodes[kMaxLevels] for the buffer's tree), its
// height in level_nodes[kLevelHeightBase + the same index],
// level_nodes[kMaxLevels + 1] receives the number of global-pass depths the
// build needed, and the device-side checks (scratch overflow, a build that
// does not end) leave their bits in *sticky_err (device) for the host's next
// check.  The host launches depth_ratio x the base budget log2(n / T) + 1
// of depths (*base_depths receives the base, 0 if the build needs no global
// pass); a cooperative kernel runs any left.  Without cooperative launch the
// host drives the rest and waits once per budget of depths (*host_waits
// counts those waits).  Returns 0 or a BDL_E* code for a launch failure.
int run_build(const JobTable& jt, BuildScratch& sc, int d, uint32_t leaf, uint32_t T,
              int rule, float depth_ratio, uint64_t* map, uint32_t idcap, hipStream_t s,
              uint32_t* level_nodes, uint32_t* sticky_err, int* base_depths,
              int64_t* host_waits, const char** err, const PhaseTimer& pt);

// Words of the device array level_nodes: node counts (kMaxLevels + 1), the
// depth count of the last build, then the trees' heights.
constexpr int kLevelHeightBase = kMaxLevels + 2;
constexpr int kLevelPubWords = kLevelHeightBase + kMaxLevels + 1;

// Node counts of the trees k-NN visits, from level_nodes (after every
// upload of the views), and each tree's kViewBalanced flag: set when its
// height is at most ceil(log2(slots / leaf)) + kBalancedMargin and
// `balanced_ok` (trees whose leaves grow past the leaf size get none).
void launch_patch_views(LevelViews* views, const uint32_t* level_nodes, uint32_t leaf,
                        bool balanced_ok, hipStream_t s);

// small utilities
void launch_store_u32(uint32_t* dst, const uint32_t* vals, int n, hipStream_t s);
void launch_fill_u32(uint32_t* dst, uint32_t v, uint64_t n, hipStream_t s);
void launch_store_views(LevelViews* dst, const LevelViews& v, hipStream_t s);

}  // namespace bdl
