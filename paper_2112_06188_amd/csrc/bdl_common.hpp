// Shared definitions of the BDL-tree HIP library (device and host).
//
// Storage formats
//  * record: one point as `rec_stride(d)` floats: coordinates 0..d-1, the
//    uint32 id (bit pattern) at index d, zero padding up to a multiple of 4
//    floats so that a record is a whole number of 16-byte vectors.  Static
//    trees store their points as records in slot order (leaves contiguous).
//  * node: `node_stride(d)` floats: [split, dim, a, b, parent, lo[d], hi[d]]
//    padded to a multiple of 4; the last word (always padding, since 5 + 2d
//    is odd) holds the number of points under the node when it was built,
//    as uint32 bits.  dim < 0 marks a leaf, whose a/b are the slot range
//    begin/count; an internal node's a/b are its children.  Nodes of one
//    tree are stored in van Emde Boas order (Alg. 1).
//  * build buffers: structure of arrays, coordinate j of position i at
//    soa[j * cap + i], id at soa[d * cap + i].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdl {

constexpr int kMaxDim = 16;
constexpr int kMaxDepth = 63;     // a node at this depth is a leaf
constexpr int kMaxLevels = 48;
constexpr int kMaxJobs = 64;
constexpr uint32_t kTomb = 0xFFFFFFFFu;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kMapInvalid = ~0ull;
constexpr uint32_t kBufferLevel = 63;  // map entries of buffered points
constexpr int kTile = 2048;            // points per tile of a global pass
constexpr int kPassThreads = 256;
constexpr int kItems = kTile / kPassThreads;
// spare records after every record array: the k-NN kernel reads leaves in
// groups of four records and may read up to three past a leaf's end
constexpr int kRecPad = 4;

__host__ __device__ inline int rec_stride(int d) { return (d + 1 + 3) & ~3; }
__host__ __device__ inline int node_stride(int d) { return (5 + 2 * d + 3) & ~3; }
__host__ __device__ inline int emit_stride(int d) { return (10 + 2 * d + 1) & ~1; }

enum NodeField { NF_SPLIT = 0, NF_DIM = 1, NF_A = 2, NF_B = 3, NF_PARENT = 4, NF_BOX = 5 };
// index of a node's point count (build time; B2 inserts leave it unchanged)
__host__ __device__ inline int node_count_field(int d) { return node_stride(d) - 1; }
// emitted (unordered) node: u32 words
enum EmitField {
  EF_PATH_LO = 0, EF_PATH_HI = 1, EF_DEPTH = 2, EF_JOB = 3, EF_PARENT = 4, EF_SIDE = 5,
  EF_BEGIN = 6, EF_COUNT = 7, EF_SPLIT = 8, EF_DIM = 9, EF_BOX = 10
};

// Order-preserving map float -> uint32 for atomic min/max.  -0.0 maps like
// +0.0, so boxes hold +0.0 for a zero coordinate of either sign.
__host__ __device__ inline uint32_t f2o_bits(uint32_t u) {
  if (u == 0x80000000u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline uint32_t o2f_bits(uint32_t o) {
  return (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
}
__device__ inline uint32_t f2o(float f) { return f2o_bits(__float_as_uint(f)); }
__device__ inline float o2f(uint32_t o) { return __uint_as_float(o2f_bits(o)); }

__host__ __device__ inline int hyperceil_i(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Position of the node at (depth, path) in the van Emde Boas order of a
// complete binary tree with H levels: the top l_t levels come first, then
// the 2^l_t bottom subtrees of l_b levels, left to right, each recursively,
// with l_b = hyperceil(floor((H+1)/2)) and l_t = H - l_b (Alg. 1 and its
// worked example under Fig. 3).  A spatial-median tree is not complete; its
// nodes are stored in the order of this index, which is the recursive layout
// with absent nodes skipped.
__host__ __device__ inline uint64_t veb_key(int H, int depth, uint64_t path) {
  uint64_t base = 0;
  while (H > 1) {
    int lb = hyperceil_i((H + 1) / 2);
    int lt = H - lb;
    if (depth < lt) {
      H = lt;
    } else {
      int rel = depth - lt;
      uint64_t j = rel >= 64 ? 0 : (path >> rel);
      base += ((1ull << lt) - 1ull) + j * ((1ull << lb) - 1ull);
      path = rel == 0 ? 0ull : (path & ((rel >= 64) ? ~0ull : ((1ull << rel) - 1ull)));
      depth = rel;
      H = lb;
    }
  }
  return base;
}

// Optional phase timing: mark(ctx, phase, 0) before and mark(ctx, phase, 1)
// after the phase's kernels are enqueued.
struct PhaseTimer {
  void* ctx = nullptr;
  void (*mark)(void* ctx, int phase, int is_end) = nullptr;
  void begin(int ph) const {
    if (mark) mark(ctx, ph, 0);
  }
  void end(int ph) const {
    if (mark) mark(ctx, ph, 1);
  }
};

// One tree being built by an Insert_L call.
struct Job {
  uint32_t base;    // first position of the job's points in the build buffers
  uint32_t count;
  uint32_t level;   // static tree index, or kBufferLevel for the buffer's tree
  uint32_t write_map;
  float* rec;       // output records, slot = position - base
  float* nodes;     // output nodes
  uint32_t node_cap;  // nodes the output array holds
  uint32_t pad_;
};

struct JobTable {
  int32_t n;
  int32_t pad_;
  Job jobs[kMaxJobs];
};

// A segment (node with more points than fit the LDS finisher) at one depth of
// the global passes.
struct Seg {
  uint32_t begin, count, job, depth;
  uint64_t path;
  uint32_t parent_emit, side;
  uint32_t emit;
  int32_t dim;         // split dimension; -1 = leaf that is copied out whole
  float split;
  uint32_t tile_begin, ntiles, nleft;
  uint32_t child[2];   // index in the next depth's list, or kNone
  uint32_t sel_key;    // object median: ordered-u32 digits selected so far
  uint32_t sel_rank;   // object median: rank still sought among matching keys
  uint32_t box[2 * kMaxDim];  // ordered-u32 lo[j] at j, hi[j] at kMaxDim + j
};

// Split heuristics of Section V-C.
constexpr int kSplitSpatial = 0;  // midpoint of the node's tight extent
constexpr int kSplitObject = 1;   // median of the node's coordinates

// A subtree small enough to be finished in LDS by one workgroup.
struct Fin {
  uint32_t begin, count, job, depth;
  uint64_t path;
  uint32_t parent_emit, side, bufsel, pad_;
};

struct BuildCounters {
  uint32_t nseg[2];    // segment list sizes by depth parity
  uint32_t ntiles[2];  // tiles of the segment lists, by depth parity
  uint32_t ebase[2];   // emit index of each list's first segment, by depth parity
  uint32_t nfin;
  uint32_t nemit;
  uint32_t err;
  uint32_t fin_next;   // next finisher entry to take
  uint32_t retry;      // the finisher found segments left above the threshold
  uint32_t par_final;  // parity of the depth list the finisher starts from
  uint32_t max_height;  // layout: the tallest job's height (vEB key bits)
  uint32_t job_bits;    // layout: bits of a job index
  uint32_t sort_sel;    // layout: buffer pair holding the sorted nodes
  uint32_t deepest;     // global-pass depths this build needed
  uint32_t job_nodes[kMaxJobs];
  uint32_t job_height[kMaxJobs];
  uint32_t job_node_off[kMaxJobs];
  uint32_t job_box[kMaxJobs][2 * kMaxDim];
};

// Sources of the pool of Insert_L: the buffer's records in arrival order
// followed by the batch (caller rows [n][d] + ids, or records).
struct PoolSrc {
  const float* bufrec;
  uint64_t bn;
  const float* batch;
  const uint32_t* batch_ids;  // null when the batch is records
  uint64_t n;
};

// One static tree (or the buffer's tree) as seen by the k-NN kernel.  Its
// node count is filled in on the device from the builds' counts (slot
// kMaxLevels of that array is the buffer's tree).
// flags of a LevelView
constexpr uint32_t kViewBalanced = 1u;  // height within log2(slots / leaf) + kBalancedMargin
constexpr int kBalancedMargin = 6;

struct LevelView {
  const float* rec;
  const float* nodes;
  uint32_t n_slots;
  uint32_t n_nodes;
  uint32_t level;  // static tree index, or kMaxLevels for the buffer's tree
  uint32_t flags;  // kViewBalanced, set on the device with the node count
};

constexpr int kMaxViews = kMaxLevels + 1;
constexpr int kMaxBatchReqs = 65536;  // requests per batched k-NN launch
struct LevelViews {
  int32_t n;
  uint32_t flags;  // kViewBalanced when every view has it
  LevelView v[kMaxViews];
};

}  // namespace bdl
