// Host side of the batched k-NN query (kNN_L, Alg. 5): Hilbert-curve ordering of
// query batches, concatenation of request tables, and the dispatch of
// traversal launches to the kernel instantiations (knn_traverse.hpp).
#include <map>
#include <mutex>
#include <tuple>

#include "bdl.h"
#include "hilbert.hpp"
#include "knn.hpp"
#include "primitives.hpp"

namespace bdl {
namespace knn_detail {

// Defined, per dimension, in knn_dN_M.hip.
template <int D>
void launch_d(const KnnLaunch& L, int kmax, const KnnQueries& Q, uint64_t grid_q,
              const uint32_t* order, const LevelViews* views, uint32_t* err,
              unsigned long long* st, hipStream_t s);

// Workgroups of `bs` threads of kernel `kern` that fit on the device at once
// (a multiple of 8, so that every XCD gets as many), cached per device.
uint64_t resident_blocks(const void* kern, int bs) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int>, uint64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, kern, bs);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, bs, 0) != hipSuccess)
    return 0;
  const uint64_t v = ((uint64_t)cus * (uint64_t)per) & ~7ull;
  cache.emplace(key, v);
  return v;
}

__global__ void k_zero_queue(uint32_t* queue) {
  if (threadIdx.x < 8) queue[threadIdx.x * kKnnQueueStride] = 0u;
}

void zero_queue(uint32_t* queue, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, s, queue);
}

__global__ void k_query_box_init(uint32_t* box) {
  const int t = threadIdx.x;
  if (t < kMaxDim) {
    box[t] = 0xFFFFFFFFu;
    box[kMaxDim + t] = 0u;
  }
}

// Tight box of a query batch.  The queries are read as one flat array of
// nq * d floats; every thread strides over it by a multiple of d, so it only
// ever sees one coordinate and keeps one pair of bounds.  Bounds are merged
// per coordinate in LDS, then with one pair of device atomics per workgroup.
__global__ void __launch_bounds__(256)
k_query_box(const float* q, const uint64_t* nq_dev, uint64_t nq_host, int d, uint32_t* box) {
  __shared__ uint32_t smn[kMaxDim], smx[kMaxDim];
  const uint64_t nq = nq_dev ? *nq_dev : nq_host;
  const uint64_t total = nq * (uint64_t)d;
  const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t stride = nthreads - nthreads % (uint64_t)d;
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.x < kMaxDim) {
    smn[threadIdx.x] = 0xFFFFFFFFu;
    smx[threadIdx.x] = 0u;
  }
  __syncthreads();
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
  if (t < stride) {
    // eight independent loads per step; an index past the end repeats this
    // thread's first element, which does not change a bound
    for (uint64_t i0 = t; i0 < total; i0 += 8 * stride) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint64_t i = i0 + (uint64_t)u * stride;
        v[u] = q[i < total ? i : i0];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t o = f2o(v[u]);
        mn = o < mn ? o : mn;
        mx = o > mx ? o : mx;
      }
    }
  }
  const int j = (int)(t % (uint64_t)d);
  atomicMin(&smn[j], mn);
  atomicMax(&smx[j], mx);
  __syncthreads();
  if ((int)threadIdx.x < d) {
    atomicMin(&box[threadIdx.x], smn[threadIdx.x]);
    atomicMax(&box[kMaxDim + threadIdx.x], smx[threadIdx.x]);
  }
}

// Hilbert key with floor(30 / D) bits per dimension; positions from nq up
// to cap get the key 0xFFFFFFFF, which sorts after every real key.
template <int D>
__global__ void k_hilbert(const float* q, const uint64_t* nq_dev, uint64_t nq_host, uint64_t cap,
                          const uint32_t* box, uint32_t* keys, uint32_t* vals) {
  constexpr int kBits = 30 / D > 0 ? 30 / D : 1;
  const uint64_t nq = nq_dev ? *nq_dev : nq_host;
  const float cells = (float)(1u << kBits);
  float lo[D], ext[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    lo[j] = o2f(box[j]);
    ext[j] = o2f(box[kMaxDim + j]) - lo[j];
  }
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
       i += (uint64_t)gridDim.x * blockDim.x) {
    vals[i] = (uint32_t)i;
    if (i >= nq) {
      keys[i] = 0xFFFFFFFFu;
      continue;
    }
    uint32_t cell[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const float u = ext[j] > 0.0f ? (q[i * D + j] - lo[j]) / ext[j] : 0.0f;
      int c = (int)(u * cells);
      c = c < 0 ? 0 : (c >= (1 << kBits) ? (1 << kBits) - 1 : c);
      cell[j] = (uint32_t)c;
    }
    keys[i] = hilbert_key<D, kBits>(cell);
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

}  // namespace knn_detail

using namespace knn_detail;


size_t query_scratch_bytes(uint64_t cap) {
  return 4 * (size_t)cap * 4 + radix_tmp_words(cap) * 4 + 2 * kMaxDim * 4;
}

const uint32_t* spatial_order(int d, const float* q, const uint64_t* nq_dev, uint64_t nq_host,
                             uint64_t cap, QueryScratch& qs, hipStream_t s) {
  hipLaunchKernelGGL(k_query_box_init, dim3(1), dim3(64), 0, s, qs.box);
  unsigned g = (unsigned)((cap * (uint64_t)d + 4095) / 4096);
  if (g > 512) g = 512;
  hipLaunchKernelGGL(k_query_box, dim3(g), dim3(256), 0, s, q, nq_dev, nq_host, d, qs.box);
  unsigned g2 = (unsigned)((cap + 255) / 256);
  if (g2 > 4096) g2 = 4096;
  switch (d) {
#define BDL_HILBERT_CASE(DD)                                                                    \
  case DD:                                                                                      \
    hipLaunchKernelGGL(k_hilbert<DD>, dim3(g2), dim3(256), 0, s, q, nq_dev, nq_host, cap, qs.box, \
                       qs.keys[0], qs.vals[0]);                                                 \
    break;
    BDL_HILBERT_CASE(1) BDL_HILBERT_CASE(2) BDL_HILBERT_CASE(3) BDL_HILBERT_CASE(4)
    BDL_HILBERT_CASE(5) BDL_HILBERT_CASE(6) BDL_HILBERT_CASE(7) BDL_HILBERT_CASE(8)
    BDL_HILBERT_CASE(9) BDL_HILBERT_CASE(10) BDL_HILBERT_CASE(11) BDL_HILBERT_CASE(12)
    BDL_HILBERT_CASE(13) BDL_HILBERT_CASE(14) BDL_HILBERT_CASE(15) BDL_HILBERT_CASE(16)
#undef BDL_HILBERT_CASE
    default:
      break;
  }
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
