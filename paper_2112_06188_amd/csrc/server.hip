// Request loop of the served form (bdl_server.h): admission by slots and a
// device-memory budget, snapshot epochs in admission order, continuous
// batching of k-NN requests into bdl_knn_batch launches, and copies that
// overlap device work on two copy streams.
//
// One worker thread owns the tree and only orchestrates device work.  The
// host copies run on the client threads: a submission copies its inputs
// into pinned staging, and handing out a completion copies its outputs from
// pinned staging into the client's buffers.  Client threads touch the
// pending queue and the completion table under one mutex, and the pinned
// cache under another.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "bdl.h"
#include "bdl_server.h"
#include "tree_access.hpp"

namespace {

using Clock = std::chrono::steady_clock;

// Cached allocations in power-of-two size classes (device or pinned host).
// A request's staging is taken from here at admission and returned at
// completion, so a steady stream of requests allocates nothing.
class SizeClassCache {
 public:
  explicit SizeClassCache(bool host) : host_(host) {}
  ~SizeClassCache() {
    for (auto& kv : free_)
      for (void* p : kv.second) release(p);
  }
  static size_t round(size_t bytes) {
    size_t c = 1 << 16;
    while (c < bytes) c <<= 1;
    return c;
  }
  void* take(size_t cls) {
    auto& v = free_[cls];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      return p;
    }
    void* p = nullptr;
    hipError_t e = host_ ? hipHostMalloc(&p, cls, hipHostMallocDefault) : hipMalloc(&p, cls);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void give(void* p, size_t cls) {
    if (p) free_[cls].push_back(p);
  }

 private:
  void release(void* p) {
    if (host_)
      (void)hipHostFree(p);
    else
      (void)hipFree(p);
  }
  bool host_;
  std::map<size_t, std::vector<void*>> free_;
};

struct Req {
  uint64_t ticket = 0;
  size_t h_in_bytes = 0, h_out_bytes = 0;  // pinned staging size classes
  bdl_request r{};
  bdl_completion c{};
  size_t in_bytes = 0, out_bytes = 0;  // staging sizes (rounded classes)
  void* d_in = nullptr;                // device: points then ids (updates), queries (k-NN)
  void* d_out = nullptr;               // device: ids then d2 (k-NN)
  void* h_in = nullptr;                // pinned copies of the same
  void* h_out = nullptr;
  hipEvent_t ev_in = nullptr;          // staging copy done
};

struct Launch {
  std::vector<Req*> reqs;
  hipEvent_t ev_done = nullptr;        // outputs back in pinned memory
};

}  // namespace

struct bdl_server {
  bdl_tree* t = nullptr;
  bdl_server_config cfg{};
  int d = 0;
  hipStream_t cs = nullptr;            // the tree's stream (compute)
  hipStream_t h2d = nullptr, d2h = nullptr;
  Clock::time_point t0;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work;     // new submissions / stop
  std::condition_variable cv_done;     // completions
  bool stop = false;
  std::deque<Req*> pending;            // submitted, not admitted (arrival order)
  std::unordered_map<uint64_t, Req*> done;  // completed, not handed out
  std::deque<uint64_t> done_order;
  std::unordered_set<uint64_t> outstanding;  // submitted, completion not handed out
  uint64_t next_ticket = 1;
  uint64_t submitted = 0, completed = 0;
  std::mutex hmu;                      // guards hcache (client threads)
  SizeClassCache hcache{true};
  // worker-only state
  SizeClassCache dcache{false};
  std::vector<hipEvent_t> free_events;
  uint64_t next_seq = 0;
  int64_t next_launch = 0;
  int inflight = 0;
  uint64_t used = 0;
  std::deque<Req*> staged;             // admitted and staged, not launched
  std::deque<Launch> running;          // launched, not completed
};

namespace {

double ms_since(const bdl_server* s) {
  return std::chrono::duration<double, std::milli>(Clock::now() - s->t0).count();
}

void staging_sizes(int d, const bdl_request& r, size_t* in, size_t* out) {
  const size_t n = (size_t)r.n;
  if (r.kind == BDL_REQ_KNN) {
    *in = SizeClassCache::round(n * d * 4);
    *out = SizeClassCache::round(n * (size_t)r.k * 8);
  } else {
    *in = SizeClassCache::round(n * d * 4 + n * 4);
    *out = 0;
  }
}

hipEvent_t get_event(bdl_server* s) {
  if (!s->free_events.empty()) {
    hipEvent_t e = s->free_events.back();
    s->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void put_event(bdl_server* s, hipEvent_t e) {
  if (e) s->free_events.push_back(e);
}

// Pinned staging of a request, filled with its inputs (client thread, at
// submission).  Returns false if pinned memory is short.
bool host_stage(bdl_server* s, Req* q) {
  const size_t n = (size_t)q->r.n;
  {
    std::lock_guard<std::mutex> lk(s->hmu);
    q->h_in = s->hcache.take(q->h_in_bytes);
    q->h_out = q->h_out_bytes ? s->hcache.take(q->h_out_bytes) : nullptr;
  }
  if (!q->h_in || (q->h_out_bytes && !q->h_out)) return false;
  const size_t pb = n * s->d * 4;
  if (n) {
    std::memcpy(q->h_in, q->r.pts, pb);
    if (q->r.kind != BDL_REQ_KNN) std::memcpy((char*)q->h_in + pb, q->r.ids, n * 4);
  }
  return true;
}

void host_unstage(bdl_server* s, Req* q) {
  std::lock_guard<std::mutex> lk(s->hmu);
  s->hcache.give(q->h_in, q->h_in_bytes);
  s->hcache.give(q->h_out, q->h_out_bytes);
  q->h_in = q->h_out = nullptr;
}

// Hand a completed request to a client: outputs into its buffers, pinned
// staging back to the cache (client thread).
bdl_completion hand_out(bdl_server* s, Req* q) {
  if (q->c.status == BDL_OK && q->r.kind == BDL_REQ_KNN && q->r.n) {
    const size_t m = (size_t)q->r.n * q->r.k;
    std::memcpy(q->r.out_ids, q->h_out, m * 4);
    std::memcpy(q->r.out_d2, (char*)q->h_out + m * 4, m * 4);
  }
  host_unstage(s, q);
  const bdl_completion c = q->c;
  delete q;
  return c;
}

// Give the request its device staging and start its input copy on the h2d
// stream.  Returns false (status set) if memory is short.
bool stage(bdl_server* s, Req* q) {
  const size_t n = (size_t)q->r.n;
  q->d_in = s->dcache.take(q->in_bytes);
  if (q->out_bytes) q->d_out = s->dcache.take(q->out_bytes);
  q->ev_in = get_event(s);
  if (!q->d_in || (q->out_bytes && !q->d_out) || !q->ev_in) {
    q->c.status = BDL_ENOMEM;
    return false;
  }
  const size_t pb = n * s->d * 4;
  const size_t bytes = pb + (q->r.kind != BDL_REQ_KNN ? n * 4 : 0);
  if ((bytes && hipMemcpyAsync(q->d_in, q->h_in, bytes, hipMemcpyHostToDevice, s->h2d) !=
                    hipSuccess) ||
      hipEventRecord(q->ev_in, s->h2d) != hipSuccess) {
    q->c.status = BDL_EHIP;
    return false;
  }
  return true;
}

void unstage(bdl_server* s, Req* q) {
  s->dcache.give(q->d_in, q->in_bytes);
  if (q->out_bytes) s->dcache.give(q->d_out, q->out_bytes);
  put_event(s, q->ev_in);
  q->d_in = q->d_out = nullptr;
  q->ev_in = nullptr;
}

// The request's device work and output copy are done: free its device
// staging and slot and post its completion (the outputs are copied to the
// client's buffers when the completion is handed out).
void finish(bdl_server* s, Req* q) {
  unstage(s, q);
  q->c.t_done_ms = ms_since(s);
  --s->inflight;
  s->used -= q->in_bytes + q->out_bytes;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->done.emplace(q->ticket, q);
    s->done_order.push_back(q->ticket);
    ++s->completed;
  }
  s->cv_done.notify_all();
}

// Admit pending requests in arrival order while a slot is free and their
// staging fits the budget; stage each one.  Returns how many were admitted.
int admit(bdl_server* s, int limit) {
  std::vector<Req*> got;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->pending.empty() && (int)got.size() < limit && s->inflight < s->cfg.max_inflight) {
      Req* q = s->pending.front();
      const uint64_t need = q->in_bytes + q->out_bytes;
      if (s->cfg.mem_budget && s->used + need > s->cfg.mem_budget) break;
      s->pending.pop_front();
      ++s->inflight;
      s->used += need;
      got.push_back(q);
    }
  }
  for (Req* q : got) {
    q->c.admit_seq = s->next_seq++;
    q->c.t_admit_ms = ms_since(s);
    if (!stage(s, q)) {
      finish(s, q);
      continue;
    }
    s->staged.push_back(q);
  }
  return (int)got.size();
}

// Enqueue the outputs' copy back to pinned memory after the launch.
bool return_outputs(bdl_server* s, Launch& L, hipEvent_t computed) {
  if (hipStreamWaitEvent(s->d2h, computed, 0) != hipSuccess) return false;
  for (Req* q : L.reqs) {
    if (q->r.kind != BDL_REQ_KNN || q->r.n == 0 || q->c.status != BDL_OK) continue;
    const size_t m = (size_t)q->r.n * q->r.k;
    const char* ids = (const char*)q->d_out;
    if (hipMemcpyAsync(q->h_out, ids, m * 8, hipMemcpyDeviceToHost, s->d2h) != hipSuccess)
      return false;
  }
  return hipEventRecord(L.ev_done, s->d2h) == hipSuccess;
}

// Launch the head of the staged queue: one update, or the k-NN requests up
// to the next update (within the batch limits).
bool launch_next(bdl_server* s) {
  if (s->staged.empty()) return false;
  Launch L;
  L.ev_done = get_event(s);
  hipEvent_t computed = get_event(s);
  const int64_t id = s->next_launch++;
  const double now = ms_since(s);
  Req* head = s->staged.front();
  if (head->r.kind != BDL_REQ_KNN) {
    s->staged.pop_front();
    L.reqs.push_back(head);
    head->c.launch = id;
    head->c.t_start_ms = now;
    (void)hipStreamWaitEvent(s->cs, head->ev_in, 0);
    const size_t n = (size_t)head->r.n;
    const float* p = (const float*)head->d_in;
    const uint32_t* ids = (const uint32_t*)((const char*)head->d_in + n * s->d * 4);
    int rc;
    if (head->r.kind == BDL_REQ_INSERT) {
      rc = bdl_insert(s->t, p, ids, (int64_t)n);
    } else {
      int64_t ne = 0;
      rc = bdl_erase(s->t, p, ids, (int64_t)n, &ne);
      head->c.n_erased = ne;
    }
    head->c.status = rc;
  } else {
    // The k-NN requests up to the next update read one snapshot, so they
    // may run in any order.  Small ones go together into one batched
    // launch, ahead of large ones; a large request (more than
    // kAloneQueries queries) runs alone as a plain call, so that it neither
    // holds small requests back until it ends nor waits for them.
    constexpr int64_t kAloneQueries = 16384;
    std::vector<Req*> pick;
    int64_t nq = 0;
    for (auto it = s->staged.begin(); it != s->staged.end();) {
      Req* q = *it;
      if (q->r.kind != BDL_REQ_KNN) break;
      if (q->r.n > kAloneQueries) {
        ++it;
        continue;
      }
      if (!pick.empty() && ((int)pick.size() >= s->cfg.max_batch_requests ||
                            nq + q->r.n > s->cfg.max_batch_queries))
        break;
      pick.push_back(q);
      nq += q->r.n;
      it = s->staged.erase(it);
    }
    if (pick.empty()) {
      pick.push_back(s->staged.front());  // the run holds only large requests
      s->staged.pop_front();
    }
    std::vector<bdl_knn_request> kr;
    for (Req* q : pick) {
      L.reqs.push_back(q);
      q->c.launch = id;
      q->c.t_start_ms = now;
      (void)hipStreamWaitEvent(s->cs, q->ev_in, 0);
      if (q->r.n == 0) continue;
      bdl_knn_request r;
      r.q = (const float*)q->d_in;
      r.nq = q->r.n;
      r.k = q->r.k;
      r.pad_ = 0;
      r.out_ids = (uint32_t*)q->d_out;
      r.out_d2 = (float*)((char*)q->d_out + (size_t)q->r.n * q->r.k * 4);
      kr.push_back(r);
    }
    // a lone request runs as a plain call (same results; no request table,
    // gather or graph bucket to pay for)
    int rc = kr.empty() ? BDL_OK
                        : (kr.size() > 1 ? bdl_knn_batch(s->t, kr.data(), (int32_t)kr.size())
                                         : bdl_knn(s->t, kr[0].q, kr[0].nq, kr[0].k,
                                                   kr[0].out_ids, kr[0].out_d2));
    for (Req* q : L.reqs) q->c.status = rc;
  }
  if (!L.ev_done || !computed || hipEventRecord(computed, s->cs) != hipSuccess ||
      !return_outputs(s, L, computed)) {
    for (Req* q : L.reqs) {
      if (q->c.status == BDL_OK) q->c.status = BDL_EHIP;
    }
    (void)hipStreamSynchronize(s->cs);
    (void)hipStreamSynchronize(s->d2h);
  }
  put_event(s, computed);  // reusable once recorded: later waits use the copy
  s->running.push_back(L);
  return true;
}

// Complete launches whose outputs are back, oldest first.
int reap(bdl_server* s, bool block) {
  int n = 0;
  while (!s->running.empty()) {
    Launch& L = s->running.front();
    if (block) {
      (void)hipEventSynchronize(L.ev_done);
    } else if (hipEventQuery(L.ev_done) != hipSuccess) {
      break;
    }
    for (Req* q : L.reqs) finish(s, q);
    put_event(s, L.ev_done);
    s->running.pop_front();
    ++n;
    block = false;
  }
  return n;
}

void loop_batched(bdl_server* s) {
  for (;;) {
    bool progress = false;
    progress |= reap(s, false) > 0;
    progress |= admit(s, 1 << 30) > 0;
    while ((int)s->running.size() < s->cfg.max_launches && !s->staged.empty()) {
      // an erase blocks this thread until the device has done it (it reads
      // the live counts back); launch it only once earlier launches are
      // reaped, so that their completions are not held back behind it
      if (s->staged.front()->r.kind == BDL_REQ_ERASE && !s->running.empty()) break;
      progress |= launch_next(s);
    }
    if (progress) continue;
    if (!s->running.empty()) {
      // device work outstanding and nothing to admit: wait for the oldest
      // launch (a timed sleep would add the timer's slack, tens of
      // microseconds, to every completion); requests that arrive meanwhile
      // are admitted as soon as it is done
      bool idle;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        idle = s->pending.empty();
      }
      if (idle)
        (void)hipEventSynchronize(s->running.front().ev_done);
      else
        std::this_thread::yield();  // pending work waits for a slot or budget
      continue;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop && s->pending.empty() && s->staged.empty() && s->running.empty()) return;
    // nothing on the device: sleep until a submission arrives
    if (s->pending.empty()) s->cv_work.wait_for(lk, std::chrono::microseconds(5000));
  }
}

void loop_fifo(bdl_server* s) {
  for (;;) {
    if (admit(s, 1) > 0) {
      if (!s->staged.empty()) {
        launch_next(s);
        reap(s, true);
      }
      continue;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop && s->pending.empty()) return;
    s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
  }
}

}  // namespace

extern "C" {

int bdl_server_create(bdl_tree* t, const bdl_server_config* cfg, bdl_server** out) {
  if (!t || !cfg || !out) return bdl::tree_fail(BDL_EINVAL, "null argument");
  *out = nullptr;
  if ((cfg->mode != BDL_SERVE_FIFO && cfg->mode != BDL_SERVE_BATCHED) || cfg->max_inflight < 1 ||
      cfg->max_batch_requests < 1 || cfg->max_batch_requests > 65536 ||
      cfg->max_launches < 1 || cfg->max_launches > 8 || cfg->max_batch_queries < 1)
    return bdl::tree_fail(BDL_EINVAL, "bad server configuration");
  bdl_server* s = new bdl_server();
  s->t = t;
  s->cfg = *cfg;
  s->d = bdl::tree_dim(t);
  s->cs = bdl::tree_stream(t);
  s->t0 = Clock::now();
  if (hipStreamCreateWithFlags(&s->h2d, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->d2h, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    if (s->h2d) (void)hipStreamDestroy(s->h2d);
    delete s;
    return bdl::tree_fail(BDL_EHIP, "cannot create copy streams");
  }
  s->worker = std::thread(cfg->mode == BDL_SERVE_FIFO ? loop_fifo : loop_batched, s);
  *out = s;
  return BDL_OK;
}

int bdl_server_submit(bdl_server* s, const bdl_request* r, uint64_t* ticket) {
  if (!s || !r) return bdl::tree_fail(BDL_EINVAL, "null argument");
  const double t_arrive = ms_since(s);
  if (r->kind != BDL_REQ_KNN && r->kind != BDL_REQ_INSERT && r->kind != BDL_REQ_ERASE)
    return bdl::tree_fail(BDL_EINVAL, "unknown request kind");
  if (r->n < 0) return bdl::tree_fail(BDL_EINVAL, "negative size");
  if (r->kind == BDL_REQ_KNN && (r->k < 1 || r->k > BDL_MAX_K))
    return bdl::tree_fail(BDL_EINVAL, "k must be in 1..64");
  if (r->n > 0 && (!r->pts || (r->kind == BDL_REQ_KNN ? (!r->out_ids || !r->out_d2) : !r->ids)))
    return bdl::tree_fail(BDL_EINVAL, "null request buffer");
  if (r->n >= (1ll << 31)) return bdl::tree_fail(BDL_EINVAL, "request too large");
  Req* q = new Req();
  q->r = *r;
  staging_sizes(s->d, *r, &q->in_bytes, &q->out_bytes);
  if (s->cfg.mem_budget && q->in_bytes + q->out_bytes > s->cfg.mem_budget) {
    delete q;
    return bdl::tree_fail(BDL_EINVAL, "request larger than the memory budget");
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete q;
      return bdl::tree_fail(BDL_EINVAL, "server is stopping");
    }
  }
  q->h_in_bytes = q->in_bytes;
  q->h_out_bytes = q->out_bytes;
  if (!host_stage(s, q)) {
    host_unstage(s, q);
    delete q;
    return bdl::tree_fail(BDL_ENOMEM, "cannot allocate pinned staging");
  }
  q->c.kind = r->kind;
  q->c.launch = -1;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      host_unstage(s, q);
      delete q;
      return bdl::tree_fail(BDL_EINVAL, "server is stopping");
    }
    q->ticket = s->next_ticket++;
    q->c.ticket = q->ticket;
    q->c.t_submit_ms = t_arrive;
    s->pending.push_back(q);
    s->outstanding.insert(q->ticket);
    ++s->submitted;
    if (ticket) *ticket = q->ticket;
  }
  s->cv_work.notify_one();
  return BDL_OK;
}

int bdl_server_wait(bdl_server* s, uint64_t ticket, bdl_completion* out) {
  if (!s) return bdl::tree_fail(BDL_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->outstanding.count(ticket))
    return bdl::tree_fail(BDL_EINVAL, "unknown ticket, or its completion was handed out");
  s->cv_done.wait(lk, [&] { return s->done.count(ticket) > 0; });
  auto it = s->done.find(ticket);
  Req* q = it->second;
  s->done.erase(it);
  s->outstanding.erase(ticket);
  lk.unlock();
  const bdl_completion c = hand_out(s, q);
  if (out) *out = c;
  return BDL_OK;
}

int bdl_server_poll(bdl_server* s, bdl_completion* out, int32_t max, int32_t* n) {
  if (!s || (max > 0 && !out)) return bdl::tree_fail(BDL_EINVAL, "null argument");
  std::vector<Req*> got;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while ((int32_t)got.size() < max && !s->done_order.empty()) {
      const uint64_t tk = s->done_order.front();
      s->done_order.pop_front();
      auto it = s->done.find(tk);
      if (it == s->done.end()) continue;  // handed out by bdl_server_wait
      got.push_back(it->second);
      s->done.erase(it);
      s->outstanding.erase(tk);
    }
  }
  for (size_t i = 0; i < got.size(); ++i) out[i] = hand_out(s, got[i]);
  if (n) *n = (int32_t)got.size();
  return BDL_OK;
}

int bdl_server_drain(bdl_server* s) {
  if (!s) return bdl::tree_fail(BDL_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  const uint64_t target = s->submitted;
  s->cv_done.wait(lk, [&] { return s->completed >= target; });
  return BDL_OK;
}

void bdl_server_destroy(bdl_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->done) {
    host_unstage(s, kv.second);
    delete kv.second;
  }
  s->done.clear();
  (void)hipStreamSynchronize(s->h2d);
  (void)hipStreamSynchronize(s->d2h);
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  (void)hipStreamDestroy(s->h2d);
  (void)hipStreamDestroy(s->d2h);
  delete s;
}

}  // extern "C"
