/* Served form of the BDL-tree: a request loop that keeps one tree resident
 * in device memory and serves interleaved kNN_L, Insert_L and Erase_L
 * requests from client threads.
 *
 * Requests are admitted in arrival order while a request slot is free and
 * the device staging memory they need fits the budget.  Admission order is
 * the order of the semantics: every k-NN request sees exactly the updates
 * admitted before it (a snapshot epoch), so its result equals that of the
 * plain calls bdl_insert / bdl_erase / bdl_knn replayed one at a time in
 * admission order.
 *
 * In the batched mode the loop keeps the device busy with continuous
 * batching: the k-NN requests admitted between two updates run together
 * as one bdl_knn_batch launch; requests that arrive while a launch runs are
 * copied to the device on a copy stream meanwhile and join the next launch,
 * and results return on a second copy stream while later launches compute.
 * The FIFO mode is the plain loop it is compared with: one request at a
 * time, copy in, plain call, copy out, then the next.
 *
 * All pointers in a request are HOST memory owned by the client; they must
 * stay valid, and outputs untouched, until the request's completion has
 * been handed out (bdl_server_wait or bdl_server_poll).  While a server
 * exists, only its loop may use the tree.
 */
#ifndef BDL_SERVER_H
#define BDL_SERVER_H

#include "bdl.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bdl_server bdl_server; /* opaque, owned by the library */

#define BDL_REQ_KNN 0
#define BDL_REQ_INSERT 1
#define BDL_REQ_ERASE 2

#define BDL_SERVE_FIFO 0    /* one request at a time, plain calls, no overlap */
#define BDL_SERVE_BATCHED 1 /* continuous batching with overlapped copies */

typedef struct {
  int32_t mode;               /* BDL_SERVE_FIFO or BDL_SERVE_BATCHED */
  int32_t max_inflight;       /* request slots: admitted, not yet completed (>= 1) */
  int32_t max_batch_requests; /* k-NN requests per batched launch (1..65536) */
  int32_t max_launches;       /* launches queued on the device at once (1..8) */
  int64_t max_batch_queries;  /* queries per batched launch (>= 1) */
  uint64_t mem_budget;        /* device staging bytes (inputs and outputs of
                                 admitted requests) held at once; 0 = no limit */
} bdl_server_config;

typedef struct {
  int32_t kind;        /* BDL_REQ_* */
  int32_t k;           /* k-NN: 1..BDL_MAX_K; ignored otherwise */
  int64_t n;           /* points or queries (>= 0) */
  const float* pts;    /* host [n][dim]: points (updates) or queries (k-NN) */
  const uint32_t* ids; /* host [n]: ids of inserted / erased points */
  uint32_t* out_ids;   /* host [n][k] (k-NN) */
  float* out_d2;       /* host [n][k] (k-NN) */
} bdl_request;

typedef struct {
  uint64_t ticket;
  uint64_t admit_seq;  /* position in admission order, from 0 */
  int32_t kind;
  int32_t status;      /* BDL_OK or the failing call's code */
  int64_t n_erased;    /* Erase_L: points erased */
  int64_t launch;      /* index of the device launch that served it */
  double t_submit_ms;  /* times since the server's creation */
  double t_admit_ms;
  double t_start_ms;   /* its launch was enqueued */
  double t_done_ms;    /* outputs written to the client's buffers */
} bdl_completion;

/* Start a request loop (one worker thread) over tree t.  BDL_EINVAL on a
 * bad configuration, BDL_ENOMEM / BDL_EHIP if streams or events cannot be
 * made. */
int bdl_server_create(bdl_tree* t, const bdl_server_config* cfg, bdl_server** out);

/* Queue a request (any thread).  *ticket receives its ticket.  BDL_EINVAL
 * for a malformed request, or one whose staging exceeds the whole budget;
 * nothing is queued then. */
int bdl_server_submit(bdl_server* s, const bdl_request* r, uint64_t* ticket);

/* Block until request `ticket` has completed and hand out its completion.
 * BDL_EINVAL for an unknown ticket or one already handed out. */
int bdl_server_wait(bdl_server* s, uint64_t ticket, bdl_completion* out);

/* Hand out up to max completions (in completion order) without blocking;
 * *n receives how many. */
int bdl_server_poll(bdl_server* s, bdl_completion* out, int32_t max, int32_t* n);

/* Block until every request submitted so far has completed. */
int bdl_server_drain(bdl_server* s);

/* Completes every submitted request, stops the loop and frees the server's
 * memory (the tree stays). */
void bdl_server_destroy(bdl_server* s);

#ifdef __cplusplus
}
#endif
#endif /* BDL_SERVER_H */
