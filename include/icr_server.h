/*
 * icr_server.h - served ICR: continuous batching of forward / adjoint / metric requests
 * on one GPU (the serving mode of the ICR library declared in icr.h).
 *
 * Requests against registered plans (or against prior configurations, whose plans the
 * server builds on first use and caches) are queued, and a worker thread launches them:
 *  - grouped mode (cfg.grouped): requests of ANY prior (1-D, 2-D, 3-D, any level sizes,
 *    depth, matrices and precision) and any op are grouped, oldest first, up to
 *    max_batch: the k-th launch of a group applies the k-th step of every request's sweep
 *    (level 0 or one refinement level, forward or adjoint) from a device table of steps,
 *    one table copy per group. A request is admitted when its workspace fits the arena;
 *    its own completion event follows its last step. At most group_streams groups run at
 *    once, so requests that arrive while groups run are gathered into the next one. A
 *    request with a refinement level of at least large_step fine pixels (bandwidth-bound,
 *    not launch-bound), or on a 1-D prior (whose own sweep runs its small levels in one
 *    fused launch), runs as below instead, with the specialised kernels.
 *  - homogeneous batches: pending requests with the same (plan, op), oldest first, in
 *    batches of a power of two up to max_batch, admitted when the batch's buffers fit the
 *    arena (first fit): gather the inputs into a contiguous batch, run the batched sweep (a
 *    hipGraph captured once per (plan, op, batch size) when use_graphs is set and the
 *    batch needs at most 1/32 of the arena; larger batches launch eagerly), scatter the
 *    outputs, record a completion event (a single request without a graph, or with input
 *    rows of 1 MiB or more, sweeps its own buffers, only its workspace taken from the
 *    arena).
 * Requests that arrive while others run are admitted as streams and memory free up, so
 * work of different priors overlaps on the device. max_batch = 1, n_streams = 1,
 * use_graphs = 0, grouped = 0 is the one-launch-per-request baseline.
 *
 * Conventions: as in icr.h (status codes, icr_last_error, caller-owned device buffers).
 * The server allocates its arena once at creation; nothing is allocated per request
 * except when a new graph is captured (from the arena) or a plan is built for a new
 * prior configuration. A request's buffers must stay
 * valid and untouched until icr_server_query reports it done (see icr_server_submit for
 * the ordering with the caller's stream). Results are identical
 * whether a request runs alone or in a batch or group (each sample is computed by the
 * same kernels in the same order; which path a request takes depends only on its prior
 * and the server's configuration).
 */
#ifndef ICR_SERVER_H
#define ICR_SERVER_H

#include <stdint.h>

#include "icr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum icr_op {
  ICR_OP_FORWARD = 0,  /* in: xi [n_xi]     out: s [n_out]       */
  ICR_OP_ADJOINT = 1,  /* in: s_bar [n_out] out: xi_bar [n_xi]   */
  ICR_OP_METRIC = 2    /* in: v [n_xi], w [n_out]  out: [n_xi]   */
} icr_op;

typedef struct icr_server_config {
  int64_t hbm_budget_bytes;  /* size of the arena batches and captured graphs live in */
  int32_t max_batch;         /* 1..64 requests per launch (batch or group) */
  int32_t n_streams;         /* 1..16 batches or groups in flight at once */
  int32_t use_graphs;        /* replay captured hipGraphs for homogeneous batched sweeps */
  int32_t grouped;           /* group requests of any prior and op (see above) */
  int64_t large_step;        /* grouped mode: fine pixels of a refinement level from which a
                                request runs on its own; 0 = 1048576 */
  int32_t group_streams;     /* grouped mode: groups in flight at once, 1..n_streams; 0 = 1 */
  int32_t max_plans;         /* prior configurations whose plans stay cached; 0 = 256 */
} icr_server_config;

typedef struct icr_server_statistics {
  int64_t completed;
  int64_t pending;
  int64_t batches;             /* launches */
  int64_t batched_requests;    /* requests over all launches */
  int64_t graph_captures;
  int64_t admissions_deferred; /* batches that had to wait for (or shrink to fit) memory */
  int64_t arena_bytes;
  int64_t arena_in_use;
  int64_t groups;              /* grouped launches sequences (one per group) */
  int64_t grouped_requests;    /* requests served in groups */
  int64_t plans_built;         /* plans the server built for prior configurations */
  int64_t plan_cache_hits;     /* submissions by configuration whose plan was cached or in build */
} icr_server_statistics;

typedef struct icr_server icr_server;

/* Create a server on the current device (arena, streams, worker thread). */
icr_status icr_server_create(const icr_server_config* cfg, icr_server** out);

/* Register a plan (it must outlive the server); returns its id. */
icr_status icr_server_register_plan(icr_server* server, const icr_plan* plan, int32_t* plan_id);

/* Queue one request (a single sample). `w` (metric only) is [n_out] in the plan's
 * arithmetic type. ICR_ERR_OUT_OF_MEMORY if a single request cannot fit the arena.
 * Ordering: `in` and `w` may still be in production on hip_stream (NULL = the legacy
 * default stream): the server records an event there at submission and the request's
 * first read waits for it, so work the caller queued on that stream before this call
 * is complete before the request starts. `in`, `out` and `w` must stay allocated and
 * must not be written by the caller until icr_server_query reports the request done;
 * `out` is complete once it does. */
icr_status icr_server_submit(icr_server* server, int32_t plan_id, int32_t op, const void* in, void* out,
                             const void* w, void* hip_stream, int64_t* request_id);

/*
 * Queue one request against a prior configuration instead of a registered plan. The
 * server keeps a cache of plans keyed by the whole configuration (dimension, level-0
 * shape, depth, kernel, length scale, chart, precision, ...); on a miss a builder thread
 * runs icr_build_matrices while the worker keeps serving other requests, and the
 * request (and every later one for that configuration) starts once the plan is built:
 * the build is part of its latency. The least recently used idle plans are destroyed
 * beyond max_plans. If the build fails, icr_server_query reports the request done and
 * returns the build's status. Other arguments as for icr_server_submit.
 */
icr_status icr_server_submit_prior(icr_server* server, const icr_config* cfg, int32_t op, const void* in,
                                   void* out, const void* w, void* hip_stream, int64_t* request_id);

/* State of a request; times are host steady-clock seconds (submit, launch of its batch,
 * observed completion). Returns the build status of a request whose prior's plan could
 * not be built (with *done = 1). */
icr_status icr_server_query(icr_server* server, int64_t request_id, int32_t* done, double* t_submit,
                            double* t_launch, double* t_done, int32_t* batch_size);

/* Wait until no request is pending or in flight (timeout_s <= 0: no limit). */
icr_status icr_server_drain(icr_server* server, double timeout_s);

icr_status icr_server_stats(icr_server* server, icr_server_statistics* stats);

/* Stop the worker, wait for in-flight work, free the arena, graphs and streams. */
icr_status icr_server_destroy(icr_server* server);

#ifdef __cplusplus
}
#endif

#endif /* ICR_SERVER_H */
