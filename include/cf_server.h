/*
 * cf_server.h -- a serving loop over many resident cuckoo filters (part of
 * libcf.so; built on the filter sets of cf_set.h).
 *
 * Filters are declared up front and admitted into device memory in
 * declaration order while their tables fit the HBM budget; the others wait
 * and are admitted as released filters free memory.  Clients submit
 * requests -- one operation kind (CF_OP_*) on one filter for n keys -- from
 * any thread; a scheduler thread owned by the server forms batches
 * continuously: whenever a batch slot is free it takes the pending requests,
 * in arrival order, that fit the batch (max_batch operations, max_requests
 * requests) and executes them as one mixed batch of the filter set, while
 * the previous batches are still on the device.  Each of the `depth` slots
 * has a stream and a scratch lane of its own, so batches in different slots
 * run on the device at the same time; a batch waits (on the device, by
 * event) only for the in-flight batches that touch one of its filters.
 * Server batches always run the set's class-kernel form with the class
 * chains on the slot's stream (the persistent form takes the whole device).
 * Each operation is the filter operation of Cuckoo-GPU (arXiv 2603.15486):
 * Alg. 2 query, Alg. 3 delete, Alg. 1 insert with the eviction search of
 * Sec. 4.6.1.
 *
 * Ordering.  Requests on one filter take effect in arrival order: a request
 * joins a batch only if every earlier pending request on its filter has
 * joined and the batch's phase order (queries, then deletes, then inserts,
 * see cf_set.h) agrees with arrival order on that filter.  So a request's
 * results are those of running all requests one at a time in arrival order.
 *
 * Modes.  CF_SERVE_BATCHED is the loop above.  CF_SERVE_PER_REQUEST runs
 * each request alone as one kernel launch on its filter (cf_set_apply), in
 * arrival order, with up to `depth` requests in flight: the baseline.  A
 * mixed batch costs a fixed chain of launches (table copy, gather, the set's
 * partition and phase kernels, scatter), so batched mode adapts to the load
 * (direct_below): while fewer than direct_below requests are pending, each
 * free slot takes one request and runs it as one launch, so a light load is
 * served with the per-request latency and requests still run side by side
 * in different slots; once that many are pending, slots take whole batches;
 * and a batch that still holds fewer than direct_below requests (its other
 * candidates waiting on filter order) runs them one launch each.  Large
 * requests (solo_above keys or more) run alone in a slot of their own while
 * fewer than 4 x direct_below requests are pending: they fill the device by
 * themselves, and in a batch they would hold back the small requests batched
 * with them; under a longer backlog they join batches, which serve more
 * operations per second.  The results are the same either way.
 *
 * Buffers.  d_keys (uint64[n]) and d_results (uint8[n]) must be readable and
 * writable by the device (device memory or mapped host memory) and stay
 * valid until the request completes.  The server works on a stream of its
 * own that does not wait for the caller's streams: the keys must be written
 * (and no other work may still target either buffer) when the request is
 * submitted, e.g. by synchronising the producing stream first.  Results:
 * 1 found / removed / stored, 0 not, 0xFF if the request failed (released
 * filter).
 */
#ifndef CF_SERVER_H
#define CF_SERVER_H

#include <stdint.h>

#include "cf.h"
#include "cf_set.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cf_server cf_server;

enum { CF_SERVE_BATCHED = 0, CF_SERVE_PER_REQUEST = 1 };

typedef struct {
    uint64_t hbm_budget;   /* bytes of tables kept resident; 0 = no limit        */
    uint64_t max_batch;    /* operations per batch (>= the largest request)      */
    uint32_t max_requests; /* requests per batch (slots), 1..65536               */
    uint32_t mode;         /* CF_SERVE_BATCHED or CF_SERVE_PER_REQUEST           */
    uint32_t depth;        /* batches (or requests) in flight, 1..8: one stream
                              and one scratch lane each                          */
    uint32_t direct_below; /* batched mode: with fewer requests pending than
                              this, a slot takes a single request; a batch of
                              fewer requests than this runs them one launch
                              each, in arrival order; 0 = default (16),
                              1 = always form batches                           */
    uint32_t solo_above;   /* batched mode, short backlog: a request of at least
                              this many keys runs alone, one launch in a slot
                              of its own; 0 = default (2^16), UINT32_MAX = never */
    uint32_t reserved;     /* must be 0                                          */
} cf_server_config;

typedef struct {
    uint64_t id;
    uint64_t t_submit_ns;  /* steady-clock times since the server started        */
    uint64_t t_start_ns;   /* when its batch was handed to the device            */
    uint64_t t_done_ns;    /* when the scheduler saw its batch complete          */
    uint64_t batch;        /* sequence number of the batch that carried it       */
    int32_t status;        /* CF_OK; CF_EINVAL for a released filter; CF_EDEVICE if
                            * its batch failed to launch (results undefined)     */
    uint32_t reserved;
} cf_request_info;

typedef struct {
    uint64_t requests;       /* completed                                      */
    uint64_t operations;     /* keys of completed requests                     */
    uint64_t batches;        /* device batches (requests in per-request mode)  */
    uint64_t held;           /* pending requests on filters not yet admitted   */
    uint64_t resident_bytes; /* tables currently in device memory              */
    uint32_t resident;       /* filters admitted                               */
    uint32_t reserved;
} cf_server_stats;

/* Declare nfilters filters and start the scheduler thread on the current
 * device.  Filters are admitted in order while they fit hbm_budget.  When
 * all of them fit, their tables share one allocation (cf_set_create), and a
 * released filter's table stays allocated until the server is destroyed
 * (no filter waits for that memory).  Errors: CF_EINVAL (config), those of
 * cf_set_create. */
cf_status cf_server_create(const cf_params *params, uint32_t nfilters,
                           const cf_server_config *config, cf_server **out);

/* Stop the scheduler after the requests already taken complete; requests
 * still pending are completed with status CF_EINVAL.  NULL accepted. */
cf_status cf_server_destroy(cf_server *server);

/* Enqueue a request; *id_out receives its id.  n <= max_batch.  Returns
 * CF_EINVAL for a bad filter id, kind, size or NULL buffer. */
cf_status cf_server_submit(cf_server *server, uint32_t fid, uint32_t op, const uint64_t *d_keys,
                           uint64_t n, uint8_t *d_results, uint64_t *id_out);

/* Block until request `id` has completed; fill *info (nullable). */
cf_status cf_server_wait(cf_server *server, uint64_t id, cf_request_info *info);

/* Block until every request on an admitted filter has completed (requests
 * held for filters that are not admitted stay pending). */
cf_status cf_server_drain(cf_server *server);

/* Drop an admitted filter after its pending requests completed, free its
 * table (see cf_server_create) and admit waiting filters that now fit.
 * Later requests on it fail. */
cf_status cf_server_release(cf_server *server, uint32_t fid);

/* 1 if the filter is admitted (its table is in device memory), else 0. */
cf_status cf_server_resident(cf_server *server, uint32_t fid, int *out);

cf_status cf_server_stats_get(cf_server *server, cf_server_stats *out);

/* The server's filter set (for counts, export and import; use only while
 * no request is pending). */
cf_set *cf_server_set(cf_server *server);

/* Replay a request trace from a client thread owned by the server: request
 * k is submitted at t0 + arrival_ns[k] (t0 = the call), with filter fids[k],
 * kind ops[k], keys d_keys + key_off[k], results d_results + key_off[k] and
 * n[k] keys.  Returns at once; ids are first_id_out .. first_id_out+count-1
 * in trace order, and each request's t_submit_ns is its scheduled arrival
 * time (so latencies include any delay in handing it over).  cf_server_drain
 * waits for the whole trace.  Replays may be started from several threads,
 * but not while cf_server_destroy runs; destroy waits for every trace to
 * have been submitted. */
cf_status cf_server_replay(cf_server *server, uint64_t count, const uint64_t *arrival_ns,
                           const uint32_t *fids, const uint32_t *ops, const uint64_t *key_off,
                           const uint64_t *n, const uint64_t *d_keys, uint8_t *d_results,
                           uint64_t *first_id_out);

#ifdef __cplusplus
}
#endif
#endif /* CF_SERVER_H */
