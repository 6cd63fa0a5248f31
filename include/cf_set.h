/*
 * cf_set.h -- many cuckoo filters resident on one device, driven by mixed
 * batches (part of libcf.so; see cf.h for the filter itself).
 *
 * A set holds up to 65536 filters, each with its own cf_params (bucket
 * count, slots per bucket, fingerprint width, hash, eviction policy), with
 * all tables in one device arena.  A mixed batch is n operations given as
 * three device arrays: kind (CF_OP_*), filter id and key.  Every operation
 * is the filter operation of Cuckoo-GPU (arXiv 2603.15486): Alg. 2 query,
 * Alg. 3 delete, Alg. 1 insert with the eviction search of Sec. 4.6.1 (or the
 * random walk), on the table of its filter.
 *
 * Batch semantics.  Because a query must not overlap writes to its filter
 * (Sec. 4.4), a batch runs in three phases: every query sees its filter as it
 * was before the batch; then all deletes run; then all inserts.  For each
 * filter the result equals applying the batch's queries, then its deletes,
 * then its inserts, each group in any order.  Results: uint8 per operation,
 * 1 = found / removed / stored, 0 = not, 0xFF = invalid operation (unknown
 * kind or filter id), which is otherwise ignored.
 *
 * Conventions as in cf.h: d_* are caller-owned device pointers valid until
 * the stream work completes; stream is a hipStream_t as void*; batch calls
 * only enqueue work.
 *
 * One batch at a time per set.  cf_set_execute, cf_graph_launch of the
 * set's graphs and cf_set_apply all use the set's one batch scratch (the
 * chunks' sorted operation indices, bin offsets and eviction queue), so two
 * of them in flight at once would read each other's indices.  Order every
 * batch call on a set on one stream, or synchronise between streams.  The
 * rules of cf.h hold per filter inside a batch by construction (the phase
 * order), and across batches by this ordering.  Breaking it is not
 * detected: results are undefined.
 */
#ifndef CF_SET_H
#define CF_SET_H

#include <stdint.h>

#include "cf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cf_set cf_set;     /* opaque, owned by the library */
typedef struct cf_graph cf_graph; /* a captured batch execution  */

enum { CF_OP_QUERY = 0, CF_OP_DELETE = 1, CF_OP_INSERT = 2 };

/* Launch shape of a batch, chosen by cf_set_tune or by hand.  A batch runs
 * in one of two forms with the same results:
 *  - class kernels (persistent = 0): a partition launch, then per class
 *    (f, b, hash, placement) a query, a delete and an insert launch;
 *  - persistent (persistent = 1): one cooperative launch whose resident
 *    blocks run the partition and the three phases, separated by grid-wide
 *    barriers.  Only for sets whose filters all share f, hash and placement
 *    (b may differ); others get CF_EUNSUPPORTED.
 * chunk: operations per chunk; a block works on whole chunks (64..4096, a
 * multiple of 64; 0 = default 2048).
 * streams (class kernels): on how many streams the classes run their
 * query-delete-insert chains at the same time (filters of different classes
 * share no state, so only each chain is ordered).  Classes go round-robin
 * onto the streams; stream 0 is the caller's, the others are the set's own,
 * forked from and joined back into the caller's stream by events (so graph
 * capture sees the same dependencies).  1 = every chain on the caller's
 * stream, one after another; 0 = default (the class count, at most 4); at
 * most 8.
 * block (persistent): threads per block, 256 or 512 (0 = 256).
 * blocks_per_cu (persistent): resident blocks per compute unit, at most
 * cf_set_persistent_capacity (0 = that many; cf_set_get_shape then reports
 * the number).
 * wave_bfs: how the breadth-first eviction search (Sec. 4.6.1) of a key
 * whose two buckets are full runs: 0 = one lane per key, loading the other
 * buckets of up to 128 bytes' worth of candidates together; 1 = one wave per
 * key, each lane probing one of the b/2 candidates and a ballot choosing the
 * lowest that fits (one dependent probe per level; the block's waves take
 * the keys in turn).  Both choose the same candidate on an unchanged table.
 * The random walk is one lane per key either way.
 * fused (class kernels only): 1 = one launch per phase instead of one per
 * (phase, class): after the partition, one query launch covers the queries
 * of every class (the class's b chosen per block at run time), then one
 * delete and one insert launch, all on the caller's stream (streams is then
 * unused).  Same results; needs the same as the persistent form (every
 * filter sharing f, hash and placement), else CF_EUNSUPPORTED.  0 = one
 * launch per (phase, class). */
typedef struct {
    uint32_t chunk;
    uint32_t streams;
    uint32_t persistent;
    uint32_t block;
    uint32_t blocks_per_cu;
    uint32_t wave_bfs;
    uint32_t fused;
} cf_set_shape;

/* Flags of cf_set_create. */
enum { CF_SET_DEFER_TABLES = 1 }; /* allocate no table until cf_set_attach */

/* Create nfilters filters (params[0..nfilters-1], each validated as in
 * cf_create) able to take batches of up to max_batch operations.  Every
 * filter's table is allocated (empty) unless flags has CF_SET_DEFER_TABLES,
 * in which case filters start detached.  A set created with its tables holds
 * them in one device allocation (each table at a 256-byte boundary), or in
 * one allocation per table when the device has no block that large.
 * Synchronous.  Errors: CF_EINVAL, CF_EUNSUPPORTED, CF_ENOMEM (tables,
 * scratch or counters do not fit). */
cf_status cf_set_create(const cf_params *params, uint32_t nfilters, uint64_t max_batch,
                        uint32_t flags, cf_set **out);

/* Device bytes of the set's fixed part (per-filter counters and logs, batch
 * scratch) and of all its tables; 0 for invalid parameters.  A filter's
 * table takes cf_table_bytes of its params, rounded up to 256 bytes. */
uint64_t cf_set_bytes(const cf_params *params, uint32_t nfilters, uint64_t max_batch);

/* Attach (allocate an empty table for, and clear the counters of) or detach
 * (free the table of) one filter.  In a set created with its tables, a
 * detached filter's table keeps its place in the set's allocation, and
 * attaching it again clears that place.  Operations on a detached filter
 * are invalid (result 0xFF).  Both synchronise the device; not for hot
 * paths.  cf_set_attached writes 1 or 0 to *out. */
cf_status cf_set_attach(cf_set *set, uint32_t fid);
cf_status cf_set_detach(cf_set *set, uint32_t fid);
cf_status cf_set_attached(const cf_set *set, uint32_t fid, int *out);

/* One operation kind on one attached filter of the set, as cf_query /
 * cf_delete / cf_insert would run it: a single launch, no batching.  n <=
 * max_batch; d_results: uint8[n] (flags as in cf.h).  Stream-ordered with the
 * set's other calls (it shares the set's scratch). */
cf_status cf_set_apply(cf_set *set, uint32_t fid, uint32_t op, const uint64_t *d_keys,
                       uint64_t n, uint8_t *d_results, void *stream);

cf_status cf_set_destroy(cf_set *set); /* NULL accepted; synchronises */

/* Execute one mixed batch (see batch semantics above).  n <= max_batch.
 * d_ops: uint8[n]; d_fids: uint32[n]; d_keys: uint64[n], 8-byte aligned;
 * d_results: uint8[n].  n = 0 is a no-op. */
cf_status cf_set_execute(cf_set *set, const uint8_t *d_ops, const uint32_t *d_fids,
                         const uint64_t *d_keys, uint64_t n, uint8_t *d_results, void *stream);

/* Capture the batch execution for fixed buffers into a HIP graph.  The
 * operation count is read at run time from d_n (device uint64, <= max_batch),
 * so one graph serves batches of any size: fill the buffers and d_n, then
 * cf_graph_launch.  The graph is tied to the set's current launch shape. */
cf_status cf_set_graph_create(cf_set *set, const uint8_t *d_ops, const uint32_t *d_fids,
                              const uint64_t *d_keys, const uint64_t *d_n, uint8_t *d_results,
                              cf_graph **out);
cf_status cf_graph_launch(cf_graph *graph, void *stream);
cf_status cf_graph_destroy(cf_graph *graph); /* NULL accepted */

/* Per-filter occupancy and failure counts: out[nfilters], host or device
 * memory, stream-ordered. */
cf_status cf_set_counts(cf_set *set, uint64_t *out, void *stream);
cf_status cf_set_failures(cf_set *set, uint64_t *out, void *stream);

/* One filter's table in the layout of cf_export (nbytes must equal
 * cf_table_bytes of its params); import recounts that filter and clears its
 * failures.  Stream-ordered. */
cf_status cf_set_export(cf_set *set, uint32_t fid, void *dst, uint64_t nbytes, void *stream);
cf_status cf_set_import(cf_set *set, uint32_t fid, const void *src, uint64_t nbytes,
                        void *stream);

/* The dropped-tag log of one filter (as cf_lost).  Synchronous. */
cf_status cf_set_lost(cf_set *set, uint32_t fid, uint64_t *buckets, uint32_t *tags,
                      uint64_t cap, uint64_t *n_out);

/* Launch shape: read, or set (graphs created earlier keep their shape).
 * Setting a shape synchronises the device and clears the persistent form's
 * control block (and with it a recorded error, see cf_set_status).  Errors:
 * CF_EINVAL (a field out of range, or more blocks per compute unit than
 * fit), CF_EUNSUPPORTED (persistent on a set whose filters differ in f, hash
 * or placement). */
cf_status cf_set_get_shape(const cf_set *set, cf_set_shape *out);
cf_status cf_set_set_shape(cf_set *set, const cf_set_shape *shape);

/* Largest blocks_per_cu the persistent form takes with `block` threads per
 * block on this set's device (0 if the set cannot run it): the blocks that
 * are resident at once, measured.  The occupancy the runtime reports from the
 * kernel's resources can exceed what the device places together, so on the
 * first call per kernel an empty persistent batch (barriers only, each wait
 * bounded by 50 ms) runs with that count and then one fewer at a time until
 * its barriers complete; the result is kept for the process.  Synchronous
 * on that first call; set-up only.  Two persistent batches in flight at once
 * on one device (of any sets) may not all be resident: order them. */
uint32_t cf_set_persistent_capacity(cf_set *set, uint32_t block);

/* The persistent form's grid barriers wait for at most a bounded time
 * (10 s; the environment variable CF_SET_BARRIER_US, read at cf_set_create,
 * sets it in microseconds).  A barrier that waits longer -- blocks not all
 * resident at once, which the cooperative launch is there to rule out --
 * abandons its batch: every block leaves the kernel without touching the
 * batch further, results are undefined, and later persistent batches return
 * at once without running until the error is cleared by cf_set_set_shape.
 * *error_out = 1 if that happened, else 0.  Synchronises the device. */
cf_status cf_set_status(cf_set *set, uint32_t *error_out);

/* Where the last persistent batch run on this set spent its time: ticks[0]
 * is the wall-clock tick when its first block started, ticks[1..3] the ticks
 * when its three grid barriers completed (after the partition, the queries
 * and the deletes); the inserts ran from ticks[3] to the kernel's end.
 * *ticks_per_s (nullable) receives the clock's rate.  Values are those of
 * the last batch that reached each point (zero before any).  Synchronises
 * the device.  CF_EUNSUPPORTED if the set cannot run the persistent form. */
cf_status cf_set_phase_ticks(cf_set *set, uint64_t ticks[4], uint64_t *ticks_per_s);

#ifdef __cplusplus
}
#endif
#endif /* CF_SET_H */
