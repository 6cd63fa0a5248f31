/*
 * cf_tune.h -- choosing a filter's geometry and a filter set's launch shape
 * by measurement on the device (part of libcf.so).
 *
 * Geometry.  For the filter of Cuckoo-GPU (arXiv 2603.15486), the
 * fingerprint width f and the bucket size b fix the false-positive rate
 * through Eq. (4) (Sec. 2.1): eps(alpha) ~= 1 - (1 - 2^-f)^(2 b alpha) at load
 * factor alpha, so smaller buckets and wider fingerprints lower it.  The
 * table takes m*b*f/8 bytes, with m a power of two (the XOR placement of
 * Eq. (3), Sec. 4.6.2).  Throughput depends on both through the memory
 * behaviour of the kernels (Sec. 5.3: a larger bucket lets a positive query
 * finish after one transaction; eviction gets harder as b shrinks), and is
 * measured here rather than modelled.  cf_tune_geometry enumerates every
 * compiled (f, b) under both placements and sizes m for the capacity: the
 * smallest power of two under XOR, the exact bucket count under the offset
 * policy of Sec. 4.6.2 (whose fingerprint loses its top bit to the choice
 * bit; its FPR is taken as 1 - (1 - 2^-(f-1))^(b alpha), which the choice
 * bit keeps equal to Eq. (4) to first order).  It keeps the candidates that
 * meet the FPR and memory goals, and ranks them by the mix-weighted time
 * per operation timed on the current device -- times within a tolerance of
 * the fastest count as equal, and the smallest table among them comes
 * first -- or, without measurement, by table bytes, then larger b, smaller
 * f, XOR before offset.
 *
 * Launch shape.  cf_set_tune times one mixed batch of a filter set under
 * candidate launch shapes (cf_set_shape: the class-kernel or the persistent
 * form, chunk, block size and blocks per compute unit) and keeps the
 * fastest.
 *
 * Both calls are for set-up time, not for hot paths: they synchronise the
 * device and allocate device memory for their duration.
 */
#ifndef CF_TUNE_H
#define CF_TUNE_H

#include <stdint.h>

#include "cf.h"
#include "cf_set.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint64_t capacity;       /* keys the filter must hold; > 0                        */
    double max_load;         /* load factor the filter may reach at capacity, in
                                (0, 1]; 0 = 0.95                                       */
    double max_fpr;          /* Eq. (4) at the load reached at capacity must not
                                exceed this; 0 = no limit                              */
    uint64_t max_bytes;      /* table bytes limit; 0 = none                            */
    double mix[3];           /* relative weights of queries, deletes and inserts
                                (CF_OP_* order); all 0 = equal weights                 */
    double positive_share;   /* share of queries for stored keys, in [0, 1]            */
    uint32_t hash;           /* CF_HASH_* of the filter                                */
    uint32_t evict;          /* CF_EVICT_* of the filter                               */
    uint32_t max_evict;      /* eviction bound; 0 = 128 (BFS) or 500 (DFS)             */
    uint32_t measure;        /* 1: time every feasible candidate on the current
                                device; 0: rank by the model alone (host only)         */
    uint64_t probe_bytes;    /* tables larger than this are timed on a probe of at
                                most this size (same per-operation memory
                                behaviour once far beyond the caches); 0 = 1 GiB       */
    uint64_t seed;           /* keys of the probes and seed of the chosen params       */
    uint32_t placements;     /* placements to consider: bit CF_PLACE_XOR, bit
                                CF_PLACE_OFFSET; 0 = both                              */
    uint32_t tie_permille;   /* measured times within this many per mille of the
                                fastest feasible candidate count as equal, and the
                                smallest table among them wins; 0 = 50 (5%)           */
} cf_tune_goal;

typedef struct {
    cf_params params;        /* sized for the goal's capacity                          */
    uint64_t bytes;          /* cf_table_bytes(&params)                                */
    uint64_t probe_buckets;  /* buckets of the table timed (0 if not timed)            */
    double load;             /* capacity / (m * b)                                     */
    double fpr;              /* Eq. (4) at `load` (offset: the form above)             */
    double rate[3];          /* measured operations per second for queries, deletes
                                and inserts at `load` (0 if not timed)                 */
    double ns_per_op;        /* mix-weighted time per operation (0 if not timed)       */
    uint32_t feasible;       /* 1 if it meets max_fpr and max_bytes and, when timed,
                                its probe had no failed insertion                      */
    uint32_t probe_failures; /* insertions that failed while timing                    */
} cf_tune_candidate;

/* Enumerate the compiled geometries for the goal (at most 24 candidates;
 * cands may be NULL to count them), write min(cap, count) of them to cands
 * sorted best first (feasible ones first), *n_out = count, and the best
 * feasible candidate's params to *best (nullable).  With goal->measure = 1,
 * each feasible candidate is filled on the device to its load at capacity
 * minus 2% of its slots, then timed three times -- insert of the next 2% of
 * slots, a query batch of 2^22 keys with the goal's positive share, delete of
 * the same 2% -- and the median rates are kept; probe results are cached per
 * process.  stream: where the probes run (NULL = the default stream).
 * Errors: CF_EINVAL (bad goal, or no candidate is feasible: then cands and
 * *n_out are still written and *best is not), CF_ENOMEM, CF_EDEVICE. */
cf_status cf_tune_geometry(const cf_tune_goal *goal, cf_tune_candidate *cands, uint32_t cap,
                           uint32_t *n_out, cf_params *best, void *stream);

typedef struct {
    cf_set_shape shape;      /* launch shape tried                                     */
    double ms;               /* median time of the batch over the repetitions          */
} cf_set_trial;

/* Most default candidates cf_set_tune tries (the size trials may need). */
#define CF_SET_TUNE_MAX_TRIALS 64

/* cf_set_tune flags: time cf_set_execute calls instead of launches of a
 * graph captured per candidate (cf_set_graph_create). */
#define CF_SET_TUNE_EAGER 1u

/* Time one mixed batch (d_ops, d_fids, d_keys, n: as in cf_set_execute,
 * device memory) under each candidate launch shape, reps times each (0 = 3),
 * and set the fastest as the set's shape (*out, nullable, receives it).
 * Each candidate is timed as the batch will run: by default as launches of
 * a graph captured for it (cf_set_graph_create, the form a batch loop
 * replays); with flags = CF_SET_TUNE_EAGER as cf_set_execute calls.  The
 * two can rank shapes differently: a graph's parallel branches (the class
 * streams) are placed on streams the runtime chooses.
 * shapes[0..nshapes-1]: the candidates, each valid for cf_set_set_shape on
 * this set; shapes = NULL tries the defaults: the class kernels with chunks
 * of 512, 1024, 2048 and 4096 operations, with the class chains on one
 * stream and on the set's current streams, and,
 * when the set can run the persistent form, the same chunks with one launch
 * per phase (fused = 1) and the persistent form with blocks of 256 and 512
 * threads x 1, 2 and the most blocks per compute unit that fit x chunks of
 * 1024, 2048 and 4096; each with the breadth-first search one lane and one
 * wave per key (wave_bfs 0 and 1).  trials (nullable): one entry per
 * candidate tried, at most trials_cap; *ntrials_out (nullable) receives the
 * number of candidates tried.
 *
 * In every execution the batch's insert keys are replaced by fresh keys
 * mixed from them (a different mix each time; queries and deletes keep the
 * batch's keys): an execution that re-inserted the keys the previous undo
 * removed would find their slots just emptied and never run an eviction
 * search, which would favour shapes that are slow at it.
 * Every timed execution is followed by its undo: each insert that stored its
 * key is deleted and each delete that removed a copy is re-inserted, so
 * every filter ends with the multiset of (bucket pair, fingerprint) it
 * started with (queries and deletes see the same answers as before; slots
 * may be placed differently).  The batch itself is not left applied.  If an
 * insertion fails during tuning (a nearly full filter) the failed insertion
 * dropped a fingerprint and the set changed: *failures_out (nullable)
 * receives the number of insertions that failed.  Synchronous; allocates
 * 10n bytes of device memory for its duration.  Errors: those of
 * cf_set_execute and cf_set_set_shape, CF_EINVAL for a bad candidate or no
 * candidate, unknown flags, CF_ENOMEM, CF_EDEVICE if a persistent trial
 * abandoned its batch (cf_set_status). */
cf_status cf_set_tune(cf_set *set, const uint8_t *d_ops, const uint32_t *d_fids,
                      const uint64_t *d_keys, uint64_t n, const cf_set_shape *shapes,
                      uint32_t nshapes, uint32_t reps, uint32_t flags, cf_set_trial *trials,
                      uint32_t trials_cap, uint32_t *ntrials_out, cf_set_shape *out,
                      uint64_t *failures_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CF_TUNE_H */
