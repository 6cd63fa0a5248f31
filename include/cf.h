/*
 * cf.h -- C ABI of the MI355X (gfx950) partial-key cuckoo filter library
 * (libcf.so).
 *
 * The operations are those of Cuckoo-GPU (arXiv 2603.15486): batched
 * insertion with a bounded eviction search (Alg. 1 and Sec. 4.6.1), query
 * (Alg. 2) and deletion (Alg. 3) on a table of m buckets with b slots of
 * f-bit fingerprints, packed into little-endian words as in Sec. 4.2 / Fig. 2.
 * For a key x with 64-bit hash h = H(x), under the XOR placement
 * (CF_PLACE_XOR, the default):
 *     fp = (h >> 32) mod 2^f, replaced by 1 when it is 0 (0 marks EMPTY)
 *     i1 = (h mod 2^32) mod m
 *     i2 = i1 XOR (H(fp) mod m)                          (Sec. 2.1, Eqs. 1-3)
 * so m must be a power of two.  Under the offset placement of Sec. 4.6.2
 * (CF_PLACE_OFFSET) any m in [1, 2^32) is allowed: the fingerprint v has
 * f-1 bits ((h >> 32) mod 2^(f-1), 0 -> 1) and the top bit of each f-bit
 * slot is a choice bit,
 *     i1 = (h mod 2^32) mod m,   offset(v) = 1 + ((H(v) mod 2^32) mod (m-1))
 *     i2 = (i1 + offset(v)) mod m                         (offset(v) = 0 if m = 1)
 * and a tag is written v in i1 and v | 2^(f-1) in i2; moving a tag during an
 * eviction flips the bit.
 *
 * Conventions for every call below:
 *  - Pointers named d_* are device pointers (hipMalloc'd or equivalent) that
 *    the caller owns; they must stay valid until the work enqueued on the
 *    given stream has completed.  Keys are uint64 and 8-byte aligned.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *  - Batch operations only enqueue work and return; results are valid after
 *    the stream is synchronised.  Argument errors are detected before any
 *    work is enqueued and return CF_EINVAL; launch errors return CF_EDEVICE.
 *    cf_last_error() gives a message for the last failing call on the
 *    calling thread.
 *  - One kind of batch operation runs at a time on a filter: a query must
 *    not overlap an insert or delete on the same filter (Sec. 4.4: its
 *    vector loads are not atomic), and inserts must not overlap deletes.
 *    An insert must not overlap another insert on the same filter either:
 *    every insert launch of a filter uses the filter's one eviction queue,
 *    so two in flight at once would read each other's queued keys.  Only
 *    queries may overlap queries (and deletes deletes).  Order calls on
 *    one stream, or synchronise between streams.
 *  - Breaking these rules is not detected and corrupts results: a query
 *    overlapping a write may miss a stored key; a delete clears its slot
 *    with a fetch-AND that relies on no insert running (Alg. 3's CAS would
 *    merely fail), so an insert overlapping a delete can have a slot it
 *    just refilled cleared, silently removing an unrelated fingerprint
 *    (a false negative).
 *  - An insertion failure is not an error: the key's d_ok entry is 0, the
 *    failure counter grows, and the fingerprint that was in flight when the
 *    eviction bound was reached is dropped and logged (Alg. 1: the caller
 *    has to rebuild the filter).
 */
#ifndef CF_H
#define CF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cf_filter cf_filter; /* opaque; owned by the library */

typedef enum {
    CF_OK = 0,
    CF_EINVAL = 1,       /* invalid argument                            */
    CF_ENOMEM = 2,       /* device allocation failed                    */
    CF_EDEVICE = 3,      /* HIP runtime or kernel launch error          */
    CF_EUNSUPPORTED = 4  /* parameters outside the compiled set         */
} cf_status;

enum { CF_HASH_FMIX64 = 0, CF_HASH_XXH64 = 1 };
enum { CF_EVICT_BFS = 0, CF_EVICT_DFS = 1 };
enum { CF_PLACE_XOR = 0, CF_PLACE_OFFSET = 1 };

typedef struct {
    uint64_t num_buckets;      /* m: power of two, 1 <= m <= 2^32                  */
    uint32_t slots_per_bucket; /* b: 4, 8, 16 or 32                                */
    uint32_t fp_bits;          /* f: 8, 16 or 32                                   */
    uint32_t hash;             /* CF_HASH_FMIX64 (MurmurHash3 finalizer) or
                                  CF_HASH_XXH64 (xxHash64, Sec. 4.3 step 1)        */
    uint32_t evict;            /* CF_EVICT_BFS (Sec. 4.6.1) or CF_EVICT_DFS (Alg. 1) */
    uint32_t max_evict;        /* bound D on evict-and-carry steps per insert      */
    uint32_t lost_capacity;    /* entries kept in the dropped-tag log (0: 65536)   */
    uint64_t seed;             /* seed of the eviction policies' random choices    */
    uint32_t placement;        /* CF_PLACE_XOR (Eq. 3) or CF_PLACE_OFFSET (Sec. 4.6.2) */
    uint32_t reserved;         /* 0                                                */
} cf_params;

/* Bytes of the bucket table for these parameters: ceil(m*b*f/64) words of
 * 8 bytes.  Returns 0 for invalid parameters. */
uint64_t cf_table_bytes(const cf_params *params);

/* Allocate an empty filter on the current HIP device (all slots EMPTY = 0).
 * Synchronous.  *out receives the handle; free it with cf_destroy.
 * Errors: CF_EINVAL (NULL; XOR: m not a power of two or > 2^32; offset: m
 * = 0 or >= 2^32; unknown placement), CF_EUNSUPPORTED (b or f outside the
 * compiled set), CF_ENOMEM.
 * Launch shape: 256-thread blocks, at most 1024 blocks per compute unit for
 * queries, deletes and whole-table kernels (one key per thread up to that,
 * then grid-stride) and 128 per compute unit for inserts.  The environment
 * variable CF_GRID_PER_CU (1..1024), read here, sets both caps to that many
 * blocks per compute unit for this filter; results do not depend on it. */
cf_status cf_create(const cf_params *params, cf_filter **out);

/* As cf_create, with the table in caller-owned device memory: d_table
 * (16-byte aligned, on the current device, at least cf_table_bytes(params)
 * bytes) is zeroed and used as the table until cf_destroy, which does not
 * free it.  The library still allocates the small counters and the
 * dropped-tag log.  Lets a caller account for and place the table itself
 * (a memory pool, a tensor).  Synchronous.  Errors: as cf_create, and
 * CF_EINVAL for a NULL, misaligned or too small buffer. */
cf_status cf_create_in(const cf_params *params, void *d_table, uint64_t nbytes,
                       cf_filter **out);

/* Free the filter's device memory (synchronises the device first).
 * NULL is accepted. */
cf_status cf_destroy(cf_filter *flt);

/* Reserve internal scratch for batches of up to max_batch keys so that later
 * inserts of that size do not allocate.  Synchronous. */
cf_status cf_reserve(cf_filter *flt, uint64_t max_batch);

/* Alg. 1 + Sec. 4.6.1: insert n keys.  d_ok (nullable): uint8[n], 1 if the
 * key's fingerprint was stored.  d_kicks (nullable): uint32[n], fingerprints
 * displaced by that key's insertion.  The occupancy count grows by the
 * number of successes.  Keys may repeat (each copy is stored).  The first
 * call with a batch larger than any before it allocates scratch and
 * synchronises the stream (see cf_reserve).  On tables of at most 16 MiB the
 * breadth-first search loads a level's candidates' other buckets in groups
 * (as many as 128 bytes hold) instead of one by one; it picks the same
 * candidate either way. */
cf_status cf_insert(cf_filter *flt, const uint64_t *d_keys, uint64_t n,
                    uint8_t *d_ok, uint32_t *d_kicks, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cf_insert
 * with the same arguments, results and rules, except that the eviction queue
 * is not the filter's own (which cf_insert grows on demand) but a fixed array
 * of CF_NOALLOC_MAX_KEYS uint32 entries (16 MiB) that the library keeps on
 * every GPU it runs on until the process ends.  The call allocates and frees
 * nothing; its first call on a device looks up that device's copy of the
 * array (hipGetSymbolAddress), later calls reuse the address.
 *  - n <= CF_NOALLOC_MAX_KEYS (2^22), else CF_EINVAL.  Also CF_EINVAL if the
 *    filter's launch shape (see CF_GRID_PER_CU) needs more queue entries for
 *    n keys than the array holds; with the default shape every n up to the
 *    limit fits on a GPU of 128 or more compute units.
 *  - Every call on one GPU shares that GPU's array, for any filter: two calls
 *    that overlap in time on one GPU (on different streams, or from different
 *    host threads) race on it and corrupt each other's insertions.  Order
 *    them on one stream, or synchronise between them.
 *  - The array keeps the last call's contents; nothing needs clearing, since
 *    a launch writes every queue entry it reads.
 *  - CF_EDEVICE if the array's address cannot be obtained or the launch
 *    fails. */
#define CF_NOALLOC_MAX_KEYS (1u << 22)
cf_status cf_insert_noalloc(cf_filter *flt, const uint64_t *d_keys, uint64_t n,
                            uint8_t *d_ok, uint32_t *d_kicks, void *stream);

/* Alg. 2: d_found (required): uint8[n], 1 if fp(key) is in bucket i1 or i2.
 * Read-only; false positives occur at the rate of Eq. (4). */
cf_status cf_query(cf_filter *flt, const uint64_t *d_keys, uint64_t n,
                   uint8_t *d_found, void *stream);

/* Alg. 3: remove one copy of fp(key) from bucket i1, else from i2.
 * d_ok (nullable): uint8[n], 1 if a copy was removed.  The occupancy count
 * shrinks by the number of successes.  Deleting a key that was never
 * inserted may remove another key's colliding fingerprint (Sec. 2.1). */
cf_status cf_delete(cf_filter *flt, const uint64_t *d_keys, uint64_t n,
                    uint8_t *d_ok, void *stream);

/* Occupancy (non-empty slots), kept by the hierarchical reduction of
 * Sec. 4.3.  *out may be host or device memory; stream-ordered copy. */
cf_status cf_count(cf_filter *flt, uint64_t *out, void *stream);

/* Number of failed insertions since creation, reset or import.  Host or
 * device *out; stream-ordered copy. */
cf_status cf_failures(cf_filter *flt, uint64_t *out, void *stream);

/* Copy the dropped-tag log: for each failed insertion, the bucket and the
 * fingerprint that was in flight.  Up to `cap` entries are copied into the
 * host arrays buckets[] and tags[]; *n_out receives the number copied, which
 * is less than the failure count only if the log overflowed.  Synchronous. */
cf_status cf_lost(cf_filter *flt, uint64_t *buckets, uint32_t *tags,
                  uint64_t cap, uint64_t *n_out);

/* Copy the raw table (cf_table_bytes bytes, the layout of Fig. 2) to dst,
 * host or device memory; nbytes must equal cf_table_bytes.  Stream-ordered. */
cf_status cf_export(cf_filter *flt, void *dst, uint64_t nbytes, void *stream);

/* Replace the table with nbytes (== cf_table_bytes) from src, host or device
 * memory, recount the occupancy on the device and clear the failure counter
 * and log.  Stream-ordered. */
cf_status cf_import(cf_filter *flt, const void *src, uint64_t nbytes, void *stream);

/* Empty the table and clear all counters.  Stream-ordered. */
cf_status cf_reset(cf_filter *flt, void *stream);

/* Copy of the filter's parameters. */
cf_status cf_get_params(const cf_filter *flt, cf_params *out);

/* Message describing the last failing call on this thread ("" if none). */
const char *cf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CF_H */
