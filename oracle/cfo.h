/*
 * cfo.h -- plain sequential CPU oracle for the partial-key cuckoo filter.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the GPU library.
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline leg may load it.  It shares no code, header, table or constant
 * generator with the GPU library, and the GPU library never calls it.
 *
 * What it computes (Cuckoo-GPU, arXiv 2603.15486):
 *   - derived values fp, i1, i2 of a key: Sec. 2.1 Eqs. (1)-(3) and Sec. 4.3
 *     step 1 (upper 32 hash bits -> fingerprint, lower 32 bits -> bucket);
 *   - the packed bucket layout of Sec. 4.2 / Fig. 2 (slot k of a 64-bit word
 *     at bits [k*f, (k+1)*f));
 *   - Insert with direct attempt and bounded eviction (Alg. 1, Sec. 4.3),
 *     with either the greedy random-walk (DFS) chain of Alg. 1 or the
 *     breadth-first heuristic of Sec. 4.6.1;
 *   - Contains (Alg. 2, Sec. 4.4) and Remove (Alg. 3, Sec. 4.5);
 *   - both bucket placement policies: XOR (Eq. (3)) and the offset policy
 *     with a choice bit (Sec. 4.6.2).
 *
 * Everything is done one slot at a time with plain loops: no SWAR, no
 * blocking, no concurrency.  Readings taken where the paper is silent are
 * listed at the top of cfo.c.
 */
#ifndef CFO_H
#define CFO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CFO_HASH_FMIX64 = 0, CFO_HASH_XXH64 = 1 };
enum { CFO_EVICT_BFS = 0, CFO_EVICT_DFS = 1 };
enum { CFO_PLACE_XOR = 0, CFO_PLACE_OFFSET = 1 };

typedef struct cfo_filter cfo_filter;

/* Hash functions, exposed so tests can pin them against known answers. */
uint64_t cfo_fmix64(uint64_t x);            /* MurmurHash3 64-bit finalizer   */
uint64_t cfo_xxh64_u64(uint64_t x);         /* xxHash64 of 8 LE bytes, seed 0 */
uint64_t cfo_hash(uint32_t kind, uint64_t x);
/* Counter-based generator: k-th output (k >= 0) of SplitMix64 started at
 * state s.  Used for the eviction policies' random choices. */
uint64_t cfo_splitmix64_at(uint64_t s, uint64_t k);

/* Create an empty filter.  m must be a power of two (XOR policy, Sec. 4.6.2),
 * b in {4,8,16,32}, f in {8,16,32}.  Returns NULL on invalid parameters. */
cfo_filter *cfo_create(uint64_t m, uint32_t b, uint32_t f, uint32_t hash_kind,
                       uint32_t evict, uint32_t max_evict, uint64_t seed);
/* The same with a bucket placement policy: CFO_PLACE_XOR (Eq. (3), m a power
 * of two) or CFO_PLACE_OFFSET (Sec. 4.6.2: offset and choice bit, any m in
 * [1, 2^32), fingerprints of f-1 bits). */
cfo_filter *cfo_create_placed(uint64_t m, uint32_t b, uint32_t f, uint32_t hash_kind,
                              uint32_t evict, uint32_t max_evict, uint64_t seed,
                              uint32_t placement);
void cfo_destroy(cfo_filter *flt);

/* Derived values of a key (Eqs. (1)-(3); Sec. 4.6.2 for the offset policy).
 * cfo_derive gives the tag as written in i1; cfo_derive_tags also the tag as
 * written in i2 (the same under XOR; with the choice bit set under offset). */
void cfo_derive(const cfo_filter *flt, uint64_t key, uint32_t *fp,
                uint64_t *i1, uint64_t *i2);
void cfo_derive_tags(const cfo_filter *flt, uint64_t key, uint32_t *t1, uint32_t *t2,
                     uint64_t *i1, uint64_t *i2);
/* Other bucket of a tag stored in `bucket`; cfo_move also gives the tag as
 * it is written there. */
uint64_t cfo_alt(const cfo_filter *flt, uint64_t bucket, uint32_t tag);
uint64_t cfo_move(const cfo_filter *flt, uint64_t bucket, uint32_t tag, uint32_t *tag_out);

/* Memory traffic of the operations so far, as the algorithm's steps define
 * it: bucket reads (one per bucket a step inspects) and word writes (one per
 * slot a step stores).  Counting only; used for algorithmic-byte figures. */
void cfo_io_counts(const cfo_filter *flt, uint64_t *reads, uint64_t *writes);
void cfo_io_reset(cfo_filter *flt);

/* Single-key operations.  Return 1 on success, 0 on failure. */
int cfo_insert(cfo_filter *flt, uint64_t key, uint32_t *kicks_out);
int cfo_query(const cfo_filter *flt, uint64_t key);
int cfo_delete(cfo_filter *flt, uint64_t key);

/* Batch wrappers: a plain loop over the keys in index order.
 * ok/kicks/found may be NULL where noted. */
void cfo_insert_batch(cfo_filter *flt, const uint64_t *keys, uint64_t n,
                      uint8_t *ok /*nullable*/, uint32_t *kicks /*nullable*/);
void cfo_query_batch(const cfo_filter *flt, const uint64_t *keys, uint64_t n,
                     uint8_t *found);
void cfo_delete_batch(cfo_filter *flt, const uint64_t *keys, uint64_t n,
                      uint8_t *ok /*nullable*/);

/* Slot access by (bucket, slot), and raw table words. */
uint32_t cfo_get_slot(const cfo_filter *flt, uint64_t bucket, uint32_t slot);
uint64_t cfo_num_words(const cfo_filter *flt);
const uint64_t *cfo_words(const cfo_filter *flt);
/* Replace the table with the given words; the count is recomputed. */
void cfo_load_words(cfo_filter *flt, const uint64_t *words, uint64_t nwords);

uint64_t cfo_count(const cfo_filter *flt);      /* non-empty slots     */
uint64_t cfo_failures(const cfo_filter *flt);   /* failed inserts      */
uint64_t cfo_lost_count(const cfo_filter *flt); /* == failures         */
/* Copy up to cap dropped (bucket, tag) pairs; returns the number copied. */
uint64_t cfo_lost(const cfo_filter *flt, uint64_t *buckets, uint32_t *tags,
                  uint64_t cap);

/* Batch forms of cfo_derive, for checkers: fp[i], i1[i], i2[i] of keys[i]. */
void cfo_derive_batch(const cfo_filter *flt, const uint64_t *keys, uint64_t n,
                      uint32_t *fp, uint64_t *i1, uint64_t *i2);

/* The stored multiset as (low bucket of the pair, high bucket, tag) triples
 * -- under the offset policy (primary, alternate, fingerprint without the
 * choice bit) -- one per non-empty slot, in slot order.  Arrays must hold
 * count() entries; returns the number written. */
uint64_t cfo_stored_groups(const cfo_filter *flt, uint64_t *lo, uint64_t *hi,
                           uint32_t *tag, uint64_t cap);
/* The group each key's tag joins (the triple cfo_stored_groups reports for
 * it once stored). */
uint64_t cfo_key_groups(const cfo_filter *flt, const uint64_t *keys, uint64_t n,
                        uint64_t *lo, uint64_t *hi, uint32_t *tag);
/* The group of each explicit (bucket, tag) pair, e.g. the dropped-tag log. */
uint64_t cfo_pair_groups(const cfo_filter *flt, const uint64_t *buckets, const uint32_t *tags,
                         uint64_t n, uint64_t *lo, uint64_t *hi, uint32_t *tag);

/* Order-independent 64-bit digest of a multiset of (low bucket, high bucket,
 * tag) triples: the wrapping sum of a mixed value per triple.  Equal
 * multisets give equal digests; different ones collide with probability
 * about 2^-64.  _keys digests the pairs of the given keys, _table the stored
 * slots of buckets [j0, j1). */
uint64_t cfo_group_digest_keys(const cfo_filter *flt, const uint64_t *keys, uint64_t n);
uint64_t cfo_group_digest_table(const cfo_filter *flt, uint64_t j0, uint64_t j1);
/* Digest of explicit (bucket, tag) pairs, e.g. the dropped-tag log. */
uint64_t cfo_group_digest_pairs(const cfo_filter *flt, const uint64_t *buckets,
                                const uint32_t *tags, uint64_t n);
/* Replace the table words without recounting (for very large tables whose
 * count the caller checks separately). */
void cfo_load_words_nocount(cfo_filter *flt, const uint64_t *words, uint64_t nwords);

/* Table-exact false-positive probability for a uniformly random negative
 * key given the current table (see cfo.c). */
double cfo_table_fpr(const cfo_filter *flt);

#ifdef __cplusplus
}
#endif
#endif /* CFO_H */
