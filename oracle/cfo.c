/*
 * cfo.c -- plain sequential CPU oracle for the partial-key cuckoo filter.
 *
 * TEST INFRASTRUCTURE ONLY: see cfo.h.  Nothing in the GPU library calls,
 * links or includes this file.
 *
 * Source: Cuckoo-GPU (arXiv 2603.15486).  Each function names the passage it
 * follows.  Readings taken where the paper is silent or leaves a choice open:
 *
 *  R1  Hash H: the paper hashes with xxHash64 (Sec. 4.3, step 1).  Both that
 *      and the 64-bit MurmurHash3 finalizer (fmix64) are offered; the caller
 *      picks one.  H(fp) in Eq. (3) hashes the fingerprint zero-extended to
 *      64 bits with the same function.
 *  R2  EMPTY is the all-zero tag (Sec. 4.5); a fingerprint that comes out as
 *      0 is replaced by 1.
 *  R3  i1 = lower 32 hash bits mod m, fp = upper 32 hash bits mod 2^f
 *      (Sec. 4.3, step 1); alt(i, v) = i XOR (H(v) mod m) (Eq. (3)).
 *  R5  Slot k of a 64-bit word occupies bits [k*f, (k+1)*f) (Fig. 2); global
 *      slot g = j*b + s of bucket j lives in word g / (64/f).  When b*f < 64,
 *      several buckets share one word.
 *  R8  Random choices (which bucket starts an eviction chain, which slot is
 *      displaced) come from a counter-based SplitMix64 stream seeded by
 *      (key XOR filter seed); the draw for eviction level n is output n.
 *  R8b BFS (Sec. 4.6.1) inspects b/2 consecutive slots starting at a random
 *      slot; the "last candidate" is the b/2-th of them.
 *  R10 max_evict (D) bounds the number of evict-and-carry steps for both
 *      policies; a kick is one fingerprint displaced from its slot.
 *  R12 When the bound is reached the in-flight tag is dropped, the insert
 *      reports failure and the dropped (bucket, tag) pair is recorded.
 *  R13 Duplicate keys are stored as separate copies (multiset semantics).
 *  R17 Load factor = non-empty slots / (m*b).
 *  R20 Offset placement (Sec. 4.6.2): the fingerprint v has f-1 bits (upper
 *      32 hash bits mod 2^(f-1), 0 -> 1) and the choice bit is the top bit
 *      of the f-bit slot; i1 = lower 32 hash bits mod m, for any m in
 *      [1, 2^32); offset(v) = 1 + (lower 32 bits of H(v)) mod (m-1) for
 *      m >= 2, so that i2 != i1, and 0 for m = 1.  A tag with choice bit 0
 *      sits in its primary bucket i1 and is written v; in i2 it is written
 *      v | choice bit.  Moving a tag flips the bit.
 *  R21 Under the offset policy a stored tag stands for the keys with its
 *      primary bucket and fingerprint: its group is the ordered triple
 *      (primary, alternate, v).  (Under XOR the pair is unordered.)
 */
#include "cfo.h"

#include <stdlib.h>
#include <string.h>

struct cfo_filter {
    uint64_t m;          /* number of buckets (power of two for XOR) */
    uint32_t placement;  /* CFO_PLACE_XOR or CFO_PLACE_OFFSET */
    uint32_t b;          /* slots per bucket                 */
    uint32_t f;          /* fingerprint bits                 */
    uint32_t hash_kind;
    uint32_t evict;
    uint32_t max_evict;
    uint64_t seed;
    uint64_t nwords;
    uint64_t *words;
    uint64_t count;
    uint64_t failures;
    uint64_t lost_n, lost_cap;
    uint64_t *lost_bucket;
    uint32_t *lost_tag;
    uint64_t *io;        /* io[0]: bucket reads, io[1]: word writes (counters
                            only; see cfo_io_counts) */
};

/* ---------------------------------------------------------------- hashes */

/* MurmurHash3's 64-bit finalizer (fmix64), as published with MurmurHash3. */
uint64_t cfo_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

static uint64_t rotl64(uint64_t x, unsigned r)
{
    return (x << r) | (x >> (64u - r));
}

/* xxHash64 (Y. Collet's published specification) of the 8-byte little-endian
 * encoding of x with seed 0: the short-input path (length < 32) processing a
 * single 8-byte lane, then the final avalanche. */
uint64_t cfo_xxh64_u64(uint64_t x)
{
    const uint64_t P1 = 0x9E3779B185EBCA87ULL;
    const uint64_t P2 = 0xC2B2AE3D27D4EB4FULL;
    const uint64_t P3 = 0x165667B19E3779F9ULL;
    const uint64_t P4 = 0x85EBCA77C2B2AE63ULL;
    const uint64_t P5 = 0x27D4EB2F165667C5ULL;
    uint64_t acc = 0 /* seed */ + P5;
    acc += 8; /* input length in bytes */
    uint64_t lane = rotl64(x * P2, 31) * P1; /* round(0, x) */
    acc ^= lane;
    acc = rotl64(acc, 27) * P1 + P4;
    acc ^= acc >> 33;
    acc *= P2;
    acc ^= acc >> 29;
    acc *= P3;
    acc ^= acc >> 32;
    return acc;
}

uint64_t cfo_hash(uint32_t kind, uint64_t x)
{
    return kind == CFO_HASH_XXH64 ? cfo_xxh64_u64(x) : cfo_fmix64(x);
}

/* SplitMix64 (Steele, Lea, Flood 2014): state advances by the golden gamma,
 * output is the state passed through the mixing function.  Output k of the
 * stream that starts at state s is mix(s + (k+1)*gamma). */
uint64_t cfo_splitmix64_at(uint64_t s, uint64_t k)
{
    uint64_t z = s + (k + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------- creation */

static int is_pow2(uint64_t x) { return x != 0 && (x & (x - 1)) == 0; }

cfo_filter *cfo_create(uint64_t m, uint32_t b, uint32_t f, uint32_t hash_kind,
                       uint32_t evict, uint32_t max_evict, uint64_t seed)
{
    return cfo_create_placed(m, b, f, hash_kind, evict, max_evict, seed, CFO_PLACE_XOR);
}

cfo_filter *cfo_create_placed(uint64_t m, uint32_t b, uint32_t f, uint32_t hash_kind,
                              uint32_t evict, uint32_t max_evict, uint64_t seed,
                              uint32_t placement)
{
    if (placement == CFO_PLACE_XOR) {
        if (!is_pow2(m) || m > (1ULL << 32)) return NULL;
    } else if (placement == CFO_PLACE_OFFSET) {
        if (m == 0 || m >= (1ULL << 32)) return NULL;
    } else {
        return NULL;
    }
    if (!(b == 4 || b == 8 || b == 16 || b == 32)) return NULL;
    if (!(f == 8 || f == 16 || f == 32)) return NULL;
    if (hash_kind > CFO_HASH_XXH64 || evict > CFO_EVICT_DFS) return NULL;
    cfo_filter *flt = (cfo_filter *)calloc(1, sizeof(*flt));
    if (!flt) return NULL;
    flt->m = m; flt->b = b; flt->f = f; flt->placement = placement;
    flt->hash_kind = hash_kind; flt->evict = evict;
    flt->max_evict = max_evict; flt->seed = seed;
    uint64_t bits = m * (uint64_t)b * f;
    flt->nwords = (bits + 63) / 64;
    flt->words = (uint64_t *)calloc(flt->nwords, sizeof(uint64_t));
    flt->io = (uint64_t *)calloc(2, sizeof(uint64_t));
    if (!flt->words || !flt->io) { free(flt->words); free(flt->io); free(flt); return NULL; }
    return flt;
}

void cfo_destroy(cfo_filter *flt)
{
    if (!flt) return;
    free(flt->words);
    free(flt->io);
    free(flt->lost_bucket);
    free(flt->lost_tag);
    free(flt);
}

/* --------------------------------------------------------- derived values */

static uint32_t tag_mask(const cfo_filter *flt)
{
    return flt->f == 32 ? 0xffffffffu : ((1u << flt->f) - 1u);
}

/* The choice bit of the offset policy (R20): the top bit of a slot. */
static uint32_t choice_bit(const cfo_filter *flt)
{
    return 1u << (flt->f - 1);
}

/* offset(v) of Sec. 4.6.2 (R20). */
static uint64_t offset_of(const cfo_filter *flt, uint32_t v)
{
    if (flt->m < 2) return 0;
    uint64_t h = cfo_hash(flt->hash_kind, (uint64_t)v) & 0xffffffffULL;
    return 1 + h % (flt->m - 1);
}

/* Sec. 2.1 Eqs. (1)-(3) with the split of Sec. 4.3 step 1 (R1-R3); under
 * the offset policy, Sec. 4.6.2 (R20).  t1 and t2 are the tag as written in
 * i1 and in i2 (equal under XOR). */
void cfo_derive_tags(const cfo_filter *flt, uint64_t key, uint32_t *t1, uint32_t *t2,
                     uint64_t *i1, uint64_t *i2)
{
    uint64_t h = cfo_hash(flt->hash_kind, key);
    uint64_t lo = h & 0xffffffffULL;
    if (flt->placement == CFO_PLACE_OFFSET) {
        uint32_t v = (uint32_t)(h >> 32) & (choice_bit(flt) - 1u);
        if (v == 0) v = 1;
        uint64_t p = lo % flt->m;
        *t1 = v;
        *t2 = v | choice_bit(flt);
        *i1 = p;
        *i2 = (p + offset_of(flt, v)) % flt->m;
        return;
    }
    uint32_t v = (uint32_t)(h >> 32) & tag_mask(flt);
    if (v == 0) v = 1;
    *t1 = *t2 = v;
    *i1 = lo & (flt->m - 1);
    *i2 = cfo_alt(flt, *i1, v);
}

void cfo_derive(const cfo_filter *flt, uint64_t key, uint32_t *fp,
                uint64_t *i1, uint64_t *i2)
{
    uint32_t t2;
    cfo_derive_tags(flt, key, fp, &t2, i1, i2);
}

/* Where a tag goes when it is moved out of `bucket`, and how it is written
 * there: Eq. (3) under XOR (the tag is unchanged); under the offset policy
 * the two equations of Sec. 4.6.2, with the choice bit flipped. */
uint64_t cfo_move(const cfo_filter *flt, uint64_t bucket, uint32_t tag, uint32_t *tag_out)
{
    if (flt->placement == CFO_PLACE_OFFSET) {
        uint32_t cb = choice_bit(flt);
        uint64_t off = offset_of(flt, tag & ~cb);
        if (tag & cb) {
            *tag_out = tag & ~cb;
            return (bucket + flt->m - off) % flt->m;
        }
        *tag_out = tag | cb;
        return (bucket + off) % flt->m;
    }
    *tag_out = tag;
    return bucket ^ (cfo_hash(flt->hash_kind, (uint64_t)tag) & (flt->m - 1));
}

uint64_t cfo_alt(const cfo_filter *flt, uint64_t bucket, uint32_t tag)
{
    uint32_t t;
    return cfo_move(flt, bucket, tag, &t);
}

/* The group of a tag v stored in bucket j (R21): (low, high, v) of its
 * unordered bucket pair under XOR; (primary, alternate, v without the
 * choice bit) under the offset policy. */
static void group_of(const cfo_filter *flt, uint64_t j, uint32_t v, uint64_t *lo,
                     uint64_t *hi, uint32_t *t)
{
    uint32_t moved;
    uint64_t a = cfo_move(flt, j, v, &moved);
    if (flt->placement == CFO_PLACE_OFFSET) {
        int in_alt = (v & choice_bit(flt)) != 0;
        *lo = in_alt ? a : j;
        *hi = in_alt ? j : a;
        *t = v & ~choice_bit(flt);
        return;
    }
    *lo = j < a ? j : a;
    *hi = j < a ? a : j;
    *t = v;
}

/* The group a key's tag joins (the same triple as group_of gives for it). */
static void key_group(const cfo_filter *flt, uint64_t key, uint64_t *lo, uint64_t *hi,
                      uint32_t *t)
{
    uint32_t t1, t2;
    uint64_t i1, i2;
    cfo_derive_tags(flt, key, &t1, &t2, &i1, &i2);
    group_of(flt, i1, t1, lo, hi, t);
}

/* -------------------------------------------------------- slot storage */

/* Sec. 4.2 / Fig. 2 (R5): slot s of bucket j is global slot j*b+s. */
uint32_t cfo_get_slot(const cfo_filter *flt, uint64_t bucket, uint32_t slot)
{
    uint64_t g = bucket * flt->b + slot;
    uint64_t per_word = 64 / flt->f;
    uint64_t w = flt->words[g / per_word];
    unsigned shift = (unsigned)((g % per_word) * flt->f);
    return (uint32_t)((w >> shift) & tag_mask(flt));
}

static void set_slot(cfo_filter *flt, uint64_t bucket, uint32_t slot,
                     uint32_t tag)
{
    uint64_t g = bucket * flt->b + slot;
    uint64_t per_word = 64 / flt->f;
    unsigned shift = (unsigned)((g % per_word) * flt->f);
    uint64_t field = (uint64_t)tag_mask(flt) << shift;
    uint64_t *w = &flt->words[g / per_word];
    *w = (*w & ~field) | ((uint64_t)tag << shift);
}

/* Scan order of a bucket for tag v (Alg. 1 TryInsert, Alg. 3 TryRemove):
 * words start, start+1, ... wrapping, with start = (v mod b) / tagsPerWord;
 * within a word, slots from low bits to high bits.  Position p of the scan
 * (0 <= p < b) maps to slot scan_slot(flt, v, p). */
static uint32_t scan_slot(const cfo_filter *flt, uint32_t v, uint32_t p)
{
    uint32_t tpw = 64 / flt->f;               /* tags per word */
    if (tpw > flt->b) tpw = flt->b;           /* bucket smaller than a word */
    uint32_t wpb = flt->b / tpw;              /* words per bucket */
    uint32_t start = (v % flt->b) / tpw;
    uint32_t w = (start + p / tpw) % wpb;
    return w * tpw + p % tpw;
}

/* Memory traffic of the algorithm's steps, counted for the roofline's
 * algorithmic bytes (it changes no result): one bucket read per bucket a step
 * inspects (TryInsert, Find, TryRemove, the current bucket of an eviction
 * level), one word write per slot a step stores (a claimed, cleared, swapped
 * or replaced slot: one 64-bit CAS or fetch-AND on a GPU). */
static void count_read(const cfo_filter *flt) { flt->io[0]++; }
static void count_write(const cfo_filter *flt) { flt->io[1]++; }

/* Alg. 1 TryInsert: first empty slot in scan order gets the tag. */
static int try_insert(cfo_filter *flt, uint64_t bucket, uint32_t tag)
{
    count_read(flt);
    for (uint32_t p = 0; p < flt->b; p++) {
        uint32_t s = scan_slot(flt, tag, p);
        if (cfo_get_slot(flt, bucket, s) == 0) {
            set_slot(flt, bucket, s, tag);
            count_write(flt);
            return 1;
        }
    }
    return 0;
}

/* Alg. 2 Find: does the bucket hold the tag in any slot? */
static int find(const cfo_filter *flt, uint64_t bucket, uint32_t tag)
{
    count_read(flt);
    for (uint32_t s = 0; s < flt->b; s++)
        if (cfo_get_slot(flt, bucket, s) == tag) return 1;
    return 0;
}

/* Alg. 3 TryRemove: first slot in scan order holding the tag is cleared. */
static int try_remove(cfo_filter *flt, uint64_t bucket, uint32_t tag)
{
    count_read(flt);
    for (uint32_t p = 0; p < flt->b; p++) {
        uint32_t s = scan_slot(flt, tag, p);
        if (cfo_get_slot(flt, bucket, s) == tag) {
            set_slot(flt, bucket, s, 0);
            count_write(flt);
            return 1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------ insertion */

static void record_lost(cfo_filter *flt, uint64_t bucket, uint32_t tag)
{
    if (flt->lost_n == flt->lost_cap) {
        uint64_t cap = flt->lost_cap ? 2 * flt->lost_cap : 64;
        uint64_t *nb = (uint64_t *)realloc(flt->lost_bucket, cap * sizeof(uint64_t));
        if (nb) flt->lost_bucket = nb;
        uint32_t *nt = (uint32_t *)realloc(flt->lost_tag, cap * sizeof(uint32_t));
        if (nt) flt->lost_tag = nt;
        if (!nb || !nt) { flt->lost_n++; return; }  /* out of memory: count only */
        flt->lost_cap = cap;
    }
    flt->lost_bucket[flt->lost_n] = bucket;
    flt->lost_tag[flt->lost_n] = tag;
    flt->lost_n++;
}

/* Random draw number n for the insert of `key` (R8). */
static uint64_t draw(const cfo_filter *flt, uint64_t key, uint64_t n)
{
    return cfo_splitmix64_at(key ^ flt->seed, n);
}

/* Alg. 1 eviction chain (greedy random walk): displace a random slot of the
 * current bucket, carry the displaced tag to its other bucket, try there. */
static int evict_dfs(cfo_filter *flt, uint64_t key, uint64_t cur, uint32_t tag,
                     uint32_t *kicks)
{
    for (uint32_t n = 1; n <= flt->max_evict; n++) {
        uint32_t s = (uint32_t)(draw(flt, key, n) % flt->b);
        uint32_t evicted = cfo_get_slot(flt, cur, s);
        set_slot(flt, cur, s, tag);
        count_read(flt);
        count_write(flt);
        cur = cfo_move(flt, cur, evicted, &tag);
        (*kicks)++;
        if (try_insert(flt, cur, tag)) return 1;
    }
    record_lost(flt, cur, tag);
    return 0;
}

/* Sec. 4.6.1 breadth-first heuristic: look at half the slots of the current
 * bucket; if one of them can move to an empty slot of its other bucket, move
 * it and take its place.  Otherwise displace the last one inspected, carry it
 * to its other bucket and search again from there. */
static int evict_bfs(cfo_filter *flt, uint64_t key, uint64_t cur, uint32_t tag,
                     uint32_t *kicks)
{
    uint32_t half = flt->b / 2;
    for (uint32_t n = 1; n <= flt->max_evict; n++) {
        uint32_t r0 = (uint32_t)(draw(flt, key, n) % flt->b);
        count_read(flt);  /* the current bucket's candidates */
        for (uint32_t j = 0; j < half; j++) {
            uint32_t s = (r0 + j) % flt->b;
            uint32_t c = cfo_get_slot(flt, cur, s), moved;
            uint64_t a = cfo_move(flt, cur, c, &moved);
            if (a != cur && try_insert(flt, a, moved)) {
                set_slot(flt, cur, s, tag);
                count_write(flt);
                (*kicks)++;
                return 1;
            }
        }
        uint32_t s_last = (r0 + half - 1) % flt->b;
        uint32_t evicted = cfo_get_slot(flt, cur, s_last);
        set_slot(flt, cur, s_last, tag);
        count_write(flt);
        cur = cfo_move(flt, cur, evicted, &tag);
        (*kicks)++;
        if (try_insert(flt, cur, tag)) return 1;
    }
    record_lost(flt, cur, tag);
    return 0;
}

/* Bucket reads and word writes counted since creation or the last reset. */
void cfo_io_counts(const cfo_filter *flt, uint64_t *reads, uint64_t *writes)
{
    *reads = flt->io[0];
    *writes = flt->io[1];
}

void cfo_io_reset(cfo_filter *flt)
{
    flt->io[0] = flt->io[1] = 0;
}

/* Alg. 1 Insert. */
int cfo_insert(cfo_filter *flt, uint64_t key, uint32_t *kicks_out)
{
    uint32_t t1, t2, kicks = 0;
    uint64_t i1, i2;
    int ok;
    cfo_derive_tags(flt, key, &t1, &t2, &i1, &i2);
    if (try_insert(flt, i1, t1) || try_insert(flt, i2, t2)) {
        ok = 1;
    } else {
        int second = (draw(flt, key, 0) & 1) != 0;
        uint64_t cur = second ? i2 : i1;
        uint32_t tag = second ? t2 : t1;
        if (flt->evict == CFO_EVICT_DFS)
            ok = evict_dfs(flt, key, cur, tag, &kicks);
        else
            ok = evict_bfs(flt, key, cur, tag, &kicks);
    }
    if (ok) flt->count++;
    else flt->failures++;
    if (kicks_out) *kicks_out = kicks;
    return ok;
}

/* Alg. 2 Contains. */
int cfo_query(const cfo_filter *flt, uint64_t key)
{
    uint32_t t1, t2;
    uint64_t i1, i2;
    cfo_derive_tags(flt, key, &t1, &t2, &i1, &i2);
    return find(flt, i1, t1) || find(flt, i2, t2);
}

/* Alg. 3 Remove. */
int cfo_delete(cfo_filter *flt, uint64_t key)
{
    uint32_t t1, t2;
    uint64_t i1, i2;
    cfo_derive_tags(flt, key, &t1, &t2, &i1, &i2);
    int ok = try_remove(flt, i1, t1) || try_remove(flt, i2, t2);
    if (ok) flt->count--;
    return ok;
}

/* ------------------------------------------------------------- batches */

void cfo_insert_batch(cfo_filter *flt, const uint64_t *keys, uint64_t n,
                      uint8_t *ok, uint32_t *kicks)
{
    for (uint64_t i = 0; i < n; i++) {
        uint32_t k = 0;
        int r = cfo_insert(flt, keys[i], &k);
        if (ok) ok[i] = (uint8_t)r;
        if (kicks) kicks[i] = k;
    }
}

void cfo_query_batch(const cfo_filter *flt, const uint64_t *keys, uint64_t n,
                     uint8_t *found)
{
    for (uint64_t i = 0; i < n; i++) found[i] = (uint8_t)cfo_query(flt, keys[i]);
}

void cfo_delete_batch(cfo_filter *flt, const uint64_t *keys, uint64_t n,
                      uint8_t *ok)
{
    for (uint64_t i = 0; i < n; i++) {
        int r = cfo_delete(flt, keys[i]);
        if (ok) ok[i] = (uint8_t)r;
    }
}

/* ------------------------------------------------------------ accessors */

uint64_t cfo_num_words(const cfo_filter *flt) { return flt->nwords; }
const uint64_t *cfo_words(const cfo_filter *flt) { return flt->words; }

void cfo_load_words(cfo_filter *flt, const uint64_t *words, uint64_t nwords)
{
    uint64_t n = nwords < flt->nwords ? nwords : flt->nwords;
    memcpy(flt->words, words, n * sizeof(uint64_t));
    uint64_t c = 0;
    for (uint64_t j = 0; j < flt->m; j++)
        for (uint32_t s = 0; s < flt->b; s++)
            c += cfo_get_slot(flt, j, s) != 0;
    flt->count = c;
}

uint64_t cfo_count(const cfo_filter *flt) { return flt->count; }
uint64_t cfo_failures(const cfo_filter *flt) { return flt->failures; }
uint64_t cfo_lost_count(const cfo_filter *flt) { return flt->lost_n; }

uint64_t cfo_lost(const cfo_filter *flt, uint64_t *buckets, uint32_t *tags,
                  uint64_t cap)
{
    uint64_t n = flt->lost_n < flt->lost_cap ? flt->lost_n : flt->lost_cap;
    if (n > cap) n = cap;
    for (uint64_t i = 0; i < n; i++) {
        buckets[i] = flt->lost_bucket[i];
        tags[i] = flt->lost_tag[i];
    }
    return n;
}

void cfo_derive_batch(const cfo_filter *flt, const uint64_t *keys, uint64_t n,
                      uint32_t *fp, uint64_t *i1, uint64_t *i2)
{
    for (uint64_t i = 0; i < n; i++) cfo_derive(flt, keys[i], &fp[i], &i1[i], &i2[i]);
}

/* Each stored tag v in bucket j belongs to the bucket pair {j, alt(j, v)}
 * (Eq. (3) is an involution), which identifies the keys it can stand for;
 * under the offset policy, to its ordered (primary, alternate) pair (R21). */
uint64_t cfo_stored_groups(const cfo_filter *flt, uint64_t *lo, uint64_t *hi,
                           uint32_t *tag, uint64_t cap)
{
    uint64_t n = 0;
    for (uint64_t j = 0; j < flt->m; j++)
        for (uint32_t s = 0; s < flt->b; s++) {
            uint32_t v = cfo_get_slot(flt, j, s);
            if (v == 0) continue;
            if (n == cap) return n;
            group_of(flt, j, v, &lo[n], &hi[n], &tag[n]);
            n++;
        }
    return n;
}

uint64_t cfo_key_groups(const cfo_filter *flt, const uint64_t *keys, uint64_t n,
                        uint64_t *lo, uint64_t *hi, uint32_t *tag)
{
    for (uint64_t i = 0; i < n; i++) key_group(flt, keys[i], &lo[i], &hi[i], &tag[i]);
    return n;
}

uint64_t cfo_pair_groups(const cfo_filter *flt, const uint64_t *buckets, const uint32_t *tags,
                         uint64_t n, uint64_t *lo, uint64_t *hi, uint32_t *tag)
{
    for (uint64_t i = 0; i < n; i++) group_of(flt, buckets[i], tags[i], &lo[i], &hi[i], &tag[i]);
    return n;
}

static uint64_t group_mix(uint64_t lo, uint64_t hi, uint32_t tag)
{
    uint64_t z = cfo_splitmix64_at(tag, 0);
    z = cfo_splitmix64_at(hi ^ z, 0);
    return cfo_splitmix64_at(lo ^ z, 0);
}

uint64_t cfo_group_digest_keys(const cfo_filter *flt, const uint64_t *keys, uint64_t n)
{
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t lo, hi;
        uint32_t t;
        key_group(flt, keys[i], &lo, &hi, &t);
        acc += group_mix(lo, hi, t);
    }
    return acc;
}

uint64_t cfo_group_digest_table(const cfo_filter *flt, uint64_t j0, uint64_t j1)
{
    uint64_t acc = 0;
    if (j1 > flt->m) j1 = flt->m;
    for (uint64_t j = j0; j < j1; j++)
        for (uint32_t s = 0; s < flt->b; s++) {
            uint32_t v = cfo_get_slot(flt, j, s);
            if (v == 0) continue;
            uint64_t lo, hi;
            uint32_t t;
            group_of(flt, j, v, &lo, &hi, &t);
            acc += group_mix(lo, hi, t);
        }
    return acc;
}

uint64_t cfo_group_digest_pairs(const cfo_filter *flt, const uint64_t *buckets,
                                const uint32_t *tags, uint64_t n)
{
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t lo, hi;
        uint32_t t;
        group_of(flt, buckets[i], tags[i], &lo, &hi, &t);
        acc += group_mix(lo, hi, t);
    }
    return acc;
}

void cfo_load_words_nocount(cfo_filter *flt, const uint64_t *words, uint64_t nwords)
{
    uint64_t n = nwords < flt->nwords ? nwords : flt->nwords;
    memcpy(flt->words, words, n * sizeof(uint64_t));
}

/* ------------------------------------------------------------------ FPR */

typedef struct { uint64_t bucket; uint32_t tag; } pair_t;

static int pair_cmp(const void *pa, const void *pb)
{
    const pair_t *a = (const pair_t *)pa, *b = (const pair_t *)pb;
    if (a->bucket != b->bucket) return a->bucket < b->bucket ? -1 : 1;
    if (a->tag != b->tag) return a->tag < b->tag ? -1 : 1;
    return 0;
}

static double table_fpr_offset(const cfo_filter *flt)
{
    uint64_t cap = flt->count + 1, n = 0;
    pair_t *u = (pair_t *)malloc(cap * sizeof(pair_t));
    if (!u) return -1.0;
    for (uint64_t j = 0; j < flt->m; j++)
        for (uint32_t s = 0; s < flt->b; s++) {
            uint32_t v = cfo_get_slot(flt, j, s);
            if (v == 0 || n + 1 > cap) continue;
            uint64_t lo, hi;
            uint32_t t;
            group_of(flt, j, v, &lo, &hi, &t);
            u[n].bucket = lo; u[n].tag = t; n++;
        }
    qsort(u, n, sizeof(pair_t), pair_cmp);
    double unit = 1.0;
    for (uint32_t i = 0; i + 1 < flt->f; i++) unit *= 0.5;
    double total = 0.0;
    for (uint64_t i = 0; i < n; i++) {
        if (i > 0 && pair_cmp(&u[i], &u[i - 1]) == 0) continue;
        total += u[i].tag == 1 ? 2.0 * unit : unit;
    }
    free(u);
    return total / (double)flt->m;
}

/* A negative key y is reported present iff fp(y) sits in i1(y) or in
 * i2(y) = alt(i1(y), fp(y)) (Alg. 2).  With i1 uniform over the m buckets
 * and fp distributed as P(v) (1/2^f each, 2/2^f for v = 1 because 0 is
 * remapped to 1), the probability is (1/m) * sum over the set
 * U = {(j, v), (alt(j, v), v) : v stored in bucket j} of P(v).
 * Under the offset policy y is present iff some stored tag has y's group
 * (primary i1(y), fingerprint v(y)), so U is the set of (primary, v) of the
 * stored tags and P(v) uses 2^(f-1); i1 = lower 32 bits mod m is uniform up
 * to a bias below m/2^32, which this ignores. */
double cfo_table_fpr(const cfo_filter *flt)
{
    if (flt->placement == CFO_PLACE_OFFSET) return table_fpr_offset(flt);
    uint64_t cap = 2 * flt->count + 2, n = 0;
    pair_t *u = (pair_t *)malloc(cap * sizeof(pair_t));
    if (!u) return -1.0;
    for (uint64_t j = 0; j < flt->m; j++)
        for (uint32_t s = 0; s < flt->b; s++) {
            uint32_t v = cfo_get_slot(flt, j, s);
            if (v == 0 || n + 2 > cap) continue;
            u[n].bucket = j; u[n].tag = v; n++;
            u[n].bucket = cfo_alt(flt, j, v); u[n].tag = v; n++;
        }
    qsort(u, n, sizeof(pair_t), pair_cmp);
    double total = 0.0;
    double unit = 1.0;
    for (uint32_t i = 0; i < flt->f; i++) unit *= 0.5;
    for (uint64_t i = 0; i < n; i++) {
        if (i > 0 && pair_cmp(&u[i], &u[i - 1]) == 0) continue;
        total += u[i].tag == 1 ? 2.0 * unit : unit;
    }
    free(u);
    return total / (double)flt->m;
}
