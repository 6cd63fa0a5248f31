"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests runs GPU code.  Each pin is chosen so that a plausible
slip in the oracle (a dropped term, a wrong shift, a swapped operand, a wrong
index) fails at least one of them:

* hash functions: published known-answer values (MurmurHash3 x64 128 whose
  last step is fmix64; the SplitMix64 reference stream) and the xxhash library;
* derived values: the upper/lower 32-bit split of Sec. 4.3 checked across
  parameter choices, and the involution of Eq. (3);
* storage layout: Fig. 2's packing, checked by viewing the exported words as
  an array of little-endian f-bit integers;
* query/delete/insert: brute force against the exact multiset predicate on
  tiny inputs, Hall's bound on insert failures, the eviction bound;
* false-positive rate: Eq. (4) and the paper's measured point (Sec. 5.3).
"""
import collections
import math
import os

import numpy as np
import pytest
import xxhash

import oracle
from oracle import OracleFilter
from workloads import keys as K

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --------------------------------------------------------------- hashes

def _rotl(x, r):
    return ((x << r) | (x >> (64 - r))) & M64


def _murmur3_x64_128(data: bytes, seed: int):
    """MurmurHash3_x64_128 body (A. Appleby); the two halves are finished with
    the oracle's fmix64, so the known answer pins that function."""
    c1, c2 = 0x87C37B91114253D5, 0x4CF5AD432745937F
    h1 = h2 = seed
    nblocks = len(data) // 16
    for i in range(nblocks):
        k1 = int.from_bytes(data[16 * i:16 * i + 8], "little")
        k2 = int.from_bytes(data[16 * i + 8:16 * i + 16], "little")
        k1 = (_rotl((k1 * c1) & M64, 31) * c2) & M64
        h1 ^= k1
        h1 = (_rotl(h1, 27) + h2) & M64
        h1 = (h1 * 5 + 0x52DCE729) & M64
        k2 = (_rotl((k2 * c2) & M64, 33) * c1) & M64
        h2 ^= k2
        h2 = (_rotl(h2, 31) + h1) & M64
        h2 = (h2 * 5 + 0x38495AB5) & M64
    tail = data[16 * nblocks:]
    if len(tail) > 8:
        k2 = int.from_bytes(tail[8:], "little")
        h2 ^= (_rotl((k2 * c2) & M64, 33) * c1) & M64
    if tail:
        k1 = int.from_bytes(tail[:8], "little")
        h1 ^= (_rotl((k1 * c1) & M64, 31) * c2) & M64
    h1 ^= len(data)
    h2 ^= len(data)
    h1 = (h1 + h2) & M64
    h2 = (h2 + h1) & M64
    h1 = oracle.fmix64(h1)
    h2 = oracle.fmix64(h2)
    h1 = (h1 + h2) & M64
    h2 = (h2 + h1) & M64
    return h1, h2


def test_fmix64_known_answer():
    for text, seed, s1, s2, hexbytes in _golden("murmur3_x64_128_kat.txt"):
        h1, h2 = _murmur3_x64_128(text.encode(), int(seed))
        assert h1 == int(s1) & M64 and h2 == int(s2) & M64
        assert (h1.to_bytes(8, "little") + h2.to_bytes(8, "little")).hex() == hexbytes


def test_fmix64_fixed_point_and_bijection_sample():
    assert oracle.fmix64(0) == 0
    rng = np.random.default_rng(1)
    xs = rng.integers(0, 2**63, size=20000, dtype=np.int64).astype(np.uint64)
    outs = {oracle.fmix64(int(x)) for x in xs}
    assert len(outs) == len(set(int(x) for x in xs))


def test_xxh64_matches_library():
    rng = np.random.default_rng(2)
    vals = [0, 1, 2, 0xFFFF, 0xFFFFFFFF, M64] + [int(v) for v in
                                                   rng.integers(0, 2**63, 5000, dtype=np.int64)]
    for v in vals:
        assert oracle.xxh64_u64(v) == xxhash.xxh64_intdigest(v.to_bytes(8, "little"), seed=0)


def test_splitmix64_reference_stream():
    for row in _golden("splitmix64_kat.txt"):
        seed, outs = int(row[0]), [int(x) for x in row[1:]]
        assert [oracle.splitmix64_at(seed, k) for k in range(len(outs))] == outs
        # the shared key generator implements the same published stream
        assert [int(v) for v in K.keys(seed, 0, len(outs))] == outs


def test_keygen_positive_negative_disjoint():
    seed = K.workload_seed(0)
    pos = K.keys(seed, 0, 200000)
    neg = K.negatives(seed, 0, 200000)
    assert np.unique(pos).size == pos.size
    assert np.intersect1d(pos, neg).size == 0


# ------------------------------------------------------- derived values

@pytest.mark.parametrize("hk", [oracle.HASH_FMIX64, oracle.HASH_XXH64])
def test_derive_uses_upper_bits_for_fp_lower_for_index(hk):
    """Sec. 4.3 step 1: the upper 32 hash bits give the fingerprint and the
    lower 32 bits the primary bucket.  With f = 32 the fingerprint is the
    whole upper half; smaller m and f keep the low bits of each half."""
    full = OracleFilter(1 << 20, 4, 32, hash_kind=hk)
    rng = np.random.default_rng(3)
    for key in [int(k) for k in rng.integers(0, 2**63, 300, dtype=np.int64)] + [0, M64]:
        h = oracle.hash64(hk, key)
        fp32, i1_20, _ = full.derive(key)
        assert fp32 == ((h >> 32) or 1)
        assert i1_20 == (h & 0xFFFFFFFF) & ((1 << 20) - 1)
        for f in (8, 16):
            small = OracleFilter(1 << 6, 4, f, hash_kind=hk)
            fp, i1, _ = small.derive(key)
            want = (h >> 32) & ((1 << f) - 1)
            assert fp == (want if want else 1)
            assert i1 == i1_20 & 63
            small.close()
    full.close()


@pytest.mark.parametrize("m", [1, 2, 64, 1 << 18])
def test_alt_is_involution_and_pairs_consistent(m):
    flt = OracleFilter(m, 4, 16)
    rng = np.random.default_rng(4)
    for key in rng.integers(0, 2**63, 500, dtype=np.int64):
        fp, i1, i2 = flt.derive(int(key))
        assert 0 < fp < 1 << 16
        assert 0 <= i1 < m and 0 <= i2 < m
        assert flt.alt(i1, fp) == i2 and flt.alt(i2, fp) == i1
    flt.close()


# -------------------------------------------------------------- layout

def _slot_view(words: np.ndarray, f: int) -> np.ndarray:
    dt = {8: "<u1", 16: "<u2", 32: "<u4"}[f]
    return words.astype("<u8").view(dt)


@pytest.mark.parametrize("b", [4, 8, 16, 32])
@pytest.mark.parametrize("f", [8, 16, 32])
def test_layout_matches_little_endian_packing(b, f):
    """Fig. 2: slot k of a word sits at bits [k*f, (k+1)*f).  Viewing the
    little-endian words as an array of f-bit integers therefore lists the
    slots in global order j*b + s."""
    m = 64
    flt = OracleFilter(m, b, f, seed=9)
    flt.insert_batch(K.keys(11, 0, int(0.8 * m * b)))
    view = _slot_view(flt.words(), f)
    assert view.size >= m * b
    for j in range(m):
        for s in range(b):
            assert flt.slot(j, s) == int(view[j * b + s])
    assert flt.count == int(np.count_nonzero(view[: m * b]))
    flt.close()


@pytest.mark.parametrize("b,f", [(16, 16), (8, 8), (32, 16), (4, 32)])
def test_first_insert_starts_at_fingerprint_word(b, f):
    """Alg. 1 TryInsert: into an empty bucket the tag lands in the first slot
    of word (fp mod b) / tagsPerWord."""
    tpw = 64 // f
    flt = OracleFilter(1 << 16, b, f)
    key = 12345
    fp, i1, _ = flt.derive(key)
    ok, _ = flt.insert(key)
    assert ok
    start = (fp % b) // tpw
    assert flt.slot(i1, start * tpw) == fp
    occupied = [s for s in range(b) if flt.slot(i1, s)]
    assert occupied == [start * tpw]
    flt.close()


def test_subword_buckets_do_not_touch_neighbours():
    """b*f = 32 < 64: two buckets share a word.  Every stored tag must sit in
    a bucket of its own pair, so filling one bucket cannot spill into the
    bucket sharing its word."""
    flt = OracleFilter(1 << 8, 4, 8, seed=3)
    flt.insert_batch(K.keys(5, 0, 1000))
    view = _slot_view(flt.words(), 8)
    assert view.size == (1 << 8) * 4
    for j in range(1 << 8):
        for s in range(4):
            assert flt.slot(j, s) == int(view[j * 4 + s])
    flt.close()


# -------------------------------------------------- brute-force semantics

def _group(flt, key):
    fp, i1, i2 = flt.derive(key)
    return (min(i1, i2), max(i1, i2), fp)


def _table_multiset(flt):
    ms = collections.Counter()
    for j in range(flt.m):
        for s in range(flt.b):
            v = flt.slot(j, s)
            if v:
                a = flt.alt(j, v)
                ms[(min(j, a), max(j, a), v)] += 1
    return ms


@pytest.mark.parametrize("m,b,f", [(1, 4, 8), (2, 4, 8), (4, 4, 8), (8, 4, 8), (8, 8, 8),
                                   (4, 4, 16), (16, 8, 16), (8, 16, 16), (4, 4, 32)])
@pytest.mark.parametrize("evict", [oracle.EVICT_BFS, oracle.EVICT_DFS])
def test_bruteforce_against_multiset_predicate(m, b, f, evict):
    """Query(x) holds iff some live copy shares x's (bucket pair, fingerprint);
    Delete(x) succeeds iff such a copy exists and removes exactly one; the
    stored multiset equals inserted minus deleted minus dropped tags."""
    flt = OracleFilter(m, b, f, evict=evict, max_evict=8, seed=77)
    rng = np.random.default_rng(m * 131 + b * 7 + f + evict)
    universe = [int(k) for k in K.keys(1000 + m, 0, 6 * m * b)]
    # small fingerprints make group collisions common; force some duplicates
    universe += universe[:4]
    G = collections.Counter()
    live = []
    lost_seen = 0
    for step in range(12 * m * b):
        op = rng.integers(0, 10)
        if op < 5 or not live:
            key = universe[int(rng.integers(0, len(universe)))]
            ok, kicks = flt.insert(key)
            assert kicks <= flt.max_evict
            G[_group(flt, key)] += 1
            if ok:
                live.append(key)
            else:
                assert kicks == flt.max_evict
                lb, lt = flt.lost()
                assert len(lb) == lost_seen + 1
                j, v = int(lb[-1]), int(lt[-1])
                a = flt.alt(j, v)
                G[(min(j, a), max(j, a), v)] -= 1
                lost_seen += 1
        elif op < 8:
            key = universe[int(rng.integers(0, len(universe)))]
            assert flt.query(key) == (G[_group(flt, key)] > 0)
        else:
            key = live[int(rng.integers(0, len(live)))] if rng.integers(0, 2) else \
                universe[int(rng.integers(0, len(universe)))]
            expect = G[_group(flt, key)] > 0
            assert flt.delete(key) == expect
            if expect:
                G[_group(flt, key)] -= 1
        if step % 7 == 0:
            assert _table_multiset(flt) == +G
            assert flt.count == sum(G.values())
    assert _table_multiset(flt) == +G
    assert flt.failures == lost_seen
    flt.close()


def _max_matching(keys_pairs, m, b):
    """Max number of keys placeable with each key in one of its two buckets
    and at most b keys per bucket (augmenting paths on slot copies)."""
    owner = {}  # (bucket, slot) -> key index

    def try_assign(k, seen):
        for j in set(keys_pairs[k]):
            for s in range(b):
                node = (j, s)
                if node in seen:
                    continue
                seen.add(node)
                if node not in owner or try_assign(owner[node], seen):
                    owner[node] = k
                    return True
        return False

    return sum(1 for k in range(len(keys_pairs)) if try_assign(k, set()))


@pytest.mark.parametrize("m,b", [(2, 4), (4, 4), (8, 4), (4, 8)])
@pytest.mark.parametrize("evict", [oracle.EVICT_BFS, oracle.EVICT_DFS])
def test_failures_respect_halls_bound(m, b, evict):
    flt = OracleFilter(m, b, 8, evict=evict, max_evict=50, seed=1)
    keys = [int(k) for k in K.keys(2024 + m + b, 0, 3 * m * b)]
    pairs = []
    for key in keys:
        _, i1, i2 = flt.derive(key)
        pairs.append((i1, i2))
    ok = flt.insert_batch(keys)
    assert int(ok.sum()) <= _max_matching(pairs, m, b)
    assert flt.count == int(ok.sum())
    flt.close()


@pytest.mark.parametrize("evict", [oracle.EVICT_BFS, oracle.EVICT_DFS])
def test_duplicates_fill_two_buckets_then_fail(evict):
    b = 4
    flt = OracleFilter(1 << 10, b, 16, evict=evict, max_evict=10)
    key = 987654321
    fp, i1, i2 = flt.derive(key)
    assert i1 != i2
    results = [flt.insert(key)[0] for _ in range(2 * b + 1)]
    assert results == [True] * (2 * b) + [False]
    lb, lt = flt.lost()
    assert list(lt) == [fp] and int(lb[0]) in (i1, i2)
    assert flt.count == 2 * b
    # every delete removes one copy; the ninth finds none
    assert [flt.delete(key) for _ in range(2 * b + 1)] == [True] * (2 * b) + [False]
    assert flt.count == 0
    flt.close()


def test_no_false_negatives_and_counts_2e18_buckets_b4_f16():
    """2^18 buckets x 4 slots, f = 16, filled to LF 0.9 in one batch."""
    seed = K.workload_seed(0)
    n = 943718
    flt = OracleFilter(1 << 18, 4, 16, max_evict=128, seed=seed)
    pos = K.keys(seed, 0, n)
    ok = flt.insert_batch(pos)
    assert flt.failures == 0 and ok.all()
    assert flt.count == n
    assert flt.query_batch(pos).all()
    half = K.seeded_subset(seed, n, n // 2)
    assert flt.delete_batch(pos[half]).all()
    assert flt.count == n - n // 2
    keep = np.setdiff1d(np.arange(n), half)
    assert flt.query_batch(pos[keep]).all()
    flt.close()


# ----------------------------------------------------------- false positives

def _eq4(b, f, alpha):
    return 1.0 - (1.0 - 2.0 ** -f) ** (2 * b * alpha)


def test_fpr_2e18_buckets_b4_f16_within_table_exact_and_eq4():
    seed = K.workload_seed(0)
    n = 943718
    flt = OracleFilter(1 << 18, 4, 16, max_evict=128, seed=seed)
    flt.insert_batch(K.keys(seed, 0, n))
    neg = K.negatives(seed, 0, 1_000_000)
    fps = int(flt.query_batch(neg).sum())
    eps_t = flt.table_fpr()
    N = neg.size
    sigma = math.sqrt(N * eps_t * (1 - eps_t))
    assert abs(fps - N * eps_t) <= 5 * sigma
    # Eq. (4) with the 0 -> 1 fingerprint remap is within a few percent of the table value
    alpha = flt.load_factor
    assert abs(eps_t - _eq4(4, 16, alpha)) / _eq4(4, 16, alpha) < 0.05
    # the crude first-order bound 2b/2^f * alpha holds
    assert eps_t <= 2 * 4 / (2 ** 16 - 1) * alpha
    flt.close()


def test_fpr_matches_paper_point():
    """Sec. 5.3: about 0.045% for b = 16, f = 16 at load 0.95, with keys from
    [0, 2^32) inserted and keys from [2^32, 2^64) queried."""
    (b, f, alpha, pct), = [(int(r[0]), int(r[1]), float(r[2]), float(r[3]))
                           for r in _golden("fpr_paper_point.txt")]
    m = 1 << 14
    target = int(alpha * m * b)
    cand = np.unique(K.keys(31, 0, 3 * target) & np.uint64(0xFFFFFFFF))
    rng = np.random.default_rng(5)
    ins = rng.permutation(cand)[:target]
    flt = OracleFilter(m, b, f, max_evict=128, seed=3)
    flt.insert_batch(ins)
    assert flt.failures == 0
    neg = K.keys(32, 0, 4_000_000)
    neg = neg[neg >= np.uint64(1 << 32)]
    rate = flt.query_batch(neg).mean()
    sigma = math.sqrt(rate * (1 - rate) / neg.size)
    # the paper's rounded figure, and Eq. (4)'s 0.0464%, within sampling noise
    assert abs(rate * 100 - pct) < 0.006 + 5 * sigma * 100
    assert abs(rate - _eq4(b, f, alpha)) < 5 * sigma + 2e-5
    flt.close()


def test_bfs_suppresses_tail_kicks_vs_dfs():
    """Sec. 5.4.1 / Fig. 5: near full load the breadth-first heuristic keeps
    the tail of kicks per insert well below the random walk's."""
    m, b, f = 1 << 14, 4, 8
    n = int(0.95 * m * b)
    keys = K.keys(77, 0, n)
    stats = {}
    for ev in (oracle.EVICT_BFS, oracle.EVICT_DFS):
        flt = OracleFilter(m, b, f, evict=ev, max_evict=500, seed=1)
        ok, kicks = flt.insert_batch(keys, with_kicks=True)
        assert ok.all()
        last = kicks[int(0.93 * m * b):]
        stats[ev] = (np.percentile(last, 99), kicks.max(), int(kicks.sum()))
        flt.close()
    bfs, dfs = stats[oracle.EVICT_BFS], stats[oracle.EVICT_DFS]
    assert bfs[0] < dfs[0] and bfs[1] < dfs[1] and bfs[2] < dfs[2]


@pytest.mark.parametrize("evict,D", [(oracle.EVICT_BFS, 2), (oracle.EVICT_DFS, 5)])
def test_group_digest_tracks_the_stored_multiset(evict, D):
    """The digests used by the full-size GPU checks: the table's digest equals
    the keys' digest minus the dropped tags', and moves with any change."""
    m, b, f = 1 << 8, 4, 8
    flt = OracleFilter(m, b, f, evict=evict, max_evict=D, seed=3)
    keys = K.keys(44, 0, int(1.02 * m * b))
    flt.insert_batch(keys)
    assert flt.failures > 0
    lb, lt = flt.lost()
    M = (1 << 64) - 1
    assert flt.digest_table() == (flt.digest_keys(keys) - flt.digest_pairs(lb, lt)) & M
    assert (flt.digest_table(0, 100) + flt.digest_table(100, m)) & M == flt.digest_table()
    # keys' digest is order independent and sensitive to one key
    assert flt.digest_keys(keys[::-1]) == flt.digest_keys(keys)
    assert flt.digest_keys(keys[1:]) != flt.digest_keys(keys)
    # deleting one live key changes the table digest by exactly its group
    live = [int(k) for k in keys if flt.query(int(k))]
    before = flt.digest_table()
    assert flt.delete(live[0])
    assert (before - flt.digest_table()) & M == flt.digest_keys([live[0]])
    flt.close()


def test_load_words_recounts():
    flt = OracleFilter(1 << 10, 8, 16, seed=2)
    flt.insert_batch(K.keys(3, 0, 5000))
    w = flt.words()
    other = OracleFilter(1 << 10, 8, 16)
    other.load_words(w)
    assert other.count == flt.count
    assert np.array_equal(other.words(), w)
    flt.close()
    other.close()


def test_io_counts_follow_the_algorithm_steps():
    """The oracle's traffic counters (bucket reads, word writes) that price
    the roofline's algorithmic bytes: an insert into an empty table reads one
    bucket and writes one word; a query reads one bucket when i1 holds the
    fingerprint and two when it misses; a delete found in i1 reads one bucket
    and clears one slot.  Counting changes no result."""
    f = OracleFilter(1 << 10, 16, 16, max_evict=128, seed=1)
    keys = K.keys(1, 0, 200)
    f.insert_batch(keys)
    assert f.io_counts() == (200, 200)
    f.io_reset()
    fp, i1, i2 = f.derive_batch(keys)
    in_i1 = np.array([any(f.slot(int(j), s) == int(v) for s in range(16))
                      for j, v in zip(i1, fp)])
    assert in_i1.all()  # a near-empty table takes every key in i1
    f.query_batch(keys)
    assert f.io_counts() == (200, 0)
    f.io_reset()
    neg = K.negatives(1, 0, 300)
    found = f.query_batch(neg)
    assert not found.any()  # no false positive at this load: both buckets read
    assert f.io_counts() == (600, 0)
    f.io_reset()
    f.delete_batch(keys[:50])
    assert f.io_counts() == (50, 50)
    full = OracleFilter(1 << 8, 4, 16, max_evict=64, seed=2)
    ks = K.keys(2, 0, int(0.97 * 1024))
    ok, kicks = full.insert_batch(ks, with_kicks=True)
    r, w = full.io_counts()
    # every stored fingerprint took exactly one write per slot it was put in:
    # one per success plus one per kick (a displaced tag is rewritten)
    assert w == int(ok.sum()) + int(kicks.sum())
    assert r >= ks.size
    f.close()
    full.close()
