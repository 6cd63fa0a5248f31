"""Pins of the oracle's offset placement policy (Sec. 4.6.2): a tag with its
choice bit clear sits in its primary bucket i1, a tag with the bit set in
i2 = (i1 + offset(fp)) mod m, and moving a tag between the two flips the bit;
any m is allowed.  The paper fixes the two equations and the flip, not the
offset function, so the pins check what follows from those:

* moving is an involution and never maps i1 to itself (m >= 2);
* the fingerprint and primary bucket come from the hash the way the XOR
  policy's do (upper / lower 32 bits), which they equal at power-of-two m;
* brute force on tiny tables: a query holds exactly when a live copy shares
  the key's (primary bucket, fingerprint); a delete removes exactly one;
* Hall's bound on insert failures; no false negatives at load 0.95 with a
  bucket count that is not a power of two;
* the false-positive rate: the table-exact value against sampled negatives,
  and against the first-order closed form b*alpha / 2^(f-1) (the choice bit
  is compared too, so this equals Eq. (4)'s 2*b*alpha / 2^f).
"""
import collections
import math

import numpy as np
import pytest

import oracle
from oracle import OracleFilter
from workloads import keys as K

OFF = oracle.PLACE_OFFSET
M32 = (1 << 32) - 1


def _flt(m, b, f, **kw):
    kw.setdefault("max_evict", 16)
    return OracleFilter(m, b, f, placement=OFF, **kw)


def test_parameters():
    for m in (1, 3, 1000, (1 << 32) - 1):
        _flt(m, 4, 8).close()
    with pytest.raises(ValueError):
        _flt(0, 4, 8)
    with pytest.raises(ValueError):
        _flt(1 << 32, 4, 8)
    with pytest.raises(ValueError):
        OracleFilter(3, 4, 8)  # XOR needs a power of two


@pytest.mark.parametrize("m", [1, 2, 3, 7, 1000, 12289, (1 << 31) + 11])
@pytest.mark.parametrize("f", [8, 16, 32])
def test_move_is_an_involution_and_flips_the_choice_bit(m, f):
    flt = _flt(m, 4, f)
    cb = 1 << (f - 1)
    rng = np.random.default_rng(m + f)
    for _ in range(300):
        j = int(rng.integers(0, m))
        v = int(rng.integers(1, cb))
        for t in (v, v | cb):
            a, t2 = flt.move(j, t)
            assert 0 <= a < m
            assert t2 == t ^ cb  # the bit flips, the fingerprint stays
            assert flt.move(a, t2) == (j, t)
            if m >= 2:
                assert a != j
    flt.close()


@pytest.mark.parametrize("m", [1, 5, 1 << 12, 3 * (1 << 12) + 1])
@pytest.mark.parametrize("f", [8, 16, 32])
def test_derive_structure(m, f):
    flt = _flt(m, 16, f)
    cb = 1 << (f - 1)
    xor = OracleFilter(m, 16, f) if m & (m - 1) == 0 else None
    for key in K.keys(9, 0, 400):
        key = int(key)
        t1, t2, i1, i2 = flt.derive_tags(key)
        assert 1 <= t1 < cb and t2 == t1 | cb
        assert 0 <= i1 < m and 0 <= i2 < m
        # the key's tag moved out of i1 lands in i2, written as t2
        assert flt.move(i1, t1) == (i2, t2)
        h = oracle.hash64(oracle.HASH_FMIX64, key)
        # i1 depends on the lower 32 hash bits only, the fingerprint on the upper
        assert i1 == (h & M32) % m
        fp_hi = (h >> 32) & (cb - 1)
        assert t1 == (fp_hi if fp_hi else 1)
        if xor is not None:
            # at power-of-two m the primary bucket is the XOR policy's
            _, x1, _ = xor.derive(key)
            assert x1 == i1
    flt.close()
    if xor is not None:
        xor.close()


def _group(flt, key):
    lo, hi, t = flt.key_groups([key])
    return (int(lo[0]), int(hi[0]), int(t[0]))


def _table_multiset(flt):
    """(primary, alternate, fingerprint) of every stored tag, from the raw
    slots: the choice bit tells which of the two buckets the tag is in."""
    cb = 1 << (flt.f - 1)
    ms = collections.Counter()
    for j in range(flt.m):
        for s in range(flt.b):
            v = flt.slot(j, s)
            if v:
                a, _ = flt.move(j, v)
                ms[(a, j, v & ~cb) if v & cb else (j, a, v)] += 1
    return ms


@pytest.mark.parametrize("m,b,f", [(1, 4, 8), (2, 4, 8), (3, 4, 8), (5, 4, 8), (7, 8, 8),
                                   (3, 4, 16), (13, 8, 16), (6, 16, 16), (5, 4, 32)])
@pytest.mark.parametrize("evict", [oracle.EVICT_BFS, oracle.EVICT_DFS])
def test_bruteforce_against_group_predicate(m, b, f, evict):
    flt = _flt(m, b, f, evict=evict, max_evict=8, seed=77)
    rng = np.random.default_rng(m * 131 + b * 7 + f + evict)
    universe = [int(k) for k in K.keys(2000 + m, 0, 6 * m * b)]
    universe += universe[:4]
    G = collections.Counter()
    live = []
    lost_seen = 0
    cb = 1 << (f - 1)
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
                a, _ = flt.move(j, v)
                G[(a, j, v & ~cb) if v & cb else (j, a, v)] -= 1
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
            lo, hi, tg = flt.stored_groups()
            assert collections.Counter(zip(lo.tolist(), hi.tolist(), tg.tolist())) == +G
    assert _table_multiset(flt) == +G
    assert flt.failures == lost_seen
    flt.close()


def _max_matching(pairs, b):
    owner = {}

    def try_assign(k, seen):
        for j in set(pairs[k]):
            for s in range(b):
                node = (j, s)
                if node in seen:
                    continue
                seen.add(node)
                if node not in owner or try_assign(owner[node], seen):
                    owner[node] = k
                    return True
        return False

    return sum(1 for k in range(len(pairs)) if try_assign(k, set()))


@pytest.mark.parametrize("m,b", [(3, 4), (5, 4), (6, 8)])
@pytest.mark.parametrize("evict", [oracle.EVICT_BFS, oracle.EVICT_DFS])
def test_failures_respect_halls_bound(m, b, evict):
    flt = _flt(m, b, 8, evict=evict, max_evict=50, seed=1)
    keys = [int(k) for k in K.keys(3030 + m + b, 0, 3 * m * b)]
    pairs = [flt.derive_tags(k)[2:] for k in keys]
    ok = flt.insert_batch(keys)
    assert int(ok.sum()) <= _max_matching(pairs, b)
    assert flt.count == int(ok.sum())
    flt.close()


def test_no_false_negatives_at_high_load_with_any_bucket_count():
    m, b, f = 3 * (1 << 12) + 7, 16, 16  # not a power of two
    n = int(0.95 * m * b)
    flt = _flt(m, b, f, max_evict=128, seed=5)
    pos = K.keys(44, 0, n)
    ok = flt.insert_batch(pos)
    assert ok.all() and flt.failures == 0 and flt.count == n
    assert flt.query_batch(pos).all()
    half = K.seeded_subset(44, n, n // 2)
    assert flt.delete_batch(pos[half]).all()
    keep = np.setdiff1d(np.arange(n), half)
    assert flt.query_batch(pos[keep]).all()
    assert flt.count == n - n // 2
    flt.close()


@pytest.mark.parametrize("b,f", [(4, 8), (16, 8)])
def test_fpr_table_exact_and_closed_form(b, f):
    m = 1000 * 3 + 1
    n = int(0.9 * m * b)
    flt = _flt(m, b, f, max_evict=500, seed=2)
    flt.insert_batch(K.keys(60, 0, n))
    assert flt.failures == 0
    neg = K.negatives(60, 0, 400_000)
    rate = flt.query_batch(neg).mean()
    eps_t = flt.table_fpr()
    sigma = math.sqrt(eps_t * (1 - eps_t) / neg.size)
    assert abs(rate - eps_t) <= 5 * sigma
    alpha = flt.load_factor
    closed = 1.0 - (1.0 - 2.0 ** -(f - 1)) ** (b * alpha)
    # the closed form ignores collisions of groups and the 0 -> 1 remap
    assert abs(eps_t - closed) / closed < 0.05
    xor_eq4 = 1.0 - (1.0 - 2.0 ** -f) ** (2 * b * alpha)
    assert abs(closed - xor_eq4) / xor_eq4 < 0.01
    flt.close()


def test_xor_and_offset_agree_on_membership_answers_for_stored_keys():
    """Both policies hold every stored key; negatives differ only by chance."""
    m, b, f = 1 << 12, 8, 16
    keys = K.keys(71, 0, int(0.9 * m * b))
    for place in (oracle.PLACE_XOR, OFF):
        flt = OracleFilter(m, b, f, max_evict=128, seed=4, placement=place)
        assert flt.insert_batch(keys).all()
        assert flt.query_batch(keys).all()
        flt.close()
