"""GPU parity of the offset placement policy (Sec. 4.6.2): any bucket count,
the fingerprint's choice bit tells a tag's primary bucket from its
alternate, and moving a tag flips the bit.

The bar is the XOR policy's: queries and deletes on an oracle-built table
are bit-exact, inserts one key per launch reproduce the oracle's table,
evictions and failures exactly, and concurrent inserts store the oracle's
(primary, alternate, fingerprint) multiset with every dropped tag logged.
Bucket counts are not powers of two, down to a single bucket and up to
2^32 - 5 (the largest the 32-bit bucket index allows, where i1 + offset
exceeds 2^32 before the modulo).
"""
import numpy as np
import pytest

import oracle
from oracle import OracleFilter
from gpu_util import (GEOMS, dev_u64, dev_zeros_u8, dev_zeros_u32, expected_groups, host_u64,
                      multiset_equal)
from workloads import keys as K

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
OFF = oracle.PLACE_OFFSET


@pytest.fixture(scope="module")
def cf():
    import paper_2603_15486_amd as mod
    return mod


def _pair(cf, m, b, f, hk=0, ev=0, D=128, seed=0):
    g = cf.CuckooFilter(m, b, f, hash=hk, evict=ev, max_evict=D, seed=seed,
                        placement=cf.CF_PLACE_OFFSET)
    r = OracleFilter(m, b, f, hash_kind=hk, evict=ev, max_evict=D, seed=seed, placement=OFF)
    return g, r


def _table(g):
    torch.cuda.synchronize()
    return host_u64(g.export_table())


def _load(g, words):
    g.import_table(dev_u64(words))
    torch.cuda.synchronize()


@pytest.mark.parametrize("b,f", GEOMS)
@pytest.mark.parametrize("hk", [oracle.HASH_FMIX64, oracle.HASH_XXH64])
def test_query_bit_exact_on_oracle_table(cf, b, f, hk):
    m = 1531 + b  # not a power of two
    seed = 5000 + b + f
    g, r = _pair(cf, m, b, f, hk=hk, seed=seed)
    pos = K.keys(seed, 0, int(0.9 * m * b))
    r.insert_batch(pos)
    _load(g, r.words())
    assert g.count() == r.count
    keys = np.concatenate([pos, K.negatives(seed, 0, 30_011)])
    got = g.query(dev_u64(keys)).cpu().numpy()
    assert np.array_equal(got, r.query_batch(keys))
    g.close()


@pytest.mark.parametrize("b,f", GEOMS)
def test_delete_bit_exact_on_oracle_table(cf, b, f):
    m = 1733 + 3 * b
    seed = 6000 + b + f
    g, r = _pair(cf, m, b, f, seed=seed)
    n = int(0.9 * m * b)
    pos = K.keys(seed, 0, n)
    r.insert_batch(pos)
    assert r.failures == 0
    _load(g, r.words())
    # only stored keys: deleting a non-member may remove a colliding copy, and
    # which one then depends on the order of the concurrent deletes
    sub = pos[K.seeded_subset(seed, n, n // 2)]
    ok = dev_zeros_u8(sub.size)
    g.delete(dev_u64(sub), ok)
    assert np.array_equal(ok.cpu().numpy(), r.delete_batch(sub))
    assert np.array_equal(_table(g), r.words())
    assert g.count() == r.count
    g.close()


@pytest.mark.parametrize("b,f", GEOMS)
@pytest.mark.parametrize("ev,D", [(oracle.EVICT_BFS, 8), (oracle.EVICT_DFS, 30)])
def test_insert_serial_bit_exact(cf, b, f, ev, D):
    """One key per launch: the oracle's sequential table, evictions (with
    their choice-bit flips) and failures exactly."""
    m = 61
    seed = 7000 + b + f + ev
    g, r = _pair(cf, m, b, f, ev=ev, D=D, seed=seed)
    keys = K.keys(seed, 0, int(0.99 * m * b))
    want_ok, want_kicks = r.insert_batch(keys, with_kicks=True)
    d_keys = dev_u64(keys)
    ok = dev_zeros_u8(keys.size)
    kicks = dev_zeros_u32(keys.size)
    for i in range(keys.size):
        g.insert(d_keys[i:i + 1], ok[i:i + 1], kicks[i:i + 1])
    assert np.array_equal(_table(g), r.words())
    assert np.array_equal(ok.cpu().numpy(), want_ok)
    assert np.array_equal(kicks.cpu().numpy().astype(np.uint32), want_kicks)
    assert g.count() == r.count and g.failures() == r.failures
    lb, lt = g.lost()
    rb, rt = r.lost()
    assert np.array_equal(lb, rb) and np.array_equal(lt, rt)
    g.close()


def _check_concurrent(g, r, keys, ok, kicks, D):
    torch.cuda.synchronize()
    fails = g.failures()
    assert int(ok.cpu().numpy().sum()) == keys.size - fails
    lost = g.lost()
    assert len(lost[0]) == fails
    r.load_words(_table(g))
    assert g.count() == r.count == keys.size - fails
    assert multiset_equal(r.stored_groups(), expected_groups(r, keys, lost=lost))
    assert kicks.cpu().numpy().max(initial=0) <= D
    if fails == 0:
        assert g.query(dev_u64(keys)).cpu().numpy().all()


@pytest.mark.parametrize("b,f", GEOMS)
@pytest.mark.parametrize("ev", [oracle.EVICT_BFS, oracle.EVICT_DFS])
def test_insert_concurrent_invariants(cf, b, f, ev):
    m = 3001
    seed = 8000 + b + f + ev
    D = 128 if ev == oracle.EVICT_BFS else 500
    g, r = _pair(cf, m, b, f, ev=ev, D=D, seed=seed)
    lf = 0.9 if b == 4 else 0.95
    keys = K.keys(seed, 0, int(lf * m * b))
    ok, kicks = dev_zeros_u8(keys.size), dev_zeros_u32(keys.size)
    g.insert(dev_u64(keys), ok, kicks)
    _check_concurrent(g, r, keys, ok, kicks, D)
    g.close()


@pytest.mark.parametrize("m,b,f,ev", [(31, 4, 8, 0), (7, 16, 16, 0), (1, 32, 8, 1), (3, 4, 32, 0)])
def test_insert_overfull_accounts_for_every_dropped_tag(cf, m, b, f, ev):
    g, r = _pair(cf, m, b, f, ev=ev, D=4, seed=19)
    keys = np.concatenate([K.keys(19, 0, 3 * m * b), K.keys(19, 0, 8)])  # duplicates too
    ok, kicks = dev_zeros_u8(keys.size), dev_zeros_u32(keys.size)
    g.insert(dev_u64(keys), ok, kicks)
    assert g.failures() > 0
    _check_concurrent(g, r, keys, ok, kicks, 4)
    g.close()


def test_largest_bucket_count(cf):
    """m = 2^32 - 5 buckets of 4 x 8 bits (16 GiB): keys inserted one per
    launch land in exactly the oracle's slots, so i1 = (h mod 2^32) mod m and
    both modular steps are exact over the whole 32-bit range."""
    m, b, f = (1 << 32) - 5, 4, 8
    g, r = _pair(cf, m, b, f, seed=23)
    keys = K.keys(23, 0, 300)
    want = r.insert_batch(keys)
    d_keys = dev_u64(keys)
    ok = dev_zeros_u8(keys.size)
    for i in range(keys.size):
        g.insert(d_keys[i:i + 1], ok[i:i + 1])
    assert np.array_equal(ok.cpu().numpy(), want) and g.count() == r.count == keys.size
    words = g.export_table()  # int64 view of the packed table, on the device
    nz = torch.nonzero(words).flatten()
    vals = host_u64(words[nz])
    nz = nz.cpu().numpy()
    torch.cuda.synchronize()
    slots = 0
    for w, v in zip(nz, vals):
        for k in range(8):  # 8-bit slots, 8 per word; global slot = bucket * 4 + s
            g_slot = int(w) * 8 + k
            tag = (int(v) >> (8 * k)) & 0xFF
            assert tag == r.slot(g_slot // 4, g_slot % 4)
            slots += tag != 0
    assert slots == r.count
    assert g.query(d_keys).cpu().numpy().all()
    del words
    g.close()


def test_set_and_invalid_parameters(cf):
    with pytest.raises(cf.CfError):
        cf.CuckooFilter(0, 4, 8, placement=cf.CF_PLACE_OFFSET)
    with pytest.raises(cf.CfError):
        cf.CuckooFilter(1 << 32, 4, 8, placement=cf.CF_PLACE_OFFSET)
    with pytest.raises(cf.CfError):
        cf.CuckooFilter(1000, 4, 8)  # XOR needs a power of two
    with pytest.raises(cf.CfError):
        cf.CuckooFilter(1024, 4, 8, placement=7)
