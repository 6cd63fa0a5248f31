"""GPU parity: libcf.so (HIP, gfx950) against the CPU oracle, through the C ABI.

* query on an oracle-built table: bit-exact per key;
* delete on an oracle-built table: bit-exact final table and per-key flags;
* insert one key per launch: bit-exact table, flags, kicks and dropped tags;
* concurrent insert: the stored (bucket pair, fingerprint) multiset equals the
  inserted keys' minus the dropped tags, zero false negatives, exact counts,
  and the kick bound.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import OracleFilter
from gpu_util import (GEOMS, dev_u64, dev_zeros_u8, dev_zeros_u32, expected_groups,
                            host_u64, multiset_equal)
from workloads import keys as K

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cf():
    import paper_2603_15486_amd as mod
    return mod


def _pair(cf, m, b, f, hk=0, ev=0, D=128, seed=0, grid_per_cu=None):
    if grid_per_cu is not None:
        os.environ["CF_GRID_PER_CU"] = str(grid_per_cu)
    try:
        g = cf.CuckooFilter(m, b, f, hash=hk, evict=ev, max_evict=D, seed=seed)
    finally:
        os.environ.pop("CF_GRID_PER_CU", None)
    r = OracleFilter(m, b, f, hash_kind=hk, evict=ev, max_evict=D, seed=seed)
    return g, r


def _table(g):
    torch.cuda.synchronize()
    return host_u64(g.export_table())


def _load(g, words):
    g.import_table(dev_u64(words))
    torch.cuda.synchronize()


# ------------------------------------------------------------------ keygen

@pytest.mark.parametrize("seed,start,n", [(0, 0, 1000), (K.workload_seed(1), 12345, 100_003),
                                          (7, K.NEG_BASE, 4097), (9, 2**64 - 100, 300)])
def test_keygen_matches_host_generator(cf, seed, start, n):
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    cf.cf_keygen(out, seed, start)
    assert np.array_equal(host_u64(out), K.keys(seed, start, n))
    ctr = np.arange(n, dtype=np.uint64)[::-1].copy()
    out2 = torch.empty(n, dtype=torch.int64, device="cuda")
    cf.cf_keygen_at(out2, dev_u64(ctr), seed)
    assert np.array_equal(host_u64(out2), K.splitmix64(seed, ctr))


# ------------------------------------------------------------------- query

@pytest.mark.parametrize("b,f", GEOMS)
@pytest.mark.parametrize("hk", [oracle.HASH_FMIX64, oracle.HASH_XXH64])
def test_query_bit_exact_on_oracle_table(cf, b, f, hk):
    m = 1 << 11
    seed = 1000 + b + f
    g, r = _pair(cf, m, b, f, hk=hk, seed=seed)
    pos = K.keys(seed, 0, int(0.9 * m * b))
    r.insert_batch(pos)
    _load(g, r.words())
    assert g.count() == r.count
    keys = np.concatenate([pos, K.negatives(seed, 0, 30_011)])
    got = g.query(dev_u64(keys)).cpu().numpy()
    want = r.query_batch(keys)
    assert np.array_equal(got, want)
    assert got[:pos.size].all() or r.failures > 0
    g.close()


def test_query_multi_pass_grid_and_ragged_tail(cf):
    """Small grid (one block per CU) so every lane walks many grid strides;
    the batch size is not a multiple of the block."""
    m, b, f = 1 << 14, 16, 16
    g, r = _pair(cf, m, b, f, seed=3, grid_per_cu=1)
    r.insert_batch(K.keys(3, 0, int(0.95 * m * b)))
    _load(g, r.words())
    keys = np.concatenate([K.keys(3, 0, 200_000), K.negatives(3, 0, 333_337)])
    got = g.query(dev_u64(keys)).cpu().numpy()
    assert np.array_equal(got, r.query_batch(keys))
    g.close()


def test_query_empty_and_single(cf):
    g, r = _pair(cf, 1 << 8, 16, 16)
    empty = torch.empty(0, dtype=torch.int64, device="cuda")
    out = g.query(empty)
    assert out.numel() == 0
    one = K.keys(5, 0, 1)
    assert g.query(dev_u64(one)).cpu().numpy().tolist() == [0]
    g.insert(dev_u64(one))
    assert g.query(dev_u64(one)).cpu().numpy().tolist() == [1]
    g.close()


# ------------------------------------------------------------------ delete

@pytest.mark.parametrize("b,f", GEOMS)
@pytest.mark.parametrize("hk", [oracle.HASH_FMIX64, oracle.HASH_XXH64])
def test_delete_bit_exact_on_oracle_table(cf, b, f, hk):
    m = 1 << 11
    seed = 2000 + b + f
    g, r = _pair(cf, m, b, f, hk=hk, seed=seed)
    n = int(0.9 * m * b)
    pos = K.keys(seed, 0, n)
    r.insert_batch(pos)
    assert r.failures == 0
    _load(g, r.words())
    sub = pos[K.seeded_subset(seed, n, n // 2)]
    ok = dev_zeros_u8(sub.size)
    g.delete(dev_u64(sub), ok)
    want_ok = r.delete_batch(sub)
    assert np.array_equal(ok.cpu().numpy(), want_ok)
    assert np.array_equal(_table(g), r.words())
    assert g.count() == r.count
    g.close()


def test_delete_duplicates_and_repeats(cf):
    """Keys deleted more often than inserted: per-group success counts and the
    final table are exact whatever the interleaving."""
    m, b, f = 1 << 6, 8, 8
    g, r = _pair(cf, m, b, f, seed=4)
    base = K.keys(4, 0, 150)
    ins = np.concatenate([base, base[:40], base[:10]])
    r.insert_batch(ins)
    _load(g, r.words())
    dels = np.concatenate([base[:60], base[:60], base[:20]])
    ok = dev_zeros_u8(dels.size)
    g.delete(dev_u64(dels), ok)
    want = r.delete_batch(dels)
    assert int(ok.sum()) == int(want.sum())
    assert np.array_equal(_table(g), r.words())
    assert g.count() == r.count
    g.close()


# ---------------------------------------------------- insert, one per launch

@pytest.mark.parametrize("b,f", GEOMS)
@pytest.mark.parametrize("ev,D", [(oracle.EVICT_BFS, 8), (oracle.EVICT_DFS, 30)])
def test_insert_serial_bit_exact(cf, b, f, ev, D):
    """One key per launch: no concurrency, so the GPU must reproduce the
    oracle's sequential table exactly, including evictions and failures."""
    m = 1 << 6
    seed = 3000 + b + f + ev
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


@pytest.mark.parametrize("m,b,f,lf,ev,D", [(1 << 20, 16, 16, 0.97, oracle.EVICT_BFS, 8),
                                           (1 << 20, 16, 16, 0.97, oracle.EVICT_DFS, 30),
                                           (1 << 21, 4, 32, 0.93, oracle.EVICT_BFS, 8)])
def test_insert_serial_bit_exact_large_table(cf, m, b, f, lf, ev, D):
    """Tables above the size up to which the breadth-first search probes
    candidates in groups (32 MiB here) take the one-by-one probe: the same
    serial parity, one key per launch, on an oracle-built table near full,
    so that most keys run the eviction search."""
    seed = 3200 + b + f + ev
    g, r = _pair(cf, m, b, f, ev=ev, D=D, seed=seed)
    assert cf.cf_table_bytes(g.params) > 16 << 20
    r.insert_batch(K.keys(seed, 0, int(lf * m * b)))
    _load(g, r.words())
    f0, lost0 = r.failures, len(r.lost()[0])
    keys = K.keys(seed, 1 << 40, 300)
    want_ok, want_kicks = r.insert_batch(keys, with_kicks=True)
    assert (np.asarray(want_kicks) > 0).sum() > 100  # the search really ran
    d_keys = dev_u64(keys)
    ok = dev_zeros_u8(keys.size)
    kicks = dev_zeros_u32(keys.size)
    for i in range(keys.size):
        g.insert(d_keys[i:i + 1], ok[i:i + 1], kicks[i:i + 1])
    assert np.array_equal(_table(g), r.words())
    assert np.array_equal(ok.cpu().numpy(), want_ok)
    assert np.array_equal(kicks.cpu().numpy().astype(np.uint32), want_kicks)
    assert g.count() == r.count and g.failures() == r.failures - f0
    lb, lt = g.lost()
    rb, rt = r.lost()
    assert np.array_equal(lb, rb[lost0:]) and np.array_equal(lt, rt[lost0:])
    g.close()
    r.close()


@pytest.mark.parametrize("m", [1, 2])
@pytest.mark.parametrize("b,f", [(4, 8), (16, 16), (32, 32)])
@pytest.mark.parametrize("ev,D", [(oracle.EVICT_BFS, 8), (oracle.EVICT_DFS, 30)])
def test_one_and_two_bucket_tables_bit_exact(cf, m, b, f, ev, D):
    """The degenerate XOR tables: with m = 1 a key's two buckets are both
    bucket 0, with m = 2 they are {0, 1} or one bucket twice, so the
    breadth-first search skips every candidate whose other bucket is the
    current one (R4) and the table overflows after m*b keys.  One key per
    launch, 2mb + 3 keys: table, flags, kicks, failures and the dropped-tag
    log equal the oracle's; then queries of every key and of negatives, and
    deletes of every key one per launch, equal the oracle's too."""
    seed = 3100 + 10 * m + b + f + ev
    g, r = _pair(cf, m, b, f, ev=ev, D=D, seed=seed)
    keys = K.keys(seed, 0, 2 * m * b + 3)
    want_ok, want_kicks = r.insert_batch(keys, with_kicks=True)
    d_keys = dev_u64(keys)
    ok = dev_zeros_u8(keys.size)
    kicks = dev_zeros_u32(keys.size)
    for i in range(keys.size):
        g.insert(d_keys[i:i + 1], ok[i:i + 1], kicks[i:i + 1])
    assert np.array_equal(_table(g), r.words())
    assert np.array_equal(ok.cpu().numpy(), want_ok)
    assert np.array_equal(kicks.cpu().numpy().astype(np.uint32), want_kicks)
    assert g.count() == r.count <= m * b and g.failures() == r.failures > 0
    lb, lt = g.lost()
    rb, rt = r.lost()
    assert np.array_equal(lb, rb) and np.array_equal(lt, rt)
    q = np.concatenate([keys, K.negatives(seed, 0, 2000)])
    assert np.array_equal(g.query(dev_u64(q)).cpu().numpy(), r.query_batch(q))
    dok = dev_zeros_u8(keys.size)
    for i in range(keys.size):
        g.delete(d_keys[i:i + 1], dok[i:i + 1])
    assert np.array_equal(dok.cpu().numpy(), r.delete_batch(keys))
    assert np.array_equal(_table(g), r.words())
    assert g.count() == r.count
    g.close()
    r.close()


# ---------------------------------------------------- insert, concurrent

def _check_concurrent(g, r, keys, ok, kicks, D):
    torch.cuda.synchronize()
    okh = ok.cpu().numpy()
    fails = g.failures()
    assert int(okh.sum()) == keys.size - fails
    lost = g.lost()
    assert len(lost[0]) == fails
    words = _table(g)
    r.load_words(words)
    assert g.count() == r.count == keys.size - fails
    assert multiset_equal(r.stored_groups(), expected_groups(r, keys, lost=lost))
    kk = kicks.cpu().numpy()
    assert kk.max(initial=0) <= D
    if fails == 0:
        assert g.query(dev_u64(keys)).cpu().numpy().all()


@pytest.mark.parametrize("b,f", GEOMS)
@pytest.mark.parametrize("ev", [oracle.EVICT_BFS, oracle.EVICT_DFS])
def test_insert_concurrent_invariants(cf, b, f, ev):
    m = 1 << 12
    seed = 4000 + b + f + ev
    D = 128 if ev == oracle.EVICT_BFS else 500
    g, r = _pair(cf, m, b, f, ev=ev, D=D, seed=seed)
    lf = 0.9 if b == 4 else 0.95
    keys = K.keys(seed, 0, int(lf * m * b))
    ok, kicks = dev_zeros_u8(keys.size), dev_zeros_u32(keys.size)
    g.insert(dev_u64(keys), ok, kicks)
    _check_concurrent(g, r, keys, ok, kicks, D)
    g.close()


@pytest.mark.parametrize("b,f,ev", [(4, 8, 0), (16, 16, 0), (4, 16, 1), (32, 32, 0)])
def test_insert_overfull_accounts_for_every_dropped_tag(cf, b, f, ev):
    """Far past capacity: failures happen under heavy contention; every
    dropped fingerprint is logged and the multiset still balances."""
    m = 1 << 5
    g, r = _pair(cf, m, b, f, ev=ev, D=4, seed=9)
    keys = K.keys(9, 0, 3 * m * b)
    ok, kicks = dev_zeros_u8(keys.size), dev_zeros_u32(keys.size)
    g.insert(dev_u64(keys), ok, kicks)
    assert g.failures() > 0
    _check_concurrent(g, r, keys, ok, kicks, 4)
    g.close()


def test_insert_contention_on_few_buckets(cf):
    """Many keys on very few buckets with shared fingerprints: CAS retries."""
    m, b, f = 1, 32, 8
    g, r = _pair(cf, m, b, f, D=3, seed=2)
    keys = np.concatenate([K.keys(2, 0, 20)] * 5)  # duplicates too
    ok, kicks = dev_zeros_u8(keys.size), dev_zeros_u32(keys.size)
    g.insert(dev_u64(keys), ok, kicks)
    _check_concurrent(g, r, keys, ok, kicks, 3)
    assert g.count() == 32
    g.close()


def test_insert_edge_keys_and_empty_batch(cf):
    g, r = _pair(cf, 1 << 10, 8, 16)
    g.insert(torch.empty(0, dtype=torch.int64, device="cuda"))
    assert g.count() == 0
    keys = np.array([0, 2**64 - 1, 1, 2**63, 0, 0], dtype=np.uint64)
    ok, kicks = dev_zeros_u8(keys.size), dev_zeros_u32(keys.size)
    g.insert(dev_u64(keys), ok, kicks)
    _check_concurrent(g, r, keys, ok, kicks, 128)
    found = g.query(dev_u64(keys)).cpu().numpy()
    assert found.all()
    g.close()


def test_insert_multi_pass_grid_then_delete(cf):
    """Grid of one block per CU, ragged batch; then concurrent deletes of a
    half: the remaining multiset is the other half's, none lost."""
    m, b, f = 1 << 14, 16, 16
    seed = 11
    g, r = _pair(cf, m, b, f, seed=seed, grid_per_cu=1)
    n = int(0.95 * m * b)
    keys = K.keys(seed, 0, n)
    ok, kicks = dev_zeros_u8(n), dev_zeros_u32(n)
    g.insert(dev_u64(keys), ok, kicks)
    _check_concurrent(g, r, keys, ok, kicks, 128)
    assert g.failures() == 0
    idx = K.seeded_subset(seed, n, n // 2)
    dok = dev_zeros_u8(idx.size)
    g.delete(dev_u64(keys[idx]), dok)
    assert dok.cpu().numpy().all()
    rest = np.setdiff1d(np.arange(n), idx)
    r.load_words(_table(g))
    assert g.count() == r.count == rest.size
    assert multiset_equal(r.stored_groups(), r.key_groups(keys[rest]))
    assert g.query(dev_u64(keys[rest])).cpu().numpy().all()
    g.close()


# ------------------------------------------------------------- whole config

def test_2e18_buckets_b4_f16_end_to_end(cf):
    """2^18 buckets x 4 slots, f = 16, fmix64: insert 943,718 keys (LF 0.9),
    query them plus 10^6 negatives, delete a seeded half, query again.
    GPU results are compared with the oracle run on the GPU's own table."""
    seed = K.workload_seed(0)
    m, b, f, n = 1 << 18, 4, 16, 943_718
    g, r = _pair(cf, m, b, f, seed=seed)
    pos = K.keys(seed, 0, n)
    neg = K.negatives(seed, 0, 1_000_000)
    # positives and negatives interleaved in a seeded random order
    qkeys = np.concatenate([pos, neg])[K.seeded_permutation(seed, n + neg.size)]
    ok, kicks = dev_zeros_u8(n), dev_zeros_u32(n)
    g.insert(dev_u64(pos), ok, kicks)
    _check_concurrent(g, r, pos, ok, kicks, 128)
    assert g.failures() == 0
    got = g.query(dev_u64(qkeys)).cpu().numpy()
    assert np.array_equal(got, r.query_batch(qkeys))
    fp_count = int(g.query(dev_u64(neg)).cpu().numpy().sum())
    eps = r.table_fpr()
    assert abs(fp_count - eps * neg.size) <= 5 * np.sqrt(eps * neg.size) + 1
    half = pos[K.seeded_subset(seed, n, n // 2)]
    dok = dev_zeros_u8(half.size)
    g.delete(dev_u64(half), dok)
    assert np.array_equal(dok.cpu().numpy(), r.delete_batch(half))
    assert np.array_equal(_table(g), r.words())
    got2 = g.query(dev_u64(qkeys)).cpu().numpy()
    assert np.array_equal(got2, r.query_batch(qkeys))
    g.close()


# ------------------------------------------------------------- error paths

def test_invalid_batches_raise(cf):
    g = cf.CuckooFilter(1 << 8, 16, 16)
    k = dev_u64(K.keys(1, 0, 16))
    assert cf.LIB.cf_query(g.handle, None, 5, None, None) == cf.CF_EINVAL
    assert cf.LIB.cf_query(g.handle, k.data_ptr(), 5, None, None) == cf.CF_EINVAL
    # keys must be 8-byte aligned
    assert cf.LIB.cf_insert(g.handle, k.data_ptr() + 4, 3, None, None, None) == cf.CF_EINVAL
    with pytest.raises(cf.CfError, match="CF_EINVAL"):
        cf.cf_export(g.handle, torch.empty(3, dtype=torch.int64, device="cuda"), 24)
    assert g.count() == 0
    g.close()


def test_table_in_caller_memory(cf):
    """cf_create_in: the caller's tensor is the table (zeroed, filled by the
    inserts, exported identically), answers match a library-owned table, and
    the tensor outlives the filter."""
    m, b, f = 1 << 12, 16, 16
    nbytes = cf.cf_table_bytes(cf.make_params(m, b, f))
    buf = torch.full((nbytes + 256,), 0x5A, dtype=torch.uint8, device="cuda")
    table = buf[256:]  # an offset view, 16-byte aligned
    g = cf.CuckooFilter(m, b, f, seed=3, table=table)
    ref = cf.CuckooFilter(m, b, f, seed=3)
    keys = dev_u64(K.keys(31, 0, int(0.9 * m * b)))
    g.insert(keys)
    ref.insert(keys)
    torch.cuda.synchronize()
    assert g.count() == ref.count() == keys.numel()
    assert torch.equal(table.view(torch.int64), g.export_table())
    probe = torch.cat([keys, dev_u64(K.negatives(31, 0, 50_000))])
    assert torch.equal(g.query(probe), ref.query(probe))
    assert bool((buf[:256] == 0x5A).all())  # nothing outside the table was touched
    snap = table.clone()
    g.close()
    ref.close()
    assert torch.equal(table, snap)  # still valid after cf_destroy
    with pytest.raises(cf.CfError):
        cf.CuckooFilter(m, b, f, table=buf[8:8 + nbytes])  # misaligned
    with pytest.raises(cf.CfError):
        cf.CuckooFilter(m, b, f, table=buf[:nbytes // 2])  # too small


def test_xor_largest_bucket_count(cf):
    """m = 2^32 buckets of 4 x 8 bits (16 GiB), the most the XOR placement
    takes: keys inserted one per launch land in exactly the oracle's slots,
    so i1 = (lower 32 hash bits) & (m - 1) and the alternate bucket agree over
    the whole 32-bit range; every key is found; deleting half of them leaves
    exactly the oracle's slots."""
    m, b, f = 1 << 32, 4, 8
    g, r = _pair(cf, m, b, f, seed=29)
    keys = K.keys(29, 0, 300)
    want = r.insert_batch(keys)
    d_keys = dev_u64(keys)
    ok = dev_zeros_u8(keys.size)
    for i in range(keys.size):
        g.insert(d_keys[i:i + 1], ok[i:i + 1])
    assert np.array_equal(ok.cpu().numpy(), want) and g.count() == r.count == keys.size

    def check_slots():
        words = g.export_table()  # int64 view of the packed table, on the device
        step = 1 << 30  # torch.nonzero over 2^31 elements overflows; scan in parts
        parts = [torch.nonzero(words[o:o + step]).flatten() + o
                 for o in range(0, words.numel(), step)]
        nz = torch.cat(parts)
        vals = host_u64(words[nz])
        nz = nz.cpu().numpy()
        del words, parts
        torch.cuda.synchronize()
        slots = 0
        for w, v in zip(nz, vals):
            for k in range(8):  # 8-bit slots, 8 per word; global slot = bucket * 4 + s
                g_slot = int(w) * 8 + k
                tag = (int(v) >> (8 * k)) & 0xFF
                assert tag == r.slot(g_slot // 4, g_slot % 4)
                slots += tag != 0
        assert slots == r.count

    check_slots()
    assert g.query(d_keys).cpu().numpy().all()
    half = keys[:150]
    dok = dev_zeros_u8(half.size)
    g.delete(dev_u64(half), dok)
    assert np.array_equal(dok.cpu().numpy(), r.delete_batch(half))
    assert g.count() == r.count == keys.size - half.size
    check_slots()
    g.close()
    r.close()


def test_table_larger_than_the_device_is_refused(cf):
    """2^32 buckets x 32 slots x 32 bits is 512 GiB, more than the device
    holds: cf_create reports CF_ENOMEM and leaves no error behind, so the next
    filter works; a set whose tables do not fit is refused the same way and
    frees what it had allocated."""
    with pytest.raises(cf.CfError, match="CF_ENOMEM"):
        cf.CuckooFilter(1 << 32, 32, 32)
    g, r = _pair(cf, 1 << 10, 16, 16, seed=3)
    keys = K.keys(3, 0, 1000)
    ok = dev_zeros_u8(keys.size)
    g.insert(dev_u64(keys), ok)
    assert bool(ok.all()) and g.count() == r.count + 1000
    assert g.query(dev_u64(keys)).cpu().numpy().all()
    g.close()
    r.close()
    big = [cf.make_params(1 << 31, 32, 32, seed=i) for i in range(2)]  # 2 x 256 GiB
    with pytest.raises(cf.CfError, match="CF_ENOMEM"):
        cf.CuckooFilterSet(big, 1024)
    torch.cuda.empty_cache()  # earlier tests' cached tensors do not count
    free, _ = torch.cuda.mem_get_info()
    assert free > 200 * 2**30  # nothing of the refused set stayed allocated
    s = cf.CuckooFilterSet([cf.make_params(1 << 10, 16, 16)], 1024)
    s.close()
