"""GPU checks at the benchmark's full sizes, in the launch configuration the
benchmark times (same entry points, batch sizes and grid).

The oracle cannot replay 2 x 10^9 sequential inserts in test time, so these
tests check properties that hold at any size, computed by the oracle from the
keys and from the table the GPU built:
  * the stored multiset of (bucket pair, fingerprint) equals the inserted
    keys' minus the dropped tags (order-independent 64-bit digests);
  * occupancy count, zero false negatives when nothing was dropped, and the
    false-positive rate against Eq. (4).
On the 4 GiB and the 3 GiB offset tables the oracle also takes the GPU's table
as it is after the fill and answers 2^20 mixed queries and a 2^20-key delete,
which are compared with the GPU's element by element (flags, and the whole
table after the delete, bit for bit).
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from oracle import OracleFilter
from gpu_util import dev_u64, dev_zeros_u8, host_u64
from workloads import keys as K

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
M64 = (1 << 64) - 1
THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def cf():
    import paper_2603_15486_amd as mod
    return mod


def _digest_keys(ref, seed, start, n, chunk=1 << 23):
    """Digest of the groups of keys (seed, start .. start+n-1), computed by the
    oracle on disjoint chunks in parallel threads (ctypes drops the GIL)."""
    def work(off):
        return ref.digest_keys(K.keys(seed, start + off, min(chunk, n - off)))
    with ThreadPoolExecutor(THREADS) as ex:
        return sum(ex.map(work, range(0, n, chunk))) & M64


def _digest_table(ref, chunk=1 << 22):
    def work(j0):
        return ref.digest_table(j0, min(ref.m, j0 + chunk))
    with ThreadPoolExecutor(THREADS) as ex:
        return sum(ex.map(work, range(0, ref.m, chunk))) & M64


def _elementwise(cf, g, ref, seed, lo, hi, n_ops=1 << 20):
    """With the oracle holding the GPU's table: n_ops mixed queries (half
    inserted keys from counters [0, hi), half negatives) compared per key, then
    one delete of n_ops distinct inserted keys from counters [lo, hi), run on
    the GPU as the benchmark runs it, compared per key and by the whole
    table, bit for bit.  The deleted keys are inserted again afterwards."""
    rng = np.random.default_rng(seed ^ 0xE1E7)
    pos = K.splitmix64(seed, rng.integers(0, hi, n_ops // 2, dtype=np.uint64))
    q = np.concatenate([pos, K.negatives(seed, 1 << 40, n_ops - n_ops // 2)])
    q = q[rng.permutation(q.size)]
    got = g.query(dev_u64(q)).cpu().numpy()
    want = ref.query_batch(q)
    assert np.array_equal(got, want)
    assert int(want[np.isin(q, pos)].min()) == 1
    ctr = np.unique(rng.integers(lo, hi, n_ops + n_ops // 8, dtype=np.uint64))
    ctr = ctr[rng.permutation(ctr.size)[:n_ops]]
    assert ctr.size == n_ops
    dk = K.splitmix64(seed, ctr)
    d_dk = dev_u64(dk)
    dok = dev_zeros_u8(n_ops)
    g.delete(d_dk, dok)
    want = ref.delete_batch(dk)
    assert bool(want.all()) and np.array_equal(dok.cpu().numpy(), want)
    assert np.array_equal(host_u64(g.export_table()), ref.words(copy=False))
    ok = dev_zeros_u8(n_ops)
    g.insert(d_dk, ok)
    torch.cuda.synchronize()
    assert bool(ok.all())


def _eq4(b, f, alpha):
    return 1.0 - (1.0 - 2.0 ** -f) ** (2 * b * alpha)


def _fill(cf, g, seed, start, n, batch, lost_ok=False):
    buf = torch.empty(batch, dtype=torch.int64, device="cuda")
    ok = dev_zeros_u8(batch)
    placed = 0
    for off in range(0, n, batch):
        cnt = min(batch, n - off)
        cf.cf_keygen(buf[:cnt], seed, start + off)
        g.insert(buf[:cnt], ok[:cnt])
        placed += int(ok[:cnt].sum())
    torch.cuda.synchronize()
    return placed


def _all_found(cf, g, seed, start, n, batch=1 << 26):
    buf = torch.empty(batch, dtype=torch.int64, device="cuda")
    missing = 0
    for off in range(0, n, batch):
        cnt = min(batch, n - off)
        cf.cf_keygen(buf[:cnt], seed, start + off)
        found = g.query(buf[:cnt])
        missing += int(cnt - found.sum())
    return missing


def test_large_table_full_size(cf):
    """2^27 buckets x 16 slots x 16-bit (4 GiB), inserts in batches of 2^24
    up to LF 0.95, queries in batches of 2^26, then one delete of 2^28 keys."""
    m, b, f = 1 << 27, 16, 16
    seed = K.workload_seed(1)
    n = int(0.95 * m * b)
    g = cf.CuckooFilter(m, b, f, max_evict=128, seed=seed)
    placed = _fill(cf, g, seed, 0, n, 1 << 24)
    assert g.failures() == 0 and placed == n and g.count() == n
    assert _all_found(cf, g, seed, 0, n) == 0
    # false positives on 2^26 fresh negatives, against Eq. (4)
    neg = torch.empty(1 << 26, dtype=torch.int64, device="cuda")
    cf.cf_keygen(neg, seed, K.NEG_BASE)
    rate = float(g.query(neg).float().mean())
    eps = _eq4(b, f, n / (m * b))
    sigma = math.sqrt(eps / neg.numel())
    assert abs(rate - eps) < 5 * sigma + 0.05 * eps
    del neg
    # stored multiset == inserted keys' groups
    ref = OracleFilter(m, b, f, max_evict=128, seed=seed)
    words = host_u64(g.export_table())
    ref.load_words_nocount(words)
    del words
    assert _digest_table(ref) == _digest_keys(ref, seed, 0, n)
    # element by element against the oracle on the GPU's own table
    print("full size: element-wise queries and delete, 4 GiB table", flush=True)
    _elementwise(cf, g, ref, seed, 1 << 28, n)
    assert g.count() == n and g.failures() == 0
    # delete 2^28 inserted keys in one batch
    nd = 1 << 28
    dk = torch.empty(nd, dtype=torch.int64, device="cuda")
    cf.cf_keygen(dk, seed, 0)
    dok = dev_zeros_u8(nd)
    g.delete(dk, dok)
    torch.cuda.synchronize()
    assert bool(dok.all()) and g.count() == n - nd
    del dk, dok
    assert _all_found(cf, g, seed, nd, n - nd) == 0
    words = host_u64(g.export_table())
    ref.load_words_nocount(words)
    del words
    assert _digest_table(ref) == _digest_keys(ref, seed, nd, n - nd)
    ref.close()
    g.close()


@pytest.mark.parametrize("evict,D", [(0, 4), (1, 500)])
def test_eviction_stress_full_size(cf, evict, D):
    """2^24 buckets x 4 slots x 8-bit, filled towards LF 0.98 in 1% bands:
    failures are expected; every dropped fingerprint is logged and the stored
    multiset equals the inserted keys' minus the logged ones."""
    m, b, f = 1 << 24, 4, 8
    seed = K.workload_seed(2)
    n = int(0.98 * m * b)
    band = int(0.01 * m * b)
    g = cf.CuckooFilter(m, b, f, evict=evict, max_evict=D, seed=seed, lost_capacity=1 << 22)
    placed = _fill(cf, g, seed, 0, n, band)
    fails = g.failures()
    assert placed == n - fails
    assert g.count() == n - fails
    lb, lt = g.lost(1 << 22)
    assert len(lb) == fails
    ref = OracleFilter(m, b, f, evict=evict, max_evict=D, seed=seed)
    ref.load_words_nocount(host_u64(g.export_table()))
    want = (_digest_keys(ref, seed, 0, n) - ref.digest_pairs(lb, lt)) & M64
    assert _digest_table(ref) == want
    # a false negative needs a dropped fingerprint
    assert _all_found(cf, g, seed, 0, n) <= fails
    ref.close()
    g.close()


def test_offset_placement_full_size(cf):
    """The offset placement at 0.75 * 2^27 buckets x 16 x 16-bit (3 GiB, a
    bucket count XOR cannot have), filled to LF 0.95 in batches of 2^24: the
    (primary, alternate, fingerprint) multiset digest, zero false negatives,
    FPR against 1 - (1 - 2^-(f-1))^(b alpha), then a delete of 2^27 keys."""
    m, b, f = 3 << 25, 16, 16
    seed = K.workload_seed(1) + 7
    n = int(0.95 * m * b)
    g = cf.CuckooFilter(m, b, f, max_evict=128, seed=seed, placement=cf.CF_PLACE_OFFSET)
    placed = _fill(cf, g, seed, 0, n, 1 << 24)
    assert g.failures() == 0 and placed == n and g.count() == n
    assert _all_found(cf, g, seed, 0, n) == 0
    neg = torch.empty(1 << 26, dtype=torch.int64, device="cuda")
    cf.cf_keygen(neg, seed, K.NEG_BASE)
    rate = float(g.query(neg).float().mean())
    alpha = n / (m * b)
    eps = 1.0 - (1.0 - 2.0 ** -(f - 1)) ** (b * alpha)
    sigma = math.sqrt(eps / neg.numel())
    assert abs(rate - eps) < 5 * sigma + 0.05 * eps
    del neg
    ref = OracleFilter(m, b, f, max_evict=128, seed=seed, placement=oracle.PLACE_OFFSET)
    ref.load_words_nocount(host_u64(g.export_table()))
    assert _digest_table(ref) == _digest_keys(ref, seed, 0, n)
    print("full size: element-wise queries and delete, 3 GiB offset table", flush=True)
    _elementwise(cf, g, ref, seed, 1 << 27, n)
    assert g.count() == n and g.failures() == 0
    nd = 1 << 27
    dk = torch.empty(nd, dtype=torch.int64, device="cuda")
    cf.cf_keygen(dk, seed, 0)
    dok = dev_zeros_u8(nd)
    g.delete(dk, dok)
    torch.cuda.synchronize()
    assert bool(dok.all()) and g.count() == n - nd
    del dk, dok
    assert _all_found(cf, g, seed, nd, n - nd) == 0
    ref.load_words_nocount(host_u64(g.export_table()))
    assert _digest_table(ref) == _digest_keys(ref, seed, nd, n - nd)
    ref.close()
    g.close()
