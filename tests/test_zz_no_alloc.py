"""cf_insert_noalloc (the insert that allocates nothing: its eviction queue is
the library's fixed per-GPU array) against cf_insert, through the C ABI.

Two calls in a row on the same filters, the second with a smaller batch:
  * one key per launch (deterministic): tables, flags, kicks and dropped-tag
    logs bit-identical to cf_insert's;
  * whole batches (concurrent): the stored (bucket pair, fingerprint)
    multiset equals cf_insert's and the oracle's key-derived one, counts and
    failures agree, no false negatives.
Keys are chosen so that many reach the eviction search, which is the part
that uses the queue.  Sizes beyond the limit are refused before any work.
"""
import numpy as np
import pytest

import oracle
from oracle import OracleFilter
from gpu_util import dev_u64, dev_zeros_u8, dev_zeros_u32, expected_groups, host_u64, \
    multiset_equal
from workloads import keys as K

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cf():
    import paper_2603_15486_amd as mod
    return mod


def _table(g):
    torch.cuda.synchronize()
    return host_u64(g.export_table())


def _run(g, keys, noalloc):
    ok, kicks = dev_zeros_u8(keys.size), dev_zeros_u32(keys.size)
    (g.insert_noalloc if noalloc else g.insert)(dev_u64(keys), ok, kicks)
    torch.cuda.synchronize()
    return ok.cpu().numpy(), kicks.cpu().numpy()


@pytest.mark.parametrize("b,f,ev", [(4, 16, 0), (16, 16, 0), (8, 8, 1)])
def test_noalloc_serial_bit_identical(cf, b, f, ev):
    """One key per launch, two rounds (the second shorter): bit-identical
    tables, flags, kicks and lost logs."""
    m = 1 << 6
    seed = 77 + b + f + ev
    D = 128 if ev == oracle.EVICT_BFS else 500
    ga = cf.CuckooFilter(m, b, f, evict=ev, max_evict=D, seed=seed)
    gb = cf.CuckooFilter(m, b, f, evict=ev, max_evict=D, seed=seed)
    keys = K.keys(seed, 0, int(0.97 * m * b))
    for part in (keys[:int(0.9 * m * b)], keys[int(0.9 * m * b):]):
        for k in part:
            one = np.array([k], dtype=np.uint64)
            oa, ka = _run(ga, one, False)
            ob, kb = _run(gb, one, True)
            assert oa[0] == ob[0] and ka[0] == kb[0]
        assert np.array_equal(_table(ga), _table(gb))
        assert ga.count() == gb.count() and ga.failures() == gb.failures()
        la, lb = ga.lost(), gb.lost()
        assert np.array_equal(la[0], lb[0]) and np.array_equal(la[1], lb[1])
    ga.close()
    gb.close()


@pytest.mark.parametrize("m,b,f,ev", [(1 << 16, 16, 16, 0), (1 << 18, 4, 16, 0),
                                      (1 << 15, 8, 8, 1)])
def test_noalloc_batches_match_insert(cf, m, b, f, ev):
    """Two whole-batch calls in a row, the second smaller: same multiset,
    count and failures as cf_insert, and the oracle's key-derived multiset."""
    seed = 900 + b + f + ev
    D = 128 if ev == oracle.EVICT_BFS else 500
    ga = cf.CuckooFilter(m, b, f, evict=ev, max_evict=D, seed=seed)
    gb = cf.CuckooFilter(m, b, f, evict=ev, max_evict=D, seed=seed)
    ref = OracleFilter(m, b, f, evict=ev, max_evict=D, seed=seed)
    slots = m * b
    lf_hi = 0.9 if b == 4 else 0.95
    n1 = min(int(0.85 * slots), cf.CF_NOALLOC_MAX_KEYS)
    n2 = int(lf_hi * slots) - n1
    assert 0 < n2 < n1
    allk = K.keys(seed, 0, n1 + n2)
    done = 0
    for n in (n1, n2):
        part = allk[done:done + n]
        oa, ka = _run(ga, part, False)
        ob, kb = _run(gb, part, True)
        done += n
        seen = allk[:done]
        fa, fb = ga.failures(), gb.failures()
        for g, okv, kk, fails in ((ga, oa, ka, fa), (gb, ob, kb, fb)):
            assert kk.max(initial=0) <= D
            words = _table(g)
            ref.load_words(words)
            assert ref.count == g.count() == done - fails
            lost = g.lost()
            assert len(lost[0]) == fails
            assert multiset_equal(ref.stored_groups(), expected_groups(ref, seen, lost=lost))
        if fa == 0 and fb == 0:
            assert oa.all() and ob.all()
            assert multiset_equal(_groups(ref, _table(ga)), _groups(ref, _table(gb)))
            assert ga.query(dev_u64(seen)).cpu().numpy().all()
            assert gb.query(dev_u64(seen)).cpu().numpy().all()
    ga.close()
    gb.close()
    ref.close()


def _groups(ref, words):
    ref.load_words(words)
    return ref.stored_groups()


def test_noalloc_rejects_oversize_before_any_work(cf):
    g = cf.CuckooFilter(1 << 10, 16, 16, seed=3)
    keys = torch.zeros(cf.CF_NOALLOC_MAX_KEYS + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(RuntimeError, match="limit"):
        g.insert_noalloc(keys)
    torch.cuda.synchronize()
    assert g.count() == 0
    g.insert_noalloc(keys[:0])
    assert g.count() == 0
    g.close()
