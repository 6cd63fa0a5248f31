"""GPU parity of filter sets driven by mixed batches (include/cf_set.h).

Batch semantics under test: per filter, every query sees the state before the
batch, then the batch's deletes apply, then its inserts.  Queries and delete
flags depend only on the stored multiset, so they are compared bit-exactly
with the oracle; insert placement is concurrent, so the stored multiset is
compared.  The same batch run alone per filter through the single-filter API
must give the same results ("alone and in the mix"), and a captured graph
replayed on batches of several sizes must match eager execution.
"""
import numpy as np
import pytest

import oracle
from oracle import OracleFilter
from gpu_util import GEOMS, dev_u64, expected_groups, host_u64, multiset_equal
from workloads import keys as K

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

QUERY, DELETE, INSERT = 0, 1, 2


@pytest.fixture(scope="module")
def cf():
    import paper_2603_15486_amd as mod
    return mod


def _specs(seed, nf):
    """Filter specs (m, b, f, hash, evict, D, seed) with mixed geometries."""
    rng = np.random.default_rng(seed)
    geoms = [(8, 16), (16, 16), (4, 8), (32, 32), (8, 8), (16, 32)]
    out = []
    for i in range(nf):
        b, f = geoms[i % len(geoms)]
        m = 1 << int(rng.integers(8, 12))
        hk = int(rng.integers(0, 2))
        ev = int(rng.integers(0, 2))
        out.append((m, b, f, hk, ev, 128 if ev == 0 else 500, 1000 + i))
    return out


def _build(cf, specs, max_batch, fill_seed):
    """A set plus one oracle per filter, both holding the same prefilled table."""
    params = [cf.make_params(m, b, f, hk, ev, D, sd) for (m, b, f, hk, ev, D, sd) in specs]
    s = cf.CuckooFilterSet(params, max_batch)
    refs, pre = [], []
    for fid, (m, b, f, hk, ev, D, sd) in enumerate(specs):
        r = OracleFilter(m, b, f, hash_kind=hk, evict=ev, max_evict=D, seed=sd)
        keys = K.keys(fill_seed + fid, 0, int(0.6 * m * b))
        r.insert_batch(keys)
        s.import_table(fid, dev_u64(r.words()))
        refs.append(r)
        pre.append(keys)
    torch.cuda.synchronize()
    return s, refs, pre


def _batch(specs, pre, n, seed):
    """A mixed batch: 60% query (half positive), 30% insert (fresh keys), 10%
    delete (distinct prefilled keys), filters drawn in proportion to size."""
    rng = np.random.default_rng(seed)
    sizes = np.array([m * b for (m, b, *_rest) in specs], dtype=np.float64)
    fids = rng.choice(len(specs), size=n, p=sizes / sizes.sum()).astype(np.uint32)
    u = rng.random(n)
    ops = np.where(u < 0.6, QUERY, np.where(u < 0.9, INSERT, DELETE)).astype(np.uint8)
    keys = np.zeros(n, dtype=np.uint64)
    fresh = K.keys(seed + 77, 0, n)
    neg = K.negatives(seed, 0, n)
    used = [set() for _ in specs]
    for i in range(n):
        f = int(fids[i])
        if ops[i] == INSERT:
            keys[i] = fresh[i]
        elif ops[i] == QUERY:
            keys[i] = pre[f][rng.integers(0, pre[f].size)] if rng.random() < 0.5 else neg[i]
        else:
            cand = [j for j in rng.integers(0, pre[f].size, 8) if j not in used[f]]
            if not cand:
                ops[i], keys[i] = QUERY, neg[i]
                continue
            used[f].add(int(cand[0]))
            keys[i] = pre[f][cand[0]]
    return ops, fids, keys


def _forget_deleted(pre, ops, fids, keys):
    """Drop a batch's deleted keys from the prefilled key lists, so a later
    batch deletes only keys still stored.  Deleting a key again could take
    the copy of another key with the same bucket pair and fingerprint, and two
    deletes then compete for one copy: which of them succeeds depends on the
    order they run in (Alg. 3 on concurrent threads), and no exact flag
    comparison holds."""
    for f in range(len(pre)):
        gone = keys[(ops == DELETE) & (fids == f)]
        if gone.size:
            pre[f] = pre[f][~np.isin(pre[f], gone)]


def _expected_query_delete(refs, ops, fids, keys):
    """Oracle results for queries (pre-batch state) and deletes, applied to
    the oracles in place; returns the expected result array (inserts 1)."""
    res = np.ones(keys.size, dtype=np.uint8)
    for i in np.nonzero(ops == QUERY)[0]:
        res[i] = refs[fids[i]].query(int(keys[i]))
    for i in np.nonzero(ops == DELETE)[0]:
        res[i] = refs[fids[i]].delete(int(keys[i]))
    return res


def _check_tables(cf, s, refs, ops, fids, keys, results):
    """After the batch: each filter's stored multiset equals the post-delete
    oracle multiset plus the batch's inserted keys minus dropped tags."""
    counts = s.counts()
    fails = s.failures()
    for fid, r in enumerate(refs):
        ins = keys[(ops == INSERT) & (fids == fid)]
        lo0, hi0, t0 = r.stored_groups()
        lo1, hi1, t1 = r.key_groups(ins)
        want = (np.concatenate([lo0, lo1]), np.concatenate([hi0, hi1]),
                np.concatenate([t0, t1]))
        g = OracleFilter(r.m, r.b, r.f, hash_kind=r.hash_kind)
        g.load_words(host_u64(s.export_table(fid)))
        if fails[fid] == 0:
            assert multiset_equal(g.stored_groups(), want), f"filter {fid}"
        assert counts[fid] == g.count, f"filter {fid}"
        g.close()


@pytest.mark.parametrize("streams,wave_bfs", [(1, 0), (0, 0), (8, 0), (0, 1)])
def test_set_batch_matches_oracle(cf, streams, wave_bfs):
    """streams: class chains one after another (1), the default, and eight
    at once (the 14 filters fall into 12 classes); the breadth-first search
    one lane or one wave per key."""
    specs = _specs(1, 14)
    s, refs, pre = _build(cf, specs, 1 << 16, 500)
    s.streams = streams
    s.set_shape(wave_bfs=wave_bfs)
    assert s.streams == streams and s.shape["wave_bfs"] == wave_bfs
    ops, fids, keys = _batch(specs, pre, 40_000, 9)
    # a few invalid operations
    ops[5], fids[17] = 7, 10_000
    res = s.execute(torch.from_numpy(ops).cuda(), torch.from_numpy(fids.view(np.int32)).cuda(),
                    dev_u64(keys)).cpu().numpy()
    assert res[5] == 0xFF and res[17] == 0xFF
    valid = np.ones(keys.size, dtype=bool)
    valid[[5, 17]] = False
    want = _expected_query_delete(refs, np.where(valid, ops, 9), fids, keys)
    qd = valid & (ops != INSERT)
    assert np.array_equal(res[qd], want[qd])
    assert (res[valid & (ops == INSERT)] == 1).all() or s.failures().sum() > 0
    ops2 = np.where(valid, ops, 9).astype(np.uint8)
    _check_tables(cf, s, refs, ops2, fids, keys, res)
    s.close()


@pytest.mark.parametrize("chunk,streams", [(64, 1), (512, 0), (4096, 8), (256, 3)])
def test_set_alone_equals_mix(cf, chunk, streams):
    """Each operation's result is the same in the mixed batch and when its
    filter's operations run alone through the single-filter entry points."""
    specs = _specs(2, 9)
    s, refs, pre = _build(cf, specs, 1 << 15, 600)
    s.chunk = chunk
    s.streams = streams
    ops, fids, keys = _batch(specs, pre, 20_000, 10)
    res = s.execute(torch.from_numpy(ops).cuda(), torch.from_numpy(fids.view(np.int32)).cuda(),
                    dev_u64(keys)).cpu().numpy()
    assert s.failures().sum() == 0
    alone = np.zeros_like(res)
    for fid, (m, b, f, hk, ev, D, sd) in enumerate(specs):
        g = cf.CuckooFilter(m, b, f, hash=hk, evict=ev, max_evict=D, seed=sd)
        g.import_table(dev_u64(refs[fid].words()))
        for kind in (QUERY, DELETE, INSERT):
            idx = np.nonzero((fids == fid) & (ops == kind))[0]
            if idx.size == 0:
                continue
            out = torch.zeros(idx.size, dtype=torch.uint8, device="cuda")
            k = dev_u64(keys[idx])
            if kind == QUERY:
                g.query(k, out)
            elif kind == DELETE:
                g.delete(k, out)
            else:
                g.insert(k, out)
            alone[idx] = out.cpu().numpy()
        solo = OracleFilter(m, b, f, hash_kind=hk)
        solo.load_words(host_u64(g.export_table()))
        mixd = OracleFilter(m, b, f, hash_kind=hk)
        mixd.load_words(host_u64(s.export_table(fid)))
        assert multiset_equal(solo.stored_groups(), mixd.stored_groups())
        g.close()
    assert np.array_equal(res, alone)
    s.close()


def test_set_graph_replays_match_eager(cf):
    """One captured graph, three batches of different sizes through fixed
    buffers; eager execution on a twin set with synchronisation between
    replays; every replay's results and tables must match.  The graph runs
    eight class chains at once, the eager twin one after another."""
    specs = _specs(3, 10)
    nmax = 1 << 15
    a, refs, pre = _build(cf, specs, nmax, 700)
    b, _, _ = _build(cf, specs, nmax, 700)
    a.chunk = 1024
    a.streams = 8
    b.streams = 1
    d_ops = torch.zeros(nmax, dtype=torch.uint8, device="cuda")
    d_fids = torch.zeros(nmax, dtype=torch.int32, device="cuda")
    d_keys = torch.zeros(nmax, dtype=torch.int64, device="cuda")
    d_res = torch.zeros(nmax, dtype=torch.uint8, device="cuda")
    d_n = torch.zeros(1, dtype=torch.int64, device="cuda")
    graph = a.graph(d_ops, d_fids, d_keys, d_n, d_res)
    for step, n in enumerate((nmax, 5000, 12_345)):
        ops, fids, keys = _batch(specs, pre, n, 100 + step)
        _forget_deleted(pre, ops, fids, keys)
        d_ops[:n].copy_(torch.from_numpy(ops))
        d_fids[:n].copy_(torch.from_numpy(fids.view(np.int32)))
        d_keys[:n].copy_(torch.from_numpy(keys.view(np.int64)))
        d_n.fill_(n)
        cf.cf_graph_launch(graph)
        torch.cuda.synchronize()
        got = d_res[:n].cpu().numpy()
        want = b.execute(torch.from_numpy(ops).cuda(),
                         torch.from_numpy(fids.view(np.int32)).cuda(),
                         dev_u64(keys)).cpu().numpy()
        assert np.array_equal(got, want), f"replay {step}"
        for fid in range(len(specs)):
            ga = OracleFilter(specs[fid][0], specs[fid][1], specs[fid][2],
                              hash_kind=specs[fid][3])
            gb = OracleFilter(specs[fid][0], specs[fid][1], specs[fid][2],
                              hash_kind=specs[fid][3])
            ga.load_words(host_u64(a.export_table(fid)))
            gb.load_words(host_u64(b.export_table(fid)))
            assert multiset_equal(ga.stored_groups(), gb.stored_groups())
            ga.close()
            gb.close()
        assert np.array_equal(a.counts(), b.counts())
    a.close()
    b.close()


def test_set_many_filters_counts(cf):
    """More filters than the LDS tally holds: per-operation atomics path."""
    nf = 5000
    params = [cf.make_params(1 << 2, 8, 16, seed=i) for i in range(nf)]
    s = cf.CuckooFilterSet(params, 1 << 16)
    rng = np.random.default_rng(4)
    n = 60_000
    fids = rng.integers(0, nf, n).astype(np.uint32)
    keys = K.keys(5, 0, n)
    ops = np.full(n, INSERT, dtype=np.uint8)
    res = s.execute(torch.from_numpy(ops).cuda(), torch.from_numpy(fids.view(np.int32)).cuda(),
                    dev_u64(keys)).cpu().numpy()
    counts = s.counts()
    fails = s.failures()
    per = np.bincount(fids, minlength=nf)
    assert np.array_equal(counts + fails, per)
    assert int(res.sum()) == int(counts.sum())
    # spot-check a few filters' tables against their counts
    for fid in (0, 1, 4999):
        g = OracleFilter(4, 8, 16)
        g.load_words(host_u64(s.export_table(fid)))
        assert g.count == counts[fid]
        g.close()
    s.close()


@pytest.mark.parametrize("wave_bfs", [0, 1])
def test_set_degenerate_filters_serial_bit_exact(cf, wave_bfs):
    """Filters of one, two and three buckets in one set (XOR with i2 = i1, and
    the offset placement at m = 1 and 3), driven one operation per filter per
    batch: 2mb + 3 inserts each, so every filter overflows; then one batch of
    queries over every key and some negatives; then the keys deleted one per
    filter per batch.  Flags, tables, counts, failures and dropped-tag logs
    equal the oracle's sequential run of each filter."""
    XOR, OFF = oracle.PLACE_XOR, oracle.PLACE_OFFSET
    geo = [(1, 4, 8, 0, XOR), (2, 16, 16, 1, XOR), (1, 32, 32, 0, XOR), (2, 8, 8, 0, XOR),
           (1, 8, 16, 0, OFF), (3, 4, 8, 1, OFF), (1, 16, 32, 0, OFF)]
    D = 8
    params = [cf.make_params(m, b, f, hk, oracle.EVICT_BFS, D, 4000 + i, placement=pl)
              for i, (m, b, f, hk, pl) in enumerate(geo)]
    s = cf.CuckooFilterSet(params, 4096)
    s.set_shape(wave_bfs=wave_bfs)
    refs = [OracleFilter(m, b, f, hash_kind=hk, evict=oracle.EVICT_BFS, max_evict=D,
                         seed=4000 + i, placement=pl) for i, (m, b, f, hk, pl) in enumerate(geo)]
    keys = [K.keys(4100 + i, 0, 2 * m * b + 3) for i, (m, b, *_) in enumerate(geo)]

    def serial(kind):
        got = [np.zeros(k.size, dtype=np.uint8) for k in keys]
        for t in range(max(k.size for k in keys)):
            live = [i for i in range(len(geo)) if t < keys[i].size]
            res = s.execute(torch.full((len(live),), kind, dtype=torch.uint8).cuda(),
                            torch.tensor(live, dtype=torch.int32).cuda(),
                            dev_u64(np.array([keys[i][t] for i in live], dtype=np.uint64)))
            res = res.cpu().numpy()
            for j, i in enumerate(live):
                got[i][t] = res[j]
        return got

    got = serial(INSERT)
    fails = s.failures()
    counts = s.counts()
    for i, r in enumerate(refs):
        assert np.array_equal(got[i], r.insert_batch(keys[i])), f"filter {i} insert flags"
        assert np.array_equal(host_u64(s.export_table(i)), r.words()), f"filter {i} table"
        assert fails[i] == r.failures > 0 and counts[i] == r.count
        lb, lt = s.lost(i)
        rb, rt = r.lost()
        assert np.array_equal(lb, rb) and np.array_equal(lt, rt), f"filter {i} lost log"

    qk, qf = [], []
    for i in range(len(geo)):
        qk.append(np.concatenate([keys[i], K.negatives(4200 + i, 0, 300)]))
        qf.append(np.full(qk[-1].size, i, dtype=np.int32))
    qk, qf = np.concatenate(qk), np.concatenate(qf)
    res = s.execute(torch.zeros(qk.size, dtype=torch.uint8).cuda(), torch.from_numpy(qf).cuda(),
                    dev_u64(qk)).cpu().numpy()
    for i, r in enumerate(refs):
        assert np.array_equal(res[qf == i], r.query_batch(qk[qf == i])), f"filter {i} queries"

    got = serial(DELETE)
    counts = s.counts()
    for i, r in enumerate(refs):
        assert np.array_equal(got[i], r.delete_batch(keys[i])), f"filter {i} delete flags"
        assert np.array_equal(host_u64(s.export_table(i)), r.words()), f"filter {i} table"
        assert counts[i] == r.count
        r.close()
    s.close()


@pytest.mark.parametrize("wave_bfs", [0, 1])
def test_set_insert_serial_bit_exact(cf, wave_bfs):
    """Each batch holds one insert per filter, so every filter sees one key
    per launch: the set's insert kernel, with its grouped breadth-first
    probe (2, 4 or 8 candidates' buckets loaded together, or 1 for 128-byte
    buckets; wave_bfs = 0) or its wave probe (one candidate per lane and a
    ballot; wave_bfs = 1), must reproduce the oracle's sequential tables,
    flags, failure counts and dropped-tag logs exactly, up to load 0.99 with
    D = 8."""
    XOR, OFF = oracle.PLACE_XOR, oracle.PLACE_OFFSET
    geo = [(64, 16, 16, 0, XOR), (64, 16, 8, 1, XOR), (64, 4, 8, 0, XOR), (64, 32, 32, 0, XOR),
           (64, 8, 16, 1, XOR), (61, 16, 16, 0, OFF), (61, 8, 8, 1, OFF), (61, 4, 32, 0, OFF),
           (61, 32, 16, 0, OFF), (61, 16, 32, 1, OFF)]
    D = 8
    params = [cf.make_params(m, b, f, hk, oracle.EVICT_BFS, D, 2000 + i, placement=pl)
              for i, (m, b, f, hk, pl) in enumerate(geo)]
    s = cf.CuckooFilterSet(params, 64)
    s.set_shape(wave_bfs=wave_bfs)
    refs, keys = [], []
    for i, (m, b, f, hk, pl) in enumerate(geo):
        refs.append(OracleFilter(m, b, f, hash_kind=hk, evict=oracle.EVICT_BFS, max_evict=D,
                                 seed=2000 + i, placement=pl))
        keys.append(K.keys(2100 + i, 0, int(0.99 * m * b)))
    rounds = max(k.size for k in keys)
    got = [np.zeros(k.size, dtype=np.uint8) for k in keys]
    for t in range(rounds):
        live = [i for i in range(len(geo)) if t < keys[i].size]
        fids = np.array(live, dtype=np.uint32)
        kk = np.array([keys[i][t] for i in live], dtype=np.uint64)
        ops = np.full(len(live), INSERT, dtype=np.uint8)
        res = s.execute(torch.from_numpy(ops).cuda(), torch.from_numpy(fids.view(np.int32)).cuda(),
                        dev_u64(kk)).cpu().numpy()
        for j, i in enumerate(live):
            got[i][t] = res[j]
    fails = s.failures()
    assert fails.sum() > 0  # the search gave up somewhere: the failure path is covered
    for i, r in enumerate(refs):
        want = r.insert_batch(keys[i])
        assert np.array_equal(got[i], want), f"filter {i} flags"
        assert np.array_equal(host_u64(s.export_table(i)), r.words()), f"filter {i} table"
        assert fails[i] == r.failures
        lb, lt = s.lost(i)
        rb, rt = r.lost()
        assert np.array_equal(lb, rb) and np.array_equal(lt, rt), f"filter {i} lost log"
        r.close()
    s.close()


def test_set_largest_filter_count(cf):
    """65536 filters, the most a set takes, created with deferred tables and
    three of them attached (ids 0, 40000, 65535).  Operations on detached
    filters come back invalid (0xFF) and change nothing; on the attached
    ones an insert batch stores the oracle's multiset, and a query / delete
    batch gives the oracle's answers.  Beyond 4096 filters the per-filter
    counts take the per-operation atomic path.  A 65537th filter is refused."""
    nf = 65536
    m, b, f = 64, 4, 8
    params = [cf.make_params(m, b, f, seed=i, lost_capacity=16) for i in range(nf)]
    with pytest.raises(cf.CfError, match="CF_EINVAL"):
        cf.CuckooFilterSet(params + params[:1], 1024, defer_tables=True)
    s = cf.CuckooFilterSet(params, 1 << 14, defer_tables=True)
    live = [0, 40000, nf - 1]
    for fid in live:
        s.attach(fid)
    rng = np.random.default_rng(31)
    per = 150  # LF 0.59 in each attached filter
    dead = rng.integers(1, 40000, 3000).astype(np.uint32)  # detached ids
    fids = np.concatenate([np.repeat(np.array(live, dtype=np.uint32), per), dead])
    keys = K.keys(32, 0, fids.size)
    order = rng.permutation(fids.size)
    fids, keys = fids[order], keys[order]
    ops = np.full(fids.size, INSERT, dtype=np.uint8)
    res = s.execute(torch.from_numpy(ops).cuda(), torch.from_numpy(fids.view(np.int32)).cuda(),
                    dev_u64(keys)).cpu().numpy()
    is_live = np.isin(fids, live)
    assert (res[~is_live] == 0xFF).all() and (res[is_live] == 1).all()
    counts = s.counts()
    assert s.failures().sum() == 0
    assert counts.sum() == 3 * per and all(counts[fid] == per for fid in live)
    refs = {}
    for fid in live:
        r = OracleFilter(m, b, f, seed=fid)
        mine = keys[fids == fid]
        r.insert_batch(mine)
        g = OracleFilter(m, b, f)
        g.load_words(host_u64(s.export_table(fid)))
        assert multiset_equal(g.stored_groups(), r.stored_groups()), f"filter {fid}"
        g.close()
        refs[fid] = (r, mine)
    # queries (half stored keys, half never inserted) and deletes of distinct
    # stored keys on the attached filters, plus operations on detached ones
    q_f, q_k, q_o = [], [], []
    for fid in live:
        mine = refs[fid][1]
        pick = rng.permutation(mine.size)
        q_f += [fid] * 140
        q_k += list(mine[pick[:70]]) + list(K.negatives(33 + fid, 0, 70))
        q_o += [QUERY] * 140
        q_f += [fid] * 40
        q_k += list(mine[pick[70:110]])
        q_o += [DELETE] * 40
    q_f += list(dead[:500])
    q_k += list(K.keys(34, 0, 500))
    q_o += list(rng.integers(0, 3, 500))
    q_f = np.array(q_f, dtype=np.uint32)
    q_k = np.array(q_k, dtype=np.uint64)
    q_o = np.array(q_o, dtype=np.uint8)
    res = s.execute(torch.from_numpy(q_o).cuda(), torch.from_numpy(q_f.view(np.int32)).cuda(),
                    dev_u64(q_k)).cpu().numpy()
    for fid in live:
        r = refs[fid][0]
        sel = q_f == fid
        want = [r.query(int(k)) for k in q_k[sel & (q_o == QUERY)]]
        assert np.array_equal(res[sel & (q_o == QUERY)], np.array(want, dtype=np.uint8))
        want = [r.delete(int(k)) for k in q_k[sel & (q_o == DELETE)]]
        assert np.array_equal(res[sel & (q_o == DELETE)], np.array(want, dtype=np.uint8))
        assert s.counts()[fid] == r.count == per - 40
        r.close()
    assert (res[~np.isin(q_f, live)] == 0xFF).all()
    s.close()


def test_set_largest_max_batch(cf):
    """max_batch = 2^31, the most a set takes, sizes its scratch (sorted
    indices, eviction queue, bin offsets) at the maximum; a small mixed batch
    through it matches the oracle, and 2^31 + 1 is refused."""
    specs = _specs(7, 4)
    params = [cf.make_params(m, b, f, hk, ev, D, sd) for (m, b, f, hk, ev, D, sd) in specs]
    with pytest.raises(cf.CfError, match="CF_EINVAL"):
        cf.CuckooFilterSet(params, (1 << 31) + 1)
    assert cf.cf_set_bytes(params, 1 << 31) > (1 << 31) * 8
    s = cf.CuckooFilterSet(params, 1 << 31)
    refs, pre = [], []
    for fid, (m, b, f, hk, ev, D, sd) in enumerate(specs):
        r = OracleFilter(m, b, f, hash_kind=hk, evict=ev, max_evict=D, seed=sd)
        keys = K.keys(900 + fid, 0, int(0.6 * m * b))
        r.insert_batch(keys)
        s.import_table(fid, dev_u64(r.words()))
        refs.append(r)
        pre.append(keys)
    torch.cuda.synchronize()
    ops, fids, keys = _batch(specs, pre, 5000, 41)
    res = s.execute(torch.from_numpy(ops).cuda(), torch.from_numpy(fids.view(np.int32)).cuda(),
                    dev_u64(keys)).cpu().numpy()
    want = _expected_query_delete(refs, ops, fids, keys)
    qd = ops != INSERT
    assert np.array_equal(res[qd], want[qd])
    _check_tables(cf, s, refs, ops, fids, keys, res)
    s.close()
    for r in refs:
        r.close()


def test_set_reattach_clears_only_that_table(cf):
    """A set created with its tables holds them in one allocation: detaching
    a filter keeps its place, and attaching it again gives an empty table and
    a zero count there while every other filter's table, count and answers
    stay as they were; the re-attached filter then takes inserts like new."""
    specs = _specs(12, 8)
    s, refs, pre = _build(cf, specs, 1 << 14, 960)
    before = [host_u64(s.export_table(fid)) for fid in range(len(specs))]
    counts = s.counts()
    fid = 5
    s.detach(fid)
    assert not s.attached(fid)
    q = np.full(100, QUERY, dtype=np.uint8)
    res = s.execute(torch.from_numpy(q).cuda(),
                    torch.from_numpy(np.full(100, fid, dtype=np.int32)).cuda(),
                    dev_u64(pre[fid][:100])).cpu().numpy()
    assert (res == 0xFF).all()
    s.attach(fid)
    assert s.attached(fid)
    after = s.counts()
    assert after[fid] == 0 and not host_u64(s.export_table(fid)).any()
    for g in range(len(specs)):
        if g != fid:
            assert after[g] == counts[g]
            assert np.array_equal(host_u64(s.export_table(g)), before[g]), f"filter {g}"
    m, b, f, hk, ev, D, sd = specs[fid]
    fresh = OracleFilter(m, b, f, hash_kind=hk, evict=ev, max_evict=D, seed=sd)
    keys = pre[fid]
    ins = np.full(keys.size, INSERT, dtype=np.uint8)
    s.execute(torch.from_numpy(ins).cuda(),
              torch.from_numpy(np.full(keys.size, fid, dtype=np.int32)).cuda(), dev_u64(keys))
    fresh.insert_batch(keys)
    assert s.counts()[fid] == fresh.count
    g = OracleFilter(m, b, f, hash_kind=hk, evict=ev, max_evict=D, seed=sd)
    g.load_words(host_u64(s.export_table(fid)))
    assert multiset_equal(g.stored_groups(), expected_groups(g, keys, lost=s.lost(fid)))
    for r in refs + [fresh, g]:
        r.close()
    s.close()


def test_set_empty_batch_and_errors(cf):
    specs = _specs(5, 3)
    s, refs, pre = _build(cf, specs, 1024, 800)
    z8 = torch.zeros(0, dtype=torch.uint8, device="cuda")
    z32 = torch.zeros(0, dtype=torch.int32, device="cuda")
    z64 = torch.zeros(0, dtype=torch.int64, device="cuda")
    s.execute(z8, z32, z64)
    big = torch.zeros(2048, dtype=torch.int64, device="cuda")
    with pytest.raises(cf.CfError, match="CF_EINVAL"):
        s.execute(torch.zeros(2048, dtype=torch.uint8, device="cuda"),
                  torch.zeros(2048, dtype=torch.int32, device="cuda"), big)
    with pytest.raises(cf.CfError):
        s.chunk = 100
    with pytest.raises(cf.CfError):
        s.streams = 9
    assert s.streams == 0 and s.chunk == 2048
    assert np.array_equal(s.counts(), np.array([r.count for r in refs], dtype=np.uint64))
    s.close()


def test_set_tune_leaves_the_set_unchanged(cf):
    """cf_set_tune executes and undoes the batch per trial: afterwards every
    filter stores the multiset it started with, and the batch executed for
    real gives the oracle's answers."""
    specs = _specs(3, 10)
    s, refs, pre = _build(cf, specs, 1 << 16, 700)
    ops, fids, keys = _batch(specs, pre, 30_000, 13)
    d_ops = torch.from_numpy(ops).cuda()
    d_fids = torch.from_numpy(fids.view(np.int32)).cuda()
    d_keys = dev_u64(keys)
    counts0 = s.counts()
    cands = [{"chunk": c} for c in (64, 512, 4096)] + [{"chunk": 1024, "streams": 1}]
    if s.persistent_capacity(256):
        cands += [{"chunk": 1024, "persistent": 1, "block": 256, "blocks_per_cu": 1},
                  {"chunk": 2048, "persistent": 1, "block": 512},
                  {"chunk": 512, "fused": 1}]
    key = ("chunk", "streams", "persistent", "fused")
    for eager in (False, True):  # timed as graph launches, then as cf_set_execute calls
        shape, trials, fails = s.tune(d_ops, d_fids, d_keys, shapes=cands, reps=2, eager=eager)
        assert fails == 0 and s.status() == 0
        assert shape == s.shape
        assert [tuple(t[k] for k in key) for t, _ in trials] == \
            [tuple(c.get(k, 0) for k in key) for c in cands]
        assert all(ms > 0 for _, ms in trials)
        assert tuple(shape[k] for k in key) in [tuple(t[k] for k in key) for t, _ in trials]
        assert np.array_equal(s.counts(), counts0)
    for fid, r in enumerate(refs):
        g = OracleFilter(r.m, r.b, r.f, hash_kind=r.hash_kind)
        g.load_words(host_u64(s.export_table(fid)))
        assert multiset_equal(g.stored_groups(), r.stored_groups()), f"filter {fid}"
        g.close()
    res = s.execute(d_ops, d_fids, d_keys).cpu().numpy()
    want = _expected_query_delete(refs, ops, fids, keys)
    qd = ops != INSERT
    assert np.array_equal(res[qd], want[qd])
    _check_tables(cf, s, refs, ops, fids, keys, res)
    with pytest.raises(cf.CfError):
        s.tune(d_ops, d_fids, d_keys, shapes=[{"chunk": 100}])
    s.close()


def test_set_mixed_placements_match_oracle(cf):
    """XOR and offset filters (any bucket count) in one set: each placement
    is its own class, and the batch's answers and tables match the oracle."""
    rng = np.random.default_rng(21)
    geoms = [(16, 16), (8, 8), (4, 16), (32, 32)]
    specs, places = [], []
    for i in range(8):
        b, f = geoms[i % len(geoms)]
        off = i % 2 == 1
        m = int(rng.integers(300, 1500)) if off else 1 << int(rng.integers(8, 11))
        specs.append((m, b, f, i % 3 == 0, 0, 128, 1200 + i))
        places.append(oracle.PLACE_OFFSET if off else oracle.PLACE_XOR)
    _check_placed_batch(cf, specs, places, 0, 900, 17)


def _sixteen_classes():
    """16 filters, each its own class: the 12 (b, f) with fmix64 and XOR,
    then four more with xxHash64 or the offset placement."""
    combos = [(b, f, 0, oracle.PLACE_XOR) for (b, f) in GEOMS]
    combos += [(16, 16, 1, oracle.PLACE_XOR), (8, 8, 0, oracle.PLACE_OFFSET),
               (4, 32, 1, oracle.PLACE_OFFSET), (32, 16, 0, oracle.PLACE_OFFSET)]
    specs = [((1 << 8) if pl == oracle.PLACE_XOR else 301 + i, b, f, hk, i % 2, 128 if i % 2 == 0
              else 500, 1500 + i) for i, (b, f, hk, pl) in enumerate(combos)]
    return specs, [pl for (_, _, _, pl) in combos]


@pytest.mark.parametrize("streams", [1, 0, 8])
def test_set_sixteen_classes(cf, streams):
    """The most classes a set takes (16, so 48 bins per chunk), with the
    class chains on one stream, the default four and eight: every answer
    and table matches the oracle.  A 17th class is refused."""
    specs, places = _sixteen_classes()
    assert len({(b, f, hk, pl) for (m, b, f, hk, *_), pl in zip(specs, places)}) == 16
    _check_placed_batch(cf, specs, places, streams, 1700, 23)
    extra = cf.make_params(1 << 8, 16, 16, 1, placement=oracle.PLACE_OFFSET)
    params = [cf.make_params(m, b, f, int(hk), ev, D, sd, placement=pl)
              for (m, b, f, hk, ev, D, sd), pl in zip(specs, places)]
    with pytest.raises(cf.CfError, match="CF_EUNSUPPORTED"):
        cf.CuckooFilterSet(params + [extra], 1024)


def _check_placed_batch(cf, specs, places, streams, fill_seed, batch_seed, shape=None):
    """One mixed batch on a set of the given filters (prefilled from the
    oracle to LF 0.6): queries and deletes bit-exact, inserts stored as the
    oracle's multiset, counts equal.  shape: cf_set_shape fields to set."""
    params = [cf.make_params(m, b, f, int(hk), ev, D, sd, placement=pl)
              for (m, b, f, hk, ev, D, sd), pl in zip(specs, places)]
    s = cf.CuckooFilterSet(params, 1 << 16)
    s.streams = streams
    if shape:
        s.set_shape(**shape)
    refs, pre = [], []
    for fid, ((m, b, f, hk, ev, D, sd), pl) in enumerate(zip(specs, places)):
        r = OracleFilter(m, b, f, hash_kind=int(hk), evict=ev, max_evict=D, seed=sd,
                         placement=pl)
        keys = K.keys(fill_seed + fid, 0, int(0.6 * m * b))
        r.insert_batch(keys)
        s.import_table(fid, dev_u64(r.words()))
        refs.append(r)
        pre.append(keys)
    torch.cuda.synchronize()
    ops, fids, keys = _batch(specs, pre, 30_000, batch_seed)
    res = s.execute(torch.from_numpy(ops).cuda(), torch.from_numpy(fids.view(np.int32)).cuda(),
                    dev_u64(keys)).cpu().numpy()
    want = _expected_query_delete(refs, ops, fids, keys)
    qd = ops != INSERT
    assert np.array_equal(res[qd], want[qd])
    assert s.failures().sum() == 0 and (res[ops == INSERT] == 1).all()
    assert s.status() == 0
    counts = s.counts()
    for fid, r in enumerate(refs):
        ins = keys[(ops == INSERT) & (fids == fid)]
        lo0, hi0, t0 = r.stored_groups()
        lo1, hi1, t1 = r.key_groups(ins)
        want_g = (np.concatenate([lo0, lo1]), np.concatenate([hi0, hi1]),
                  np.concatenate([t0, t1]))
        g = OracleFilter(r.m, r.b, r.f, hash_kind=r.hash_kind, placement=r.placement)
        g.load_words(host_u64(s.export_table(fid)))
        assert multiset_equal(g.stored_groups(), want_g), f"filter {fid}"
        assert counts[fid] == g.count
        g.close()
    s.close()
