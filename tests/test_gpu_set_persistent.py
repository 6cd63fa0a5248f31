"""GPU tests of a filter set's persistent form (cf_set_shape.persistent = 1):
one cooperative launch per mixed batch, with grid barriers between the
partition and the query, delete and insert phases.

* A mixed batch against per-filter oracles (queries see the pre-batch state,
  deletes bit-exact, inserts keep the multiset, invalid operations 0xFF) for
  both block sizes, one and the most blocks per compute unit, three chunks,
  both hashes and both placements, BFS and DFS filters, b = 4..32 in one set.
* The same batch on a twin set in the class-kernel form gives the same
  answers and multisets.
* A captured graph (one cooperative kernel node) replayed on batches of
  three sizes equals eager execution of the class-kernel form.
* More filters than the LDS tally holds (per-operation atomics), detached
  filters.
* The shape is refused on a set whose filters differ in f, hash or placement,
  and with more blocks per compute unit than fit.
* The capacity reported is what is resident at once: for every fingerprint
  width, hash and block size, a batch at that many blocks per compute unit
  completes its barriers.
* A barrier given no time at all (CF_SET_BARRIER_US=0, set from the host)
  abandons its batch: the error is reported, no delete or insert ran, later
  batches do nothing until the shape is set again, then batches are exact.
"""
import os

import numpy as np
import pytest

from oracle import OracleFilter
from gpu_util import dev_u64, host_u64, multiset_equal
from test_gpu_set import (INSERT, QUERY, _batch, _build, _check_placed_batch, _check_tables,
                          _expected_query_delete, _forget_deleted)
from workloads import keys as K

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cf():
    import paper_2603_15486_amd as mod
    return mod


def _specs(seed, nf, f=16, hk=0):
    """Filters sharing f and the hash: b = 4, 8, 16, 32 in turn, BFS and DFS."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nf):
        b = (4, 8, 16, 32)[i % 4]
        m = 1 << int(rng.integers(7, 11))
        ev = int(rng.integers(0, 2))
        out.append((m, b, f, hk, ev, 128 if ev == 0 else 500, 2000 + i))
    return out


def _dev(ops, fids, keys):
    return (torch.from_numpy(ops).cuda(), torch.from_numpy(fids.view(np.int32)).cuda(),
            dev_u64(keys))


def _run_checked(cf, s, specs, refs, pre, n, seed):
    ops, fids, keys = _batch(specs, pre, n, seed)
    ops[3], fids[11] = 9, 70_000  # an unknown kind and an unknown filter
    res = s.execute(*_dev(ops, fids, keys)).cpu().numpy()
    assert s.status() == 0
    assert res[3] == 0xFF and res[11] == 0xFF
    valid = np.ones(n, dtype=bool)
    valid[[3, 11]] = False
    ops2 = np.where(valid, ops, 9).astype(np.uint8)
    want = _expected_query_delete(refs, ops2, fids, keys)
    qd = valid & (ops != INSERT)
    assert np.array_equal(res[qd], want[qd])
    assert (res[valid & (ops == INSERT)] == 1).all() or s.failures().sum() > 0
    _check_tables(cf, s, refs, ops2, fids, keys, res)


@pytest.mark.parametrize("block,per_cu,chunk,wave_bfs", [(256, 1, 2048, 0), (256, 0, 64, 0),
                                                         (512, 0, 4096, 0), (512, 1, 1024, 0),
                                                         (256, 0, 2048, 1), (512, 2, 512, 1)])
def test_persistent_batch_matches_oracle(cf, block, per_cu, chunk, wave_bfs):
    specs = _specs(block + per_cu + chunk, 12)
    s, refs, pre = _build(cf, specs, 1 << 16, 800)
    assert s.persistent_capacity(block) >= 1
    s.set_shape(chunk=chunk, persistent=1, block=block, blocks_per_cu=per_cu, wave_bfs=wave_bfs)
    sh = s.shape
    assert sh["persistent"] == 1 and sh["block"] == block
    assert sh["blocks_per_cu"] == (per_cu or s.persistent_capacity(block))
    print(f"persistent: block={block} per_cu={per_cu} chunk={chunk}", flush=True)
    _run_checked(cf, s, specs, refs, pre, 40_000, 31)
    s.close()


@pytest.mark.parametrize("f,hk,placement", [(8, 1, 0), (32, 0, 0), (16, 1, 1)])
def test_persistent_hashes_widths_placements(cf, f, hk, placement):
    specs = _specs(40 + f, 8, f=f, hk=hk)
    if placement:
        # the offset placement takes any bucket count
        specs = [(m - 3, b, ff, h, ev, D, sd) for (m, b, ff, h, ev, D, sd) in specs]
    print(f"persistent: f={f} hash={hk} placement={placement}", flush=True)
    _check_placed_batch(cf, specs, [placement] * len(specs), 0, 900 + f, 41,
                        shape={"persistent": 1, "chunk": 512})


def test_persistent_equals_class_kernels(cf):
    specs = _specs(5, 10)
    a, refs, pre = _build(cf, specs, 1 << 16, 850)
    b, _, _ = _build(cf, specs, 1 << 16, 850)
    a.set_shape(persistent=1, block=512, chunk=1024)
    for step in range(3):
        # 3 x 10k operations take the filters from load 0.6 to about 0.75
        ops, fids, keys = _batch(specs, pre, 10_000, 50 + step)
        _forget_deleted(pre, ops, fids, keys)
        ra = a.execute(*_dev(ops, fids, keys)).cpu().numpy()
        rb = b.execute(*_dev(ops, fids, keys)).cpu().numpy()
        assert a.status() == 0
        assert a.failures().sum() == 0 and b.failures().sum() == 0
        assert np.array_equal(ra, rb), f"batch {step}"
        assert np.array_equal(a.counts(), b.counts())
        for fid, (m, bb, f, hk, *_r) in enumerate(specs):
            ga, gb = OracleFilter(m, bb, f, hash_kind=hk), OracleFilter(m, bb, f, hash_kind=hk)
            ga.load_words(host_u64(a.export_table(fid)))
            gb.load_words(host_u64(b.export_table(fid)))
            assert multiset_equal(ga.stored_groups(), gb.stored_groups())
            ga.close()
            gb.close()
    a.close()
    b.close()


def test_persistent_graph_replays_match_eager(cf):
    specs = _specs(6, 10)
    nmax = 1 << 15
    a, refs, pre = _build(cf, specs, nmax, 860)
    b, _, _ = _build(cf, specs, nmax, 860)
    a.set_shape(persistent=1, chunk=1024)
    b.streams = 1
    d_ops = torch.zeros(nmax, dtype=torch.uint8, device="cuda")
    d_fids = torch.zeros(nmax, dtype=torch.int32, device="cuda")
    d_keys = torch.zeros(nmax, dtype=torch.int64, device="cuda")
    d_res = torch.zeros(nmax, dtype=torch.uint8, device="cuda")
    d_n = torch.zeros(1, dtype=torch.int64, device="cuda")
    graph = a.graph(d_ops, d_fids, d_keys, d_n, d_res)
    for step, n in enumerate((nmax, 5000, 12_345)):
        ops, fids, keys = _batch(specs, pre, n, 150 + step)
        _forget_deleted(pre, ops, fids, keys)
        d_ops[:n].copy_(torch.from_numpy(ops))
        d_fids[:n].copy_(torch.from_numpy(fids.view(np.int32)))
        d_keys[:n].copy_(torch.from_numpy(keys.view(np.int64)))
        d_n.fill_(n)
        print(f"persistent graph replay {step}: n={n}", flush=True)
        cf.cf_graph_launch(graph)
        torch.cuda.synchronize()
        assert a.status() == 0
        got = d_res[:n].cpu().numpy()
        want = b.execute(*_dev(ops, fids, keys)).cpu().numpy()
        assert np.array_equal(got, want), f"replay {step}"
        assert np.array_equal(a.counts(), b.counts())
        for fid, (m, bb, f, hk, *_r) in enumerate(specs):
            ga, gb = OracleFilter(m, bb, f, hash_kind=hk), OracleFilter(m, bb, f, hash_kind=hk)
            ga.load_words(host_u64(a.export_table(fid)))
            gb.load_words(host_u64(b.export_table(fid)))
            assert multiset_equal(ga.stored_groups(), gb.stored_groups())
            ga.close()
            gb.close()
    a.drop_graph(graph)
    a.close()
    b.close()


def test_persistent_many_filters_and_detached(cf):
    """5000 filters (beyond the 4096 the LDS tally holds: per-operation
    atomics), three of them detached (their operations give 0xFF)."""
    nf = 5000
    params = [cf.make_params(64, (8, 16)[i % 2], 16, seed=i) for i in range(nf)]
    s = cf.CuckooFilterSet(params, 1 << 16)
    for fid in (7, 1234, 4999):
        s.detach(fid)
    s.set_shape(persistent=1)
    rng = np.random.default_rng(3)
    n = 50_000
    fids = rng.integers(0, nf, n).astype(np.uint32)
    ops = np.full(n, INSERT, dtype=np.uint8)
    keys = K.keys(77, 0, n)
    res = s.execute(*_dev(ops, fids, keys)).cpu().numpy()
    assert s.status() == 0
    det = np.isin(fids, [7, 1234, 4999])
    assert (res[det] == 0xFF).all() and (res[~det] == 1).all()
    counts = s.counts()
    want = np.bincount(fids[~det], minlength=nf)
    assert np.array_equal(counts, want.astype(np.uint64))
    q = s.execute(*_dev(np.full(n, QUERY, dtype=np.uint8), fids, keys)).cpu().numpy()
    assert (q[~det] == 1).all() and (q[det] == 0xFF).all()
    s.close()


def test_persistent_refused_where_it_cannot_run(cf):
    mixed = [cf.make_params(256, 16, 16), cf.make_params(256, 16, 8)]
    s = cf.CuckooFilterSet(mixed, 1 << 12)
    assert s.persistent_capacity(256) == 0
    with pytest.raises(cf.CfError, match="CF_EUNSUPPORTED"):
        s.set_shape(persistent=1)
    assert s.shape["persistent"] == 0
    s.close()
    same = cf.CuckooFilterSet([cf.make_params(256, 16, 16), cf.make_params(256, 8, 16)], 1 << 12)
    fit = same.persistent_capacity(256)
    assert fit >= 1
    with pytest.raises(cf.CfError, match="CF_EINVAL"):
        same.set_shape(persistent=1, blocks_per_cu=fit + 1)
    with pytest.raises(cf.CfError, match="CF_EINVAL"):
        same.set_shape(persistent=1, block=384)
    same.set_shape(persistent=1, blocks_per_cu=fit)
    same.close()


def test_persistent_abandoned_batch_is_reported(cf):
    specs = _specs(9, 6)
    os.environ["CF_SET_BARRIER_US"] = "0"
    try:
        s, refs, pre = _build(cf, specs, 1 << 15, 880)
    finally:
        os.environ.pop("CF_SET_BARRIER_US", None)
    s.set_shape(persistent=1)
    before = [host_u64(s.export_table(fid)).copy() for fid in range(len(specs))]
    ops, fids, keys = _batch(specs, pre, 20_000, 61)
    d = _dev(ops, fids, keys)
    res = torch.full((keys.size,), 0x5A, dtype=torch.uint8, device="cuda")
    print("persistent: batch with no barrier time", flush=True)
    s.execute(*d, results=res)
    torch.cuda.synchronize()
    if s.status() == 0:
        # every block reached every barrier in time: the batch is exact
        _check_tables(cf, s, refs, *_apply_expected(refs, ops, fids, keys, res))
        s.close()
        return
    # no delete or insert ran: every table is as it was
    for fid in range(len(specs)):
        assert np.array_equal(host_u64(s.export_table(fid)), before[fid])
    # later batches do nothing until the shape is set again, which clears it
    res.fill_(0x5A)
    s.execute(*d, results=res)
    assert bool((res == 0x5A).all()) and s.status() == 1
    s.set_shape(persistent=1)
    assert s.status() == 0
    s.close()
    # a set created with the usual bound runs the same batch exactly
    s2, refs2, pre2 = _build(cf, specs, 1 << 15, 880)
    s2.set_shape(persistent=1)
    _run_checked(cf, s2, specs, refs2, pre2, 20_000, 61)
    s2.close()


def _apply_expected(refs, ops, fids, keys, res):
    r = res.cpu().numpy()
    want = _expected_query_delete(refs, ops, fids, keys)
    qd = ops != INSERT
    assert np.array_equal(r[qd], want[qd])
    return ops, fids, keys, r


@pytest.mark.parametrize("f", [8, 16, 32])
@pytest.mark.parametrize("hk", [0, 1])
def test_persistent_capacity_is_resident(cf, f, hk):
    """At the reported capacity every barrier completes (the runtime's
    occupancy figure alone overstates it for one kernel)."""
    specs = [(1 << 9, b, f, hk, 0, 128, 3000 + b) for b in (4, 8, 16, 32)]
    s, refs, pre = _build(cf, specs, 1 << 15, 890)
    for block in (256, 512):
        cap = s.persistent_capacity(block)
        assert cap >= 1
        s.set_shape(persistent=1, block=block, blocks_per_cu=cap, chunk=256)
        print(f"persistent capacity: f={f} hash={hk} block={block} cap={cap}", flush=True)
        ops, fids, keys = _batch(specs, pre, 8000, 70 + block)
        q = np.where(ops == INSERT, QUERY, ops).astype(np.uint8)  # queries and deletes
        _forget_deleted(pre, q, fids, keys)
        res = s.execute(*_dev(q, fids, keys)).cpu().numpy()
        assert s.status() == 0
        assert np.array_equal(res, _expected_query_delete(refs, q, fids, keys))
    s.close()


def _specs_b16(seed, nf, f=16, hk=0):
    """Filters whose buckets have at most 16 slots (b = 4, 8, 16 in turn): the
    set gets the kernels compiled without the 32-slot path."""
    return [(m, (4, 8, 16)[i % 3], ff, h, ev, D, sd)
            for i, (m, _b, ff, h, ev, D, sd) in enumerate(_specs(seed, nf, f, hk))]


@pytest.mark.parametrize("block,f,hk", [(256, 16, 0), (512, 8, 1), (256, 32, 0)])
def test_persistent_small_buckets_match_oracle(cf, block, f, hk):
    specs = _specs_b16(300 + block + f, 9, f=f, hk=hk)
    s, refs, pre = _build(cf, specs, 1 << 16, 820)
    cap = s.persistent_capacity(block)
    assert cap >= 1
    s.set_shape(chunk=1024, persistent=1, block=block, blocks_per_cu=cap)
    print(f"persistent, buckets <= 16: block={block} f={f} hash={hk} cap={cap}", flush=True)
    _run_checked(cf, s, specs, refs, pre, 30_000, 53)
    s.close()


def test_persistent_phase_ticks_are_ordered(cf):
    """cf_set_phase_ticks: after a persistent batch, the start and the three
    barrier times are set and in order; a set that cannot run the form is
    refused."""
    specs = _specs(77, 6)
    s, refs, pre = _build(cf, specs, 1 << 15, 840)
    s.set_shape(persistent=1, chunk=512)
    ops, fids, keys = _batch(specs, pre, 20_000, 91)
    s.execute(*_dev(ops, fids, keys))
    assert s.status() == 0
    t, hz = cf.cf_set_phase_ticks(s.handle)
    assert hz > 0 and 0 < t[0] <= t[1] <= t[2] <= t[3]
    assert all(x >= 0 for x in s.persistent_phase_us())
    s.close()
    mixed = cf.CuckooFilterSet([cf.make_params(256, 16, 16), cf.make_params(256, 16, 8)], 1 << 12)
    with pytest.raises(cf.CfError, match="CF_EUNSUPPORTED"):
        cf.cf_set_phase_ticks(mixed.handle)
    mixed.close()
