"""GPU tests of a filter set's phase form (cf_set_shape.fused = 1): after the
partition, one launch per phase covers every class (the class's b chosen per
block at run time), all on the caller's stream.

* A mixed batch against per-filter oracles (queries see the pre-batch state,
  deletes bit-exact, inserts keep the multiset, invalid operations 0xFF) at
  four chunks and both breadth-first searches, b = 4..32 in one set.
* Both hashes, the three fingerprint widths and both placements.
* The same batches on a twin set in the class-kernel form give the same
  answers, counts and multisets.
* A captured graph (a straight chain of four kernels) replayed on batches of
  three sizes equals eager execution of the class-kernel form.
* More filters than the LDS tally holds, detached filters.
* The shape is refused on a set whose filters differ in f, and together with
  the persistent form.
"""
import numpy as np
import pytest

from oracle import OracleFilter
from gpu_util import host_u64, multiset_equal
from test_gpu_set import INSERT, QUERY, _batch, _build, _check_placed_batch, _forget_deleted
from test_gpu_set_persistent import _dev, _run_checked, _specs
from workloads import keys as K

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cf():
    import paper_2603_15486_amd as mod
    return mod


def _same_tables(a, b, specs):
    for fid, (m, bb, f, hk, *_r) in enumerate(specs):
        ga, gb = OracleFilter(m, bb, f, hash_kind=hk), OracleFilter(m, bb, f, hash_kind=hk)
        ga.load_words(host_u64(a.export_table(fid)))
        gb.load_words(host_u64(b.export_table(fid)))
        assert multiset_equal(ga.stored_groups(), gb.stored_groups()), f"filter {fid}"
        ga.close()
        gb.close()


@pytest.mark.parametrize("chunk,wave_bfs", [(64, 0), (512, 1), (2048, 0), (4096, 1)])
def test_fused_batch_matches_oracle(cf, chunk, wave_bfs):
    specs = _specs(chunk + wave_bfs, 12)
    s, refs, pre = _build(cf, specs, 1 << 16, 810)
    s.set_shape(chunk=chunk, fused=1, wave_bfs=wave_bfs)
    sh = s.shape
    assert sh["fused"] == 1 and sh["persistent"] == 0 and sh["chunk"] == chunk
    print(f"fused: chunk={chunk} wave_bfs={wave_bfs}", flush=True)
    _run_checked(cf, s, specs, refs, pre, 40_000, 37)
    s.close()


@pytest.mark.parametrize("f,hk,placement", [(8, 1, 0), (32, 0, 0), (16, 1, 1), (16, 0, 1)])
def test_fused_hashes_widths_placements(cf, f, hk, placement):
    specs = _specs(60 + f, 8, f=f, hk=hk)
    if placement:
        # the offset placement takes any bucket count
        specs = [(m - 5, b, ff, h, ev, D, sd) for (m, b, ff, h, ev, D, sd) in specs]
    print(f"fused: f={f} hash={hk} placement={placement}", flush=True)
    _check_placed_batch(cf, specs, [placement] * len(specs), 0, 700 + f, 43,
                        shape={"fused": 1, "chunk": 1024})


def test_fused_equals_class_kernels(cf):
    specs = _specs(9, 10)
    a, refs, pre = _build(cf, specs, 1 << 16, 870)
    b, _, _ = _build(cf, specs, 1 << 16, 870)
    a.set_shape(fused=1, chunk=1024)
    for step in range(3):
        ops, fids, keys = _batch(specs, pre, 10_000, 60 + step)
        _forget_deleted(pre, ops, fids, keys)
        ra = a.execute(*_dev(ops, fids, keys)).cpu().numpy()
        rb = b.execute(*_dev(ops, fids, keys)).cpu().numpy()
        assert a.failures().sum() == 0 and b.failures().sum() == 0
        assert np.array_equal(ra, rb), f"batch {step}"
        assert np.array_equal(a.counts(), b.counts())
        _same_tables(a, b, specs)
    a.close()
    b.close()


def test_fused_graph_replays_match_eager(cf):
    specs = _specs(11, 10)
    nmax = 1 << 15
    a, refs, pre = _build(cf, specs, nmax, 880)
    b, _, _ = _build(cf, specs, nmax, 880)
    a.set_shape(fused=1, chunk=512)
    b.streams = 1
    d_ops = torch.zeros(nmax, dtype=torch.uint8, device="cuda")
    d_fids = torch.zeros(nmax, dtype=torch.int32, device="cuda")
    d_keys = torch.zeros(nmax, dtype=torch.int64, device="cuda")
    d_res = torch.zeros(nmax, dtype=torch.uint8, device="cuda")
    d_n = torch.zeros(1, dtype=torch.int64, device="cuda")
    graph = a.graph(d_ops, d_fids, d_keys, d_n, d_res)
    for step, n in enumerate((nmax, 5000, 12_345)):
        ops, fids, keys = _batch(specs, pre, n, 170 + step)
        _forget_deleted(pre, ops, fids, keys)
        d_ops[:n].copy_(torch.from_numpy(ops))
        d_fids[:n].copy_(torch.from_numpy(fids.view(np.int32)))
        d_keys[:n].copy_(torch.from_numpy(keys.view(np.int64)))
        d_n.fill_(n)
        print(f"fused graph replay {step}: n={n}", flush=True)
        cf.cf_graph_launch(graph)
        torch.cuda.synchronize()
        got = d_res[:n].cpu().numpy()
        want = b.execute(*_dev(ops, fids, keys)).cpu().numpy()
        assert np.array_equal(got, want), f"replay {step}"
        assert np.array_equal(a.counts(), b.counts())
        _same_tables(a, b, specs)
    a.drop_graph(graph)
    a.close()
    b.close()


def test_fused_many_filters_and_detached(cf):
    """5000 filters (beyond the 4096 the LDS tally holds: per-operation
    atomics), three of them detached (their operations give 0xFF)."""
    nf = 5000
    params = [cf.make_params(64, (8, 16)[i % 2], 16, seed=i) for i in range(nf)]
    s = cf.CuckooFilterSet(params, 1 << 16)
    for fid in (3, 2500, 4998):
        s.detach(fid)
    s.set_shape(fused=1)
    rng = np.random.default_rng(5)
    n = 50_000
    fids = rng.integers(0, nf, n).astype(np.uint32)
    keys = K.keys(79, 0, n)
    res = s.execute(*_dev(np.full(n, INSERT, dtype=np.uint8), fids, keys)).cpu().numpy()
    det = np.isin(fids, [3, 2500, 4998])
    assert (res[det] == 0xFF).all() and (res[~det] == 1).all()
    want = np.bincount(fids[~det], minlength=nf)
    assert np.array_equal(s.counts(), want.astype(np.uint64))
    q = s.execute(*_dev(np.full(n, QUERY, dtype=np.uint8), fids, keys)).cpu().numpy()
    assert (q[~det] == 1).all() and (q[det] == 0xFF).all()
    s.close()


def test_fused_refused_where_it_cannot_run(cf):
    mixed = [cf.make_params(256, 16, 16), cf.make_params(256, 16, 8)]
    s = cf.CuckooFilterSet(mixed, 1 << 12)
    with pytest.raises(cf.CfError, match="CF_EUNSUPPORTED"):
        s.set_shape(fused=1)
    assert s.shape["fused"] == 0
    s.close()
    same = [cf.make_params(256, 16, 16), cf.make_params(512, 8, 16)]
    s = cf.CuckooFilterSet(same, 1 << 12)
    with pytest.raises(cf.CfError, match="CF_EINVAL"):
        s.set_shape(fused=1, persistent=1)
    s.set_shape(fused=1)
    assert s.shape["fused"] == 1
    s.close()


@pytest.mark.parametrize("f,hk,wave_bfs", [(16, 0, 0), (8, 1, 1)])
def test_fused_small_buckets_match_oracle(cf, f, hk, wave_bfs):
    """Buckets of at most 16 slots: the phase kernels compiled without the
    32-slot path."""
    from test_gpu_set_persistent import _specs_b16
    specs = _specs_b16(400 + f, 9, f=f, hk=hk)
    s, refs, pre = _build(cf, specs, 1 << 16, 830)
    s.set_shape(chunk=2048, fused=1, wave_bfs=wave_bfs)
    print(f"fused, buckets <= 16: f={f} hash={hk} wave_bfs={wave_bfs}", flush=True)
    _run_checked(cf, s, specs, refs, pre, 30_000, 59)
    s.close()
