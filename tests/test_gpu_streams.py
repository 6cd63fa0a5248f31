"""Stream ordering of the C ABI's asynchronous calls, on streams other than
the default one.

Each call enqueues on the stream it is given (the binding passes torch's
current stream when none is named), so work on one stream must see the
effects of earlier work on that stream with no device-wide synchronisation,
and work on another stream only after an event says so.  A filter set forks
its class chains onto its own streams and joins them back into the caller's
stream: the caller's next work on that stream, here a torch reduction, must
see every result of the batch."""
import numpy as np
import pytest

import oracle
from oracle import OracleFilter
from gpu_util import dev_u64
from workloads import keys as K

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cf():
    import paper_2603_15486_amd as mod
    return mod


def test_filters_follow_their_streams(cf):
    """Two filters, each driven on its own stream with insert, query, delete
    and query again back to back; each stream is synchronised alone."""
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    out = {}
    for name, st, seed in (("a", s1, 1), ("b", s2, 2)):
        with torch.cuda.stream(st):
            g = cf.CuckooFilter(1 << 14, 16, 16, seed=seed)
            keys = torch.empty(150_000, dtype=torch.int64, device="cuda")
            cf.cf_keygen(keys, seed)  # on the current stream
            ok = torch.zeros(keys.numel(), dtype=torch.uint8, device="cuda")
            g.insert(keys, ok)
            found = g.query(keys)
            dok = torch.zeros(keys.numel() // 2, dtype=torch.uint8, device="cuda")
            g.delete(keys[: keys.numel() // 2], dok)
            after = g.query(keys)
            # reductions on the same stream see every result above
            out[name] = (g, st, ok.sum(dtype=torch.int64), found.sum(dtype=torch.int64),
                         dok.sum(dtype=torch.int64), after[keys.numel() // 2:].sum(dtype=torch.int64))
    for name, (g, st, n_ok, n_found, n_del, n_rest) in out.items():
        st.synchronize()
        assert int(n_ok) == int(n_found) == 150_000, name
        assert int(n_del) == 75_000 and int(n_rest) == 75_000, name
        g.close()


def test_event_orders_work_across_streams(cf):
    """Inserts on one stream, an event, queries on another stream that waits
    for it: every key is found."""
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    g = cf.CuckooFilter(1 << 14, 16, 16, seed=5)
    keys = dev_u64(K.keys(5, 0, 200_000))
    torch.cuda.synchronize()
    ev = torch.cuda.Event()
    with torch.cuda.stream(s1):
        g.insert(keys)
        ev.record(s1)
    s2.wait_event(ev)
    with torch.cuda.stream(s2):
        n = g.query(keys).sum(dtype=torch.int64)
    s2.synchronize()
    assert int(n) == keys.numel()
    g.close()


@pytest.mark.parametrize("graph", [False, True])
def test_set_batch_joins_back_into_the_callers_stream(cf, graph):
    """A set of four classes run on its own streams from a user stream; a
    torch reduction queued next on that stream sees all of the batch's
    results, eagerly and through a replayed graph."""
    specs = [(1 << 10, 16, 16), (1 << 11, 8, 16), (1 << 10, 4, 8), (1 << 9, 32, 32)]
    params = [cf.make_params(m, b, f, seed=10 + i) for i, (m, b, f) in enumerate(specs)]
    n_per = [int(0.5 * m * b) for m, b, f in specs]
    total = sum(n_per)
    s = cf.CuckooFilterSet(params, total)
    assert s.streams == 0  # the default: one stream per class, here four
    fids = np.concatenate([np.full(n, i, dtype=np.int32) for i, n in enumerate(n_per)])
    keys = np.concatenate([K.keys(30 + i, 0, n) for i, n in enumerate(n_per)])
    d_ops = torch.full((total,), 2, dtype=torch.uint8, device="cuda")
    d_fids = torch.from_numpy(fids).cuda()
    d_keys = dev_u64(keys)
    d_res = torch.zeros(total, dtype=torch.uint8, device="cuda")
    d_n = torch.full((1,), total, dtype=torch.int64, device="cuda")
    gr = s.graph(d_ops, d_fids, d_keys, d_n, d_res) if graph else None
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        if graph:
            cf.cf_graph_launch(gr, stream=st.cuda_stream)
        else:
            s.execute(d_ops, d_fids, d_keys, d_res)
        stored = d_res.sum(dtype=torch.int64)
        d_ops.fill_(0)  # then every key again, as queries
        if graph:
            cf.cf_graph_launch(gr, stream=st.cuda_stream)
        else:
            s.execute(d_ops, d_fids, d_keys, d_res)
        found = d_res.sum(dtype=torch.int64)
    st.synchronize()
    assert int(stored) == total and int(found) == total
    assert s.failures().sum() == 0
    refs = [OracleFilter(m, b, f, seed=10 + i) for i, (m, b, f) in enumerate(specs)]
    for i, r in enumerate(refs):
        r.insert_batch(keys[fids == i])
        g = OracleFilter(r.m, r.b, r.f)
        g.load_words(s.export_table(i).cpu().numpy().view(np.uint64))
        assert g.count == r.count
        lo0, hi0, t0 = g.stored_groups()
        lo1, hi1, t1 = r.stored_groups()
        assert sorted(zip(lo0, hi0, t0)) == sorted(zip(lo1, hi1, t1))
        g.close()
        r.close()
    s.close()
