"""Host model of the filter set's scratch indexing (csrc/cf_set.hip,
csrc/cf_set_kernels.hpp), checked on the CPU at the multi-filter benchmark's
exact shape: 256 filters in two classes, batches of 2^22 operations, every
chunk the tuner may pick, eager and graph launches, and at the set's limits
(16 classes, 48 bins).

The model restates, for every block of a launch, the indices the kernels
compute into the set's three scratch arrays and into the batch:
  * partition_kernel: its chunk [lo, hi), the per-bin histogram, the bin
    offsets it stores at binoff[block * (nb + 1) + j] and the sorted positions
    it stores at sorted[lo + pos];
  * the class kernels: bin_range's reads of binoff, the reads of
    sorted[block * chunk + p] for p in [b0, b1), the batch index each read
    yields, and the insert kernel's queue slice [block * chunk + b0,
    block * chunk + b1);
  * cf_set_apply's single-filter insert: queue[block * seg + pos], pos < seg;
and asserts that every index lies inside the allocation the set makes for
max_batch (layout_of), every batch index inside [0, n), and that the bins of
one block tile its chunk exactly (so concurrent class kernels never share a
queue or result entry).
"""
import numpy as np
import pytest

K_BLOCK = 256
K_MAX_CHUNK, K_MIN_CHUNK = 4096, 64
K_MAX_CLASSES = 16
K_MAX_BINS = 3 * K_MAX_CLASSES
K_APPLY_GRID = 4096


def layout(max_batch):
    """Entries of the scratch arrays, as layout_of computes them."""
    return {
        "sorted": max_batch + K_MAX_CHUNK,
        "queue": max_batch + K_APPLY_GRID * K_BLOCK,
        "binoff": ((max_batch + K_MIN_CHUNK - 1) // K_MIN_CHUNK + 1) * (K_MAX_BINS + 1),
    }


def model_batch(ops, fids, cls, ncls, chunk, n, grid, max_batch):
    """Index every scratch and batch access of one batch; returns the
    largest index seen per array."""
    L = layout(max_batch)
    nb = 3 * ncls
    nfilters = cls.size
    top = {"sorted": -1, "queue": -1, "binoff": -1}
    assert grid * chunk >= n
    binoff = np.zeros(grid * (nb + 1), dtype=np.int64)
    sorted_ = np.full(grid * chunk, -1, dtype=np.int64)
    for blk in range(grid):
        lo = blk * chunk
        hi = min(lo + chunk, n)
        idx = np.arange(lo, max(hi, lo), dtype=np.int64)
        op, fid = ops[idx].astype(np.int64), fids[idx].astype(np.int64)
        valid = (op <= 2) & (fid < nfilters)
        c = np.where(valid, cls[np.minimum(fid, nfilters - 1)], 0xFF).astype(np.int64)
        b = np.where(valid & (c < ncls), op * ncls + c, nb)
        hist = np.bincount(b, minlength=nb + 1)
        base = np.concatenate([[0], np.cumsum(hist)[:-1]])
        off = blk * (nb + 1) + np.arange(nb + 1)
        assert off.max() < L["binoff"]
        top["binoff"] = max(top["binoff"], int(off.max()))
        binoff[off] = base
        # scatter: bin j's operations take positions base[j] .. base[j]+hist[j]-1
        order = np.argsort(b, kind="stable")
        pos = np.arange(idx.size)  # position of order[k] is k (bins contiguous)
        if idx.size:
            assert pos.max() < hi - lo <= chunk
            w = lo + pos
            assert w.max() < L["sorted"]
            top["sorted"] = max(top["sorted"], int(w.max()))
            sorted_[w] = idx[order]
    # class kernels: every (kind, class) bin of every block
    seen = np.zeros(max(n, 1), dtype=np.int64)
    for blk in range(grid):
        for binj in range(nb):
            b0 = int(binoff[blk * (nb + 1) + binj])
            b1 = int(binoff[blk * (nb + 1) + binj + 1]) if binj + 1 <= nb else b0
            assert 0 <= b0 <= b1 <= chunk
            rd = blk * chunk + np.arange(b0, b1)
            if rd.size:
                assert rd.max() < L["sorted"]
                i = sorted_[rd]
                assert (i >= 0).all() and (i < n).all()
                seen[i] += 1
                if binj >= 2 * ncls:  # insert bins: the queue slice of the bin
                    q = blk * chunk + b0 + np.arange(b1 - b0)
                    assert q.max() < L["queue"]
                    top["queue"] = max(top["queue"], int(q.max()))
    # each valid operation is handled by exactly one class kernel
    valid_all = (ops[:n] <= 2) & (fids[:n] < nfilters)
    valid_all &= cls[np.minimum(fids[:n], nfilters - 1)] < ncls
    assert np.array_equal(seen[:n], valid_all.astype(np.int64))
    return top


def model_apply(n, apply_grid, max_batch):
    L = layout(max_batch)
    grid = min((n + K_BLOCK - 1) // K_BLOCK, apply_grid)
    per = grid * K_BLOCK
    seg = ((n + per - 1) // per) * K_BLOCK
    assert grid * seg <= L["queue"], (n, grid, seg)
    return grid * seg - 1


def _multi_batch(rng, nf, n, classes):
    """The multi-filter benchmark's batch shape: filters drawn in proportion
    to slot count (2^12..2^26), kinds 60/30/10."""
    e = rng.integers(12, 27, nf)
    w = (2.0 ** e) / (2.0 ** e).sum()
    fids = rng.choice(nf, n, p=w).astype(np.uint32)
    u = rng.random(n)
    ops = np.where(u < 0.6, 0, np.where(u < 0.9, 2, 1)).astype(np.uint8)
    cls = rng.integers(0, classes, nf).astype(np.uint8)
    return ops, fids, cls


@pytest.mark.parametrize("chunk", [64, 512, 2048, 4096])
def test_multi_benchmark_shape_stays_in_bounds(chunk):
    rng = np.random.default_rng(chunk)
    max_batch = n = 1 << 22
    ops, fids, cls = _multi_batch(rng, 256, n, 2)
    grid = (n + chunk - 1) // chunk
    top = model_batch(ops, fids, cls, 2, chunk, n, grid, max_batch)
    L = layout(max_batch)
    assert all(top[k] < L[k] for k in top)


@pytest.mark.parametrize("n", [0, 1, 1000, (1 << 22) - 5])
def test_graph_launch_grid_for_max_batch_with_smaller_batches(n):
    """A graph is captured with the grid for max_batch and reads n on the
    device: blocks past n see an empty chunk and all-zero bin offsets."""
    rng = np.random.default_rng(n)
    max_batch, chunk = 1 << 22, 2048
    ops, fids, cls = _multi_batch(rng, 256, max_batch, 2)
    grid = (max_batch + chunk - 1) // chunk
    model_batch(ops, fids, cls, 2, chunk, n, grid, max_batch)


def test_sixteen_classes_and_invalid_operations():
    rng = np.random.default_rng(16)
    max_batch, n, chunk = 1 << 18, (1 << 18) - 77, 64
    ops, fids, cls = _multi_batch(rng, 300, max_batch, 16)
    ops[rng.integers(0, n, 500)] = 7           # unknown kind
    fids[rng.integers(0, n, 500)] = 10_000     # unknown filter
    cls[rng.integers(0, 300, 20)] = 0xFF       # detached filters
    grid = (n + chunk - 1) // chunk
    model_batch(ops, fids, cls, 16, chunk, n, grid, max_batch)


@pytest.mark.parametrize("n", [1, 255, 256, 257, 1 << 20, 1 << 22])
@pytest.mark.parametrize("apply_grid", [16 * 256, 4096, 16])
def test_apply_insert_queue_in_bounds(n, apply_grid):
    model_apply(n, min(apply_grid, K_APPLY_GRID), 1 << 22)


@pytest.mark.parametrize("ncls,grid", [(1, 1), (2, 2048), (16, 64), (3, 4097)])
def test_phase_kernels_give_each_chunk_and_class_one_block(ncls, grid):
    """The one-launch-per-phase form (cf_set_shape.fused) launches grid x ncls
    blocks and block k works on chunk k / ncls, class k % ncls, bin
    phase * ncls + class: every (chunk, bin) of a phase is visited by exactly
    one block, so the reads, result writes and queue slices are the class
    kernels' own (checked above), only launched together."""
    nb = 3 * ncls
    for phase in range(3):
        seen = np.zeros((grid, nb), dtype=np.int64)
        k = np.arange(grid * ncls)
        cid, c = k // ncls, k % ncls
        assert cid.max() == grid - 1
        np.add.at(seen, (cid, phase * ncls + c), 1)
        want = np.zeros((grid, nb), dtype=np.int64)
        want[:, phase * ncls:(phase + 1) * ncls] = 1
        assert np.array_equal(seen, want)
