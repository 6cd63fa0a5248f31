"""Helpers shared by the GPU tests: host <-> device copies of uint64 arrays
(carried as int64 tensors, same bits) and the multiset comparison used for
concurrent inserts."""
from __future__ import annotations

import numpy as np

GEOMS = [(4, 8), (8, 8), (16, 8), (32, 8), (4, 16), (8, 16), (16, 16), (32, 16),
         (4, 32), (8, 32), (16, 32), (32, 32)]  # (b, f)


def dev_u64(arr):
    import torch
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.uint64))
    return torch.from_numpy(a.view(np.int64)).to("cuda")


def host_u64(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def dev_zeros_u8(n):
    import torch
    return torch.zeros(max(n, 1), dtype=torch.uint8, device="cuda")[:n]


def dev_zeros_u32(n):
    import torch
    return torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")[:n]


def _rows(lo, hi, tag):
    rows = np.empty(len(lo), dtype=[("lo", "<u8"), ("hi", "<u8"), ("t", "<u4")])
    rows["lo"], rows["hi"], rows["t"] = lo, hi, tag
    rows.sort(order=("lo", "hi", "t"))
    return rows


def multiset_equal(a, b) -> bool:
    """Two (lo, hi, tag) triple lists hold the same multiset."""
    ra, rb = _rows(*a), _rows(*b)
    return ra.shape == rb.shape and bool(np.array_equal(ra, rb))


def expected_groups(ref, keys, ok_mask=None, lost=None):
    """Key-derived multiset: one (pair, fp) per inserted key (those with
    ok_mask set, if given), minus the dropped (bucket, tag) pairs."""
    lo, hi, fp = ref.key_groups(keys)
    if ok_mask is not None and lost is None:
        lo, hi, fp = lo[ok_mask], hi[ok_mask], fp[ok_mask]
    if lost is not None:
        lb, lt = lost
        alo, ahi, at = ref.pair_groups(lb, lt)
        rows = _rows(lo, hi, fp)
        drop = _rows(alo, ahi, at)
        # multiset difference rows - drop
        keep = np.ones(rows.size, dtype=bool)
        j = 0
        for r in drop:
            while j < rows.size and (rows[j]["lo"], rows[j]["hi"], rows[j]["t"]) < \
                    (r["lo"], r["hi"], r["t"]):
                j += 1
            assert j < rows.size and rows[j] == r, "dropped tag not among inserted keys"
            keep[j] = False
            j += 1
        rows = rows[keep]
        return rows["lo"], rows["hi"], rows["t"]
    return lo, hi, fp
