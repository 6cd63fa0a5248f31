"""MI355X-native partial-key cuckoo filter (Cuckoo-GPU, arXiv 2603.15486).

The filter's work runs in hand-written HIP kernels for gfx950 behind the C ABI
of ``include/cf.h`` (``libcf.so``).  This package is the thin Python layer:
``_binding`` mirrors the C functions one for one and ``CuckooFilter`` wraps a
handle for use with torch device tensors and streams.
"""
from __future__ import annotations

from typing import Optional

from ._binding import (  # noqa: F401
    CF_SERVE_BATCHED, CF_SERVE_PER_REQUEST, cf_request_info, cf_server_config, cf_server_create,
    cf_server_destroy, cf_server_drain, cf_server_release, cf_server_replay, cf_server_resident,
    cf_server_set, cf_server_stats, cf_server_stats_get, cf_server_submit, cf_server_wait,
    CF_OP_DELETE, CF_OP_INSERT, CF_OP_QUERY, CF_SET_DEFER_TABLES, cf_set_apply, cf_set_attach,
    cf_set_attached, cf_set_detach, cf_graph_destroy, cf_graph_launch, cf_set_bytes,
    cf_set_counts, cf_set_create, cf_set_destroy, cf_set_execute, cf_set_export,
    cf_set_failures, cf_set_get_shape, cf_set_graph_create, cf_set_import, cf_set_lost,
    cf_set_set_shape, cf_set_shape, CF_EDEVICE, CF_EINVAL, CF_ENOMEM, CF_EUNSUPPORTED, CF_OK, EXPORTED, CF_EVICT_BFS, CF_EVICT_DFS, CF_HASH_FMIX64, CF_HASH_XXH64, CF_PLACE_XOR, CF_PLACE_OFFSET, LIB, LIB_PATH, CfError, cf_count,
    cf_create, cf_create_in, cf_delete, cf_destroy, cf_export, cf_failures, cf_get_params, cf_import, cf_insert,
    cf_keygen, cf_keygen_at, cf_probe_atomics, cf_probe_lines, cf_lost, cf_params, cf_query, cf_reserve, cf_reset, cf_table_bytes)
from ._binding import cf_set_trial, cf_set_tune, cf_tune_candidate, cf_tune_geometry, cf_tune_goal  # noqa: F401,E501
from ._binding import cf_set_persistent_capacity, cf_set_phase_ticks, cf_set_status  # noqa: F401
from ._binding import CF_NOALLOC_MAX_KEYS, cf_insert_noalloc  # noqa: F401


def tune_geometry(capacity: int, max_fpr: float = 0.0, max_load: float = 0.95,
                  max_bytes: int = 0, mix=(1.0, 1.0, 1.0), positive_share: float = 0.5,
                  hash: int = CF_HASH_FMIX64, evict: int = CF_EVICT_BFS, max_evict: int = 0,
                  measure: bool = True, probe_bytes: int = 0, seed: int = 0, stream=None,
                  raise_infeasible: bool = True, placements: int = 0,
                  tie_permille: int = 0):
    """Choose (b, f, m) for a filter of `capacity` keys (cf_tune_geometry).
    mix: weights of (query, delete, insert).  Returns (params or None, list
    of candidate dicts, best first)."""
    goal = cf_tune_goal(capacity, max_load, max_fpr, max_bytes, (ctypes_double3(mix)),
                        positive_share, hash, evict, max_evict, 1 if measure else 0,
                        probe_bytes, seed & (2**64 - 1), placements, tie_permille)
    best, cands = cf_tune_geometry(goal, stream, raise_infeasible)
    rows = [{"slots_per_bucket": c.params.slots_per_bucket, "fp_bits": c.params.fp_bits,
             "placement": c.params.placement,
             "num_buckets": c.params.num_buckets, "bytes": c.bytes, "load": c.load,
             "fpr": c.fpr, "feasible": bool(c.feasible), "probe_buckets": c.probe_buckets,
             "query_per_s": c.rate[0], "delete_per_s": c.rate[1], "insert_per_s": c.rate[2],
             "ns_per_op": c.ns_per_op, "probe_failures": c.probe_failures} for c in cands]
    return best, rows


def ctypes_double3(v):
    import ctypes
    return (ctypes.c_double * 3)(*[float(x) for x in v])


def make_params(num_buckets: int, slots_per_bucket: int = 16, fp_bits: int = 16,
                hash: int = CF_HASH_FMIX64, evict: int = CF_EVICT_BFS, max_evict: int = 128,
                seed: int = 0, lost_capacity: int = 0,
                placement: int = CF_PLACE_XOR) -> cf_params:
    return cf_params(num_buckets, slots_per_bucket, fp_bits, hash, evict, max_evict,
                     lost_capacity, seed & (2**64 - 1), placement, 0)


class CuckooFilter:
    """One filter on one device: m buckets x b slots x f-bit fingerprints."""

    def __init__(self, num_buckets: int, slots_per_bucket: int = 16, fp_bits: int = 16,
                 hash: int = CF_HASH_FMIX64, evict: int = CF_EVICT_BFS, max_evict: int = 128,
                 seed: int = 0, lost_capacity: int = 0, device=None,
                 placement: int = CF_PLACE_XOR, table=None):
        """table (optional): a device tensor of at least cf_table_bytes bytes,
        16-byte aligned, that holds the table (cf_create_in); it is zeroed, and
        kept referenced here for the filter's lifetime."""
        import torch
        self.params = make_params(num_buckets, slots_per_bucket, fp_bits, hash, evict,
                                  max_evict, seed, lost_capacity, placement)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self._table = table
        with torch.cuda.device(self.device):
            if table is None:
                self.handle = cf_create(self.params)
            else:
                torch.cuda.synchronize(self.device)  # the table's prior writers are done
                self.handle = cf_create_in(self.params, table)
        self.table_bytes = cf_table_bytes(self.params)

    @property
    def num_buckets(self) -> int:
        return self.params.num_buckets

    @property
    def slots_per_bucket(self) -> int:
        return self.params.slots_per_bucket

    @property
    def fp_bits(self) -> int:
        return self.params.fp_bits

    @property
    def capacity(self) -> int:
        return self.params.num_buckets * self.params.slots_per_bucket

    def close(self) -> None:
        if getattr(self, "handle", None):
            cf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, max_batch: int) -> None:
        cf_reserve(self.handle, max_batch)

    def insert(self, keys, ok=None, kicks=None, stream=None):
        cf_insert(self.handle, keys, ok, kicks, stream)
        return ok

    def insert_noalloc(self, keys, ok=None, kicks=None, stream=None):
        """insert() on the library's fixed per-GPU queue: no device
        allocation, at most CF_NOALLOC_MAX_KEYS keys, and calls on one GPU
        must not overlap in time."""
        cf_insert_noalloc(self.handle, keys, ok, kicks, stream)
        return ok

    def query(self, keys, found=None, stream=None):
        import torch
        if found is None:
            found = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        cf_query(self.handle, keys, found, stream)
        return found

    def delete(self, keys, ok=None, stream=None):
        cf_delete(self.handle, keys, ok, stream)
        return ok

    def count(self, stream=None) -> int:
        return cf_count(self.handle, stream)

    def failures(self, stream=None) -> int:
        return cf_failures(self.handle, stream)

    def lost(self, cap: int = 1 << 16):
        return cf_lost(self.handle, cap)

    def export_table(self, out=None, stream=None):
        """Raw table words as a device int64 tensor (bits of the uint64 words, Fig. 2)."""
        import torch
        if out is None:
            out = torch.empty(self.table_bytes // 8, dtype=torch.int64, device=self.device)
        cf_export(self.handle, out, self.table_bytes, stream)
        return out

    def import_table(self, words, stream=None) -> None:
        cf_import(self.handle, words, self.table_bytes, stream)

    def reset(self, stream=None) -> None:
        cf_reset(self.handle, stream)


class CuckooFilterSet:
    """Many filters on one device, driven by mixed batches of (kind, filter id,
    key) operations: queries see the state before the batch, then deletes,
    then inserts run (per filter)."""

    def __init__(self, params, max_batch: int, device=None, defer_tables: bool = False):
        import torch
        self.params = list(params)
        self.nfilters = len(self.params)
        self.max_batch = int(max_batch)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            self.handle = cf_set_create(self.params, self.max_batch,
                                        CF_SET_DEFER_TABLES if defer_tables else 0)
        self._graphs = []

    def close(self) -> None:
        for g in self._graphs:
            cf_graph_destroy(g)
        self._graphs = []
        if getattr(self, "handle", None):
            cf_set_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def table_bytes(self, fid: int) -> int:
        return cf_table_bytes(self.params[fid])

    def execute(self, ops, fids, keys, results=None, stream=None):
        import torch
        if results is None:
            results = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        cf_set_execute(self.handle, ops, fids, keys, results, stream)
        return results

    def graph(self, ops, fids, keys, d_n, results) -> int:
        """Capture the batch execution for these fixed buffers; d_n (device
        uint64) holds the operation count at launch time.  The set owns the
        graph: close() or drop_graph() destroys it (never cf_graph_destroy
        on it directly, which would free it twice)."""
        g = cf_set_graph_create(self.handle, ops, fids, keys, d_n, results)
        self._graphs.append(g)
        return g

    def drop_graph(self, g: int) -> None:
        """Destroy one graph made by graph()."""
        self._graphs.remove(g)
        cf_graph_destroy(g)

    def attach(self, fid: int) -> None:
        cf_set_attach(self.handle, fid)

    def detach(self, fid: int) -> None:
        cf_set_detach(self.handle, fid)

    def attached(self, fid: int) -> bool:
        return cf_set_attached(self.handle, fid)

    def apply(self, fid: int, op: int, keys, results=None, stream=None):
        """One operation kind on one filter, as a single launch."""
        import torch
        if results is None:
            results = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        cf_set_apply(self.handle, fid, op, keys, results, stream)
        return results

    def counts(self, stream=None):
        return cf_set_counts(self.handle, self.nfilters, stream)

    def failures(self, stream=None):
        return cf_set_failures(self.handle, self.nfilters, stream)

    def lost(self, fid: int, cap: int = 1 << 16):
        return cf_set_lost(self.handle, fid, cap)

    def export_table(self, fid: int, stream=None):
        import torch
        out = torch.empty(self.table_bytes(fid) // 8, dtype=torch.int64, device=self.device)
        cf_set_export(self.handle, fid, out, self.table_bytes(fid), stream)
        return out

    def import_table(self, fid: int, words, stream=None) -> None:
        cf_set_import(self.handle, fid, words, self.table_bytes(fid), stream)

    def tune(self, ops, fids, keys, shapes=None, reps: int = 0, stream=None,
             eager: bool = False):
        """Time this batch under candidate launch shapes (dicts of cf_set_shape
        fields; None = the library's defaults) and keep the fastest
        (cf_set_tune; the batch is undone after every trial).  Each candidate
        is timed as launches of a graph captured for it, or with eager=True as
        cf_set_execute calls.  Returns (shape dict, [(shape dict, median ms)],
        failed insertions)."""
        return cf_set_tune(self.handle, ops, fids, keys, shapes, reps, stream, eager)

    @property
    def shape(self) -> dict:
        return cf_set_get_shape(self.handle).as_dict()

    def set_shape(self, **fields) -> None:
        """Change some cf_set_shape fields (chunk, streams, persistent, block,
        blocks_per_cu, wave_bfs, fused); the others keep their values."""
        cf_set_set_shape(self.handle, **fields)

    def persistent_capacity(self, block: int = 256) -> int:
        """Most blocks per compute unit of the persistent form (0: not
        available for this set)."""
        return cf_set_persistent_capacity(self.handle, block)

    def status(self) -> int:
        """1 if a persistent batch abandoned its work (cf_set_status)."""
        return cf_set_status(self.handle)

    def persistent_phase_us(self):
        """Microseconds the last persistent batch spent partitioning, then on
        its queries and its deletes (between its barriers), from
        cf_set_phase_ticks; the inserts run from the third barrier to the
        kernel's end."""
        t, hz = cf_set_phase_ticks(self.handle)
        return [round((t[k + 1] - t[k]) * 1e6 / hz, 1) for k in range(3)]

    @property
    def chunk(self) -> int:
        return cf_set_get_shape(self.handle).chunk

    @chunk.setter
    def chunk(self, value: int) -> None:
        cf_set_set_shape(self.handle, chunk=value)

    @property
    def streams(self) -> int:
        """Streams the class chains run on concurrently (cf_set_shape.streams;
        0 = default)."""
        return cf_set_get_shape(self.handle).streams

    @streams.setter
    def streams(self, value: int) -> None:
        cf_set_set_shape(self.handle, streams=value)

    @property
    def persistent(self) -> bool:
        return bool(cf_set_get_shape(self.handle).persistent)

    @persistent.setter
    def persistent(self, value: bool) -> None:
        cf_set_set_shape(self.handle, persistent=int(bool(value)))


class _SetView(CuckooFilterSet):
    """A CuckooFilterSet over a set owned by someone else (a server)."""

    def __init__(self, handle, params, max_batch, device):
        self.handle = handle
        self.params = list(params)
        self.nfilters = len(self.params)
        self.max_batch = max_batch
        self.device = device
        self._graphs = []

    def close(self) -> None:
        self.handle = None


class CuckooServer:
    """Continuous-batching request loop over many resident filters (or, with
    per_request=True, one launch per request: the baseline)."""

    def __init__(self, params, max_batch: int, hbm_budget: int = 0, max_requests: int = 4096,
                 depth: int = 2, per_request: bool = False, direct_below: int = 0,
                 solo_above: int = 0, device=None):
        import torch
        self.params = list(params)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        cfg = cf_server_config(hbm_budget, max_batch, max_requests,
                               CF_SERVE_PER_REQUEST if per_request else CF_SERVE_BATCHED,
                               depth, direct_below, solo_above)
        with torch.cuda.device(self.device):
            self.handle = cf_server_create(self.params, cfg)
        self.set = _SetView(cf_server_set(self.handle), self.params, max_batch, self.device)

    def close(self) -> None:
        if getattr(self, "handle", None):
            cf_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, fid: int, op: int, keys, results) -> int:
        return cf_server_submit(self.handle, fid, op, keys, results)

    def wait(self, rid: int):
        return cf_server_wait(self.handle, rid)

    def drain(self) -> None:
        cf_server_drain(self.handle)

    def release(self, fid: int) -> None:
        cf_server_release(self.handle, fid)

    def resident(self, fid: int) -> bool:
        return cf_server_resident(self.handle, fid)

    def stats(self):
        return cf_server_stats_get(self.handle)

    def replay(self, arrival_ns, fids, ops, key_off, n, keys, results) -> int:
        return cf_server_replay(self.handle, arrival_ns, fids, ops, key_off, n, keys, results)
