"""ctypes binding of libcf.so (include/cf.h, include/cf_keygen.h).

Argument marshalling only: every step of insert, query and delete runs in the
HIP kernels of libcf.so.  Functions keep the C names; tensors are passed as
raw device pointers and the stream defaults to torch's current stream on the
tensor's device.  If libcf.so has not been built the import of this module
fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcf.so")

CF_OK, CF_EINVAL, CF_ENOMEM, CF_EDEVICE, CF_EUNSUPPORTED = 0, 1, 2, 3, 4
CF_HASH_FMIX64, CF_HASH_XXH64 = 0, 1
CF_EVICT_BFS, CF_EVICT_DFS = 0, 1
CF_PLACE_XOR, CF_PLACE_OFFSET = 0, 1

_STATUS = {0: "CF_OK", 1: "CF_EINVAL", 2: "CF_ENOMEM", 3: "CF_EDEVICE", 4: "CF_EUNSUPPORTED"}


class CfError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


class cf_params(ctypes.Structure):  # noqa: N801 (C name)
    _fields_ = [
        ("num_buckets", ctypes.c_uint64),
        ("slots_per_bucket", ctypes.c_uint32),
        ("fp_bits", ctypes.c_uint32),
        ("hash", ctypes.c_uint32),
        ("evict", ctypes.c_uint32),
        ("max_evict", ctypes.c_uint32),
        ("lost_capacity", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("placement", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


EXPORTED = [
    "cf_table_bytes", "cf_create", "cf_create_in", "cf_destroy", "cf_reserve", "cf_insert",
    "cf_query",
    "cf_delete", "cf_count", "cf_failures", "cf_lost", "cf_export", "cf_import", "cf_reset",
    "cf_get_params", "cf_last_error", "cf_keygen", "cf_keygen_at", "cf_probe_lines",
    "cf_probe_atomics", "cf_insert_noalloc",
    "cf_set_create", "cf_set_bytes", "cf_set_destroy", "cf_set_execute", "cf_set_graph_create",
    "cf_graph_launch", "cf_graph_destroy", "cf_set_counts", "cf_set_failures", "cf_set_export",
    "cf_set_import", "cf_set_lost", "cf_set_get_shape", "cf_set_set_shape",
    "cf_set_persistent_capacity", "cf_set_status", "cf_set_phase_ticks",
    "cf_set_attach", "cf_set_detach", "cf_set_attached", "cf_set_apply",
]

CF_SET_DEFER_TABLES = 1

CF_OP_QUERY, CF_OP_DELETE, CF_OP_INSERT = 0, 1, 2


class cf_set_shape(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("persistent", ctypes.c_uint32), ("block", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32), ("wave_bfs", ctypes.c_uint32),
                ("fused", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {"chunk": self.chunk, "streams": self.streams, "persistent": self.persistent,
                "block": self.block, "blocks_per_cu": self.blocks_per_cu,
                "wave_bfs": self.wave_bfs, "fused": self.fused}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
            f"g.build()'` (hipcc, gfx950). There is no CPU fallback.")
    # torch ships its own HIP runtime under the soname libamdhip64.so.7.  Loading
    # it first makes libcf.so bind to that same runtime; loaded the other way
    # round, the process would map two runtimes and the library would not see
    # the device, streams or allocations torch set up.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    u64, u32, vp, st = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "cf_table_bytes": (u64, [P(cf_params)]),
        "cf_create": (st, [P(cf_params), P(vp)]),
        "cf_create_in": (st, [P(cf_params), vp, u64, P(vp)]),
        "cf_destroy": (st, [vp]),
        "cf_reserve": (st, [vp, u64]),
        "cf_insert": (st, [vp, vp, u64, vp, vp, vp]),
        "cf_insert_noalloc": (st, [vp, vp, u64, vp, vp, vp]),
        "cf_query": (st, [vp, vp, u64, vp, vp]),
        "cf_delete": (st, [vp, vp, u64, vp, vp]),
        "cf_count": (st, [vp, vp, vp]),
        "cf_failures": (st, [vp, vp, vp]),
        "cf_lost": (st, [vp, vp, vp, u64, P(u64)]),
        "cf_export": (st, [vp, vp, u64, vp]),
        "cf_import": (st, [vp, vp, u64, vp]),
        "cf_reset": (st, [vp, vp]),
        "cf_get_params": (st, [vp, P(cf_params)]),
        "cf_last_error": (ctypes.c_char_p, []),
        "cf_keygen": (st, [vp, u64, u64, u64, vp]),
        "cf_keygen_at": (st, [vp, vp, u64, u64, vp]),
        "cf_probe_lines": (st, [vp, u64, u32, u32, u64, u64, vp, vp]),
        "cf_probe_atomics": (st, [vp, u64, u32, u32, u64, u64, vp, vp]),
        "cf_set_create": (st, [P(cf_params), u32, u64, u32, P(vp)]),
        "cf_set_attach": (st, [vp, u32]),
        "cf_set_detach": (st, [vp, u32]),
        "cf_set_attached": (st, [vp, u32, P(ctypes.c_int)]),
        "cf_set_apply": (st, [vp, u32, u32, vp, u64, vp, vp]),
        "cf_set_bytes": (u64, [P(cf_params), u32, u64]),
        "cf_set_destroy": (st, [vp]),
        "cf_set_execute": (st, [vp, vp, vp, vp, u64, vp, vp]),
        "cf_set_graph_create": (st, [vp, vp, vp, vp, vp, vp, P(vp)]),
        "cf_graph_launch": (st, [vp, vp]),
        "cf_graph_destroy": (st, [vp]),
        "cf_set_counts": (st, [vp, vp, vp]),
        "cf_set_failures": (st, [vp, vp, vp]),
        "cf_set_export": (st, [vp, u32, vp, u64, vp]),
        "cf_set_import": (st, [vp, u32, vp, u64, vp]),
        "cf_set_lost": (st, [vp, u32, vp, vp, u64, P(u64)]),
        "cf_set_get_shape": (st, [vp, P(cf_set_shape)]),
        "cf_set_set_shape": (st, [vp, P(cf_set_shape)]),
        "cf_set_persistent_capacity": (u32, [vp, u32]),
        "cf_set_status": (st, [vp, P(u32)]),
        "cf_set_phase_ticks": (st, [vp, P(u64), P(u64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


LIB = _load()


def _check(status: int, where: str) -> None:
    if status != CF_OK:
        msg = LIB.cf_last_error()
        raise CfError(status, where, msg.decode() if msg else "")


def _ptr(t) -> Optional[int]:
    """Device pointer of a tensor (or an int address); None stays None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("tensors passed to libcf must be contiguous")
    return t.data_ptr()


def _stream(stream, *tensors) -> Optional[int]:
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    for t in tensors:
        if t is not None and not isinstance(t, int) and t.is_cuda:
            return torch.cuda.current_stream(t.device).cuda_stream
    return torch.cuda.current_stream().cuda_stream


def _keys_arg(keys):
    import torch
    if isinstance(keys, int):
        raise TypeError("pass keys as a device tensor (or use the *_ptr variants)")
    if not keys.is_cuda:
        raise ValueError("keys must be a device tensor")
    if keys.dtype not in (torch.int64, torch.uint64):
        raise TypeError(f"keys must be 64-bit integers, got {keys.dtype}")
    return keys


def _out_arg(t, n: int, dtype, name: str):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or t.numel() < n:
        raise ValueError(f"{name} must be a device {dtype} tensor of at least {n} elements")
    return t


# ----------------------------------------------------------------- C names

def cf_table_bytes(params: cf_params) -> int:
    return LIB.cf_table_bytes(ctypes.byref(params))


def cf_create(params: cf_params) -> int:
    h = ctypes.c_void_p()
    _check(LIB.cf_create(ctypes.byref(params), ctypes.byref(h)), "cf_create")
    return h.value


def cf_create_in(params: cf_params, table, nbytes: int = None) -> int:
    """A filter whose table is the caller's device buffer `table` (a tensor
    or an address); the caller keeps it alive until cf_destroy."""
    h = ctypes.c_void_p()
    if nbytes is None:
        nbytes = table.numel() * table.element_size()
    _check(LIB.cf_create_in(ctypes.byref(params), _ptr(table), nbytes, ctypes.byref(h)),
           "cf_create_in")
    return h.value


def cf_destroy(handle: int) -> None:
    _check(LIB.cf_destroy(handle), "cf_destroy")


def cf_reserve(handle: int, max_batch: int) -> None:
    _check(LIB.cf_reserve(handle, max_batch), "cf_reserve")


def cf_insert(handle: int, keys, ok=None, kicks=None, stream=None) -> None:
    import torch
    keys = _keys_arg(keys)
    n = keys.numel()
    ok = _out_arg(ok, n, torch.uint8, "ok")
    if kicks is not None:
        kicks = _out_arg(kicks, n, kicks.dtype if kicks.dtype in (torch.int32, torch.uint32)
                         else torch.int32, "kicks")
    _check(LIB.cf_insert(handle, _ptr(keys), n, _ptr(ok), _ptr(kicks),
                         _stream(stream, keys)), "cf_insert")


def cf_insert_noalloc(handle: int, keys, ok=None, kicks=None, stream=None) -> None:
    """cf_insert on the library's fixed per-GPU queue (allocates nothing on
    the device; n <= CF_NOALLOC_MAX_KEYS)."""
    import torch
    keys = _keys_arg(keys)
    n = keys.numel()
    ok = _out_arg(ok, n, torch.uint8, "ok")
    if kicks is not None:
        kicks = _out_arg(kicks, n, kicks.dtype if kicks.dtype in (torch.int32, torch.uint32)
                         else torch.int32, "kicks")
    _check(LIB.cf_insert_noalloc(handle, _ptr(keys), n, _ptr(ok), _ptr(kicks),
                                 _stream(stream, keys)), "cf_insert_noalloc")


CF_NOALLOC_MAX_KEYS = 1 << 22


def cf_query(handle: int, keys, found, stream=None) -> None:
    import torch
    keys = _keys_arg(keys)
    n = keys.numel()
    found = _out_arg(found, n, torch.uint8, "found")
    _check(LIB.cf_query(handle, _ptr(keys), n, _ptr(found), _stream(stream, keys)), "cf_query")


def cf_delete(handle: int, keys, ok=None, stream=None) -> None:
    import torch
    keys = _keys_arg(keys)
    n = keys.numel()
    ok = _out_arg(ok, n, torch.uint8, "ok")
    _check(LIB.cf_delete(handle, _ptr(keys), n, _ptr(ok), _stream(stream, keys)), "cf_delete")


def cf_count(handle: int, stream=None) -> int:
    """Occupancy, copied to the host after the given stream's prior work."""
    import torch
    out = ctypes.c_uint64()
    s = _stream(stream)
    _check(LIB.cf_count(handle, ctypes.addressof(out), s), "cf_count")
    torch.cuda.synchronize()
    return out.value


def cf_failures(handle: int, stream=None) -> int:
    import torch
    out = ctypes.c_uint64()
    _check(LIB.cf_failures(handle, ctypes.addressof(out), _stream(stream)), "cf_failures")
    torch.cuda.synchronize()
    return out.value


def cf_lost(handle: int, cap: int = 1 << 16):
    import numpy as np
    b = np.zeros(max(cap, 1), dtype=np.uint64)
    t = np.zeros(max(cap, 1), dtype=np.uint32)
    n = ctypes.c_uint64()
    _check(LIB.cf_lost(handle, b.ctypes.data, t.ctypes.data, cap, ctypes.byref(n)), "cf_lost")
    return b[:n.value], t[:n.value]


def cf_export(handle: int, dst, nbytes: int, stream=None) -> None:
    _check(LIB.cf_export(handle, _ptr(dst), nbytes, _stream(stream)), "cf_export")


def cf_import(handle: int, src, nbytes: int, stream=None) -> None:
    _check(LIB.cf_import(handle, _ptr(src), nbytes, _stream(stream)), "cf_import")


def cf_reset(handle: int, stream=None) -> None:
    _check(LIB.cf_reset(handle, _stream(stream)), "cf_reset")


def cf_get_params(handle: int) -> cf_params:
    p = cf_params()
    _check(LIB.cf_get_params(handle, ctypes.byref(p)), "cf_get_params")
    return p


def cf_keygen(out, seed: int, start: int = 0, stream=None) -> None:
    _check(LIB.cf_keygen(_ptr(out), out.numel(), seed & (2**64 - 1), start & (2**64 - 1),
                         _stream(stream, out)), "cf_keygen")


def cf_probe_lines(buf, line_bytes: int, width: int, n_reads: int, seed: int, sink,
                   stream=None) -> None:
    """Random single reads of `width` bytes at line starts of the device
    tensor `buf`, whose byte size must be a power-of-two number of lines."""
    nbytes = buf.numel() * buf.element_size()
    n_lines = nbytes // line_bytes
    if n_lines * line_bytes != nbytes or n_lines & (n_lines - 1):
        raise ValueError("buffer must hold a power-of-two number of whole lines")
    _check(LIB.cf_probe_lines(_ptr(buf), n_lines, line_bytes, width, n_reads, seed & (2**64 - 1),
                              _ptr(sink), _stream(stream, buf)), "cf_probe_lines")


def cf_probe_atomics(buf, line_bytes: int, read_first: bool, n_ops: int, seed: int, sink,
                     stream=None) -> None:
    """Random 64-bit CAS at line starts of the device tensor `buf` (scratch:
    its words change), whose byte size must be a power-of-two number of
    lines; with read_first the word is loaded before its CAS."""
    nbytes = buf.numel() * buf.element_size()
    n_lines = nbytes // line_bytes
    if n_lines * line_bytes != nbytes or n_lines & (n_lines - 1):
        raise ValueError("buffer must hold a power-of-two number of whole lines")
    _check(LIB.cf_probe_atomics(_ptr(buf), n_lines, line_bytes, int(bool(read_first)), n_ops,
                                seed & (2**64 - 1), _ptr(sink), _stream(stream, buf)),
           "cf_probe_atomics")


def cf_keygen_at(out, counters, seed: int, stream=None) -> None:
    _check(LIB.cf_keygen_at(_ptr(out), _ptr(counters), out.numel(), seed & (2**64 - 1),
                            _stream(stream, out)), "cf_keygen_at")


# ----------------------------------------------------------------- sets

def _params_array(params):
    arr = (cf_params * len(params))()
    for i, p in enumerate(params):
        arr[i] = p
    return arr


def cf_set_bytes(params, max_batch: int) -> int:
    return LIB.cf_set_bytes(_params_array(params), len(params), max_batch)


def cf_set_create(params, max_batch: int, flags: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(LIB.cf_set_create(_params_array(params), len(params), max_batch, flags,
                             ctypes.byref(h)), "cf_set_create")
    return h.value


def cf_set_attach(handle: int, fid: int) -> None:
    _check(LIB.cf_set_attach(handle, fid), "cf_set_attach")


def cf_set_detach(handle: int, fid: int) -> None:
    _check(LIB.cf_set_detach(handle, fid), "cf_set_detach")


def cf_set_attached(handle: int, fid: int) -> bool:
    out = ctypes.c_int()
    _check(LIB.cf_set_attached(handle, fid, ctypes.byref(out)), "cf_set_attached")
    return bool(out.value)


def cf_set_apply(handle: int, fid: int, op: int, keys, results, stream=None) -> None:
    n = keys.numel()
    if results.numel() < n:
        raise ValueError("results must hold at least len(keys) entries")
    _check(LIB.cf_set_apply(handle, fid, op, _ptr(keys), n, _ptr(results),
                            _stream(stream, keys)), "cf_set_apply")


def cf_set_destroy(handle: int) -> None:
    _check(LIB.cf_set_destroy(handle), "cf_set_destroy")


def cf_set_execute(handle: int, ops, fids, keys, results, stream=None) -> None:
    n = keys.numel()
    if ops.numel() < n or fids.numel() < n or results.numel() < n:
        raise ValueError("ops, fids and results must hold at least len(keys) entries")
    _check(LIB.cf_set_execute(handle, _ptr(ops), _ptr(fids), _ptr(keys), n, _ptr(results),
                              _stream(stream, keys)), "cf_set_execute")


def cf_set_graph_create(handle: int, ops, fids, keys, d_n, results) -> int:
    g = ctypes.c_void_p()
    _check(LIB.cf_set_graph_create(handle, _ptr(ops), _ptr(fids), _ptr(keys), _ptr(d_n),
                                   _ptr(results), ctypes.byref(g)), "cf_set_graph_create")
    return g.value


def cf_graph_launch(graph: int, stream=None) -> None:
    _check(LIB.cf_graph_launch(graph, _stream(stream)), "cf_graph_launch")


def cf_graph_destroy(graph: int) -> None:
    _check(LIB.cf_graph_destroy(graph), "cf_graph_destroy")


def _set_totals(fn, name, handle: int, nfilters: int, stream=None):
    import numpy as np
    import torch
    out = np.zeros(nfilters, dtype=np.uint64)
    _check(fn(handle, out.ctypes.data, _stream(stream)), name)
    torch.cuda.synchronize()
    return out


def cf_set_counts(handle: int, nfilters: int, stream=None):
    return _set_totals(LIB.cf_set_counts, "cf_set_counts", handle, nfilters, stream)


def cf_set_failures(handle: int, nfilters: int, stream=None):
    return _set_totals(LIB.cf_set_failures, "cf_set_failures", handle, nfilters, stream)


def cf_set_export(handle: int, fid: int, dst, nbytes: int, stream=None) -> None:
    _check(LIB.cf_set_export(handle, fid, _ptr(dst), nbytes, _stream(stream)), "cf_set_export")


def cf_set_import(handle: int, fid: int, src, nbytes: int, stream=None) -> None:
    _check(LIB.cf_set_import(handle, fid, _ptr(src), nbytes, _stream(stream)), "cf_set_import")


def cf_set_lost(handle: int, fid: int, cap: int = 1 << 16):
    import numpy as np
    b = np.zeros(max(cap, 1), dtype=np.uint64)
    t = np.zeros(max(cap, 1), dtype=np.uint32)
    n = ctypes.c_uint64()
    _check(LIB.cf_set_lost(handle, fid, b.ctypes.data, t.ctypes.data, cap, ctypes.byref(n)),
           "cf_set_lost")
    return b[:n.value], t[:n.value]


def cf_set_get_shape(handle: int) -> cf_set_shape:
    sh = cf_set_shape()
    _check(LIB.cf_set_get_shape(handle, ctypes.byref(sh)), "cf_set_get_shape")
    return sh


def cf_set_set_shape(handle: int, chunk: int | None = None, streams: int | None = None,
                     persistent: int | None = None, block: int | None = None,
                     blocks_per_cu: int | None = None, wave_bfs: int | None = None,
                     fused: int | None = None) -> None:
    """Fields as in cf_set_shape; a field left None keeps the set's value."""
    cur = cf_set_get_shape(handle)
    sh = cf_set_shape(cur.chunk if chunk is None else chunk,
                      cur.streams if streams is None else streams,
                      cur.persistent if persistent is None else persistent,
                      cur.block if block is None else block,
                      cur.blocks_per_cu if blocks_per_cu is None else blocks_per_cu,
                      cur.wave_bfs if wave_bfs is None else wave_bfs,
                      cur.fused if fused is None else fused)
    _check(LIB.cf_set_set_shape(handle, ctypes.byref(sh)), "cf_set_set_shape")


def cf_set_persistent_capacity(handle: int, block: int = 256) -> int:
    return LIB.cf_set_persistent_capacity(handle, block)


def cf_set_phase_ticks(handle: int):
    """(ticks[4], ticks per second) of the last persistent batch: its start
    and its three barriers (cf_set_phase_ticks)."""
    t = (ctypes.c_uint64 * 4)()
    hz = ctypes.c_uint64()
    _check(LIB.cf_set_phase_ticks(handle, t, ctypes.byref(hz)), "cf_set_phase_ticks")
    return list(t), hz.value


def cf_set_status(handle: int) -> int:
    """1 if a persistent batch abandoned its work (cf_set_status), else 0."""
    e = ctypes.c_uint32()
    _check(LIB.cf_set_status(handle, ctypes.byref(e)), "cf_set_status")
    return e.value


# --------------------------------------------------------------- server

CF_SERVE_BATCHED, CF_SERVE_PER_REQUEST = 0, 1


class cf_server_config(ctypes.Structure):  # noqa: N801 (C name)
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_batch", ctypes.c_uint64),
                ("max_requests", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("depth", ctypes.c_uint32), ("direct_below", ctypes.c_uint32),
                ("solo_above", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class cf_request_info(ctypes.Structure):  # noqa: N801 (C name)
    _fields_ = [("id", ctypes.c_uint64), ("t_submit_ns", ctypes.c_uint64),
                ("t_start_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64),
                ("batch", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_uint32)]


class cf_server_stats(ctypes.Structure):  # noqa: N801 (C name)
    _fields_ = [("requests", ctypes.c_uint64), ("operations", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("held", ctypes.c_uint64),
                ("resident_bytes", ctypes.c_uint64), ("resident", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


def _server_sigs():
    u64, u32, vp, st = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "cf_server_create": (st, [P(cf_params), u32, P(cf_server_config), P(vp)]),
        "cf_server_destroy": (st, [vp]),
        "cf_server_submit": (st, [vp, u32, u32, vp, u64, vp, P(u64)]),
        "cf_server_wait": (st, [vp, u64, P(cf_request_info)]),
        "cf_server_drain": (st, [vp]),
        "cf_server_release": (st, [vp, u32]),
        "cf_server_resident": (st, [vp, u32, P(ctypes.c_int)]),
        "cf_server_stats_get": (st, [vp, P(cf_server_stats)]),
        "cf_server_set": (vp, [vp]),
        "cf_server_replay": (st, [vp, u64, vp, vp, vp, vp, vp, vp, vp, P(u64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(LIB, name)
        fn.restype = res
        fn.argtypes = args
    EXPORTED.extend(sig)


_server_sigs()


def cf_server_create(params, config: cf_server_config) -> int:
    h = ctypes.c_void_p()
    _check(LIB.cf_server_create(_params_array(params), len(params), ctypes.byref(config),
                                ctypes.byref(h)), "cf_server_create")
    return h.value


def cf_server_destroy(handle: int) -> None:
    _check(LIB.cf_server_destroy(handle), "cf_server_destroy")


def cf_server_submit(handle: int, fid: int, op: int, keys, results) -> int:
    rid = ctypes.c_uint64()
    n = keys.numel()
    _check(LIB.cf_server_submit(handle, fid, op, _ptr(keys), n, _ptr(results),
                                ctypes.byref(rid)), "cf_server_submit")
    return rid.value


def cf_server_wait(handle: int, rid: int) -> cf_request_info:
    info = cf_request_info()
    _check(LIB.cf_server_wait(handle, rid, ctypes.byref(info)), "cf_server_wait")
    return info


def cf_server_drain(handle: int) -> None:
    _check(LIB.cf_server_drain(handle), "cf_server_drain")


def cf_server_release(handle: int, fid: int) -> None:
    _check(LIB.cf_server_release(handle, fid), "cf_server_release")


def cf_server_resident(handle: int, fid: int) -> bool:
    out = ctypes.c_int()
    _check(LIB.cf_server_resident(handle, fid, ctypes.byref(out)), "cf_server_resident")
    return bool(out.value)


def cf_server_stats_get(handle: int) -> cf_server_stats:
    out = cf_server_stats()
    _check(LIB.cf_server_stats_get(handle, ctypes.byref(out)), "cf_server_stats_get")
    return out


def cf_server_set(handle: int) -> int:
    return LIB.cf_server_set(handle)


def cf_server_replay(handle: int, arrival_ns, fids, ops, key_off, n, keys, results) -> int:
    """Replay a trace (host numpy arrays) against device key/result pools."""
    import numpy as np
    arrs = [np.ascontiguousarray(a, dtype=d) for a, d in
            ((arrival_ns, np.uint64), (fids, np.uint32), (ops, np.uint32),
             (key_off, np.uint64), (n, np.uint64))]
    first = ctypes.c_uint64()
    _check(LIB.cf_server_replay(handle, arrs[0].size, *[a.ctypes.data for a in arrs],
                                _ptr(keys), _ptr(results), ctypes.byref(first)),
           "cf_server_replay")
    return first.value


# ----------------------------------------------------------------- tuning

class cf_tune_goal(ctypes.Structure):  # noqa: N801 (C name)
    _fields_ = [("capacity", ctypes.c_uint64), ("max_load", ctypes.c_double),
                ("max_fpr", ctypes.c_double), ("max_bytes", ctypes.c_uint64),
                ("mix", ctypes.c_double * 3), ("positive_share", ctypes.c_double),
                ("hash", ctypes.c_uint32), ("evict", ctypes.c_uint32),
                ("max_evict", ctypes.c_uint32), ("measure", ctypes.c_uint32),
                ("probe_bytes", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("placements", ctypes.c_uint32), ("tie_permille", ctypes.c_uint32)]


class cf_tune_candidate(ctypes.Structure):  # noqa: N801 (C name)
    _fields_ = [("params", cf_params), ("bytes", ctypes.c_uint64),
                ("probe_buckets", ctypes.c_uint64), ("load", ctypes.c_double),
                ("fpr", ctypes.c_double), ("rate", ctypes.c_double * 3),
                ("ns_per_op", ctypes.c_double), ("feasible", ctypes.c_uint32),
                ("probe_failures", ctypes.c_uint32)]


class cf_set_trial(ctypes.Structure):  # noqa: N801 (C name)
    _fields_ = [("shape", cf_set_shape), ("ms", ctypes.c_double)]


CF_SET_TUNE_MAX_TRIALS = 64


def _tune_sigs():
    u64, u32, vp, st = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "cf_tune_geometry": (st, [P(cf_tune_goal), vp, u32, P(u32), P(cf_params), vp]),
        "cf_set_tune": (st, [vp, vp, vp, vp, u64, vp, u32, u32, u32, vp, u32, P(u32),
                             P(cf_set_shape), P(u64), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(LIB, name)
        fn.restype = res
        fn.argtypes = args
    EXPORTED.extend(sig)


_tune_sigs()


def cf_tune_geometry(goal: cf_tune_goal, stream=None, raise_infeasible: bool = True):
    """Returns (best params or None, list of candidates, best first)."""
    n = ctypes.c_uint32()
    cands = (cf_tune_candidate * 24)()
    best = cf_params()
    # the model alone touches no device: no stream is resolved for it
    st = _stream(stream) if goal.measure else None
    status = LIB.cf_tune_geometry(ctypes.byref(goal), ctypes.cast(cands, ctypes.c_void_p), 24,
                                  ctypes.byref(n), ctypes.byref(best), st)
    out = [cands[k] for k in range(min(n.value, 24))]
    if status != CF_OK:
        if status == CF_EINVAL and out and not raise_infeasible:
            return None, out
        _check(status, "cf_tune_geometry")
    return best, out


CF_SET_TUNE_EAGER = 1


def cf_set_tune(handle: int, ops, fids, keys, shapes=None, reps: int = 0, stream=None,
                eager: bool = False):
    """shapes: None (the library's default candidates) or a list of dicts with
    cf_set_shape's fields (missing fields 0).  eager: time cf_set_execute
    calls instead of launches of a graph captured per candidate.  Returns
    (chosen shape dict, [(shape dict, median ms)], failed insertions)."""
    n = keys.numel()
    if shapes is None:
        arr, ns = None, 0
    else:
        arr = (cf_set_shape * max(len(shapes), 1))()
        for k, d in enumerate(shapes):
            arr[k] = cf_set_shape(d.get("chunk", 0), d.get("streams", 0),
                                  d.get("persistent", 0), d.get("block", 0),
                                  d.get("blocks_per_cu", 0), d.get("wave_bfs", 0),
                                  d.get("fused", 0))
        ns = len(shapes)
    cap = max(ns, CF_SET_TUNE_MAX_TRIALS)
    trials = (cf_set_trial * cap)()
    ntr = ctypes.c_uint32()
    shape = cf_set_shape()
    fails = ctypes.c_uint64()
    _check(LIB.cf_set_tune(handle, _ptr(ops), _ptr(fids), _ptr(keys), n,
                           None if arr is None else ctypes.cast(arr, ctypes.c_void_p), ns, reps,
                           CF_SET_TUNE_EAGER if eager else 0,
                           ctypes.cast(trials, ctypes.c_void_p), cap, ctypes.byref(ntr),
                           ctypes.byref(shape), ctypes.byref(fails), _stream(stream, keys)),
           "cf_set_tune")
    done = [(t.shape.as_dict(), t.ms) for t in trials[:min(ntr.value, cap)]]
    return shape.as_dict(), done, fails.value
