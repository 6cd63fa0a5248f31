"""Plain sequential CPU oracle for the partial-key cuckoo filter.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the benchmark's ``cpu_baseline`` leg may import this package.  It shares no
code with the GPU library (``paper_2603_15486_amd``) and never imports it.

The arithmetic lives in ``cfo.c`` (plain C, one slot at a time); this module
only loads it with ctypes and marshals numpy arrays.  Function-level citations
of the paper (Cuckoo-GPU, arXiv 2603.15486) are in ``cfo.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cfo.c")
_LIB = os.path.join(_HERE, "libcfo.so")

HASH_FMIX64 = 0
HASH_XXH64 = 1
EVICT_BFS = 0
EVICT_DFS = 1
PLACE_XOR = 0      # Eq. (3), m a power of two
PLACE_OFFSET = 1   # Sec. 4.6.2, offset + choice bit, any m


def build(force: bool = False) -> str:
    """Compile cfo.c into libcfo.so with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        vp = ctypes.c_void_p
        L.cfo_fmix64.restype = u64
        L.cfo_fmix64.argtypes = [u64]
        L.cfo_xxh64_u64.restype = u64
        L.cfo_xxh64_u64.argtypes = [u64]
        L.cfo_hash.restype = u64
        L.cfo_hash.argtypes = [u32, u64]
        L.cfo_splitmix64_at.restype = u64
        L.cfo_splitmix64_at.argtypes = [u64, u64]
        L.cfo_create.restype = vp
        L.cfo_create.argtypes = [u64, u32, u32, u32, u32, u32, u64]
        L.cfo_destroy.restype = None
        L.cfo_destroy.argtypes = [vp]
        L.cfo_derive.restype = None
        L.cfo_derive.argtypes = [vp, u64, ctypes.POINTER(u32), ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.cfo_alt.restype = u64
        L.cfo_alt.argtypes = [vp, u64, u32]
        L.cfo_insert.restype = i32
        L.cfo_insert.argtypes = [vp, u64, ctypes.POINTER(u32)]
        L.cfo_query.restype = i32
        L.cfo_query.argtypes = [vp, u64]
        L.cfo_delete.restype = i32
        L.cfo_delete.argtypes = [vp, u64]
        L.cfo_insert_batch.restype = None
        L.cfo_insert_batch.argtypes = [vp, vp, u64, vp, vp]
        L.cfo_query_batch.restype = None
        L.cfo_query_batch.argtypes = [vp, vp, u64, vp]
        L.cfo_delete_batch.restype = None
        L.cfo_delete_batch.argtypes = [vp, vp, u64, vp]
        L.cfo_get_slot.restype = u32
        L.cfo_get_slot.argtypes = [vp, u64, u32]
        L.cfo_num_words.restype = u64
        L.cfo_num_words.argtypes = [vp]
        L.cfo_words.restype = vp
        L.cfo_words.argtypes = [vp]
        L.cfo_load_words.restype = None
        L.cfo_load_words.argtypes = [vp, vp, u64]
        for name in ("cfo_count", "cfo_failures", "cfo_lost_count"):
            getattr(L, name).restype = u64
            getattr(L, name).argtypes = [vp]
        L.cfo_lost.restype = u64
        L.cfo_lost.argtypes = [vp, vp, vp, u64]
        L.cfo_derive_batch.restype = None
        L.cfo_derive_batch.argtypes = [vp, vp, u64, vp, vp, vp]
        L.cfo_stored_groups.restype = u64
        L.cfo_stored_groups.argtypes = [vp, vp, vp, vp, u64]
        L.cfo_group_digest_keys.restype = u64
        L.cfo_group_digest_keys.argtypes = [vp, vp, u64]
        L.cfo_group_digest_table.restype = u64
        L.cfo_group_digest_table.argtypes = [vp, u64, u64]
        L.cfo_group_digest_pairs.restype = u64
        L.cfo_group_digest_pairs.argtypes = [vp, vp, vp, u64]
        L.cfo_load_words_nocount.restype = None
        L.cfo_load_words_nocount.argtypes = [vp, vp, u64]
        L.cfo_table_fpr.restype = ctypes.c_double
        L.cfo_table_fpr.argtypes = [vp]
        L.cfo_create_placed.restype = vp
        L.cfo_create_placed.argtypes = [u64, u32, u32, u32, u32, u32, u64, u32]
        L.cfo_derive_tags.restype = None
        L.cfo_derive_tags.argtypes = [vp, u64, ctypes.POINTER(u32), ctypes.POINTER(u32),
                                      ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.cfo_move.restype = u64
        L.cfo_move.argtypes = [vp, u64, u32, ctypes.POINTER(u32)]
        L.cfo_key_groups.restype = u64
        L.cfo_key_groups.argtypes = [vp, vp, u64, vp, vp, vp]
        L.cfo_pair_groups.restype = u64
        L.cfo_pair_groups.argtypes = [vp, vp, vp, u64, vp, vp, vp]
        L.cfo_io_counts.restype = None
        L.cfo_io_counts.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.cfo_io_reset.restype = None
        L.cfo_io_reset.argtypes = [vp]
        _lib = L
    return _lib


def fmix64(x: int) -> int:
    return lib().cfo_fmix64(x)


def xxh64_u64(x: int) -> int:
    return lib().cfo_xxh64_u64(x)


def hash64(kind: int, x: int) -> int:
    return lib().cfo_hash(kind, x)


def splitmix64_at(state: int, k: int) -> int:
    return lib().cfo_splitmix64_at(state, k)


def _keys(keys) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))


class OracleFilter:
    """Sequential cuckoo filter: m buckets x b slots x f-bit fingerprints."""

    def __init__(self, m: int, b: int, f: int, hash_kind: int = HASH_FMIX64,
                 evict: int = EVICT_BFS, max_evict: int = 16, seed: int = 0,
                 placement: int = 0):
        self.m, self.b, self.f = int(m), int(b), int(f)
        self.hash_kind, self.evict, self.max_evict, self.seed = hash_kind, evict, max_evict, seed
        self.placement = placement
        self._h = lib().cfo_create_placed(self.m, self.b, self.f, hash_kind, evict, max_evict,
                                          seed & 0xFFFFFFFFFFFFFFFF, placement)
        if not self._h:
            raise ValueError(f"invalid oracle filter parameters m={m} b={b} f={f}")

    def close(self):
        if self._h:
            lib().cfo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # derived values -------------------------------------------------
    def derive(self, key: int):
        fp, i1, i2 = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
        lib().cfo_derive(self._h, key, ctypes.byref(fp), ctypes.byref(i1), ctypes.byref(i2))
        return fp.value, i1.value, i2.value

    def derive_batch(self, keys):
        k = _keys(keys)
        fp = np.zeros(k.size, dtype=np.uint32)
        i1 = np.zeros(k.size, dtype=np.uint64)
        i2 = np.zeros(k.size, dtype=np.uint64)
        lib().cfo_derive_batch(self._h, k.ctypes.data, k.size, fp.ctypes.data,
                               i1.ctypes.data, i2.ctypes.data)
        return fp, i1, i2

    def derive_tags(self, key: int):
        """(t1, t2, i1, i2): the tag as written in i1 and in i2."""
        t1, t2 = ctypes.c_uint32(), ctypes.c_uint32()
        i1, i2 = ctypes.c_uint64(), ctypes.c_uint64()
        lib().cfo_derive_tags(self._h, key, ctypes.byref(t1), ctypes.byref(t2),
                              ctypes.byref(i1), ctypes.byref(i2))
        return t1.value, t2.value, i1.value, i2.value

    def move(self, bucket: int, tag: int):
        """(other bucket, tag as written there) for a tag stored in bucket."""
        t = ctypes.c_uint32()
        a = lib().cfo_move(self._h, bucket, tag, ctypes.byref(t))
        return a, t.value

    def key_groups(self, keys):
        """The group each key's tag joins, as three arrays: (low bucket, high
        bucket, fp) of its pair under XOR; (primary, alternate, fingerprint)
        under the offset policy."""
        k = _keys(keys)
        lo = np.zeros(max(k.size, 1), dtype=np.uint64)
        hi = np.zeros(max(k.size, 1), dtype=np.uint64)
        tg = np.zeros(max(k.size, 1), dtype=np.uint32)
        lib().cfo_key_groups(self._h, k.ctypes.data, k.size, lo.ctypes.data, hi.ctypes.data,
                             tg.ctypes.data)
        return lo[:k.size], hi[:k.size], tg[:k.size]

    def pair_groups(self, buckets, tags):
        """The group of each (bucket, tag) pair, as key_groups gives them."""
        bk = np.ascontiguousarray(np.asarray(buckets, dtype=np.uint64))
        tt = np.ascontiguousarray(np.asarray(tags, dtype=np.uint32))
        n = bk.size
        lo = np.zeros(max(n, 1), dtype=np.uint64)
        hi = np.zeros(max(n, 1), dtype=np.uint64)
        tg = np.zeros(max(n, 1), dtype=np.uint32)
        lib().cfo_pair_groups(self._h, bk.ctypes.data, tt.ctypes.data, n, lo.ctypes.data,
                              hi.ctypes.data, tg.ctypes.data)
        return lo[:n], hi[:n], tg[:n]

    def stored_groups(self):
        """(low bucket, high bucket, tag) of every non-empty slot."""
        n = self.count
        lo = np.zeros(max(n, 1), dtype=np.uint64)
        hi = np.zeros(max(n, 1), dtype=np.uint64)
        tg = np.zeros(max(n, 1), dtype=np.uint32)
        got = lib().cfo_stored_groups(self._h, lo.ctypes.data, hi.ctypes.data, tg.ctypes.data, n)
        return lo[:got], hi[:got], tg[:got]

    def digest_keys(self, keys) -> int:
        """Multiset digest of the keys' (bucket pair, fingerprint) groups."""
        k = _keys(keys)
        return lib().cfo_group_digest_keys(self._h, k.ctypes.data, k.size)

    def digest_table(self, j0: int = 0, j1: int = None) -> int:
        """Multiset digest of the stored groups of buckets [j0, j1)."""
        return lib().cfo_group_digest_table(self._h, j0, self.m if j1 is None else j1)

    def digest_pairs(self, buckets, tags) -> int:
        b = np.ascontiguousarray(np.asarray(buckets, dtype=np.uint64))
        t = np.ascontiguousarray(np.asarray(tags, dtype=np.uint32))
        return lib().cfo_group_digest_pairs(self._h, b.ctypes.data, t.ctypes.data, b.size)

    def load_words_nocount(self, words) -> None:
        w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
        lib().cfo_load_words_nocount(self._h, w.ctypes.data, w.size)

    def alt(self, bucket: int, tag: int) -> int:
        return lib().cfo_alt(self._h, bucket, tag)

    # single-key ops -------------------------------------------------
    def insert(self, key: int):
        k = ctypes.c_uint32()
        ok = lib().cfo_insert(self._h, key, ctypes.byref(k))
        return bool(ok), k.value

    def query(self, key: int) -> bool:
        return bool(lib().cfo_query(self._h, key))

    def delete(self, key: int) -> bool:
        return bool(lib().cfo_delete(self._h, key))

    # batch ops ------------------------------------------------------
    def insert_batch(self, keys, with_kicks: bool = False):
        k = _keys(keys)
        ok = np.zeros(k.size, dtype=np.uint8)
        kicks = np.zeros(k.size, dtype=np.uint32) if with_kicks else None
        lib().cfo_insert_batch(self._h, k.ctypes.data, k.size, ok.ctypes.data,
                               kicks.ctypes.data if kicks is not None else None)
        return (ok, kicks) if with_kicks else ok

    def query_batch(self, keys) -> np.ndarray:
        k = _keys(keys)
        out = np.zeros(k.size, dtype=np.uint8)
        lib().cfo_query_batch(self._h, k.ctypes.data, k.size, out.ctypes.data)
        return out

    def delete_batch(self, keys) -> np.ndarray:
        k = _keys(keys)
        ok = np.zeros(k.size, dtype=np.uint8)
        lib().cfo_delete_batch(self._h, k.ctypes.data, k.size, ok.ctypes.data)
        return ok

    # state ----------------------------------------------------------
    def slot(self, bucket: int, s: int) -> int:
        return lib().cfo_get_slot(self._h, bucket, s)

    def words(self, copy: bool = True) -> np.ndarray:
        """The table's words; copy=False gives a read-only view that is valid
        only while this filter lives and is not modified."""
        n = lib().cfo_num_words(self._h)
        ptr = lib().cfo_words(self._h)
        buf = (ctypes.c_uint64 * n).from_address(ptr)
        view = np.frombuffer(buf, dtype=np.uint64)
        if copy:
            return view.copy()
        view.flags.writeable = False
        return view

    def load_words(self, words) -> None:
        w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
        lib().cfo_load_words(self._h, w.ctypes.data, w.size)

    @property
    def count(self) -> int:
        return lib().cfo_count(self._h)

    @property
    def failures(self) -> int:
        return lib().cfo_failures(self._h)

    def lost(self):
        n = lib().cfo_lost_count(self._h)
        b = np.zeros(max(n, 1), dtype=np.uint64)
        t = np.zeros(max(n, 1), dtype=np.uint32)
        got = lib().cfo_lost(self._h, b.ctypes.data, t.ctypes.data, n)
        return b[:got], t[:got]

    def io_counts(self):
        """(bucket reads, word writes) of the operations since the last
        io_reset(): the memory traffic the algorithm's steps define."""
        r, w = ctypes.c_uint64(), ctypes.c_uint64()
        lib().cfo_io_counts(self._h, ctypes.byref(r), ctypes.byref(w))
        return r.value, w.value

    def io_reset(self) -> None:
        lib().cfo_io_reset(self._h)

    def table_fpr(self) -> float:
        return lib().cfo_table_fpr(self._h)

    @property
    def load_factor(self) -> float:
        return self.count / float(self.m * self.b)
