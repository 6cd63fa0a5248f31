"""Pin of Eq. (3): the alternate bucket is i1 XOR H(fp), with H a uniform hash
applied to the fingerprint (Sec. 2.1).

The involution test in test_oracle.py holds for any XOR offset that depends
on the fingerprint alone, so it cannot tell i2 = i1 ^ H(fp) from i2 = i1 ^ fp.
What Eq. (3) adds is that the offset is the *hash* of the fingerprint, so it
spreads over the whole bucket range however few fingerprint bits there are.
The checks below pin exactly that, without restating the oracle's formula:

* the offset i1 ^ i2 depends on the fingerprint alone (keys sharing a
  fingerprint share it, whatever their bucket);
* with 8-bit fingerprints and 2^20 buckets the 255 offsets reach far beyond
  2^8 and land in both halves of the table;
* with 16-bit fingerprints and 2^20 buckets the offsets' top four bits are
  uniform (chi-square), and over 2^28 buckets nearly all 65535 offsets are
  distinct (a uniform hash gives about 8 collisions).

Planting either of two plausible slips in a copy of the oracle -- dropping H
(offset = fp) or reducing H(fp) to f bits instead of log2(m) -- makes the pin
fail (test_pin_rejects_planted_mistakes).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from workloads import keys as K

SRC = os.path.join(os.path.dirname(oracle.__file__), "cfo.c")
# the line of cfo_move that computes the XOR placement's other bucket
XOR_MOVE = "return bucket ^ (cfo_hash(flt->hash_kind, (uint64_t)tag) & (flt->m - 1));"
MUTANTS = {
    "H dropped": "return bucket ^ ((uint64_t)tag & (flt->m - 1));",
    "H(fp) reduced to f bits": "return bucket ^ (cfo_hash(flt->hash_kind, (uint64_t)tag) & "
                               "((1ULL << flt->f) - 1) & (flt->m - 1));",
}
SHAPES = ((1 << 20, 8), (1 << 20, 16), (1 << 28, 16))  # (m, f), b = 4


class _Lib:
    """alt() and derive() of a filter built by a cfo.c library (the oracle,
    or a planted copy of it).  The 2^28-bucket table is calloc'ed and never
    touched, so it costs no memory."""

    def __init__(self, L, hk):
        self.L, self.hk = L, hk
        L.cfo_create.restype = ctypes.c_void_p
        L.cfo_create.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint64]
        L.cfo_alt.restype = ctypes.c_uint64
        L.cfo_alt.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32]
        L.cfo_derive.restype = None
        L.cfo_derive.argtypes = [ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_uint32),
                                 ctypes.POINTER(ctypes.c_uint64),
                                 ctypes.POINTER(ctypes.c_uint64)]
        L.cfo_destroy.restype = None
        L.cfo_destroy.argtypes = [ctypes.c_void_p]
        self.h = {}
        for m, f in SHAPES:
            h = L.cfo_create(m, 4, f, hk, 0, 16, 0)
            assert h, f"cannot create an oracle filter with m={m} f={f}"
            self.h[(m, f)] = h

    def alt(self, shape):
        L, h = self.L, self.h[shape]
        return lambda j, v: L.cfo_alt(h, j, v)

    def derive(self, shape):
        L, h = self.L, self.h[shape]

        def d(key):
            fp, i1, i2 = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
            L.cfo_derive(h, key, ctypes.byref(fp), ctypes.byref(i1), ctypes.byref(i2))
            return fp.value, i1.value, i2.value
        return d

    def close(self):
        for h in self.h.values():
            self.L.cfo_destroy(h)
        self.h = {}


def _offsets(alt, f):
    """XOR offset alt(0, v) for every non-zero f-bit fingerprint v."""
    return np.array([alt(0, v) for v in range(1, 1 << f)], dtype=np.uint64)


def eq3_violations(lib):
    """The Eq. (3) properties that the library's alt() and derive() violate."""
    bad = []
    a8 = lib.alt((1 << 20, 8))
    # the offset depends on the fingerprint alone
    rng = np.random.default_rng(5)
    for v in (1, 2, 77, 255):
        d = a8(0, v)
        if any(a8(int(j), v) ^ int(j) != d for j in rng.integers(0, 1 << 20, 64)):
            bad.append(f"offset of fp {v} depends on the bucket")
    seen = {}
    derive = lib.derive((1 << 20, 8))
    for key in K.keys(21, 0, 4000):
        fp, i1, i2 = derive(int(key))
        if seen.setdefault(fp, i1 ^ i2) != i1 ^ i2:
            bad.append("two keys with one fingerprint have different offsets")
            break
    # f = 8, m = 2^20: without H the offset would stay below 2^8
    d8 = _offsets(a8, 8)
    far = int((d8 >= 256).sum())
    if far < 250:  # a uniform 20-bit offset is below 2^8 with chance 2^-12
        bad.append(f"only {far} of 255 offsets reach past 2^8")
    top = int((d8 >> np.uint64(19)).sum())
    if not 88 <= top <= 168:  # Binomial(255, 1/2) within 5 sigma
        bad.append(f"{top} of 255 offsets in the upper half of the table")
    # f = 16, m = 2^20: top 4 offset bits uniform over the 65535 fingerprints
    d16 = _offsets(lib.alt((1 << 20, 16)), 16)
    hist = np.bincount((d16 >> np.uint64(16)).astype(np.int64), minlength=16)
    exp = d16.size / 16
    chi2 = float(((hist - exp) ** 2 / exp).sum())
    if chi2 > 60:  # 15 degrees of freedom: P(chi2 > 60) < 1e-6
        bad.append(f"top offset bits not uniform (chi2 {chi2:.1f})")
    # f = 16, m = 2^28: expected collisions C(65535, 2) / 2^28 = 8
    d28 = _offsets(lib.alt((1 << 28, 16)), 16)
    distinct = np.unique(d28).size
    if distinct < 65500:
        bad.append(f"only {distinct} distinct offsets over 2^28 buckets")
    return bad


@pytest.mark.parametrize("hk", [oracle.HASH_FMIX64, oracle.HASH_XXH64])
def test_eq3_offset_is_a_hash_of_the_fingerprint(hk):
    lib = _Lib(oracle.lib(), hk)
    try:
        bad = eq3_violations(lib)
    finally:
        lib.close()
    assert not bad, bad


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_rejects_planted_mistakes(name, tmp_path):
    """A copy of the oracle with the mistake planted in cfo_move fails the
    pin (the real oracle passes it, above)."""
    src = open(SRC).read()
    assert src.count(XOR_MOVE) == 1, "cfo_move's XOR line changed; update the planted copies"
    mutant = tmp_path / "cfo_mut.c"
    mutant.write_text(src.replace(XOR_MOVE, MUTANTS[name]))
    so = tmp_path / "libcfo_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-I", os.path.dirname(SRC), "-o", str(so), str(mutant)])
    lib = _Lib(ctypes.CDLL(str(so)), oracle.HASH_FMIX64)
    try:
        bad = eq3_violations(lib)
    finally:
        lib.close()
    assert bad, f"planted mistake '{name}' passed the Eq. (3) pin"
