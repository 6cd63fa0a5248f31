"""A CPU model of the concurrent insert algorithm of the GPU kernels, run
under random interleavings.

The device code's steps are restated over a word-granular table: the direct
attempts of Alg. 1 (first empty slot in scan order, CAS retried with the
returned word), then the eviction search -- the breadth-first relocation of
Sec. 4.6.1 in the kernels' displacement-first order (replace the candidate
while the slot still holds it, insert it into its other bucket, else carry
it) or the random walk.  Every shared-memory step is a yield point, so a
random scheduler interleaves many inserting threads; every plain load may
return any value the word held earlier (a stale cached copy).  After each
schedule the table must hold exactly one fingerprint per successful insert,
in its key's bucket pair, minus the dropped fingerprints the failures log.

This checks the algorithm, not the compiled kernels: it is the evidence that
a fingerprint lost on the GPU comes from how the code was built, not from
the interleavings the algorithm allows.  Not a copy of any device source.
"""
import collections
import random

import pytest

M64 = (1 << 64) - 1


def _mix(z):
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 & M64
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB & M64
    return z ^ (z >> 31)


class Table:
    """m buckets x b slots of f bits, packed into words of tpw lanes."""

    def __init__(self, m, b, f, tpw):
        self.m, self.b, self.f, self.tpw = m, b, f, tpw
        self.wpb = b // tpw
        self.words = [0] * (m * self.wpb)
        self.history = [[0] for _ in self.words]  # every value each word held

    def cas(self, w, expected, desired):
        old = self.words[w]
        if old == expected:
            self.words[w] = desired
            self.history[w].append(desired)
        return old

    def lane(self, word, k):
        return (word >> (k * self.f)) & ((1 << self.f) - 1)

    def set_lane(self, word, k, v):
        mask = ((1 << self.f) - 1) << (k * self.f)
        return (word & ~mask) | (v << (k * self.f))


class Model:
    def __init__(self, m, b, f, tpw, evict_bfs, max_evict, rng):
        self.t = Table(m, b, f, tpw)
        self.bfs = evict_bfs
        self.D = max_evict
        self.rng = rng
        self.lost = []

    # derived values (XOR placement over a power-of-two m)
    def derive(self, key):
        h = _mix(key)
        fp = (h >> 32) & ((1 << self.t.f) - 1) or 1
        i1 = h & (self.t.m - 1)
        return fp, i1, self.alt(i1, fp)

    def alt(self, j, tag):
        return j ^ (_mix(tag + 0x9E3779B97F4A7C15) & (self.t.m - 1))

    # ---- shared-memory steps (each is a yield point) -------------------
    def load_bucket(self, j):
        """Plain load: every word of the bucket may be any earlier value."""
        out = []
        for k in range(self.t.wpb):
            w = j * self.t.wpb + k
            yield
            out.append(self.rng.choice(self.t.history[w][-3:]))
        return out

    def try_insert(self, j, tag, bk):
        t = self.t
        start = (tag % t.b) // t.tpw
        while True:
            idx = lane = None
            for p in range(t.wpb):
                k = (start + p) % t.wpb
                zs = [q for q in range(t.tpw) if t.lane(bk[k], q) == 0]
                if zs:
                    idx, lane = k, zs[0]
                    break
            if idx is None:
                return -1
            w = bk[idx]
            yield
            old = t.cas(j * t.wpb + idx, w, t.set_lane(w, lane, tag))
            if old == w:
                bk[idx] = t.set_lane(w, lane, tag)
                return idx * t.tpw + lane
            bk[idx] = old

    def replace_if(self, j, s, expect, tag, bk):
        t = self.t
        idx, q = divmod(s, t.tpw)
        w = bk[idx]
        while t.lane(w, q) == expect:
            yield
            old = t.cas(j * t.wpb + idx, w, t.set_lane(w, q, tag))
            if old == w:
                bk[idx] = t.set_lane(w, q, tag)
                return True
            w = old
        bk[idx] = w
        return False

    def swap(self, j, s, tag, bk):
        t = self.t
        idx, q = divmod(s, t.tpw)
        w = bk[idx]
        while True:
            yield
            old = t.cas(j * t.wpb + idx, w, t.set_lane(w, q, tag))
            if old == w:
                bk[idx] = t.set_lane(w, q, tag)
                return t.lane(w, q)
            w = old

    # ---- one insert ----------------------------------------------------
    def insert(self, key, out):
        fp, i1, i2 = self.derive(key)
        bk = yield from self.load_bucket(i1)
        if (yield from self.try_insert(i1, fp, bk)) >= 0:
            out.append(True)
            return
        bk = yield from self.load_bucket(i2)
        if (yield from self.try_insert(i2, fp, bk)) >= 0:
            out.append(True)
            return
        rs = _mix(key ^ 0x5EED)
        cur, tag = (i2 if rs & 1 else i1), fp
        b, half = self.t.b, self.t.b // 2
        for n in range(1, self.D + 1):
            r = _mix(rs + n)
            cb = yield from self.load_bucket(cur)
            if (yield from self.try_insert(cur, tag, cb)) >= 0:
                out.append(True)
                return
            if self.bfs:
                r0 = r % b
                carried = False
                for jj in range(half):
                    s = (r0 + jj) % b
                    c = self.t.lane(cb[s // self.t.tpw], s % self.t.tpw)
                    if c == 0:
                        continue
                    a = self.alt(cur, c)
                    if a == cur:
                        continue
                    ab = yield from self.load_bucket(a)
                    if all(self.t.lane(w, q) != 0 for w in ab for q in range(self.t.tpw)):
                        continue
                    if not (yield from self.replace_if(cur, s, c, tag, cb)):
                        continue
                    if (yield from self.try_insert(a, c, ab)) >= 0:
                        out.append(True)
                        return
                    tag, cur, carried = c, a, True  # `a` filled meanwhile: carry c
                    break
                if carried:
                    continue
                s = (r0 + half - 1) % b
            else:
                s = r % b
            ev = yield from self.swap(cur, s, tag, cb)
            if ev == 0:
                out.append(True)
                return
            tag, cur = ev, self.alt(cur, ev)
            nb = yield from self.load_bucket(cur)
            if (yield from self.try_insert(cur, tag, nb)) >= 0:
                out.append(True)
                return
        self.lost.append((cur, tag))
        out.append(False)

    def groups_stored(self):
        t = self.t
        g = collections.Counter()
        for j in range(t.m):
            for k in range(t.wpb):
                for q in range(t.tpw):
                    v = t.lane(t.words[j * t.wpb + k], q)
                    if v:
                        a = self.alt(j, v)
                        g[(min(j, a), max(j, a), v)] += 1
        return g


def _run(seed, m, b, f, tpw, nkeys, bfs, D):
    rng = random.Random(seed)
    md = Model(m, b, f, tpw, bfs, D, rng)
    keys = [rng.getrandbits(64) for _ in range(nkeys)]
    keys += keys[: nkeys // 8]  # duplicates too
    outs = [[] for _ in keys]
    threads = [md.insert(k, o) for k, o in zip(keys, outs)]
    live = list(range(len(threads)))
    while live:  # random interleaving, one step at a time
        i = rng.randrange(len(live))
        try:
            next(threads[live[i]])
        except StopIteration:
            live.pop(i)
    ok = [o[0] for o in outs]
    want = collections.Counter()
    for k, _ in zip(keys, ok):
        fp, i1, i2 = md.derive(k)
        want[(min(i1, i2), max(i1, i2), fp)] += 1
    for j, v in md.lost:
        a = md.alt(j, v)
        want[(min(j, a), max(j, a), v)] -= 1
    stored = md.groups_stored()
    assert sum(stored.values()) == sum(ok), (seed, "slots != successes")
    assert stored == +want, (seed, "stored multiset != keys' groups - dropped")
    assert len(md.lost) == ok.count(False)
    return sum(ok), len(md.lost)


@pytest.mark.parametrize("bfs", [True, False])
@pytest.mark.parametrize("m,b,f,tpw", [(4, 4, 8, 4), (8, 8, 16, 4), (4, 16, 16, 4), (16, 4, 8, 2)])
def test_random_interleavings_keep_every_fingerprint(bfs, m, b, f, tpw):
    D = 4 if bfs else 12
    total_lost = 0
    for seed in range(150):
        _, lost = _run(seed * 7919 + m * 31 + b, m, b, f, tpw, int(1.05 * m * b), bfs, D)
        total_lost += lost
    # over-full tables: failures happen, and each one was accounted for above
    assert total_lost > 0
