"""The exact per-lane zero test used by the device code to find empty slots
and matching fingerprints (reading R7): with H the top bit of every f-bit
lane and L the other bits, lane k of w is zero iff bit (k*f + f-1) of
~(((w & L) + L) | w) & H is set.  Checked here against a plain per-lane
scan: exhaustively for every value of one 8-bit lane (the other lanes
random), and on random words for 16- and 32-bit lanes, with zero lanes
planted.  Also shows why the classic borrow test (w - 0x01..01) & ~w & H is
not used: it flags a 0x01 lane sitting above a zero lane."""
import numpy as np

M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _masks(f):
    lanes = 64 // f
    hi = np.uint64(0)
    for k in range(lanes):
        hi |= np.uint64(1) << np.uint64(k * f + f - 1)
    return hi, hi ^ M64


def _exact(w, f):
    hi, lo = _masks(f)
    with np.errstate(over="ignore"):
        return ~(((w & lo) + lo) | w) & hi


def _scan(w, f):
    out = np.zeros_like(w)
    mask = np.uint64((1 << f) - 1)
    for k in range(64 // f):
        lane = (w >> np.uint64(k * f)) & mask
        out |= np.where(lane == 0, np.uint64(1) << np.uint64(k * f + f - 1), np.uint64(0))
    return out


def test_every_8bit_lane_value_in_every_position():
    rng = np.random.default_rng(1)
    for pos in range(8):
        base = rng.integers(0, 2**63, 256, dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, 256, dtype=np.uint64)
        vals = np.arange(256, dtype=np.uint64)
        sh = np.uint64(8 * pos)
        w = (base & ~(np.uint64(0xFF) << sh)) | (vals << sh)
        # neighbours take every value too, zero included
        w2 = w.copy()
        for nb in (pos - 1, pos + 1):
            if 0 <= nb < 8:
                w2 &= ~(np.uint64(0xFF) << np.uint64(8 * nb))
        for ww in (w, w2):
            assert np.array_equal(_exact(ww, 8), _scan(ww, 8))


def test_random_words_16_and_32_bit_lanes():
    rng = np.random.default_rng(2)
    for f in (16, 32):
        w = rng.integers(0, 2**63, 1_000_000, dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, 1_000_000, dtype=np.uint64)
        mask = np.uint64((1 << f) - 1)
        for k in range(64 // f):  # plant zero lanes and lanes equal to 1
            sel = rng.random(w.size) < 0.3
            w[sel] &= ~(mask << np.uint64(k * f))
            one = rng.random(w.size) < 0.1
            w[one] = (w[one] & ~(mask << np.uint64(k * f))) | (np.uint64(1) << np.uint64(k * f))
        assert np.array_equal(_exact(w, f), _scan(w, f))


def test_borrow_test_is_not_exact():
    f = 8
    hi, _ = _masks(f)
    ones = np.uint64(0x0101010101010101)
    w = np.array([0x0100], dtype=np.uint64)  # lane 0 zero, lane 1 holds 0x01
    with np.errstate(over="ignore"):
        borrow = (w - ones) & ~w & hi
    assert int(borrow[0]) & 0x8000  # lane 1 wrongly flagged
    assert not int(_exact(w, f)[0]) & 0x8000
    assert int(_exact(w, f)[0]) & 0x80
