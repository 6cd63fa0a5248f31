"""Host-only checks of the geometry tuner's model (cf_tune_geometry with
measure = 0): every compiled (b, f) is enumerated, m is the smallest power
of two that holds the capacity at the load limit, the false-positive rate is
Eq. (4) of Sec. 2.1 at the load reached, and candidates are ranked by
feasibility, table bytes, then larger buckets.  No device is touched."""
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    import paper_2603_15486_amd._binding as mod
    return mod


def _tune(B, capacity, **kw):
    import paper_2603_15486_amd as cf
    return cf.tune_geometry(capacity, measure=False, **kw)


def _paper_point():
    with open(os.path.join(ROOT, "tests", "golden", "fpr_paper_point.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                b, f, lf, pct = line.split()
                return int(b), int(f), float(lf), float(pct)


def test_large_filter_goal_picks_the_papers_gpu_geometry(B):
    # 0.95 * 2^31 keys at an FPR of at most 0.05%: f = 8 fails the FPR at any
    # b, f = 16 with b = 32 fails it (Eq. 4 gives about 0.093%), f = 32 costs
    # twice the bytes, so b = 16, f = 16 (the paper's GPU configuration) wins.
    cap = int(0.95 * 2**31)
    best, rows = _tune(B, cap, max_fpr=5e-4)
    # 2^31 slots is a power of two, so both placements need the same table
    # and the tie goes to XOR
    assert (best.slots_per_bucket, best.fp_bits, best.placement) == (16, 16, 0)
    assert best.num_buckets * best.slots_per_bucket == 2**31
    assert len(rows) == 24
    for pl in (0, 1):
        feas = {(r["slots_per_bucket"], r["fp_bits"]) for r in rows
                if r["feasible"] and r["placement"] == pl}
        assert feas == {(4, 16), (8, 16), (16, 16), (4, 32), (8, 32), (16, 32), (32, 32)}
    # rows are ranked: feasible first, then bytes, then larger b
    keys = [(not r["feasible"], r["bytes"], -r["slots_per_bucket"]) for r in rows]
    assert keys == sorted(keys)
    # the paper reports about 0.045% at b = 16, f = 16, load 0.95
    b, f, lf, pct = _paper_point()
    r = next(r for r in rows
             if (r["slots_per_bucket"], r["fp_bits"], r["placement"]) == (b, f, 0))
    assert abs(r["load"] - lf) < 1e-6
    assert abs(100 * r["fpr"] - pct) < 0.005


def test_fpr_matches_eq4_and_limits_of_small_fingerprints(B):
    best, rows = _tune(B, 1000)
    need = math.ceil(1000 / 0.95)
    for r in rows:
        b, f = r["slots_per_bucket"], r["fp_bits"]
        slots = r["num_buckets"] * b
        assert r["load"] == pytest.approx(1000 / slots)
        if r["placement"] == 0:
            assert slots == 2048  # smallest power of two >= 1000 / 0.95
            # Eq. (4) as a product of per-slot collision chances
            q = 1.0 - 2.0 ** -f
            assert r["fpr"] == pytest.approx(1.0 - q ** (2 * b * r["load"]), rel=1e-9)
        else:
            assert r["num_buckets"] == math.ceil(need / b)  # any bucket count
            q = 1.0 - 2.0 ** -(f - 1)
            assert r["fpr"] == pytest.approx(1.0 - q ** (b * r["load"]), rel=1e-9)
        # the closed-form bound 2 b alpha / 2^f is never exceeded
        assert r["fpr"] <= 2 * b * r["load"] / 2 ** f * (1 + 1e-12)
    # with no FPR limit the smallest table wins: 8-bit fingerprints, b = 32,
    # offset placement (1056 slots instead of 2048)
    assert (best.slots_per_bucket, best.fp_bits, best.placement) == (32, 8, 1)


def test_memory_limit_and_infeasible_goal(B):
    cap = int(0.95 * 2**31)
    best, rows = _tune(B, cap, max_fpr=5e-4, max_bytes=2**32 - 1, raise_infeasible=False)
    assert best is None and not any(r["feasible"] for r in rows)
    import paper_2603_15486_amd as cf
    with pytest.raises(cf.CfError):
        _tune(B, cap, max_fpr=5e-4, max_bytes=2**32 - 1)
    # the byte limit alone, without an FPR goal: 8-bit fingerprints fit in 2 GiB
    best, _ = _tune(B, cap, max_bytes=2**31)
    assert best.fp_bits == 8


def test_offset_placement_saves_memory_above_a_power_of_two(B):
    # 1.25 * 2^20 slots at load 0.95: XOR rounds up to 2^21 slots
    cap = int(0.95 * 1.25 * 2**20)
    best, rows = _tune(B, cap, max_fpr=5e-4)
    assert (best.slots_per_bucket, best.fp_bits, best.placement) == (16, 16, 1)
    assert best.num_buckets * best.slots_per_bucket < 1.26 * 2**20
    xor = next(r for r in rows if (r["slots_per_bucket"], r["fp_bits"], r["placement"]) ==
               (16, 16, 0))
    assert xor["num_buckets"] * 16 == 2**21
    # asked for XOR only, the tuner keeps to powers of two
    best, rows = _tune(B, cap, max_fpr=5e-4, placements=1)
    assert best.placement == 0 and len(rows) == 12


def test_capacity_beyond_the_largest_table_drops_small_buckets(B):
    # m is at most 2^32, so 2^34 slots need b >= 4; 2^36 slots need b >= 16
    best, rows = _tune(B, int(0.95 * 2**36))
    assert {r["slots_per_bucket"] for r in rows} == {16, 32}


@pytest.mark.parametrize("kw", [dict(max_load=1.5), dict(positive_share=2.0),
                                dict(max_fpr=-1.0), dict(mix=(-1, 1, 1))])
def test_bad_goals_are_rejected(B, kw):
    import paper_2603_15486_amd as cf
    with pytest.raises(cf.CfError):
        _tune(B, 1000, **kw)
    with pytest.raises(cf.CfError):
        _tune(B, 0)


def test_counting_call(B):
    import ctypes
    goal = B.cf_tune_goal(1000, 0.95, 0.0, 0, (ctypes.c_double * 3)(1, 1, 1), 0.5, 0, 0, 0, 0,
                          0, 0)
    n = ctypes.c_uint32()
    assert B.LIB.cf_tune_geometry(ctypes.byref(goal), None, 0, ctypes.byref(n), None,
                                  None) == B.CF_OK
    assert n.value == 24
    assert math.isfinite(goal.max_load)
