"""The benchmark's host-side measurement helpers (no device needed), on
synthetic files shaped like rocprofv3's csv output: how dispatches map to
counters, how the timed steps' launches are found in a counter run, how
filter-set batches are grouped in a kernel trace, and the percentile rule."""
import csv
import os

import pytest

import bench


def _write(dirpath, name, rows):
    sub = os.path.join(dirpath, "vm")
    os.makedirs(sub, exist_ok=True)
    path = os.path.join(sub, name)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)
    return path


def _counter_rows(kernels, counter="FETCH_SIZE"):
    """One row per (dispatch, counter) the way a --pmc run writes them, with
    two rows for one dispatch (a counter summed over instances)."""
    rows = []
    for d, k in enumerate(kernels, start=1):
        rows.append({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": counter,
                     "Counter_Value": 10.0 * d})
        rows.append({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": counter,
                     "Counter_Value": 1.0})
    return rows


INS = "void cfk::insert_kernel<cfk::Geom<16, 16>, 0, 0, 0, 1>(unsigned long*, ...)"
QRY = "void cfk::query_kernel<cfk::Geom<16, 16>, 0, 0>(unsigned long const*, ...)"
DEL = "void cfk::delete_kernel<cfk::Geom<16, 16>, 0, 0>(unsigned long*, ...)"
KEY = "keygen_kernel(unsigned long*, unsigned long, unsigned long, unsigned long)"


def test_counter_by_dispatch_sums_instances_and_filters_kernels(tmp_path):
    _write(tmp_path, "1_counter_collection.csv", _counter_rows([INS, KEY, QRY]))
    got = bench._counter_by_dispatch(str(tmp_path), r"query_kernel|insert_")
    assert sorted(got) == [1, 3]
    assert got[1]["FETCH_SIZE"] == 11.0 and got[3]["FETCH_SIZE"] == 31.0


def test_timed_step_launches_skip_the_prefill_and_warmup(tmp_path):
    """prefill inserts, then W + S steps of (insert, 3 queries, delete), then
    the large delete; key generation in between is ignored."""
    step = [KEY, INS, QRY, QRY, QRY, DEL]
    kernels = [KEY, INS, INS, INS] + step * 5 + [DEL]
    _write(tmp_path, "1_counter_collection.csv", _counter_rows(kernels))
    groups = bench._timed_step_launches(str(tmp_path), 2, 3)
    assert len(groups) == 3
    ids = {d: k for d, k in enumerate(kernels, start=1)}
    for g in groups:
        assert [ids[d] for d in g] == [INS, QRY, QRY, QRY, DEL]
    # the first timed step is the third step of the run
    first_query = kernels.index(QRY) + 1
    assert groups[0][1] == first_query + 2 * len(step)


def test_timed_step_launches_refuse_a_run_that_is_not_the_step(tmp_path):
    kernels = [INS, INS, QRY, QRY, DEL, DEL]  # a query missing from the step
    _write(tmp_path, "1_counter_collection.csv", _counter_rows(kernels))
    with pytest.raises(AssertionError):
        bench._timed_step_launches(str(tmp_path), 0, 1)


def _trace_row(name, t0, t1, q=1):
    return {"Kernel_Name": name, "Start_Timestamp": t0, "End_Timestamp": t1, "Queue_Id": q}


def test_set_batch_spans_group_batches_by_launch_sequence():
    part = "void cfs::partition_kernel(cfs::Batch, ...)"
    q16 = "void cfs::set_query_kernel<cfk::Geom<16, 16>, 0, 0>(cfs::Batch, ...)"
    q8 = "void cfs::set_query_kernel<cfk::Geom<16, 8>, 0, 0>(cfs::Batch, ...)"
    pq = "void cfs::phase_query_kernel<16, 0, 0, 16>(cfs::Batch, ...)"
    trace, t = [], 0
    for _ in range(3):  # three class-kernel batches on one queue
        trace += [_trace_row(part, t, t + 20_000), _trace_row(q16, t + 21_000, t + 101_000),
                  _trace_row(q8, t + 102_000, t + 142_000)]
        t += 200_000
    for _ in range(3):  # three phase-form batches, the query on a second queue
        trace += [_trace_row(part, t, t + 10_000), _trace_row(pq, t + 11_000, t + 71_000, q=2)]
        t += 100_000
    out = bench._set_batch_spans(trace)
    text = "\n".join(out)
    assert "3 batches, 1 queue(s): span 142.0, gap 58.0" in text
    assert "partition 20.0, query b16 80.0, query b8 40.0" in text
    assert "3 batches, 2 queue(s): span 71.0, gap 29.0" in text
    assert "partition 10.0, query* 60.0" in text


def test_set_batch_spans_empty_without_set_kernels():
    trace = [_trace_row(QRY, 0, 10), _trace_row(INS, 20, 30)]
    assert bench._set_batch_spans(trace) == []


@pytest.mark.parametrize("xs,q,want", [([3, 1, 2], 50, 2), ([1, 2, 3, 4], 50, 2.5),
                                       ([5], 99, 5), ([1, 2], 0, 1), ([1, 2], 100, 2),
                                       ([], 50, None)])
def test_percentile_interpolates_between_order_statistics(xs, q, want):
    assert bench.pct(xs, q) == want
