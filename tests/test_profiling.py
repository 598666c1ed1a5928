"""CPU check of the serving-overlap summary over a small hand-made kernel
trace: which streams count as serving streams, busy time, and the time with
two or more streams running."""
import csv

from paper_1610_05994_amd import profiling


def _trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Stream_Id", "Queue_Id"])
        w.writeheader()
        for name, s, e, stream, queue in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": s, "End_Timestamp": e, "Stream_Id": stream,
                        "Queue_Id": queue})


def test_serving_overlap_counts_single_builds_on_serving_streams(tmp_path):
    p = tmp_path / "run_kernel_trace.csv"
    _trace(p, [
        ("void wt::k_batch_level<2, 32, true>(wt::BatchClass)", 0, 100, 1, 1),
        ("void wt::k_level<4, 128, false>(wt::LevelArgs)", 100, 300, 1, 1),   # a long request, built alone
        ("void wt::k_small_batch<1, 1u>(wt::SmallJob const*)", 200, 400, 2, 2),
        ("void wt::k_query_multi(wt::QueryArgs)", 400, 450, 2, 2),
        ("__amd_rocclr_copyBuffer", 450, 460, 2, 2),                          # not a library kernel
        ("void wt::k_level<1, 32, false>(wt::LevelArgs)", 1000, 2000, 3, 3),  # not a serving stream
    ])
    res = profiling.overlap(profiling.serving_dispatches(str(p)))
    assert res["dispatches"] == 4 and res["streams"] == [1, 2]
    assert res["window_ms"] == 450 / 1e6
    assert res["busy_ms"] == 450 / 1e6
    assert res["two_or_more_streams_ms"] == 100 / 1e6   # [200, 300): both streams
    assert abs(res["overlap_frac_of_busy"] - 100 / 450) < 1e-12
    # explicit patterns keep their old meaning (name filter only)
    res = profiling.overlap(profiling.read_dispatches(str(p), ("k_level",)))
    assert res["dispatches"] == 2 and res["streams"] == [1, 3] and res["two_or_more_streams_ms"] == 0.0
