"""CPU checks of bench.py's bookkeeping: per-column launches per reduction and
the per-evaluation averages read back from a (synthetic) rocprofv3 kernel
trace."""
import csv
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_column_launches():
    # the LDS tail takes the last <= 256 columns from a 32-column panel
    # boundary; panels whose trailing order is at most 4000 are fused (kind 8)
    assert bench.column_launches(6000) == {0: 2016, 8: 3744}
    assert sum(bench.column_launches(6000).values()) == 5760
    assert bench.column_launches(256) == {0: 0, 8: 0}
    assert bench.column_launches(257) == {0: 0, 8: 32}
    assert bench.column_launches(289) == {0: 0, 8: 64}
    assert bench.column_launches(2) == {0: 0, 8: 0}
    assert bench.column_launches(6000, fused_max=0) == {0: 5760, 8: 0}
    # the panel starting at k0 = 2016 has trailing order 3983 <= 4000
    assert bench.column_launches(6000, fused_max=3983)[0] == 2016
    assert bench.column_launches(6000, fused_max=3982)[0] == 2048


def test_trace_summary_averages(tmp_path, capsys):
    per = bench.column_launches(6000)
    steps, warmup = 2, 1
    rows = []
    t = 0
    # autotuner candidates (10 us), warm-up (4 us), timed (2 us), profiled (6 us);
    # each column takes a SYMV launch + finish, or one fused launch (half the
    # time); every reduction ends with one tail launch
    for dur, reps in ((10000, 3), (4000, 1), (2000, steps), (6000, 1)):
        for _ in range(reps):
            for _ in range(per[0]):
                rows.append({"Kernel_Name": "void sytrd_symv_kernel<float, 32>(SytrdWs<float>, int, int, int)",
                             "Start_Timestamp": t, "End_Timestamp": t + dur})
                rows.append({"Kernel_Name": "void sytrd_finish_kernel<float, 32>(SytrdWs<float>, int, int)",
                             "Start_Timestamp": t + dur + 10, "End_Timestamp": t + dur + 20})
                t += dur + 100
            for _ in range(per[8]):
                rows.append({"Kernel_Name": "void sytrd_col_kernel<float, 32>(SytrdWs<float>, int, int, int)",
                             "Start_Timestamp": t, "End_Timestamp": t + dur // 2})
                t += dur + 100
            rows.append({"Kernel_Name": "void sytrd_tail_kernel<float>(SytrdWs<float>)",
                         "Start_Timestamp": t, "End_Timestamp": t + 50})
            t += 100
    path = tmp_path / "x_kernel_trace.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerows(rows)
    bench.trace_summary(str(tmp_path), steps, warmup)
    out = capsys.readouterr().out.splitlines()
    assert out[0] == "sytrd_symv_kernel<float>: %d launches per reduction" % per[0]
    assert out[1].endswith("%.2f us" % ((4 + 2 * 2 + 6) / 4.0))
    assert out[2].endswith("2.00 us")
    assert out[3].endswith("6.00 us")
    assert out[4] == "sytrd_col_kernel<float>: %d launches per reduction" % per[8]
    assert out[5].endswith("%.2f us" % ((4 + 2 * 2 + 6) / 8.0))
    assert out[6].endswith("1.00 us")
    assert out[7].endswith("3.00 us")
