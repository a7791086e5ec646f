"""CPU checks of bench.py's bookkeeping: SYMV launches per reduction and the
per-evaluation average read back from a (synthetic) rocprofv3 kernel trace."""
import csv
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_symv_launches():
    # the LDS tail takes the last <= 256 columns from a 32-column panel boundary
    assert bench.symv_launches(6000) == 5760
    assert bench.symv_launches(256) == 0
    assert bench.symv_launches(257) == 32
    assert bench.symv_launches(289) == 64
    assert bench.symv_launches(2) == 0


def test_trace_summary_averages(tmp_path, capsys):
    per = bench.symv_launches(6000)
    steps, warmup = 2, 1
    rows = []
    t = 0
    # autotuner candidates (10 us), warm-up (4 us), timed (2 us), profiled (6 us)
    for dur, count in ((10000, 3 * per), (4000, per), (2000, steps * per), (6000, per)):
        for _ in range(count):
            rows.append({"Kernel_Name": "void sytrd_symv_kernel<float, 32>(SytrdWs<float>, int, int, int)",
                         "Start_Timestamp": t, "End_Timestamp": t + dur})
            rows.append({"Kernel_Name": "void sytrd_finish_kernel<float, 32>(SytrdWs<float>, int, int)",
                         "Start_Timestamp": t + dur + 10, "End_Timestamp": t + dur + 20})
            t += dur + 100
    path = tmp_path / "x_kernel_trace.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerows(rows)
    bench.trace_summary(str(tmp_path), steps, warmup)
    out = capsys.readouterr().out.splitlines()
    assert out[1].endswith("%.2f us" % ((4 + 2 * 2 + 6) / 4.0))
    assert out[2].endswith("2.00 us")
    assert out[3].endswith("6.00 us")
