"""The rocprofv3 summary tool on a synthetic kernel trace whose answers are
known by construction: per-kernel totals, the idle gaps between kernels and
the idle time inside a run of factorisation kernels."""
import csv

from paper_1508_02599_amd import prof_summary as ps


def _trace(tmp_path, rows):
    d = tmp_path / "run" / "host"
    d.mkdir(parents=True)
    with open(d / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for name, a, b in rows:
            w.writerow([name, a * 1000, b * 1000])   # microseconds -> ns
    return str(tmp_path / "run")


def _rows():
    # two updates with a 10 us gap, an axpby after a 30 us gap, 25 panel
    # solves 10 us apart (25 x 10 us busy, 24 x 10 us idle inside the run),
    # then a gather after a 1210 us gap
    rows = [("void feti::k_update_db<double, 32, false>(feti::Task const*)", 0, 100),
            ("void feti::k_update_db<double, 32, false>(feti::Task const*)", 110, 200),
            ("feti::k_axpby(long, double)", 230, 240)]
    rows += [("void feti::k_trsm<double>(feti::Task const*)", 300 + 20 * i, 310 + 20 * i) for i in range(25)]
    rows += [("feti::k_gather(long)", 2000, 2010)]
    return rows


def test_trace_table_totals(tmp_path):
    d = _trace(tmp_path, _rows())
    out = ps.trace_table(d, top=10, min_us=10)
    assert "| `k_update_db<double, 32, false>` | 2 | 0.190 |" in out
    assert "| `k_trsm<double>` | 25 | 0.250 |" in out
    assert "over 29 launches" in out


def test_gaps_table(tmp_path):
    d = _trace(tmp_path, _rows())
    out = ps.gaps_table(d)
    # idle: 10 + 30 + 60 + 24 x 10 + 1210 = 1550 us of a 2010 us span
    assert out.startswith("span 2.0 ms, idle 1.5 ms (77.1%), kernels 29")
    assert "before k_gather: 1.2 ms over 1 gaps (1210.0 us mean)" in out
    assert "before k_trsm<double>: 0.3 ms over 25 gaps (12.0 us mean)" in out


def test_factor_gaps_table(tmp_path):
    d = _trace(tmp_path, _rows())
    out = ps.factor_gaps_table(d)
    # the two updates form a run too short to count; the 25 panel solves span
    # 490 us with 240 us idle between them
    assert out == "factor phase: 25 launches, span 0.49 ms, idle gaps 0.24 ms (49.0%)"
