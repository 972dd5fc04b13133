"""bench.py's command line on the CPU: more than one GPU is refused with a
message before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_gate_reads_the_counter_summary():
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.main_pass_sources_sha256()
    assert len(sha) == 64
    t = bench.counter_traffic()
    # either the summary matches the current kernel sources, or the figure is withheld
    assert t is None or (t[0] > 0 and t[1] > 0)


def test_roofline_fraction_is_cells_over_the_issue_ceiling():
    sys.path.insert(0, ROOT)
    import bench
    # the ceiling is one packed lane-instruction per cell on every lane of every CU
    assert bench.PEAK_ISSUE_CELLS == 256 * 64 * 2.4e9
    rec = bench.roofline(1.154e13, 0.465, "k", traffic=9.2e10, algorithmic_bytes=1.2e8)
    assert rec["bound"] == "alu"
    assert abs(rec["frac"] - 1.154e13 / 0.465 / bench.PEAK_ISSUE_CELLS) < 1e-4
    assert 0 < rec["frac"] <= 1
    assert abs(rec["achieved"] / rec["peak"] - rec["frac"]) < 1e-3
    assert rec["traffic_over_algorithmic"] == round(9.2e10 / 1.2e8, 2)
