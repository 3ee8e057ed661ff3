"""Host-side checks of bench.py's command line and of the stability-map table (no GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workloads_are_listed():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for w in ("step", "step3d", "hybrid", "ensemble", "surrogate"):
        assert w in r.stdout


def test_stability_table_layout():
    from paper_2501_03759_amd import stability
    res = [{"model": m, "mobility": M, "eps_reg": e, "s_j": stability.flux_rate(M), "stable": (e < 1.0) or m == "trt",
            "max_abs_phi": 1.0} for m in ("mrt", "srt", "trt") for M in (0.1, 1.0) for e in (0.03, 1.0)]
    t = stability.table(res)
    assert t.count("| 0.1 (1.250) |") == 3 and t.count("| 1 (0.286) |") == 3
    assert "MRT:" in t and "SRT:" in t and "TRT:" in t
    assert t.splitlines()[2] == "| M (s_j) | eps 0.03 | eps 1 |"
    assert "| 0.1 (1.250) | o | x |" in t and "| 0.1 (1.250) | o | o |" in t
    assert abs(stability.flux_rate(0.1) - 1.25) < 1e-15
