"""CPU checks of bench.py's contract: one GPU only, per-workload step counts,
and the algorithmic-byte formula the roofline is computed from."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_default_steps_are_the_workloads_run_lengths(monkeypatch):
    import bench
    for wl, steps in (("turbulence", 500), ("ensemble", 100), ("weibel", 200), ("shock", 50)):
        monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", wl])
        assert bench.parse().steps == steps
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "7"])
    assert bench.parse().steps == 7


def test_algorithmic_bytes_of_the_turbulence_step():
    import bench
    # 33.5 M particles (D = 2) and 1.05 M cells in FP32: positions and momenta
    # read and written once (40 B per particle), E and B read and written and
    # J written and read once (72 B per cell)
    n_p, n_c = 33_554_432, 1_048_576
    assert bench.algorithmic_bytes(2, 4, n_p, n_c) == n_p * 40 + n_c * 72
    assert abs(bench.algorithmic_bytes(2, 4, n_p, n_c) / 1e9 - 1.4177) < 1e-3
    # the push alone: particles plus E, B read and J written (9 words per cell)
    assert bench.push_bytes(2, 4, n_p, n_c) == n_p * 40 + n_c * 36
    # FP64 words double every term
    assert bench.push_bytes(2, 8, n_p, n_c) == 2 * bench.push_bytes(2, 4, n_p, n_c)
