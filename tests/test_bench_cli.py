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


def test_code_hash_ignores_comments_and_follows_code(tmp_path, monkeypatch):
    """The stored traffic and instruction counts are keyed by a hash of the
    kernel code without comments: editing a comment keeps the key, editing
    code (or a string literal) changes it."""
    import bench
    src = tmp_path / "paper_1906_06306_amd" / "csrc"
    src.mkdir(parents=True)
    f = src / "k.hpp"
    base = 'int a = 1; // note\n/* block\n comment */ const char *s = "// kept"; char c = \'/\';\n'
    f.write_text(base)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    f.write_text(base.replace("// note", "// another note").replace("block", "other words"))
    assert bench.kernel_source_hash() == h0
    f.write_text(base.replace("  ", " ") + "\n\n")           # whitespace only
    assert bench.kernel_source_hash() == h0
    f.write_text(base.replace("int a = 1", "int a = 2"))
    assert bench.kernel_source_hash() != h0
    f.write_text(base.replace('"// kept"', '"// changed"'))  # inside a string literal: code
    assert bench.kernel_source_hash() != h0
    assert bench.strip_comments('x = 1; // y\n/* z */ w = "/*s*/";') == 'x = 1; w = "/*s*/";'


def test_valu_roofline_of_a_stored_count(monkeypatch):
    import types
    import bench
    key = ("feedfacefeedface", "fp32", 16, 1024, 16)
    monkeypatch.setitem(bench.MEASURED_PUSH_VALU_PER_64, key, 400.0)
    args = types.SimpleNamespace(n=1024, ppc=16)
    # 400 instructions per 64 particles for 2^25 particles in 0.5 ms
    r = bench.valu_roofline("feedfacefeedface", "fp32", 16, args, 1 << 25, 0.5)
    assert abs(r["achieved"] - 400.0 * (1 << 19) / 0.5e-3) < 1.0
    assert abs(r["peak"] - 256 * 4 * 2.4e9 / 4) < 1.0 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    assert bench.valu_roofline("0000000000000000", "fp32", 16, args, 1 << 25, 0.5) is None
