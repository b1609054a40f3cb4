"""Host-side parts of bench.py: the one-GPU contract, the source digest that
ties recorded HBM traffic to the kernel code, and the CPU-baseline helpers."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_source_digest_ignores_comments_only(tmp_path):
    a = tmp_path / "a.h"
    b = tmp_path / "b.h"
    c = tmp_path / "c.h"
    a.write_text("// header\nint f(int x) {  // add one\n  return x + 1;\n}\n")
    b.write_text("// another header\n\nint f(int x) {\n  return x + 1;  // same code\n}\n\n")
    c.write_text("// header\nint f(int x) {  // add one\n  return x + 2;\n}\n")
    assert bench.source_digest(str(a)) == bench.source_digest(str(b))
    assert bench.source_digest(str(a)) != bench.source_digest(str(c))


def test_source_digest_stops_at_the_triangular_solves(tmp_path):
    a = tmp_path / "a.h"
    b = tmp_path / "b.h"
    a.write_text("int strip(int x) { return x; }\n" + bench.SOLVE_MARK + "\nint solve() { return 1; }\n")
    b.write_text("int strip(int x) { return x; }\n" + bench.SOLVE_MARK + "\nint solve() { return 2; }\n")
    assert bench.source_digest(str(a)) == bench.source_digest(str(b))


def test_recorded_traffic_matches_the_current_kernel_or_is_absent():
    v = bench.recorded_traffic("lu_strip_kernel<float>")
    assert v is None or v > 1e8
    assert bench.recorded_traffic("some_other_kernel") is None


def test_cpu_model_is_text_or_none():
    m = bench.cpu_model()
    assert m is None or (isinstance(m, str) and m)
