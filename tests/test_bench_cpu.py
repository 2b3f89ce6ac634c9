"""bench.py's contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_dsb_stream_bytes_formula():
    sys.path.insert(0, ROOT)
    import bench
    n, nnz, M = 100, 300, 130
    # x, y in place (16 B per spin-update), 3 sign words per spin read and
    # written, column and coupling per stored coupling, 12 B per row
    assert bench.stream_bytes_dsb(n, nnz, M) == 16 * n * M + 16 * n * 3 + 8 * nnz + 12 * n
    assert bench.stream_bytes(n, nnz, M, 1) == 16 * n * M + 5 * nnz + 12 * n
