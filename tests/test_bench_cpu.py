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


def test_measured_lds_normalises_by_chip_cu_cycles(tmp_path, monkeypatch):
    import json

    sys.path.insert(0, ROOT)
    import bench
    from paper_2402_14718_amd import rocprof_summary as rs

    (tmp_path / "profiles").mkdir()
    # GRBM_GUI_ACTIVE summed over 8 XCDs of 1000 active cycles each: 256 CUs
    # x 1000 = 256000 CU cycles
    rec = {"family": "sb_batch", "sources_sha": rs.sources_hash("sb_batch"),
           "sq": {"GRBM_GUI_ACTIVE": 8000.0, "SQ_LDS_IDX_ACTIVE": 128000.0,
                  "SQ_LDS_BANK_CONFLICT": 25600.0}}

    def write(r):
        (tmp_path / "profiles" / "k.md").write_text(
            "# k\n\n## Record\n\n```json\n" + json.dumps(r) + "\n```\n")

    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    write(rec)
    lds = bench.measured_lds("k.md")
    assert lds["busy_frac"] == 0.5 and lds["bank_conflict_frac"] == 0.1
    # stale counters (sources changed) and records without the LDS pass give None
    write(dict(rec, sources_sha="0" * 16))
    assert bench.measured_lds("k.md") is None
    write(dict(rec, sq={"SQ_WAVES": 1.0}))
    assert bench.measured_lds("k.md") is None
