"""The batch tuning interface without a GPU: the cache key, the cache
lookup (exact key, nearest histogram, defaults), the validation of a
tuning, and the committed cache file's format."""
import json
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

sbt = pytest.importorskip("paper_2402_14718_amd")
from paper_2402_14718_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_key_is_mode_precision_agents_and_size_histogram():
    # buckets: n <= 64, <= 128, ..., <= 16384
    n = [10, 64, 65, 128, 129, 4096, 4097, 9216]
    assert sbt.batch_tuning_key(n, "dsb", "bf16", 128) == "dsb bf16 M128 h=2,2,1,0,0,0,1,1,1"
    assert sbt.batch_tuning_key([1], "bsb", "fp16", 7) == "bsb fp16 M7 h=1,0,0,0,0,0,0,0,0"
    with pytest.raises(sbt.SbtError):
        sbt.batch_tuning_key([1], "dsb", "fp32", 7)


def test_defaults_and_validation():
    t = sbt.batch_tuning()
    assert sbt.tuning_dict(t) == {"split_n": 0, "tail_words": 8192, "fill": 1.0,
                                  "band_rows": 0, "from_cache": False}
    n = np.array([300, 5000, 60], np.int32)
    nnz = np.array([900, 15000, 100], np.int64)
    p = sbt.solve_params(agents=128, steps=100)
    lib = sbt.load()
    P = lambda a, t: a.ctypes.data_as(t)
    import ctypes as C
    w = lambda t: lib.sbt_batch_workspace_bytes_tuned(P(n, C.POINTER(C.c_int32)),
                                                      P(nnz, C.POINTER(C.c_int64)), 3,
                                                      C.byref(p), C.byref(t))
    base = w(sbt.batch_tuning())
    assert base == lib.sbt_batch_workspace_bytes(P(n, C.POINTER(C.c_int32)),
                                                 P(nnz, C.POINTER(C.c_int64)), 3, C.byref(p))
    # half-full items: more work items, so at least as much workspace
    assert w(sbt.batch_tuning(fill=0.5)) >= base
    assert w(sbt.batch_tuning(split_n=4608)) >= base
    for bad in (dict(fill=0.0), dict(fill=1.5), dict(tail_words=9000), dict(tail_words=-1),
                dict(split_n=-3), dict(band_rows=-1), dict(band_rows=9217)):
        assert w(sbt.batch_tuning(**bad)) == 0
        assert "tuning" in lib.sbt_last_error().decode()
    t = sbt.batch_tuning()
    t.reserved = 1
    assert w(t) == 0


LOOKUP_SCRIPT = textwrap.dedent("""
    import json, sys
    sys.path.insert(0, {root!r})
    import paper_2402_14718_amd as sbt
    out = {{}}
    for name, sizes, mode, prec, m in {cases!r}:
        out[name] = sbt.tuning_dict(sbt.batch_tuning_lookup(sizes, mode, prec, m))
    print(json.dumps(out))
""")


def test_lookup_exact_nearest_and_default(tmp_path):
    sizes_a = [100] * 10 + [3000] * 10          # h = 0,10,0,0,0,0,10,...
    key_a = sbt.batch_tuning_key(sizes_a, "dsb", "bf16", 128)
    key_b = sbt.batch_tuning_key([9000] * 20, "dsb", "bf16", 128)
    cache = {"format": "sbtrack batch tuning 1", "entries": [
        {"key": key_a, "split_n": 2304, "tail_words": 4096, "fill": 0.5, "seconds": 1.0},
        {"key": key_b, "split_n": 0, "tail_words": 8192, "fill": 1.0, "seconds": 2.0},
        {"key": "dsb fp16 M128 h=0,0,0,0,0,0,0,0,1", "split_n": 64, "tail_words": 0,
         "fill": 0.25, "band_rows": 3000}]}
    path = tmp_path / "cache.json"
    path.write_text(json.dumps(cache, indent=1))
    cases = [("exact", sizes_a, "dsb", "bf16", 128),
             ("near", [100] * 9 + [3000] * 11, "dsb", "bf16", 128),   # distance 0.1
             ("far", [100] * 20, "dsb", "bf16", 128),                 # distance 1.0
             ("other_mode", sizes_a, "bsb", "bf16", 128),
             ("other_agents", sizes_a, "dsb", "bf16", 64),
             ("fp16", [9000], "dsb", "fp16", 128)]
    env = dict(os.environ, SBT_BATCH_TUNING_CACHE=str(path))
    r = subprocess.run([sys.executable, "-c", LOOKUP_SCRIPT.format(root=ROOT, cases=cases)],
                       capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr
    got = json.loads(r.stdout.strip().splitlines()[-1])
    assert got["exact"] == {"split_n": 2304, "tail_words": 4096, "fill": 0.5, "band_rows": 0,
                            "from_cache": True}
    assert got["near"] == got["exact"]
    default = {"split_n": 0, "tail_words": 8192, "fill": 1.0, "band_rows": 0,
               "from_cache": False}
    assert got["far"] == default and got["other_mode"] == default
    assert got["other_agents"] == default
    assert got["fp16"] == {"split_n": 64, "tail_words": 0, "fill": 0.25, "band_rows": 3000,
                           "from_cache": True}


def test_committed_cache_is_well_formed():
    path = os.path.join(ROOT, "paper_2402_14718_amd", "tuning", "batch_tuning.json")
    if not os.path.exists(path):
        pytest.skip("no tuning cache committed yet")
    data = json.load(open(path))
    assert data["format"] == "sbtrack batch tuning 1"
    for e in data["entries"]:
        mode, prec, m, h = e["key"].split(" ")
        assert mode in ("bsb", "dsb", "asb") and prec in ("fp16", "bf16")
        assert m.startswith("M") and h.startswith("h=") and len(h[2:].split(",")) == 9
        assert 0 <= e["split_n"] and 0 <= e["tail_words"] <= 8192 and 0 < e["fill"] <= 1
        assert e["seconds"] <= e["default_seconds"]
