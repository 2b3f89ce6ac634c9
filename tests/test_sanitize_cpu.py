"""The library's host code under sanitizers (no GPU).

The pure host sources -- QUBO construction, spin order and relabelling,
FP64 energy, the simulated-annealing comparator, QUBO validation and error
reporting -- are compiled with g++ together with the driver
``tests/sanitize/host_abi_check.cpp`` twice: with AddressSanitizer +
UndefinedBehaviorSanitizer (any report aborts the run) and with
ThreadSanitizer (the annealer's host threads).  The driver runs every host
entry point on generated events and on malformed inputs; its outputs must
equal the regular library's bit for bit, so the sanitized code is the code
that ships.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import trackgen as tg

sbt = pytest.importorskip("paper_2402_14718_amd")

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_14718_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in
           ("status.cpp", "validate.cpp", "build_qubo.cpp", "order.cpp", "anneal.cpp")]
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_abi_check.cpp")
FLAVOURS = {
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
    "tsan": ["-fsanitize=thread"],
}
EVENTS = [(tg.tiny_spec(), 1), (tg.tiny_spec(), 3), (tg.plain_spec(), 100),
          (tg.plain_spec(300), 7), (tg.EventSpec(n_particles=200, eta_max=0.8, noise_frac=0.4), 2)]


def _build(flavour, out_dir):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = os.path.join(out_dir, f"host_abi_check_{flavour}")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           *FLAVOURS[flavour], f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", *SOURCES,
           DRIVER, "-o", exe, "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _write_events(path):
    hits = []
    with open(path, "wb") as f:
        for spec, seed in EVENTS:
            h = np.ascontiguousarray(tg.generate(spec, seed).hits_struct(), dtype=sbt.HIT_DTYPE)
            np.array([h.shape[0]], dtype=np.int64).tofile(f)
            h.tofile(f)
            hits.append(h)
    return hits


def _read(buf, off, dtype, count):
    a = np.frombuffer(buf, dtype=dtype, count=count, offset=off)
    return a, off + a.nbytes


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("sanitize"))


@pytest.mark.parametrize("flavour", sorted(FLAVOURS))
def test_host_code_clean_under_sanitizer_and_equal_to_library(flavour, workdir):
    exe = _build(flavour, workdir)
    ev_path = os.path.join(workdir, f"events_{flavour}.bin")
    out_path = os.path.join(workdir, f"out_{flavour}.bin")
    hits = _write_events(ev_path)
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
    r = subprocess.run([exe, ev_path, out_path], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.strip() == f"events {len(EVENTS)}, ok"
    buf = open(out_path, "rb").read()
    off = 0
    for h in hits:
        q = sbt.build_qubo(h)
        n, off = _read(buf, off, np.int32, 1)
        nnz, off = _read(buf, off, np.int64, 1)
        assert (int(n[0]), int(nnz[0])) == (q.n, q.nnz)
        for want, dt, cnt in ((q.a, np.float64, q.n), (q.row_ptr, np.int64, q.n + 1),
                              (q.col, np.int32, q.nnz), (q.b, np.float64, q.nnz),
                              (q.trip_hits.reshape(-1), np.int64, 3 * q.n)):
            got, off = _read(buf, off, dt, cnt)
            assert np.array_equal(got, want)
        if q.n == 0:
            continue
        perm = sbt.phi_order(q, h)
        got, off = _read(buf, off, np.int32, q.n)
        assert np.array_equal(got, perm)
        qp = sbt.permute_qubo(q, perm)
        for want, dt, cnt in ((qp.row_ptr, np.int64, q.n + 1), (qp.col, np.int32, q.nnz),
                              (qp.b, np.float64, q.nnz)):
            got, off = _read(buf, off, dt, cnt)
            assert np.array_equal(got, want)
        T = np.array([(i * 7 + 3) % 5 < 2 for i in range(q.n)], dtype=np.int8)
        got, off = _read(buf, off, np.float64, 1)
        assert got[0] == sbt.energy(q, T)
        ann = sbt.anneal_cpu(q, shots=6, sweeps=20, seed=11, threads=2)
        got, off = _read(buf, off, np.float64, 6)
        assert np.array_equal(got, ann["shot_energy"])
    assert off == len(buf)
