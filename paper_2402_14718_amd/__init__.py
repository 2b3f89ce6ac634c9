"""Python binding of libsbtrack: MI355X simulated bifurcation for track QUBOs.

Method: Okawa, Zeng, Tao, Yung, "Quantum-Annealing-Inspired Algorithms for
Track Reconstruction at High-Energy Colliders" -- hits -> triplet QUBO
(Eq. 13-17) -> ballistic / discrete simulated bifurcation (Eq. 5-12).

Every function here only marshals arguments into the C ABI declared in
include/sbtrack.h; all computation happens in the library (host C++ for
the QUBO construction, HIP kernels for the solver).  PyTorch is used only
to hold device memory and to name the HIP stream for ``solve_dev``.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import numpy as np

from . import _lib
from ._lib import (SBT_BSB, SBT_DSB, SBT_KERNEL_AUTO, SBT_KERNEL_RESIDENT, SBT_KERNEL_STREAM,
                   SbtError, check, load)

MODES = {"bsb": SBT_BSB, "dsb": SBT_DSB, "asb": _lib.SBT_ASB}
KERNELS = {"auto": SBT_KERNEL_AUTO, "resident": SBT_KERNEL_RESIDENT, "stream": SBT_KERNEL_STREAM,
           "stream_tile": _lib.SBT_KERNEL_STREAM_TILE, "stream_rows": _lib.SBT_KERNEL_STREAM_ROWS,
           "stream_mfma": _lib.SBT_KERNEL_STREAM_MFMA}
PRECISIONS = {"fp32": _lib.SBT_PREC_FP32, "fp16": _lib.SBT_PREC_FP16, "bf16": _lib.SBT_PREC_BF16,
              "fp8": _lib.SBT_PREC_FP8, "fp8_block": _lib.SBT_PREC_FP8_BLOCK,
              "bf16x2": _lib.SBT_PREC_BF16X2}
KERNEL_NAMES = {v: k for k, v in KERNELS.items()}

HIT_DTYPE = np.dtype([("hit_id", "<i8"), ("layer", "<i4"), ("pad", "<i4"),
                      ("x", "<f8"), ("y", "<f8"), ("z", "<f8")])


@dataclasses.dataclass
class Qubo:
    """Host copy of an sbt_qubo (b symmetric CSR, ascending columns)."""
    n: int
    a: np.ndarray          # float64 [n]
    row_ptr: np.ndarray    # int64 [n+1]
    col: np.ndarray        # int32 [nnz]
    b: np.ndarray          # float64 [nnz]
    trip_hits: np.ndarray  # int64 [n, 3]

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def max_row_nnz(self) -> int:
        return int(np.diff(self.row_ptr).max()) if self.n else 0

    def as_struct(self):
        """A ctypes sbt_qubo viewing this object's arrays (kept alive by it)."""
        self.a = np.ascontiguousarray(self.a, dtype=np.float64)
        self.row_ptr = np.ascontiguousarray(self.row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(self.col, dtype=np.int32)
        self.b = np.ascontiguousarray(self.b, dtype=np.float64)
        self.trip_hits = np.ascontiguousarray(self.trip_hits, dtype=np.int64)
        return _lib.SbtQubo(
            self.n, self.nnz,
            self.a.ctypes.data_as(C.POINTER(C.c_double)),
            self.row_ptr.ctypes.data_as(C.POINTER(C.c_int64)),
            self.col.ctypes.data_as(C.POINTER(C.c_int32)),
            self.b.ctypes.data_as(C.POINTER(C.c_double)),
            self.trip_hits.ctypes.data_as(C.POINTER(C.c_int64)))


def version() -> str:
    return load().sbt_version().decode()


def build_params_default() -> _lib.SbtBuildParams:
    p = _lib.SbtBuildParams()
    load().sbt_build_params_default(C.byref(p))
    return p


def build_qubo(hits: np.ndarray, params: Optional[_lib.SbtBuildParams] = None) -> Qubo:
    """sbt_build_qubo: hits (record array of HIT_DTYPE) -> Qubo."""
    lib = load()
    hits = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    out = C.POINTER(_lib.SbtQubo)()
    check(lib.sbt_build_qubo(hits.ctypes.data_as(C.POINTER(_lib.SbtHit)), hits.shape[0],
                             C.byref(params) if params is not None else None, C.byref(out)))
    return _take_qubo(out)


def build_qubo_gpu(hits: np.ndarray, params: Optional[_lib.SbtBuildParams] = None):
    """sbt_build_qubo_gpu: the same QUBO built on the GPU.  Returns
    (Qubo, device seconds of the construction)."""
    lib = load()
    hits = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    out = C.POINTER(_lib.SbtQubo)()
    t = C.c_double()
    check(lib.sbt_build_qubo_gpu(hits.ctypes.data_as(C.POINTER(_lib.SbtHit)), hits.shape[0],
                                 C.byref(params) if params is not None else None, C.byref(out),
                                 C.byref(t)))
    return _take_qubo(out), float(t.value)


def _take_qubo(out) -> Qubo:
    """Copy a library-owned sbt_qubo into a Qubo and free it."""
    lib = load()
    try:
        q = out.contents
        n, nnz = int(q.n), int(q.nnz)

        def arr(ptr, count, dtype):
            if count == 0:
                return np.zeros(0, dtype=dtype)
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)

        res = Qubo(n=n, a=arr(q.a, n, np.float64), row_ptr=arr(q.row_ptr, n + 1, np.int64),
                   col=arr(q.col, nnz, np.int32), b=arr(q.b, nnz, np.float64),
                   trip_hits=arr(q.trip_hits, 3 * n, np.int64).reshape(n, 3))
    finally:
        lib.sbt_qubo_free(out)
    return res


def anneal_cpu(q: Qubo, shots: int = 50, sweeps: int = 1000, beta_hot: float = 0.0,
               beta_cold: float = 0.0, seed: int = 0, threads: int = 0) -> dict:
    """sbt_anneal_cpu: single-flip Metropolis annealing on the host."""
    p = _lib.SbtAnnealParams()
    load().sbt_anneal_params_default(C.byref(p))
    p.shots, p.sweeps, p.beta_hot, p.beta_cold = shots, sweeps, beta_hot, beta_cold
    p.seed, p.threads = seed & 0xFFFFFFFFFFFFFFFF, threads
    T = np.zeros(q.n, dtype=np.int8)
    se = np.zeros(shots)
    e, t = C.c_double(), C.c_double()
    s = q.as_struct()
    check(load().sbt_anneal_cpu(C.byref(s), C.byref(p), T.ctypes.data_as(C.POINTER(C.c_int8)),
                                C.byref(e), se.ctypes.data_as(C.POINTER(C.c_double)), C.byref(t)))
    return {"T": T, "energy": float(e.value), "shot_energy": se, "elapsed_s": float(t.value)}


def phi_order(q: Qubo, hits: np.ndarray) -> np.ndarray:
    """sbt_phi_order: triplets sorted by the azimuth (then z) of their
    middle hit; perm[k] = original index of the triplet placed at k."""
    hits = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    perm = np.zeros(max(q.n, 1), dtype=np.int32)
    s = q.as_struct()
    check(load().sbt_phi_order(C.byref(s), hits.ctypes.data_as(C.POINTER(_lib.SbtHit)),
                               hits.shape[0], perm.ctypes.data_as(C.POINTER(C.c_int32))))
    return perm[:q.n]


def permute_qubo(q: Qubo, perm: np.ndarray) -> Qubo:
    """sbt_qubo_permute: spin k of the result is spin perm[k] of q."""
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    if perm.shape != (q.n,):
        raise ValueError("perm must have shape (n,)")
    s = q.as_struct()
    out = C.POINTER(_lib.SbtQubo)()
    check(load().sbt_qubo_permute(C.byref(s), perm.ctypes.data_as(C.POINTER(C.c_int32)),
                                  C.byref(out)))
    return _take_qubo(out)


def energy(q: Qubo, T: np.ndarray) -> float:
    """sbt_energy: FP64 O(T) of Eq. 13 on the host."""
    T = np.ascontiguousarray(T, dtype=np.int8)
    if T.shape != (q.n,):
        raise ValueError("T must have shape (n,)")
    s = q.as_struct()
    e = C.c_double()
    check(load().sbt_energy(C.byref(s), T.ctypes.data_as(C.POINTER(C.c_int8)), C.byref(e)))
    return float(e.value)


def solve_params(agents: int = 32, steps: int = 2000, dt: float = 1.0, a0: float = 1.0,
                 c0: float = 0.0, seed: int = 0, event: int = 0, kernel: str = "auto",
                 energy_every: int = 0, tpb: int = 0,
                 precision: str = "fp32") -> _lib.SbtSolveParams:
    p = _lib.SbtSolveParams()
    load().sbt_solve_params_default(C.byref(p))
    p.agents, p.steps, p.dt, p.a0, p.c0 = agents, steps, dt, a0, c0
    p.seed = seed & 0xFFFFFFFFFFFFFFFF
    p.event = event
    p.kernel = KERNELS[kernel]
    p.energy_every = energy_every
    p.tpb = tpb
    p.precision = PRECISIONS[precision]
    return p


def solve(q: Qubo, mode: str, agents: int = 32, steps: int = 2000, dt: float = 1.0,
          a0: float = 1.0, c0: float = 0.0, seed: int = 0, event: int = 0,
          kernel: str = "auto", energy_every: int = 0, want_state: bool = False,
          want_trace: bool = False, tpb: int = 0, precision: str = "fp32") -> dict:
    """sbt_solve: host QUBO in, host results out (the library uploads,
    solves on the GPU and downloads)."""
    p = solve_params(agents, steps, dt, a0, c0, seed, event, kernel, energy_every, tpb,
                     precision)
    s = q.as_struct()
    T = np.zeros(q.n, dtype=np.int8)
    E = np.zeros(agents, dtype=np.float64)
    n_ck = steps // energy_every if energy_every > 0 else 0
    trace = np.zeros(n_ck, dtype=np.float64) if want_trace else None
    atrace = np.zeros((n_ck, agents), dtype=np.float64) if want_trace and n_ck else None
    xf = np.zeros((q.n, agents), dtype=np.float32) if want_state else None
    yf = np.zeros((q.n, agents), dtype=np.float32) if want_state else None
    r = _lib.SbtResult()
    r.T = T.ctypes.data_as(C.POINTER(C.c_int8))
    r.agent_energy = E.ctypes.data_as(C.POINTER(C.c_double))
    if trace is not None:
        r.trace = trace.ctypes.data_as(C.POINTER(C.c_double))
    if atrace is not None:
        r.agent_trace = atrace.ctypes.data_as(C.POINTER(C.c_double))
    if xf is not None:
        r.x_final = xf.ctypes.data_as(C.POINTER(C.c_float))
        r.y_final = yf.ctypes.data_as(C.POINTER(C.c_float))
    check(load().sbt_solve(C.byref(s), MODES[mode], C.byref(p), C.byref(r)))
    return {"T": T, "agent_energy": E, "energy": r.energy, "best_agent": int(r.best_agent),
            "c0": r.c0, "ising_offset": r.ising_offset, "trace": trace, "agent_trace": atrace,
            "x": xf, "y": yf,
            "kernel": KERNEL_NAMES[int(r.kernel_used)], "elapsed_s": r.elapsed_s,
            "trace_len": int(r.trace_len)}


def workspace_bytes(n: int, nnz: int, mode: str, params: _lib.SbtSolveParams) -> int:
    v = load().sbt_workspace_bytes(n, nnz, MODES[mode], C.byref(params))
    if v == 0:
        raise SbtError(_lib.SBT_EINVAL, load().sbt_last_error().decode())
    return int(v)


def select_kernel(n: int, nnz: int, max_row_nnz: int, mode: str,
                  params: _lib.SbtSolveParams) -> str:
    rc = load().sbt_select_kernel(n, nnz, max_row_nnz, MODES[mode], C.byref(params))
    if rc < 0:
        check(rc)
    return KERNEL_NAMES[rc]


class DeviceSolver:
    """sbt_solve_dev with every buffer held by torch on a HIP device.

    The QUBO is uploaded once; ``run()`` enqueues a complete solve (Ising
    preparation, initial draw, all SB steps, FP64 energies, best agent) on
    the current torch stream and returns without synchronising."""

    def __init__(self, q: Qubo, mode: str, params: _lib.SbtSolveParams, device="cuda",
                 want_state: bool = False, want_trace: bool = False):
        import torch
        self.torch = torch
        self.q = q
        self.mode = mode
        self.params = params
        dev = torch.device(device)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)
        self.a = t(q.a, torch.float64)
        self.row_ptr = t(q.row_ptr.astype(np.int32), torch.int32)
        self.col = t(q.col if q.nnz else np.zeros(1, np.int32), torch.int32)
        self.b = t(q.b if q.nnz else np.zeros(1), torch.float64)
        M = params.agents
        self.ws_bytes = workspace_bytes(q.n, q.nnz, mode, params)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.T = torch.empty(q.n, dtype=torch.int8, device=dev)
        self.agent_energy = torch.empty(M, dtype=torch.float64, device=dev)
        self.best_energy = torch.empty(1, dtype=torch.float64, device=dev)
        self.best_agent = torch.empty(1, dtype=torch.int32, device=dev)
        self.scalars = torch.empty(4, dtype=torch.float64, device=dev)
        self.x = torch.empty((q.n, M), dtype=torch.float32, device=dev) if want_state else None
        self.y = torch.empty((q.n, M), dtype=torch.float32, device=dev) if want_state else None
        n_ck = params.steps // params.energy_every if params.energy_every > 0 else 0
        self.trace = (torch.empty(n_ck, dtype=torch.float64, device=dev)
                      if want_trace and n_ck > 0 else None)
        self.agent_trace = (torch.empty((n_ck, M), dtype=torch.float64, device=dev)
                            if want_trace and n_ck > 0 else None)
        self._dq = _lib.SbtDevQubo(q.n, q.nnz, self.a.data_ptr(), self.row_ptr.data_ptr(),
                                   self.col.data_ptr(), self.b.data_ptr())
        ptr = lambda x: x.data_ptr() if x is not None else None
        self._dr = _lib.SbtDevResult(self.T.data_ptr(), self.agent_energy.data_ptr(),
                                     self.best_energy.data_ptr(), self.best_agent.data_ptr(),
                                     self.scalars.data_ptr(), ptr(self.x), ptr(self.y),
                                     ptr(self.trace), None, None, ptr(self.agent_trace))
        self.max_row = q.max_row_nnz()
        self.kernel = select_kernel(q.n, q.nnz, self.max_row, mode, params)

    def run(self, stream=None) -> None:
        torch = self.torch
        st = stream if stream is not None else torch.cuda.current_stream()
        check(load().sbt_solve_dev(C.byref(self._dq), self.max_row, MODES[self.mode],
                                   C.byref(self.params), C.c_void_p(self.workspace.data_ptr()),
                                   self.ws_bytes, C.byref(self._dr), C.c_void_p(st.cuda_stream)))

    def run_noalloc(self, stream=None) -> None:
        """The same solve through sbt_solve_dev_noalloc: scratch from the
        library's fixed per-device array instead of this object's
        workspace (for callers that cannot allocate)."""
        torch = self.torch
        st = stream if stream is not None else torch.cuda.current_stream()
        check(load().sbt_solve_dev_noalloc(C.byref(self._dq), self.max_row, MODES[self.mode],
                                           C.byref(self.params), C.byref(self._dr),
                                           C.c_void_p(st.cuda_stream)))

    def result(self) -> dict:
        self.torch.cuda.synchronize()
        return {"T": self.T.cpu().numpy(), "agent_energy": self.agent_energy.cpu().numpy(),
                "energy": float(self.best_energy.item()),
                "best_agent": int(self.best_agent.item()),
                "c0": float(self.scalars[0].item()), "ising_offset": float(self.scalars[1].item()),
                "x": None if self.x is None else self.x.cpu().numpy(),
                "y": None if self.y is None else self.y.cpu().numpy(),
                "trace": None if self.trace is None else self.trace.cpu().numpy(),
                "agent_trace": (None if self.agent_trace is None
                                else self.agent_trace.cpu().numpy()),
                "kernel": self.kernel}




def top_k(energy, k: int, stream=None):
    """The k lowest energies of a CUDA float64 vector and their indices,
    ascending, ties to the lower index (sbt_top_k_dev, on the GPU)."""
    import torch
    if not (energy.is_cuda and energy.dtype == torch.float64 and energy.dim() == 1):
        raise ValueError("top_k: energy must be a 1-D float64 CUDA tensor")
    e = energy.contiguous()
    vals = torch.empty(k, dtype=torch.float64, device=e.device)
    idx = torch.empty(k, dtype=torch.int32, device=e.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    check(load().sbt_top_k_dev(C.c_void_p(e.data_ptr()), e.numel(), k, C.c_void_p(vals.data_ptr()),
                               C.c_void_p(idx.data_ptr()), C.c_void_p(st.cuda_stream)))
    return vals, idx


def _concat_batch(qubos):
    n = np.array([q.n for q in qubos], dtype=np.int32)
    nnz = np.array([q.nnz for q in qubos], dtype=np.int64)
    a = np.concatenate([q.a for q in qubos]).astype(np.float64)
    rp = np.concatenate([q.row_ptr.astype(np.int32) for q in qubos])
    col = np.concatenate([q.col for q in qubos] + [np.zeros(1, np.int32)]).astype(np.int32)
    b = np.concatenate([q.b for q in qubos] + [np.zeros(1)]).astype(np.float64)
    return n, nnz, a, rp, col, b


def _split(flat, sizes):
    out, o = [], 0
    for s in sizes:
        out.append(flat[o:o + s])
        o += s
    return out


def solve_batch(qubos, mode: str, precision: str = "fp16", agents: int = 128,
                steps: int = 3000, dt: float = 1.0, a0: float = 1.0, c0: float = 0.0,
                seed: int = 0, event: int = 0, energy_every: int = 0,
                want_agent_energy: bool = False, want_trace: bool = False) -> dict:
    """sbt_solve_batch: host QUBOs in, per-event host results out."""
    p = solve_params(agents, steps, dt, a0, c0, seed, event, "auto", energy_every)
    structs = [q.as_struct() for q in qubos]
    arr = (C.POINTER(_lib.SbtQubo) * len(qubos))(*[C.pointer(s) for s in structs])
    E = len(qubos)
    energy_ = np.zeros(E)
    best = np.zeros(E, dtype=np.int32)
    T = np.zeros(sum(q.n for q in qubos), dtype=np.int8)
    ae = np.zeros(E * agents) if want_agent_energy else None
    n_ck = steps // energy_every if energy_every > 0 else 0
    tr = np.zeros(E * n_ck) if want_trace else None
    atr = np.zeros(E * n_ck * agents) if want_trace and n_ck else None
    r = _lib.SbtBatchResult()
    r.energy = energy_.ctypes.data_as(C.POINTER(C.c_double))
    r.best_agent = best.ctypes.data_as(C.POINTER(C.c_int32))
    r.T = T.ctypes.data_as(C.POINTER(C.c_int8))
    if ae is not None:
        r.agent_energy = ae.ctypes.data_as(C.POINTER(C.c_double))
    if tr is not None:
        r.trace = tr.ctypes.data_as(C.POINTER(C.c_double))
    if atr is not None:
        r.agent_trace = atr.ctypes.data_as(C.POINTER(C.c_double))
    check(load().sbt_solve_batch(arr, E, MODES[mode], PRECISIONS[precision], C.byref(p),
                                 C.byref(r)))
    return {"energy": energy_, "best_agent": best, "T": _split(T, [q.n for q in qubos]),
            "agent_energy": None if ae is None else ae.reshape(E, agents),
            "trace": None if tr is None else tr.reshape(E, n_ck),
            "agent_trace": None if atr is None else atr.reshape(E, n_ck, agents),
            "elapsed_s": r.elapsed_s}


def wall_clock_hz() -> float:
    """sbt_wall_clock_hz: tick rate of the device wall clock."""
    hz = C.c_double()
    check(load().sbt_wall_clock_hz(C.byref(hz)))
    return float(hz.value)


def c0_scan(q: Qubo, mode: str, factors, precision: str = "fp16", agents: int = 128,
            steps: int = 3000, dt: float = 1.0, a0: float = 1.0, c0: float = 0.0,
            seed: int = 0, event: int = 0) -> dict:
    """sbt_c0_scan: one batch solving q once per c0 factor from one start."""
    p = solve_params(agents, steps, dt, a0, c0, seed, event)
    f = np.ascontiguousarray(factors, dtype=np.float64)
    e = np.zeros(f.shape[0])
    ba = np.zeros(f.shape[0], dtype=np.int32)
    best = C.c_int32()
    s = q.as_struct()
    check(load().sbt_c0_scan(C.byref(s), MODES[mode], PRECISIONS[precision], C.byref(p),
                             f.ctypes.data_as(C.POINTER(C.c_double)), f.shape[0],
                             e.ctypes.data_as(C.POINTER(C.c_double)),
                             ba.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(best)))
    return {"energy": e, "best_agent": ba, "best_factor": int(best.value),
            "factor": float(f[best.value])}


def batch_tuning(split_n: int = 0, tail_words: int = 8192, fill: float = 1.0,
                 band_rows: int = 0):
    """An explicit sbt_batch_tuning."""
    t = _lib.SbtBatchTuning()
    load().sbt_batch_tuning_default(C.byref(t))
    t.split_n, t.tail_words, t.fill = int(split_n), int(tail_words), float(fill)
    t.band_rows = int(band_rows)
    return t


def tuning_dict(t: _lib.SbtBatchTuning) -> dict:
    return {"split_n": int(t.split_n), "tail_words": int(t.tail_words), "fill": float(t.fill),
            "band_rows": int(t.band_rows), "from_cache": bool(t.from_cache)}


def batch_tuning_key(sizes, mode: str, precision: str, agents: int) -> str:
    """sbt_batch_tuning_key of a batch of events with these n."""
    n = np.ascontiguousarray(sizes, dtype=np.int32)
    buf = C.create_string_buffer(256)
    check(load().sbt_batch_tuning_key(n.ctypes.data_as(C.POINTER(C.c_int32)), n.shape[0],
                                      MODES[mode], PRECISIONS[precision], agents, buf, 256))
    return buf.value.decode()


def batch_tuning_lookup(sizes, mode: str, precision: str, agents: int) -> _lib.SbtBatchTuning:
    """sbt_batch_tuning_lookup: the cached tuning of a batch, or the defaults."""
    n = np.ascontiguousarray(sizes, dtype=np.int32)
    t = _lib.SbtBatchTuning()
    check(load().sbt_batch_tuning_lookup(n.ctypes.data_as(C.POINTER(C.c_int32)), n.shape[0],
                                         MODES[mode], PRECISIONS[precision], agents, C.byref(t)))
    return t


class DeviceBatchSolver:
    """sbt_batch_plan once, then sbt_batch_run per call, every buffer held by
    torch on a HIP device (events concatenated).  `tuning`: None = the
    library's cached tuning for this batch (sbt_batch_tuning_lookup),
    "default" = the untuned schedule, or an sbt_batch_tuning."""

    def __init__(self, qubos, mode: str, precision: str, params: _lib.SbtSolveParams,
                 device="cuda", want_agent_energy: bool = False, want_trace: bool = False,
                 want_agent_state: bool = False, c0_scale=None, same_start: bool = False,
                 want_clock: bool = False, tuning=None, target=None):
        import torch
        self.torch = torch
        self.mode, self.precision, self.params = mode, precision, params
        dev = torch.device(device)
        n, nnz, a, rp, col, b = _concat_batch(qubos)
        self.n_host, self.nnz_host = n, nnz
        self.sizes = [int(v) for v in n]
        t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt).to(dev)
        self.a, self.rp, self.col, self.b = (t(a, torch.float64), t(rp, torch.int32),
                                             t(col, torch.int32), t(b, torch.float64))
        E, M = len(qubos), params.agents
        self.E = E
        lib = load()
        np_ = n.ctypes.data_as(C.POINTER(C.c_int32))
        nz_ = nnz.ctypes.data_as(C.POINTER(C.c_int64))
        if tuning is None:
            tuning = batch_tuning_lookup(n, mode, precision, params.agents)
        elif isinstance(tuning, str) and tuning == "default":
            tuning = batch_tuning()
        self.tuning = tuning
        self.ws_bytes = int(lib.sbt_batch_workspace_bytes_tuned(np_, nz_, E, C.byref(params),
                                                                C.byref(tuning)))
        if self.ws_bytes == 0:
            raise SbtError(_lib.SBT_EINVAL, lib.sbt_last_error().decode())
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.best_energy = torch.empty(E, dtype=torch.float64, device=dev)
        self.best_agent = torch.empty(E, dtype=torch.int32, device=dev)
        self.best_T = torch.empty(int(n.sum()), dtype=torch.int8, device=dev)
        self.offset = torch.empty(E, dtype=torch.float64, device=dev)
        self.agent_energy = (torch.empty(E * M, dtype=torch.float64, device=dev)
                             if want_agent_energy else None)
        n_ck = params.steps // params.energy_every if params.energy_every > 0 else 0
        self.n_ckpt = n_ck
        self.trace = (torch.empty(E * n_ck, dtype=torch.float64, device=dev)
                      if want_trace and n_ck > 0 else None)
        self.agent_trace = (torch.empty(E * n_ck * M, dtype=torch.float64, device=dev)
                            if want_trace and n_ck > 0 else None)
        self.ckpt_clock = (torch.zeros(E * (n_ck + 1) * M, dtype=torch.int64, device=dev)
                           if want_clock else None)
        st = torch.cuda.current_stream()
        self._c0_scale = (None if c0_scale is None
                          else np.ascontiguousarray(c0_scale, dtype=np.float64))
        if self._c0_scale is not None and self._c0_scale.shape != (E,):
            raise ValueError("c0_scale must have one entry per event")
        cs = (None if self._c0_scale is None
              else self._c0_scale.ctypes.data_as(C.POINTER(C.c_double)))
        rc = lib.sbt_batch_plan_tuned(np_, nz_, E, cs, 1 if same_start else 0, C.byref(params),
                                      C.byref(tuning), C.c_void_p(self.workspace.data_ptr()),
                                      self.ws_bytes, C.c_void_p(st.cuda_stream))
        if rc < 0:
            check(rc)
        self.n_items = rc
        # target mode: per-event energies at which the event's work stops
        self.target = (None if target is None else
                       t(np.asarray(target, dtype=np.float64).reshape(E), torch.float64))
        self._db = _lib.SbtDevBatch(E, np_, nz_, self.a.data_ptr(), self.rp.data_ptr(),
                                    self.col.data_ptr(), self.b.data_ptr(),
                                    None if self.target is None else self.target.data_ptr())
        tot = int(n.sum()) * M
        self.agent_T = torch.empty(tot, dtype=torch.int8, device=dev) if want_agent_state else None
        self.agent_x = torch.empty(tot, dtype=torch.float32, device=dev) if want_agent_state else None
        ptr = lambda x: x.data_ptr() if x is not None else None
        self._dr = _lib.SbtDevBatchResult(self.best_energy.data_ptr(), self.best_agent.data_ptr(),
                                          self.best_T.data_ptr(), ptr(self.agent_energy),
                                          self.offset.data_ptr(), ptr(self.trace), None, None,
                                          ptr(self.agent_T), ptr(self.agent_x),
                                          ptr(self.agent_trace), ptr(self.ckpt_clock))

    def run(self, stream=None) -> None:
        st = stream if stream is not None else self.torch.cuda.current_stream()
        check(load().sbt_batch_run_tuned(C.byref(self._db), MODES[self.mode],
                                         PRECISIONS[self.precision], C.byref(self.params),
                                         C.byref(self.tuning),
                                         C.c_void_p(self.workspace.data_ptr()), self.ws_bytes,
                                         C.byref(self._dr), C.c_void_p(st.cuda_stream)))

    def plan_info(self) -> dict:
        """The tuning this batch runs with and its work-item count."""
        return dict(tuning_dict(self.tuning), work_items=self.n_items)

    def result(self) -> dict:
        self.torch.cuda.synchronize()
        M = self.params.agents
        return {"energy": self.best_energy.cpu().numpy(),
                "best_agent": self.best_agent.cpu().numpy(),
                "T": _split(self.best_T.cpu().numpy(), self.sizes),
                "offset": self.offset.cpu().numpy(),
                "agent_energy": (None if self.agent_energy is None
                                 else self.agent_energy.cpu().numpy().reshape(self.E, M)),
                "trace": (None if self.trace is None
                          else self.trace.cpu().numpy().reshape(self.E, self.n_ckpt)),
                "agent_trace": (None if self.agent_trace is None else
                                self.agent_trace.cpu().numpy().reshape(self.E, self.n_ckpt, M)),
                "ckpt_clock": (None if self.ckpt_clock is None else
                               self.ckpt_clock.cpu().numpy().reshape(self.E, self.n_ckpt + 1, M)),
                "agent_T": (None if self.agent_T is None else
                            [v.reshape(-1, M) for v in _split(self.agent_T.cpu().numpy(),
                                                              [s * M for s in self.sizes])]),
                "agent_x": (None if self.agent_x is None else
                            [v.reshape(-1, M) for v in _split(self.agent_x.cpu().numpy(),
                                                              [s * M for s in self.sizes])])}


__all__ = ["Qubo", "DeviceSolver", "DeviceBatchSolver", "build_qubo", "energy", "solve",
           "phi_order", "permute_qubo", "build_qubo_gpu", "c0_scan", "anneal_cpu",
           "solve_batch", "solve_params", "wall_clock_hz", "batch_tuning",
           "batch_tuning_key", "batch_tuning_lookup", "tuning_dict", "workspace_bytes", "select_kernel",
           "build_params_default", "version", "load", "SbtError", "HIT_DTYPE", "MODES",
           "KERNELS", "PRECISIONS"]
