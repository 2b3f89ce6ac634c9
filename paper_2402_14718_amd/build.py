"""Build libsbtrack.so in-tree for gfx950.

Host C++ (QUBO construction, FP64 energy, status) is compiled with g++
without floating-point contraction, so every cut decision is a fixed IEEE
expression.  Host orchestration (solve.cpp) uses only the HIP runtime API.
Kernels are compiled by hipcc for gfx950 with packed-FP32 instruction
selection disabled.  Run ``python -m paper_2402_14718_amd.build``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB_NAME = "libsbtrack.so"
LIB_PATH = os.path.join(PKG, LIB_NAME)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HOST_SOURCES = ["status.cpp", "validate.cpp", "build_qubo.cpp", "order.cpp", "anneal.cpp",
                "batch_tuning.cpp"]
RUNTIME_SOURCES = ["solve.cpp", "solve_batch.cpp"]
HIP_SOURCES = ["sb_kernels.hip", "sb_resident_reg.hip", "sb_resident_reg_bsb.hip",
               "sb_resident_reg_dsb.hip", "sb_resident_reg_asb.hip", "sb_batch.hip",
               "sb_stream.hip", "build_qubo_gpu.hip", "solve_noalloc.hip", "sb_batch_gang.hip",
               "sb_stream_tile.hip", "topk.hip", "sb_stream_quad.hip", "sb_stream_mfma.hip"]
# one source built several times: (source, object tag, extra flags) -- the
# batched step kernel once per (mode, coupling format, workgroup shape), in
# parallel
HIP_VARIANTS = [("sb_batch_mode.hip", f"{m}_{j}_{tpb}",
                 [f"-DSBT_BATCH_MODE={mi}", f"-DSBT_BATCH_JP={ji}", f"-DSBT_BATCH_TPB={tpb}"])
                for mi, m in enumerate(("bsb", "dsb", "asb")) for ji, j in enumerate(("fp16", "bf16"))
                for tpb in (1024, 512)]
# the GPU QUBO builder evaluates the host builder's cut expressions: no
# floating-point contraction, like the host file
HIP_EXTRA_FLAGS = {"build_qubo_gpu.hip": ["-ffp-contract=off"]}

HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
              "-Wall", "-Wextra", "-Wno-unused-parameter", f"-I{INCLUDE}", f"-I{CSRC}"]
HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-parameter", f"-I{INCLUDE}", f"-I{CSRC}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path.
    Sources compile in parallel (the kernel files take minutes each)."""
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    gxx = shutil.which("g++") or "g++"
    os.makedirs(BUILD, exist_ok=True)
    jobs = []  # (command, object)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(([gxx, *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    for src in RUNTIME_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(([gxx, *HOST_FLAGS, "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-c",
                      os.path.join(CSRC, src), "-o", obj], obj))
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(([hipcc, *HIP_FLAGS, *HIP_EXTRA_FLAGS.get(src, []), "-c",
                      os.path.join(CSRC, src), "-o", obj], obj))
    for src, tag, flags in HIP_VARIANTS:
        obj = os.path.join(BUILD, f"{src}.{tag}.o")
        jobs.append(([hipcc, *HIP_FLAGS, *flags, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        for f in [pool.submit(_run, cmd, verbose) for cmd, _ in jobs]:
            f.result()
    objs = [obj for _, obj in jobs]
    tmp = LIB_PATH + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
          f"-L{ROCM}/lib", "-lamdhip64", "-ldl", "-pthread", f"-Wl,-rpath,{ROCM}/lib"], verbose)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
