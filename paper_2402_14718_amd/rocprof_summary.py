"""Summarise rocprofv3 CSV output into a short markdown profile record.

    python -m paper_2402_14718_amd.rocprof_summary --title T --kernel REGEX \\
        --trace DIR --fetch DIR --write DIR [--sq DIR ...] \\
        --copy-fetch DIR --copy-write DIR --command CMD ... > profiles/NAME.md

Each DIR is a rocprofv3 output directory (``-f csv``).  FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) are scaled by what the same counters read for
a plain device-to-device copy of known size (``bench.py --copy-calibration``
copies 256 MiB three times), giving HBM bytes per launch of the kernel that
matches REGEX.  The record ends with a JSON block (sources hash included) so
the benchmark can tell whether the counters still describe the current
kernel.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {
    "sb_resident_reg": ["csrc/sb_resident_reg.hip", "csrc/sb_resident_reg_step.hpp",
                        "csrc/sb_resident_reg_bsb.hip", "csrc/sb_resident_reg_dsb.hip",
                        "csrc/sb_resident_reg_asb.hip", "csrc/sb_device.hpp", "csrc/sb_kernels.hpp"],
    "sb_stream": ["csrc/sb_stream.hip", "csrc/sb_stream_quad.hip", "csrc/sb_stream_chunk.hpp",
                  "csrc/sb_stream_kernels.hpp", "csrc/sb_device.hpp", "csrc/sb_kernels.hpp"],
    "sb_batch": ["csrc/sb_batch.hip", "csrc/sb_batch_step.hpp", "csrc/sb_batch_mode.hip",
                 "csrc/sb_device.hpp", "csrc/sb_kernels.hpp"],
    "sb_batch_gang": ["csrc/sb_batch_gang.hip", "csrc/sb_device.hpp", "csrc/sb_kernels.hpp"],
    "sb_stream_mfma": ["csrc/sb_stream_mfma.hip", "csrc/sb_stream_mfma.hpp", "csrc/sb_stream_kernels.hpp",
                       "csrc/sb_stream_chunk.hpp", "csrc/sb_device.hpp", "csrc/sb_kernels.hpp"],
}
COPY_BYTES = 256 << 20


def sources_hash(kernel_family: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel_family]:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _one(d, pattern):
    files = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not files:
        raise FileNotFoundError(f"{pattern} under {d}")
    return files[0]


def counters(d):
    """{kernel name: {counter: [values per dispatch]}}"""
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(_one(d, "*counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            out[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def pick(table, regex):
    for name, v in table.items():
        if re.search(regex, name):
            return name, v
    raise KeyError(regex)


def pick_all(table, regex):
    """Every kernel whose name matches: [(name, {counter: [values]})]."""
    out = [(name, v) for name, v in table.items() if re.search(regex, name)]
    if not out:
        raise KeyError(regex)
    return out


def per_solve(matches, counter):
    """Sum over the matched kernels (one launch each per solve, e.g. the
    batch kernel's two workgroup shapes) of the counter's mean per
    dispatch."""
    return sum(sum(v[counter]) / len(v[counter]) for _, v in matches if counter in v)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--title", required=True)
    ap.add_argument("--kernel", required=True, help="regex of the dominant kernel")
    ap.add_argument("--family", required=True, choices=sorted(KERNEL_SOURCES))
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--sq", action="append", default=[],
                    help="folder of one SQ counter pass (repeatable; passes are merged)")
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--note", action="append", default=[])
    a = ap.parse_args(argv)

    lines = [f"# {a.title}", ""]
    if a.command:
        lines += ["Commands (run from /tmp with TMPDIR=/tmp; R = repository root):", "", "```"]
        lines += a.command + ["```", ""]
    lines += ["## Kernel time (rocprofv3 --kernel-trace --stats)", "",
              "| kernel | calls | avg us | total us | % |", "|---|---|---|---|---|"]
    with open(_one(a.trace, "*kernel_stats.csv")) as f:
        rows = list(csv.DictReader(f))
    for r in rows[:12]:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs'])/1e3:.2f} | "
                     f"{float(r['TotalDurationNs'])/1e3:.1f} | {float(r['Percentage']):.1f} |")
    # per launch of the kernel; when the regex matches several kernels (one
    # launch each per solve), the sum of their mean durations: per solve
    dom = [r for r in rows if re.search(a.kernel, r["Name"])]
    avg_ns = sum(float(r["TotalDurationNs"]) / max(1, int(r["Calls"])) for r in dom)

    cf = counters(a.copy_fetch)
    cw = counters(a.copy_write)
    _, cfv = pick(cf, "copyBuffer")
    _, cwv = pick(cw, "copyBuffer")
    fetch_copy_kib = max(cfv["FETCH_SIZE"])
    write_copy_kib = max(cwv["WRITE_SIZE"])
    f_fac = COPY_BYTES / 1024.0 / fetch_copy_kib
    w_fac = COPY_BYTES / 1024.0 / write_copy_kib

    mf = pick_all(counters(a.fetch), a.kernel)
    mw = pick_all(counters(a.write), a.kernel)
    fetch_kib = per_solve(mf, "FETCH_SIZE")
    write_kib = per_solve(mw, "WRITE_SIZE")
    hbm_bytes = fetch_kib * 1024 * f_fac + write_kib * 1024 * w_fac
    names = ", ".join(f"`{n}`" for n, _ in mf)

    lines += ["", "## HBM bytes of the dominant kernel (rocprofv3 --pmc, one pass each)", "",
              f"Kernel: {names}" + (" (one launch of each per solve; figures summed)"
                                    if len(mf) > 1 else ""), "",
              "| counter | KiB per dispatch | copy calibration (KiB read for 256 MiB) | factor | bytes per launch |",
              "|---|---|---|---|---|",
              f"| FETCH_SIZE | {fetch_kib:.1f} | {fetch_copy_kib:.1f} | {f_fac:.3f} | {fetch_kib*1024*f_fac:.4g} |",
              f"| WRITE_SIZE | {write_kib:.1f} | {write_copy_kib:.1f} | {w_fac:.3f} | {write_kib*1024*w_fac:.4g} |",
              "", f"Average duration of that kernel: {avg_ns/1e3:.2f} us; HBM traffic "
              f"{hbm_bytes/1e6:.2f} MB per launch = {hbm_bytes/avg_ns:.2f} GB/s.", ""]
    sq = None
    if a.sq:
        sq = {}
        for d in a.sq:
            m = pick_all(counters(d), a.kernel)
            sq.update({c: per_solve(m, c) for c in {c for _, vs in m for c in vs}})
        lines += ["## Instruction counters (SQ, summed over the chip, per dispatch)", "",
                  "| counter | value |", "|---|---|"]
        for c, v in sorted(sq.items()):
            lines.append(f"| {c} | {v:.4g} |")
        if "SQ_INSTS_VALU" in sq:
            slots = 256 * 4 * 2.4e9 * avg_ns * 1e-9 / 4.0
            lines += ["", f"VALU issue: {sq['SQ_INSTS_VALU']:.4g} wave-instructions against "
                      f"{slots:.4g} wave64 issue slots in the kernel's duration "
                      f"(256 CU x 4 SIMD x 2.4 GHz / 4 cycles) = {sq['SQ_INSTS_VALU']/slots:.2f}."]
        if "SQ_LDS_IDX_ACTIVE" in sq and "GRBM_GUI_ACTIVE" in sq:
            # GRBM_GUI_ACTIVE comes summed over the 8 XCDs: per-XCD active
            # cycles x 32 CUs per XCD = CU cycles of the chip
            cu_cycles = sq["GRBM_GUI_ACTIVE"] / 8 * 256
            lines += ["", f"LDS: indexed-access cycles {sq['SQ_LDS_IDX_ACTIVE']:.4g} = "
                      f"{sq['SQ_LDS_IDX_ACTIVE']/cu_cycles:.2f} of the CU cycles "
                      f"(GRBM_GUI_ACTIVE / 8 XCDs x 256 CUs); bank-conflict cycles "
                      f"{sq.get('SQ_LDS_BANK_CONFLICT', 0.0):.4g} = "
                      f"{sq.get('SQ_LDS_BANK_CONFLICT', 0.0)/cu_cycles:.2f} of the CU cycles, "
                      f"{sq.get('SQ_LDS_BANK_CONFLICT', 0.0)/max(1.0, sq['SQ_LDS_IDX_ACTIVE']):.2f} "
                      f"of the LDS cycles; out-of-range LDS accesses "
                      f"{sq.get('SQ_LDS_MEM_VIOLATIONS', 0.0):.0f}."]
        lines.append("")
    for n in a.note:
        lines += [n, ""]
    rec = {"kernel_regex": a.kernel, "family": a.family, "sources_sha": sources_hash(a.family),
           "avg_launch_us": avg_ns / 1e3, "fetch_kib": fetch_kib, "write_kib": write_kib,
           "fetch_factor": f_fac, "write_factor": w_fac, "hbm_bytes_per_launch": hbm_bytes,
           "sq": sq}
    lines += ["## Record", "", "```json", json.dumps(rec, indent=1), "```", ""]
    sys.stdout.write("\n".join(lines))


def read_record(md_path):
    """The JSON record of a profile markdown file, or None."""
    try:
        text = open(md_path).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    return json.loads(m.group(1)) if m else None


if __name__ == "__main__":
    main()
