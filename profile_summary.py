"""Summaries of rocprofv3 databases for ``profiles/`` (text only).

    python profile_summary.py kernels DB TITLE COMMAND
        per-kernel calls / total / average duration (``--kernel-trace --stats``)

    python profile_summary.py traffic FETCH_DB WRITE_DB WORKLOAD COMMAND_FETCH COMMAND_WRITE
        FETCH_SIZE and WRITE_SIZE per dispatch (two ``--pmc`` runs of
        ``bench.py --copy-probe-mib 256``), scaled by what the counters read for
        the 256 MiB device copy in the same run, per kernel class of the solve's
        kernel timer; ends with a JSON block that ``bench.py`` reads for the
        roofline ``traffic`` field (with a digest of the kernel sources: a
        changed source makes the figure stale, and bench reports null).

    python profile_summary.py mfma DB KERNEL SIMDS COMMAND
        matrix-core counters of one kernel (a ``--pmc`` run with
        SQ_INSTS_VALU_MFMA_MOPS_F32, SQ_INSTS_VALU_MFMA_F32,
        SQ_VALU_MFMA_BUSY_CYCLES, SQ_BUSY_CYCLES, GRBM_GUI_ACTIVE)

Only reads the databases; runs nothing.
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
import sqlite3
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_1712_08740_amd", "csrc")

# kernel class of the solve's kernel timer -> (kernel-name prefix, source files)
CLASSES = {
    # the fine down leg is a tiled kernel or, on large grids, the marching one:
    # a launch is either (one component, pooled over its alternatives)
    "vc_down": ((("k_down<Fine5", "k_down_zmarch"),), ["vcycle_tiled.hip", "hh_internal.h"]),
    "vc_up": ("k_up<Fine5", ["vcycle_tiled.hip", "hh_internal.h"]),
    "vc_down_coarse": ("k_down<Coarse9", ["vcycle_tiled.hip", "hh_internal.h"]),
    "vc_up_coarse": ("k_up<Coarse9", ["vcycle_tiled.hip", "hh_internal.h"]),
    # one launch of the class: the single-source product, or for a batch the
    # matrix-core product and the sum of its k-split partials
    "gemv": (("k_gemv_pred", "k_coarsest_mfma", "k_coarsest_sum"),
             ["coarsest.hip", "hh_internal.h"]),
    "apply_dot": ("k_apply_dot", ["krylov.hip", "hh_internal.h", "givens.h"]),
    "axpy_dot": ("k_axpy_dcgs", ["krylov.hip", "hh_internal.h", "givens.h"]),
    "axpy_norm": ("k_dot_blocks", ["krylov.hip", "hh_internal.h", "givens.h"]),
    "givens": ("k_givens_tail", ["krylov.hip", "hh_internal.h", "givens.h"]),
    "reduce": ("k_reduce_pred", ["krylov.hip", "hh_internal.h", "givens.h"]),
    "pcr": ("k_pcr_apply", ["pcr.hip", "hh_internal.h"]),
}
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_KIB = 256 * 1024


def source_digest(kernel_class: str) -> str:
    h = hashlib.sha256()
    for f in CLASSES[kernel_class][1]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    return name.replace("hh::(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def kernels(db: str, title: str, cmd: str) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels").fetchall()
    out = [f"# {title}", "", "Command (on the MI355X, from the repository root):", "",
           f"    {cmd}", "",
           "Kernel durations from `rocprofv3 --kernel-trace --stats` (top_kernels); "
           "times in microseconds. Set-up kernels (Galerkin products, banded LU and "
           "inverse of the coarsest operator) run once per problem.", "",
           "| kernel | calls | total us | avg us | % |", "|---|---:|---:|---:|---:|"]
    for n, c, t, a, p in rows:
        out.append(f"| {_short(n)} | {c} | {t:.1f} | {a:.3f} | {p:.1f} |")
    return "\n".join(out) + "\n"


def _counter(db: str, ctr: str):
    con = sqlite3.connect(db)
    d = collections.defaultdict(list)
    for name, v in con.execute("select kernel_name, value from counters_collection "
                               "where counter_name=?", (ctr,)):
        d[_short(name)].append(v)
    return d


def traffic(fetch_db: str, write_db: str, workload: str, cmd_f: str, cmd_w: str) -> str:
    f = _counter(fetch_db, "FETCH_SIZE")
    w = _counter(write_db, "WRITE_SIZE")
    # the probe is the largest device copy of the run
    fc, wc = max(f[COPY_KERNEL]), max(w[COPY_KERNEL])
    ff, fw = COPY_KIB / fc, COPY_KIB / wc
    out = [f"# HBM traffic per launch, {workload}", "",
           "Commands (on the MI355X, from /tmp with TMPDIR=/tmp):", "",
           f"    {cmd_f}", f"    {cmd_w}", "",
           f"Scale: the 256 MiB device copy reads {fc:.0f} KiB "
           f"(FETCH_SIZE) and writes {wc:.0f} KiB (WRITE_SIZE); "
           f"factors {ff:.3f} and {fw:.3f} are applied below. FETCH_SIZE counts L2 misses "
           "served by the fabric (Infinity Cache or HBM).", "",
           "| kernel class | launches | fetch KiB/launch | write KiB/launch | scaled MB/launch |",
           "|---|---:|---:|---:|---:|"]
    table = {}
    for cls, (prefixes, _) in CLASSES.items():
        if isinstance(prefixes, str):
            prefixes = (prefixes,)
        # a launch of the class dispatches each of its kernels once: sum their means
        fk = wk = 0.0
        n = 0
        for prefix in prefixes:     # a str, or a tuple of alternative kernels
            fv = [v for k, vs in f.items() if k.startswith(prefix) for v in vs]
            wv = [v for k, vs in w.items() if k.startswith(prefix) for v in vs]
            if not fv or not wv:
                continue
            # launches of steps the device had already closed return at once: drop them
            fv = [v for v in fv if v > 0.05 * max(fv)]
            wv = [v for v in wv if v > 0.05 * max(wv)]
            fk += statistics.mean(fv)
            wk += statistics.mean(wv)
            n = max(n, len(fv))
        if n == 0:
            continue
        b = (fk * ff + wk * fw) * 1024.0
        table[cls] = {"bytes_per_launch": b, "digest": source_digest(cls)}
        out.append(f"| {cls} | {n} | {fk:.1f} | {wk:.1f} | {b / 1e6:.3f} |")
    out += ["", "```json", json.dumps({workload: table}, indent=1), "```", ""]
    return "\n".join(out)


def mfma(db: str, kernel: str, simds: int, cmd: str) -> str:
    """Matrix-core counters of one kernel (mean per dispatch): the flops its MFMA
    ops stand for (SQ_INSTS_VALU_MFMA_MOPS_F32 counts units of 512) and the share
    of SIMD cycles the matrix cores were busy (SQ_VALU_MFMA_BUSY_CYCLES summed
    over the SIMDs, GRBM_GUI_ACTIVE summed over the 8 XCDs)."""
    con = sqlite3.connect(db)
    d = collections.defaultdict(list)
    for name, c, v in con.execute("select kernel_name, counter_name, value "
                                  "from counters_collection"):
        if _short(name).startswith(kernel):
            d[c].append(v)
    m = {c: statistics.mean(v) for c, v in d.items()}
    n = len(next(iter(d.values())))
    gflop = m["SQ_INSTS_VALU_MFMA_MOPS_F32"] * 512 / 1e9
    cycles = m["GRBM_GUI_ACTIVE"] / 8
    busy = m["SQ_VALU_MFMA_BUSY_CYCLES"] / (simds * cycles)
    out = [f"# Matrix-core counters of {kernel}", "", "Command (on the MI355X, from /tmp with "
           "TMPDIR=/tmp):", "", f"    {cmd}", "",
           f"Mean over {n} dispatches.", "",
           "| counter | mean per dispatch |", "|---|---:|"]
    for c in sorted(m):
        out.append(f"| {c} | {m[c]:.0f} |")
    out += ["", f"MFMA work: {gflop:.2f} GFLOP per dispatch (MOPS x 512); "
            f"{m['SQ_INSTS_VALU_MFMA_F32']:.0f} MFMA instructions x 2048 flops = "
            f"{m['SQ_INSTS_VALU_MFMA_F32'] * 2048 / 1e9:.2f} GFLOP.",
            f"Duration: {cycles:.0f} cycles per XCD = {cycles / 2.4e3:.0f} us at 2.4 GHz.",
            f"Matrix cores busy: {100 * busy:.1f}% of the SIMD cycles ({simds} SIMDs).", ""]
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "kernels":
        sys.stdout.write(kernels(*sys.argv[2:5]))
    elif sys.argv[1] == "traffic":
        sys.stdout.write(traffic(*sys.argv[2:7]))
    elif sys.argv[1] == "mfma":
        sys.stdout.write(mfma(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5]))
    else:
        raise SystemExit(__doc__)
