"""Summaries of rocprofv3 CSV output for the library's kernels.

    python -m paper_1703_06999_amd.profiling stats  <kernel_stats.csv>  <title>  <command>
    python -m paper_1703_06999_amd.profiling traffic <fetch counter_collection.csv> \\
        <write counter_collection.csv> <title> <command> <calibration MiB>
    python -m paper_1703_06999_amd.profiling counters <title> <command ;; command ...> \\
        <kernel_stats.csv> <counter_collection.csv> [<counter_collection.csv> ...]

`stats` tabulates calls and durations per kernel.  `traffic` turns per-dispatch FETCH_SIZE and
WRITE_SIZE (KiB) into bytes per launch for every stage of an evaluation.  Each counter is scaled
by what it reads for a plain streaming kernel of known size in the same run: torch's `neg` over a
buffer of the size given by bench.py's --copy-calibration-mb, which reads and writes that many
bytes.  `counters` tabulates any SQ/TCP/GRBM counters per stage (average per launch) with the
VALU issue time they imply next to the measured duration.  The outputs record the SHA-256 of the
kernel sources, so a stale summary can be detected.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1703_06999_amd/csrc/kernels.h", "paper_1703_06999_amd/csrc/fft_lds.h",
                  "paper_1703_06999_amd/csrc/vdwxc_gpu.hip"]

# kernel symbol -> stage name, in launch order within one potential evaluation
_STAGE_ORDER = [
    ("k_theta_zfwd", "theta_zfwd"), ("k_ypass_fwd", "y_fwd"), ("k_xcontract", "x_contract"),
    ("k_ypass_inv", "y_inv"), ("k_zinv_assemble", "z_assemble"),
    ("k_div_z", "div_z"), ("k_div_y", "div_y"), ("k_div_x", "div_x"), ("k_lda_pw92", "lda"),
]


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    s = re.sub(r"\(.*", "", name).replace("void ", "").replace("vdwxc::", "")
    if s.startswith("k_ypass"):
        s = s.replace("k_ypass", "k_ypass_fwd" if ", -1>" in s else "k_ypass_inv")
    return s


def kernel_stats(path: str, title: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}", "", "Command (repository root, one MI355X):", "", "    " + command, "",
           "Library kernels only; durations in microseconds.", "",
           "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in rows:
        if "vdwxc::" not in r["Name"]:
            continue
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")
    return "\n".join(out) + "\n"


def _dispatches(path):
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
    return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows]


def _per_stage(disp):
    """Assign library dispatches to stages in launch order; average over evaluations."""
    acc = collections.defaultdict(list)
    lib = [(n, v) for n, v in disp if "vdwxc::" in n]
    i = 0
    while i < len(lib):
        for sym, stage in _STAGE_ORDER:
            if i < len(lib) and _short(lib[i][0]).startswith(sym):
                acc[stage].append(lib[i][1])
                i += 1
        if i < len(lib) and not any(_short(lib[i][0]).startswith(s) for s, _ in _STAGE_ORDER[:1]):
            i += 1   # unexpected kernel: skip it
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic(fetch_csv: str, write_csv: str, title: str, command: str, calib_bytes: float) -> str:
    fd, wd = _dispatches(fetch_csv), _dispatches(write_csv)
    cal_f = [v for n, v in fd if "neg_kernel" in n]
    cal_w = [v for n, v in wd if "neg_kernel" in n]
    f_scale = calib_bytes / (cal_f[-1] * 1024.0)
    w_scale = calib_bytes / (cal_w[-1] * 1024.0)
    fs, ws = _per_stage(fd), _per_stage(wd)
    out = [f"# {title}", "", "Commands (repository root, one MI355X), one counter per run:", ""]
    out += ["    " + c for c in command.split(" ;; ")]
    out += ["", f"source_sha256: {source_hash()}", "",
            f"Calibration: a plain streaming kernel (torch neg) reads and writes {calib_bytes / 2**20:.0f} MiB;",
            f"FETCH_SIZE reported {cal_f[-1]:.0f} KiB (scale {f_scale:.4f}), "
            f"WRITE_SIZE {cal_w[-1]:.0f} KiB (scale {w_scale:.4f}).", "",
            "| stage | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch |", "|---|---|---|---|"]
    for _, stage in _STAGE_ORDER:
        if stage in fs and stage in ws:
            b = fs[stage] * 1024.0 * f_scale + ws[stage] * 1024.0 * w_scale
            out.append(f"| `{stage}` | {fs[stage]:.1f} | {ws[stage]:.1f} | {b:.0f} |")
    return "\n".join(out) + "\n"


# ---- counters per stage, by kernel name ---------------------------------------------------------

# MI355X: 256 compute units of 4 SIMDs; a wave64 VALU instruction occupies its SIMD for 4 cycles
CUS, SIMDS_PER_CU, CLOCK_HZ = 256, 4, 2.4e9


def stage_of(kernel_name: str):
    """Stage of an evaluation a library kernel belongs to (None for other kernels)."""
    s = _short(kernel_name)
    for sym, stage in _STAGE_ORDER + [("k_grad_z", "grad_z"), ("k_grad_y", "grad_y"), ("k_grad_x", "grad_x")]:
        if s.startswith(sym):
            return stage
    return None


def _counter_rows(path):
    """{(stage, counter): [values per dispatch]} of one counter_collection.csv."""
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        st = stage_of(r["Kernel_Name"])
        if st is not None:
            acc[(st, r["Counter_Name"])].append(float(r["Counter_Value"]))
    return acc


def counters(title: str, command: str, stats_csv: str, counter_csvs) -> str:
    durations = {}
    for r in csv.DictReader(open(stats_csv)):
        st = stage_of(r["Name"])
        if st is not None:
            durations[st] = float(r["AverageNs"]) * 1e-9
    acc = collections.defaultdict(list)
    for p in counter_csvs:
        for k, v in _counter_rows(p).items():
            acc[k].extend(v)
    names = sorted({c for _, c in acc})
    stages = [st for _, st in _STAGE_ORDER if any((st, c) in acc for c in names)]
    out = [f"# {title}", "", "Commands (repository root, one MI355X, TMPDIR=/tmp), one counter set per run:", ""]
    out += ["    " + c for c in command.split(" ;; ")]
    out += ["", f"source_sha256: {source_hash()}", "",
            "Average per launch of each library kernel; durations from the kernel-trace run.", "",
            "| counter | " + " | ".join(f"`{st}`" for st in stages) + " |",
            "|---|" + "---|" * len(stages)]
    for c in names:
        out.append(f"| {c} | " + " | ".join(f"{sum(acc[(st, c)]) / len(acc[(st, c)]):.4g}" if acc.get((st, c)) else "-"
                                             for st in stages) + " |")
    if "SQ_INSTS_VALU" in names:
        # the least time the SIMDs need to issue the VALU instructions, all 1024 busy
        row_t, row_d, row_f = [], [], []
        for st in stages:
            v = acc.get((st, "SQ_INSTS_VALU"))
            t_valu = (sum(v) / len(v)) * 4.0 / (CUS * SIMDS_PER_CU * CLOCK_HZ) if v else None
            d = durations.get(st)
            row_t.append(f"{t_valu * 1e3:.3f}" if t_valu else "-")
            row_d.append(f"{d * 1e3:.3f}" if d else "-")
            row_f.append(f"{t_valu / d:.2f}" if t_valu and d else "-")
        out.append("| VALU issue time at full rate, ms (SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz)) | "
                   + " | ".join(row_t) + " |")
        out.append("| measured duration, ms | " + " | ".join(row_d) + " |")
        out.append("| VALU issue time / duration | " + " | ".join(row_f) + " |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "stats":
        print(kernel_stats(sys.argv[2], sys.argv[3], sys.argv[4]), end="")
    elif mode == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], float(sys.argv[6]) * 2**20), end="")
    elif mode == "counters":
        print(counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5:]), end="")
    else:
        raise SystemExit(__doc__)
