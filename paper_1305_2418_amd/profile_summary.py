"""Summarise rocprofv3 CSV output into the short text records kept under profiles/.

    python -m paper_1305_2418_amd.profile_summary stats  <rocprof dir> <out.txt> "<command>"
    python -m paper_1305_2418_amd.profile_summary pmc    <rocprof dir> <out.txt> "<command>"
    python -m paper_1305_2418_amd.profile_summary traffic <fetch dir> <write dir> <mesh> <out.json>

`traffic` converts the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) of
the sweep kernels into bytes per launch, scaled by what the same counters read
for the streaming kernel the benchmark runs with --calibrate-copy (a bitwise
NOT of 1 GiB of int32 into another buffer: it reads and writes exactly 1 GiB).
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_OPS = "paper_1305_2418_amd/csrc/mgfr_ops.h"
SWEEPS = {"k_mx_colour": ["paper_1305_2418_amd/csrc/mgfr_mixed.hip", _OPS],
          "k_mx_sweep2": ["paper_1305_2418_amd/csrc/mgfr_mixed.hip", _OPS],
          "k_sweep_fused": ["paper_1305_2418_amd/csrc/mgfr_solver.hip", _OPS]}
BY_GRID = ("k_mx_colour", "k_sweep_fused", "k_mx_correct_residual", "k_mx_restrict_pass", "k_mx_sweep2",
           "k_amrx_sweep", "k_amrx_restrict")
COPY = "bitwise_not"


def _short(name: str) -> str:
    base = name.replace("(anonymous namespace)::", "").split("(")[0]
    return base.replace("void ", "").replace("mgfr::", "")[:70]


def _rows(d, pattern):
    out = []
    for f in glob.glob(os.path.join(d, "**", pattern), recursive=True):
        with open(f) as fh:
            out.extend(csv.DictReader(fh))
    return out


def stats(d, out, cmd):
    rows = _rows(d, "*kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {cmd}", "",
             f"{'kernel':70s} {'calls':>6s} {'total ms':>10s} {'avg us':>10s} {'min us':>9s} {'max us':>9s} {'%':>6s}"]
    for r in rows[:40]:
        lines.append(f"{_short(r['Name']):70s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:9.2f} "
                     f"{float(r['MaxNs']) / 1e3:9.2f} {float(r['Percentage']):6.2f}")
    # the dominant kernels run on every mesh level: split their launches by grid size
    trace = _rows(d, "*kernel_trace.csv")
    if trace:
        gkey = next((k for k in trace[0] if k.startswith("Grid_Size")), None)
        per = collections.defaultdict(list)
        for r in trace:
            name = _short(r["Kernel_Name"])
            if gkey and any(name.startswith(k) for k in BY_GRID):
                per[(name, int(r[gkey]))].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        if per:
            lines += ["", f"# by grid size ({gkey}, work-items; the largest grid is the finest level)",
                      f"{'kernel':40s} {'grid':>12s} {'calls':>6s} {'avg us':>10s} {'min us':>9s} {'max us':>9s}"]
            for (name, grid), v in sorted(per.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
                lines.append(f"{name:40s} {grid:12d} {len(v):6d} {sum(v) / len(v):10.2f} {min(v):9.2f} {max(v):9.2f}")
    open(out, "w").write("\n".join(lines) + "\n")


def _counters(d):
    agg = collections.defaultdict(list)
    for r in _rows(d, "*counter_collection.csv"):
        agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return agg


def pmc(d, out, cmd):
    agg = _counters(d)
    lines = [f"# rocprofv3 counters (mean per dispatch)", f"# command: {cmd}", ""]
    for (k, c), v in sorted(agg.items(), key=lambda kv: (_short(kv[0][0]), kv[0][1])):
        if any(s in k for s in list(SWEEPS) + [COPY, "k_mx_correct", "k_mx_restrict", "k_mx_prolong", "k_conv3d", "k_cic", "k_force"]):
            lines.append(f"{_short(k):70s} {c:22s} n={len(v):5d} mean={sum(v) / len(v):.5g} max={max(v):.5g}")
    open(out, "w").write("\n".join(lines) + "\n")


def _hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic(dfetch, dwrite, mesh, out):
    fa, wa = _counters(dfetch), _counters(dwrite)

    def pick(agg, counter, name, largest=True, exact=True):
        # exact: the kernel itself (k_mx_colour, not k_mx_colour_zero); else a substring of its name
        vals = [max(v) if largest else sum(v) / len(v) for (k, c), v in agg.items()
                if c == counter and (_short(k).split("<")[0] == name if exact else name in k)]
        return max(vals) if vals else None

    cf = pick(fa, "FETCH_SIZE", COPY, exact=False)
    cw = pick(wa, "WRITE_SIZE", COPY, exact=False)
    gib_kib = float(1 << 20)
    res = {"calibration": {"copy_fetch_kib": cf, "copy_write_kib": cw, "copy_bytes": 1 << 30}}
    for name, src in SWEEPS.items():
        # the finest-level launches are the largest dispatches of the kernel
        fv = pick(fa, "FETCH_SIZE", name)
        wv = pick(wa, "WRITE_SIZE", name)
        if fv is None or wv is None or not cf or not cw:
            continue
        ff, fw = gib_kib / cf, gib_kib / cw
        res[name] = {"mesh": mesh, "fetch_kib": fv, "write_kib": wv, "fetch_scale": ff, "write_scale": fw,
                     "bytes_per_launch": (fv * ff + wv * fw) * 1024.0, "source_hash": _hash(src)}
    json.dump(res, open(out, "w"), indent=1)


if __name__ == "__main__":
    kind = sys.argv[1]
    if kind == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif kind == "pmc":
        pmc(sys.argv[2], sys.argv[3], sys.argv[4])
    elif kind == "traffic":
        traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5])
    else:
        raise SystemExit(__doc__)
