"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_1401_7441_amd.profiling stats <kernel_trace.csv> <out.md> <command...>
    python -m paper_1401_7441_amd.profiling traffic <fetch_csv> <write_csv> <copy_bytes>
                                             <workload> <dtype> <out.json>

`stats` turns the kernel_trace.csv of a `rocprofv3 --kernel-trace --stats
--output-format csv` run into a short Markdown table per kernel kind
(dispatches, average, min, max and total duration) headed by the command
that produced it.

`traffic` reads the per-dispatch counter_collection.csv of two counter runs
(FETCH_SIZE, then WRITE_SIZE, both in KiB per dispatch) of the native
driver, whose first kernel is a plain copy of `copy_bytes` bytes (read
`copy_bytes`, written `copy_bytes`).  Each counter is scaled by the ratio of
the copy's true bytes to what the counter read for it, and the per-launch
averages of every kernel kind are merged into out.json under
"<workload>/<dtype>/<kind>", stamped with the hash of the kernel sources
they were taken on.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("wvl_kernels.hip", "wvl_fused.hip", "wvl_static.hip", "wvl_host.cpp",
              "wvl_internal.h", "wvl_filters.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


_KIN_AXIS = {"0": "kin_xcol", "1": "kin_ycol", "2": "kin_zcol"}


def kind_of(name: str):
    """Kernel kind (the library's profiling names) of a demangled kernel
    name, or None for kernels that are not the library's."""
    if "k_copy" in name:
        return "copy"
    m = re.search(r"wvl::k_(\w+)(?:<([^>]*)>)?", name)
    if not m:
        return None
    base, targs = m.group(1), m.group(2) or ""
    if base == "kin_col":
        return _KIN_AXIS[targs.split(",")[-1].strip()]
    if base == "gather":
        return "uncompress"
    if base == "scatter":
        return "compress"
    if base == "back_out":       # the x analysis pass, writing the compressed output
        return "back_x"
    return base          # sparse_values is split into S and H by dispatch order


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def stats_markdown(trace_csv: str, command: str) -> str:
    """Per-kind dispatch statistics of the library's kernels from a
    rocprofv3 kernel_trace.csv (other kernels, e.g. input generation, are
    left out; sparse_values dispatches alternate S and H)."""
    rows = _rows(trace_csv)
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    per = {}
    cfg = {}
    nsparse = 0
    for r in rows:
        k = kind_of(r["Kernel_Name"])
        if k is None or k == "copy":
            continue
        if k == "sparse_values":
            k = "sparse_s" if nsparse % 2 == 0 else "sparse_h"
            nsparse += 1
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        per.setdefault(k, {"name": re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", ""),
                           "ms": []})["ms"].append(d)
        cfg.setdefault(k, {}).setdefault((r.get("Grid_Size_X"), r.get("Grid_Size_Y")),
                                         []).append(d)
    tot = sum(sum(v["ms"]) for v in per.values())
    out = ["Command:", "", "```", command, "```", "",
           "| kind | kernel | dispatches | avg ms | min ms | max ms | total ms | % of library time |",
           "|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1]["ms"])):
        ms = v["ms"]
        out.append(f"| {k} | `{v['name']}` | {len(ms)} | {sum(ms) / len(ms):.3f} | {min(ms):.3f} | "
                   f"{max(ms):.3f} | {sum(ms):.3f} | {100 * sum(ms) / tot:.1f} |")
    # per launch configuration: a kind launches once per bin with its own
    # grid; configurations seen at least 5 times are the timed layout (the
    # others are autotuner candidates or side runs)
    out += ["", "Launch configurations seen at least 5 times (grid x, y; the timed layout):", "",
            "| kind | grid | dispatches | avg ms |", "|---|---|---|---|"]
    for k in sorted(cfg):
        for g, ms in sorted(cfg[k].items(), key=lambda kv: -len(kv[1])):
            if len(ms) >= 5:
                out.append(f"| {k} | {g[0]} x {g[1]} | {len(ms)} | {sum(ms) / len(ms):.3f} |")
    return "\n".join(out) + "\n"


def _per_kind(path, counter):
    """{kind: [values per dispatch]} for one counter; sparse_values
    dispatches alternate S (first) and H."""
    rows = [r for r in _rows(path) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    out = {}
    nsparse = 0
    for r in rows:
        k = kind_of(r["Kernel_Name"])
        if k is None:
            continue
        if k == "sparse_values":
            k = "sparse_s" if nsparse % 2 == 0 else "sparse_h"
            nsparse += 1
        out.setdefault(k, []).append(float(r["Counter_Value"]))
    return out


def traffic(fetch_csv, write_csv, copy_bytes, workload, dtype, out_json):
    fk = _per_kind(fetch_csv, "FETCH_SIZE")
    wk = _per_kind(write_csv, "WRITE_SIZE")
    f_copy = sum(fk["copy"]) / len(fk["copy"]) * 1024.0
    w_copy = sum(wk["copy"]) / len(wk["copy"]) * 1024.0
    fs, ws = copy_bytes / f_copy, copy_bytes / w_copy
    tab = {}
    if os.path.exists(out_json):
        with open(out_json) as f:
            tab = json.load(f)
    h = source_hash()
    for k in sorted(set(fk) & set(wk)):
        if k == "copy":
            continue
        fb = sum(fk[k]) / len(fk[k]) * 1024.0 * fs
        wb = sum(wk[k]) / len(wk[k]) * 1024.0 * ws
        tab[f"{workload}/{dtype}/{k}"] = {"bytes_per_launch": fb + wb, "read_bytes": fb,
                                          "write_bytes": wb, "fetch_scale": fs,
                                          "write_scale": ws, "source_hash": h}
    with open(out_json, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    return tab


if __name__ == "__main__":
    if len(sys.argv) >= 4 and sys.argv[1] == "stats":
        with open(sys.argv[3], "w") as f:
            f.write(stats_markdown(sys.argv[2], " ".join(sys.argv[4:])))
    elif len(sys.argv) == 8 and sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6], sys.argv[7])
    else:
        sys.exit(__doc__)
