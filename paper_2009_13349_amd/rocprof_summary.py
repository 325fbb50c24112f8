"""Summaries of rocprofv3 CSV output for the CCD kernels.

    python -m paper_2009_13349_amd.rocprof_summary stats <kernel_stats.csv>
    python -m paper_2009_13349_amd.rocprof_summary traffic <fetch_counter_collection.csv> \
        <write_counter_collection.csv> [--copy-bytes N] [--tuning k=v,...]
    python -m paper_2009_13349_amd.rocprof_summary counters <counter_collection.csv>... \
        [--tuning k=v,...]

`stats` prints the per-kernel duration table of a --kernel-trace --stats run.
`traffic` prints per-dispatch HBM bytes of FETCH_SIZE and WRITE_SIZE runs
(counters in KiB), each scaled by the ratio of a known device-to-device copy's
size to what the same counter read for it (the largest __amd_rocclr_copyBuffer
dispatch), and writes a JSON record of the scaled figures keyed by the
SHA-256 of the kernel sources they were taken with.
`counters` prints and records (same keying) the per-dispatch mean of every
counter in the given --pmc runs, per CCD kernel.  With --tuning the records
also carry the ccd_tuning the profiled run used.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in
                  ("ccd_kernels.hip", "ccd_device.hpp", "ccd_internal.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name: str) -> str:
    return name.split("(")[0].replace("void ", "") if name.startswith(("void ccd", "ccd")) else name[:48]


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg ms | min ms | max ms | % |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                   f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out)


def _per_kernel(path: str):
    agg = defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def traffic(fetch_path: str, write_path: str, copy_bytes: int = 256 << 20):
    fetch, write = _per_kernel(fetch_path), _per_kernel(write_path)
    cf = max(fetch.get("__amd_rocclr_copyBuffer", [0]))
    cw = max(write.get("__amd_rocclr_copyBuffer", [0]))
    sf = copy_bytes / (cf * 1024) if cf else None
    sw = copy_bytes / (cw * 1024) if cw else None
    out = ["| kernel | dispatches | FETCH_SIZE KiB (raw) | WRITE_SIZE KiB (raw) | read GB (scaled) | "
           "written GB (scaled) |", "|---|---|---|---|---|---|"]
    rec = {"kernel_source_sha256": kernel_source_hash(), "copy_bytes": copy_bytes,
           "fetch_scale": sf, "write_scale": sw, "kernels": {}}
    for name in fetch:
        if not name.startswith(("void ccd", "ccd")):
            continue
        f = sum(fetch[name]) / len(fetch[name])
        w = sum(write.get(name, [0])) / max(1, len(write.get(name, [0])))
        fb = f * 1024 * sf if sf else None
        wb = w * 1024 * sw if sw else None
        out.append(f"| `{short(name)}` | {len(fetch[name])} | {f:.0f} | {w:.0f} | "
                   f"{fb / 1e9 if fb else float('nan'):.3f} | {wb / 1e9 if wb else float('nan'):.3f} |")
        rec["kernels"][short(name)] = {"fetch_bytes": fb, "write_bytes": wb}
    out.append("")
    out.append(f"copy calibration: {copy_bytes} B copied; FETCH_SIZE read {cf:.0f} KiB "
               f"(scale {sf:.4f}), WRITE_SIZE read {cw:.0f} KiB (scale {sw:.4f})")
    return "\n".join(out), rec


def counters(paths):
    """Per-dispatch means of every counter of the CCD kernels over --pmc runs."""
    agg = defaultdict(lambda: defaultdict(list))
    for path in paths:
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            if not name.startswith(("void ccd", "ccd")):
                continue
            agg[short(name)][r["Counter_Name"]].append(float(r["Counter_Value"]))
    rec = {"kernel_source_sha256": kernel_source_hash(), "kernels": {}}
    out = ["| kernel | counter | dispatches | per dispatch |", "|---|---|---|---|"]
    for k in sorted(agg):
        rec["kernels"][k] = {}
        for c in sorted(agg[k]):
            v = agg[k][c]
            rec["kernels"][k][c] = sum(v) / len(v)
            out.append(f"| `{k}` | {c} | {len(v)} | {sum(v) / len(v):.4g} |")
    return "\n".join(out), rec


def _tuning(argv):
    if "--tuning" not in argv:
        return None
    kv = argv[argv.index("--tuning") + 1]
    return {k: int(v) for k, v in (x.split("=") for x in kv.split(",") if x)}


def main(argv):
    if argv[0] == "stats":
        print(stats(argv[1]))
    elif argv[0] == "traffic":
        copy_bytes = 256 << 20
        if "--copy-bytes" in argv:
            copy_bytes = int(argv[argv.index("--copy-bytes") + 1])
        table, rec = traffic(argv[1], argv[2], copy_bytes)
        rec["tuning"] = _tuning(argv)
        print(table)
        print()
        print(json.dumps(rec))
    elif argv[0] == "counters":
        paths = argv[1:argv.index("--tuning")] if "--tuning" in argv else argv[1:]
        table, rec = counters(paths)
        rec["tuning"] = _tuning(argv)
        print(table)
        print()
        print(json.dumps(rec))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
