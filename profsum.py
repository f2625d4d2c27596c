"""Condense rocprofv3 output into the short summaries kept with the code.

Kernel table (kernel, calls, average / total milliseconds, share) from a
``--kernel-trace --stats --output-format csv`` run:

    python profsum.py <run>_kernel_stats.csv

HBM traffic of one kernel from ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``
runs (each its own run, counter values in KiB per dispatch) of a program
that first copied ``copy_mib`` MiB device to device: each counter is scaled
by the bytes that copy moved over what the counter read for it.

    python profsum.py traffic KERNEL COPY_MIB SOURCE OUT.json \\
        plain=<fetch_csv>,<write_csv> [packed=<fetch_csv>,<write_csv>]

(the last 10 dispatches of KERNEL are averaged: one reconstruction's
iterations, after any autotuner passes).
"""
import csv
import hashlib
import json
import re
import sys


def short_name(name: str) -> str:
    name = name.replace("void ", "").replace("lmtof::(anonymous namespace)::", "")
    m = re.match(r"([A-Za-z_0-9:]+(?:<[^>]*>)?)", name)
    return m.group(1) if m else name


def table(path: str) -> str:
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    out = ["| kernel | calls | avg ms | total ms | % of GPU time |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def counter_values(path: str, kernel: str):
    """Per-dispatch values of the one counter in a counter_collection.csv:
    (values of `kernel`'s dispatches, values of the device copies).  A
    kernel name "a+b" adds the dispatches of a and b pairwise (a stage of
    one launch of each per iteration)."""
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    parts = kernel.split("+")
    mine, copies = {k: [] for k in parts}, []
    for r in rows:
        name = short_name(r["Kernel_Name"]).split("<")[0]
        if name in mine:
            mine[name].append(float(r["Counter_Value"]))
        elif "copyBuffer" in r["Kernel_Name"]:
            copies.append(float(r["Counter_Value"]))
    n = min(len(v) for v in mine.values())
    total = [sum(mine[k][len(mine[k]) - n + q] for k in parts) for q in range(n)]
    return total, copies


def traffic(kernel: str, copy_mib: int, source: str, storages: dict, last: int = 10) -> dict:
    ref_kib = copy_mib * 1024.0
    rec = {"kernel": kernel, "source_sha256": hashlib.sha256(open(source, "rb").read()).hexdigest(),
           "copy_reference_mib": copy_mib,
           "note": f"KiB per dispatch, averaged over the last {last} {kernel} launches of the run (one "
                   "reconstruction's iterations); a scale is the bytes the device-to-device copy moved over "
                   "what the counter read for it"}
    scales = {}
    for storage, (fetch_csv, write_csv) in storages.items():
        out = {}
        for what, path in (("fetch", fetch_csv), ("write", write_csv)):
            vals, copies = counter_values(path, kernel)
            vals = vals[-last:]
            if not vals or not copies:
                raise SystemExit(f"{path}: no {kernel} dispatch or no copy reference")
            scales.setdefault(what, []).append(ref_kib / max(copies))
            out[f"{what}_kib"] = sum(vals) / len(vals)
            out[f"{what}_dispatches"] = len(vals)
        rec[storage] = out
    rec["fetch_scale"] = round(sum(scales["fetch"]) / len(scales["fetch"]), 4)
    rec["write_scale"] = round(sum(scales["write"]) / len(scales["write"]), 4)
    return rec


if __name__ == "__main__":
    if sys.argv[1] == "traffic":
        kernel, copy_mib, source, out = sys.argv[2], int(sys.argv[3]), sys.argv[4], sys.argv[5]
        storages = {}
        for arg in sys.argv[6:]:
            k, v = arg.split("=", 1)
            storages[k] = tuple(v.split(","))
        rec = traffic(kernel, copy_mib, source, storages)
        with open(out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec, indent=1))
    else:
        print(table(sys.argv[1]))
