"""Summaries of rocprofv3 runs of the step kernel.

stats:   kernel-trace statistics (``rocprofv3 --kernel-trace --stats``) into a
         short markdown table.
traffic: HBM bytes per step launch from two counter runs (FETCH_SIZE, then
         WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
         reads for the library's plain copy kernel of known size; written as
         JSON (read by bench.py, tagged with the kernel source hash) and markdown.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "csrc", "mlb_kernels.hip")


STEP_IMPL = os.path.join(HERE, "csrc", "mlb_step_impl.h")
STEP_UNITS = ("mlb_kernels.hip", "mlb_kernels2.hip", "mlb_persist.hip")


def kernel_sha(src: str = KERNEL_SRC) -> str:
    """Short hash of a kernel source file (default: the one-step kernels); for
    the step kernels' translation units it covers the device code they share
    (mlb_step_impl.h) as well."""
    h = hashlib.sha256()
    with open(src, "rb") as f:
        h.update(f.read())
    if os.path.basename(src) in STEP_UNITS:
        with open(STEP_IMPL, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return hits[-1]


def _col(row: dict, *names):
    for n in names:
        for k in row:
            if k.strip().lower() == n.lower():
                return row[k]
    raise KeyError(names)


def kernel_stats(d: str):
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    out = []
    for r in rows:
        out.append({"name": _col(r, "Name", "KernelName"), "calls": int(_col(r, "Calls")),
                    "total_ns": float(_col(r, "TotalDurationNs")), "avg_ns": float(_col(r, "AverageNs")),
                    "min_ns": float(_col(r, "MinNs")), "max_ns": float(_col(r, "MaxNs")),
                    "pct": float(_col(r, "Percentage"))})
    return out


def counter_per_dispatch(d: str, kernel_substr: str, counter: str) -> float:
    """Mean over matching dispatches of the counter's value (summed over its
    per-dispatch records)."""
    per = {}
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        if kernel_substr not in _col(r, "Kernel_Name"):
            continue
        if _col(r, "Counter_Name") != counter:
            continue
        key = _col(r, "Dispatch_Id")
        per[key] = per.get(key, 0.0) + float(_col(r, "Counter_Value"))
    if not per:
        raise ValueError("no %s records for kernels matching %r in %s" % (counter, kernel_substr, d))
    return sum(per.values()) / len(per)


def cmd_stats(a):
    st = kernel_stats(a.dir)
    lines = ["# rocprofv3 kernel statistics: %s" % a.title, "",
             "Command (from the repository root):", "", "```", a.command, "```", "",
             "| kernel | calls | avg [us] | min [us] | max [us] | total [ms] | % |",
             "|---|---|---|---|---|---|---|"]
    for k in sorted(st, key=lambda k: -k["total_ns"])[:12]:
        lines.append("| `%s` | %d | %.2f | %.2f | %.2f | %.3f | %.1f |" % (
            k["name"][:90], k["calls"], k["avg_ns"] / 1e3, k["min_ns"] / 1e3, k["max_ns"] / 1e3,
            k["total_ns"] / 1e6, k["pct"]))
    if a.extra:
        lines += ["", a.extra]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print(open(a.out).read())


def cmd_traffic(a):
    f_k = counter_per_dispatch(a.fetch, a.kernel, "FETCH_SIZE")
    w_k = counter_per_dispatch(a.write, a.kernel, "WRITE_SIZE")
    f_c = counter_per_dispatch(a.copy_fetch, "copy_probe", "FETCH_SIZE")
    w_c = counter_per_dispatch(a.copy_write, "copy_probe", "WRITE_SIZE")
    kib = a.copy_bytes / 1024.0
    sf, sw = kib / f_c, kib / w_c          # counter KiB -> true KiB
    fetch_b = f_k * sf * 1024.0
    write_b = w_k * sw * 1024.0
    alg = a.bytes_per_unit * a.nodes
    src = os.path.join(HERE, "csrc", a.source)
    res = {"kernel": a.kernel, "kernel_source": a.source, "kernel_sha": kernel_sha(src), "nodes": a.nodes,
           "tile_rows": a.tile_rows,
           "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
           "bytes_per_launch": fetch_b + write_b, "algorithmic_bytes_per_launch": alg,
           "fetch_scale": sf, "write_scale": sw,
           "raw_fetch_kib": f_k, "raw_write_kib": w_k, "copy_fetch_kib": f_c, "copy_write_kib": w_c,
           "copy_bytes": a.copy_bytes}
    json.dump(res, open(a.out_json, "w"), indent=1)
    md = ["# HBM traffic of `%s` (%s)" % (a.kernel, a.title), "",
          "Counter runs (from the repository root), one counter per run:", "", "```"] + \
         a.commands.split(";;") + ["```", "",
          "| quantity | value |", "|---|---|",
          "| FETCH_SIZE per step launch (raw) | %.0f KiB |" % f_k,
          "| WRITE_SIZE per step launch (raw) | %.0f KiB |" % w_k,
          "| copy kernel, %d bytes: FETCH_SIZE / WRITE_SIZE | %.0f / %.0f KiB |" % (a.copy_bytes, f_c, w_c),
          "| scale factors (true / counter) | %.4f / %.4f |" % (sf, sw),
          "| measured HBM bytes per launch | %.1f MB (read %.1f + write %.1f) |" % (
              (fetch_b + write_b) / 1e6, fetch_b / 1e6, write_b / 1e6),
          "| algorithmic bytes per launch | %.1f MB (%d B x %d nodes) |" % (alg / 1e6, a.bytes_per_unit, a.nodes),
          "| measured / algorithmic | %.3f |" % ((fetch_b + write_b) / alg),
          "", "Kernel source (`%s`) sha256[:16]: `%s`" % (a.source, res["kernel_sha"])]
    open(a.out_md, "w").write("\n".join(md) + "\n")
    print("\n".join(md))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--command", required=True)
    s.add_argument("--extra", default="")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--kernel", default="step_kernel")
    t.add_argument("--tile-rows", type=int, default=None, help="tile rows of the profiled launches (recorded)")
    t.add_argument("--nodes", type=int, required=True)
    t.add_argument("--bytes-per-unit", type=int, default=28)
    t.add_argument("--source", default="mlb_kernels.hip", help="kernel source file under csrc/ (for its hash)")
    t.add_argument("--title", default="")
    t.add_argument("--commands", required=True)
    t.add_argument("--out-json", required=True)
    t.add_argument("--out-md", required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic}[a.cmd](a)


if __name__ == "__main__":
    main()
