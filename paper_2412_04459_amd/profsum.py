"""Summaries of rocprofv3 runs of bench.py, written as short markdown files.

    python -m paper_2412_04459_amd.profsum --trace DIR [--fetch DIR --write DIR]
        --out profiles/NAME.md --cmd "<the commands that produced DIR...>"

--trace   output directory of `rocprofv3 --kernel-trace --stats --output-format csv`
--fetch   output directory of `rocprofv3 --pmc FETCH_SIZE --output-format csv`
--write   output directory of `rocprofv3 --pmc WRITE_SIZE --output-format csv`
--pmc     output directory of any other `rocprofv3 --pmc ... --output-format csv`
          run (repeatable): every counter in it, mean per dispatch per kernel

The counter runs are expected to include the 1 GiB device copy that
`bench.py --calibrate` performs; the ratio of its known bytes to what the
counter reports scales the counter values of the other kernels.  The summary
ends with a JSON block (kernel -> average duration, calls, traffic per
dispatch) stamped with a hash of the HIP sources, which bench.py uses to
report measured traffic only while the kernels are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
CALIB_BYTES = 1 << 30


def source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(PKG, "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    n = name.split("(")[0]
    n = re.sub(r"^void ", "", n)
    return n.replace("svr::", "")


def _find(d, pattern):
    hits = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not hits:
        raise FileNotFoundError("%s not found under %s" % (pattern, d))
    return hits[0]


def read_stats(d):
    rows = list(csv.DictReader(open(_find(d, "*kernel_stats.csv"))))
    out = {}
    for r in rows:
        out[short_name(r["Name"])] = {"calls": int(r["Calls"]),
                                      "avg_us": float(r["AverageNs"]) / 1e3,
                                      "total_ms": float(r["TotalDurationNs"]) / 1e6,
                                      "pct": float(r["Percentage"])}
    return out


def read_counter(d, counter):
    """(mean KiB per dispatch, max KiB of one dispatch) per kernel."""
    rows = list(csv.DictReader(open(_find(d, "*counter_collection.csv"))))
    acc = defaultdict(float)
    cnt = defaultdict(int)
    mx = defaultdict(float)
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        k = short_name(r["Kernel_Name"])
        v = float(r["Counter_Value"])
        acc[k] += v
        cnt[k] += 1
        mx[k] = max(mx[k], v)
    return {k: acc[k] / cnt[k] for k in acc}, dict(mx)


def read_all_counters(d):
    """{kernel: {counter: mean value per dispatch}} of one --pmc run."""
    rows = list(csv.DictReader(open(_find(d, "*counter_collection.csv"))))
    acc = defaultdict(float)
    cnt = defaultdict(int)
    for r in rows:
        key = (short_name(r["Kernel_Name"]), r["Counter_Name"])
        acc[key] += float(r["Counter_Value"])
        cnt[key] += 1
    out = defaultdict(dict)
    for (k, c), v in acc.items():
        out[k][c] = v / cnt[(k, c)]
    return dict(out)


# kernels whose counters the summary tabulates (all are kept in the JSON block)
COUNTER_TABLE = ("k_render_fwd", "k_render_bwd", "k_atomic_probe", "k_project", "k_emit",
                 "k_sort_pass", "k_sh_bwd", "k_grid_gather")


def calib_factor(per_kernel_max_kib):
    """Known bytes / counted bytes of the largest single copy dispatch (the
    1 GiB copy of bench.py --calibrate; the same kernel also serves small
    copies, so the largest dispatch is the one of known size)."""
    cands = {k: v for k, v in per_kernel_max_kib.items() if "copy" in k.lower()}
    if not cands:
        return None, None
    k = max(cands, key=cands.get)
    return k, CALIB_BYTES / (cands[k] * 1024.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--pmc", action="append", default=[])
    ap.add_argument("--out", required=True)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--title", default="rocprofv3 summary")
    args = ap.parse_args()
    stats = read_stats(args.trace)
    fetch, fetch_max = read_counter(args.fetch, "FETCH_SIZE") if args.fetch else ({}, {})
    write, write_max = read_counter(args.write, "WRITE_SIZE") if args.write else ({}, {})
    fk, ff = calib_factor(fetch_max) if fetch else (None, None)
    wk, wf = calib_factor(write_max) if write else (None, None)
    lines = ["# %s" % args.title, "", "Commands (run from the repository root on the GPU box):", ""]
    lines += ["    " + c for c in args.cmd.split(" ;; ")]
    lines += ["", "Kernel time (`--kernel-trace --stats`):", "",
              "| kernel | calls | avg µs | total ms | % |", "|---|---|---|---|---|"]
    for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["total_ms"]):
        lines.append("| %s | %d | %.1f | %.2f | %.1f |" % (k, v["calls"], v["avg_us"],
                                                         v["total_ms"], v["pct"]))
    traffic = {}
    if fetch or write:
        lines += ["", "HBM traffic per dispatch (FETCH_SIZE and WRITE_SIZE, KiB, two runs):", ""]
        if ff:
            lines.append("Calibration: the largest `%s` dispatch (the 1 GiB device copy) "
                         "gives FETCH_SIZE factor %.4f and WRITE_SIZE factor %.4f (known bytes / "
                         "counted bytes); values below are means per dispatch." % (
                             fk, ff, wf if wf else float("nan")))
        lines += ["", "| kernel | FETCH KiB | WRITE KiB | scaled MB |", "|---|---|---|---|"]
        for k in sorted(set(fetch) | set(write)):
            f = fetch.get(k, 0.0)
            w = write.get(k, 0.0)
            scaled = (f * (ff or 1.0) + w * (wf or 1.0)) * 1024.0
            traffic[k] = {"fetch_kib": f, "write_kib": w, "bytes_scaled": scaled}
            lines.append("| %s | %.0f | %.0f | %.2f |" % (k, f, w, scaled / 1e6))
    counters = defaultdict(dict)
    for d in args.pmc:
        for k, cs in read_all_counters(d).items():
            counters[k].update(cs)
    if counters:
        names = sorted({c for cs in counters.values() for c in cs})
        lines += ["", "Hardware counters per dispatch (`--pmc`, mean over dispatches; "
                  "VALUBusy and VALUUtilization in %):", ""]
        lines += ["| kernel | " + " | ".join(names) + " |",
                  "|---|" + "---|" * len(names)]
        for k in sorted(counters):
            if not k.startswith(COUNTER_TABLE):
                continue
            lines.append("| %s | " % k + " | ".join(
                ("%.4g" % counters[k][c]) if c in counters[k] else "" for c in names) + " |")
    block = {"source_hash": source_hash(), "kernels": stats, "traffic": traffic,
             "fetch_factor": ff, "write_factor": wf,
             "counters": {k: v for k, v in counters.items() if k.startswith(COUNTER_TABLE)}}
    lines += ["", "```json", json.dumps(block, sort_keys=True), "```", ""]
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    open(args.out, "w").write("\n".join(lines))
    print("wrote", args.out)


if __name__ == "__main__":
    main()
