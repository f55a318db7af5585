"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_2505_01231_amd.profile_summary \
        --trace DIR/trace_kernel_stats.csv [--kernel-trace DIR/trace_kernel_trace.csv] \
        --fetch DIR/fetch_counter_collection.csv --write DIR/write_counter_collection.csv \
        [--traffic-json OUT.json --kernel k_s3]
    python -m paper_2505_01231_amd.profile_summary --counters A_counter_collection.csv [B_...csv ...]

The counter runs must include the plain 1 GiB copy that ``bench.py
--copy-calibration`` launches first (three dispatches of torch's elementwise
kernel reading and writing 2^28 floats): ``FETCH_SIZE`` and ``WRITE_SIZE`` are
scaled by what they read for that copy of known size.  Prints a markdown table
of average duration and calibrated HBM bytes per dispatch; with
``--traffic-json`` also stores the calibrated bytes of one kernel together with
a digest of that kernel's source, which ``bench.py`` checks before it reports
the figure as ``roofline.traffic``.  With ``--counters`` it prints instead, per
kernel, the mean over dispatches of every counter or derived metric that the
given ``--pmc`` runs collected (unit utilisation, instruction counts).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_KERNEL = "vectorized_elementwise_kernel"
GIB_KIB = 1024 * 1024


def s3_source_digest() -> str:
    """sha256 over the source text of the S3 kernel and of the code that decides
    its work split, tile order and barriers; any change to them invalidates
    stored traffic counters."""
    csrc = os.path.join(HERE, "csrc")
    with open(os.path.join(csrc, "ps_moments.hip")) as f:
        src = f.read()
    with open(os.path.join(csrc, "ps_internal.h")) as f:
        inc = f.read()
    with open(os.path.join(csrc, "ps_api.cpp")) as f:
        api = f.read()
    pats = [
        (api, r"void tile_order\(.*?\n\}\n"),
        (api, r"int tile_group = \d+;"),
        (api, r"int64_t units_per_block\(.*?\n\}\n"),
        (api, r"int32_t seg_blocks\(.*?\n\}\n"),
        (inc, r"__device__ __forceinline__ void lds_barrier\(\) \{.*?\n\}\n"),
        (src, r"__device__ __forceinline__ bool resolve_block\(.*?\n\}\n"),
        (src, r"__device__ __forceinline__ bool next_item\(.*?\n\}\n"),
        (src, r"template <int FB, bool DIAG>\n__device__ __forceinline__ void s3_item\(.*?\n\}\n"),
        (src, r"template <int FB>\n__global__ __launch_bounds__\(kS3Threads, 2\) void k_s3\(BatchArgs p\) \{.*?\n\}\n"),
        (inc, r"struct Sched \{.*?\n\};\n"),
    ]
    h = hashlib.sha256()
    for text, pat in pats:
        m = re.search(pat, text, re.S)
        if not m:
            raise RuntimeError(f"source pattern not found: {pat[:40]}")
        h.update(m.group(0).encode())
    return h.hexdigest()


def _pmc(path: str) -> dict:
    agg = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            agg[r["Kernel_Name"].split("(")[0]].append(float(r["Counter_Value"]))
    return agg


def _timed_avg_us(kernel_trace: str) -> dict:
    """Per kernel: mean duration (us) of its dispatches after the first (the
    first is the warm-up step's, with cold caches)."""
    d = collections.defaultdict(list)
    with open(kernel_trace) as f:
        for r in csv.DictReader(f):
            d[r["Kernel_Name"].split("(")[0]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return {k: sum(v[1:]) / len(v[1:]) for k, v in d.items() if len(v) > 1}


def counter_table(paths: list[str]) -> tuple[list[str], dict]:
    """Mean value per (kernel, counter) over the dispatches of the given runs."""
    names: list[str] = []
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                c = r["Counter_Name"]
                if c not in names:
                    names.append(c)
                vals[r["Kernel_Name"].split("(")[0]][c].append(float(r["Counter_Value"]))
    return names, {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in vals.items()}


def summarize(trace: str, fetch: str, write: str, kernel_trace: str | None = None):
    with open(trace) as f:
        stats = list(csv.DictReader(f))
    timed = _timed_avg_us(kernel_trace) if kernel_trace else {}
    fe, wr = _pmc(fetch), _pmc(write)
    # dispatches 2..4 of the copy kernel are the three 1 GiB copies (the first is a fill)
    fcal = GIB_KIB / (sum(fe[COPY_KERNEL][1:4]) / 3)
    wcal = GIB_KIB / (sum(wr[COPY_KERNEL][1:4]) / 3)
    rows = []
    for r in stats:
        k = r["Name"].split("(")[0]
        f_, w_ = fe.get(k, []), wr.get(k, [])
        fa = sum(f_) / len(f_) if f_ else float("nan")
        wa = sum(w_) / len(w_) if w_ else float("nan")
        rows.append({"kernel": k, "calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                     "timed_us": timed.get(k, float("nan")),
                     "fetch_kib_raw": fa, "write_kib_raw": wa,
                     "read_bytes": fa * fcal * 1024, "write_bytes": wa * wcal * 1024})
    return fcal, wcal, rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--counters", nargs="+", help="*_counter_collection.csv files: print a per-kernel counter table")
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel-trace", help="the per-dispatch *_kernel_trace.csv of the trace run")
    ap.add_argument("--traffic-json")
    ap.add_argument("--kernel", default="k_s3")
    ap.add_argument("--command", default="", help="the rocprofv3 command lines, recorded in the JSON")
    a = ap.parse_args(argv)
    if a.counters:
        names, table = counter_table(a.counters)
        print("| kernel | " + " | ".join(names) + " |")
        print("|---|" + "---|" * len(names))
        for k, d in table.items():
            print(f"| {k} | " + " | ".join(f"{d[c]:.4g}" if c in d else "" for c in names) + " |")
        return
    if not (a.trace and a.fetch and a.write):
        ap.error("--trace, --fetch and --write are required without --counters")
    fcal, wcal, rows = summarize(a.trace, a.fetch, a.write, a.kernel_trace)
    print(f"calibration: FETCH_SIZE x{fcal:.3f}, WRITE_SIZE x{wcal:.3f} (1 GiB copy)\n")
    print("| kernel | calls | avg us (all) | avg us (after the first) | FETCH KiB raw | WRITE KiB raw | "
          "HBM read GB (cal.) | HBM write GB (cal.) |")
    print("|---|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['kernel']} | {r['calls']} | {r['avg_us']:.1f} | {r['timed_us']:.1f} | {r['fetch_kib_raw']:.0f} | "
              f"{r['write_kib_raw']:.0f} | {r['read_bytes'] / 1e9:.3f} | {r['write_bytes'] / 1e9:.3f} |")
    if a.traffic_json:
        r = next(x for x in rows if x["kernel"] == a.kernel)
        if a.kernel != "k_s3":
            raise SystemExit("only the S3 kernel's source digest is defined")
        out = {"kernel": a.kernel, "source_sha256": s3_source_digest(),
               "hbm_read_bytes_per_launch": r["read_bytes"], "hbm_write_bytes_per_launch": r["write_bytes"],
               "avg_launch_us_kernel_trace": r["timed_us"] if r["timed_us"] == r["timed_us"] else r["avg_us"],
               "fetch_scale": fcal, "write_scale": wcal,
               "command": a.command}
        with open(a.traffic_json, "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
