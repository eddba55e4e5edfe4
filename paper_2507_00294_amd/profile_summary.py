"""Summaries of rocprofv3 output for the measurement records.

    python -m paper_2507_00294_amd.profile_summary trace <dir> <out.md> "<command>"
        Per-kernel launch counts and durations from a --kernel-trace --stats run
        (the *_kernel_stats.csv files under <dir>), full kernel names.

    python -m paper_2507_00294_amd.profile_summary counters <out.md> <record.txt> \
        <bench.json> <trace_dir> <copy_fetch_dir> <copy_write_dir> <pass_dir> [<pass_dir> ...]
        Per-dispatch counter averages of the arrival query's kernels from
        --pmc passes, HBM bytes calibrated by a plain device copy of 1 GiB,
        VALU instructions and FLOPs per causal pair of the far kernels, and
        the record bench.py reads (valid while the device sources hash to the
        recorded value).

    python -m paper_2507_00294_amd.profile_summary visits <out.md> <trace_dir> "<command>" \
        <n_visits> <pass_dir> [<pass_dir> ...]
        Counters of the general visit list's kernels (arrival and final map of
        one list of n_visits visits with the map at n_visits pixels), taken
        from each kernel's largest dispatch (the list's own; the bench's
        many-list leg launches the same kernels with small grids).

FLOPs are counted from the instruction counters as the FLOP counters count
them: 2 per FMA, 1 per add, multiply or transcendental, per lane.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEVICE_SOURCES = ("dd_device.h", "dd_internal.h", "dd_items.h", "dd_kernels.hip", "dd_queries.cpp",
                  "dd_host.cpp")
FAR32 = "k_arrival_far32<4, 0>"
FAR64 = "k_arrival_far64<2, 0>"
COPY_BYTES = 1 << 30


def device_source_hash() -> str:
    h = hashlib.sha256()
    for name in DEVICE_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_00294_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def demangle(name: str) -> str:
    """A name the profiler left mangled, through c++filt; BF16 (DF16b, which
    c++filt does not know) is spelt as the vendor type __bf16 first."""
    import subprocess

    try:
        out = subprocess.run(["c++filt", name.replace("DF16b", "u6__bf16")],
                             capture_output=True, text=True, timeout=10).stdout.strip()
        return out or name
    except (OSError, subprocess.SubprocessError):
        return name


def short_name(name: str) -> str:
    """Kernel name without its parameter list (the last balanced (...) at the
    end), keeping '(anonymous namespace)' and template arguments."""
    name = name.strip()
    if name.startswith("_Z"):
        name = demangle(name)
    if name.endswith(")"):
        depth = 0
        for i in range(len(name) - 1, -1, -1):
            if name[i] == ")":
                depth += 1
            elif name[i] == "(":
                depth -= 1
                if depth == 0:
                    name = name[:i]
                    break
    name = re.sub(r"^void ", "", name)
    return name.replace("(anonymous namespace)::", "")


def _csvs(d: str, suffix: str):
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def kernel_stats(d: str):
    rows = []
    for path in _csvs(d, "kernel_stats.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.append({"name": short_name(r["Name"]), "calls": int(r["Calls"]),
                             "avg_us": float(r["AverageNs"]) / 1e3,
                             "min_us": float(r["MinNs"]) / 1e3, "max_us": float(r["MaxNs"]) / 1e3,
                             "total_us": float(r["TotalDurationNs"]) / 1e3})
    return rows


def counter_means(d: str):
    """{kernel: {counter: mean per dispatch}} over every dispatch in <d>."""
    acc = defaultdict(lambda: defaultdict(dict))  # kernel -> counter -> dispatch -> value
    for path in _csvs(d, "counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                k = short_name(r["Kernel_Name"])
                c = r["Counter_Name"]
                did = (path, r.get("Dispatch_Id", r.get("Correlation_Id")))
                acc[k][c][did] = acc[k][c].get(did, 0.0) + float(r["Counter_Value"])
    return {k: {c: sum(v.values()) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


def write_trace(d: str, out: str, command: str):
    rows = sorted(kernel_stats(d), key=lambda r: -r["total_us"])
    total = sum(r["total_us"] for r in rows) or 1.0
    lines = ["# Kernel trace: " + os.path.basename(out).rsplit(".", 1)[0], "",
             "Command (rocprofv3 on MI355X):", "", "    " + command, "",
             "Durations in microseconds per launch (rocprofv3 --stats).", "",
             "| Kernel | Calls | Average us | Min us | Max us | Share |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['name']}` | {r['calls']} | {r['avg_us']:.1f} | {r['min_us']:.1f} | "
                     f"{r['max_us']:.1f} | {100 * r['total_us'] / total:.1f}% |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _find(means, key):
    for k, v in means.items():
        if k.endswith(key) or k == key:
            return v
    return None


def write_counters(out_md, record, bench_json, trace_dir, fetch_dir, write_dir, passes):
    with open(bench_json) as f:
        line = json.loads(f.read().strip().splitlines()[-1])
    pairs = {FAR32: line["roofline"]["pairs_per_launch"],
             FAR64: line["other_precision"]["roofline"]["pairs_per_launch"]}
    merged = defaultdict(dict)
    for d in passes:
        for k, cs in counter_means(d).items():
            merged[k].update(cs)
    fetch = _find(counter_means(fetch_dir), "copyBuffer")["FETCH_SIZE"]
    write = _find(counter_means(write_dir), "copyBuffer")["WRITE_SIZE"]
    f_fac = COPY_BYTES / (fetch * 1024.0)
    w_fac = COPY_BYTES / (write * 1024.0)
    trace = {r["name"]: r for r in kernel_stats(trace_dir)}

    def resolve(d, key):  # full name of the kernel `key` in d (names carry the namespace)
        return next((n for n in d if n == key or n.endswith("::" + key)), None)

    def per_pair(k, c):
        return 64.0 * cs.get(c, 0.0) / pairs[k]

    rec = {"source_sha256": device_source_hash()}
    derived = []
    for k, tag in ((FAR32, ""), (FAR64, "fp64_")):
        name = resolve(merged, k)
        if name is None:
            continue
        cs = merged[name]
        f32 = 2 * cs.get("SQ_INSTS_VALU_FMA_F32", 0) + cs.get("SQ_INSTS_VALU_MUL_F32", 0) + \
            cs.get("SQ_INSTS_VALU_ADD_F32", 0) + cs.get("SQ_INSTS_VALU_TRANS_F32", 0)
        f64 = 2 * cs.get("SQ_INSTS_VALU_FMA_F64", 0) + cs.get("SQ_INSTS_VALU_MUL_F64", 0) + \
            cs.get("SQ_INSTS_VALU_ADD_F64", 0) + cs.get("SQ_INSTS_VALU_TRANS_F64", 0)
        flops_pair = 64.0 * (f32 + f64) / pairs[k]
        ipp = per_pair(k, "SQ_INSTS_VALU")
        rec[tag + "valu_lane_instructions_per_pair"] = f"{ipp:.4f}"
        rec[tag + "flops_per_pair"] = f"{flops_pair:.4f}"
        if not tag:
            rec["valu_transcendental_per_pair"] = f"{per_pair(k, 'SQ_INSTS_VALU_TRANS_F32'):.4f}"
            rec["fetch_bytes"] = f"{cs.get('FETCH_SIZE', 0) * 1024 * f_fac:.6e}"
            rec["write_bytes"] = f"{cs.get('WRITE_SIZE', 0) * 1024 * w_fac:.6e}"
        tn = resolve(trace, k)
        t = trace[tn] if tn else None
        if t:
            rec[tag + "rocprof_avg_launch_ms"] = f"{t['avg_us'] / 1e3:.4f}"
            peak = 157.3e12 if not tag else 78.6e12
            derived.append(
                f"* `{k}`: {pairs[k]:.4e} causal pairs per launch; {ipp:.2f} VALU lane-instructions "
                f"and {flops_pair:.2f} FLOPs per pair (FP32 {64 * f32 / pairs[k]:.2f}, FP64 "
                f"{64 * f64 / pairs[k]:.2f}); rocprof average {t['avg_us'] / 1e3:.3f} ms per launch "
                f"-> {flops_pair * pairs[k] / (t['avg_us'] * 1e-6) / 1e12:.2f} TFLOP/s = "
                f"{flops_pair * pairs[k] / (t['avg_us'] * 1e-6) / peak:.4f} of "
                f"{peak / 1e12:.1f} TFLOP/s; issue {ipp * pairs[k] / (t['avg_us'] * 1e-6):.3e} "
                f"lane-instructions/s = "
                f"{ipp * pairs[k] / (t['avg_us'] * 1e-6) / (256 * 64 * 2.4e9):.3f} of 3.93e13/s.")
    with open(record, "w") as f:
        f.write("# Counter record of the far kernels on the 512x512 random-scan arrival query,\n"
                "# written by paper_2507_00294_amd/profile_summary.py from the passes in\n"
                "# k_arrival_far_512x512_random_counters.md; bench.py uses it only while the\n"
                "# device sources hash to source_sha256.\n")
        for k, v in rec.items():
            f.write(f"{k} = {v}\n")
    cols = sorted({c for cs in merged.values() for c in cs})
    lines = ["# Counters: arrival query of the 512x512 random scan (mixed and FP64)", "",
             "Each pass is its own run (rocprofv3 does not split counters over passes); values "
             "are per dispatch, averaged over the profiled dispatches of each kernel.", "",
             f"Copy calibration (1 GiB device copy): FETCH_SIZE {fetch:.0f} KiB -> bytes = KiB x "
             f"1024 x {f_fac:.3f}; WRITE_SIZE {write:.0f} KiB -> x {w_fac:.3f}.", "",
             "| Kernel | " + " | ".join(c.replace("SQ_INSTS_", "") for c in cols) + " |",
             "|---|" + "---|" * len(cols)]
    for k in sorted(merged):
        lines.append(f"| `{k}` | " + " | ".join(f"{merged[k].get(c, float('nan')):.4g}"
                                              for c in cols) + " |")
    lines += ["", "Derived:", ""] + derived
    if "fetch_bytes" in rec:
        lines.append(f"* HBM bytes per launch of `{FAR32}`: read {float(rec['fetch_bytes']):.3e}, "
                     f"written {float(rec['write_bytes']):.3e} (calibrated).")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def counter_max(d: str):
    """{kernel: {counter: largest per-dispatch value}} over the dispatches in <d>."""
    acc = defaultdict(lambda: defaultdict(dict))
    for path in _csvs(d, "counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                k = short_name(r["Kernel_Name"])
                did = (path, r.get("Dispatch_Id", r.get("Correlation_Id")))
                c = acc[k][r["Counter_Name"]]
                c[did] = c.get(did, 0.0) + float(r["Counter_Value"])
    return {k: {c: max(v.values()) for c, v in cs.items()} for k, cs in acc.items()}


def write_visits(out_md, trace_dir, command, n_visits, passes):
    n = int(n_visits)
    pairs = {"arrival": n * (n - 1) / 2.0, "map": float(n) * n}
    merged = defaultdict(dict)
    for d in passes:
        for k, cs in counter_max(d).items():
            merged[k].update(cs)
    trace = {r["name"]: r for r in kernel_stats(trace_dir)}
    lines = [f"# Counters: general visit list of {n} visits (arrival and final map)", "",
             "Commands (each counter pass and the trace its own run):", "",
             "    " + command, "",
             "Values are those of each kernel's largest dispatch (the list's own call; the "
             "many-list leg of the same run launches the same kernels with small grids); the "
             "duration is the trace's longest launch of the kernel.", "",
             "| Kernel | pairs | ms | pair-terms/s | VALU / pair | FMA64 / pair | FMA32 / pair | "
             "CVT / pair | TRANS32 / pair | SALU / wave-step | LDS / wave-step | issue / 3.93e13 |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k in sorted(merged):
        if "k_visit_arrival" not in k and "k_visit_map" not in k:
            continue
        cs = merged[k]
        p = pairs["map" if "k_visit_map" in k else "arrival"]
        t = trace.get(k)
        ms = t["max_us"] / 1e3 if t else float("nan")

        def per(c):
            return 64.0 * cs.get(c, 0.0) / p
        issue = 64.0 * cs.get("SQ_INSTS_VALU", 0.0) / (ms * 1e-3) / (256 * 64 * 2.4e9)
        lines.append(f"| `{k}` | {p:.4e} | {ms:.3f} | {p / (ms * 1e-3):.3e} | "
                     f"{per('SQ_INSTS_VALU'):.1f} | {per('SQ_INSTS_VALU_FMA_F64'):.1f} | "
                     f"{per('SQ_INSTS_VALU_FMA_F32'):.1f} | {per('SQ_INSTS_VALU_CVT'):.1f} | "
                     f"{per('SQ_INSTS_VALU_TRANS_F32'):.2f} | {per('SQ_INSTS_SALU'):.1f} | "
                     f"{per('SQ_INSTS_LDS'):.2f} | {issue:.3f} |")
    lines += ["", "Per pair: lane-instructions per causal pair (counter x 64 / pairs). Per "
              "wave-step: wave instructions per 64 pairs. The issue rate is VALU lane-instructions "
              "per second against one per lane per clock on 256 CUs at 2.4 GHz."]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv):
    if len(argv) >= 4 and argv[0] == "trace":
        write_trace(argv[1], argv[2], argv[3])
    elif len(argv) >= 8 and argv[0] == "counters":
        write_counters(argv[1], argv[2], argv[3], argv[4], argv[5], argv[6], argv[7:])
    elif len(argv) >= 6 and argv[0] == "visits":
        write_visits(argv[1], argv[2], argv[3], argv[4], argv[5:])
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
