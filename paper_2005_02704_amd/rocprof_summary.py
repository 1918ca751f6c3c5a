"""Condense rocprofv3 CSV output of a bench.py run into the text summaries kept
in profiles/ (and the traffic JSON bench.py reads).

Usage:
  python -m paper_2005_02704_amd.rocprof_summary --trace DIR [--fetch DIR --write DIR]
         --command "the rocprofv3 command" --out profiles/NAME.txt [--traffic-json FILE]
  python -m paper_2005_02704_amd.rocprof_summary --sq DIR [DIR ...]
         --command "the rocprofv3 commands" --out profiles/NAME.txt

--sq takes the output folders of --pmc runs of SQ counters (any counters, one
value per dispatch) and writes their average per dispatch by kernel, with the
busy ratios and per-wave counts that follow from them.

The profiled run launches only the batched chain (bench.py --forms graph).
HBM bytes are FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the
same counters read for the plain device copy bench.py --copy-calibration runs
(the largest copy dispatch of the run).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kname(s: str) -> str:
    m = re.search(r"::(k_\w+)<", s)
    if m:
        return m.group(1)
    return s.split("(")[0][:48]


def _csv(d: str, suffix: str):
    files = glob.glob(os.path.join(d, f"*{suffix}"))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def kernel_source_hash():
    """Hash of the kernels' code (the same as bench.py's): comments and blank
    space left out, so that an edit of a comment keeps the counters valid."""
    import re
    h = hashlib.sha256()
    for name in ("lidarseg_kernels.hip", "lidarseg_internal.h"):
        with open(os.path.join(ROOT, "paper_2005_02704_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def trace_summary(d: str):
    """Durations by kernel.  The profiled run launches only the batched chain
    (bench.py --forms graph), so every dispatch of a library kernel is batched."""
    rows = _csv(d, "kernel_trace.csv")
    by = collections.defaultdict(list)
    for r in rows:
        by[kname(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return by


def counter_summary(d: str):
    rows = _csv(d, "counter_collection.csv")
    by = collections.defaultdict(list)
    copies = []
    for r in rows:
        name = kname(r["Kernel_Name"])
        v = float(r["Counter_Value"])
        if "copyBuffer" in name:
            copies.append((int(r["Grid_Size"]), v))
        elif name.startswith("k_"):
            by[name].append(v)
    # the calibration copy is the largest copy dispatch (the others stage inputs)
    gmax = max(g for g, _ in copies)
    return by, [v for g, v in copies if g == gmax]


def sq_summary(dirs):
    """Average per dispatch of every counter, by library kernel."""
    tot = collections.defaultdict(lambda: collections.defaultdict(float))
    cnt = collections.defaultdict(collections.Counter)
    for d in dirs:
        for r in _csv(d, "counter_collection.csv"):
            k = kname(r["Kernel_Name"])
            if not k.startswith("k_"):
                continue
            tot[k][r["Counter_Name"]] += float(r["Counter_Value"])
            cnt[k][r["Counter_Name"]] += 1
    return {k: {c: v / cnt[k][c] for c, v in d.items()} for k, d in tot.items()}


# (label, numerator, denominator).  SQ_ACTIVE_INST_* count quad-cycles summed
# over the SIMDs, SQ_BUSY_CU_CYCLES cycles summed over the compute units: with
# four SIMDs per compute unit the busy ratios are the fraction of a busy
# compute unit's cycles in which one SIMD issues that kind of instruction.
SQ_RATIOS = [
    ("VALU busy", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CU_CYCLES"),
    ("scalar busy", "SQ_ACTIVE_INST_SCA", "SQ_BUSY_CU_CYCLES"),
    ("LDS busy", "SQ_ACTIVE_INST_LDS", "SQ_BUSY_CU_CYCLES"),
    ("VALU instructions per wave", "SQ_INSTS_VALU", "SQ_WAVES"),
    ("scalar instructions per wave", "SQ_INSTS_SALU", "SQ_WAVES"),
    ("LDS instructions per wave", "SQ_INSTS_LDS", "SQ_WAVES"),
    ("vector memory reads per wave", "SQ_INSTS_VMEM_RD", "SQ_WAVES"),
    ("vector memory writes per wave", "SQ_INSTS_VMEM_WR", "SQ_WAVES"),
    ("wave cycles waiting on a dependency", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES"),
    ("wave cycles waiting (any)", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES"),
]


def sq_lines(by):
    out = []
    kernels = sorted(by, key=lambda k: -by[k].get("SQ_BUSY_CU_CYCLES", 0.0))
    counters = sorted({c for d in by.values() for c in d})
    out.append("counter (average per dispatch)   " + " ".join(f"{k:>13}" for k in kernels))
    for c in counters:
        out.append(f"{c:<32} " + " ".join(f"{by[k].get(c, float('nan')):13.4g}" for k in kernels))
    out += ["", "ratio (numerator / denominator)  " + " ".join(f"{k:>13}" for k in kernels)]
    for label, num, den in SQ_RATIOS:
        if not any(num in by[k] and by[k].get(den) for k in kernels):
            continue
        vals = [by[k][num] / by[k][den] if num in by[k] and by[k].get(den) else float("nan") for k in kernels]
        out.append(f"{label:<32} " + " ".join(f"{v:13.4g}" for v in vals) + f"   [{num} / {den}]")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace")
    ap.add_argument("--sq", nargs="+", help="output folders of --pmc runs of SQ counters")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--command", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic-json")
    ap.add_argument("--kernel", default="k_geom")
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--alg-bytes", type=float, default=0.0,
                    help="algorithmic bytes per launch of --kernel (from bench.py's roofline)")
    a = ap.parse_args()
    if a.sq:
        lines = ["# rocprofv3 SQ counters of the batched chain, bench.py workload",
                 f"kernel source hash: {kernel_source_hash()}", f"command: {a.command}", ""]
        lines += sq_lines(sq_summary(a.sq))
        with open(a.out, "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    if not a.trace:
        ap.error("--trace or --sq is required")
    lines = [f"# rocprofv3 summary: {a.kernel} and the rest of the chain, bench.py workload",
             f"command: {a.command}", ""]
    tr = trace_summary(a.trace)
    lines.append("kernel            calls   avg_us    min_us    total_us")
    for k, v in sorted(tr.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{k:<17} {len(v):6d} {sum(v) / len(v) / 1e3:9.2f} {min(v) / 1e3:9.2f} {sum(v) / 1e3:11.1f}")
    traffic = None
    if a.fetch and a.write:
        fb, fcopy = counter_summary(a.fetch)
        wb, wcopy = counter_summary(a.write)
        copy_kib = a.copy_mib * 1024.0
        f_scale = copy_kib / (sum(fcopy) / len(fcopy))
        w_scale = copy_kib / (sum(wcopy) / len(wcopy))
        lines += ["", f"calibration: {a.copy_mib} MiB device copy reads FETCH_SIZE "
                      f"{sum(fcopy) / len(fcopy):.1f} KiB, WRITE_SIZE {sum(wcopy) / len(wcopy):.1f} KiB "
                      f"-> scale fetch x{f_scale:.3f}, write x{w_scale:.3f}",
                  "kernel            fetch_MB  write_MB  hbm_MB (scaled, per dispatch)"]
        for k in sorted(fb, key=lambda k: -sum(fb[k]) / len(fb[k])):
            fm = sum(fb[k]) / len(fb[k]) * f_scale * 1024 / 1e6
            wm = sum(wb.get(k, [0])) / max(1, len(wb.get(k, [0]))) * w_scale * 1024 / 1e6
            lines.append(f"{k:<17} {fm:9.1f} {wm:9.1f} {fm + wm:9.1f}")
            if k == a.kernel:
                traffic = (fm + wm) * 1e6
        if a.kernel in tr and traffic is not None:
            v = tr[a.kernel]
            avg_s = sum(v) / len(v) / 1e9
            lines += ["", f"{a.kernel}: avg {avg_s * 1e6:.2f} us, HBM traffic {traffic / 1e6:.1f} MB "
                          f"-> {traffic / avg_s / 1e9:.1f} GB/s"]
            if a.alg_bytes:
                lines.append(f"algorithmic bytes {a.alg_bytes / 1e6:.1f} MB -> "
                             f"{a.alg_bytes / avg_s / 1e9:.1f} GB/s ({a.alg_bytes / avg_s / 8e12:.3f} of 8 TB/s)")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    if a.traffic_json and traffic is not None:
        with open(a.traffic_json, "w") as f:
            json.dump({"kernel": a.kernel, "hbm_bytes_per_launch": round(traffic),
                       "kernel_source_hash": kernel_source_hash(), "frames": a.frames, "seed": a.seed,
                       "command": a.command}, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
