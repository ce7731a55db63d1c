"""HBM bytes per kernel launch from two rocprofv3 counter passes.

    rocprofv3 --pmc FETCH_SIZE ... -f csv -d F -o run -- python3 bench.py ... --calib-copy-mb M
    rocprofv3 --pmc WRITE_SIZE ... -f csv -d W -o run -- python3 bench.py ... --calib-copy-mb M
    python -m paper_1811_07717_amd.counters --fetch F/run_counter_collection.csv \
        --write W/run_counter_collection.csv --copy-mib 2048 --workload sphere2mm_L128 \
        --bench bench.json --update profiles/traffic.json --md profiles/x.md

Both counters report KiB per dispatch.  Each is calibrated on the library's
plain copy (zi_copy_probe, kernel k_copy2) recorded in the same pass, whose
true traffic is known (copy_mib read and copy_mib written per launch):
factor = true KiB / counted KiB.  The solver kernels' calibrated bytes per
launch go to traffic.json together with a hash of the kernel sources, so
that bench.py reports them only while the kernels are unchanged.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1811_07717_amd/csrc/k_pcg.hip",
                  "paper_1811_07717_amd/csrc/k_assemble.hip"]

# rocprofv3 kernel name -> solver kernel key used by bench.py
KERNELS = [(re.compile(r"k_spmm<.*, true>"), "spmm_pq"),
           (re.compile(r"k_spmm_sr<|k_spmm_ring<double, true>"), "spmm_sr"),
           (re.compile(r"k_spmm_ring<.*, false>"), "spmm_pq"),
           (re.compile(r"k_update<"), "update"),
           (re.compile(r"k_pupdate<"), "pupdate"),
           (re.compile(r"k_xflush<"), "xflush"),
           (re.compile(r"k_pflush<"), "pflush"),
           (re.compile(r"k_copy2"), "copy")]


def source_hash():
    """Hash of the sources that define the solver kernels and the row order."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def per_kernel(path, spmm_args=None):
    """Mean counter value (KiB) and launch count per solver kernel key.
    spmm_args ("16, 2"): count only SpMM launches of that tile (the run's
    tuned tile; the autotuner's launches of other tiles are left out)."""
    vals = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"]
            for pat, key in KERNELS:
                if pat.search(name):
                    if (spmm_args and key.startswith("spmm")
                            and (f"<{spmm_args}" if spmm_args != "ring" else "k_spmm_ring<")
                            not in name):
                        break
                    vals[key].append(float(r["Counter_Value"]))
                    break
    return {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}


def summarize(fetch_csv, write_csv, copy_mib, spmm_args=None):
    fe, wr = per_kernel(fetch_csv, spmm_args), per_kernel(write_csv, spmm_args)
    if "copy" not in fe or "copy" not in wr:
        raise SystemExit("no k_copy2 launch in the counter files (run bench.py --calib-copy-mb)")
    true_kib = copy_mib * 1024.0
    ff, wf = true_kib / fe["copy"][0], true_kib / wr["copy"][0]
    out = {}
    for k in fe:
        if k == "copy" or k not in wr:
            continue
        fk, wk = fe[k][0], wr[k][0]
        # the solver's SpMM runs as several slab launches per product (one
        # residual update per product): bytes per product = slabs x per launch
        slabs = 1
        if k.startswith("spmm") and "update" in fe:
            slabs = max(1, round(fe[k][1] / fe["update"][1]))
        out[k] = dict(fetch_kib=round(fk, 1), write_kib=round(wk, 1),
                      bytes_per_launch=int(round((fk * ff + wk * wf) * 1024 * slabs)),
                      launches=fe[k][1], slabs=slabs)
    return out, ff, wf


def phase_gaps(trace_csv, marker="k_copy2"):
    """Busy and idle time of the GPU in a rocprofv3 kernel trace, cut into
    phases at the dispatches of `marker`: per phase the span from the first
    kernel's start to the last kernel's end, the time some kernel runs (the
    union of the kernels' intervals on all queues), the rest (idle), the
    dispatch count and the longest idle stretches (microseconds)."""
    rows = []
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    phases, cur = [], []
    for s, e, name in rows:
        if marker in name:
            phases.append(cur)
            cur = []
        else:
            cur.append((s, e))
    phases.append(cur)
    out = []
    for ph in phases:
        if not ph:
            out.append(None)
            continue
        busy, gaps, lo, hi = 0, [], ph[0][0], ph[0][1]
        for s, e in ph[1:]:
            if s > hi:
                busy += hi - lo
                gaps.append(s - hi)
                lo, hi = s, e
            else:
                hi = max(hi, e)
        busy += hi - lo
        span = max(e for _, e in ph) - ph[0][0]
        gaps.sort(reverse=True)
        out.append(dict(span_us=span / 1e3, busy_us=busy / 1e3, idle_us=(span - busy) / 1e3,
                        dispatches=len(ph), gaps_over_50us=sum(g > 50e3 for g in gaps),
                        longest_gaps_us=[round(g / 1e3, 1) for g in gaps[:5]]))
    return out


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    if "--gaps" in sys.argv:   # phase busy/idle table of a kernel trace
        g = argparse.ArgumentParser()
        g.add_argument("--gaps", required=True, help="rocprofv3 run_kernel_trace.csv")
        g.add_argument("--marker", default="k_copy2")
        ga = g.parse_args()
        print(json.dumps(phase_gaps(ga.gaps, ga.marker), indent=1))
        return
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--copy-mib", type=float, required=True,
                   help="MiB read (and written) by each calibration copy launch")
    p.add_argument("--workload", required=True)
    p.add_argument("--bench", help="bench.py JSON line (for the algorithmic bytes)")
    p.add_argument("--update", help="traffic.json to update")
    p.add_argument("--md", help="write a markdown table here")
    p.add_argument("--command", default="", help="command line to record in the table")
    a = p.parse_args()
    alg, spmm_args, tuned = {}, None, None
    if a.bench:
        with open(a.bench) as f:
            line = [ln for ln in f.read().splitlines() if ln.startswith("{")][-1]
        b = json.loads(line)
        alg = {k: v["bytes_per_launch"] for k, v in b["solver_kernels"].items()}
        tuned = (b.get("autotune") or {}).get("tile") or b.get("config", {}).get("tile_name")
        if not tuned and isinstance(b.get("config", {}).get("tile"), int):
            from paper_1811_07717_amd import zi
            tuned = zi.tile_names()[b["config"]["tile"]]
        m = re.match(r"lpr(\d+)_nv(\d+)_", tuned or "")
        if m:
            spmm_args = f"{m.group(1)}, {m.group(2)}"
        elif (tuned or "").startswith("ring"):
            spmm_args = "ring"
    res, ff, wf = summarize(a.fetch, a.write, a.copy_mib, spmm_args)
    h = source_hash()
    if a.update:
        d = {}
        if os.path.exists(a.update):
            with open(a.update) as f:
                d = json.load(f)
        w = d.setdefault(a.workload, {})
        for k, v in res.items():
            # the SpMM's traffic depends on its tile: one entry per tile
            key = f"{k}@{tuned}" if (k.startswith("spmm") and tuned) else k
            w[key] = dict(v, source_hash=h, fetch_factor=round(ff, 4), write_factor=round(wf, 4))
        with open(a.update, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
            f.write("\n")
    rows = ["| kernel | dispatches | launches per product | FETCH_SIZE KiB per dispatch | "
            "WRITE_SIZE KiB per dispatch | HBM bytes per product (calibrated) | "
            "algorithmic bytes | ratio |", "|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(res.items()):
        ab = alg.get(k)
        ratio = f"{v['bytes_per_launch'] / ab:.3f}" if ab else "-"
        rows.append(f"| {k} | {v['launches']} | {v['slabs']} | {v['fetch_kib']:.1f} | "
                    f"{v['write_kib']:.1f} | {v['bytes_per_launch']:,} | "
                    + (f"{ab:,} | {ratio} |" if ab else "- | - |"))
    text = "\n".join(rows) + (f"\n\nCalibration on k_copy2 ({a.copy_mib:g} MiB read + written per "
                              f"launch): FETCH_SIZE factor {ff:.4f}, WRITE_SIZE factor {wf:.4f}. "
                              f"Kernel source hash {h}.\n")
    if a.md:
        with open(a.md, "w") as f:
            if a.command:
                f.write(a.command.strip() + "\n\n")
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
