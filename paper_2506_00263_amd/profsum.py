"""Summaries of rocprofv3 runs of bench.py (kernel statistics and counters).

Reads the CSV output of rocprofv3 runs made with

    rocprofv3 --kernel-trace --stats -d <dir>/trace_<sched> -o run --output-format csv -- \
        python3 bench.py --sched <sched> --steps S --warmup 1 --no-extras --no-cpu
    rocprofv3 --pmc <counters> -d <dir>/<pass>_<sched> -o run --output-format csv -- \
        python3 bench.py --sched <sched> --steps 1 --warmup 1 --no-extras --no-cpu --copy-mib 1024

and writes, per scheduler kernel, a short markdown summary and the HBM
traffic per launch used by bench.py's roofline record.  Byte counters are
scaled by what the same counter reads for the final 1 GiB device-to-device
copy of the run (a kernel of known traffic).

The kernel-trace run's standard output (bench.py's JSON line) is kept as
<dir>/trace_<sched>/bench.json; for the stack scheduler, whose every
remapping round is a launch, the summary then lists each round of the last
run: its input population (from bench.py) and its duration (from the
trace).

Usage: python -m paper_2506_00263_amd.profsum <dir> <out_dir> [--workload NAME] [--decomp split]
           [--bench-args "..."]
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
from collections import defaultdict

from . import build

# the kernels a scheduler launches for its work (the asynchronous scheme runs
# the block-shared stash kernel for decomposed events of large runs)
KERNELS = {"naive": ("naive_kernel",), "stack": ("stack_round",), "async": ("async_kernel", "async_shared_kernel")}
PASSES = {
    "fetch": ["FETCH_SIZE"],
    "write": ["WRITE_SIZE", "TCC_HIT_sum", "TCC_MISS_sum"],
    "sq1": ["SQ_WAVES", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU",
            "SQ_THREAD_CYCLES_VALU", "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY", "GRBM_GUI_ACTIVE"],
    "sq2": ["SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_FLAT",
            "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_ACTIVE_INST_ANY"],
}
COPY_BYTES = 1 << 30
XCDS = 8           # GRBM_GUI_ACTIVE is summed over the eight XCDs
CUS = 256


def _csv(path_glob):
    files = glob.glob(path_glob, recursive=True)
    rows = []
    for f in files:
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def counters(d: str, pass_name: str, sched: str):
    """{kernel_short: {counter: per-dispatch mean}}, dispatch counts, copy values."""
    rows = _csv(os.path.join(d, f"{pass_name}_{sched}", "**", "*counter_collection.csv"))
    per = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    copy = {}
    by_dispatch = defaultdict(dict)
    for r in rows:
        name = r["Kernel_Name"]
        by_dispatch[(r["Dispatch_Id"], name)][r["Counter_Name"]] = float(r["Counter_Value"])
    for (did, name), cs in by_dispatch.items():
        short = next((v for vs in KERNELS.values() for v in vs if v in name), None)
        if short is None:
            if "copyBuffer" in name and cs.get("FETCH_SIZE", cs.get("WRITE_SIZE", 0.0)) * 1024 > COPY_BYTES / 4:
                copy = cs
            continue
        for c, v in cs.items():
            per[short][c] += v
        disp[short].add(did)
    out = {}
    for k, cs in per.items():
        n = len(disp[k])
        out[k] = {c: v / n for c, v in cs.items()}
        out[k]["_dispatches"] = n
    return out, copy


def kernel_stats(d: str, sched: str, kern: str):
    rows = _csv(os.path.join(d, f"trace_{sched}", "**", "*kernel_stats.csv"))
    for r in rows:
        if kern in r["Name"]:
            return {"calls": int(r["Calls"]), "total_ns": float(r["TotalDurationNs"]),
                    "avg_ns": float(r["AverageNs"]), "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"])}
    return None


def launch_durations(d: str, sched: str, kern: str):
    """Durations (ns) of kernel `kern`'s dispatches in start order."""
    rows = _csv(os.path.join(d, f"trace_{sched}", "**", "*kernel_trace.csv"))
    ds = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
          for r in rows if kern in r["Kernel_Name"]]
    return [dur for _, dur in sorted(ds)]


def round_table(d: str, sched: str, kern: str):
    """Per-round rows (round, input particles, duration us) of the last run
    of a stack trace, or None."""
    try:
        with open(os.path.join(d, f"trace_{sched}", "bench.json")) as fh:
            bench = json.loads(fh.read().strip().splitlines()[-1])
    except (OSError, ValueError, IndexError):
        return None
    rounds = bench.get("stack_rounds")
    n = bench.get("counters", {}).get("launches")
    durs = launch_durations(d, sched, kern)
    if not rounds or not n or len(durs) < n:
        return None
    last = durs[-n:]
    return [(r, rounds[r] if r < len(rounds) else 0, last[r] / 1e3) for r in range(n)]


def summarise(d: str, out_dir: str, workload: str, decomp: str = "fused", bench_args: str = "") -> dict:
    src = build.source_hash()
    traffic = {}
    for sched, kern in ((s, k) for s, ks in KERNELS.items() for k in ks):
        f, fcopy = counters(d, "fetch", sched)
        w, wcopy = counters(d, "write", sched)
        if kern not in f or kern not in w:
            continue
        st = kernel_stats(d, sched, kern)
        s1, _ = counters(d, "sq1", sched)
        s2, _ = counters(d, "sq2", sched)
        rf = COPY_BYTES / (fcopy["FETCH_SIZE"] * 1024) if fcopy.get("FETCH_SIZE") else None
        rw = COPY_BYTES / (wcopy["WRITE_SIZE"] * 1024) if wcopy.get("WRITE_SIZE") else None
        rd = f[kern]["FETCH_SIZE"] * 1024 * rf if rf else None
        wr = w[kern]["WRITE_SIZE"] * 1024 * rw if rw else None
        lines = [f"# {kern} — {workload}", ""]
        lines.append(f"Build source hash: `{src}`.  Commands (from the repository root):")
        lines.append("")
        lines.append("```")
        dflag = "" if decomp == "fused" else f" --decomp {decomp}"
        bflag = f" {bench_args}" if bench_args else ""
        lines.append(f"rocprofv3 --kernel-trace --stats -d <dir>/trace_{sched} -o run --output-format csv -- "
                     f"python3 bench.py --sched {sched}{dflag}{bflag} --steps 5 --warmup 1 --no-extras --no-cpu"
                     f" > <dir>/trace_{sched}/bench.json")
        for p, cs in PASSES.items():
            lines.append(f"rocprofv3 --pmc {' '.join(cs)} -d <dir>/{p}_{sched} -o run --output-format csv -- "
                         f"python3 bench.py --sched {sched}{dflag}{bflag} --steps 1 --warmup 1 --no-extras --no-cpu "
                         f"--copy-mib 1024")
        wflag = f" --workload {workload}"
        aflag = f" --bench-args '{bench_args}'" if bench_args else ""
        lines.append(f"python3 -m paper_2506_00263_amd.profsum <dir> profiles{dflag}{wflag}{aflag}")
        lines.append("```")
        lines.append("")
        if st:
            lines.append("| kernel-trace | value |")
            lines.append("|---|---|")
            lines.append(f"| dispatches | {st['calls']} |")
            lines.append(f"| average duration | {st['avg_ns'] / 1e3:.1f} us |")
            lines.append(f"| min / max | {st['min_ns'] / 1e3:.1f} / {st['max_ns'] / 1e3:.1f} us |")
            lines.append(f"| total | {st['total_ns'] / 1e6:.3f} ms |")
            lines.append("")
        lines.append("| counters (mean per dispatch) | value |")
        lines.append("|---|---|")
        lines.append(f"| dispatches per pass | {f[kern]['_dispatches']} |")
        if rf:
            lines.append(f"| FETCH_SIZE scale (1 GiB copy reads {fcopy['FETCH_SIZE']:.0f} KiB) | x{rf:.3f} |")
        if rw:
            lines.append(f"| WRITE_SIZE scale (1 GiB copy writes {wcopy['WRITE_SIZE']:.0f} KiB) | x{rw:.3f} |")
        if rd is not None:
            lines.append(f"| HBM read per dispatch (scaled) | {rd / 1e6:.2f} MB |")
        if wr is not None:
            lines.append(f"| HBM write per dispatch (scaled) | {wr / 1e6:.2f} MB |")
        lines.append(f"| L2 hit rate | {w[kern]['TCC_HIT_sum'] / max(1.0, w[kern]['TCC_HIT_sum'] + w[kern]['TCC_MISS_sum']):.3f} |")
        if kern in s1:
            a = s1[kern]
            util = a["SQ_THREAD_CYCLES_VALU"] / max(1.0, 64.0 * a["SQ_ACTIVE_INST_VALU"])
            occ = 4.0 * a["SQ_WAVE_CYCLES"] / max(1.0, a["GRBM_GUI_ACTIVE"] / XCDS) / CUS
            lines.append(f"| active lanes per VALU instruction (THREAD_CYCLES_VALU / 64 ACTIVE_INST_VALU) | {util:.3f} |")
            lines.append(f"| mean resident waves per CU (4 WAVE_CYCLES / GUI_ACTIVE per XCD / 256 CUs) | {occ:.2f} of 32 |")
            lines.append(f"| wave time waiting (WAIT_ANY / WAVE_CYCLES) | {a['SQ_WAIT_ANY'] / max(1.0, a['SQ_WAVE_CYCLES']):.3f} |")
            lines.append(f"| VALU instructions | {a['SQ_INSTS_VALU']:.4g} |")
        if kern in s2:
            b = s2[kern]
            for c in PASSES["sq2"]:
                lines.append(f"| {c} | {b[c]:.4g} |")
        lines.append("")
        rt = round_table(d, sched, kern) if sched == "stack" else None
        if rt:
            lines.append("Remapping rounds of the last run (input particles from bench.py's `stack_rounds`, "
                         "duration from the kernel trace; rounds past the last one are queued launches that "
                         "exit at once):")
            lines.append("")
            lines.append("| round | input particles | duration (us) |")
            lines.append("|---|---|---|")
            for r, n_in, us in rt:
                lines.append(f"| {r} | {n_in} | {us:.1f} |")
            tot = sum(us for _, _, us in rt)
            big = sum(us for _, n_in, us in rt if n_in >= 100_000)
            lines.append("")
            lines.append(f"Total {tot:.1f} us over {len(rt)} launches; rounds with at least 1e5 input particles "
                         f"{big:.1f} us, the rest {tot - big:.1f} us.")
            lines.append("")
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, f"{kern}_{workload.replace(' ', '_')}.md"), "w") as fh:
            fh.write("\n".join(lines))
        if rd is not None and wr is not None:
            traffic[kern] = {"bytes_per_launch": rd + wr, "read": rd, "write": wr, "source_hash": src,
                             "workload": workload, "read_scale": rf, "write_scale": rw}
    # the default (fused lattice) figures are the ones bench.py reports
    tname = {"lattice_1e6": "traffic.json", "lattice_1e6_split": "traffic_split.json"}.get(
        workload, f"traffic_{workload}.json")
    with open(os.path.join(out_dir, tname), "w") as fh:
        json.dump(traffic, fh, indent=1, sort_keys=True)
    return traffic


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("out")
    ap.add_argument("--workload", default=None)
    ap.add_argument("--decomp", default="fused", choices=["fused", "split"])
    ap.add_argument("--bench-args", default="", help="extra bench.py arguments the profiled runs used")
    a = ap.parse_args()
    wl = a.workload or ("lattice_1e6" if a.decomp == "fused" else f"lattice_1e6_{a.decomp}")
    print(json.dumps(summarise(a.dir, a.out, wl, a.decomp, a.bench_args), indent=1))


if __name__ == "__main__":
    main()
