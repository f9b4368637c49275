"""Benchmark: particle histories per second on one MI355X.

Workload: the multigroup pin lattice (17x17 pins, 7 materials x 7 groups,
reflective box, uniform source, 51x51x20x7 mesh tally), 1e6 histories.
One step = one forward transport run of all histories through the selected
thread-data-remapping scheduler, with inputs resident in HBM.  Also
reported: the other schedulers (naive one-lane-per-history baseline, stack,
async; fused and split events), the score-function backward/forward time
ratio, the batched 256-problem launch, the roofline of the dominant kernel
and the CPU oracle timed on the host cores over the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sched async|stack|naive] [--decomp fused|split]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
N_HIST = 1_000_000
NEUTRON_SPEED = 1.383e6        # cm/s per sqrt(eV)


def algorithmic_bytes(c: dict, d: dict | None = None, lookup: str = "hash") -> float:
    """Bytes the method itself must touch over a run with counters `c`: one
    int64 tally update per scored piece (8 B); multigroup: Sigma_t per flight,
    Sigma_s per collision and every transfer-CDF entry a scatter reads (8 B
    each); continuous energy: one cross-section lookup per flight
    (ce_lookup_bytes)."""
    if d is not None and int(d.get("energy_mode", 0)) == 1:
        return 8.0 * c["pieces"] + c["flights"] * ce_lookup_bytes(d, lookup)
    return 8.0 * (c["pieces"] + c["flights"] + c["collisions"] + c["cdf_scans"])


def ce_lookup_bytes(d: dict, lookup: str) -> float:
    """Table bytes of one continuous-energy lookup, per species: the bracket
    search (binary: ceil(log2(n-1)) probes of 8 B over the whole grid; hashed:
    the 8-byte bin entry plus ceil(log2 width) probes, averaged over the hash
    bins as the library builds them) and 48 B of interpolation (E, sigma_a,
    sigma_s at both ends of the bracket)."""
    S, n = int(d["n_species"]), int(d["grid_len"])
    if lookup == "binary":
        return S * (8.0 * math.ceil(math.log2(n - 1)) + 48.0)
    g = np.asarray(d["e_grid"], np.float64).reshape(S, n)
    M = int(d.get("hash_bins", 0) or 0) or max(64, n // 8)
    lo, hi = math.log(g[:, 0].min()), math.log(g[:, -1].max())
    inv = M / (hi - lo)
    b = np.arange(M, dtype=np.float64)
    e0, e1 = np.exp(lo + b / inv), np.exp(lo + (b + 1) / inv)
    per = 0.0
    for s in range(S):
        lo_i = np.maximum(np.clip(np.searchsorted(g[s], e0, side="right") - 1, 0, n - 2) - 1, 0)
        hi_i = np.minimum(np.clip(np.searchsorted(g[s], e1, side="right") - 1, 0, n - 2) + 2, n - 1)
        probes = np.ceil(np.log2(np.maximum(hi_i - lo_i, 1)))
        per += 8.0 + 8.0 * float(probes.mean()) + 48.0
    return per


def backward_bytes(c: dict, n_hist: int) -> float:
    """Algorithmic bytes of the two replays of the score-function backward,
    from the forward's counters of the same histories: pass A gathers dL/dT
    per tally piece and writes G_h; both passes read Sigma_t per flight,
    Sigma_s per collision and the CDF entries a scatter reads; pass B reads
    G_h (the three per-(material, group) sums stay on chip)."""
    replay = 8.0 * (c["flights"] + c["collisions"] + c["cdf_scans"])
    return 8.0 * c["pieces"] + 2.0 * replay + 16.0 * n_hist


def roofline_block(bytes_per_launch: float, mean_launch_ms: float, kernel: str, traffic=None, **extra) -> dict:
    achieved = bytes_per_launch / (mean_launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "mean_launch_ms": mean_launch_ms, "bytes_per_launch": bytes_per_launch, **extra}


def main_launches(c: dict, sched: str) -> int:
    """Launches of the scheduler's main kernel in one run (the stack scheme
    launches one per remapping round; the others one)."""
    return int(c["rounds"]) if sched == "stack" else 1


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/traffic.json), or None if those counters were taken
    from a different build of the device code."""
    from paper_2506_00263_amd import build
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            rec = json.load(f).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != build.source_hash():
        return None
    return rec["bytes_per_launch"]


def timed_runs(P, reps, **kw):
    """Wall times of `reps` runs (no per-launch events: they cost host time
    between the stack scheduler's launches), then the kernel time of one
    more run timed with HIP events."""
    import torch
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.run(**kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    P.run(time_kernels=True, **kw)
    return times, [P.counters()["kernel_ms"]]


def _wall(P, reps, **kw):
    ts, _ = timed_runs(P, reps + 1, **kw)
    return float(np.median(ts[1:]))


def _kernel_ms(P, reps, **kw) -> float:
    ks = []
    for _ in range(reps):
        P.run(time_kernels=True, **kw)
        ks.append(P.counters()["kernel_ms"])
    return float(np.median(ks))


def latency_block(P, n_hist: int) -> dict:
    """Where the asynchronous kernel's time goes on the lattice (default
    knobs): its kernel time against the number of histories (the slope over
    the two largest runs is the marginal cost of a history, the intercept the
    fixed cost of a run's start and end), the latency of one wavefront
    running a single history (a fit of kernel time against that history's
    flights over 20 seeds), and the headline run's longest history, whose
    flights times that latency bound the run's end from below."""
    import torch
    from paper_2506_00263_amd import inputs, mcx
    by_n = []
    for n in (250_000, 500_000, 1_000_000, 2_000_000):
        Q = mcx.Problem(inputs.cfg2_lattice(n))
        Q.run(sched="async")
        by_n.append((n, _kernel_ms(Q, 5, sched="async")))
        del Q
    (n1, t1), (n2, t2) = by_n[-2], by_n[-1]
    slope = (t2 - t1) / (n2 - n1)
    lone = []
    for seed in range(1, 21):
        Q = mcx.Problem(dict(inputs.cfg2_lattice(1), seed=seed))
        dg = torch.zeros(24, dtype=torch.uint8, device="cuda")
        Q.run(sched="async", digest=dg)
        fl = int(dg.cpu().numpy().view(mcx.DIGEST_DTYPE)["flights"][0])
        lone.append((fl, _kernel_ms(Q, 3, sched="async")))
        del Q
    fl = np.array([x[0] for x in lone], dtype=np.float64)
    tk = np.array([x[1] for x in lone])
    per_flight, lone_fixed = np.linalg.lstsq(np.vstack([fl, np.ones_like(fl)]).T, tk, rcond=None)[0]
    dg = torch.zeros(24 * n_hist, dtype=torch.uint8, device="cuda")
    P.run(sched="async", digest=dg)
    longest = int(dg.cpu().numpy().view(mcx.DIGEST_DTYPE)["flights"].max())
    return {"scheduler": "async", "decomposition": "fused",
            "kernel_ms_by_histories": {str(n): t for n, t in by_n},
            "marginal_ns_per_history": 1e6 * slope, "fixed_ms": t2 - slope * n2,
            "lone_us_per_flight": 1e3 * float(per_flight), "lone_fixed_us": 1e3 * float(lone_fixed),
            "longest_history_flights": longest, "tail_floor_ms": longest * float(per_flight)}


SWEEP_PARTS = ("box", "lattice", "pincell_ce", "pincell_time", "tally_path", "eigen", "async_waves", "weights",
               "backward", "batch")


def eigen_run(P, n, cycles, **kw):
    """Wall time of one k-eigenvalue run (cycles, 25 % inactive) and its
    histories (the source sizes summed over cycles)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = P.run_eigen(n, cycles, cycles // 4, **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, int(r["n_source"].sum()), r


def sweep(parts=SWEEP_PARTS) -> dict:
    """Measurement sweep (tuned knobs from the autotuner next to the defaults)."""
    from paper_2506_00263_amd import autotune, inputs, mcx
    out = {k: [] for k in parts}
    scheds = (("naive", "fused"), ("async", "fused"), ("async", "split"), ("stack", "fused"), ("stack", "split"))
    for n in ((10_000, 100_000, 1_000_000, 10_000_000) if "box" in parts else ()):
        P = mcx.Problem(inputs.cfg1_box(n))
        for s, dc in scheds:
            t = _wall(P, 3, sched=s, decomp=dc)
            out["box"].append({"histories": n, "sched": s, "decomp": dc, "ms": 1e3 * t, "hist_per_s": n / t})
            print("sweep box", out["box"][-1], file=sys.stderr, flush=True)
        del P
    for n in ((100_000, 1_000_000, 10_000_000) if "lattice" in parts else ()):
        P = mcx.Problem(inputs.cfg2_lattice(n))
        reps = 3 if n < 10_000_000 else 2
        for s, dc in scheds:
            t = _wall(P, reps, sched=s, decomp=dc)
            knobs = autotune.tune(P, sched=s, decomp=dc, use_cache=False, reps=1)
            tt = _wall(P, reps, sched=s, decomp=dc, **knobs)
            out["lattice"].append({"histories": n, "sched": s, "decomp": dc, "ms": 1e3 * t, "hist_per_s": n / t,
                                   "tuned_ms": 1e3 * tt, "tuned_hist_per_s": n / tt, "knobs": knobs})
            print("sweep lattice", out["lattice"][-1], file=sys.stderr, flush=True)
        del P
    for nb in ((100, 1000, 10000) if "pincell_ce" in parts else ()):
        for lookup in ("binary", "hash"):
            P = mcx.Problem(inputs.cfg3_pincell(n_ebins=nb, n_histories=1_000_000))
            for s, dc in scheds:
                t = _wall(P, 2, sched=s, decomp=dc, lookup=lookup)
                out["pincell_ce"].append({"bins": nb, "lookup": lookup, "sched": s, "decomp": dc, "ms": 1e3 * t,
                                          "hist_per_s": 1e6 / t})
                print("sweep pincell", out["pincell_ce"][-1], file=sys.stderr, flush=True)
            del P
    # temporal tally resolution (paper Sec. 4): the continuous-energy pin cell
    # with 100 energy bins times 1..128 time bins over [0, 5e-7 s), a window
    # every history ends in (absorbed) at neutron speeds
    for n in ((100_000, 1_000_000) if "pincell_time" in parts else ()):
        for nt in (1, 2, 4, 8, 16, 32, 64, 128):
            d = inputs.with_time_bins(inputs.cfg3_pincell(n_ebins=100, n_histories=n), nt, 5e-7,
                                      speed_coef=NEUTRON_SPEED)
            P = mcx.Problem(d)
            for s, dc in scheds:
                t = _wall(P, 2, sched=s, decomp=dc)
                c = P.counters()
                out["pincell_time"].append({"histories": n, "time_bins": nt, "sched": s, "decomp": dc,
                                            "ms": 1e3 * t, "hist_per_s": n / t, "cutoffs": c["cutoffs"],
                                            "pieces": c["pieces"]})
                print("sweep pincell_time", out["pincell_time"][-1], file=sys.stderr, flush=True)
            del P
    # where the tally adds go (per-block LDS sums, 16 replicas, direct), per
    # scheduler and tally size
    if "tally_path" in parts:
        cases = [("box, 2000 mesh bins", inputs.cfg1_box(1_000_000))]
        for nt in (1, 8, 16, 32, 64):
            cases.append((f"pin cell, 100 energy x {nt} time bins",
                          inputs.with_time_bins(inputs.cfg3_pincell(n_ebins=100, n_histories=1_000_000), nt, 5e-7,
                                                speed_coef=NEUTRON_SPEED)))
        cases.append(("lattice, 364140 mesh bins", inputs.cfg2_lattice(1_000_000)))
        for name, d in cases:
            P = mcx.Problem(d)
            nb = inputs.n_bins(d)
            for s, dc in scheds:
                for path in ("lds", "replicas", "direct"):
                    if path == "lds" and nb > 4096:
                        continue
                    t = _wall(P, 2, sched=s, decomp=dc, tally_path=path)
                    out["tally_path"].append({"case": name, "bins": nb, "sched": s, "decomp": dc, "path": path,
                                              "ms": 1e3 * t, "hist_per_s": d["n_histories"] / t})
                    print("sweep tally_path", out["tally_path"][-1], file=sys.stderr, flush=True)
            del P
    # k-eigenvalue power iteration (the paper's C5G7 experiment, §4-5.1):
    # histories/s against histories per cycle, 24 and 48 cycles (25 % inactive)
    if "eigen" in parts:
        P = mcx.Problem(inputs.with_fission(inputs.cfg2_lattice(1)))
        for cycles in (24, 48):
            for n in (10_000, 100_000, 1_000_000, 10_000_000):
                if cycles == 48 and n == 10_000_000:
                    continue
                for s, dc in scheds:
                    eigen_run(P, n, 2, sched=s, decomp=dc)
                    ts = []
                    for _ in range(2):
                        t, nh, r = eigen_run(P, n, cycles, sched=s, decomp=dc)
                        ts.append(t)
                    t = float(np.median(ts))
                    out["eigen"].append({"cycles": cycles, "per_cycle": n, "sched": s, "decomp": dc,
                                         "ms": 1e3 * t, "hist_per_s": nh / t,
                                         "k_active": float(np.mean(r["k"][cycles // 4:]))})
                    print("sweep eigen", out["eigen"][-1], file=sys.stderr, flush=True)
        del P
    # wavefronts per asynchronous block (each with its own stash; the block
    # shares the LDS tables and tally sums)
    if "async_waves" in parts:
        cases = [("lattice 1e5", inputs.cfg2_lattice(100_000), {}), ("lattice 1e6", inputs.cfg2_lattice(1_000_000), {}),
                 ("lattice 1e7", inputs.cfg2_lattice(10_000_000), {}), ("box 1e6", inputs.cfg1_box(1_000_000), {})]
        for nt in (1, 16, 32):
            cases.append((f"pin cell 100 x {nt} time bins, LDS sums",
                          inputs.with_time_bins(inputs.cfg3_pincell(n_ebins=100, n_histories=1_000_000), nt, 5e-7,
                                                speed_coef=NEUTRON_SPEED), {"tally_path": "lds"}))
        for name, d, kw in cases:
            P = mcx.Problem(d)
            for dc in ("fused", "split"):
                for wpb in (1, 2, 4):
                    t = _wall(P, 2, sched="async", decomp=dc, async_block_waves=wpb, **kw)
                    c = P.counters()
                    out["async_waves"].append({"case": name, "decomp": dc, "waves_per_block": wpb, "ms": 1e3 * t,
                                               "hist_per_s": d["n_histories"] / t, "grid_blocks": c["grid_blocks"],
                                               "block_threads": c["block_threads"], "lds_bytes": c["lds_bytes"]})
                    print("sweep async_waves", out["async_waves"][-1], file=sys.stderr, flush=True)
            del P
    # non-analog weights: implicit capture with roulette below 0.25 to 0.5
    # against analog histories (histories run longer: more flights each)
    if "weights" in parts:
        for name, d0 in (("lattice 1e6", inputs.cfg2_lattice(1_000_000)), ("box 1e6", inputs.cfg1_box(1_000_000))):
            for label, d in (("analog", d0), ("implicit capture", inputs.with_implicit_capture(d0, 0.25, 0.5))):
                P = mcx.Problem(d)
                for s, dc in scheds:
                    t = _wall(P, 2, sched=s, decomp=dc)
                    c = P.counters()
                    out["weights"].append({"case": name, "weights": label, "sched": s, "decomp": dc, "ms": 1e3 * t,
                                           "hist_per_s": d["n_histories"] / t,
                                           "flights_per_history": c["flights"] / d["n_histories"]})
                    print("sweep weights", out["weights"][-1], file=sys.stderr, flush=True)
                del P
    import torch
    d = inputs.cfg4_lattice_grad(1_000_000)
    P = mcx.Problem(d) if "backward" in parts else None
    w = np.random.default_rng(4).normal(size=inputs.n_bins(d))
    for s, dc in ((("naive", "fused"), ("async", "fused"), ("stack", "fused")) if P else ()):
        tf = _wall(P, 3, sched=s, decomp=dc)
        tb = []
        for _ in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            P.backward(w, sched=s, decomp=dc)
            torch.cuda.synchronize()
            tb.append(time.perf_counter() - t1)
        out["backward"].append({"sched": s, "decomp": dc, "fwd_ms": 1e3 * tf, "bwd_ms": 1e3 * float(np.median(tb)),
                                "ratio": float(np.median(tb)) / tf})
        print("sweep backward", out["backward"][-1], file=sys.stderr, flush=True)
    if "batch" not in parts:
        return out
    out["batch"] = {}
    probs = inputs.cfg5_batch()
    nb = sum(p["n_histories"] for p in probs)
    B = mcx.Problem(probs)
    singles = [mcx.Problem(p) for p in probs]
    for s in ("async", "stack", "naive"):
        t_one = _wall(B, 2, sched=s)
        t_seq = []
        for _ in range(2):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for Q in singles:
                Q.run(sched=s)
            torch.cuda.synchronize()
            t_seq.append(time.perf_counter() - t1)
        wb = np.concatenate([np.random.default_rng(k).normal(size=inputs.n_bins(p)) for k, p in enumerate(probs)])
        B.run(sched=s)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.backward(wb, problem=-1, sched=s)
        torch.cuda.synchronize()
        tbw = time.perf_counter() - t1
        out["batch"][s] = {"one_launch_ms": 1e3 * t_one, "hist_per_s": nb / t_one,
                           "sequential_ms": 1e3 * float(np.median(t_seq)), "backward_ms": 1e3 * tbw}
        print("sweep batch", s, out["batch"][s], file=sys.stderr, flush=True)
    out["batch"]["histories"] = nb
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sched", default="async")
    ap.add_argument("--decomp", default="fused")
    ap.add_argument("--workload", default="lattice", choices=["lattice", "pincell"],
                    help="lattice: the multigroup pin lattice (the benchmark); pincell: the continuous-energy pin "
                         "cell (for profiling its kernels; implies --no-extras)")
    ap.add_argument("--lookup", default="hash", choices=["hash", "binary"], help="pincell: cross-section lookup")
    ap.add_argument("--ebins", type=int, default=100, help="pincell: energy bins")
    ap.add_argument("--histories", type=int, default=0, help="histories (0: 1e6)")
    ap.add_argument("--no-extras", action="store_true", help="time only the headline configuration")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--latency", action="store_true",
                    help="lattice: also report where the asynchronous kernel's time goes (with --no-extras too)")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line, print one JSON object with the measurement sweep: "
                         "box histories 1e4..1e7, lattice histories 1e5..1e7, the continuous-energy pin cell over bins, lookups and "
                         "event decompositions, the pin cell over 1..128 time bins, backward/forward per scheduler "
                         "and the batch as one launch vs one launch per problem")
    ap.add_argument("--sweep-parts", default=",".join(SWEEP_PARTS),
                    help="comma-separated parts of the sweep to run (default: all)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="finish with one device-to-device copy of this many MiB (a kernel of known traffic "
                         "against which profiler byte counters are scaled)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (histories would shard "
              "across GPUs with one int64 all-reduce of the tallies; not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_00263_amd import inputs, mcx

    torch.cuda.set_device(0)
    if args.sweep:
        parts = tuple(p for p in args.sweep_parts.split(",") if p)
        bad = [p for p in parts if p not in SWEEP_PARTS]
        if bad:
            ap.error(f"unknown sweep parts {bad}; known: {SWEEP_PARTS}")
        print(json.dumps(sweep(parts)))
        return
    n_hist = args.histories or N_HIST
    run_kw = {}
    if args.workload == "pincell":
        d = inputs.cfg3_pincell(n_ebins=args.ebins, n_histories=n_hist)
        run_kw = {"lookup": args.lookup}
        args.no_extras = True
        args.no_cpu = True
        workload = (f"continuous-energy pin cell, 3 species x 1e5-point tables, {args.lookup} lookup, "
                    f"{n_hist:.0e} histories, {args.ebins} energy bins")
    else:
        d = inputs.cfg2_lattice(n_hist)
        workload = f"multigroup 17x17 pin lattice, 7 materials x 7 groups, {n_hist:.0e} histories, 51x51x20x7 mesh tally"
    P = mcx.Problem(d)
    stream = torch.cuda.current_stream()

    # headline: warmup, then exactly `steps` timed steps (no per-launch
    # events and no host reads inside the timed region)
    for _ in range(args.warmup):
        P.run(sched=args.sched, decomp=args.decomp, stream=stream, **run_kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P.run(sched=args.sched, decomp=args.decomp, stream=stream, **run_kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = n_hist / (wall / args.steps)
    c = P.counters()
    tally = P.tallies()

    # roofline of the dominant kernel: algorithmic bytes per launch over the
    # mean launch duration, timed with HIP events on the run's stream over
    # the same number of steps right after the timed region
    kernel_ms, launches = 0.0, 0
    for _ in range(args.steps):
        P.run(sched=args.sched, decomp=args.decomp, stream=stream, time_kernels=True, **run_kw)
        ck = P.counters()
        kernel_ms += ck["kernel_ms"]
        launches += main_launches(ck, args.sched)
    torch.cuda.synchronize()
    kern = {"async": "async_kernel", "stack": "stack_round", "naive": "naive_kernel"}[args.sched]
    roofline = roofline_block(algorithmic_bytes(c, d, args.lookup) / max(1, launches // args.steps),
                              kernel_ms / max(1, launches), kern,
                              measured_traffic(kern) if args.workload == "lattice" else None)

    out = {
        "metric": "particle histories/sec on 1 GPU (stack vs async TDR); backward/forward time ratio",
        "value": value, "unit": "histories/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload, "histories": n_hist, "scheduler": args.sched, "decomposition": args.decomp},
        "roofline": roofline,
        "counters": {k: c[k] for k in ("flights", "collisions", "cdf_scans", "crossings", "pieces", "events", "lane_slots",
                                       "dispatches", "spills", "refills", "rounds", "launches", "grid_blocks",
                                       "block_threads", "lds_bytes")},
        "active_lane_frac": c["events"] / max(1, c["lane_slots"]),
    }
    if args.sched == "stack":
        # input population of each remapping round of the last timed run
        out["stack_rounds"] = [int(v) for v in P.stack_rounds()]

    if args.latency and args.no_extras and args.workload == "lattice":
        out["latency"] = latency_block(P, N_HIST)
    if not args.no_extras:
        from paper_2506_00263_amd import autotune
        sched = {}
        for s, dc in (("naive", "fused"), ("stack", "fused"), ("stack", "split"), ("async", "fused"), ("async", "split")):
            rec = {}
            for label, knobs in (("default", {}), ("tuned", None)):
                if knobs is None:
                    knobs = autotune.tune(P, sched=s, decomp=dc, use_cache=False, reps=1)
                P.run(sched=s, decomp=dc, **knobs)
                ts, kms = timed_runs(P, 5, sched=s, decomp=dc, **knobs)
                cc = P.counters()
                rec[label] = {"hist_per_s": N_HIST / float(np.median(ts)), "ms": 1e3 * float(np.median(ts)),
                              "kernel_ms": float(np.median(kms)),
                              "active_lane_frac": cc["events"] / max(1, cc["lane_slots"]),
                              "launches": cc["launches"], "knobs": knobs}
                if not np.array_equal(P.tallies(), tally):
                    raise SystemExit(f"tally mismatch between schedulers: {s}/{dc} {knobs}")
            sched[f"{s}_{dc}"] = rec
        out["schedulers"] = sched
        # backward: two replays (pass A, pass B) of the same histories
        w = np.random.default_rng(4).normal(size=inputs.n_bins(d))
        P.run(sched=args.sched, decomp=args.decomp)
        fwd = []
        bwd = []
        for _ in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            P.run(sched=args.sched, decomp=args.decomp)
            torch.cuda.synchronize()
            fwd.append(time.perf_counter() - t1)
            t1 = time.perf_counter()
            P.backward(w, sched=args.sched, decomp=args.decomp)
            torch.cuda.synchronize()
            bwd.append(time.perf_counter() - t1)
        P.run(sched=args.sched, decomp=args.decomp)
        cf = P.counters()
        P.backward(w, sched=args.sched, decomp=args.decomp, time_kernels=True)
        cb = P.counters()
        out["backward"] = {"fwd_ms": 1e3 * float(np.median(fwd)), "bwd_ms": 1e3 * float(np.median(bwd)),
                           "bwd_fwd_ratio": float(np.median(bwd) / np.median(fwd)),
                           "roofline": roofline_block(backward_bytes(cf, N_HIST), cb["kernel_ms"], kern + " x2",
                                                      passes=2)}
        # batched: 256 problems of uneven size in one launch
        probs = inputs.cfg5_batch()
        B = mcx.Problem(probs)
        nb = sum(p["n_histories"] for p in probs)
        bres = {}
        bref = None
        for s in ("async", "stack", "naive"):
            rec = {}
            for label, knobs in (("default", {}), ("tuned", None)):
                if knobs is None:
                    knobs = autotune.tune(B, sched=s, decomp="fused", use_cache=False, reps=1)
                B.run(sched=s, **knobs)
                ts, kms = timed_runs(B, 3, sched=s, **knobs)
                cc = B.counters()
                bk = {"async": "async_kernel", "stack": "stack_round", "naive": "naive_kernel"}[s]
                nl = main_launches(cc, s)
                rec[label] = {"hist_per_s": nb / float(np.median(ts)), "ms": 1e3 * float(np.median(ts)),
                              "kernel_ms": float(np.median(kms)), "knobs": knobs,
                              "roofline": roofline_block(algorithmic_bytes(cc) / nl, float(np.median(kms)) / nl, bk)}
                t = [B.tallies(k) for k in range(len(probs))]
                if bref is None:
                    bref = t
                elif not all(np.array_equal(a, b) for a, b in zip(bref, t)):
                    raise SystemExit(f"batched tally mismatch: {s} {knobs}")
            bres[s] = rec
        # batched backward (both replays, every problem), async
        wb = np.concatenate([np.random.default_rng(k).normal(size=inputs.n_bins(p)) for k, p in enumerate(probs)])
        B.run(sched="async")
        cf = B.counters()
        B.backward(wb, problem=-1, sched="async", time_kernels=True)
        cb = B.counters()
        bres["async_backward"] = {"kernel_ms": cb["kernel_ms"],
                                  "roofline": roofline_block(backward_bytes(cf, nb), cb["kernel_ms"],
                                                             "async_kernel x2", passes=2)}
        out["batched"] = {"problems": len(probs), "histories": nb, **bres}
        # continuous-energy pin cell (3 species x 1e5-point tables in HBM):
        # hashed and binary lookups, fused and split events, 1e6 and 1e7
        # histories, every scheduler
        ce = []
        ce_cases = [(1_000_000, 100, "hash"), (1_000_000, 10000, "hash"), (1_000_000, 100, "binary"),
                    (10_000_000, 100, "hash")]
        ce_ref = {}
        for n_ce, bins, lookup in ce_cases:
            dce = inputs.cfg3_pincell(n_ebins=bins, n_histories=n_ce)
            Q = mcx.Problem(dce)
            per_lookup = ce_lookup_bytes(dce, lookup)
            for s, dc in (("naive", "fused"), ("stack", "fused"), ("stack", "split"), ("async", "fused"),
                          ("async", "split")):
                Q.run(sched=s, decomp=dc, lookup=lookup)
                ts, kms = timed_runs(Q, 2, sched=s, decomp=dc, lookup=lookup)
                cc = Q.counters()
                key = (n_ce, bins)
                tq = Q.tallies()
                if key not in ce_ref:
                    ce_ref[key] = tq
                elif not np.array_equal(ce_ref[key], tq):
                    raise SystemExit(f"CE tally mismatch: {n_ce} {bins} {lookup} {s}/{dc}")
                bk = {"async": "async_kernel", "stack": "stack_round", "naive": "naive_kernel"}[s]
                nl = main_launches(cc, s)
                ce.append({"histories": n_ce, "bins": bins, "lookup": lookup, "sched": s, "decomp": dc,
                           "ms": 1e3 * float(np.median(ts)), "hist_per_s": n_ce / float(np.median(ts)),
                           "kernel_ms": float(np.median(kms)), "flights": cc["flights"],
                           "lookup_bytes": per_lookup,
                           "roofline": roofline_block(algorithmic_bytes(cc, dce, lookup) / nl,
                                                      float(np.median(kms)) / nl, bk)})
                print("bench pincell_ce", {k: v for k, v in ce[-1].items() if k != "roofline"},
                      ce[-1]["roofline"]["frac"], file=sys.stderr, flush=True)
            del Q
        out["pincell_ce"] = ce
        # k-eigenvalue: the lattice with synthetic fission, 1e6 particles per
        # cycle, 24 cycles (6 inactive), default knobs
        E = mcx.Problem(inputs.with_fission(inputs.cfg2_lattice(1)))
        eres = {}
        eref = None
        for s, dc in (("naive", "fused"), ("stack", "fused"), ("async", "fused")):
            eigen_run(E, N_HIST, 2, sched=s, decomp=dc)
            ts = []
            for _ in range(2):
                t, nh, r = eigen_run(E, N_HIST, 24, sched=s, decomp=dc)
                ts.append(t)
            if eref is None:
                eref = (r["k"], E.tallies())
            elif not (np.array_equal(eref[0], r["k"]) and np.array_equal(eref[1], E.tallies())):
                raise SystemExit(f"k-eigenvalue mismatch between schedulers: {s}/{dc}")
            t = float(np.median(ts))
            eres[f"{s}_{dc}"] = {"ms": 1e3 * t, "hist_per_s": nh / t}
        out["eigen"] = {"per_cycle": N_HIST, "cycles": 24, "inactive": 6,
                        "k_active_mean": float(np.mean(eref[0][6:])), **eres}
        if args.workload == "lattice":
            out["latency"] = latency_block(P, N_HIST)

    if not args.no_cpu:
        # the oracle as it stands, on the host cores: the whole workload,
        # repeated until about 5 s have passed; and a 1e5-history prefix on one
        # core (histories are independent and keyed, so a prefix is a fair sample)
        from oracle import oracle as O
        threads = min(16, os.cpu_count() or 1)
        reps, cpu_s, ref = 0, 0.0, None
        while cpu_s < 10.0 and reps < 100:
            t1 = time.perf_counter()
            ref = O.run(d, threads=threads)
            cpu_s += time.perf_counter() - t1
            reps += 1
        n1 = 100_000
        t1 = time.perf_counter()
        O.run(d, 0, n1, threads=1)
        one_s = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": reps * N_HIST / cpu_s, "unit": "histories/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"all {N_HIST} histories of the benchmark workload, {reps} times "
                                         f"({cpu_s:.1f} s)",
                               "single_core": {"value": n1 / one_s, "sample": f"histories [0, {n1}) on 1 core "
                                                                               f"({one_s:.1f} s)"}}
        out["oracle_match"] = bool(np.array_equal(ref["tally"], tally))
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": n * 8, "bytes_written": n * 8}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
