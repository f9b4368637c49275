"""Autotuner for the remapping schedulers.

Grid search over the tuning knobs of a scheduler (async: wavefronts per
block, resident wavefronts per CU, stash links, events a drained wavefront
runs in place, and a stash per wavefront or one per block; stack: events a popped particle runs before it is
pushed again, at least and in the tail, the make_work threshold and resident
wavefronts per CU; naive: block size) on a calibration run, timed with HIP
events inside the library.  Knobs never
change results: every candidate's tally is checked against the first
candidate's.  The best choice is cached per (problem class, scheduler,
decomposition, device).
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import mcx

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_autotune_cache.json")


def candidates(sched: str, decomp: str, histories: int = 0) -> list:
    """Knob settings tried for one scheduler (0 = library default); the
    first, with no knob set, is the library's own default choice.  Stack
    thresholds are fractions of the run's histories (the default stack
    capacity holds them all, so no candidate can run out of room)."""
    events = 4 if decomp == "split" else 1
    out = [dict()]
    if sched == "async":
        for wpb in (4, 2, 1):
            for wpc in (0, 4, 8):
                for links in sorted({events + 1, events + 2, events + 3}):
                    out.append(dict(async_block_waves=wpb, waves_per_cu=wpc, stash_links=links))
        out += [dict(async_drain_events=k) for k in (1, 4, 16, 64)]
        if decomp == "fused":
            out += [dict(async_bulk_events=k) for k in (1, 8)]
        for shared in (1, 2):
            for wpb in (4, 2):
                for links in (0, events + wpb + 1, events + 2 * wpb + 2):
                    out.append(dict(async_shared_stash=shared, async_block_waves=wpb, stash_links=links))
        return out
    if sched == "stack":
        out += [dict(stack_min_events=m, stack_tail_events=t) for m in (1, 2, 4, 6, 8) for t in (16, 64, 256)]
        out += [dict(waves_per_cu=w) for w in (4, 8)]
        if decomp == "fused":
            out += [dict(stack_bulk_events=1)]
        if histories >= 4096:
            out += [dict(stack_threshold=max(256, histories // f)) for f in (2, 8, 32)]
        return out
    return out + [dict(block_size=b) for b in (64, 128, 256)]


def problem_key(P: "mcx.Problem", sched: str, decomp: str, lookup: str, device: str) -> str:
    d0 = P.descs[0]
    shape = dict(n=P.n_problems, geometry=int(d0["geometry"]), energy=int(d0["energy_mode"]),
                 tally=int(d0["tally_kind"]), n_mat=int(d0["n_mat"]), n_grp=int(d0["n_grp"]),
                 hist=int(sum(d["n_histories"] for d in P.descs)), sched=sched, decomp=decomp, lookup=lookup,
                 device=device)
    return hashlib.sha1(json.dumps(shape, sort_keys=True).encode()).hexdigest()[:16]


def _load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c: dict) -> None:
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def tune(P: "mcx.Problem", sched: str = "async", decomp: str = "fused", lookup: str = "binary",
         calib_histories: int | None = None, reps: int = 2, use_cache: bool = True, device: str = "gpu0",
         stream=None) -> dict:
    """Return the fastest knob setting for this problem and scheduler."""
    key = problem_key(P, sched, decomp, lookup, device)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key]["best"]
    run_kw = dict(sched=sched, decomp=decomp, lookup=lookup, stream=stream)
    if P.n_problems == 1 and calib_histories:
        run_kw.update(first=0, n=min(calib_histories, P.descs[0]["n_histories"]))
    results = []
    ref = None
    hist = run_kw.get("n") or sum(int(d["n_histories"]) for d in P.descs)
    for cand in candidates(sched, decomp, hist):
        times = []
        for _ in range(reps + 1):
            P.run(time_kernels=True, **run_kw, **cand)
            times.append(P.counters()["kernel_ms"])
        tally = [P.tallies(k) for k in range(P.n_problems)]
        if ref is None:
            ref = tally
        elif not all(np.array_equal(a, b) for a, b in zip(ref, tally)):
            raise RuntimeError(f"tuning knob changed the result: {cand}")
        results.append((float(np.median(times[1:])), cand))
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    if use_cache:
        cache[key] = dict(best=best, table=[dict(ms=t, **c) for t, c in results])
        _save_cache(cache)
    return best
