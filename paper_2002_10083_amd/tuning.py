"""Measurement-driven tuner for the per-bin launch shapes and the table
sizing margin of the expansion kernels.

The numeric phase runs one kernel per table bin, and the library reports
each bin kernel's time (HIP events).  Launch shapes of different bins are
independent, so the search is a coordinate descent: for every bin, every
launch variant is timed with the other bins fixed and the fastest kept; then
the estimate scale (table sizing margin) is chosen from a short list by the
whole step time.  Results do not depend on the choice (the accumulation
order is fixed), only the speed does.  The chosen policy is stored in
``tuned.json`` next to this file, keyed by workload name.
"""
from __future__ import annotations

import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "tuned.json")
VARIANTS = [2, 2, 2, 6, 7, 8, 15]       # launch variants per LDS bin
SCALES = (1.0, 1.25, 1.6)
KEYS = (5, 8, 12)                       # Cohen keys per vertex


def pack(variants) -> int:
    return sum((int(v) & 15) << (4 * b) for b, v in enumerate(variants))


def unpack(policy: int):
    return [(policy >> (4 * b)) & 15 for b in range(len(VARIANTS))]



def load_policy(key: str, default=(0, 1.0, 5)):
    """(bin_policy, est_scale, cohen_keys) stored for `key`, else `default`."""
    try:
        with open(TUNED) as f:
            d = json.load(f)
        e = d[key]
        return int(e["bin_policy"], 0), float(e["est_scale"]), int(e.get("cohen_keys", default[2]))
    except (OSError, KeyError, ValueError):
        return default


def has_policy(key: str) -> bool:
    try:
        with open(TUNED) as f:
            return key in json.load(f)
    except (OSError, ValueError):
        return False


def save_policy(key: str, policy: int, scale: float, keys: int, info: dict, path: str = TUNED):
    d = {}
    if os.path.exists(path):
        with open(path) as f:
            d = json.load(f)
    d[key] = dict(bin_policy=hex(policy), est_scale=scale, cohen_keys=keys, **info)
    with open(path, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)


#: bin_policy flags: accumulate LDS bins 0-6 in one persistent launch, and
#: its queue order (lightest bins first instead of heaviest)
PERSIST = 1 << 28
LIGHT_FIRST = 1 << 29


def decide_persist(run, policy: int, scale: float, keys: int, reps: int = 2, log=print):
    """Times the stored launch shapes with per-bin launches and with the
    persistent accumulation in both queue orders (whole-step wall time, best
    of `reps`); returns the fastest policy and the three times."""
    import torch
    base = policy & ~(PERSIST | LIGHT_FIRST)
    trials = {"off_ms": base, "on_ms": base | PERSIST, "on_light_first_ms": base | PERSIST | LIGHT_FIRST}
    ms = {}
    for name, pol in trials.items():
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            run(pol, scale, keys)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) * 1e3
            best = dt if best is None else min(best, dt)
        ms[name] = round(best, 3)
        log("persistent accumulation %s: %.1f ms" % (name[:-3].replace("_", " "), best))
    win = min(ms, key=lambda k: ms[k])
    return trials[win], ms


def candidates_from(key: str, slack: float = 1.3):
    """Per bin, the variants whose time in the stored tuning of `key` was
    within `slack` of that bin's best (all variants where none is stored)."""
    out = [list(range(n)) for n in VARIANTS]
    try:
        with open(TUNED) as f:
            bins = json.load(f)[key]["bins"]
    except (OSError, KeyError, ValueError):
        return out
    for b, times in bins.items():
        b = int(b)
        if b < len(out) and len(times) == VARIANTS[b]:
            best = min(times)
            out[b] = [v for v, t in enumerate(times) if t <= slack * best]
    return out


def tune(run, reps=2, log=print, candidates=None, scales=SCALES, keys=KEYS):
    """run(policy, scale, keys) -> stats dict of one step (bin_ms, t_total_ms).
    candidates: per bin, the variants to try (default all).  Returns
    (policy, scale, keys, report)."""
    import torch

    def measure(policy, scale, keys=5):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = run(policy, scale, keys)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) * 1e3
            if best is None or dt < best[0]:
                best = (dt, st)
        return best

    variants = [0] * len(VARIANTS)
    scale = 1.0
    report = {"bins": {}}
    base_ms, base_st = measure(pack(variants), scale)
    report["start_ms"] = base_ms
    for b in range(len(VARIANTS)):
        cand = candidates[b] if candidates else list(range(VARIANTS[b]))
        times = {}
        for v in cand:
            trial = list(variants)
            trial[b] = v
            ms, st = measure(pack(trial), scale)
            times[v] = st["bin_ms"][b]
        if st["bin_cols"][b] == 0:
            continue
        variants[b] = min(times, key=lambda v: times[v])
        report["bins"][b] = [round(times[v], 3) if v in times else None for v in range(VARIANTS[b])]
        log("bin %d variant times %s -> %d" % (b, report["bins"][b], variants[b]))
    best_scale, best_keys, best_ms = scale, 5, None
    for r in keys:
        for sc in scales:
            ms, st = measure(pack(variants), sc, r)
            log("keys %d scale %.2f: %.1f ms (overflow %d)" % (r, sc, ms, st["n_overflow"]))
            if best_ms is None or ms < best_ms:
                best_scale, best_keys, best_ms = sc, r, ms
    report["final_ms"] = best_ms
    return pack(variants), best_scale, best_keys, report
