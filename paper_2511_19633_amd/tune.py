"""Launch autotuner of the persistent shower kernel.

The paper tunes its kernels' block size by measurement (section 3.2, the
scan over threads per block) and measures where its event partitioning pays
(section 3.1).  Here the launch shape of the one persistent kernel is chosen
the same way, by timing: `autotune` runs the library's gaps_tune over a grid
of candidate shapes -- threads per block, cycles between wave refills
(compaction interval), resident waves per SIMD (occupancy), and the fraction
of the GPU-filling grid (the events in flight, i.e. the batch the kernel
works on at a time, whose working storage competes for the caches) -- on
calibration batches of the caller's workload, and keeps the fastest.  The
choice is stored per (device, workload, mode, form, slots) in a JSON file
and reused without timing when the same key comes back.

Every shape gives bitwise the same events (each random number is keyed by
the event id), so tuning changes only the speed.
"""
from __future__ import annotations

import json
import os
import time

DEFAULT = dict(block=512, compact_every=8, waves_per_simd=2, fill=1.0)


def default_space(retain: bool):
    """The candidate shapes: blocks of 256 and 512 threads at two waves per
    SIMD, refills every 4, 8, 16, 24 or 32 cycles, 100 %, 75 % or 50 % of the
    filling grid; with retained trials also the three-wave kernel (384
    threads)."""
    pts = []
    for block in (512, 256):
        for ce in (4, 8, 16, 24, 32):
            for fill in (1.0, 0.75, 0.5):
                pts.append(dict(block=block, compact_every=ce, waves_per_simd=2, fill=fill))
    if retain:
        for ce in (8, 16):
            pts.append(dict(block=384, compact_every=ce, waves_per_simd=3, fill=1.0))
    return pts


def cache_path():
    return os.environ.get("GAPS_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "gaps",
                                                             "tune.json")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home: the choice is simply not kept


def tuning_key(device_name: str, workload: str, mode: int, retain: bool, max_slots: int) -> str:
    return f"{device_name}|{workload}|mode{mode}|{'retain' if retain else 'regenerate'}|slots{max_slots}"


def autotune(G, batches, seed: int, workload: str, mode: int, retain: bool, space=None, repeats: int = 3,
             use_cache: bool = True, stream=None):
    """Choose the launch shape for `batches` (the calibration batches of the
    workload).  Returns a dict: `params` (block, grid, compact_every,
    waves_per_simd for gaps_shower / gaps_shower_stream), `chosen` and
    `default` points with their times, every timed point, the tuning's wall
    time and whether the choice came from the cache."""
    import torch
    name = torch.cuda.get_device_name(torch.cuda.current_device())
    slots = min(int(b[1].max_slots) for b in batches)
    key = tuning_key(name, workload, mode, retain, slots)
    path = cache_path()
    table = _load(path) if use_cache else {}
    if use_cache and key in table:
        rec = dict(table[key])
        rec["cached"] = True
        return rec
    pts = list(space or default_space(retain))
    if not any(all(p[k] == v for k, v in DEFAULT.items()) for p in pts):
        pts.insert(0, dict(DEFAULT))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = G.tune(batches, seed, pts, repeats=repeats, stream=stream, mode=mode, retain=retain)
    wall = time.perf_counter() - t0
    ok = [r for r in res if r["ms"] > 0.0]
    if not ok:
        raise RuntimeError("gaps_tune: no runnable launch shape")
    best = min(ok, key=lambda r: r["ms"])
    dflt = next(r for r in res if all(r[k] == v for k, v in DEFAULT.items()))
    rec = {"key": key, "params": {k: best[k] for k in ("block", "grid", "compact_every", "waves_per_simd")},
           "chosen": best, "default": dflt, "points": res, "tune_s": wall, "repeats": repeats,
           "calibration_events": int(sum(b[2] if len(b) > 2 else b[0].cap for b in batches)), "cached": False}
    if use_cache:
        table[key] = {k: v for k, v in rec.items() if k != "cached"}
        _store(path, table)
    return rec
