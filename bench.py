"""Benchmark: showered events per second for NLO pp -> Z at 13 TeV on one MI355X.

A step is one pass of the whole shower (gaps_shower, every step of the veto
algorithm) over one batch of 10^6 NLO S/H events that already sit in HBM.
Hard-event generation and observables are timed separately, as the paper's
component table does, and are not part of `value`.

Prints one JSON line.  Extra objects:
  roofline      the shower kernel against the FP64 vector peak, with the
                algorithmic operation count of the launches that were timed
  cpu_baseline  the CPU oracle on the host cores on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
# algorithmic FP64 work per unit (a transcendental counted as 20 operations)
OPS_TRIAL = 6 + 20            # one log, the key arithmetic and the compare
OPS_WINNER = 200 + 2 * 50     # z/phi sampling, maps, weight; two PDF lookups
OPS_ACCEPT_BASE = 150         # emission kinematics and bookkeeping
OPS_ACCEPT_PER_PARTON = 28    # II boost: a 4x4 transformation per parton


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, n_sample, seed):
    from oracle.pyoracle import Oracle
    threads = min(16, os.cpu_count() or 1)
    o = Oracle(cfg)
    ev = o.hard_events(0, n_sample, seed)
    t0 = time.perf_counter()
    o.shower(ev, seed, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_sample} NLO pp->Z event ids (seed {seed}), shower only, "
                      f"{threads} threads over contiguous id ranges, {dt:.2f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=1_000_000)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--compact-every", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=150_000)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (events shard trivially by id range; "
              "no multi-GPU path is built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from gapsinputs import workloads
    from paper_2511_19633_amd import binding

    torch.cuda.set_device(0)
    cfg = workloads.config_dict(workloads.PP_NLO)
    seed = 1
    n = args.events
    G = binding.Gaps(cfg)
    stream = torch.cuda.current_stream()

    # hard events (timed separately, not part of the metric)
    t0 = time.perf_counter()
    ev_in = G.hard_events(0, n, seed)
    torch.cuda.synchronize()
    t_hard = time.perf_counter() - t0
    ev_out = binding.DeviceEvents(n, workloads.MAX_SLOTS)
    stats = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")

    for _ in range(args.warmup):
        G.shower(ev_in, seed, out=ev_out, block=args.block, compact_every=args.compact_every,
                 variant=args.variant)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(args.steps):
        stats.zero_()
        starts[k].record(stream)
        G.shower(ev_in, seed, out=ev_out, block=args.block, compact_every=args.compact_every,
                 variant=args.variant, stats=stats)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    log("step ms: " + ", ".join(f"{m:.1f}" for m in ms))
    st = stats.cpu().numpy().astype(float)  # counters of the last step

    ms_per_step = wall * 1e3 / args.steps
    value = n * args.steps / wall
    mean_launch_s = sum(ms) / len(ms) / 1e3

    # observables (timed separately)
    t0 = time.perf_counter()
    obs = G.observables(ev_out)
    torch.cuda.synchronize()
    t_obs = time.perf_counter() - t0

    nfin = ev_out.n.double().mean().item()
    trials, winners, accepts = st[binding.ST_TRIALS], st[binding.ST_CYCLES], st[binding.ST_ACCEPT]
    ops = (trials * OPS_TRIAL + winners * OPS_WINNER +
           accepts * (OPS_ACCEPT_BASE + OPS_ACCEPT_PER_PARTON * 0.5 * nfin))
    achieved = ops / mean_launch_s / 1e12
    viol = int(st[binding.ST_VIOL])

    out = {
        "metric": "showered events/sec, NLO pp→Z 13 TeV, 1 MI355X; plain vs learned-proposal",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pp_nlo_1m: NLO-matched Z production at 13 TeV, MC@NLO-style S/H "
                               "events, toy PDF grid 100x50, 10^6 events per step, FP64 kinematics",
                   "events_per_step": n, "mode": "plain", "max_slots": workloads.MAX_SLOTS,
                   "kernel": "k_shower_lanes" if args.variant == 1 else "k_shower_wave",
                   "block": args.block or 256, "compact_every": args.compact_every or 4},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_shower_lanes" if args.variant == 1 else "k_shower_wave",
                     "launch_ms": mean_launch_s * 1e3,
                     "ops_per_launch": ops},
        "shower_stats": {"trials_per_event": trials / n, "winner_cycles_per_event": winners / n,
                         "accepted_per_event": accepts / n,
                         "veto_trials_per_accepted_emission": winners / max(accepts, 1.0),
                         "channel_trials_per_accepted_emission": trials / max(accepts, 1.0),
                         "weight_violations": viol, "mean_final_multiplicity": nfin,
                         "active_lane_fraction": (st[binding.ST_LANE_ACTIVE] / st[binding.ST_LANE_ITERS]
                                                  if st[binding.ST_LANE_ITERS] > 0 else None)},
        "component_s": {"hard_events": t_hard, "shower_per_step": ms_per_step / 1e3, "observables": t_obs},
    }
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample, seed)
    print(json.dumps(out))
    del obs


if __name__ == "__main__":
    main()
