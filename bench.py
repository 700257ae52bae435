"""Benchmark: showered events per second for NLO pp -> Z at 13 TeV on one MI355X.

A step is one pass of the whole shower (every step of the veto algorithm) over
one batch of 10^6 NLO S/H events that already sit in HBM; step k showers event
ids k*10^6 .. (k+1)*10^6-1.  By default the timed steps' batches are streamed
through one persistent launch captured in a HIP graph (gaps_shower_stream), so
lanes refill across batch boundaries; --launch per-step launches gaps_shower
once per batch instead.  Hard-event generation and observables are timed
separately, as the paper's component table does, and are not part of `value`.

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

import numpy as np

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


def source_hash():
    """Hash of the shower kernel sources: a stored traffic figure is used only
    while it matches (the counters describe one build of the kernel)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_19633_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per event of `kernel` from the committed counter summary, or None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_pp_nlo.traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    return d


def copy_probe(nbytes):
    """A plain device copy of known size: the calibration run for the HBM byte counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=1_000_000, help="events per step (one batch)")
    ap.add_argument("--launch", choices=["stream", "per-step"], default="stream",
                    help="stream: the timed steps' batches go through one graph-captured persistent "
                         "launch; per-step: one launch per step")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--compact-every", type=int, default=0)
    ap.add_argument("--waves-per-simd", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=150_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a device copy of this many bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the shower runs on one GPU only (events shard trivially by id range; "
              "no multi-GPU path is built)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.launch == "stream" and args.variant != 0:
        ap.error("only the wave kernel (variant 0) streams batches")

    import torch
    from gapsinputs import workloads
    from paper_2511_19633_amd import binding

    torch.cuda.set_device(0)
    cfg = workloads.config_dict(workloads.PP_NLO)
    seed = 1
    n, K = args.events, args.steps
    G = binding.Gaps(cfg)
    kw = dict(block=args.block, compact_every=args.compact_every, waves_per_simd=args.waves_per_simd,
              variant=args.variant)
    stats = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")

    # hard events of every step (ids k*n .. (k+1)*n-1); timed separately, not part of the metric
    t0 = time.perf_counter()
    ins = [G.hard_events(k * n, n, seed, max_slots=8) for k in range(K)]
    torch.cuda.synchronize()
    t_hard = (time.perf_counter() - t0) / K
    outs = [binding.DeviceEvents(n, workloads.MAX_SLOTS) for _ in range(K)]
    batches = [(ins[k], outs[k], n) for k in range(K)]

    if args.launch == "stream":
        stream = torch.cuda.Stream()
        graph = G.capture(batches, seed, stream, stats=stats, **kw)
        run = lambda: graph.launch(stream)  # noqa: E731
    else:
        stream = torch.cuda.current_stream()
        def run():
            for k in range(K):
                G.shower(ins[k], seed, out=outs[k], stats=stats, stream=stream, **kw)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} passes over {K} batches)")

    # timed: K steps; HIP events on the stream the shower kernel runs on
    stats.zero_()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    start.record(stream)
    run()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    launch_ms = start.elapsed_time(end)
    launches = 1 if args.launch == "stream" else K
    log(f"timed {K} steps: wall {wall * 1e3:.1f} ms, device {launch_ms:.1f} ms")
    st = stats.cpu().numpy().astype(float)

    ms_per_step = wall * 1e3 / K
    value = n * K / wall
    mean_launch_s = launch_ms / 1e3 / launches
    nev_launch = n * K / launches

    # observables of the last batch (timed separately)
    t0 = time.perf_counter()
    obs = G.observables(outs[-1])
    torch.cuda.synchronize()
    t_obs = time.perf_counter() - t0

    nfin = float(np.mean([o.n.double().mean().item() for o in outs]))
    flags = torch.cat([o.flags.to(torch.int64) for o in outs])
    overflow = int(((flags & 1) != 0).sum().item())
    trials, winners, accepts = st[binding.ST_TRIALS], st[binding.ST_CYCLES], st[binding.ST_ACCEPT]
    ops = (trials * OPS_TRIAL + winners * OPS_WINNER +
           accepts * (OPS_ACCEPT_BASE + OPS_ACCEPT_PER_PARTON * 0.5 * nfin)) / launches
    achieved = ops / mean_launch_s / 1e12
    viol = int(st[binding.ST_VIOL])
    kernel = {1: "k_shower_lanes", 0: {0: "k_shower_wave", 2: "k_shower_wave", 3: "k_shower_wave3",
                                       4: "k_shower_wave4"}[args.waves_per_simd]}[args.variant]
    tr = stored_traffic(kernel)
    traffic = None if tr is None else tr["bytes_per_event"] * nev_launch
    nev = n * K

    out = {
        "metric": "showered events/sec, NLO pp→Z 13 TeV, 1 MI355X; plain vs learned-proposal",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pp_nlo_1m: NLO-matched Z production at 13 TeV (MC@NLO-style S/H events, "
                               "toy PDF grid 100x50), one step = one batch of 10^6 events with its own ids, "
                               "FP64 kinematics, up to 128 partons per event",
                   "events_per_step": n, "mode": "plain", "launch": args.launch,
                   "max_slots": workloads.MAX_SLOTS, "kernel": kernel, "block": args.block or "auto",
                   "compact_every": args.compact_every or 4},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": kernel, "launch_ms": mean_launch_s * 1e3, "events_per_launch": nev_launch,
                     "ops_per_launch": ops,
                     "hbm_gbs": None if traffic is None else traffic / mean_launch_s / 1e9},
        "shower_stats": {"trials_per_event": trials / nev, "winner_cycles_per_event": winners / nev,
                         "accepted_per_event": accepts / nev,
                         "veto_trials_per_accepted_emission": winners / max(accepts, 1.0),
                         "channel_trials_per_accepted_emission": trials / max(accepts, 1.0),
                         "weight_violations": viol, "overflow_events": overflow,
                         "mean_final_multiplicity": nfin,
                         "active_lane_fraction": (st[binding.ST_LANE_ACTIVE] / st[binding.ST_LANE_ITERS]
                                                  if st[binding.ST_LANE_ITERS] > 0 else None)},
        "component_s": {"hard_events_per_step": t_hard, "shower_per_step": ms_per_step / 1e3,
                        "observables_per_step": t_obs},
    }
    if args.launch == "stream":
        graph.close()
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample, seed)
    print(json.dumps(out))
    del obs


if __name__ == "__main__":
    main()
