"""Benchmark: showered events per second for NLO pp -> Z at 13 TeV on one MI355X.

A step is one pass of the whole shower (every step of the veto algorithm) over
one batch of 10^6 NLO S/H events that already sit in HBM; step k showers event
ids k*10^6 .. (k+1)*10^6-1.  The K timed steps' batches are streamed through
one persistent launch captured in a HIP graph (gaps_shower_stream), so lanes
refill across batch boundaries.  Every timed figure is the median of --repeats
(default 5) timed passes over all K steps, each bracketed by device
synchronisations, after --warmup untimed passes; the spread (min, max) is
reported beside it.  Hard-event generation and observables are timed
separately, as the paper's component table does, and are not part of `value`.

With --mode learned (default) the learned initial-state bound is first
trained on the GPU (trial log of the plain shower on separate event ids,
training, calibration, tabulation; reported under "learned"), then the same
batches are showered plain and learned; `value` is the learned shower and the
plain one is reported beside it.  The launch shape of each mode (block,
refill interval, waves per SIMD, lanes in flight) comes from the library's
autotuner on the first batch (reported under "autotune", with the
hand-picked default shape's time on the full run beside it).

Reported beside `value`:
  plain, learned, cellmax, cellmax_adaptive   the plain shower, the trained
      bound and the cell-maximum comparators on the same batches
  histograms    chi^2 of Z pT, phi* and the jet count of each form against a
      plain shower of independent events (ids K*10^6 .. 2K*10^6 - 1, the
      output weights), and the plain-vs-plain control under the same protocol
  paper_form    the same batches with every channel redrawn each cycle
  stream_uneven the same 10^7 events in batches of uniform sizes 10^4..5*10^5
      (the batched-stream configuration), one captured launch
  table1        hard events / shower / observables at 10^4, 10^5, 10^6 events
      (the paper's component table), median of the repeats
  competition_forms, matching, dy_nlo   the other forms and workloads
  roofline      the shower kernel against the FP64 vector peak: the
      algorithmic floating-point operations (transcendentals excluded,
      reported as counts) per launch over the median launch time
  cpu_baseline  the CPU oracle on one thread and on all the host's cores
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
LOG_ID0 = 1 << 40  # event ids of the trial-log run (disjoint from the timed steps)
# algorithmic work per unit of the veto algorithm, floating-point operations
# without the transcendental functions (counted separately)
FLOPS_TRIAL = 6               # the trial key ln T + ln(u)/c, its compare
FLOPS_WINNER = 200            # term choice, z/phi sampling, maps, kernel, weight
FLOPS_ACCEPT_BASE = 150       # emission kinematics and bookkeeping
FLOPS_ACCEPT_PER_PARTON = 28  # the initial-initial boost: a 4x4 transformation per parton
# transcendental evaluations per unit: a trial's log; a winner's exp of its
# scale, the coupling's log, z sampling (one log or exp), the PDF lookups'
# logs of x (two) and of Q^2, the trial log's and map's sqrt/cos/sin counted
# with the accepts
TRANS_TRIAL = 1
TRANS_WINNER = 6
PDF_LOOKUPS_WINNER = 2
TRANS_ACCEPT = 6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, seed, retain, n_single, n_all):
    """The oracle (test infrastructure, not tuned) on one thread, then on every
    core this process may run on, over contiguous event-id ranges."""
    from oracle.pyoracle import Oracle
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    o = Oracle(cfg)
    ev1 = o.hard_events(0, n_single, seed)
    t0 = time.perf_counter()
    o.shower(ev1, seed, nthreads=1, retain=retain)
    dt1 = time.perf_counter() - t0
    evn = o.hard_events(0, n_all, seed)
    t0 = time.perf_counter()
    o.shower(evn, seed, nthreads=cores, retain=retain)
    dtn = time.perf_counter() - t0
    form = "retained trials" if retain else "every channel redrawn each cycle"
    return {"value": n_all / dtn, "unit": "events/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n_all} NLO pp->Z event ids (seed {seed}), plain shower ({form}), {cores} threads "
                      f"over contiguous id ranges, {dtn:.2f} s wall; single thread: first {n_single} ids, "
                      f"{dt1:.2f} s",
            "single_thread_value": n_single / dt1, "host_cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
            "single_thread_per_workload": single_thread_rates(seed, retain)}


def single_thread_rates(seed, retain, m=10_000):
    """The oracle on one thread over the first m event ids of each workload
    (e+e- -> q qbar at 91.2 GeV, LO and NLO pp -> Z at 13 TeV), plain shower."""
    from gapsinputs import workloads
    from oracle.pyoracle import Oracle
    out = {}
    for name, wcfg in (("ee", workloads.EE), ("pp_lo", workloads.PP_LO), ("pp_nlo", workloads.PP_NLO)):
        o = Oracle(workloads.config_dict(wcfg))
        ev = o.hard_events(0, m, seed)
        t0 = time.perf_counter()
        o.shower(ev, seed, nthreads=1, retain=retain)
        dt = time.perf_counter() - t0
        out[name] = {"events": m, "events_per_s": m / dt, "wall_s": dt}
    return out


SHOWER_SOURCES = ("capi.hip", "device.hpp", "kernels.hpp", "shower_wave.hip")


def code_text(src):
    """Source text without comments and blank space (what the compiler sees
    of it)."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def source_hash(read=None):
    """Hash of the shower kernel's code (its device code, record layouts and
    launch plan, comments excluded): a stored traffic figure is used only while
    it matches (the counters describe one build of the kernel).  read(name)
    gives a source's text (default: the working tree's)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_19633_amd", "csrc")
    for name in SHOWER_SOURCES:
        if read is None:
            with open(os.path.join(csrc, name)) as f:
                text = f.read()
        else:
            text = read(name)
        h.update((name + "\n" + code_text(text)).encode())
    return h.hexdigest()[:16]


def stored_traffic(kernel, mode):
    """HBM bytes per event of `kernel` in `mode` from the committed counter
    summary, or None (no summary, or taken with other sources)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_pp_nlo.traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("modes", {}).get(mode)


def counted_fp64(tr, events_per_s):
    """FP64 rates from the committed counter summary's per-event figures at
    the measured events/s: the flops the SIMDs issued (SQ_INSTS_VALU_FLOPS_FP64
    and _TRANS, one count per wave instruction, times 64) and those weighted by
    the fraction of lanes active in a VALU instruction; None without a
    summary of these sources."""
    fp = None if tr is None else tr.get("fp64")
    if fp is None:
        return None
    issued = fp["issued_flop_per_event"] * events_per_s / 1e12
    lane = fp["lane_flop_per_event"] * events_per_s / 1e12
    return {"unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS, "issued": issued, "issued_frac": issued / FP64_PEAK_TFLOPS,
            "lane_weighted": lane, "lane_weighted_frac": lane / FP64_PEAK_TFLOPS,
            "issued_flop_per_event": fp["issued_flop_per_event"], "lane_flop_per_event": fp["lane_flop_per_event"],
            "trans_f64_per_event": fp["trans_per_event"]}


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


def counter_dispatches(args):
    """One gaps_shower dispatch of the first batch (10^6 events) per mode, in a
    fixed order (plain, learned after the training, cell maxima fixed and
    adaptive), at the hand-picked launch shape: the run that hardware
    counters are collected on, one dispatch per mode.  Prints the order."""
    import torch
    from gapsinputs import workloads
    from paper_2511_19633_amd import binding
    torch.cuda.set_device(0)
    G = binding.Gaps(workloads.config_dict(workloads.PP_NLO))
    retain = args.trials == "retain"
    n = args.events
    ev_in = G.hard_events(0, n, 1, max_slots=8)
    ev_out = binding.DeviceEvents(n, workloads.MAX_SLOTS)
    order = []

    def run(name, mode):
        G.shower(ev_in, 1, out=ev_out, mode=mode, retain=retain)
        torch.cuda.synchronize()
        order.append(name)
    run("plain", binding.MODE_PLAIN)
    _, rows = learned_pipeline(G, args, 1, retain)
    run("learned", binding.MODE_LEARNED)
    for adaptive, key in ((False, "cellmax"), (True, "cellmax_adaptive")):
        G.cellmax_table(rows, int(0.8 * rows.shape[0]), adaptive=adaptive)
        run(key, binding.MODE_LEARNED)
    print(json.dumps({"dispatch_order": order, "events_per_dispatch": n,
                      "kernel": "k_shower_wave_rt" if retain else "k_shower_wave"}))


def fisher_p(ps):
    """Fisher's combination of independent p-values: -2 sum ln p follows chi^2
    with 2 k degrees of freedom when all k are uniform; its upper tail."""
    from scipy import stats as sstats
    ps = np.maximum(np.asarray(ps, dtype=np.float64), 1e-300)
    return float(sstats.chi2.sf(-2.0 * np.sum(np.log(ps)), 2 * len(ps)))


def scan_sample(G, binding, first, mode, n, K, ev_in, ev_out):
    """Histograms of one independent sample: K batches of n NLO events with ids
    from `first`, showered (retained trials) in `mode`."""
    h = None
    for k in range(K):
        G.hard_events(first + k * n, n, 1, out=ev_in)
        G.shower(ev_in, 1, out=ev_out, retain=True, mode=mode)
        hk = histograms(G, [(ev_out, n)])
        h = hk if h is None else [(a + c, b + d) for (a, b), (c, d) in zip(h, hk)]
    return h


class IndependentScan:
    """The histogram comparison repeated on independent samples: for sample
    k = 1..S, the plain, learned and cell-maximum showers of K n NLO events
    (event ids from 2 k K n) each against a plain reference of the next K n
    ids, all independent of every other sample and of the benchmark's own
    comparison (ids below 2 K n).  Under no bias each p-value is uniform and
    the S p-values of a form and observable combine by Fisher's method
    (-2 sum ln p, chi^2 with 2 S degrees of freedom); one comparison's p-value
    alone says little.  A form's samples are showered while its table is the
    context's bound."""

    def __init__(self, G, binding, S, n, K):
        from gapsinputs import workloads
        self.G, self.binding, self.S, self.n, self.K = G, binding, S, n, K
        self.ev_in = binding.DeviceEvents(n, 8)
        self.ev_out = binding.DeviceEvents(n, workloads.MAX_SLOTS)
        self.refs, self.hs = [], {}

    def base(self, k):
        return 2 * (k + 1) * self.K * self.n

    def run(self, form, mode):
        b = self.binding
        if not self.refs:
            self.refs = [scan_sample(self.G, b, self.base(k) + self.K * self.n, b.MODE_PLAIN, self.n, self.K,
                                     self.ev_in, self.ev_out) for k in range(self.S)]
        self.hs[form] = [scan_sample(self.G, b, self.base(k), mode, self.n, self.K, self.ev_in, self.ev_out)
                         for k in range(self.S)]

    def result(self):
        res = {"events_per_sample": self.K * self.n, "samples": self.S,
               "ids": "sample k = 1..S: ids from 2 k K n, reference the next K n ids",
               "p_values": {f: {} for f in self.hs}, "chi2_ndf": {f: {} for f in self.hs}}
        for f, hl in self.hs.items():
            for k in range(self.S):
                for o, v in chi2(self.refs[k], hl[k]).items():
                    if isinstance(v, dict):
                        res["p_values"][f].setdefault(o, []).append(round(v["p_value"], 4))
                        res["chi2_ndf"][f].setdefault(o, []).append(round(v["chi2_ndf"], 3))
        res["fisher_p"] = {f: {o: fisher_p(ps) for o, ps in res["p_values"][f].items()} for f in self.hs}
        return res


def seed_scan(args):
    """Only the independent-sample histogram comparison (IndependentScan) with
    a bound trained here, args.seed_scan samples."""
    import torch
    from gapsinputs import workloads
    from paper_2511_19633_amd import binding
    torch.cuda.set_device(0)
    G = binding.Gaps(workloads.config_dict(workloads.PP_NLO))
    _, rows = learned_pipeline(G, args, 1, True)
    sc = IndependentScan(G, binding, args.seed_scan, args.events, args.steps)
    sc.run("plain", binding.MODE_PLAIN)
    sc.run("learned", binding.MODE_LEARNED)
    log("plain and learned samples done")
    G.cellmax_table(rows, int(0.8 * rows.shape[0]))
    sc.run("cellmax", binding.MODE_LEARNED)
    print(json.dumps(sc.result()))


def learned_pipeline(G, args, seed, retain):
    """Trial log of the plain shower, training, calibration and tabulation, all
    on the GPU with the library's kernels (untimed for `value`, reported)."""
    import torch
    rep = {}
    G.mlp_init(seed + 10)
    t0 = time.perf_counter()
    hin = G.hard_events(LOG_ID0, args.log_events, seed, max_slots=8)
    _, rows, cnt = G.shower_log(hin, seed, args.log_rows, retain=retain)
    torch.cuda.synchronize()
    rep["log_s"], rep["log_events"], rep["log_rows"] = time.perf_counter() - t0, args.log_events, int(rows.shape[0])
    del hin
    t0 = time.perf_counter()
    x, y, _, cell = G.mlp_features(rows)
    ntr = int(0.8 * x.shape[0])
    loss = G.mlp_train(x[:ntr], y[:ntr], steps=args.train_steps, batch=args.train_batch, lr=3e-3, tau=args.train_tau,
                       seed=seed)
    torch.cuda.synchronize()
    rep["train_s"] = time.perf_counter() - t0
    rep["train_steps"], rep["train_batch"], rep["train_tau"] = args.train_steps, args.train_batch, args.train_tau
    lv = loss.cpu().numpy()
    rep["loss_first"], rep["loss_last"] = float(lv[:10].mean()), float(lv[-10:].mean())
    t0 = time.perf_counter()
    G.mlp_calibrate(x[ntr:], y[ntr:], cell[ntr:])
    G.mlp_tabulate()
    torch.cuda.synchronize()
    rep["calibrate_tabulate_s"] = time.perf_counter() - t0
    rep["mean_bound_over_analytic"] = bound_over_analytic(G)
    del x, y, cell
    return rep, rows


def bound_over_analytic(G):
    """Mean over the cells of the current learned table of its ratio to the analytic bound."""
    tab = G.learned_table()
    R = np.repeat(G.bounds()[8:72, :, None], 8, axis=2)
    return float(np.mean(tab[tab > 0] / R[tab > 0]))


HIST_SPEC = (("z_pt", 0, 0.0, 60.0, 30), ("phi_star", 3, 0.0, 1.0, 30), ("n_jets", 4, -0.5, 6.5, 7))


def histograms(G, pairs):
    """Weighted histograms (sum w, sum w^2, with each event's output weight)
    of Z pT, phi* and the jet count over (record, n) pairs."""
    acc = [None] * len(HIST_SPEC)
    for ev, n in pairs:
        ob = G.observables(ev, n=n)
        for k, (_, col, lo, hi, nb) in enumerate(HIST_SPEC):
            sw, sw2 = G.histogram(ob, ev.w[:n], col, lo, hi, nb)
            acc[k] = (sw, sw2) if acc[k] is None else (acc[k][0] + sw, acc[k][1] + sw2)
        del ob
    return [(a.cpu().numpy(), b.cpu().numpy()) for a, b in acc]


def chi2(h_ref, h_other):
    """chi^2 per degree of freedom of two independent sets of weighted
    histograms, bin by bin over the bins with content, with p-values."""
    from scipy import stats as sstats
    out = {}
    for (name, *_), (a, a2), (b, b2) in zip(HIST_SPEC, h_ref, h_other):
        m = (a2 + b2) > 0
        c2, ndf = float(np.sum((a[m] - b[m]) ** 2 / (a2[m] + b2[m]))), int(max(m.sum(), 1))
        pulls = np.where(m, (b - a) / np.sqrt(np.where(m, a2 + b2, 1.0)), 0.0)
        out[name] = {"chi2_ndf": c2 / ndf, "ndf": ndf, "p_value": float(sstats.chi2.sf(c2, ndf)),
                     "pulls": [round(float(v), 2) for v in pulls]}
    obs = [v for v in out.values() if isinstance(v, dict)]
    out["gate_chi2_ndf_below_1_5"] = all(v["chi2_ndf"] < 1.5 for v in obs)
    # at few degrees of freedom chi^2/ndf < 1.5 fails often for identical
    # distributions (16 % of runs at ndf 7); the p-value gate does not
    out["gate_p_above_0_01"] = all(v["p_value"] > 0.01 for v in obs)
    return out


def timed_stream(G, binding, batches, seed, args, kw, mode, repeats=None, warmup=None):
    """Warm-up passes, then `repeats` timed passes of the graph-captured
    stream (all batches in one launch), each bracketed by synchronisations;
    HIP events on the launch's stream give its device time."""
    import torch
    repeats = args.repeats if repeats is None else repeats
    warmup = args.warmup if warmup is None else warmup
    torch.cuda.synchronize()  # the input batches may still be in the making on another stream
    stats = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
    stream = torch.cuda.Stream()
    graph = G.capture(batches, seed, stream, stats=stats, mode=mode, **kw)
    try:
        for _ in range(warmup):
            graph.launch(stream)
        torch.cuda.synchronize()
        walls, launches = [], []
        for r in range(repeats):
            if r == repeats - 1:
                stats.zero_()  # the last pass's counters (every pass does the same work)
            start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            start.record(stream)
            graph.launch(stream)
            end.record(stream)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - w0)
            launches.append(start.elapsed_time(end))
    finally:
        graph.close()
    n = sum(b[2] for b in batches)
    return {"wall_s": float(np.median(walls)), "wall_s_min": min(walls), "wall_s_max": max(walls),
            "launch_ms": float(np.median(launches)), "launch_ms_min": min(launches), "launch_ms_max": max(launches),
            "repeats": repeats, "events": n, "stats": stats.cpu().numpy().astype(float)}


def shower_stats(st, nev, nfin, overflow):
    trials, winners, accepts = st[1], st[0], st[2]
    return {"trials_per_event": trials / nev, "winner_cycles_per_event": winners / nev,
            "accepted_per_event": accepts / nev,
            "veto_trials_per_accepted_emission": winners / max(accepts, 1.0),
            "channel_trials_per_accepted_emission": trials / max(accepts, 1.0),
            "weight_violations": int(st[3]), "overflow_events": overflow,
            "fallback_events": int(st[6]), "null_winners_per_event": st[7] / nev,
            "mean_final_multiplicity": nfin,
            "active_lane_fraction": st[5] / st[4] if st[4] > 0 else None}


def summarise(r, outs, kernel, mode_name, K):
    """events/s (median pass), ms per step, the roofline entry and the shower statistics of a timed stream."""
    import torch
    nfin = float(np.mean([o.n.double().mean().item() for o in outs]))
    flags = torch.cat([o.flags.to(torch.int64) for o in outs])
    overflow = int(((flags & 1) != 0).sum().item())
    st = r["stats"]
    launch_s = r["launch_ms"] / 1e3
    flops = st[1] * FLOPS_TRIAL + st[0] * FLOPS_WINNER + st[2] * (FLOPS_ACCEPT_BASE +
                                                                  FLOPS_ACCEPT_PER_PARTON * 0.5 * nfin)
    trans = st[1] * TRANS_TRIAL + st[0] * TRANS_WINNER + st[2] * TRANS_ACCEPT
    achieved = flops / launch_s / 1e12
    tr = stored_traffic(kernel, mode_name)
    traffic = None if tr is None else tr["bytes_per_event"] * r["events"]
    roof = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic, "kernel": kernel,
            "launch_ms": r["launch_ms"], "launch_ms_min": r["launch_ms_min"], "launch_ms_max": r["launch_ms_max"],
            "events_per_launch": r["events"], "flops_per_launch": flops,
            "transcendentals_per_launch": trans, "pdf_lookups_per_launch": st[0] * PDF_LOOKUPS_WINNER,
            "philox_blocks_per_launch": st[1] / 4.0 + st[0],
            "transcendentals_per_s": trans / launch_s,
            "hbm_gbs": None if traffic is None else traffic / launch_s / 1e9,
            "counted_fp64": counted_fp64(tr, r["events"] / launch_s)}
    value = r["events"] / r["wall_s"]
    return {"value": value, "value_min": r["events"] / r["wall_s_max"], "value_max": r["events"] / r["wall_s_min"],
            "repeats": r["repeats"], "ms_per_step": r["wall_s"] * 1e3 / K, "roofline": roof,
            "shower_stats": shower_stats(st, r["events"], nfin, overflow)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--repeats", type=int, default=5, help="timed passes per figure (the median is reported)")
    ap.add_argument("--events", type=int, default=1_000_000, help="events per step (one batch)")
    ap.add_argument("--mode", choices=["learned", "plain"], default="learned",
                    help="learned: train the bound first and report the learned shower as `value`, "
                         "the plain shower beside it; plain: the plain shower only")
    ap.add_argument("--log-events", type=int, default=460_000, help="events whose trials train the bound")
    ap.add_argument("--log-rows", type=int, default=52_000_000)
    ap.add_argument("--train-steps", type=int, default=1500)
    ap.add_argument("--train-batch", type=int, default=65536)
    ap.add_argument("--train-tau", type=float, default=0.9999, help="quantile of the learned bound's pinball loss")
    ap.add_argument("--trials", choices=["retain", "regenerate"], default="retain",
                    help="retain: a losing channel keeps its trial scale (the same Markov chain, fewer draws); "
                         "regenerate: every channel draws again each cycle")
    ap.add_argument("--no-tune", action="store_true", help="use the hand-picked default launch shape")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--compact-every", type=int, default=0)
    ap.add_argument("--waves-per-simd", type=int, default=0)
    ap.add_argument("--lite", action="store_true",
                    help="only the timed plain and learned legs (no comparators, forms, workloads, table, CPU)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-single", type=int, default=60_000, help="events of the single-thread oracle run")
    ap.add_argument("--cpu-all", type=int, default=300_000, help="events of the all-core oracle run")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a device copy of this many bytes")
    ap.add_argument("--dispatches", action="store_true",
                    help="only one shower dispatch of the first batch per mode (for hardware counters)")
    ap.add_argument("--scan-samples", type=int, default=5,
                    help="independent samples of the histogram comparison in the default run (0: none)")
    ap.add_argument("--seed-scan", type=int, default=0,
                    help="only the histogram comparison of plain, learned and cell-maximum showers against "
                         "plain references, on this many independent samples (no timing)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the shower runs on one GPU only (events shard trivially by id range; "
              "no multi-GPU path is built)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.dispatches:
        counter_dispatches(args)
        return
    if args.seed_scan:
        seed_scan(args)
        return

    import torch
    from gapsinputs import workloads
    from paper_2511_19633_amd import binding
    from paper_2511_19633_amd import tune as tuner

    torch.cuda.set_device(0)
    cfg = workloads.config_dict(workloads.PP_NLO)
    seed = 1
    n, K = args.events, args.steps
    retain = args.trials == "retain"
    G = binding.Gaps(cfg)
    kernel = "k_shower_wave_rt" if retain else "k_shower_wave"

    # hard events of every step (ids k*n .. (k+1)*n-1); timed separately
    ins = [G.hard_events(k * n, n, seed, max_slots=8) for k in range(K)]
    torch.cuda.synchronize()
    outs = [binding.DeviceEvents(n, workloads.MAX_SLOTS) for _ in range(K)]
    batches = [(ins[k], outs[k], n) for k in range(K)]
    out = {}

    def shape_for(mode):
        """The launch shape of a mode: the autotuner's choice on the first batch
        (or the command line's / the default shape)."""
        if args.no_tune or args.block or args.compact_every or args.waves_per_simd:
            return dict(block=args.block, compact_every=args.compact_every, waves_per_simd=args.waves_per_simd), None
        rec = tuner.autotune(G, batches[:1], seed, "pp_nlo", mode, retain, repeats=3, use_cache=False)
        log(f"autotune mode {mode}: {rec['chosen']} (default {rec['default']['ms']:.2f} ms)")
        rep = {k: rec[k] for k in ("params", "chosen", "default", "tune_s", "repeats", "calibration_events")}
        rep["points"] = rec["points"]
        return dict(rec["params"]), rep

    def is_default(kw):
        return all(kw.get(k, 0) in (0, v) for k, v in (("block", 512), ("compact_every", 8), ("waves_per_simd", 2))) \
            and not kw.get("grid")

    # ---- plain
    kw_plain, tune_plain = shape_for(binding.MODE_PLAIN)
    s_plain = summarise(timed_stream(G, binding, batches, seed, args, dict(kw_plain, retain=retain),
                                     binding.MODE_PLAIN), outs, kernel, "plain", K)
    log(f"plain: {s_plain['value']:.4g} events/s")
    out["plain"] = s_plain
    autotune = {"plain": tune_plain}
    if not args.lite:
        # the reference sample: a plain shower of independent events (ids K n ..
        # 2 K n - 1), one batch at a time through one spare record
        ref_in = binding.DeviceEvents(n, 8)
        ref_out = binding.DeviceEvents(n, workloads.MAX_SLOTS)
        h_ref = None
        for k in range(K):
            G.hard_events((K + k) * n, n, seed, out=ref_in)
            G.shower(ref_in, seed, out=ref_out, retain=retain)
            h = histograms(G, [(ref_out, n)])
            h_ref = h if h_ref is None else [(a + c, b + d) for (a, b), (c, d) in zip(h_ref, h)]
        del ref_in, ref_out
        t0 = time.perf_counter()
        h_plain = histograms(G, [(o, n) for o in outs])
        torch.cuda.synchronize()
        t_obs = (time.perf_counter() - t0) / K
        hist = {"reference": "plain shower of event ids %d .. %d" % (K * n, 2 * K * n - 1),
                "plain_control": chi2(h_ref, h_plain)}
    value, ms_per_step, roof, stats_main = s_plain["value"], s_plain["ms_per_step"], s_plain["roofline"], \
        s_plain["shower_stats"]
    kw_main, mode_main = dict(kw_plain, retain=retain), binding.MODE_PLAIN

    # ---- learned
    log_rows = None
    if args.mode == "learned":
        rep, log_rows = learned_pipeline(G, args, seed, retain)
        log(f"trained bound: {rep}")
        kw_l, tune_l = shape_for(binding.MODE_LEARNED)
        autotune["learned"] = tune_l
        s_l = summarise(timed_stream(G, binding, batches, seed, args, dict(kw_l, retain=retain),
                                     binding.MODE_LEARNED), outs, kernel, "learned", K)
        log(f"learned: {s_l['value']:.4g} events/s")
        neg = int(sum(((o.w < 0) & ((o.flags.to(torch.int64) & binding.F_FALLBACK) != 0)).sum().item() for o in outs))
        out["learned"] = dict(rep, **s_l, speedup_over_plain=s_l["value"] / s_plain["value"],
                              fallback_events_negative_weight=neg)
        if not args.lite:
            hist["learned"] = chi2(h_ref, histograms(G, [(o, n) for o in outs]))
            if args.scan_samples > 0:
                scan = IndependentScan(G, binding, args.scan_samples, n, K)
                scan.run("plain", binding.MODE_PLAIN)
                scan.run("learned", binding.MODE_LEARNED)
                log("independent samples: plain and learned done")
        if tune_l is not None and not is_default(kw_l):
            s_d = summarise(timed_stream(G, binding, batches, seed, args, dict(retain=retain), binding.MODE_LEARNED),
                            outs, kernel, "learned", K)
            autotune["learned_default_shape_value"] = s_d["value"]
            autotune["learned_tuned_over_default"] = s_l["value"] / s_d["value"]
        value, ms_per_step, roof, stats_main = s_l["value"], s_l["ms_per_step"], s_l["roofline"], s_l["shower_stats"]
        kw_main, mode_main = dict(kw_l, retain=retain), binding.MODE_LEARNED
    out["autotune"] = autotune

    if not args.lite:
        # ---- the batched-stream configuration: the same events in uneven
        # batches (sizes uniform in [10^4, 5*10^5], seed 1), views of the
        # records above split where they cross a record's end
        sizes = workloads.batch_sizes(n * K, seed=1)
        ub, pos = [], 0
        for m in sizes:
            while m > 0:
                k, off = divmod(pos, n)
                take = min(m, n - off)
                ub.append((ins[k].view(off, take), outs[k].view(off, take), take))
                pos += take
                m -= take
        r = timed_stream(G, binding, ub, seed, args, kw_main, mode_main)
        s_u = summarise(r, outs, kernel, "learned" if mode_main == binding.MODE_LEARNED else "plain", K)
        out["stream_uneven"] = {"value": s_u["value"], "value_min": s_u["value_min"], "value_max": s_u["value_max"],
                                "batch_sizes": len(sizes), "stream_batches": len(ub),
                                "active_lane_fraction": s_u["shower_stats"]["active_lane_fraction"],
                                "launch_ms": s_u["roofline"]["launch_ms"],
                                "mode": "learned" if mode_main == binding.MODE_LEARNED else "plain"}
        log(f"uneven stream: {s_u['value']:.4g} events/s")

        # ---- the paper's form of the competition on the same batches
        pf = {"kernel": "k_shower_wave"}
        for md, nm in ((binding.MODE_PLAIN, "plain"), (binding.MODE_LEARNED, "learned")):
            if md == binding.MODE_LEARNED and args.mode != "learned":
                continue
            if not retain:
                break
            s = summarise(timed_stream(G, binding, batches, seed, args, dict(retain=False), md), outs,
                          "k_shower_wave", nm, K)
            log(f"paper form {nm}: {s['value']:.4g} events/s")
            pf[nm] = s
        out["paper_form"] = pf

        # ---- the non-learned comparators from the same logged trials
        if args.mode == "learned":
            for adaptive, key in ((False, "cellmax"), (True, "cellmax_adaptive")):
                t0 = time.perf_counter()
                G.cellmax_table(log_rows, int(0.8 * log_rows.shape[0]), adaptive=adaptive)
                torch.cuda.synchronize()
                t_tab = time.perf_counter() - t0
                s = summarise(timed_stream(G, binding, batches, seed, args, kw_main, binding.MODE_LEARNED), outs,
                              kernel, key, K)
                log(f"{key}: {s['value']:.4g} events/s")
                hist[key] = chi2(h_ref, histograms(G, [(o, n) for o in outs]))
                if args.scan_samples > 0 and not adaptive:
                    scan.run("cellmax", binding.MODE_LEARNED)
                out[key] = dict(s, speedup_over_plain=s["value"] / s_plain["value"],
                                speedup_over_learned=s["value"] / out["learned"]["value"], table_s=t_tab,
                                mean_bound_over_analytic=bound_over_analytic(G))
            # back to the trained bound for the legs below
            G.mlp_tabulate()
        out["histograms"] = hist
        if args.mode == "learned" and args.scan_samples > 0:
            out["histograms_independent"] = scan.result()
            del scan
        del log_rows

        # ---- the paper's component table: hard events, shower, observables
        # at 10^4, 10^5 and 10^6 events (views of the first batch)
        t1 = {}
        for m in (10_000, 100_000, 1_000_000):
            if m > n:
                continue
            vi, vo = ins[0].view(0, m), outs[0].view(0, m)
            row = {}
            for what in ("hard", "shower_plain", "shower_" + args.mode, "observables"):
                if what == "shower_learned" and args.mode != "learned":
                    continue
                ts = []
                for r in range(args.repeats + 1):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    if what == "hard":
                        G.hard_events(0, m, seed, out=vi)
                    elif what == "observables":
                        histograms(G, [(vo, m)])
                    else:
                        md = binding.MODE_LEARNED if what == "shower_learned" else binding.MODE_PLAIN
                        G.shower(vi, seed, n=m, out=vo, mode=md, **(kw_main if md == mode_main else
                                                                    dict(kw_plain, retain=retain)))
                    torch.cuda.synchronize()
                    if r:
                        ts.append(time.perf_counter() - t0)
                row[what + "_s"] = float(np.median(ts))
            t1[str(m)] = row
        out["table1"] = t1

        # ---- the three forms of the competition in the one-event-per-lane
        # kernels (where the other two forms run), on the first two batches
        sub = batches[:2]
        forms = {"kernel": "k_shower_lanes", "events": sum(b[2] for b in sub)}
        for nm, kwf in (("max_veto", dict(variant=1)), ("generate_select", dict(variant=1, gen_select=True)),
                        ("veto_max", dict(variant=1, veto_max=True))):
            ts = []
            st = None
            for r in range(3):
                stt = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for ev_in, ev_out, m in sub:
                    G.shower(ev_in, seed, out=ev_out, stats=stt, **kwf)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                st = stt.cpu().numpy().astype(float)
            ev = forms["events"]
            forms[nm] = {"value": ev / float(np.median(ts[1:])), "draws_per_event": st[1] / ev,
                         "cycles_per_event": st[0] / ev, "accepted_per_event": st[2] / ev}
            log(f"{nm} (one event per lane): {forms[nm]['value']:.4g} events/s")
        out["competition_forms"] = forms

        # ---- the matching variants and the NLO Z/photon workload, plain, on
        # their own hard events with the ids of the first two batches
        mt = {"events": 2 * n, "kernel": kernel}
        for nm, wl in (("mcatnlo_start_mz2", workloads.PP_NLO_MUQ), ("powheg", workloads.PP_NLO_POWHEG),
                       ("dy_nlo", workloads.PP_DY_NLO)):
            Gm = binding.Gaps(workloads.config_dict(wl))
            ins_m = [Gm.hard_events(k * n, n, seed, max_slots=8) for k in range(2)]
            r = timed_stream(Gm, binding, [(ins_m[k], outs[k], n) for k in range(2)], seed, args,
                             dict(kw_plain, retain=retain), binding.MODE_PLAIN, repeats=3)
            st = r["stats"]
            w = torch.cat([i.w for i in ins_m])
            mt[nm] = {"value": r["events"] / r["wall_s"], "cycles_per_event": st[0] / r["events"],
                      "accepted_per_event": st[2] / r["events"], "violations": int(st[3]),
                      "sigma_per_event": float(w.mean().item()),
                      "negative_weight_fraction": float((w < 0).double().mean().item())}
            log(f"matching {nm}: {mt[nm]['value']:.4g} events/s")
            del ins_m
            Gm.close()
        mt["mcatnlo_power_shower_sigma_per_event"] = float(torch.cat([b[0].w for b in batches[:2]]).mean().item())
        out["dy_nlo"] = mt.pop("dy_nlo")
        out["matching"] = mt
        out["component_s"] = {"hard_events_per_step": out["table1"].get(str(n), {}).get("hard_s"),
                              "shower_per_step": ms_per_step / 1e3, "observables_per_step": t_obs}

    line = {
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
                   "events_per_step": n, "mode": args.mode, "trials": args.trials, "launch": "stream",
                   "repeats": args.repeats, "max_slots": workloads.MAX_SLOTS, "kernel": kernel,
                   "launch_shape": {k: v for k, v in kw_main.items() if k != "retain"}},
        "roofline": roof,
        "shower_stats": stats_main,
    }
    line.update(out)
    if not args.no_cpu and not args.lite:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(cfg, seed, retain, args.cpu_single, args.cpu_all)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
