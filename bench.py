"""Benchmark: showered events per second for NLO pp -> Z at 13 TeV on one MI355X.

A step is one pass of the whole shower (every step of the veto algorithm) over
one batch of 10^6 NLO S/H events that already sit in HBM; step k showers event
ids k*10^6 .. (k+1)*10^6-1.  By default the timed steps' batches are streamed
through one persistent launch captured in a HIP graph (gaps_shower_stream), so
lanes refill across batch boundaries; --launch per-step launches gaps_shower
once per batch instead.  Hard-event generation and observables are timed
separately, as the paper's component table does, and are not part of `value`.

With --mode learned (default) the learned initial-state bound is first
trained on the GPU (trial log of the plain shower on separate event ids,
training, calibration, tabulation; reported under "learned"), then the same
batches are showered plain and learned; `value` is the learned shower and the
plain one is reported beside it.

--trials retain (default) runs the competition of the veto algorithm in its
retained-trial form (a losing channel keeps its trial scale; the same Markov
chain with fewer draws); the same batches are then also timed with every
channel redrawn each cycle, the paper's form, and reported under
"paper_form".

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
LOG_ID0 = 1 << 40  # event ids of the trial-log run (disjoint from the timed steps)
HBM_PEAK_GBS = 8000.0
# algorithmic FP64 work per unit (a transcendental counted as 20 operations)
OPS_TRIAL = 6 + 20            # one log, the key arithmetic and the compare
OPS_WINNER = 200 + 2 * 50     # z/phi sampling, maps, weight; two PDF lookups
OPS_ACCEPT_BASE = 150         # emission kinematics and bookkeeping
OPS_ACCEPT_PER_PARTON = 28    # II boost: a 4x4 transformation per parton


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, n_sample, seed, retain):
    from oracle.pyoracle import Oracle
    threads = min(16, os.cpu_count() or 1)
    o = Oracle(cfg)
    ev = o.hard_events(0, n_sample, seed)
    t0 = time.perf_counter()
    o.shower(ev, seed, nthreads=threads, retain=retain)
    dt = time.perf_counter() - t0
    form = "retained trials" if retain else "every channel redrawn each cycle"
    return {"value": n_sample / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_sample} NLO pp->Z event ids (seed {seed}), plain shower ({form}), "
                      f"{threads} threads over contiguous id ranges, {dt:.2f} s wall"}


SHOWER_SOURCES = ("capi.hip", "device.hpp", "kernels.hpp", "shower_wave.hip")


def source_hash():
    """Hash of the shower kernel's sources (its device code, record layouts and
    launch plan): a stored traffic figure is used only while it matches (the
    counters describe one build of the kernel)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_19633_amd", "csrc")
    for name in SHOWER_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, mode):
    """HBM bytes per event of `kernel` in `mode` ("plain" or "learned") from the
    committed counter summary, or None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_pp_nlo.traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("modes", {}).get(mode)


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


def learned_pipeline(G, binding, args, seed):
    """Trial log of the plain shower, training, calibration and tabulation, all
    on the GPU with the library's kernels (untimed for `value`, reported)."""
    import torch
    rep = {}
    G.mlp_init(seed + 10)
    t0 = time.perf_counter()
    hin = G.hard_events(LOG_ID0, args.log_events, seed, max_slots=8)
    _, rows, cnt = G.shower_log(hin, seed, args.log_rows, retain=args.trials == "retain")
    torch.cuda.synchronize()
    rep["log_s"], rep["log_events"], rep["log_rows"] = time.perf_counter() - t0, args.log_events, int(rows.shape[0])
    del hin
    t0 = time.perf_counter()
    x, y, ent = G.mlp_features(rows)
    ntr = int(0.8 * x.shape[0])
    loss = G.mlp_train(x[:ntr], y[:ntr], steps=args.train_steps, batch=args.train_batch, lr=3e-3, tau=args.train_tau,
                       seed=seed)
    torch.cuda.synchronize()
    rep["train_s"] = time.perf_counter() - t0
    rep["train_steps"], rep["train_batch"] = args.train_steps, args.train_batch
    rep["train_tau"] = args.train_tau
    lv = loss.cpu().numpy()
    rep["loss_first"], rep["loss_last"] = float(lv[:10].mean()), float(lv[-10:].mean())
    t0 = time.perf_counter()
    G.mlp_calibrate(x[ntr:], y[ntr:], ent[ntr:])
    G.mlp_tabulate()
    torch.cuda.synchronize()
    rep["calibrate_tabulate_s"] = time.perf_counter() - t0
    rep["mean_bound_over_analytic"] = bound_over_analytic(G)
    del x, y, ent
    return rep, rows


def bound_over_analytic(G):
    """Mean over the cells of the current learned table of its ratio to the analytic bound."""
    tab = G.learned_table()
    R = np.repeat(G.bounds()[8:72, :, None], 8, axis=2)
    return float(np.mean(tab[tab > 0] / R[tab > 0]))


def chi_vs_plain(h_plain, h_other):
    """chi^2 of two sets of weighted histograms (sum w, sum w^2) bin by bin."""
    from scipy import stats as sstats
    chi = {}
    for name, (a, a2), (b, b2) in zip(("z_pt", "phi_star", "n_jets"), h_plain, h_other):
        m = (a2 + b2) > 0
        c2, ndf = float(np.sum((a[m] - b[m]) ** 2 / (a2[m] + b2[m]))), int(max(m.sum(), 1))
        chi[name] = {"chi2_ndf": c2 / ndf, "ndf": ndf, "p_value": float(sstats.chi2.sf(c2, ndf))}
    return chi


def timed_stream(G, binding, batches, seed, args, kw, mode):
    """Warm-up passes and one timed pass of the graph-captured stream."""
    import torch
    # the input batches may still be in the making on another stream
    torch.cuda.synchronize()
    stats = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
    K = len(batches)
    if args.launch == "stream":
        stream = torch.cuda.Stream()
        graph = G.capture(batches, seed, stream, stats=stats, mode=mode, **kw)
        run = lambda: graph.launch(stream)  # noqa: E731
    else:
        stream = torch.cuda.current_stream()
        graph = None

        def run():
            for ev_in, ev_out, _ in batches:
                G.shower(ev_in, seed, out=ev_out, stats=stats, stream=stream, mode=mode, **kw)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
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
    if graph is not None:
        graph.close()
    n = sum(b[2] for b in batches)
    return {"wall_s": wall, "launch_ms": launch_ms, "events": n, "stats": stats.cpu().numpy().astype(float),
            "launches": 1 if args.launch == "stream" else len(batches)}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=1_000_000, help="events per step (one batch)")
    ap.add_argument("--mode", choices=["learned", "plain"], default="learned",
                    help="learned: train the bound first and report the learned shower as `value`, "
                         "the plain shower beside it; plain: the plain shower only")
    ap.add_argument("--batches", choices=["even", "uneven"], default="even",
                    help="even: one batch of --events per step; uneven: the same events in batches of "
                         "10^4..5*10^5 (uniform sizes, seed 1) streamed through the same launch")
    ap.add_argument("--launch", choices=["stream", "per-step"], default="stream",
                    help="stream: the timed steps' batches go through one graph-captured persistent "
                         "launch; per-step: one launch per step")
    ap.add_argument("--log-events", type=int, default=420_000, help="events whose trials train the bound")
    ap.add_argument("--log-rows", type=int, default=50_000_000)
    ap.add_argument("--train-steps", type=int, default=1500)
    ap.add_argument("--train-batch", type=int, default=65536)
    ap.add_argument("--train-tau", type=float, default=0.999, help="quantile of the learned bound's pinball loss")
    ap.add_argument("--trials", choices=["retain", "regenerate"], default="retain",
                    help="retain: a losing channel keeps its trial scale (the same Markov chain, fewer draws); "
                         "regenerate: every channel draws again each cycle")
    ap.add_argument("--no-paper-form", action="store_true",
                    help="with --trials retain: skip timing the same batches with every channel redrawn each "
                         "cycle (the paper's form of the competition), reported under \"paper_form\"")
    ap.add_argument("--no-cellmax", action="store_true",
                    help="with --mode learned: skip timing the cell-maximum bound (the non-learned comparator "
                         "built from the same logged trials), reported under \"cellmax\"")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip timing max-veto, generate-select and veto-max in the one-event-per-lane "
                         "kernels on the first two batches, reported under \"competition_forms\"")
    ap.add_argument("--no-matching", action="store_true",
                    help="skip timing the plain shower of the matching variants (MC@NLO started at mZ^2, "
                         "POWHEG-like events with the first-emission correction) and of NLO pp -> Z/photon -> "
                         "e+e- events on two batches of their own events, reported under \"matching\" and "
                         "\"dy_nlo\"")
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
    if args.variant != 0 and (args.launch == "stream" or args.mode == "learned"):
        ap.error("only the wave kernel (variant 0) streams batches and runs the learned mode")

    import torch
    from gapsinputs import workloads
    from paper_2511_19633_amd import binding

    torch.cuda.set_device(0)
    cfg = workloads.config_dict(workloads.PP_NLO)
    seed = 1
    n, K = args.events, args.steps
    G = binding.Gaps(cfg)
    kw = dict(block=args.block, compact_every=args.compact_every, waves_per_simd=args.waves_per_simd,
              variant=args.variant, retain=args.trials == "retain")

    # hard events of every step (ids k*n .. (k+1)*n-1); timed separately, not part of the metric
    t0 = time.perf_counter()
    # even: K batches of n events; uneven: the same n*K events in batches whose
    # sizes are uniform integers in [10^4, 5*10^5] (the last one truncated)
    sizes = workloads.batch_sizes(n * K, seed=1) if args.batches == "uneven" else [n] * K
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    ins = [G.hard_events(int(a), int(m), seed, max_slots=8) for a, m in zip(starts, sizes)]
    torch.cuda.synchronize()
    t_hard = (time.perf_counter() - t0) / K
    outs = [binding.DeviceEvents(int(m), workloads.MAX_SLOTS) for m in sizes]
    batches = [(ins[k], outs[k], int(sizes[k])) for k in range(len(sizes))]
    kernel = {1: "k_shower_lanes", 0: {0: "k_shower_wave", 2: "k_shower_wave", 3: "k_shower_wave3",
                                       4: "k_shower_wave4"}[args.waves_per_simd]}[args.variant]
    if args.trials == "retain":
        kernel = "k_shower_wave_rt3" if args.waves_per_simd == 3 else "k_shower_wave_rt"

    def summarise(r, mode, kname=None):
        nfin = float(np.mean([o.n.double().mean().item() for o in outs]))
        flags = torch.cat([o.flags.to(torch.int64) for o in outs])
        overflow = int(((flags & 1) != 0).sum().item())
        st = r["stats"]
        nev_launch = r["events"] / r["launches"]
        mean_launch_s = r["launch_ms"] / 1e3 / r["launches"]
        ops = (st[1] * OPS_TRIAL + st[0] * OPS_WINNER +
               st[2] * (OPS_ACCEPT_BASE + OPS_ACCEPT_PER_PARTON * 0.5 * nfin)) / r["launches"]
        achieved = ops / mean_launch_s / 1e12
        kname = kname or kernel
        tr = stored_traffic(kname, mode)
        traffic = None if tr is None else tr["bytes_per_event"] * nev_launch
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic, "kernel": kname,
                "launch_ms": mean_launch_s * 1e3, "events_per_launch": nev_launch, "ops_per_launch": ops,
                "hbm_gbs": None if traffic is None else traffic / mean_launch_s / 1e9}
        return (r["events"] / r["wall_s"], r["wall_s"] * 1e3 / K, roof,
                shower_stats(st, r["events"], nfin, overflow))

    def histos():
        """Weighted histograms (sum w, sum w^2) over every timed batch: Z pT and
        phi* in 30 bins, the jet count one bin per integer."""
        spec = ((0, 0.0, 60.0, 30), (3, 0.0, 1.0, 30), (4, -0.5, 6.5, 7))
        acc = [None] * len(spec)
        for ev_in, ev_out, _ in batches:
            ob = G.observables(ev_out)
            for k, (col, lo, hi, nb) in enumerate(spec):
                sw, sw2 = G.histogram(ob, ev_in.w, col, lo, hi, nb)
                acc[k] = (sw, sw2) if acc[k] is None else (acc[k][0] + sw, acc[k][1] + sw2)
            del ob
        return [(a.cpu().numpy(), b.cpu().numpy()) for a, b in acc]

    out_extra = {}
    r_plain = timed_stream(G, binding, batches, seed, args, kw, binding.MODE_PLAIN)
    v_plain, ms_plain, roof_plain, st_plain = summarise(r_plain, "plain")
    t0 = time.perf_counter()
    h_plain = histos()
    torch.cuda.synchronize()
    t_obs = (time.perf_counter() - t0) / K  # observables and histograms of one step
    log(f"plain: {v_plain:.4g} events/s")
    if args.mode == "learned":
        rep, log_rows = learned_pipeline(G, binding, args, seed)
        log(f"trained bound: {rep}")
        r_l = timed_stream(G, binding, batches, seed, args, kw, binding.MODE_LEARNED)
        v_l, ms_l, roof_l, st_l = summarise(r_l, "learned")
        # a weight above its bound that was used without the plain fallback
        unhandled = int(sum(((o.flags.to(torch.int64) & binding.F_VIOL) != 0).sum().item() for o in outs))
        log(f"learned: {v_l:.4g} events/s")
        chi = chi_vs_plain(h_plain, histos())
        value, ms_per_step, roof, stats_main = v_l, ms_l, roof_l, st_l
        out_extra["plain"] = {"value": v_plain, "ms_per_step": ms_plain, "roofline": roof_plain,
                              "shower_stats": st_plain}
        out_extra["learned"] = dict(rep, speedup_over_plain=v_l / v_plain,
                                    histogram_chi2_ndf_vs_plain=chi,
                                    unhandled_bound_violations=unhandled)
    else:
        value, ms_per_step, roof, stats_main = v_plain, ms_plain, roof_plain, st_plain
    if args.trials == "retain" and not args.no_paper_form and args.variant == 0:
        # the same batches with every channel redrawn each cycle (same Markov chain)
        kw_p = dict(kw, retain=False)
        kname_p = {0: "k_shower_wave", 2: "k_shower_wave", 3: "k_shower_wave3",
                   4: "k_shower_wave4"}[args.waves_per_simd]
        pf = {"kernel": kname_p}
        for md, nm in ((binding.MODE_PLAIN, "plain"), (binding.MODE_LEARNED, "learned")):
            if md == binding.MODE_LEARNED and args.mode != "learned":
                continue
            r = timed_stream(G, binding, batches, seed, args, kw_p, md)
            v, ms, rf, st = summarise(r, nm, kname_p)
            log(f"paper form {nm}: {v:.4g} events/s")
            pf[nm] = {"value": v, "ms_per_step": ms, "roofline": rf, "shower_stats": st}
        out_extra["paper_form"] = pf
    if args.mode == "learned" and not args.no_cellmax:
        # the non-learned comparator: cell maxima of the same logged trials
        t0 = time.perf_counter()
        G.cellmax_table(log_rows, int(0.8 * log_rows.shape[0]))
        torch.cuda.synchronize()
        t_tab = time.perf_counter() - t0
        r = timed_stream(G, binding, batches, seed, args, kw, binding.MODE_LEARNED)
        v, ms, rf, st = summarise(r, "cellmax")
        log(f"cell-maximum bound: {v:.4g} events/s")
        out_extra["cellmax"] = {"value": v, "ms_per_step": ms, "speedup_over_plain": v / v_plain,
                                "speedup_over_learned": v / v_l, "table_s": t_tab,
                                "mean_bound_over_analytic": bound_over_analytic(G),
                                "histogram_chi2_ndf_vs_plain": chi_vs_plain(h_plain, histos()),
                                "roofline": rf, "shower_stats": st}
        # the same with adaptive cell sizes (each cell from the finest block
        # around it with enough logged trials)
        t0 = time.perf_counter()
        G.cellmax_table(log_rows, int(0.8 * log_rows.shape[0]), adaptive=True)
        torch.cuda.synchronize()
        t_tab = time.perf_counter() - t0
        r = timed_stream(G, binding, batches, seed, args, kw, binding.MODE_LEARNED)
        v, ms, rf, st = summarise(r, "cellmax_adaptive")
        log(f"cell-maximum bound, adaptive cells: {v:.4g} events/s")
        out_extra["cellmax_adaptive"] = {"value": v, "ms_per_step": ms, "speedup_over_plain": v / v_plain,
                                         "speedup_over_learned": v / v_l, "table_s": t_tab,
                                         "mean_bound_over_analytic": bound_over_analytic(G),
                                         "histogram_chi2_ndf_vs_plain": chi_vs_plain(h_plain, histos()),
                                         "roofline": rf, "shower_stats": st}
    if args.mode == "learned":
        del log_rows
    if not args.no_forms:
        # the three forms of the competition section 2 names, on the same
        # first two batches, plain, in the one-event-per-lane kernels (the
        # other two forms run there only): max-veto with every channel
        # redrawn, generate-select, veto-max
        import argparse as _ap
        a1 = _ap.Namespace(**vars(args))
        a1.launch, a1.warmup = "per-step", 1
        sub = batches[:2]
        forms = {"kernel": "k_shower_lanes", "events": sum(b[2] for b in sub)}
        for nm, kwf in (("max_veto", dict(variant=1)), ("generate_select", dict(variant=1, gen_select=True)),
                        ("veto_max", dict(variant=1, veto_max=True))):
            r = timed_stream(G, binding, sub, seed, a1, kwf, binding.MODE_PLAIN)
            st = r["stats"]
            forms[nm] = {"value": r["events"] / r["wall_s"], "draws_per_event": st[1] / r["events"],
                         "cycles_per_event": st[0] / r["events"], "accepted_per_event": st[2] / r["events"]}
            log(f"{nm} (one event per lane): {forms[nm]['value']:.4g} events/s")
        out_extra["competition_forms"] = forms
    if not args.no_matching:
        # the matching variants: their own hard events (the same ids as the
        # first two batches), the plain shower in the benchmark's launch
        sub_n = [b[2] for b in batches[:2]]
        nb = len(sub_n)
        mt = {"events": int(sum(sub_n)), "kernel": kernel}
        for nm, wl in (("mcatnlo_start_mz2", workloads.PP_NLO_MUQ), ("powheg", workloads.PP_NLO_POWHEG),
                       ("dy_nlo", workloads.PP_DY_NLO)):
            Gm = binding.Gaps(workloads.config_dict(wl))
            ins_m = [Gm.hard_events(int(a), int(m), seed, max_slots=8) for a, m in zip(starts[:nb], sub_n)]
            sub = [(ins_m[k], outs[k], sub_n[k]) for k in range(nb)]
            r = timed_stream(Gm, binding, sub, seed, args, kw, binding.MODE_PLAIN)
            st = r["stats"]
            w = torch.cat([i.w for i in ins_m])
            mt[nm] = {"value": r["events"] / r["wall_s"], "cycles_per_event": st[0] / r["events"],
                      "accepted_per_event": st[2] / r["events"], "violations": int(st[3]),
                      "sigma_per_event": float(w.mean().item()),
                      "negative_weight_fraction": float((w < 0).double().mean().item())}
            log(f"matching {nm}: {mt[nm]['value']:.4g} events/s")
            del ins_m, sub
            Gm.close()
        w0 = torch.cat([b[0].w for b in batches[:nb]])
        mt["mcatnlo_power_shower_sigma_per_event"] = float(w0.mean().item())
        # the second workload at NLO (pp -> Z/photon -> e+e-, power shower) is
        # reported with them, beside the matchings of the first
        out_extra["dy_nlo"] = mt.pop("dy_nlo")
        out_extra["matching"] = mt

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
                   "events_per_step": n, "mode": args.mode, "trials": args.trials, "launch": args.launch,
                   "batches": args.batches, "n_batches": len(batches),
                   "max_slots": workloads.MAX_SLOTS, "kernel": kernel, "block": args.block or "auto",
                   "compact_every": args.compact_every or 8},
        "roofline": roof,
        "shower_stats": stats_main,
        "component_s": {"hard_events_per_step": t_hard, "shower_per_step": ms_per_step / 1e3,
                        "observables_per_step": t_obs},
    }
    out.update(out_extra)
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample, seed, args.trials == "retain")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
