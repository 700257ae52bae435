"""Retained trials on the GPU (libgaps through the C-ABI) against the oracle's
retained-trial form, event by event, with the same bar as the paper's form:
integer, flavour and colour data bit-exact, >= 99.9 % of events with identical
emission sequences, momenta within 1e-9 relative to the event's scale.  Then
the retained form against the paper's form on the GPU, in distribution."""
import sys

import numpy as np
import pytest

from gapsinputs import records, workloads
from tests.test_gpu_parity import SCALE, compare_events

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu(cfgs):
    import torch
    from paper_2511_19633_amd import binding
    assert torch.cuda.is_available()
    return {k: binding.Gaps(v) for k, v in cfgs.items()}


def _same(a, b, what):
    for name in a.fields():
        assert np.array_equal(getattr(a, name), getattr(b, name)), (what, name)


@pytest.mark.parametrize("key,n", [("ee", 10000), ("lo", 10000), ("nlo", 10000), ("dy", 10000),
                                   ("dynlo", 10000)])
def test_retained_shower_parity(gpu, oracles, key, n):
    say(f"retained parity {key} n={n}")
    G, O = gpu[key], oracles[key]
    gout = G.shower(G.hard_events(0, n, 1), 7, retain=True).to_host()
    oout = O.shower(O.hard_events(0, n, 1), 7, nthreads=8, retain=True)
    frac, worst, _ = compare_events(oout, gout, SCALE[key])
    say(f"  identical {frac:.5f}  worst rel diff {worst:.2e}  trials/event {gout.n_trials.mean():.1f}")
    assert frac >= 0.999
    assert worst < 1e-9
    assert int(gout.n_viol.sum()) == 0
    assert np.all((gout.flags & ~np.uint32(records.FLAG_HEVENT)) == 0)


def test_retained_ragged_overflow_and_scheduling(gpu, oracles):
    """Ragged launches, the slot limit and every scheduling knob leave each
    retained-trial event unchanged (the event id keys every draw)."""
    G, O = gpu["nlo"], oracles["nlo"]
    for n in (1, 63, 65, 257):
        gout = G.shower(G.hard_events(100, n, 3), 9, block=64, retain=True).to_host()
        oout = O.shower(O.hard_events(100, n, 3), 9, retain=True)
        frac, _, _ = compare_events(oout, gout, SCALE["nlo"])
        assert frac == 1.0, n
    # a slot limit that overflows some events
    gout = G.shower(G.hard_events(0, 500, 5), 3, max_slots=8, retain=True).to_host()
    oout = O.shower(O.hard_events(0, 500, 5), 3, max_slots=8, retain=True)
    assert np.any(oout.flags & records.FLAG_OVERFLOW)
    assert np.array_equal(gout.flags & records.FLAG_OVERFLOW, oout.flags & records.FLAG_OVERFLOW)
    frac, _, _ = compare_events(oout, gout, SCALE["nlo"])
    assert frac >= 0.99
    n = 4000
    gin = G.hard_events(0, n, 11)
    a = G.shower(gin, 5, block=512, retain=True).to_host()
    for kw in (dict(block=64, grid=7), dict(block=128, compact_every=1), dict(compact_every=33),
               dict(tail_every=16), dict(tail_every=3, block=256), dict(waves_per_simd=3),
               dict(waves_per_simd=3, block=128, tail_every=5)):
        _same(a, G.shower(gin, 5, retain=True, **kw).to_host(), kw)


def test_retained_rejects_other_kernels(gpu):
    from paper_2511_19633_amd import binding
    G = gpu["nlo"]
    gin = G.hard_events(0, 64, 1)
    for kw in (dict(variant=1), dict(waves_per_simd=4), dict(waves_per_simd=3, block=448)):
        with pytest.raises(binding.GapsError):
            G.shower(gin, 1, retain=True, **kw)


def test_retained_stream_and_graph(gpu):
    """Uneven batches in one persistent launch, and graph replays, equal a
    launch per batch."""
    import torch
    from paper_2511_19633_amd import binding
    G = gpu["nlo"]
    sizes = [700, 1500, 64, 900]
    h = G.hard_events(0, sum(sizes), 17).to_host()
    ins, at = [], 0
    for n in sizes:
        ins.append(binding.DeviceEvents.from_host(h.subset(np.arange(at, at + n))))
        at += n
    refs = [G.shower(ev, 8, retain=True).to_host() for ev in ins]
    outs = [binding.DeviceEvents(n, workloads.MAX_SLOTS) for n in sizes]
    batches = list(zip(ins, outs, sizes))
    G.shower_stream(batches, 8, retain=True, block=128)
    for ref, o in zip(refs, outs):
        _same(ref, o.to_host(), "stream")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = G.capture(batches, 8, side, retain=True)
    try:
        for rep in range(3):
            for o in outs:
                o.n.zero_()
                o.E.zero_()
            torch.cuda.synchronize()
            g.launch(side)
            side.synchronize()
            for ref, o in zip(refs, outs):
                _same(ref, o.to_host(), ("replay", rep))
            G.shower(ins[0], 3)  # eager library work between replays
            torch.cuda.synchronize()
    finally:
        g.close()


def test_retained_learned_matches_oracle(gpu, oracles):
    """Learned mode with retained trials: cell constants, null trials at cell
    edges, the per-trial bound check and the plain fallback, against the
    oracle.  The table is the analytic bound cut to an eighth in every third
    eta bin of cells 2-4, so that nulls, refreshed cells and fallbacks (about
    4 % of events) all occur."""
    from paper_2511_19633_amd import binding
    G, O = gpu["nlo"], oracles["nlo"]
    B = O.bounds()
    tab = np.ascontiguousarray(np.broadcast_to(B[8:72, :, None], (64, 48, 8))).copy()
    tab[:, ::3, 2:5] *= 0.125
    G.learned_set_table(tab)
    n = 3000
    gin = G.hard_events(0, n, 2)
    gout = G.shower(gin, 6, mode=binding.MODE_LEARNED, retain=True).to_host()
    oout = O.shower_learned(O.hard_events(0, n, 2), 6, tab, nthreads=8, retain=True)
    fb = (oout.flags & records.FLAG_FALLBACK) != 0
    say(f"  fallbacks {fb.mean():.4f}")
    assert fb.any() and not fb.all()
    frac, worst, _ = compare_events(oout, gout, 13000.0)
    say(f"  identical {frac:.5f}  worst rel diff {worst:.3g}")
    assert frac >= 0.999 and worst < 1e-9
    for kw in (dict(block=64, grid=5, compact_every=1), dict(tail_every=4, block=256)):
        _same(gout, G.shower(gin, 6, mode=binding.MODE_LEARNED, retain=True, **kw).to_host(), kw)


def test_retained_matches_regenerated_in_distribution(gpu):
    """10^6 NLO events showered in both forms on the GPU: the same
    distributions (emissions, Z pT, phi*, jet count) with far fewer draws."""
    import torch
    from paper_2511_19633_amd import binding
    G = gpu["nlo"]
    n = 1_000_000
    gin = G.hard_events(0, n, 1, max_slots=8)
    sa = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
    sb = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
    a = G.shower(gin, 2, stats=sa, max_slots=workloads.MAX_SLOTS)
    b = G.shower(gin, 3, stats=sb, retain=True, max_slots=workloads.MAX_SLOTS)
    ta, tb = sa.cpu().numpy().astype(float), sb.cpu().numpy().astype(float)
    say(f"  trials/event {ta[1] / n:.1f} -> {tb[1] / n:.1f}, cycles {ta[0] / n:.1f} / {tb[0] / n:.1f}")
    assert tb[1] < 0.35 * ta[1]
    assert abs(tb[0] - ta[0]) / ta[0] < 0.01
    from tests.histcheck import chi2_compare
    w = gin.w.cpu().numpy()
    one = np.ones(n)
    na, nb = a.n_accept.cpu().numpy(), b.n_accept.cpu().numpy()
    chi, ndf, p = chi2_compare(na, nb, one, one, np.arange(-0.5, 40.0))
    say(f"  emissions chi2/ndf {chi / ndf:.3f} (p {p:.3g})")
    assert p > 1e-3
    assert not np.any(a.flags.cpu().numpy() & records.FLAG_OVERFLOW)
    oa, ob = G.observables(a).cpu().numpy(), G.observables(b).cpu().numpy()
    for col, edges in ((0, np.linspace(0.0, 60.0, 31)), (3, np.linspace(0.0, 1.0, 31)), (4, np.arange(-0.5, 7.0)),
                       (9, np.arange(3.5, 31.0))):
        chi, ndf, p = chi2_compare(oa[:, col], ob[:, col], w, w, edges)
        say(f"  column {col}: chi2/ndf {chi / ndf:.3f} (ndf {ndf}, p {p:.3g})")
        assert p > 1e-3
