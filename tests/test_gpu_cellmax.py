"""The cell-maximum bound on the GPU (libgaps through the C-ABI) against the
oracle: the table from the same logged trials, the learned-mode shower with
that table event by event, and at 10^6 events the same distributions as the
plain shower with fewer veto cycles."""
import sys

import numpy as np
import pytest

from gapsinputs import records, workloads
from oracle import cellmax
from tests.test_gpu_parity import compare_events

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G(cfgs):
    import torch
    from paper_2511_19633_amd import binding
    assert torch.cuda.is_available()
    return binding.Gaps(cfgs["nlo"])


@pytest.fixture(scope="module")
def logged(oracles):
    """Trial log of 20 000 NLO events from the oracle, and its table."""
    o = oracles["nlo"]
    _, rows, cnt = o.shower_log(o.hard_events(3_000_000, 20_000, 5), 5, 5_000_000, nthreads=8)
    nf = int(0.8 * cnt)
    tab, delta, n = cellmax.cellmax_table(rows[:nf], rows[nf:], o.bounds(), o.cell_edges())
    return rows, nf, tab, delta, n


def test_cellmax_table_matches_oracle(G, oracles, logged):
    import torch
    O = oracles["nlo"]
    rows, nf, tab, delta, n = logged
    say(f"rows {rows.shape[0]}, fitted cells {int(((n >= cellmax.MIN_CELL) & np.isfinite(delta)[:, None, None]).sum())}")
    G.cellmax_table(torch.from_numpy(np.ascontiguousarray(rows)).cuda(), nf)
    g = G.learned_table()
    diff = g != tab
    say(f"  cells differing {int(diff.sum())}")
    assert not diff.any()
    # a second call with other rows starts from cleared counters
    G.cellmax_table(torch.from_numpy(np.ascontiguousarray(rows[:nf // 2])).cuda(), nf // 4)
    o2, _, _ = cellmax.cellmax_table(rows[:nf // 4], rows[nf // 4:nf // 2], O.bounds(), O.cell_edges())
    assert np.array_equal(G.learned_table(), o2)


def test_cellmax_rejects_bad_arguments(G):
    import torch
    from paper_2511_19633_amd import binding
    rows = torch.zeros((10, 5), dtype=torch.float32, device="cuda")
    with pytest.raises(binding.GapsError):
        G.cellmax_table(rows, 0)
    with pytest.raises(binding.GapsError):
        G.cellmax_table(rows, 11)


def test_cellmax_shower_matches_oracle(G, oracles, logged):
    """The learned-mode shower with the oracle's cell-maximum table, both trial
    forms, event by event."""
    from paper_2511_19633_amd import binding
    O = oracles["nlo"]
    tab = logged[2]
    G.learned_set_table(tab)
    n = 3000
    gin = G.hard_events(0, n, 2)
    for retain in (True, False):
        gout = G.shower(gin, 6, mode=binding.MODE_LEARNED, retain=retain).to_host()
        oout = O.shower_learned(O.hard_events(0, n, 2), 6, tab, nthreads=8, retain=retain)
        fb = (oout.flags & records.FLAG_FALLBACK) != 0
        frac, worst, _ = compare_events(oout, gout, 13000.0)
        say(f"  retain={retain}: identical {frac:.5f}, worst rel diff {worst:.3g}, fallbacks {fb.mean():.4f}")
        assert frac >= 0.999 and worst < 1e-9


def test_cellmax_distributions_and_gain(G):
    """10^6 NLO events with a cell-maximum table from 4 * 10^5 logged events:
    the plain shower's distributions, rare fallbacks, fewer veto cycles."""
    import torch
    from paper_2511_19633_amd import binding
    from tests.histcheck import chi2_compare
    _, rows, cnt = G.shower_log(G.hard_events(1 << 40, 400_000, 1, max_slots=8), 1, 50_000_000)
    G.cellmax_table(rows, int(0.8 * rows.shape[0]))
    n = 1_000_000
    gin = G.hard_events(0, n, 1, max_slots=8)
    sp = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
    sl = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
    a = G.shower(gin, 3, stats=sp, retain=True, max_slots=workloads.MAX_SLOTS)
    b = G.shower(gin, 3, stats=sl, mode=binding.MODE_LEARNED, retain=True, max_slots=workloads.MAX_SLOTS)
    tp, tl = sp.cpu().numpy().astype(float), sl.cpu().numpy().astype(float)
    fb = int(((b.flags.cpu().numpy() & records.FLAG_FALLBACK) != 0).sum())
    say(f"  rows {cnt}; cycles/event {tp[0] / n:.1f} -> {tl[0] / n:.1f}; fallbacks {fb}")
    assert tl[0] < 0.85 * tp[0]
    assert fb < 1e-3 * n
    w = gin.w.cpu().numpy()
    oa, ob = G.observables(a).cpu().numpy(), G.observables(b).cpu().numpy()
    for col, edges in ((0, np.linspace(0.0, 60.0, 31)), (4, np.arange(-0.5, 7.0)), (9, np.arange(3.5, 31.0))):
        chi, ndf, p = chi2_compare(oa[:, col], ob[:, col], w, w, edges)
        say(f"  column {col}: chi2/ndf {chi / ndf:.3f} (p {p:.3g})")
        assert p > 1e-3


def test_cellmax_adaptive_table_matches_oracle(G, oracles, logged):
    """Adaptive cell sizes: the GPU table equals the oracle's bit for bit."""
    import torch
    O = oracles["nlo"]
    rows, nf = logged[0], logged[1]
    G.cellmax_table(torch.from_numpy(np.ascontiguousarray(rows)).cuda(), nf, adaptive=True)
    g = G.learned_table()
    o, _, na = cellmax.cellmax_table(rows[:nf], rows[nf:], O.bounds(), O.cell_edges(), adaptive=True)
    say(f"  adaptive: cells differing {int((g != o).sum())}, cells with a block {int((na > 0).sum())}")
    assert np.array_equal(g, o)


def test_cellmax_adaptive_distributions_and_gain(G):
    """10^6 NLO events with adaptive cells from 4 * 10^5 logged events: the
    plain shower's distributions, rare fallbacks, no more veto cycles than the
    fixed cells."""
    import torch
    from paper_2511_19633_amd import binding
    from tests.histcheck import chi2_compare
    _, rows, cnt = G.shower_log(G.hard_events(1 << 40, 400_000, 1, max_slots=8), 1, 50_000_000)
    n = 1_000_000
    gin = G.hard_events(0, n, 1, max_slots=8)
    outs, cyc = {}, {}
    for adaptive in (False, True):
        G.cellmax_table(rows, int(0.8 * rows.shape[0]), adaptive=adaptive)
        st = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
        outs[adaptive] = G.shower(gin, 3, stats=st, mode=binding.MODE_LEARNED, retain=True,
                                  max_slots=workloads.MAX_SLOTS)
        cyc[adaptive] = float(st.cpu().numpy().astype(float)[0]) / n
    a = G.shower(gin, 3, retain=True, max_slots=workloads.MAX_SLOTS)
    b = outs[True]
    fb = int(((b.flags.cpu().numpy() & records.FLAG_FALLBACK) != 0).sum())
    say(f"  cycles/event fixed {cyc[False]:.1f}, adaptive {cyc[True]:.1f}; fallbacks {fb}")
    assert cyc[True] <= cyc[False] * 1.01
    assert fb < 1e-3 * n
    w = gin.w.cpu().numpy()
    oa, ob = G.observables(a).cpu().numpy(), G.observables(b).cpu().numpy()
    for col, edges in ((0, np.linspace(0.0, 60.0, 31)), (4, np.arange(-0.5, 7.0)), (9, np.arange(3.5, 31.0))):
        chi, ndf, p = chi2_compare(oa[:, col], ob[:, col], w, w, edges)
        say(f"  column {col}: chi2/ndf {chi / ndf:.3f} (p {p:.3g})")
        assert p > 1e-3
