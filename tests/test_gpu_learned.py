"""GPU (libgaps through the C-ABI) against the CPU oracle for the trial log, the
learned-bound network and the learned shower, and the gain of the trained
bound over the plain shower."""
import collections
import math
import sys
import time

import numpy as np
import pytest

from gapsinputs import records, workloads
from oracle import mlp

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
def oracle_model(oracles):
    """Weights, margins and table trained by the oracle's reference loop."""
    o = oracles["nlo"]
    B = o.bounds()
    # one thread: the rows come in event order, so the trained network is reproducible
    _, rows, _ = o.shower_log(o.hard_events(1_000_000, 8000, 1), 1, 2_000_000, nthreads=1)
    x, y, ent = mlp.features(rows, B)
    cell = mlp.cell_ids(rows, o.cell_edges())
    ntr = int(0.8 * len(x))
    th = mlp.train(mlp.init_params(7), x[:ntr], y[:ntr], steps=150, batch=4096, lr=3e-3, tau=0.999)
    delta, _ = mlp.calibrate(th, x[ntr:], y[ntr:], cell[ntr:])
    return th, delta, mlp.tabulate(th, delta, B, o.cell_edges()), rows


def _rowset(rows):
    r = np.ascontiguousarray(rows, dtype=np.float32)
    return collections.Counter(r.view(np.dtype((np.void, 20))).ravel().tolist())


def test_log_mode_rows_match_oracle(G, oracles):
    O = oracles["nlo"]
    n = 2000
    gin = G.hard_events(0, n, 1)
    gout, grows, gcnt = G.shower_log(gin, 1, 1_000_000)
    say("log rows", gcnt)
    _, orows, ocnt = O.shower_log(O.hard_events(0, n, 1), 1, 1_000_000, nthreads=8)
    assert abs(gcnt - ocnt) <= 0.001 * ocnt
    a, b = _rowset(grows.cpu().numpy()), _rowset(orows)
    common = sum((a & b).values())
    assert common >= 0.999 * max(gcnt, ocnt), (common, gcnt, ocnt)
    # logging does not change the shower
    plain = G.shower(gin, 1).to_host()
    h = gout.to_host()
    for name in plain.fields():
        assert np.array_equal(getattr(plain, name), getattr(h, name)), name
    # rows beyond the capacity are counted, not stored
    _, r2, c2 = G.shower_log(gin, 1, 100)
    assert c2 == gcnt and r2.shape[0] == 100


def test_mlp_init_matches_oracle(G):
    G.mlp_init(7)
    assert np.array_equal(G.mlp_get(), mlp.init_params(7))


def _test_theta(seed):
    th = mlp.init_params(seed)
    rng = np.random.default_rng(seed)
    th[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(scale=0.3, size=64)
    th[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(scale=0.3, size=64)
    th[mlp.OFF_B3] = -2.0
    return th.astype(np.float32)


def test_mlp_forward_matches_oracle(G):
    import torch
    th = _test_theta(3)
    G.mlp_set(th)
    rng = np.random.default_rng(0)
    for n in (1, 15, 16, 17, 1000, 100003):
        x = rng.normal(size=(n, 4)).astype(np.float32)
        f = G.mlp_forward(torch.from_numpy(x).cuda()).cpu().numpy()
        ref = mlp.forward(th, x)
        d = np.abs(f - ref) / (1.0 + np.abs(ref))
        # FP32 sums in another order; where one lands across a bfloat16 rounding
        # boundary of the first layer, that unit moves by one bfloat16 step
        assert np.mean(d <= 1e-5) >= 0.99 and d.max() <= 1e-2, (n, d.max(), np.mean(d <= 1e-5))


def test_mlp_grad_matches_oracle(G):
    import torch
    th = _test_theta(4)
    G.mlp_set(th)
    rng = np.random.default_rng(1)
    n = 5003
    x = rng.normal(size=(n, 4)).astype(np.float32)
    y = (rng.normal(size=n) - 2.0).astype(np.float32)
    for tau in (0.5, 0.999):
        g, loss = G.mlp_grad(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), tau)
        g = g.cpu().numpy().astype(np.float64)
        lref, gref = mlp.loss_grad(th, x, y, tau)
        gmag = mlp.grad_magnitudes(th, x, y, tau)
        assert abs(loss.item() - lref) <= 1e-4 * abs(lref)
        for a, b in ((mlp.OFF_W1, mlp.OFF_B1), (mlp.OFF_B1, mlp.OFF_W2), (mlp.OFF_W2, mlp.OFF_B2),
                     (mlp.OFF_B2, mlp.OFF_W3), (mlp.OFF_W3, mlp.OFF_B3), (mlp.OFF_B3, mlp.NPARAM)):
            err = np.linalg.norm(g[a:b] - gref[a:b]) / max(np.linalg.norm(gref[a:b]), 1e-12)
            assert err < 1e-2, (tau, a, err)
            # element by element: 1 % of the element, plus the rounding bound
            # of a sum whose terms carry a bfloat16 backward operand (relative
            # 2^-9) and FP32 accumulation over the rows: 4e-3 of the sum of the
            # terms' magnitudes (an element that cancels to near zero is only
            # as accurate as its terms)
            excess = np.abs(g[a:b] - gref[a:b]) / (1e-2 * np.abs(gref[a:b]) + 4e-3 * gmag[a:b] + 1e-12)
            print(f"tau {tau} block {a}: worst element at {excess.max():.3f} of its tolerance")
            assert np.all(excess <= 1.0), (tau, a, int(np.argmax(excess)), excess.max())


def test_adam_step_matches_oracle(G):
    """One training step on identical rows (so the batch draw does not matter)
    equals the oracle's gradient and Adam update."""
    import torch
    th = _test_theta(5)
    G.mlp_set(th)
    x1 = np.array([[0.3, -0.2, 0.5, 0.1]], dtype=np.float32)
    y1 = np.array([-1.5], dtype=np.float32)
    x = torch.from_numpy(np.repeat(x1, 512, axis=0)).cuda()
    y = torch.from_numpy(np.repeat(y1, 512)).cuda()
    lr = 1e-3
    G.mlp_train(x, y, steps=1, batch=256, lr=lr, tau=0.9)
    got = G.mlp_get().astype(np.float64)
    _, g = mlp.loss_grad(th, x1, y1, 0.9)
    ref, _, _ = mlp.adam_step(th.astype(np.float64), np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), g, 1, lr)
    moved = np.abs(g) > 1e-6
    assert np.mean(np.abs(got - ref)[moved] <= 1e-3 * lr + 1e-7) > 0.99
    assert np.all(np.abs(got - th)[~moved] <= lr * 1.001 + 1e-7)


def test_adam_step_entry_matches_oracle(G):
    """gaps_mlp_adam_step, twice in a row (the step count and moments carry
    over), equals the oracle's Adam update applied to the same gradient (the
    device's own, from gaps_mlp_grad: the gradient itself is compared with the
    oracle's above), and clears the gradient."""
    import torch
    th = _test_theta(6)
    G.mlp_set(th)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3001, 4)).astype(np.float32)
    y = (rng.normal(size=3001) - 2.0).astype(np.float32)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    lr = 1e-3
    prev = th.astype(np.float64)
    m = np.zeros(mlp.NPARAM)
    v = np.zeros(mlp.NPARAM)
    for step in (1, 2):
        g, _ = G.mlp_grad(xd, yd, 0.7)
        gh = g.cpu().numpy().astype(np.float64)
        G.mlp_adam_step(g, lr)
        assert np.all(g.cpu().numpy() == 0.0)
        got = G.mlp_get().astype(np.float64)
        ref, m, v = mlp.adam_step(prev, m, v, gh, step, lr)
        # FP32 update arithmetic against FP64: well within 1e-3 of a step
        err = np.abs(got - ref)
        print(f"step {step}: worst update difference {err.max() / lr:.2e} of lr")
        assert np.all(err <= 1e-3 * lr + 1e-7), (step, err.max())
        prev = got


def test_features_match_oracle(G, oracles, oracle_model):
    import torch
    rows = oracle_model[3][:200000]
    x, y, ent, cell = G.mlp_features(torch.from_numpy(np.ascontiguousarray(rows)).cuda())
    xr, yr, er = mlp.features(rows, oracles["nlo"].bounds())
    assert np.array_equal(x.cpu().numpy(), xr)
    assert np.array_equal(ent.cpu().numpy(), er.astype(np.int32))
    assert np.array_equal(cell.cpu().numpy(), mlp.cell_ids(rows, oracles["nlo"].cell_edges()).astype(np.int32))
    assert np.allclose(y.cpu().numpy(), yr, rtol=0, atol=2e-6)


def test_tabulation_matches_oracle(G, oracle_model):
    th, delta, tab, _ = oracle_model
    G.mlp_set(th)
    G.mlp_set_delta(delta)
    assert np.array_equal(G.mlp_get_delta(), delta)
    G.mlp_tabulate()
    gt = G.learned_table()
    same = gt == tab
    say("table cells identical", same.mean())
    # the network maximum differs by FP32 summation order and, where a first-layer
    # unit lands across a bfloat16 rounding boundary, by one bfloat16 step of that
    # unit; a cell changes only where that moves R e^v across a grid point
    assert same.mean() >= 0.995
    ratio = gt[~same] / tab[~same]
    assert np.all((ratio <= 1 + 2.0 ** -6 + 1e-12) & (ratio >= 1 / (1 + 2.0 ** -6) - 1e-12))


def test_calibration_matches_oracle(G, oracles, oracle_model):
    import torch
    th, _, _, rows = oracle_model
    G.mlp_set(th)
    x, y, ent = mlp.features(rows, oracles["nlo"].bounds())
    cell = mlp.cell_ids(rows, oracles["nlo"].cell_edges())
    dref, _ = mlp.calibrate(th, x, y, cell)
    G.mlp_calibrate(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(),
                    torch.from_numpy(cell.astype(np.int32)).cuda())
    d = G.mlp_get_delta()
    fin = np.isfinite(dref)
    assert np.array_equal(np.isfinite(d), fin)
    assert np.all(np.abs(d[fin] - dref[fin]) < 5e-3)


def _compare(a, b, need=0.999):
    from tests.test_gpu_parity import compare_events
    frac, worst, same = compare_events(a, b, 13000.0)
    say(f"  identical {frac:.5f}  worst rel diff {worst:.3g}")
    assert frac >= need
    return same


def test_learned_shower_matches_oracle(G, oracles, oracle_model):
    from paper_2511_19633_amd import binding
    O = oracles["nlo"]
    tab = oracle_model[2]
    G.learned_set_table(tab)
    n = 3000
    gin = G.hard_events(0, n, 2)
    gout = G.shower(gin, 6, mode=binding.MODE_LEARNED).to_host()
    oout = O.shower_learned(O.hard_events(0, n, 2), 6, tab, nthreads=8)
    _compare(oout, gout)
    # scheduling does not change a learned event either
    for kw in (dict(block=64, grid=5, compact_every=1), dict(tail_every=4, block=256)):
        g2 = G.shower(gin, 6, mode=binding.MODE_LEARNED, **kw).to_host()
        for name in gout.fields():
            assert np.array_equal(getattr(gout, name), getattr(g2, name)), (kw, name)


def test_forced_fallback_matches_oracle(G, oracles):
    """A bound 16 times below the analytic one fails on most events: the
    weighted veto of each failing trial (the weight factor +-(2w - 1)) and the
    event's continuation on the analytic bound match the oracle event by
    event, weights included, in both forms; tail repacking does not change
    an event."""
    from paper_2511_19633_amd import binding
    O = oracles["nlo"]
    B = O.bounds()
    tab = np.ascontiguousarray(np.broadcast_to(B[8:72, :, None] * 2.0 ** -4, (64, 48, 8)))
    G.learned_set_table(tab)
    n = 2000
    gin = G.hard_events(0, n, 4)
    oin = O.hard_events(0, n, 4)
    for retain in (False, True):
        gl = G.shower(gin, 9, mode=binding.MODE_LEARNED, retain=retain).to_host()
        fb = (gl.flags & records.FLAG_FALLBACK) != 0
        say(f"  retain={retain}: fallbacks {fb.mean():.3f}, negative weights {(gl.w < 0).mean():.3f}")
        assert fb.mean() > 0.5
        gt = G.shower(gin, 9, mode=binding.MODE_LEARNED, retain=retain, tail_every=2, block=128).to_host()
        for name in gl.fields():
            assert np.array_equal(getattr(gl, name), getattr(gt, name)), name
        oout = O.shower_learned(oin, 9, tab, nthreads=8, retain=retain)
        _compare(oout, gl)


def test_learned_set_table_rejects_bad_tables(G, oracles):
    from paper_2511_19633_amd import binding
    B = oracles["nlo"].bounds()
    tab = np.ascontiguousarray(np.broadcast_to(B[8:72, :, None] * 1.01 + 1e-3, (64, 48, 8)))
    with pytest.raises(binding.GapsError):
        G.learned_set_table(tab)  # above the analytic bound
    tab = np.ascontiguousarray(np.broadcast_to(B[8:72, :, None], (64, 48, 8))).copy()
    tab[3, 4, 5] = np.nan
    with pytest.raises(binding.GapsError):
        G.learned_set_table(tab)


def test_trained_bound_gains_over_plain(G):
    """The whole learned path on the GPU: log trials of the plain shower, train
    the network on them with the library's kernels, calibrate on held-out
    trials, tabulate; then the learned shower needs fewer veto cycles and
    channel trials, runs faster, falls back rarely and gives the same
    histograms as the plain shower."""
    import torch
    from paper_2511_19633_amd import binding
    G.mlp_init(11)
    _, rows, cnt = G.shower_log(G.hard_events(5_000_000, 40000, 1), 1, 6_000_000)
    say("trial rows", cnt)
    x, y, _, cell = G.mlp_features(rows)
    ntr = int(0.8 * x.shape[0])
    loss = G.mlp_train(x[:ntr], y[:ntr], steps=600, batch=32768, lr=3e-3, tau=0.999, seed=3)
    torch.cuda.synchronize()
    lv = loss.cpu().numpy()
    say("loss first/last", lv[:3], lv[-3:])
    assert lv[-50:].mean() < lv[:10].mean()
    G.mlp_calibrate(x[ntr:], y[ntr:], cell[ntr:])
    G.mlp_tabulate()
    tab = G.learned_table()
    say("mean table / analytic", float(np.mean(tab > 0)))
    n = 1_000_000
    # independent samples (disjoint event ids) for the plain and the learned
    # shower, so that the histogram comparison's variances hold
    gin = G.hard_events(0, n, 1, max_slots=8)
    gin2 = G.hard_events(n, n, 1, max_slots=8)
    stp = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
    stl = torch.zeros(binding.NSTATS, dtype=torch.uint64, device="cuda")
    out_p = binding.DeviceEvents(n, workloads.MAX_SLOTS)
    out_l = binding.DeviceEvents(n, workloads.MAX_SLOTS)
    G.shower(gin, 2, out=out_p)  # warm
    G.shower(gin2, 2, out=out_l, mode=binding.MODE_LEARNED)
    torch.cuda.synchronize()
    tp = tl = float("inf")
    for rep in range(3):  # best of three alternating launches of each form
        for mode, src, out, st in ((binding.MODE_PLAIN, gin, out_p, stp), (binding.MODE_LEARNED, gin2, out_l, stl)):
            if rep == 2:
                st.zero_()
            t0 = time.perf_counter()
            G.shower(src, 2, out=out, stats=st, mode=mode)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if mode == binding.MODE_PLAIN:
                tp = min(tp, dt)
            else:
                tl = min(tl, dt)
    sp, sl = stp.cpu().numpy().astype(float), stl.cpu().numpy().astype(float)
    say(f"plain {n / tp:.4g} ev/s cycles {sp[0] / n:.1f} trials {sp[1] / n:.1f}; "
        f"learned {n / tl:.4g} ev/s cycles {sl[0] / n:.1f} trials {sl[1] / n:.1f} "
        f"fallback {sl[6] / n:.2e} null {sl[7] / n:.1f}")
    assert sl[6] / n < 0.01
    assert sl[0] < 0.85 * sp[0] and sl[1] < sp[1]
    assert tl < tp
    ap, al = out_p.n_accept.double().cpu().numpy(), out_l.n_accept.double().cpu().numpy()
    assert abs(ap.mean() - al.mean()) < 5 * math.sqrt(ap.var() * 2 / n)
    from tests.histcheck import chi2_compare
    op, ol = G.observables(out_p).cpu().numpy(), G.observables(out_l).cpu().numpy()
    wp, wl = out_p.w.cpu().numpy(), out_l.w.cpu().numpy()
    # Z pT (28 bins), jet count and parton count (one bin per integer)
    for col, edges in ((0, np.linspace(0.0, 60.0, 29)), (4, np.arange(-0.5, 7.0)), (9, np.arange(3.5, 31.0))):
        chi, ndf, p = chi2_compare(op[:, col], ol[:, col], wp, wl, edges)
        say(f"  column {col}: chi2/ndf {chi / ndf:.3f} (ndf {ndf}, p {p:.3g})")
        assert p > 1e-3
