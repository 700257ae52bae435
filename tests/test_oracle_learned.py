"""Pins of the oracle's learned initial-state bound: the network arithmetic
(closed forms, finite differences, the first Adam step), the tabulation rules,
and the learned shower (exact first-emission distribution with null trials,
the weighted veto of a violated bound (forced everywhere, and planted in one
cell: exact first-emission distribution, where discarding and re-showering
is not), histograms against plain)."""
import math

import numpy as np
import pytest

from gapsinputs import records, toypdf, workloads
from oracle import mlp
from tests import sudakov_pins as pins
from tests.test_oracle_sudakov import PDF, _ii_channel, compare, delta_curve, replicate


def test_bf16_rounding():
    v = np.array([1.0, 3.14159265, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 0.0, 1e-30], dtype=np.float32)
    r = mlp.bf16(v)
    # 8 significant bits, nearest, ties to even
    assert r[0] == 1.0 and r[1] == np.float32(3.140625) and r[2] == 1.0 and r[3] == np.float32(1.0 + 2 ** -6)
    assert r[4] == -2.5 and r[5] == 0.0
    assert abs(r[6] - 1e-30) / 1e-30 < 2 ** -8


def _identity_net():
    th = np.zeros(mlp.NPARAM, dtype=np.float32)
    W1 = th[mlp.OFF_W1:mlp.OFF_B1].reshape(64, 4)
    W2 = th[mlp.OFF_W2:mlp.OFF_B2].reshape(64, 64)
    for c in range(4):
        W1[c, c] = 1.0
        W2[c, c] = 1.0
    th[mlp.OFF_W3:mlp.OFF_W3 + 4] = 1.0
    th[mlp.OFF_B3] = 0.25
    return th


def test_forward_closed_form():
    """A network that routes each input through one ReLU unit per layer sums
    the positive parts: f = sum_c max(x_c, 0) + b3."""
    rng = np.random.default_rng(3)
    x = rng.normal(size=(257, 4)).astype(np.float32)
    th = _identity_net()
    f = mlp.forward(th, x, dtype=np.float64, round_bf16=False)
    assert np.allclose(f, np.maximum(x, 0).astype(np.float64).sum(axis=1) + 0.25, rtol=0, atol=1e-12)
    fb = mlp.forward(th, x)  # bf16 first layer: the positive parts rounded to 8 bits
    ref = mlp.bf16(np.maximum(x, 0)).astype(np.float64).sum(axis=1) + 0.25
    assert np.allclose(fb, ref, rtol=1e-6, atol=1e-6)


def test_gradient_finite_differences():
    rng = np.random.default_rng(5)
    th = mlp.init_params(11).astype(np.float64)
    th[mlp.OFF_B1:mlp.OFF_W2] = 0.1
    th[mlp.OFF_B2:mlp.OFF_W3] = 0.1
    x = rng.normal(size=(64, 4))
    y = rng.normal(size=64)
    tau = 0.9

    def loss(t):
        W1, b1, W2, b2, W3, b3 = mlp.unpack(t)
        h1 = np.maximum(x @ W1.T + b1, 0)
        h2 = np.maximum(h1 @ W2.T + b2, 0)
        r = y - (h2 @ W3 + b3)
        return np.mean(np.where(r >= 0, tau * r, (tau - 1) * r))

    # the oracle's analytic gradient at FP64 parameters (no rounding)
    W1, b1, W2, b2, W3, b3 = [np.asarray(a, dtype=np.float64) for a in mlp.unpack(th)]
    _, g = mlp.loss_grad(th.astype(np.float32), x, y, tau, round_bf16=False)
    # recompute at the float32 parameters the gradient used
    th32 = th.astype(np.float32).astype(np.float64)
    idx = np.concatenate([rng.choice(np.arange(mlp.OFF_W1, mlp.OFF_B1), 10),
                          rng.choice(np.arange(mlp.OFF_B1, mlp.OFF_W2), 5),
                          rng.choice(np.arange(mlp.OFF_W2, mlp.OFF_B2), 15),
                          rng.choice(np.arange(mlp.OFF_B2, mlp.OFF_W3), 5),
                          rng.choice(np.arange(mlp.OFF_W3, mlp.OFF_B3), 5), [mlp.OFF_B3]])
    h = 1e-6
    for p in idx:
        tp, tm = th32.copy(), th32.copy()
        tp[p] += h
        tm[p] -= h
        fd = (loss(tp) - loss(tm)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 + 1e-5 * abs(fd), (p, fd, g[p])


def test_grad_magnitudes_bound_rounded_backward():
    """grad_magnitudes bounds every gradient element, and a gradient whose
    backward operand dA2 is rounded to bfloat16 (as the matrix-core kernels
    take it) differs from the oracle's by at most 2^-8 of it, element by
    element: the scale of the GPU gradient test's tolerance."""
    rng = np.random.default_rng(8)
    th = rng.normal(scale=0.3, size=mlp.NPARAM).astype(np.float32)
    x = rng.normal(size=(3001, 4)).astype(np.float32)
    y = (rng.normal(size=3001) - 2.0).astype(np.float32)
    for tau in (0.5, 0.999):
        _, g = mlp.loss_grad(th, x, y, tau)
        gm = mlp.grad_magnitudes(th, x, y, tau)
        assert np.all(gm >= np.abs(g) * (1 - 1e-12))
        # the same gradient with dA2 rounded to bfloat16 before both products
        W1, b1, W2, b2, W3, b3 = [mlp.bf16(np.float32(a)).astype(np.float64)
                                  for a in mlp.unpack(th)[:5]] + [float(mlp.unpack(th)[5])]
        xd = x.astype(np.float64)
        a1 = xd @ W1.T + b1
        h1q = mlp.bf16(np.maximum(a1, 0.0).astype(np.float32)).astype(np.float64)
        a2 = h1q @ W2.T + b2
        f = np.maximum(a2, 0.0) @ W3 + b3
        r = y - f
        gf = -np.where(r >= 0, tau, tau - 1.0) / len(y)
        da2 = mlp.bf16((np.outer(gf, W3) * (a2 > 0)).astype(np.float32)).astype(np.float64)
        gw2 = (da2.T @ h1q).ravel()
        gw1 = (((da2 @ W2) * (a1 > 0)).T @ xd).ravel()
        for blk, (a, b) in ((gw2, (mlp.OFF_W2, mlp.OFF_B2)), (gw1, (mlp.OFF_W1, mlp.OFF_B1))):
            assert np.all(np.abs(blk - g[a:b]) <= 2.0 ** -8 * gm[a:b] + 1e-15)
        # while a purely relative criterion would fail on elements that cancel
        assert np.any(np.abs(gw1 - g[mlp.OFF_W1:mlp.OFF_B1]) > 1e-3 * np.abs(g[mlp.OFF_W1:mlp.OFF_B1]))


def test_adam_first_step_closed_form():
    """Bias correction makes the first Adam step lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    th, g = rng.normal(size=50), rng.normal(size=50)
    t1, m, v = mlp.adam_step(th, np.zeros(50), np.zeros(50), g, 1, 0.01)
    assert np.allclose(t1, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_init_distribution():
    th = mlp.init_params(2)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th)
    assert not b1.any() and not b2.any() and b3 == 0.0
    for W, fan in ((W1, 4), (W2, 64), (W3, 64)):
        lim = math.sqrt(6.0 / fan)
        assert np.all(np.abs(W) <= lim)
        assert abs(W.mean()) < 0.1 * lim
        assert abs(W.var() - lim * lim / 3) < 0.15 * lim * lim / 3
    assert np.array_equal(th, mlp.init_params(2)) and not np.array_equal(th, mlp.init_params(3))


def test_up6_and_tabulation(oracles):
    v = np.array([1.0, 0.3, 1.7, 1e-5, 123.456])
    u = mlp.up6(v)
    assert np.all(u >= v) and np.all(u <= v * (1 + 2.0 ** -6))
    m, _ = np.frexp(u)
    assert np.all(m * 128 == np.round(m * 128))
    assert np.array_equal(mlp.up6(u), u)
    o = oracles["nlo"]
    B = o.bounds()
    R = B[8:72]
    fm = np.zeros((64, 48, 8), dtype=np.float32)
    # no margins: the analytic table in every cell
    t0 = mlp.tabulate(None, np.full(64, np.inf), B, o.cell_edges(), fmax=fm)
    assert np.array_equal(t0, np.broadcast_to(R[:, :, None], t0.shape))
    # v = delta + max f, clipped to [-20, 0], applied as R e^v rounded up
    d = np.full(64, -1.0)
    d[5] = 3.0
    fm[:, :, 2] = -30.0
    t1 = mlp.tabulate(None, d, B, o.cell_edges(), fmax=fm)
    for e in (0, 9, 17, 45):
        assert np.array_equal(t1[e, :, 0], np.minimum(R[e], mlp.up6(R[e] * math.exp(-1.0))))
        assert np.array_equal(t1[e, :, 2], np.minimum(R[e], mlp.up6(R[e] * math.exp(-20.0))))
    assert np.array_equal(t1[5, :, 0], R[5])  # v clipped at 0: the analytic constant
    assert np.array_equal(t1[5, :, 2], np.minimum(R[5], mlp.up6(R[5] * math.exp(-20.0))))
    assert np.all(t1 <= R[:, :, None])


def test_calibration_margins_closed_form(oracles):
    """With a network that outputs a constant f, the residual of a row is
    y - f: a cell with MIN_CAL_CELL rows gets its own largest residual + 2^-6;
    a thinner cell that of its (entry, eta bin) when the bin's cells hold
    MIN_CAL_BIN rows together, else that of its entry; an entry with fewer than
    MIN_CAL rows keeps the analytic bound (+inf); and the cell of a row is the
    ln t cell the shower takes for its scale (the lower edge itself belongs to
    the cell below)."""
    o = oracles["nlo"]
    E = o.cell_edges()
    th = np.zeros(mlp.NPARAM, dtype=np.float32)
    th[mlp.OFF_B3] = -1.0  # f = -1 everywhere
    lne_bin = lambda b: mlp.LNETA0 + (b + 0.5) * mlp.DLE
    rows, ys = [], []

    def add(ent, b, k, y, count, lnt=None):
        lt = 0.5 * (E[k] + E[k + 1]) if lnt is None else lnt
        for _ in range(count):
            rows.append((lt, lne_bin(b), 0.5, ent, 0.0))
            ys.append(y)
    # entry 10: a full cell (3, 2), a thin cell (3, 5) in a full bin, a thin bin 7
    add(10, 3, 2, -0.5, mlp.MIN_CAL_CELL)
    add(10, 3, 5, -0.2, 10)
    add(10, 7, 1, -0.9, 10)
    add(10, 9, 4, -0.3, mlp.MIN_CAL - mlp.MIN_CAL_CELL - 20)
    # entry 20: too few rows in all
    add(20, 0, 0, 0.0, 50)
    # a row on the lower edge of cell 4 (as stored: the float at or just below
    # it) belongs to cell 3
    lt32 = np.float32(E[4])
    if float(lt32) > E[4]:
        lt32 = np.nextafter(lt32, np.float32(-np.inf))
    add(10, 11, 3, -0.1, 1, lnt=float(lt32))
    rows = np.asarray(rows, dtype=np.float32)
    x = np.zeros((len(rows), 4), dtype=np.float32)
    y = np.asarray(ys, dtype=np.float32)
    cell = mlp.cell_ids(rows, E)
    assert cell[-1] == ((10 - 8) * 48 + 11) * 8 + 3
    d, cnt = mlp.calibrate(th, x, y, cell, round_bf16=False)
    m = mlp.CAL_MARGIN
    f = -1.0
    y32 = lambda v: float(np.float32(v))
    assert d[2, 3, 2] == y32(-0.5) - f + m                      # its own
    assert d[2, 3, 5] == max(y32(-0.5), y32(-0.2)) - f + m     # its bin's (two cells)
    assert d[2, 3, 0] == d[2, 3, 5]                            # an empty cell of a full bin
    assert d[2, 7, 1] == y32(-0.1) - f + m                     # a thin bin: the entry's maximum
    assert d[2, 47, 7] == d[2, 7, 1]
    assert np.all(np.isinf(d[12]))                             # entry 20: analytic
    assert cnt[2, 3, 2] == mlp.MIN_CAL_CELL and cnt[2, 11, 3] == 1


def test_forced_fallback_weighted(oracles):
    """A bound 16 times below the analytic one fails on most events' first
    initial-state winners.  Each failing trial goes through the weighted veto:
    the event's weight is multiplied by +-(2w - 1) (w > 1, so at least one in
    size) and the event continues on the analytic bound; events that never
    fail keep their weight bit for bit, and on average the factor is one
    (the weighted veto conserves the total rate)."""
    o = oracles["nlo"]
    B = o.bounds()
    tab = np.ascontiguousarray(np.broadcast_to(B[8:72, :, None] * 2.0 ** -4, (64, 48, 8)))
    ev = o.hard_events(0, 4000, 4)
    l = o.shower_learned(ev, 9, tab, nthreads=8)
    fb = (l.flags & records.FLAG_FALLBACK) != 0
    assert fb.mean() > 0.5
    f = l.w / ev.w
    assert np.all(f[~fb] == 1.0)
    assert np.all(np.abs(f[fb]) >= 1.0) and np.any(f[fb] < 0.0)
    assert abs(f.mean() - 1.0) < 5.0 * f.std() / math.sqrt(len(f))
    assert int(l.n_viol.sum()) == 0  # learned-bound failures are not analytic violations


@pytest.mark.slow
@pytest.mark.parametrize("retain", [False, True], ids=["regenerate", "retain"])
def test_learned_too_low_everywhere_first_emission(oracles, cfgs, retain):
    """Every cell 16 times below the analytic bound: the weighted first-emission
    distribution of a u ubar Born still equals the Sudakov quadrature."""
    o, pdf = oracles["lo"], PDF(cfgs["lo"]["pdf"])
    B = o.bounds()
    tab = np.ascontiguousarray(np.broadcast_to(B[8:72, :, None] * 2.0 ** -4, (64, 48, 8)))
    base = o.hard_events(0, 64, 3)
    k = next(e for e in range(64) if abs(base.pid[0, e]) == 2)
    n = 20000
    ev = replicate(base, k, n)
    out = o.shower_learned(ev, 5, tab, nthreads=8, retain=retain)
    assert ((out.flags & records.FLAG_FALLBACK) != 0).mean() > 0.2
    S = 13000.0 ** 2
    ea, eb = 2 * base.E[0, k] / 13000.0, 2 * base.E[1, k] / 13000.0
    s = ea * eb * S
    chans = [_ii_channel(pdf, s, ea, toypdf.TABLE_NAMES.index("u" if base.pid[0, k] == 2 else "ubar")),
             _ii_channel(pdf, s, eb, toypdf.TABLE_NAMES.index("u" if base.pid[1, k] == 2 else "ubar"))]
    tgrid = np.array([1.7, 3.0, 10.0, 30.0, 100.0, 1000.0, 1e4, 1e5])
    pins.compare(out.t1, tgrid, delta_curve(chans, 1.69, tgrid), w=out.w / ev.w)


@pytest.mark.slow
@pytest.mark.parametrize("retain", [False, True], ids=["regenerate", "retain"])
def test_learned_planted_low_cell(oracles, cfgs, retain):
    """One cell planted 64 times below the analytic bound (family A of both
    quarks of a u ubar Born, ln t cell 2, i.e. t in [16.9, 169) GeV^2): the
    weighted first-emission distribution equals the Sudakov quadrature, while
    the rule that discards a violating event and showers it again on the
    analytic bound, applied to the same events, is off by many standard
    errors (events that drew no trial in the cell keep too low an emission
    rate there)."""
    worst, old = pins.check_learned_planted(oracles["lo"], PDF(cfgs["lo"]["pdf"]), retain)
    assert worst < 1.0
    assert old > 8.0, old


@pytest.mark.slow
@pytest.mark.parametrize("retain", [False, True], ids=["regenerate", "retain"])
def test_learned_first_emission_with_null_trials(oracles, cfgs, retain):
    """With the analytic constants in every cell, learned mode draws each
    initial-state channel cell by cell (a null at every cell edge it crosses);
    the first-emission distribution still equals the Sudakov quadrature."""
    o, pdf = oracles["lo"], PDF(cfgs["lo"]["pdf"])
    B = o.bounds()
    tab = np.ascontiguousarray(np.broadcast_to(B[8:72, :, None], (64, 48, 8)))
    base = o.hard_events(0, 64, 3)
    k = next(e for e in range(64) if abs(base.pid[0, e]) == 2)
    n = 20000
    ev = replicate(base, k, n)
    out = o.shower_learned(ev, 5, tab, nthreads=8, retain=retain)
    assert not np.any(out.flags & records.FLAG_FALLBACK)
    plain = o.shower(ev, 5, nthreads=8, retain=retain)
    assert out.n_cycles.mean() > plain.n_cycles.mean()  # the null winners
    S = 13000.0 ** 2
    ea, eb = 2 * base.E[0, k] / 13000.0, 2 * base.E[1, k] / 13000.0
    s = ea * eb * S
    chans = [_ii_channel(pdf, s, ea, toypdf.TABLE_NAMES.index("u" if base.pid[0, k] == 2 else "ubar")),
             _ii_channel(pdf, s, eb, toypdf.TABLE_NAMES.index("u" if base.pid[1, k] == 2 else "ubar"))]
    tgrid = np.array([1.7, 3.0, 10.0, 30.0, 100.0, 1000.0, 1e4, 1e5])
    compare(out.t1, tgrid, delta_curve(chans, 1.69, tgrid))


@pytest.fixture(scope="module")
def trained(oracles):
    """A bound trained by the oracle's own reference loop on oracle trial logs."""
    o = oracles["nlo"]
    B = o.bounds()
    # one thread: the rows come in event order, so the trained bound is reproducible
    _, rows, _ = o.shower_log(o.hard_events(1_000_000, 12000, 1), 1, 3_000_000, nthreads=1)
    x, y, ent = mlp.features(rows, B)
    cell = mlp.cell_ids(rows, o.cell_edges())
    ntr = int(0.8 * len(x))
    th = mlp.train(mlp.init_params(7), x[:ntr], y[:ntr], steps=250, batch=4096, lr=3e-3, tau=0.999)
    delta, _ = mlp.calibrate(th, x[ntr:], y[ntr:], cell[ntr:])
    return th, delta, mlp.tabulate(th, delta, B, o.cell_edges())


@pytest.mark.slow
@pytest.mark.parametrize("retain", [False, True], ids=["regenerate", "retain"])
def test_learned_histograms_match_plain(oracles, trained, retain):
    """Learned and plain showers of independent NLO samples agree in
    distribution (Z pT, number of partons, with the output weights), with
    fewer cycles and rare fallbacks."""
    o = oracles["nlo"]
    _, _, tab = trained
    n = 20000
    # independent samples: the plain and learned showers get disjoint event
    # ids (so neither the hard events nor the random numbers are shared)
    ev = o.hard_events(0, n, 1)
    ev2 = o.hard_events(n, n, 1)
    p = o.shower(ev, 3, nthreads=8, retain=retain)
    l = o.shower_learned(ev2, 3, tab, nthreads=8, retain=retain)
    fb = (l.flags & records.FLAG_FALLBACK) != 0
    assert fb.mean() < 0.02
    assert l.n_cycles[~fb].mean() < 0.8 * p.n_cycles.mean()
    assert l.n_trials[~fb].mean() < p.n_trials.mean()
    op, ol = o.observables(p), o.observables(l)
    chi = []
    for col, lo, hi in ((0, 0.0, 60.0), (9, 3.5, 30.5)):
        hp, _ = np.histogram(op[:, col], bins=27, range=(lo, hi), weights=p.w)
        hp2, _ = np.histogram(op[:, col], bins=27, range=(lo, hi), weights=p.w ** 2)
        hl, _ = np.histogram(ol[:, col], bins=27, range=(lo, hi), weights=l.w)
        hl2, _ = np.histogram(ol[:, col], bins=27, range=(lo, hi), weights=l.w ** 2)
        m = (hp2 + hl2) > 0
        chi.append(np.sum((hp[m] - hl[m]) ** 2 / (hp2[m] + hl2[m])) / m.sum())
    assert max(chi) < 2.0, chi  # p < 0.2 % at 27 degrees of freedom
