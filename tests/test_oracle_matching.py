"""Pins of the oracle's matching variants (the alternatives to the paper's
MC@NLO power shower of appendix C.4): MC@NLO with the start scale mu_Q^2, and
POWHEG-like Born events whose first emission is corrected to the real matrix
element.

The real matrix elements are written here from the textbook 2 -> 2 results
(q qbar -> Z g, and q g -> Z q by crossing), independently of the oracle's
closed forms of R - S and of the dipole sum S; the first-emission CDF of the
corrected shower is integrated from them over the real emission's phase space
in the initial-initial variables (x, v)."""
import math

import numpy as np
import pytest
from scipy import interpolate

from gapsinputs import records, toypdf, workloads
from oracle.pyoracle import Oracle

CF, TR = 4.0 / 3.0, 0.5
MZ = 91.1876


def textbook_r(kind, s, t, u, m2):
    """|M|^2 of the real emission over 8 pi alpha_s |M_B|^2 / m^2 and the
    colour factor: q qbar -> Z g (kind 0; t, u against the two quarks) and
    g q -> Z q (kind 1; u the gluon against the outgoing quark)."""
    if kind == 0:
        return (t * t + u * u + 2.0 * m2 * s) / (t * u)
    return -(s * s + u * u + 2.0 * m2 * t) / (s * u)


def test_dipole_sum_plus_printed_r_minus_s_is_the_real_matrix_element(oracles):
    """S (the oracle's dipole sum) + (R - S) (appendix C.2, printed) = R at
    random real configurations, for q qbar -> Z g and both gluon orientations."""
    o = oracles["nlo"]
    m2 = MZ * MZ
    rng = np.random.default_rng(3)
    for _ in range(200):
        x = rng.uniform(1e-3, 0.999)
        va = (1.0 - x) * rng.uniform(1e-4, 1.0 - 1e-4)
        sb = m2 / x
        ub, tb = -va * sb, -(1.0 - x - va) * sb  # ubar against beam A, tbar against beam B
        a_s = o.cfg["alphas_mz"]
        for kind, cf in ((0, CF), (1, TR), (2, TR)):
            pre = 8.0 * math.pi * a_s * cf / m2
            if kind == 0:
                rs = o.rs(0, sb, tb, ub, 1.0)
                ref = textbook_r(0, sb, tb, ub, m2)
            elif kind == 1:
                rs = o.rs(1, sb, tb, ub, 1.0)
                ref = textbook_r(1, sb, tb, ub, m2)
            else:
                rs = o.rs(1, sb, ub, tb, 1.0)
                ref = textbook_r(1, sb, ub, tb, m2)
            got = rs / pre + o.nlo_sub(kind, x, va)
            assert abs(got - ref) <= 1e-12 * abs(ref), (kind, x, va, got, ref)


def test_correction_factor_is_r_over_the_shower_density(oracles):
    """The first-emission factor of family A is R over both quarks' dipoles and
    of family B R over the gluon's dipole (their sum S pinned above); family A
    lies in [1/2, 1] and family B below the bound its overestimate carries."""
    o = oracles["nlo"]
    m2 = MZ * MZ
    xs = np.linspace(1e-3, 0.999, 199)
    worst_b, lo_a = 0.0, 2.0
    for x in xs:
        for f in np.linspace(1e-3, 1.0 - 1e-3, 101):
            v = (1.0 - x) * f
            sb = m2 / x
            ub, tb = -v * sb, -(1.0 - x - v) * sb
            ra = o.mec_ratio(0, x, v)
            rb = o.mec_ratio(1, x, v)
            assert abs(ra - textbook_r(0, sb, tb, ub, m2) / o.nlo_sub(0, x, v)) < 1e-12
            assert abs(rb - textbook_r(1, sb, tb, ub, m2) / o.nlo_sub(1, x, v)) < 1e-12 * rb
            lo_a = min(lo_a, ra)
            worst_b = max(worst_b, rb)
            assert 0.5 <= ra <= 1.0
    golden2 = ((1.0 + math.sqrt(5.0)) / 2.0) ** 2
    assert worst_b <= golden2 + 1e-12 and worst_b > golden2 - 5e-3
    assert o.mec_bound() > golden2


def _totals(ev):
    n = len(ev.w)
    h = (ev.flags & records.FLAG_HEVENT) != 0
    return (ev.w.sum() / n, ev.w.std() / math.sqrt(n), ev.w[h].sum() / n, ev.w[~h].sum() / n)


@pytest.fixture(scope="module")
def nlo_sets(oracles):
    n = 300_000
    return {k: oracles[k].hard_events(0, n, 1, max_slots=8) for k in ("nlo", "muq", "powheg")}


def test_start_scale_at_hadronic_s_is_the_power_shower(cfgs):
    """mu_Q^2 = S: no emission reaches it, so every event is the power
    shower's, bit for bit."""
    a = Oracle(cfgs["nlo"]).hard_events(0, 20000, 4, max_slots=8)
    b = Oracle(dict(cfgs["nlo"], matching=1, mu_q2=13000.0 ** 2)).hard_events(0, 20000, 4, max_slots=8)
    for name in a.fields():
        assert np.array_equal(getattr(a, name), getattr(b, name)), name


def test_start_scale_moves_the_dipoles_above_it(nlo_sets):
    """With mu_Q = mZ the total cross section is unchanged: what the H events
    gain (the dipole sum above mu_Q) the S events lose, and every event starts
    its shower at mu_Q^2."""
    t0, e0, h0, s0 = _totals(nlo_sets["nlo"])
    t1, e1, h1, s1 = _totals(nlo_sets["muq"])
    ev = nlo_sets["muq"]
    assert np.all(ev.t_start == MZ ** 2)
    assert np.all(nlo_sets["nlo"].t_start == 13000.0 ** 2)
    # the H events gain a sizeable amount (about half of R - S), the S events lose it
    assert h1 - h0 > 0.3 * h0
    assert abs((h1 - h0) + (s1 - s0)) < 4.0 * math.hypot(e0, e1), (h1 - h0, s1 - s0)
    assert abs(t1 - t0) < 4.0 * math.hypot(e0, e1)


def test_powheg_born_events_carry_the_nlo_cross_section(nlo_sets):
    """POWHEG-like events are Born events (four particles, flag MEC, the power
    shower's start) whose weights B + V + I + C + int (R - S) sum to the same
    NLO cross section as the S and H events; almost none are negative."""
    ev = nlo_sets["powheg"]
    assert np.all(ev.n == 4) and np.all(ev.flags == records.FLAG_MEC)
    assert np.all(ev.t_start == 13000.0 ** 2)
    t0, e0, h0, _ = _totals(nlo_sets["nlo"])
    t2, e2, _, _ = _totals(ev)
    assert abs(t2 - t0) < 4.0 * math.hypot(e0, e2), (t2, t0)
    # int (R - S) is the H events' total: a wrong share would move t2 by it
    assert abs(h0) > 15.0 * math.hypot(e0, e2)
    assert np.mean(ev.w < 0) < 0.01


def test_matching_is_rejected_where_undefined(cfgs):
    for key in ("ee", "dy"):
        with pytest.raises(ValueError):
            Oracle(dict(cfgs[key], matching=2)).hard_events(0, 10, 1)
    with pytest.raises(ValueError):
        Oracle(dict(cfgs["nlo"], matching=1, mu_q2=0.0)).hard_events(0, 10, 1)
    with pytest.raises(ValueError):
        Oracle(dict(cfgs["nlo"], matching=3)).hard_events(0, 10, 1)


# ---------------------------------------------------------------------------
# the corrected first emission against the POWHEG Sudakov of the real matrix
# element


class PDFv:
    """f(x, Q^2) from the grid's x f nodes with a library interpolator, with a
    scale per point."""

    def __init__(self, grid):
        lnx, lnq = toypdf.grid_axes()
        self.f = [interpolate.RegularGridInterpolator((lnq, lnx), grid[t].astype(np.float64),
                                                      bounds_error=False, fill_value=0.0) for t in range(8)]
        self.lq0, self.lq1, self.lx0 = lnq[0], lnq[-1], lnx[0]

    def __call__(self, tab, x, q2):
        x, q2 = np.broadcast_arrays(np.asarray(x, dtype=np.float64), np.asarray(q2, dtype=np.float64))
        lx = np.log(np.clip(x, 1e-300, None))
        lq = np.log(q2)
        ok = (x < 1.0) & (lx >= self.lx0) & (lq >= self.lq0) & (lq <= self.lq1)
        v = self.f[tab](np.stack([lq, lx], axis=-1))
        return np.where(ok, v / x, 0.0)


def alphas(t):
    b0 = 23.0 / (12.0 * math.pi)
    return 0.118 / (1.0 + 0.118 * b0 * np.log(t / MZ ** 2))


def emission_above(pdf, s, eta, tq, t, corrected=True, npts=160):
    """Integral over the real emissions of one leg (quark table tq at momentum
    fraction eta, Born invariant s) with kT^2 > t of R / B (corrected) or of
    the leg's dipoles over B (the shower's own density): R is q qbar -> Z g in
    the share of this leg's dipole (1 - x - v) / (1 - x) plus the
    gluon-initiated configuration, each with alpha_s and the PDF ratio at kT^2
    (the shower's scales); x in ln(1 - x), v in ln(v / (1 - x - v))."""
    GX, GWX = np.polynomial.legendre.leggauss(npts)
    r = t / s
    xmax = 1.0 + 2.0 * r - math.sqrt((1.0 + 2.0 * r) ** 2 - 1.0)
    if not xmax > eta:
        return 0.0
    ya, yb = math.log(1.0 - xmax), math.log(1.0 - eta)
    y = 0.5 * (yb - ya) * GX + 0.5 * (yb + ya)
    x = 1.0 - np.exp(y)
    jx = 0.5 * (yb - ya) * GWX * np.exp(y)
    omx = 1.0 - x
    disc = np.sqrt(np.clip(omx * omx - 4.0 * r * x, 0.0, None))
    vm, vp = 0.5 * (omx - disc), 0.5 * (omx + disc)
    wa, wb = np.log(vm / (omx - vm)), np.log(vp / (omx - vp))
    w = 0.5 * (wb - wa)[:, None] * GX[None, :] + 0.5 * (wb + wa)[:, None]
    X = x[:, None]
    O = omx[:, None]
    v = O / (1.0 + np.exp(-w))
    jv = 0.5 * (wb - wa)[:, None] * GWX[None, :] * v * (O - v) / O
    kt2 = v * (O - v) * s / X
    den = pdf(tq, eta, kt2)
    safe = np.where(den > 0, den, 1.0)
    rq = np.where(den > 0, pdf(tq, eta / X, kt2) / (X * safe), 0.0)
    rg = np.where(den > 0, pdf(0, eta / X, kt2) / (X * safe), 0.0)
    if corrected:
        kq = CF * (v * v + (O - v) ** 2 + 2.0 * X) / (v * (O - v)) * (O - v) / O
        kg = TR * (1.0 + v * v - 2.0 * X * (O - v)) / v
    else:
        kq = CF * (1.0 + X * X) / (O * v)
        kg = TR * (X * X + O * O) / v
    f = alphas(kt2) / (2.0 * math.pi) * (kq * rq + kg * rg)
    return float(np.sum(f * jv * jx[:, None]))


def replicate(ev, k, n):
    out = records.Events(n, ev.max_slots)
    for name in ev.fields():
        src = getattr(ev, name)
        if src.ndim == 1:
            getattr(out, name)[:] = src[k]
        else:
            getattr(out, name)[:] = src[:, k:k + 1]
    out.id[:] = np.arange(n)
    return out


FORMS = pytest.mark.parametrize("form", [dict(retain=False), dict(retain=True), dict(gen_select=True),
                                         dict(veto_max=True)], ids=["regenerate", "retain", "gen_select",
                                                                    "veto_max"])


@pytest.mark.slow
@FORMS
def test_corrected_first_emission_follows_the_real_matrix_element(oracles, cfgs, form):
    """Copies of one u ubar Born event: with the correction flag the CDF of the
    first emission scale is exp(-int_{kT^2 > t} R / B) summed over both legs,
    without it the same with the legs' dipoles in place of R (the shower's
    density), in every form of the competition; the two curves are resolved."""
    o, pdf = oracles["lo"], PDFv(cfgs["lo"]["pdf"])
    base = o.hard_events(0, 64, 3)
    k = next(e for e in range(64) if abs(base.pid[0, e]) == 2)
    n = 100_000
    ev = replicate(base, k, n)
    ea, eb = 2 * base.E[0, k] / 13000.0, 2 * base.E[1, k] / 13000.0
    s = ea * eb * 13000.0 ** 2
    ta = toypdf.TABLE_NAMES.index("u" if base.pid[0, k] == 2 else "ubar")
    tb = toypdf.TABLE_NAMES.index("u" if base.pid[1, k] == 2 else "ubar")
    tgrid = np.array([1.7, 3.0, 10.0, 30.0, 100.0, 300.0, 1000.0, 3e3, 1e4])
    curves = {c: np.array([math.exp(-emission_above(pdf, s, ea, ta, t, c) - emission_above(pdf, s, eb, tb, t, c))
                           for t in tgrid]) for c in (True, False)}
    tol = 4.5 * np.sqrt(np.maximum(curves[True] * (1 - curves[True]), 1e-4) / n) + 1e-3
    assert np.max(np.abs(curves[True] - curves[False]) - 2.0 * tol) > 0.0
    for corrected in (True, False):
        ev.flags[:] = records.FLAG_MEC if corrected else 0
        out = o.shower(ev, 5, nthreads=8, **form)
        assert int(out.n_viol.sum()) == 0
        emp = np.array([np.mean(out.t1 <= t) for t in tgrid])
        assert np.all(np.abs(emp - curves[corrected]) < tol), (corrected, emp, curves[corrected])
