"""Pins of the oracle's NLO building blocks (appendix C) and observables."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from gapsinputs import records

CF, TR = 4.0 / 3.0, 0.5


def test_bvi_factor_matches_printed_value(oracles):
    # the paper states that the B+V+I term multiplies the Born by about 1.05
    assert oracles["nlo"].bvi_factor() == pytest.approx(1.05, abs=1e-3)


def test_aqq_from_delta_coefficients(oracles):
    # A^qq collects the delta(1-x) coefficients of Kbar, Ktilde and P (logs 0)
    a = 0.118
    delta_coeff = -(5.0 - math.pi ** 2) - math.pi ** 2 / 3.0
    assert oracles["nlo"].aqq() == pytest.approx(CF * a / (2 * math.pi) * delta_coeff, rel=1e-14)


@pytest.mark.parametrize("x", [0.0, 1e-6, 0.1, 0.3, 0.5, 0.51, 0.9, 0.999999, 1.0, -0.5, -3.0])
def test_li2_matches_library(oracles, x):
    assert oracles["nlo"].li2(x) == pytest.approx(float(special.spence(1.0 - x)), rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("eta", [1e-4, 0.01, 0.2, 0.6, 0.95])
def test_bqq_is_integral_of_gqq(oracles, eta):
    o = oracles["nlo"]
    val, _ = integrate.quad(o.gqq, 0.0, eta, limit=400, epsabs=1e-13, epsrel=1e-11)
    assert o.bqq(eta) == pytest.approx(val, rel=1e-8, abs=1e-12)


def test_real_minus_subtraction_identities(oracles):
    """R - S in closed form equals the printed real matrix elements minus the
    printed dipoles, in the II-map Mandelstams t = -(1-x-v)s, u = -v s."""
    o = oracles["nlo"]
    rng = np.random.default_rng(2)
    a = 0.118
    m2 = 91.1876 ** 2
    mb2 = 1.234e-3  # any Born |M|^2: both sides are linear in it
    for _ in range(200):
        x = rng.uniform(0.01, 0.99)
        v = rng.uniform(1e-3, 1 - x - 1e-3)
        s = m2 / x
        t, u = -(1 - x - v) * s, -v * s
        R_qq = 8 * math.pi * a * CF / m2 * mb2 * (t / u + u / t + 2 * m2 * s / (t * u))
        # printed dipoles (with the printed 1/u, negative here); the subtraction
        # term that cancels the collinear poles of R is S = -(D(u) + D(t))
        D = lambda uu: 8 * math.pi * a * CF * mb2 / x / uu * (2 / (1 - x) - (1 + x))
        S_qq = -D(u) - D(t)
        assert o.rs(0, s, t, u, mb2) == pytest.approx(R_qq - S_qq, rel=1e-9)
        R_gq = 8 * math.pi * a * TR / m2 * mb2 * (-u / s - s / u - 2 * m2 * t / (s * u))
        S_gq = 8 * math.pi * a * TR / m2 * mb2 * (-m2 / x) / u * (1 - 2 * x * (1 - x))
        assert o.rs(1, s, t, u, mb2) == pytest.approx(R_gq - S_gq, rel=1e-9)


def test_hard_events_shapes(oracles):
    lo = oracles["lo"].hard_events(0, 4000, 1)
    assert not np.any(lo.flags & records.FLAG_HARDFAIL)
    mll = []
    cos = []
    for e in range(lo.cap):
        P = lo.momenta(e)
        Z = P[2] + P[3]
        mll.append(math.sqrt(Z[0] ** 2 - (Z[1:] ** 2).sum()))
        # lepton angle in the Z rest frame along the beam
        bz = Z[3] / Z[0]
        g = 1 / math.sqrt(1 - bz * bz)
        ez, pz = g * (P[2][0] - bz * P[2][3]), g * (P[2][3] - bz * P[2][0])
        cos.append(pz / ez)
    mll = np.array(mll)
    assert mll.min() >= 66.0 and mll.max() <= 116.0
    # Breit-Wigner core: most events within a few widths of the Z mass
    assert np.mean(np.abs(mll - 91.1876) < 5.0) > 0.6
    h, _ = np.histogram(cos, bins=10, range=(-1, 1))
    edges = np.linspace(-1, 1, 11)
    cdf = lambda c: (c + c ** 3 / 3 + 4 / 3) / (8 / 3)
    exp = np.diff(cdf(edges)) * len(cos)
    assert ((h - exp) ** 2 / exp).sum() < 30.0

    nlo = oracles["nlo"].hard_events(0, 4000, 1)
    hfrac = np.mean((nlo.flags & records.FLAG_HEVENT) > 0)
    assert 0.22 < hfrac < 0.28  # p_s = 0.75
    for e in range(0, 4000, 13):
        P = nlo.momenta(e)
        st = nlo.status[: nlo.n[e], e]
        bal = (P * st[:, None]).sum(0)
        assert np.abs(bal).max() < 1e-9 * 13000
        nn = nlo.n[e]
        Z = P[nn - 2] + P[nn - 1]
        assert math.sqrt(Z[0] ** 2 - (Z[1:] ** 2).sum()) == pytest.approx(91.1876, rel=1e-9)
    # H events: q qbar -> Z g carry negative weight and g q -> Z q positive, by
    # the closed forms of R - S (S events may go negative through the one-point
    # sample of the collinear integral)
    h = (nlo.flags & records.FLAG_HEVENT) > 0
    assert np.all(nlo.w[h & (nlo.pid[2] == 21)] < 0)
    assert np.all(nlo.w[h & (nlo.pid[2] != 21)] > 0)
    assert np.mean(nlo.w[~h] > 0) > 0.95


def _single(cap_slots, parts):
    ev = records.Events(1, cap_slots)
    ev.n[0] = len(parts)
    for q, (p, pid, st) in enumerate(parts):
        ev.E[q, 0], ev.px[q, 0], ev.py[q, 0], ev.pz[q, 0] = p
        ev.pid[q, 0], ev.status[q, 0] = pid, st
    return ev


def test_thrust_and_durham_hand_events(oracles):
    o = oracles["ee"]
    E = 45.6
    # back to back: T = 1, y23 = 0
    ev = _single(8, [((E, 0, 0, E), 1, 1), ((E, 0, 0, -E), -1, 1)])
    obs = o.observables(ev)
    assert obs[0, 0] == pytest.approx(0.0, abs=1e-15)
    # symmetric three-parton (Mercedes) event: T = 2/3, y23 = 2 E^2 (1 - cos 120) / Evis^2 = 1/3
    Ep = 91.2 / 3
    parts = []
    for k in range(3):
        ph = 2 * math.pi * k / 3
        parts.append(((Ep, Ep * math.cos(ph), Ep * math.sin(ph), 0.0), 21, 1))
    obs = o.observables(_single(8, parts))
    assert 1 - obs[0, 0] == pytest.approx(2.0 / 3.0, rel=1e-12)
    assert obs[0, 1] == pytest.approx(2 * Ep * Ep * 1.5 / (3 * Ep) ** 2, rel=1e-12)


def test_antikt_hand_event(oracles):
    o = oracles["lo"]
    def pt_eta_phi(pt, eta, phi):
        return (pt * math.cosh(eta), pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta))
    parts = [((100.0, 0, 0, 100.0), 2, -1), ((100.0, 0, 0, -100.0), -2, -1),
             (pt_eta_phi(40.0, 0.1, 0.0), 21, 1), (pt_eta_phi(10.0, 0.3, 0.1), 21, 1),
             (pt_eta_phi(30.0, -1.0, 3.0), 21, 1), (pt_eta_phi(3.0, 2.0, 1.0), 21, 1)]
    ev = _single(8, parts)
    obs = o.observables(ev)
    # first two partons merge (Delta R ~ 0.22 < 0.4): jets ~50, 30 (>5), 3 (<5)
    assert obs[0, 4] == 2
    assert obs[0, 5] == pytest.approx(49.9, abs=0.2)
    assert obs[0, 7] == pytest.approx(30.0, rel=1e-12)
