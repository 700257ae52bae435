"""Pins of the oracle's LO pp -> Z/photon -> e+e- events (the second
workload: the photon, the Z and their interference).  The angular and mass
distributions of the generated events are checked against the cross section
written in helicity amplitudes, A_ij = Q_q Q_e + g_i^q g_j^e chi' (chiral
couplings g_L = T3 - Q sin^2, g_R = -Q sin^2, chi' = s / (s - mZ^2 + i mZ GZ) /
(sin^2 cos^2)): (1 + cos^2) sum |A_ij|^2 + 2 cos (|A_LL|^2 + |A_RR|^2 - |A_LR|^2
- |A_RL|^2), and at the pole against the electroweak asymmetry parameters."""
import math

import numpy as np
import pytest

from gapsinputs import workloads

# PDF table of each quark and antiquark flavour (the grid's layout)
TAB = {1: 1, 2: 2, 3: 3, 4: 4, 5: 5, -1: 6, -2: 7, -3: 3, -4: 4, -5: 5}


def helicity_f12(up, m2, cfg):
    """(sum |A|^2 / 4, (|A_LL|^2 + |A_RR|^2 - |A_LR|^2 - |A_RL|^2) / 4)."""
    sw2, mz, gz = cfg["sw2"], cfg["mz"], cfg["gz"]
    Qq, T3 = (2.0 / 3.0, 0.5) if up else (-1.0 / 3.0, -0.5)
    Qe, T3e = -1.0, -0.5
    gq = {"L": T3 - Qq * sw2, "R": -Qq * sw2}
    ge = {"L": T3e - Qe * sw2, "R": -Qe * sw2}
    chi = m2 / complex(m2 - mz * mz, mz * gz) / (sw2 * (1.0 - sw2))
    A = {(i, j): abs(Qq * Qe + gq[i] * ge[j] * chi) ** 2 for i in "LR" for j in "LR"}
    return sum(A.values()) / 4.0, (A["L", "L"] + A["R", "R"] - A["L", "R"] - A["R", "L"]) / 4.0


@pytest.fixture(scope="module")
def dy(oracles, cfgs):
    o = oracles["dy"]
    n = 200_000
    ev = o.hard_events(0, n, 1)
    assert np.all(ev.flags == 0) and np.all(ev.n == 4)
    pa = ev.pid[0]
    up = (np.abs(pa) % 2) == 0
    sq = np.where(pa > 0, 1.0, -1.0)  # the quark moves along +z when beam A carries it
    em = np.stack([ev.E[2], ev.px[2], ev.py[2], ev.pz[2]])
    ep = np.stack([ev.E[3], ev.px[3], ev.py[3], ev.pz[3]])
    P = em + ep
    m2 = P[0] ** 2 - P[1] ** 2 - P[2] ** 2 - P[3] ** 2
    # the electron in the pair's rest frame (the pair moves along z at LO)
    b = P[3] / P[0]
    g = 1.0 / np.sqrt(1.0 - b * b)
    pz = g * (em[3] - b * em[0])
    pabs = np.sqrt(em[1] ** 2 + em[2] ** 2 + pz ** 2)
    c = sq * pz / pabs
    return o, cfgs["dy"], np.sqrt(m2), up, c, ev


def test_angular_distribution(dy):
    """Each event's cos(theta*) against its expectation F2 / (2 F1) from the
    helicity amplitudes at its mass and flavour (variance 2/5 - mean^2)."""
    o, cfg, m, up, c, _ = dy
    F = np.array([helicity_f12(u, mm * mm, cfg) for u, mm in zip(up, m)])
    mu = F[:, 1] / (2.0 * F[:, 0])
    z = np.sum(c - mu) / math.sqrt(np.sum(0.4 - mu * mu))
    assert abs(z) < 4.0, z
    # the asymmetry changes sign across the pole: negative below (interference)
    lo, hi = m < 80.0, m > 100.0
    assert c[lo].mean() < -0.05 and c[hi].mean() > 0.1
    # the second moment of 1 + cos^2 plus the odd term
    assert abs(np.mean(c * c) - 0.4) < 0.01


def test_pole_asymmetry(dy):
    """At the pole the Z dominates: <cos theta*> = A_q A_e / 2 with
    A_f = 2 v a / (v^2 + a^2) (v = T3 - 2 Q sin^2, a = T3)."""
    o, cfg, m, up, c, _ = dy
    sw2 = cfg["sw2"]

    def A(T3, Q):
        v, a = T3 - 2.0 * Q * sw2, T3
        return 2.0 * v * a / (v * v + a * a)

    Ae = A(-0.5, -1.0)
    win = np.abs(m - cfg["mz"]) < 0.5
    for sel, Aq in ((up, A(0.5, 2.0 / 3.0)), (~up, A(-0.5, -1.0 / 3.0))):
        s = win & sel
        mean, err = c[s].mean(), math.sqrt(0.4 / s.sum())
        assert abs(mean - 0.5 * Aq * Ae) < 4.0 * err + 2e-3, (mean, 0.5 * Aq * Ae, err)


def test_mass_spectrum(dy):
    """The pair-mass histogram against d sigma / dm = 2m / m^4 * sum over
    flavours and orientations of x f x f * F1, integrated over the rapidity on
    a grid with the oracle's PDF lookup."""
    o, cfg, m, _, _, _ = dy
    edges = np.linspace(cfg["mll_min"], cfg["mll_max"], 26)
    h, _ = np.histogram(m, edges)
    S = cfg["sqrt_s"]
    exp = []
    for k in range(25):
        acc = 0.0
        for mm in np.linspace(edges[k], edges[k + 1], 5)[:4] + (edges[1] - edges[0]) / 8.0:
            m2 = mm * mm
            Y = math.log(S / mm)
            ys = np.linspace(-Y, Y, 241)
            tot = np.zeros_like(ys)
            for f in range(1, 6):
                F1, _ = helicity_f12(f % 2 == 0, m2, cfg)
                for i, y in enumerate(ys):
                    x1, x2 = mm / S * math.exp(y), mm / S * math.exp(-y)
                    tot[i] += F1 * (o.pdf_xf(TAB[f], x1, m2) * o.pdf_xf(TAB[-f], x2, m2) +
                                    o.pdf_xf(TAB[-f], x1, m2) * o.pdf_xf(TAB[f], x2, m2))
            acc += np.trapezoid(tot, ys) * 2.0 * mm / (m2 * m2)
        exp.append(acc)
    exp = np.array(exp) * h.sum() / np.sum(exp)
    chi2 = np.sum((h - exp) ** 2 / exp)
    from scipy import stats
    p = stats.chi2.sf(chi2, 24)
    assert p > 1e-3, (chi2, h, exp.round())
