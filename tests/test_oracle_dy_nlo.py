"""Pins of the oracle's NLO pp -> Z/photon -> e+e- events (process 4): the
real emission by the Kleiss trick and the subtraction by the dipoles with the
Born at mapped lepton momenta, against the textbook on-shell Z matrix elements
once the lepton angles are averaged (the lepton tensor integrates to the sum
over the vector boson's polarisations), pointwise in the collinear limits, and
the balance of S and H events against the on-shell Z workload at the pole."""
import math

import numpy as np
import pytest

from gapsinputs import records
from oracle.pyoracle import Oracle

CF, TR = 4.0 / 3.0, 0.5


def textbook(kind, s, t, u, m2):
    """q qbar -> V g (kind 0) and the crossed g q -> V q with u against the gluon."""
    if kind == 0:
        return (t * t + u * u + 2.0 * m2 * s) / (t * u)
    return -(s * s + u * u + 2.0 * m2 * t) / (s * u)


CS, WC = np.polynomial.legendre.leggauss(6)
PHIS = (np.arange(8) + 0.5) / 8


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("o2", [0, 1])
def test_lepton_average_is_the_z_matrix_element(oracles, kind, o2):
    """<R>_leptons = <|M_0|^2>_leptons * 8 pi alpha_s C / m^2 * textbook R, and
    the same for the dipole sum with the on-shell dipoles, at several real
    configurations and flavours (<|M_0|^2> = (a + b) / 3)."""
    o = oracles["dynlo"]
    a_s = o.cfg["alphas_mz"]
    for f, (m, x, y, fv) in ((2, (85.0, 0.3, 0.2, 0.1)), (1, (95.0, 0.05, -1.0, 0.6)), (5, (70.0, 0.7, 0.5, 0.2)),
                             (4, (110.0, 0.01, 1.5, 0.95))):
        m2, v = m * m, fv * (1.0 - x)
        R = S = 0.0
        for c, w in zip(CS, WC):
            for u in PHIS:
                r = o.dy_real(f, kind, o2, m2, x, y, v, 0.4, c, u)
                R += w * r[0] / 16.0
                S += w * r[1] / 16.0
        al, be = r[2], r[3]
        sb = m2 / x
        ub, tb = -v * sb, -(1.0 - x - v) * sb
        X = textbook(kind, sb, tb, ub, m2) if kind < 2 else textbook(1, sb, ub, tb, m2)
        pre = (al + be) / 3.0 * 8.0 * math.pi * a_s * (CF if kind == 0 else TR) / m2
        assert abs(R / (pre * X) - 1.0) < 1e-12
        assert abs(S / (pre * o.nlo_sub(kind, x, v)) - 1.0) < 1e-12


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_collinear_limits(oracles, kind):
    """R / S -> 1 pointwise (fixed lepton angles) as the emission becomes
    collinear to the emitting beam, as the square root of v (the terms linear
    in the transverse momentum that the azimuthal average removes)."""
    o = oracles["dynlo"]
    for o2 in (0, 1):
        d = []
        for v in (1e-4, 1e-6):
            x = 0.3
            vv = v * (1 - x) if kind != 2 else (1 - x) * (1 - v)
            r = o.dy_real(3, kind, o2, 88.0 ** 2, x, -0.4, vv, 1.1, -0.35, 0.8)
            d.append(abs(r[0] / r[1] - 1.0))
        assert d[1] < 2e-3 and d[1] < 0.15 * d[0]


def test_events_and_the_balance_of_s_and_h(cfgs):
    """In a narrow window at the pole the H events' share of the NLO cross
    section and their emission spectrum are the on-shell Z workload's (the
    lepton-averaged R - S and Born are the Z's), and the events are well
    formed: leptons in the window, H events with a parton, the S fraction p_S."""
    n = 300_000
    win = dict(mll_min=91.0, mll_max=91.4)
    dy = Oracle(dict(cfgs["dynlo"], **win)).hard_events(0, n, 1, max_slots=8)
    z = Oracle(cfgs["nlo"]).hard_events(0, n, 1, max_slots=8)
    for ev in (dy, z):
        assert np.all(np.isfinite(ev.w))
    h = (dy.flags & records.FLAG_HEVENT) != 0
    assert abs(h.mean() - 0.25) < 0.005
    assert np.all(dy.n[h] == 5) and np.all(dy.n[~h] == 4)
    sl = np.where(h, 3, 2)
    idx = np.arange(n)
    em = np.stack([dy.E[sl, idx], dy.px[sl, idx], dy.py[sl, idx], dy.pz[sl, idx]])
    ep = np.stack([dy.E[sl + 1, idx], dy.px[sl + 1, idx], dy.py[sl + 1, idx], dy.pz[sl + 1, idx]])
    P = em + ep
    m = np.sqrt(P[0] ** 2 - P[1] ** 2 - P[2] ** 2 - P[3] ** 2)
    assert np.all((m > 91.0 - 1e-6) & (m < 91.4 + 1e-6))
    hz = (z.flags & records.FLAG_HEVENT) != 0
    fdy, fz = dy.w[h].sum() / dy.w.sum(), z.w[hz].sum() / z.w.sum()
    edy = dy.w[h].std() * math.sqrt(h.sum()) / dy.w.sum()
    ez = z.w[hz].std() * math.sqrt(hz.sum()) / z.w.sum()
    assert abs(fdy - fz) < 4.0 * math.hypot(edy, ez) + 2e-3, (fdy, fz, edy, ez)
    assert fz > 0.02
    # the H events' emission spectrum (the parton's pT, as a fraction of the
    # NLO cross section) is the Z's: chi^2 over 12 bins
    edges = np.array([0.0, 1.0, 2.0, 4.0, 7.0, 10.0, 15.0, 20.0, 30.0, 45.0, 70.0, 120.0, 300.0])

    def spectrum(ev, hh):
        pt = np.hypot(ev.px[2], ev.py[2])[hh]
        w = ev.w[hh] / ev.w.sum()
        return np.histogram(pt, edges, weights=w)[0], np.histogram(pt, edges, weights=w * w)[0]

    (a, va), (b, vb) = spectrum(dy, h), spectrum(z, hz)
    chi2 = float(np.sum((a - b) ** 2 / (va + vb)))
    from scipy import stats
    assert stats.chi2.sf(chi2, len(edges) - 1) > 1e-3, (chi2, a, b)
