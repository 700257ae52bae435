"""Pins of the oracle's building blocks: random numbers, coupling, PDF grid.

Each check compares the oracle with something other than itself: published
known-answer vectors, a library interpolator, a differential equation the
coupling must satisfy, or the analytic toy PDF's sum rule.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, interpolate

from gapsinputs import toypdf
from oracle import pyoracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(w, 16) for w in line.split()])
    assert len(rows) == 3
    for r in rows:
        assert pyoracle.philox4x32(r[0:4], r[4:6]) == r[6:10]


def test_philox_uniforms_open_interval_and_flat():
    # u = (w + 1/2) 2^-32 never reaches 0 or 1; words are flat in [0, 2^32)
    words = []
    for c in range(4000):
        words += pyoracle.philox4x32([c, 0, 7, 0], [1, 0])
    u = (np.array(words, dtype=np.float64) + 0.5) * 2.0 ** -32
    assert u.min() > 0.0 and u.max() < 1.0
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    expect = len(u) / 20
    chi2 = ((hist - expect) ** 2 / expect).sum()
    assert chi2 < 50.0  # 19 dof


def test_alphas_rge_and_reference(oracles):
    o = oracles["lo"]
    mz2 = 91.1876 ** 2
    assert o.alphas(mz2) == pytest.approx(0.118, rel=1e-15)
    b0 = (33.0 - 2 * 5) / (12.0 * math.pi)
    for t in (1.0, 10.0, 1e3, 1e6):
        h = 1e-4
        d = (o.alphas(t * math.exp(h)) - o.alphas(t * math.exp(-h))) / (2 * h)
        a = o.alphas(t)
        assert d == pytest.approx(-b0 * a * a, rel=1e-6)
    # the overestimate alpha_s(t_c) at t_c = 1 GeV^2
    assert o.alphas(1.0) == pytest.approx(0.336931, abs=2e-6)


def test_coupling_and_pdf_at_ln_t(oracles):
    """The veto weight evaluates the coupling and the PDF interpolation at the
    trial's ln t: the same functions as at t, to rounding (the coupling's
    logarithm ln(t / mZ^2) taken as ln t - ln mZ^2), and exactly the same PDF
    value when the ln Q^2 given is log(Q^2)."""
    o = oracles["lo"]
    for t in (1.0, 2.5, 91.1876 ** 2, 1e4, 1e7):
        lnt = math.log(t)
        assert o.alphas_ln(lnt) == pytest.approx(o.alphas(t), rel=1e-14)
    assert o.alphas_ln(math.log(91.1876 ** 2)) == pytest.approx(0.118, rel=1e-15)
    for tab in (0, 1, 2, 7):
        for x, q2 in ((1e-4, 3.0), (0.05, 91.0), (0.3, 1e4), (0.9, 2e6)):
            assert o.pdf_f_lq(tab, x, q2, math.log(q2)) == o.pdf_xf(tab, x, q2) / x


def test_pdf_nodes_exact(oracles, cfgs):
    o, grid = oracles["lo"], cfgs["lo"]["pdf"]
    lnx, lnq = toypdf.grid_axes()
    rng = np.random.default_rng(3)
    for _ in range(200):
        t = int(rng.integers(0, 8))
        i = int(rng.integers(0, toypdf.NX - 1))
        j = int(rng.integers(0, toypdf.NQ))
        x, q2 = math.exp(lnx[i]), math.exp(lnq[j])
        if j == toypdf.NQ - 1:
            q2 = math.exp(lnq[j]) * (1 - 1e-15)
        assert o.pdf_xf(t, x, q2) == pytest.approx(float(grid[t, j, i]), rel=1e-9, abs=1e-30)


def test_pdf_matches_library_bilinear(oracles, cfgs):
    o, grid = oracles["nlo"], cfgs["nlo"]["pdf"]
    lnx, lnq = toypdf.grid_axes()
    rng = np.random.default_rng(5)
    for t in range(8):
        f = interpolate.RegularGridInterpolator((lnq, lnx), grid[t].astype(np.float64), method="linear")
        for _ in range(100):
            lx = rng.uniform(lnx[0], -1e-6)
            lq = rng.uniform(lnq[0], lnq[-1])
            ref = float(f([[lq, lx]])[0])
            got = o.pdf_xf(t, math.exp(lx), math.exp(lq))
            assert got == pytest.approx(ref, rel=1e-10, abs=1e-14)


def test_pdf_zero_outside(oracles):
    o = oracles["lo"]
    for t in range(8):
        assert o.pdf_xf(t, 1.0, 100.0) == 0.0
        assert o.pdf_xf(t, 1.5, 100.0) == 0.0
        assert o.pdf_xf(t, 5e-8, 100.0) == 0.0
        assert o.pdf_xf(t, 0.1, 1.0) == 0.0
        assert o.pdf_xf(t, 0.1, 2e8) == 0.0
    # heavy flavours vanish at their threshold rows
    assert o.pdf_xf(4, 0.01, 1.69 * (1 + 1e-12)) == pytest.approx(0.0, abs=1e-6)
    assert o.pdf_xf(5, 0.01, 15.0) == 0.0


@pytest.mark.parametrize("q2", [1.69, 100.0, 8315.0, 1.0e6, 1.69e8])
def test_toy_pdf_momentum_sum_rule(q2):
    tot = 0.0
    for t in range(toypdf.NTAB):
        val, _ = integrate.quad(lambda x: float(toypdf.analytic_xf(t, x, q2)), 0.0, 1.0,
                                limit=400, points=[1e-6, 1e-3, 0.1])
        tot += toypdf.TABLE_MULT[t] * val
    assert tot == pytest.approx(1.0, abs=2e-6)


def test_overestimate_table_quarter_octaves(oracles):
    b = oracles["nlo"].bounds()
    pos = b[b > 0]
    k = np.log2(pos) * 4
    assert np.allclose(k, np.round(k), atol=1e-9)
    # every transition the shower can reach has a finite, positive bound
    assert np.all(b[0:8] > 0)          # final-initial spectators
    assert np.all(b[8 + 1:8 + 8] > 0)  # q <- q
    assert np.all(b[24] > 0)           # g <- g
