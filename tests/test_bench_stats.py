"""The benchmark's histogram statistics (host code, no GPU): the chi^2 of two
independent weighted histograms and Fisher's combination of p-values, pinned
by hand-computed values, closed forms and their null distributions."""
import numpy as np
import pytest
from scipy import stats

import bench


def _hists(rng, n, shift=0.0, neg=0.08):
    """Weighted histograms of the three benchmark observables from n events
    with signed weights (a fraction neg negative, as NLO events have)."""
    w = np.where(rng.random(n) < neg, -1.0, 1.0) * rng.uniform(0.5, 1.5, n)
    out = []
    for name, _, lo, hi, nb in bench.HIST_SPEC:
        if name == "n_jets":
            x = rng.poisson(1.5 + shift, n).astype(float)
        else:
            x = rng.exponential((hi - lo) / 4.0 * (1.0 + shift), n) + lo
        a, _ = np.histogram(x, bins=nb, range=(lo, hi), weights=w)
        a2, _ = np.histogram(x, bins=nb, range=(lo, hi), weights=w * w)
        out.append((a, a2))
    return out


def test_chi2_hand_computed():
    """(a - b)^2 / (sigma_a^2 + sigma_b^2) summed over the bins with content,
    divided by their number."""
    spec_bins = [nb for *_, nb in bench.HIST_SPEC]
    ref, oth = [], []
    for nb in spec_bins:
        a = np.zeros(nb); a2 = np.zeros(nb); b = np.zeros(nb); b2 = np.zeros(nb)
        a[0], a2[0], b[0], b2[0] = 1.0, 1.0, 2.0, 2.0   # (1)^2 / 3
        a[1], a2[1], b[1], b2[1] = 4.0, 2.0, 4.0, 2.0   # 0
        ref.append((a, a2)); oth.append((b, b2))
    c = bench.chi2(ref, oth)
    for name, *_ in bench.HIST_SPEC:
        assert c[name]["ndf"] == 2
        assert c[name]["chi2_ndf"] == pytest.approx((1.0 / 3.0) / 2.0, rel=1e-15)
        assert c[name]["p_value"] == pytest.approx(stats.chi2.sf(1.0 / 3.0, 2), rel=1e-12)
        assert c[name]["pulls"][0] == round(1.0 / np.sqrt(3.0), 2)


def test_chi2_p_values_uniform_under_the_null():
    """Two independent samples of one distribution with signed weights: the
    p-values are uniform (Kolmogorov-Smirnov), and the gates pass at their
    stated rates."""
    rng = np.random.default_rng(7)
    ps = {name: [] for name, *_ in bench.HIST_SPEC}
    for _ in range(300):
        c = bench.chi2(_hists(rng, 20000), _hists(rng, 20000))
        for name, *_ in bench.HIST_SPEC:
            ps[name].append(c[name]["p_value"])
    for name, p in ps.items():
        assert stats.kstest(p, "uniform").pvalue > 0.001, name
        assert 0.0 <= np.mean(np.asarray(p) < 0.01) < 0.04, name


def test_chi2_detects_a_shift():
    rng = np.random.default_rng(8)
    c = bench.chi2(_hists(rng, 200000), _hists(rng, 200000, shift=0.05))
    assert c["z_pt"]["p_value"] < 1e-6 and not c["gate_p_above_0_01"]


def test_fisher_closed_forms():
    """One p-value combines to itself (chi^2 with 2 degrees of freedom has
    the tail exp(-x/2)); k p-values equal to p give the tail of chi^2 with
    2 k degrees of freedom at -2 k ln p."""
    for p in (0.9, 0.37, 0.01, 1e-9):
        assert bench.fisher_p([p]) == pytest.approx(p, rel=1e-12)
    k, p = 5, 0.5
    assert bench.fisher_p([p] * k) == pytest.approx(stats.chi2.sf(-2 * k * np.log(p), 2 * k), rel=1e-12)
    # order does not matter; a single tiny p dominates
    assert bench.fisher_p([0.2, 0.7, 0.5]) == pytest.approx(bench.fisher_p([0.5, 0.2, 0.7]), rel=1e-15)
    assert bench.fisher_p([1e-12, 0.9, 0.9, 0.9, 0.9]) < 1e-6


def test_fisher_uniform_under_the_null():
    rng = np.random.default_rng(9)
    comb = [bench.fisher_p(rng.random(5)) for _ in range(4000)]
    assert stats.kstest(comb, "uniform").pvalue > 0.001
