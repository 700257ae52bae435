"""Histogram agreement of two weighted samples: chi^2 over the bins that have
content in either sample, with the variance of each bin from its sum of
squared weights (independent samples; samples that share their hard events
are positively correlated, which only makes the test conservative)."""
import numpy as np
from scipy import stats


def chi2_compare(xa, xb, wa, wb, edges):
    """Returns (chi2, ndf, p-value)."""
    a, _ = np.histogram(xa, edges, weights=wa)
    a2, _ = np.histogram(xa, edges, weights=wa * wa)
    b, _ = np.histogram(xb, edges, weights=wb)
    b2, _ = np.histogram(xb, edges, weights=wb * wb)
    m = (a2 + b2) > 0
    chi = float(np.sum((a[m] - b[m]) ** 2 / (a2[m] + b2[m])))
    ndf = int(m.sum())
    return chi, ndf, float(stats.chi2.sf(chi, ndf))
