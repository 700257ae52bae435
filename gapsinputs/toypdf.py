"""Synthetic stand-in for the CT14lo grid: a toy proton PDF tabulated on a
100 (ln x) x 50 (ln Q^2) grid, node values x*f(x,Q^2) stored as float32.

This module is an *input generator*: it produces the data table that both the
CPU oracle and the GPU library read (as the paper's generator reads an LHAPDF
grid, section 2 and section 4.1).  It contains none of the shower arithmetic:
interpolation, PDF ratios and overestimates live separately in each of the two
implementations.

Functional form (one power law per table, as fixed for the toy PDF):

    x f_T(x, Q^2) = A_T(s) * x^(1 - a_T(s)) * (1 - x)^(b_T(s))

with the evolution variable s = ln[ ln(Q^2/L^2) / ln(Q0^2/L^2) ], L = 0.088 GeV
and Q0 = 1.3 GeV (the lower edge of the grid, the CT14lo boundary analogue).
A_T is fixed by the momentum fraction M_T(s) the table carries:
integral_0^1 x f_T dx = A_T * B(2 - a_T, 1 + b_T) = M_T, and the M_T sum to one
(s, c and b tables count twice: quark and antiquark share them).  Charm and
bottom vanish at and below their masses and grow like ln(Q^2/m^2) above.

Table order (index): 0 g, 1 d, 2 u, 3 s (= sbar), 4 c (= cbar), 5 b (= bbar),
6 dbar, 7 ubar.
"""
from __future__ import annotations

import math

import numpy as np

NTAB = 8
NX = 100
NQ = 50
X_MIN = 1e-7
Q2_MIN = 1.69          # (1.3 GeV)^2
Q2_MAX = 1.69e8        # (13 TeV)^2
LAMBDA2 = 0.088 ** 2
M_C = 1.3
M_B = 4.75

TABLE_NAMES = ("g", "d", "u", "s", "c", "b", "dbar", "ubar")
# multiplicity of each table in the momentum sum rule
TABLE_MULT = (1, 1, 1, 2, 2, 2, 1, 1)


def _evol_s(q2: float) -> float:
    return math.log(math.log(q2 / LAMBDA2) / math.log(Q2_MIN / LAMBDA2))


def _shape(s: float, q2: float):
    """Per-table (a, b, M) at evolution variable s (Q^2 = q2)."""
    sat = s / (1.0 + s)
    a = np.empty(NTAB)
    b = np.empty(NTAB)
    m = np.empty(NTAB)
    # gluon
    a[0], b[0], m[0] = 1.15 + 0.08 * s, 4.5 + 1.0 * s, 0.40 + 0.06 * sat
    # sea-like tables: s, c, b, dbar, ubar
    for t in (3, 4, 5, 6, 7):
        a[t], b[t] = 1.12 + 0.08 * s, 6.0 + 1.0 * s
    m[3] = 0.020 + 0.012 * sat
    lc = math.log(q2 / M_C ** 2) if q2 > M_C ** 2 else 0.0
    lb = math.log(q2 / M_B ** 2) if q2 > M_B ** 2 else 0.0
    m[4] = 0.018 * (1.0 - math.exp(-lc))
    m[5] = 0.014 * (1.0 - math.exp(-lb))
    m[6] = 0.036 + 0.010 * sat
    m[7] = 0.030 + 0.010 * sat
    # valence-dominated u, d share the rest of the momentum
    rest = 1.0 - m[0] - m[6] - m[7] - 2.0 * (m[3] + m[4] + m[5])
    a[2], b[2], m[2] = 0.75 + 0.10 * s, 3.0 + 0.9 * s, 0.66 * rest
    a[1], b[1], m[1] = 0.78 + 0.10 * s, 3.6 + 0.9 * s, 0.34 * rest
    return a, b, m


def _beta(p: float, q: float) -> float:
    return math.exp(math.lgamma(p) + math.lgamma(q) - math.lgamma(p + q))


def analytic_xf(tab: int, x, q2: float):
    """x f_T(x, Q^2) of the analytic toy form (numpy, float64)."""
    s = _evol_s(q2)
    a, b, m = _shape(s, q2)
    if m[tab] <= 0.0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    norm = m[tab] / _beta(2.0 - a[tab], 1.0 + b[tab])
    x = np.asarray(x, dtype=np.float64)
    return norm * x ** (1.0 - a[tab]) * (1.0 - x) ** b[tab]


def momentum_fractions(q2: float):
    """Per-table momentum fraction M_T at Q^2 (the sum rule weights)."""
    return _shape(_evol_s(q2), q2)[2]


def grid_axes():
    """Node coordinates: ln x (NX, last node x = 1) and ln Q^2 (NQ)."""
    lnx = np.linspace(math.log(X_MIN), 0.0, NX)
    lnq2 = np.linspace(math.log(Q2_MIN), math.log(Q2_MAX), NQ)
    return lnx, lnq2


def make_grid() -> np.ndarray:
    """float32 array [NTAB][NQ][NX] of node values x*f at (x_i, Q^2_j)."""
    lnx, lnq2 = grid_axes()
    x = np.exp(lnx)
    x[-1] = 1.0
    out = np.zeros((NTAB, NQ, NX), dtype=np.float32)
    for j, lq in enumerate(lnq2):
        q2 = math.exp(lq)
        for t in range(NTAB):
            v = analytic_xf(t, x, q2)
            v[-1] = 0.0
            out[t, j, :] = v.astype(np.float32)
    return out


def grid_config():
    """Everything the two implementations need to rebuild the grid geometry."""
    lnx, lnq2 = grid_axes()
    return dict(nx=NX, nq=NQ, ntab=NTAB, lnx0=float(lnx[0]), lnx1=float(lnx[-1]),
                lnq0=float(lnq2[0]), lnq1=float(lnq2[-1]))
