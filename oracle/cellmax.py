"""CPU oracle of the cell-maximum initial-state bound (TEST INFRASTRUCTURE ONLY).

Plain numpy, written from the definitions below; only tests/, the smoke check
and bench.py's CPU baseline may use it.

The non-learned comparator of the learned bound.  The paper replaces Herwig's
adaptive overestimates (ExSample) with large fixed ones and names adaptive
overestimation as future work (section 5); the first half of such a scheme is
presampling: run trials, record the veto weight each one would have had, and
set each cell's overestimate from the largest weight seen there.  This module
does that on the same cells the learned bound uses, so that the shower's
per-trial check and plain-mode fallback keep it exact in the same way, and the
two bounds can be compared on the same logged trials.

Cell of a logged trial (ln t, ln eta, z, entry, ln W):
    (entry - 8, eta bin of ln eta, ln t cell), the ln t cell being the largest
    k in 1..7 with edge[k] < ln t, else 0 (the cell the shower takes for a scale)
Target: y = ln W - ln R[entry][eta bin], rounded to float32 (as for the network).
Fitting rows: ymax[cell] = the largest y, n[cell] = the number of rows.
Held-out rows, per entry, over cells with n >= MIN_CELL:
    r_e = the largest y - ymax[cell]; delta_e = max(r_e, 0) + 2^-6,
    entries with fewer than MIN_CAL such rows keep the analytic bound.
Table: min(R, up6(R exp(v))), v = clip(ymax + delta_e, -20, 0), for cells with
n >= MIN_CELL in calibrated entries; R (the analytic bound) elsewhere.

Adaptive cell sizes (adaptive=True): in the spirit of ExSample's cell
splitting, every cell takes the finest block around it that holds enough
presampled trials.  The blocks are dyadic in (eta bin, ln t cell): level l
groups the cells whose indices agree after shifting right by SHIFTS[l]
(level 0 is the cell itself, the last level the whole entry).  A cell's
maximum is the largest y of the first level whose block has at least MIN_CELL
fitting rows; cells of entries with fewer rows keep the analytic bound.  The
held-out margin of a cell at level 0 is its entry's, as on the fixed cells;
cells at a coarser level l share one margin per level, from the held-out rows
of all such cells of every entry (with the same MIN_CAL threshold), so that
thinly sampled cells do not loosen the well sampled ones of their entry.

Pinned by tests/test_oracle_cellmax.py (every fitting row covered, closed-form
cells, calibration raising the bound over held-out rows, untouched cells, the
adaptive blocks).
"""
from __future__ import annotations

import numpy as np

from oracle.mlp import CAL_MARGIN, DLE, IS0, LNETA0, MIN_CAL, NB, NENT_IS, NTB, V_MIN, up6

MIN_CELL = 16
NCELL = NENT_IS * NB * NTB
# (eta bin, ln t cell) shifts of the dyadic blocks of each level
SHIFTS = ((0, 0), (1, 1), (2, 2), (3, 3), (4, 3), (5, 3), (6, 3))


def adaptive_cells(ymax, n):
    """Per cell the maximum, row count and level of the finest block around it
    with at least MIN_CELL rows (-inf, 0 and -1 where even the whole entry has
    fewer)."""
    ym = ymax.reshape(NENT_IS, NB, NTB)
    nn = n.reshape(NENT_IS, NB, NTB)
    out_y = np.full(ym.shape, -np.inf)
    out_n = np.zeros(nn.shape, dtype=np.int64)
    out_l = np.full(nn.shape, -1, dtype=np.int64)
    done = np.zeros(ym.shape, dtype=bool)
    bi = np.arange(NB)[:, None]
    ki = np.arange(NTB)[None, :]
    for lev, (sb, sk) in enumerate(SHIFTS):
        for e in range(NENT_IS):
            for b in range(NB):
                for k in range(NTB):
                    if done[e, b, k]:
                        continue
                    blk = ((bi >> sb) == (b >> sb)) & ((ki >> sk) == (k >> sk))
                    cnt = int(nn[e][blk].sum())
                    if cnt >= MIN_CELL:
                        out_y[e, b, k] = ym[e][blk].max()
                        out_n[e, b, k] = cnt
                        out_l[e, b, k] = lev
                        done[e, b, k] = True
    return out_y.reshape(-1), out_n.reshape(-1), out_l.reshape(-1)


def cells(rows, bounds, cell_edges):
    """Cell index, target y (float64 of the float32 value) and entry of each
    logged trial whose entry is an initial-state one (others are dropped)."""
    r = np.asarray(rows, dtype=np.float32).reshape(-1, 5).astype(np.float64)
    lnt, lne, lnw = r[:, 0], r[:, 1], r[:, 4]
    ent = r[:, 3].astype(np.int64)
    keep = (ent >= IS0) & (ent < IS0 + NENT_IS)
    lnt, lne, lnw, ent = lnt[keep], lne[keep], lnw[keep], ent[keep]
    b = np.floor((lne - LNETA0) / DLE)
    b = np.where(b >= 0.0, b, 0.0)  # below the first bin, or not a number
    b = np.minimum(b, NB - 1).astype(np.int64)
    E = np.asarray(cell_edges, dtype=np.float64)
    k = np.zeros(lnt.shape, dtype=np.int64)
    for j in range(1, NTB):
        k = np.where(E[j] < lnt, j, k)
    y = (lnw - np.log(np.asarray(bounds, dtype=np.float64)[ent, b])).astype(np.float32).astype(np.float64)
    return ((ent - IS0) * NB + b) * NTB + k, y, ent


def cellmax_table(rows_fit, rows_cal, bounds, cell_edges, adaptive=False):
    """The cell-maximum table [64][48][8] (doubles), the per-entry delta of the
    entries' own cells (inf: analytic) and the fitting-row count of each cell
    (adaptive: of its block)."""
    c, y, _ = cells(rows_fit, bounds, cell_edges)
    ymax = np.full(NCELL, -np.inf)
    np.maximum.at(ymax, c, y)
    n = np.bincount(c, minlength=NCELL)
    # calibration group of each cell: its entry (the cell's own rows), or one
    # group per coarser level of the adaptive blocks
    grp = np.repeat(np.arange(NENT_IS), NB * NTB)
    if adaptive:
        ymax, n, lev = adaptive_cells(ymax, n)
        grp = np.where(lev > 0, NENT_IS + lev - 1, grp)
    ngrp = NENT_IS + len(SHIFTS) - 1
    cc, yc, ec = cells(rows_cal, bounds, cell_edges)
    use = n[cc] >= MIN_CELL
    g = grp[cc[use]]
    excess = np.full(ngrp, -np.inf)
    np.maximum.at(excess, g, yc[use] - ymax[cc[use]])
    ncal = np.bincount(g, minlength=ngrp)
    dgrp = np.where(ncal >= MIN_CAL, np.maximum(excess, 0.0) + CAL_MARGIN, np.inf)
    delta = dgrp[:NENT_IS]
    dcell = dgrp[grp].reshape(NENT_IS, NB, NTB)
    R = np.broadcast_to(np.asarray(bounds, dtype=np.float64)[IS0:IS0 + NENT_IS, :, None], (NENT_IS, NB, NTB))
    ym = ymax.reshape(NENT_IS, NB, NTB)
    fitted = (n.reshape(NENT_IS, NB, NTB) >= MIN_CELL) & np.isfinite(dcell) & (R > 0.0)
    with np.errstate(invalid="ignore", over="ignore"):
        v = np.clip(ym + dcell, V_MIN, 0.0)
        tab = np.where(fitted, np.minimum(R, up6(R * np.exp(v))), R)
    return np.ascontiguousarray(tab, dtype=np.float64), delta, n.reshape(NENT_IS, NB, NTB)
