"""Pins of the oracle's cell-maximum bound (the non-learned comparator of the
learned bound): where a logged trial lands, closed-form cells, the calibration
margin, the row thresholds, and on logged trials of the NLO shower, that every
fitting row is covered and the bound never exceeds the analytic one."""
import math

import numpy as np
import pytest

from oracle import cellmax, mlp


@pytest.fixture(scope="module")
def nlo(oracles):
    o = oracles["nlo"]
    return o, o.bounds(), o.cell_edges()


def _row(e, b, k, y, B, E, z=0.5, lnt=None):
    """A logged trial of entry e in the middle of eta bin b and ln t cell k
    whose target ln W - ln R is y (in float32)."""
    lne = mlp.LNETA0 + (b + 0.5) * mlp.DLE
    if lnt is None:
        lnt = 0.5 * (E[k] + E[k + 1])
    lnw = y + math.log(B[e, b])
    return [lnt, lne, z, float(e), lnw]


def test_cell_of_a_logged_trial(nlo):
    o, B, E = nlo
    picks = [(9, 0, 0), (9, 47, 7), (33, 17, 3), (71, 5, 6), (55, 33, 1)]
    rows = np.array([_row(e, b, k, -1.0, B, E) for e, b, k in picks], dtype=np.float32)
    c, y, ent = cellmax.cells(rows, B, E)
    got = np.stack(np.unravel_index(c, (64, 48, 8)), axis=1)
    assert np.array_equal(got, [[e - 8, b, k] for e, b, k in picks])
    assert np.array_equal(ent, [e for e, _, _ in picks])
    # the target is the log of the weight over the analytic bound
    assert np.allclose(y, -1.0, atol=1e-6)
    # scales outside the cell grid belong to the outermost cells; final-state
    # entries are not cells of the initial-state bound
    out = np.array([_row(20, 3, 0, -1.0, B, E, lnt=E[0] - 3.0), _row(20, 3, 0, -1.0, B, E, lnt=E[8] + 3.0),
                    _row(3, 3, 0, -1.0, B, E)], dtype=np.float32)
    c, _, _ = cellmax.cells(out, B, E)
    assert [int(v) % 8 for v in c] == [0, 7]


def _table(rows_fit, rows_cal, B, E):
    return cellmax.cellmax_table(np.array(rows_fit, dtype=np.float32).reshape(-1, 5),
                                 np.array(rows_cal, dtype=np.float32).reshape(-1, 5), B, E)


def test_closed_form_cell(nlo):
    o, B, E = nlo
    e, b, k = 33, 17, 3
    R = B[e, b]
    ys = np.linspace(-3.0, -2.5, 20)
    fit = [_row(e, b, k, y, B, E) for y in ys]
    cal = [_row(e, b, k, -2.75, B, E)] * 2000  # all below the fitted maximum: the bare margin
    tab, delta, n = _table(fit, cal, B, E)
    assert n[e - 8, b, k] == 20 and delta[e - 8] == 2.0 ** -6
    top = float(np.float32(-2.5))
    lo = R * math.exp(top + 2.0 ** -6)
    v = tab[e - 8, b, k]
    assert lo <= v <= lo * (1 + 2.0 ** -6)
    m, _ = math.frexp(v)
    assert m * 128 == round(m * 128)  # on the 7-bit grid
    # every other cell keeps the analytic bound
    R3 = np.broadcast_to(B[8:72, :, None], tab.shape)
    mask = np.ones(tab.shape, dtype=bool)
    mask[e - 8, b, k] = False
    assert np.array_equal(tab[mask], R3[mask])


def test_calibration_covers_held_out_rows(nlo):
    o, B, E = nlo
    e, b, k = 50, 9, 5
    fit = [_row(e, b, k, y, B, E) for y in np.linspace(-4.0, -2.5, 30)]
    cal = [_row(e, b, k, -3.0, B, E)] * 1999 + [_row(e, b, k, -2.0, B, E)]
    tab, delta, _ = _table(fit, cal, B, E)
    assert abs(delta[e - 8] - (0.5 + 2.0 ** -6)) < 1e-6
    assert tab[e - 8, b, k] >= B[e, b] * math.exp(-2.0)  # the held-out row is under the bound
    # the margin of an entry applies to all its cells
    fit2 = fit + [_row(e, 2, 6, y, B, E) for y in np.linspace(-5.0, -4.0, 16)]
    tab2, _, _ = _table(fit2, cal, B, E)
    assert tab2[e - 8, 2, 6] >= B[e, 2] * math.exp(-4.0 + 0.5)


def test_row_thresholds_and_clip(nlo):
    o, B, E = nlo
    R3 = np.broadcast_to(B[8:72, :, None], (64, 48, 8))
    e, b, k = 20, 30, 2
    # 15 fitting rows: too few for the cell
    tab, _, _ = _table([_row(e, b, k, -2.0, B, E)] * 15, [_row(e, b, k, -2.0, B, E)] * 2000, B, E)
    assert np.array_equal(tab, R3)
    # 1999 held-out rows: too few for the entry
    tab, delta, _ = _table([_row(e, b, k, -2.0, B, E)] * 16, [_row(e, b, k, -2.0, B, E)] * 1999, B, E)
    assert np.array_equal(tab, R3) and np.isinf(delta[e - 8])
    # held-out rows of thin cells do not count towards the entry
    fit = [_row(e, b, k, -2.0, B, E)] * 16 + [_row(e, b, 7, -2.0, B, E)] * 3
    cal = [_row(e, b, k, -2.0, B, E)] * 1990 + [_row(e, b, 7, -2.0, B, E)] * 10
    tab, _, _ = _table(fit, cal, B, E)
    assert np.array_equal(tab, R3)
    # a target above the analytic bound clips to it; the floor is e^-20 of it
    tab, _, _ = _table([_row(e, b, k, 0.3, B, E)] * 16, [_row(e, b, k, -1.0, B, E)] * 2000, B, E)
    assert tab[e - 8, b, k] == B[e, b]
    tab, _, _ = _table([_row(e, b, k, -40.0, B, E)] * 16, [_row(e, b, k, -50.0, B, E)] * 2000, B, E)
    assert B[e, b] * math.exp(-20.0) <= tab[e - 8, b, k] <= B[e, b] * math.exp(-20.0) * (1 + 2.0 ** -6)


def test_logged_trials_are_covered(nlo):
    """On logged trials of 6000 NLO events: every fitting row lies under the
    bound of its cell, the bound never exceeds the analytic one, it is tighter
    where rows exist, and held-out rows above it are rare."""
    o, B, E = nlo
    # one thread: rows in event order, so the fitting / held-out split is reproducible
    _, rows, cnt = o.shower_log(o.hard_events(2_000_000, 6000, 3), 3, 3_000_000, nthreads=1)
    assert cnt == rows.shape[0] and cnt > 300_000
    nf = int(0.8 * cnt)
    tab, delta, n = cellmax.cellmax_table(rows[:nf], rows[nf:], B, E)
    R3 = np.broadcast_to(B[8:72, :, None], tab.shape)
    assert np.all(tab <= R3) and np.all(tab[R3 > 0] > 0)
    c, y, _ = cellmax.cells(rows[:nf], B, E)
    flat = tab.reshape(-1)
    rflat = R3.reshape(-1)
    assert np.all(rflat[c] * np.exp(y) <= flat[c] * (1 + 1e-12))
    fitted = (n >= cellmax.MIN_CELL) & np.isfinite(delta)[:, None, None] & (R3 > 0)
    assert fitted.sum() > 500
    assert np.mean(tab[fitted] < R3[fitted]) > 0.5
    cc, yc, _ = cellmax.cells(rows[nf:], B, E)
    over = rflat[cc] * np.exp(yc) > flat[cc]
    assert over.mean() < 1e-3


def test_adaptive_blocks_closed_form(nlo):
    """Adaptive cell sizes: a well sampled cell keeps its own maximum, a thin
    neighbour takes the maximum of the smallest dyadic block with enough rows,
    an empty corner of the entry the whole entry's, each coarser level with a
    margin of its own (analytic without enough held-out rows), and an entry
    with too few rows in all keeps the analytic bound."""
    o, B, E = nlo
    e = 33
    rich = [_row(e, 16, 3, y, B, E) for y in np.linspace(-3.0, -2.5, 20)]
    thin = [_row(e, 17, 3, -1.0, B, E)] * 5
    lone = [_row(50, 9, 5, -2.0, B, E)] * 10
    cal = ([_row(e, 16, 3, -2.75, B, E)] * 2000 + [_row(e, 17, 3, -1.5, B, E)] * 2000 +
           [_row(e, 47, 7, -2.0, B, E)] * 2000 + [_row(50, 9, 5, -2.0, B, E)] * 2000)
    tab, delta, n = _table(rich + thin + lone, cal, B, E)
    taba, deltaa, na = cellmax.cellmax_table(np.array(rich + thin + lone, dtype=np.float32),
                                             np.array(cal, dtype=np.float32), B, E, adaptive=True)
    R = B[e]
    top_rich, top_thin = float(np.float32(-2.5)), float(np.float32(-1.0))
    m = 2.0 ** -6
    # the rich cell: its own maximum, as on the fixed grid
    assert taba[e - 8, 16, 3] == tab[e - 8, 16, 3]
    assert R[16] * math.exp(top_rich + m) <= taba[e - 8, 16, 3] <= R[16] * math.exp(top_rich + m) * (1 + m)
    # the thin cell: the 2 x 2 block (eta bins 16-17, ln t cells 2-3) with 25 rows
    assert na[e - 8, 17, 3] == 25 and n[e - 8, 17, 3] == 5
    assert tab[e - 8, 17, 3] == R[17]
    assert R[17] * math.exp(top_thin + m) <= taba[e - 8, 17, 3] <= R[17] * math.exp(top_thin + m) * (1 + m)
    # far corners of the entry: the whole entry (25 rows) at the last level
    assert na[e - 8, 47, 7] == 25 and na[e - 8, 0, 0] == 25
    assert R[47] * math.exp(top_thin + m) <= taba[e - 8, 47, 7] <= R[47] * math.exp(top_thin + m) * (1 + m)
    # a 4 x 4 block holds the thin and rich cells at level 2; no held-out rows
    # there, so the level has no margin and its cells stay analytic
    assert na[e - 8, 19, 0] == 25 and taba[e - 8, 19, 0] == R[19]
    # a held-out row above a coarse block raises that level's margin only
    cal2 = cal + [_row(e, 17, 3, -0.5, B, E)]
    taba2, _, _ = cellmax.cellmax_table(np.array(rich + thin + lone, dtype=np.float32),
                                        np.array(cal2, dtype=np.float32), B, E, adaptive=True)
    assert taba2[e - 8, 16, 3] == taba[e - 8, 16, 3] and taba2[e - 8, 47, 7] == taba[e - 8, 47, 7]
    assert taba2[e - 8, 17, 3] >= R[17] * math.exp(-0.5)
    # entry 50 has 10 rows in all: analytic everywhere
    R3 = np.broadcast_to(B[8:72, :, None], tab.shape)
    assert np.array_equal(taba[50 - 8], R3[50 - 8]) and np.isinf(deltaa[50 - 8])
    # entries without rows are untouched
    assert np.array_equal(taba[20 - 8], R3[20 - 8])


def test_adaptive_logged_trials(nlo):
    """On logged trials of 6000 NLO events: with adaptive cells every fitting
    row stays under its cell's bound, well sampled cells keep their own
    maximum, fewer cells of calibrated entries stay analytic, and held-out
    rows above the bound are rare."""
    o, B, E = nlo
    _, rows, cnt = o.shower_log(o.hard_events(2_000_000, 6000, 3), 3, 3_000_000, nthreads=1)
    nf = int(0.8 * cnt)
    tab, delta, n = cellmax.cellmax_table(rows[:nf], rows[nf:], B, E)
    taba, deltaa, na = cellmax.cellmax_table(rows[:nf], rows[nf:], B, E, adaptive=True)
    R3 = np.broadcast_to(B[8:72, :, None], tab.shape)
    assert np.all(taba <= R3) and np.all(taba[R3 > 0] > 0)
    c, y, _ = cellmax.cells(rows[:nf], B, E)
    flat, rflat = taba.reshape(-1), R3.reshape(-1)
    assert np.all(rflat[c] * np.exp(y) <= flat[c] * (1 + 1e-12))
    own = n >= cellmax.MIN_CELL
    assert np.array_equal(na[own], n[own])
    cal = np.isfinite(deltaa)
    live = cal[:, None, None] & (R3 > 0)
    assert np.sum(live & (taba == R3)) < np.sum(live & (tab == R3))
    cc, yc, _ = cellmax.cells(rows[nf:], B, E)
    assert np.mean(rflat[cc] * np.exp(yc) > flat[cc]) < 1e-3
