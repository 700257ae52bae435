"""Event-by-event comparison of two shower outputs (the oracle's and the GPU
library's), shared by the GPU parity tests and the smoke check.

An event counts as identical when its integer data are equal (multiplicity,
flags, cycle/trial/accept/violation counters, and every parton's flavour,
colour tags and status), its weight agrees to wtol relative, and every
parton's four-momentum components agree to tol relative to that parton's own
energy (|dp| <= tol * max(E_i, 1 GeV)).  The per-parton scale is at most the
collision energy, so this is stricter than a tolerance relative to sqrt(s).
Transcendental functions differ by an ulp between the device and host
libraries; that is the only expected source of disagreement.
"""
from __future__ import annotations

import numpy as np

from gapsinputs import records


def compare_events(a: records.Events, b: records.Events, scale: float = None, need=0.999, tol=1e-9, wtol=1e-9):
    """a: oracle, b: GPU.  Returns (fraction identical, the worst per-parton
    relative momentum difference among the identical events, mask of the
    identical events).  `scale` is accepted for the callers that quote it; the
    criterion is per parton."""
    n = a.cap
    same = np.ones(n, dtype=bool)
    same &= a.n == b.n
    same &= a.flags == b.flags
    for name in ("n_cycles", "n_trials", "n_accept", "n_viol"):
        same &= getattr(a, name) == getattr(b, name)
    wrel = np.abs(a.w - b.w) / np.maximum(np.abs(a.w), 1e-300)
    int_ok = same.copy()
    M = min(a.max_slots, b.max_slots)
    slot_ok = np.arange(M)[:, None] < a.n[None, :]
    for name in ("pid", "col", "acol", "status"):
        eq = (getattr(a, name)[:M] == getattr(b, name)[:M]) | ~slot_ok
        same &= eq.all(axis=0)
    ref = np.maximum(np.abs(a.E[:M]), 1.0)
    rel = np.zeros(n)
    for name in ("E", "px", "py", "pz"):
        d = np.abs(getattr(a, name)[:M] - getattr(b, name)[:M]) / ref
        d = np.where(slot_ok, d, 0.0)
        rel = np.maximum(rel, np.nan_to_num(d, nan=np.inf).max(axis=0))
    int_ok &= same
    same &= (rel <= tol) & (wrel <= wtol)
    worst = float(rel[same].max()) if same.any() else 0.0
    if not same.all():
        bad = ~same
        print(f"  compare_events: {int(bad.sum())} of {n} differ: {int((~int_ok).sum())} in integer data, "
              f"{int((int_ok & (wrel > wtol)).sum())} in the weight (worst {float(wrel[int_ok].max()) if int_ok.any() else 0.0:.3g}), "
              f"{int((int_ok & (rel > tol)).sum())} in momenta (worst {float(rel[int_ok].max()) if int_ok.any() else 0.0:.3g})", flush=True)
    return float(same.mean()), worst, same
