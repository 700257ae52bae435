"""Event-record layout shared by both implementations' Python bindings.

An event record is a structure of arrays, slot-major: a per-slot field is a
[max_slots, cap] array and particle q of event e sits at [q, e].  Per-event
fields are [cap] arrays.  This module only allocates and compares storage.
"""
from __future__ import annotations

import numpy as np

PER_EVENT = (
    ("id", np.int64), ("w", np.float64), ("t_start", np.float64), ("n", np.int32),
    ("flags", np.uint32),
)
PER_SLOT = (
    ("E", np.float64), ("px", np.float64), ("py", np.float64), ("pz", np.float64),
    ("pid", np.int32), ("col", np.int32), ("acol", np.int32), ("status", np.int8),
)
COUNTERS = (
    ("n_cycles", np.uint32), ("n_trials", np.uint32), ("n_accept", np.uint32),
    ("n_viol", np.uint32), ("t1", np.float64),
)

FLAG_OVERFLOW = 1
FLAG_COLOUR = 2
FLAG_NAN = 4
FLAG_FALLBACK = 8
FLAG_VIOL = 16
FLAG_HARDFAIL = 32
FLAG_HEVENT = 64
FLAG_MAXCYC = 128
FLAG_MEC = 256


class Events:
    """numpy-backed event record (host memory)."""

    def __init__(self, cap: int, max_slots: int):
        self.cap = int(cap)
        self.max_slots = int(max_slots)
        for name, dt in PER_EVENT + COUNTERS:
            setattr(self, name, np.zeros(self.cap, dtype=dt))
        for name, dt in PER_SLOT:
            setattr(self, name, np.zeros((self.max_slots, self.cap), dtype=dt))

    def fields(self):
        return [n for n, _ in PER_EVENT + PER_SLOT + COUNTERS]

    def subset(self, idx) -> "Events":
        idx = np.asarray(idx)
        out = Events(len(idx), self.max_slots)
        for name, _ in PER_EVENT + COUNTERS:
            getattr(out, name)[:] = getattr(self, name)[idx]
        for name, _ in PER_SLOT:
            getattr(out, name)[:] = getattr(self, name)[:, idx]
        return out

    def momenta(self, e: int) -> np.ndarray:
        n = int(self.n[e])
        return np.stack([self.E[:n, e], self.px[:n, e], self.py[:n, e], self.pz[:n, e]], axis=1)
