"""The event comparison the GPU parity tests use (tests/parity.py), on the
CPU: identical outputs compare equal; a momentum off by more than 1e-9 of the
parton's own energy, a weight off by more than 1e-9 relative, or one colour
tag changed, each make exactly that event differ."""
import numpy as np

from tests.parity import compare_events


def test_compare_events_catches_each_kind_of_difference(oracles):
    o = oracles["nlo"]
    ev = o.hard_events(0, 200, 3)
    a = o.shower(ev, 5)
    b = o.shower(ev, 5)
    frac, worst, same = compare_events(a, b)
    assert frac == 1.0 and worst == 0.0
    # a soft parton: 1e-9 of sqrt(S) would hide this, 1e-9 of its own energy does not
    e = int(np.argmax(a.n))
    q = int(np.argmin(a.E[:a.n[e], e]))
    b.px[q, e] += 3e-9 * max(a.E[q, e], 1.0)
    b.w[e + 1] *= 1.0 + 3e-9
    b.col[0, e + 2] += 1
    b.pz[1, e + 3] += 0.5e-9 * max(a.E[1, e + 3], 1.0)  # within tolerance
    frac, worst, same = compare_events(a, b)
    assert not same[e] and not same[e + 1] and not same[e + 2] and same[e + 3]
    assert same.sum() == 197 and 0.0 < worst <= 1e-9
