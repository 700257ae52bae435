"""Pins of the oracle's FF/FI/IF/II maps (appendix B): the Catani-Seymour
variables recomputed from the produced momenta with the printed definitions
must equal the inputs; momenta stay massless; momentum is conserved; the II
transformation maps K' onto K and preserves the metric."""
import math

import numpy as np
import pytest

from oracle import pyoracle

FF, FI, IF, II = 0, 1, 2, 3


def dot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def massless(rng, emin=1.0, emax=100.0):
    e = rng.uniform(emin, emax)
    c = rng.uniform(-1, 1)
    ph = rng.uniform(0, 2 * math.pi)
    s = math.sqrt(1 - c * c)
    return np.array([e, e * s * math.cos(ph), e * s * math.sin(ph), e * c])


def beam(e, sign):
    return np.array([e, 0.0, 0.0, sign * e])


def test_ff_map():
    rng = np.random.default_rng(11)
    for _ in range(300):
        pij, pk = massless(rng), massless(rng)
        z, y, phi = rng.uniform(0.01, 0.99), rng.uniform(1e-4, 0.9), rng.uniform(0, 6.28)
        (pi, pj, pk2), _ = pyoracle.kin_map(FF, pij, pk, z, y, phi)
        scale = dot(pij, pk)
        for p in (pi, pj, pk2):
            assert abs(dot(p, p)) < 1e-11 * scale
        assert np.allclose(pi + pj + pk2, pij + pk, atol=1e-11 * pij[0])
        zz = dot(pi, pk2) / (dot(pi, pk2) + dot(pj, pk2))
        yy = dot(pi, pj) / (dot(pi, pj) + dot(pi, pk2) + dot(pj, pk2))
        assert zz == pytest.approx(z, rel=1e-9)
        assert yy == pytest.approx(y, rel=1e-9)


def test_fi_map():
    rng = np.random.default_rng(12)
    for _ in range(300):
        pij, pa = massless(rng), beam(rng.uniform(10, 500), rng.choice([-1, 1]))
        z, x, phi = rng.uniform(0.01, 0.99), rng.uniform(0.05, 0.999), rng.uniform(0, 6.28)
        (pi, pj, pa2), _ = pyoracle.kin_map(FI, pij, pa, z, x, phi)
        scale = dot(pij, pa)
        for p in (pi, pj, pa2):
            assert abs(dot(p, p)) < 1e-11 * scale
        assert np.allclose(pi + pj - pa2, pij - pa, atol=1e-11 * pa2[0])
        zz = dot(pi, pa2) / (dot(pi, pa2) + dot(pj, pa2))
        xx = (dot(pi, pa2) + dot(pj, pa2) - dot(pi, pj)) / (dot(pi, pa2) + dot(pj, pa2))
        assert zz == pytest.approx(z, rel=1e-9)
        assert xx == pytest.approx(x, rel=1e-9)
        assert pa2[1] == 0 and pa2[2] == 0  # stays on the beam axis


def test_if_map():
    rng = np.random.default_rng(13)
    for _ in range(300):
        paj, pk = beam(rng.uniform(10, 500), rng.choice([-1, 1])), massless(rng)
        x, u, phi = rng.uniform(0.05, 0.999), rng.uniform(1e-3, 0.999), rng.uniform(0, 6.28)
        (pa, pj, pk2), _ = pyoracle.kin_map(IF, paj, pk, x, u, phi)
        scale = dot(paj, pk)
        for p in (pa, pj, pk2):
            assert abs(dot(p, p)) < 1e-11 * scale
        assert np.allclose(pa - pj - pk2, paj - pk, atol=1e-10 * pa[0])
        xx = (dot(pa, pj) + dot(pa, pk2) - dot(pj, pk2)) / (dot(pa, pj) + dot(pa, pk2))
        uu = dot(pa, pj) / (dot(pa, pj) + dot(pa, pk2))
        assert xx == pytest.approx(x, rel=1e-9)
        assert uu == pytest.approx(u, rel=1e-9)
        # forward momentum fraction and the ordering variable, printed forms
        z = dot(pa - pj, pk) / dot(pa, pk)
        assert z == pytest.approx(1 - (1 - x) * (1 - u), rel=1e-9)


def test_ii_map_and_boost():
    rng = np.random.default_rng(14)
    for _ in range(300):
        sign = rng.choice([-1, 1])
        paj, pb = beam(rng.uniform(10, 500), sign), beam(rng.uniform(10, 500), -sign)
        # a colour-neutral final state carrying K' = paj + pb: two massless momenta
        Kp = paj + pb
        M = math.sqrt(dot(Kp, Kp))
        c, ph = rng.uniform(-1, 1), rng.uniform(0, 6.28)
        s = math.sqrt(1 - c * c)
        k1 = np.array([M / 2, M / 2 * s * math.cos(ph), M / 2 * s * math.sin(ph), M / 2 * c])
        bz = Kp[3] / Kp[0]
        g = 1 / math.sqrt(1 - bz * bz)
        def boostz(k):
            return np.array([g * (k[0] + bz * k[3]), k[1], k[2], g * (k[3] + bz * k[0])])
        k1 = boostz(k1)
        k2 = Kp - k1
        x, phi = rng.uniform(0.05, 0.999), rng.uniform(0, 6.28)
        v = rng.uniform(1e-4, 1 - x - 1e-4)
        (pa, pj, pb2), rest = pyoracle.kin_map(II, paj, pb, x, v, phi, rest=np.stack([k1, k2]))
        scale = dot(paj, pb)
        for p in (pa, pj, pb2, rest[0], rest[1]):
            assert abs(dot(p, p)) < 1e-10 * scale
        assert np.allclose(pb2, pb)
        K = pa + pb2 - pj
        assert dot(K, K) == pytest.approx(dot(Kp, Kp), rel=1e-10)
        assert np.allclose(rest[0] + rest[1], K, atol=1e-9 * K[0])
        assert dot(rest[0], rest[1]) == pytest.approx(dot(k1, k2), rel=1e-10)
        xx = (dot(pa, pb2) - dot(pa, pj) - dot(pb2, pj)) / dot(pa, pb2)
        vv = dot(pa, pj) / dot(pa, pb2)
        assert xx == pytest.approx(x, rel=1e-9)
        assert vv == pytest.approx(v, rel=1e-8)
        z = dot(pa - pj, pb) / dot(pa, pb)
        assert z == pytest.approx(x + v, rel=1e-9)


@pytest.mark.parametrize("typ", [IF, II])
def test_is_variable_round_trip(typ):
    rng = np.random.default_rng(20 + typ)
    for _ in range(500):
        s = 10 ** rng.uniform(2, 8)
        z = rng.uniform(1e-3, 1 - 1e-6)
        r = 10 ** rng.uniform(-9, -0.5)
        t = r * s
        x, uv = pyoracle.is_vars(typ, z, t, s)
        if typ == IF:
            assert 1 - (1 - x) * (1 - uv) == pytest.approx(z, rel=1e-12, abs=1e-14)
            assert uv * (1 - uv) * (1 - x) / x * s == pytest.approx(t, rel=1e-9)
            # the printed root, where it is well conditioned
            if r > 1e-4:
                pr = (1 - z + r) / (2 * r) * (1 - math.sqrt(1 - 4 * r * z * (1 - z) / (1 - z + r) ** 2))
                assert x == pytest.approx(pr, rel=1e-8)
        else:
            assert x + uv == pytest.approx(z, rel=1e-12)
            assert uv * (1 - x - uv) / x * s == pytest.approx(t, rel=1e-9)


@pytest.mark.parametrize("typ", [IF, II])
def test_z_limits_put_x_at_eta(typ):
    """At the printed z+- the Catani-Seymour x equals the momentum fraction."""
    rng = np.random.default_rng(30 + typ)
    for _ in range(200):
        eta = 10 ** rng.uniform(-5, -0.3)
        s = 10 ** rng.uniform(3, 8)
        tlim = s / 4 * (1 - eta) / eta if typ == IF else s / 4 * (1 - eta) ** 2 / eta
        t = tlim * 10 ** rng.uniform(-6, -0.01)
        d = 4 * t * eta / (s * (1 - eta)) if typ == IF else 4 * t * eta / (s * (1 - eta) ** 2)
        for sgn in (-1, 1):
            z = 0.5 * ((1 + eta) + sgn * (1 - eta) * math.sqrt(1 - d))
            x, _ = pyoracle.is_vars(typ, z, t, s)
            assert x == pytest.approx(eta, rel=1e-6)
