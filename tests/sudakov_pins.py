"""First-emission pins of the oracle's splitting kernels, shared by the pin
tests and the mutation tests.

Each check showers many copies of one hard configuration with the oracle and
compares the empirical distribution of the first emission scale with the
no-emission probability Delta(t) = exp(-sum_ch int_t dt'/t' F_ch(t')), where
every integrand F_ch is written here, independently of the oracle, from the
printed kernels, kinematics and Sudakov factors of appendix B (FF B.2, FI B.3,
IF B.4, II B.5) and the PDF ratio of appendix A.1, and integrated numerically
with SciPy's grid interpolator for the PDFs.  The veto algorithm reproduces
Delta whatever the overestimates, so a kernel with a wrong colour factor, a
dropped term, a wrong PDF ratio or a wrong measure moves the distribution.

Families whose integrand can turn negative somewhere are clipped at zero: the
veto never accepts a negative weight, and every term of a channel is its own
competing process.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import interpolate

from gapsinputs import records, toypdf

CF, CA, TR, NF = 4.0 / 3.0, 3.0, 0.5, 5
NODES, WEIGHTS = np.polynomial.legendre.leggauss(600)
TAB = {name: i for i, name in enumerate(toypdf.TABLE_NAMES)}
# the ten quark flavours a gluon can evolve back to, by PDF table (the sea
# antiquarks s-bar, c-bar, b-bar share the quarks' tables)
QUARK_TABLES = [TAB["d"], TAB["u"], TAB["s"], TAB["c"], TAB["b"],
                TAB["dbar"], TAB["ubar"], TAB["s"], TAB["c"], TAB["b"]]


def table_of(pid):
    return {21: TAB["g"], 1: TAB["d"], 2: TAB["u"], 3: TAB["s"], 4: TAB["c"], 5: TAB["b"],
            -1: TAB["dbar"], -2: TAB["ubar"], -3: TAB["s"], -4: TAB["c"], -5: TAB["b"]}[int(pid)]


class PDF:
    """f(x, Q^2) from the toy grid: linear in (ln Q^2, ln x) of x f, zero
    outside the grid and at x >= 1 (appendix B.6)."""

    def __init__(self, grid):
        lnx, lnq = toypdf.grid_axes()
        self.f = [interpolate.RegularGridInterpolator((lnq, lnx), grid[t].astype(np.float64),
                                                      bounds_error=False, fill_value=0.0)
                  for t in range(8)]
        self.lq0, self.lq1, self.lx0 = lnq[0], lnq[-1], lnx[0]

    def __call__(self, tab, x, q2):
        x = np.asarray(x, dtype=np.float64)
        lx = np.log(np.clip(x, 1e-300, None))
        lq = np.full_like(lx, math.log(q2))
        ok = (x < 1.0) & (lx >= self.lx0) & (lq >= self.lq0) & (lq <= self.lq1)
        v = self.f[tab](np.stack([lq, lx], axis=-1))
        r = np.where(ok, v / x, 0.0)
        return r if np.ndim(r) else float(r)


def alphas(t):
    """One-loop running from alpha_s(m_Z^2) = 0.118, five flavours."""
    b0 = (33.0 - 2.0 * NF) / (12.0 * math.pi)
    return 0.118 / (1.0 + 0.118 * b0 * math.log(t / 91.1876 ** 2))


def zint(fun, zlo, zhi):
    """int_zlo^zhi fun(z) dz, Gauss-Legendre in the variable ln(z/(1-z))."""
    a, b = math.log(zlo / (1 - zlo)), math.log(zhi / (1 - zhi))
    v = 0.5 * (b - a) * NODES + 0.5 * (b + a)
    z = 1.0 / (1.0 + np.exp(-v))
    return 0.5 * (b - a) * float(np.sum(WEIGHTS * fun(z) * z * (1 - z)))


def delta_curve(channels, tgrid):
    """Delta(t) on tgrid for channels (F, t_low, t_high): each contributes
    int dt'/t' F(t') over [max(t, t_low), t_high]."""
    out = []
    for t in tgrid:
        tot = 0.0
        for F, tlo, thi in channels:
            a = max(t, tlo)
            if a >= thi:
                continue
            l = np.linspace(math.log(a), math.log(thi), 241)
            vals = np.array([F(math.exp(x)) for x in l])
            tot += np.trapezoid(vals, l)
        out.append(math.exp(-tot))
    return np.array(out)


def compare(t1, tgrid, delta, w=None, tol_abs=4e-3, nsig=4.5):
    """Empirical (weighted: the mean of w * [t1 <= t]) first-emission CDF
    against Delta, within nsig standard errors plus tol_abs (quadrature)."""
    n = len(t1)
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    worst = 0.0
    for t, d in zip(tgrid, delta):
        v = w * (t1 <= t)
        emp = float(np.mean(v))
        sig = math.sqrt(max(float(np.var(v)), d * (1 - d), 1e-4) / n)
        worst = max(worst, abs(emp - d) / (nsig * sig + tol_abs))
        assert abs(emp - d) < nsig * sig + tol_abs, (t, emp, d, sig)
    return worst


def deviation(t1, tgrid, delta):
    """Largest |empirical - Delta| in standard errors (unweighted)."""
    n = len(t1)
    return max(abs(float(np.mean(t1 <= t)) - d) / math.sqrt(max(d * (1 - d), 1e-4) / n)
               for t, d in zip(tgrid, delta))


def replicate(ev, k, n):
    """n copies of event k with ids 0..n-1."""
    out = records.Events(n, ev.max_slots)
    for name in ev.fields():
        src = getattr(ev, name)
        if src.ndim == 1:
            getattr(out, name)[:] = src[k]
        else:
            getattr(out, name)[:] = src[:, k:k + 1]
    out.id[:] = np.arange(n)
    return out


def form_kwargs(form):
    return {"paper": {}, "retain": dict(retain=True), "gen_select": dict(gen_select=True),
            "veto_max": dict(veto_max=True)}[form]


FORMS = ["paper", "retain", "gen_select", "veto_max"]


# ---- integrands (appendix B) ----

def ff_channel(s, gluon, tc=1.0):
    """FF end of s_ik (B.2): (1 - y) P(z, y) over z in z_+-; a quark emits
    q -> q g, a gluon g -> g g and g -> q qbar for NF flavours."""
    def F(t):
        d = 4.0 * t / s
        if d >= 1.0:
            return 0.0
        zm = 0.5 * (1.0 - math.sqrt(1.0 - d))

        def f(z):
            y = t / (z * (1 - z) * s)
            soft = 2.0 / (1.0 - z * (1.0 - y))
            if gluon:
                P = 0.5 * CA * (soft - 2.0 + z * (1 - z)) + NF * 0.5 * TR * (1.0 - 2.0 * z * (1 - z))
            else:
                P = CF * (soft - (1.0 + z))
            return np.where(y < 1.0, (1.0 - y) * P, 0.0)
        return alphas(t) / (2 * math.pi) * zint(f, zm, 1 - zm)
    return F, tc, s / 4.0


def fi_channel(pdf, s, eta, spec_tab, gluon, tc=1.69):
    """FI end (B.3): x from t = z(1 - z)(1 - x)/x s, the spectator's PDF ratio
    f_a(eta/x)/f_a(eta); q -> q g, or g -> g g and g -> q qbar."""
    def F(t):
        d = 4.0 * t / s * eta / (1.0 - eta)
        if d >= 1.0:
            return 0.0
        sq = math.sqrt(1.0 - d)
        den = pdf(spec_tab, eta, t)
        if den <= 0.0:
            return 0.0

        def f(z):
            kap = t / (z * (1 - z) * s)
            x = 1.0 / (1.0 + kap)
            ok = x > eta
            xs = np.where(ok, x, 0.5)
            ratio = pdf(spec_tab, eta / xs, t) / den
            soft = 2.0 / (1.0 - z + (1.0 - xs))
            if gluon:
                P = np.maximum(0.5 * CA * (soft - 2.0 + z * (1 - z)), 0.0) + \
                    NF * 0.5 * TR * (1.0 - 2.0 * z * (1 - z))
            else:
                P = np.maximum(CF * (soft - (1.0 + z)), 0.0)
            return np.where(ok, P * ratio, 0.0)
        return alphas(t) / (2 * math.pi) * zint(f, 0.5 * (1 - sq), 0.5 * (1 + sq))
    return F, tc, s / 4.0 * (1.0 - eta) / eta


def is_channel(pdf, kind, s, eta, pid, tc=1.69):
    """IF (kind "IF", B.4) or II ("II", B.5) end of an incoming parton of
    flavour pid at momentum fraction eta with dipole invariant s.  A quark has
    families A (q <- q, gluon emitted) and B (q <- g); a gluon C (g <- g) and
    D (g <- q for the ten quark flavours).  The measure dt/t (for a c or b
    quark, appendix A.2's dt/(t - m^2) times (t - m^2)/t, the same), the
    Jacobian 1/(u + x - 2ux) (IF) or 1/z (II) and the PDF ratio
    f_a(eta/x)/f_emitter(eta) at Q^2 = t."""
    ii = kind == "II"
    tab = table_of(pid)
    gluon = pid == 21

    def F(t):
        r = t / s
        d = 4.0 * t * eta / (s * (1.0 - eta) ** (2 if ii else 1))
        if d >= 1.0:
            return 0.0
        sq = math.sqrt(1.0 - d)
        zlo, zhi = 0.5 * ((1 + eta) - (1 - eta) * sq), 0.5 * ((1 + eta) + (1 - eta) * sq)
        den = pdf(tab, eta, t)
        if den <= 0.0:
            return 0.0

        def f(z):
            if ii:
                x = z * (1 - z) / (1 - z + r)
            else:
                # the printed root of B.4, in a form that does not cancel
                D = 1 - z + r
                dd = 4 * r * z * (1 - z) / D ** 2
                x = 2 * z * (1 - z) / (D * (1 + np.sqrt(1 - dd)))
            u = x * r / (1 - z)
            ok = (x > eta) & (u < 1)
            xs, us = np.where(ok, x, 0.5), np.where(ok, u, 0.5)
            omx = 1.0 - xs
            J = 1.0 / z if ii else 1.0 / (us + xs - 2 * us * xs)
            soft = omx if ii else omx + us
            if gluon:
                PC = CA * (1.0 / soft + omx / xs - 1.0 + xs * omx)
                PD = CF * (xs + 2.0 * omx / xs)
                num_c = pdf(TAB["g"], eta / xs, t)
                num_d = sum(pdf(T, eta / xs, t) for T in QUARK_TABLES)
                val = np.maximum(PC, 0.0) * num_c + np.maximum(PD, 0.0) * num_d
            else:
                PA = CF * (2.0 / soft - (1.0 + xs))
                PB = TR * (1.0 - 2.0 * xs * omx)
                val = np.maximum(PA, 0.0) * pdf(tab, eta / xs, t) + np.maximum(PB, 0.0) * pdf(TAB["g"], eta / xs, t)
            return np.where(ok, J * val / den, 0.0)
        return alphas(t) / (2 * math.pi) * zint(f, zlo, zhi)
    lim = s / 4.0 * (1.0 - eta) ** (2 if ii else 1) / eta
    return F, tc, lim


# ---- configurations ----

def qqg_event(n, sqrt_s=91.2, x=(0.9, 0.8, 0.3)):
    """n copies of an e+e- -> q qbar g configuration at sqrt(s) (energy
    fractions x_q, x_qbar, x_g summing to 2, massless, in the x-z plane): a d
    quark (colour 1), a gluon (colour 2, anticolour 1) and a d antiquark
    (anticolour 2), starting at s."""
    E = [xi * sqrt_s / 2 for xi in x]
    # quark along +z; the antiquark's angle from the gluon's momentum balance
    c12 = (E[2] ** 2 - E[0] ** 2 - E[1] ** 2) / (2 * E[0] * E[1])
    p_q = np.array([E[0], 0.0, 0.0, E[0]])
    p_qb = np.array([E[1], E[1] * math.sqrt(1 - c12 ** 2), 0.0, E[1] * c12])
    p_g = np.array([sqrt_s, 0.0, 0.0, 0.0]) - p_q - p_qb
    ev = records.Events(n, 128)
    for q, (p, pid, col, acol) in enumerate(((p_q, 1, 1, 0), (p_g, 21, 2, 1), (p_qb, -1, 0, 2))):
        ev.E[q], ev.px[q], ev.py[q], ev.pz[q] = p
        ev.pid[q], ev.col[q], ev.acol[q], ev.status[q] = pid, col, acol, 1
    ev.n[:] = 3
    ev.w[:] = 1.0
    ev.t_start[:] = sqrt_s ** 2
    ev.id[:] = np.arange(n)
    return ev, (p_q, p_g, p_qb)


def dot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def momentum(ev, q, e):
    return np.array([ev.E[q, e], ev.px[q, e], ev.py[q, e], ev.pz[q, e]])


# ---- the checks (each raises AssertionError on a mismatch) ----

def check_ff_qqg(o, form, n=20000, seed=11):
    """e+e- -> q qbar g: FF q -> q g with a gluon spectator and the gluon's two
    ends (g -> g g and g -> q qbar) with the quark and antiquark spectators."""
    ev, (pq, pg, pqb) = qqg_event(n)
    out = o.shower(ev, seed, nthreads=8, **form_kwargs(form))
    chans = [ff_channel(2 * dot(pq, pg), False), ff_channel(2 * dot(pg, pqb), True),
             ff_channel(2 * dot(pg, pq), True), ff_channel(2 * dot(pqb, pg), False)]
    tgrid = np.array([1.0, 1.5, 3.0, 10.0, 30.0, 100.0, 300.0, 1000.0])
    return compare(out.t1, tgrid, delta_curve(chans, tgrid))


def gluon_h_event(o, pick, nsample=400, seed=9):
    """An NLO H event q g -> Z q (incoming d or u quark and gluon, outgoing
    quark at slot 2) from the oracle's generator.  pick "fi": of those in the
    sample, the one whose outgoing quark has the largest transverse momentum
    (where the quark's FI end has the largest share of the emission
    probability); "is": the one whose gluon has the smallest momentum
    fraction (where the gluon's backward steps to a quark, family D, weigh
    most)."""
    base = o.hard_events(0, nsample, seed)
    best, which = -math.inf, -1
    for e in range(nsample):
        if (base.flags[e] & records.FLAG_HEVENT) and 21 in (base.pid[0, e], base.pid[1, e]) \
                and abs(base.pid[2, e]) in (1, 2):
            if pick == "fi":
                score = math.hypot(base.px[2, e], base.py[2, e])
            else:
                score = -base.E[0 if base.pid[0, e] == 21 else 1, e]
            if score > best:
                best, which = score, e
    assert which >= 0, "no q g -> Z q event in the sample"
    return base, which


def check_h_gluon(o, pdf, form, pick, n=40000, seed=13):
    """q g -> Z q: the incoming gluon's IF (outgoing quark spectator) and II
    (incoming quark spectator) ends, families C and D; the incoming quark's II
    end, families A and B; the outgoing quark's FI end q -> q g with the
    gluon's PDF ratio."""
    base, k = gluon_h_event(o, pick)
    ev = replicate(base, k, n)
    out = o.shower(ev, seed, nthreads=8, **form_kwargs(form))
    sq = 13000.0
    gslot = 0 if base.pid[0, k] == 21 else 1
    qslot = 1 - gslot
    pg, pq, pout = momentum(base, gslot, k), momentum(base, qslot, k), momentum(base, 2, k)
    eg, eq = 2 * pg[0] / sq, 2 * pq[0] / sq
    chans = [is_channel(pdf, "IF", 2 * dot(pg, pout), eg, 21),
             is_channel(pdf, "II", 2 * dot(pg, pq), eg, 21),
             is_channel(pdf, "II", 2 * dot(pq, pg), eq, int(base.pid[qslot, k])),
             fi_channel(pdf, 2 * dot(pout, pg), eg, TAB["g"], False)]
    tgrid = np.array([1.7, 3.0, 10.0, 30.0, 100.0, 300.0, 1000.0, 1e4])
    return compare(out.t1, tgrid, delta_curve(chans, tgrid))


def heavy_born(o, flavour, nsample=2000, seed=3):
    base = o.hard_events(0, nsample, seed)
    for e in range(nsample):
        if abs(base.pid[0, e]) == flavour:
            return base, e
    raise AssertionError(f"no flavour-{flavour} Born in the sample")


def check_heavy_born(o, pdf, form, flavour, n=20000, seed=17):
    """q qbar -> Z for a c or b quark: both II ends with appendix A.2's heavy
    quark measure.  The cutoff is m^2 + t_c; the density is the massless one
    (dt/(t - m^2) times (t - m^2)/t)."""
    base, k = heavy_born(o, flavour)
    ev = replicate(base, k, n)
    out = o.shower(ev, seed, nthreads=8, **form_kwargs(form))
    sq = 13000.0
    m2 = {4: 1.3 ** 2, 5: 4.75 ** 2}[flavour]
    tc = m2 + 1.0
    pa, pb = momentum(base, 0, k), momentum(base, 1, k)
    ea, eb = 2 * pa[0] / sq, 2 * pb[0] / sq
    s = 2 * dot(pa, pb)
    chans = [is_channel(pdf, "II", s, ea, int(base.pid[0, k]), tc=tc),
             is_channel(pdf, "II", s, eb, int(base.pid[1, k]), tc=tc)]
    tgrid = tc * np.array([0.9, 1.05, 1.2, 1.5, 2.0, 3.0, 6.0, 20.0, 100.0])
    return compare(out.t1, tgrid, delta_curve(chans, tgrid))


# ---- learned bound below the weight ----

def eta_bin(eta):
    """The overestimate table's eta bin: 48 bins uniform in ln eta on [1e-6, 1)."""
    l0 = math.log(1e-6)
    return int(min(47, max(0, math.floor((math.log(eta) - l0) / (-l0 / 48)))))


def check_learned_planted(o, pdf, retain, kappa=1.0 / 64, cell=2, n=20000, seed=5):
    """Learned mode with the analytic table in every cell except one: the
    family-A (q <- q) constant of both incoming quarks of a u ubar Born,
    at their eta bins, in ln t cell `cell`, lowered to kappa times the
    analytic one, far below the weights of the trials that land there.  With
    the weighted veto the weighted first-emission distribution is still the
    Sudakov quadrature.  Returns (worst/limit of that comparison, the largest
    deviation in standard errors of the rule that discards a violating event
    and showers it again on the analytic bound, applied to the same events)."""
    B = o.bounds()
    tab = np.ascontiguousarray(np.broadcast_to(B[8:72, :, None], (64, 48, 8))).copy()
    base = o.hard_events(0, 64, 3)
    k = next(e for e in range(64) if abs(base.pid[0, e]) == 2)
    sq = 13000.0
    ea, eb = 2 * base.E[0, k] / sq, 2 * base.E[1, k] / sq
    for pid, eta in ((base.pid[0, k], ea), (base.pid[1, k], eb)):
        ent = 8 + table_of(pid)  # family A of the quark's table
        tab[ent - 8, eta_bin(eta), cell] *= kappa
    ev = replicate(base, k, n)
    kw = dict(retain=True) if retain else {}
    out = o.shower_learned(ev, seed, tab, nthreads=8, **kw)
    fb = (out.flags & records.FLAG_FALLBACK) != 0
    assert fb.mean() > 0.01  # the planted cell is reached
    wfac = out.w / ev.w
    assert np.all(wfac[~fb] == 1.0) and np.all(np.abs(wfac[fb]) >= 1.0)
    s = 2 * dot(momentum(base, 0, k), momentum(base, 1, k))
    chans = [is_channel(pdf, "II", s, ea, int(base.pid[0, k])), is_channel(pdf, "II", s, eb, int(base.pid[1, k]))]
    tgrid = np.array([1.7, 3.0, 10.0, 30.0, 100.0, 300.0, 1000.0, 1e4, 1e5])
    delta = delta_curve(chans, tgrid)
    worst = compare(out.t1, tgrid, delta, w=wfac)
    plain = o.shower(ev, seed, nthreads=8, **kw)
    old = np.where(fb, plain.t1, out.t1)
    return worst, deviation(old, tgrid, delta)
