/* CPU oracle: hard-process events that feed the shower (appendix C and the
 * workload definitions).  Test infrastructure only. */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_int.h"

#define STREAM_HARD 2u
#define LO_MAXATT 1000

/* Li2 by its power series on [0, 1/2] and the reflection
 * Li2(x) = pi^2/6 - ln(x) ln(1-x) - Li2(1-x) above; x < 0 through
 * Li2(x) = -Li2(x/(x-1)) - ln^2(1-x)/2. */
double or_li2(double x) {
    if (x == 1.0) return OR_PI * OR_PI / 6.0;
    if (x < 0.0) {
        double l = log(1.0 - x);
        return -or_li2(x / (x - 1.0)) - 0.5 * l * l;
    }
    if (x > 0.5) return OR_PI * OR_PI / 6.0 - log(x) * log(1.0 - x) - or_li2(1.0 - x);
    double sum = 0.0, xk = x;
    for (int k = 1; k < 200; ++k) {
        double term = xk / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
        xk *= x;
    }
    return sum;
}

/* cos(theta) distributed as 1 + cos^2(theta): invert the cubic CDF (Cardano) */
static double cos_1pc2(double u) {
    double q = 4.0 - 8.0 * u;
    double sd = sqrt(0.25 * q * q + 1.0);
    return cbrt(-0.5 * q + sd) + cbrt(-0.5 * q - sd);
}

/* V^2 + A^2 of the Z coupling to quark flavour |f| */
static double zcoup(const or_state* s, int f) {
    int a = abs(f);
    double V, A;
    if (a % 2 == 0) { V = 0.5 - 4.0 / 3.0 * s->c.sw2; A = 0.5; }
    else { V = -0.5 + 2.0 / 3.0 * s->c.sw2; A = -0.5; }
    return V * V + A * A;
}

static double xfp(const or_state* s, int pid, double x, double q2) {
    return or_pdf_xf(s, or_pdf_table(pid), x, q2);
}

static void put(or_events* o, int64_t e, int slot, const double* p, int pid, int col, int acol,
                int st) {
    int64_t k = (int64_t)slot * o->cap + e;
    o->E[k] = p[0]; o->px[k] = p[1]; o->py[k] = p[2]; o->pz[k] = p[3];
    o->pid[k] = pid; o->col[k] = col; o->acol[k] = acol; o->status[k] = (int8_t)st;
}

/* the pair of mass m and momentum pZ decays to e- e+, the electron at polar
 * cosine c (about +z) and azimuth 2 pi uphi in the pair's rest frame, boosted
 * along pZ */
static void decay_zc(const double* pZ, double m, double c, double uphi, double* em, double* ep) {
    double st = sqrt(fmax(0.0, 1.0 - c * c)), ph = 2.0 * OR_PI * uphi;
    double k[4] = {0.5 * m, 0.5 * m * st * cos(ph), 0.5 * m * st * sin(ph), 0.5 * m * c};
    double pk = pZ[1] * k[1] + pZ[2] * k[2] + pZ[3] * k[3];
    double E1 = (pZ[0] * k[0] + pk) / m;
    double f = (k[0] + E1) / (pZ[0] + m);
    em[0] = E1;
    for (int m3 = 1; m3 < 4; ++m3) em[m3] = k[m3] + f * pZ[m3];
    for (int m3 = 0; m3 < 4; ++m3) ep[m3] = pZ[m3] - em[m3];
}

/* Z -> e- e+ with 1 + cos^2 in the Z rest frame */
static void decay_z(const double* pZ, double m, double ucos, double uphi, double* em, double* ep) {
    decay_zc(pZ, m, cos_1pc2(ucos), uphi, em, ep);
}

/* q qbar -> Z/photon -> e- e+ at s = m2 for quark flavour f: the coefficients
 * of (1 + cos^2 theta) and of 2 cos theta in the cross section over its
 * photon-only value for unit charges, theta the angle between the incoming
 * quark and the electron in the pair's rest frame.  Couplings v = T3 - 2 Q
 * sin^2(theta_W), a = T3; chi = s / (s - mZ^2 + i mZ GammaZ) /
 * (4 sin^2 cos^2). */
static void dy_f12(const or_state* s, int f, double m2, double* F1, double* F2) {
    const double sw2 = s->c.sw2, mz2 = s->c.mz * s->c.mz, mg = s->c.mz * s->c.gz;
    const int up = abs(f) % 2 == 0;
    const double Qq = up ? 2.0 / 3.0 : -1.0 / 3.0, Qe = -1.0;
    const double vq = up ? 0.5 - 4.0 / 3.0 * sw2 : -0.5 + 2.0 / 3.0 * sw2, aq = up ? 0.5 : -0.5;
    const double ve = -0.5 + 2.0 * sw2, ae = -0.5;
    const double kap = 1.0 / (4.0 * sw2 * (1.0 - sw2));
    const double d = m2 - mz2, D = d * d + mg * mg;
    const double rechi = kap * m2 * d / D, chi2 = kap * kap * m2 * m2 / D;
    *F1 = Qq * Qq * Qe * Qe + 2.0 * Qq * Qe * vq * ve * rechi + (vq * vq + aq * aq) * (ve * ve + ae * ae) * chi2;
    *F2 = 2.0 * Qq * Qe * aq * ae * rechi + 4.0 * vq * aq * ve * ae * chi2;
}

static void clear_counters(or_events* o, int64_t e) {
    if (o->n_cycles) o->n_cycles[e] = 0;
    if (o->n_trials) o->n_trials[e] = 0;
    if (o->n_accept) o->n_accept[e] = 0;
    if (o->n_viol) o->n_viol[e] = 0;
    if (o->t1) o->t1[e] = 0.0;
}

static void gen_ee(const or_state* s, int64_t id, uint64_t seed, or_events* o, int64_t e) {
    double u[4];
    or_rng_block(seed, STREAM_HARD, id, 0u, 0u, u);
    int f = 1 + (int)(u[0] * s->c.nf);
    if (f > s->c.nf) f = s->c.nf;
    double c = cos_1pc2(u[1]), st = sqrt(fmax(0.0, 1.0 - c * c)), ph = 2.0 * OR_PI * u[2];
    double E = 0.5 * s->sqrtS;
    double q[4] = {E, E * st * cos(ph), E * st * sin(ph), E * c};
    double qb[4] = {E, -q[1], -q[2], -q[3]};
    put(o, e, 0, q, f, 1, 0, 1);
    put(o, e, 1, qb, -f, 0, 1, 1);
    o->n[e] = 2; o->w[e] = 1.0; o->t_start[e] = s->S; o->flags[e] = 0;
}

/* Drell-Yan luminosity sum over the ten q qbar orientations at (m, y) */
static double lo_lumi(const or_state* s, double m, double y, double* csub) {
    double m2 = m * m;
    double e1 = m / s->sqrtS * exp(y), e2 = m / s->sqrtS * exp(-y);
    double L = 0.0;
    for (int f = 1; f <= s->c.nf; ++f) {
        double v = zcoup(s, f);
        double a = v * xfp(s, f, e1, m2) * xfp(s, -f, e2, m2);
        double b = v * xfp(s, -f, e1, m2) * xfp(s, f, e2, m2);
        if (csub) { csub[2 * (f - 1)] = a; csub[2 * (f - 1) + 1] = b; }
        L += a + b;
    }
    return L;
}

/* The same with the Z/photon cross section: per q qbar orientation the
 * luminosity times F1 (m^2 - mZ^2)^2 + mZ^2 GammaZ^2) / m^4, the density of
 * d sigma / dm^2 dy over the Breit-Wigner the masses are drawn from */
static double dy_lumi(const or_state* s, double m, double y, double* csub) {
    double m2 = m * m;
    double e1 = m / s->sqrtS * exp(y), e2 = m / s->sqrtS * exp(-y);
    const double d = m2 - s->c.mz * s->c.mz, mg = s->c.mz * s->c.gz;
    const double bw = (d * d + mg * mg) / (m2 * m2);
    double L = 0.0;
    for (int f = 1; f <= s->c.nf; ++f) {
        double F1, F2;
        dy_f12(s, f, m2, &F1, &F2);
        double g = F1 * bw;
        double a = g * xfp(s, f, e1, m2) * xfp(s, -f, e2, m2);
        double b = g * xfp(s, -f, e1, m2) * xfp(s, f, e2, m2);
        if (csub) { csub[2 * (f - 1)] = a; csub[2 * (f - 1) + 1] = b; }
        L += a + b;
    }
    return L;
}

double or_lo_scan_wmax(const or_state* s) {
    double best = 0.0;
    for (int i = 0; i < 64; ++i) {
        double m = s->c.mll_min + (s->c.mll_max - s->c.mll_min) * i / 63.0;
        double Y = log(s->sqrtS / m);
        for (int j = 0; j < 128; ++j) {
            double y = -Y + 2.0 * Y * (j + 0.5) / 128.0;
            double W = (s->c.process == 3 ? dy_lumi(s, m, y, NULL) : lo_lumi(s, m, y, NULL)) * 2.0 * Y;
            if (W > best) best = W;
        }
    }
    return or_quarter_octave_up(1.25 * best);
}

static void gen_lo(const or_state* s, int64_t id, uint64_t seed, or_events* o, int64_t e) {
    double mz2 = s->c.mz * s->c.mz, mg = s->c.mz * s->c.gz;
    double r1 = atan((s->c.mll_min * s->c.mll_min - mz2) / mg);
    double r2 = atan((s->c.mll_max * s->c.mll_max - mz2) / mg);
    double csub[10];
    for (int k = 0; k < LO_MAXATT; ++k) {
        double u[4];
        or_rng_block(seed, STREAM_HARD, id, (uint32_t)k, 0u, u);
        double m2 = mz2 + mg * tan(r1 + u[0] * (r2 - r1));
        double m = sqrt(m2);
        double Y = log(s->sqrtS / m), y = -Y + 2.0 * Y * u[1];
        double L = lo_lumi(s, m, y, csub);
        if (!(u[2] * s->lo_wmax < L * 2.0 * Y)) continue;
        double target = u[3] * L, cum = 0.0;
        int sel = 2 * s->c.nf - 1;
        for (int q = 0; q < 2 * s->c.nf; ++q) {
            cum += csub[q];
            if (target < cum) { sel = q; break; }
        }
        int f = sel / 2 + 1;
        int pa = (sel % 2 == 0) ? f : -f, pb = -pa;
        double e1 = m / s->sqrtS * exp(y), e2 = m / s->sqrtS * exp(-y);
        double Ea = 0.5 * e1 * s->sqrtS, Eb = 0.5 * e2 * s->sqrtS;
        double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
        put(o, e, 0, A, pa, pa > 0 ? 1 : 0, pa > 0 ? 0 : 1, -1);
        put(o, e, 1, B, pb, pb > 0 ? 1 : 0, pb > 0 ? 0 : 1, -1);
        double pZ[4] = {A[0] + B[0], 0.0, 0.0, A[3] + B[3]}, em[4], ep[4];
        double ud[4];
        or_rng_block(seed, STREAM_HARD, id, 0xFFFFFFFFu, 0u, ud);
        decay_z(pZ, m, ud[0], ud[1], em, ep);
        put(o, e, 2, em, 11, 0, 0, 1);
        put(o, e, 3, ep, -11, 0, 0, 1);
        o->n[e] = 4; o->w[e] = 1.0;
        o->t_start[e] = s->c.matching == 1 ? s->c.mu_q2 : s->S;
        o->flags[e] = s->c.matching == 2 ? OR_F_MEC : 0u;
        return;
    }
    o->n[e] = 0; o->w[e] = 0.0; o->t_start[e] = s->S; o->flags[e] = OR_F_HARDFAIL;
}

/* pp -> Z/photon -> e- e+ at LO with the photon, the Z and their
 * interference: (m, y) and the q qbar orientation as for the Z alone with the
 * Z/photon weight, then cos(theta) between the quark and the electron by
 * accept-reject on (1 + c^2) F1 + 2 c F2 from proposals distributed as 1 + c^2
 * (block (id, 2^32 - 1, j) of attempt j: proposal, acceptance, azimuth) */
static void gen_dy(const or_state* s, int64_t id, uint64_t seed, or_events* o, int64_t e) {
    double mz2 = s->c.mz * s->c.mz, mg = s->c.mz * s->c.gz;
    double r1 = atan((s->c.mll_min * s->c.mll_min - mz2) / mg);
    double r2 = atan((s->c.mll_max * s->c.mll_max - mz2) / mg);
    double csub[10];
    for (int k = 0; k < LO_MAXATT; ++k) {
        double u[4];
        or_rng_block(seed, STREAM_HARD, id, (uint32_t)k, 0u, u);
        double m2 = mz2 + mg * tan(r1 + u[0] * (r2 - r1));
        double m = sqrt(m2);
        double Y = log(s->sqrtS / m), y = -Y + 2.0 * Y * u[1];
        double L = dy_lumi(s, m, y, csub);
        if (!(u[2] * s->lo_wmax < L * 2.0 * Y)) continue;
        double target = u[3] * L, cum = 0.0;
        int sel = 2 * s->c.nf - 1;
        for (int q = 0; q < 2 * s->c.nf; ++q) {
            cum += csub[q];
            if (target < cum) { sel = q; break; }
        }
        int f = sel / 2 + 1;
        int pa = (sel % 2 == 0) ? f : -f, pb = -pa;
        double e1 = m / s->sqrtS * exp(y), e2 = m / s->sqrtS * exp(-y);
        double Ea = 0.5 * e1 * s->sqrtS, Eb = 0.5 * e2 * s->sqrtS;
        double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
        double pZ[4] = {A[0] + B[0], 0.0, 0.0, A[3] + B[3]}, em[4], ep[4];
        double F1, F2;
        dy_f12(s, f, m2, &F1, &F2);
        const double sq = pa > 0 ? 1.0 : -1.0; /* the quark moves along +z when beam A carries it */
        for (int j = 0; j < LO_MAXATT; ++j) {
            double ud[4];
            or_rng_block(seed, STREAM_HARD, id, 0xFFFFFFFFu, (uint32_t)j, ud);
            const double c = cos_1pc2(ud[0]);
            const double acc = ((1.0 + c * c) * F1 + 2.0 * c * F2) / ((1.0 + c * c) * (F1 + fabs(F2)));
            if (!(ud[1] < acc)) continue;
            put(o, e, 0, A, pa, pa > 0 ? 1 : 0, pa > 0 ? 0 : 1, -1);
            put(o, e, 1, B, pb, pb > 0 ? 1 : 0, pb > 0 ? 0 : 1, -1);
            decay_zc(pZ, m, sq * c, ud[2], em, ep);
            put(o, e, 2, em, 11, 0, 0, 1);
            put(o, e, 3, ep, -11, 0, 0, 1);
            o->n[e] = 4; o->w[e] = 1.0; o->t_start[e] = s->S; o->flags[e] = 0;
            return;
        }
        break;
    }
    o->n[e] = 0; o->w[e] = 0.0; o->t_start[e] = s->S; o->flags[e] = OR_F_HARDFAIL;
}

/* NLO building blocks of appendix C.3-C.4 at muF = muR = mZ (the logarithms of
 * muF^2/m^2 vanish) */
double or_nlo_bvi_factor(const or_state* s) {
    return 1.0 + OR_CF * s->c.alphas_mz / (2.0 * OR_PI) * 2.0;
}
double or_nlo_aqq(const or_state* s) {
    return OR_CF * s->c.alphas_mz / (2.0 * OR_PI) * (-5.0 + 2.0 * OR_PI * OR_PI / 3.0);
}
double or_nlo_bqq(const or_state* s, double eta) {
    double l = log(1.0 - eta);
    return OR_CF * s->c.alphas_mz / (2.0 * OR_PI) * 2.0 *
           (OR_PI * OR_PI / 6.0 - l * l - or_li2(1.0 - eta));
}
double or_nlo_gqq(const or_state* s, double x) {
    double L = log((1.0 - x) / x) + log(1.0 - x);
    return OR_CF * s->c.alphas_mz / (2.0 * OR_PI) * (2.0 / (1.0 - x)) * L;
}
static double nlo_hqq(const or_state* s, double x) {
    double L = log((1.0 - x) / x) + log(1.0 - x);
    return OR_CF * s->c.alphas_mz / (2.0 * OR_PI) * (-(1.0 + x) * L + (1.0 - x));
}
static double nlo_hqg(const or_state* s, double x) {
    double L = log((1.0 - x) / x) + log(1.0 - x);
    return OR_TR * s->c.alphas_mz / (2.0 * OR_PI) *
           (2.0 * x * (1.0 - x) + (x * x + (1.0 - x) * (1.0 - x)) * L);
}

/* collinear insertion for one leg with Born parton b at eta, one-point sample x */
static double k_leg(const or_state* s, int b, double eta, double x, double q2) {
    double den = or_pdf_f(s, or_pdf_table(b), eta, q2);
    if (!(den > 0.0)) return 0.0;
    double rq = or_pdf_f(s, or_pdf_table(b), eta / x, q2) / (x * den);
    double rg = or_pdf_f(s, 0, eta / x, q2) / (x * den);
    return or_nlo_aqq(s) - or_nlo_bqq(s, eta) +
           (1.0 - eta) * ((rq - 1.0) * or_nlo_gqq(s, x) + rq * nlo_hqq(s, x) + rg * nlo_hqg(s, x));
}

/* Radiation integral of one leg of a Born event at fixed Born kinematics, as a
 * one-point estimate (x uniform on [eta, 1], v uniform on [0, 1 - x]) relative
 * to the Born.  It covers the real configurations that the initial-initial map
 * with this leg as emitter (appendix B.5) sends onto the Born: the leg's parton
 * then carries eta / x, and the gluon-initiated ones take the gluon PDF.  Per
 * unit Born the real emission's measure is m^2 / (16 pi^2 |M_B|^2) dx dv times
 * the PDF ratio.
 *   matching 1: minus the leg's dipoles (appendix C.2) where the emission's
 *               kT^2 = v (1 - x - v) m^2 / x reaches mu_q2 (the region that the
 *               S events' shower, started at mu_q2, no longer subtracts)
 *   matching 2: R - S assigned to this leg's map; for q qbar -> Z g the share
 *               of this leg's dipole in the dipole sum, (1 - x - v) / (1 - x) */
static double leg_rad(const or_state* s, int b, double eta, double x, double v, double q2) {
    double den = or_pdf_f(s, or_pdf_table(b), eta, q2);
    if (!(den > 0.0)) return 0.0;
    double rq = or_pdf_f(s, or_pdf_table(b), eta / x, q2) / (x * den);
    double rg = or_pdf_f(s, 0, eta / x, q2) / (x * den);
    double aq = OR_CF * s->c.alphas_mz / (2.0 * OR_PI), ag = OR_TR * s->c.alphas_mz / (2.0 * OR_PI);
    double omx = 1.0 - x, m2 = s->c.mz * s->c.mz, g;
    if (s->c.matching == 1) {
        double kt2 = v * (omx - v) * m2 / x;
        if (!(kt2 >= s->c.mu_q2)) return 0.0;
        g = -(aq * (1.0 + x * x) / (omx * v) * rq + ag * (x * x + omx * omx) / v * rg);
    } else {
        g = -2.0 * aq * (omx - v) / omx * rq + ag * (2.0 * x + v) * rg;
    }
    return (1.0 - eta) * omx * g;
}

/* The dipole sum S of a real configuration (appendix C.2) in the variables of
 * its generation, x = m^2/sbar and va = -ubar/sbar (the emitted parton against
 * beam A): for q qbar -> Z g (kind 0) the two initial-state q -> q g dipoles,
 * for g q (kind 1: gluon at A, kind 2: gluon at B) the gluon's g -> q qbar
 * dipole; in units of 8 pi alpha_s |M_B|^2 / m^2 times C_F (kind 0) or T_R, so
 * that with or_nlo_rs it gives R = S + (R - S). */
double or_nlo_sub(int kind, double x, double va) {
    double vb = 1.0 - x - va;
    if (kind == 0) return (1.0 + x * x) / (va * vb);
    return (x * x + (1.0 - x) * (1.0 - x)) / (kind == 1 ? va : vb);
}

/* real minus subtraction in closed form (appendix C.2); kind 0: q qbar -> Z g,
 * kind 1: g q -> Z q with ubar measured from the gluon */
void or_nlo_rs(const or_state* s, int kind, double sbar, double tbar, double ubar, double mborn2,
               double* r_minus_s) {
    double m2 = s->c.mz * s->c.mz;
    (void)tbar;
    if (kind == 0) *r_minus_s = 8.0 * OR_PI * s->c.alphas_mz * OR_CF / m2 * mborn2 * (-2.0);
    else *r_minus_s = 8.0 * OR_PI * s->c.alphas_mz * OR_TR / m2 * mborn2 * ((2.0 * m2 - ubar) / sbar);
}

static double mborn2(const or_state* s, int f) {
    double m2 = s->c.mz * s->c.mz;
    return 1.0 / OR_NC * 0.25 * sqrt(2.0) * s->c.gf * m2 * m2 * zcoup(s, f);
}

static void gen_nlo(const or_state* s, int64_t id, uint64_t seed, or_events* o, int64_t e) {
    double u0[4], u1[4];
    or_rng_block(seed, STREAM_HARD, id, 0u, 0u, u0);
    or_rng_block(seed, STREAM_HARD, id, 1u, 0u, u1);
    const double m = s->c.mz, m2 = m * m, q2 = m2;
    const int nf = s->c.nf;
    const int mt = s->c.matching;
    if (mt == 2 || u0[0] < s->c.p_s) {
        /* S event: Born x (B + V + I + collinear); matching 1 and 2 add the
         * legs' radiation integrals (x of the collinear term, v from u1[2] and
         * block (id, 2)) */
        double Y = log(s->sqrtS / m), y = -Y + 2.0 * Y * u0[2];
        double e1 = m / s->sqrtS * exp(y), e2 = m / s->sqrtS * exp(-y);
        double xa = e1 + (1.0 - e1) * u1[0], xb = e2 + (1.0 - e2) * u1[1];
        double va = 0.0, vb = 0.0;
        if (mt != 0) {
            double u2[4];
            or_rng_block(seed, STREAM_HARD, id, 2u, 0u, u2);
            va = (1.0 - xa) * u1[2];
            vb = (1.0 - xb) * u2[0];
        }
        double csub[10], W = 0.0;
        for (int f = 1; f <= nf; ++f)
            for (int o2 = 0; o2 < 2; ++o2) {
                int a = o2 == 0 ? f : -f, b = -a;
                double born = OR_PI / (m2 * m2) * mborn2(s, f) * xfp(s, a, e1, q2) * xfp(s, b, e2, q2);
                double corr = or_nlo_bvi_factor(s) + k_leg(s, a, e1, xa, q2) + k_leg(s, b, e2, xb, q2);
                if (mt != 0) corr += leg_rad(s, a, e1, xa, va, q2) + leg_rad(s, b, e2, xb, vb, q2);
                csub[2 * (f - 1) + o2] = born * corr;
                W += fabs(born * corr);
            }
        double target = u0[1] * W, cum = 0.0;
        int sel = 2 * nf - 1;
        for (int q = 0; q < 2 * nf; ++q) {
            cum += fabs(csub[q]);
            if (target < cum) { sel = q; break; }
        }
        int f = sel / 2 + 1, a = (sel % 2 == 0) ? f : -f, b = -a;
        double Ea = 0.5 * e1 * s->sqrtS, Eb = 0.5 * e2 * s->sqrtS;
        double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
        put(o, e, 0, A, a, a > 0 ? 1 : 0, a > 0 ? 0 : 1, -1);
        put(o, e, 1, B, b, b > 0 ? 1 : 0, b > 0 ? 0 : 1, -1);
        double pZ[4] = {A[0] + B[0], 0.0, 0.0, A[3] + B[3]}, em[4], ep[4];
        decay_z(pZ, m, u0[3], u1[3], em, ep);
        put(o, e, 2, em, 11, 0, 0, 1);
        put(o, e, 3, ep, -11, 0, 0, 1);
        o->n[e] = 4;
        o->w[e] = (csub[sel] < 0.0 ? -W : W) * 2.0 * Y / (mt == 2 ? 1.0 : s->c.p_s);
        o->t_start[e] = mt == 1 ? s->c.mu_q2 : s->S;
        o->flags[e] = mt == 2 ? OR_F_MEC : 0u;
        return;
    }
    /* H event: real minus subtraction, kinematics from the II map with j = 2 */
    double xmin = m2 / s->S;
    double x = xmin + (1.0 - xmin) * u1[0], sbar = m2 / x;
    double YH = 0.5 * log(s->S * x / m2), y = -YH + 2.0 * YH * u0[2];
    double ea = exp(y) * sqrt(sbar / s->S), eb = exp(-y) * sqrt(sbar / s->S);
    double v = (1.0 - x) * u1[1], ph = 2.0 * OR_PI * u1[2];
    double Ea = 0.5 * ea * s->sqrtS, Eb = 0.5 * eb * s->sqrtS;
    double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
    double kt0 = sqrt(v * (1.0 - x - v) * sbar);
    double J[4];
    for (int k = 0; k < 4; ++k) J[k] = (1.0 - x - v) * A[k] + v * B[k];
    J[1] -= kt0 * cos(ph);
    J[2] -= kt0 * sin(ph);
    double pZ[4];
    for (int k = 0; k < 4; ++k) pZ[k] = A[k] + B[k] - J[k];
    double ubar = -2.0 * (A[0] * J[0] - A[1] * J[1] - A[2] * J[2] - A[3] * J[3]);
    double tbar = -2.0 * (B[0] * J[0] - B[1] * J[1] - B[2] * J[2] - B[3] * J[3]);
    double csub[30], W = 0.0;
    int pa[30], pb[30], kind[30];
    int q = 0;
    /* matching 1: above the start scale the S events' shower subtracts
     * nothing, so there the H events keep the dipole sum (their weight is R) */
    const int above = mt == 1 && v * (1.0 - x - v) * sbar >= s->c.mu_q2;
    const double sq = 8.0 * OR_PI * s->c.alphas_mz * OR_CF / m2, sg = 8.0 * OR_PI * s->c.alphas_mz * OR_TR / m2;
    for (int f = 1; f <= nf; ++f) {
        double mb = mborn2(s, f), rs;
        or_nlo_rs(s, 0, sbar, tbar, ubar, mb, &rs);
        if (above) rs += sq * mb * or_nlo_sub(0, x, v);
        pa[q] = f; pb[q] = -f; kind[q] = 0; csub[q++] = rs;
        pa[q] = -f; pb[q] = f; kind[q] = 0; csub[q++] = rs;
        or_nlo_rs(s, 1, sbar, tbar, ubar, mb, &rs);
        if (above) rs += sg * mb * or_nlo_sub(1, x, v);
        pa[q] = 21; pb[q] = f; kind[q] = 1; csub[q++] = rs;
        pa[q] = 21; pb[q] = -f; kind[q] = 1; csub[q++] = rs;
        or_nlo_rs(s, 1, sbar, ubar, tbar, mb, &rs);
        if (above) rs += sg * mb * or_nlo_sub(2, x, v);
        pa[q] = f; pb[q] = 21; kind[q] = 2; csub[q++] = rs;
        pa[q] = -f; pb[q] = 21; kind[q] = 2; csub[q++] = rs;
    }
    for (int k = 0; k < q; ++k) {
        csub[k] *= xfp(s, pa[k], ea, q2) * xfp(s, pb[k], eb, q2) / (16.0 * OR_PI * m2);
        W += fabs(csub[k]);
    }
    double target = u0[1] * W, cum = 0.0;
    int sel = q - 1;
    for (int k = 0; k < q; ++k) {
        cum += fabs(csub[k]);
        if (target < cum) { sel = k; break; }
    }
    int a = pa[sel], b = pb[sel];
    int ca, aa, cb, ab, jp, cj, aj;
    if (kind[sel] == 0) {
        /* q qbar -> Z g: quark colour 1, antiquark anticolour 2, gluon (1, 2) */
        ca = a > 0 ? 1 : 0; aa = a > 0 ? 0 : 2;
        cb = b > 0 ? 1 : 0; ab = b > 0 ? 0 : 2;
        jp = 21; cj = 1; aj = 2;
    } else {
        int qk = kind[sel] == 1 ? b : a; /* the incoming (anti)quark */
        int cg = 1, ag = 2, cq, aq;
        if (qk > 0) { cq = 2; aq = 0; cj = 1; aj = 0; }
        else { cq = 0; aq = 1; cj = 0; aj = 2; }
        jp = qk;
        if (kind[sel] == 1) { ca = cg; aa = ag; cb = cq; ab = aq; }
        else { ca = cq; aa = aq; cb = cg; ab = ag; }
    }
    put(o, e, 0, A, a, ca, aa, -1);
    put(o, e, 1, B, b, cb, ab, -1);
    put(o, e, 2, J, jp, cj, aj, 1);
    double em[4], ep[4];
    decay_z(pZ, m, u0[3], u1[3], em, ep);
    put(o, e, 3, em, 11, 0, 0, 1);
    put(o, e, 4, ep, -11, 0, 0, 1);
    o->n[e] = 5;
    o->w[e] = (csub[sel] < 0.0 ? -W : W) * 2.0 * YH * (1.0 - xmin) * (1.0 - x) / (1.0 - s->c.p_s);
    o->t_start[e] = mt == 1 ? s->c.mu_q2 : s->S;
    o->flags[e] = OR_F_HEVENT;
}

/* ---------------------------------------------------------------------------
 * pp -> Z/photon -> e- e+ at NLO (the second workload at NLO, MC@NLO S and H
 * events with the power shower), the real emission by the Kleiss trick.
 *
 * Born q(p_q) qbar -> e-(p3) e+(p4) at s = m^2, in units common to S and H
 * events (coupling and colour constants dropped):
 *   |M_0|^2 = (a(s) u^2 + b(s) t^2) / s^2,  t = (p_q - p3)^2,  u = (p_q - p4)^2,
 *   a = |A_LL|^2 + |A_RR|^2,  b = |A_LR|^2 + |A_RL|^2,
 *   A_ij = Q_q Q_e + g_i^q g_j^e s / (s - mZ^2 + i mZ GZ) / (sin^2 cos^2),
 * chiral couplings g_L = T3 - Q sin^2, g_R = -Q sin^2 (helicity amplitudes;
 * (1 + c^2) F1 + 2 c F2 of process 3 in other variables).
 * Real q qbar -> e- e+ g by the Kleiss trick (every NLO matrix element from
 * LO ones): with t' = (p_qbar - p4)^2, u' = (p_qbar - p3)^2 and s' = m^2,
 *   |M_R|^2 = g^2 C_F (a(s') (u^2 + u'^2) + b(s') (t^2 + t'^2)) /
 *             (2 s' (p_q.k)(p_qbar.k)),
 * g^2 = 4 pi alpha_s; g qbar -> e- e+ qbar and g q -> e- e+ q by crossing
 * (p_q = -p_j or p_qbar = -p_j, k = -p_g), times -3/8 (the colour and spin
 * averages of a gluon, the fermion sign).  The subtraction is the sum of the
 * initial-initial dipoles (appendix C.2) with the Born at the mapped momenta
 * (appendix B.5's map backwards: the emitter x p_e, the leptons transformed
 * by the Lorentz map of K = p_a + p_b - k onto x p_e + p_s).  The PDFs are at
 * mu_F^2 = m^2; alpha_s is alpha_s(mZ) as for the Z. */
static void dy_hel(const or_state* s, int f, double m2, double* al, double* be) {
    const double sw2 = s->c.sw2, mz2 = s->c.mz * s->c.mz, mg = s->c.mz * s->c.gz;
    const int up = abs(f) % 2 == 0;
    const double Qq = up ? 2.0 / 3.0 : -1.0 / 3.0, T3 = up ? 0.5 : -0.5, Qe = -1.0, T3e = -0.5;
    const double gq[2] = {T3 - Qq * sw2, -Qq * sw2}, ge[2] = {T3e - Qe * sw2, -Qe * sw2};
    const double d = m2 - mz2, D = d * d + mg * mg, k = 1.0 / (sw2 * (1.0 - sw2));
    const double rex = k * m2 * d / D, imx = -k * m2 * mg / D; /* s / (s - mZ^2 + i mZ GZ) */
    double A2[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double re = Qq * Qe + gq[i] * ge[j] * rex, im = gq[i] * ge[j] * imx;
            A2[i][j] = re * re + im * im;
        }
    *al = A2[0][0] + A2[1][1];
    *be = A2[0][1] + A2[1][0];
}

static double dot(const double* a, const double* b) {
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

static double born_dy(double al, double be, const double* pq, const double* p3, const double* p4) {
    double t = -2.0 * dot(pq, p3), u = -2.0 * dot(pq, p4), s = 2.0 * dot(p3, p4);
    return (al * u * u + be * t * t) / (s * s);
}

/* the Kleiss-trick real matrix element of q(pq) qbar(pqb) -> e-(p3) e+(p4) g(k)
 * over g^2 C_F (momenta may be crossed, i.e. negative) */
static double kleiss(double al, double be, const double* pq, const double* pqb, const double* k,
                     const double* p3, const double* p4) {
    double t = -2.0 * dot(pq, p3), u = -2.0 * dot(pq, p4);
    double tp = -2.0 * dot(pqb, p4), up = -2.0 * dot(pqb, p3);
    double sp = 2.0 * dot(p3, p4);
    return (al * (u * u + up * up) + be * (t * t + tp * tp)) / (2.0 * sp * dot(pq, k) * dot(pqb, k));
}

/* the lepton momenta p of a real configuration mapped onto its Born by the
 * initial-initial dipole of emitter pe (and spectator ps, emitted k): the
 * Lorentz map of pe + ps - k onto x pe + ps */
static void dy_project(const double* pe, const double* ps, const double* k, double x, double* p) {
    double K[4], Kt[4], S[4];
    for (int m = 0; m < 4; ++m) {
        K[m] = pe[m] + ps[m] - k[m];
        Kt[m] = x * pe[m] + ps[m];
        S[m] = K[m] + Kt[m];
    }
    double c1 = 2.0 * dot(S, p) / dot(S, S), c2 = 2.0 * dot(K, p) / dot(K, K);
    for (int m = 0; m < 4; ++m) p[m] = p[m] - c1 * S[m] + c2 * Kt[m];
}

/* the dipole sum of a real configuration, over 8 pi alpha_s: beams A (pa) and
 * B (pb) with flavours fa, fb (21: gluon), emitted parton k, leptons p3, p4,
 * the Born's angular weights al, be at the pair mass (the map keeps it) */
static double dy_dipoles(int fa, int fb, const double* pa, const double* pb, const double* k, const double* p3,
                         const double* p4, double x, double al, double be) {
    double sum = 0.0;
    for (int side = 0; side < 2; ++side) {
        const int fe = side == 0 ? fa : fb, fs = side == 0 ? fb : fa;
        const double *pe = side == 0 ? pa : pb, *ps = side == 0 ? pb : pa;
        if (fs == 21) continue; /* the spectator of a Born leg is a quark */
        double q3[4], q4[4], pem[4];
        memcpy(q3, p3, sizeof(q3));
        memcpy(q4, p4, sizeof(q4));
        dy_project(pe, ps, k, x, q3);
        dy_project(pe, ps, k, x, q4);
        for (int m = 0; m < 4; ++m) pem[m] = x * pe[m];
        /* the Born's quark flavour at the emitter: the emitter's own, or (gluon)
         * the one conjugate to the spectator */
        const int qe = fe == 21 ? -fs : fe;
        const double* pq = qe > 0 ? pem : ps;
        double B = born_dy(al, be, pq, q3, q4);
        double V = fe == 21 ? OR_TR * (1.0 - 2.0 * x * (1.0 - x)) : OR_CF * (1.0 + x * x) / (1.0 - x);
        sum += V / (x * 2.0 * dot(pe, k)) * B;
    }
    return sum;
}

/* The momenta of a real configuration: beams A, B, the emitted parton J (the
 * initial-initial map's variables x = m^2/sbar, v against beam A, azimuth
 * phi, rapidity y of the pair of beams), the leptons from the pair's decay at
 * polar cosine c and azimuth 2 pi uphi in its rest frame. */
static void dy_real_kin(const or_state* s, double m2, double x, double y, double v, double ph, double c,
                        double uphi, double* A, double* B, double* J, double* em, double* ep) {
    double sbar = m2 / x;
    double ea = exp(y) * sqrt(sbar / s->S), eb = exp(-y) * sqrt(sbar / s->S);
    double Ea = 0.5 * ea * s->sqrtS, Eb = 0.5 * eb * s->sqrtS;
    A[0] = Ea; A[1] = 0.0; A[2] = 0.0; A[3] = Ea;
    B[0] = Eb; B[1] = 0.0; B[2] = 0.0; B[3] = -Eb;
    double kt0 = sqrt(v * (1.0 - x - v) * sbar), pZ[4];
    for (int k = 0; k < 4; ++k) J[k] = (1.0 - x - v) * A[k] + v * B[k];
    J[1] -= kt0 * cos(ph);
    J[2] -= kt0 * sin(ph);
    for (int k = 0; k < 4; ++k) pZ[k] = A[k] + B[k] - J[k];
    decay_zc(pZ, sqrt(m2), c, uphi, em, ep);
}

/* R and the dipole sum S of one channel of a real configuration: kind 0
 * q qbar -> e- e+ g with the quark at A (fa > 0) or B; kind 1 the gluon at A,
 * kind 2 at B, the (anti)quark fa or fb at the other beam */
static void dy_real_rs(const or_state* s, int kind, int fa, int fb, double al, double be, const double* A,
                       const double* B, const double* J, const double* em, const double* ep, double x, double* R,
                       double* S) {
    const double g2 = 4.0 * OR_PI * s->c.alphas_mz;
    double mJ[4], mA[4], mB[4];
    for (int k = 0; k < 4; ++k) { mJ[k] = -J[k]; mA[k] = -A[k]; mB[k] = -B[k]; }
    if (kind == 0) {
        *R = g2 * OR_CF * kleiss(al, be, fa > 0 ? A : B, fa > 0 ? B : A, J, em, ep);
    } else if (kind == 1) {
        /* the outgoing parton is the same as B's */
        *R = -0.375 * g2 * OR_CF * (fb > 0 ? kleiss(al, be, B, mJ, mA, em, ep) : kleiss(al, be, mJ, B, mA, em, ep));
    } else {
        *R = -0.375 * g2 * OR_CF * (fa > 0 ? kleiss(al, be, A, mJ, mB, em, ep) : kleiss(al, be, mJ, A, mB, em, ep));
    }
    *S = 8.0 * OR_PI * s->c.alphas_mz * dy_dipoles(fa, fb, A, B, J, em, ep, x, al, be);
}

/* for the pins: R and S of channel (flavour f, kind, orientation o2) at one
 * real configuration, and the Born weights al, be at m2 */
void or_dy_real(const or_state* s, int f, int kind, int o2, double m2, double x, double y, double v, double ph,
                double c, double uphi, double out[4]) {
    double A[4], B[4], J[4], em[4], ep[4], al, be;
    dy_real_kin(s, m2, x, y, v, ph, c, uphi, A, B, J, em, ep);
    dy_hel(s, f, m2, &al, &be);
    int fa, fb;
    if (kind == 0) { fa = o2 == 0 ? f : -f; fb = -fa; }
    else if (kind == 1) { fa = 21; fb = o2 == 0 ? f : -f; }
    else { fa = o2 == 0 ? f : -f; fb = 21; }
    dy_real_rs(s, kind, fa, fb, al, be, A, B, J, em, ep, x, &out[0], &out[1]);
    out[2] = al;
    out[3] = be;
}

/* NLO pp -> Z/photon -> e- e+ event: blocks (id, 0): S/H choice, channel,
 * rapidity, lepton polar cosine; (id, 1): x_a and x_b of the collinear terms
 * (S) or x and v (H), the emission azimuth (H), the lepton azimuth; (id, 2):
 * the pair mass on the Breit-Wigner of the window. */
static void gen_dy_nlo(const or_state* s, int64_t id, uint64_t seed, or_events* o, int64_t e) {
    double u0[4], u1[4], u2[4];
    or_rng_block(seed, STREAM_HARD, id, 0u, 0u, u0);
    or_rng_block(seed, STREAM_HARD, id, 1u, 0u, u1);
    or_rng_block(seed, STREAM_HARD, id, 2u, 0u, u2);
    const double mz2 = s->c.mz * s->c.mz, mg = s->c.mz * s->c.gz;
    const double r1 = atan((s->c.mll_min * s->c.mll_min - mz2) / mg);
    const double r2 = atan((s->c.mll_max * s->c.mll_max - mz2) / mg);
    const double m2 = mz2 + mg * tan(r1 + u2[0] * (r2 - r1)), m = sqrt(m2), q2 = m2;
    const double jm = (r2 - r1) * ((m2 - mz2) * (m2 - mz2) + mg * mg) / mg; /* d m^2 / d u */
    const double c = 2.0 * u0[3] - 1.0;
    const int nf = s->c.nf;
    if (u0[0] < s->c.p_s) {
        double Y = log(s->sqrtS / m), y = -Y + 2.0 * Y * u0[2];
        double e1 = m / s->sqrtS * exp(y), e2 = m / s->sqrtS * exp(-y);
        double xa = e1 + (1.0 - e1) * u1[0], xb = e2 + (1.0 - e2) * u1[1];
        double Ea = 0.5 * e1 * s->sqrtS, Eb = 0.5 * e2 * s->sqrtS;
        double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
        double pZ[4] = {A[0] + B[0], 0.0, 0.0, A[3] + B[3]}, em[4], ep[4];
        decay_zc(pZ, m, c, u1[3], em, ep);
        double csub[10], W = 0.0;
        for (int f = 1; f <= nf; ++f) {
            double al, be;
            dy_hel(s, f, m2, &al, &be);
            for (int o2 = 0; o2 < 2; ++o2) {
                int a = o2 == 0 ? f : -f, b = -a;
                double M0 = born_dy(al, be, a > 0 ? A : B, em, ep);
                double born = xfp(s, a, e1, q2) * xfp(s, b, e2, q2) * M0 / (16.0 * OR_PI * m2 * m2);
                double corr = or_nlo_bvi_factor(s) + k_leg(s, a, e1, xa, q2) + k_leg(s, b, e2, xb, q2);
                csub[2 * (f - 1) + o2] = born * corr;
                W += fabs(born * corr);
            }
        }
        double target = u0[1] * W, cum = 0.0;
        int sel = 2 * nf - 1;
        for (int q = 0; q < 2 * nf; ++q) {
            cum += fabs(csub[q]);
            if (target < cum) { sel = q; break; }
        }
        int f = sel / 2 + 1, a = (sel % 2 == 0) ? f : -f, b = -a;
        put(o, e, 0, A, a, a > 0 ? 1 : 0, a > 0 ? 0 : 1, -1);
        put(o, e, 1, B, b, b > 0 ? 1 : 0, b > 0 ? 0 : 1, -1);
        put(o, e, 2, em, 11, 0, 0, 1);
        put(o, e, 3, ep, -11, 0, 0, 1);
        o->n[e] = 4;
        o->w[e] = (csub[sel] < 0.0 ? -W : W) * 2.0 * Y * jm / s->c.p_s;
        o->t_start[e] = s->S;
        o->flags[e] = 0u;
        return;
    }
    double xmin = m2 / s->S;
    double x = xmin + (1.0 - xmin) * u1[0];
    double YH = 0.5 * log(s->S * x / m2), y = -YH + 2.0 * YH * u0[2];
    double v = (1.0 - x) * u1[1], ph = 2.0 * OR_PI * u1[2];
    double ea = exp(y) * sqrt(m2 / x / s->S), eb = exp(-y) * sqrt(m2 / x / s->S);
    double A[4], B[4], J[4], em[4], ep[4];
    dy_real_kin(s, m2, x, y, v, ph, c, u1[3], A, B, J, em, ep);
    double csub[30], W = 0.0;
    int pa[30], pb[30], kind[30];
    int q = 0;
    for (int f = 1; f <= nf; ++f) {
        double al, be;
        dy_hel(s, f, m2, &al, &be);
        for (int kd = 0; kd < 3; ++kd)
            for (int o2 = 0; o2 < 2; ++o2) {
                int fa, fb;
                if (kd == 0) { fa = o2 == 0 ? f : -f; fb = -fa; }
                else if (kd == 1) { fa = 21; fb = o2 == 0 ? f : -f; }
                else { fa = o2 == 0 ? f : -f; fb = 21; }
                double R, S;
                dy_real_rs(s, kd, fa, fb, al, be, A, B, J, em, ep, x, &R, &S);
                pa[q] = fa; pb[q] = fb; kind[q] = kd; csub[q++] = R - S;
            }
    }
    for (int k = 0; k < q; ++k) {
        csub[k] *= xfp(s, pa[k], ea, q2) * xfp(s, pb[k], eb, q2) / (16.0 * OR_PI * m2) / (16.0 * OR_PI * OR_PI);
        W += fabs(csub[k]);
    }
    double target = u0[1] * W, cum = 0.0;
    int sel = q - 1;
    for (int k = 0; k < q; ++k) {
        cum += fabs(csub[k]);
        if (target < cum) { sel = k; break; }
    }
    int a = pa[sel], b = pb[sel];
    int ca, aa, cb, ab, jp, cj, aj;
    if (kind[sel] == 0) {
        ca = a > 0 ? 1 : 0; aa = a > 0 ? 0 : 2;
        cb = b > 0 ? 1 : 0; ab = b > 0 ? 0 : 2;
        jp = 21; cj = 1; aj = 2;
    } else {
        int qk = kind[sel] == 1 ? b : a;
        int cq, aq;
        if (qk > 0) { cq = 2; aq = 0; cj = 1; aj = 0; }
        else { cq = 0; aq = 1; cj = 0; aj = 2; }
        jp = qk;
        if (kind[sel] == 1) { ca = 1; aa = 2; cb = cq; ab = aq; }
        else { ca = cq; aa = aq; cb = 1; ab = 2; }
    }
    put(o, e, 0, A, a, ca, aa, -1);
    put(o, e, 1, B, b, cb, ab, -1);
    put(o, e, 2, J, jp, cj, aj, 1);
    put(o, e, 3, em, 11, 0, 0, 1);
    put(o, e, 4, ep, -11, 0, 0, 1);
    o->n[e] = 5;
    o->w[e] = (csub[sel] < 0.0 ? -W : W) * 2.0 * YH * (1.0 - xmin) * (1.0 - x) * jm / (1.0 - s->c.p_s);
    o->t_start[e] = s->S;
    o->flags[e] = OR_F_HEVENT;
}

int or_hard_events(const or_state* s, int64_t first_id, int64_t n, uint64_t seed, or_events* out) {
    const int mt = s->c.matching;
    if (mt < 0 || mt > 2) return -1;
    if (mt != 0 && s->c.process != 1 && s->c.process != 2) return -1;
    if (mt == 1 && !(s->c.mu_q2 > 0.0)) return -1;
    for (int64_t e = 0; e < n; ++e) {
        int64_t id = first_id + e;
        out->id[e] = id;
        clear_counters(out, e);
        if (s->c.process == 0) gen_ee(s, id, seed, out, e);
        else if (s->c.process == 1) gen_lo(s, id, seed, out, e);
        else if (s->c.process == 3) gen_dy(s, id, seed, out, e);
        else if (s->c.process == 4) gen_dy_nlo(s, id, seed, out, e);
        else gen_nlo(s, id, seed, out, e);
    }
    return 0;
}
