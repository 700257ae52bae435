/* CPU oracle: the dipole-shower veto algorithm (paper section 2 and appendices
 * A and B), one event at a time, FP64.  Test infrastructure only. */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_int.h"

enum { T_FF = 0, T_FI = 1, T_IF = 2, T_II = 3 };
enum { SH_SOFT = 0, SH_FLAT = 1, SH_S1 = 2, SH_S3 = 3 };
/* splitting families: final-state emitters, then backward (initial-state) steps */
enum { K_QQG = 0, K_GGG = 1, K_GQQ = 2, K_A = 3, K_B = 4, K_C = 5, K_D = 6 };

typedef struct {
    int n, maxtag;
    int mec; /* the next emission is corrected to the real matrix element */
    double p[OR_MAXM][4];
    int pid[OR_MAXM], col[OR_MAXM], acol[OR_MAXM], st[OR_MAXM];
} ev_t;

/* coefR: the term's constant in front of its z shape, mul times the table's */
typedef struct { int kern, shape, flav, ent; double coefR, c, mul; } term_t;

typedef struct {
    int i, k, side, type, alive, heavy, ebin, mec;
    int shared; /* an incoming gluon: the terms after the first share one shape */
    double s, eta, etak, tlim, lntlim, tcut, lntcut, m2;
    double zlo, zhi, omzlo, omzhi;
    int nterm;
    term_t term[12];
    double c, invc;
} chan_t;

static double dot4(const double* a, const double* b) {
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* colours seen as if every parton were outgoing: an incoming parton's colour
 * and anticolour swap roles */
static int effc(const ev_t* e, int i) { return e->st[i] < 0 ? e->acol[i] : e->col[i]; }
static int effa(const ev_t* e, int i) { return e->st[i] < 0 ? e->col[i] : e->acol[i]; }
static void set_eff(ev_t* e, int i, int c, int a) {
    if (e->st[i] < 0) { e->col[i] = a; e->acol[i] = c; }
    else { e->col[i] = c; e->acol[i] = a; }
}

static int eta_bin(double eta) {
    double dle = -OR_LNETA0 / OR_NB;
    double b = floor((log(eta) - OR_LNETA0) / dle);
    if (b < 0.0) return 0;
    if (b > OR_NB - 1) return OR_NB - 1;
    return (int)b;
}

static double shape_int(int sh, const chan_t* ch) {
    switch (sh) {
    case SH_SOFT: return log(ch->omzlo / ch->omzhi);
    case SH_FLAT: return ch->zhi - ch->zlo;
    case SH_S1: return log(ch->zhi / ch->omzhi) - log(ch->zlo / ch->omzlo);
    default: return log(ch->zhi / ch->zlo);
    }
}

static void shape_sample(int sh, const chan_t* ch, double I, double u, double* z, double* omz) {
    switch (sh) {
    case SH_SOFT: *omz = ch->omzlo * exp(-u * I); *z = 1.0 - *omz; break;
    case SH_FLAT: *z = ch->zlo + u * (ch->zhi - ch->zlo); *omz = 1.0 - *z; break;
    case SH_S1: {
        double L = log(ch->zlo / ch->omzlo) + u * I;
        double e = exp(-L);
        *z = 1.0 / (1.0 + e);
        *omz = e / (1.0 + e);
        break;
    }
    default: *z = ch->zlo * exp(u * I); *omz = 1.0 - *z; break;
    }
}

static double shape_val(int sh, double z, double omz) {
    switch (sh) {
    case SH_SOFT: return 1.0 / omz;
    case SH_FLAT: return 1.0;
    case SH_S1: return 1.0 / (z * omz);
    default: return 1.0 / z;
    }
}

/* The overestimate constant of a channel is the sum over its terms of
 * af R_m I_m (appendix A.1: alpha_s(t_c)/(2 pi), the term's PDF-ratio and
 * kernel bound R_m, the z integral I_m of its shape).  The terms of an
 * incoming gluon after the first (g <- q for every quark flavour) all have the
 * same shape, and their part is taken as one product, af (sum of their R_m) I
 * (R summed in term order).  The running sum that picks the winner's term is
 * written the same way.  R: each term's constant (table value times mul). */
static double terms_total(const or_state* S, const chan_t* ch, const double* R) {
    const double af = S->as_over / (2.0 * OR_PI) * S->c.over_scale;
    if (ch->shared) {
        double sum = 0.0;
        for (int m = 1; m < ch->nterm; ++m) sum += R[m];
        return af * R[0] * shape_int(ch->term[0].shape, ch) + af * sum * shape_int(ch->term[1].shape, ch);
    }
    double c = 0.0;
    for (int m = 0; m < ch->nterm; ++m) c += af * R[m] * shape_int(ch->term[m].shape, ch);
    return c;
}

/* the first term whose running sum of constants exceeds target (-1: none) */
static int terms_pick(const or_state* S, const chan_t* ch, const double* R, double target) {
    const double af = S->as_over / (2.0 * OR_PI) * S->c.over_scale;
    if (ch->shared) {
        const double c0 = af * R[0] * shape_int(ch->term[0].shape, ch);
        if (target < c0) return 0;
        const double I = shape_int(ch->term[1].shape, ch);
        double sum = 0.0;
        for (int m = 1; m < ch->nterm; ++m) {
            sum += R[m];
            if (target < c0 + af * sum * I) return m;
        }
        return -1;
    }
    double cum = 0.0;
    for (int m = 0; m < ch->nterm; ++m) {
        cum += af * R[m] * shape_int(ch->term[m].shape, ch);
        if (target < cum) return m;
    }
    return -1;
}

/* if rounding leaves a draw past every term: the last term of positive
 * (analytic) constant */
static int terms_last(const chan_t* ch) {
    for (int m = ch->nterm - 1; m >= 0; --m)
        if (ch->term[m].c > 0.0) return m;
    return 0;
}

static void add_term(chan_t* ch, int kern, int shape, int flav, double coefR, int ent) {
    term_t* t = &ch->term[ch->nterm++];
    t->kern = kern; t->shape = shape; t->flav = flav; t->coefR = coefR; t->c = 0.0; t->ent = ent;
    t->mul = 1.0;
}

/* First-emission correction of a POWHEG-like event (flag OR_F_MEC): the real
 * matrix element over the shower's own density at the same real
 * configuration, at the initial-initial variables (x, v) of the emission
 * (appendix B.5; the shower's initial-initial density is the dipole of
 * appendix C.2).  q qbar -> Z g is reached from both incoming quarks' q -> q g
 * (family A): R / (D_a + D_b) = 1 - 2 v (1 - x - v) / (1 + x^2), in [1/2, 1].
 * A quark from a gluon (family B, g qbar -> Z qbar) has only its own dipole:
 * R / D = 1 + v (2 x + v) / (x^2 + (1 - x)^2), at most the square of the golden
 * ratio (2.618...).  While the correction applies, family B's overestimate
 * comes from a table of its own (the kernel bound times the correction's
 * largest value at each momentum fraction, scanned like the others); a learned
 * constant carries the factor OR_MEC_KB. */
#define OR_MEC_KB 2.625
double or_mec_ratio(int family_b, double x, double v) {
    double omx = 1.0 - x;
    if (!family_b) return 1.0 - 2.0 * v * (omx - v) / (1.0 + x * x);
    return 1.0 + v * (2.0 * x + v) / (x * x + omx * omx);
}
double or_mec_bound(void) { return OR_MEC_KB; }

/* Channel constants (dipole end i with spectator k on colour side `side`):
 * invariant mass, momentum fractions, kinematic limit, the widest z range (at
 * the cutoff), the overestimate terms and their integrals. */
static void setup_channel(const or_state* S, const ev_t* e, int i, int side, int k, chan_t* ch) {
    memset(ch, 0, sizeof(*ch));
    ch->i = i; ch->k = k; ch->side = side;
    int isE = e->st[i] < 0, isS = e->st[k] < 0;
    ch->type = isE ? (isS ? T_II : T_IF) : (isS ? T_FI : T_FF);
    ch->s = 2.0 * dot4(e->p[i], e->p[k]);
    ch->eta = isE ? 2.0 * e->p[i][0] / S->sqrtS : 0.0;
    ch->etak = isS ? 2.0 * e->p[k][0] / S->sqrtS : 0.0;
    double tc = ch->type == T_FF ? S->c.t_cut : S->tc_is;
    double s = ch->s, eta = ch->eta, etak = ch->etak, d;
    if (!(s > 0.0)) return;
    switch (ch->type) {
    case T_FF: ch->tlim = s / 4.0; d = 4.0 * tc / s; break;
    case T_FI: ch->tlim = s * (1.0 - etak) / (4.0 * etak); d = 4.0 * tc * etak / (s * (1.0 - etak)); break;
    case T_IF: ch->tlim = s * (1.0 - eta) / (4.0 * eta); d = 4.0 * tc * eta / (s * (1.0 - eta)); break;
    default: ch->tlim = s * (1.0 - eta) * (1.0 - eta) / (4.0 * eta);
        d = 4.0 * tc * eta / (s * (1.0 - eta) * (1.0 - eta)); break;
    }
    ch->tcut = tc;
    if (isE) {
        int ap = abs(e->pid[i]);
        if (ap == 4) ch->m2 = S->c.mc * S->c.mc;
        if (ap == 5) ch->m2 = S->c.mb * S->c.mb;
        if (ch->m2 > 0.0) {
            ch->heavy = 1;
            double th = ch->m2 + S->c.t_cut;
            if (th > ch->tcut) ch->tcut = th;
        }
    }
    if (!(d < 1.0) || !(ch->tlim > ch->tcut)) return;
    ch->lntlim = log(ch->tlim);
    ch->lntcut = log(ch->tcut);
    double sq = sqrt(1.0 - d);
    if (ch->type == T_FF || ch->type == T_FI) {
        ch->zlo = 0.5 * d / (1.0 + sq);
        ch->omzhi = ch->zlo;
        ch->zhi = 1.0 - ch->zlo;
        ch->omzlo = 1.0 - ch->zlo;
    } else {
        ch->omzhi = 0.5 * (1.0 - eta) * d / (1.0 + sq);
        ch->zhi = 1.0 - ch->omzhi;
        ch->zlo = (4.0 * eta + (1.0 - eta) * (1.0 - eta) * d) /
                  (2.0 * ((1.0 + eta) + (1.0 - eta) * sq));
        ch->omzlo = 1.0 - ch->zlo;
    }
    /* overestimate terms */
    if (!isE) {
        double R = 1.0;
        int ent = -1;
        if (ch->type == T_FI) {
            ent = OR_ENT_FI(or_pdf_table(e->pid[k]));
            R = S->bound[ent][eta_bin(etak)];
        }
        if (e->pid[i] == 21) {
            add_term(ch, K_GGG, SH_SOFT, 0, OR_CA * R, ent);
            for (int f = 1; f <= S->c.nf; ++f) add_term(ch, K_GQQ, SH_FLAT, f, 0.5 * OR_TR * R, ent);
        } else {
            add_term(ch, K_QQG, SH_SOFT, 0, 2.0 * OR_CF * R, ent);
        }
    } else {
        int bin = eta_bin(eta);
        ch->ebin = bin;
        int sh2 = ch->type == T_II ? SH_S3 : SH_S1;
        if (e->pid[i] == 21) {
            add_term(ch, K_C, SH_S1, 0, S->bound[OR_ENT_S1(FAM_C, 0)][bin], OR_ENT_S1(FAM_C, 0));
            static const int par[10] = {1, 2, 3, 4, 5, -1, -2, -3, -4, -5};
            for (int m = 0; m < 10; ++m) {
                int a = par[m];
                if (abs(a) > S->c.nf) continue;
                int T = or_pdf_table(a);
                int ent = ch->type == T_II ? OR_ENT_S3(FAM_D, T) : OR_ENT_S1(FAM_D, T);
                add_term(ch, K_D, sh2, a, S->bound[ent][bin], ent);
            }
        } else {
            int T = or_pdf_table(e->pid[i]);
            add_term(ch, K_A, SH_S1, 0, S->bound[OR_ENT_S1(FAM_A, T)][bin], OR_ENT_S1(FAM_A, T));
            int ent = ch->type == T_II ? OR_ENT_S3(FAM_B, T) : OR_ENT_S1(FAM_B, T);
            add_term(ch, K_B, sh2, 0, S->bound[ent][bin], ent);
            if (e->mec && ch->type == T_II) {
                /* plain: the corrected family-B table; learned: the learned
                 * constant times the correction's bound */
                term_t* tb = &ch->term[ch->nterm - 1];
                tb->mul = OR_MEC_KB;
                tb->coefR = S->bound_mec[T][bin];
                ch->mec = 1;
            }
        }
    }
    double af = S->as_over / (2.0 * OR_PI) * S->c.over_scale;
    double R[12];
    ch->shared = isE && e->pid[i] == 21;
    for (int m = 0; m < ch->nterm; ++m) {
        term_t* t = &ch->term[m];
        t->c = af * t->coefR * shape_int(t->shape, ch);
        R[m] = t->coefR;
    }
    double c = terms_total(S, ch, R);
    if (!(c > 0.0)) return;
    ch->c = c;
    ch->invc = 1.0 / c;
    ch->alive = 1;
}

/* channel list in (parton slot, side) order; returns -1 on a broken colour flow */
static int build_channels(const or_state* S, const ev_t* e, chan_t* ch, int* nch) {
    int m = 0;
    for (int i = 0; i < e->n; ++i) {
        if (e->col[i] == 0 && e->acol[i] == 0) continue;
        for (int side = 0; side < 2; ++side) {
            int tag = side == 0 ? effc(e, i) : effa(e, i);
            if (!tag) continue;
            int k = -1;
            for (int j = 0; j < e->n; ++j) {
                if (j == i) continue;
                int other = side == 0 ? effa(e, j) : effc(e, j);
                if (other == tag) { k = j; break; }
            }
            if (k < 0) return -1;
            setup_channel(S, e, i, side, k, &ch[m++]);
        }
    }
    *nch = m;
    return 0;
}

/* transverse momentum of size sqrt(tp) at azimuth phi, orthogonal to pa and pb */
static void kperp(const double* pa, const double* pb, double tp, double phi, double* kt) {
    double pab = dot4(pa, pb);
    double na = sqrt(pa[1] * pa[1] + pa[2] * pa[2] + pa[3] * pa[3]);
    double nb = sqrt(pb[1] * pb[1] + pb[2] * pb[2] + pb[3] * pb[3]);
    double d[3];
    for (int m = 0; m < 3; ++m) d[m] = pb[m + 1] / nb - pa[m + 1] / na;
    int ax = 0;
    double best = fabs(d[0]);
    for (int m = 1; m < 3; ++m)
        if (fabs(d[m]) < best) { best = fabs(d[m]); ax = m; }
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    r[ax + 1] = 1.0;
    double ra = dot4(r, pa), rb = dot4(r, pb);
    double n1[4];
    for (int m = 0; m < 4; ++m) n1[m] = r[m] - rb / pab * pa[m] - ra / pab * pb[m];
    double n1n = sqrt(-dot4(n1, n1));
    for (int m = 0; m < 4; ++m) n1[m] /= n1n;
    double A[4] = {pa[0], -pa[1], -pa[2], -pa[3]};
    double B[4] = {pb[0], -pb[1], -pb[2], -pb[3]};
    double C[4] = {n1[0], -n1[1], -n1[2], -n1[3]};
    double n2[4];
    for (int mu = 0; mu < 4; ++mu) {
        int cc[3], q = 0;
        for (int m = 0; m < 4; ++m)
            if (m != mu) cc[q++] = m;
        int c0 = cc[0], c1 = cc[1], c2 = cc[2];
        double det = A[c0] * (B[c1] * C[c2] - B[c2] * C[c1]) -
                     A[c1] * (B[c0] * C[c2] - B[c2] * C[c0]) +
                     A[c2] * (B[c0] * C[c1] - B[c1] * C[c0]);
        n2[mu] = (mu & 1) ? -det : det;
    }
    double n2n = sqrt(-dot4(n2, n2));
    for (int m = 0; m < 4; ++m) n2[m] /= n2n;
    double kt0 = sqrt(tp), cp = cos(phi), sp = sin(phi);
    for (int m = 0; m < 4; ++m) kt[m] = kt0 * (cp * n1[m] + sp * n2[m]);
}

/* II recoil: the Lorentz transformation of appendix B.5 mapping K' onto K,
 * applied to one momentum */
static void ii_lambda(const double* Kp, const double* K, double* p) {
    double KK[4];
    for (int m = 0; m < 4; ++m) KK[m] = K[m] + Kp[m];
    double KK2 = dot4(KK, KK), Kp2 = dot4(Kp, Kp);
    double c1 = 2.0 * dot4(KK, p) / KK2;
    double c2 = 2.0 * dot4(Kp, p) / Kp2;
    for (int m = 0; m < 4; ++m) p[m] = p[m] - c1 * KK[m] + c2 * K[m];
}

/* IF and II: Catani-Seymour variables from the shower's (z, t) (appendix B.4
 * and B.5).  The IF x is written as 2z(1-z)/((1-z+r)(1+sqrt(1-d))), an exact
 * rearrangement of the printed root that does not cancel at small r. */
static void is_vars(int type, double z, double omz, double t, double s, double* x, double* uv) {
    double r = t / s;
    if (type == T_IF) {
        double D = omz + r;
        double dd = 4.0 * r * z * omz / (D * D);
        *x = 2.0 * z * omz / (D * (1.0 + sqrt(1.0 - dd)));
    } else {
        *x = z * omz / (omz + r);
    }
    *uv = *x * r / omz;
}

void or_is_vars(int type, double z, double t, double s, double* x, double* uv) {
    is_vars(type, z, 1.0 - z, t, s, x, uv);
}

/* Momenta after the emission; out = {emitter', emitted, spectator'}. */
static void do_map(int type, const double* pe, const double* ps, double s, double z, double omz,
                   double v1, double v2, double phi, double* pi, double* pj, double* pk) {
    double kt[4], tp;
    if (type == T_FF) { /* v1 = y */
        double y = v1;
        tp = z * omz * y * s;
        kperp(pe, ps, tp, phi, kt);
        for (int m = 0; m < 4; ++m) {
            pi[m] = z * pe[m] + y * omz * ps[m] + kt[m];
            pj[m] = omz * pe[m] + y * z * ps[m] - kt[m];
            pk[m] = (1.0 - y) * ps[m];
        }
    } else if (type == T_FI) { /* v1 = x, v2 = 1 - x */
        double x = v1, omx = v2;
        tp = z * omz * omx / x * s;
        kperp(pe, ps, tp, phi, kt);
        double a = omz * omx / x, b = z * omx / x;
        for (int m = 0; m < 4; ++m) {
            pi[m] = z * pe[m] + a * ps[m] + kt[m];
            pj[m] = omz * pe[m] + b * ps[m] - kt[m];
            pk[m] = ps[m] / x;
        }
    } else if (type == T_IF) { /* v1 = x, v2 = u */
        double x = v1, u = v2, omx = 1.0 - x;
        tp = u * (1.0 - u) * omx / x * s;
        kperp(pe, ps, tp, phi, kt);
        double a = (1.0 - u) * omx / x, b = u * omx / x;
        for (int m = 0; m < 4; ++m) {
            pi[m] = pe[m] / x;
            pj[m] = a * pe[m] + u * ps[m] - kt[m];
            pk[m] = b * pe[m] + (1.0 - u) * ps[m] + kt[m];
        }
    } else { /* II: v1 = x, v2 = v */
        double x = v1, v = v2;
        tp = v * (1.0 - x - v) / x * s;
        kperp(pe, ps, tp, phi, kt);
        double a = (1.0 - x - v) / x;
        for (int m = 0; m < 4; ++m) {
            pi[m] = pe[m] / x;
            pj[m] = a * pe[m] + v * ps[m] - kt[m];
            pk[m] = ps[m];
        }
    }
}

void or_map(int type, const double pe[4], const double ps[4], double v1, double v2, double phi,
            double out[12], double* rest, int nrest) {
    double s = 2.0 * dot4(pe, ps);
    double z = 0.0, omz = 0.0, a1 = v1, a2 = v2;
    if (type == T_FF || type == T_FI) { z = v1; omz = 1.0 - v1; a1 = v2; a2 = 1.0 - v2; }
    if (type == T_FF) a2 = 0.0;
    do_map(type, pe, ps, s, z, omz, a1, a2, phi, out, out + 4, out + 8);
    if (type == T_II) {
        double Kp[4], K[4];
        for (int m = 0; m < 4; ++m) {
            Kp[m] = pe[m] + ps[m];
            K[m] = out[m] + out[8 + m] - out[4 + m];
        }
        for (int q = 0; q < nrest; ++q) ii_lambda(Kp, K, rest + 4 * q);
    }
}

typedef struct {
    int ok;
    double x, omx, y, uv, w;
    double wn; /* the weight before division by the table constant: w * over_scale * coefR */
} veto_t;

/* acceptance weight of the winner trial (term tm, scale t with its ln t lnt as
 * drawn, momentum fraction z); the PDF ratio and the coupling are evaluated at
 * that ln t */
static veto_t weight(const or_state* S, const ev_t* e, const chan_t* ch, const term_t* tm,
                     double t, double lnt, double z, double omz) {
    veto_t r;
    memset(&r, 0, sizeof(r));
    double W = 0.0, s = ch->s;
    if (ch->type == T_FF) {
        double y = t / (z * omz * s);
        if (!(y < 1.0)) return r;
        double den1 = omz + z * y;
        double P;
        if (tm->kern == K_QQG) P = OR_CF * (2.0 / den1 - (1.0 + z));
        else if (tm->kern == K_GGG) P = 0.5 * OR_CA * (2.0 / den1 - 2.0 + z * omz);
        else P = 0.5 * OR_TR * (1.0 - 2.0 * z * omz);
        W = (1.0 - y) * P;
        r.y = y;
    } else if (ch->type == T_FI) {
        double kap = t / (z * omz * s);
        double x = 1.0 / (1.0 + kap), omx = kap * x;
        if (!(x > ch->etak)) return r;
        double den1 = omz + omx;
        double P;
        if (tm->kern == K_QQG) P = OR_CF * (2.0 / den1 - (1.0 + z));
        else if (tm->kern == K_GGG) P = 0.5 * OR_CA * (2.0 / den1 - 2.0 + z * omz);
        else P = 0.5 * OR_TR * (1.0 - 2.0 * z * omz);
        int Tk = or_pdf_table(e->pid[ch->k]);
        double den = or_pdf_f_lq(S, Tk, ch->etak, t, lnt);
        double pr = den > 0.0 ? or_pdf_f_lq(S, Tk, ch->etak / x, t, lnt) / den : 0.0;
        W = P * pr;
        r.x = x; r.omx = omx;
    } else {
        double x, uv;
        is_vars(ch->type, z, omz, t, s, &x, &uv);
        if (!(x > ch->eta)) return r;
        if (ch->type == T_IF && !(uv < 1.0)) return r;
        double omx = 1.0 - x, P, J;
        int Ti = or_pdf_table(e->pid[ch->i]);
        int Tnum, Tden;
        if (ch->type == T_IF) {
            J = 1.0 / (uv + x - 2.0 * uv * x);
            switch (tm->kern) {
            case K_A: P = OR_CF * (2.0 / (omx + uv) - (1.0 + x)); break;
            case K_B: P = OR_TR * (1.0 - 2.0 * x * omx); break;
            case K_C: P = OR_CA * (1.0 / (omx + uv) + omx / x - 1.0 + x * omx); break;
            default: P = OR_CF * (x + 2.0 * omx / x); break;
            }
        } else {
            J = 1.0 / z;
            switch (tm->kern) {
            case K_A: P = OR_CF * (2.0 / omx - (1.0 + x)); break;
            case K_B: P = OR_TR * (1.0 - 2.0 * x * omx); break;
            case K_C: P = OR_CA * (1.0 / omx + omx / x - 1.0 + x * omx); break;
            default: P = OR_CF * (x + 2.0 * omx / x); break;
            }
        }
        switch (tm->kern) {
        case K_A: Tnum = Ti; Tden = Ti; break;
        case K_B: Tnum = 0; Tden = Ti; break;
        case K_C: Tnum = 0; Tden = 0; break;
        default: Tnum = or_pdf_table(tm->flav); Tden = 0; break;
        }
        double den = or_pdf_f_lq(S, Tden, ch->eta, t, lnt);
        double pr = den > 0.0 ? or_pdf_f_lq(S, Tnum, ch->eta / x, t, lnt) / den : 0.0;
        double hf = ch->heavy ? (t - ch->m2) / t : 1.0;
        W = J * P * pr * hf;
        if (ch->mec) W *= or_mec_ratio(tm->kern == K_B, x, uv);
        r.x = x; r.omx = omx; r.uv = uv;
    }
    double over = S->c.over_scale * tm->coefR * shape_val(tm->shape, z, omz);
    double ar = or_alphas_ln(S, lnt) / S->as_over;
    r.w = ar * W / over;
    r.wn = ar * W / shape_val(tm->shape, z, omz);
    r.ok = 1;
    return r;
}

/* apply the accepted emission: momenta, flavours and colour tags; j appended */
static void emit(const or_state* S, ev_t* e, const chan_t* ch, const term_t* tm, double z,
                 double omz, const veto_t* v, double phi) {
    int i = ch->i, k = ch->k, j = e->n;
    double pe[4], ps[4], pi[4], pj[4], pk[4];
    memcpy(pe, e->p[i], sizeof(pe));
    memcpy(ps, e->p[k], sizeof(ps));
    double a1 = 0.0, a2 = 0.0;
    if (ch->type == T_FF) a1 = v->y;
    else if (ch->type == T_FI) { a1 = v->x; a2 = v->omx; }
    else { a1 = v->x; a2 = v->uv; }
    do_map(ch->type, pe, ps, ch->s, z, omz, a1, a2, phi, pi, pj, pk);
    if (ch->type == T_II) {
        double Kp[4], K[4];
        for (int m = 0; m < 4; ++m) { Kp[m] = pe[m] + ps[m]; K[m] = pi[m] + pk[m] - pj[m]; }
        for (int q = 0; q < e->n; ++q)
            if (q != i && q != k && e->st[q] > 0) ii_lambda(Kp, K, e->p[q]);
    }
    memcpy(e->p[i], pi, sizeof(pi));
    memcpy(e->p[k], pk, sizeof(pk));
    memcpy(e->p[j], pj, sizeof(pj));
    e->st[j] = 1;
    int ec = effc(e, i), ea = effa(e, i), jc = 0, ja = 0;
    switch (tm->kern) {
    case K_QQG: case K_GGG: case K_A: case K_C: {
        int N = ++e->maxtag;
        if (ch->side == 0) { set_eff(e, i, N, ea); jc = ec; ja = N; }
        else { set_eff(e, i, ec, N); jc = N; ja = ea; }
        e->pid[j] = 21;
        break;
    }
    case K_GQQ: {
        int f = tm->flav;
        if (ch->side == 0) { e->pid[i] = f; set_eff(e, i, ec, 0); e->pid[j] = -f; jc = 0; ja = ea; }
        else { e->pid[i] = -f; set_eff(e, i, 0, ea); e->pid[j] = f; jc = ec; ja = 0; }
        break;
    }
    case K_B: {
        int N = ++e->maxtag;
        e->pid[j] = -e->pid[i];
        if (ec == 0) { set_eff(e, i, N, ea); jc = 0; ja = N; }
        else { set_eff(e, i, ec, N); jc = N; ja = 0; }
        e->pid[i] = 21;
        break;
    }
    default: { /* K_D */
        int a = tm->flav;
        if (a > 0) { set_eff(e, i, 0, ea); jc = ec; ja = 0; }
        else { set_eff(e, i, ec, 0); jc = 0; ja = ea; }
        e->pid[i] = a;
        e->pid[j] = a;
        break;
    }
    }
    e->col[j] = jc;
    e->acol[j] = ja;
    e->n += 1;
    e->mec = 0;
}

static int finite4(const double* p) {
    return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]) && isfinite(p[3]);
}

/* ---- learned bound (LEARNED mode) ----
 * An initial-state channel's overestimate constant depends on the cell of its
 * current scale: c_k = sum over terms of alpha_s(t_c)/(2 pi) * R_theta[entry][eta
 * bin][k] * (z integral of the term's shape).  Cell k spans (edge[k], edge[k+1]]. */
static double lrn(const double* L, int ent, int ebin, int k) {
    return L[((ent - OR_IS0) * OR_NB + ebin) * OR_NTB + k];
}

/* the cell of a scale: the largest k with edge[k] < ln t (0 if none) */
static int cell_of(const or_state* S, double lnt) {
    int k = OR_NTB - 1;
    while (k > 0 && !(S->cell_edge[k] < lnt)) --k;
    return k;
}

/* the terms' learned constants in cell k */
static void learned_R(const chan_t* ch, const double* L, int k, double* R) {
    for (int m = 0; m < ch->nterm; ++m) R[m] = lrn(L, ch->term[m].ent, ch->ebin, k) * ch->term[m].mul;
}

static double learned_c(const or_state* S, const chan_t* ch, const double* L, int k) {
    double R[12];
    learned_R(ch, L, k, R);
    return terms_total(S, ch, R);
}

/* trial log shared by the threads of one or_shower_ex call */
typedef struct {
    const or_opts* o;
    pthread_mutex_t mu;
} logsink_t;

/* one row per initial-state winner trial with a positive weight (LOG mode) */
static void log_trial(logsink_t* L, double t, double eta, double z, int ent, double wn) {
    pthread_mutex_lock(&L->mu);
    int64_t k = *L->o->log_count;
    *L->o->log_count = k + 1;
    if (k < L->o->log_cap) {
        float* r = L->o->log + 5 * k;
        r[0] = (float)log(t);
        r[1] = (float)log(eta);
        r[2] = (float)z;
        r[3] = (float)ent;
        r[4] = (float)log(wn);
    }
    pthread_mutex_unlock(&L->mu);
}

/* One trial of channel C from the evolution scale (T, lnT), with the random
 * number of its entry 2i+side at cycle cyc.  Returns the key ln t of the trial,
 * or -INFINITY when the channel has no trial above its cutoff (then nothing is
 * counted).  In learned mode an initial-state channel of the incoming partons
 * draws against the constant of the cell of its starting scale, and a trial
 * below that cell is a null at the cell's lower edge (*isnull, *cell). */
static double draw_trial(const or_state* S, const chan_t* C, double T, double lnT, uint64_t seed,
                         uint32_t stream, int64_t id, uint32_t cyc, int learned, const double* Lt,
                         uint32_t* ntri, int* isnull, int* cell) {
    *isnull = 0;
    *cell = 0;
    if (!C->alive) return -INFINITY;
    double Tch = T < C->tlim ? T : C->tlim;
    double lnTch = lnT < C->lntlim ? lnT : C->lntlim;
    if (!(Tch > C->tcut)) return -INFINITY;
    uint32_t slot = 2u * (uint32_t)C->i + (uint32_t)C->side;
    double ub[4];
    or_rng_block(seed, stream, id, cyc, slot >> 2, ub);
    double lu = log(ub[slot & 3u]);
    *ntri += 1;
    double invc = C->invc, floor = -INFINITY;
    int lch = learned && (C->type == T_IF || C->type == T_II) && C->i < 2, k = 0;
    if (lch) {
        k = cell_of(S, lnTch);
        invc = 1.0 / learned_c(S, C, Lt, k);
        floor = S->cell_edge[k];
    }
    double key;
    if (!C->heavy) key = lnTch + lu * invc;
    else key = log(C->m2 + (Tch - C->m2) * exp(lu * invc));
    if (lch && key < floor && floor > C->lntcut) { key = floor; *isnull = 1; }
    *cell = k;
    if (key < C->lntcut) return -INFINITY;
    return key;
}

/* ---- one event ----
 * The working state of one event while it is showered: its record and channel
 * list, the evolution scale, the random-number coordinates and the counters
 * that go to the output.  lrn: the initial-state channels of the incoming
 * partons still draw against the learned cell constants (LEARNED mode until
 * the first violation of the learned bound); wfac: the weight factor that the
 * weighted veto of such a violation leaves on the event. */
typedef struct {
    const or_state* S;
    ev_t* ev;
    chan_t* ch;
    int nch, M;
    int64_t id;
    uint64_t seed;
    uint32_t stream;
    int lrn;
    const double* Lt;
    logsink_t* L;
    double T, lnT, t1, wfac;
    uint32_t cycle, ntri, nacc, nviol, flags;
} sh_t;

/* the learned cells apply to the initial-state channels of the incoming
 * partons (emitter slot 0 or 1) */
static int learned_chan(const sh_t* r, const chan_t* C) {
    return r->lrn && (C->type == T_IF || C->type == T_II) && C->i < 2;
}

/* read event e of the input into the working record; returns 0 when the event
 * can be showered (it fits and its colour lines pair up) */
static int sh_load(sh_t* r, const or_events* in, int64_t e) {
    ev_t* ev = r->ev;
    const int64_t ci = in->cap;
    ev->n = in->n[e];
    ev->maxtag = 0;
    r->flags = in->flags ? in->flags[e] : 0u;
    ev->mec = (r->flags & OR_F_MEC) != 0u;
    for (int q = 0; q < ev->n && q < OR_MAXM; ++q) {
        int64_t o = (int64_t)q * ci + e;
        ev->p[q][0] = in->E[o]; ev->p[q][1] = in->px[o];
        ev->p[q][2] = in->py[o]; ev->p[q][3] = in->pz[o];
        ev->pid[q] = in->pid[o]; ev->col[q] = in->col[o]; ev->acol[q] = in->acol[o];
        ev->st[q] = in->status[o];
        if (ev->col[q] > ev->maxtag) ev->maxtag = ev->col[q];
        if (ev->acol[q] > ev->maxtag) ev->maxtag = ev->acol[q];
    }
    r->id = in->id[e];
    r->T = in->t_start[e];
    r->lnT = log(r->T);
    r->t1 = 0.0;
    r->wfac = 1.0;
    r->cycle = r->ntri = r->nacc = r->nviol = 0u;
    r->nch = 0;
    if (ev->n > r->M) { r->flags |= OR_F_OVERFLOW; return -1; }
    if (build_channels(r->S, ev, r->ch, &r->nch) < 0) { r->flags |= OR_F_COLOUR; return -1; }
    return 0;
}

static void sh_store(const sh_t* r, const or_events* in, int64_t e_in, or_events* out, int64_t e_out) {
    const ev_t* ev = r->ev;
    const int64_t co = out->cap;
    out->id[e_out] = r->id;
    out->w[e_out] = in->w[e_in] * r->wfac;
    out->t_start[e_out] = in->t_start[e_in];
    out->n[e_out] = ev->n;
    if (out->flags) out->flags[e_out] = r->flags;
    for (int q = 0; q < ev->n && q < out->max_slots; ++q) {
        int64_t o = (int64_t)q * co + e_out;
        out->E[o] = ev->p[q][0]; out->px[o] = ev->p[q][1];
        out->py[o] = ev->p[q][2]; out->pz[o] = ev->p[q][3];
        out->pid[o] = ev->pid[q]; out->col[o] = ev->col[q]; out->acol[o] = ev->acol[q];
        out->status[o] = (int8_t)ev->st[q];
    }
    if (out->n_cycles) out->n_cycles[e_out] = r->cycle;
    if (out->n_trials) out->n_trials[e_out] = r->ntri;
    if (out->n_accept) out->n_accept[e_out] = r->nacc;
    if (out->n_viol) out->n_viol[e_out] = r->nviol;
    if (out->t1) out->t1[e_out] = r->t1;
}

/* the trial of channel C from the current scale at the current cycle */
static double sh_draw(sh_t* r, const chan_t* C, int* isnull, int* cell) {
    return draw_trial(r->S, C, r->T, r->lnT, r->seed, r->stream, r->id, r->cycle, r->lrn, r->Lt, &r->ntri,
                      isnull, cell);
}

/* what the winner of a cycle proposes */
typedef struct {
    int acc;     /* the emission is accepted */
    term_t tm;   /* splitting term */
    double z, omz, phi;
    veto_t v;
} step_t;

/* The winner trial of channel C at scale t (section 2): its splitting term in
 * proportion to the terms' overestimates (a learned channel: the cell
 * constants of cell wcell), z from the term's shape and the azimuth, from the
 * winner block of the cycle; then the weight and the veto.
 *
 * A weight above the learned bound (LEARNED mode) is handled by the weighted
 * veto algorithm (Lonnblad, Eur. Phys. J. C 73 (2013) 2350): with a proposal
 * density g below the true density f at the trial, accepting with any
 * probability eps and multiplying the event weight by f/(g eps) on acceptance
 * and by (1 - f/g)/(1 - eps) on rejection keeps the emission density exactly
 * f.  eps = w/(2w - 1) (w = f/g > 1) minimises the second moment of the
 * factor, which is then +(2w - 1) or -(2w - 1).  From this trial on the event
 * draws against the analytic overestimate (its channels draw again from the
 * new scale), so it sees no further learned-bound violation.  A weight above
 * the analytic bound is counted (n_viol, OR_F_VIOL) and accepted with
 * probability one. */
static step_t winner(sh_t* r, const chan_t* C, double t, double lnt, int lch, int wcell) {
    const or_state* S = r->S;
    const double* Lt = r->Lt;
    step_t st;
    double u[4];
    or_rng_block(r->seed, r->stream, r->id, r->cycle, 0xFFFFFFFFu, u);
    double R[12];
    if (lch) learned_R(C, Lt, wcell, R);
    else
        for (int m = 0; m < C->nterm; ++m) R[m] = C->term[m].coefR;
    const double ctot = lch ? terms_total(S, C, R) : C->c;
    int sel = terms_pick(S, C, R, u[0] * ctot);
    if (sel < 0) sel = terms_last(C);
    st.tm = C->term[sel];
    st.tm.coefR = R[sel];
    double I = shape_int(st.tm.shape, C);
    shape_sample(st.tm.shape, C, I, u[1], &st.z, &st.omz);
    st.phi = 2.0 * OR_PI * u[2];
    st.v = weight(S, r->ev, C, &st.tm, t, lnt, st.z, st.omz);
    const veto_t* v = &st.v;
    if (r->L && (C->type == T_IF || C->type == T_II) && !C->mec && v->ok && v->wn > 0.0)
        log_trial(r->L, t, C->eta, st.z, st.tm.ent, v->wn);
    if (lch && v->ok && v->w > 1.0) {
        const double g = 2.0 * v->w - 1.0;
        st.acc = u[3] < v->w / g;
        r->wfac *= st.acc ? g : -g;
        r->lrn = 0;
        r->flags |= OR_F_FALLBACK;
        return st;
    }
    if (v->ok && v->w > 1.0) { r->nviol += 1; r->flags |= OR_F_VIOL; }
    st.acc = v->ok && u[3] < v->w;
    return st;
}

/* Apply the accepted emission of channel C at scale t and rebuild the channel
 * list.  Returns 0 to go on, 1 when the event stops after this cycle (a
 * non-finite momentum or a broken colour line: the cycle counts), 2 when it
 * stops before (the record is full: the cycle does not count). */
static int emit_step(sh_t* r, const chan_t* C, const step_t* st, double t) {
    ev_t* ev = r->ev;
    if (ev->n + 1 > r->M) { r->flags |= OR_F_OVERFLOW; return 2; }
    emit(r->S, ev, C, &st->tm, st->z, st->omz, &st->v, st->phi);
    r->nacc += 1;
    if (r->t1 == 0.0) r->t1 = t;
    int bad = 0;
    for (int q = 0; q < ev->n; ++q) bad |= !finite4(ev->p[q]);
    if (bad) { r->flags |= OR_F_NAN; return 1; }
    if (build_channels(r->S, ev, r->ch, &r->nch) < 0) { r->flags |= OR_F_COLOUR; return 1; }
    return 0;
}

/* Max-veto, the paper's form (section 2): each cycle every channel draws a
 * trial scale from the current scale and the largest trial is the winner
 * (ties to the lowest channel); it is vetoed or accepted, and the evolution
 * continues from its scale.  In LEARNED mode an initial-state channel of an
 * incoming parton draws against the constant of the cell of its scale, and a
 * trial below that cell is a null at the cell's lower edge: when a null wins,
 * no channel emits above the edge and the evolution continues from it. */
static void run_max_veto(sh_t* r) {
    for (;;) {
        if (r->cycle >= OR_MAXCYC) { r->flags |= OR_F_MAXCYC; break; }
        double best = -INFINITY;
        int win = -1, wnull = 0, wcell = 0;
        for (int c = 0; c < r->nch; ++c) {
            int isnull, cell;
            const double key = sh_draw(r, &r->ch[c], &isnull, &cell);
            if (key > best) { best = key; win = c; wnull = isnull; wcell = cell; }
        }
        if (win < 0) break;
        if (wnull) {
            r->T = exp(best);
            r->lnT = best;
            r->cycle += 1;
            continue;
        }
        const double t = exp(best);
        const chan_t* C = &r->ch[win];
        const step_t st = winner(r, C, t, best, learned_chan(r, C), wcell);
        if (st.acc) {
            const int rc = emit_step(r, C, &st, t);
            if (rc == 2) break;
            if (rc == 1) { r->cycle += 1; break; }
        }
        r->T = t;
        r->lnT = best;
        r->cycle += 1;
    }
}

/* Retained trials (the same Markov chain as max-veto with fewer draws): a
 * channel's trial scales are the points of its own Poisson process of
 * intensity c/t below the current scale, so a channel that loses a cycle
 * keeps its trial, and only the winner draws again after a veto or a null.
 * After an emission a channel keeps its trial when its process is unchanged:
 * the same spectator, and neither its emitter nor its spectator is the
 * emitter, the spectator or the new parton of the emission (whose recoil is
 * local).  An initial-initial emission boosts every final-state parton, and a
 * violated learned bound changes the initial-state constants: then every
 * channel draws again. */
static void run_retained(sh_t* r) {
    static _Thread_local double key[OR_MAXCH], okey[2 * OR_MAXM];
    static _Thread_local int knull[OR_MAXCH], kcell[OR_MAXCH];
    static _Thread_local int okspec[2 * OR_MAXM], onull[2 * OR_MAXM], ocell[2 * OR_MAXM];
    for (int c = 0; c < r->nch; ++c) key[c] = sh_draw(r, &r->ch[c], &knull[c], &kcell[c]);
    for (;;) {
        if (r->cycle >= OR_MAXCYC) { r->flags |= OR_F_MAXCYC; break; }
        double best = -INFINITY;
        int win = -1;
        for (int c = 0; c < r->nch; ++c)
            if (key[c] > best) { best = key[c]; win = c; }
        if (win < 0) break;
        if (knull[win]) {
            r->T = exp(best);
            r->lnT = best;
            r->cycle += 1;
            key[win] = sh_draw(r, &r->ch[win], &knull[win], &kcell[win]);
            continue;
        }
        const double t = exp(best);
        const chan_t* C = &r->ch[win];
        const int lch = learned_chan(r, C);
        const int e_i = C->i, e_k = C->k;
        const step_t st = winner(r, C, t, best, lch, kcell[win]);
        const int fell = lch && !r->lrn;
        const int e_all = C->type == T_II || fell;
        if (st.acc) {
            /* the pending trial and spectator of every entry 2i+side */
            for (int q = 0; q < 2 * r->ev->n; ++q) okspec[q] = -1;
            for (int c = 0; c < r->nch; ++c) {
                int q = 2 * r->ch[c].i + r->ch[c].side;
                okspec[q] = r->ch[c].k;
                okey[q] = key[c];
                onull[q] = knull[c];
                ocell[q] = kcell[c];
            }
            const int rc = emit_step(r, C, &st, t);
            if (rc == 2) break;
            if (rc == 1) { r->cycle += 1; break; }
        }
        r->T = t;
        r->lnT = best;
        r->cycle += 1;
        if (!st.acc && !fell) {
            key[win] = sh_draw(r, &r->ch[win], &knull[win], &kcell[win]);
            continue;
        }
        const int j = r->ev->n - 1;
        for (int c = 0; c < r->nch; ++c) {
            const chan_t* D = &r->ch[c];
            const int q = 2 * D->i + D->side;
            const int kept = st.acc && !e_all && q < 2 * j && okspec[q] == D->k && D->i != e_i && D->i != e_k &&
                             D->i != j && D->k != e_i && D->k != e_k && D->k != j;
            if (kept) {
                key[c] = okey[q];
                knull[c] = onull[q];
                kcell[c] = ocell[q];
            } else {
                key[c] = sh_draw(r, D, &knull[c], &kcell[c]);
            }
        }
    }
}

/* generate-select: is channel D active just below T, and its share of the sum
 * over the segment whose lower end is lo */
static int gs_active(const chan_t* D, double T) {
    return D->alive && D->tlim > D->tcut && D->tlim >= T && D->tcut < T;
}
static double gs_share(const chan_t* D, double lo) {
    return D->heavy ? D->c * lo / (lo - D->m2) : D->c;
}

/* Generate-select (the alternative section 2 names): each cycle one trial
 * from the sum of the channels' overestimates, the channel picked in
 * proportion to its share.  Channel limits and cutoffs cut the scale range
 * into segments; in the segment [lo, T] the active channels sum to C/t (a
 * heavy-quark channel's c/(t - m^2) bounded by c lo/(lo - m^2)/t and thinned
 * back); a trial below lo is a null at lo, and with no channel active the
 * evolution moves to lo without a draw.  Block (id, cycle, 2^32 - 2) gives
 * the trial, the channel and the thinning; the winner block as in max-veto. */
static void run_gen_select(sh_t* r) {
    for (;;) {
        if (r->cycle >= OR_MAXCYC) { r->flags |= OR_F_MAXCYC; break; }
        /* the segment below T ends at the largest scale below T where a
         * channel starts (its limit) or stops (its cutoff) */
        double lo = -1.0, lnlo = 0.0;
        int any = 0;
        for (int c = 0; c < r->nch; ++c) {
            const chan_t* D = &r->ch[c];
            if (!D->alive || !(D->tlim > D->tcut)) continue;
            if (D->tlim < r->T) {
                if (D->tlim > lo) { lo = D->tlim; lnlo = D->lntlim; }
            } else if (D->tcut < r->T) {
                any = 1;
                if (D->tcut > lo) { lo = D->tcut; lnlo = D->lntcut; }
            }
        }
        if (lo < 0.0) break; /* no channel can emit below T */
        if (!any) {          /* none active: move to where one starts */
            r->T = lo;
            r->lnT = lnlo;
            r->cycle += 1;
            continue;
        }
        double Csum = 0.0;
        for (int c = 0; c < r->nch; ++c)
            if (gs_active(&r->ch[c], r->T)) Csum += gs_share(&r->ch[c], lo);
        double g[4];
        or_rng_block(r->seed, r->stream, r->id, r->cycle, 0xFFFFFFFEu, g);
        r->ntri += 1;
        const double lnt = r->lnT + log(g[0]) / Csum;
        if (lnt < lnlo) { /* below the segment: a null at its lower end */
            r->T = lo;
            r->lnT = lnlo;
            r->cycle += 1;
            continue;
        }
        /* the channel whose running share first exceeds u1 C */
        const double target = g[1] * Csum;
        double cum = 0.0;
        int sel = -1, last = -1;
        for (int c = 0; c < r->nch && sel < 0; ++c) {
            if (!gs_active(&r->ch[c], r->T)) continue;
            cum += gs_share(&r->ch[c], lo);
            last = c;
            if (target < cum) sel = c;
        }
        if (sel < 0) sel = last;
        if (r->ch[sel].heavy) { /* thin the bound back to c/(t - m^2) */
            const double t = exp(lnt), m2 = r->ch[sel].m2;
            const double keep = (t * (lo - m2)) / (lo * (t - m2));
            if (!(g[2] < keep)) {
                r->T = t;
                r->lnT = lnt;
                r->cycle += 1;
                continue;
            }
        }
        const double t = exp(lnt);
        const chan_t* C = &r->ch[sel];
        const step_t st = winner(r, C, t, lnt, 0, 0);
        if (st.acc) {
            const int rc = emit_step(r, C, &st, t);
            if (rc == 2) break;
            if (rc == 1) { r->cycle += 1; break; }
        }
        r->T = t;
        r->lnT = lnt;
        r->cycle += 1;
    }
}

/* veto-max: trial k of channel entry c at emission cycle j draws its scale
 * from word 0 of block (id, j, VM_BLOCK(c, k, 0)) and its term, z, azimuth and
 * acceptance from block (id, j, VM_BLOCK(c, k, 1)) */
#define VM_BLOCK(c, k, b) (0x80000000u | ((uint32_t)(c) << 20) | ((uint32_t)(k) << 1) | (uint32_t)(b))
#define VM_MAXTRIALS (1 << 19)

/* the splitting term, z, azimuth and weight of a trial of channel C at scale t
 * from the four numbers u (plain mode); returns whether it is accepted */
static int vm_veto(const or_state* S, const ev_t* ev, const chan_t* C, double t, double lnt, const double* u,
                   term_t* tsel, double* z, double* omz, double* phi, veto_t* v) {
    double R[12] = {0.0};
    for (int m = 0; m < C->nterm; ++m) R[m] = C->term[m].coefR;
    int sel = terms_pick(S, C, R, u[0] * C->c);
    if (sel < 0) sel = terms_last(C);
    *tsel = C->term[sel];
    shape_sample(tsel->shape, C, shape_int(tsel->shape, C), u[1], z, omz);
    *phi = 2.0 * OR_PI * u[2];
    *v = weight(S, ev, C, tsel, t, lnt, *z, *omz);
    return v->ok && u[3] < v->w;
}

/* veto-max: the first accepted trial of channel entry c below T, by the
 * channel's own veto loop at emission cycle j; its ln t (-INFINITY: none above
 * the cutoff) and trial index *kk.  *capped is set when the loop runs out of
 * trial indices. */
static double vm_first(const or_state* S, const ev_t* ev, const chan_t* C, int c, double T, double lnT,
                       uint64_t seed, uint32_t stream, int64_t id, uint32_t j, uint32_t* ntri, uint32_t* nviol,
                       int* kk, int* capped) {
    *kk = -1;
    if (!C->alive) return -INFINITY;
    double Tch = T < C->tlim ? T : C->tlim;
    double lnTch = lnT < C->lntlim ? lnT : C->lntlim;
    for (int k = 0; k < VM_MAXTRIALS; ++k) {
        if (!(Tch > C->tcut)) return -INFINITY;
        double ub[4], u[4];
        or_rng_block(seed, stream, id, j, VM_BLOCK(c, k, 0), ub);
        *ntri += 1;
        const double lu = log(ub[0]);
        double key;
        if (!C->heavy) key = lnTch + lu * C->invc;
        else key = log(C->m2 + (Tch - C->m2) * exp(lu * C->invc));
        if (key < C->lntcut) return -INFINITY;
        const double t = exp(key);
        or_rng_block(seed, stream, id, j, VM_BLOCK(c, k, 1), u);
        term_t tm;
        double z, omz, phi;
        veto_t v;
        const int acc = vm_veto(S, ev, C, t, key, u, &tm, &z, &omz, &phi, &v);
        if (v.ok && v.w > 1.0) *nviol += 1;
        if (acc) { *kk = k; return key; }
        Tch = t;
        lnTch = key;
    }
    *capped = 1;
    return -INFINITY;
}

/* Veto-max (the other form section 2 names): every channel runs the veto
 * algorithm on its own from the current scale down to its first accepted
 * trial, and the largest of these is the emission, applied without a further
 * veto; after it every channel runs its loop again from the emission's scale.
 * A cycle is one emission. */
static void run_veto_max(sh_t* r) {
    for (;;) {
        if (r->cycle >= OR_MAXCYC) { r->flags |= OR_F_MAXCYC; break; }
        double best = -INFINITY;
        int win = -1, wk = -1, capped = 0;
        uint32_t nv = 0;
        for (int c = 0; c < r->nch; ++c) {
            int k;
            const double key1 = vm_first(r->S, r->ev, &r->ch[c], c, r->T, r->lnT, r->seed, r->stream, r->id,
                                         r->cycle, &r->ntri, &nv, &k, &capped);
            if (key1 > best) { best = key1; win = c; wk = k; }
        }
        if (nv) { r->nviol += nv; r->flags |= OR_F_VIOL; }
        if (capped) { r->flags |= OR_F_MAXCYC; break; }
        if (win < 0) break;
        /* the winner's accepted trial again, from the same numbers */
        const chan_t* C = &r->ch[win];
        const double t = exp(best);
        double u[4];
        or_rng_block(r->seed, r->stream, r->id, r->cycle, VM_BLOCK(win, wk, 1), u);
        step_t st;
        vm_veto(r->S, r->ev, C, t, best, u, &st.tm, &st.z, &st.omz, &st.phi, &st.v);
        st.acc = 1;
        const int rc = emit_step(r, C, &st, t);
        if (rc == 2) break;
        r->cycle += 1;
        if (rc == 1) break;
        r->T = t;
        r->lnT = best;
    }
}

enum { FORM_MAX_VETO = 0, FORM_RETAINED = 1, FORM_GEN_SELECT = 2, FORM_VETO_MAX = 3 };

typedef struct {
    const or_state* S;
    const or_events* in;
    or_events* out;
    uint64_t seed;
    int64_t lo, hi;
    logsink_t* L;
    int mode;
    const double* Lt;
    int form;
} job_t;

static void* run_job(void* arg) {
    job_t* J = (job_t*)arg;
    sh_t r;
    memset(&r, 0, sizeof(r));
    r.S = J->S;
    r.ev = (ev_t*)malloc(sizeof(ev_t));
    r.ch = (chan_t*)malloc(sizeof(chan_t) * OR_MAXCH);
    r.M = J->out->max_slots < OR_MAXM ? J->out->max_slots : OR_MAXM;
    r.seed = J->seed;
    r.stream = J->mode == OR_MODE_LEARNED ? 1u : 0u;
    r.Lt = J->Lt;
    r.L = J->L;
    for (int64_t e = J->lo; e < J->hi; ++e) {
        r.lrn = J->mode == OR_MODE_LEARNED;
        if (sh_load(&r, J->in, e) == 0) {
            switch (J->form) {
            case FORM_RETAINED: run_retained(&r); break;
            case FORM_GEN_SELECT: run_gen_select(&r); break;
            case FORM_VETO_MAX: run_veto_max(&r); break;
            default: run_max_veto(&r); break;
            }
        }
        sh_store(&r, J->in, e, J->out, e);
    }
    free(r.ev);
    free(r.ch);
    return NULL;
}

int or_shower_ex(const or_state* S, const or_events* in, int64_t n, uint64_t seed, or_events* out,
                 int nthreads, const or_opts* opts) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    int mode = opts ? opts->mode : OR_MODE_PLAIN;
    if (mode != OR_MODE_PLAIN && mode != OR_MODE_LOG && mode != OR_MODE_LEARNED) return -1;
    if (mode == OR_MODE_LEARNED && !opts->learned) return -1;
    if (opts && opts->gen_select && (mode != OR_MODE_PLAIN || opts->retain)) return -1;
    if (opts && opts->veto_max && (mode != OR_MODE_PLAIN || opts->retain || opts->gen_select)) return -1;
    logsink_t sink, *L = NULL;
    if (mode == OR_MODE_LOG) {
        if (!opts->log_count || (opts->log_cap > 0 && !opts->log)) return -1;
        sink.o = opts;
        pthread_mutex_init(&sink.mu, NULL);
        L = &sink;
    }
    job_t jobs[256];
    pthread_t th[256];
    for (int k = 0; k < nthreads; ++k) {
        jobs[k].S = S; jobs[k].in = in; jobs[k].out = out; jobs[k].seed = seed;
        jobs[k].lo = n * k / nthreads;
        jobs[k].hi = n * (k + 1) / nthreads;
        jobs[k].L = L;
        jobs[k].mode = mode;
        jobs[k].Lt = mode == OR_MODE_LEARNED ? opts->learned : NULL;
        jobs[k].form = !opts ? FORM_MAX_VETO
                       : opts->retain ? FORM_RETAINED
                       : opts->gen_select ? FORM_GEN_SELECT
                       : opts->veto_max ? FORM_VETO_MAX : FORM_MAX_VETO;
    }
    if (nthreads == 1) run_job(&jobs[0]);
    else {
        for (int k = 0; k < nthreads; ++k) pthread_create(&th[k], NULL, run_job, &jobs[k]);
        for (int k = 0; k < nthreads; ++k) pthread_join(th[k], NULL);
    }
    if (L) pthread_mutex_destroy(&sink.mu);
    return 0;
}

int or_shower(const or_state* S, const or_events* in, int64_t n, uint64_t seed, or_events* out,
              int nthreads) {
    return or_shower_ex(S, in, n, seed, out, nthreads, NULL);
}
