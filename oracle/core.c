/* CPU oracle: random numbers, running coupling, PDF grid interpolation and the
 * overestimate table.  Test infrastructure only. */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_int.h"

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
 * multiplications with the published multipliers and Weyl key increments. */
void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One block of four uniforms in (0,1): counter (id, c2, c3), key (seed, stream). */
void or_rng_block(uint64_t seed, uint32_t stream, int64_t id, uint32_t c2, uint32_t c3,
                  double u[4]) {
    uint32_t ctr[4] = {(uint32_t)(uint64_t)id, (uint32_t)((uint64_t)id >> 32), c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ stream};
    uint32_t o[4];
    or_philox4x32(ctr, key, o);
    for (int k = 0; k < 4; ++k) u[k] = ((double)o[k] + 0.5) * 2.3283064365386963e-10;
}

/* One-loop running coupling with nf = 5 (alpha_s reference at mZ). */
double or_alphas(const or_state* s, double t) {
    return s->c.alphas_mz / (1.0 + s->c.alphas_mz * s->b0 * log(t / (s->c.mz * s->c.mz)));
}

/* The same coupling at ln t, with ln(t / mZ^2) = ln t - ln mZ^2. */
double or_alphas_ln(const or_state* s, double lnt) {
    return s->c.alphas_mz / (1.0 + s->c.alphas_mz * s->b0 * (lnt - s->ln_mz2));
}

int or_pdf_table(int pid) {
    switch (pid) {
    case 21: return 0;
    case 1: return 1;
    case 2: return 2;
    case 3: case -3: return 3;
    case 4: case -4: return 4;
    case 5: case -5: return 5;
    case -1: return 6;
    case -2: return 7;
    default: return -1;
    }
}

/* x*f by bilinear interpolation in (ln x, ln Q^2) of the node values.  Zero for
 * x >= 1, below the smallest x node and outside the Q^2 range: no extrapolation
 * (the paper's PDF edge policy, appendix B.6 and section 4.1). */
static double pdf_xf_lq(const or_state* s, int tab, double x, double q2, double lq) {
    if (!(x > 0.0) || x >= 1.0 || !(q2 > 0.0)) return 0.0;
    double lx = log(x);
    if (lx < s->c.lnx0 || lq < s->c.lnq0 || lq > s->c.lnq1) return 0.0;
    double fx = (lx - s->c.lnx0) / s->dlnx;
    int i = (int)fx;
    if (i > s->c.nx - 2) i = s->c.nx - 2;
    double a = fx - (double)i;
    double fq = (lq - s->c.lnq0) / s->dlnq;
    int j = (int)fq;
    if (j > s->c.nq - 2) j = s->c.nq - 2;
    double b = fq - (double)j;
    const float* F = s->pdf + (size_t)tab * s->c.nq * s->c.nx;
    double f00 = F[j * s->c.nx + i], f10 = F[j * s->c.nx + i + 1];
    double f01 = F[(j + 1) * s->c.nx + i], f11 = F[(j + 1) * s->c.nx + i + 1];
    return (1.0 - b) * ((1.0 - a) * f00 + a * f10) + b * ((1.0 - a) * f01 + a * f11);
}

double or_pdf_xf(const or_state* s, int tab, double x, double q2) {
    return q2 > 0.0 ? pdf_xf_lq(s, tab, x, q2, log(q2)) : 0.0;
}

double or_pdf_f(const or_state* s, int tab, double x, double q2) {
    double xf = or_pdf_xf(s, tab, x, q2);
    return xf > 0.0 ? xf / x : 0.0;
}

/* At a trial scale the veto algorithm has ln t itself (the trial is drawn in
 * ln t), so the interpolation's ln Q^2 is that ln t. */
double or_pdf_f_lq(const or_state* s, int tab, double x, double q2, double lq) {
    double xf = pdf_xf_lq(s, tab, x, q2, lq);
    return xf > 0.0 ? xf / x : 0.0;
}

/* Smallest value of the form m * 2^e, m in {1/2, 2^-3/4, 2^-1/2, 2^-1/4, 1}, that
 * is >= v: rounds a bound up onto a quarter-octave ladder (exact, no libm). */
double or_quarter_octave_up(double v) {
    if (!(v > 0.0)) return 0.0;
    int e;
    double m = frexp(v, &e); /* v = m 2^e, m in [0.5, 1) */
    double q;
    if (m <= 0.5) q = 0.5;
    else if (m <= 0.5946035575013605) q = 0.5946035575013605;
    else if (m <= 0.7071067811865476) q = 0.7071067811865476;
    else if (m <= 0.8408964152537145) q = 0.8408964152537145;
    else q = 1.0;
    return ldexp(q, e);
}

/* Collinear-limit bound of Jacobian x kernel divided by the z shape.
 * shape 1: 1/(z(1-z)), G = (1-x) P(x); shape 3: 1/z, G = P(x); P the II kernels
 * (appendix B.5), which the IF kernels reach at u -> 0 where the bound is largest. */
static double gbound(int shape, int fam, double x) {
    double omx = 1.0 - x;
    if (shape == 1) {
        switch (fam) {
        case FAM_A: return OR_CF * (1.0 + x * x);
        case FAM_B: return omx * OR_TR * (1.0 - 2.0 * x * omx);
        case FAM_C: return OR_CA * (1.0 + omx * omx / x - omx + x * omx * omx);
        default: return omx * OR_CF * (x + 2.0 * omx / x);
        }
    }
    if (fam == FAM_B) return OR_TR * (1.0 - 2.0 * x * omx);
    return OR_CF * (x + 2.0 * omx / x);
}

/* The first-emission correction's largest value over the initial-initial
 * phase space at momentum fraction x (family B, at v = 1 - x), and its
 * largest value over [lo, hi] (one maximum, at x = (3 - sqrt 5) / 2). */
static double mec_bmax(double x) {
    double omx = 1.0 - x;
    return 1.0 + (1.0 - x * x) / (x * x + omx * omx);
}
static double mec_bmax_range(double lo, double hi) {
    const double xs = 0.5 * (3.0 - sqrt(5.0));
    if (lo <= xs && xs <= hi) return mec_bmax(xs);
    double a = mec_bmax(lo), b = mec_bmax(hi);
    return a > b ? a : b;
}

/* x*f interpolated along ln x at row j (node column values exact). */
static double xf_row(const or_state* s, int tab, int j, double x) {
    if (!(x > 0.0) || x >= 1.0) return 0.0;
    double lx = log(x);
    if (lx < s->c.lnx0) return 0.0;
    double fx = (lx - s->c.lnx0) / s->dlnx;
    int i = (int)fx;
    if (i > s->c.nx - 2) i = s->c.nx - 2;
    double a = fx - (double)i;
    const float* F = s->pdf + ((size_t)tab * s->c.nq + j) * s->c.nx;
    return (1.0 - a) * (double)F[i] + a * (double)F[i + 1];
}

typedef struct { int kind, fam, T, num, den; double m2; } entry_t;

/* entries OR_NENT + T: family B at the initial-initial end (shape 3) under
 * the first-emission correction (kind 4) */
#define OR_NALL (OR_NENT + 8)
static int entry_info(const or_state* s, int e, entry_t* out) {
    out->m2 = 0.0;
    if (e >= OR_NENT) {
        int T = e - OR_NENT;
        if (T == 0) return 0;
        out->kind = 4; out->fam = FAM_B; out->T = T; out->num = 0; out->den = T;
        if (T == 4) out->m2 = s->c.mc * s->c.mc;
        if (T == 5) out->m2 = s->c.mb * s->c.mb;
        return 1;
    }
    if (e < 8) { out->kind = 0; out->fam = -1; out->T = e; out->num = e; out->den = e; return 1; }
    int kind = e < 40 ? 1 : 3;
    int r = e - (kind == 1 ? 8 : 40);
    int fam = r / 8, T = r % 8;
    out->kind = kind; out->fam = fam; out->T = T;
    if (fam == FAM_C) {
        if (kind != 1 || T != 0) return 0;
        out->num = 0; out->den = 0;
    } else {
        if (T == 0) return 0;
        if (kind == 3 && (fam == FAM_A)) return 0;
        if (fam == FAM_A) { out->num = T; out->den = T; }
        if (fam == FAM_B) { out->num = 0; out->den = T; }
        if (fam == FAM_D) { out->num = T; out->den = 0; }
        if (fam == FAM_A || fam == FAM_B) {
            if (T == 4) out->m2 = s->c.mc * s->c.mc;
            if (T == 5) out->m2 = s->c.mb * s->c.mb;
        }
    }
    return 1;
}

/* The overestimate table R[entry][eta bin]: for every transition, an upper
 * envelope in eta of PDF ratio x (collinear Jacobian x kernel bound), taken over
 * all scales and momentum fractions.  This is the paper's procedure of appendix
 * A.2 (tabulate the ratio against eta and take an upper envelope), made strict:
 * the scale dependence is bounded through the grid rows (the interpolant in
 * ln Q^2 is a mediant of the rows), the x dependence cell by cell through the
 * node values, and the result is multiplied by 1.5 and rounded up onto a
 * quarter-octave ladder. */
void or_compute_bounds(or_state* s) {
    const int nx = s->c.nx, nq = s->c.nq;
    const double dle = -OR_LNETA0 / OR_NB;
    double* xn = (double*)malloc(sizeof(double) * nx);
    double* qn = (double*)malloc(sizeof(double) * nq);
    for (int i = 0; i < nx; ++i) xn[i] = exp(s->c.lnx0 + i * s->dlnx);
    for (int j = 0; j < nq; ++j) qn[j] = exp(s->c.lnq0 + j * s->dlnq);
    /* per-row values v[e][j] for the current eta point */
    double* v = (double*)malloc(sizeof(double) * OR_NALL * nq);
    double* numc = (double*)malloc(sizeof(double) * 8 * nx);
    double* gc = (double*)malloc(sizeof(double) * 9 * nx); /* combos: 4 S1 + 4 S3 + corrected B */
    entry_t info[OR_NALL];
    int valid[OR_NALL];
    for (int e = 0; e < OR_NALL; ++e) valid[e] = entry_info(s, e, &info[e]);
    memset(s->bound, 0, sizeof(s->bound));
    memset(s->bound_mec, 0, sizeof(s->bound_mec));

    for (int bin = 0; bin < OR_NB; ++bin) {
        double best[OR_NALL];
        for (int e = 0; e < OR_NALL; ++e) best[e] = 0.0;
        for (int p = 0; p < 3; ++p) {
            double eta = exp(OR_LNETA0 + (bin + 0.5 * p) * dle);
            if (!(eta < 1.0)) continue;
            double fx = (log(eta) - s->c.lnx0) / s->dlnx;
            int i0 = (int)fx;
            if (i0 > nx - 2) i0 = nx - 2;
            /* G over each cell of the parent momentum fraction X in [eta, 1) */
            for (int i = i0; i <= nx - 2; ++i) {
                double xlo = (i == i0) ? eta : xn[i];
                double xhi = xn[i + 1];
                for (int f = 0; f < 4; ++f) {
                    double a1 = gbound(1, f, eta / xlo), b1 = gbound(1, f, eta / xhi);
                    gc[f * nx + i] = a1 > b1 ? a1 : b1;
                    double a3 = (f == FAM_B || f == FAM_D) ? gbound(3, f, eta / xlo) : 0.0;
                    double b3 = (f == FAM_B || f == FAM_D) ? gbound(3, f, eta / xhi) : 0.0;
                    gc[(4 + f) * nx + i] = a3 > b3 ? a3 : b3;
                }
                gc[8 * nx + i] = gc[(4 + FAM_B) * nx + i] * mec_bmax_range(eta / xhi, eta / xlo);
            }
            for (int j = 0; j < nq; ++j) {
                double den[8];
                for (int T = 0; T < 8; ++T) den[T] = xf_row(s, T, j, eta) / eta;
                for (int T = 0; T < 8; ++T) {
                    const float* F = s->pdf + ((size_t)T * nq + j) * nx;
                    for (int i = i0; i <= nx - 2; ++i) {
                        double xlo = (i == i0) ? eta : xn[i];
                        double flo = (i == i0) ? xf_row(s, T, j, eta) : (double)F[i];
                        double fhi = (double)F[i + 1];
                        numc[T * nx + i] = (flo > fhi ? flo : fhi) / xlo;
                    }
                }
                for (int e = 0; e < OR_NALL; ++e) {
                    v[e * nq + j] = -1.0; /* marks a zero denominator */
                    if (!valid[e]) continue;
                    double d = den[info[e].den];
                    if (!(d > 0.0)) continue;
                    const double* g = NULL;
                    if (info[e].kind == 1) g = gc + info[e].fam * nx;
                    if (info[e].kind == 3) g = gc + (4 + info[e].fam) * nx;
                    if (info[e].kind == 4) g = gc + 8 * nx;
                    const double* nc = numc + info[e].num * nx;
                    double m = 0.0;
                    for (int i = i0; i <= nx - 2; ++i) {
                        double val = g ? g[i] * nc[i] : nc[i];
                        if (val > m) m = val;
                    }
                    v[e * nq + j] = m / d;
                }
            }
            /* scale intervals [row j, row j+1] that reach above the channel cutoff */
            for (int e = 0; e < OR_NALL; ++e) {
                if (!valid[e]) continue;
                double m2 = info[e].m2;
                double tmin = m2 > 0.0 ? m2 + s->c.t_cut : s->tc_is;
                for (int j = 0; j + 1 < nq; ++j) {
                    if (qn[j + 1] < tmin) continue;
                    double a = v[e * nq + j], b = v[e * nq + j + 1];
                    double m = a > b ? a : b;
                    if (m < 0.0) continue;
                    if (m2 > 0.0) m *= (qn[j + 1] - m2) / qn[j + 1];
                    if (m > best[e]) best[e] = m;
                }
            }
        }
        for (int e = 0; e < OR_NENT; ++e)
            s->bound[e][bin] = valid[e] ? or_quarter_octave_up(1.5 * best[e]) : 0.0;
        for (int T = 0; T < 8; ++T)
            s->bound_mec[T][bin] = valid[OR_NENT + T] ? or_quarter_octave_up(1.5 * best[OR_NENT + T]) : 0.0;
    }
    free(xn); free(qn); free(v); free(numc); free(gc);
}

void or_bounds_shape(int* nent, int* nbin) { *nent = OR_NENT; *nbin = OR_NB; }

void or_bounds(const or_state* s, double* out) {
    memcpy(out, s->bound, sizeof(s->bound));
}

double or_lo_wmax(const or_state* s) { return s->lo_wmax; }

or_state* or_init(const or_config* cfg) {
    or_state* s = (or_state*)calloc(1, sizeof(or_state));
    s->c = *cfg;
    if (!(s->c.over_scale > 0.0)) s->c.over_scale = 1.0;
    if (s->c.nf <= 0) s->c.nf = 5;
    s->pdf = cfg->pdf;
    s->dlnx = (cfg->lnx1 - cfg->lnx0) / (cfg->nx - 1);
    s->dlnq = (cfg->lnq1 - cfg->lnq0) / (cfg->nq - 1);
    s->sqrtS = cfg->sqrt_s;
    s->S = cfg->sqrt_s * cfg->sqrt_s;
    s->b0 = (33.0 - 2.0 * 5.0) / (12.0 * OR_PI);
    s->ln_mz2 = log(cfg->mz * cfg->mz);
    s->as_over = or_alphas(s, cfg->t_cut);
    double q2min = exp(cfg->lnq0);
    s->tc_is = cfg->t_cut > q2min ? cfg->t_cut : q2min;
    for (int k = 0; k <= OR_NTB; ++k)
        s->cell_edge[k] = cfg->lnq0 + (double)k * ((cfg->lnq1 - cfg->lnq0) / OR_NTB);
    if (cfg->pdf) {
        or_compute_bounds(s);
        if (cfg->process == 1 || cfg->process == 3) s->lo_wmax = or_lo_scan_wmax(s);
    }
    return s;
}

void or_free(or_state* s) { free(s); }

void or_cell_edges(const or_state* s, double* out) {
    for (int k = 0; k <= OR_NTB; ++k) out[k] = s->cell_edge[k];
}
