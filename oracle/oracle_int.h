/* Internal declarations of the CPU oracle (test infrastructure only). */
#ifndef GAPS_ORACLE_INT_H
#define GAPS_ORACLE_INT_H

#include "oracle.h"

#define OR_PI 3.14159265358979323846
#define OR_CF (4.0 / 3.0)
#define OR_CA 3.0
#define OR_TR 0.5
#define OR_NC 3.0

/* eta bins of the overestimate table: 48 bins uniform in ln(eta) on [1e-6, 1) */
#define OR_NB 48
#define OR_LNETA0 (-13.815510557964274) /* ln(1e-6) */
/* entries: FI[T] (8), S1[family][T] (4 x 8), S3[family][T] (4 x 8) */
#define OR_NENT 72
#define OR_ENT_FI(T) (T)
#define OR_ENT_S1(f, T) (8 + 8 * (f) + (T))
#define OR_ENT_S3(f, T) (40 + 8 * (f) + (T))
enum { FAM_A = 0, FAM_B = 1, FAM_C = 2, FAM_D = 3 };

/* learned bound: initial-state entries 8..71, eta bins, OR_NTB cells uniform in
 * ln t over the PDF grid's ln Q^2 range */
#define OR_NTB 8
#define OR_NIS 64
#define OR_IS0 8

#define OR_MAXM 256
#define OR_MAXCH (2 * OR_MAXM)
#define OR_MAXCYC 2000000

struct or_state {
    or_config c;
    const float* pdf;
    double dlnx, dlnq;         /* node spacings */
    double sqrtS, S;           /* hadronic (or e+e-) energy, squared */
    double as_over;            /* alpha_s(t_c): the alpha_s overestimate */
    double tc_is;              /* cutoff of channels that need a PDF ratio */
    double b0;
    double ln_mz2;             /* log(m_Z^2): the coupling at a trial's ln t */
    double bound[OR_NENT][OR_NB];
    /* family B at the initial-initial end while the first-emission correction
     * applies (kernel bound times the correction's largest value), by the
     * quark's PDF table */
    double bound_mec[8][OR_NB];
    double cell_edge[OR_NTB + 1]; /* ln t edges of the learned-bound cells */
    double lo_wmax;
};

double or_pdf_f(const or_state* s, int tab, double x, double q2); /* f, not x*f */
/* the same at ln Q^2 = lq given by the caller (a trial's ln t) */
double or_pdf_f_lq(const or_state* s, int tab, double x, double q2, double lq);
/* the one-loop coupling at ln t (one logarithm fewer than or_alphas(exp(lnt))) */
double or_alphas_ln(const or_state* s, double lnt);
void or_compute_bounds(or_state* s);
double or_quarter_octave_up(double v);
void or_rng_block(uint64_t seed, uint32_t stream, int64_t id, uint32_t c2, uint32_t c3,
                  double u[4]);
double or_lo_scan_wmax(const or_state* s);

#endif
