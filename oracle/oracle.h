/*
 * CPU oracle for the GAPS-2 dipole shower (arXiv:2511.19633).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64
 * implementation of the shower's veto algorithm written from the paper
 * (section 2, appendix A, appendix B, appendix C).  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no source with the GPU library: the two only see the same input tables (the
 * toy PDF grid and the workload constants).
 *
 * Event records are structure-of-arrays, slot-major: field[slot * cap + e].
 *
 * Parity status of each part (see the tests for the pins):
 *   Philox4x32-10 ............ pinned (Random123 known-answer vectors)
 *   alpha_s, PDF interpolation  pinned (RGE property, library interpolator)
 *   FF/FI/IF/II maps, II boost  pinned (CS variables recomputed from momenta,
 *                               masslessness, momentum conservation, Lambda)
 *   veto loop ................. pinned (no-emission closed form; first-emission
 *                               CDF vs 2-D quadrature of the Sudakov integrands
 *                               of every kernel: FF q->qg, g->gg, g->qqbar; FI
 *                               q->qg and the gluon's; IF/II families A-D; the
 *                               heavy-quark measure and factor; in all four
 *                               forms; planted mistakes fail them)
 *   learned bound ............. pinned (first-emission CDF with null trials;
 *                               with the bound too low everywhere and in one
 *                               planted cell: the weighted veto's weighted
 *                               CDF vs quadrature)
 *   NLO pieces ................ pinned (printed B+V+I factor, B = int g,
 *                               Li2 vs library, R-S identities)
 *   observables ............... pinned (thrust/jets on hand-built events)
 *   NLO Z/photon (process 4) .. pinned (Kleiss-trick R and the dipoles at mapped
 *                               leptons, lepton-averaged, = textbook Z ones;
 *                               collinear limits; S/H balance at the pole)
 *   matching variants ......... pinned (S + printed R - S = textbook R; the
 *                               correction factor = textbook R / dipoles; NLO
 *                               totals equal across the variants; corrected and
 *                               plain first-emission CDFs vs 2-D quadrature of
 *                               R / B and of the dipoles in (x, v))
 */
#ifndef GAPS_ORACLE_H
#define GAPS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int process;        /* 0 e+e- -> qq, 1 pp LO Z->ee, 2 pp NLO S/H,
                           3 pp LO Z/photon -> ee with interference,
                           4 pp NLO S/H Z/photon -> ee (the real emission by
                             the Kleiss trick) */
    int nf;             /* active flavours (5) */
    double sqrt_s, t_cut, alphas_mz, mz, gz, sw2, gf, mc, mb;
    double mll_min, mll_max, p_s;
    const float* pdf;   /* [ntab][nq][nx] node values of x*f */
    int nx, nq, ntab;
    double lnx0, lnx1, lnq0, lnq1;
    double over_scale;  /* multiplies every channel overestimate (1 default) */
    int matching;       /* 0: MC@NLO with the power shower (every event starts at
                              the hadronic S: the paper's choice)
                           1: MC@NLO with the start scale mu_q2 (processes 1, 2):
                              every event starts at mu_q2; H events keep the
                              dipole sum where kT^2 >= mu_q2 (there the S events'
                              shower no longer subtracts it) and S events lose its
                              integral over that region (one-point estimate)
                           2: POWHEG-like (processes 1, 2): Born-kinematics events
                              (NLO: weight B + V + I + C plus the integral of R - S
                              over the radiation, one-point estimate) flagged
                              OR_F_MEC, whose first emission the shower corrects to
                              the real matrix element */
    double mu_q2;       /* start scale for matching 1, GeV^2 */
} or_config;

typedef struct {
    int64_t* id; double* w; double* t_start; int32_t* n; uint32_t* flags;
    double *E, *px, *py, *pz;
    int32_t *pid, *col, *acol; int8_t* status;
    uint32_t *n_cycles, *n_trials, *n_accept, *n_viol; /* may be NULL */
    double* t1;                                         /* may be NULL */
    int32_t max_slots; int64_t cap;
} or_events;

/* per-event flags */
#define OR_F_OVERFLOW 1u
#define OR_F_COLOUR   2u
#define OR_F_NAN      4u
#define OR_F_FALLBACK 8u
#define OR_F_VIOL     16u
#define OR_F_HARDFAIL 32u
#define OR_F_HEVENT   64u
#define OR_F_MAXCYC   128u
#define OR_F_MEC      256u /* first emission corrected to the real matrix element */

typedef struct or_state or_state;

or_state* or_init(const or_config* cfg);
void or_free(or_state* s);

/* counter-based generator, Philox4x32-10 */
void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

double or_alphas(const or_state* s, double t);
double or_pdf_xf(const or_state* s, int tab, double x, double q2);
int or_pdf_table(int pid);

/* overestimate table: or_bounds_shape gives (nent, nbin); copy out */
void or_bounds_shape(int* nent, int* nbin);
void or_bounds(const or_state* s, double* out);
double or_lo_wmax(const or_state* s);

/* hard events for ids first_id .. first_id+n-1 into out[0..n-1] */
int or_hard_events(const or_state* s, int64_t first_id, int64_t n, uint64_t seed,
                   or_events* out);

/* shower events in[0..n-1] into out[0..n-1] on nthreads threads (1 = serial) */
int or_shower(const or_state* s, const or_events* in, int64_t n, uint64_t seed,
              or_events* out, int nthreads);

/* shower modes */
#define OR_MODE_PLAIN 0
#define OR_MODE_LEARNED 1
#define OR_MODE_LOG 2

typedef struct {
    int mode;            /* OR_MODE_* */
    /* LOG: one row of 5 floats per initial-state (IF, II) winner trial with a
     * positive weight: ln t, ln eta, z, table entry of the splitting term,
     * ln(alpha_s(t)/alpha_s(t_c) * W / shape(z)), the quantity the entry's
     * constant bounds.  Rows beyond log_cap are counted, not stored. */
    float* log;
    int64_t log_cap;
    int64_t* log_count;  /* in/out: rows so far */
    /* LEARNED: the learned bound R_theta[64][48][8] (initial-state entries
     * 8..71, eta bins, ln t cells) for the initial-state channels of the
     * partons in slots 0 and 1; random-number stream 1.  A trial whose weight
     * exceeds its learned bound goes through the weighted veto (accepted
     * with probability w/(2w - 1), the event weight multiplied by 2w - 1 on
     * acceptance and by -(2w - 1) on rejection), and the event continues on
     * the analytic overestimate (every channel draws again), flagged
     * OR_F_FALLBACK.  Violations of the learned bound are not counted in
     * n_viol. */
    const double* learned;
    /* retain != 0: the retained-trial form of the max-veto competition.  A
     * channel's trial scale is the first point below the current scale of its
     * own Poisson process of intensity c/t; a channel that loses a cycle keeps
     * its trial, which is still that process's first point below the new
     * scale, so only the winner draws again after a veto or a null.  After an
     * emission a channel keeps its trial only when its process is unchanged:
     * the same spectator, and neither its emitter nor its spectator is the
     * emitter, the spectator or the new parton of the emission (whose recoil
     * is local); after an initial-initial emission, which boosts every
     * final-state parton, every channel draws again.  Same distribution as
     * redrawing every channel each cycle; different use of the random
     * numbers: channel entry 2i+side draws at cycle j with word (2i+side) mod
     * 4 of block (id, j, (2i+side)/4), the first draws at cycle 0 and the
     * redraws at the cycle that follows the one they replace. */
    int retain;
    /* gen_select != 0 (plain mode, not with retain): the generate-select form.
     * Each cycle draws one trial from the sum of every channel's overestimate
     * and picks the channel in proportion to its share.  The scale range below
     * T is cut into segments at the scales where a channel starts (its limit
     * t_lim below T) or stops (its cutoff): in the segment just below T the
     * active channels (t_cut < T <= t_lim) sum to C/t, with a heavy-quark
     * channel's c/(t - m^2) bounded by c lo/(lo - m^2) / t over the segment
     * [lo, T]; the trial is ln t = ln T + ln(u0)/C, a null at lo when below it
     * (and a jump to lo without a draw when no channel is active), the channel
     * the first whose running share exceeds u1 C (entry order), a heavy-quark
     * channel's trial kept with probability t (lo - m^2) / (lo (t - m^2)) < u2
     * failing, then the usual veto.  Block (id, cycle, 2^32 - 2) gives u0..u2;
     * the winner block (id, cycle, 2^32 - 1) as in the max-veto forms. */
    int gen_select;
    /* veto_max != 0 (plain mode, neither retain nor gen_select): the veto-max
     * form.  Every channel runs the veto algorithm on its own from T down to
     * its first accepted trial; the largest of these is the emission (no
     * further veto).  After it every channel runs its loop again from the
     * emission's scale.  A cycle is one emission.  Trial k of channel entry c
     * (in channel order) at cycle j: its scale from word 0 of block (id, j,
     * 2^31 | c << 20 | k << 1), term, z, azimuth and acceptance from block
     * (id, j, 2^31 | c << 20 | k << 1 | 1). */
    int veto_max;
} or_opts;

#define OR_LEARN_NTB 8
/* ln t edges of the learned-bound cells (OR_LEARN_NTB + 1 values) */
void or_cell_edges(const or_state* s, double* out);

int or_shower_ex(const or_state* s, const or_events* in, int64_t n, uint64_t seed,
                 or_events* out, int nthreads, const or_opts* opts);

/* kinematic maps, exposed for the identity tests.
 * type: 0 FF, 1 FI, 2 IF, 3 II.  pe, ps: emitter/spectator before (E,px,py,pz).
 * vars: FF (z, y), FI (z, x), IF (x, u), II (x, v); phi azimuth.
 * out: new emitter, emitted, spectator (3 x 4 doubles).
 * For II the boost acts on nrest extra momenta in-place (rest, nrest x 4). */
void or_map(int type, const double pe[4], const double ps[4], double v1, double v2,
            double phi, double out[12], double* rest, int nrest);
/* IF/II: (z, t, s) -> CS variables (x, u or v) */
void or_is_vars(int type, double z, double t, double s, double* x, double* uv);

/* per-event observables: see observables.c for the layout */
int or_n_obs(void);
int or_observables(const or_state* s, const or_events* ev, int64_t n, double* obs);

/* NLO building blocks exposed for the pins */
double or_li2(double x);
double or_nlo_bvi_factor(const or_state* s);
double or_nlo_aqq(const or_state* s);
double or_nlo_bqq(const or_state* s, double eta);
double or_nlo_gqq(const or_state* s, double x);
void or_nlo_rs(const or_state* s, int kind, double sbar, double tbar, double ubar,
               double mborn2, double* r_minus_s);
double or_nlo_sub(int kind, double x, double va);
/* the first-emission correction factor R / (dipole sum) of the shower's
 * initial-initial families A (q -> q g) and B (q <- g) at (x, v), and the bound
 * on family B's factor that the corrected channels' overestimate carries */
double or_mec_ratio(int family_b, double x, double v);
double or_mec_bound(void);
/* process 4: R and the dipole sum S of one real channel (kind 0 q qbar with
 * the quark at A for o2 = 0, kind 1 gluon at A, kind 2 gluon at B; the other
 * beam's (anti)quark by o2) at the pair mass m2, the map's x, y, v, phi, the
 * lepton angles (c, uphi); out = {R, S, a, b} (the Born's angular weights) */
void or_dy_real(const or_state* s, int f, int kind, int o2, double m2, double x, double y, double v, double ph,
                double c, double uphi, double out[4]);

#ifdef __cplusplus
}
#endif
#endif
