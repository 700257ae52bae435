/*
 * libgaps: MI355X (gfx950) implementation of the GAPS-2 dipole parton shower
 * (Seymour and Sule, "An NLO-Matched Initial and Final State Parton Shower on a
 * GPU", arXiv:2511.19633).
 *
 * The library showers hard-process events one event per lane: the max-veto
 * algorithm of section 2 (trial scales against overestimates, winner,
 * accept/veto, emission), initial-state backward evolution guided by PDF
 * ratios (appendix A), the FF/FI/IF/II kernels, kinematic maps and the II
 * recoil transformation (appendix B), on LO or MC@NLO-style S/H inputs
 * (appendix C).  Kinematics and weights are FP64.
 *
 * Conventions for every entry point:
 *  - Device pointers point to memory on the current HIP device; host pointers
 *    are marked as such.  The caller owns all buffers it passes; the library
 *    owns only what gaps_init uploads plus its scratch space.
 *  - Event records are structure-of-arrays, slot-major: a per-particle field
 *    of event e, slot q lives at [q * cap + e]; per-event fields at [e].
 *  - Calls taking a stream are asynchronous on that stream.  Argument and state
 *    errors are reported synchronously by the return value; device-side
 *    per-event problems are reported in the event's flags word.
 *  - Results are a pure function of the inputs, the seed and the
 *    configuration: the event id (not the array position) keys the random
 *    numbers, so block size, grid size and batching never change an event.
 */
#ifndef GAPS_H
#define GAPS_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gaps_ctx_s* gaps_ctx;

typedef enum {
    GAPS_OK = 0,
    GAPS_EINVAL = -1,    /* bad argument (null pointer, size, layout) */
    GAPS_ENOMEM = -2,    /* device allocation failed */
    GAPS_EHIP = -3,      /* a HIP call failed */
    GAPS_ECAPACITY = -4, /* a size exceeds what the context was built for */
    GAPS_ESTATE = -5     /* call not valid in the current state */
} gaps_status;

/* per-event flag bits */
#define GAPS_F_OVERFLOW 1u  /* an accepted emission would exceed max_slots */
#define GAPS_F_COLOUR 2u    /* a colour line has no partner */
#define GAPS_F_NAN 4u       /* a non-finite momentum appeared */
#define GAPS_F_FALLBACK 8u  /* learned mode: a weight exceeded the learned bound;
                               the weighted veto's factor is in the event's
                               weight and the event continued on the analytic
                               overestimate */
#define GAPS_F_VIOL 16u     /* a veto weight exceeded one (counted in n_viol) */
#define GAPS_F_HARDFAIL 32u /* the hard-event sampler found no event */
#define GAPS_F_HEVENT 64u   /* NLO H (real-emission) event */
#define GAPS_F_MAXCYC 128u  /* cycle guard reached */
#define GAPS_F_MEC 256u     /* POWHEG-like event: the shower corrects its first
                               emission to the real matrix element */

/* Physics configuration, read from host memory by gaps_init (section 4 and
 * appendix C constants; the PDF grid stands in for the paper's LHAPDF set). */
typedef struct {
    int process;        /* 0: e+e- -> q qbar (final state only)
                           1: pp -> Z -> e+e- LO,  2: pp -> Z NLO S/H events
                           3: pp -> Z/photon -> e+e- LO with the interference
                              (m_ee in the window below; cos theta of the
                              electron about the quark from (1 + cos^2) F1 +
                              2 cos F2 by accept-reject)
                           4: pp -> Z/photon -> e+e- at NLO, MC@NLO S and H
                              events (weighted, p_s; m_ee from the Z
                              Breit-Wigner on the window, the electron uniform
                              in the pair's rest frame; the real emission by the
                              Kleiss trick, the subtraction by the dipoles at
                              mapped lepton momenta; mu_F = m_ee) */
    int nf;             /* active quark flavours (5) */
    double sqrt_s;      /* collider energy, GeV */
    double t_cut;       /* shower cutoff on t = pT^2, GeV^2 */
    double alphas_mz;   /* alpha_s(mZ^2), one-loop running */
    double mz, gz;      /* Z mass and width, GeV */
    double sw2, gf;     /* sin^2(theta_W), Fermi constant */
    double mc, mb;      /* charm and bottom masses (heavy-quark measure) */
    double mll_min, mll_max; /* LO dilepton mass window, GeV */
    double p_s;         /* NLO (processes 2, 4): probability of an S event */
    const float* pdf_xf; /* HOST [ntab][nq][nx] node values of x*f(x, Q^2) */
    int nx, nq, ntab;   /* grid sizes; ntab must be 8 (g d u s c b dbar ubar) */
    double lnx0, lnx1, lnq0, lnq1; /* node ranges in ln x and ln Q^2 */
    double over_scale;  /* multiplies every overestimate (1 = default) */
    int matching;       /* how NLO events meet the shower (appendix C.4 and the
                           alternatives it names; processes 1 and 2 only):
                           0: MC@NLO with the power shower, every event starting
                              at the hadronic S (the paper's choice)
                           1: MC@NLO with the start scale mu_q2: every event
                              starts at mu_q2; H events keep the dipole sum where
                              the emission's kT^2 >= mu_q2 and S events lose its
                              integral over that region (one-point estimate, x
                              of the collinear term and v uniform on [0, 1 - x]
                              from block (id, 1) word 2 and (id, 2) word 0)
                           2: POWHEG-like: every event is a Born event (weight
                              B + V + I + C plus the one-point integral of
                              R - S, the q qbar part in the share of each leg's
                              dipole) flagged GAPS_F_MEC; for LO (process 1) the
                              LO events are flagged.  gaps_shower multiplies a
                              flagged event's first emission by R over its
                              initial-initial dipole density (meanwhile family
                              B's overestimate comes from a table of its own,
                              the kernel bound times the factor's largest value,
                              scanned like the others; a learned constant
                              carries 2.625, the factor's overall maximum).
                           GAPS_EINVAL for other values and processes. */
    double mu_q2;       /* start scale of matching 1, GeV^2 (> 0) */
} gaps_config;

/* Event record: DEVICE pointers.  The optional counters may be NULL. */
typedef struct {
    int64_t* id;         /* event id: keys the random numbers */
    double* w;           /* event weight (signed for NLO) */
    double* t_start;     /* starting scale of the evolution, GeV^2 */
    int32_t* n;          /* particles in the record */
    uint32_t* flags;     /* GAPS_F_* */
    double *E, *px, *py, *pz;   /* [max_slots][cap] momenta, GeV */
    int32_t *pid, *col, *acol;  /* [max_slots][cap] PDG id, colour tags */
    int8_t* status;             /* [max_slots][cap] -1 incoming, +1 outgoing */
    uint32_t *n_cycles, *n_trials, *n_accept, *n_viol; /* per-event counters */
    double* t1;          /* scale of the first accepted emission (0 if none) */
    int32_t max_slots;   /* slots per event (<= 256) */
    int64_t cap;         /* events the arrays hold */
} gaps_events;

#define GAPS_MODE_PLAIN 0
#define GAPS_MODE_LEARNED 1
#define GAPS_MODE_LOG 2

/* statistics accumulated by gaps_shower when params.stats != NULL
 * (device array of GAPS_NSTATS unsigned 64-bit counters, caller-zeroed) */
#define GAPS_ST_CYCLES 0      /* winner cycles, summed over events */
#define GAPS_ST_TRIALS 1      /* channel trials */
#define GAPS_ST_ACCEPT 2      /* accepted emissions */
#define GAPS_ST_VIOL 3        /* weights above one */
#define GAPS_ST_LANE_ITERS 4  /* wave iterations x 64 (lane slots offered) */
#define GAPS_ST_LANE_ACTIVE 5 /* lanes doing work in those iterations */
#define GAPS_ST_FALLBACK 6    /* learned-mode events whose bound failed (weighted
                                 veto, then the analytic overestimate) */
#define GAPS_ST_NULL 7        /* learned-mode cell boundary (null) winners */
#define GAPS_NSTATS 8

typedef struct {
    int mode;            /* GAPS_MODE_* */
    int block;           /* threads per block, multiple of 64, at most 512 for
                            the 2-wave kernel and 256 otherwise (0: largest) */
    int grid;            /* blocks of the persistent launch (0: fill the GPU) */
    int compact_every;   /* cycles between wave refills (0: 8) */
    float* trial_log;    /* LOG mode: device [log_cap][5] floats, one row per
                            initial-state winner trial with a positive weight:
                            ln t, ln eta, z, table entry, ln(alpha_s(t)/
                            alpha_s(t_c) W / shape(z)); rows beyond log_cap are
                            counted, not stored; trials of a GAPS_F_MEC event's
                            corrected first emission are not logged */
    int64_t log_cap;
    unsigned long long* log_count; /* LOG mode: device counter */
    unsigned long long* stats;     /* optional device [GAPS_NSTATS] */
    int variant;         /* 0: wave-cooperative kernel (default)
                            1: one event per lane, no cooperation (reference) */
    int waves_per_simd;  /* wave kernel register budget: 2, 3 or 4 resident
                            waves per SIMD (0: 2); blocks of at most 512
                            threads at 2, 384 at 3 with retained trials, 256
                            otherwise */
    int tail_every;      /* wave kernel: once the queue is empty, repack live
                            events into the block's first waves every this
                            many cycles (0: off) */
    int retain;          /* 0: every channel draws a new trial scale each
                            cycle (the max-veto competition of section 2);
                            1: retained trials, the same Markov chain with
                            fewer draws: a channel that loses keeps its trial
                            (still the first point of its own process below
                            the new scale), so only the winner draws again
                            after a veto or a null; after an emission only
                            the channels whose process changed (emitter or
                            spectator among the emission's emitter, spectator
                            and new parton, a new spectator, or every channel
                            after an initial-initial emission, whose recoil
                            boosts the final state).  Channel entry 2i+side draws at cycle j
                            with word (2i+side) mod 4 of block (id, j,
                            (2i+side)/4); initial draws at cycle 0, redraws at
                            the cycle after the one they replace.  Wave kernel
                            at 2 or 3 waves per SIMD (GAPS_EINVAL otherwise). */
    int gen_select;      /* 1: the generate-select form (section 2 names it as
                            the alternative to max-veto): each cycle one trial
                            from the sum of every channel's overestimate, the
                            channel picked in proportion to its share.  The
                            scale range is cut into segments where a channel
                            starts (its limit) or stops (its cutoff); in the
                            segment [lo, T] the active channels sum to C/t (a
                            heavy-quark channel's c/(t - m^2) bounded by
                            c lo/(lo - m^2)/t and thinned back), ln t = ln T +
                            ln(u0)/C, a null at lo below it (a jump to lo,
                            without a draw, when no channel is active), the
                            first channel in entry order whose running share
                            exceeds u1 C, a heavy-quark trial kept when u2 <
                            t (lo - m^2)/(lo (t - m^2)), then the usual veto.
                            u0..u2 from block (id, cycle, 2^32 - 2).  The same
                            distribution as max-veto, another use of the
                            random numbers.  Plain mode, variant 1, retain 0
                            (GAPS_EINVAL otherwise); not streamed. */
    int veto_max;        /* 1: the veto-max form (section 2 names it beside
                            max-veto): every channel runs the veto algorithm on
                            its own from the current scale down to its first
                            accepted trial, and the largest of these is the
                            emission, applied without a further veto; after it
                            every channel runs its loop again.  A cycle is one
                            emission.  Trial k of channel c (channel order) at
                            cycle j: its scale from word 0 of block (id, j,
                            2^31 | c << 20 | k << 1), term, z, azimuth and
                            acceptance from block (id, j, 2^31 | c << 20 |
                            k << 1 | 1); more than 2^19 trials in one loop
                            stop the event (GAPS_F_MAXCYC).  Plain mode,
                            variant 1, retain 0, gen_select 0 (GAPS_EINVAL
                            otherwise); not streamed. */
} gaps_params;

/* Create a context: validates the configuration, uploads the PDF grid and
 * computes the overestimate table on the device (appendix A.2 procedure).
 * Synchronous.  Returns GAPS_EINVAL for a bad configuration. */
gaps_status gaps_init(const gaps_config* cfg, gaps_ctx* out);

/* Release every device allocation of the context. */
gaps_status gaps_destroy(gaps_ctx ctx);

const char* gaps_strerror(gaps_status s);

/* Hard events (appendix C; e+e- and LO by the workload definitions) for ids
 * first_id .. first_id+n-1 into out[0..n-1].  out->cap >= n, max_slots >= 5.
 * The matching of gaps_config decides the NLO events' weights, their t_start
 * and the GAPS_F_MEC flag. */
gaps_status gaps_hard_events(gaps_ctx ctx, int64_t first_id, int64_t n, uint64_t seed,
                             gaps_events* out, hipStream_t stream);

/* Shower in[0..n-1] into out[0..n-1] (section 2, appendices A and B).
 * in and out must not alias; out->max_slots bounds the final multiplicity
 * (GAPS_F_OVERFLOW otherwise).  params may be NULL (plain mode, defaults).
 * Modes: PLAIN; LOG (plain, plus the trial log); LEARNED (needs
 * gaps_mlp_tabulate first, else GAPS_ESTATE).  LOG and LEARNED run on the wave
 * kernel (variant 0) only.  An event flagged GAPS_F_MEC has its first emission
 * corrected to the real matrix element (see gaps_config.matching), in every
 * mode, form and kernel; the flag is kept in the output. */
gaps_status gaps_shower(gaps_ctx ctx, const gaps_events* in, int64_t n, const gaps_params* params,
                        uint64_t seed, gaps_events* out, hipStream_t stream);

/* gaps_shower for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, checks and results (every event bitwise what gaps_shower
 * gives), with the per-lane working storage (event records, channel caches,
 * weight factors, the work-queue counter) in a static device array of
 * GAPS_NOALLOC_SCRATCH_BYTES per GPU instead of the context's grown
 * allocation.  The array exists on every GPU the library is loaded on until
 * the process ends; gaps_init resolves its address on the context's device.
 * The call allocates nothing: the launch's grid is cut to the blocks of lanes
 * whose storage fits the array (fewer lanes in flight than gaps_shower uses,
 * so it is slower), and the queue counter is cleared by a fill kernel (no
 * memset node under capture).  Calls on one GPU share the array and keep the
 * last call's contents: calls that overlap on one GPU (on different streams,
 * or from different contexts on the same device) race and must not be
 * issued; calls in one stream are ordered.  Errors as gaps_shower, plus
 * GAPS_ECAPACITY when one block's storage (block x per-lane bytes for
 * out->max_slots) exceeds the array and GAPS_ESTATE when the address was not
 * resolved on this device. */
#define GAPS_NOALLOC_SCRATCH_BYTES (256ull << 20)
gaps_status gaps_shower_noalloc(gaps_ctx ctx, const gaps_events* in, int64_t n, const gaps_params* params,
                                uint64_t seed, gaps_events* out, hipStream_t stream);

/* One batch of a stream: input and output records (their pointers are DEVICE
 * pointers, as in gaps_shower) and the number of events n (in->cap, out->cap >= n). */
typedef struct {
    gaps_events in;
    gaps_events out;
    int64_t n;
} gaps_batch;

#define GAPS_MAX_BATCHES 4096

/* Shower a stream of batches in ONE persistent launch (the batching of the
 * section 3 implementation): lanes take events from the batches in order and
 * refill across batch boundaries, so the drain at the end of one batch
 * overlaps the next.  batches is a HOST array of nbatch descriptors
 * (1 <= nbatch <= GAPS_MAX_BATCHES), validated like gaps_shower's arguments
 * and copied by the call (the host array may be reused at once).  The output
 * slot limit is the smallest out.max_slots of the batches; with equal limits
 * every event equals what gaps_shower gives for its batch.  Only the wave
 * kernel (params->variant 0) streams.  Calls on one context share its
 * scratch: issue them on one stream. */
gaps_status gaps_shower_stream(gaps_ctx ctx, const gaps_batch* batches, int nbatch,
                               const gaps_params* params, uint64_t seed, hipStream_t stream);

/* A HIP graph of one gaps_shower_stream call (batch table upload, queue reset
 * and the persistent launch), captured on `stream` (not the null stream).  The
 * graph owns its own scratch, so graphs and direct calls may be mixed; the
 * records the batches point to must stay valid while it is used.  Replay with
 * gaps_graph_launch (asynchronous; replays of one graph must not overlap);
 * gaps_graph_destroy frees it. */
typedef struct gaps_graph_s* gaps_graph;
gaps_status gaps_graph_capture(gaps_ctx ctx, const gaps_batch* batches, int nbatch,
                               const gaps_params* params, uint64_t seed, hipStream_t stream,
                               gaps_graph* out);
gaps_status gaps_graph_launch(gaps_graph g, hipStream_t stream);
gaps_status gaps_graph_destroy(gaps_graph g);

/* ---- Launch autotuner ----
 * The paper tunes its kernels' block size by measurement (section 3.2) and
 * finds where its event partitioning pays (section 3.1).  gaps_tune times the
 * persistent streamed launch (gaps_shower_stream) over a caller's calibration
 * batches for each candidate launch shape: threads per block, cycles between
 * wave refills, resident waves per SIMD, and the fraction of the filling grid
 * (the lanes in flight, whose working storage competes for the caches).  Each
 * point is launched once untimed and then `repeats` times between HIP events
 * on `stream`; its median time goes to ms and its resolved grid (blocks) to
 * grid, so that gaps_params {block, grid, compact_every, waves_per_simd}
 * reproduces it.  A point the kernels cannot run (a block or register budget
 * outside gaps_params' limits) gets ms = -1.  The other fields of base (mode,
 * retain, ...) apply to every point.  Synchronous (it reads the timings).
 * The outputs of the batches are overwritten.  Errors: GAPS_EINVAL for a
 * bad batch table, base, npoints < 1 or repeats < 1. */
typedef struct {
    int block;           /* threads per block (multiple of 64) */
    int compact_every;   /* cycles between wave refills (> 0) */
    int waves_per_simd;  /* 2 or 3 (retained trials), 2..4 otherwise */
    float fill;          /* fraction (0, 1] of the grid that fills the GPU */
    int grid;            /* out: blocks of the launch */
    float ms;            /* out: median launch time, ms (-1: not runnable) */
} gaps_tune_point;

gaps_status gaps_tune(gaps_ctx ctx, const gaps_batch* batches, int nbatch, const gaps_params* base, uint64_t seed,
                      gaps_tune_point* points, int npoints, int repeats, hipStream_t stream);

/* ---- Learned initial-state veto bound (LEARNED mode) ----
 * The paper bounds the PDF ratio x kernel of initial-state emissions with
 * maxima fitted against eta (appendix A.2).  LEARNED mode replaces that
 * constant, for the channels of the incoming partons (slots 0 and 1), by a
 * learned bound per (table entry, eta bin, ln t cell): 8 cells uniform in ln t
 * over the PDF grid's ln Q^2 range.  A channel draws against its cell's
 * constant; a trial below the cell is a null at the cell edge (the evolution
 * continues from there, exact by the factorisation of the no-emission
 * probability); every real trial checks its weight w against the bound.  A
 * trial with w > 1 is handled by the weighted veto algorithm (Lonnblad, Eur.
 * Phys. J. C 73 (2013) 2350): accepted with probability w/(2w - 1), the event
 * weight multiplied by 2w - 1 on acceptance and by -(2w - 1) on rejection, so
 * the emission density stays exactly the true one; the event then continues on
 * the analytic overestimate (every channel set up and drawn again), flagged
 * GAPS_F_FALLBACK.  Such violations are not counted in n_viol (which counts
 * weights above the analytic bound).  Random-number stream 1.
 *
 * The bound comes from a network 4 -> 64 -> 64 -> 1 (ReLU) on features
 * ((ln t - 10)/10, (ln eta + 7)/7, 2z - 1, (entry - 40)/32) predicting an upper
 * quantile of ln(W / R) for logged trials (LOG mode rows), trained with the
 * pinball loss: bfloat16 weights and first hidden layer, FP32 accumulation on
 * the matrix cores, FP32 master weights and Adam.  Calibration gives each cell
 * the largest residual of the held-out rows in it plus 2^-6 when it holds at
 * least GAPS_MLP_MIN_CAL_CELL of them, else that of its (entry, eta bin) when
 * those hold GAPS_MLP_MIN_CAL_BIN, else that of its entry when the entry holds
 * GAPS_MLP_MIN_CAL (entries with fewer keep the analytic bound); tabulation
 * evaluates the network on 48 probe points per cell (3 ln t x 2 ln eta x 8
 * z), takes v = clip(delta + max, -20, 0) and stores min(R, R e^v rounded up
 * to a 7-bit mantissa).  Parameter layout (4545 floats): W1[64][4] b1[64] W2[64][64]
 * b2[64] W3[64] b3. */
#define GAPS_MLP_PARAMS 4545
#define GAPS_LEARN_CELLS (64 * 48 * 8)
#define GAPS_MLP_MIN_CAL_CELL 200
#define GAPS_MLP_MIN_CAL_BIN 200
#define GAPS_MLP_MIN_CAL 2000

/* Cell-maximum bound (the non-learned comparator of the learned bound): the
 * same cells and the same check and fallback in LEARNED mode, with each cell's
 * constant set from presampled trials instead of a network, as adaptive
 * overestimation does (the paper names it as future work, section 5).  rows:
 * device [n_fit + n_cal][5] LOG-mode rows (ln t, ln eta, z, entry, ln W); the
 * first n_fit give each cell (entry, eta bin, ln t cell as the shower takes it)
 * its largest target y = ln W - ln R (rounded to float) and row count; the
 * next n_cal (held out) give each entry delta = max(0, largest y - ymax(cell))
 * + 2^-6 over rows of cells with at least GAPS_CELLMAX_MIN_CELL fitting rows.
 * A cell with at least GAPS_CELLMAX_MIN_CELL fitting rows in an entry with at
 * least GAPS_CELLMAX_MIN_CAL such held-out rows gets min(R, R e^v rounded up to
 * a 7-bit mantissa), v = clip(ymax + delta, -20, 0); every other cell keeps the
 * analytic R.  The table replaces the context's learned table (read it back
 * with gaps_learned_table).  Asynchronous on stream; rows must stay valid until
 * the stream reaches the call.  Errors: GAPS_EINVAL for a NULL context or rows,
 * n_fit <= 0 or n_cal < 0; GAPS_ENOMEM if its 1 MB of cell counters cannot
 * be allocated (first call only, shared with the adaptive variant). */
#define GAPS_CELLMAX_MIN_CELL 16
#define GAPS_CELLMAX_MIN_CAL 2000
gaps_status gaps_cellmax_table(gaps_ctx ctx, const float* rows, int64_t n_fit, int64_t n_cal, hipStream_t stream);

/* The cell-maximum bound with adaptive cell sizes, in the spirit of the
 * adaptive (ExSample) overestimates section 5 leaves for later work: as
 * gaps_cellmax_table, except that every cell takes the largest y and the row
 * count of the finest block around it holding at least GAPS_CELLMAX_MIN_CELL
 * fitting rows, the blocks being dyadic in (eta bin, ln t cell): level l groups
 * the cells whose indices agree after shifting right by (l, min(l, 3)), l = 0
 * (the cell alone) .. 6 (the whole entry).  So a thinly sampled cell is bounded
 * by the trials of its neighbourhood instead of the analytic bound, and a well
 * sampled one by its own.  The held-out margin of a level-0 cell is its
 * entry's (from level-0 rows, as above); the cells of each coarser level share
 * one margin from the held-out rows of all such cells of every entry (at least
 * GAPS_CELLMAX_MIN_CAL, else they keep R).  Cells of entries with fewer rows
 * in all keep R.  Same arguments, scratch, asynchrony and errors. */
gaps_status gaps_cellmax_table_adaptive(gaps_ctx ctx, const float* rows, int64_t n_fit, int64_t n_cal,
                                        hipStream_t stream);

/* Network weights of the context: Philox He-uniform initialisation (key
 * (seed, stream 4)) and zeroed Adam moments.  Synchronous. */
gaps_status gaps_mlp_init(gaps_ctx ctx, uint64_t seed);
/* Copy the FP32 master weights from / to HOST memory (GAPS_MLP_PARAMS floats);
 * set also resets the Adam moments.  Synchronous. */
gaps_status gaps_mlp_set(gaps_ctx ctx, const float* host_theta);
gaps_status gaps_mlp_get(gaps_ctx ctx, float* host_theta);
/* Features of n logged trials: rows device [n][5] -> x device [n][4], y [n],
 * ent [n] (the table entry; may be NULL) and cell [n] (the row's cell
 * (entry - 8) * 384 + eta bin * 8 + ln t cell, the ln t cell being the largest
 * k in 1..7 whose lower edge lies below ln t, else 0; may be NULL). */
gaps_status gaps_mlp_features(gaps_ctx ctx, const float* rows, int64_t n, float* x, float* y, int32_t* ent,
                              int32_t* cell, hipStream_t stream);
/* f[i] = network(x[i]), device arrays. */
gaps_status gaps_mlp_forward(gaps_ctx ctx, const float* x, int64_t n, float* f, hipStream_t stream);
/* Pinball-loss (quantile tau) gradient of the mean over n rows, ADDED to
 * device grad[GAPS_MLP_PARAMS] and *loss (device; may be NULL). */
gaps_status gaps_mlp_grad(gaps_ctx ctx, const float* x, const float* y, int64_t n, float tau, float* grad,
                          float* loss, hipStream_t stream);

/* One Adam step (Kingma and Ba, ICLR 2015, Algorithm 1) of the context's
 * master weights with the device gradient grad[GAPS_MLP_PARAMS] (as
 * gaps_mlp_grad accumulates it; caller-owned): moments m <- beta1 m +
 * (1 - beta1) g and v <- beta2 v + (1 - beta2) g^2, theta <- theta - lr
 * (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps) with t the context's
 * step count plus one, the bfloat16 copy refreshed, grad cleared to zero (so
 * the next gaps_mlp_grad starts from it).  FP32 throughout.  The step count is
 * shared with gaps_mlp_train and reset by gaps_mlp_init/gaps_mlp_set.
 * Asynchronous.  GAPS_EINVAL for a null pointer, lr <= 0, beta outside [0, 1)
 * or eps <= 0; GAPS_ESTATE before the weights exist. */
gaps_status gaps_mlp_adam_step(gaps_ctx ctx, float* grad, float lr, float beta1, float beta2, float eps,
                               hipStream_t stream);

typedef struct {
    int64_t steps;       /* Adam steps */
    int64_t batch;       /* rows per step, drawn at random from the n rows */
    float lr, beta1, beta2, eps, tau;
    uint64_t seed;       /* batch sampling (Philox stream 5) */
} gaps_train_params;

/* Train the context's network on device rows x [n][4], y [n]; step losses go
 * to device loss[steps] (may be NULL).  Asynchronous. */
gaps_status gaps_mlp_train(gaps_ctx ctx, const float* x, const float* y, int64_t n, const gaps_train_params* p,
                           float* loss, hipStream_t stream);
/* Calibration margins from held-out device rows (x, y, cell as
 * gaps_mlp_features gives it): one per cell, as described above (+inf: the
 * analytic bound).  Asynchronous (no stream
 * synchronisation): the network's outputs are staged through the context's
 * tabulation buffers (24 MB, allocated by the first call of either function
 * on a context), in chunks, in stream order.  GAPS_ENOMEM if they cannot be
 * allocated. */
gaps_status gaps_mlp_calibrate(gaps_ctx ctx, const float* x, const float* y, const int32_t* cell, int64_t n,
                               hipStream_t stream);
/* Margins from / to HOST memory ([64][48][8] doubles: entries 8..71, eta
 * bins, ln t cells; +inf: analytic). */
gaps_status gaps_mlp_set_delta(gaps_ctx ctx, const double* host_delta);
gaps_status gaps_mlp_get_delta(gaps_ctx ctx, double* host_delta);
/* Tabulate the learned bound from the current weights and margins and enable
 * LEARNED mode for later gaps_shower calls on the same stream.  Asynchronous. */
gaps_status gaps_mlp_tabulate(gaps_ctx ctx, hipStream_t stream);
/* Copy the learned bound [64][48][8] (doubles) to HOST memory.  Synchronous;
 * GAPS_ESTATE before gaps_mlp_tabulate. */
gaps_status gaps_learned_table(gaps_ctx ctx, double* host_out);
/* Install a learned bound [64][48][8] given in HOST memory (every value must be
 * finite and at most the analytic table's entry; GAPS_EINVAL otherwise) and
 * enable LEARNED mode.  Synchronous. */
gaps_status gaps_learned_set_table(gaps_ctx ctx, const double* host_table);

/* Per-event observables (section 4.1): obs is device [n][12], one row per
 * event.  For pp processes the columns are
 *   0 Z pT (the lepton pair's transverse momentum), 1 Z rapidity, 2 Z azimuth
 *   (0 when the pair has no transverse recoil), 3 phi*, 4 number of anti-kT
 *   jets (R = 0.4, E-scheme, pT > 5 GeV, |eta| < 5), 5 leading-jet pT
 *   (|eta| < 5), 6 leading-jet pseudorapidity (pT > 5 GeV), 7 second-jet pT
 *   (|eta| < 5), 8 Delta R of the two leading jets (both cuts; -1 with fewer
 *   than two), 9 number of final-state partons, 10 largest component of the
 *   final minus the initial total four-momentum (momentum conservation), 11
 *   unused (0);
 * for e+e- (process 0): 0 1 - thrust, 1-4 Durham y23, y34, y45, y56 (E
 *   scheme), 9 number of final-state partons, 10 momentum imbalance as above,
 *   the others 0. */
gaps_status gaps_observables(gaps_ctx ctx, const gaps_events* ev, int64_t n, double* obs,
                             hipStream_t stream);

/* Weighted histogram of column col of obs (device [n][12]) with weights w
 * (device [n], or NULL for unit weights): nbins uniform bins on [lo, hi),
 * device sumw/sumw2 [nbins] accumulated (caller zeroes them). */
gaps_status gaps_histogram(gaps_ctx ctx, const double* obs, const double* w, int64_t n, int col,
                           double lo, double hi, int nbins, double* sumw, double* sumw2,
                           hipStream_t stream);

/* Copy the overestimate table (72 entries x 48 eta bins, doubles) to HOST
 * memory host_out.  Synchronous. */
gaps_status gaps_bounds(gaps_ctx ctx, double* host_out);

/* PDF evaluation x*f(tab, x, q2) for n device points (the grid lookup of the
 * shower, exposed for tests and the lookup micro-benchmark). */
gaps_status gaps_pdf_eval(gaps_ctx ctx, const int32_t* tab, const double* x, const double* q2,
                          int64_t n, double* out, hipStream_t stream);

/* Philox4x32-10 blocks: out[4*k..4*k+3] for counter (id[k], c2[k], c3[k]) and
 * key (seed, stream id), all device arrays of length n. */
gaps_status gaps_rng_blocks(uint64_t seed, uint32_t stream_id, const int64_t* id,
                            const uint32_t* c2, const uint32_t* c3, int64_t n, uint32_t* out,
                            hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
