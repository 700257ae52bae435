// Kernel declarations shared by the translation units of libgaps.
#pragma once

#include "../../include/gaps.h"
#include "device.hpp"

namespace gaps {

// Trial data of a channel cache entry (32 bytes): the kinematic limit t_lim
// and its log, 1/c of the current overestimate (of the current cell in learned
// mode), and a copy of the entry's info word.  The info words and the pending
// trial keys of the retained form also sit in arrays of their own
// (Scratch::info, Scratch::key): the channel build's walk over an event's
// entries reads only the info words, the argmax scan only the keys, and the
// winner reads its info word from this copy, in the line it loads anyway.
// Every write of an info word writes both.
struct alignas(16) Trial {
  double tl, ltl, ic;
  uint32_t info, pad0;
};
static_assert(sizeof(Trial) == 32, "trial record layout");

// Winner data of a channel cache entry, contiguous (80 bytes): the total
// overestimate constant c (in learned mode the constant of the current cell),
// the dipole invariant s, the z limits, the z integrals of the channel's two
// shapes, the momentum fraction 2E/sqrt(S) in the PDF ratio's denominator (the
// incoming emitter's for IF and II, the incoming spectator's for FI, 0 for FF)
// and its logarithm, log(zlo / (1 - zlo)) of an incoming emitter's channel,
// and the two flavours (int8 each, emitter in the low byte).
struct Win {
  double c, s, zlo, omzhi, I1, I2, etap, lnep, lz1;
  uint32_t pid, pad0;
};
static_assert(sizeof(Win) == 80, "winner record layout");

// One channel cache entry: its winner and trial data side by side in one
// 128-byte line, so that the winner of a cycle (and its redraw) reads one line;
// for a learned channel also the learned constants of its current cell that
// its term choice reads first (lr: a quark's families A and B, a gluon's
// family C), written with the cell constant.
struct alignas(128) Ent {
  Win w;
  Trial t;
  double lr[2];
};
static_assert(sizeof(Ent) == 128, "channel cache entry layout");

// Per-lane working storage of the shower kernels: event records and channel
// caches, slot-major with stride = number of lanes (coalesced across a wave).
struct Scratch {
  int64_t lanes;
  int max_slots;
  Part* part;  // working event records (lane-major in the wave kernels: one event's partons adjacent)
  // channel cache [lanes][nch]: one event's entries contiguous (the wave's
  // passes give consecutive lanes consecutive entries of an event), one line
  // of winner and trial data per entry
  int nch;             // entries per event: 2 max_slots rounded up to a multiple of 4
  struct Ent* ent;
  // pending trial key ln t of each entry (retained form; -inf: none above the
  // cutoff), [lanes][nch] like the records: an event's keys are contiguous, so
  // the argmax scan reads 8 bytes per entry
  double* key;
  // info word of each entry, [lanes][nch]: alive | type << 1 | heavy << 3 |
  // spectator << 5 | eta bin << 13 | spectator eta bin << 19 | learned cell
  // << 25 | null << 29 | first-emission correction << 30
  uint32_t* info;
  // weight factor of the event in each state slot, written by the weighted
  // veto of a violated learned bound (valid while the event's flags carry
  // fFallback)
  double* wfac;
  // the accepted emission awaiting its channel build, per lane slot,
  // [lanes][kPendStride]: z, 1 - z, azimuth, the two map variables, the
  // dipole's s (one lane's record in one 64-byte piece of a line: accepts are
  // sparse, so a lane-major record touches one line where a slot-major one
  // would touch six)
  double* pend;
  unsigned long long* queue;  // work-queue counters
};

// doubles per lane of the pending-emission record
constexpr int kPendStride = 8;

// bytes of LDS per thread for the tail-compaction state pool of the wave kernel
constexpr size_t kLaneStateBytes = 96;

struct ShowerArgs {
  int mode;
  int gen_select;  // one event per lane kernel: the generate-select form
  int veto_max;    // one event per lane kernel: the veto-max form
  int compact_every;
  int tail_every;
  uint32_t stream;
  uint64_t seed;
  int64_t n;
  const gaps_batch* batches;  // device table of a stream (nbatch > 0), else the kernel's in/out
  const int64_t* prefix;      // device [nbatch + 1]: first stream index of each batch
  int nbatch;
  float* log;
  int64_t log_cap;
  unsigned long long* log_count;
  unsigned long long* stats;
};

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v);
__global__ void k_rng_blocks(uint64_t seed, uint32_t stream, const int64_t* id, const uint32_t* c2,
                             const uint32_t* c3, int64_t n, uint32_t* out);
__global__ void k_pdf_eval(Cfg C, const int32_t* tab, const double* x, const double* q2, int64_t n,
                           double* out);
__global__ void k_bounds(Cfg C, double* bound);
__global__ void k_bound_sums(Cfg C, double* bound);
__global__ void k_learn_sums(Cfg C, const double* learn, double* sd);
__global__ void k_lo_scan(Cfg C, double* w);
__global__ void k_lo_max(const double* w, int n, double* out);
__global__ void k_hard(Cfg C, int64_t first_id, int64_t n, uint64_t seed, gaps_events o);
__global__ void k_shower_lanes(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A);
__global__ void k_shower_lanes_gs(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A);
__global__ void k_shower_lanes_vm(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A);
__global__ void k_shower_wave(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A);
__global__ void k_shower_wave_rt(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A);
__global__ void k_shower_wave_rt3(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A);
__global__ void k_shower_wave3(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A);
__global__ void k_shower_wave4(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A);
// a chunk of a stream's batch table, passed by value (fits the kernel-argument space)
constexpr int kBatchChunk = 8;
struct BatchChunk {
  gaps_batch b[kBatchChunk];
  int64_t first[kBatchChunk];  // stream index of each batch's first event
  int count;
  int at;                      // table position of b[0]
  int64_t total;               // written to prefix[nbatch] by the last chunk
  int last;
};
__global__ void k_store_batches(BatchChunk ch, gaps_batch* table, int64_t* prefix, int nbatch);
__global__ void k_observables(Cfg C, gaps_events ev, int64_t n, double* obs);
// pp observables with one event per wave, for events of at most kObsW slots
constexpr int kObsW = 128, kObsWaves = 4;
constexpr int kHistLds = 2048;  // histograms of at most this many bins accumulate in LDS
__global__ void k_observables_pp(Cfg C, gaps_events ev, int64_t n, double* obs);

// learned bound network (4 -> 64 -> 64 -> 1)
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = 4545;
constexpr int64_t kMlpProbeRows = (int64_t)kNIS * kNB * kNTB * 48;
__global__ void k_mlp_fwd(const uint16_t* wb, const float* x, int64_t n, float* f);
__global__ void k_mlp_grad(const uint16_t* wb, const float* x, const float* y, int64_t nrows, int64_t nsrc,
                           uint64_t seed, int64_t step, int sample, float tau, float inv_n, float* grad, float* loss);
__global__ void k_adam(float* theta, uint16_t* wb, float* grad, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2);
__global__ void k_mlp_pack(const float* theta, uint16_t* wb, int n);
__global__ void k_mlp_init(uint64_t seed, float* theta, int n);
__global__ void k_mlp_features(Cfg C, const float* rows, int64_t n, const double* bound, float* x, float* y,
                               int32_t* ent, int32_t* cell);
__global__ void k_mlp_resid(const float* f, const float* y, const int32_t* cell, int64_t n,
                            unsigned long long* maxbits, unsigned long long* count);
__global__ void k_mlp_delta(const unsigned long long* maxbits, const unsigned long long* count, long long min_cell,
                            long long min_bin, long long min_entry, double margin, double* delta);
__global__ void k_mlp_probes(Cfg C, float* x);
__global__ void k_mlp_table(const float* f, const double* delta, const double* bound, double* table);
__global__ void k_cellmax_fit(Cfg C, const float* rows, int64_t n, unsigned long long* ymax, unsigned long long* count);
// calibration groups of the cell-maximum bound: one per entry, and one per
// coarser level of the adaptive blocks
constexpr int kCmGroups = kNIS + 6;
__global__ void k_cellmax_resid(Cfg C, const float* rows, int64_t n, const unsigned long long* ymax,
                                const unsigned long long* count, const unsigned long long* level, long long min_cell,
                                unsigned long long* emax, unsigned long long* ecount);
__global__ void k_cellmax_adapt(const unsigned long long* ymax, const unsigned long long* count, long long min_cell,
                                unsigned long long* aymax, unsigned long long* acount, unsigned long long* alevel);
__global__ void k_cellmax_table(const unsigned long long* ymax, const unsigned long long* count,
                                const unsigned long long* level, const unsigned long long* emax,
                                const unsigned long long* ecount, long long min_cell, long long min_cal, double margin,
                                const double* bound, double* table);
__global__ void k_histogram(const double* obs, const double* w, int64_t n, int col, double lo, double hi,
                            int nbins, double* sumw, double* sumw2);

}  // namespace gaps
