// Device-side physics of the gfx950 shower: random numbers, coupling, PDF
// lookup, channel constants, trial scales, veto weights and the kinematic maps
// (arXiv:2511.19633 section 2, appendices A and B).  FP64 throughout.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>

namespace gaps {

constexpr double kPi = 3.14159265358979323846;
constexpr double kCF = 4.0 / 3.0;
constexpr double kCA = 3.0;
constexpr double kTR = 0.5;
constexpr double kNC = 3.0;

// Overestimate table: 48 eta bins uniform in ln(eta) on [1e-6, 1); entries
// FI[T], S1[family][T], S3[family][T] (T: PDF table, family A..D).
constexpr int kNB = 48;
constexpr double kLnEta0 = -13.815510557964274;  // ln(1e-6)
constexpr int kNEnt = 72;
__host__ __device__ constexpr int ent_fi(int T) { return T; }
__host__ __device__ constexpr int ent_s1(int f, int T) { return 8 + 8 * f + T; }
__host__ __device__ constexpr int ent_s3(int f, int T) { return 40 + 8 * f + T; }

// Rows of the bound table after the entries and the corrected family-B rows:
// per eta bin the sums, in term order, of an initial-state gluon's g <- q
// constants (the D entries of every flavour) at an IF and at an II end
constexpr int kSumIF = kNEnt + 8, kSumII = kNEnt + 9;
constexpr int kBoundRows = kNEnt + 10;

// learned bound: initial-state entries kIS0.. (kNIS of them), kNTB cells in ln t
constexpr int kIS0 = 8;
constexpr int kNIS = 64;
constexpr int kNTB = 8;

constexpr int kMaxSlots = 256;
// most overestimate terms of a channel: an initial-state gluon, 1 + 2 nf (nf <= 5)
constexpr int kMaxTerms = 11;
constexpr uint32_t kMaxCycles = 2000000u;
constexpr double kMecB = 2.625;  // overestimate factor of a corrected learned family-B term

enum : int { kFF = 0, kFI = 1, kIF = 2, kII = 3 };
enum : int { kSoft = 0, kFlat = 1, kS1 = 2, kS3 = 3 };
// splitting families: final-state q->qg, g->gg, g->qqbar; backward steps
// A (q <- q, gluon emitted), B (q <- g), C (g <- g), D (g <- q)
enum : int { kQQG = 0, kGGG = 1, kGQQ = 2, kA = 3, kB = 4, kC = 5, kD = 6 };
enum : int { famA = 0, famB = 1, famC = 2, famD = 3 };

enum : uint32_t {
  fOverflow = 1u, fColour = 2u, fNaN = 4u, fFallback = 8u, fViol = 16u,
  fHardFail = 32u, fHEvent = 64u, fMaxCyc = 128u, fMEC = 256u
};

// Everything the kernels need, passed by value (kernel-argument segment).
struct Cfg {
  int process, nf, nx, nq;
  double sqrt_s, S, t_cut, tc_is, alphas_mz, mz, gz, mz2, b0, as_over;
  double ln_mz2;  // log(mz2), computed on the host
  double mc2, mb2, tch_c, tch_b, ln_tc, ln_tcis, ln_tch_c, ln_tch_b;
  double sw2, gf, mll_min, mll_max, p_s, over_scale;
  double lnx0, lnx1, lnq0, lnq1, dlnx, dlnq;
  double lo_wmax;
  int matching;
  double mu_q2;
  double cell_edge[kNTB + 1];  // ln t edges of the learned-bound cells
  const float* pdf;      // [8][nq][nx]
  const double* bound;   // [kBoundRows][48]: the entries, family B under the
                         // first-emission correction by the quark's PDF table,
                         // and the gluon's g <- q sums (kSumIF, kSumII)
  const double* learn;   // [64][48][8] learned bound (LEARNED mode), or null
  const double* learn_sd;  // [2][48][8] its g <- q sums (IF, II) per eta bin and cell
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11), counter (id_lo, id_hi, c2, c3), key
// (seed_lo, seed_hi ^ stream).
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1, uint32_t o[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32 x 32 -> 64-bit product in one multiply (its high and low words)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  o[0] = c0; o[1] = c1; o[2] = c2; o[3] = c3;
}

__device__ __forceinline__ double u01(uint32_t w) { return ((double)w + 0.5) * 2.3283064365386963e-10; }

__device__ __forceinline__ void rng4(uint64_t seed, uint32_t stream, int64_t id, uint32_t c2,
                                     uint32_t c3, double u[4]) {
  uint32_t o[4];
  philox((uint32_t)(uint64_t)id, (uint32_t)((uint64_t)id >> 32), c2, c3, (uint32_t)seed,
         (uint32_t)(seed >> 32) ^ stream, o);
  u[0] = u01(o[0]); u[1] = u01(o[1]); u[2] = u01(o[2]); u[3] = u01(o[3]);
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ double alphas(const Cfg& C, double t) {
  return C.alphas_mz / (1.0 + C.alphas_mz * C.b0 * log(t / C.mz2));
}

// the same coupling at ln t: ln(t / mZ^2) = ln t - ln mZ^2 (a trial is drawn
// in ln t, so its coupling needs no logarithm)
__device__ __forceinline__ double alphas_ln(const Cfg& C, double lnt) {
  return C.alphas_mz / (1.0 + C.alphas_mz * C.b0 * (lnt - C.ln_mz2));
}

__device__ __forceinline__ int pdf_tab(int pid) {
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

// x*f: bilinear in (ln x, ln Q^2) of the node values, zero outside the grid
// (no extrapolation, appendix B.6).
__device__ inline double pdf_xf(const Cfg& C, int tab, double x, double q2) {
  if (!(x > 0.0) || x >= 1.0 || !(q2 > 0.0)) return 0.0;
  double lx = log(x), lq = log(q2);
  if (lx < C.lnx0 || lq < C.lnq0 || lq > C.lnq1) return 0.0;
  double fx = (lx - C.lnx0) / C.dlnx;
  int i = (int)fx;
  if (i > C.nx - 2) i = C.nx - 2;
  double a = fx - (double)i;
  double fq = (lq - C.lnq0) / C.dlnq;
  int j = (int)fq;
  if (j > C.nq - 2) j = C.nq - 2;
  double b = fq - (double)j;
  const float* F = C.pdf + (size_t)tab * C.nq * C.nx;
  double f00 = F[j * C.nx + i], f10 = F[j * C.nx + i + 1];
  double f01 = F[(j + 1) * C.nx + i], f11 = F[(j + 1) * C.nx + i + 1];
  return (1.0 - b) * ((1.0 - a) * f00 + a * f10) + b * ((1.0 - a) * f01 + a * f11);
}

// the same lookup with ln(q2) supplied by the caller (shared by the two
// lookups of a PDF ratio)
__device__ inline double pdf_xf_l(const Cfg& C, int tab, double x, double q2, double lq) {
  if (!(x > 0.0) || x >= 1.0 || !(q2 > 0.0)) return 0.0;
  double lx = log(x);
  if (lx < C.lnx0 || lq < C.lnq0 || lq > C.lnq1) return 0.0;
  double fx = (lx - C.lnx0) / C.dlnx;
  int i = (int)fx;
  if (i > C.nx - 2) i = C.nx - 2;
  double a = fx - (double)i;
  double fq = (lq - C.lnq0) / C.dlnq;
  int j = (int)fq;
  if (j > C.nq - 2) j = C.nq - 2;
  double b = fq - (double)j;
  const float* F = C.pdf + (size_t)tab * C.nq * C.nx;
  double f00 = F[j * C.nx + i], f10 = F[j * C.nx + i + 1];
  double f01 = F[(j + 1) * C.nx + i], f11 = F[(j + 1) * C.nx + i + 1];
  return (1.0 - b) * ((1.0 - a) * f00 + a * f10) + b * ((1.0 - a) * f01 + a * f11);
}

// the same lookup with ln(x) supplied too (a channel's cached momentum fraction)
__device__ inline double pdf_f_lx(const Cfg& C, int tab, double x, double lx, double q2, double lq) {
  if (!(x > 0.0) || x >= 1.0 || !(q2 > 0.0)) return 0.0;
  if (lx < C.lnx0 || lq < C.lnq0 || lq > C.lnq1) return 0.0;
  double fx = (lx - C.lnx0) / C.dlnx;
  int i = (int)fx;
  if (i > C.nx - 2) i = C.nx - 2;
  double a = fx - (double)i;
  double fq = (lq - C.lnq0) / C.dlnq;
  int j = (int)fq;
  if (j > C.nq - 2) j = C.nq - 2;
  double b = fq - (double)j;
  const float* F = C.pdf + (size_t)tab * C.nq * C.nx;
  double f00 = F[j * C.nx + i], f10 = F[j * C.nx + i + 1];
  double f01 = F[(j + 1) * C.nx + i], f11 = F[(j + 1) * C.nx + i + 1];
  const double xf = (1.0 - b) * ((1.0 - a) * f00 + a * f10) + b * ((1.0 - a) * f01 + a * f11);
  return xf > 0.0 ? xf / x : 0.0;
}

__device__ __forceinline__ double pdf_f_l(const Cfg& C, int tab, double x, double q2, double lq) {
  double xf = pdf_xf_l(C, tab, x, q2, lq);
  return xf > 0.0 ? xf / x : 0.0;
}

__device__ __forceinline__ double pdf_f(const Cfg& C, int tab, double x, double q2) {
  double xf = pdf_xf(C, tab, x, q2);
  return xf > 0.0 ? xf / x : 0.0;
}

__device__ __forceinline__ double dot4(const double* a, const double* b) {
  return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

// ---------------------------------------------------------------------------
// A parton of a working event record (48 bytes, one or two cache lines):
// momentum, flavour, colour tags and status side by side.
struct alignas(16) Part {
  double E, px, py, pz;
  int32_t pid, col, acol;
  int8_t st, pad0, pad1, pad2;
};
static_assert(sizeof(Part) == 48, "parton record layout");

// one field of the partons of a record, indexed like an array
template <typename T, size_t OFF>
struct PartField {
  Part* base;
  __device__ __forceinline__ T& operator[](int64_t k) const {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base + k) + OFF);
  }
};

// Working event record of one lane: parton q of state slot `lane` is
// part[q * sq + lane * sl] (lane-major: sq = 1, sl = slots; slot-major:
// sq = lanes, sl = 1).
struct Rec {
  PartField<double, offsetof(Part, E)> E;
  PartField<double, offsetof(Part, px)> px;
  PartField<double, offsetof(Part, py)> py;
  PartField<double, offsetof(Part, pz)> pz;
  PartField<int32_t, offsetof(Part, pid)> pid;
  PartField<int32_t, offsetof(Part, col)> col;
  PartField<int32_t, offsetof(Part, acol)> acol;
  PartField<int8_t, offsetof(Part, st)> st;
  int64_t sq, sl, lane;
  __device__ __forceinline__ int64_t o(int q) const { return (int64_t)q * sq + lane * sl; }
  __device__ __forceinline__ void get(int q, double p[4]) const {
    int64_t k = o(q);
    p[0] = E[k]; p[1] = px[k]; p[2] = py[k]; p[3] = pz[k];
  }
  __device__ __forceinline__ void set(int q, const double p[4]) const {
    int64_t k = o(q);
    E[k] = p[0]; px[k] = p[1]; py[k] = p[2]; pz[k] = p[3];
  }
  // colours as if every parton were outgoing (incoming ones swap)
  __device__ __forceinline__ int effc(int q) const { int64_t k = o(q); return st[k] < 0 ? acol[k] : col[k]; }
  __device__ __forceinline__ int effa(int q) const { int64_t k = o(q); return st[k] < 0 ? col[k] : acol[k]; }
  __device__ __forceinline__ void set_eff(int q, int c, int a) const {
    int64_t k = o(q);
    if (st[k] < 0) { col[k] = a; acol[k] = c; } else { col[k] = c; acol[k] = a; }
  }
};

__device__ __forceinline__ Rec make_rec(Part* p, int64_t sq, int64_t sl, int64_t lane) {
  return Rec{{p}, {p}, {p}, {p}, {p}, {p}, {p}, {p}, sq, sl, lane};
}

// ---------------------------------------------------------------------------
// Channel: dipole end (emitter i, spectator k, colour side) with its constants.
// Its overestimate terms are enumerated on demand by term_at(); the z
// integrals of the (at most two) z shapes a channel uses are I1 and I2.
// mec: an initial-initial channel of a quark whose next emission is corrected
// to the real matrix element (see mec_ratio)
struct Chan {
  int i, k, side, type, heavy, alive, ebin, kbin, pidi, pidk, nterm, mec;
  double s, eta, etak, tlim, lntlim, tcut, lntcut, m2;
  double zlo, zhi, omzlo, omzhi, I1, I2, c, invc;
  double lz1;  // log(zlo / (1 - zlo)) of an initial-state channel (its 1/(z(1-z)) shape), else 0
  // log of the momentum fraction in the PDF ratio's denominator: the
  // emitter's eta (IF, II) or the spectator's (FI); 0 for FF
  double lnep;
};

struct Term {
  int kern, shape, flav, ent;  // ent: overestimate-table entry (-1: none)
  double coefR, I;
};

// bin of a momentum fraction, from its logarithm
__device__ __forceinline__ int eta_bin_ln(double lneta) {
  const double dle = -kLnEta0 / kNB;
  double b = floor((lneta - kLnEta0) / dle);
  if (!(b >= 0.0)) return 0;
  if (b > kNB - 1) return kNB - 1;
  return (int)b;
}

// lz1: log(zlo / omzlo), the lower end of the 1/(z(1-z)) shape's log-odds.
// The curved shapes' integrals are each one logarithm of a ratio, taken once
// with the ratio chosen per shape (lanes with different shapes share it).
__device__ __forceinline__ double shape_int(int sh, double zlo, double zhi, double omzlo, double omzhi, double lz1) {
  if (sh == kFlat) return zhi - zlo;
  const double num = sh == kSoft ? omzlo : zhi;
  const double den = sh == kS3 ? zlo : omzhi;
  const double l = log(num / den);
  return sh == kS1 ? l - lz1 : l;
}

// Inverse of the shape's integral at u I.  Every curved shape takes one
// exponential, of an argument chosen per shape, so that lanes of a wave with
// different shapes share one evaluation.
__device__ __forceinline__ void shape_sample(int sh, const Chan& ch, double I, double u, double& z,
                                             double& omz) {
  if (sh == kFlat) {
    z = ch.zlo + u * (ch.zhi - ch.zlo);
    omz = 1.0 - z;
    return;
  }
  const double uI = u * I;
  const double arg = sh == kSoft ? -uI : (sh == kS1 ? -(ch.lz1 + uI) : uI);
  const double e = exp(arg);
  if (sh == kSoft) {
    omz = ch.omzlo * e;
    z = 1.0 - omz;
  } else if (sh == kS1) {
    z = 1.0 / (1.0 + e);
    omz = e / (1.0 + e);
  } else {
    z = ch.zlo * e;
    omz = 1.0 - z;
  }
}

__device__ __forceinline__ double shape_val(int sh, double z, double omz) {
  switch (sh) {
    case kSoft: return 1.0 / omz;
    case kFlat: return 1.0;
    case kS1: return 1.0 / (z * omz);
    default: return 1.0 / z;
  }
}

__device__ __forceinline__ bool is_fs(const Chan& ch) { return ch.type == kFF || ch.type == kFI; }

__device__ __forceinline__ int n_terms(const Chan& ch, int nf) {
  if (is_fs(ch)) return ch.pidi == 21 ? 1 + nf : 1;
  return ch.pidi == 21 ? 1 + 2 * nf : 2;
}

// Term m of a channel: splitting family, z shape, flavour, and the constant in
// front of the shape (kernel coefficient, and the PDF-ratio / Jacobian bound
// of the overestimate table for initial-state and final-initial channels).
__device__ __forceinline__ Term term_at(const Cfg& C, const Chan& ch, int m) {
  Term t;
  // the two shape integrals as values (a choice between the fields' addresses
  // would keep the channel record in private memory)
  const double I1 = ch.I1, I2 = ch.I2;
  if (is_fs(ch)) {
    double R = 1.0;
    t.ent = -1;
    if (ch.type == kFI) {
      t.ent = ent_fi(pdf_tab(ch.pidk));
      R = C.bound[t.ent * kNB + ch.kbin];
    }
    if (ch.pidi == 21) {
      if (m == 0) { t.kern = kGGG; t.shape = kSoft; t.flav = 0; t.coefR = kCA * R; t.I = I1; }
      else { t.kern = kGQQ; t.shape = kFlat; t.flav = m; t.coefR = 0.5 * kTR * R; t.I = I2; }
    } else {
      t.kern = kQQG; t.shape = kSoft; t.flav = 0; t.coefR = 2.0 * kCF * R; t.I = I1;
    }
    return t;
  }
  const bool ii = ch.type == kII;
  const int sh2 = ii ? kS3 : kS1;
  if (ch.pidi == 21) {
    if (m == 0) {
      t.kern = kC; t.shape = kS1; t.flav = 0; t.ent = ent_s1(famC, 0); t.I = I1;
    } else {
      int a = m <= C.nf ? m : -(m - C.nf);
      int T = pdf_tab(a);
      t.kern = kD; t.shape = sh2; t.flav = a; t.ent = ii ? ent_s3(famD, T) : ent_s1(famD, T); t.I = I2;
    }
  } else {
    int T = pdf_tab(ch.pidi);
    if (m == 0) {
      t.kern = kA; t.shape = kS1; t.flav = 0; t.ent = ent_s1(famA, T); t.I = I1;
    } else {
      t.kern = kB; t.shape = sh2; t.flav = 0; t.ent = ii ? ent_s3(famB, T) : ent_s1(famB, T); t.I = I2;
    }
  }
  t.coefR = C.bound[t.ent * kNB + ch.ebin];  // (a corrected family B: see select_term)
  return t;
}

// Entry of the m-th g <- q term of an initial-state gluon (m = 1 .. 2 nf):
// flavours 1..nf, then -1..-nf.
__device__ __forceinline__ int gluon_d_entry(const Cfg& C, bool ii, int m) {
  const int a = m <= C.nf ? m : -(m - C.nf);
  const int T = pdf_tab(a);
  return ii ? ent_s3(famD, T) : ent_s1(famD, T);
}

// The channel's constant c: the sum over its terms of af R_m I_m.  A quark's
// two terms are added in order; the terms of a gluon after the first (g <- q
// for every flavour) share one z shape, so their part is af (sum of their R
// in term order) I2, the sum being a precomputed row (kSumIF, kSumII) of the
// table R_of reads.
template <class Tab>
__device__ __forceinline__ double is_terms_c(const Cfg& C, int type, int pidi, double I1, double I2, Tab R_of,
                                             bool mec) {
  const double af = C.as_over / (2.0 * kPi) * C.over_scale;
  const bool ii = type == kII;
  if (pidi == 21) {
    const double R0 = R_of(ent_s1(famC, 0)), sum = R_of(ii ? kSumII : kSumIF);
    return af * R0 * I1 + af * sum * I2;
  }
  const int T = pdf_tab(pidi);
  const double RA = R_of(ent_s1(famA, T));
  // a corrected channel's family B: the corrected table (entry kNEnt + T)
  const double RB = R_of(mec ? kNEnt + T : (ii ? ent_s3(famB, T) : ent_s1(famB, T)));
  double c = 0.0;
  c += af * RA * I1;
  c += af * RB * I2;
  return c;
}

// The term of an initial-state channel whose running sum of constants (in
// term order, written as in is_terms_c) first exceeds target, and its
// constant; -1 if none does.  A gluon's g <- q constants are loaded only when
// the draw passes its first term.
template <class Tab>
__device__ __forceinline__ int is_terms_pick(const Cfg& C, int type, int pidi, double I1, double I2, double target,
                                             Tab R_of, bool mec, double& Rsel) {
  const double af = C.as_over / (2.0 * kPi) * C.over_scale;
  const bool ii = type == kII;
  int sel = -1;
  Rsel = 0.0;
  if (pidi == 21) {
    const double R0 = R_of(ent_s1(famC, 0));
    const double c0 = af * R0 * I1;
    if (target < c0) {
      Rsel = R0;
      return 0;
    }
    double R[kMaxTerms];
    const int nt = 1 + 2 * C.nf;
#pragma unroll
    for (int m = 1; m < kMaxTerms; ++m) R[m] = m < nt ? R_of(gluon_d_entry(C, ii, m)) : 0.0;
    double sum = 0.0;
#pragma unroll
    for (int m = 1; m < kMaxTerms; ++m)
      if (sel < 0 && m < nt) {
        sum += R[m];
        if (target < c0 + af * sum * I2) { sel = m; Rsel = R[m]; }
      }
    return sel;
  }
  const int T = pdf_tab(pidi);
  const double RA = R_of(ent_s1(famA, T));
  const double RB = R_of(mec ? kNEnt + T : (ii ? ent_s3(famB, T) : ent_s1(famB, T)));
  double cum = 0.0;
  cum += af * RA * I1;
  if (target < cum) { sel = 0; Rsel = RA; }
  cum += af * RB * I2;
  if (sel < 0 && target < cum) { sel = 1; Rsel = RB; }
  return sel;
}

// the sum, in term order, of the g <- q constants of a gluon at an IF (ii
// false) or II end, from a table of per-entry constants
template <class Tab>
__device__ __forceinline__ double gluon_d_sum(const Cfg& C, bool ii, Tab R_of) {
  double sum = 0.0;
  for (int m = 1; m < 1 + 2 * C.nf; ++m) sum += R_of(gluon_d_entry(C, ii, m));
  return sum;
}

// Channel constants of dipole end (i, side) with spectator k: invariant,
// momentum fractions, kinematic limit (appendix B), the widest z range (at the
// cutoff), and the total overestimate c of G = c/t (appendix A.1).  mec: the
// event's next emission is corrected to the real matrix element (applies to
// its initial-initial quark channels).
__device__ inline void chan_setup(const Cfg& C, const Rec& R, int i, int side, int k, Chan& ch, bool mec) {
  ch.i = i; ch.k = k; ch.side = side; ch.alive = 0; ch.heavy = 0; ch.nterm = 0;
  ch.m2 = 0.0; ch.c = 0.0; ch.invc = 0.0; ch.ebin = 0; ch.kbin = 0;
  ch.zlo = ch.zhi = ch.omzlo = ch.omzhi = ch.I1 = ch.I2 = ch.lz1 = ch.lnep = 0.0;
  int sti = R.st[R.o(i)], stk = R.st[R.o(k)];
  bool isE = sti < 0, isS = stk < 0;
  ch.pidi = R.pid[R.o(i)];
  ch.pidk = R.pid[R.o(k)];
  ch.type = isE ? (isS ? kII : kIF) : (isS ? kFI : kFF);
  ch.mec = mec && ch.type == kII && ch.pidi != 21;
  double pi[4], pk[4];
  R.get(i, pi);
  R.get(k, pk);
  ch.s = 2.0 * dot4(pi, pk);
  ch.eta = isE ? 2.0 * pi[0] / C.sqrt_s : 0.0;
  ch.etak = isS ? 2.0 * pk[0] / C.sqrt_s : 0.0;
  double tc = ch.type == kFF ? C.t_cut : C.tc_is;
  double s = ch.s, eta = ch.eta, etak = ch.etak, d;
  ch.tcut = tc;
  ch.lntcut = ch.type == kFF ? C.ln_tc : C.ln_tcis;
  ch.tlim = 0.0;
  ch.lntlim = 0.0;
  if (!(s > 0.0)) return;
  switch (ch.type) {
    case kFF: ch.tlim = s / 4.0; d = 4.0 * tc / s; break;
    case kFI: ch.tlim = s * (1.0 - etak) / (4.0 * etak); d = 4.0 * tc * etak / (s * (1.0 - etak)); break;
    case kIF: ch.tlim = s * (1.0 - eta) / (4.0 * eta); d = 4.0 * tc * eta / (s * (1.0 - eta)); break;
    default:
      ch.tlim = s * (1.0 - eta) * (1.0 - eta) / (4.0 * eta);
      d = 4.0 * tc * eta / (s * (1.0 - eta) * (1.0 - eta));
      break;
  }
  if (isE) {
    int ap = ch.pidi < 0 ? -ch.pidi : ch.pidi;
    if (ap == 4) { ch.heavy = 1; ch.m2 = C.mc2; ch.tcut = C.tch_c; ch.lntcut = C.ln_tch_c; }
    if (ap == 5) { ch.heavy = 2; ch.m2 = C.mb2; ch.tcut = C.tch_b; ch.lntcut = C.ln_tch_b; }
    if (pdf_tab(ch.pidi) < 0) return;
  } else if (ch.type == kFI && pdf_tab(ch.pidk) < 0) {
    return;
  }
  if (!(d < 1.0) || !(ch.tlim > ch.tcut)) return;
  ch.lntlim = log(ch.tlim);
  double sq = sqrt(1.0 - d);
  if (ch.type == kFF || ch.type == kFI) {
    ch.zlo = 0.5 * d / (1.0 + sq);
    ch.omzhi = ch.zlo;
    ch.zhi = 1.0 - ch.zlo;
    ch.omzlo = 1.0 - ch.zlo;
  } else {
    ch.omzhi = 0.5 * (1.0 - eta) * d / (1.0 + sq);
    ch.zhi = 1.0 - ch.omzhi;
    ch.zlo = (4.0 * eta + (1.0 - eta) * (1.0 - eta) * d) / (2.0 * ((1.0 + eta) + (1.0 - eta) * sq));
    ch.omzlo = 1.0 - ch.zlo;
  }
  if (isE || ch.type == kFI) {  // one bin evaluation: the emitter's or the spectator's
    ch.lnep = log(isE ? eta : etak);
    const int b = eta_bin_ln(ch.lnep);
    if (isE) ch.ebin = b;
    else ch.kbin = b;
  }
  int sh1 = is_fs(ch) ? kSoft : kS1;
  int sh2 = is_fs(ch) ? kFlat : (ch.type == kII ? kS3 : kS1);
  if (isE) ch.lz1 = log(ch.zlo / ch.omzlo);
  ch.I1 = shape_int(sh1, ch.zlo, ch.zhi, ch.omzlo, ch.omzhi, ch.lz1);
  ch.I2 = shape_int(sh2, ch.zlo, ch.zhi, ch.omzlo, ch.omzhi, ch.lz1);
  ch.nterm = n_terms(ch, C.nf);
  double c = 0.0;
  if (isE) {
    const int eb = ch.ebin;
    c = is_terms_c(C, ch.type, ch.pidi, ch.I1, ch.I2, [&](int ent) { return C.bound[ent * kNB + eb]; }, ch.mec);
  } else {
    double af = C.as_over / (2.0 * kPi) * C.over_scale;
    for (int m = 0; m < ch.nterm; ++m) {
      Term t = term_at(C, ch, m);
      c += af * t.coefR * t.I;
    }
  }
  if (!(c > 0.0)) return;
  ch.c = c;
  ch.invc = 1.0 / c;
  ch.alive = 1;
}

// ---------------------------------------------------------------------------
// Learned bound (LEARNED mode): an initial-state channel's overestimate
// constant in cell k of ln t is the sum over its terms, in order, of
// alpha_s(t_c)/(2 pi) * R_theta[entry][eta bin][k] * (z integral of the shape)
// (computed for all cells at the channel build).
// (an entry kNEnt + T, family B under the first-emission correction: the
// learned family-B constant times kMecB, the correction's largest value)
__device__ __forceinline__ double learned_R(const Cfg& C, int ent, int ebin, int k) {
  if (ent >= kSumIF) return C.learn_sd[((ent - kSumIF) * kNB + ebin) * kNTB + k];
  const bool mec = ent >= kNEnt;
  const double v = C.learn[(((mec ? ent_s3(famB, ent - kNEnt) : ent) - kIS0) * kNB + ebin) * kNTB + k];
  return mec ? v * kMecB : v;
}

// Splitting family (term) of the winner in proportion to the overestimates.
// A learned channel (lrn) draws from its constant ck in cell k, and the chosen
// term carries its cell constant; if rounding leaves the draw past every term,
// the last term of positive weight in the analytic bound.
// lr: a learned channel's cell constants of its first table reads (a quark's
// families A and B, a gluon's family C), as learned_c2 gave them when the
// channel entered cell k, so that they need no load; the others (a gluon's
// g <- q terms) load.
__device__ inline Term select_term(const Cfg& C, const Chan& ch, double u, bool lrn, int k, double ck,
                                   const double* lr = nullptr) {
  double af = C.as_over / (2.0 * kPi) * C.over_scale;
  double target = u * (lrn ? ck : ch.c), cum = 0.0;
  if (ch.type == kIF || ch.type == kII) {
    const int eb = ch.ebin;
    double Rsel;
    int nread = 0;
    const int m = is_terms_pick(C, ch.type, ch.pidi, ch.I1, ch.I2, target, [&](int ent) {
      const int r = nread++;
      if (!lrn) return C.bound[ent * kNB + eb];
      // a quark reads A then B, as learned_c2 did; a gluon reads C, then its
      // g <- q terms one by one (learned_c2's second read was their sum)
      if (lr && (r == 0 || (r == 1 && ch.pidi != 21))) return lr[r];
      return learned_R(C, ent, eb, k);
    }, ch.mec, Rsel);
    if (m >= 0) {
      Term t = term_at(C, ch, m);
      t.coefR = Rsel;
      return t;
    }
  } else {
    // a final-state emitter: its first term, then (a gluon) the g -> q qbar
    // terms, which share one constant: the running sum adds it once per
    // flavour, in term order
    const Term t0 = term_at(C, ch, 0);
    cum += af * t0.coefR * t0.I;
    if (target < cum) return t0;
    if (ch.nterm > 1) {
      Term t1 = term_at(C, ch, 1);
      const double inc = af * t1.coefR * t1.I;
      for (int m = 1; m < ch.nterm; ++m) {
        cum += inc;
        if (target < cum) {
          t1.flav = m;
          return t1;
        }
      }
    }
  }
  for (int m = ch.nterm - 1; m >= 0; --m) {
    Term t = term_at(C, ch, m);
    if (af * t.coefR * t.I > 0.0) {
      if (ch.mec && t.kern == kB) t.coefR = C.bound[(kNEnt + pdf_tab(ch.pidi)) * kNB + ch.ebin];
      if (lrn) t.coefR = learned_R(C, t.ent, ch.ebin, k) * (ch.mec && t.kern == kB ? kMecB : 1.0);
      return t;
    }
  }
  Term t = term_at(C, ch, 0);
  if (lrn) t.coefR = learned_R(C, t.ent, ch.ebin, k);
  return t;
}

__device__ __forceinline__ Term select_term(const Cfg& C, const Chan& ch, double u) {
  return select_term(C, ch, u, false, 0, 0.0);
}


// constant of cell k of an initial-state channel (type IF or II) whose emitter
// has flavour pidi, from the cell constants of its terms; the values of its
// first two table reads (a quark's families A and B, a gluon's family C and
// g <- q sum) go to lr[0], lr[1]
__device__ __forceinline__ double learned_c2(const Cfg& C, int type, int pidi, int ebin, double I1, double I2, int k,
                                             bool mec, double lr[2]) {
  int nread = 0;
  lr[0] = lr[1] = 0.0;
  return is_terms_c(C, type, pidi, I1, I2, [&](int ent) {
    const double v = learned_R(C, ent, ebin, k);
    if (nread < 2) lr[nread] = v;
    ++nread;
    return v;
  }, mec);
}

// the cell of a scale: the largest k with edge[k] < ln t (0 if none), and its
// lower edge (constant indices only, so the edges stay in registers)
__device__ __forceinline__ int cell_of(const Cfg& C, double lnt, double& edge) {
  int k = 0;
  edge = C.cell_edge[0];
#pragma unroll
  for (int j = 1; j < kNTB; ++j) {
    if (C.cell_edge[j] < lnt) {
      k = j;
      edge = C.cell_edge[j];
    }
  }
  return k;
}

// transverse momentum of size sqrt(tp) at azimuth phi, orthogonal to pa, pb
__device__ inline void kperp(const double* pa, const double* pb, double tp, double phi, double* kt) {
  double pab = dot4(pa, pb);
  double na = sqrt(pa[1] * pa[1] + pa[2] * pa[2] + pa[3] * pa[3]);
  double nb = sqrt(pb[1] * pb[1] + pb[2] * pb[2] + pb[3] * pb[3]);
  double d0 = pb[1] / nb - pa[1] / na, d1 = pb[2] / nb - pa[2] / na, d2 = pb[3] / nb - pa[3] / na;
  int ax = 0;
  double best = fabs(d0);
  if (fabs(d1) < best) { best = fabs(d1); ax = 1; }
  if (fabs(d2) < best) { best = fabs(d2); ax = 2; }
  // the lab axis as a four-vector (written without an indexed store, which
  // would put the array in private memory)
  const double r[4] = {0.0, ax == 0 ? 1.0 : 0.0, ax == 1 ? 1.0 : 0.0, ax == 2 ? 1.0 : 0.0};
  double ra = dot4(r, pa), rb = dot4(r, pb);
  double n1[4];
  for (int m = 0; m < 4; ++m) n1[m] = r[m] - rb / pab * pa[m] - ra / pab * pb[m];
  double n1n = sqrt(-dot4(n1, n1));
  for (int m = 0; m < 4; ++m) n1[m] /= n1n;
  double A[4] = {pa[0], -pa[1], -pa[2], -pa[3]};
  double B[4] = {pb[0], -pb[1], -pb[2], -pb[3]};
  double Cc[4] = {n1[0], -n1[1], -n1[2], -n1[3]};
  double n2[4];
  for (int mu = 0; mu < 4; ++mu) {
    // the three columns other than mu, ascending
    int c0 = mu == 0 ? 1 : 0;
    int c1 = mu <= 1 ? 2 : 1;
    int c2 = mu <= 2 ? 3 : 2;
    double det = A[c0] * (B[c1] * Cc[c2] - B[c2] * Cc[c1]) - A[c1] * (B[c0] * Cc[c2] - B[c2] * Cc[c0]) +
                 A[c2] * (B[c0] * Cc[c1] - B[c1] * Cc[c0]);
    n2[mu] = (mu & 1) ? -det : det;
  }
  double n2n = sqrt(-dot4(n2, n2));
  for (int m = 0; m < 4; ++m) n2[m] /= n2n;
  double kt0 = sqrt(tp), cp = cos(phi), sp = sin(phi);
  for (int m = 0; m < 4; ++m) kt[m] = kt0 * (cp * n1[m] + sp * n2[m]);
}

// II recoil transformation (appendix B.5) of one momentum: maps K' to K
__device__ __forceinline__ void ii_lambda(const double* Kp, const double* K, double* p) {
  double KK[4];
  for (int m = 0; m < 4; ++m) KK[m] = K[m] + Kp[m];
  double KK2 = dot4(KK, KK), Kp2 = dot4(Kp, Kp);
  double c1 = 2.0 * dot4(KK, p) / KK2;
  double c2 = 2.0 * dot4(Kp, p) / Kp2;
  for (int m = 0; m < 4; ++m) p[m] = p[m] - c1 * KK[m] + c2 * K[m];
}

// First-emission correction of a POWHEG-like event: the real matrix element
// over the shower's own density at the same real configuration, at the
// initial-initial (x, v) of the emission (appendix B.5; the density is the
// dipole of appendix C.2).  q qbar -> Z g is reached from both incoming
// quarks' family A (q -> q g), so R / (D_a + D_b) = 1 - 2 v (1 - x - v) /
// (1 + x^2), in [1/2, 1]; a quark from a gluon (family B, g qbar -> Z qbar)
// has only its own dipole: R / D = 1 + v (2 x + v) / (x^2 + (1 - x)^2), at
// most the golden ratio squared (2.618...).  A corrected channel's family-B
// overestimate covers it with a table of its own (the kernel bound times the
// factor's largest value at each momentum fraction, scanned like the others),
// or, for a learned constant, with the factor kMecB.
__device__ __forceinline__ double mec_ratio(bool family_b, double x, double v) {
  const double omx = 1.0 - x;
  if (!family_b) return 1.0 - 2.0 * v * (omx - v) / (1.0 + x * x);
  return 1.0 + v * (2.0 * x + v) / (x * x + omx * omx);
}

struct Veto {
  int ok;
  double x, omx, y, uv, w;
  double wn;  // the weight before division by the table constant (trial log)
};

// IF and II: (z, t) -> (x, u or v); the IF root in a cancellation-free form
__device__ __forceinline__ void is_vars(int type, double z, double omz, double t, double s, double& x,
                                        double& uv) {
  double r = t / s;
  if (type == kIF) {
    double D = omz + r;
    double dd = 4.0 * r * z * omz / (D * D);
    x = 2.0 * z * omz / (D * (1.0 + sqrt(1.0 - dd)));
  } else {
    x = z * omz / (omz + r);
  }
  uv = x * r / omz;
}

// acceptance weight of the winner trial: kinematic variables and phase-space
// check per dipole type, the splitting kernel, then one shared pair of PDF
// lookups for the ratio (spectator for FI, emitter for IF and II)
// t: the trial scale, lnt: its ln t as drawn (the PDF ratio's ln Q^2 and the
// coupling's logarithm)
__device__ inline Veto veto_weight(const Cfg& C, const Rec& R, const Chan& ch, const Term& tm, double t,
                                   double lnt, double z, double omz) {
  Veto r;
  r.ok = 0; r.x = 0.0; r.omx = 0.0; r.y = 0.0; r.uv = 0.0; r.w = 0.0; r.wn = 0.0;
  const double s = ch.s;
  const int kern = tm.kern, type = ch.type;
  const bool fs = type == kFF || type == kFI;
  double x = 0.0, omx = 0.0, y = 0.0, uv = 0.0;
  if (type == kFF) {
    y = t / (z * omz * s);
    if (!(y < 1.0)) return r;
  } else if (type == kFI) {
    double kap = t / (z * omz * s);
    x = 1.0 / (1.0 + kap);
    omx = kap * x;
    if (!(x > ch.etak)) return r;
  } else {
    is_vars(type, z, omz, t, s, x, uv);
    if (!(x > ch.eta)) return r;
    if (type == kIF && !(uv < 1.0)) return r;
    omx = 1.0 - x;
  }
  // splitting kernel (and the IF/II Jacobian)
  double P, J = 1.0;
  if (fs) {
    const double den1 = type == kFF ? omz + z * y : omz + omx;
    if (kern == kQQG) P = kCF * (2.0 / den1 - (1.0 + z));
    else if (kern == kGGG) P = 0.5 * kCA * (2.0 / den1 - 2.0 + z * omz);
    else P = 0.5 * kTR * (1.0 - 2.0 * z * omz);
  } else {
    const bool iff = type == kIF;
    J = iff ? 1.0 / (uv + x - 2.0 * uv * x) : 1.0 / z;
    const double soft = iff ? omx + uv : omx;
    switch (kern) {
      case kA: P = kCF * (2.0 / soft - (1.0 + x)); break;
      case kB: P = kTR * (1.0 - 2.0 * x * omx); break;
      case kC: P = kCA * (1.0 / soft + omx / x - 1.0 + x * omx); break;
      default: P = kCF * (x + 2.0 * omx / x); break;
    }
  }
  // PDF ratio: which tables at which momentum fractions
  double pr = 1.0;
  if (type != kFF) {
    int tnum, tden;
    double xd, xn;
    if (type == kFI) {
      tnum = tden = pdf_tab(ch.pidk);
      xd = ch.etak;
      xn = ch.etak / x;
    } else {
      const int Ti = pdf_tab(ch.pidi);
      switch (kern) {
        case kA: tnum = Ti; tden = Ti; break;
        case kB: tnum = 0; tden = Ti; break;
        case kC: tnum = 0; tden = 0; break;
        default: tnum = pdf_tab(tm.flav); tden = 0; break;
      }
      xd = ch.eta;
      xn = ch.eta / x;
    }
    if (tnum < 0 || tden < 0) return r;
    const double lq = lnt;
    const double den = pdf_f_lx(C, tden, xd, ch.lnep, t, lq);
    pr = den > 0.0 ? pdf_f_l(C, tnum, xn, t, lq) / den : 0.0;
  }
  double W;
  if (type == kFF) W = (1.0 - y) * P;
  else if (type == kFI) W = P * pr;
  else W = J * P * pr * (ch.heavy ? (t - ch.m2) / t : 1.0);
  if (ch.mec) W *= mec_ratio(kern == kB, x, uv);
  r.x = x; r.omx = omx; r.y = y; r.uv = uv;
  const double over = C.over_scale * tm.coefR * shape_val(tm.shape, z, omz);
  const double ar = alphas_ln(C, lnt) / C.as_over;
  r.w = ar * W / over;
  r.wn = ar * W / shape_val(tm.shape, z, omz);
  r.ok = 1;
  return r;
}

// momenta after the emission: emitter', emitted, spectator'
__device__ inline void do_map(int type, const double* pe, const double* ps, double s, double z, double omz,
                              double v1, double v2, double phi, double* pi, double* pj, double* pk) {
  double kt[4], tp;
  // ordering variable recomputed from the map variables, so that the new
  // momenta are massless to rounding
  switch (type) {
    case kFF: tp = z * omz * v1 * s; break;
    case kFI: tp = z * omz * v2 / v1 * s; break;
    case kIF: tp = v2 * (1.0 - v2) * (1.0 - v1) / v1 * s; break;
    default: tp = v2 * (1.0 - v1 - v2) / v1 * s; break;
  }
  kperp(pe, ps, tp, phi, kt);
  if (type == kFF) {
    const double y = v1;
    for (int m = 0; m < 4; ++m) {
      pi[m] = z * pe[m] + y * omz * ps[m] + kt[m];
      pj[m] = omz * pe[m] + y * z * ps[m] - kt[m];
      pk[m] = (1.0 - y) * ps[m];
    }
  } else if (type == kFI) {
    const double x = v1, omx = v2;
    const double a = omz * omx / x, b = z * omx / x;
    for (int m = 0; m < 4; ++m) {
      pi[m] = z * pe[m] + a * ps[m] + kt[m];
      pj[m] = omz * pe[m] + b * ps[m] - kt[m];
      pk[m] = ps[m] / x;
    }
  } else if (type == kIF) {
    const double x = v1, u = v2, omx = 1.0 - x;
    const double a = (1.0 - u) * omx / x, b = u * omx / x;
    for (int m = 0; m < 4; ++m) {
      pi[m] = pe[m] / x;
      pj[m] = a * pe[m] + u * ps[m] - kt[m];
      pk[m] = b * pe[m] + (1.0 - u) * ps[m] + kt[m];
    }
  } else {
    const double x = v1, v = v2;
    const double a = (1.0 - x - v) / x;
    for (int m = 0; m < 4; ++m) {
      pi[m] = pe[m] / x;
      pj[m] = a * pe[m] + v * ps[m] - kt[m];
      pk[m] = ps[m];
    }
  }
}

// the two map variables of an accepted trial: y (FF), x and 1 - x (FI), x and
// u (IF) or v (II)
__device__ __forceinline__ void map_vars(int type, const Veto& v, double& a1, double& a2) {
  a1 = type == kFF ? v.y : v.x;
  a2 = type == kFF ? 0.0 : (type == kFI ? v.omx : v.uv);
}

// apply the accepted emission of splitting kernel kern (flavour flav for the
// flavour-changing ones) with map variables a1, a2: momenta, flavours and
// colour tags; the emitted parton is appended at slot n
__device__ inline void emit_map(const Rec& R, int n, int& maxtag, const Chan& ch, int kern, int flav, double z,
                                double omz, double a1, double a2, double phi) {
  int i = ch.i, k = ch.k, j = n;
  double pe[4], ps[4], pi[4], pj[4], pk[4];
  // everything read of the emitter and spectator, before any write (a write
  // of a status byte may alias any later read, which would then wait for it)
  const int ec = R.effc(i), ea = R.effa(i);
  const int pidi = R.pid[R.o(i)];
  R.get(i, pe);
  R.get(k, ps);
  do_map(ch.type, pe, ps, ch.s, z, omz, a1, a2, phi, pi, pj, pk);
  if (ch.type == kII) {
    double Kp[4], K[4];
    for (int q = 0; q < 4; ++q) { Kp[q] = pe[q] + ps[q]; K[q] = pi[q] + pk[q] - pj[q]; }
    for (int q = 0; q < n; ++q) {
      if (q == i || q == k || R.st[R.o(q)] <= 0) continue;
      double p[4];
      R.get(q, p);
      ii_lambda(Kp, K, p);
      R.set(q, p);
    }
  }
  R.set(i, pi);
  R.set(k, pk);
  R.set(j, pj);
  R.st[R.o(j)] = 1;
  int jc = 0, ja = 0;
  if (kern == kQQG || kern == kGGG || kern == kA || kern == kC) {
    int N = ++maxtag;
    if (ch.side == 0) { R.set_eff(i, N, ea); jc = ec; ja = N; }
    else { R.set_eff(i, ec, N); jc = N; ja = ea; }
    R.pid[R.o(j)] = 21;
  } else if (kern == kGQQ) {
    int f = flav;
    if (ch.side == 0) { R.pid[R.o(i)] = f; R.set_eff(i, ec, 0); R.pid[R.o(j)] = -f; jc = 0; ja = ea; }
    else { R.pid[R.o(i)] = -f; R.set_eff(i, 0, ea); R.pid[R.o(j)] = f; jc = ec; ja = 0; }
  } else if (kern == kB) {
    int N = ++maxtag;
    R.pid[R.o(j)] = -pidi;
    if (ec == 0) { R.set_eff(i, N, ea); jc = 0; ja = N; }
    else { R.set_eff(i, ec, N); jc = N; ja = 0; }
    R.pid[R.o(i)] = 21;
  } else {  // kD
    int a = flav;
    if (a > 0) { R.set_eff(i, 0, ea); jc = ec; ja = 0; }
    else { R.set_eff(i, ec, 0); jc = 0; ja = ea; }
    R.pid[R.o(i)] = a;
    R.pid[R.o(j)] = a;
  }
  R.col[R.o(j)] = jc;
  R.acol[R.o(j)] = ja;
}

__device__ __forceinline__ void emit(const Rec& R, int n, int& maxtag, const Chan& ch, const Term& tm, double z,
                                     double omz, const Veto& v, double phi) {
  double a1, a2;
  map_vars(ch.type, v, a1, a2);
  emit_map(R, n, maxtag, ch, tm.kern, tm.flav, z, omz, a1, a2, phi);
}

}  // namespace gaps
