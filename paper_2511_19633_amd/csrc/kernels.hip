// gfx950 kernels of libgaps: overestimate table, hard events, the shower,
// observables and small helpers (arXiv:2511.19633).
#include "kernels.hpp"

namespace gaps {

// ---------------------------------------------------------------------------
// small helpers
__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// store one chunk of a stream's batch table (and its stream offsets)
__global__ void k_store_batches(BatchChunk ch, gaps_batch* table, int64_t* prefix, int nbatch) {
  const int k = threadIdx.x;
  if (k < ch.count) {
    table[ch.at + k] = ch.b[k];
    prefix[ch.at + k] = ch.first[k];
  }
  if (k == 0 && ch.last) prefix[nbatch] = ch.total;
}

__global__ void k_rng_blocks(uint64_t seed, uint32_t stream, const int64_t* id, const uint32_t* c2,
                             const uint32_t* c3, int64_t n, uint32_t* out) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint32_t o[4];
  uint64_t u = (uint64_t)id[k];
  philox((uint32_t)u, (uint32_t)(u >> 32), c2[k], c3[k], (uint32_t)seed, (uint32_t)(seed >> 32) ^ stream, o);
  for (int m = 0; m < 4; ++m) out[4 * k + m] = o[m];
}

__global__ void k_pdf_eval(Cfg C, const int32_t* tab, const double* x, const double* q2, int64_t n,
                           double* out) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  int t = tab[k];
  out[k] = (t >= 0 && t < 8) ? pdf_xf(C, t, x[k], q2[k]) : 0.0;
}

// ---------------------------------------------------------------------------
// Overestimate table (appendix A.2 procedure made strict): one thread per
// (entry, eta bin).  Upper envelope over the grid rows (the scale
// interpolant is a mediant of rows), over cells of the parent momentum
// fraction (bounded by node values), times 1.5, rounded up to a quarter
// octave.
__device__ double gbound(int shape, int fam, double x) {
  double omx = 1.0 - x;
  if (shape == 1) {
    switch (fam) {
      case famA: return kCF * (1.0 + x * x);
      case famB: return omx * kTR * (1.0 - 2.0 * x * omx);
      case famC: return kCA * (1.0 + omx * omx / x - omx + x * omx * omx);
      default: return omx * kCF * (x + 2.0 * omx / x);
    }
  }
  if (fam == famB) return kTR * (1.0 - 2.0 * x * omx);
  return kCF * (x + 2.0 * omx / x);
}

__device__ double quarter_octave_up(double v) {
  if (!(v > 0.0)) return 0.0;
  int e;
  double m = frexp(v, &e);
  double q;
  if (m <= 0.5) q = 0.5;
  else if (m <= 0.5946035575013605) q = 0.5946035575013605;
  else if (m <= 0.7071067811865476) q = 0.7071067811865476;
  else if (m <= 0.8408964152537145) q = 0.8408964152537145;
  else q = 1.0;
  return ldexp(q, e);
}

__device__ double xf_on_row(const Cfg& C, int tab, int j, double x) {
  if (!(x > 0.0) || x >= 1.0) return 0.0;
  double lx = log(x);
  if (lx < C.lnx0) return 0.0;
  double fx = (lx - C.lnx0) / C.dlnx;
  int i = (int)fx;
  if (i > C.nx - 2) i = C.nx - 2;
  double a = fx - (double)i;
  const float* F = C.pdf + ((size_t)tab * C.nq + j) * C.nx;
  return (1.0 - a) * (double)F[i] + a * (double)F[i + 1];
}

// the first-emission correction's largest value at momentum fraction x
// (family B, v = 1 - x), and over [lo, hi] (one maximum, at (3 - sqrt 5) / 2)
__device__ double mec_bmax(double x) {
  const double omx = 1.0 - x;
  return 1.0 + (1.0 - x * x) / (x * x + omx * omx);
}
__device__ double mec_bmax_range(double lo, double hi) {
  const double xs = 0.5 * (3.0 - sqrt(5.0));
  if (lo <= xs && xs <= hi) return mec_bmax(xs);
  const double a = mec_bmax(lo), b = mec_bmax(hi);
  return a > b ? a : b;
}

// entries 0 .. kNEnt-1 of the table, then kNEnt + T: family B at the
// initial-initial end (shape 3) while the first-emission correction applies
// (kind 4: the kernel bound times the correction's largest value)
// The rows kSumIF, kSumII of the bound table: per eta bin the sum, in term
// order, of an initial-state gluon's g <- q entries (after k_bounds).
__global__ void k_bound_sums(Cfg C, double* bound) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * kNB) return;
  const int ii = t / kNB, bin = t % kNB;
  bound[(kSumIF + ii) * kNB + bin] = gluon_d_sum(C, ii != 0, [&](int ent) { return bound[ent * kNB + bin]; });
}

// The same sums of a learned table [64][48][8], per eta bin and ln t cell.
__global__ void k_learn_sums(Cfg C, const double* learn, double* sd) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * kNB * kNTB) return;
  const int ii = t / (kNB * kNTB), bin = (t / kNTB) % kNB, k = t % kNTB;
  sd[t] = gluon_d_sum(C, ii != 0, [&](int ent) { return learn[((ent - kIS0) * kNB + bin) * kNTB + k]; });
}

__global__ void k_bounds(Cfg C, double* bound) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (kNEnt + 8) * kNB) return;
  int e = t / kNB, bin = t % kNB;
  // which transition this entry bounds
  int kind, fam = -1, T, num, den;
  double m2 = 0.0;
  bool valid = true;
  if (e >= kNEnt) {
    kind = 4; fam = famB; T = e - kNEnt; num = 0; den = T;
    valid = T != 0;
    if (T == 4) m2 = C.mc2;
    if (T == 5) m2 = C.mb2;
  } else if (e < 8) {
    kind = 0; T = e; num = e; den = e;
  } else {
    kind = e < 40 ? 1 : 3;
    int r = e - (kind == 1 ? 8 : 40);
    fam = r / 8; T = r % 8;
    num = den = 0;
    if (fam == famC) {
      valid = (kind == 1 && T == 0);
    } else {
      if (T == 0 || (kind == 3 && fam == famA)) valid = false;
      if (fam == famA) { num = T; den = T; }
      if (fam == famB) { num = 0; den = T; }
      if (fam == famD) { num = T; den = 0; }
      if (fam == famA || fam == famB) {
        if (T == 4) m2 = C.mc2;
        if (T == 5) m2 = C.mb2;
      }
    }
  }
  if (!valid) { bound[e * kNB + bin] = 0.0; return; }
  const int nx = C.nx, nq = C.nq;
  const double dle = -kLnEta0 / kNB;
  double vrow[64];
  double best = 0.0;
  for (int p = 0; p < 3; ++p) {
    double eta = exp(kLnEta0 + (bin + 0.5 * p) * dle);
    if (!(eta < 1.0)) continue;
    double fx = (log(eta) - C.lnx0) / C.dlnx;
    int i0 = (int)fx;
    if (i0 > nx - 2) i0 = nx - 2;
    for (int j = 0; j < nq; ++j) {
      double d = xf_on_row(C, den, j, eta) / eta;
      vrow[j] = -1.0;
      if (!(d > 0.0)) continue;
      const float* F = C.pdf + ((size_t)num * nq + j) * nx;
      double m = 0.0;
      for (int i = i0; i <= nx - 2; ++i) {
        double xlo = (i == i0) ? eta : exp(C.lnx0 + i * C.dlnx);
        double xhi = exp(C.lnx0 + (i + 1) * C.dlnx);
        double flo = (i == i0) ? xf_on_row(C, num, j, eta) : (double)F[i];
        double fhi = (double)F[i + 1];
        double nc = (flo > fhi ? flo : fhi) / xlo;
        double val = nc;
        if (kind != 0) {
          int sh = kind == 1 ? 1 : 3;
          double ga = gbound(sh, fam, eta / xlo), gb = gbound(sh, fam, eta / xhi);
          double g = ga > gb ? ga : gb;
          if (kind == 4) g = g * mec_bmax_range(eta / xhi, eta / xlo);
          val = g * nc;
        }
        if (val > m) m = val;
      }
      vrow[j] = m / d;
    }
    double tmin = m2 > 0.0 ? m2 + C.t_cut : C.tc_is;
    for (int j = 0; j + 1 < nq; ++j) {
      double qhi = exp(C.lnq0 + (j + 1) * C.dlnq);
      if (qhi < tmin) continue;
      double a = vrow[j], b = vrow[j + 1];
      double m = a > b ? a : b;
      if (m < 0.0) continue;
      if (m2 > 0.0) m *= (qhi - m2) / qhi;
      if (m > best) best = m;
    }
  }
  bound[e * kNB + bin] = quarter_octave_up(1.5 * best);
}

// ---------------------------------------------------------------------------
// Hard events (appendix C; e+e- and LO from the workload definitions)
__device__ double cos_1pc2(double u) {
  double q = 4.0 - 8.0 * u;
  double sd = sqrt(0.25 * q * q + 1.0);
  return cbrt(-0.5 * q + sd) + cbrt(-0.5 * q - sd);
}

__device__ double zcoup(const Cfg& C, int f) {
  int a = f < 0 ? -f : f;
  double V, A;
  if (a % 2 == 0) { V = 0.5 - 4.0 / 3.0 * C.sw2; A = 0.5; }
  else { V = -0.5 + 2.0 / 3.0 * C.sw2; A = -0.5; }
  return V * V + A * A;
}

__device__ double lo_lumi(const Cfg& C, double m, double y, double* csub) {
  double m2 = m * m;
  double e1 = m / C.sqrt_s * exp(y), e2 = m / C.sqrt_s * exp(-y);
  double L = 0.0;
  for (int f = 1; f <= C.nf; ++f) {
    double v = zcoup(C, f);
    double a = v * pdf_xf(C, pdf_tab(f), e1, m2) * pdf_xf(C, pdf_tab(-f), e2, m2);
    double b = v * pdf_xf(C, pdf_tab(-f), e1, m2) * pdf_xf(C, pdf_tab(f), e2, m2);
    if (csub) { csub[2 * (f - 1)] = a; csub[2 * (f - 1) + 1] = b; }
    L += a + b;
  }
  return L;
}

// q qbar -> Z/photon -> e- e+ at s = m2 for quark flavour f: the coefficients
// of (1 + cos^2 theta) and of 2 cos theta, theta between the incoming quark
// and the electron in the pair's rest frame (couplings v = T3 - 2 Q sin^2,
// a = T3; chi = s / (s - mZ^2 + i mZ GZ) / (4 sin^2 cos^2))
__device__ void dy_f12(const Cfg& C, int f, double m2, double& F1, double& F2) {
  const double sw2 = C.sw2, mg = C.mz * C.gz;
  const int a = f < 0 ? -f : f;
  const bool up = a % 2 == 0;
  const double Qq = up ? 2.0 / 3.0 : -1.0 / 3.0, Qe = -1.0;
  const double vq = up ? 0.5 - 4.0 / 3.0 * sw2 : -0.5 + 2.0 / 3.0 * sw2, aq = up ? 0.5 : -0.5;
  const double ve = -0.5 + 2.0 * sw2, ae = -0.5;
  const double kap = 1.0 / (4.0 * sw2 * (1.0 - sw2));
  const double d = m2 - C.mz2, D = d * d + mg * mg;
  const double rechi = kap * m2 * d / D, chi2 = kap * kap * m2 * m2 / D;
  F1 = Qq * Qq * Qe * Qe + 2.0 * Qq * Qe * vq * ve * rechi + (vq * vq + aq * aq) * (ve * ve + ae * ae) * chi2;
  F2 = 2.0 * Qq * Qe * aq * ae * rechi + 4.0 * vq * aq * ve * ae * chi2;
}

// the Z/photon weight of (m, y) per q qbar orientation: luminosity times
// F1 ((m^2 - mZ^2)^2 + mZ^2 GZ^2) / m^4 (d sigma / dm^2 dy over the
// Breit-Wigner the masses are drawn from)
__device__ double dy_lumi(const Cfg& C, double m, double y, double* csub) {
  double m2 = m * m;
  double e1 = m / C.sqrt_s * exp(y), e2 = m / C.sqrt_s * exp(-y);
  const double d = m2 - C.mz2, mg = C.mz * C.gz;
  const double bw = (d * d + mg * mg) / (m2 * m2);
  double L = 0.0;
  for (int f = 1; f <= C.nf; ++f) {
    double F1, F2;
    dy_f12(C, f, m2, F1, F2);
    const double g = F1 * bw;
    double a = g * pdf_xf(C, pdf_tab(f), e1, m2) * pdf_xf(C, pdf_tab(-f), e2, m2);
    double b = g * pdf_xf(C, pdf_tab(-f), e1, m2) * pdf_xf(C, pdf_tab(f), e2, m2);
    if (csub) { csub[2 * (f - 1)] = a; csub[2 * (f - 1) + 1] = b; }
    L += a + b;
  }
  return L;
}

__global__ void k_lo_scan(Cfg C, double* w) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 64 * 128) return;
  int i = t / 128, j = t % 128;
  double m = C.mll_min + (C.mll_max - C.mll_min) * i / 63.0;
  double Y = log(C.sqrt_s / m);
  double y = -Y + 2.0 * Y * (j + 0.5) / 128.0;
  w[t] = (C.process == 3 ? dy_lumi(C, m, y, nullptr) : lo_lumi(C, m, y, nullptr)) * 2.0 * Y;
}

__global__ void k_lo_max(const double* w, int n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double best = 0.0;
  for (int k = 0; k < n; ++k) best = w[k] > best ? w[k] : best;
  *out = quarter_octave_up(1.25 * best);
}

struct HardOut {
  const gaps_events* o;
  int64_t e;
  __device__ void put(int slot, const double* p, int pid, int col, int acol, int st) const {
    int64_t k = (int64_t)slot * o->cap + e;
    o->E[k] = p[0]; o->px[k] = p[1]; o->py[k] = p[2]; o->pz[k] = p[3];
    o->pid[k] = pid; o->col[k] = col; o->acol[k] = acol; o->status[k] = (int8_t)st;
  }
};

// the pair of mass m and momentum pZ decays to e- e+, the electron at polar
// cosine c (about +z) and azimuth 2 pi uphi in the pair's rest frame
__device__ void decay_zc(const double* pZ, double m, double c, double uphi, double* em, double* ep) {
  double st = sqrt(fmax(0.0, 1.0 - c * c)), ph = 2.0 * kPi * uphi;
  double k[4] = {0.5 * m, 0.5 * m * st * cos(ph), 0.5 * m * st * sin(ph), 0.5 * m * c};
  double pk = pZ[1] * k[1] + pZ[2] * k[2] + pZ[3] * k[3];
  double E1 = (pZ[0] * k[0] + pk) / m;
  double f = (k[0] + E1) / (pZ[0] + m);
  em[0] = E1;
  for (int q = 1; q < 4; ++q) em[q] = k[q] + f * pZ[q];
  for (int q = 0; q < 4; ++q) ep[q] = pZ[q] - em[q];
}

// Z -> e- e+ with 1 + cos^2 in the Z rest frame
__device__ void decay_z(const double* pZ, double m, double ucos, double uphi, double* em, double* ep) {
  decay_zc(pZ, m, cos_1pc2(ucos), uphi, em, ep);
}

__device__ double li2(double x) {
  // power series on [0, 1/2]; reflections elsewhere
  double sign = 1.0, add = 0.0;
  if (x == 1.0) return kPi * kPi / 6.0;
  if (x < 0.0) {
    double l = log(1.0 - x);
    add = -0.5 * l * l;
    sign = -1.0;
    x = x / (x - 1.0);
  }
  double base = 0.0, s2 = 1.0;
  if (x > 0.5) {
    base = kPi * kPi / 6.0 - log(x) * log(1.0 - x);
    s2 = -1.0;
    x = 1.0 - x;
  }
  double sum = 0.0, xk = x;
  for (int k = 1; k < 200; ++k) {
    double term = xk / ((double)k * (double)k);
    sum += term;
    if (term < 1e-18 * sum) break;
    xk *= x;
  }
  return sign * (base + s2 * sum) + add;
}

__device__ double mborn2(const Cfg& C, int f) {
  return 1.0 / kNC * 0.25 * sqrt(2.0) * C.gf * C.mz2 * C.mz2 * zcoup(C, f);
}

// collinear insertion (K + P at muF = mZ) for a leg with Born parton b at eta;
// rq, rg get the leg's PDF ratios at eta / x (quark, gluon), 0 without a Born PDF
__device__ double k_leg(const Cfg& C, int b, double eta, double x, double q2, double& rq, double& rg) {
  rq = rg = 0.0;
  double den = pdf_f(C, pdf_tab(b), eta, q2);
  if (!(den > 0.0)) return 0.0;
  rq = pdf_f(C, pdf_tab(b), eta / x, q2) / (x * den);
  rg = pdf_f(C, 0, eta / x, q2) / (x * den);
  double pq = kCF * C.alphas_mz / (2.0 * kPi), pg = kTR * C.alphas_mz / (2.0 * kPi);
  double A = pq * (-5.0 + 2.0 * kPi * kPi / 3.0);
  double l = log(1.0 - eta);
  double B = pq * 2.0 * (kPi * kPi / 6.0 - l * l - li2(1.0 - eta));
  double L = log((1.0 - x) / x) + log(1.0 - x);
  double g = pq * (2.0 / (1.0 - x)) * L;
  double h = pq * (-(1.0 + x) * L + (1.0 - x));
  double hg = pg * (2.0 * x * (1.0 - x) + (x * x + (1.0 - x) * (1.0 - x)) * L);
  return A - B + (1.0 - eta) * ((rq - 1.0) * g + rq * h + rg * hg);
}

// One leg's radiation integral at fixed Born kinematics (matching 1 and 2),
// one point (x of the collinear term, v uniform on [0, 1 - x]) relative to the
// Born, from the leg's PDF ratios rq, rg at eta / x.  The real configurations
// that the initial-initial map with this leg as emitter sends onto the Born
// have the measure m^2 / (16 pi^2 |M_B|^2) dx dv per unit Born.  Matching 1:
// minus the leg's dipoles (q -> q g, and g -> q qbar for the gluon-initiated
// configuration) where kT^2 = v (1 - x - v) m^2 / x >= mu_q2.  Matching 2:
// R - S mapped by this leg, the q qbar -> Z g part in the share
// (1 - x - v) / (1 - x) of this leg's dipole in the dipole sum.
__device__ double leg_rad(const Cfg& C, double eta, double x, double v, double rq, double rg) {
  const double omx = 1.0 - x;
  const double aq = kCF * C.alphas_mz / (2.0 * kPi), ag = kTR * C.alphas_mz / (2.0 * kPi);
  double g;
  if (C.matching == 1) {
    if (!(v * (omx - v) * C.mz2 / x >= C.mu_q2)) return 0.0;
    g = -(aq * (1.0 + x * x) / (omx * v) * rq + ag * (x * x + omx * omx) / v * rg);
  } else {
    g = -2.0 * aq * (omx - v) / omx * rq + ag * (2.0 * x + v) * rg;
  }
  return (1.0 - eta) * omx * g;
}

// The dipole sum of a real configuration (appendix C.2) at x = m^2 / sbar and
// va = -ubar / sbar (the emitted parton against beam A), over
// 8 pi alpha_s |M_B|^2 / m^2 and the colour factor: both q -> q g dipoles of
// q qbar -> Z g (kind 0), the gluon's g -> q qbar dipole for the gluon at A
// (kind 1) or at B (kind 2).
__device__ __forceinline__ double dipole_sum(int kind, double x, double va) {
  const double vb = 1.0 - x - va;
  if (kind == 0) return (1.0 + x * x) / (va * vb);
  return (x * x + (1.0 - x) * (1.0 - x)) / (kind == 1 ? va : vb);
}

// ---------------------------------------------------------------------------
// NLO pp -> Z/photon -> e- e+ (process 4): MC@NLO S and H events with the power
// shower.  Born q(p_q) qbar -> e-(p3) e+(p4) at s = m^2, in units common to S
// and H events: (a u^2 + b t^2) / s^2 with t = (p_q - p3)^2, u = (p_q - p4)^2,
// a = |A_LL|^2 + |A_RR|^2, b = |A_LR|^2 + |A_RL|^2 from the helicity
// amplitudes A_ij = Q_q Q_e + g_i^q g_j^e s / (s - mZ^2 + i mZ GZ) /
// (sin^2 cos^2) (chiral couplings g_L = T3 - Q sin^2, g_R = -Q sin^2).  The
// real emission by the Kleiss trick: g^2 C_F (a (u^2 + u'^2) + b (t^2 + t'^2))
// / (2 s' (p_q.k)(p_qbar.k)), t' = (p_qbar - p4)^2, u' = (p_qbar - p3)^2,
// s' = m^2; the gluon-initiated channels by crossing, times -3/8.  The
// subtraction: the initial-initial dipoles with the Born at the mapped
// momenta (appendix B.5's map run backwards).  PDFs at mu_F^2 = m^2.
struct DyHel {
  double al, be;
};

__device__ DyHel dy_hel(const Cfg& C, int f, double m2) {
  const bool up = (f < 0 ? -f : f) % 2 == 0;
  const double Qq = up ? 2.0 / 3.0 : -1.0 / 3.0, T3 = up ? 0.5 : -0.5, Qe = -1.0, T3e = -0.5;
  const double mg = C.mz * C.gz, d = m2 - C.mz2, D = d * d + mg * mg, k = 1.0 / (C.sw2 * (1.0 - C.sw2));
  const double rex = k * m2 * d / D, imx = -k * m2 * mg / D;
  const double gq[2] = {T3 - Qq * C.sw2, -Qq * C.sw2}, ge[2] = {T3e - Qe * C.sw2, -Qe * C.sw2};
  double A2[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const double re = Qq * Qe + gq[i] * ge[j] * rex, im = gq[i] * ge[j] * imx;
      A2[i][j] = re * re + im * im;
    }
  return DyHel{A2[0][0] + A2[1][1], A2[0][1] + A2[1][0]};
}

__device__ __forceinline__ double dy_born(const DyHel& h, const double* pq, const double* p3, const double* p4) {
  const double t = -2.0 * dot4(pq, p3), u = -2.0 * dot4(pq, p4), s = 2.0 * dot4(p3, p4);
  return (h.al * u * u + h.be * t * t) / (s * s);
}

// the Kleiss-trick real matrix element over g^2 C_F (crossed momenta allowed)
__device__ __forceinline__ double dy_kleiss(const DyHel& h, const double* pq, const double* pqb, const double* k,
                                            const double* p3, const double* p4) {
  const double t = -2.0 * dot4(pq, p3), u = -2.0 * dot4(pq, p4);
  const double tp = -2.0 * dot4(pqb, p4), up = -2.0 * dot4(pqb, p3);
  const double sp = 2.0 * dot4(p3, p4);
  return (h.al * (u * u + up * up) + h.be * (t * t + tp * tp)) / (2.0 * sp * dot4(pq, k) * dot4(pqb, k));
}

// the dipole sum over 8 pi alpha_s: beams A, B of flavours fa, fb (21: gluon),
// emitted k, leptons p3, p4; each dipole's Born at x p_e, p_s and the leptons
// under the map of p_a + p_b - k onto x p_e + p_s
__device__ double dy_dipoles(int fa, int fb, const double* A, const double* B, const double* k, const double* p3,
                             const double* p4, double x, const DyHel& h) {
  double sum = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int fe = side == 0 ? fa : fb, fs = side == 0 ? fb : fa;
    if (fs == 21) continue;
    const double* pe = side == 0 ? A : B;
    const double* ps = side == 0 ? B : A;
    double K[4], Kt[4], q3[4], q4[4], pem[4];
    for (int m = 0; m < 4; ++m) {
      K[m] = pe[m] + ps[m] - k[m];
      Kt[m] = x * pe[m] + ps[m];
      q3[m] = p3[m];
      q4[m] = p4[m];
      pem[m] = x * pe[m];
    }
    ii_lambda(K, Kt, q3);
    ii_lambda(K, Kt, q4);
    const int qe = fe == 21 ? -fs : fe;  // the Born's flavour at the emitter
    const double Bn = dy_born(h, qe > 0 ? pem : ps, q3, q4);
    const double V = fe == 21 ? kTR * (1.0 - 2.0 * x * (1.0 - x)) : kCF * (1.0 + x * x) / (1.0 - x);
    sum += V / (x * 2.0 * dot4(pe, k)) * Bn;
  }
  return sum;
}

// colour tags of an NLO H event's beams and emitted parton (kind 0: q qbar ->
// V g; kind 1: gluon at A; kind 2: gluon at B)
__device__ void h_colours(int kind, int a, int b, int& ca, int& aa, int& cb, int& ab, int& jp, int& cj, int& aj) {
  if (kind == 0) {
    ca = a > 0 ? 1 : 0; aa = a > 0 ? 0 : 2;
    cb = b > 0 ? 1 : 0; ab = b > 0 ? 0 : 2;
    jp = 21; cj = 1; aj = 2;
    return;
  }
  const int qk = kind == 1 ? b : a;
  int cq, aq;
  if (qk > 0) { cq = 2; aq = 0; cj = 1; aj = 0; }
  else { cq = 0; aq = 1; cj = 0; aj = 2; }
  jp = qk;
  if (kind == 1) { ca = 1; aa = 2; cb = cq; ab = aq; }
  else { ca = cq; aa = aq; cb = 1; ab = 2; }
}

// one process-4 event: blocks (id, 0) S/H, channel, rapidity, lepton polar
// cosine; (id, 1) x_a, x_b (S) or x, v (H), emission azimuth, lepton azimuth;
// (id, 2) the pair mass on the window's Breit-Wigner
__device__ void hard_dy_nlo(const Cfg& C, int64_t id, uint64_t seed, const HardOut& H, gaps_events& o, int64_t e) {
  const uint32_t SH = 2u;
  double u0[4], u1[4], u2[4];
  rng4(seed, SH, id, 0u, 0u, u0);
  rng4(seed, SH, id, 1u, 0u, u1);
  rng4(seed, SH, id, 2u, 0u, u2);
  const double mg = C.mz * C.gz;
  const double r1 = atan((C.mll_min * C.mll_min - C.mz2) / mg), r2 = atan((C.mll_max * C.mll_max - C.mz2) / mg);
  const double m2 = C.mz2 + mg * tan(r1 + u2[0] * (r2 - r1)), m = sqrt(m2), q2 = m2;
  const double jm = (r2 - r1) * ((m2 - C.mz2) * (m2 - C.mz2) + mg * mg) / mg;
  const double c = 2.0 * u0[3] - 1.0;
  const int nf = C.nf;
  const double g2 = 4.0 * kPi * C.alphas_mz;
  if (u0[0] < C.p_s) {
    const double Y = log(C.sqrt_s / m), y = -Y + 2.0 * Y * u0[2];
    const double e1 = m / C.sqrt_s * exp(y), e2 = m / C.sqrt_s * exp(-y);
    const double xa = e1 + (1.0 - e1) * u1[0], xb = e2 + (1.0 - e2) * u1[1];
    const double Ea = 0.5 * e1 * C.sqrt_s, Eb = 0.5 * e2 * C.sqrt_s;
    double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
    double pZ[4] = {A[0] + B[0], 0.0, 0.0, A[3] + B[3]}, em[4], ep[4];
    decay_zc(pZ, m, c, u1[3], em, ep);
    const double bvi = 1.0 + kCF * C.alphas_mz / (2.0 * kPi) * 2.0;
    double csub[10], W = 0.0;
    for (int f = 1; f <= nf; ++f) {
      const DyHel h = dy_hel(C, f, m2);
      for (int o2 = 0; o2 < 2; ++o2) {
        const int a = o2 == 0 ? f : -f, b = -a;
        const double M0 = dy_born(h, a > 0 ? A : B, em, ep);
        const double born = pdf_xf(C, pdf_tab(a), e1, q2) * pdf_xf(C, pdf_tab(b), e2, q2) * M0 / (16.0 * kPi * m2 * m2);
        double rq, rg;
        const double corr = bvi + k_leg(C, a, e1, xa, q2, rq, rg) + k_leg(C, b, e2, xb, q2, rq, rg);
        csub[2 * (f - 1) + o2] = born * corr;
        W += fabs(born * corr);
      }
    }
    const double target = u0[1] * W;
    double cum = 0.0;
    int sel = 2 * nf - 1;
    for (int q = 0; q < 2 * nf; ++q) {
      cum += fabs(csub[q]);
      if (target < cum) { sel = q; break; }
    }
    const int f = sel / 2 + 1, a = (sel % 2 == 0) ? f : -f, b = -a;
    H.put(0, A, a, a > 0 ? 1 : 0, a > 0 ? 0 : 1, -1);
    H.put(1, B, b, b > 0 ? 1 : 0, b > 0 ? 0 : 1, -1);
    H.put(2, em, 11, 0, 0, 1);
    H.put(3, ep, -11, 0, 0, 1);
    o.n[e] = 4;
    o.w[e] = (csub[sel] < 0.0 ? -W : W) * 2.0 * Y * jm / C.p_s;
    o.t_start[e] = C.S;
    o.flags[e] = 0u;
    return;
  }
  const double xmin = m2 / C.S;
  const double x = xmin + (1.0 - xmin) * u1[0], sbar = m2 / x;
  const double YH = 0.5 * log(C.S * x / m2), y = -YH + 2.0 * YH * u0[2];
  const double v = (1.0 - x) * u1[1], ph = 2.0 * kPi * u1[2];
  const double ea = exp(y) * sqrt(sbar / C.S), eb = exp(-y) * sqrt(sbar / C.S);
  const double Ea = 0.5 * ea * C.sqrt_s, Eb = 0.5 * eb * C.sqrt_s;
  double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb}, J[4], pZ[4], em[4], ep[4];
  double mJ[4], mA[4], mB[4];
  const double kt0 = sqrt(v * (1.0 - x - v) * sbar);
  for (int q = 0; q < 4; ++q) J[q] = (1.0 - x - v) * A[q] + v * B[q];
  J[1] -= kt0 * cos(ph);
  J[2] -= kt0 * sin(ph);
  for (int q = 0; q < 4; ++q) {
    pZ[q] = A[q] + B[q] - J[q];
    mJ[q] = -J[q]; mA[q] = -A[q]; mB[q] = -B[q];
  }
  decay_zc(pZ, m, c, u1[3], em, ep);
  double csub[30], W = 0.0;
  int pa[30], pb[30], kind[30];
  int q = 0;
  const double as8 = 8.0 * kPi * C.alphas_mz;
  for (int f = 1; f <= nf; ++f) {
    const DyHel h = dy_hel(C, f, m2);
    for (int kd = 0; kd < 3; ++kd)
      for (int o2 = 0; o2 < 2; ++o2) {
        int fa, fb;
        double R;
        if (kd == 0) {
          fa = o2 == 0 ? f : -f; fb = -fa;
          R = g2 * kCF * dy_kleiss(h, fa > 0 ? A : B, fa > 0 ? B : A, J, em, ep);
        } else if (kd == 1) {
          fa = 21; fb = o2 == 0 ? f : -f;
          R = -0.375 * g2 * kCF * (fb > 0 ? dy_kleiss(h, B, mJ, mA, em, ep) : dy_kleiss(h, mJ, B, mA, em, ep));
        } else {
          fa = o2 == 0 ? f : -f; fb = 21;
          R = -0.375 * g2 * kCF * (fa > 0 ? dy_kleiss(h, A, mJ, mB, em, ep) : dy_kleiss(h, mJ, A, mB, em, ep));
        }
        const double S = as8 * dy_dipoles(fa, fb, A, B, J, em, ep, x, h);
        pa[q] = fa; pb[q] = fb; kind[q] = kd; csub[q++] = R - S;
      }
  }
  for (int k = 0; k < q; ++k) {
    csub[k] *= pdf_xf(C, pdf_tab(pa[k]), ea, q2) * pdf_xf(C, pdf_tab(pb[k]), eb, q2) / (16.0 * kPi * m2) /
               (16.0 * kPi * kPi);
    W += fabs(csub[k]);
  }
  const double target = u0[1] * W;
  double cum = 0.0;
  int sel = q - 1;
  for (int k = 0; k < q; ++k) {
    cum += fabs(csub[k]);
    if (target < cum) { sel = k; break; }
  }
  const int a = pa[sel], b = pb[sel];
  int ca, aa, cb, ab, jp, cj, aj;
  h_colours(kind[sel], a, b, ca, aa, cb, ab, jp, cj, aj);
  H.put(0, A, a, ca, aa, -1);
  H.put(1, B, b, cb, ab, -1);
  H.put(2, J, jp, cj, aj, 1);
  H.put(3, em, 11, 0, 0, 1);
  H.put(4, ep, -11, 0, 0, 1);
  o.n[e] = 5;
  o.w[e] = (csub[sel] < 0.0 ? -W : W) * 2.0 * YH * (1.0 - xmin) * (1.0 - x) * jm / (1.0 - C.p_s);
  o.t_start[e] = C.S;
  o.flags[e] = fHEvent;
}

__global__ void k_hard(Cfg C, int64_t first_id, int64_t n, uint64_t seed, gaps_events o) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint32_t SH = 2u;  // stream of the hard process
  int64_t id = first_id + e;
  o.id[e] = id;
  if (o.n_cycles) o.n_cycles[e] = 0;
  if (o.n_trials) o.n_trials[e] = 0;
  if (o.n_accept) o.n_accept[e] = 0;
  if (o.n_viol) o.n_viol[e] = 0;
  if (o.t1) o.t1[e] = 0.0;
  HardOut H{&o, e};
  if (C.process == 0) {
    double u[4];
    rng4(seed, SH, id, 0u, 0u, u);
    int f = 1 + (int)(u[0] * C.nf);
    if (f > C.nf) f = C.nf;
    double c = cos_1pc2(u[1]), st = sqrt(fmax(0.0, 1.0 - c * c)), ph = 2.0 * kPi * u[2];
    double E = 0.5 * C.sqrt_s;
    double q[4] = {E, E * st * cos(ph), E * st * sin(ph), E * c};
    double qb[4] = {E, -q[1], -q[2], -q[3]};
    H.put(0, q, f, 1, 0, 1);
    H.put(1, qb, -f, 0, 1, 1);
    o.n[e] = 2; o.w[e] = 1.0; o.t_start[e] = C.S; o.flags[e] = 0u;
    return;
  }
  if (C.process == 1) {
    double mg = C.mz * C.gz;
    double r1 = atan((C.mll_min * C.mll_min - C.mz2) / mg);
    double r2 = atan((C.mll_max * C.mll_max - C.mz2) / mg);
    double csub[10];
    for (int k = 0; k < 1000; ++k) {
      double u[4];
      rng4(seed, SH, id, (uint32_t)k, 0u, u);
      double m2 = C.mz2 + mg * tan(r1 + u[0] * (r2 - r1));
      double m = sqrt(m2);
      double Y = log(C.sqrt_s / m), y = -Y + 2.0 * Y * u[1];
      double L = lo_lumi(C, m, y, csub);
      if (!(u[2] * C.lo_wmax < L * 2.0 * Y)) continue;
      double target = u[3] * L, cum = 0.0;
      int sel = 2 * C.nf - 1;
      for (int q = 0; q < 2 * C.nf; ++q) {
        cum += csub[q];
        if (target < cum) { sel = q; break; }
      }
      int f = sel / 2 + 1;
      int pa = (sel % 2 == 0) ? f : -f, pb = -pa;
      double e1 = m / C.sqrt_s * exp(y), e2 = m / C.sqrt_s * exp(-y);
      double Ea = 0.5 * e1 * C.sqrt_s, Eb = 0.5 * e2 * C.sqrt_s;
      double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
      H.put(0, A, pa, pa > 0 ? 1 : 0, pa > 0 ? 0 : 1, -1);
      H.put(1, B, pb, pb > 0 ? 1 : 0, pb > 0 ? 0 : 1, -1);
      double pZ[4] = {A[0] + B[0], 0.0, 0.0, A[3] + B[3]}, em[4], ep[4], ud[4];
      rng4(seed, SH, id, 0xFFFFFFFFu, 0u, ud);
      decay_z(pZ, m, ud[0], ud[1], em, ep);
      H.put(2, em, 11, 0, 0, 1);
      H.put(3, ep, -11, 0, 0, 1);
      o.n[e] = 4; o.w[e] = 1.0;
      o.t_start[e] = C.matching == 1 ? C.mu_q2 : C.S;
      o.flags[e] = C.matching == 2 ? fMEC : 0u;
      return;
    }
    o.n[e] = 0; o.w[e] = 0.0; o.t_start[e] = C.S; o.flags[e] = fHardFail;
    return;
  }
  if (C.process == 3) {
    // LO Z/photon with interference: (m, y) and the orientation as for the Z
    // alone with the Z/photon weight, then cos(theta) between the quark and
    // the electron by accept-reject on (1 + c^2) F1 + 2 c F2 from proposals
    // distributed as 1 + c^2 (block (id, 2^32 - 1, j) of attempt j)
    double mg = C.mz * C.gz;
    double r1 = atan((C.mll_min * C.mll_min - C.mz2) / mg);
    double r2 = atan((C.mll_max * C.mll_max - C.mz2) / mg);
    double csub[10];
    for (int k = 0; k < 1000; ++k) {
      double u[4];
      rng4(seed, SH, id, (uint32_t)k, 0u, u);
      double m2 = C.mz2 + mg * tan(r1 + u[0] * (r2 - r1));
      double m = sqrt(m2);
      double Y = log(C.sqrt_s / m), y = -Y + 2.0 * Y * u[1];
      double L = dy_lumi(C, m, y, csub);
      if (!(u[2] * C.lo_wmax < L * 2.0 * Y)) continue;
      double target = u[3] * L, cum = 0.0;
      int sel = 2 * C.nf - 1;
      for (int q = 0; q < 2 * C.nf; ++q) {
        cum += csub[q];
        if (target < cum) { sel = q; break; }
      }
      int f = sel / 2 + 1;
      int pa = (sel % 2 == 0) ? f : -f, pb = -pa;
      double e1 = m / C.sqrt_s * exp(y), e2 = m / C.sqrt_s * exp(-y);
      double Ea = 0.5 * e1 * C.sqrt_s, Eb = 0.5 * e2 * C.sqrt_s;
      double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
      double pZ[4] = {A[0] + B[0], 0.0, 0.0, A[3] + B[3]}, em[4], ep[4];
      double F1, F2;
      dy_f12(C, f, m2, F1, F2);
      const double sq = pa > 0 ? 1.0 : -1.0;  // the quark moves along +z when beam A carries it
      for (int j = 0; j < 1000; ++j) {
        double ud[4];
        rng4(seed, SH, id, 0xFFFFFFFFu, (uint32_t)j, ud);
        const double c = cos_1pc2(ud[0]);
        const double acc = ((1.0 + c * c) * F1 + 2.0 * c * F2) / ((1.0 + c * c) * (F1 + fabs(F2)));
        if (!(ud[1] < acc)) continue;
        H.put(0, A, pa, pa > 0 ? 1 : 0, pa > 0 ? 0 : 1, -1);
        H.put(1, B, pb, pb > 0 ? 1 : 0, pb > 0 ? 0 : 1, -1);
        decay_zc(pZ, m, sq * c, ud[2], em, ep);
        H.put(2, em, 11, 0, 0, 1);
        H.put(3, ep, -11, 0, 0, 1);
        o.n[e] = 4; o.w[e] = 1.0; o.t_start[e] = C.S; o.flags[e] = 0u;
        return;
      }
      break;
    }
    o.n[e] = 0; o.w[e] = 0.0; o.t_start[e] = C.S; o.flags[e] = fHardFail;
    return;
  }
  if (C.process == 4) {
    hard_dy_nlo(C, id, seed, H, o, e);
    return;
  }
  // NLO S and H events
  double u0[4], u1[4];
  rng4(seed, SH, id, 0u, 0u, u0);
  rng4(seed, SH, id, 1u, 0u, u1);
  const double m = C.mz, m2 = C.mz2, q2 = m2;
  const int nf = C.nf;
  const int mt = C.matching;
  if (mt == 2 || u0[0] < C.p_s) {
    // S event (matching 2: every event, as a Born event with the radiation integral)
    double Y = log(C.sqrt_s / m), y = -Y + 2.0 * Y * u0[2];
    double e1 = m / C.sqrt_s * exp(y), e2 = m / C.sqrt_s * exp(-y);
    double xa = e1 + (1.0 - e1) * u1[0], xb = e2 + (1.0 - e2) * u1[1];
    double va = 0.0, vb = 0.0;
    if (mt != 0) {
      double u2[4];
      rng4(seed, SH, id, 2u, 0u, u2);
      va = (1.0 - xa) * u1[2];
      vb = (1.0 - xb) * u2[0];
    }
    double csub[10], W = 0.0;
    double bvi = 1.0 + kCF * C.alphas_mz / (2.0 * kPi) * 2.0;
    for (int f = 1; f <= nf; ++f)
      for (int o2 = 0; o2 < 2; ++o2) {
        int a = o2 == 0 ? f : -f, b = -a;
        double born = kPi / (m2 * m2) * mborn2(C, f) * pdf_xf(C, pdf_tab(a), e1, q2) * pdf_xf(C, pdf_tab(b), e2, q2);
        double rqa, rga, rqb, rgb;
        double corr = bvi + k_leg(C, a, e1, xa, q2, rqa, rga) + k_leg(C, b, e2, xb, q2, rqb, rgb);
        if (mt != 0) corr += leg_rad(C, e1, xa, va, rqa, rga) + leg_rad(C, e2, xb, vb, rqb, rgb);
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
    double Ea = 0.5 * e1 * C.sqrt_s, Eb = 0.5 * e2 * C.sqrt_s;
    double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
    H.put(0, A, a, a > 0 ? 1 : 0, a > 0 ? 0 : 1, -1);
    H.put(1, B, b, b > 0 ? 1 : 0, b > 0 ? 0 : 1, -1);
    double pZ[4] = {A[0] + B[0], 0.0, 0.0, A[3] + B[3]}, em[4], ep[4];
    decay_z(pZ, m, u0[3], u1[3], em, ep);
    H.put(2, em, 11, 0, 0, 1);
    H.put(3, ep, -11, 0, 0, 1);
    o.n[e] = 4;
    o.w[e] = (csub[sel] < 0.0 ? -W : W) * 2.0 * Y / (mt == 2 ? 1.0 : C.p_s);
    o.t_start[e] = mt == 1 ? C.mu_q2 : C.S;
    o.flags[e] = mt == 2 ? fMEC : 0u;
    return;
  }
  double xmin = m2 / C.S;
  double x = xmin + (1.0 - xmin) * u1[0], sbar = m2 / x;
  double YH = 0.5 * log(C.S * x / m2), y = -YH + 2.0 * YH * u0[2];
  double ea = exp(y) * sqrt(sbar / C.S), eb = exp(-y) * sqrt(sbar / C.S);
  double v = (1.0 - x) * u1[1], ph = 2.0 * kPi * u1[2];
  double Ea = 0.5 * ea * C.sqrt_s, Eb = 0.5 * eb * C.sqrt_s;
  double A[4] = {Ea, 0.0, 0.0, Ea}, B[4] = {Eb, 0.0, 0.0, -Eb};
  double kt0 = sqrt(v * (1.0 - x - v) * sbar);
  double J[4];
  for (int q = 0; q < 4; ++q) J[q] = (1.0 - x - v) * A[q] + v * B[q];
  J[1] -= kt0 * cos(ph);
  J[2] -= kt0 * sin(ph);
  double pZ[4];
  for (int q = 0; q < 4; ++q) pZ[q] = A[q] + B[q] - J[q];
  double ubar = -2.0 * (A[0] * J[0] - A[1] * J[1] - A[2] * J[2] - A[3] * J[3]);
  double tbar = -2.0 * (B[0] * J[0] - B[1] * J[1] - B[2] * J[2] - B[3] * J[3]);
  double csub[30], W = 0.0;
  int pa[30], pb[30], kind[30];
  int q = 0;
  double pre_q = 8.0 * kPi * C.alphas_mz * kCF / m2, pre_g = 8.0 * kPi * C.alphas_mz * kTR / m2;
  // matching 1: above mu_q2 the S events' shower subtracts nothing, so the H
  // events keep the dipole sum there (their weight is R)
  const bool above = mt == 1 && v * (1.0 - x - v) * sbar >= C.mu_q2;
  for (int f = 1; f <= nf; ++f) {
    double mb = mborn2(C, f);
    double rs = pre_q * mb * (-2.0);
    if (above) rs += pre_q * mb * dipole_sum(0, x, v);
    pa[q] = f; pb[q] = -f; kind[q] = 0; csub[q++] = rs;
    pa[q] = -f; pb[q] = f; kind[q] = 0; csub[q++] = rs;
    rs = pre_g * mb * ((2.0 * m2 - ubar) / sbar);
    if (above) rs += pre_g * mb * dipole_sum(1, x, v);
    pa[q] = 21; pb[q] = f; kind[q] = 1; csub[q++] = rs;
    pa[q] = 21; pb[q] = -f; kind[q] = 1; csub[q++] = rs;
    rs = pre_g * mb * ((2.0 * m2 - tbar) / sbar);
    if (above) rs += pre_g * mb * dipole_sum(2, x, v);
    pa[q] = f; pb[q] = 21; kind[q] = 2; csub[q++] = rs;
    pa[q] = -f; pb[q] = 21; kind[q] = 2; csub[q++] = rs;
  }
  for (int k = 0; k < q; ++k) {
    csub[k] *= pdf_xf(C, pdf_tab(pa[k]), ea, q2) * pdf_xf(C, pdf_tab(pb[k]), eb, q2) / (16.0 * kPi * m2);
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
  H.put(0, A, a, ca, aa, -1);
  H.put(1, B, b, cb, ab, -1);
  H.put(2, J, jp, cj, aj, 1);
  double em[4], ep[4];
  decay_z(pZ, m, u0[3], u1[3], em, ep);
  H.put(3, em, 11, 0, 0, 1);
  H.put(4, ep, -11, 0, 0, 1);
  o.n[e] = 5;
  o.w[e] = (csub[sel] < 0.0 ? -W : W) * 2.0 * YH * (1.0 - xmin) * (1.0 - x) / (1.0 - C.p_s);
  o.t_start[e] = mt == 1 ? C.mu_q2 : C.S;
  o.flags[e] = fHEvent;
}

}  // namespace gaps
