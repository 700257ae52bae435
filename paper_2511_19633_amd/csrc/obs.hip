// Observables and histograms (section 4.1: Z observables, anti-kT jets; thrust
// and Durham jet rates for the e+e- workload), one event per thread.
#include "kernels.hpp"

namespace gaps {

namespace {

constexpr int kObsMax = 256;
constexpr int kNObs = 12;

__device__ __forceinline__ bool is_parton(int pid) { return pid == 21 || (pid != 0 && pid <= 5 && pid >= -5); }
__device__ __forceinline__ double rapidity(const double* p) { return 0.5 * log((p[0] + p[3]) / (p[0] - p[3])); }
__device__ __forceinline__ double pseudorap(const double* p) {
  double pt = sqrt(p[1] * p[1] + p[2] * p[2]);
  return asinh(p[3] / pt);
}

// anti-kT with E-scheme recombination over q[0..n-1] (modified in place);
// jets written to jets[] sorted by pT (descending).  Each pseudojet's
// rapidity, azimuth and 1/pT^2 are computed once (and again after a merge),
// not for every pair of every step: the same values, so the same clustering.
__device__ int antikt(double (*q)[4], int n, double R, double (*jets)[4], bool* on, double* yv, double* phv,
                      double* ipv) {
  int alive = n, nj = 0;
  auto props = [&](int i) {
    yv[i] = rapidity(q[i]);
    phv[i] = atan2(q[i][2], q[i][1]);
    ipv[i] = 1.0 / (q[i][1] * q[i][1] + q[i][2] * q[i][2]);
  };
  for (int i = 0; i < n; ++i) {
    on[i] = true;
    props(i);
  }
  const double iR2 = R * R;
  while (alive > 0) {
    double best = INFINITY;
    int bi = -1, bj = -1;
    for (int i = 0; i < n; ++i) {
      if (!on[i]) continue;
      const double diB = ipv[i];
      if (diB < best) { best = diB; bi = i; bj = -1; }
      const double yi = yv[i], phii = phv[i];
      for (int j = i + 1; j < n; ++j) {
        if (!on[j]) continue;
        double dy = yi - yv[j];
        double dphi = fabs(phii - phv[j]);
        if (dphi > kPi) dphi = 2.0 * kPi - dphi;
        double dR2 = dy * dy + dphi * dphi;
        double dij = fmin(diB, ipv[j]) * dR2 / iR2;
        if (dij < best) { best = dij; bi = i; bj = j; }
      }
    }
    if (bj < 0) {
      for (int m = 0; m < 4; ++m) jets[nj][m] = q[bi][m];
      ++nj;
      on[bi] = false;
    } else {
      for (int m = 0; m < 4; ++m) q[bi][m] += q[bj][m];
      on[bj] = false;
      props(bi);
    }
    --alive;
  }
  for (int i = 1; i < nj; ++i) {
    double tmp[4] = {jets[i][0], jets[i][1], jets[i][2], jets[i][3]};
    double pti = tmp[1] * tmp[1] + tmp[2] * tmp[2];
    int j = i - 1;
    while (j >= 0 && jets[j][1] * jets[j][1] + jets[j][2] * jets[j][2] < pti) {
      for (int m = 0; m < 4; ++m) jets[j + 1][m] = jets[j][m];
      --j;
    }
    for (int m = 0; m < 4; ++m) jets[j + 1][m] = tmp[m];
  }
  return nj;
}

__device__ double thrust(double (*p)[4], int n) {
  double sum = 0.0;
  for (int i = 0; i < n; ++i) sum += sqrt(p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]);
  if (n < 2 || !(sum > 0.0)) return 1.0;
  if (n == 2) {
    double d0 = p[0][1] - p[1][1], d1 = p[0][2] - p[1][2], d2 = p[0][3] - p[1][3];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2) / sum;
  }
  double best = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double nv0 = p[i][2] * p[j][3] - p[i][3] * p[j][2];
      double nv1 = p[i][3] * p[j][1] - p[i][1] * p[j][3];
      double nv2 = p[i][1] * p[j][2] - p[i][2] * p[j][1];
      double P0 = 0.0, P1 = 0.0, P2 = 0.0;
      for (int k = 0; k < n; ++k) {
        if (k == i || k == j) continue;
        double d = p[k][1] * nv0 + p[k][2] * nv1 + p[k][3] * nv2;
        double sg = d >= 0.0 ? 1.0 : -1.0;
        P0 += sg * p[k][1]; P1 += sg * p[k][2]; P2 += sg * p[k][3];
      }
      for (int si = -1; si <= 1; si += 2)
        for (int sj = -1; sj <= 1; sj += 2) {
          double Q0 = P0 + si * p[i][1] + sj * p[j][1];
          double Q1 = P1 + si * p[i][2] + sj * p[j][2];
          double Q2 = P2 + si * p[i][3] + sj * p[j][3];
          double v = sqrt(Q0 * Q0 + Q1 * Q1 + Q2 * Q2);
          if (v > best) best = v;
        }
    }
  return best / sum;
}

__device__ void durham(double (*q)[4], int n, double* y, bool* on) {
  double Evis = 0.0;
  for (int i = 0; i < n; ++i) { on[i] = true; Evis += q[i][0]; }
  for (int k = 0; k < 4; ++k) y[k] = 0.0;
  int alive = n;
  while (alive > 1) {
    double best = INFINITY;
    int bi = -1, bj = -1;
    for (int i = 0; i < n; ++i) {
      if (!on[i]) continue;
      double ai = sqrt(q[i][1] * q[i][1] + q[i][2] * q[i][2] + q[i][3] * q[i][3]);
      for (int j = i + 1; j < n; ++j) {
        if (!on[j]) continue;
        double aj = sqrt(q[j][1] * q[j][1] + q[j][2] * q[j][2] + q[j][3] * q[j][3]);
        double c = (q[i][1] * q[j][1] + q[i][2] * q[j][2] + q[i][3] * q[j][3]) / (ai * aj);
        double emin = fmin(q[i][0], q[j][0]);
        double yij = 2.0 * emin * emin * (1.0 - c) / (Evis * Evis);
        if (yij < best) { best = yij; bi = i; bj = j; }
      }
    }
    int k = alive - 1;
    if (k >= 2 && k <= 5) y[k - 2] = best;
    for (int m = 0; m < 4; ++m) q[bi][m] += q[bj][m];
    on[bj] = false;
    --alive;
  }
}

}  // namespace

__global__ void __launch_bounds__(64) k_observables(Cfg C, gaps_events ev, int64_t n, double* obs) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  double ps[kObsMax][4];
  double jets[kObsMax][4];
  double yv[kObsMax], phv[kObsMax], ipv[kObsMax];
  bool on[kObsMax];
  double* o = obs + e * kNObs;
  for (int k = 0; k < kNObs; ++k) o[k] = 0.0;
  int np = 0, nn = ev.n[e];
  if (nn > ev.max_slots) nn = ev.max_slots;
  double lm[4] = {0, 0, 0, 0}, lp[4] = {0, 0, 0, 0}, bal[4] = {0, 0, 0, 0};
  for (int q = 0; q < nn; ++q) {
    int64_t k = (int64_t)q * ev.cap + e;
    double p[4] = {ev.E[k], ev.px[k], ev.py[k], ev.pz[k]};
    int st = ev.status[k];
    for (int m = 0; m < 4; ++m) bal[m] += st > 0 ? p[m] : -p[m];
    if (st <= 0) continue;
    int pid = ev.pid[k];
    if (pid == 11) { for (int m = 0; m < 4; ++m) lm[m] = p[m]; }
    else if (pid == -11) { for (int m = 0; m < 4; ++m) lp[m] = p[m]; }
    else if (is_parton(pid) && np < kObsMax) { for (int m = 0; m < 4; ++m) ps[np][m] = p[m]; ++np; }
  }
  if (C.process == 0) bal[0] -= C.sqrt_s;
  double imb = 0.0;
  for (int m = 0; m < 4; ++m) imb = fmax(imb, fabs(bal[m]));
  o[9] = np;
  o[10] = imb;
  if (C.process == 0) {
    o[0] = 1.0 - thrust(ps, np);
    double y[4];
    durham(ps, np, y, on);
    for (int k = 0; k < 4; ++k) o[1 + k] = y[k];
    return;
  }
  double Z[4];
  for (int m = 0; m < 4; ++m) Z[m] = lm[m] + lp[m];
  o[0] = sqrt(Z[1] * Z[1] + Z[2] * Z[2]);
  o[1] = rapidity(Z);
  o[2] = (Z[1] == 0.0 && Z[2] == 0.0) ? 0.0 : atan2(Z[2], Z[1]);
  double dphi = fabs(atan2(lm[2], lm[1]) - atan2(lp[2], lp[1]));
  if (dphi > kPi) dphi = 2.0 * kPi - dphi;
  double cth = tanh(0.5 * (pseudorap(lm) - pseudorap(lp)));
  o[3] = tan(0.5 * (kPi - dphi)) * sqrt(fmax(0.0, 1.0 - cth * cth));
  int nq = 0;
  for (int i = 0; i < np; ++i)
    if (ps[i][1] * ps[i][1] + ps[i][2] * ps[i][2] > 1e-18 * C.S) {
      for (int m = 0; m < 4; ++m) ps[nq][m] = ps[i][m];
      ++nq;
    }
  int nj = antikt(ps, nq, 0.4, jets, on, yv, phv, ipv);
  int njet = 0, n_eta = 0;
  double j1[4] = {0, 0, 0, 0}, j2[4] = {0, 0, 0, 0};
  double j1pt = 0.0, j2pt = 0.0, j1eta = 0.0;
  bool have1 = false;
  for (int k = 0; k < nj; ++k) {
    double pt = sqrt(jets[k][1] * jets[k][1] + jets[k][2] * jets[k][2]);
    double et = pseudorap(jets[k]);
    if (fabs(et) < 5.0) {
      if (n_eta == 0) j1pt = pt;
      else if (n_eta == 1) j2pt = pt;
      ++n_eta;
    }
    if (pt > 5.0 && !have1) { j1eta = et; have1 = true; }
    if (pt > 5.0 && fabs(et) < 5.0) {
      if (njet == 0) { for (int m = 0; m < 4; ++m) j1[m] = jets[k][m]; }
      else if (njet == 1) { for (int m = 0; m < 4; ++m) j2[m] = jets[k][m]; }
      ++njet;
    }
  }
  o[4] = njet;
  o[5] = j1pt;
  o[6] = j1eta;
  o[7] = j2pt;
  if (njet >= 2) {
    double dy = pseudorap(j1) - pseudorap(j2);
    double dp = fabs(atan2(j1[2], j1[1]) - atan2(j2[2], j2[1]));
    if (dp > kPi) dp = 2.0 * kPi - dp;
    o[8] = sqrt(dy * dy + dp * dp);
  } else {
    o[8] = -1.0;
  }
}

// ---------------------------------------------------------------------------
// The pp observables with one event per wave: the event's slots one per lane,
// its pseudojets in LDS, and every anti-kT step an argmin over the step's
// distances (each alive pseudojet's beam distance and its pairs), the pairs
// dealt to the lanes once for the whole kernel in triangular order and the
// minimum taken with the serial loop's order (emitter, beam before pairs,
// partner) as tie-break: the same clustering as the one-thread loop above,
// without its private arrays.  The transcendentals of the jet and Z
// observables run on several lanes at once.  For events of at most kObsW
// slots.
struct ObsWave {
  double q[kObsW][4];
  double y[kObsW], ph[kObsW];
  double ip[kObsW];  // 1/pT^2 of an alive pseudojet, -1 once it is merged or a jet
  int jet[kObsW];    // the pseudojets that became jets, in order (their q is final)
  int srt[kObsW];    // the jets by pT, descending, equal pT in order
};
namespace {
// item q of the triangle a <= b (row b holds a = 0 .. b): b the largest with
// b (b + 1) / 2 <= q, from the root of the quadratic corrected to the integer
__device__ __forceinline__ void obs_tri(int q, int& a, int& b) {
  b = (int)(0.5f * (sqrtf(8.0f * (float)q + 1.0f) - 1.0f));
  b = b < 0 ? 0 : b;
  while (b > 0 && b * (b + 1) / 2 > q) --b;
  while ((b + 1) * (b + 2) / 2 <= q) ++b;
  a = q - b * (b + 1) / 2;
}
// the serial loop's position of an item: emitter a, its beam distance (b ==
// a) before its pairs, then partner b
__device__ __forceinline__ int obs_ord(int a, int b) { return (a << 8) | (a == b ? 0 : b + 1); }
constexpr int kNoItem = 0x7fffffff;
constexpr int kObsPass = 4;  // items dealt once per lane: events of up to 22 pseudojets
}  // namespace

__global__ void __launch_bounds__(64 * kObsWaves, 4) k_observables_pp(Cfg C, gaps_events ev, int64_t n, double* obs) {
  __shared__ ObsWave sw[kObsWaves];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  ObsWave& W = sw[wid];
  const int64_t nwaves = (int64_t)gridDim.x * kObsWaves;
  // this lane's items of the first kObsPass passes (the same for every event)
  int pa[kObsPass], pb[kObsPass];
#pragma unroll
  for (int k = 0; k < kObsPass; ++k) obs_tri(lane + 64 * k, pa[k], pb[k]);
  for (int64_t e = (int64_t)blockIdx.x * kObsWaves + wid; e < n; e += nwaves) {
    int nn = ev.n[e];
    if (nn > ev.max_slots) nn = ev.max_slots;
    // ---- slots: momentum balance, leptons (the last of each sign), partons
    // and the pseudojets above the pT floor, both in slot order
    double bal[4] = {0.0, 0.0, 0.0, 0.0};
    double lm[4] = {0.0, 0.0, 0.0, 0.0}, lp[4] = {0.0, 0.0, 0.0, 0.0};
    int np = 0, nq = 0;
#pragma unroll
    for (int h = 0; h < kObsW / 64; ++h) {
      const int q = h * 64 + lane;
      double p[4] = {0.0, 0.0, 0.0, 0.0};
      int st = 0, pid = 0;
      if (q < nn) {
        const int64_t k = (int64_t)q * ev.cap + e;
        p[0] = ev.E[k]; p[1] = ev.px[k]; p[2] = ev.py[k]; p[3] = ev.pz[k];
        st = ev.status[k];
        pid = ev.pid[k];
        for (int m = 0; m < 4; ++m) bal[m] += st > 0 ? p[m] : -p[m];
      }
      const bool out = q < nn && st > 0;
      const unsigned long long mm = __ballot(out && pid == 11), mp = __ballot(out && pid == -11);
      if (mm) {
        const int L = 63 - __clzll((long long)mm);
        for (int m = 0; m < 4; ++m) lm[m] = __shfl(p[m], L);
      }
      if (mp) {
        const int L = 63 - __clzll((long long)mp);
        for (int m = 0; m < 4; ++m) lp[m] = __shfl(p[m], L);
      }
      const bool par = out && pid != 11 && pid != -11 && is_parton(pid);
      const unsigned long long pm = __ballot(par);
      np += __popcll(pm);
      const bool jet = par && p[1] * p[1] + p[2] * p[2] > 1e-18 * C.S;
      const unsigned long long jm = __ballot(jet);
      if (jet) {
        const int i = nq + __popcll(jm & ((1ull << lane) - 1ull));
        for (int m = 0; m < 4; ++m) W.q[i][m] = p[m];
      }
      nq += __popcll(jm);
    }
    for (int o = 32; o > 0; o >>= 1)
      for (int m = 0; m < 4; ++m) bal[m] += __shfl_xor(bal[m], o);
    __builtin_amdgcn_wave_barrier();
    // ---- anti-kT, R = 0.4, E-scheme
    auto props = [&](int i) {
      W.y[i] = rapidity(W.q[i]);
      W.ph[i] = atan2(W.q[i][2], W.q[i][1]);
      W.ip[i] = 1.0 / (W.q[i][1] * W.q[i][1] + W.q[i][2] * W.q[i][2]);
    };
    for (int i = lane; i < nq; i += 64) props(i);
    __builtin_amdgcn_wave_barrier();
    const double iR2 = 0.4 * 0.4;
    const int nitem = nq * (nq + 1) / 2;
    int nj = 0;
    for (int alive = nq; alive > 0; --alive) {
      // this lane's smallest distance, the serial loop's first on ties
      double bv = INFINITY;
      int bo = kNoItem;
      auto take = [&](int a, int b) {
        const double ipa = W.ip[a];
        if (!(ipa > 0.0)) return;
        double v = ipa;
        if (a != b) {
          const double ipb = W.ip[b];
          if (!(ipb > 0.0)) return;
          double dy = W.y[a] - W.y[b];
          double dphi = fabs(W.ph[a] - W.ph[b]);
          if (dphi > kPi) dphi = 2.0 * kPi - dphi;
          double dR2 = dy * dy + dphi * dphi;
          v = fmin(ipa, ipb) * dR2 / iR2;
        }
        const int o = obs_ord(a, b);
        if (v < bv || (v == bv && o < bo)) { bv = v; bo = o; }
      };
#pragma unroll
      for (int k = 0; k < kObsPass; ++k)
        if (lane + 64 * k < nitem) take(pa[k], pb[k]);
      for (int q = lane + 64 * kObsPass; q < nitem; q += 64) {
        int a, b;
        obs_tri(q, a, b);
        take(a, b);
      }
      double m = bv;
      for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o));
      const bool mine = bo != kNoItem && bv == m;
      const unsigned long long hit = __ballot(mine);
      if (!hit) break;  // no finite distance (no such event): stop clustering
      int wo;
      if (__popcll(hit) == 1) {
        wo = __shfl(bo, __ffsll((long long)hit) - 1);
      } else {
        int c = mine ? bo : kNoItem;
        for (int o = 32; o > 0; o >>= 1) c = min(c, __shfl_xor(c, o));
        wo = c;
      }
      const int a = wo >> 8, r = wo & 0xFF;
      if (lane == 0) {
        if (r == 0) {
          W.jet[nj] = a;
          W.ip[a] = -1.0;
        } else {
          for (int mm = 0; mm < 4; ++mm) W.q[a][mm] += W.q[r - 1][mm];
          props(a);
          W.ip[r - 1] = -1.0;
        }
      }
      if (r == 0) ++nj;
      __builtin_amdgcn_wave_barrier();
    }
    // ---- jets by pT, descending, equal pT keep their order: each jet's rank
    auto pt2 = [&](int k) { return W.q[k][1] * W.q[k][1] + W.q[k][2] * W.q[k][2]; };
    for (int k = lane; k < nj; k += 64) {
      const int t = W.jet[k];
      const double p2 = pt2(t);
      int r = 0;
      for (int mm = 0; mm < nj; ++mm) {
        const double o2 = pt2(W.jet[mm]);
        r += (o2 > p2 || (o2 == p2 && mm < k)) ? 1 : 0;
      }
      W.srt[r] = t;
    }
    __builtin_amdgcn_wave_barrier();
    // ---- jet pT and pseudorapidity of each jet on a lane of its own; items
    // nj and nj + 1 are the two leptons' pseudorapidities
    int njet = 0, n_eta = 0;
    double j1pt = 0.0, j2pt = 0.0, j1eta = 0.0, et1 = 0.0, et2 = 0.0, etm = 0.0, etp = 0.0;
    bool have1 = false;
    int i1 = -1, i2 = -1;
    for (int k0 = 0; k0 < nj + 2; k0 += 64) {
      const int k = k0 + lane;
      double p[4] = {0.0, 0.0, 0.0, 1.0};
      if (k < nj) {
        for (int mm = 0; mm < 4; ++mm) p[mm] = W.q[W.srt[k]][mm];
      } else if (k == nj) {
        for (int mm = 0; mm < 4; ++mm) p[mm] = lm[mm];
      } else if (k == nj + 1) {
        for (int mm = 0; mm < 4; ++mm) p[mm] = lp[mm];
      }
      double pt = 0.0, et = 0.0;
      if (k < nj + 2) {
        pt = sqrt(p[1] * p[1] + p[2] * p[2]);
        et = pseudorap(p);
      }
      const bool jt = k < nj;
      unsigned long long me = __ballot(jt && fabs(et) < 5.0);
      const unsigned long long mp = __ballot(jt && pt > 5.0);
      unsigned long long mb = __ballot(jt && pt > 5.0 && fabs(et) < 5.0);
      if (nj >= k0 && nj < k0 + 64) etm = __shfl(et, nj - k0);
      if (nj + 1 >= k0 && nj + 1 < k0 + 64) etp = __shfl(et, nj + 1 - k0);
      for (; n_eta < 2 && me; me &= me - 1, ++n_eta) {
        const double v = __shfl(pt, __ffsll((long long)me) - 1);
        if (n_eta == 0) j1pt = v;
        else j2pt = v;
      }
      if (!have1 && mp) {
        j1eta = __shfl(et, __ffsll((long long)mp) - 1);
        have1 = true;
      }
      for (; njet < 2 && mb; mb &= mb - 1, ++njet) {
        const int L = __ffsll((long long)mb) - 1;
        if (njet == 0) { i1 = W.srt[k0 + L]; et1 = __shfl(et, L); }
        else { i2 = W.srt[k0 + L]; et2 = __shfl(et, L); }
      }
      njet += __popcll(mb);
    }
    // ---- the azimuths (Z, leptons, the two leading jets) on a lane each
    double Z[4];
    for (int mm = 0; mm < 4; ++mm) Z[mm] = lm[mm] + lp[mm];
    double az = 0.0;
    {
      double ax = 0.0, ay = 0.0;
      bool need = false;
      if (lane == 0) { ax = Z[1]; ay = Z[2]; need = !(Z[1] == 0.0 && Z[2] == 0.0); }
      else if (lane == 1) { ax = lm[1]; ay = lm[2]; need = true; }
      else if (lane == 2) { ax = lp[1]; ay = lp[2]; need = true; }
      else if (lane == 3 && njet >= 2) { ax = W.q[i1][1]; ay = W.q[i1][2]; need = true; }
      else if (lane == 4 && njet >= 2) { ax = W.q[i2][1]; ay = W.q[i2][2]; need = true; }
      if (need) az = atan2(ay, ax);
    }
    const double phm = __shfl(az, 1), php = __shfl(az, 2), ph1 = __shfl(az, 3), ph2 = __shfl(az, 4);
    // ---- Z and jet observables (one lane)
    if (lane == 0) {
      double* o = obs + e * kNObs;
      double imb = 0.0;
      for (int mm = 0; mm < 4; ++mm) imb = fmax(imb, fabs(bal[mm]));
      o[0] = sqrt(Z[1] * Z[1] + Z[2] * Z[2]);
      o[1] = rapidity(Z);
      o[2] = az;
      double dphi = fabs(phm - php);
      if (dphi > kPi) dphi = 2.0 * kPi - dphi;
      double cth = tanh(0.5 * (etm - etp));
      o[3] = tan(0.5 * (kPi - dphi)) * sqrt(fmax(0.0, 1.0 - cth * cth));
      o[4] = njet;
      o[5] = j1pt;
      o[6] = j1eta;
      o[7] = j2pt;
      if (njet >= 2) {
        double dy = et1 - et2;
        double dp = fabs(ph1 - ph2);
        if (dp > kPi) dp = 2.0 * kPi - dp;
        o[8] = sqrt(dy * dy + dp * dp);
      } else {
        o[8] = -1.0;
      }
      o[9] = np;
      o[10] = imb;
      o[11] = 0.0;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ void k_histogram(const double* obs, const double* w, int64_t n, int col, double lo, double hi,
                            int nbins, double* sumw, double* sumw2) {
  // bins of the block in LDS when they fit (nbins <= kHistLds), one global
  // atomic per bin per block at the end; else straight to the global bins
  extern __shared__ double hs[];
  const bool lds = nbins <= kHistLds;
  if (lds) {
    for (int b = threadIdx.x; b < 2 * nbins; b += blockDim.x) hs[b] = 0.0;
    __syncthreads();
  }
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double v = obs[e * kNObs + col];
    if (!(v >= lo && v < hi)) continue;
    int b = (int)((v - lo) / (hi - lo) * nbins);
    if (b >= nbins) b = nbins - 1;
    double ww = w ? w[e] : 1.0;
    if (lds) {
      atomicAdd(hs + b, ww);
      atomicAdd(hs + nbins + b, ww * ww);
    } else {
      atomicAdd(sumw + b, ww);
      atomicAdd(sumw2 + b, ww * ww);
    }
  }
  if (lds) {
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
      if (hs[b] != 0.0) atomicAdd(sumw + b, hs[b]);
      if (hs[nbins + b] != 0.0) atomicAdd(sumw2 + b, hs[nbins + b]);
    }
  }
}

}  // namespace gaps
