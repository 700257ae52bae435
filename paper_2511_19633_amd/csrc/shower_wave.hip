// Wave-cooperative shower kernel.  One event per lane for the serial part of
// the veto algorithm (section 2: trial scales, winner, accept/veto, emission),
// and the whole wavefront for the parts that have inner parallelism:
//  - channel (re)builds after an emission or a refill: the 64 lanes take the
//    (slot, side) dipole ends of one event at a time, so a build costs about
//    one channel set-up instead of 2n sequential ones on one lane while the
//    other 63 wait;
//  - refill: finished lanes take new event ids from the work queue with one
//    atomic per wave (ballot + prefix count), every `compact_every` cycles.
// Event records are lane-major (one event contiguous) so cooperative reads of
// another lane's event coalesce; the channel cache is indexed by (slot, side),
// the coordinate that also keys the random numbers, stored [entry][lane] so
// the per-lane trial loop reads coalesce across the wave.
#include "kernels.hpp"

namespace gaps {

namespace {

// cache word: alive | type<<1 | heavy<<3 | spectator<<5 | eta bin<<13 | spectator eta bin<<19
__device__ __forceinline__ uint32_t pack(const Chan& ch) {
  return (uint32_t)ch.alive | ((uint32_t)ch.type << 1) | ((uint32_t)ch.heavy << 3) | ((uint32_t)ch.k << 5) |
         ((uint32_t)ch.ebin << 13) | ((uint32_t)ch.kbin << 19);
}

__device__ __forceinline__ unsigned long long lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

struct WaveCtx {
  const Cfg& C;
  const Scratch& S;
  int64_t wbase;  // state slot of lane 0
  int lane;
  int M;
};

__device__ __forceinline__ Rec rec_of(const Scratch& S, int64_t slot) {
  return Rec{S.E, S.px, S.py, S.pz, S.pid, S.col, S.acol, S.st, 1, S.max_slots, slot};
}

// Cooperative (re)build of every channel entry of the events whose lanes are
// set in `mask`.  For each such event, lane j holds the effective colour
// tags of particles j and j + 64, so the colour partner of every dipole end
// is found with register reads instead of a search through memory; then lane
// c sets up entry c = 2 * slot + side.  Returns (per lane) whether this
// lane's own event hit a broken colour line or a non-finite momentum.
__device__ uint32_t coop_build(const WaveCtx& W, unsigned long long mask, int n) {
  uint32_t myflags = 0u;
  __threadfence_block();
  while (mask) {
    const int L = __ffsll((long long)mask) - 1;
    mask &= mask - 1ull;
    const int nL = __shfl(n, L);
    const int64_t slot = W.wbase + L;
    const Rec R = rec_of(W.S, slot);
    // colours of particles lane and lane + 64 in registers
    int ec0 = 0, ea0 = 0, ec1 = 0, ea1 = 0;
    bool bad = false;
    for (int r = 0; r < 2; ++r) {
      const int q = W.lane + 64 * r;
      if (q >= nL) continue;
      const int64_t o = R.o(q);
      const int st = R.st[o], cl = R.col[o], al = R.acol[o];
      const int ec = st < 0 ? al : cl, ea = st < 0 ? cl : al;
      if (r == 0) { ec0 = ec; ea0 = ea; } else { ec1 = ec; ea1 = ea; }
      bad |= !(isfinite(R.E[o]) && isfinite(R.px[o]) && isfinite(R.py[o]) && isfinite(R.pz[o]));
    }
    bool missing = false;
    for (int base = 0; base < 2 * nL; base += 64) {
      const int c = base + W.lane;
      const int i = c >> 1, side = c & 1;
      // this entry's tag: colour (side 0) or anticolour (side 1) of particle i
      const int src = i & 63;
      const int tc0 = __shfl(ec0, src), ta0 = __shfl(ea0, src);
      const int tc1 = __shfl(ec1, src), ta1 = __shfl(ea1, src);
      const int tag = c < 2 * nL ? (i < 64 ? (side == 0 ? tc0 : ta0) : (side == 0 ? tc1 : ta1)) : 0;
      int k = -1;
      if (nL <= 128) {
        for (int j = 0; j < nL; ++j) {
          const int oc = j < 64 ? __shfl(ec0, j) : __shfl(ec1, j - 64);
          const int oa = j < 64 ? __shfl(ea0, j) : __shfl(ea1, j - 64);
          const int other = side == 0 ? oa : oc;
          if (k < 0 && j != i && tag != 0 && other == tag) k = j;
        }
      } else if (tag != 0) {
        for (int j = 0; j < nL; ++j) {
          if (j == i) continue;
          const int other = side == 0 ? R.effa(j) : R.effc(j);
          if (other == tag) { k = j; break; }
        }
      }
      if (c >= 2 * nL) continue;
      if (tag != 0 && k < 0) missing = true;
      const int64_t oc = (int64_t)c * W.S.lanes + slot;
      if (k < 0) { W.S.cinfo[oc] = 0u; continue; }
      Chan ch;
      chan_setup(W.C, R, i, side, k, ch);
      W.S.cinfo[oc] = pack(ch);
      W.S.ctlim[oc] = ch.tlim;
      W.S.clntlim[oc] = ch.lntlim;
      W.S.cinvc[oc] = ch.invc;
      W.S.cc[oc] = ch.c;
      W.S.cs[oc] = ch.s;
      W.S.czlo[oc] = ch.zlo;
      W.S.comzhi[oc] = ch.omzhi;
      W.S.cI1[oc] = ch.I1;
      W.S.cI2[oc] = ch.I2;
    }
    const bool anymiss = __ballot(missing) != 0ull;
    const bool anybad = __ballot(bad) != 0ull;
    if (W.lane == L) myflags = (anymiss ? fColour : 0u) | (anybad ? fNaN : 0u);
  }
  __threadfence_block();
  return myflags;
}

// rebuild the channel description of cache entry c from the cache and record
__device__ __forceinline__ void chan_from_cache(const Cfg& C, const Scratch& S, const Rec& R, int64_t slot, int c,
                                                Chan& ch) {
  const int64_t oc = (int64_t)c * S.lanes + slot;
  uint32_t info = S.cinfo[oc];
  ch.alive = 1;
  ch.i = c >> 1;
  ch.side = c & 1;
  ch.type = (info >> 1) & 3u;
  ch.heavy = (info >> 3) & 3u;
  ch.k = (info >> 5) & 0xFFu;
  ch.ebin = (info >> 13) & 0x3Fu;
  ch.kbin = (info >> 19) & 0x3Fu;
  ch.m2 = ch.heavy == 1 ? C.mc2 : (ch.heavy == 2 ? C.mb2 : 0.0);
  ch.pidi = R.pid[R.o(ch.i)];
  ch.pidk = R.pid[R.o(ch.k)];
  ch.s = S.cs[oc];
  ch.c = S.cc[oc];
  ch.zlo = S.czlo[oc];
  ch.omzhi = S.comzhi[oc];
  ch.zhi = 1.0 - ch.omzhi;
  ch.omzlo = 1.0 - ch.zlo;
  ch.I1 = S.cI1[oc];
  ch.I2 = S.cI2[oc];
  ch.eta = (ch.type == kIF || ch.type == kII) ? 2.0 * R.E[R.o(ch.i)] / C.sqrt_s : 0.0;
  ch.etak = (ch.type == kFI || ch.type == kII) ? 2.0 * R.E[R.o(ch.k)] / C.sqrt_s : 0.0;
  ch.nterm = n_terms(ch, C.nf);
}

}  // namespace

__device__ __forceinline__ void shower_wave_body(const Cfg& Cg, const gaps_events& in, const gaps_events& out,
                                                 const Scratch& S, const ShowerArgs& A) {
  // the overestimate table, staged in LDS for the term loops
  __shared__ double s_bound[kNEnt * kNB];
  for (int q = threadIdx.x; q < kNEnt * kNB; q += blockDim.x) s_bound[q] = Cg.bound[q];
  __syncthreads();
  Cfg C = Cg;
  C.bound = s_bound;
  const int lane = threadIdx.x & 63;
  const int64_t slot = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int M = out.max_slots < S.max_slots ? out.max_slots : S.max_slots;
  const WaveCtx W{C, S, slot - lane, lane, M};
  const Rec R = rec_of(S, slot);
  const int K = A.compact_every > 0 ? A.compact_every : 4;

  bool active = false, exhausted = false, loaded = false, stop = false;
  int64_t e = 0, id = 0;
  double T = 0.0, lnT = 0.0, t1 = 0.0;
  uint32_t cycle = 0, ntri = 0, nacc = 0, nviol = 0, flags = 0;
  int n = 0, maxtag = 0;
  unsigned long long st_cyc = 0, st_tri = 0, st_acc = 0, st_viol = 0, st_iters = 0, st_active = 0;
  int since = 1 << 30;

  for (;;) {
    // ---- refill finished lanes from the work queue (one atomic per wave)
    unsigned long long act = __ballot(active);
    if (!exhausted && (since >= K || act == 0ull)) {
      unsigned long long idle = ~act;
      const int cnt = __popcll(idle);
      unsigned long long base = 0ull;
      if (lane == 0) base = atomicAdd(S.queue, (unsigned long long)cnt);
      base = __shfl(base, 0);
      if (base + (unsigned long long)cnt >= (unsigned long long)A.n) exhausted = true;
      bool fresh = false;
      if (!active) {
        const unsigned long long ev = base + (unsigned long long)__popcll(idle & lanemask_lt(lane));
        if (ev < (unsigned long long)A.n) {
          e = (int64_t)ev;
          n = in.n[e];
          id = in.id[e];
          flags = in.flags ? in.flags[e] : 0u;
          T = in.t_start[e];
          lnT = log(T);
          t1 = 0.0;
          cycle = ntri = nacc = nviol = 0u;
          maxtag = 0;
          active = true;
          loaded = false;
          stop = false;
          if (n < 0 || n > M || n > in.max_slots) {
            flags |= fOverflow;
            stop = true;
          } else {
            loaded = true;
            for (int q = 0; q < n; ++q) {
              const int64_t k = (int64_t)q * in.cap + e, o = R.o(q);
              R.E[o] = in.E[k]; R.px[o] = in.px[k]; R.py[o] = in.py[k]; R.pz[o] = in.pz[k];
              R.pid[o] = in.pid[k]; R.col[o] = in.col[k]; R.acol[o] = in.acol[k]; R.st[o] = in.status[k];
              maxtag = in.col[k] > maxtag ? in.col[k] : maxtag;
              maxtag = in.acol[k] > maxtag ? in.acol[k] : maxtag;
            }
            fresh = true;
          }
        }
      }
      {
        // a broken colour line stops the event before its first cycle
        const uint32_t f = coop_build(W, __ballot(fresh), n) & fColour;
        if (fresh && f) { flags |= f; stop = true; }
      }
      since = 0;
      act = __ballot(active);
    }
    if (act == 0ull) {
      if (exhausted) break;
      continue;
    }
    st_iters += 64ull;
    st_active += (unsigned long long)__popcll(act);

    // ---- one cycle of the veto algorithm on every active lane
    bool done = false, accepted = false;
    if (active && stop) done = true;
    if (active && !done && cycle >= kMaxCycles) { flags |= fMaxCyc; done = true; }
    if (active && !done) {
      // Trial scales of every channel and the winner (largest key = ln t,
      // ties to the lowest entry).  Each key is first bounded with the
      // hardware single-precision log of u and a rigorous error margin; the
      // double-precision log is taken only where the bounds cannot decide
      // (overlapping candidates, the cutoff) and for the final winner, so the
      // result is exactly that of evaluating every key in double precision.
      int win = -1;
      bool wexact = false;
      double wlo = 0.0, whi = 0.0, wkey = 0.0, wu = 0.5, wlnT = 0.0, winv = 0.0;
      for (int c0 = 0; c0 < 2 * n; c0 += 4) {
        uint32_t inf[4];
        double tl[4], ltl[4], ic[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t oc = (int64_t)(c0 + j) * S.lanes + slot;
          inf[j] = S.cinfo[oc];
          tl[j] = S.ctlim[oc];
          ltl[j] = S.clntlim[oc];
          ic[j] = S.cinvc[oc];
        }
        if (!((inf[0] | inf[1] | inf[2] | inf[3]) & 1u)) continue;
        double ub[4];
        rng4(A.seed, A.stream, id, cycle, (uint32_t)c0 >> 2, ub);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = c0 + j;
          const uint32_t info = inf[j];
          if (c >= 2 * n || !(info & 1u)) continue;
          const int type = (info >> 1) & 3u, heavy = (info >> 3) & 3u;
          double tcut, lntcut, m2 = 0.0;
          if (heavy == 1) { tcut = C.tch_c; lntcut = C.ln_tch_c; m2 = C.mc2; }
          else if (heavy == 2) { tcut = C.tch_b; lntcut = C.ln_tch_b; m2 = C.mb2; }
          else if (type == kFF) { tcut = C.t_cut; lntcut = C.ln_tc; }
          else { tcut = C.tc_is; lntcut = C.ln_tcis; }
          const double Tch = T < tl[j] ? T : tl[j];
          const double lnTch = lnT < ltl[j] ? lnT : ltl[j];
          if (!(Tch > tcut)) continue;
          ntri += 1;
          const double u = ub[j], invc = ic[j];
          double lo, hi, key = 0.0;
          bool exact;
          if (heavy) {
            key = log(m2 + (Tch - m2) * exp(log(u) * invc));
            if (key < lntcut) continue;
            lo = hi = key;
            exact = true;
          } else {
            const double lf = (double)__builtin_amdgcn_logf((float)u) * 0.69314718055994530942;
            const double ka = lnTch + lf * invc;
            const double err = invc * (fabs(lf) * 0x1p-17 + 0x1p-19) + 1e-12;
            lo = ka - err;
            hi = ka + err;
            if (hi < lntcut) continue;
            exact = false;
            if (lo < lntcut) {
              key = lnTch + log(u) * invc;
              if (key < lntcut) continue;
              lo = hi = key;
              exact = true;
            }
          }
          if (win < 0) {
            win = c; wlo = lo; whi = hi; wkey = key; wexact = exact; wu = u; wlnT = lnTch; winv = invc;
            continue;
          }
          if (hi <= wlo) continue;
          if (!(lo > whi)) {
            // the bounds overlap: decide with exact keys
            if (!wexact) { wkey = wlnT + log(wu) * winv; wlo = whi = wkey; wexact = true; }
            if (!exact) { key = lnTch + log(u) * invc; lo = hi = key; exact = true; }
            if (!(key > wkey)) continue;
          }
          win = c; wlo = lo; whi = hi; wkey = key; wexact = exact; wu = u; wlnT = lnTch; winv = invc;
        }
      }
      double best = -INFINITY;
      if (win >= 0) best = wexact ? wkey : wlnT + log(wu) * winv;
      if (win < 0) {
        done = true;
      } else {
        const double t = exp(best);
        Chan ch;
        chan_from_cache(C, S, R, slot, win, ch);
        double u[4];
        rng4(A.seed, A.stream, id, cycle, 0xFFFFFFFFu, u);
        const Term tm = select_term(C, ch, u[0]);
        double z, omz;
        shape_sample(tm.shape, ch, tm.I, u[1], z, omz);
        const double phi = 2.0 * kPi * u[2];
        const Veto v = veto_weight(C, R, ch, tm, t, z, omz);
        if (v.ok && v.w > 1.0) { nviol += 1; flags |= fViol; }
        if (v.ok && u[3] < v.w) {
          if (n + 1 > M) {
            flags |= fOverflow;
            done = true;
          } else {
            emit(R, n, maxtag, ch, tm, z, omz, v, phi);
            n += 1;
            nacc += 1;
            if (t1 == 0.0) t1 = t;
            accepted = true;
          }
        }
        if (!done) {
          T = t;
          lnT = best;
          cycle += 1;
        }
      }
    }
    // ---- cooperative channel rebuild for the lanes that emitted
    const unsigned long long emitted = __ballot(accepted);
    if (emitted) {
      uint32_t f = coop_build(W, emitted, n);
      if (f & fNaN) f = fNaN;  // a non-finite momentum is reported before the colour check
      if (accepted && f) { flags |= f; done = true; }
    }
    // ---- finished events: write out and free the lane
    if (active && done) {
      const int64_t co = out.cap;
      const int nin = in.n[e];
      const bool fits = loaded;
      out.id[e] = id;
      out.w[e] = in.w[e];
      out.t_start[e] = in.t_start[e];
      if (fits) {
        out.n[e] = n;
        for (int q = 0; q < n; ++q) {
          const int64_t k = (int64_t)q * co + e, o = R.o(q);
          out.E[k] = R.E[o]; out.px[k] = R.px[o]; out.py[k] = R.py[o]; out.pz[k] = R.pz[o];
          out.pid[k] = R.pid[o]; out.col[k] = R.col[o]; out.acol[k] = R.acol[o]; out.status[k] = R.st[o];
        }
      } else {
        out.n[e] = nin;
        for (int q = 0; q < nin && q < out.max_slots && q < in.max_slots; ++q) {
          const int64_t k = (int64_t)q * co + e, ki = (int64_t)q * in.cap + e;
          out.E[k] = in.E[ki]; out.px[k] = in.px[ki]; out.py[k] = in.py[ki]; out.pz[k] = in.pz[ki];
          out.pid[k] = in.pid[ki]; out.col[k] = in.col[ki]; out.acol[k] = in.acol[ki];
          out.status[k] = in.status[ki];
        }
      }
      if (out.flags) out.flags[e] = flags;
      if (out.n_cycles) out.n_cycles[e] = cycle;
      if (out.n_trials) out.n_trials[e] = ntri;
      if (out.n_accept) out.n_accept[e] = nacc;
      if (out.n_viol) out.n_viol[e] = nviol;
      if (out.t1) out.t1[e] = t1;
      st_cyc += cycle; st_tri += ntri; st_acc += nacc; st_viol += nviol;
      active = false;
    }
    since += 1;
  }
  if (A.stats) {
    atomicAdd(A.stats + 0, st_cyc);
    atomicAdd(A.stats + 1, st_tri);
    atomicAdd(A.stats + 2, st_acc);
    atomicAdd(A.stats + 3, st_viol);
    if (lane == 0) {
      atomicAdd(A.stats + 4, st_iters);
      atomicAdd(A.stats + 5, st_active);
    }
  }
}

// The same body at three register budgets (waves resident per SIMD): more
// waves hide more latency, fewer registers per wave spill more.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_shower_wave(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A) {
  shower_wave_body(C, in, out, S, A);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_shower_wave3(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A) {
  shower_wave_body(C, in, out, S, A);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_shower_wave4(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A) {
  shower_wave_body(C, in, out, S, A);
}

}  // namespace gaps
