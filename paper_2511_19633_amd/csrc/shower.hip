// The shower kernel: the max-veto algorithm of section 2 with the initial-state
// extension of appendix A and the dipole kinematics of appendix B, one event
// per lane.  Lanes fetch events from a work queue, so the launch is persistent
// and finished lanes refill at once; every lane keeps its event record and its
// channel cache in slot-major scratch (stride = lanes), so a wave's accesses
// coalesce whatever events the lanes hold.
#include "kernels.hpp"

namespace gaps {

namespace {

// channel cache word: emitter slot, spectator slot, side, type, heavy flavour, alive
__device__ __forceinline__ uint32_t pack_info(const Chan& ch) {
  return (uint32_t)ch.i | ((uint32_t)ch.k << 8) | ((uint32_t)ch.side << 16) | ((uint32_t)ch.type << 17) |
         ((uint32_t)ch.heavy << 19) | ((uint32_t)ch.alive << 21);
}

// rebuild the channel list in (slot, side) order; -1 on a broken colour line
__device__ int build_channels(const Cfg& C, const Rec& R, int n, const Scratch& S, int& nch, bool mec) {
  int m = 0;
  Chan ch;
  for (int i = 0; i < n; ++i) {
    int64_t oi = R.o(i);
    if (R.col[oi] == 0 && R.acol[oi] == 0) continue;
    for (int side = 0; side < 2; ++side) {
      int tag = side == 0 ? R.effc(i) : R.effa(i);
      if (!tag) continue;
      int k = -1;
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        int other = side == 0 ? R.effa(j) : R.effc(j);
        if (other == tag) { k = j; break; }
      }
      if (k < 0) return -1;
      chan_setup(C, R, i, side, k, ch, mec);
      int64_t oc = (int64_t)R.lane * S.nch + m;
      S.info[oc] = pack_info(ch);
      S.ent[oc].t.tl = ch.tlim;
      S.ent[oc].t.ltl = ch.lntlim;
      S.ent[oc].t.ic = ch.invc;
      S.key[oc] = ch.c;  // this kernel keeps no pending trials: the slot holds c
      ++m;
    }
  }
  nch = m;
  return 0;
}

// cutoff (and ln cutoff) and heavy-quark mass^2 of a channel from its type and
// heavy flavour
__device__ __forceinline__ void chan_cut(const Cfg& C, int type, int heavy, double& tcut, double& lntcut,
                                         double& m2) {
  m2 = 0.0;
  if (heavy == 1) { tcut = C.tch_c; lntcut = C.ln_tch_c; m2 = C.mc2; }
  else if (heavy == 2) { tcut = C.tch_b; lntcut = C.ln_tch_b; m2 = C.mb2; }
  else if (type == kFF) { tcut = C.t_cut; lntcut = C.ln_tc; }
  else { tcut = C.tc_is; lntcut = C.ln_tcis; }
}

// veto-max: the Philox block of trial k of channel c (b = 0: its scale, 1:
// term, z, azimuth and acceptance), and the longest loop of one channel
__device__ __forceinline__ uint32_t vm_block(int c, int k, int b) {
  return 0x80000000u | ((uint32_t)c << 20) | ((uint32_t)k << 1) | (uint32_t)b;
}
constexpr int kVmMaxTrials = 1 << 19;

// FORM 0: max-veto (every channel draws each cycle), 1: generate-select,
// 2: veto-max; one kernel each, so that each keeps its own register budget
template <int FORM>
__device__ void shower_one(const Cfg& C, const gaps_events& in, int64_t e, const gaps_events& out,
                           const Rec& R, const Scratch& S, const ShowerArgs& A, unsigned long long* st) {
  const int M = out.max_slots < kMaxSlots ? out.max_slots : kMaxSlots;
  const int64_t ci = in.cap, co = out.cap;
  int n = in.n[e];
  uint32_t flags = in.flags ? in.flags[e] : 0u;
  int maxtag = 0;
  bool fits = n >= 0 && n <= M && n <= in.max_slots;
  if (fits) {
    for (int q = 0; q < n; ++q) {
      int64_t k = (int64_t)q * ci + e, o = R.o(q);
      R.E[o] = in.E[k]; R.px[o] = in.px[k]; R.py[o] = in.py[k]; R.pz[o] = in.pz[k];
      R.pid[o] = in.pid[k]; R.col[o] = in.col[k]; R.acol[o] = in.acol[k]; R.st[o] = in.status[k];
      maxtag = in.col[k] > maxtag ? in.col[k] : maxtag;
      maxtag = in.acol[k] > maxtag ? in.acol[k] : maxtag;
    }
  }
  const int64_t id = in.id[e];
  double T = in.t_start[e], lnT = log(T), t1 = 0.0;
  uint32_t ncyc = 0, ntri = 0, nacc = 0, nviol = 0;
  int nch = 0;
  // a flagged event's first emission is corrected to the real matrix element
  auto mec_now = [&]() { return (flags & fMEC) != 0u && t1 == 0.0; };
  if (!fits) {
    flags |= fOverflow;
  } else if (build_channels(C, R, n, S, nch, mec_now()) < 0) {
    flags |= fColour;
  } else {
    uint32_t cycle = 0;
    const uint64_t seed = A.seed;
    const uint32_t stream = A.stream;
    // veto-max: every channel runs its own veto loop down to its first
    // accepted trial; the largest of these is the emission; a cycle is one
    // emission, after which every channel runs its loop again
    for (; FORM == 2;) {
      if (cycle >= kMaxCycles) { flags |= fMaxCyc; break; }
      double best = -INFINITY;
      int win = -1, wkern = 0, wflav = 0;
      double wz = 0.0, womz = 0.0, wphi = 0.0, wa1 = 0.0, wa2 = 0.0;  // the best candidate's emission
      bool capped = false;
      for (int c = 0; c < nch && !capped; ++c) {
        const int64_t oc = (int64_t)R.lane * S.nch + c;
        const uint32_t info = S.info[oc];
        if (!((info >> 21) & 1u)) continue;
        double tcut, lntcut, m2;
        const int heavy = (info >> 19) & 3u;
        chan_cut(C, (info >> 17) & 3u, heavy, tcut, lntcut, m2);
        double Tch = S.ent[oc].t.tl, lnTch = S.ent[oc].t.ltl;
        if (T < Tch) { Tch = T; lnTch = lnT; }
        const double invc = S.ent[oc].t.ic;
        Chan ch;
        chan_setup(C, R, info & 0xFFu, (info >> 16) & 1u, (info >> 8) & 0xFFu, ch, mec_now());
        for (int k = 0;; ++k) {
          if (k >= kVmMaxTrials) { capped = true; break; }
          if (!(Tch > tcut)) break;
          double ub[4];
          rng4(seed, stream, id, cycle, vm_block(c, k, 0), ub);
          ntri += 1;
          const double lu = log(ub[0]);
          double key;
          if (!heavy) key = lnTch + lu * invc;
          else key = log(m2 + (Tch - m2) * exp(lu * invc));
          if (key < lntcut) break;
          const double t = exp(key);
          double u[4];
          rng4(seed, stream, id, cycle, vm_block(c, k, 1), u);
          const Term tm = select_term(C, ch, u[0]);
          double z, omz;
          shape_sample(tm.shape, ch, tm.I, u[1], z, omz);
          const Veto v = veto_weight(C, R, ch, tm, t, key, z, omz);
          if (v.ok && v.w > 1.0) { nviol += 1; flags |= fViol; }
          if (v.ok && u[3] < v.w) {
            if (key > best) {
              best = key;
              win = c;
              wkern = tm.kern;
              wflav = tm.flav;
              wz = z;
              womz = omz;
              wphi = 2.0 * kPi * u[2];
              map_vars(ch.type, v, wa1, wa2);
            }
            break;
          }
          Tch = t;
          lnTch = key;
        }
      }
      if (capped) { flags |= fMaxCyc; break; }
      if (win < 0) break;
      // the winner's accepted trial, as recorded
      const uint32_t info = S.info[(int64_t)R.lane * S.nch + win];
      Chan ch;
      chan_setup(C, R, info & 0xFFu, (info >> 16) & 1u, (info >> 8) & 0xFFu, ch, mec_now());
      const double t = exp(best);
      if (n + 1 > M) { flags |= fOverflow; break; }
      emit_map(R, n, maxtag, ch, wkern, wflav, wz, womz, wa1, wa2, wphi);
      n += 1;
      nacc += 1;
      if (t1 == 0.0) t1 = t;
      cycle += 1;
      bool bad = false;
      for (int q = 0; q < n; ++q) {
        const int64_t o = R.o(q);
        bad |= !(isfinite(R.E[o]) && isfinite(R.px[o]) && isfinite(R.py[o]) && isfinite(R.pz[o]));
      }
      if (bad) { flags |= fNaN; break; }
      if (build_channels(C, R, n, S, nch, mec_now()) < 0) { flags |= fColour; break; }
      T = t;
      lnT = best;
    }
    for (; FORM != 2;) {
      if (cycle >= kMaxCycles) { flags |= fMaxCyc; break; }
      double best = -INFINITY;
      int win = -1;
      uint32_t curblk = 0xFFFFFFFFu;
      double ub[4] = {0.0, 0.0, 0.0, 0.0};
      if constexpr (FORM == 1) {
        // generate-select: the segment below T ends at the largest scale below
        // T where a channel starts (its limit) or stops (its cutoff); its
        // active channels' shares sum to C, a heavy-quark channel's bound
        // c lo/(lo - m^2) over the segment
        double lo = -1.0, lnlo = 0.0;
        bool any = false;
        for (int c = 0; c < nch; ++c) {
          const int64_t oc = (int64_t)R.lane * S.nch + c;
          const uint32_t info = S.info[oc];
          if (!((info >> 21) & 1u)) continue;
          const double tlim = S.ent[oc].t.tl;
          double tcut, lntcut, m2;
          chan_cut(C, (info >> 17) & 3u, (info >> 19) & 3u, tcut, lntcut, m2);
          if (!(tlim > tcut)) continue;
          if (tlim < T) {
            if (tlim > lo) { lo = tlim; lnlo = S.ent[oc].t.ltl; }
          } else if (tcut < T) {
            any = true;
            if (tcut > lo) { lo = tcut; lnlo = lntcut; }
          }
        }
        if (lo < 0.0) break;  // no channel can emit below T
        if (!any) {           // none active: move to where one starts
          T = lo;
          lnT = lnlo;
          cycle += 1;
          continue;
        }
        // active channels in entry order: their share of the segment's sum
        auto share = [&](int c, double& sh) -> bool {
          const int64_t oc = (int64_t)R.lane * S.nch + c;
          const uint32_t info = S.info[oc];
          if (!((info >> 21) & 1u)) return false;
          const double tlim = S.ent[oc].t.tl;
          double tcut, lntcut, m2;
          const int heavy = (info >> 19) & 3u;
          chan_cut(C, (info >> 17) & 3u, heavy, tcut, lntcut, m2);
          if (!(tlim > tcut && tlim >= T && tcut < T)) return false;
          const double cc = S.key[oc];
          sh = heavy ? cc * lo / (lo - m2) : cc;
          return true;
        };
        double Csum = 0.0;
        for (int c = 0; c < nch; ++c) {
          double sh;
          if (share(c, sh)) Csum += sh;
        }
        double g[4];
        rng4(seed, stream, id, cycle, 0xFFFFFFFEu, g);
        ntri += 1;
        const double lnt = lnT + log(g[0]) / Csum;
        if (lnt < lnlo) {  // below the segment: a null at its lower end
          T = lo;
          lnT = lnlo;
          cycle += 1;
          continue;
        }
        const double target = g[1] * Csum;
        double cum = 0.0;
        int sel = -1, last = -1;
        for (int c = 0; c < nch && sel < 0; ++c) {
          double sh;
          if (!share(c, sh)) continue;
          cum += sh;
          last = c;
          if (target < cum) sel = c;
        }
        if (sel < 0) sel = last;
        const uint32_t sinfo = S.info[(int64_t)R.lane * S.nch + sel];
        const int sheavy = (sinfo >> 19) & 3u;
        if (sheavy) {  // thin the bound back to c/(t - m^2)
          double tcut, lntcut, m2;
          chan_cut(C, (sinfo >> 17) & 3u, sheavy, tcut, lntcut, m2);
          const double t = exp(lnt);
          const double keep = (t * (lo - m2)) / (lo * (t - m2));
          if (!(g[2] < keep)) {
            T = t;
            lnT = lnt;
            cycle += 1;
            continue;
          }
        }
        best = lnt;
        win = sel;
      }
      for (int c = 0; FORM == 0 && c < nch; ++c) {
        int64_t oc = (int64_t)R.lane * S.nch + c;
        uint32_t info = S.info[oc];
        if (!((info >> 21) & 1u)) continue;
        double tlim = S.ent[oc].t.tl, lntlim = S.ent[oc].t.ltl;
        int type = (info >> 17) & 3u, heavy = (info >> 19) & 3u;
        double tcut, lntcut, m2 = 0.0;
        if (heavy == 1) { tcut = C.tch_c; lntcut = C.ln_tch_c; m2 = C.mc2; }
        else if (heavy == 2) { tcut = C.tch_b; lntcut = C.ln_tch_b; m2 = C.mb2; }
        else if (type == kFF) { tcut = C.t_cut; lntcut = C.ln_tc; }
        else { tcut = C.tc_is; lntcut = C.ln_tcis; }
        double Tch = T < tlim ? T : tlim;
        double lnTch = lnT < lntlim ? lnT : lntlim;
        if (!(Tch > tcut)) continue;
        uint32_t slot = 2u * (info & 0xFFu) + ((info >> 16) & 1u);
        if ((slot >> 2) != curblk) {
          curblk = slot >> 2;
          rng4(seed, stream, id, cycle, curblk, ub);
        }
        double lu = log(ub[slot & 3u]);
        ntri += 1;
        double invc = S.ent[oc].t.ic;
        double key;
        if (!heavy) key = lnTch + lu * invc;
        else key = log(m2 + (Tch - m2) * exp(lu * invc));
        if (key < lntcut) continue;
        if (key > best) { best = key; win = c; }
      }
      if (win < 0) break;
      double t = exp(best);
      uint32_t info = S.info[(int64_t)R.lane * S.nch + win];
      Chan ch;
      chan_setup(C, R, info & 0xFFu, (info >> 16) & 1u, (info >> 8) & 0xFFu, ch, mec_now());
      double u[4];
      rng4(seed, stream, id, cycle, 0xFFFFFFFFu, u);
      Term tm = select_term(C, ch, u[0]);
      double z, omz;
      shape_sample(tm.shape, ch, tm.I, u[1], z, omz);
      double phi = 2.0 * kPi * u[2];
      Veto v = veto_weight(C, R, ch, tm, t, best, z, omz);
      if (v.ok && v.w > 1.0) { nviol += 1; flags |= fViol; }
      if (v.ok && u[3] < v.w) {
        if (n + 1 > M) { flags |= fOverflow; break; }
        emit(R, n, maxtag, ch, tm, z, omz, v, phi);
        n += 1;
        nacc += 1;
        if (t1 == 0.0) t1 = t;
        bool bad = false;
        for (int q = 0; q < n; ++q) {
          int64_t o = R.o(q);
          bad |= !(isfinite(R.E[o]) && isfinite(R.px[o]) && isfinite(R.py[o]) && isfinite(R.pz[o]));
        }
        if (bad) { flags |= fNaN; cycle += 1; break; }
        if (build_channels(C, R, n, S, nch, mec_now()) < 0) { flags |= fColour; cycle += 1; break; }
      }
      T = t;
      lnT = best;
      cycle += 1;
    }
    ncyc = cycle;
  }
  out.id[e] = id;
  out.w[e] = in.w[e];
  out.t_start[e] = in.t_start[e];
  out.n[e] = fits ? n : in.n[e];
  if (out.flags) out.flags[e] = flags;
  if (fits) {
    for (int q = 0; q < n && q < out.max_slots; ++q) {
      int64_t k = (int64_t)q * co + e, o = R.o(q);
      out.E[k] = R.E[o]; out.px[k] = R.px[o]; out.py[k] = R.py[o]; out.pz[k] = R.pz[o];
      out.pid[k] = R.pid[o]; out.col[k] = R.col[o]; out.acol[k] = R.acol[o]; out.status[k] = R.st[o];
    }
  } else {
    // record larger than the output capacity: pass the slots that fit through
    for (int q = 0; q < n && q < out.max_slots && q < in.max_slots; ++q) {
      int64_t k = (int64_t)q * co + e, ki = (int64_t)q * ci + e;
      out.E[k] = in.E[ki]; out.px[k] = in.px[ki]; out.py[k] = in.py[ki]; out.pz[k] = in.pz[ki];
      out.pid[k] = in.pid[ki]; out.col[k] = in.col[ki]; out.acol[k] = in.acol[ki]; out.status[k] = in.status[ki];
    }
  }
  if (out.n_cycles) out.n_cycles[e] = ncyc;
  if (out.n_trials) out.n_trials[e] = ntri;
  if (out.n_accept) out.n_accept[e] = nacc;
  if (out.n_viol) out.n_viol[e] = nviol;
  if (out.t1) out.t1[e] = t1;
  if (st) {
    atomicAdd(st + 0, (unsigned long long)ncyc);
    atomicAdd(st + 1, (unsigned long long)ntri);
    atomicAdd(st + 2, (unsigned long long)nacc);
    atomicAdd(st + 3, (unsigned long long)nviol);
  }
}

}  // namespace

template <int FORM>
__device__ __forceinline__ void lanes_body(const Cfg& C, const gaps_events& in, const gaps_events& out,
                                           const Scratch& S, const ShowerArgs& A) {
  const int64_t lane = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  Rec R = make_rec(S.part, S.lanes, 1, lane);
  for (;;) {
    unsigned long long e = atomicAdd(S.queue, 1ULL);
    if (e >= (unsigned long long)A.n) break;
    shower_one<FORM>(C, in, (int64_t)e, out, R, S, A, A.stats);
  }
}

__global__ void __launch_bounds__(256) k_shower_lanes(Cfg C, gaps_events in, gaps_events out, Scratch S,
                                                      ShowerArgs A) {
  lanes_body<0>(C, in, out, S, A);
}
__global__ void __launch_bounds__(256) k_shower_lanes_gs(Cfg C, gaps_events in, gaps_events out, Scratch S,
                                                         ShowerArgs A) {
  lanes_body<1>(C, in, out, S, A);
}
__global__ void __launch_bounds__(256) k_shower_lanes_vm(Cfg C, gaps_events in, gaps_events out, Scratch S,
                                                         ShowerArgs A) {
  lanes_body<2>(C, in, out, S, A);
}

}  // namespace gaps
