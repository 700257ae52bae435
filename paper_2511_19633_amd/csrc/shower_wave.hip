// Wave-cooperative shower kernel.  One event per lane for the serial part of
// the veto algorithm (section 2: trial scales, winner, accept/veto, emission),
// and the whole wavefront for the parts that have inner parallelism:
//  - channel (re)builds after an emission or a refill: the 64 lanes take the
//    (slot, side) dipole ends of one event at a time, so a build costs about
//    one channel set-up instead of 2n sequential ones on one lane while the
//    other 63 wait;
//  - refill: finished lanes take new event ids from the work queue with one
//    atomic per wave (ballot + prefix count), every `compact_every` cycles;
//  - tail compaction: once the queue is empty, waves drain and would keep
//    paying full price per cycle for a few live lanes.  When every wave of the
//    block has seen the queue empty (an LDS counter, no barrier before that),
//    the block switches to tail mode: every 16 iterations it pools the
//    register state of its live events in LDS and packs them into its first
//    waves (each event keeps its state slot, so records and channel caches
//    stay where they are); emptied waves park at the block barrier.
// Event records are lane-major (one event contiguous) so cooperative reads of
// another lane's event coalesce; the channel cache is indexed by (slot, side),
// the coordinate that also keys the random numbers, stored [entry][lane] so
// the per-lane trial loop reads coalesce across the wave.
#include "kernels.hpp"

namespace gaps {

namespace {

// cache word: alive | type<<1 | heavy<<3 | spectator<<5 | eta bin<<13 | spectator eta bin<<19 |
// learned cell<<25 (the cell whose 1/c the trial entry holds; 15: none yet) | null<<29 |
// first-emission correction<<30
constexpr uint32_t kCellShift = 25u, kCellMask = 15u << kCellShift, kCellNone = 15u;
// retained trials: the entry's pending trial is a null at its cell's lower edge
constexpr uint32_t kNullBit = 1u << 29;
constexpr uint32_t kMecBit = 1u << 30;
__device__ __forceinline__ uint32_t pack(const Chan& ch) {
  return (uint32_t)ch.alive | ((uint32_t)ch.type << 1) | ((uint32_t)ch.heavy << 3) | ((uint32_t)ch.k << 5) |
         ((uint32_t)ch.ebin << 13) | ((uint32_t)ch.kbin << 19) | (kCellNone << kCellShift) |
         (ch.mec ? kMecBit : 0u);
}

__device__ __forceinline__ unsigned long long lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

// element j of a four-element register array, by selects (no private-memory
// indexing), so that a per-entry loop can stay rolled and its body is emitted
// once rather than four times
template <typename T>
__device__ __forceinline__ T pick4(const T (&a)[4], int j) {
  return j == 0 ? a[0] : (j == 1 ? a[1] : (j == 2 ? a[2] : a[3]));
}

struct WaveCtx {
  const Cfg& C;
  const Scratch& S;
  int lane;
  int M;
};

// register state of one in-flight event (what moves when the tail compacts)
struct LaneState {
  int64_t e, id, slot;
  int32_t b, lrn;
  double T, lnT, t1;
  uint32_t cycle, ntri, nacc, nviol, flags;
  int32_t n, maxtag;
  uint32_t bits;  // loaded | stop << 1 | rebuild << 3 | em_all << 4
  int32_t emik;   // emitter | spectator << 8 of the emission awaiting its channel rebuild
};
static_assert(sizeof(LaneState) <= kLaneStateBytes, "lane state exceeds its LDS budget");

// sum of a per-lane count over the wave, as a wave-uniform value
__device__ __forceinline__ unsigned long long wave_total(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
         (unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)v);
}

__device__ __forceinline__ Rec rec_of(const Scratch& S, int64_t slot) {
  return make_rec(S.part, 1, S.max_slots, slot);
}

// LDS of one wave for the cooperative channel build: a ring of entries that
// need their constants set up, and one flag word per lane.
constexpr int kBuildRing = 128;
// deferred rebuilds after emissions: build when this many lanes want one, when
// one has waited this many iterations, or when fewer lanes are left to trial
constexpr int kDeferLanes = 8, kDeferWait = 4, kDeferMin = 16;
// entries per lane in a pass of the retained form's argmax scan
constexpr int kScanGroup = 16;

struct BuildLds {
  uint32_t ring[kBuildRing];  // lane L | particle q << 6 | side << 14 | spectator k << 15
  uint32_t flags[64];
  uint32_t count[64];         // retained trials: draws per lane's event in a build
  int tag[64];                // refill: the largest colour tag of each lane's new event
};

// Owner lane of item g when every lane L contributes items
// [incl_L - count_L, incl_L) (incl: inclusive prefix of the counts over the
// wave): the number of lanes whose inclusive prefix is <= g.
__device__ __forceinline__ int owner_of(int incl, int g) {
  int L = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1) {
    const int v = __shfl(incl, L + step - 1);
    if (v <= g) L += step;
  }
  return L > 63 ? 63 : L;
}

// inclusive prefix sum of v over the wave
__device__ __forceinline__ int wave_incl(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, (unsigned)o);
    if (lane >= o) v += u;
  }
  return v;
}

// Retained trials: draw a new trial for cache entry c of the event in state
// slot `slot` from the evolution scale (T, lnT), with random number u.  The key
// ln t is stored in the entry (-inf: no trial above the cutoff) with its null
// bit; in learned mode an initial-state entry of the incoming partons draws
// against the constant of its scale's cell (refreshed here when the cell
// changed), and a trial below the cell is a null at the cell's lower edge.
// Returns whether a trial was drawn (the channel is open at this scale); kout
// gets the stored key.
__device__ __forceinline__ bool draw_entry(const Cfg& C, const Scratch& S, int64_t slot, int c, uint32_t info,
                                           double tl, double ltl, double ic, double u, double T, double lnT,
                                           bool lrn, double& kout) {
  const int64_t oc = (int64_t)slot * S.nch + c;
  double key = -INFINITY;
  bool isnull = false, tried = false;
  const uint32_t info0 = info;
  if (info & 1u) {
    const int type = (info >> 1) & 3u, heavy = (info >> 3) & 3u;
    double tcut, lntcut, m2 = 0.0;
    if (heavy == 1) { tcut = C.tch_c; lntcut = C.ln_tch_c; m2 = C.mc2; }
    else if (heavy == 2) { tcut = C.tch_b; lntcut = C.ln_tch_b; m2 = C.mb2; }
    else if (type == kFF) { tcut = C.t_cut; lntcut = C.ln_tc; }
    else { tcut = C.tc_is; lntcut = C.ln_tcis; }
    const double Tch = T < tl ? T : tl;
    const double lnTch = lnT < ltl ? lnT : ltl;
    if (Tch > tcut) {
      tried = true;
      double invc = ic, floor = -INFINITY;
      if (lrn && c < 4 && (type == kIF || type == kII)) {
        const int cell = cell_of(C, lnTch, floor);
        if ((int)((info & kCellMask) >> kCellShift) != cell) {
          // the emitter's flavour, I1 and I2 from the entry's own line
          const Win& wd = S.ent[oc].w;
          double lr[2];
          const double ck = learned_c2(C, type, (int)(int8_t)(wd.pid & 0xFFu), (int)((info >> 13) & 0x3Fu), wd.I1,
                                       wd.I2, cell, (info & kMecBit) != 0u, lr);
          invc = 1.0 / ck;
          S.ent[oc].t.ic = invc;
          S.ent[oc].w.c = ck;
          S.ent[oc].lr[0] = lr[0];
          S.ent[oc].lr[1] = lr[1];
          info = (info & ~kCellMask) | ((uint32_t)cell << kCellShift);
        }
        if (!(floor > lntcut)) floor = -INFINITY;  // the cutoff lies inside this cell
      }
      const double lu = log(u);  // one evaluation for the light and heavy measures
      if (heavy) key = log(m2 + (Tch - m2) * exp(lu * invc));
      else key = lnTch + lu * invc;
      if (key < floor) { key = floor; isnull = true; }
      if (key < lntcut) { key = -INFINITY; isnull = false; }
    }
    // the word is written only when its cell or null bit changed, so that a
    // plain redraw dirties no line of the info array
    const uint32_t nw = isnull ? (info | kNullBit) : (info & ~kNullBit);
    if (nw != info0) {
      S.info[oc] = nw;
      S.ent[oc].t.info = nw;
    }
  }
  S.key[oc] = key;
  kout = key;
  return tried;
}

// LDS of one wave for the trial tournament: the winner of each lane's group
// of four entries (bits: entry | exact << 9 | null << 10 | cell << 11 |
// valid << 15) and its trial count.
struct TrialCand {
  double lo, hi, key, u, lnT, invc;
  uint32_t bits, ntri;
};
struct TrialLds {
  TrialCand c[64];
};

// Retained trials: what a lane's event needs for its entries to draw new
// trials while they are built (scale, cycle, id, stream).
struct DrawState {
  double T, lnT;
  int64_t id;
  uint32_t cycle;
  bool lrn;       // learned cells (else the analytic constants)
  uint32_t strm;  // random-number stream of the event
  uint64_t seed;
  bool mec;  // the event's next emission is corrected to the real matrix element
};

// set up the channel constants of up to 64 queued entries, one per lane
// (DRAW: and draw each entry's first trial from its event's scale)
template <bool DRAW>
__device__ __forceinline__ void build_setup(const WaveCtx& W, BuildLds& B, int head, int cnt, int64_t myslot,
                                            const DrawState& D) {
  const bool valid = W.lane < cnt;
  const uint32_t it = valid ? B.ring[(head + W.lane) & (kBuildRing - 1)] : 0u;
  const int L = (int)(it & 63u);
  const int64_t slot = __shfl(myslot, L);
  double TL = 0.0, lnTL = 0.0;
  int64_t idL = 0;
  uint32_t cyL = 0, stL = 0;
  bool lrnL = false;
  if constexpr (DRAW) {
    TL = __shfl(D.T, L); lnTL = __shfl(D.lnT, L); idL = __shfl(D.id, L);
    cyL = (uint32_t)__shfl((int)D.cycle, L); lrnL = __shfl((int)D.lrn, L) != 0;
    stL = (uint32_t)__shfl((int)D.strm, L);
  }
  const bool mecL = __shfl((int)D.mec, L) != 0;
  if (!valid) return;
  const int q = (int)((it >> 6) & 0xFFu), side = (int)((it >> 14) & 1u), k = (int)(it >> 15);
  const Rec R = rec_of(W.S, slot);
  Chan ch;
  chan_setup(W.C, R, q, side, k, ch, mecL);
  const int c = 2 * q + side;
  const int64_t oc = (int64_t)slot * W.S.nch + c;
  const uint32_t pw = pack(ch);
  W.S.info[oc] = pw;
  W.S.ent[oc].t.info = pw;
  W.S.ent[oc].t.tl = ch.tlim;
  W.S.ent[oc].t.ltl = ch.lntlim;
  W.S.ent[oc].t.ic = ch.invc;
  Win wd;
  wd.c = ch.c; wd.s = ch.s; wd.zlo = ch.zlo; wd.omzhi = ch.omzhi; wd.I1 = ch.I1; wd.I2 = ch.I2;
  wd.etap = ch.type == kFI ? ch.etak : ch.eta;
  wd.lnep = ch.lnep;
  wd.lz1 = ch.lz1;
  wd.pid = (uint32_t)(ch.pidi & 0xFF) | ((uint32_t)(ch.pidk & 0xFF) << 8);
  wd.pad0 = 0u;
  W.S.ent[oc].w = wd;
  if constexpr (DRAW) {
    double ub[4];
    rng4(D.seed, stL, idL, cyL, (uint32_t)c >> 2, ub);
    double key;
    if (draw_entry(W.C, W.S, slot, c, pack(ch), ch.tlim, ch.lntlim, ch.invc, pick4(ub, c & 3), TL, lnTL, lrnL,
                   key))
      atomicAdd(&B.count[L], 1u);
  }
}

// The entries a rebuild after a local emission visits: the two of the
// emitter i, of the spectator k and of the new parton j, then the entries
// paired with the old colour partners of the emitter's and the spectator's
// entries (rp: the partner slots of (i, 0), (i, 1), (k, 0), (k, 1), eight bits
// each, i where there was none), each entry once.  Colour partnership is
// mutual: when (q, side) pairs with p, (p, 1 - side) pairs with q, so an entry
// whose old partner was i or k is one of these.  Returns the entry (2 q +
// side) of item e, or for e < 0 the number of items.
__device__ __forceinline__ int partial_item(int e, int i, int k, int j, uint32_t rp) {
  if (e >= 0 && e < 6) {
    const int x = e < 2 ? i : (e < 4 ? k : j);
    return 2 * x + (e & 1);
  }
  int m = 6;
  int seen[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int p = (int)((rp >> (8 * u)) & 0xFFu);
    const int c = 2 * p + ((u & 1) ^ 1);
    bool ok = p != i && p != k && p != j;
#pragma unroll
    for (int v = 0; v < u; ++v) ok = ok && seen[v] != c;
    seen[u] = ok ? c : -1;
    if (ok) {
      if (m == e) return c;
      ++m;
    }
  }
  return e < 0 ? m : -1;
}

// Cooperative (re)build of the channel entries of the events whose lanes are
// set in `mask`.  The entries (slot, side) these events visit are laid end to
// end and the wave walks them 64 at a time: each lane finds the colour partner
// of one entry by scanning its event's colour tags.  Only entries whose
// constants can have changed are set up again: all of them after a refill
// (`all`) or an initial-initial emission (whose recoil boosts every
// final-state momentum), which visit every entry; otherwise those of emitter
// `ei`, spectator `ek` and the new parton n - 1, entries whose partner is one
// of those three, and entries whose partner changed (its old partner was the
// emitter), and only those candidates are visited (partial_item).  The others
// are bitwise what a full set-up would write, because their inputs did not
// change.  Entries to set up are
// queued in LDS and set up 64 at a time, one per lane.  Returns (per lane)
// whether this lane's own event has a broken colour line or a non-finite
// momentum.  DRAW (retained trials): every entry that is set up also draws a
// new trial from its event's scale at its current cycle; an unchanged entry
// keeps its pending trial (its overestimate process is unchanged).  `drawn`
// gets the number of trials drawn for this lane's event.
template <bool DRAW>
__device__ uint32_t coop_build(const WaveCtx& W, BuildLds& B, unsigned long long mask, int n, int64_t myslot,
                               bool fresh, bool all, int ei, int ek, const DrawState& D, uint32_t& drawn) {
  __threadfence_block();
  const bool mine = (mask >> W.lane) & 1ull;
  // after an emission, the old partners of the emitter's and the spectator's
  // entries, read before any entry is rewritten: the candidates of a local
  // rebuild's walk, and (the emitter's) of the partner searches
  uint32_t rp = 0u;
  if (mine && !fresh) {
    const int64_t b = myslot * W.S.nch;
    const uint32_t w0 = W.S.info[b + 2 * ei], w1 = W.S.info[b + 2 * ei + 1];
    const uint32_t w2 = W.S.info[b + 2 * ek], w3 = W.S.info[b + 2 * ek + 1];
    const auto pt = [&](uint32_t w) -> uint32_t { return w ? (w >> 5) & 0xFFu : (uint32_t)ei; };
    rp = pt(w0) | (pt(w1) << 8) | (pt(w2) << 16) | (pt(w3) << 24);
  }
  const int ne = mine ? (all ? 2 * n : partial_item(-1, ei, ek, n - 1, rp)) : 0;
  int incl = ne;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, (unsigned)o);
    if (W.lane >= o) incl += v;
  }
  const int total = __shfl(incl, 63);
  if (mine) B.flags[W.lane] = 0u;
  if constexpr (DRAW) B.count[W.lane] = 0u;
  __builtin_amdgcn_wave_barrier();
  int head = 0, cnt = 0;
  for (int g0 = 0; g0 < total; g0 += 64) {
    const int g = g0 + W.lane;
    // owner lane: the number of lanes whose inclusive prefix is <= g
    int L = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
      const int v = __shfl(incl, L + step - 1);
      if (v <= g) L += step;
    }
    L = L > 63 ? 63 : L;
    const int nL = __shfl(n, L);
    const int firstL = __shfl(incl - ne, L);
    const int64_t slot = __shfl(myslot, L);
    const bool allL = __shfl((int)all, L) != 0, freshL = __shfl((int)fresh, L) != 0;
    const int iL = __shfl(ei, L), kL = __shfl(ek, L);
    const uint32_t rpL = (uint32_t)__shfl((int)rp, L);
    bool queue = false;
    int q = 0, side = 0, k = -1;
    if (g < total) {
      const int e = allL ? g - firstL : partial_item(g - firstL, iL, kL, nL - 1, rpL);
      q = e >> 1;
      side = e & 1;
      const Rec R = rec_of(W.S, slot);
      // its cache word and (for the finiteness check) its parton's momentum:
      // an emission changes only the momenta of its emitter, spectator and
      // new parton, and an initial-initial one (a full build) every
      // final-state momentum, so only those are checked (the others were
      // checked when they last changed)
      const int64_t oc = (int64_t)slot * W.S.nch + e;
      const uint32_t old = W.S.info[oc];
      const int64_t oq = R.o(q);
      const int jL = nL - 1;
      bool fin = true;
      if (side == 0 && (allL || q == iL || q == kL || q == jL))
        fin = isfinite(R.E[oq]) && isfinite(R.px[oq]) && isfinite(R.py[oq]) && isfinite(R.pz[oq]);
      const int kold = old ? (int)((old >> 5) & 0xFFu) : -1;
      // this entry's tag: colour (side 0) or anticolour (side 1), as if outgoing
      const int stq = R.st[oq], clq = R.col[oq], alq = R.acol[oq];
      const int tag = side == 0 ? (stq < 0 ? alq : clq) : (stq < 0 ? clq : alq);
      // After an emission the partner can only be among the emitter, the new
      // parton and the emitter's old partners (no other parton's tags
      // changed), so their opposite tags are read together with the entry's
      // word, in the same memory round trip; the full scan below is the
      // fallback if none of them matches.
      int cand[4], ctag[4];
      if (!freshL) {
        cand[0] = iL;
        cand[1] = jL;
        cand[2] = (int)(rpL & 0xFFu);
        cand[3] = (int)((rpL >> 8) & 0xFFu);
#pragma unroll
        for (int u = 0; u < 4; ++u) ctag[u] = cand[u] < nL ? (side == 0 ? R.effa(cand[u]) : R.effc(cand[u])) : 0;
      }
      // An emission changes colour tags only on the emitter (which only ever
      // takes a new tag) and the new parton (which takes the emitter's old
      // tags or the new one), and each tag sits on exactly one pair of
      // partons.  So another parton keeps its partner unless that partner was
      // the emitter; only those entries, the emitter's and the new parton's
      // search, as every entry of a refilled event does.
      if (freshL || q == iL || q == jL || (old != 0u && kold == iL)) {
        if (tag != 0) {
          if (!freshL) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (cand[u] != q && cand[u] < nL && ctag[u] == tag && (k < 0 || cand[u] < k)) k = cand[u];
          }
          if (k < 0) {
            // the partner: the first other parton whose opposite tag matches,
            // eight partons at a time
            int oth[8];
            for (int j0 = 0; j0 < nL && k < 0; j0 += 8) {
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                const int j = j0 + u;
                oth[u] = j < nL ? (side == 0 ? R.effa(j) : R.effc(j)) : 0;
              }
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                const int j = j0 + u;
                if (k < 0 && j < nL && j != q && oth[u] == tag) k = j;
              }
            }
          }
          if (k < 0) atomicOr(&B.flags[L], fColour);
        }
      } else {
        k = kold;
      }
      if (!fin) atomicOr(&B.flags[L], fNaN);
      const bool dirty = allL || k != kold || q == iL || q == kL || q == jL || k == iL || k == kL || k == jL;
      if (dirty) {
        if (k < 0) {
          W.S.info[oc] = 0u;
          W.S.ent[oc].t.info = 0u;
        }
        else queue = true;
      }
      // retained trials: an unchanged entry keeps its pending trial (its
      // process is unchanged); an entry without a partner has none
      if constexpr (DRAW)
        if (k < 0) W.S.key[oc] = -INFINITY;
    }
    const unsigned long long qm = __ballot(queue);
    if (queue) {
      const int r = __popcll(qm & lanemask_lt(W.lane));
      B.ring[(head + cnt + r) & (kBuildRing - 1)] =
          (uint32_t)L | ((uint32_t)q << 6) | ((uint32_t)side << 14) | ((uint32_t)k << 15);
    }
    cnt += __popcll(qm);
    __builtin_amdgcn_wave_barrier();
    if (cnt >= 64) {
      build_setup<DRAW>(W, B, head, 64, myslot, D);
      head = (head + 64) & (kBuildRing - 1);
      cnt -= 64;
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (cnt > 0) build_setup<DRAW>(W, B, head, cnt, myslot, D);
  __builtin_amdgcn_wave_barrier();
  __threadfence_block();
  if constexpr (DRAW) drawn = mine ? B.count[W.lane] : 0u;
  return mine ? B.flags[W.lane] : 0u;
}

// rebuild the channel description of cache entry c from the cache and record
__device__ __forceinline__ void chan_from_cache(const Cfg& C, const Scratch& S, const Rec& R, int64_t slot, int c,
                                                Chan& ch) {
  const int64_t oc = (int64_t)slot * S.nch + c;
  uint32_t info = S.ent[oc].t.info;
  ch.alive = 1;
  ch.i = c >> 1;
  ch.side = c & 1;
  ch.type = (info >> 1) & 3u;
  ch.heavy = (info >> 3) & 3u;
  ch.k = (info >> 5) & 0xFFu;
  ch.ebin = (info >> 13) & 0x3Fu;
  ch.kbin = (info >> 19) & 0x3Fu;
  ch.mec = (info & kMecBit) != 0u;
  ch.m2 = ch.heavy == 1 ? C.mc2 : (ch.heavy == 2 ? C.mb2 : 0.0);
  const Win wd = S.ent[oc].w;
  const uint32_t pk = wd.pid;
  ch.pidi = (int)(int8_t)(pk & 0xFFu);
  ch.pidk = (int)(int8_t)((pk >> 8) & 0xFFu);
  ch.s = wd.s;
  ch.c = wd.c;
  ch.zlo = wd.zlo;
  ch.omzhi = wd.omzhi;
  ch.zhi = 1.0 - ch.omzhi;
  ch.omzlo = 1.0 - ch.zlo;
  ch.I1 = wd.I1;
  ch.I2 = wd.I2;
  // the winner needs only the PDF ratio's momentum fraction: the emitter's
  // (IF, II) or the spectator's (FI)
  ch.eta = ch.type == kFI ? 0.0 : wd.etap;
  ch.etak = ch.type == kFI ? wd.etap : 0.0;
  ch.lnep = wd.lnep;
  ch.lz1 = wd.lz1;
  ch.nterm = n_terms(ch, C.nf);
}

// Retained trials: the winner entry c of a vetoed or null cycle draws again,
// in its own lane, at the new cycle from the new scale (T, lnT).
// info, tl, ltl, ic: the entry's cache word and trial constants; kout gets
// the new key.
__device__ __forceinline__ bool redraw_winner(const Cfg& C, const Scratch& S, uint64_t seed, uint32_t strm,
                                              int64_t id, uint32_t cycle, int64_t slot, int c, uint32_t info,
                                              double tl, double ltl, double ic, double T, double lnT, bool lrn,
                                              double& kout) {
  double ub[4];
  rng4(seed, strm, id, cycle, (uint32_t)c >> 2, ub);
  return draw_entry(C, S, slot, c, info, tl, ltl, ic, pick4(ub, c & 3), T, lnT, lrn, kout);
}

// batch of global queue index g: the last b with prefix[b] <= g
__device__ __forceinline__ int batch_of(const ShowerArgs& A, int64_t g) {
  int lo = 0, hi = A.nbatch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.prefix[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace

// Wave-uniform values held in vector registers.  The compiler keeps uniform
// values in scalar registers, and the shower kernel runs out of them: its
// arguments and hot constants end up spilled to lanes of vector registers and
// restored (one instruction per dword) at every use.  An empty asm with a
// vector-register operand moves a value into vector registers once, at the
// start; a pointer keeps its global address space by a cast back.
template <typename T>
__device__ __forceinline__ T* vreg_ptr(T* p) {
  uint64_t v = (uint64_t)p;
  asm volatile("" : "+v"(v));
  typedef __attribute__((address_space(1))) T GT;
  return (T*)(GT*)v;
}
__device__ __forceinline__ void vreg(double& d) { asm volatile("" : "+v"(d)); }
__device__ __forceinline__ uint64_t vreg_u64(uint64_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// RETAIN: the retained-trial form of the competition (a losing channel keeps
// its trial; only the winner draws again after a veto or a null, every channel
// after an emission); otherwise every channel draws again each cycle.
template <bool RETAIN>
__device__ __forceinline__ void shower_wave_body(const Cfg& Cg, const gaps_events& in1, const gaps_events& out1,
                                                 const Scratch& Sg, const ShowerArgs& A) {
  // the scratch pointers and the seed in vector registers
  Scratch S = Sg;
  S.part = vreg_ptr(S.part);
  S.ent = vreg_ptr(S.ent);
  S.key = vreg_ptr(S.key);
  S.info = vreg_ptr(S.info);
  S.wfac = vreg_ptr(S.wfac);
  S.pend = vreg_ptr(S.pend);
  const uint64_t seed = vreg_u64(A.seed);
  // the overestimate table, staged in LDS for the term loops
  __shared__ double s_bound[kBoundRows * kNB];
  __shared__ int s_cnt[16], s_nexh;
  __shared__ BuildLds s_build[8];  // one per wave (blocks of at most 512 threads)
  __shared__ TrialLds s_trial[8];
  extern __shared__ LaneState s_pool[];
  for (int q = threadIdx.x; q < kBoundRows * kNB; q += blockDim.x) s_bound[q] = Cg.bound[q];
  if (threadIdx.x == 0) s_nexh = 0;
  __syncthreads();
  Cfg C = Cg;
  C.bound = s_bound;
  // the table pointers and the constants of the draws, the PDF lookups and
  // the coupling in vector registers
  C.learn = vreg_ptr(C.learn);
  C.learn_sd = vreg_ptr(C.learn_sd);
  C.pdf = vreg_ptr(C.pdf);
  vreg(C.t_cut); vreg(C.tc_is); vreg(C.ln_tc); vreg(C.ln_tcis);
  vreg(C.tch_c); vreg(C.ln_tch_c); vreg(C.tch_b); vreg(C.ln_tch_b);
  vreg(C.mc2); vreg(C.mb2);
  vreg(C.lnx0); vreg(C.dlnx); vreg(C.lnq0); vreg(C.dlnq);
  vreg(C.b0); vreg(C.ln_mz2); vreg(C.as_over); vreg(C.over_scale);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t slot = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // every batch's output has at least S.max_slots slots (checked by the host)
  const int M = S.max_slots;
  const WaveCtx W{C, S, lane, M};
  Rec R = rec_of(S, slot);
  const int K = A.compact_every > 0 ? A.compact_every : 8;
  const unsigned KC = A.tail_every > 0 ? (unsigned)A.tail_every : 16u;
  const bool compact = A.tail_every > 0;
  const bool learned_mode = A.mode == GAPS_MODE_LEARNED;
  const bool log_mode = A.mode == GAPS_MODE_LOG;

  bool active = false, exhausted = false, loaded = false, stop = false;
  // this event draws its initial-state channels against the learned bound
  // (LEARNED mode until the bound fails; the event keeps random-number stream 1
  // after that, marked by fFallback in its flags)
  bool lrn = false;
  int64_t e = 0, id = 0;
  int b = 0;
  double T = 0.0, lnT = 0.0, t1 = 0.0;
  uint32_t cycle = 0, ntri = 0, nacc = 0, nviol = 0, flags = 0;
  int n = 0, maxtag = 0;
  // statistics, per lane (summed over the wave once, at the end: wave-uniform
  // accumulators would hold scalar registers, which the loop is short of)
  unsigned long long st_cyc = 0, st_tri = 0, st_acc = 0, st_viol = 0, st_iters = 0, st_active = 0;
  unsigned long long st_fb = 0, st_null = 0;
  int since = 1 << 30;
  int rwait = 0;  // iterations an emission's rebuild has been deferred
  // the accepted emission awaiting its application (pe): its channel entry
  // (bits 0-8), splitting kernel (9-11), flavour + 8 (12-15), dipole type
  // (16-17) and spectator (18-25) in pe_code; z, 1 - z, azimuth, the map
  // variables and the dipole invariant s in the lane slot's pending-emission
  // record (memory: they would otherwise hold twelve registers through the
  // whole loop).  Applying it needs no channel-cache read: the partons'
  // momenta are the only memory round trip.
  bool pe = false;
  uint32_t pe_code = 0u;
  // apply it: the new parton goes to slot n
  auto apply_emission = [&]() {
    const double* P = S.pend + kPendStride * slot;
    const double pz = P[0], pomz = P[1], pphi = P[2], pa1 = P[3], pa2 = P[4], ps = P[5];
    const int c = (int)(pe_code & 0x1FFu);
    Chan ch;
    ch.i = c >> 1;
    ch.side = c & 1;
    ch.type = (int)((pe_code >> 16) & 3u);
    ch.k = (int)((pe_code >> 18) & 0xFFu);
    ch.s = ps;
    emit_map(R, n, maxtag, ch, (int)((pe_code >> 9) & 7u), (int)((pe_code >> 12) & 15u) - 8, pz, pomz, pa1, pa2,
             pphi);
    n += 1;
    pe = false;
  };
  // the last cycle's accepted emission, whose channels are rebuilt at the top
  // of the next iteration together with the refilled lanes
  bool rebuild = false, em_all = false;
  int em_i = 0, em_k = 0;
  // retained trials: the second-largest pending trial (sec_k at entry sec_c)
  // of the last scan, valid while no other entry's trial changed, and the last
  // winner pw with its new trial pk; together they give the next winner
  // without a scan
  bool sec_ok = false;
  int sec_c = -1, pw = -1;
  double sec_k = -INFINITY, pk = -INFINITY;
  bool counted = false, tail = false;
  unsigned it_tail = 0;

  // load the header of event e of batch b; false if the event does not fit
  // this lane's record
  auto load = [&](bool learned) -> bool {
    const gaps_events& in = A.nbatch > 0 ? A.batches[b].in : in1;
    n = in.n[e];
    id = in.id[e];
    flags = in.flags ? in.flags[e] : 0u;
    T = in.t_start[e];
    lnT = log(T);
    t1 = 0.0;
    cycle = ntri = nacc = nviol = 0u;
    maxtag = 0;
    stop = false;
    lrn = learned;
    if (n < 0 || n > M || n > in.max_slots) {
      flags |= fOverflow;
      stop = true;
      loaded = false;
      return false;
    }
    loaded = true;
    return true;  // the partons are copied by the whole wave (below)
  };

  bool owed = false;
  // write out the events of the owed lanes (finished, not yet written): the
  // headers per lane, then the partons one per lane over the whole wave
  auto flush_owed = [&]() {
    if (owed) {
      const gaps_events& in = A.nbatch > 0 ? A.batches[b].in : in1;
      const gaps_events& out = A.nbatch > 0 ? A.batches[b].out : out1;
      const int64_t co = out.cap;
      const int nin = in.n[e];
      const bool fits = loaded;
      out.id[e] = id;
      // a violated learned bound leaves the weighted veto's factor on the event
      out.w[e] = (flags & fFallback) ? in.w[e] * S.wfac[slot] : in.w[e];
      out.t_start[e] = in.t_start[e];
      if (fits) {
        out.n[e] = n;
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
    }
    if (owed) {
      st_cyc += cycle;
      st_tri += ntri;
      st_acc += nacc;
      st_viol += nviol;
    }
    {
      // finished events' partons to their outputs, one parton per lane
      const int np = owed && loaded ? n : 0;
      const int incl = wave_incl(np, lane);
      const int total = __shfl(incl, 63);
      for (int g0 = 0; g0 < total; g0 += 64) {
        const int g = g0 + lane;
        const int L = owner_of(incl, g);
        const int nL = __shfl(n, L), fL = __shfl(incl, L) - nL, bL = __shfl(b, L);
        const int64_t sL = __shfl(slot, L), eL = __shfl(e, L);
        if (g < total) {
          const gaps_events& out = A.nbatch > 0 ? A.batches[bL].out : out1;
          const int q = g - fL;
          const int64_t k = (int64_t)q * out.cap + eL, o = rec_of(S, sL).o(q);
          const Part pt = S.part[o];
          out.E[k] = pt.E; out.px[k] = pt.px; out.py[k] = pt.py; out.pz[k] = pt.pz;
          out.pid[k] = pt.pid; out.col[k] = pt.col; out.acol[k] = pt.acol; out.status[k] = pt.st;
        }
      }
    }
    owed = false;
  };

  for (unsigned it = 0;; ++it) {
    if (__ballot(owed) && (exhausted || since >= K || __ballot(active) == 0ull)) flush_owed();
    // ---- tail mode starts when every wave of the block has seen the queue empty
    if (compact && !tail && exhausted) {
      if (!counted) {
        if (lane == 0) atomicAdd(&s_nexh, 1);
        counted = true;
      }
      tail = __builtin_amdgcn_readfirstlane(*(volatile int*)&s_nexh) == nw;
      if (tail) it_tail = it;
    }
    // ---- tail mode: block bookkeeping, termination and compaction
    if (tail && (it - it_tail) % KC == 0u) {
      const bool live = active;
      const unsigned long long a0 = __ballot(live);
      if (lane == 0) s_cnt[wid] = __popcll(a0);
      __syncthreads();
      int total = 0, used = 0, prefix = 0;
      for (int w = 0; w < nw; ++w) {
        const int cw = s_cnt[w];
        if (w < wid) prefix += cw;
        total += cw;
        used += cw > 0 ? 1 : 0;
      }
      if (total == 0) break;
      if ((total + 63) / 64 < used) {
        if (pe) apply_emission();  // the lane state does not carry a pending emission
        if (live) {
          LaneState& X = s_pool[prefix + __popcll(a0 & lanemask_lt(lane))];
          X.e = e; X.id = id; X.slot = slot; X.b = b; X.lrn = lrn; X.T = T; X.lnT = lnT; X.t1 = t1;
          X.cycle = cycle; X.ntri = ntri; X.nacc = nacc; X.nviol = nviol; X.flags = flags;
          X.n = n; X.maxtag = maxtag;
          X.bits = (uint32_t)loaded | ((uint32_t)stop << 1) | ((uint32_t)rebuild << 3) | ((uint32_t)em_all << 4);
          X.emik = (em_i & 0xFF) | ((em_k & 0xFF) << 8);
        }
        __syncthreads();
        const bool got = (int)threadIdx.x < total;
        active = false;
        rebuild = false;
        sec_ok = false;
        if (got) {
          const LaneState& X = s_pool[threadIdx.x];
          e = X.e; id = X.id; slot = X.slot; b = X.b; lrn = X.lrn != 0; T = X.T; lnT = X.lnT; t1 = X.t1;
          cycle = X.cycle; ntri = X.ntri; nacc = X.nacc; nviol = X.nviol; flags = X.flags;
          n = X.n; maxtag = X.maxtag;
          loaded = (X.bits & 1u) != 0; stop = (X.bits & 2u) != 0;
          rebuild = (X.bits & 8u) != 0; em_all = (X.bits & 16u) != 0;
          em_i = X.emik & 0xFF; em_k = (X.emik >> 8) & 0xFF;
          active = true;
          R = rec_of(S, slot);
        }
      }
      __syncthreads();
    }
    // ---- refill finished lanes from the work queue (one atomic per wave)
    unsigned long long act = __ballot(active);
    bool fresh = false;
    if (!exhausted && (since >= K || act == 0ull)) {
      const unsigned long long idle = ~act;
      const int cnt = __popcll(idle);
      unsigned long long base = 0ull;
      if (lane == 0) base = atomicAdd(S.queue, (unsigned long long)cnt);
      base = __shfl(base, 0);
      if (base + (unsigned long long)cnt >= (unsigned long long)A.n) exhausted = true;
      if (!active) {
        const unsigned long long ev = base + (unsigned long long)__popcll(idle & lanemask_lt(lane));
        if (ev < (unsigned long long)A.n) {
          b = A.nbatch > 0 ? batch_of(A, (int64_t)ev) : 0;
          e = (int64_t)ev - (A.nbatch > 0 ? A.prefix[b] : 0);
          active = true;
          fresh = load(learned_mode);
        }
      }
      since = 0;
      act = __ballot(active);
      // the refilled events' partons into their records, one parton per lane,
      // and the largest colour tag of each event
      const int np = fresh ? n : 0;
      const int incl = wave_incl(np, lane);
      const int total = __shfl(incl, 63);
      if (total > 0) {
        BuildLds& B = s_build[wid];
        B.tag[lane] = 0;
        __builtin_amdgcn_wave_barrier();
        for (int g0 = 0; g0 < total; g0 += 64) {
          const int g = g0 + lane;
          const int L = owner_of(incl, g);
          const int nL = __shfl(n, L), fL = __shfl(incl, L) - nL, bL = __shfl(b, L);
          const int64_t sL = __shfl(slot, L), eL = __shfl(e, L);
          if (g < total) {
            const gaps_events& in = A.nbatch > 0 ? A.batches[bL].in : in1;
            const int q = g - fL;
            const int64_t k = (int64_t)q * in.cap + eL, o = rec_of(S, sL).o(q);
            const int cl = in.col[k], al = in.acol[k];
            Part pt;
            pt.E = in.E[k]; pt.px = in.px[k]; pt.py = in.py[k]; pt.pz = in.pz[k];
            pt.pid = in.pid[k]; pt.col = cl; pt.acol = al; pt.st = in.status[k];
            pt.pad0 = pt.pad1 = pt.pad2 = 0;
            S.part[o] = pt;
            atomicMax(&B.tag[L], cl > al ? cl : al);
          }
        }
        __builtin_amdgcn_wave_barrier();
        if (fresh) maxtag = B.tag[lane];
      }
    }
    // ---- one cooperative channel build for the refilled lanes and the lanes
    // that emitted in the last cycle.  A broken colour line stops a refilled
    // event before its first cycle; after an emission a non-finite momentum
    // (reported first) or a broken colour line stops the event (its cycle
    // was already counted).
    // A build pass costs about the same for one lane as for many (its memory
    // round trips), so the rebuilds after emissions wait, without trialing,
    // until kDeferLanes lanes want one, one has waited kDeferWait iterations,
    // fewer than kDeferMin other lanes are left to trial, or refilled lanes
    // are built anyway.  Results do not depend on it (every draw is keyed by
    // the event id and cycle).
    bool go = true;
    {
      const unsigned long long rm = __ballot(rebuild);
      if (rm && !__ballot(fresh)) {
        const bool aged = __ballot(rebuild && rwait >= kDeferWait) != 0ull;
        go = aged || __popcll(rm) >= kDeferLanes || __popcll(__ballot(active) & ~rm) < kDeferMin;
      }
      rwait = rebuild ? rwait + 1 : 0;
    }
    const bool built = fresh || (rebuild && go);
    if (built) sec_ok = false;
    if (built && pe) apply_emission();
    {
      const unsigned long long bm = __ballot(built);
      if (bm) {
        const DrawState D{T, lnT, id, cycle, lrn, (lrn || (flags & fFallback)) ? 1u : 0u, seed,
                          (flags & fMEC) != 0u && t1 == 0.0};
        uint32_t drawn = 0;
        uint32_t f =
            coop_build<RETAIN>(W, s_build[wid], bm, n, slot, fresh, fresh || em_all, em_i, em_k, D, drawn);
        if (fresh) f &= fColour;
        if (f & fNaN) f = fNaN;
        // an event stopped here draws nothing (its draws are not counted)
        if (built && f) { flags |= f; stop = true; }
        else ntri += drawn;
        if (built) rebuild = false;
      }
    }
    if (act == 0ull) {
      if (!compact && exhausted) break;  // no tail mode: a drained wave just leaves
      if (exhausted && !tail) __builtin_amdgcn_s_sleep(2);
      continue;
    }
    st_iters += 1ull;
    st_active += active ? 1ull : 0ull;

    // ---- one cycle of the veto algorithm on every active lane
    bool done = false;
    if (active && stop) done = true;
    if (active && !done && cycle >= kMaxCycles) { flags |= fMaxCyc; done = true; }
    // Trial scales of every channel and the winner (largest key = ln t, ties
    // to the lowest entry), for every lane that has a cycle to run.  Each key
    // is first bounded with the hardware single-precision log of u and a
    // rigorous error margin; the double-precision log is taken only where the
    // bounds cannot decide (overlapping candidates, the cutoff, a cell edge)
    // and for the final winner, so the result is exactly that of evaluating
    // every key in double precision.  In learned mode an initial-state channel
    // of the incoming partons draws against its cell constant, and a trial
    // below the cell is a null candidate at the cell's lower edge.
    //
    // The work is spread over the whole wave: the events' groups of four
    // entries (one random block each) are laid end to end and taken 64 at a
    // time, one per lane, so that a lane whose event has few channels works on
    // another event's groups instead of idling.  Each group yields its own
    // winner; the owner lane of each event then merges its groups' winners in
    // entry order with the same rule, which gives the same winner as one pass
    // over all entries.
    const bool trialing = active && !done && !rebuild;  // a deferred rebuild waits
    const uint32_t strm = (lrn || (flags & fFallback)) ? 1u : 0u;
    int win = -1, wcell = 0;
    bool wexact = false, wnull = false;
    double wlo = 0.0, whi = 0.0, wkey = RETAIN ? -INFINITY : 0.0, wu = 0.5, wlnT = 0.0, winv = 0.0;
    uint32_t rinfo = 0u;
    double rtl = 0.0, rltl = 0.0, ric = 0.0;
    if constexpr (RETAIN) {
      // ---- retained trials: the winner is the largest pending trial, ties
      // to the lowest entry.  An event whose cached second-largest trial is
      // valid takes the larger of it and its last winner's new trial; the
      // others scan their entries, in groups of kScanGroup (one 128-byte line
      // of keys) spread over the wave, one group per lane, and each owner
      // merges its groups' two largest in order (keeping the two largest for
      // the cache).  A pass over 64 groups costs one memory round trip, and
      // some lane scans in almost every iteration, so the groups are large.
      TrialLds& TQ = s_trial[wid];
      const bool scan = trialing && !sec_ok;
      const int ng = scan ? (2 * n + kScanGroup - 1) / kScanGroup : 0;
      const int incl = wave_incl(ng, lane);
      const int total = __shfl(incl, 63);
      const int first = incl - ng;
      double k2 = -INFINITY;
      int c2 = -1;
      for (int g0 = 0; g0 < total; g0 += 64) {
        const int g = g0 + lane;
        const int L = owner_of(incl, g);
        const int64_t sL = __shfl(slot, L);
        const int nL = __shfl(n, L), fL = __shfl(first, L);
        double b1 = -INFINITY, b2 = -INFINITY;
        int i1 = -1, i2 = -1;
        if (g < total) {
          const int c0 = kScanGroup * (g - fL);
          const double* kr = S.key + (int64_t)sL * S.nch + c0;
          double kk[kScanGroup];
          if (c0 + kScanGroup <= S.nch) {
            // the whole group lies in the event's row: one vector load per
            // two keys, entries past the event's masked afterwards
            const double2* k2 = reinterpret_cast<const double2*>(kr);
#pragma unroll
            for (int j = 0; j < kScanGroup / 2; ++j) {
              const double2 v = k2[j];
              kk[2 * j] = v.x;
              kk[2 * j + 1] = v.y;
            }
#pragma unroll
            for (int j = 0; j < kScanGroup; ++j)
              if (c0 + j >= 2 * nL) kk[j] = -INFINITY;
          } else {
#pragma unroll
            for (int j = 0; j < kScanGroup; ++j) kk[j] = c0 + j < 2 * nL ? kr[j] : -INFINITY;
          }
#pragma unroll
          for (int j = 0; j < kScanGroup; ++j) {
            const double k = kk[j];
            if (k > b1) { b2 = b1; i2 = i1; b1 = k; i1 = c0 + j; }
            else if (k > b2) { b2 = k; i2 = c0 + j; }
          }
        }
        TQ.c[lane].key = b1;
        TQ.c[lane].bits = (uint32_t)i1;
        TQ.c[lane].hi = b2;
        TQ.c[lane].ntri = (uint32_t)i2;
        __builtin_amdgcn_wave_barrier();
        if (scan) {
          const int kb = (first > g0 ? first : g0) - g0;
          const int ke = (incl < g0 + 64 ? incl : g0 + 64) - g0;
          for (int k = kb; k < ke; ++k) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const double y = h == 0 ? TQ.c[k].key : TQ.c[k].hi;
              const int yi = (int)(h == 0 ? TQ.c[k].bits : TQ.c[k].ntri);
              if (y > wkey) { k2 = wkey; c2 = win; wkey = y; win = yi; }
              else if (y > k2) { k2 = y; c2 = yi; }
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
      if (scan) {
        sec_k = k2;
        sec_c = c2;
        sec_ok = true;
      } else if (trialing) {
        // every entry other than pw and sec_c is at most sec_k (and after sec_c
        // if equal): the winner is the larger of the two, ties to the lower entry
        if (pk > sec_k || (pk == sec_k && pw < sec_c)) {
          wkey = pk;
          win = pw;
        } else {
          wkey = sec_k;
          win = sec_c;
          sec_ok = false;  // the next winner needs a scan
        }
        if (!(wkey > -INFINITY)) win = -1;
      }
      if (trialing && win >= 0) {
        // the winner's entry: null and cell bits now, trial constants for its
        // redraw after a veto (loaded together, one memory round trip)
        const int64_t ow = (int64_t)slot * S.nch + win;
        rinfo = S.ent[ow].t.info;
        rtl = S.ent[ow].t.tl;
        rltl = S.ent[ow].t.ltl;
        ric = S.ent[ow].t.ic;
        wnull = (rinfo & kNullBit) != 0u;
        wcell = (int)((rinfo & kCellMask) >> kCellShift);
      }
      wexact = true;
    } else {
      TrialLds& TQ = s_trial[wid];
      const int ng = trialing ? (2 * n + 3) >> 2 : 0;
      int incl = ng;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, (unsigned)o);
        if (lane >= o) incl += v;
      }
      const int total = __shfl(incl, 63);
      const int first = incl - ng;
      for (int g0 = 0; g0 < total; g0 += 64) {
        const int g = g0 + lane;
        int L = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const int v = __shfl(incl, L + step - 1);
          if (v <= g) L += step;
        }
        L = L > 63 ? 63 : L;
        const int64_t sL = __shfl(slot, L);
        const int64_t idL = __shfl(id, L);
        const uint32_t cyL = (uint32_t)__shfl((int)cycle, L);
        const double TL = __shfl(T, L), lnTL = __shfl(lnT, L);
        const int nL = __shfl(n, L), fL = __shfl(first, L);
        const bool lrnL = __shfl((int)lrn, L) != 0;
        const uint32_t stL = (uint32_t)__shfl((int)strm, L);
        // this lane's group: its winner (gw < 0: none) and trial count
        int gw = -1, gcell = 0;
        bool gexact = false, gnull = false;
        double glo = 0.0, ghi = 0.0, gkey = 0.0, gu = 0.5, glnT = 0.0, ginv = 0.0;
        uint32_t gtri = 0;
        if (g < total) {
          const int c0 = 4 * (g - fL);
          uint32_t inf[4];
          double tl[4], ltl[4], ic[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int64_t oc = (int64_t)sL * S.nch + (c0 + j);
            inf[j] = S.info[oc];
            tl[j] = S.ent[oc].t.tl;
            ltl[j] = S.ent[oc].t.ltl;
            ic[j] = S.ent[oc].t.ic;
          }
          if ((inf[0] | inf[1] | inf[2] | inf[3]) & 1u) {
            double ub[4];
            rng4(seed, stL, idL, cyL, (uint32_t)c0 >> 2, ub);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int c = c0 + j;
              const uint32_t info = pick4(inf, j);
              if (c >= 2 * nL || !(info & 1u)) continue;
              const int type = (info >> 1) & 3u, heavy = (info >> 3) & 3u;
              double tcut, lntcut, m2 = 0.0;
              if (heavy == 1) { tcut = C.tch_c; lntcut = C.ln_tch_c; m2 = C.mc2; }
              else if (heavy == 2) { tcut = C.tch_b; lntcut = C.ln_tch_b; m2 = C.mb2; }
              else if (type == kFF) { tcut = C.t_cut; lntcut = C.ln_tc; }
              else { tcut = C.tc_is; lntcut = C.ln_tcis; }
              const double Tch = TL < pick4(tl, j) ? TL : pick4(tl, j);
              const double lnTch = lnTL < pick4(ltl, j) ? lnTL : pick4(ltl, j);
              if (!(Tch > tcut)) continue;
              gtri += 1;
              const double u = pick4(ub, j);
              double invc = pick4(ic, j), floor = -INFINITY;
              int cell = 0;
              if (lrnL && c < 4 && (type == kIF || type == kII)) {
                cell = cell_of(C, lnTch, floor);
                if ((int)((info & kCellMask) >> kCellShift) != cell) {
                  // the scale entered a new cell: that cell's constant replaces the
                  // entry's (1/c for the trials, c for the winner's term choice)
                  const int64_t oc = (int64_t)sL * S.nch + c;
                  const Win& wd = S.ent[oc].w;
                  double lr[2];
                  const double ck = learned_c2(C, type, (int)(int8_t)(wd.pid & 0xFFu), (int)((info >> 13) & 0x3Fu),
                                               wd.I1, wd.I2, cell, (info & kMecBit) != 0u, lr);
                  invc = 1.0 / ck;
                  S.ent[oc].t.ic = invc;
                  S.ent[oc].w.c = ck;
                  S.ent[oc].lr[0] = lr[0];
                  S.ent[oc].lr[1] = lr[1];
                  const uint32_t nw = (info & ~kCellMask) | ((uint32_t)cell << kCellShift);
                  S.info[oc] = nw;
                  S.ent[oc].t.info = nw;
                }
                if (!(floor > lntcut)) floor = -INFINITY;  // the cutoff lies inside this cell
              }
              double lo, hi, key = 0.0;
              bool exact, isnull = false;
              if (heavy) {
                key = log(m2 + (Tch - m2) * exp(log(u) * invc));
                if (key < floor) { key = floor; isnull = true; }
                if (key < lntcut) continue;
                lo = hi = key;
                exact = true;
              } else {
                const double lf = (double)__builtin_amdgcn_logf((float)u) * 0.69314718055994530942;
                const double ka = lnTch + lf * invc;
                const double err = invc * (fabs(lf) * 0x1p-17 + 0x1p-19) + 1e-12;
                lo = ka - err;
                hi = ka + err;
                exact = false;
                if (hi < floor) {
                  key = floor; lo = hi = key; exact = true; isnull = true;
                } else if (lo < floor) {
                  key = lnTch + log(u) * invc;
                  if (key < floor) { key = floor; isnull = true; }
                  lo = hi = key;
                  exact = true;
                }
                if (hi < lntcut) continue;
                if (lo < lntcut) {
                  key = lnTch + log(u) * invc;
                  if (key < lntcut) continue;
                  lo = hi = key;
                  exact = true;
                }
              }
              if (gw >= 0) {
                if (hi <= glo) continue;
                if (!(lo > ghi)) {
                  // the bounds overlap: decide with exact keys (a null key is exact)
                  if (!gexact) { gkey = glnT + log(gu) * ginv; glo = ghi = gkey; gexact = true; }
                  if (!exact) { key = lnTch + log(u) * invc; lo = hi = key; exact = true; }
                  if (!(key > gkey)) continue;
                }
              }
              gw = c; glo = lo; ghi = hi; gkey = key; gexact = exact; gu = u; glnT = lnTch; ginv = invc;
              gnull = isnull; gcell = cell;
            }
          }
        }
        TrialCand& X = TQ.c[lane];
        X.lo = glo; X.hi = ghi; X.key = gkey; X.u = gu; X.lnT = glnT; X.invc = ginv;
        X.bits = (uint32_t)(gw & 0x1FF) | ((uint32_t)gexact << 9) | ((uint32_t)gnull << 10) |
                 ((uint32_t)gcell << 11) | ((uint32_t)(gw >= 0) << 15);
        X.ntri = gtri;
        __builtin_amdgcn_wave_barrier();
        // owner: merge the winners of this event's groups in this pass, in order
        if (trialing) {
          const int kb = (first > g0 ? first : g0) - g0;
          const int ke = (incl < g0 + 64 ? incl : g0 + 64) - g0;
          for (int k = kb; k < ke; ++k) {
            const TrialCand& Y = TQ.c[k];
            ntri += Y.ntri;
            const uint32_t yb = Y.bits;
            if (!(yb & (1u << 15))) continue;
            double lo = Y.lo, hi = Y.hi, key = Y.key;
            bool exact = (yb >> 9) & 1u;
            if (win >= 0) {
              if (hi <= wlo) continue;
              if (!(lo > whi)) {
                if (!wexact) { wkey = wlnT + log(wu) * winv; wlo = whi = wkey; wexact = true; }
                if (!exact) { key = Y.lnT + log(Y.u) * Y.invc; lo = hi = key; exact = true; }
                if (!(key > wkey)) continue;
              }
            }
            win = (int)(yb & 0x1FFu); wlo = lo; whi = hi; wkey = key; wexact = exact; wu = Y.u; wlnT = Y.lnT;
            winv = Y.invc; wnull = (yb >> 10) & 1u; wcell = (int)((yb >> 11) & 15u);
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
      // learned mode: cell constants written by one lane are read by the owner
      if (learned_mode) __threadfence_block();
    }
    bool rdw = false;  // retained trials: the winner of a vetoed or null cycle draws again
    bool nulled = false, fellback = false;  // this cycle: a null winner, a failed learned bound
    if (trialing) {
      double best = -INFINITY;
      if (win >= 0) best = wexact ? wkey : wlnT + log(wu) * winv;
      // the winner's scale, one evaluation for null and real winners alike
      const double tbest = win >= 0 ? exp(best) : 0.0;
      if (win < 0) {
        done = true;
      } else if (wnull) {
        // no channel emits above the cell edge: continue the evolution from it
        T = tbest;
        lnT = best;
        cycle += 1;
        nulled = true;
        rdw = true;
      } else {
        const double t = tbest;
        Chan ch;
        chan_from_cache(C, S, R, slot, win, ch);
        const bool lch = lrn && win < 4 && (ch.type == kIF || ch.type == kII);
        double u[4];
        rng4(seed, strm, id, cycle, 0xFFFFFFFFu, u);
        // a learned channel's cached c is that of its current cell (the winner's)
        double lr[2] = {0.0, 0.0};
        if (lch) {
          lr[0] = S.ent[(int64_t)slot * S.nch + win].lr[0];
          lr[1] = S.ent[(int64_t)slot * S.nch + win].lr[1];
        }
        const Term tm = select_term(C, ch, u[0], lch, wcell, ch.c, lr);
        double z, omz;
        shape_sample(tm.shape, ch, tm.I, u[1], z, omz);
        const double phi = 2.0 * kPi * u[2];
        const Veto v = veto_weight(C, R, ch, tm, t, best, z, omz);
        if (log_mode) {
          // trial log: one atomic for the lanes of this branch that log
          const bool dolog = (ch.type == kIF || ch.type == kII) && !ch.mec && v.ok && v.wn > 0.0;
          const unsigned long long lm = __ballot(dolog);
          if (lm) {
            const int leader = __ffsll((long long)lm) - 1;
            unsigned long long base = 0ull;
            if (lane == leader) base = atomicAdd(A.log_count, (unsigned long long)__popcll(lm));
            base = __shfl(base, leader);
            const unsigned long long r = base + (unsigned long long)__popcll(lm & lanemask_lt(lane));
            if (dolog && r < (unsigned long long)A.log_cap) {
              float* row = A.log + 5ull * r;
              row[0] = (float)log(t); row[1] = (float)ch.lnep; row[2] = (float)z;
              row[3] = (float)tm.ent; row[4] = (float)log(v.wn);
            }
          }
        }
        // A weight above the learned bound goes through the weighted veto
        // (Lonnblad, Eur. Phys. J. C 73 (2013) 2350): accepted with probability
        // w/(2w - 1), the event weight multiplied by 2w - 1 on acceptance and by
        // -(2w - 1) on rejection, which keeps the emission density exact; the
        // event then continues on the analytic overestimate (every channel set
        // up and drawn again by a full rebuild), so it meets no further learned
        // bound.  A weight above the analytic bound is counted and accepted.
        bool acc;
        if (lch && v.ok && v.w > 1.0) {
          const double g = 2.0 * v.w - 1.0;
          acc = u[3] < v.w / g;
          S.wfac[slot] = acc ? g : -g;
          flags |= fFallback;
          lrn = false;
          fellback = true;
        } else {
          if (v.ok && v.w > 1.0) { nviol += 1; flags |= fViol; }
          acc = v.ok && u[3] < v.w;
        }
        if (acc) {
          if (n + 1 > M) {
            flags |= fOverflow;
            done = true;
          } else {
            // the emission is applied by the next channel build, together
            // with the other lanes' (one pass of the emission code for all)
            pe_code = (uint32_t)win | ((uint32_t)tm.kern << 9) | ((uint32_t)(tm.flav + 8) << 12) |
                      ((uint32_t)ch.type << 16) | ((uint32_t)ch.k << 18);
            double a1, a2;
            map_vars(ch.type, v, a1, a2);
            double* P = S.pend + kPendStride * slot;
            P[0] = z;
            P[1] = omz;
            P[2] = phi;
            P[3] = a1;
            P[4] = a2;
            P[5] = ch.s;
            pe = true;
            // an initial-initial recoil boosts every final-state momentum
            rebuild = true;
            em_all = ch.type == kII;
            em_i = ch.i;
            em_k = ch.k;
            nacc += 1;
            if (t1 == 0.0) t1 = t;
          }
        }
        if (fellback) {
          rebuild = true;
          em_all = true;
        }
        if (!done) {
          T = t;
          lnT = best;
          cycle += 1;
          // retained trials: after a veto only the winner draws again
          rdw = !rebuild;
        }
      }
    }
    if constexpr (RETAIN)
      if (rdw) {
        ntri += redraw_winner(C, S, seed, strm, id, cycle, slot, win, rinfo, rtl, rltl, ric, T, lnT, lrn, pk)
                    ? 1u : 0u;
        pw = win;
      }
    st_null += nulled ? 1ull : 0ull;
    st_fb += fellback ? 1ull : 0ull;
    // ---- finished events: their outputs are owed until the next flush (a
    // pass for all of them: before the next refill, or at once when the
    // queue is drained)
    if (active && done && pe) apply_emission();  // stopped while its rebuild waited
    if (active && done) {
      owed = true;
      active = false;
    }
    since += 1;
  }
  if (A.stats) {  // wave totals, one atomic each
    const unsigned long long v[8] = {wave_total(st_cyc), wave_total(st_tri), wave_total(st_acc), wave_total(st_viol),
                                     wave_total(st_iters), wave_total(st_active), wave_total(st_fb),
                                     wave_total(st_null)};
    if (lane == 0)
      for (int k = 0; k < 8; ++k) atomicAdd(A.stats + k, v[k]);
  }
}

// The same body at three register budgets (waves resident per SIMD): more
// waves hide more latency, fewer registers per wave spill more.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
k_shower_wave(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A) {
  shower_wave_body<false>(C, in, out, S, A);
}
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
k_shower_wave_rt(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A) {
  shower_wave_body<true>(C, in, out, S, A);
}
// retained trials at three waves per SIMD (blocks of 384 threads, two per CU)
__global__ void __launch_bounds__(384) __attribute__((amdgpu_waves_per_eu(3)))
k_shower_wave_rt3(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A) {
  shower_wave_body<true>(C, in, out, S, A);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_shower_wave3(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A) {
  shower_wave_body<false>(C, in, out, S, A);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_shower_wave4(Cfg C, gaps_events in, gaps_events out, Scratch S, ShowerArgs A) {
  shower_wave_body<false>(C, in, out, S, A);
}

}  // namespace gaps
