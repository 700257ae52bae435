// Host side of the C-ABI declared in include/gaps.h.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "kernels.hpp"

using gaps::Cfg;

#define GAPS_HIP(call)                       \
  do {                                       \
    if ((call) != hipSuccess) return GAPS_EHIP; \
  } while (0)

namespace {

bool bad_events(const gaps_events* e, int64_t n, int min_slots) {
  if (!e || n < 0 || e->cap < n) return true;
  if (n == 0) return false;  // nothing to touch: the arrays may be empty
  if (e->max_slots < min_slots || e->max_slots > gaps::kMaxSlots) return true;
  return !e->id || !e->w || !e->t_start || !e->n || !e->flags || !e->E || !e->px || !e->py || !e->pz ||
         !e->pid || !e->col || !e->acol || !e->status;
}

unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Per-lane shower scratch held in one allocation (grown on demand).
struct ScratchMem {
  void* mem = nullptr;
  size_t bytes = 0;
  gaps::Scratch S{};
};

// bytes of per-lane working storage for events of `slots` slots
size_t scratch_per_lane(int slots) {
  const int nch = (2 * slots + 3) & ~3;  // whole chunks of four entries
  return (size_t)slots * sizeof(gaps::Part) +
         (size_t)nch * (sizeof(gaps::Ent) + sizeof(double) + sizeof(uint32_t)) + (1 + gaps::kPendStride) * sizeof(double);
}

// bytes the working storage of `lanes` lanes needs, alignment included
size_t scratch_bytes(int64_t lanes, int slots) { return scratch_per_lane(slots) * (size_t)lanes + 256 * 10 + 64; }

// Lay out the working storage of `lanes` lanes over [base, base + bytes).
gaps_status scratch_layout(char* base, size_t bytes, int64_t lanes, int slots, gaps::Scratch& S) {
  const int nch = (2 * slots + 3) & ~3;
  char* p = base;
  auto take = [&](size_t n) {
    char* r = p;
    p += (n + 255) & ~(size_t)255;
    return (void*)r;
  };
  S.lanes = lanes;
  S.max_slots = slots;
  const size_t ps = (size_t)slots * lanes, cs = (size_t)nch * lanes;
  S.part = (gaps::Part*)take(ps * sizeof(gaps::Part));
  S.nch = nch;
  S.ent = (gaps::Ent*)take(cs * sizeof(gaps::Ent));
  S.key = (double*)take(cs * sizeof(double));
  S.info = (uint32_t*)take(cs * sizeof(uint32_t));
  S.wfac = (double*)take((size_t)lanes * sizeof(double));
  S.pend = (double*)take((size_t)gaps::kPendStride * lanes * sizeof(double));
  S.queue = (unsigned long long*)take(64);
  return (size_t)(p - base) > bytes ? GAPS_ECAPACITY : GAPS_OK;
}

gaps_status ensure_scratch(ScratchMem& m, int64_t lanes, int slots) {
  const size_t need = scratch_bytes(lanes, slots);
  if (need > m.bytes || m.S.lanes != lanes || m.S.max_slots != slots) {
    if (need > m.bytes) {
      if (m.mem) (void)hipFree(m.mem);
      m.mem = nullptr;
      m.bytes = 0;
      if (hipMalloc(&m.mem, need) != hipSuccess) return GAPS_ENOMEM;
      m.bytes = need;
    }
    if (scratch_layout((char*)m.mem, m.bytes, lanes, slots, m.S) != GAPS_OK) return GAPS_ENOMEM;
  }
  return GAPS_OK;
}

// The working storage of gaps_shower_noalloc: a static device array, one per
// GPU (its name on the host is only a stand-in; kernels get the device
// address that gaps_init resolves per device with hipGetSymbolAddress).
static __device__ __align__(256) unsigned char scratch[GAPS_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// resolve the array's address on the current device (once per device)
gaps_status resolve_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return GAPS_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return GAPS_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GAPS_EHIP;
  g_scratch_ptr[device] = ptr;
  return GAPS_OK;
}

void* static_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

// Device copy of a stream's batch table and its offsets (grown on demand).
struct BatchMem {
  gaps_batch* table = nullptr;
  int64_t* prefix = nullptr;
  int cap = 0;
};

gaps_status ensure_batches(BatchMem& m, int nbatch) {
  if (nbatch <= m.cap) return GAPS_OK;
  if (m.table) (void)hipFree(m.table);
  if (m.prefix) (void)hipFree(m.prefix);
  m.table = nullptr;
  m.prefix = nullptr;
  m.cap = 0;
  if (hipMalloc((void**)&m.table, sizeof(gaps_batch) * (size_t)nbatch) != hipSuccess) return GAPS_ENOMEM;
  if (hipMalloc((void**)&m.prefix, sizeof(int64_t) * ((size_t)nbatch + 1)) != hipSuccess) return GAPS_ENOMEM;
  m.cap = nbatch;
  return GAPS_OK;
}

void free_batches(BatchMem& m) {
  if (m.table) (void)hipFree(m.table);
  if (m.prefix) (void)hipFree(m.prefix);
  m = BatchMem{};
}

}  // namespace

struct gaps_ctx_s {
  gaps_config cfg;
  Cfg C;
  int device = 0;
  int cus = 0;
  float* d_pdf = nullptr;
  double* d_bound = nullptr;
  ScratchMem scratch;  // shower scratch, grown on demand
  BatchMem batches;    // batch table of gaps_shower_stream
  // learned-bound network: one allocation for weights, Adam state, margins, table
  void* mlp_mem = nullptr;
  float *theta = nullptr, *mom1 = nullptr, *mom2 = nullptr, *grad = nullptr;
  uint16_t* wb = nullptr;
  double *delta = nullptr, *table = nullptr, *table_sd = nullptr;
  unsigned long long *maxbits = nullptr, *count = nullptr;
  float *probe_x = nullptr, *probe_f = nullptr;
  // cell-maximum bound: per-cell largest target and row count, per-entry
  // largest held-out excess and row count
  unsigned long long* cm_mem = nullptr;
  int64_t adam_step = 0;
};

struct gaps_graph_s {
  ScratchMem scratch;
  BatchMem batches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* gaps_strerror(gaps_status s) {
  switch (s) {
    case GAPS_OK: return "ok";
    case GAPS_EINVAL: return "invalid argument";
    case GAPS_ENOMEM: return "device allocation failed";
    case GAPS_EHIP: return "HIP call failed";
    case GAPS_ECAPACITY: return "size exceeds capacity";
    case GAPS_ESTATE: return "invalid state";
  }
  return "unknown status";
}

gaps_status gaps_init(const gaps_config* cfg, gaps_ctx* out) {
  if (!cfg || !out || !cfg->pdf_xf) return GAPS_EINVAL;
  if (cfg->process < 0 || cfg->process > 4 || cfg->nf < 1 || cfg->nf > 5) return GAPS_EINVAL;
  if (cfg->ntab != 8 || cfg->nx < 4 || cfg->nx > 1024 || cfg->nq < 4 || cfg->nq > 64) return GAPS_EINVAL;
  if (!(cfg->sqrt_s > 0.0) || !(cfg->t_cut > 0.0) || !(cfg->alphas_mz > 0.0) || !(cfg->mz > 0.0))
    return GAPS_EINVAL;
  if (!(cfg->lnx1 > cfg->lnx0) || !(cfg->lnq1 > cfg->lnq0)) return GAPS_EINVAL;
  if ((cfg->process == 2 || cfg->process == 4) && !(cfg->p_s > 0.0 && cfg->p_s < 1.0)) return GAPS_EINVAL;
  if (cfg->process == 4 && !(cfg->mll_min > 0.0 && cfg->mll_max > cfg->mll_min)) return GAPS_EINVAL;
  if (cfg->matching < 0 || cfg->matching > 2) return GAPS_EINVAL;
  if (cfg->matching != 0 && cfg->process != 1 && cfg->process != 2) return GAPS_EINVAL;
  if (cfg->matching == 1 && !(cfg->mu_q2 > 0.0)) return GAPS_EINVAL;
  gaps_ctx c = new (std::nothrow) gaps_ctx_s();
  if (!c) return GAPS_ENOMEM;
  c->cfg = *cfg;
  c->cfg.pdf_xf = nullptr;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return GAPS_EHIP; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) { delete c; return GAPS_EHIP; }
  c->cus = prop.multiProcessorCount;
  // the allocation-free shower's static working storage on this device
  if (resolve_static_scratch(c->device) != GAPS_OK) { delete c; return GAPS_EHIP; }
  size_t npdf = (size_t)cfg->ntab * cfg->nq * cfg->nx;
  if (hipMalloc(&c->d_pdf, npdf * sizeof(float)) != hipSuccess ||
      hipMalloc(&c->d_bound, gaps::kBoundRows * gaps::kNB * sizeof(double)) != hipSuccess) {
    gaps_destroy(c);
    return GAPS_ENOMEM;
  }
  if (hipMemcpy(c->d_pdf, cfg->pdf_xf, npdf * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    gaps_destroy(c);
    return GAPS_EHIP;
  }
  Cfg& C = c->C;
  memset(&C, 0, sizeof(C));
  C.process = cfg->process; C.nf = cfg->nf; C.nx = cfg->nx; C.nq = cfg->nq;
  C.sqrt_s = cfg->sqrt_s; C.S = cfg->sqrt_s * cfg->sqrt_s;
  C.t_cut = cfg->t_cut; C.alphas_mz = cfg->alphas_mz; C.mz = cfg->mz; C.gz = cfg->gz;
  C.mz2 = cfg->mz * cfg->mz;
  C.b0 = (33.0 - 2.0 * 5.0) / (12.0 * gaps::kPi);
  C.as_over = cfg->alphas_mz / (1.0 + cfg->alphas_mz * C.b0 * log(cfg->t_cut / C.mz2));
  C.ln_mz2 = log(C.mz2);
  double q2min = exp(cfg->lnq0);
  C.tc_is = cfg->t_cut > q2min ? cfg->t_cut : q2min;
  C.mc2 = cfg->mc * cfg->mc;
  C.mb2 = cfg->mb * cfg->mb;
  C.tch_c = C.mc2 + cfg->t_cut > C.tc_is ? C.mc2 + cfg->t_cut : C.tc_is;
  C.tch_b = C.mb2 + cfg->t_cut > C.tc_is ? C.mb2 + cfg->t_cut : C.tc_is;
  C.ln_tc = log(cfg->t_cut); C.ln_tcis = log(C.tc_is);
  C.ln_tch_c = log(C.tch_c); C.ln_tch_b = log(C.tch_b);
  C.sw2 = cfg->sw2; C.gf = cfg->gf; C.mll_min = cfg->mll_min; C.mll_max = cfg->mll_max; C.p_s = cfg->p_s;
  C.over_scale = cfg->over_scale > 0.0 ? cfg->over_scale : 1.0;
  C.matching = cfg->matching;
  C.mu_q2 = cfg->mu_q2;
  C.lnx0 = cfg->lnx0; C.lnx1 = cfg->lnx1; C.lnq0 = cfg->lnq0; C.lnq1 = cfg->lnq1;
  for (int k = 0; k <= gaps::kNTB; ++k)
    C.cell_edge[k] = cfg->lnq0 + (double)k * ((cfg->lnq1 - cfg->lnq0) / gaps::kNTB);
  C.learn = nullptr;
  C.dlnx = (cfg->lnx1 - cfg->lnx0) / (cfg->nx - 1);
  C.dlnq = (cfg->lnq1 - cfg->lnq0) / (cfg->nq - 1);
  C.pdf = c->d_pdf;
  C.bound = c->d_bound;
  // the overestimate table, computed on the device
  int nthr = (gaps::kNEnt + 8) * gaps::kNB;
  hipLaunchKernelGGL(gaps::k_bounds, dim3(grid_for(nthr, 64)), dim3(64), 0, 0, C, c->d_bound);
  hipLaunchKernelGGL(gaps::k_bound_sums, dim3(grid_for(2 * gaps::kNB, 64)), dim3(64), 0, 0, C, c->d_bound);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    gaps_destroy(c);
    return GAPS_EHIP;
  }
  if (cfg->process == 1 || cfg->process == 3) {
    double *scan = nullptr, *wmax = nullptr;
    if (hipMalloc(&scan, 64 * 128 * sizeof(double)) != hipSuccess || hipMalloc(&wmax, sizeof(double)) != hipSuccess) {
      gaps_destroy(c);
      return GAPS_ENOMEM;
    }
    hipLaunchKernelGGL(gaps::k_lo_scan, dim3(64 * 128 / 128), dim3(128), 0, 0, C, scan);
    hipLaunchKernelGGL(gaps::k_lo_max, dim3(1), dim3(64), 0, 0, scan, 64 * 128, wmax);
    double h = 0.0;
    hipError_t err = hipMemcpy(&h, wmax, sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(scan);
    (void)hipFree(wmax);
    if (err != hipSuccess) { gaps_destroy(c); return GAPS_EHIP; }
    C.lo_wmax = h;
  }
  *out = c;
  return GAPS_OK;
}

gaps_status gaps_destroy(gaps_ctx c) {
  if (!c) return GAPS_EINVAL;
  if (c->d_pdf) (void)hipFree(c->d_pdf);
  if (c->d_bound) (void)hipFree(c->d_bound);
  if (c->scratch.mem) (void)hipFree(c->scratch.mem);
  free_batches(c->batches);
  if (c->mlp_mem) (void)hipFree(c->mlp_mem);
  if (c->probe_x) (void)hipFree(c->probe_x);
  if (c->cm_mem) (void)hipFree(c->cm_mem);
  if (c->probe_f) (void)hipFree(c->probe_f);
  delete c;
  return GAPS_OK;
}

gaps_status gaps_bounds(gaps_ctx c, double* host_out) {
  if (!c || !host_out) return GAPS_EINVAL;
  GAPS_HIP(hipMemcpy(host_out, c->d_bound, gaps::kNEnt * gaps::kNB * sizeof(double), hipMemcpyDeviceToHost));
  return GAPS_OK;
}

gaps_status gaps_hard_events(gaps_ctx c, int64_t first_id, int64_t n, uint64_t seed, gaps_events* out,
                             hipStream_t stream) {
  if (!c || first_id < 0 || bad_events(out, n, 5)) return GAPS_EINVAL;
  if (n == 0) return GAPS_OK;
  hipLaunchKernelGGL(gaps::k_hard, dim3(grid_for(n, 128)), dim3(128), 0, stream, c->C, first_id, n, seed, *out);
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

}  // extern "C"

namespace {

// Kernel, block and grid of a shower launch over n events.
struct Plan {
  const void* kern;
  int block;
  int64_t grid;
  size_t dyn;
  gaps::ShowerArgs A;
};

gaps_status plan_shower(gaps_ctx c, const gaps_params* params, int64_t n, uint64_t seed, Plan& pl) {
  gaps_params P{};
  if (params) P = *params;
  if (P.variant < 0 || P.variant > 1) return GAPS_EINVAL;
  if (P.mode != GAPS_MODE_PLAIN) {
    if (P.variant != 0) return GAPS_EINVAL;  // the reference variant runs plain mode only
    if (P.mode == GAPS_MODE_LEARNED) {
      if (!c->C.learn) return GAPS_ESTATE;
    } else if (P.mode == GAPS_MODE_LOG) {
      if (!P.log_count || P.log_cap < 0 || (P.log_cap > 0 && !P.trial_log)) return GAPS_EINVAL;
    } else {
      return GAPS_EINVAL;
    }
  }
  const int wps = P.waves_per_simd > 0 ? P.waves_per_simd : 2;
  if (wps < 2 || wps > 4) return GAPS_EINVAL;
  if (P.retain != 0 && (P.retain != 1 || P.variant != 0 || wps > 3)) return GAPS_EINVAL;
  if (P.gen_select != 0 && (P.gen_select != 1 || P.variant != 1 || P.retain || P.mode != GAPS_MODE_PLAIN))
    return GAPS_EINVAL;
  if (P.veto_max != 0 &&
      (P.veto_max != 1 || P.variant != 1 || P.retain || P.gen_select || P.mode != GAPS_MODE_PLAIN))
    return GAPS_EINVAL;
  // the 2-wave kernels compact their tail across up to 8 waves of a block
  const int max_block = (P.variant == 0 && wps == 2) ? 512 : (P.retain && wps == 3) ? 384 : 256;
  pl.block = P.block > 0 ? P.block : max_block;
  if (pl.block % 64 != 0 || pl.block > max_block) return GAPS_EINVAL;
  if (P.grid < 0 || P.compact_every < 0 || P.tail_every < 0) return GAPS_EINVAL;
  // the lane-state pool is used only by tail repacking
  pl.dyn = (P.variant == 1 || P.tail_every == 0) ? 0 : (size_t)pl.block * gaps::kLaneStateBytes;
  pl.kern = P.variant == 1 ? (P.gen_select ? (const void*)gaps::k_shower_lanes_gs
                             : P.veto_max ? (const void*)gaps::k_shower_lanes_vm
                                          : (const void*)gaps::k_shower_lanes)
            : P.retain     ? (wps == 3 ? (const void*)gaps::k_shower_wave_rt3 : (const void*)gaps::k_shower_wave_rt)
            : wps == 2     ? (const void*)gaps::k_shower_wave
            : wps == 3     ? (const void*)gaps::k_shower_wave3
                           : (const void*)gaps::k_shower_wave4;
  int per_cu = 0;
  GAPS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pl.kern, pl.block, pl.dyn));
  if (per_cu < 1) per_cu = 1;
  pl.grid = P.grid > 0 ? P.grid : (int64_t)per_cu * c->cus;
  const int64_t need_blocks = (n + pl.block - 1) / pl.block;
  if (pl.grid > need_blocks) pl.grid = need_blocks;
  if (pl.grid < 1) pl.grid = 1;
  gaps::ShowerArgs& A = pl.A;
  A = gaps::ShowerArgs{};
  A.mode = P.mode;
  A.gen_select = P.gen_select;
  A.veto_max = P.veto_max;
  A.compact_every = P.compact_every > 0 ? P.compact_every : 8;
  A.tail_every = P.tail_every;
  A.stream = 0u;
  A.seed = seed;
  A.n = n;
  A.stats = P.stats;
  A.log = P.trial_log;
  A.log_cap = P.log_cap;
  A.log_count = P.log_count;
  return GAPS_OK;
}

// Validate a host batch table; total events and the smallest output slot limit.
gaps_status check_batches(const gaps_batch* b, int nbatch, int64_t& total, int& slots) {
  if (!b || nbatch < 1 || nbatch > GAPS_MAX_BATCHES) return GAPS_EINVAL;
  total = 0;
  slots = gaps::kMaxSlots;
  for (int k = 0; k < nbatch; ++k) {
    const gaps_batch& x = b[k];
    if (bad_events(&x.in, x.n, 1) || bad_events(&x.out, x.n, 1)) return GAPS_EINVAL;
    if (x.n > 0 && (x.in.E == x.out.E || x.in.n == x.out.n)) return GAPS_EINVAL;
    if (x.n > 0 && x.out.max_slots < slots) slots = x.out.max_slots;
    total += x.n;
  }
  return GAPS_OK;
}

// Upload a host batch table, by value in kernel arguments (stream-ordered and
// capturable; the host table is not referenced after the calls return).
gaps_status store_batches(const gaps_batch* b, int nbatch, int64_t total, BatchMem& m, hipStream_t stream) {
  int64_t first = 0;
  for (int at = 0; at < nbatch; at += gaps::kBatchChunk) {
    gaps::BatchChunk ch{};
    ch.at = at;
    ch.count = nbatch - at < gaps::kBatchChunk ? nbatch - at : gaps::kBatchChunk;
    for (int k = 0; k < ch.count; ++k) {
      ch.b[k] = b[at + k];
      ch.first[k] = first;
      first += b[at + k].n;
    }
    ch.last = at + ch.count == nbatch;
    ch.total = total;
    hipLaunchKernelGGL(gaps::k_store_batches, dim3(1), dim3(64), 0, stream, ch, m.table, m.prefix, nbatch);
    GAPS_HIP(hipGetLastError());
  }
  return GAPS_OK;
}

// Queue reset and the persistent launch.
gaps_status launch_shower(gaps_ctx c, const Plan& pl, const gaps_events* in, const gaps_events* out,
                          const gaps::Scratch& S, hipStream_t stream) {
  hipLaunchKernelGGL(gaps::k_fill_u64, dim3(1), dim3(64), 0, stream, S.queue, (int64_t)1, 0ULL);
  GAPS_HIP(hipGetLastError());
  gaps_events none{};
  void* args[] = {(void*)&c->C, (void*)(in ? in : &none), (void*)(out ? out : &none), (void*)&S,
                  (void*)&pl.A};
  GAPS_HIP(hipLaunchKernel(pl.kern, dim3((unsigned)pl.grid), dim3(pl.block), args, pl.dyn, stream));
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

// Batch upload, plan and scratch of a stream call into (scratch, batches).
gaps_status prepare_stream(gaps_ctx c, const gaps_batch* batches, int nbatch, const gaps_params* params,
                           uint64_t seed, ScratchMem& sm, BatchMem& bm, Plan& pl, int64_t& total) {
  int slots = 0;
  gaps_status s = check_batches(batches, nbatch, total, slots);
  if (s != GAPS_OK) return s;
  if (params && params->variant != 0) return GAPS_EINVAL;
  s = plan_shower(c, params, total, seed, pl);
  if (s != GAPS_OK) return s;
  s = ensure_scratch(sm, pl.grid * pl.block, slots);
  if (s != GAPS_OK) return s;
  s = ensure_batches(bm, nbatch);
  if (s != GAPS_OK) return s;
  pl.A.batches = bm.table;
  pl.A.prefix = bm.prefix;
  pl.A.nbatch = nbatch;
  return GAPS_OK;
}

}  // namespace

extern "C" {

gaps_status gaps_shower(gaps_ctx c, const gaps_events* in, int64_t n, const gaps_params* params, uint64_t seed,
                        gaps_events* out, hipStream_t stream) {
  if (!c || bad_events(in, n, 1) || bad_events(out, n, 1)) return GAPS_EINVAL;
  if (n > 0 && (in->E == out->E || in->n == out->n)) return GAPS_EINVAL;
  Plan pl;
  gaps_status s = plan_shower(c, params, n, seed, pl);
  if (s != GAPS_OK || n == 0) return s;
  s = ensure_scratch(c->scratch, pl.grid * pl.block, out->max_slots);
  if (s != GAPS_OK) return s;
  return launch_shower(c, pl, in, out, c->scratch.S, stream);
}

gaps_status gaps_shower_noalloc(gaps_ctx c, const gaps_events* in, int64_t n, const gaps_params* params,
                                uint64_t seed, gaps_events* out, hipStream_t stream) {
  if (!c || bad_events(in, n, 1) || bad_events(out, n, 1)) return GAPS_EINVAL;
  if (n > 0 && (in->E == out->E || in->n == out->n)) return GAPS_EINVAL;
  Plan pl;
  gaps_status s = plan_shower(c, params, n, seed, pl);
  if (s != GAPS_OK || n == 0) return s;
  void* base = static_scratch(c->device);
  if (!base) return GAPS_ESTATE;
  // as many whole blocks of lanes as the static storage holds (the grid only
  // changes the speed: every event's result is keyed by its id)
  const size_t per_lane = scratch_per_lane(out->max_slots);
  const size_t fixed = scratch_bytes(0, out->max_slots) + 256 * 6;
  const int64_t lanes_cap = GAPS_NOALLOC_SCRATCH_BYTES > fixed
                                ? (int64_t)((GAPS_NOALLOC_SCRATCH_BYTES - fixed) / per_lane) : 0;
  const int64_t blocks_cap = lanes_cap / pl.block;
  if (blocks_cap < 1) return GAPS_ECAPACITY;
  if (pl.grid > blocks_cap) pl.grid = blocks_cap;
  gaps::Scratch S{};
  s = scratch_layout((char*)base, GAPS_NOALLOC_SCRATCH_BYTES, pl.grid * pl.block, out->max_slots, S);
  if (s != GAPS_OK) return s;
  return launch_shower(c, pl, in, out, S, stream);
}

gaps_status gaps_shower_stream(gaps_ctx c, const gaps_batch* batches, int nbatch, const gaps_params* params,
                               uint64_t seed, hipStream_t stream) {
  if (!c) return GAPS_EINVAL;
  Plan pl;
  int64_t total = 0;
  gaps_status s = prepare_stream(c, batches, nbatch, params, seed, c->scratch, c->batches, pl, total);
  if (s != GAPS_OK || total == 0) return s;
  s = store_batches(batches, nbatch, total, c->batches, stream);
  if (s != GAPS_OK) return s;
  return launch_shower(c, pl, nullptr, nullptr, c->scratch.S, stream);
}

gaps_status gaps_graph_capture(gaps_ctx c, const gaps_batch* batches, int nbatch, const gaps_params* params,
                               uint64_t seed, hipStream_t stream, gaps_graph* out) {
  if (!c || !out || stream == nullptr) return GAPS_EINVAL;
  *out = nullptr;
  gaps_graph g = new gaps_graph_s();
  Plan pl;
  int64_t total = 0;
  gaps_status s = prepare_stream(c, batches, nbatch, params, seed, g->scratch, g->batches, pl, total);
  if (s == GAPS_OK && hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) s = GAPS_EHIP;
  if (s == GAPS_OK) {
    gaps_status s1 = store_batches(batches, nbatch, total, g->batches, stream);
    if (s1 == GAPS_OK && total > 0) s1 = launch_shower(c, pl, nullptr, nullptr, g->scratch.S, stream);
    hipError_t e = hipStreamEndCapture(stream, &g->graph);
    if (s1 != GAPS_OK) s = s1;
    else if (e != hipSuccess) s = GAPS_EHIP;
  }
  if (s == GAPS_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) s = GAPS_EHIP;
  if (s != GAPS_OK) {
    gaps_graph_destroy(g);
    return s;
  }
  *out = g;
  return GAPS_OK;
}

gaps_status gaps_tune(gaps_ctx c, const gaps_batch* batches, int nbatch, const gaps_params* base, uint64_t seed,
                      gaps_tune_point* pts, int npts, int repeats, hipStream_t stream) {
  if (!c || !pts || npts < 1 || repeats < 1 || repeats > 64) return GAPS_EINVAL;
  int64_t total = 0;
  int slots = 0;
  gaps_status s = check_batches(batches, nbatch, total, slots);
  if (s != GAPS_OK) return s;
  if (base && base->variant != 0) return GAPS_EINVAL;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return GAPS_EHIP;
  }
  gaps_status out = GAPS_OK;
  float times[64];
  for (int k = 0; k < npts && out == GAPS_OK; ++k) {
    gaps_tune_point& q = pts[k];
    q.grid = 0;
    q.ms = -1.0f;
    gaps_params P{};
    if (base) P = *base;
    P.block = q.block;
    P.compact_every = q.compact_every;
    P.waves_per_simd = q.waves_per_simd;
    P.grid = 0;
    P.stats = nullptr;
    if (q.block <= 0 || q.compact_every <= 0 || !(q.fill > 0.0f && q.fill <= 1.0f)) continue;
    Plan pl;
    int64_t tot = 0;
    s = prepare_stream(c, batches, nbatch, &P, seed, c->scratch, c->batches, pl, tot);
    if (s == GAPS_EINVAL) continue;  // a shape the kernels cannot run
    if (s != GAPS_OK) { out = s; break; }
    if (tot == 0) { q.ms = 0.0f; continue; }
    int64_t g = (int64_t)((double)pl.grid * (double)q.fill + 0.5);
    pl.grid = g < 1 ? 1 : g;
    q.grid = (int)pl.grid;
    s = store_batches(batches, nbatch, tot, c->batches, stream);
    for (int r = 0; r <= repeats && s == GAPS_OK; ++r) {
      if (hipEventRecord(e0, stream) != hipSuccess) { s = GAPS_EHIP; break; }
      s = launch_shower(c, pl, nullptr, nullptr, c->scratch.S, stream);
      if (s != GAPS_OK) break;
      if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { s = GAPS_EHIP; break; }
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { s = GAPS_EHIP; break; }
      if (r > 0) times[r - 1] = ms;  // the first launch is a warm-up
    }
    if (s != GAPS_OK) { out = s; break; }
    // median of the timed launches (insertion sort of at most 64)
    for (int i = 1; i < repeats; ++i)
      for (int j = i; j > 0 && times[j - 1] > times[j]; --j) {
        const float t = times[j];
        times[j] = times[j - 1];
        times[j - 1] = t;
      }
    q.ms = repeats % 2 ? times[repeats / 2] : 0.5f * (times[repeats / 2 - 1] + times[repeats / 2]);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return out;
}

gaps_status gaps_graph_launch(gaps_graph g, hipStream_t stream) {
  if (!g || !g->exec) return GAPS_EINVAL;
  GAPS_HIP(hipGraphLaunch(g->exec, stream));
  return GAPS_OK;
}

gaps_status gaps_graph_destroy(gaps_graph g) {
  if (!g) return GAPS_EINVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->scratch.mem) (void)hipFree(g->scratch.mem);
  free_batches(g->batches);
  delete g;
  return GAPS_OK;
}

gaps_status gaps_observables(gaps_ctx c, const gaps_events* ev, int64_t n, double* obs, hipStream_t stream) {
  if (!c || !obs || bad_events(ev, n, 1)) return GAPS_EINVAL;
  if (n == 0) return GAPS_OK;
  if (c->C.process != 0 && ev->max_slots <= gaps::kObsW) {
    // pp: one event per wave
    const int64_t blocks = (n + gaps::kObsWaves - 1) / gaps::kObsWaves;
    const unsigned grid = (unsigned)(blocks < 2048 ? blocks : 2048);
    hipLaunchKernelGGL(gaps::k_observables_pp, dim3(grid), dim3(64 * gaps::kObsWaves), 0, stream, c->C, *ev, n, obs);
  } else {
    hipLaunchKernelGGL(gaps::k_observables, dim3(grid_for(n, 64)), dim3(64), 0, stream, c->C, *ev, n, obs);
  }
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_histogram(gaps_ctx c, const double* obs, const double* w, int64_t n, int col, double lo, double hi,
                           int nbins, double* sumw, double* sumw2, hipStream_t stream) {
  if (!c || !obs || !sumw || !sumw2 || n < 0 || col < 0 || col >= 12 || nbins < 1 || !(hi > lo))
    return GAPS_EINVAL;
  if (n == 0) return GAPS_OK;
  const unsigned hg = grid_for(n, 256) < 1024 ? grid_for(n, 256) : 1024;
  const size_t hl = nbins <= gaps::kHistLds ? (size_t)2 * nbins * sizeof(double) : 0;
  hipLaunchKernelGGL(gaps::k_histogram, dim3(hg), dim3(256), hl, stream, obs, w, n, col, lo, hi, nbins, sumw, sumw2);
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_pdf_eval(gaps_ctx c, const int32_t* tab, const double* x, const double* q2, int64_t n, double* out,
                          hipStream_t stream) {
  if (!c || !tab || !x || !q2 || !out || n < 0) return GAPS_EINVAL;
  if (n == 0) return GAPS_OK;
  hipLaunchKernelGGL(gaps::k_pdf_eval, dim3(grid_for(n, 256)), dim3(256), 0, stream, c->C, tab, x, q2, n, out);
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_rng_blocks(uint64_t seed, uint32_t stream_id, const int64_t* id, const uint32_t* c2,
                            const uint32_t* c3, int64_t n, uint32_t* out, hipStream_t stream) {
  if (!id || !c2 || !c3 || !out || n < 0) return GAPS_EINVAL;
  if (n == 0) return GAPS_OK;
  hipLaunchKernelGGL(gaps::k_rng_blocks, dim3(grid_for(n, 256)), dim3(256), 0, stream, seed, stream_id, id, c2, c3,
                     n, out);
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

// ---------------------------------------------------------------------------
// Learned initial-state veto bound: network state, training, tabulation

}  // extern "C"

namespace {

constexpr int kNP = gaps::kMlpParams;

// Make the context's learned table the one LEARNED mode reads, with its
// g <- q sums (stream-ordered after the table's writers on `stream`).
gaps_status learn_enable(gaps_ctx c, hipStream_t stream) {
  const int n = 2 * gaps::kNB * gaps::kNTB;
  hipLaunchKernelGGL(gaps::k_learn_sums, dim3(grid_for(n, 128)), dim3(128), 0, stream, c->C, c->table, c->table_sd);
  GAPS_HIP(hipGetLastError());
  c->C.learn = c->table;
  c->C.learn_sd = c->table_sd;
  return GAPS_OK;
}

gaps_status mlp_alloc(gaps_ctx c) {
  if (c->mlp_mem) return GAPS_OK;
  const size_t fl = ((size_t)kNP * 4 + 255) & ~(size_t)255;
  const size_t need = 4 * fl + (((size_t)kNP * 2 + 255) & ~(size_t)255) + (size_t)GAPS_LEARN_CELLS * 8 +
                      (size_t)GAPS_LEARN_CELLS * 8 + 2 * gaps::kNB * gaps::kNTB * 8 +
                      2 * (size_t)GAPS_LEARN_CELLS * 8 + 1280;
  if (hipMalloc(&c->mlp_mem, need) != hipSuccess) return GAPS_ENOMEM;
  char* p = (char*)c->mlp_mem;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~(size_t)255;
    return (void*)r;
  };
  c->theta = (float*)take((size_t)kNP * 4);
  c->mom1 = (float*)take((size_t)kNP * 4);
  c->mom2 = (float*)take((size_t)kNP * 4);
  c->grad = (float*)take((size_t)kNP * 4);
  c->wb = (uint16_t*)take((size_t)kNP * 2);
  c->delta = (double*)take((size_t)GAPS_LEARN_CELLS * 8);
  c->table = (double*)take((size_t)GAPS_LEARN_CELLS * 8);
  c->table_sd = (double*)take(2 * gaps::kNB * gaps::kNTB * 8);
  c->maxbits = (unsigned long long*)take((size_t)GAPS_LEARN_CELLS * 8);
  c->count = (unsigned long long*)take((size_t)GAPS_LEARN_CELLS * 8);
  return GAPS_OK;
}

// fresh optimiser state and analytic margins around new weights in c->theta
gaps_status mlp_reset(gaps_ctx c) {
  GAPS_HIP(hipMemset(c->mom1, 0, (size_t)kNP * 4));
  GAPS_HIP(hipMemset(c->mom2, 0, (size_t)kNP * 4));
  GAPS_HIP(hipMemset(c->grad, 0, (size_t)kNP * 4));
  hipLaunchKernelGGL(gaps::k_mlp_pack, dim3((kNP + 255) / 256), dim3(256), 0, 0, c->theta, c->wb, kNP);
  GAPS_HIP(hipGetLastError());
  hipLaunchKernelGGL(gaps::k_fill_u64, dim3(grid_for(GAPS_LEARN_CELLS, 256)), dim3(256), 0, 0,
                     (unsigned long long*)c->delta, (int64_t)GAPS_LEARN_CELLS, 0x7FF0000000000000ull);  // +inf
  GAPS_HIP(hipGetLastError());
  GAPS_HIP(hipDeviceSynchronize());
  c->adam_step = 0;
  return GAPS_OK;
}

unsigned mlp_grid(int64_t rows, unsigned cap) {
  const int64_t tiles = (rows + 15) / 16;
  int64_t blocks = (tiles + 3) / 4;
  if (blocks < 1) blocks = 1;
  return (unsigned)(blocks < cap ? blocks : cap);
}

}  // namespace

extern "C" {

gaps_status gaps_mlp_init(gaps_ctx c, uint64_t seed) {
  if (!c) return GAPS_EINVAL;
  gaps_status s = mlp_alloc(c);
  if (s != GAPS_OK) return s;
  hipLaunchKernelGGL(gaps::k_mlp_init, dim3((kNP + 255) / 256), dim3(256), 0, 0, seed, c->theta, kNP);
  GAPS_HIP(hipGetLastError());
  return mlp_reset(c);
}

gaps_status gaps_mlp_set(gaps_ctx c, const float* host_theta) {
  if (!c || !host_theta) return GAPS_EINVAL;
  gaps_status s = mlp_alloc(c);
  if (s != GAPS_OK) return s;
  GAPS_HIP(hipMemcpy(c->theta, host_theta, (size_t)kNP * 4, hipMemcpyHostToDevice));
  return mlp_reset(c);
}

gaps_status gaps_mlp_get(gaps_ctx c, float* host_theta) {
  if (!c || !host_theta) return GAPS_EINVAL;
  if (!c->mlp_mem) return GAPS_ESTATE;
  GAPS_HIP(hipDeviceSynchronize());
  GAPS_HIP(hipMemcpy(host_theta, c->theta, (size_t)kNP * 4, hipMemcpyDeviceToHost));
  return GAPS_OK;
}

gaps_status gaps_mlp_features(gaps_ctx c, const float* rows, int64_t n, float* x, float* y, int32_t* ent,
                              int32_t* cell, hipStream_t stream) {
  if (!c || n < 0 || (n > 0 && (!rows || !x || !y))) return GAPS_EINVAL;
  if (n == 0) return GAPS_OK;
  hipLaunchKernelGGL(gaps::k_mlp_features, dim3(grid_for(n, 256)), dim3(256), 0, stream, c->C, rows, n, c->d_bound,
                     x, y, ent, cell);
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_mlp_forward(gaps_ctx c, const float* x, int64_t n, float* f, hipStream_t stream) {
  if (!c || n < 0 || (n > 0 && (!x || !f))) return GAPS_EINVAL;
  if (!c->mlp_mem) return GAPS_ESTATE;
  if (n == 0) return GAPS_OK;
  hipLaunchKernelGGL(gaps::k_mlp_fwd, dim3(mlp_grid(n, 4096)), dim3(256), 0, stream, c->wb, x, n, f);
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_mlp_grad(gaps_ctx c, const float* x, const float* y, int64_t n, float tau, float* grad, float* loss,
                          hipStream_t stream) {
  if (!c || n <= 0 || !x || !y || !grad || !(tau > 0.f && tau < 1.f)) return GAPS_EINVAL;
  if (!c->mlp_mem) return GAPS_ESTATE;
  hipLaunchKernelGGL(gaps::k_mlp_grad, dim3(mlp_grid(n, 256)), dim3(256), 0, stream, c->wb, x, y, n, n, 0ull,
                     (int64_t)0, 0, tau, (float)(1.0 / (double)n), grad, loss);
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_mlp_train(gaps_ctx c, const float* x, const float* y, int64_t n, const gaps_train_params* p,
                           float* loss, hipStream_t stream) {
  if (!c || !p || n <= 0 || !x || !y || p->steps < 0 || p->batch <= 0) return GAPS_EINVAL;
  if (!(p->tau > 0.f && p->tau < 1.f) || !(p->lr > 0.f) || !(p->beta1 >= 0.f && p->beta1 < 1.f) ||
      !(p->beta2 >= 0.f && p->beta2 < 1.f) || !(p->eps > 0.f))
    return GAPS_EINVAL;
  if (!c->mlp_mem) return GAPS_ESTATE;
  const float inv_n = (float)(1.0 / (double)p->batch);
  const unsigned gg = mlp_grid(p->batch, 256);
  for (int64_t k = 0; k < p->steps; ++k) {
    const int64_t t = c->adam_step + 1;
    hipLaunchKernelGGL(gaps::k_mlp_grad, dim3(gg), dim3(256), 0, stream, c->wb, x, y, p->batch, n, p->seed, t, 1, p->tau,
                       inv_n, c->grad, loss ? loss + k : (float*)nullptr);
    const float bc1 = (float)(1.0 - pow((double)p->beta1, (double)t));
    const float bc2 = (float)(1.0 - pow((double)p->beta2, (double)t));
    hipLaunchKernelGGL(gaps::k_adam, dim3((kNP + 255) / 256), dim3(256), 0, stream, c->theta, c->wb, c->grad, c->mom1,
                       c->mom2, kNP, p->lr, p->beta1, p->beta2, p->eps, bc1, bc2);
    c->adam_step = t;
  }
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_mlp_adam_step(gaps_ctx c, float* grad, float lr, float beta1, float beta2, float eps,
                               hipStream_t stream) {
  if (!c || !grad || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return GAPS_EINVAL;
  if (!c->mlp_mem) return GAPS_ESTATE;
  const int64_t t = c->adam_step + 1;
  const float bc1 = (float)(1.0 - pow((double)beta1, (double)t));
  const float bc2 = (float)(1.0 - pow((double)beta2, (double)t));
  hipLaunchKernelGGL(gaps::k_adam, dim3((kNP + 255) / 256), dim3(256), 0, stream, c->theta, c->wb, grad, c->mom1,
                     c->mom2, kNP, lr, beta1, beta2, eps, bc1, bc2);
  GAPS_HIP(hipGetLastError());
  c->adam_step = t;
  return GAPS_OK;
}

// the probe buffers of the tabulation (allocated once per context), also the
// staging of the network's outputs for the calibration's residuals
static gaps_status ensure_probes(gaps_ctx c) {
  const int64_t np = gaps::kMlpProbeRows;
  if (!c->probe_x) {
    if (hipMalloc((void**)&c->probe_x, (size_t)np * 16) != hipSuccess) return GAPS_ENOMEM;
    if (hipMalloc((void**)&c->probe_f, (size_t)np * 4) != hipSuccess) return GAPS_ENOMEM;
  }
  return GAPS_OK;
}

gaps_status gaps_mlp_calibrate(gaps_ctx c, const float* x, const float* y, const int32_t* cell, int64_t n,
                               hipStream_t stream) {
  if (!c || n <= 0 || !x || !y || !cell) return GAPS_EINVAL;
  if (!c->mlp_mem) return GAPS_ESTATE;
  const gaps_status st = ensure_probes(c);
  if (st != GAPS_OK) return st;
  hipLaunchKernelGGL(gaps::k_fill_u64, dim3(grid_for(GAPS_LEARN_CELLS, 256)), dim3(256), 0, stream, c->maxbits,
                     (int64_t)GAPS_LEARN_CELLS, 0ull);
  hipLaunchKernelGGL(gaps::k_fill_u64, dim3(grid_for(GAPS_LEARN_CELLS, 256)), dim3(256), 0, stream, c->count,
                     (int64_t)GAPS_LEARN_CELLS, 0ull);
  // the rows in chunks that fit the probe output buffer, in stream order
  const int64_t chunk = gaps::kMlpProbeRows;
  for (int64_t off = 0; off < n; off += chunk) {
    const int64_t m = n - off < chunk ? n - off : chunk;
    hipLaunchKernelGGL(gaps::k_mlp_fwd, dim3(mlp_grid(m, 4096)), dim3(256), 0, stream, c->wb, x + 4 * off, m,
                       c->probe_f);
    hipLaunchKernelGGL(gaps::k_mlp_resid, dim3(grid_for(m, 256) < 1024 ? grid_for(m, 256) : 1024), dim3(256), 0,
                       stream, c->probe_f, y + off, cell + off, m, c->maxbits, c->count);
  }
  hipLaunchKernelGGL(gaps::k_mlp_delta, dim3(gaps::kNIS), dim3(gaps::kNB * gaps::kNTB), 0, stream, c->maxbits,
                     c->count, (long long)GAPS_MLP_MIN_CAL_CELL, (long long)GAPS_MLP_MIN_CAL_BIN,
                     (long long)GAPS_MLP_MIN_CAL, 0.015625, c->delta);
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_mlp_set_delta(gaps_ctx c, const double* host_delta) {
  if (!c || !host_delta) return GAPS_EINVAL;
  if (!c->mlp_mem) return GAPS_ESTATE;
  GAPS_HIP(hipDeviceSynchronize());
  GAPS_HIP(hipMemcpy(c->delta, host_delta, (size_t)GAPS_LEARN_CELLS * sizeof(double), hipMemcpyHostToDevice));
  return GAPS_OK;
}

gaps_status gaps_mlp_get_delta(gaps_ctx c, double* host_delta) {
  if (!c || !host_delta) return GAPS_EINVAL;
  if (!c->mlp_mem) return GAPS_ESTATE;
  GAPS_HIP(hipDeviceSynchronize());
  GAPS_HIP(hipMemcpy(host_delta, c->delta, (size_t)GAPS_LEARN_CELLS * sizeof(double), hipMemcpyDeviceToHost));
  return GAPS_OK;
}

gaps_status gaps_mlp_tabulate(gaps_ctx c, hipStream_t stream) {
  if (!c) return GAPS_EINVAL;
  if (!c->mlp_mem) return GAPS_ESTATE;
  const int64_t np = gaps::kMlpProbeRows;
  const gaps_status st = ensure_probes(c);
  if (st != GAPS_OK) return st;
  hipLaunchKernelGGL(gaps::k_mlp_probes, dim3(grid_for(np, 256)), dim3(256), 0, stream, c->C, c->probe_x);
  hipLaunchKernelGGL(gaps::k_mlp_fwd, dim3(mlp_grid(np, 4096)), dim3(256), 0, stream, c->wb, c->probe_x, np,
                     c->probe_f);
  hipLaunchKernelGGL(gaps::k_mlp_table, dim3(grid_for(GAPS_LEARN_CELLS, 256)), dim3(256), 0, stream, c->probe_f,
                     c->delta, c->d_bound, c->table);
  GAPS_HIP(hipGetLastError());
  return learn_enable(c, stream);
}

static gaps_status cellmax_table(gaps_ctx c, const float* rows, int64_t n_fit, int64_t n_cal, bool adaptive,
                                 hipStream_t stream) {
  if (!c || !rows || n_fit <= 0 || n_cal < 0) return GAPS_EINVAL;
  gaps_status s = mlp_alloc(c);
  if (s != GAPS_OK) return s;
  const int64_t nc = GAPS_LEARN_CELLS, words = 5 * nc + 2 * 128;
  if (!c->cm_mem && hipMalloc((void**)&c->cm_mem, (size_t)words * 8) != hipSuccess) return GAPS_ENOMEM;
  static_assert(gaps::kCmGroups <= 128, "calibration groups");
  unsigned long long *ymax = c->cm_mem, *cnt = ymax + nc, *emax = cnt + nc, *ecnt = emax + 128;
  unsigned long long *aymax = ecnt + 128, *acnt = aymax + nc, *alvl = acnt + nc, *lvl = nullptr;
  // fill kernels, not memsets, so that the call may be captured in a graph
  hipLaunchKernelGGL(gaps::k_fill_u64, dim3(grid_for(words, 256)), dim3(256), 0, stream, c->cm_mem, words, 0ull);
  hipLaunchKernelGGL(gaps::k_cellmax_fit, dim3(grid_for(n_fit, 256) < 2048 ? grid_for(n_fit, 256) : 2048), dim3(256),
                     0, stream, c->C, rows, n_fit, ymax, cnt);
  if (adaptive) {
    // every cell's block maximum and count then stand in for its own
    hipLaunchKernelGGL(gaps::k_cellmax_adapt, dim3(grid_for(nc, 256)), dim3(256), 0, stream, ymax, cnt,
                       (long long)GAPS_CELLMAX_MIN_CELL, aymax, acnt, alvl);
    ymax = aymax;
    cnt = acnt;
    lvl = alvl;
  }
  if (n_cal > 0)
    hipLaunchKernelGGL(gaps::k_cellmax_resid, dim3(grid_for(n_cal, 256) < 1024 ? grid_for(n_cal, 256) : 1024),
                       dim3(256), 0, stream, c->C, rows + 5 * n_fit, n_cal, ymax, cnt, lvl,
                       (long long)GAPS_CELLMAX_MIN_CELL, emax, ecnt);
  hipLaunchKernelGGL(gaps::k_cellmax_table, dim3(grid_for(nc, 256)), dim3(256), 0, stream, ymax, cnt, lvl, emax, ecnt,
                     (long long)GAPS_CELLMAX_MIN_CELL, (long long)GAPS_CELLMAX_MIN_CAL, 0.015625, c->d_bound, c->table);
  GAPS_HIP(hipGetLastError());
  return learn_enable(c, stream);
}

gaps_status gaps_cellmax_table(gaps_ctx c, const float* rows, int64_t n_fit, int64_t n_cal, hipStream_t stream) {
  return cellmax_table(c, rows, n_fit, n_cal, false, stream);
}

gaps_status gaps_cellmax_table_adaptive(gaps_ctx c, const float* rows, int64_t n_fit, int64_t n_cal,
                                        hipStream_t stream) {
  return cellmax_table(c, rows, n_fit, n_cal, true, stream);
}

gaps_status gaps_learned_table(gaps_ctx c, double* host_out) {
  if (!c || !host_out) return GAPS_EINVAL;
  if (!c->C.learn) return GAPS_ESTATE;
  GAPS_HIP(hipDeviceSynchronize());
  GAPS_HIP(hipMemcpy(host_out, c->table, (size_t)GAPS_LEARN_CELLS * 8, hipMemcpyDeviceToHost));
  return GAPS_OK;
}

gaps_status gaps_learned_set_table(gaps_ctx c, const double* host_table) {
  if (!c || !host_table) return GAPS_EINVAL;
  gaps_status s = mlp_alloc(c);
  if (s != GAPS_OK) return s;
  double* an = (double*)malloc(sizeof(double) * gaps::kNEnt * gaps::kNB);
  if (!an) return GAPS_ENOMEM;
  hipError_t e = hipMemcpy(an, c->d_bound, sizeof(double) * gaps::kNEnt * gaps::kNB, hipMemcpyDeviceToHost);
  bool ok = e == hipSuccess;
  for (int q = 0; ok && q < GAPS_LEARN_CELLS; ++q) {
    const int ent = q / (gaps::kNB * gaps::kNTB) + gaps::kIS0, b = (q / gaps::kNTB) % gaps::kNB;
    const double v = host_table[q];
    ok = isfinite(v) && v >= 0.0 && v <= an[ent * gaps::kNB + b];
  }
  free(an);
  if (e != hipSuccess) return GAPS_EHIP;
  if (!ok) return GAPS_EINVAL;
  GAPS_HIP(hipDeviceSynchronize());
  GAPS_HIP(hipMemcpy(c->table, host_table, (size_t)GAPS_LEARN_CELLS * 8, hipMemcpyHostToDevice));
  const gaps_status st = learn_enable(c, nullptr);
  if (st != GAPS_OK) return st;
  GAPS_HIP(hipDeviceSynchronize());
  return GAPS_OK;
}

}  // extern "C"
