// Host side of the C-ABI declared in include/gaps.h.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "kernels.hpp"

using gaps::Cfg;

struct gaps_ctx_s {
  gaps_config cfg;
  Cfg C;
  int device = 0;
  int cus = 0;
  float* d_pdf = nullptr;
  double* d_bound = nullptr;
  // shower scratch, grown on demand
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  gaps::Scratch S{};
};

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

gaps_status ensure_scratch(gaps_ctx c, int64_t lanes, int slots) {
  const int nch = (2 * slots + 3) & ~3;  // whole chunks of four entries
  size_t per_lane = (size_t)slots * (4 * sizeof(double) + 3 * sizeof(int32_t) + sizeof(int8_t)) +
                    (size_t)nch * (sizeof(uint32_t) + 9 * sizeof(double));
  size_t need = per_lane * (size_t)lanes + 256 * 24 + 64;
  if (need > c->scratch_bytes || c->S.lanes != lanes || c->S.max_slots != slots) {
    if (need > c->scratch_bytes) {
      if (c->scratch) (void)hipFree(c->scratch);
      c->scratch = nullptr;
      c->scratch_bytes = 0;
      if (hipMalloc(&c->scratch, need) != hipSuccess) return GAPS_ENOMEM;
      c->scratch_bytes = need;
    }
    char* p = (char*)c->scratch;
    auto take = [&](size_t bytes) {
      char* r = p;
      p += (bytes + 255) & ~(size_t)255;
      return (void*)r;
    };
    gaps::Scratch& S = c->S;
    S.lanes = lanes;
    S.max_slots = slots;
    size_t ps = (size_t)slots * lanes, cs = (size_t)nch * lanes;
    S.E = (double*)take(ps * 8); S.px = (double*)take(ps * 8);
    S.py = (double*)take(ps * 8); S.pz = (double*)take(ps * 8);
    S.pid = (int32_t*)take(ps * 4); S.col = (int32_t*)take(ps * 4); S.acol = (int32_t*)take(ps * 4);
    S.st = (int8_t*)take(ps);
    S.cinfo = (uint32_t*)take(cs * 4);
    S.ctlim = (double*)take(cs * 8); S.clntlim = (double*)take(cs * 8); S.cinvc = (double*)take(cs * 8);
    S.cc = (double*)take(cs * 8); S.cs = (double*)take(cs * 8); S.czlo = (double*)take(cs * 8);
    S.comzhi = (double*)take(cs * 8); S.cI1 = (double*)take(cs * 8); S.cI2 = (double*)take(cs * 8);
    S.queue = (unsigned long long*)take(64);
    if ((size_t)(p - (char*)c->scratch) > c->scratch_bytes) return GAPS_ENOMEM;
  }
  return GAPS_OK;
}

}  // namespace

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
  if (cfg->process < 0 || cfg->process > 2 || cfg->nf < 1 || cfg->nf > 5) return GAPS_EINVAL;
  if (cfg->ntab != 8 || cfg->nx < 4 || cfg->nx > 1024 || cfg->nq < 4 || cfg->nq > 64) return GAPS_EINVAL;
  if (!(cfg->sqrt_s > 0.0) || !(cfg->t_cut > 0.0) || !(cfg->alphas_mz > 0.0) || !(cfg->mz > 0.0))
    return GAPS_EINVAL;
  if (!(cfg->lnx1 > cfg->lnx0) || !(cfg->lnq1 > cfg->lnq0)) return GAPS_EINVAL;
  if (cfg->process == 2 && !(cfg->p_s > 0.0 && cfg->p_s < 1.0)) return GAPS_EINVAL;
  gaps_ctx c = new (std::nothrow) gaps_ctx_s();
  if (!c) return GAPS_ENOMEM;
  c->cfg = *cfg;
  c->cfg.pdf_xf = nullptr;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return GAPS_EHIP; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) { delete c; return GAPS_EHIP; }
  c->cus = prop.multiProcessorCount;
  size_t npdf = (size_t)cfg->ntab * cfg->nq * cfg->nx;
  if (hipMalloc(&c->d_pdf, npdf * sizeof(float)) != hipSuccess ||
      hipMalloc(&c->d_bound, gaps::kNEnt * gaps::kNB * sizeof(double)) != hipSuccess) {
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
  C.lnx0 = cfg->lnx0; C.lnx1 = cfg->lnx1; C.lnq0 = cfg->lnq0; C.lnq1 = cfg->lnq1;
  C.dlnx = (cfg->lnx1 - cfg->lnx0) / (cfg->nx - 1);
  C.dlnq = (cfg->lnq1 - cfg->lnq0) / (cfg->nq - 1);
  C.pdf = c->d_pdf;
  C.bound = c->d_bound;
  // the overestimate table, computed on the device
  int nthr = gaps::kNEnt * gaps::kNB;
  hipLaunchKernelGGL(gaps::k_bounds, dim3(grid_for(nthr, 64)), dim3(64), 0, 0, C, c->d_bound);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    gaps_destroy(c);
    return GAPS_EHIP;
  }
  if (cfg->process == 1) {
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
  if (c->scratch) (void)hipFree(c->scratch);
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

gaps_status gaps_shower(gaps_ctx c, const gaps_events* in, int64_t n, const gaps_params* params, uint64_t seed,
                        gaps_events* out, hipStream_t stream) {
  if (!c || bad_events(in, n, 1) || bad_events(out, n, 1)) return GAPS_EINVAL;
  if (n > 0 && (in->E == out->E || in->n == out->n)) return GAPS_EINVAL;
  gaps_params P{};
  if (params) P = *params;
  if (P.mode != GAPS_MODE_PLAIN) return GAPS_ESTATE;
  int block = P.block > 0 ? P.block : 256;
  if (block % 64 != 0 || block > 256) return GAPS_EINVAL;
  if (n == 0) return GAPS_OK;
  if (P.variant < 0 || P.variant > 1) return GAPS_EINVAL;
  const int wps = P.waves_per_simd > 0 ? P.waves_per_simd : 2;
  if (wps < 2 || wps > 4) return GAPS_EINVAL;
  const void* kern = P.variant == 1 ? (const void*)gaps::k_shower_lanes
                     : wps == 2     ? (const void*)gaps::k_shower_wave
                     : wps == 3     ? (const void*)gaps::k_shower_wave3
                                    : (const void*)gaps::k_shower_wave4;
  int per_cu = 0;
  GAPS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, 0));
  if (per_cu < 1) per_cu = 1;
  int64_t grid = P.grid > 0 ? P.grid : (int64_t)per_cu * c->cus;
  int64_t need_blocks = (n + block - 1) / block;
  if (grid > need_blocks) grid = need_blocks;
  int64_t lanes = grid * block;
  gaps_status s = ensure_scratch(c, lanes, out->max_slots);
  if (s != GAPS_OK) return s;
  hipLaunchKernelGGL(gaps::k_fill_u64, dim3(1), dim3(64), 0, stream, c->S.queue, (int64_t)1, 0ULL);
  gaps::ShowerArgs A{};
  A.mode = P.mode;
  A.compact_every = P.compact_every > 0 ? P.compact_every : 4;
  A.stream = 0u;
  A.seed = seed;
  A.n = n;
  A.stats = P.stats;
  void* args[] = {(void*)&c->C, (void*)in, (void*)out, (void*)&c->S, (void*)&A};
  GAPS_HIP(hipLaunchKernel(kern, dim3((unsigned)grid), dim3(block), args, 0, stream));
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_observables(gaps_ctx c, const gaps_events* ev, int64_t n, double* obs, hipStream_t stream) {
  if (!c || !obs || bad_events(ev, n, 1)) return GAPS_EINVAL;
  if (n == 0) return GAPS_OK;
  hipLaunchKernelGGL(gaps::k_observables, dim3(grid_for(n, 64)), dim3(64), 0, stream, c->C, *ev, n, obs);
  GAPS_HIP(hipGetLastError());
  return GAPS_OK;
}

gaps_status gaps_histogram(gaps_ctx c, const double* obs, const double* w, int64_t n, int col, double lo, double hi,
                           int nbins, double* sumw, double* sumw2, hipStream_t stream) {
  if (!c || !obs || !sumw || !sumw2 || n < 0 || col < 0 || col >= 12 || nbins < 1 || !(hi > lo))
    return GAPS_EINVAL;
  if (n == 0) return GAPS_OK;
  hipLaunchKernelGGL(gaps::k_histogram, dim3(grid_for(n, 256)), dim3(256), 0, stream, obs, w, n, col, lo, hi, nbins,
                     sumw, sumw2);
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

}  // extern "C"
