// Learned initial-state veto bound: the network 4 -> 64 -> 64 -> 1 (ReLU) on
// the matrix cores, its training (pinball loss, Adam) and the tabulation of
// the bound per (table entry, eta bin, ln t cell).
//
// Arithmetic: weights and the first hidden layer in bfloat16 (round to
// nearest even), products accumulated in FP32.  The 64x64 layer and the two
// backward products through it are v_mfma_f32_16x16x16_bf16 tiles: a wave
// takes 16 rows at a time.  Operand layouts of that instruction (lane l,
// g = l / 16, r = l % 16): A[i][k] with i = r, k = 4g + j; B[k][n] with
// n = r, k = 4g + j; D[i][n] with n = r, i = 4g + j (j = 0..3 the packed
// values).
#include "kernels.hpp"

namespace gaps {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int H = kMlpHidden;
constexpr int OW1 = 0, OB1 = 256, OW2 = 320, OB2 = 4416, OW3 = 4480, OB3 = 4544;
static_assert(OB3 + 1 == kMlpParams, "parameter layout");
constexpr double kLnEta0d = -13.815510557964274;  // eta bins: uniform in ln eta on [1e-6, 1)
constexpr double kDle = 13.815510557964274 / 48.0;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bf16x4 load4(const uint16_t* p) {
  bf16x4 v;
  v[0] = (short)p[0]; v[1] = (short)p[1]; v[2] = (short)p[2]; v[3] = (short)p[3];
  return v;
}

// small layers (W1, b1, b2, W3, b3) staged in LDS as floats
struct Small {
  float W1[H * 4], b1[H], b2[H], W3[H], b3;
};

__device__ __forceinline__ void load_small(const uint16_t* wb, Small& s) {
  for (int q = threadIdx.x; q < H * 4; q += blockDim.x) s.W1[q] = bf2f(wb[OW1 + q]);
  for (int q = threadIdx.x; q < H; q += blockDim.x) {
    s.b1[q] = bf2f(wb[OB1 + q]);
    s.b2[q] = bf2f(wb[OB2 + q]);
    s.W3[q] = bf2f(wb[OW3 + q]);
  }
  if (threadIdx.x == 0) s.b3 = bf2f(wb[OB3]);
}

// first layer of one row for hidden unit u
__device__ __forceinline__ float layer1(const Small& s, int u, float x0, float x1, float x2, float x3) {
  float a = s.b1[u];
  a = a + s.W1[u * 4 + 0] * x0;
  a = a + s.W1[u * 4 + 1] * x1;
  a = a + s.W1[u * 4 + 2] * x2;
  a = a + s.W1[u * 4 + 3] * x3;
  return a;
}

// random batch row of training step `step` (Philox, stream 5)
__device__ __forceinline__ int64_t sample_row(uint64_t seed, int64_t step, int64_t i, int64_t nsrc) {
  uint32_t o[4];
  philox((uint32_t)step, (uint32_t)((uint64_t)step >> 32), (uint32_t)(i >> 2), 7u, (uint32_t)seed,
         (uint32_t)(seed >> 32) ^ 5u, o);
  const double u = ((double)o[i & 3] + 0.5) * 0x1p-32;
  int64_t k = (int64_t)(u * (double)nsrc);
  return k < nsrc ? k : nsrc - 1;
}

}  // namespace

// f[i] = network(x[i]) for i < n; x is [n][4] floats
__global__ void __launch_bounds__(256) k_mlp_fwd(const uint16_t* __restrict__ wb, const float* __restrict__ x,
                                                 int64_t n, float* __restrict__ f) {
  __shared__ Small s;
  load_small(wb, s);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  bf16x4 B[4][4];  // B[nt][kb]: W2[n = 16 nt + r][k = 16 kb + 4 g + j]
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) B[nt][kb] = load4(wb + OW2 + (nt * 16 + r16) * H + kb * 16 + 4 * g);
  const int64_t ntiles = (n + 15) / 16;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
    const int64_t row = tile * 16 + r16;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f;
    if (row < n) { x0 = x[row * 4]; x1 = x[row * 4 + 1]; x2 = x[row * 4 + 2]; x3 = x[row * 4 + 3]; }
    bf16x4 A[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
        A[kb][jj] = (short)f2bf(fmaxf(layer1(s, kb * 16 + 4 * g + jj, x0, x1, x2, x3), 0.f));
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 D = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) D = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[kb], B[nt][kb], D, 0, 0, 0);
      const int nn = nt * 16 + r16;
#pragma unroll
      for (int j = 0; j < 4; ++j) part[j] += s.W3[nn] * fmaxf(D[j] + s.b2[nn], 0.f);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) part[j] += __shfl_xor(part[j], off);
    if (r16 == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t ri = tile * 16 + 4 * g + j;
        if (ri < n) f[ri] = part[j] + s.b3;
      }
    }
  }
}

// Pinball-loss gradient of a batch of nrows rows, accumulated into grad[4545]
// (and the loss into *loss): rows are x[i], y[i] for i < nrows, or, with
// sample != 0, random rows of the nsrc source rows for training step `step`.
__global__ void __launch_bounds__(256) k_mlp_grad(const uint16_t* __restrict__ wb, const float* __restrict__ x,
                                                  const float* __restrict__ y, int64_t nrows, int64_t nsrc,
                                                  uint64_t seed, int64_t step, int sample, float tau, float inv_n,
                                                  float* __restrict__ grad, float* __restrict__ loss) {
  __shared__ Small s;
  __shared__ uint16_t sH[4][16][H];  // first hidden layer (bf16) of the wave's tile, [row][unit]
  __shared__ uint16_t sD[4][16][H];  // d loss / d a2 (bf16), [row][unit]
  __shared__ float sX[4][16][4], sY[4][16];
  load_small(wb, s);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15, w = threadIdx.x >> 6;
  bf16x4 Bf[4][4], Bt[4][4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) Bf[nt][kb] = load4(wb + OW2 + (nt * 16 + r16) * H + kb * 16 + 4 * g);
  // Bt[nb][kt]: B[k = n][col = k'] = W2[n = 16 nb + 4 g + j][k' = 16 kt + r]
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
      for (int j = 0; j < 4; ++j) Bt[nb][kt][j] = (short)wb[OW2 + (nb * 16 + 4 * g + j) * H + kt * 16 + r16];
  f32x4 accW2[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) accW2[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  float accW1[4][4] = {}, accb1[4] = {}, accb2[4] = {}, accW3[4] = {}, accb3 = 0.f, accloss = 0.f;

  const int64_t ntiles = (nrows + 15) / 16;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
    wave_sync();
    const int64_t row = tile * 16 + r16;
    const bool valid = row < nrows;
    const int64_t src = !valid ? 0 : (sample ? sample_row(seed, step, row, nsrc) : row);
    float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f, yv = 0.f;
    if (valid) { x0 = x[src * 4]; x1 = x[src * 4 + 1]; x2 = x[src * 4 + 2]; x3 = x[src * 4 + 3]; yv = y[src]; }
    if (g == 0) {
      sX[w][r16][0] = x0; sX[w][r16][1] = x1; sX[w][r16][2] = x2; sX[w][r16][3] = x3;
      sY[w][r16] = yv;
    }
    bf16x4 A[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int u = kb * 16 + 4 * g + jj;
        const uint16_t hb = f2bf(fmaxf(layer1(s, u, x0, x1, x2, x3), 0.f));
        A[kb][jj] = (short)hb;
        sH[w][r16][u] = hb;
      }
    f32x4 D[4];
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      D[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) D[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[kb], Bf[nt][kb], D[nt], 0, 0, 0);
      const int nn = nt * 16 + r16;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        D[nt][j] += s.b2[nn];  // a2
        part[j] += s.W3[nn] * fmaxf(D[nt][j], 0.f);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) part[j] += __shfl_xor(part[j], off);
    wave_sync();
    // output layer: d loss / d f per row 4g + j
    float gf[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * g + j;
      const bool vi = tile * 16 + i < nrows;
      const float r = sY[w][i] - (part[j] + s.b3);
      gf[j] = vi ? -(r >= 0.f ? tau : tau - 1.f) * inv_n : 0.f;
      if (r16 == 0 && vi) {
        accloss += (r >= 0.f ? tau * r : (tau - 1.f) * r) * inv_n;
        accb3 += gf[j];
      }
    }
    // second layer: d a2, and the products through W2
    bf16x4 Ad[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int nn = nt * 16 + r16;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float a2 = D[nt][j];
        accW3[nt] += gf[j] * fmaxf(a2, 0.f);
        const float da2 = a2 > 0.f ? gf[j] * s.W3[nn] : 0.f;
        accb2[nt] += da2;
        const uint16_t db = f2bf(da2);
        Ad[nt][j] = (short)db;
        sD[w][4 * g + j][nn] = db;
      }
    }
    wave_sync();
    // dW2[n][k] += sum_rows d a2[row][n] h1[row][k]: A = d a2 (D layout), B = h1 rows
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      bf16x4 Bh;
#pragma unroll
      for (int j = 0; j < 4; ++j) Bh[j] = (short)sH[w][4 * g + j][kt * 16 + r16];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) accW2[mt][kt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ad[mt], Bh, accW2[mt][kt], 0, 0, 0);
    }
    // d h1[row][k] = sum_n d a2[row][n] W2[n][k]
    bf16x4 Ar[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) Ar[nb] = load4(&sD[w][r16][nb * 16 + 4 * g]);
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      f32x4 dh = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) dh = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ar[nb], Bt[nb][kt], dh, 0, 0, 0);
      const int k = kt * 16 + r16;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = 4 * g + j;
        const float xi0 = sX[w][i][0], xi1 = sX[w][i][1], xi2 = sX[w][i][2], xi3 = sX[w][i][3];
        const float a1 = layer1(s, k, xi0, xi1, xi2, xi3);
        const float da1 = a1 > 0.f ? dh[j] : 0.f;
        accb1[kt] += da1;
        accW1[kt][0] += da1 * xi0;
        accW1[kt][1] += da1 * xi1;
        accW1[kt][2] += da1 * xi2;
        accW1[kt][3] += da1 * xi3;
      }
    }
  }
  // flush: dW2 is owned lane by lane; the rest is summed over the four row groups
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        atomicAdd(grad + OW2 + (mt * 16 + 4 * g + j) * H + kt * 16 + r16, accW2[mt][kt][j]);
  auto red = [&](float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
  };
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float w3 = red(accW3[t]), b2 = red(accb2[t]), b1 = red(accb1[t]);
    const float w10 = red(accW1[t][0]), w11 = red(accW1[t][1]), w12 = red(accW1[t][2]), w13 = red(accW1[t][3]);
    if (g == 0) {
      const int u = t * 16 + r16;
      atomicAdd(grad + OW3 + u, w3);
      atomicAdd(grad + OB2 + u, b2);
      atomicAdd(grad + OB1 + u, b1);
      atomicAdd(grad + OW1 + u * 4 + 0, w10);
      atomicAdd(grad + OW1 + u * 4 + 1, w11);
      atomicAdd(grad + OW1 + u * 4 + 2, w12);
      atomicAdd(grad + OW1 + u * 4 + 3, w13);
    }
  }
  const float b3 = red(accb3), ls = red(accloss);
  if (lane == 0) {
    atomicAdd(grad + OB3, b3);
    if (loss) atomicAdd(loss, ls);
  }
}

// One Adam step (Kingma and Ba) on the FP32 master weights; refreshes the
// bfloat16 copy and clears the gradient for the next step.
__global__ void k_adam(float* theta, uint16_t* wb, float* grad, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float gr = grad[p];
  const float mm = b1 * m[p] + (1.f - b1) * gr;
  const float vv = b2 * v[p] + (1.f - b2) * gr * gr;
  m[p] = mm;
  v[p] = vv;
  const float th = theta[p] - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
  theta[p] = th;
  wb[p] = f2bf(th);
  grad[p] = 0.f;
}

// bfloat16 copy of the master weights
__global__ void k_mlp_pack(const float* theta, uint16_t* wb, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) wb[p] = f2bf(theta[p]);
}

// He-uniform weights from Philox4x32-10 (key (seed, stream 4), counter
// (p / 4, 0, 0, 0), word p % 4), zero biases
__global__ void k_mlp_init(uint64_t seed, float* theta, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double fan = 0.0;
  if (p < OB1) fan = 4.0;
  else if (p >= OW2 && p < OB2) fan = 64.0;
  else if (p >= OW3 && p < OB3) fan = 64.0;
  if (fan == 0.0) { theta[p] = 0.f; return; }
  uint32_t o[4];
  philox((uint32_t)(p >> 2), 0u, 0u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32) ^ 4u, o);
  const double u = ((double)o[p & 3] + 0.5) / 4294967296.0;
  theta[p] = (float)((2.0 * u - 1.0) * sqrt(6.0 / fan));
}

// features and target of logged trials (rows of 5 floats: ln t, ln eta, z,
// table entry, ln weight); bound is the analytic table [72][48]
__global__ void k_mlp_features(Cfg C, const float* rows, int64_t n, const double* bound, float* x, float* y,
                               int32_t* ent, int32_t* cell) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lnt = rows[5 * i], lne = rows[5 * i + 1], z = rows[5 * i + 2], lnw = rows[5 * i + 4];
  int e = (int)rows[5 * i + 3];
  e = e < kIS0 ? kIS0 : (e > kIS0 + kNIS - 1 ? kIS0 + kNIS - 1 : e);
  double bb = floor((lne - kLnEta0d) / kDle);
  const int b = !(bb >= 0.0) ? 0 : (bb > 47.0 ? 47 : (int)bb);
  x[4 * i] = (float)((lnt - 10.0) / 10.0);
  x[4 * i + 1] = (float)((lne + 7.0) / 7.0);
  x[4 * i + 2] = (float)(2.0 * z - 1.0);
  x[4 * i + 3] = (float)((e - 40.0) / 32.0);
  y[i] = (float)(lnw - log(bound[e * kNB + b]));
  if (ent) ent[i] = e;
  if (cell) {
    // the ln t cell the shower takes for that scale
    int k = 0;
#pragma unroll
    for (int j = 1; j < kNTB; ++j)
      if (C.cell_edge[j] < lnt) k = j;
    cell[i] = ((e - kIS0) * kNB + b) * kNTB + k;
  }
}

namespace {
// doubles as unsigned keys of the same order (for atomicMax), and back
__device__ __forceinline__ unsigned long long ord64(double d) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double unord64(unsigned long long o) {
  const unsigned long long u = (o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o;
  return __longlong_as_double((long long)u);
}
}  // namespace

// largest residual y - f and row count per cell (entry, eta bin, ln t cell)
__global__ void k_mlp_resid(const float* f, const float* y, const int32_t* cell, int64_t n,
                            unsigned long long* maxbits, unsigned long long* count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = cell[i];
    if (c < 0 || c >= kNIS * kNB * kNTB) continue;
    const double r = (double)y[i] - (double)f[i];
    atomicMax(maxbits + c, ord64(r));
    atomicAdd(count + c, 1ull);
  }
}

// Calibration margin of each cell, one block per entry and one thread per
// cell: the cell's largest residual + margin when it has min_cell rows, else
// its eta bin's (all its cells) when that has min_bin, else its entry's when
// that has min_entry; +inf (the analytic bound) when the entry has fewer.
__global__ void __launch_bounds__(kNB * kNTB) k_mlp_delta(const unsigned long long* maxbits,
                                                         const unsigned long long* count, long long min_cell,
                                                         long long min_bin, long long min_entry, double margin,
                                                         double* delta) {
  __shared__ unsigned long long bm[kNB], bc[kNB], em, ec;
  const int e = blockIdx.x, q = threadIdx.x, b = q / kNTB;
  const int c = (e * kNB + b) * kNTB + q % kNTB;
  if (q < kNB) { bm[q] = 0ull; bc[q] = 0ull; }
  if (q == 0) { em = 0ull; ec = 0ull; }
  __syncthreads();
  const unsigned long long m = maxbits[c], n = count[c];
  if (n) {
    atomicMax(&bm[b], m);
    atomicAdd(&bc[b], n);
    atomicMax(&em, m);
    atomicAdd(&ec, n);
  }
  __syncthreads();
  double d;
  if ((long long)ec < min_entry) d = INFINITY;
  else if ((long long)n >= min_cell) d = unord64(m) + margin;
  else if ((long long)bc[b] >= min_bin) d = unord64(bm[b]) + margin;
  else d = unord64(em) + margin;
  delta[c] = d;
}

// probe inputs of every cell (entry, eta bin, ln t cell): 3 ln t x 2 ln eta x 8 z
__global__ void k_mlp_probes(Cfg C, float* x) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpProbeRows) return;
  const int q = p % 8, j = (p / 8) % 2, i = (p / 16) % 3, k = (p / 48) % kNTB, b = (p / 384) % kNB;
  const int e = (int)(p / 18432);
  const double lo = kLnEta0d + b * kDle;
  const double le = j == 0 ? lo : lo + kDle;
  const double etalo = exp(lo);
  double ek = 0.0, ek1 = 0.0;
#pragma unroll
  for (int m = 0; m < kNTB; ++m)
    if (m == k) { ek = C.cell_edge[m]; ek1 = C.cell_edge[m + 1]; }
  const double lt = i == 0 ? ek : (i == 1 ? 0.5 * (ek + ek1) : ek1);
  const double z = etalo + (1.0 - etalo) * (q / 7.0);
  x[4 * p] = (float)((lt - 10.0) / 10.0);
  x[4 * p + 1] = (float)((le + 7.0) / 7.0);
  x[4 * p + 2] = (float)(2.0 * z - 1.0);
  x[4 * p + 3] = (float)((e + kIS0 - 40.0) / 32.0);
}

// the learned bound of every cell: min(R, up6(R exp(clip(delta + max f, -20, 0))))
__global__ void k_mlp_table(const float* f, const double* delta, const double* bound, double* table) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= kNIS * kNB * kNTB) return;
  const int e = cell / (kNB * kNTB), b = (cell / kNTB) % kNB;
  float fm = f[(int64_t)cell * 48];
  for (int q = 1; q < 48; ++q) fm = fmaxf(fm, f[(int64_t)cell * 48 + q]);
  const double R = bound[(e + kIS0) * kNB + b];
  const double d = delta[cell];
  if (!isfinite(d) || !(R > 0.0)) { table[cell] = R; return; }
  double v = d + (double)fm;
  v = v < -20.0 ? -20.0 : (v > 0.0 ? 0.0 : v);
  int ex;
  const double m = frexp(R * exp(v), &ex);
  const double up = ldexp(ceil(m * 128.0) / 128.0, ex);
  table[cell] = up < R ? up : R;
}

// ---------------------------------------------------------------------------
// Cell-maximum bound: the same cells and shower check as the learned bound,
// with each cell's constant taken from the largest logged weight in the cell
// (presampled maxima, the first half of adaptive overestimation) instead of
// a network.  The non-learned comparator of the learned bound.

namespace {
// cell of a logged trial (entry, eta bin, ln t cell: the cell the shower
// takes for that scale) and its target y = ln W - ln R rounded to FP32 like
// the network's target; -1 for rows outside the initial-state entries
__device__ __forceinline__ int cm_cell(const Cfg& C, const float* row, double& y) {
  const double lnt = row[0], lne = row[1], lnw = row[4];
  const int e = (int)row[3];
  if (e < kIS0 || e >= kIS0 + kNIS) return -1;
  const double bb = floor((lne - kLnEta0d) / kDle);
  const int b = !(bb >= 0.0) ? 0 : (bb > 47.0 ? 47 : (int)bb);
  double edge;
  const int k = cell_of(C, lnt, edge);
  y = (double)(float)(lnw - log(C.bound[e * kNB + b]));
  return ((e - kIS0) * kNB + b) * kNTB + k;
}
}  // namespace

// largest target and row count per cell over the fitting rows
__global__ void k_cellmax_fit(Cfg C, const float* rows, int64_t n, unsigned long long* ymax,
                              unsigned long long* count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double y;
    const int c = cm_cell(C, rows + 5 * i, y);
    if (c < 0) continue;
    atomicMax(ymax + c, ord64(y));
    atomicAdd(count + c, 1ull);
  }
}

// largest excess y - ymax(cell) of the held-out rows per entry, over cells
// with at least min_cell fitting rows, and the number of such rows
// Adaptive cell sizes: each cell takes the finest dyadic block of (eta bin,
// ln t cell) around it with at least min_cell fitting rows (level l: indices
// equal after shifting right by (l, l) up to the ln t range, then the eta
// range), and that block's largest target, row count and level; none: 0, 0, 0
// (the cell then keeps the analytic bound).  ymax holds order-preserving bit
// patterns with 0 for an empty cell, below every value.
__global__ void k_cellmax_adapt(const unsigned long long* ymax, const unsigned long long* count, long long min_cell,
                                unsigned long long* aymax, unsigned long long* acount, unsigned long long* alevel) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= kNIS * kNB * kNTB) return;
  const int e = cell / (kNB * kNTB), b = (cell / kNTB) % kNB, k = cell % kNTB;
  unsigned long long ay = 0ull, an = 0ull, al = 0ull;
  for (int l = 0; l < 7; ++l) {
    const int sb = l, sk = l < 3 ? l : 3;
    const int b0 = (b >> sb) << sb, k0 = (k >> sk) << sk;
    const int b1 = b0 + (1 << sb) < kNB ? b0 + (1 << sb) : kNB, k1 = k0 + (1 << sk) < kNTB ? k0 + (1 << sk) : kNTB;
    unsigned long long m = 0ull, n = 0ull;
    for (int bb = b0; bb < b1; ++bb)
      for (int kk = k0; kk < k1; ++kk) {
        const int q = (e * kNB + bb) * kNTB + kk;
        n += count[q];
        m = ymax[q] > m ? ymax[q] : m;
      }
    if ((long long)n >= min_cell) { ay = m; an = n; al = (unsigned long long)l; break; }
  }
  aymax[cell] = ay;
  acount[cell] = an;
  alevel[cell] = al;
}

// calibration group of a cell: its entry, or (adaptive cells at a coarser
// level l > 0) group kNIS + l - 1 shared by all entries
__device__ __forceinline__ int cm_group(const unsigned long long* level, int cell) {
  const int l = level ? (int)level[cell] : 0;
  return l > 0 ? kNIS + l - 1 : cell / (kNB * kNTB);
}

__global__ void k_cellmax_resid(Cfg C, const float* rows, int64_t n, const unsigned long long* ymax,
                                const unsigned long long* count, const unsigned long long* level, long long min_cell,
                                unsigned long long* emax, unsigned long long* ecount) {
  __shared__ unsigned long long sm[kCmGroups], sc[kCmGroups];
  for (int q = threadIdx.x; q < kCmGroups; q += blockDim.x) { sm[q] = 0ull; sc[q] = 0ull; }
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double y;
    const int c = cm_cell(C, rows + 5 * i, y);
    if (c < 0 || (long long)count[c] < min_cell) continue;
    const int g = cm_group(level, c);
    atomicMax(&sm[g], ord64(y - unord64(ymax[c])));
    atomicAdd(&sc[g], 1ull);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kCmGroups; q += blockDim.x) {
    if (sc[q]) {
      atomicMax(emax + q, sm[q]);
      atomicAdd(ecount + q, sc[q]);
    }
  }
}

// the bound of every cell: min(R, up6(R exp(clip(ymax + delta_e, -20, 0))))
// with delta_e = max(largest excess, 0) + margin, for cells with at least
// min_cell fitting rows in entries with at least min_cal held-out rows; R
// (the analytic bound) elsewhere
__global__ void k_cellmax_table(const unsigned long long* ymax, const unsigned long long* count,
                                const unsigned long long* level, const unsigned long long* emax,
                                const unsigned long long* ecount, long long min_cell, long long min_cal, double margin,
                                const double* bound, double* table) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= kNIS * kNB * kNTB) return;
  const int e = cell / (kNB * kNTB), b = (cell / kNTB) % kNB;
  const int g = cm_group(level, cell);
  const double R = bound[(e + kIS0) * kNB + b];
  if ((long long)count[cell] < min_cell || (long long)ecount[g] < min_cal || !(R > 0.0)) {
    table[cell] = R;
    return;
  }
  const double r = unord64(emax[g]);
  const double d = (r > 0.0 ? r : 0.0) + margin;
  double v = unord64(ymax[cell]) + d;
  v = v < -20.0 ? -20.0 : (v > 0.0 ? 0.0 : v);
  int ex;
  const double m = frexp(R * exp(v), &ex);
  const double up = ldexp(ceil(m * 128.0) / 128.0, ex);
  table[cell] = up < R ? up : R;
}

}  // namespace gaps
