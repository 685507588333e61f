// Learned warm start: training (forward, backward, Adam) and inference of the
// marker-forcing network on MFMA, and its extern "C" entry points.
#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>

#include "prs_internal.h"
#include "prs_mlp.h"

namespace prs {

// Per-wave LDS scratch: BF16 tiles stored [row][marker] so the weight
// gradients (products over the 16 markers of a tile) can read them in the
// A/B operand layout.
struct MlpWaveScratch {
  unsigned short xt[kMlpIn * 16];
  unsigned short a1[kMlpHid * 16];
  unsigned short a2[kMlpHid * 16];
  unsigned short dz1[kMlpHid * 16];
  unsigned short dz2[kMlpHid * 16];
  unsigned short dy[kMlpOut * 16];
};

constexpr int kMlpWaves = 4;   // waves per training workgroup

// One training pass over a batch of standardised inputs X [B][16] and
// targets T [B][3]: loss (1/(3B)) sum (Y - T)^2 and the gradient of every
// parameter, as one partial per wave (reduced in fixed order afterwards).
__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_train(
    const unsigned short *__restrict__ wbf, const float *__restrict__ master,
    const float *__restrict__ X, const float *__restrict__ T, int B, int tiles_per_wave,
    float *__restrict__ partial, float *__restrict__ loss_part) {
  __shared__ MlpLds L;
  __shared__ MlpWaveScratch WS[kMlpWaves];
  mlp_stage(L, wbf, master, true);
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int r = threadIdx.x & 15, q = (threadIdx.x >> 4) & 3;
  const int gwave = blockIdx.x * kMlpWaves + wave;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 gW1[4], gW2[16], gW3[4], gb1[4], gb2[4], gb3 = zero;
  for (int t = 0; t < 4; ++t) gW1[t] = gW3[t] = gb1[t] = gb2[t] = zero;
  for (int t = 0; t < 16; ++t) gW2[t] = zero;
  float lsum = 0.f;
  const float inv = 2.0f / (3.0f * (float)B);
  MlpWaveScratch &W = WS[wave];
  for (int it = 0; it < tiles_per_wave; ++it) {
    const int m0 = (gwave * tiles_per_wave + it) * 16;
    const int m = m0 + r;
    const bool valid = m < B;
    f32x4 xv = zero;
    if (valid) xv = *reinterpret_cast<const f32x4 *>(X + (size_t)m * kMlpIn + 4 * q);
    MlpFwd s;
    mlp_forward_tile(L, pack4(xv), s);
    f32x4 dy;
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * q + i;
      float e = 0.f;
      if (valid && o < kMlpUsed) e = s.y[i] - T[(size_t)m * kMlpUsed + o];
      dy[i] = inv * e;
      lsum += e * e;
    }
    const bf16x4 dyb = pack4(dy);
    f32x4 dz2[4], dz1[4];
    bf16x4 dz2b[4], dz1b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const f32x4 da = mfma(L.g3[t][threadIdx.x & 63], dyb, zero);
      for (int i = 0; i < 4; ++i) dz2[t][i] = da[i] * gelu_d(s.z2[t][i]);
      dz2b[t] = pack4(dz2[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 da = zero;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        da = mfma(L.g2[t][kc][threadIdx.x & 63], dz2b[kc], da);
      for (int i = 0; i < 4; ++i) dz1[t][i] = da[i] * gelu_d(s.z1[t][i]);
      dz1b[t] = pack4(dz1[t]);
    }
    gb3 += dy;
    for (int t = 0; t < 4; ++t) {
      gb2[t] += dz2[t];
      gb1[t] += dz1[t];
    }
    // tiles to LDS, [row][marker]
    for (int j = 0; j < 4; ++j) {
      W.xt[(4 * q + j) * 16 + r] = (unsigned short)s.xb[j];
      W.dy[(4 * q + j) * 16 + r] = (unsigned short)dyb[j];
    }
    for (int t = 0; t < 4; ++t)
      for (int i = 0; i < 4; ++i) {
        const int row = (16 * t + 4 * q + i) * 16 + r;
        W.a1[row] = (unsigned short)s.a1b[t][i];
        W.a2[row] = (unsigned short)s.a2b[t][i];
        W.dz1[row] = (unsigned short)dz1b[t][i];
        W.dz2[row] = (unsigned short)dz2b[t][i];
      }
    __syncthreads();
    // weight gradients: products over the tile's 16 markers
#pragma unroll
    for (int t = 0; t < 4; ++t)
      gW1[t] = mfma(lds4(&W.dz1[(16 * t + r) * 16 + 4 * q]), lds4(&W.xt[r * 16 + 4 * q]), gW1[t]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int t2 = 0; t2 < 4; ++t2)
        gW2[4 * t + t2] = mfma(lds4(&W.dz2[(16 * t + r) * 16 + 4 * q]),
                               lds4(&W.a1[(16 * t2 + r) * 16 + 4 * q]), gW2[4 * t + t2]);
#pragma unroll
    for (int t2 = 0; t2 < 4; ++t2)
      gW3[t2] = mfma(lds4(&W.dy[r * 16 + 4 * q]), lds4(&W.a2[(16 * t2 + r) * 16 + 4 * q]),
                     gW3[t2]);
    __syncthreads();
  }
  float *P = partial + (size_t)gwave * kMlpParams;
  for (int t = 0; t < 4; ++t)
    for (int i = 0; i < 4; ++i) {
      P[kOffW1 + (16 * t + 4 * q + i) * kMlpIn + r] = gW1[t][i];
      for (int t2 = 0; t2 < 4; ++t2)
        P[kOffW2 + (16 * t + 4 * q + i) * kMlpHid + 16 * t2 + r] = gW2[4 * t + t2][i];
      P[kOffW3 + (4 * q + i) * kMlpHid + 16 * t + r] = gW3[t][i];
    }
  // bias gradients: sum over the 16 markers (lanes r) of each lane group q
  for (int t = 0; t < 4; ++t)
    for (int i = 0; i < 4; ++i) {
      float a = gb1[t][i], b = gb2[t][i];
      for (int off = 1; off < 16; off <<= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
      }
      if (r == 0) {
        P[kOffB1 + 16 * t + 4 * q + i] = a;
        P[kOffB2 + 16 * t + 4 * q + i] = b;
      }
    }
  for (int i = 0; i < 4; ++i) {
    float a = gb3[i];
    for (int off = 1; off < 16; off <<= 1) a += __shfl_xor(a, off);
    if (r == 0) P[kOffB3 + 4 * q + i] = a;
  }
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
  if ((threadIdx.x & 63) == 0) loss_part[gwave] = lsum;
}

// grad[i] = sum over waves w of partial[w][i], in a fixed order that does
// not depend on the launch: block b takes parameters 64 b .. 64 b + 63;
// wave v of the block sums (FP64) the partials of waves v, v + 16, v + 32,
// ... in that order, then lane i of wave 0 adds the 16 wave sums in wave
// order.  Reads are coalesced rows of 64 parameters.
constexpr int kRedWaves = 16;

__global__ __launch_bounds__(64 * kRedWaves) void k_mlp_reduce(const float *__restrict__ partial,
                                                              int nwaves, float *grad) {
  __shared__ double s[kRedWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double a = 0.0;
  if (i < kMlpParams)
    for (int w = wv; w < nwaves; w += kRedWaves) a += (double)partial[(size_t)w * kMlpParams + i];
  s[wv][lane] = a;
  __syncthreads();
  if (wv == 0 && i < kMlpParams) {
    double t = s[0][lane];
    for (int v = 1; v < kRedWaves; ++v) t += s[v][lane];
    grad[i] = (float)t;
  }
}

// *out = scale * sum of part[0 .. n-1]: thread t sums part[t], part[t + 1024],
// ... in that order, then thread 0 adds the 1024 thread sums in order.
__global__ __launch_bounds__(1024) void k_sum_ordered(const float *__restrict__ part, int n,
                                                      double scale, double *out) {
  __shared__ double s[1024];
  double a = 0.0;
  for (int w = threadIdx.x; w < n; w += blockDim.x) a += (double)part[w];
  s[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < (int)blockDim.x; ++k) t += s[k];
    *out = scale * t;
  }
}

// Adam on the FP32 master weights; refreshes their BF16 copy.
__global__ void k_mlp_adam(float *master, float *m, float *v, const float *__restrict__ g,
                           unsigned short *wbf, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = master[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  master[i] = w;
  wbf[i] = to_bf16(w);
}

// Table of the GELU of the fused learned pass (gelu_tab): piece i on
// [z_i, z_i + h], z_i = -6 + i h, h = 1/16, the cubic through Phi at
// z_i + {0, 1/3, 2/3, 1} h (Newton's forward differences written in powers
// of f), Phi(z) = erfc(-z / sqrt 2) / 2 in double precision.
__global__ void k_gelu_table(float4 *tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kGeluTabN) return;
  const double h = 1.0 / (double)kGeluInvStep, z = (double)kGeluZ0 + i * h;
  auto Phi = [](double v) { return 0.5 * erfc(-v * 0.70710678118654752440); };
  const double p0 = Phi(z), p1 = Phi(z + h / 3.0), p2 = Phi(z + 2.0 * h / 3.0), p3 = Phi(z + h);
  const double d1 = p1 - p0, d2 = p2 - 2.0 * p1 + p0, d3 = p3 - 3.0 * p2 + 3.0 * p1 - p0;
  tab[i] = make_float4((float)p0, (float)(3.0 * d1 - 1.5 * d2 + d3), (float)(4.5 * (d2 - d3)),
                       (float)(4.5 * d3));
}

__global__ void k_mlp_round(const float *__restrict__ master, unsigned short *wbf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpParams) wbf[i] = to_bf16(master[i]);
}

// Standalone inference: Y [B][3] for inputs X [B][16].  raw != 0: X are raw
// features (standardised here with the stored statistics) and Y is returned
// in target units; raw == 0: both in the network's standardised units.
__global__ __launch_bounds__(256) void k_mlp_forward(const unsigned short *__restrict__ wbf,
                                                     const float *__restrict__ master,
                                                     const float *__restrict__ norm,
                                                     const float *__restrict__ X, int B, int raw,
                                                     float *__restrict__ Y) {
  __shared__ MlpLds L;
  mlp_stage(L, wbf, master, false);
  __syncthreads();
  const int r = threadIdx.x & 15, q = (threadIdx.x >> 4) & 3;
  const int waves = blockDim.x >> 6;
  const int ntiles = (B + 15) / 16;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  for (int tile = blockIdx.x * waves + (threadIdx.x >> 6); tile < ntiles;
       tile += gridDim.x * waves) {
    const int m = tile * 16 + r;
    const bool valid = m < B;
    f32x4 xv = zero;
    if (valid) {
      xv = *reinterpret_cast<const f32x4 *>(X + (size_t)m * kMlpIn + 4 * q);
      if (raw)
        for (int j = 0; j < 4; ++j)
          xv[j] = (xv[j] - norm[4 * q + j]) / norm[kMlpIn + 4 * q + j];
    }
    MlpFwd s;
    mlp_forward_tile(L, pack4(xv), s);
    if (valid && q == 0)
      for (int i = 0; i < kMlpUsed; ++i) {
        float y = s.y[i];
        if (raw) y = y * norm[2 * kMlpIn + kMlpUsed + i] + norm[2 * kMlpIn + i];
        Y[(size_t)m * kMlpUsed + i] = y;
      }
  }
}

// Loss of standardised inputs X [B][16] against standardised targets T
// [B][3]: block b writes the sum of (Y - T)^2 over its tiles (wave sums in
// wave order) to part[b].
__global__ __launch_bounds__(256) void k_mlp_loss(const unsigned short *__restrict__ wbf,
                                                  const float *__restrict__ master,
                                                  const float *__restrict__ X,
                                                  const float *__restrict__ T, int B,
                                                  float *__restrict__ part) {
  __shared__ MlpLds L;
  __shared__ float wsum[4];
  mlp_stage(L, wbf, master, false);
  __syncthreads();
  const int r = threadIdx.x & 15, q = (threadIdx.x >> 4) & 3, wave = threadIdx.x >> 6;
  const int ntiles = (B + 15) / 16;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  float e2 = 0.f;
  for (int tile = blockIdx.x * 4 + wave; tile < ntiles; tile += gridDim.x * 4) {
    const int m = tile * 16 + r;
    const bool valid = m < B;
    f32x4 xv = zero;
    if (valid) xv = *reinterpret_cast<const f32x4 *>(X + (size_t)m * kMlpIn + 4 * q);
    MlpFwd s;
    mlp_forward_tile(L, pack4(xv), s);
    if (valid && q == 0)
      for (int i = 0; i < kMlpUsed; ++i) {
        const float e = s.y[i] - T[(size_t)m * kMlpUsed + i];
        e2 += e * e;
      }
  }
  for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off);
  if ((threadIdx.x & 63) == 0) wsum[wave] = e2;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

// Training-set statistics: column c < 16 of X [m][16], column 16 + c of T
// [m][3].  pass 0: per-block sums of the columns; pass 1: per-block sums of
// the squared deviations from mean[].  Thread t of block b takes rows
// b * 256 + t, then + gridDim * 256, ... (FP64, fixed order), the block adds
// its threads in a fixed tree; out[b][19].
constexpr int kStatCols = kMlpIn + kMlpUsed;
constexpr int kStatBlocks = 256;

__global__ __launch_bounds__(256) void k_col_sums(const float *__restrict__ X,
                                                  const float *__restrict__ T, long long m,
                                                  const double *__restrict__ mean, int pass,
                                                  double *__restrict__ out) {
  __shared__ double s[256];
  double a[kStatCols];
  for (int c = 0; c < kStatCols; ++c) a[c] = 0.0;
  for (long long row = (long long)blockIdx.x * blockDim.x + threadIdx.x; row < m;
       row += (long long)gridDim.x * blockDim.x) {
    for (int c = 0; c < kStatCols; ++c) {
      double v = c < kMlpIn ? (double)X[row * kMlpIn + c] : (double)T[row * kMlpUsed + c - kMlpIn];
      if (pass) {
        v -= mean[c];
        v *= v;
      }
      a[c] += v;
    }
  }
  for (int c = 0; c < kStatCols; ++c) {
    s[threadIdx.x] = a[c];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x * kStatCols + c] = s[0];
    __syncthreads();
  }
}

// dst[c] = sum over blocks of part[b][c] in block order, times scale (or,
// with root = 1, the square root of that times scale).
__global__ void k_col_final(const double *__restrict__ part, int nblocks, double scale, int root,
                            double *dst) {
  const int c = threadIdx.x;
  if (c >= kStatCols) return;
  double t = 0.0;
  for (int b = 0; b < nblocks; ++b) t += part[b * kStatCols + c];
  t *= scale;
  dst[c] = root ? sqrt(t) : t;
}

// Xs = (X - mean) / std, Ts = (T - tmean) / tstd with the network's
// statistics, each value formed in FP64 and rounded to FP32.
__global__ void k_standardize(const float *__restrict__ norm, const float *__restrict__ X,
                              const float *__restrict__ T, long long m, float *__restrict__ Xs,
                              float *__restrict__ Ts) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m * kMlpIn) {
    const int c = (int)(e % kMlpIn);
    Xs[e] = (float)(((double)X[e] - (double)norm[c]) / (double)norm[kMlpIn + c]);
  }
  if (T && e < m * kMlpUsed) {
    const int c = (int)(e % kMlpUsed);
    Ts[e] = (float)(((double)T[e] - (double)norm[2 * kMlpIn + c]) /
                    (double)norm[2 * kMlpIn + kMlpUsed + c]);
  }
}

}  // namespace prs

using namespace prs;

struct prs_mlp {
  float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *partial = nullptr;
  float *loss_part = nullptr, *norm = nullptr;
  float4 *gelu_tab = nullptr;
  double *loss = nullptr;
  unsigned short *wbf = nullptr;
  int t = 0;
  int max_waves = 1024 + kMlpWaves;
  std::string err;
};

void prs::mlp_buffers(const prs_mlp *mlp, prs::LearnArgs *la) {
  la->wbf = mlp->wbf;
  la->master = mlp->master;
  la->norm = mlp->norm;
  la->gelu_tab = reinterpret_cast<const float *>(mlp->gelu_tab);
}

namespace {

int mfail(prs_mlp *m, int code, const char *msg, hipError_t e = hipSuccess) {
  if (m) {
    m->err = msg;
    if (e != hipSuccess) m->err += std::string(": ") + hipGetErrorString(e);
  }
  return code;
}

#define MLP_TRY(mlp, expr)                                   \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return mfail((mlp), PRS_EHIP, #expr, e_); \
  } while (0)

hipStream_t st(void *s) { return static_cast<hipStream_t>(s); }

// Gradient and loss of one batch into mlp->grad / mlp->loss.
int mlp_grad(prs_mlp *mlp, hipStream_t s, const float *X, const float *T, int B) {
  const int tiles = (B + 15) / 16;
  const int cap = mlp->max_waves - kMlpWaves;
  const int tpw = (tiles + cap - 1) / cap;
  const int nwg = (tiles + kMlpWaves * tpw - 1) / (kMlpWaves * tpw);
  hipLaunchKernelGGL(k_mlp_train, dim3(nwg), dim3(64 * kMlpWaves), 0, s, mlp->wbf, mlp->master, X,
                     T, B, tpw, mlp->partial, mlp->loss_part);
  MLP_TRY(mlp, hipGetLastError());
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 63) / 64), dim3(64 * kRedWaves), 0, s,
                     mlp->partial, nwg * kMlpWaves, mlp->grad);
  hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(1024), 0, s, mlp->loss_part, nwg * kMlpWaves,
                     1.0 / (3.0 * (double)B), mlp->loss);
  MLP_TRY(mlp, hipGetLastError());
  return PRS_OK;
}

// One bias-corrected Adam step on the master weights from g (device).
int mlp_adam(prs_mlp *m, hipStream_t s, const float *g, float lr) {
  m->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, m->t)), c2 = (float)(1.0 - std::pow(0.999, m->t));
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, m->master, m->m,
                     m->v, g, m->wbf, lr, b1, b2, 1e-8f, c1, c2);
  MLP_TRY(m, hipGetLastError());
  return PRS_OK;
}

int copy_loss(prs_mlp *m, hipStream_t s, double *loss) {
  if (!loss) return PRS_OK;
  MLP_TRY(m, hipMemcpyAsync(loss, m->loss, sizeof(double), hipMemcpyDeviceToHost, s));
  MLP_TRY(m, hipStreamSynchronize(s));
  return PRS_OK;
}

// Training-set statistics into norm (host) with the caller's scratch: part
// [kStatBlocks][kStatCols] and stat [2][kStatCols] doubles on the device.
// Every entry of the scratch is written before it is read.
int fit_norm_with(hipStream_t s, const float *X, const float *T, int64_t count, double *part,
                  double *stat, float *norm) {
  double host[2 * kStatCols];
  hipLaunchKernelGGL(k_col_sums, dim3(kStatBlocks), dim3(256), 0, s, X, T, (long long)count,
                     nullptr, 0, part);
  hipLaunchKernelGGL(k_col_final, dim3(1), dim3(64), 0, s, part, kStatBlocks,
                     1.0 / (double)count, 0, stat);
  hipLaunchKernelGGL(k_col_sums, dim3(kStatBlocks), dim3(256), 0, s, X, T, (long long)count,
                     stat, 1, part);
  // sample standard deviation (n - 1 in the denominator)
  hipLaunchKernelGGL(k_col_final, dim3(1), dim3(64), 0, s, part, kStatBlocks,
                     1.0 / (double)(count - 1), 1, stat + kStatCols);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(host, stat, sizeof host, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return PRS_EHIP;
  // the padding features stay unscaled; a constant column keeps std 1
  for (int c = 0; c < kMlpIn; ++c) {
    const bool pad = c >= kMlpFeat;
    norm[c] = pad ? 0.f : (float)host[c];
    const double sd = host[kStatCols + c];
    norm[kMlpIn + c] = (pad || !(sd > 0)) ? 1.f : (float)sd;
  }
  for (int c = 0; c < kMlpUsed; ++c) {
    norm[2 * kMlpIn + c] = (float)host[kMlpIn + c];
    const double sd = host[kStatCols + kMlpIn + c];
    norm[2 * kMlpIn + kMlpUsed + c] = sd > 0 ? (float)sd : 1.f;
  }
  return PRS_OK;
}

// Scratch of prs_mlp_fit_norm_noalloc: the per-block partial sums and the
// statistics.  Every device the library runs on holds its own instance of
// this array until the process ends; host code never passes its name to a
// kernel (on the host the name is only a stand-in), but the device address
// looked up once per device with that device current.
constexpr int kNoAllocDoubles = kStatBlocks * kStatCols + 2 * kStatCols;
__device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there).
int scratch_address(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PRS_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PRS_EHIP;
    g_scratch[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch[dev];
  return PRS_OK;
}

}  // namespace

extern "C" {

int prs_mlp_create(const float *params, const float *norm, prs_mlp **out) {
  if (!params || !norm || !out) return PRS_EINVAL;
  *out = nullptr;
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(params[i])) return PRS_EINVAL;
  for (int i = 0; i < kMlpNorm; ++i)
    if (!std::isfinite(norm[i]) || (i >= kMlpIn && i < 2 * kMlpIn && !(norm[i] > 0)) ||
        (i >= 2 * kMlpIn + kMlpUsed && !(norm[i] > 0)))
      return PRS_EINVAL;
  prs_mlp *m = new prs_mlp();
  const size_t P = kMlpParams;
  bool ok = hipMalloc(&m->master, P * 4) == hipSuccess && hipMalloc(&m->m, P * 4) == hipSuccess &&
            hipMalloc(&m->v, P * 4) == hipSuccess && hipMalloc(&m->grad, P * 4) == hipSuccess &&
            hipMalloc(&m->partial, (size_t)m->max_waves * P * 4) == hipSuccess &&
            hipMalloc(&m->loss_part, (size_t)m->max_waves * 4) == hipSuccess &&
            hipMalloc(&m->norm, kMlpNorm * 4) == hipSuccess &&
            hipMalloc(&m->loss, sizeof(double)) == hipSuccess &&
            hipMalloc(&m->wbf, P * 2) == hipSuccess &&
            hipMalloc(&m->gelu_tab, kGeluTabN * sizeof(float4)) == hipSuccess;
  ok = ok && hipMemcpy(m->master, params, P * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(m->norm, norm, kMlpNorm * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(m->m, 0, P * 4) == hipSuccess && hipMemset(m->v, 0, P * 4) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(k_mlp_round, dim3((kMlpParams + 255) / 256), dim3(256), 0, nullptr,
                       m->master, m->wbf);
    hipLaunchKernelGGL(k_gelu_table, dim3((kGeluTabN + 255) / 256), dim3(256), 0, nullptr,
                       m->gelu_tab);
    ok = hipDeviceSynchronize() == hipSuccess;
  }
  if (!ok) {
    prs_mlp_destroy(m);
    return PRS_EHIP;
  }
  *out = m;
  return PRS_OK;
}

void prs_mlp_destroy(prs_mlp *m) {
  if (!m) return;
  void *ptrs[] = {m->master, m->m, m->v, m->grad, m->partial, m->loss_part, m->norm, m->loss,
                  m->wbf, m->gelu_tab};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
}

const char *prs_mlp_last_error(const prs_mlp *m) {
  if (!m) return "null network";
  return m->err.empty() ? "ok" : m->err.c_str();
}

int prs_mlp_get(prs_mlp *m, float *params, float *norm) {
  if (!m) return PRS_EINVAL;
  if (params)
    MLP_TRY(m, hipMemcpy(params, m->master, kMlpParams * 4, hipMemcpyDeviceToHost));
  if (norm) MLP_TRY(m, hipMemcpy(norm, m->norm, kMlpNorm * 4, hipMemcpyDeviceToHost));
  return PRS_OK;
}

int prs_mlp_forward(prs_mlp *m, void *stream, const float *X, int32_t B, int raw, float *Y) {
  if (!m) return PRS_EINVAL;
  if (B < 0 || (B > 0 && (!X || !Y))) return mfail(m, PRS_EINVAL, "forward: bad arguments");
  if (B == 0) return PRS_OK;
  const int tiles = (B + 15) / 16;
  const int grid = (tiles + 3) / 4 < 2048 ? (tiles + 3) / 4 : 2048;
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, st(stream), m->wbf, m->master,
                     m->norm, X, B, raw, Y);
  MLP_TRY(m, hipGetLastError());
  return PRS_OK;
}

int prs_mlp_backward(prs_mlp *m, void *stream, const float *X, const float *T, int32_t B,
                     float *grad, double *loss) {
  if (!m) return PRS_EINVAL;
  if (B <= 0 || !X || !T) return mfail(m, PRS_EINVAL, "backward: bad arguments");
  hipStream_t s = st(stream);
  if (int rc = mlp_grad(m, s, X, T, B)) return rc;
  if (grad)
    MLP_TRY(m, hipMemcpyAsync(grad, m->grad, kMlpParams * 4, hipMemcpyDeviceToDevice, s));
  return copy_loss(m, s, loss);
}

int prs_mlp_adam(prs_mlp *m, void *stream, const float *grad, float lr) {
  if (!m) return PRS_EINVAL;
  if (!(lr > 0)) return mfail(m, PRS_EINVAL, "adam: learning rate must be positive");
  return mlp_adam(m, st(stream), grad ? grad : m->grad, lr);
}

int prs_mlp_train_step(prs_mlp *m, void *stream, const float *X, const float *T, int32_t B,
                       float lr, double *loss) {
  if (!m) return PRS_EINVAL;
  if (B <= 0 || !X || !T || !(lr > 0)) return mfail(m, PRS_EINVAL, "train: bad arguments");
  hipStream_t s = st(stream);
  if (int rc = mlp_grad(m, s, X, T, B)) return rc;
  if (int rc = mlp_adam(m, s, m->grad, lr)) return rc;
  return copy_loss(m, s, loss);
}

int prs_mlp_loss(prs_mlp *m, void *stream, const float *X, const float *T, int32_t B,
                 double *loss) {
  if (!m) return PRS_EINVAL;
  if (B <= 0 || !X || !T || !loss) return mfail(m, PRS_EINVAL, "loss: bad arguments");
  hipStream_t s = st(stream);
  const int tiles = (B + 15) / 16;
  int grid = (tiles + 3) / 4;
  if (grid > m->max_waves) grid = m->max_waves;
  hipLaunchKernelGGL(k_mlp_loss, dim3(grid), dim3(256), 0, s, m->wbf, m->master, X, T, B,
                     m->loss_part);
  hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(1024), 0, s, m->loss_part, grid,
                     1.0 / (3.0 * (double)B), m->loss);
  MLP_TRY(m, hipGetLastError());
  return copy_loss(m, s, loss);
}

int prs_mlp_standardize(prs_mlp *m, void *stream, const float *X, const float *T, int64_t count,
                        float *Xs, float *Ts) {
  if (!m) return PRS_EINVAL;
  if (count < 0 || (count > 0 && (!X || !Xs || (T && !Ts))))
    return mfail(m, PRS_EINVAL, "standardize: bad arguments");
  if (count == 0) return PRS_OK;
  const long long n = (long long)count * kMlpIn;
  hipLaunchKernelGGL(k_standardize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st(stream),
                     m->norm, X, T, (long long)count, Xs, Ts);
  MLP_TRY(m, hipGetLastError());
  return PRS_OK;
}

int prs_mlp_fit_norm(void *stream, const float *X, const float *T, int64_t count, float *norm) {
  if (count < 2 || !X || !T || !norm) return PRS_EINVAL;
  double *part = nullptr, *stat = nullptr;
  if (hipMalloc(&part, sizeof(double) * kStatBlocks * kStatCols) != hipSuccess) return PRS_EHIP;
  if (hipMalloc(&stat, sizeof(double) * 2 * kStatCols) != hipSuccess) {
    (void)hipFree(part);
    return PRS_EHIP;
  }
  const int rc = fit_norm_with(st(stream), X, T, count, part, stat, norm);
  (void)hipFree(part);
  (void)hipFree(stat);
  return rc;
}

int prs_mlp_fit_norm_noalloc(void *stream, const float *X, const float *T, int64_t count,
                             float *norm) {
  if (count < 2 || !X || !T || !norm) return PRS_EINVAL;
  double *base = nullptr;
  if (int rc = scratch_address(&base)) return rc;
  return fit_norm_with(st(stream), X, T, count, base, base + kStatBlocks * kStatCols, norm);
}

}  // extern "C"
