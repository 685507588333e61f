// Learned warm start: a 16 -> 64 -> GELU -> 64 -> GELU -> 16 perceptron on
// gfx950 matrix cores (v_mfma_f32_16x16x16_bf16: BF16 operands, FP32
// accumulation).  The network is an addition to the method (the paper has
// no learned component); the plain multi-direct forcing runs after it
// unchanged.
//
// Work layout: one wave evaluates 16 markers at a time with the markers as
// the N dimension of every product, Z^T = W * X^T.  With the MFMA lane layout
// (lane l holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16] and C[4(l/16)+i][l%16])
// each layer's output tile is exactly the next layer's B operand, so the
// forward pass chains MFMAs without data movement.
#pragma once

#include "prs_device.h"

namespace prs {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 16, kMlpHid = 64, kMlpOut = 16, kMlpUsed = 3, kMlpFeat = 12;
// flat parameter vector, row-major (out x in)
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHid * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpHid;
constexpr int kMlpParams = kOffB3 + kMlpOut;   // 6288
constexpr int kMlpNorm = 2 * kMlpIn + 2 * kMlpUsed;   // feature mean/std, target mean/std

// FP32 -> BF16 bits, round to nearest even (the gfx950 conversion
// instruction).
__device__ inline unsigned short to_bf16(float x) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(x));
}

__device__ inline float from_bf16(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Four FP32 values -> BF16 (round to nearest even), two per conversion.
__device__ inline bf16x4 pack4(float a, float b, float c, float d) {
  const bf16x2_t lo = __builtin_convertvector((f32x2){a, b}, bf16x2_t);
  const bf16x2_t hi = __builtin_convertvector((f32x2){c, d}, bf16x2_t);
  const unsigned ulo = __builtin_bit_cast(unsigned, lo), uhi = __builtin_bit_cast(unsigned, hi);
  bf16x4 v;
  v.x = (short)(ulo & 0xffffu);
  v.y = (short)(ulo >> 16);
  v.z = (short)(uhi & 0xffffu);
  v.w = (short)(uhi >> 16);
  return v;
}

__device__ inline bf16x4 pack4(const f32x4 &v) { return pack4(v.x, v.y, v.z, v.w); }

// Standard normal distribution Phi(z) = erfc(-z / sqrt 2) / 2 and density
// phi(z), branch-free.  erfc(x), x >= 0, is the Chebyshev fit of Press et
// al., Numerical Recipes (2nd ed., sec. 6.2, "erfcc"), fractional error below
// 1.2e-7 for every x: erfc(x) = t exp(-x^2 + P(t)), t = 1 / (1 + x / 2).
__device__ inline void normal_cdf_pdf(float z, float &Phi, float &phi) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  p = fmaf(p, t, -1.26551223f);
  const float ex2 = __builtin_amdgcn_exp2f(-x * x * 1.4426950408889634f);   // exp(-x^2)
  const float half_erfc = 0.5f * t * ex2 * __builtin_amdgcn_exp2f(p * 1.4426950408889634f);
  Phi = z >= 0.f ? 1.0f - half_erfc : half_erfc;
  phi = ex2 * 0.39894228040143268f;   // exp(-z^2 / 2) / sqrt(2 pi)
}

// GELU(z) = z Phi(z), with the erfcc fit above evaluated in base 2 so that
// one exponential serves: erfc(x) / 2 = t 2^(log2(e) (P(t) - x^2) - 1).
__device__ inline float gelu(float z) {
  constexpr float L2E = 1.4426950408889634f;
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
  float p = 0.17087277f * L2E;
  p = fmaf(p, t, -0.82215223f * L2E);
  p = fmaf(p, t, 1.48851587f * L2E);
  p = fmaf(p, t, -1.13520398f * L2E);
  p = fmaf(p, t, 0.27886807f * L2E);
  p = fmaf(p, t, -0.18628806f * L2E);
  p = fmaf(p, t, 0.09678418f * L2E);
  p = fmaf(p, t, 0.37409196f * L2E);
  p = fmaf(p, t, 1.00002368f * L2E);
  p = fmaf(p, t, -1.26551223f * L2E - 1.0f);
  const float half_erfc = t * __builtin_amdgcn_exp2f(fmaf(z * (-0.5f * L2E), z, p));
  return z * (z >= 0.f ? 1.0f - half_erfc : half_erfc);
}

// GELU from a table of Phi: cubic pieces on [-6, 6) with step 1/16,
// Phi(z_i + f h) = c0 + f (c1 + f (c2 + f c3)), f in [0, 1), through Phi at
// z_i + {0, 1/3, 2/3, 1} h (interpolation error below 5e-9: h^4 / 24 times
// the largest fourth derivative of Phi, < 0.55, times the largest
// |f (f - 1/3) (f - 2/3) (f - 1)|, < 0.0124); outside [-6, 6] Phi is within
// 1e-9 of 0 or 1 and the end pieces are used.  Nine vector operations and one
// LDS read instead of the erfcc fit's exponential and reciprocal: the fused
// learned pass evaluates 128 GELUs per marker.
constexpr int kGeluTabN = 192;
constexpr float kGeluZ0 = -6.0f, kGeluInvStep = 16.0f;

__device__ inline float gelu_tab(const float4 *tab, float z) {
  const float u = fminf(fmaxf(fmaf(z, kGeluInvStep, -kGeluZ0 * kGeluInvStep), 0.0f),
                        (float)kGeluTabN - 0.001f);
  // u >= 0: the piece is the truncation, f its exact fractional part
  const float f = __builtin_amdgcn_fractf(u);
  const float4 c = tab[(int)u];
  return z * fmaf(f, fmaf(f, fmaf(f, c.w, c.z), c.y), c.x);
}

// The activation of the forward pass: the erfcc fit, or the table.
struct GeluFit {
  __device__ float operator()(float z) const { return gelu(z); }
};
struct GeluTable {
  const float4 *tab;
  __device__ float operator()(float z) const { return gelu_tab(tab, z); }
};

__device__ inline float gelu_d(float z) {
  float Phi, phi;
  normal_cdf_pdf(z, Phi, phi);
  return Phi + z * phi;
}

__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 4 consecutive BF16 values from LDS (8-byte aligned).
__device__ inline bf16x4 lds4(const unsigned short *p) {
  return *reinterpret_cast<const bf16x4 *>(p);
}

// Weights staged in LDS as BF16 MFMA operand fragments, fragment-major: entry
// [..][lane] is the bf16x4 that lane (q = lane / 16, r = lane % 16) passes to
// the product, so the 64 lanes of a wave read 512 consecutive bytes (no bank
// conflicts, whatever the row length of the matrix):
//   f1[t][lane]     = W1[16t + r][4q .. 4q+3]          (layer 1, output tile t)
//   f2[t][kc][lane] = W2[16t + r][16kc + 4q .. +3]     (layer 2)
//   f3[kc][lane]    = W3[r][16kc + 4q .. +3]           (layer 3)
//   g2[t][kc][lane] = W2[16kc + 4q + j][16t + r], j = 0..3   (W2^T, backward)
//   g3[t][lane]     = W3[4q + j][16t + r], j = 0..3          (W3^T, backward)
// plus the FP32 biases.
// The forward pass's part (the fused learned pass stages only this).
struct alignas(16) MlpFwdLds {
  bf16x4 f1[4][64];
  bf16x4 f2[4][4][64];
  bf16x4 f3[4][64];
  float b1[kMlpHid], b2[kMlpHid], b3[kMlpOut];
};
struct alignas(16) MlpLds : MlpFwdLds {
  bf16x4 g2[4][4][64];
  bf16x4 g3[4][64];
};

constexpr size_t kMlpLdsBytes = (sizeof(MlpLds) + 15) & ~(size_t)15;
constexpr size_t kMlpFwdLdsBytes = (sizeof(MlpFwdLds) + 15) & ~(size_t)15;

// Whole workgroup: stage the forward pass's BF16 weight fragments and FP32
// biases.
__device__ inline void mlp_stage_fwd(MlpFwdLds &L, const unsigned short *__restrict__ wbf,
                                     const float *__restrict__ master) {
  auto frag = [&](int off) { return *reinterpret_cast<const bf16x4 *>(wbf + off); };
  for (int e = threadIdx.x; e < 4 * 64; e += blockDim.x) {
    const int t = e >> 6, lane = e & 63, r = lane & 15, q = lane >> 4;
    L.f1[t][lane] = frag(kOffW1 + (16 * t + r) * kMlpIn + 4 * q);
    L.f3[t][lane] = frag(kOffW3 + r * kMlpHid + 16 * t + 4 * q);
  }
  for (int e = threadIdx.x; e < 16 * 64; e += blockDim.x) {
    const int t = e >> 8, kc = (e >> 6) & 3, lane = e & 63, r = lane & 15, q = lane >> 4;
    L.f2[t][kc][lane] = frag(kOffW2 + (16 * t + r) * kMlpHid + 16 * kc + 4 * q);
  }
  for (int i = threadIdx.x; i < kMlpHid; i += blockDim.x) {
    L.b1[i] = master[kOffB1 + i];
    L.b2[i] = master[kOffB2 + i];
  }
  for (int i = threadIdx.x; i < kMlpOut; i += blockDim.x) L.b3[i] = master[kOffB3 + i];
}

// Whole workgroup: the forward part, and with transposed also the W2^T and
// W3^T fragments of the backward pass.
__device__ inline void mlp_stage(MlpLds &L, const unsigned short *__restrict__ wbf,
                                 const float *__restrict__ master, bool transposed) {
  mlp_stage_fwd(L, wbf, master);
  if (transposed) {
    for (int e = threadIdx.x; e < 16 * 64; e += blockDim.x) {
      const int t = e >> 8, kc = (e >> 6) & 3, lane = e & 63, r = lane & 15, q = lane >> 4;
      bf16x4 v;
      for (int j = 0; j < 4; ++j)
        v[j] = (short)wbf[kOffW2 + (16 * kc + 4 * q + j) * kMlpHid + 16 * t + r];
      L.g2[t][kc][lane] = v;
    }
    for (int e = threadIdx.x; e < 4 * 64; e += blockDim.x) {
      const int t = e >> 6, lane = e & 63, r = lane & 15, q = lane >> 4;
      bf16x4 v;
      for (int j = 0; j < 4; ++j) v[j] = (short)wbf[kOffW3 + (4 * q + j) * kMlpHid + 16 * t + r];
      L.g3[t][lane] = v;
    }
  }
}

// Activations of one 16-marker tile in the C/B lane layout: lane (q = l/16,
// r = l%16) holds rows 16t + 4q + i of marker r.
struct MlpFwd {
  f32x4 z1[4], z2[4], y;
  bf16x4 xb, a1b[4], a2b[4];
};

// Forward pass of one tile.  xb: B operand of the standardised input, lane
// (q, r) holding features 4q..4q+3 of marker r.  act: the GELU evaluation.
template <class Act = GeluFit>
__device__ inline void mlp_forward_tile(const MlpFwdLds &L, bf16x4 xb, MlpFwd &s, Act act = Act{}) {
  const int lane = threadIdx.x & 63, q = lane >> 4;
  s.xb = xb;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const f32x4 b = *reinterpret_cast<const f32x4 *>(&L.b1[16 * t + 4 * q]);
    f32x4 z = mfma(L.f1[t][lane], xb, b);
    s.z1[t] = z;
    s.a1b[t] = pack4(act(z[0]), act(z[1]), act(z[2]), act(z[3]));
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 z = *reinterpret_cast<const f32x4 *>(&L.b2[16 * t + 4 * q]);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
      z = mfma(L.f2[t][kc][lane], s.a1b[kc], z);
    s.z2[t] = z;
    s.a2b[t] = pack4(act(z[0]), act(z[1]), act(z[2]), act(z[3]));
  }
  f32x4 y = *reinterpret_cast<const f32x4 *>(&L.b3[4 * q]);
#pragma unroll
  for (int kc = 0; kc < 4; ++kc)
    y = mfma(L.f3[kc][lane], s.a2b[kc], y);
  s.y = y;
}

}  // namespace prs
