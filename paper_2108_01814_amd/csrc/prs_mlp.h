// Learned warm start: a 16 -> 64 -> GELU -> 64 -> GELU -> 16 perceptron on
// gfx950 matrix cores (v_mfma_f32_16x16x16_bf16: BF16 operands, FP32
// accumulation).  The network is the build's own addition to the method
// (the paper has no learned component); the plain multi-direct forcing runs
// after it unchanged.
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

// FP32 -> BF16 bits, round to nearest even (NaN/inf passed through).
__device__ inline unsigned short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline float from_bf16(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ inline bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 v;
  v.x = (short)to_bf16(a);
  v.y = (short)to_bf16(b);
  v.z = (short)to_bf16(c);
  v.w = (short)to_bf16(d);
  return v;
}

__device__ inline bf16x4 pack4(const f32x4 &v) { return pack4(v.x, v.y, v.z, v.w); }

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ inline float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 4 consecutive BF16 values from LDS (8-byte aligned).
__device__ inline bf16x4 lds4(const unsigned short *p) {
  return *reinterpret_cast<const bf16x4 *>(p);
}

// Weights staged in LDS as BF16: the parameter vector (W1, W2, W3 in their
// row-major places; bias slots unused) plus transposed copies of W2 and W3
// for the backward products, and the FP32 biases.
struct MlpLds {
  unsigned short w[kMlpParams];
  unsigned short w2t[kMlpHid * kMlpHid];
  unsigned short w3t[kMlpHid * kMlpOut];
  float b1[kMlpHid], b2[kMlpHid], b3[kMlpOut];
};

constexpr size_t kMlpLdsBytes = (sizeof(MlpLds) + 15) & ~(size_t)15;

// Whole workgroup: copy the BF16 weights and FP32 biases into LDS.
__device__ inline void mlp_stage(MlpLds &L, const unsigned short *__restrict__ wbf,
                                 const float *__restrict__ master, bool transposed) {
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) L.w[i] = wbf[i];
  if (transposed) {
    for (int i = threadIdx.x; i < kMlpHid * kMlpHid; i += blockDim.x) {
      const int r = i / kMlpHid, c = i % kMlpHid;   // w2t[r][c] = W2[c][r]
      L.w2t[i] = wbf[kOffW2 + c * kMlpHid + r];
    }
    for (int i = threadIdx.x; i < kMlpHid * kMlpOut; i += blockDim.x) {
      const int r = i / kMlpOut, c = i % kMlpOut;   // w3t[r][c] = W3[c][r]
      L.w3t[i] = wbf[kOffW3 + c * kMlpHid + r];
    }
  }
  for (int i = threadIdx.x; i < kMlpHid; i += blockDim.x) {
    L.b1[i] = master[kOffB1 + i];
    L.b2[i] = master[kOffB2 + i];
  }
  for (int i = threadIdx.x; i < kMlpOut; i += blockDim.x) L.b3[i] = master[kOffB3 + i];
}

// Activations of one 16-marker tile in the C/B lane layout: lane (q = l/16,
// r = l%16) holds rows 16t + 4q + i of marker r.
struct MlpFwd {
  f32x4 z1[4], z2[4], y;
  bf16x4 xb, a1b[4], a2b[4];
};

// Forward pass of one tile.  xb: B operand of the standardised input, lane
// (q, r) holding features 4q..4q+3 of marker r.
__device__ inline void mlp_forward_tile(const MlpLds &L, bf16x4 xb, MlpFwd &s) {
  const int r = threadIdx.x & 15, q = (threadIdx.x >> 4) & 3;
  s.xb = xb;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 z = mfma(lds4(&L.w[kOffW1 + (16 * t + r) * kMlpIn + 4 * q]), xb, zero);
    for (int i = 0; i < 4; ++i) z[i] += L.b1[16 * t + 4 * q + i];
    s.z1[t] = z;
    s.a1b[t] = pack4(gelu(z[0]), gelu(z[1]), gelu(z[2]), gelu(z[3]));
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 z = zero;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
      z = mfma(lds4(&L.w[kOffW2 + (16 * t + r) * kMlpHid + 16 * kc + 4 * q]), s.a1b[kc], z);
    for (int i = 0; i < 4; ++i) z[i] += L.b2[16 * t + 4 * q + i];
    s.z2[t] = z;
    s.a2b[t] = pack4(gelu(z[0]), gelu(z[1]), gelu(z[2]), gelu(z[3]));
  }
  f32x4 y = zero;
#pragma unroll
  for (int kc = 0; kc < 4; ++kc)
    y = mfma(lds4(&L.w[kOffW3 + r * kMlpHid + 16 * kc + 4 * q]), s.a2b[kc], y);
  for (int i = 0; i < 4; ++i) y[i] += L.b3[4 * q + i];
  s.y = y;
}

}  // namespace prs
