// Delta-kernel stencils and block reductions shared by the interpolation and
// spreading kernels.
#pragma once

#include "prs_device.h"

namespace prs {

// Three-point kernel weights of the nodes ic-1, ic, ic+1 for the offset
// r0 = s - ic in [-1/2, 1/2) (s in node units): with q = sqrt(1 - 3 r0^2),
// w(ic) = (1+q)/3 and w(ic+-1) = (2 +- 3 r0 - q)/6.  Interpolation and
// spreading use this one function, so they are exact adjoints.
template <typename T>
__device__ inline void kernel3(double s, int &ic, T w[3]) {
  const double c = floor(s + 0.5);
  ic = (int)c;
  const T r = (T)(s - c);
  const T q = sqrt((T)1 - (T)3 * r * r);
  w[0] = ((T)2 - (T)3 * r - q) * (T)(1.0 / 6.0);
  w[1] = ((T)1 + q) * (T)(1.0 / 3.0);
  w[2] = ((T)2 + (T)3 * r - q) * (T)(1.0 / 6.0);
}

// Staggering of component c in units of h: u on x-faces, v on y-faces, w on
// z-faces.
__device__ inline double stagger(int c, int axis) { return c == axis ? 0.0 : 0.5; }

// Stencil of one marker for one component: centre node per axis (unwrapped)
// and the three weights per axis.
template <typename T>
struct Stencil {
  int ic[3];
  T w[3][3];
};

template <typename T>
__device__ inline void make_stencil(const Geom &G, int c, const double X[3], Stencil<T> &S) {
  for (int a = 0; a < 3; ++a) kernel3<T>(X[a] * G.inv_h - stagger(c, a), S.ic[a], S.w[a]);
}

// First node row of the brick of a sphere of centre xc for component c along
// one axis: the lowest stencil node any marker of the sphere can reach.
__device__ inline int brick_lo(double xc, double R, double inv_h, double o) {
  return (int)floor((xc - R) * inv_h - o + 0.5) - 1;
}

// ---- per-sphere block reductions -----------------------------------------
// 6 compensated pairs (force and torque sums) + 2 plain sums.
struct Red {
  double s[6], c[6];
  double q[2];
};

__device__ inline void red_zero(Red &r) {
  for (int k = 0; k < 6; ++k) r.s[k] = r.c[k] = 0.0;
  r.q[0] = r.q[1] = 0.0;
}

__device__ inline void red_set_ft(Red &r, const double rl[3], const double d[3]) {
  r.s[0] = d[0];
  r.s[1] = d[1];
  r.s[2] = d[2];
  r.s[3] = rl[1] * d[2] - rl[2] * d[1];
  r.s[4] = rl[2] * d[0] - rl[0] * d[2];
  r.s[5] = rl[0] * d[1] - rl[1] * d[0];
}

// Inside a wave a plain FP64 butterfly (at most 6 roundings per term, far
// below the single-precision inputs' own error); the compensated sums start
// at the cross-wave level.
__device__ inline void wave_reduce(Red &r) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 6; ++k) r.s[k] += __shfl_xor(r.s[k], off);
    r.q[0] += __shfl_xor(r.q[0], off);
    r.q[1] += __shfl_xor(r.q[1], off);
  }
}

// Result valid in thread 0.  All threads of the block must call it.
__device__ inline void block_reduce(Red &r) {
  __shared__ double lds[16][14];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  wave_reduce(r);
  if (lane == 0) {
    for (int k = 0; k < 6; ++k) {
      lds[wave][k] = r.s[k];
      lds[wave][6 + k] = r.c[k];
    }
    lds[wave][12] = r.q[0];
    lds[wave][13] = r.q[1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int wv = 1; wv < nw; ++wv) {
      for (int k = 0; k < 6; ++k) comp_add(r.s[k], r.c[k], lds[wv][k], lds[wv][6 + k]);
      r.q[0] += lds[wv][12];
      r.q[1] += lds[wv][13];
    }
  }
}

}  // namespace prs
