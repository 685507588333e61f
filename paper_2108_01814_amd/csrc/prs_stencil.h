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
// Eight columns per lane: the force and torque terms (0..5) and two slip
// sums (6: with forcing, 7: zero forcing).
enum { kColF = 0, kColSlip = 6, kColSlip0 = 7 };
struct Red {
  double v[8];
};

__device__ inline void red_zero(Red &r) {
  for (int k = 0; k < 8; ++k) r.v[k] = 0.0;
}

__device__ inline void red_set_ft(Red &r, const double rl[3], const double d[3]) {
  r.v[0] = d[0];
  r.v[1] = d[1];
  r.v[2] = d[2];
  r.v[3] = rl[1] * d[2] - rl[2] * d[1];
  r.v[4] = rl[2] * d[0] - rl[0] * d[2];
  r.v[5] = rl[0] * d[1] - rl[1] * d[0];
}

// Block sums of the columns in MASK: a plain FP64 sum inside each wave (at
// most 6 roundings per term, far below the single-precision inputs' own
// error), compensated across waves.  On return thread t < 8 holds column t's
// sum as a compensated pair (s, c); other threads get zeros.  All threads of
// the block must call it; blockDim.x is a multiple of 64.
template <unsigned MASK>
__device__ inline void block_reduce(Red &r, double &s, double &c) {
  __shared__ double lds[16][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if ((MASK >> k) & 1u) r.v[k] = wave_sum_last(r.v[k]);
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if ((MASK >> k) & 1u) lds[wave][k] = r.v[k];
  }
  __syncthreads();
  s = c = 0.0;
  const int t = threadIdx.x;
  if (t < 8 && ((MASK >> t) & 1u)) {
    s = lds[0][t];
    for (int wv = 1; wv < nw; ++wv) comp_add(s, c, lds[wv][t], 0.0);
  }
}

}  // namespace prs
