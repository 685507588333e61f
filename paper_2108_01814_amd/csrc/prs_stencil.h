// Delta-kernel stencils and block reductions shared by the interpolation and
// spreading kernels.
#pragma once

#include "prs_device.h"

namespace prs {

// ---- stencil geometry shared by the interpolation and the spreading ------
// Both operations evaluate a marker's delta-kernel weights with the same
// arithmetic from the same inputs, so they are exact adjoints:
//   - the sphere centre in node units, s = x / h, is split once per sphere
//     into an integer node I = floor(s) and a fraction phi = s - I in [0, 1)
//     (double precision), and fo = phi - o for the two staggering offsets
//     o = 0 (the component along the axis) and o = 1/2 (the other two),
//     rounded to the grid precision;
//   - the marker offset (R / h) t_l in node units is a per-template value
//     (m_hi + m_lo in single precision: m_hi = the offset rounded, m_lo its
//     remainder; m_lo = 0 in double precision);
//   - the stencil centre c = floor(fo + m_hi + 1/2) and the offset of the
//     marker from it, r = ((m_hi - c) + fo) + m_lo, which is within a few
//     rounding errors of the exact offset even though |fo + m| reaches R/h
//     (m_hi - c is exact or nearly so, and |r| <= 1/2);
//   - the three-point kernel (regularised delta function) at the nodes
//     I + c - 1, I + c, I + c + 1: with q = sqrt(1 - 3 r^2),
//     w(c) = (1 + q) / 3, w(c -+ 1) = (2 -+ 3 r - q) / 6, evaluated as
//     (2 - q) / 6 -+ r / 2.
// Near r = +-1/2 the floor may pick either neighbour; both choices give the
// same weights on the same nodes (w = 0, 1/2, 1/2 and 1/2, 1/2, 0), so the
// stencil is continuous there.

// Integer node and staggered fractions of one coordinate of a sphere centre.
template <typename T>
__device__ inline void sphere_axis(double x, double inv_h, int &I, T fo[2]) {
  const double s = x * inv_h;
  const double fl = floor(s);
  I = (int)fl;
  const T phi = (T)(s - fl);
  fo[0] = phi;
  fo[1] = phi - (T)0.5;
}

// Square root of the kernel's 1 - 3 r^2 (in [1/4, 1]): the hardware
// instruction in single precision (within about one unit in the last place;
// the correctly rounded library form costs a dozen more instructions per
// stencil), the correctly rounded one in double precision.
__device__ inline float kernel_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double kernel_sqrt(double x) { return sqrt(x); }

// Stencil along one axis: centre offset c (nodes I + c - 1 .. I + c + 1)
// and the three weights.  Written with explicit fused operations so that
// every inlined copy rounds identically.
template <typename T>
__device__ inline int stencil_axis(T fo, T mhi, T mlo, T w[3]) {
  const T cf = floor((fo + mhi) + (T)0.5);
  const T r = ((mhi - cf) + fo) + mlo;
  const T q = kernel_sqrt(fma((T)-3 * r, r, (T)1));
  const T a6 = fma(q, (T)(-1.0 / 6.0), (T)(1.0 / 3.0));   // (2 - q) / 6
  w[0] = fma((T)-0.5, r, a6);
  w[1] = fma(q, (T)(1.0 / 3.0), (T)(1.0 / 3.0));
  w[2] = fma((T)0.5, r, a6);
  return (int)cf;
}

// Staggering index of component c along axis a: 0 for the component along
// the axis (nodes on cell faces), 1 for the others (cell centres).
__device__ inline constexpr int stag(int c, int a) { return c == a ? 0 : 1; }

// Per-template marker offsets in node units, float4 pairs (hi xyz, lo xyz)
// in single precision or one double4 (xyz) in double precision.
template <typename T>
struct MarkerOffset;
template <>
struct MarkerOffset<float> {
  __device__ static inline void load(const float *tm, int l, float hi[3], float lo[3]) {
    const float4 a = reinterpret_cast<const float4 *>(tm)[2 * l];
    const float4 b = reinterpret_cast<const float4 *>(tm)[2 * l + 1];
    hi[0] = a.x; hi[1] = a.y; hi[2] = a.z;
    lo[0] = b.x; lo[1] = b.y; lo[2] = b.z;
  }
};
template <>
struct MarkerOffset<double> {
  __device__ static inline void load(const double *tm, int l, double hi[3], double lo[3]) {
    const double *p = tm + 4 * l;
    hi[0] = p[0]; hi[1] = p[1]; hi[2] = p[2];
    lo[0] = lo[1] = lo[2] = 0.0;
  }
};

// Brick of one sphere in the interpolation: nodes I - E .. I - E + nb - 1 per
// axis, with E = ceil(R/h) + 1 and nb = 2 ceil(R/h) + 4, which holds every
// node of every marker's stencil (|m| < R/h, fo in [-1/2, 1)).
__host__ __device__ inline int brick_reach(double R, double h) { return (int)ceil(R / h - 1e-9) + 1; }

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

__device__ inline void red_add_ft(Red &r, const double rl[3], const double d[3]) {
  r.v[0] += d[0];
  r.v[1] += d[1];
  r.v[2] += d[2];
  r.v[3] += rl[1] * d[2] - rl[2] * d[1];
  r.v[4] += rl[2] * d[0] - rl[0] * d[2];
  r.v[5] += rl[0] * d[1] - rl[1] * d[0];
}

// Wave sums of eight columns at once, each step halving the columns a lane
// carries: a lane keeps one half and adds its partner's copy of that half
// (partners differ in lane bit 0, then bit 1), so the last four steps move
// two values instead of eight.  The steps over lane bits 2 and 3 rotate
// within a row, those over bits 4 and 5 cross rows through the LDS
// crossbar.  On return every lane holds the wave sums of columns
// 4 b0 + 2 b1 and 4 b0 + 2 b1 + 1 (b0, b1: bits 0 and 1 of its lane), in
// w0 and w1.  Every lane of the wave must be active.
__device__ inline void wave_sum8(const double v[8], double &w0, double &w1) {
  const int lane = threadIdx.x & 63;
  const bool b0 = lane & 1, b1 = (lane >> 1) & 1;
  double a[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double keep = b0 ? v[i + 4] : v[i];
    const double send = b0 ? v[i] : v[i + 4];
    a[i] = keep + dpp_move<kDppXor1, 0xF>(send);
  }
  double b[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double keep = b1 ? a[i + 2] : a[i];
    const double send = b1 ? a[i] : a[i + 2];
    b[i] = keep + dpp_move<kDppXor2, 0xF>(send);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    b[i] += dpp_move<kDppRor4, 0xF>(b[i]);
    b[i] += dpp_move<kDppRor8, 0xF>(b[i]);
    b[i] += __shfl_xor(b[i], 16);
    b[i] += __shfl_xor(b[i], 32);
  }
  w0 = b[0];
  w1 = b[1];
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
  if constexpr (__builtin_popcount(MASK) >= 4) {
    double w0, w1;
    wave_sum8(r.v, w0, w1);
    if (lane < 4) {
      const int c0 = 4 * (lane & 1) + 2 * (lane >> 1);
      if ((MASK >> c0) & 1u) lds[wave][c0] = w0;
      if ((MASK >> (c0 + 1)) & 1u) lds[wave][c0 + 1] = w1;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if ((MASK >> k) & 1u) r.v[k] = wave_sum_last(r.v[k]);
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if ((MASK >> k) & 1u) lds[wave][k] = r.v[k];
    }
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
