// Device helpers shared by the HIP translation units of the library.
#pragma once

#include "prs_internal.h"

namespace prs {

// Grid-stride style XCD-aware mapping: consecutive block ids are dispatched
// round-robin over the 8 XCDs, so give every XCD a contiguous run of work
// items (spheres in cell order) to keep neighbouring spheres in one L2.
__device__ inline int xcd_item(int block, int n) {
  const int per = (n + 7) >> 3;
  const int item = (block & 7) * per + (block >> 3);
  return item < n ? item : -1;
}

inline int xcd_grid(int n) { return 8 * ((n + 7) >> 3); }

// Error-free sum of two doubles (Knuth's TwoSum).
__device__ inline void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Compensated accumulation of (s2, c2) into (s, c).
__device__ inline void comp_add(double &s, double &c, double s2, double c2) {
  double t, e;
  two_sum(s, s2, t, e);
  s = t;
  c = c + c2 + e;
}

// max(a, b) that keeps a NaN of either argument.
__device__ inline float nan_max(float a, float b) { return (b > a || b != b) ? b : a; }

// ---- wave reductions on DPP lane moves (VALU only, no LDS traffic) -------
// A DPP move reads another lane of the same wave; rows are 16 lanes.  Lanes
// of rows outside ROW_MASK receive 0.  Every lane of the wave must be active.
enum : int {
  kDppXor1 = 0xB1,          // quad_perm [1,0,3,2]
  kDppXor2 = 0x4E,          // quad_perm [2,3,0,1]
  kDppHalfMirror = 0x141,   // lane i <- 7 - i within each 8 lanes
  kDppMirror = 0x140,       // lane i <- 15 - i within each row
  kDppBcast15 = 0x142,      // lane 15 of each row -> the next row
  kDppBcast31 = 0x143,      // lane 31 -> rows 2 and 3
  kDppRor4 = 0x124,         // lane i <- (i + 4) mod 16 within each row
  kDppRor8 = 0x128,         // lane i <- (i + 8) mod 16 within each row
};

// One 32-bit word: with every row written (ROW_MASK 0xF) the plain move,
// else the update with 0 for the lanes of the rows left out.
template <int CTRL, int ROW_MASK>
__device__ inline int dpp_word(int v) {
  if constexpr (ROW_MASK == 0xF)
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
  else
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK>
__device__ inline double dpp_move(double v) {
  const int lo = dpp_word<CTRL, ROW_MASK>(__double2loint(v));
  const int hi = dpp_word<CTRL, ROW_MASK>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

template <int CTRL, int ROW_MASK>
__device__ inline float dpp_move(float v) {
  return __int_as_float(dpp_word<CTRL, ROW_MASK>(__float_as_int(v)));
}

template <int CTRL, int ROW_MASK>
__device__ inline int dpp_move(int v) {
  return dpp_word<CTRL, ROW_MASK>(v);
}

// Sum over the wave, valid in lane 63: butterflies inside each quad, mirrors
// fold quads into rows, row broadcasts fold rows 0..2 into row 3.
template <typename T>
__device__ inline T wave_sum_last(T v) {
  v += dpp_move<kDppXor1, 0xF>(v);
  v += dpp_move<kDppXor2, 0xF>(v);
  v += dpp_move<kDppHalfMirror, 0xF>(v);
  v += dpp_move<kDppMirror, 0xF>(v);
  v += dpp_move<kDppBcast15, 0xA>(v);
  v += dpp_move<kDppBcast31, 0xC>(v);
  return v;
}

// |v| as its bit pattern: for values with the sign bit clear the unsigned
// order of the patterns is the numeric order, and every NaN sorts above
// +inf, so the largest pattern is the largest |v| or a NaN.
__device__ inline unsigned abs_bits(float v) { return __float_as_uint(fabsf(v)); }

// Largest pattern over the wave, valid in lane 63.
__device__ inline unsigned wave_max_last(unsigned v) {
  v = max(v, (unsigned)dpp_move<kDppXor1, 0xF>((int)v));
  v = max(v, (unsigned)dpp_move<kDppXor2, 0xF>((int)v));
  v = max(v, (unsigned)dpp_move<kDppHalfMirror, 0xF>((int)v));
  v = max(v, (unsigned)dpp_move<kDppMirror, 0xF>((int)v));
  v = max(v, (unsigned)dpp_move<kDppBcast15, 0xA>((int)v));
  v = max(v, (unsigned)dpp_move<kDppBcast31, 0xC>((int)v));
  return v;
}

__device__ inline int wrap_once(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

__device__ inline double min_image(double d, double L) {
  if (d > 0.5 * L)
    d -= L;
  else if (d < -0.5 * L)
    d += L;
  return d;
}

__device__ inline int cell_coord(double v, double cs, int n) {
  int c = (int)floor(v / cs);
  return c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
}

__device__ inline int cell_key(const Cells &C, int cx, int cy, int cz) {
  const int tile = ((cz >> 2) * C.nty + (cy >> 2)) * C.ntx + (cx >> 2);
  const int m = (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2) | ((cx & 2) << 2) | ((cy & 2) << 3) |
                ((cz & 2) << 4);
  return tile * 64 + m;
}

// Sanitise one coordinate of a sphere centre: returns a value that keeps
// every index computation in bounds and reports what was wrong.
__device__ inline double sane_coord(double v, double L, bool closed, uint32_t &flags) {
  if (!isfinite(v)) {
    flags |= kFlagNonFinite;
    return 0.0;
  }
  if (v < 0.0 || (closed ? v > L : v >= L)) {
    flags |= kFlagDomain;
    return 0.0;
  }
  return v;
}

}  // namespace prs
