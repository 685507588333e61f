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
