// Fluid inside the spheres: the fluid velocity and its moment about the
// centre integrated over each sphere's volume, the momentum whose rate of
// change joins minus the marker forces in the hydrodynamic force of the
// direct-forcing method (eqs. 7-8).  The integral is the midpoint rule over
// the staggered nodes inside the sphere, |x_n - x_p| < R with the minimum
// image in x and z, each weighted h^3 (wall faces and nodes outside the
// fluid excluded).
//
// One workgroup per sphere; threads stride over the nodes of the box that
// holds the sphere, per component.  Compiled with -ffp-contract=off: the
// inside test (dx dx + dy dy) + dz dz < R^2 is evaluated exactly as written,
// so the set of nodes is reproducible bit for bit.
#include "prs_device.h"

namespace prs {

constexpr int kInnerThreads = 256;

// Integrals over sphere p of the field a + adt b (b == nullptr: a alone):
// out[0..2] = h^3 sum u_c, out[3..5] = h^3 sum r x (e_c u_c).  On return
// thread 0 holds them.  xc: the centre.
template <typename T>
__device__ inline void inner_sums(const Geom &G, const T *const a[3], const T *const b[3],
                                  double adt, const double xc[3], double out[6]) {
  __shared__ double red[kInnerThreads / 64][6];
  const double h = G.h, R = G.R;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int c = 0; c < 3; ++c) {
    const double o[3] = {c == 0 ? 0.0 : 0.5, c == 1 ? 0.0 : 0.5, c == 2 ? 0.0 : 0.5};
    long lo[3], ext[3];
    for (int q = 0; q < 3; ++q) {
      lo[q] = (long)floor((xc[q] - R) / h - o[q]) - 1;
      ext[q] = (long)floor((xc[q] + R) / h - o[q]) + 1 - lo[q] + 1;
    }
    const int nyc = G.ny + (c == 1 ? 1 : 0);
    const long count = ext[0] * ext[1] * ext[2];
    for (long e = threadIdx.x; e < count; e += blockDim.x) {
      const long i = lo[0] + e % ext[0];
      const long j = lo[1] + (e / ext[0]) % ext[1];
      const long k = lo[2] + e / (ext[0] * ext[1]);
      const double r0 = min_image(((double)i + o[0]) * h - xc[0], G.Lx);
      const double r1 = ((double)j + o[1]) * h - xc[1];
      const double r2 = min_image(((double)k + o[2]) * h - xc[2], G.Lz);
      if (!((r0 * r0 + r1 * r1) + r2 * r2 < R * R)) continue;
      if (c == 1 ? (j < 1 || j > G.ny - 1) : (j < 0 || j > G.ny - 1)) continue;
      long iw = i % G.nx, kw = k % G.nz;
      if (iw < 0) iw += G.nx;
      if (kw < 0) kw += G.nz;
      const size_t g = ((size_t)kw * nyc + (size_t)j) * G.nx + (size_t)iw;
      double uc = (double)a[c][g];
      if (b) uc += adt * (double)b[c][g];
      acc[c] += uc;
      if (c == 0) {
        acc[4] += r2 * uc;
        acc[5] -= r1 * uc;
      } else if (c == 1) {
        acc[3] -= r2 * uc;
        acc[5] += r0 * uc;
      } else {
        acc[3] += r1 * uc;
        acc[4] -= r0 * uc;
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = 0; q < 6; ++q) {
    const double v = wave_sum_last(acc[q]);
    if (lane == 63) red[wave][q] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double h3 = h * h * h;
    for (int q = 0; q < 6; ++q) {
      double s = red[0][q];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s += red[w][q];
      out[q] = h3 * s;
    }
  }
}

// Caller-ordered spheres: inner[i][6] of the field a.
template <typename T>
__global__ __launch_bounds__(kInnerThreads) void k_inner_fluid(Geom G, const T *a0, const T *a1,
                                                               const T *a2,
                                                               const double *__restrict__ x,
                                                               int n, double *inner,
                                                               uint32_t *status) {
  const int p = xcd_item(blockIdx.x, n);
  if (p < 0) return;
  uint32_t fl = 0;
  const double xc[3] = {sane_coord(x[3 * p], G.Lx, false, fl),
                        sane_coord(x[3 * p + 1], G.Ly, true, fl),
                        sane_coord(x[3 * p + 2], G.Lz, false, fl)};
  if (fl && threadIdx.x == 0) atomicOr(status, fl);
  const T *a[3] = {a0, a1, a2};
  const T *b[3] = {nullptr, nullptr, nullptr};
  double out[6];
  inner_sums<T>(G, a, nullptr, 0.0, xc, out);
  (void)b;
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) inner[6 * (size_t)p + q] = out[q];
}

// Sorted spheres inside the step: integrals of u** = u-hat + adt f; adds
// rho_f (I - I_prev) / adt to the sorted hydrodynamic force and torque
// (prev nullable: no term) and writes I to inner_out (nullable), both in
// caller order.
template <typename T>
__global__ __launch_bounds__(kInnerThreads) void k_inner_step(
    Geom G, const T *a0, const T *a1, const T *a2, const T *b0, const T *b1, const T *b2,
    double adt, double rho_f, const double *__restrict__ xs, const int *__restrict__ perm, int n,
    const double *__restrict__ prev, double *inner_out, double *fh, double *th) {
  const int p = xcd_item(blockIdx.x, n);
  if (p < 0) return;
  const size_t N = (size_t)n;
  const double xc[3] = {xs[p], xs[N + p], xs[2 * N + p]};
  const T *a[3] = {a0, a1, a2};
  const T *b[3] = {b0, b1, b2};
  double out[6];
  inner_sums<T>(G, a, b, adt, xc, out);
  if (threadIdx.x == 0) {
    const size_t i = (size_t)perm[p];
    if (prev)
      for (int q = 0; q < 3; ++q) {
        fh[q * N + p] += rho_f * (out[q] - prev[6 * i + q]) / adt;
        th[q * N + p] += rho_f * (out[3 + q] - prev[6 * i + 3 + q]) / adt;
      }
    if (inner_out)
      for (int q = 0; q < 6; ++q) inner_out[6 * i + q] = out[q];
  }
}

template <typename T>
hipError_t launch_inner_fluid(hipStream_t s, const Geom &G, const Scratch &S, const T *u[3],
                              const double *x, int n, double *inner) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_inner_fluid<T>, dim3(xcd_grid(n)), dim3(kInnerThreads), 0, s, G, u[0],
                     u[1], u[2], x, n, inner, S.status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_inner_step(hipStream_t s, const Geom &G, const Scratch &S, const T *uh[3],
                             const T *f[3], double adt, double rho_f, int n, const double *prev,
                             double *inner_out) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_inner_step<T>, dim3(xcd_grid(n)), dim3(kInnerThreads), 0, s, G, uh[0],
                     uh[1], uh[2], f[0], f[1], f[2], adt, rho_f, S.xs[0], S.perm, n, prev,
                     inner_out, S.fh, S.th);
  return hipGetLastError();
}

template hipError_t launch_inner_fluid<float>(hipStream_t, const Geom &, const Scratch &,
                                              const float *[3], const double *, int, double *);
template hipError_t launch_inner_fluid<double>(hipStream_t, const Geom &, const Scratch &,
                                               const double *[3], const double *, int, double *);
template hipError_t launch_inner_step<float>(hipStream_t, const Geom &, const Scratch &,
                                             const float *[3], const float *[3], double, double,
                                             int, const double *, double *);
template hipError_t launch_inner_step<double>(hipStream_t, const Geom &, const Scratch &,
                                              const double *[3], const double *[3], double,
                                              double, int, const double *, double *);

}  // namespace prs
