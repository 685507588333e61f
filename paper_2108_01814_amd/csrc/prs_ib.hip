// Immersed-boundary kernels: marker template, interpolation of the staggered
// fluid velocity at the Lagrangian markers, the direct-forcing correction,
// and diffusion (spreading) of marker forces back to the grid (sec. 3.3 and
// eq. 4 of the paper; the regularised delta function is the three-point
// kernel, the iteration is multi-direct forcing in Jacobi form).
//
// Work decomposition: one workgroup per sphere, one lane per marker, so
// every workgroup carries the same number of markers however dense the bed
// is around it (the marker-based balancing of sec. 3.3 on one GPU), and the
// per-sphere force and torque are workgroup reductions.
#include "prs_device.h"

namespace prs {

// ---------------------------------------------------------------------------
// template
// ---------------------------------------------------------------------------
__global__ void k_template(double *t, int nl) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nl) return;
  const double golden = M_PI * (3.0 - sqrt(5.0));
  const double zp = 1.0 - (2.0 * l + 1.0) / nl;
  const double rho = sqrt(1.0 - zp * zp);
  const double th = l * golden;
  t[3 * l + 0] = rho * cos(th);
  t[3 * l + 1] = zp;
  t[3 * l + 2] = rho * sin(th);
}

hipError_t launch_template(hipStream_t s, double *t, int nl) {
  hipLaunchKernelGGL(k_template, dim3((nl + 255) / 256), dim3(256), 0, s, t, nl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stencil of one marker for one staggered component
// ---------------------------------------------------------------------------
// Three-point kernel weights of the nodes ic-1, ic, ic+1 for the offset
// r0 = s - ic in [-1/2, 1/2) (s in node units): with q = sqrt(1 - 3 r0^2),
// w(ic) = (1+q)/3 and w(ic+-1) = (2 +- 3 r0 - q)/6.
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

template <typename T>
struct Stencil {
  int ix[3];
  int kz[3];
  int j0;        // first row (may be out of range; masked by jok)
  bool jok[3];
  T wx[3], wy[3], wz[3];
  int nyc;
};

template <typename T>
__device__ inline void make_stencil(const Geom &G, int c, const double X[3], Stencil<T> &S) {
  const double ox = c == 0 ? 0.0 : 0.5, oy = c == 1 ? 0.0 : 0.5, oz = c == 2 ? 0.0 : 0.5;
  int icx, icy, icz;
  kernel3<T>(X[0] * G.inv_h - ox, icx, S.wx);
  kernel3<T>(X[1] * G.inv_h - oy, icy, S.wy);
  kernel3<T>(X[2] * G.inv_h - oz, icz, S.wz);
  for (int a = 0; a < 3; ++a) {
    S.ix[a] = wrap_once(icx - 1 + a, G.nx);
    S.kz[a] = wrap_once(icz - 1 + a, G.nz);
  }
  S.j0 = icy - 1;
  const int jlo = (c == 1) ? 1 : 0;
  for (int a = 0; a < 3; ++a) {
    const int j = S.j0 + a;
    S.jok[a] = (j >= jlo) && (j <= G.ny - 1);
  }
  S.nyc = G.ny + (c == 1 ? 1 : 0);
}

// a1 = I[g1], a2 = I[g2] (g2 may be null).
template <typename T, bool TWO>
__device__ inline void gather(const Geom &G, const Stencil<T> &S, const T *__restrict__ g1,
                              const T *__restrict__ g2, T &a1, T &a2) {
  T s1 = 0, s2 = 0;
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      if (!S.jok[jj]) continue;
      const size_t row = ((size_t)S.kz[kk] * S.nyc + (size_t)(S.j0 + jj)) * (size_t)G.nx;
      const T wzy = S.wz[kk] * S.wy[jj];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        const T w = wzy * S.wx[ii];
        s1 += g1[row + S.ix[ii]] * w;
        if (TWO) s2 += g2[row + S.ix[ii]] * w;
      }
    }
  }
  a1 = s1;
  a2 = s2;
}

template <typename T>
__device__ inline void scatter(const Geom &G, const Stencil<T> &S, T *__restrict__ g, T val) {
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      if (!S.jok[jj]) continue;
      const size_t row = ((size_t)S.kz[kk] * S.nyc + (size_t)(S.j0 + jj)) * (size_t)G.nx;
      const T wzy = S.wz[kk] * S.wy[jj];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) atomicAdd(&g[row + S.ix[ii]], val * (wzy * S.wx[ii]));
    }
  }
}

__device__ inline void load_sphere_aos(const Geom &G, const double *x, const double *up,
                                       const double *om, int p, double xp[3], double u[3],
                                       double w[3]) {
  uint32_t fl = 0;
  xp[0] = sane_coord(x[3 * p + 0], G.Lx, false, fl);
  xp[1] = sane_coord(x[3 * p + 1], G.Ly, true, fl);
  xp[2] = sane_coord(x[3 * p + 2], G.Lz, false, fl);
  for (int a = 0; a < 3; ++a) {
    u[a] = up ? up[3 * p + a] : 0.0;
    w[a] = om ? om[3 * p + a] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// plain interpolation / spreading (caller order, one field set)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_interp_plain(Geom G, const double *__restrict__ templ,
                                                       const T *__restrict__ gu,
                                                       const T *__restrict__ gv,
                                                       const T *__restrict__ gw,
                                                       const double *x, const double *up,
                                                       const double *om, int n, T *U, T *Ud) {
  const int p = xcd_item(blockIdx.x, n);
  const int l = threadIdx.x;
  if (p < 0 || l >= G.nl) return;
  double xp[3], u[3], w[3];
  load_sphere_aos(G, x, up, om, p, xp, u, w);
  const double r[3] = {G.R * templ[3 * l], G.R * templ[3 * l + 1], G.R * templ[3 * l + 2]};
  const double X[3] = {xp[0] + r[0], xp[1] + r[1], xp[2] + r[2]};
  const T *g[3] = {gu, gv, gw};
  const size_t m = (size_t)p * G.nl + l;
  for (int c = 0; c < 3; ++c) {
    Stencil<T> S;
    make_stencil<T>(G, c, X, S);
    T a, b;
    gather<T, false>(G, S, g[c], nullptr, a, b);
    U[3 * m + c] = a;
  }
  if (Ud) {
    Ud[3 * m + 0] = (T)(u[0] + (w[1] * r[2] - w[2] * r[1]));
    Ud[3 * m + 1] = (T)(u[1] + (w[2] * r[0] - w[0] * r[2]));
    Ud[3 * m + 2] = (T)(u[2] + (w[0] * r[1] - w[1] * r[0]));
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_spread_plain(Geom G, const double *__restrict__ templ,
                                                       const double *x, int n,
                                                       const T *__restrict__ F, T *fu, T *fv,
                                                       T *fw) {
  const int p = xcd_item(blockIdx.x, n);
  const int l = threadIdx.x;
  if (p < 0 || l >= G.nl) return;
  double xp[3], u[3], w[3];
  load_sphere_aos(G, x, nullptr, nullptr, p, xp, u, w);
  const double X[3] = {xp[0] + G.R * templ[3 * l], xp[1] + G.R * templ[3 * l + 1],
                       xp[2] + G.R * templ[3 * l + 2]};
  const T scale = (T)(G.dV * G.inv_h * G.inv_h * G.inv_h);
  T *g[3] = {fu, fv, fw};
  const size_t m = (size_t)p * G.nl + l;
  for (int c = 0; c < 3; ++c) {
    Stencil<T> S;
    make_stencil<T>(G, c, X, S);
    scatter<T>(G, S, g[c], F[3 * m + c] * scale);
  }
}

static inline int block_for(int nl) { return ((nl + 63) / 64) * 64; }

template <typename T>
hipError_t launch_interp_plain(hipStream_t s, const Geom &G, const double *templ, const T *gu,
                               const T *gv, const T *gw, const double *x, const double *up,
                               const double *om, int n, T *U, T *Ud) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_interp_plain<T>, dim3(xcd_grid(n)), dim3(block_for(G.nl)), 0, s, G, templ,
                     gu, gv, gw, x, up, om, n, U, Ud);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread_plain(hipStream_t s, const Geom &G, const double *templ, const double *x,
                               int n, const T *F, T *fu, T *fv, T *fw) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spread_plain<T>, dim3(xcd_grid(n)), dim3(block_for(G.nl)), 0, s, G, templ,
                     x, n, F, fu, fv, fw);
  return hipGetLastError();
}

template hipError_t launch_interp_plain<float>(hipStream_t, const Geom &, const double *,
                                               const float *, const float *, const float *,
                                               const double *, const double *, const double *,
                                               int, float *, float *);
template hipError_t launch_interp_plain<double>(hipStream_t, const Geom &, const double *,
                                                const double *, const double *, const double *,
                                                const double *, const double *, const double *,
                                                int, double *, double *);
template hipError_t launch_spread_plain<float>(hipStream_t, const Geom &, const double *,
                                               const double *, int, const float *, float *,
                                               float *, float *);
template hipError_t launch_spread_plain<double>(hipStream_t, const Geom &, const double *,
                                                const double *, int, const double *, double *,
                                                double *, double *);

// ---------------------------------------------------------------------------
// block reduction of the per-marker force/torque and slip contributions
// ---------------------------------------------------------------------------
// v: 6 compensated pairs (force, torque) + 2 plain sums (slip^2, zero-forcing
// slip^2).  Result valid in thread 0.
struct Red {
  double s[6], c[6];
  double q[2];
};

__device__ inline void wave_reduce(Red &r) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double s2 = __shfl_xor(r.s[k], off);
      const double c2 = __shfl_xor(r.c[k], off);
      comp_add(r.s[k], r.c[k], s2, c2);
    }
    r.q[0] += __shfl_xor(r.q[0], off);
    r.q[1] += __shfl_xor(r.q[1], off);
  }
}

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

// ---------------------------------------------------------------------------
// multi-direct forcing on the sorted spheres
// ---------------------------------------------------------------------------
// Interpolation pass of one iteration.  u** = u-hat + alpha dt f is formed on
// the fly from the two fields.  Per marker: U = I[u**], r = U_d - U,
// dF = r/(alpha dt) stored for the spreading pass; per sphere: the slip
// partials (sum of r^2, and of (U_d - I[u-hat])^2 for the relative slip).
template <typename T>
__global__ __launch_bounds__(1024) void k_interp_mdf(
    Geom G, const double *__restrict__ templ, const T *__restrict__ uh0,
    const T *__restrict__ uh1, const T *__restrict__ uh2, const T *__restrict__ f0,
    const T *__restrict__ f1, const T *__restrict__ f2, const double *__restrict__ xs,
    const double *__restrict__ us, const double *__restrict__ ws, int n, double adt,
    T *__restrict__ dF, double *__restrict__ slip_part) {
  const int p = xcd_item(blockIdx.x, n);
  if (p < 0) return;
  const int l = threadIdx.x;
  Red red;
  for (int k = 0; k < 6; ++k) red.s[k] = red.c[k] = 0.0;
  red.q[0] = red.q[1] = 0.0;
  if (l < G.nl) {
    const double r[3] = {G.R * templ[3 * l], G.R * templ[3 * l + 1], G.R * templ[3 * l + 2]};
    const double X[3] = {xs[p] + r[0], xs[n + p] + r[1], xs[2 * n + p] + r[2]};
    const double w[3] = {ws[p], ws[n + p], ws[2 * n + p]};
    const double Ud[3] = {us[p] + (w[1] * r[2] - w[2] * r[1]),
                          us[n + p] + (w[2] * r[0] - w[0] * r[2]),
                          us[2 * n + p] + (w[0] * r[1] - w[1] * r[0])};
    const T *uh[3] = {uh0, uh1, uh2};
    const T *ff[3] = {f0, f1, f2};
    const size_t M = (size_t)n * G.nl;
    const size_t m = (size_t)p * G.nl + l;
    const T tadt = (T)adt;
    for (int c = 0; c < 3; ++c) {
      Stencil<T> S;
      make_stencil<T>(G, c, X, S);
      T iu, ifc;
      gather<T, true>(G, S, uh[c], ff[c], iu, ifc);
      const T U = iu + tadt * ifc;
      const T res = (T)Ud[c] - U;
      const T corr = res / tadt;
      dF[c * M + m] = corr;
      red.q[0] += (double)res * (double)res;
      const double z = Ud[c] - (double)iu;
      red.q[1] += z * z;
    }
  }
  block_reduce(red);
  if (threadIdx.x == 0) {
    slip_part[p] = red.q[0];
    slip_part[n + p] = red.q[1];
  }
}

// Spreading pass: f += S[dF] (sorted spheres, corrections from the buffer),
// and the compensated per-sphere sums of dF and (R t) x dF added to the
// force/torque accumulators; or, with F0 != null, the spread of a
// caller-ordered initial marker force whose sums seed the accumulators.
template <typename T>
__global__ __launch_bounds__(1024) void k_spread_mdf(Geom G, const double *__restrict__ templ,
                                                     const double *__restrict__ xs, int n,
                                                     const T *__restrict__ dF,
                                                     const T *__restrict__ F0,
                                                     const int *__restrict__ perm, T *f0, T *f1,
                                                     T *f2, double *__restrict__ acc) {
  const int p = xcd_item(blockIdx.x, n);
  if (p < 0) return;
  const int l = threadIdx.x;
  Red red;
  for (int k = 0; k < 6; ++k) red.s[k] = red.c[k] = 0.0;
  red.q[0] = red.q[1] = 0.0;
  if (l < G.nl) {
    const double r[3] = {G.R * templ[3 * l], G.R * templ[3 * l + 1], G.R * templ[3 * l + 2]};
    const double X[3] = {xs[p] + r[0], xs[n + p] + r[1], xs[2 * n + p] + r[2]};
    const size_t M = (size_t)n * G.nl;
    T v[3];
    if (F0) {
      const size_t mc = (size_t)perm[p] * G.nl + l;
      for (int c = 0; c < 3; ++c) v[c] = F0[3 * mc + c];
    } else {
      const size_t m = (size_t)p * G.nl + l;
      for (int c = 0; c < 3; ++c) v[c] = dF[c * M + m];
    }
    const T scale = (T)(G.dV * G.inv_h * G.inv_h * G.inv_h);
    T *g[3] = {f0, f1, f2};
    for (int c = 0; c < 3; ++c) {
      Stencil<T> S;
      make_stencil<T>(G, c, X, S);
      scatter<T>(G, S, g[c], v[c] * scale);
    }
    const double d[3] = {(double)v[0], (double)v[1], (double)v[2]};
    red.s[0] = d[0];
    red.s[1] = d[1];
    red.s[2] = d[2];
    red.s[3] = r[1] * d[2] - r[2] * d[1];
    red.s[4] = r[2] * d[0] - r[0] * d[2];
    red.s[5] = r[0] * d[1] - r[1] * d[0];
  }
  block_reduce(red);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 6; ++k) {
      double S = 0.0, C = 0.0;
      if (!F0) {
        S = acc[(2 * k) * (size_t)n + p];
        C = acc[(2 * k + 1) * (size_t)n + p];
      }
      comp_add(S, C, red.s[k], red.c[k]);
      acc[(2 * k) * (size_t)n + p] = S;
      acc[(2 * k + 1) * (size_t)n + p] = C;
    }
  }
}

template <typename T>
hipError_t launch_interp_mdf(hipStream_t s, const Geom &G, const Scratch &S, const T *uh[3],
                             const T *f[3], int n, double adt, int iter, int want_den) {
  (void)iter;
  (void)want_den;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_interp_mdf<T>, dim3(xcd_grid(n)), dim3(block_for(G.nl)), 0, s, G, S.templ,
                     uh[0], uh[1], uh[2], f[0], f[1], f[2], S.xs[0], S.us[0], S.ws[0], n, adt,
                     (T *)S.dF, S.slip_part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread_mdf(hipStream_t s, const Geom &G, const Scratch &S, T *f[3], int n,
                             const T *F0) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spread_mdf<T>, dim3(xcd_grid(n)), dim3(block_for(G.nl)), 0, s, G, S.templ,
                     S.xs[0], n, (const T *)S.dF, F0, S.perm, f[0], f[1], f[2], S.ft_acc);
  return hipGetLastError();
}

template hipError_t launch_interp_mdf<float>(hipStream_t, const Geom &, const Scratch &,
                                             const float *[3], const float *[3], int, double, int,
                                             int);
template hipError_t launch_interp_mdf<double>(hipStream_t, const Geom &, const Scratch &,
                                              const double *[3], const double *[3], int, double,
                                              int, int);
template hipError_t launch_spread_mdf<float>(hipStream_t, const Geom &, const Scratch &,
                                             float *[3], int, const float *);
template hipError_t launch_spread_mdf<double>(hipStream_t, const Geom &, const Scratch &,
                                              double *[3], int, const double *);

// ---------------------------------------------------------------------------
// bookkeeping
// ---------------------------------------------------------------------------
__global__ void k_zero_f64(double *p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t launch_ib_begin(hipStream_t s, const Scratch &S, int n) {
  const size_t count = 12 * (size_t)n;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f64, dim3(1024), dim3(256), 0, s, S.ft_acc, count);
  return hipGetLastError();
}

// Deterministic reduction of the per-sphere slip partials of one iteration
// into slip_hist[iter] (and the zero-forcing denominator into slot kMaxSlip).
__global__ __launch_bounds__(1024) void k_slip_reduce(const double *part, int n, double *hist,
                                                      int iter, int want_den) {
  __shared__ double lds[2][1024];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a += part[i];
    b += part[n + i];
  }
  lds[0][threadIdx.x] = a;
  lds[1][threadIdx.x] = b;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      lds[0][threadIdx.x] += lds[0][threadIdx.x + off];
      lds[1][threadIdx.x] += lds[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    hist[iter] = lds[0][0];
    if (want_den) hist[PRS_MAX_SLIP + 0] = lds[1][0];
  }
}

hipError_t launch_slip_reduce(hipStream_t s, const Scratch &S, int n, int iter, int want_den) {
  hipLaunchKernelGGL(k_slip_reduce, dim3(1), dim3(1024), 0, s, S.slip_part, n, S.slip_hist, iter,
                     want_den);
  return hipGetLastError();
}

__global__ void k_ib_finish(const double *acc, int n, double scale, double *fh, double *th) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  for (int a = 0; a < 3; ++a) {
    fh[a * (size_t)n + p] = scale * (acc[(2 * a) * (size_t)n + p] + acc[(2 * a + 1) * (size_t)n + p]);
    th[a * (size_t)n + p] =
        scale * (acc[(2 * (a + 3)) * (size_t)n + p] + acc[(2 * (a + 3) + 1) * (size_t)n + p]);
  }
}

hipError_t launch_ib_finish(hipStream_t s, const Scratch &S, const Geom &G, int n, double rho_f) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ib_finish, dim3((n + 255) / 256), dim3(256), 0, s, S.ft_acc, n,
                     -rho_f * G.dV, S.fh, S.th);
  return hipGetLastError();
}

template <typename T>
__global__ void k_fill_zero(T *p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = (T)0;
}

template <typename T>
hipError_t launch_fill_zero(hipStream_t s, T *p, size_t count) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_zero<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

template hipError_t launch_fill_zero<float>(hipStream_t, float *, size_t);
template hipError_t launch_fill_zero<double>(hipStream_t, double *, size_t);
template hipError_t launch_fill_zero<int>(hipStream_t, int *, size_t);

}  // namespace prs
