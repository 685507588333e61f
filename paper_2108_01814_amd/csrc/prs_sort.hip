// Mapping of spheres to collision cells (the "mapping" and "collision
// search" subprocedures of sec. 3.5): a counting sort of the spheres by cell
// number, cells numbered in 4x4x4 tiles with Morton order inside a tile, so
// spheres that are close in space are close in memory.  Also the copies
// between the caller's arrays (caller order, [n][3]) and the sorted
// structure-of-arrays state the kernels work on.
#include "prs_device.h"

namespace prs {

// ---------------------------------------------------------------------------
// exclusive scan of int32 (in place; data[n] receives the total)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int block_exclusive_scan(int v, int &total) {
  __shared__ int s[kScanThreads];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  total = s[kScanThreads - 1];
  const int incl = s[threadIdx.x];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(int *data, int n, int *sums) {
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int local = 0;
  for (int a = 0; a < kScanItems; ++a) {
    v[a] = (base + a < (size_t)n) ? data[base + a] : 0;
    local += v[a];
  }
  int total;
  int run = block_exclusive_scan(local, total);
  for (int a = 0; a < kScanItems; ++a) {
    if (base + a < (size_t)n) data[base + a] = run;
    run += v[a];
  }
  if (threadIdx.x == 0) {
    if (sums)
      sums[blockIdx.x] = total;
    else
      data[n] = total;
  }
}

__global__ void k_scan_add(int *data, int n, const int *sums, int nb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (size_t)n) data[i] += sums[i / kScanTile];
  if (i == 0) data[n] = sums[nb];
}

hipError_t launch_scan(hipStream_t s, int *data, int n, int *tmp) {
  if (n <= kScanTile) {
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, data, n, nullptr);
    return hipGetLastError();
  }
  const int nb = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kScanThreads), 0, s, data, n, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan(s, tmp, nb, tmp + nb + 1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((n + 255) / 256), dim3(256), 0, s, data, n, tmp, nb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// counting sort by cell
// ---------------------------------------------------------------------------
__global__ void k_zero_int(int *p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

__global__ void k_cell_keys(const double *__restrict__ x, int n, Cells C, Geom G, int *key,
                            int *count, uint32_t *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t fl = 0;
  const double px = sane_coord(x[3 * i + 0], G.Lx, false, fl);
  const double py = sane_coord(x[3 * i + 1], G.Ly, true, fl);
  const double pz = sane_coord(x[3 * i + 2], G.Lz, false, fl);
  if (fl) atomicOr(status, fl);
  const int k = cell_key(C, cell_coord(px, C.csx, C.ncx), cell_coord(py, C.csy, C.ncy),
                         cell_coord(pz, C.csz, C.ncz));
  key[i] = k;
  atomicAdd(&count[k], 1);
}

__global__ void k_scatter(const int *__restrict__ key, int n, const int *__restrict__ start,
                          int *fill, int *perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = key[i];
  perm[start[k] + atomicAdd(&fill[k], 1)] = i;
}

// The atomic scatter leaves the order inside a cell arbitrary; sort each
// cell's (few) entries by caller index so the layout is reproducible.
__global__ void k_cell_order(const int *__restrict__ start, int nkeys, int *perm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nkeys) return;
  const int b = start[k], e = start[k + 1];
  for (int a = b + 1; a < e; ++a) {
    const int v = perm[a];
    int c = a - 1;
    while (c >= b && perm[c] > v) {
      perm[c + 1] = perm[c];
      --c;
    }
    perm[c + 1] = v;
  }
}

hipError_t launch_sort(hipStream_t s, const Scratch &S, const Cells &C, const Geom &G,
                       const double *x, int n, int /*unused*/) {
  const int nk = C.nkeys;
  hipLaunchKernelGGL(k_zero_int, dim3((nk + 1 + 255) / 256), dim3(256), 0, s, S.start, nk + 1);
  hipLaunchKernelGGL(k_zero_int, dim3((nk + 255) / 256), dim3(256), 0, s, S.fill, nk);
  if (n > 0)
    hipLaunchKernelGGL(k_cell_keys, dim3((n + 255) / 256), dim3(256), 0, s, x, n, C, G, S.key,
                       S.start, S.status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan(s, S.start, nk, S.scan_tmp);
  if (e != hipSuccess) return e;
  if (n > 0)
    hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, s, S.key, n, S.start,
                       S.fill, S.perm);
  hipLaunchKernelGGL(k_cell_order, dim3((nk + 255) / 256), dim3(256), 0, s, S.start, nk, S.perm);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// caller arrays <-> sorted state
// ---------------------------------------------------------------------------
__global__ void k_gather_state(const int *__restrict__ perm, int n, Geom G,
                               const double *__restrict__ x, const double *__restrict__ u,
                               const double *__restrict__ om, const int32_t *__restrict__ hp,
                               const double *__restrict__ hd, const double *__restrict__ hu,
                               const int8_t *__restrict__ hc, double *xs, double *us, double *ws,
                               double *x0, double *pk, int *inv_perm, int *h_cnt, int *h_id,
                               double *h_dt, double *h_uin, uint32_t *status) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int i = perm[j];
  inv_perm[i] = j;
  uint32_t fl = 0;
  const double L[3] = {G.Lx, G.Ly, G.Lz};
  for (int a = 0; a < 3; ++a) {
    const double v = sane_coord(x[3 * i + a], L[a], a == 1, fl);
    xs[a * (size_t)n + j] = v;
    x0[a * (size_t)n + j] = v;
    const double uv = u[3 * i + a], wv = om[3 * i + a];
    if (!isfinite(uv) || !isfinite(wv)) fl |= kFlagNonFinite;
    us[a * (size_t)n + j] = uv;
    ws[a * (size_t)n + j] = wv;
    pk[pk_pos(j, n) + a] = v;
    pk[pk_vel(j, n) + a] = uv;
    pk[pk_vel(j, n) + 4 + a] = wv;
  }
  int c = hc[i];
  if (c < 0 || c > kSlots) {
    fl |= kFlagSlots;
    c = c < 0 ? 0 : kSlots;
  }
  h_cnt[j] = c;
  // only the slots in use (the substeps read no slot at or past the count)
  for (int sl = 0; sl < kSlots; ++sl) {
    if (sl >= c) break;
    h_id[sl * (size_t)n + j] = hp[(size_t)i * kSlots + sl];
    h_uin[sl * (size_t)n + j] = hu[(size_t)i * kSlots + sl];
    for (int a = 0; a < 3; ++a)
      h_dt[(sl * 3 + a) * (size_t)n + j] = hd[((size_t)i * kSlots + sl) * 3 + a];
  }
  if (fl) atomicOr(status, fl);
}

hipError_t launch_gather_state(hipStream_t s, const Scratch &S, const Geom &G, const double *x,
                               const double *u, const double *om, const prs_history *H, int n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_state, dim3((n + 255) / 256), dim3(256), 0, s, S.perm, n, G, x, u,
                     om, H->partner, H->delta_t, H->u_in, H->count, S.xs[0], S.us[0], S.ws[0],
                     S.x0, S.pk[0], S.inv_perm, S.h_cnt[0], S.h_id[0], S.h_dt[0], S.h_uin[0],
                     S.status);
  return hipGetLastError();
}

// Positions (and, when u and om are given, velocities) in sorted SoA order.
__global__ void k_gather_pos(const int *__restrict__ perm, int n, Geom G,
                             const double *__restrict__ x, const double *__restrict__ u,
                             const double *__restrict__ om, double *xs, double *us, double *ws,
                             int *inv_perm, uint32_t *status) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int i = perm[j];
  inv_perm[i] = j;
  uint32_t fl = 0;
  const double L[3] = {G.Lx, G.Ly, G.Lz};
  for (int a = 0; a < 3; ++a) xs[a * (size_t)n + j] = sane_coord(x[3 * i + a], L[a], a == 1, fl);
  if (u)
    for (int a = 0; a < 3; ++a) {
      const double uv = u[3 * i + a], wv = om[3 * i + a];
      if (!isfinite(uv) || !isfinite(wv)) fl |= kFlagNonFinite;
      us[a * (size_t)n + j] = uv;
      ws[a * (size_t)n + j] = wv;
    }
  if (fl && status) atomicOr(status, fl);
}

hipError_t launch_gather_pos(hipStream_t s, const Scratch &S, const Geom &G, const double *x,
                             int n, const double *u, const double *om) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_pos, dim3((n + 255) / 256), dim3(256), 0, s, S.perm, n, G, x, u, om,
                     S.xs[0], S.us[0], S.ws[0], S.inv_perm, S.status);
  return hipGetLastError();
}

constexpr uint32_t kErrorMask = kFlagSlots | kFlagCand | kFlagNonFinite | kFlagDomain | kFlagSkin;

// Write the advanced state back in caller order -- only when the step raised
// no error, so a failed step leaves the caller's state untouched.
__global__ void k_writeback(const int *__restrict__ perm, int n, const uint32_t *status,
                            const double *__restrict__ xs, const double *__restrict__ us,
                            const double *__restrict__ ws, const double *__restrict__ fh,
                            const double *__restrict__ th, const int *__restrict__ h_cnt,
                            const int *__restrict__ h_id, const double *__restrict__ h_dt,
                            const double *__restrict__ h_uin, double *x, double *u, double *om,
                            double *Fh, double *Th, int32_t *hp, double *hd, double *hu,
                            int8_t *hc, int vec) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int i = perm[j];
  for (int a = 0; a < 3; ++a) {
    Fh[3 * i + a] = fh[a * (size_t)n + j];
    Th[3 * i + a] = th[a * (size_t)n + j];
  }
  if (*status & kErrorMask) return;
  for (int a = 0; a < 3; ++a) {
    x[3 * i + a] = xs[a * (size_t)n + j];
    u[3 * i + a] = us[a * (size_t)n + j];
    om[3 * i + a] = ws[a * (size_t)n + j];
  }
  const int c = h_cnt[j];
  hc[i] = (int8_t)c;
  // the caller's rows, two slots per round with 8- and 16-byte stores when
  // the arrays allow (zeros past the count); the sorted slots read only
  // where in use
  static_assert(kSlots % 2 == 0, "slot pairs");
  for (int sl = 0; sl < kSlots; sl += 2) {
    int id[2] = {0, 0};
    double ui[2] = {0.0, 0.0}, dt[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = 0; e < 2; ++e)
      if (sl + e < c) {
        id[e] = h_id[(sl + e) * (size_t)n + j];
        ui[e] = h_uin[(sl + e) * (size_t)n + j];
        for (int a = 0; a < 3; ++a) dt[3 * e + a] = h_dt[((sl + e) * 3 + a) * (size_t)n + j];
      }
    const size_t r = (size_t)i * kSlots + sl;
    if (vec) {
      *reinterpret_cast<int2 *>(hp + r) = make_int2(id[0], id[1]);
      *reinterpret_cast<double2 *>(hu + r) = make_double2(ui[0], ui[1]);
      for (int q = 0; q < 3; ++q)
        reinterpret_cast<double2 *>(hd + 3 * r)[q] = make_double2(dt[2 * q], dt[2 * q + 1]);
    } else {
      for (int e = 0; e < 2; ++e) {
        hp[r + e] = id[e];
        hu[r + e] = ui[e];
      }
      for (int q = 0; q < 6; ++q) hd[3 * r + q] = dt[q];
    }
  }
}

hipError_t launch_writeback(hipStream_t s, const Scratch &S, double *x, double *u, double *om,
                            const prs_history *H, double *Fh, double *Th, int n, int buf) {
  if (n == 0) return hipSuccess;
  // slot pairs of a row start at multiples of 8 (partners) and 16 bytes
  // (u_in, delta_t) when the arrays themselves are 16-byte aligned
  const int vec = ((reinterpret_cast<uintptr_t>(H->partner) | reinterpret_cast<uintptr_t>(H->delta_t) |
                    reinterpret_cast<uintptr_t>(H->u_in)) & 15u) == 0;
  hipLaunchKernelGGL(k_writeback, dim3((n + 255) / 256), dim3(256), 0, s, S.perm, n, S.status,
                     S.xs[buf], S.us[buf], S.ws[buf], S.fh, S.th, S.h_cnt[buf], S.h_id[buf],
                     S.h_dt[buf], S.h_uin[buf], x, u, om, Fh, Th, H->partner, H->delta_t, H->u_in,
                     H->count, vec);
  return hipGetLastError();
}

__global__ void k_reset_status(uint32_t *status, unsigned long long *counters) {
  if (threadIdx.x == 0) *status = 0u;
  if (threadIdx.x < 4) counters[threadIdx.x] = 0ull;
}

hipError_t launch_reset_status(hipStream_t s, const Scratch &S) {
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, S.status, S.counters);
  return hipGetLastError();
}

}  // namespace prs
