// Soft-sphere contacts and Newton-Euler substeps.
//
// Collision search (once per fluid step, sec. 3.5's "collision search"):
// every sphere lists the spheres within 2R + skin from the 27 cells around
// it, sorted by caller index.  Each particle substep then tests only those
// candidates (exactly: d^2 < (2R)^2), which finds every contact as long as no
// sphere moves more than skin/2 during the step -- checked on every substep.
//
// Contact force (eqs. 9-10 and Appendix A): linear spring-dashpot normal
// force, tangential spring-dashpot on the rotated tangential displacement
// (A.9-A.11) capped by Coulomb friction.  Each sphere gathers its own
// contacts (no atomics), so the substep is deterministic.  The contact
// history follows sec. 3.4: the slots of the previous substep (M_temp) are
// matched against the contacts found now (M_p) by partner index; unmatched
// old slots are dropped.
//
// Compiled with -ffp-contract=off: the contact test d^2 < (2R)^2 must be
// evaluated exactly as written so the contact lists are reproducible bit for
// bit.
#include "prs_device.h"

namespace prs {

// Partner order inside a history: spheres by index, then bottom wall, then
// top wall.
__device__ inline unsigned order_key(int id) {
  return id >= 0 ? (unsigned)id : (id == PRS_WALL_BOTTOM ? 0x7ffffffeu : 0x7fffffffu);
}

// Sphere k's coordinate a is xs[a * cs + k * ss]: SoA [3][n] (cs = n, ss =
// 1) or the packed state [n][12] (cs = 1, ss = 12), whose three coordinates
// share a cache line.
template <typename F>
__device__ inline void for_each_near(const Cells &C, const Geom &G, const int *start,
                                     const double *xs, size_t cs, size_t ss, int j, double cut2,
                                     F fn) {
  const double px = xs[j * ss], py = xs[cs + j * ss], pz = xs[2 * cs + j * ss];
  const int cx = cell_coord(px, C.csx, C.ncx), cy = cell_coord(py, C.csy, C.ncy),
            cz = cell_coord(pz, C.csz, C.ncz);
  for (int dz = -1; dz <= 1; ++dz) {
    const int kz = wrap_once(cz + dz, C.ncz);
    for (int dy = -1; dy <= 1; ++dy) {
      const int ky = cy + dy;
      if (ky < 0 || ky >= C.ncy) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int kx = wrap_once(cx + dx, C.ncx);
        const int key = cell_key(C, kx, ky, kz);
        const int e = start[key + 1];
        for (int k = start[key]; k < e; ++k) {
          if (k == j) continue;
          const double *q = xs + k * ss;
          const double ddx = min_image(q[0] - px, G.Lx);
          const double ddy = q[cs] - py;
          const double ddz = min_image(q[2 * cs] - pz, G.Lz);
          const double d2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
          if (d2 < cut2) fn(k);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// collision search
// ---------------------------------------------------------------------------
// pk: the packed sphere state (positions [n][4] first).  Each thread keeps
// its sorted candidate list in its own LDS column (an array indexed at run
// time in registers would live in scratch memory).
constexpr int kCandThreads = 128;
__global__ __launch_bounds__(kCandThreads) void k_candidates(
    Cells C, Geom G, const int *__restrict__ start, const int *__restrict__ perm,
    const double *__restrict__ pk, int n, double cut2, int *__restrict__ ncand,
    int *__restrict__ cand, uint32_t *status) {
  __shared__ int s_key[kCandCap][kCandThreads];
  __shared__ int s_loc[kCandCap][kCandThreads];
  const int t = threadIdx.x;
  const int j = blockIdx.x * blockDim.x + t;
  if (j >= n) return;
  int cnt = 0;
  bool over = false;
  for_each_near(C, G, start, pk, 1, PRS_PK_SPLIT ? 4 : 12, j, cut2, [&](int k) {
    if (cnt < kCandCap) {
      const int id = perm[k];
      int c = cnt - 1;
      while (c >= 0 && s_key[c][t] > id) {
        s_key[c + 1][t] = s_key[c][t];
        s_loc[c + 1][t] = s_loc[c][t];
        --c;
      }
      s_key[c + 1][t] = id;
      s_loc[c + 1][t] = k;
      ++cnt;
    } else {
      over = true;
    }
  });
  if (over) atomicOr(status, kFlagCand);
  ncand[j] = cnt;
  for (int c = 0; c < cnt; ++c) cand[c * (size_t)n + j] = s_loc[c][t];
}

hipError_t launch_candidates(hipStream_t s, const Scratch &S, const Cells &C, const Geom &G,
                             int n, double cut) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_candidates, dim3((n + kCandThreads - 1) / kCandThreads), dim3(kCandThreads),
                     0, s, C, G, S.start, S.perm,
                     S.pk[0], n, cut * cut, S.ncand, S.cand, S.status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// one contact
// ---------------------------------------------------------------------------
struct ContactOut {
  double F[3], T[3], dnew[3], un;
};

// n: unit normal from p towards the partner; xi: overlap; ucp: contact-point
// relative velocity (A.5 / A.6); dprev: stored tangential displacement.
__device__ inline void contact_law(const Mech &M, double R, double kn, double dn, double kt,
                                   double dt, const double n[3], double xi, const double ucp[3],
                                   const double dprev[3], ContactOut &o) {
  const double un = (ucp[0] * n[0] + ucp[1] * n[1]) + ucp[2] * n[2];
  double ut[3];
  for (int a = 0; a < 3; ++a) ut[a] = ucp[a] - un * n[a];
  o.un = fabs(un);
  // rotate the stored displacement onto the tangent plane, keep its length
  const double dpn = (dprev[0] * n[0] + dprev[1] * n[1]) + dprev[2] * n[2];
  double dtil[3];
  for (int a = 0; a < 3; ++a) dtil[a] = dprev[a] - dpn * n[a];
  const double lt = sqrt((dtil[0] * dtil[0] + dtil[1] * dtil[1]) + dtil[2] * dtil[2]);
  const double lp = sqrt((dprev[0] * dprev[0] + dprev[1] * dprev[1]) + dprev[2] * dprev[2]);
  for (int a = 0; a < 3; ++a) {
    const double dh = lt > 0.0 ? (lp / lt) * dtil[a] : 0.0;
    o.dnew[a] = dh + M.dtp * ut[a];
  }
  const double fn = kn * xi + dn * un;
  double Ft[3];
  for (int a = 0; a < 3; ++a) Ft[a] = -kt * o.dnew[a] - dt * ut[a];
  const double FN = fn > 0.0 ? fn : 0.0;
  const double lft = sqrt((Ft[0] * Ft[0] + Ft[1] * Ft[1]) + Ft[2] * Ft[2]);
  if (lft > M.mu * FN) {
    const double sc = lft > 0.0 ? M.mu * FN / lft : 0.0;
    for (int a = 0; a < 3; ++a) {
      Ft[a] = sc * Ft[a];
      o.dnew[a] = -(Ft[a] + dt * ut[a]) / kt;
    }
  }
  o.T[0] = R * (n[1] * Ft[2] - n[2] * Ft[1]);
  o.T[1] = R * (n[2] * Ft[0] - n[0] * Ft[2]);
  o.T[2] = R * (n[0] * Ft[1] - n[1] * Ft[0]);
  for (int a = 0; a < 3; ++a) o.F[a] = -fn * n[a] + Ft[a];
}

// ---------------------------------------------------------------------------
// one particle substep
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_substep(
    Geom G, Mech M, int n, const int *__restrict__ perm, const int *__restrict__ ncand,
    const int *__restrict__ cand, const double *__restrict__ x0, const double *__restrict__ xs,
    const double *__restrict__ us, const double *__restrict__ ws, const double *__restrict__ pk,
    const double *__restrict__ fh, const double *__restrict__ th, const int *__restrict__ o_cnt,
    const int *__restrict__ o_id, const double *__restrict__ o_dt,
    const double *__restrict__ o_uin, double *__restrict__ xd, double *__restrict__ ud,
    double *__restrict__ wd, double *__restrict__ pd, int *__restrict__ n_cnt,
    int *__restrict__ n_id, double *__restrict__ n_dt, double *__restrict__ n_uin,
    uint32_t *status, unsigned long long *counters, int last) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  int my_pp = 0, my_wall = 0;
  if (j < n) {
    const double R = G.R;
    const size_t N = (size_t)n;
    double xp[3], up[3], wp[3];
    for (int a = 0; a < 3; ++a) {
      xp[a] = xs[a * N + j];
      up[a] = us[a * N + j];
      wp[a] = ws[a * N + j];
    }
    uint32_t fl = 0;
    {
      const double ex = min_image(xp[0] - x0[j], G.Lx), ey = xp[1] - x0[N + j],
                   ez = min_image(xp[2] - x0[2 * N + j], G.Lz);
      if ((ex * ex + ey * ey) + ez * ez > M.skin_half2) fl |= kFlagSkin;
    }
    const int cnt_old = o_cnt[j];
    int o = 0;
    int nc = 0;
    double Fc[3] = {0.0, 0.0, 0.0}, Tc[3] = {0.0, 0.0, 0.0};
    const int nk = ncand[j];
    const double four_r2 = (2.0 * R) * (2.0 * R);

    auto emit = [&](int id, const double nrm[3], double xi, const double ucp[3], bool wall) {
      const unsigned key = order_key(id);
      while (o < cnt_old && order_key(o_id[o * N + j]) < key) ++o;
      const bool exist = (o < cnt_old) && (o_id[o * N + j] == id);
      double dprev[3] = {0.0, 0.0, 0.0};
      if (exist)
        for (int a = 0; a < 3; ++a) dprev[a] = o_dt[(o * 3 + a) * N + j];
      ContactOut c;
      contact_law(M, R, wall ? M.kn_pw : M.kn_pp, wall ? M.dn_pw : M.dn_pp,
                  wall ? M.kt_pw : M.kt_pp, wall ? M.dt_pw : M.dt_pp, nrm, xi, ucp, dprev, c);
      if (nc < kSlots) {
        n_id[nc * N + j] = id;
        n_uin[nc * N + j] = exist ? o_uin[o * N + j] : c.un;
        for (int a = 0; a < 3; ++a) n_dt[(nc * 3 + a) * N + j] = c.dnew[a];
      }
      ++nc;
      for (int a = 0; a < 3; ++a) {
        Fc[a] += c.F[a];
        Tc[a] += c.T[a];
      }
    };

    // Which candidates touch: a first pass over their positions, branch-free
    // and unrolled so the gathers overlap, marks them in a bit mask; the
    // contacts are then evaluated in candidate order.
    static_assert(kCandCap <= 32, "candidate mask");
    uint32_t touching = 0;
#pragma unroll 4
    for (int a = 0; a < nk; ++a) {
      const double *q = pk + pk_pos((size_t)cand[a * N + j], N);
      const double dx = min_image(q[0] - xp[0], G.Lx);
      const double dy = q[1] - xp[1];
      const double dz = min_image(q[2] - xp[2], G.Lz);
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      touching |= (d2 < four_r2 ? 1u : 0u) << a;
    }
    for (; touching; touching &= touching - 1u) {
      const int a = __builtin_ctz(touching);
      const int k = cand[a * N + j];
      const double *q = pk + pk_pos((size_t)k, N);
      const double *qv = pk + pk_vel((size_t)k, N);   // u at +0, omega at +4
      const double dx = min_image(q[0] - xp[0], G.Lx);
      const double dy = q[1] - xp[1];
      const double dz = min_image(q[2] - xp[2], G.Lz);
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      const double dist = sqrt(d2);
      const double nrm[3] = {dx / dist, dy / dist, dz / dist};
      const double sw[3] = {wp[0] + qv[4], wp[1] + qv[5], wp[2] + qv[6]};
      const double wxn[3] = {sw[1] * nrm[2] - sw[2] * nrm[1], sw[2] * nrm[0] - sw[0] * nrm[2],
                             sw[0] * nrm[1] - sw[1] * nrm[0]};
      const double ucp[3] = {(up[0] - qv[0]) + R * wxn[0], (up[1] - qv[1]) + R * wxn[1],
                             (up[2] - qv[2]) + R * wxn[2]};
      emit(perm[k], nrm, 2.0 * R - dist, ucp, false);
      ++my_pp;
    }
    if (my_pp > kMaxPP) fl |= kFlagSlots;
    for (int wall = 0; wall < 2; ++wall) {
      const bool touch = wall == 0 ? (xp[1] < R) : (G.Ly - xp[1] < R);
      if (!touch) continue;
      const double nrm[3] = {0.0, wall == 0 ? -1.0 : 1.0, 0.0};
      const double xi = wall == 0 ? R - xp[1] : R - (G.Ly - xp[1]);
      const double wxn[3] = {wp[1] * nrm[2] - wp[2] * nrm[1], wp[2] * nrm[0] - wp[0] * nrm[2],
                             wp[0] * nrm[1] - wp[1] * nrm[0]};
      const double ucp[3] = {up[0] + R * wxn[0], up[1] + R * wxn[1], up[2] + R * wxn[2]};
      emit(wall == 0 ? PRS_WALL_BOTTOM : PRS_WALL_TOP, nrm, xi, ucp, true);
      ++my_wall;
    }
    n_cnt[j] = nc < kSlots ? nc : kSlots;

    // Newton-Euler, symplectic Euler with the hydrodynamic load held fixed
    for (int a = 0; a < 3; ++a) {
      const double Ftot = (fh[a * N + j] + M.fg[a]) + Fc[a];
      up[a] += M.dtp * Ftot / M.m;
      wp[a] += M.dtp * (th[a * N + j] + Tc[a]) / M.I;
      xp[a] += M.dtp * up[a];
    }
    if (xp[0] < 0.0) xp[0] += G.Lx;
    if (xp[0] >= G.Lx) xp[0] -= G.Lx;
    if (xp[2] < 0.0) xp[2] += G.Lz;
    if (xp[2] >= G.Lz) xp[2] -= G.Lz;
    for (int a = 0; a < 3; ++a) {
      if (!isfinite(up[a]) || !isfinite(wp[a]) || !isfinite(xp[a])) fl |= kFlagNonFinite;
      xd[a * N + j] = xp[a];
      ud[a * N + j] = up[a];
      wd[a * N + j] = wp[a];
      pd[pk_pos(j, N) + a] = xp[a];
      pd[pk_vel(j, N) + a] = up[a];
      pd[pk_vel(j, N) + 4 + a] = wp[a];
    }
    if (!(xp[1] >= 0.0 && xp[1] <= G.Ly)) fl |= kFlagDomain;
    if (fl) atomicOr(status, fl);
  }
  // contact counters: one atomic per wave (a wave's counts fit in 32 bits)
  const int c1 = wave_sum_last(my_pp), c2 = wave_sum_last(my_wall);
  if ((threadIdx.x & 63) == 63) {
    const unsigned long long c0 = (unsigned long long)c1 + (unsigned long long)c2;
    if (c0) atomicAdd(&counters[0], c0);
    if (last) {
      if (c1) atomicAdd(&counters[1], (unsigned long long)c1);
      if (c2) atomicAdd(&counters[2], (unsigned long long)c2);
    }
  }
}

hipError_t launch_substep(hipStream_t s, const Scratch &S, const Geom &G, const Mech &M, int n,
                          int src, int last) {
  if (n == 0) return hipSuccess;
  const int dst = 1 - src;
  hipLaunchKernelGGL(k_substep, dim3((n + 255) / 256), dim3(256), 0, s, G, M, n, S.perm, S.ncand,
                     S.cand, S.x0, S.xs[src], S.us[src], S.ws[src], S.pk[src], S.fh, S.th,
                     S.h_cnt[src], S.h_id[src], S.h_dt[src], S.h_uin[src], S.xs[dst], S.us[dst],
                     S.ws[dst], S.pk[dst], S.h_cnt[dst], S.h_id[dst], S.h_dt[dst], S.h_uin[dst],
                     S.status, S.counters, last);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// canonical contact list
// ---------------------------------------------------------------------------
// phase 0: per caller index i, count contacts (i, j > i) and walls, flag a
// sphere with more than twelve sphere contacts.  phase 1: write the rows of
// sphere i at its scanned offset, partners ascending, walls last.
__global__ void k_contact_list(Cells C, Geom G, const int *__restrict__ start,
                               const int *__restrict__ perm, const int *__restrict__ inv_perm,
                               const double *__restrict__ xs, int n, int *__restrict__ ccount,
                               const int *__restrict__ coffset, int32_t *pairs, long long cap,
                               uint32_t *status, int phase) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = inv_perm[i];
  const double R = G.R;
  int upper[kMaxPP];
  int nu = 0, all = 0;
  for_each_near(C, G, start, xs, (size_t)n, 1, j, (2.0 * R) * (2.0 * R), [&](int k) {
    const int id = perm[k];
    ++all;
    if (id > i && nu < kMaxPP) upper[nu++] = id;
  });
  const double y = xs[n + j];
  const bool wb = y < R, wt = (G.Ly - y) < R;
  if (phase == 0) {
    if (all > kMaxPP) atomicOr(status, kFlagSlots);
    ccount[i] = nu + (wb ? 1 : 0) + (wt ? 1 : 0);
    return;
  }
  for (int a = 1; a < nu; ++a) {
    const int v = upper[a];
    int c = a - 1;
    while (c >= 0 && upper[c] > v) {
      upper[c + 1] = upper[c];
      --c;
    }
    upper[c + 1] = v;
  }
  long long row = coffset[i];
  auto put = [&](int a, int b) {
    if (row < cap) {
      pairs[2 * row] = a;
      pairs[2 * row + 1] = b;
    }
    ++row;
  };
  for (int a = 0; a < nu; ++a) put(i, upper[a]);
  if (wb) put(i, PRS_WALL_BOTTOM);
  if (wt) put(i, PRS_WALL_TOP);
}

hipError_t launch_contact_list(hipStream_t s, const Scratch &S, const Cells &C, const Geom &G,
                               int n, int32_t *pairs, long long cap, int phase) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_contact_list, dim3((n + 127) / 128), dim3(128), 0, s, C, G, S.start,
                     S.perm, S.inv_perm, S.xs[0], n, S.ccount, S.coffset, pairs, cap, S.status,
                     phase);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// bed and flying spheres (sec. 4.3.1, step (1))
// ---------------------------------------------------------------------------
// A sphere with its centre below one diameter is bed, and so is every sphere
// touching a bed sphere, directly or through a chain of contacts.  The
// touching partners (A.3) of every sphere are listed once (sorted indices,
// [slot][n] in cand, counts in ncand); bed[] starts at the bottom layer and
// passes over the spheres mark each one touching a marked partner, in place
// (a mark made in a pass is seen by later reads of the same pass), until a
// pass marks nothing.  Marks only ever go from 0 to 1, so the result is the
// unique smallest closed set, whatever the order of the updates.
__global__ void k_bed_seed(Cells C, Geom G, const int *__restrict__ start,
                           const double *__restrict__ xs, int n, int *__restrict__ ncand,
                           int *__restrict__ cand, int *__restrict__ bed, uint32_t *status) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double R = G.R;
  int cnt = 0, all = 0;
  for_each_near(C, G, start, xs, (size_t)n, 1, j, (2.0 * R) * (2.0 * R), [&](int k) {
    if (cnt < kMaxPP) cand[cnt++ * (size_t)n + j] = k;
    ++all;
  });
  if (all > kMaxPP) atomicOr(status, kFlagSlots);
  ncand[j] = cnt;
  bed[j] = xs[n + j] < 2.0 * R ? 1 : 0;
}

__global__ void k_bed_pass(int n, const int *__restrict__ ncand, const int *__restrict__ cand,
                           int *bed, unsigned long long *changed) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  int mark = 0;
  if (j < n && !bed[j]) {
    const int cnt = ncand[j];
    for (int c = 0; c < cnt && !mark; ++c)
      if (__atomic_load_n(&bed[cand[c * (size_t)n + j]], __ATOMIC_RELAXED)) mark = 1;
    if (mark) __atomic_store_n(&bed[j], 1, __ATOMIC_RELAXED);
  }
  const int w = wave_sum_last(mark);
  if ((threadIdx.x & 63) == 63 && w) atomicAdd(changed, (unsigned long long)w);
}

// flags[perm[j]] = bed[j]; counters[3] += bed spheres.
__global__ void k_bed_out(int n, const int *__restrict__ perm, const int *__restrict__ bed,
                          int8_t *__restrict__ flags, unsigned long long *count) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  if (j < n) {
    b = bed[j];
    flags[perm[j]] = (int8_t)b;
  }
  const int w = wave_sum_last(b);
  if ((threadIdx.x & 63) == 63 && w) atomicAdd(count, (unsigned long long)w);
}

hipError_t launch_bed_seed(hipStream_t s, const Scratch &S, const Cells &C, const Geom &G, int n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bed_seed, dim3((n + 127) / 128), dim3(128), 0, s, C, G, S.start, S.xs[0],
                     n, S.ncand, S.cand, S.bed, S.status);
  return hipGetLastError();
}

hipError_t launch_bed_pass(hipStream_t s, const Scratch &S, int n, unsigned long long *changed) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bed_pass, dim3((n + 255) / 256), dim3(256), 0, s, n, S.ncand, S.cand,
                     S.bed, changed);
  return hipGetLastError();
}

hipError_t launch_bed_out(hipStream_t s, const Scratch &S, int n, int8_t *flags,
                          unsigned long long *count) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bed_out, dim3((n + 255) / 256), dim3(256), 0, s, n, S.perm, S.bed, flags,
                     count);
  return hipGetLastError();
}

}  // namespace prs
