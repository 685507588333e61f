// extern "C" boundary of the library: argument validation, context and
// scratch management, and the host-side sequencing of the kernels on the
// caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "prs_internal.h"

using namespace prs;

// Phases of the step timed by prs_timing_* (one slot each).
enum Phase { kZeroF = 0, kSort, kInterp, kSpread, kSearch, kSubstep, kWriteback, kLearned, kRecord };
constexpr int kPhases = 9;

struct prs_ctx {
  prs_params p{};
  Geom G{};
  Cells C_step{}, C_touch{};
  Mech M{};
  Scratch S{};
  int device = 0;
  std::vector<void *> allocs;
  std::string err;
  double *host_pinned = nullptr;   // staging for statistics
  // phase timing (prs_timing_*)
  bool timing = false;
  std::vector<hipEvent_t> events;
  size_t events_used = 0;
  struct Mark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  hipEvent_t open_ev = nullptr;
  double ms[kPhases] = {};
  int64_t launches[kPhases] = {};
  const prs_mlp *mlp = nullptr;   // learned warm start (prs_set_learned)
  int64_t steps = 0;
};

namespace {

int fail(prs_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail((ctx), PRS_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

template <typename T>
int alloc(prs_ctx *c, T **p, size_t count) {
  void *q = nullptr;
  const size_t bytes = (count ? count : 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess)
    return fail(c, PRS_EHIP, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  c->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return PRS_OK;
}

// Cells of edge >= cut (with a relative margin so that rounding never puts
// two spheres closer than cut into non-adjacent cells).
Cells make_cells(const Geom &G, double cut) {
  Cells C{};
  const double c = cut * (1.0 + 1e-9);
  C.ncx = (int)std::floor(G.Lx / c);
  C.ncy = (int)std::floor(G.Ly / c);
  C.ncz = (int)std::floor(G.Lz / c);
  if (C.ncy < 1) C.ncy = 1;
  C.csx = G.Lx / (C.ncx > 0 ? C.ncx : 1);
  C.csy = G.Ly / C.ncy;
  C.csz = G.Lz / (C.ncz > 0 ? C.ncz : 1);
  C.ntx = (C.ncx + 3) / 4;
  C.nty = (C.ncy + 3) / 4;
  C.ntz = (C.ncz + 3) / 4;
  C.nkeys = C.ntx * C.nty * C.ntz * 64;
  return C;
}

double damping(double k, double e, double m_eff) {
  const double le = std::log(e);
  return -2.0 * le * std::sqrt(m_eff * k) / std::sqrt(M_PI * M_PI + le * le);
}

size_t grid_count(const prs_ctx *c, int comp) {
  return (size_t)c->p.nz * (size_t)(c->p.ny + (comp == 1 ? 1 : 0)) * (size_t)c->p.nx;
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

int status_code(uint32_t st) {
  if (st & kFlagNonFinite) return PRS_ENONFINITE;
  if (st & kFlagDomain) return PRS_EDOMAIN;
  if (st & (kFlagSlots | kFlagCand)) return PRS_ECAPACITY;
  if (st & kFlagSkin) return PRS_ESKIN;
  return PRS_OK;
}

const char *status_text(uint32_t st) {
  if (st & kFlagNonFinite) return "non-finite value in the sphere state";
  if (st & kFlagDomain) return "a sphere centre lies outside the box";
  if (st & kFlagSlots) return "a sphere touches more than twelve spheres";
  if (st & kFlagCand) return "more than 32 collision-search candidates on one sphere";
  if (st & kFlagSkin) return "a sphere moved farther than skin/2 within the step";
  return "ok";
}

int check_n(prs_ctx *c, int32_t n) {
  if (n < 0 || n > c->p.max_particles)
    return fail(c, PRS_EINVAL, "n = %d outside 0..max_particles (%d)", n, c->p.max_particles);
  return PRS_OK;
}


hipError_t next_event(prs_ctx *c, hipEvent_t *ev) {
  if (c->events_used == c->events.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    c->events.push_back(e);
  }
  *ev = c->events[c->events_used++];
  return hipSuccess;
}

hipError_t phase_begin(prs_ctx *c, hipStream_t s) {
  if (!c->timing) return hipSuccess;
  hipError_t r = next_event(c, &c->open_ev);
  return r != hipSuccess ? r : hipEventRecord(c->open_ev, s);
}

hipError_t phase_end(prs_ctx *c, hipStream_t s, int phase) {
  if (!c->timing) return hipSuccess;
  hipEvent_t e;
  hipError_t r = next_event(c, &e);
  if (r != hipSuccess) return r;
  r = hipEventRecord(e, s);
  c->marks.push_back({phase, c->open_ev, e});
  return r;
}

// After the stream has been synchronised: fold the recorded intervals in.
hipError_t phase_collect(prs_ctx *c) {
  if (!c->timing) return hipSuccess;
  for (const auto &m : c->marks) {
    float ms = 0.f;
    hipError_t r = hipEventElapsedTime(&ms, m.a, m.b);
    if (r != hipSuccess) return r;
    c->ms[m.phase] += ms;
    c->launches[m.phase] += 1;
  }
  c->marks.clear();
  c->events_used = 0;
  c->steps += 1;
  return hipSuccess;
}

template <typename T>
int clear_field(prs_ctx *c, hipStream_t s, void *const f[3]) {
  for (int k = 0; k < 3; ++k) HIP_TRY(c, launch_fill_zero<T>(s, (T *)f[k], grid_count(c, k)));
  return PRS_OK;
}

// Multi-direct forcing on the sorted spheres (Jacobi): every iteration
// interpolates u** = u-hat + alpha dt f at all markers, then spreads the
// corrections into f.  In tolerance mode the relative slip of each pass is
// read back and the loop stops before spreading once it is below tol.
//   F0      : caller-ordered initial marker force, spread first (or NULL);
//   learned : start from the attached network's prediction (f is zero);
//   target  : when set, alpha dt times every correction is accumulated into
//             it (training samples).
template <typename T>
int run_forcing(prs_ctx *c, hipStream_t s, double adt, const void *const uhat[3],
                void *const f[3], int n, const void *F0, bool need_den, bool learned, int n_fixed,
                float *target, int &iters, int &n_slip, int &rejected, bool clear_f = false) {
  Scratch &S = c->S;
  const prs_params &q = c->p;
  const T *uh[3] = {(const T *)uhat[0], (const T *)uhat[1], (const T *)uhat[2]};
  T *ff[3] = {(T *)f[0], (T *)f[1], (T *)f[2]};
  const T *fc[3] = {ff[0], ff[1], ff[2]};
  double *hist_host = c->host_pinned;
  bool den_ready = false;
  // the first spreading pass of the step records each tile's culled markers,
  // the later ones replay them (the spheres do not move during the forcing)
  int spreads = 0;
  // clear_f: f is to be cleared; nothing reads it before the first spreading
  // pass, which overwrites every node instead of adding
  bool pending_clear = clear_f;
  auto tile_cache = [&]() {
    TileCache tc{2, S.tc_cap, S.tc_items, S.tc_count, S.tc_ncand};
    tc.overwrite = pending_clear ? 1 : 0;
    pending_clear = false;
    return tc;
  };
  // the tiles' records, before the step's first spreading pass (a phase of
  // its own)
  auto record_tiles = [&]() -> hipError_t {
    if (spreads++ > 0) return hipSuccess;
    hipError_t e = phase_begin(c, s);
    if (e == hipSuccess) e = launch_tile_record<T>(s, c->G, c->C_step, S, n);
    if (e == hipSuccess) e = phase_end(c, s, kRecord);
    return e;
  };
  if (learned) {
    // features, zero-forcing slip and the prediction F0 -> dF in one pass
    LearnArgs la{};
    mlp_buffers(c->mlp, &la);
    HIP_TRY(c, phase_begin(c, s));
    HIP_TRY(c, launch_interp_learned<T>(s, c->G, S, uh, n, adt, la));
    HIP_TRY(c, phase_end(c, s, kLearned));
    HIP_TRY(c, launch_slip_reduce(s, S, n, 0, 1));
    HIP_TRY(c, launch_ib_begin(s, S, n));
    HIP_TRY(c, launch_ft_commit(s, S, n));
    HIP_TRY(c, record_tiles());
    HIP_TRY(c, phase_begin(c, s));
    HIP_TRY(c, launch_spread_tiles<T>(s, c->G, c->C_step, S, ff, n, nullptr, tile_cache()));
    HIP_TRY(c, phase_end(c, s, kSpread));
    den_ready = true;
  } else {
    if (need_den) {
      HIP_TRY(c, phase_begin(c, s));
      HIP_TRY(c, launch_interp_mdf<T>(s, c->G, S, uh, fc, n, adt, 1));
      HIP_TRY(c, phase_end(c, s, kInterp));
      HIP_TRY(c, launch_slip_reduce(s, S, n, 0, 1));
      den_ready = true;
    }
    if (F0) {
      HIP_TRY(c, launch_marker_sums<T>(s, c->G, S, n, (const T *)F0));
      HIP_TRY(c, record_tiles());
      HIP_TRY(c, phase_begin(c, s));
      HIP_TRY(c, launch_spread_tiles<T>(s, c->G, c->C_step, S, ff, n, (const T *)F0,
                                        tile_cache()));
      HIP_TRY(c, phase_end(c, s, kSpread));
    } else {
      HIP_TRY(c, launch_ib_begin(s, S, n));
    }
  }
  const bool tol_mode = q.tol_mode && n_fixed < 0;
  const int n_iter = n_fixed >= 0 ? n_fixed : q.n_iter;
  const int limit = q.max_iter;
  for (int it = 0;; ++it) {
    if (!tol_mode && it >= n_iter) break;
    HIP_TRY(c, phase_begin(c, s));
    // the first pass after a cleared field with no initial force reads u-hat only
    const T *fnone[3] = {nullptr, nullptr, nullptr};
    HIP_TRY(c, launch_interp_mdf<T>(s, c->G, S, uh, it == 0 && !den_ready ? fnone : fc, n, adt,
                                    0));
    HIP_TRY(c, phase_end(c, s, kInterp));
    HIP_TRY(c, launch_slip_reduce(s, S, n, it, 0));
    if (it == 0 && !den_ready) {
      // f = 0 and no initial force: this pass saw u** = u-hat
      HIP_TRY(c, launch_copy_scalar(s, S.slip_hist, S.slip_hist + PRS_MAX_SLIP));
      den_ready = true;
    }
    n_slip = it + 1;
    if (tol_mode || learned) {
      HIP_TRY(c, hipMemcpyAsync(hist_host, S.slip_hist, sizeof(double) * (PRS_MAX_SLIP + 1),
                                hipMemcpyDeviceToHost, s));
      HIP_TRY(c, hipStreamSynchronize(s));
      const double den = std::sqrt(hist_host[PRS_MAX_SLIP]);
      const double rel = den > 0 ? std::sqrt(hist_host[it]) / den : 0.0;
      if (learned && ((it == 0 && !(rel < 1.0)) || (it > 0 && hist_host[it] > hist_host[it - 1]))) {
        // the prediction made things worse: restart from zero forcing
        rejected = 1;
        learned = false;
        HIP_TRY(c, phase_begin(c, s));
        if (int rc = clear_field<T>(c, s, f)) return rc;
        HIP_TRY(c, phase_end(c, s, kZeroF));
        HIP_TRY(c, launch_ib_begin(s, S, n));
        iters = 0;
        it = -1;
        continue;
      }
      if (tol_mode && (rel < q.tol || it >= limit)) break;
    }
    if (target) HIP_TRY(c, launch_accum_target<T>(s, c->G, S, n, adt, target));
    HIP_TRY(c, launch_ft_commit(s, S, n));
    HIP_TRY(c, record_tiles());
    HIP_TRY(c, phase_begin(c, s));
    HIP_TRY(c, launch_spread_tiles<T>(s, c->G, c->C_step, S, ff, n, nullptr, tile_cache()));
    HIP_TRY(c, phase_end(c, s, kSpread));
    iters = it + 1;
  }
  if (pending_clear) {
    // no spreading pass ran (zero iterations, or the tolerance met at once)
    HIP_TRY(c, phase_begin(c, s));
    if (int rc = clear_field<T>(c, s, f)) return rc;
    HIP_TRY(c, phase_end(c, s, kZeroF));
  }
  return PRS_OK;
}

void fill_stats(prs_stats *stats, const double *hist_host, int iters, int n_slip) {
  memset(stats, 0, sizeof *stats);
  stats->iterations = iters;
  stats->n_slip = n_slip;
  const double den = std::sqrt(hist_host[PRS_MAX_SLIP]);
  for (int k = 0; k < n_slip; ++k)
    stats->rel_slip[k] = den > 0 ? std::sqrt(hist_host[k]) / den : 0.0;
}

}  // namespace

extern "C" {

int prs_create(const prs_params *p, prs_ctx **out) {
  if (!p || !out) return PRS_EINVAL;
  *out = nullptr;
  const prs_params &q = *p;
  auto bad = [&](const char *what) {
    (void)what;
    return PRS_EINVAL;
  };
  if (q.nx < 1 || q.ny < 1 || q.nz < 1 || !(q.h > 0) || !(q.radius > 0)) return bad("grid");
  if (q.n_markers < 1 || q.n_markers > kMaxMarkers) return bad("n_markers");
  if (!(q.rho_p > 0) || !(q.rho_f >= 0) || !(q.dt_f > 0) || !(q.alpha > 0)) return bad("phys");
  if (q.n_iter < 0 || q.max_iter < 0 || q.max_iter > PRS_MAX_SLIP - 1 ||
      q.n_iter > PRS_MAX_SLIP - 1)
    return bad("iter");
  if (q.tol_mode != 0 && q.tol_mode != 1) return bad("tol_mode");
  if (q.n_sub < 0 || !(q.e_n > 0 && q.e_n <= 1) || !(q.mu >= 0) || !(q.skin >= 0))
    return bad("contact");
  if (q.contact_model == PRS_CONTACT_FIXED) {
    if (!(q.k_n > 0) || !(q.kt_ratio > 0) || !(q.dt_ratio >= 0)) return bad("contact");
  } else if (q.contact_model == PRS_CONTACT_COLLISION_TIME) {
    if (!(q.t_c > 0) || !(q.e_t > 0 && q.e_t <= 1)) return bad("contact");
  } else {
    return bad("contact_model");
  }
  if (q.precision != PRS_F32 && q.precision != PRS_F64) return bad("precision");
  if (q.max_particles < 0) return bad("max_particles");
  for (double gv : q.gravity)
    if (!std::isfinite(gv)) return bad("gravity");

  prs_ctx *c = new prs_ctx();
  c->p = q;
  Geom &G = c->G;
  G.nx = q.nx;
  G.ny = q.ny;
  G.nz = q.nz;
  G.h = q.h;
  G.inv_h = 1.0 / q.h;
  G.Lx = q.nx * q.h;
  G.Ly = q.ny * q.h;
  G.Lz = q.nz * q.h;
  G.R = q.radius;
  G.nl = q.n_markers;
  G.dV = M_PI * q.h * (12.0 * q.radius * q.radius + q.h * q.h) / (3.0 * q.n_markers);
  {
    // A node's stencil weights are products of three one-dimensional
    // kernel values (each <= 2/3) and it is reached by markers within
    // rho = 1.5 sqrt(3) h.  Those markers of one sphere lie on the part of
    // the sphere inside a ball of radius rho, a cap of area at most
    // 2 pi R (R - sqrt(R^2 - rho^2)) (the whole sphere when rho >= R), against
    // 4 pi R^2 / n_markers per marker; the Fibonacci points are within a
    // factor 1.5 of uniform, and four extra markers cover the cap's rim.
    const double R = q.radius;
    const double rho = 1.5 * std::sqrt(3.0) * q.h + 1e-9 * q.h;
    const double area =
        rho < R ? 2.0 * M_PI * R * (R - std::sqrt(R * R - rho * rho)) : 4.0 * M_PI * R * R;
    const double per_marker = 4.0 * M_PI * R * R / q.n_markers;
    const double markers = std::min((double)q.n_markers, std::ceil(1.5 * area / per_marker) + 4.0);
    G.wsum_bound = markers * (8.0 / 27.0);
  }
  // the stencil of a marker must not wrap twice around the periodic box
  if (!(G.Lx > q.radius + 3 * q.h) || !(G.Lz > q.radius + 3 * q.h)) {
    delete c;
    return PRS_EINVAL;
  }
  c->C_step = make_cells(G, 2.0 * q.radius + q.skin);
  c->C_touch = make_cells(G, 2.0 * q.radius);
  if (c->C_step.ncx < 3 || c->C_step.ncz < 3) {
    delete c;
    return PRS_EINVAL;
  }
  // the interpolation brick of one sphere must fit in the periodic box, and
  // a spreading tile must see each sphere that reaches it through one
  // periodic image only
  const int nb = brick_edge(q.radius, q.h);
  {
    const int esz = q.precision == PRS_F64 ? 8 : 4;
    const int reach = 2 * (int)std::ceil(q.radius / q.h - 1e-9) + 6;
    if (q.nx <= nb || q.nz <= nb || q.nx < spread_tile_dim(esz, 0) + reach ||
        q.nz < spread_tile_dim(esz, 2) + reach) {
      delete c;
      return PRS_EINVAL;
    }
  }
  // every argument check above runs before the first HIP call
  (void)hipGetDevice(&c->device);
  {
    hipDeviceProp_t prop;
    const size_t need = interp_lds_bytes(nb, q.precision == PRS_F64 ? 8 : 4) + 4096;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && need > prop.sharedMemPerBlock) {
      delete c;
      return PRS_EINVAL;
    }
  }
  Mech &M = c->M;
  const double R = q.radius;
  M.m = q.rho_p * (4.0 / 3.0) * M_PI * R * R * R;
  M.I = 0.4 * M.m * R * R;
  const double V = (4.0 / 3.0) * M_PI * R * R * R;
  for (int a = 0; a < 3; ++a) M.fg[a] = (q.rho_p - q.rho_f) * V * q.gravity[a];
  if (q.contact_model == PRS_CONTACT_COLLISION_TIME) {
    // a damped oscillator of mass m lasting t_c with restitution e
    auto calib = [&](double m, double e, double &k, double &d) {
      const double le = std::log(e);
      d = -2.0 * m * le / q.t_c;
      k = m * (M_PI * M_PI + le * le) / (q.t_c * q.t_c);
    };
    calib(0.5 * M.m, q.e_n, M.kn_pp, M.dn_pp);
    calib(M.m, q.e_n, M.kn_pw, M.dn_pw);
    calib((2.0 / 7.0) * 0.5 * M.m, q.e_t, M.kt_pp, M.dt_pp);
    calib((2.0 / 7.0) * M.m, q.e_t, M.kt_pw, M.dt_pw);
  } else {
    M.kn_pp = M.kn_pw = q.k_n;
    M.dn_pp = damping(q.k_n, q.e_n, 0.5 * M.m);
    M.dn_pw = damping(q.k_n, q.e_n, M.m);
    M.kt_pp = M.kt_pw = q.kt_ratio * q.k_n;
    M.dt_pp = q.dt_ratio * M.dn_pp;
    M.dt_pw = q.dt_ratio * M.dn_pw;
  }
  M.mu = q.mu;
  M.dtp = q.n_sub > 0 ? q.dt_f / q.n_sub : 0.0;
  M.skin_half2 = 0.25 * q.skin * q.skin;

  Scratch &S = c->S;
  const size_t n = (size_t)(q.max_particles > 0 ? q.max_particles : 1);
  const int nkeys = c->C_step.nkeys > c->C_touch.nkeys ? c->C_step.nkeys : c->C_touch.nkeys;
  const size_t scan_max = (size_t)(nkeys > (int)n ? nkeys : (int)n) + 1;
  S.cap_n = (int)n;
  S.scan_tmp_elems = scan_max / 1024 + 64;
  const size_t esz = q.precision == PRS_F64 ? 8 : 4;
  int rc = PRS_OK;
  rc |= alloc(c, &S.key, n);
  rc |= alloc(c, &S.start, (size_t)nkeys + 1);
  rc |= alloc(c, &S.fill, (size_t)nkeys);
  rc |= alloc(c, &S.perm, n);
  rc |= alloc(c, &S.inv_perm, n);
  rc |= alloc(c, &S.scan_tmp, S.scan_tmp_elems);
  for (int b = 0; b < 2; ++b) {
    rc |= alloc(c, &S.xs[b], 3 * n);
    rc |= alloc(c, &S.us[b], 3 * n);
    rc |= alloc(c, &S.ws[b], 3 * n);
    rc |= alloc(c, &S.pk[b], 12 * n);
    rc |= alloc(c, &S.h_cnt[b], n);
    rc |= alloc(c, &S.h_id[b], kSlots * n);
    rc |= alloc(c, &S.h_dt[b], 3 * kSlots * n);
    rc |= alloc(c, &S.h_uin[b], kSlots * n);
  }
  rc |= alloc(c, &S.x0, 3 * n);
  rc |= alloc(c, &S.fh, 3 * n);
  rc |= alloc(c, &S.th, 3 * n);
  rc |= alloc(c, &S.ft_acc, 12 * n);
  rc |= alloc(c, &S.ft_part, 12 * n);
  rc |= alloc(c, &S.slip_part, 2 * n);
  rc |= alloc(c, &S.vmax, n);
  rc |= alloc(c, &S.slip_hist, PRS_MAX_SLIP + 1 + 256);
  rc |= alloc(c, &S.ncand, n);
  rc |= alloc(c, &S.cand, (size_t)kCandCap * n);
  rc |= alloc(c, &S.bed, n);
  rc |= alloc(c, &S.ccount, n + 1);
  S.coffset = S.ccount;
  char *dF = nullptr;
  rc |= alloc(c, &dF, 3 * n * (size_t)q.n_markers * esz);
  S.dF = dF;
  char *u0 = nullptr;
  rc |= alloc(c, &u0, 3 * n * (size_t)q.n_markers * esz);
  S.u0 = u0;
  {
    // record of the spreading's culled markers per grid tile, reused by the
    // later passes of a step: 2048 markers and 256 candidate spheres per tile
    // (a tile with more is culled again instead)
    const int ntiles = esz == 8 ? spread_tile_count<double>(c->G) : spread_tile_count<float>(c->G);
    S.tc_cap = kTileRecord;
    rc |= alloc(c, &S.tc_items, (size_t)ntiles * S.tc_cap);
    rc |= alloc(c, &S.tc_count, (size_t)ntiles);
    rc |= alloc(c, &S.tc_ncand, (size_t)ntiles);
  }
  rc |= alloc(c, &S.status, 4);
  rc |= alloc(c, &S.counters, 4);
  rc |= alloc(c, &S.templ, 3 * (size_t)q.n_markers);
  rc |= alloc(c, &S.lane_order, (size_t)q.n_markers);
  rc |= alloc(c, &S.tm32, 8 * (size_t)q.n_markers);
  rc |= alloc(c, &S.tm64, 4 * (size_t)q.n_markers);
  rc |= alloc(c, &S.tm32_lane, 8 * (size_t)q.n_markers);
  rc |= alloc(c, &S.tm64_lane, 4 * (size_t)q.n_markers);
  if (rc != PRS_OK) {
    prs_destroy(c);
    return PRS_EHIP;
  }
  if (hipHostMalloc((void **)&c->host_pinned, 256 * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    prs_destroy(c);
    return PRS_EHIP;
  }
  if (launch_template(nullptr, S.templ, S.tm32, S.tm64, S.tm32_lane, S.tm64_lane, S.lane_order,
                      q.n_markers,
                      q.radius / q.h) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    prs_destroy(c);
    return PRS_EHIP;
  }
  *out = c;
  return PRS_OK;
}

void prs_destroy(prs_ctx *c) {
  if (!c) return;
  for (void *q : c->allocs) (void)hipFree(q);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->host_pinned) (void)hipHostFree(c->host_pinned);
  delete c;
}

const char *prs_last_error(const prs_ctx *c) {
  if (!c) return "null context";
  return c->err.empty() ? "ok" : c->err.c_str();
}

int prs_template(prs_ctx *c, double *t_host, double *dV) {
  if (!c) return PRS_EINVAL;
  if (!t_host || !dV) return fail(c, PRS_EINVAL, "template: null output");
  HIP_TRY(c, hipMemcpy(t_host, c->S.templ, sizeof(double) * 3 * c->p.n_markers,
                       hipMemcpyDeviceToHost));
  *dV = c->G.dV;
  return PRS_OK;
}

int prs_interpolate(prs_ctx *c, void *stream, const void *gu, const void *gv, const void *gw,
                    const double *x, const double *up, const double *om, int32_t n, void *U,
                    void *Ud) {
  if (!c) return PRS_EINVAL;
  if (int rc = check_n(c, n)) return rc;
  if (n == 0) return PRS_OK;
  if (!gu || !gv || !gw || !x || !U) return fail(c, PRS_EINVAL, "interpolate: null array");
  if (Ud && (!up || !om))
    return fail(c, PRS_EINVAL, "interpolate: Ud needs up and om");
  hipStream_t s = as_stream(stream);
  if (c->p.precision == PRS_F64)
    HIP_TRY(c, launch_interp_plain<double>(s, c->G, c->S, (const double *)gu,
                                           (const double *)gv, (const double *)gw, x, up, om, n,
                                           (double *)U, (double *)Ud));
  else
    HIP_TRY(c, launch_interp_plain<float>(s, c->G, c->S, (const float *)gu,
                                          (const float *)gv, (const float *)gw, x, up, om, n,
                                          (float *)U, (float *)Ud));
  return PRS_OK;
}

int prs_spread(prs_ctx *c, void *stream, const double *x, int32_t n, const void *F, void *fu,
               void *fv, void *fw, int accumulate) {
  if (!c) return PRS_EINVAL;
  if (int rc = check_n(c, n)) return rc;
  if (!fu || !fv || !fw) return fail(c, PRS_EINVAL, "spread: null field");
  if (n > 0 && (!x || !F)) return fail(c, PRS_EINVAL, "spread: null array");
  hipStream_t s = as_stream(stream);
  void *g[3] = {fu, fv, fw};
  Scratch &S = c->S;
  HIP_TRY(c, launch_reset_status(s, S));
  if (n == 0) {
    // nothing to spread: accumulate leaves the field, otherwise it is cleared
    if (!accumulate)
      return c->p.precision == PRS_F64 ? clear_field<double>(c, s, g) : clear_field<float>(c, s, g);
    return PRS_OK;
  }
  HIP_TRY(c, launch_sort(s, S, c->C_step, c->G, x, n, 0));
  HIP_TRY(c, launch_gather_pos(s, S, c->G, x, n, nullptr, nullptr));
  // without accumulate the pass overwrites every node (the field is not read)
  TileCache tc{0, 0, nullptr, nullptr, nullptr};
  tc.overwrite = accumulate ? 0 : 1;
  if (c->p.precision == PRS_F64)
    HIP_TRY(c, launch_spread_tiles<double>(s, c->G, c->C_step, S, (double **)g, n,
                                           (const double *)F, tc));
  else
    HIP_TRY(c, launch_spread_tiles<float>(s, c->G, c->C_step, S, (float **)g, n,
                                          (const float *)F, tc));
  return PRS_OK;
}

int prs_contacts(prs_ctx *c, void *stream, const double *x, int32_t n, int32_t *pairs,
                 int64_t cap, int64_t *n_out) {
  if (!c) return PRS_EINVAL;
  if (int rc = check_n(c, n)) return rc;
  if (!n_out) return fail(c, PRS_EINVAL, "contacts: null n_out");
  if (cap < 0 || (cap > 0 && !pairs)) return fail(c, PRS_EINVAL, "contacts: bad pairs/cap");
  if (n > 0 && !x) return fail(c, PRS_EINVAL, "contacts: null positions");
  *n_out = 0;
  hipStream_t s = as_stream(stream);
  Scratch &S = c->S;
  HIP_TRY(c, launch_reset_status(s, S));
  HIP_TRY(c, launch_sort(s, S, c->C_touch, c->G, x, n, 0));
  HIP_TRY(c, launch_gather_pos(s, S, c->G, x, n, nullptr, nullptr));
  HIP_TRY(c, launch_contact_list(s, S, c->C_touch, c->G, n, pairs, cap, 0));
  if (n > 0) HIP_TRY(c, launch_scan(s, S.ccount, n, S.scan_tmp));
  HIP_TRY(c, launch_contact_list(s, S, c->C_touch, c->G, n, pairs, cap, 1));
  int total = 0;
  uint32_t st = 0;
  if (n > 0)
    HIP_TRY(c, hipMemcpyAsync(&total, S.ccount + n, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(&st, S.status, sizeof st, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (int code = status_code(st)) return fail(c, code, "contacts: %s", status_text(st));
  *n_out = total;
  if (total > cap)
    return fail(c, PRS_ECAPACITY, "contacts: %d contacts exceed cap %lld", total, (long long)cap);
  return PRS_OK;
}

int prs_bed_flags(prs_ctx *c, void *stream, const double *x, int32_t n, int8_t *flags,
                  int64_t *n_bed) {
  if (!c) return PRS_EINVAL;
  if (int rc = check_n(c, n)) return rc;
  if (!n_bed) return fail(c, PRS_EINVAL, "bed_flags: null n_bed");
  if (n > 0 && (!x || !flags)) return fail(c, PRS_EINVAL, "bed_flags: null array");
  *n_bed = 0;
  if (n == 0) return PRS_OK;
  hipStream_t s = as_stream(stream);
  Scratch &S = c->S;
  HIP_TRY(c, launch_reset_status(s, S));
  HIP_TRY(c, launch_sort(s, S, c->C_touch, c->G, x, n, 0));
  HIP_TRY(c, launch_gather_pos(s, S, c->G, x, n, nullptr, nullptr));
  HIP_TRY(c, launch_bed_seed(s, S, c->C_touch, c->G, n));
  // passes in groups of four between reads of the change count (a pass
  // after the last change changes nothing); every pass marks at least one
  // sphere until the last, so n + 1 passes always suffice
  unsigned long long *host = reinterpret_cast<unsigned long long *>(c->host_pinned);
  for (int64_t done = 0; done <= (int64_t)n; done += 4) {
    HIP_TRY(c, hipMemsetAsync(S.counters + 3, 0, sizeof(unsigned long long), s));
    for (int k = 0; k < 4; ++k) HIP_TRY(c, launch_bed_pass(s, S, n, S.counters + 3));
    HIP_TRY(c, hipMemcpyAsync(host, S.counters + 3, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (host[0] == 0) break;
  }
  HIP_TRY(c, hipMemsetAsync(S.counters + 3, 0, sizeof(unsigned long long), s));
  HIP_TRY(c, launch_bed_out(s, S, n, flags, S.counters + 3));
  uint32_t st = 0;
  HIP_TRY(c, hipMemcpyAsync(host, S.counters + 3, sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(&st, S.status, sizeof st, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (int code = status_code(st)) return fail(c, code, "bed_flags: %s", status_text(st));
  *n_bed = (int64_t)host[0];
  return PRS_OK;
}

int prs_step_particles_ex(prs_ctx *c, void *stream, const prs_step_args *A, prs_stats *stats) {
  if (!c) return PRS_EINVAL;
  if (!A) return fail(c, PRS_EINVAL, "step: null arguments");
  const void *const *uhat = A->uhat;
  void *const *f = A->f;
  const int zero_f = A->zero_f;
  double *x = A->x, *u = A->u, *om = A->om;
  const int32_t n = A->n;
  const prs_history *H = A->hist;
  double *Fh = A->Fh, *Th = A->Th;
  const void *F0 = A->F0;
  if (int rc = check_n(c, n)) return rc;
  if (!uhat || !f || !uhat[0] || !uhat[1] || !uhat[2] || !f[0] || !f[1] || !f[2])
    return fail(c, PRS_EINVAL, "step: null field");
  if (n > 0 && (!x || !u || !om || !Fh || !Th || !H || !H->partner || !H->delta_t || !H->u_in ||
                !H->count))
    return fail(c, PRS_EINVAL, "step: null particle array");
  if (c->mlp && (!zero_f || F0))
    return fail(c, PRS_EINVAL, "step: a learned start needs zero_f = 1 and no F0");
  if (!(A->alpha >= 0) || !std::isfinite(A->alpha))
    return fail(c, PRS_EINVAL, "step: alpha must be finite and >= 0 (0: the context's)");
  if (n > 0 && A->inner_prev && !A->inner_out)
    return fail(c, PRS_EINVAL, "step: inner_prev needs inner_out");
  hipStream_t s = as_stream(stream);
  Scratch &S = c->S;
  const prs_params &q = c->p;
  const bool f64 = q.precision == PRS_F64;
  const double adt = (A->alpha > 0 ? A->alpha : q.alpha) * q.dt_f;

  HIP_TRY(c, launch_reset_status(s, S));
  c->marks.clear();
  c->events_used = 0;
  if (zero_f && n == 0) {
    // (with spheres the forcing's first spreading pass overwrites f)
    HIP_TRY(c, phase_begin(c, s));
    if (int rc = f64 ? clear_field<double>(c, s, f) : clear_field<float>(c, s, f)) return rc;
    HIP_TRY(c, phase_end(c, s, kZeroF));
  }
  if (n > 0) {
    HIP_TRY(c, phase_begin(c, s));
    HIP_TRY(c, launch_sort(s, S, c->C_step, c->G, x, n, 0));
    HIP_TRY(c, launch_gather_state(s, S, c->G, x, u, om, H, n));
    HIP_TRY(c, phase_end(c, s, kSort));
  }

  // ---- immersed-boundary forcing (multi-direct forcing, Jacobi) ----
  int iters = 0, n_slip = 0, rejected = 0;
  double *hist_host = c->host_pinned;   // [0..63] slip^2, [64] zero-forcing slip^2
  if (n > 0) {
    // the first pass sees f = 0 only when the field was cleared here and no
    // initial marker force is spread; otherwise the zero-forcing slip needs a
    // pass of its own
    const bool need_den = !zero_f || F0 != nullptr;
    const bool learned = c->mlp != nullptr;
    const int rc =
        f64 ? run_forcing<double>(c, s, adt, uhat, f, n, F0, need_den, learned, -1, nullptr, iters,
                                  n_slip, rejected, zero_f != 0)
            : run_forcing<float>(c, s, adt, uhat, f, n, F0, need_den, learned, -1, nullptr, iters,
                                 n_slip, rejected, zero_f != 0);
    if (rc != PRS_OK) return rc;
    HIP_TRY(c, launch_ib_finish(s, S, c->G, n, q.rho_f));
    if (A->inner_out) {
      // fluid inside the spheres: rho_f d/dt int u** dV joins the force
      if (f64) {
        const double *uh[3] = {(const double *)uhat[0], (const double *)uhat[1],
                               (const double *)uhat[2]};
        const double *ff[3] = {(const double *)f[0], (const double *)f[1], (const double *)f[2]};
        HIP_TRY(c, launch_inner_step<double>(s, c->G, S, uh, ff, adt, q.rho_f, n, A->inner_prev,
                                             A->inner_out));
      } else {
        const float *uh[3] = {(const float *)uhat[0], (const float *)uhat[1],
                              (const float *)uhat[2]};
        const float *ff[3] = {(const float *)f[0], (const float *)f[1], (const float *)f[2]};
        HIP_TRY(c, launch_inner_step<float>(s, c->G, S, uh, ff, adt, q.rho_f, n, A->inner_prev,
                                            A->inner_out));
      }
    }

    // ---- contacts and Newton-Euler substeps ----
    const int n_sub = A->advance ? q.n_sub : 0;
    if (n_sub > 0) {
      HIP_TRY(c, phase_begin(c, s));
      HIP_TRY(c, launch_candidates(s, S, c->C_step, c->G, n, 2.0 * q.radius + q.skin));
      HIP_TRY(c, phase_end(c, s, kSearch));
    }
    for (int sub = 0; sub < n_sub; ++sub) {
      HIP_TRY(c, phase_begin(c, s));
      HIP_TRY(c, launch_substep(s, S, c->G, c->M, n, sub & 1, sub == n_sub - 1));
      HIP_TRY(c, phase_end(c, s, kSubstep));
    }
    HIP_TRY(c, phase_begin(c, s));
    HIP_TRY(c, launch_writeback(s, S, x, u, om, H, Fh, Th, n, n_sub & 1));
    HIP_TRY(c, phase_end(c, s, kWriteback));
  }

  uint32_t st = 0;
  unsigned long long cnt[4] = {0, 0, 0, 0};
  HIP_TRY(c, hipMemcpyAsync(&st, S.status, sizeof st, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(cnt, S.counters, sizeof cnt, hipMemcpyDeviceToHost, s));
  if (n_slip > 0)
    HIP_TRY(c, hipMemcpyAsync(hist_host, S.slip_hist, sizeof(double) * (PRS_MAX_SLIP + 1),
                              hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  HIP_TRY(c, phase_collect(c));
  if (stats) {
    fill_stats(stats, hist_host, iters, n_slip);
    stats->rejected_learned = rejected;
    stats->contacts = (int64_t)cnt[0];
    stats->pairs_last = (int64_t)cnt[1] / 2;
    stats->wall_last = (int64_t)cnt[2];
    stats->flags = st;
  }
  if (int code = status_code(st)) return fail(c, code, "step: %s", status_text(st));
  return PRS_OK;
}

int prs_step_particles(prs_ctx *c, void *stream, const void *const uhat[3], void *const f[3],
                       int zero_f, double *x, double *u, double *om, int32_t n,
                       const prs_history *H, double *Fh, double *Th, const void *F0,
                       prs_stats *stats) {
  prs_step_args A{};
  A.uhat = uhat;
  A.f = f;
  A.zero_f = zero_f;
  A.x = x;
  A.u = u;
  A.om = om;
  A.n = n;
  A.hist = H;
  A.Fh = Fh;
  A.Th = Th;
  A.F0 = F0;
  A.alpha = 0.0;
  A.advance = 1;
  return prs_step_particles_ex(c, stream, &A, stats);
}

int prs_inner_fluid(prs_ctx *c, void *stream, const void *const u[3], const double *x, int32_t n,
                    double *inner) {
  if (!c) return PRS_EINVAL;
  if (int rc = check_n(c, n)) return rc;
  if (!u || !u[0] || !u[1] || !u[2]) return fail(c, PRS_EINVAL, "inner_fluid: null field");
  if (n > 0 && (!x || !inner)) return fail(c, PRS_EINVAL, "inner_fluid: null array");
  if (n == 0) return PRS_OK;
  hipStream_t s = as_stream(stream);
  Scratch &S = c->S;
  HIP_TRY(c, launch_reset_status(s, S));
  if (c->p.precision == PRS_F64) {
    const double *g[3] = {(const double *)u[0], (const double *)u[1], (const double *)u[2]};
    HIP_TRY(c, launch_inner_fluid<double>(s, c->G, S, g, x, n, inner));
  } else {
    const float *g[3] = {(const float *)u[0], (const float *)u[1], (const float *)u[2]};
    HIP_TRY(c, launch_inner_fluid<float>(s, c->G, S, g, x, n, inner));
  }
  uint32_t st = 0;
  HIP_TRY(c, hipMemcpyAsync(&st, S.status, sizeof st, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (int code = status_code(st)) return fail(c, code, "inner_fluid: %s", status_text(st));
  return PRS_OK;
}

int prs_set_learned(prs_ctx *c, const prs_mlp *mlp) {
  if (!c) return PRS_EINVAL;
  if (mlp) {
    const int nb = brick_edge(c->p.radius, c->p.h);
    const size_t need =
        learned_lds_bytes(c->p.n_markers, nb, c->p.precision == PRS_F64 ? 8 : 4) + 4096;
    hipDeviceProp_t prop;
    HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
    if (need > prop.sharedMemPerBlock)
      return fail(c, PRS_EINVAL, "set_learned: %zu bytes of LDS needed, %zu available", need,
                  (size_t)prop.sharedMemPerBlock);
  }
  c->mlp = mlp;
  return PRS_OK;
}

int prs_forcing_samples(prs_ctx *c, void *stream, const void *const uhat[3], void *const f[3],
                        const double *x, const double *u, const double *om, int32_t n,
                        int32_t n_iter, float *feat, float *target, prs_stats *stats) {
  if (!c) return PRS_EINVAL;
  if (int rc = check_n(c, n)) return rc;
  if (!uhat || !f || !uhat[0] || !uhat[1] || !uhat[2] || !f[0] || !f[1] || !f[2])
    return fail(c, PRS_EINVAL, "samples: null field");
  if (n_iter < 1 || n_iter > PRS_MAX_SLIP - 1)
    return fail(c, PRS_EINVAL, "samples: n_iter = %d outside 1..%d", n_iter, PRS_MAX_SLIP - 1);
  if (n > 0 && (!x || !u || !om || !feat || !target))
    return fail(c, PRS_EINVAL, "samples: null particle or output array");
  hipStream_t s = as_stream(stream);
  Scratch &S = c->S;
  const bool f64 = c->p.precision == PRS_F64;
  HIP_TRY(c, launch_reset_status(s, S));
  c->marks.clear();
  c->events_used = 0;
  int rc = f64 ? clear_field<double>(c, s, f) : clear_field<float>(c, s, f);
  if (rc) return rc;
  int iters = 0, n_slip = 0, rejected = 0;
  if (n > 0) {
    HIP_TRY(c, launch_sort(s, S, c->C_step, c->G, x, n, 0));
    HIP_TRY(c, launch_gather_pos(s, S, c->G, x, n, u, om));
    const size_t M = (size_t)n * c->p.n_markers;
    HIP_TRY(c, launch_fill_zero<float>(s, target, 3 * M));
    if (f64) {
      const double *uh[3] = {(const double *)uhat[0], (const double *)uhat[1],
                             (const double *)uhat[2]};
      HIP_TRY(c, launch_interp_feat<double>(s, c->G, S, uh, n, feat));
    } else {
      const float *uh[3] = {(const float *)uhat[0], (const float *)uhat[1],
                            (const float *)uhat[2]};
      HIP_TRY(c, launch_interp_feat<float>(s, c->G, S, uh, n, feat));
    }
    // f = 0: the first iteration's slip is the zero-forcing slip
    const double adt = c->p.alpha * c->p.dt_f;
    rc = f64 ? run_forcing<double>(c, s, adt, uhat, f, n, nullptr, false, false, n_iter, target,
                                   iters, n_slip, rejected)
             : run_forcing<float>(c, s, adt, uhat, f, n, nullptr, false, false, n_iter, target,
                                  iters, n_slip, rejected);
    if (rc) return rc;
  }
  uint32_t st = 0;
  double *hist_host = c->host_pinned;
  HIP_TRY(c, hipMemcpyAsync(&st, S.status, sizeof st, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(hist_host, S.slip_hist, sizeof(double) * (PRS_MAX_SLIP + 1),
                            hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->marks.clear();
  c->events_used = 0;
  if (stats) {
    fill_stats(stats, hist_host, iters, n_slip);
    stats->flags = st;
  }
  if (int code = status_code(st)) return fail(c, code, "samples: %s", status_text(st));
  return PRS_OK;
}

int prs_timing_enable(prs_ctx *c, int enable) {
  if (!c) return PRS_EINVAL;
  c->timing = enable != 0;
  c->marks.clear();
  c->events_used = 0;
  return PRS_OK;
}

int prs_timing_read(prs_ctx *c, prs_timing *out, int reset) {
  if (!c || !out) return PRS_EINVAL;
  out->steps = c->steps;
  out->ms_zero_f = c->ms[kZeroF];
  out->ms_sort = c->ms[kSort];
  out->ms_interp = c->ms[kInterp];
  out->ms_spread = c->ms[kSpread];
  out->ms_search = c->ms[kSearch];
  out->ms_substep = c->ms[kSubstep];
  out->ms_writeback = c->ms[kWriteback];
  out->n_interp = c->launches[kInterp];
  out->n_spread = c->launches[kSpread];
  out->n_substep = c->launches[kSubstep];
  out->ms_learned = c->ms[kLearned];
  out->n_learned = c->launches[kLearned];
  out->ms_record = c->ms[kRecord];
  out->n_record = c->launches[kRecord];
  if (reset) {
    for (int k = 0; k < kPhases; ++k) {
      c->ms[k] = 0.0;
      c->launches[k] = 0;
    }
    c->steps = 0;
  }
  return PRS_OK;
}

}  // extern "C"
