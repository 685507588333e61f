// Internal declarations of the HIP implementation behind include/prs.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "prs.h"

namespace prs {

constexpr int kSlots = PRS_SLOTS;
constexpr int kMaxPP = PRS_MAX_PP;
constexpr int kCandCap = 32;   // collision-search candidates per sphere
constexpr int kMaxMarkers = 1024;

// Device status word bits.
enum : uint32_t {
  kFlagSlots = 1u << 0,      // a sphere touches more than twelve spheres
  kFlagCand = 1u << 1,       // more than kCandCap search candidates
  kFlagNonFinite = 1u << 2,  // NaN / inf in the sphere state
  kFlagDomain = 1u << 3,     // a centre outside the box
  kFlagSkin = 1u << 4,       // displacement beyond skin/2 within a step
};

// Box, grid and sphere geometry as seen by the kernels.
struct Geom {
  int nx, ny, nz;
  double h, inv_h;
  double Lx, Ly, Lz;
  double R;
  int nl;
  double dV;
  // bound on the sum of one sphere's stencil weights at any node, in units
  // of the sphere's largest marker value (fixed-point spreading)
  double wsum_bound;
};

// Collision cells: an ncx*ncy*ncz partition of the box, cell edges >= the
// search cut-off; cells are numbered by 4x4x4 tiles (tile-major, Morton order
// inside a tile) so that spheres sorted by cell number are close in space.
struct Cells {
  int ncx, ncy, ncz;
  double csx, csy, csz;
  int ntx, nty, ntz;
  int nkeys;
};

// Sphere mechanics.
struct Mech {
  double m, I;
  double fg[3];           // buoyant weight (rho_p - rho_f) V g
  // normal and tangential stiffness and damping, sphere-sphere (pp) and
  // sphere-wall (pw)
  double kn_pp, kn_pw, dn_pp, dn_pw, kt_pp, kt_pw, dt_pp, dt_pw, mu;
  double dtp;             // particle substep
  double skin_half2;      // (skin/2)^2
};

// Entries of a spreading tile's record: candidate sphere indices, then the
// culled (candidate << 10 | marker) codes; a tile with more is not recorded.
constexpr int kTileRecord = 2304;

// Scratch owned by a context.
struct Scratch {
  int cap_n;
  // sorting / cell list
  int *key, *count, *fill, *start, *perm, *inv_perm;
  int *scan_tmp;
  size_t scan_tmp_elems;
  // sorted sphere state, double-buffered SoA [3][n]
  double *xs[2], *us[2], *ws[2], *x0;
  // the same state packed per sphere, double-buffered like xs: positions
  // [n][4] (x, 0), then velocities [n][8] (u, 0, omega, 0) -- the substeps'
  // gathers of a partner's state touch one or two cache lines, not nine,
  // and the contact test's gathers of positions four spheres a 128-byte line
  // (see PkPos / PkVel)
  double *pk[2];
  double *fh, *th;            // [3][n] sorted
  double *ft_acc;             // [12][n]: (sum, compensation) x (Fx Fy Fz Tx Ty Tz)
  double *ft_part;            // [12][n]: the same for the latest interpolation pass
  double *slip_part;          // [2][n]: slip^2 and zero-forcing slip^2 per sphere
  float *vmax;                // [n]: largest |marker value| per sphere (latest spread source)
  // per-tile record of the spreading (TileCache), kTileRecord entries a tile
  unsigned *tc_items;
  int *tc_count, *tc_ncand;
  int tc_cap;
  double *slip_hist;          // [kMaxSlip + 1 + 256]: per pass, zero-forcing, block partials
  int *ncand, *cand;          // [n], [kCandCap][n]
  int *bed;                   // [n]: bed marks of the bed / flying detection (sorted order)
  // contact history, internal SoA layout [slot][n], double-buffered
  int *h_cnt[2], *h_id[2];
  double *h_dt[2], *h_uin[2];
  // contact listing
  int *ccount, *coffset;
  // marker corrections dF [3][n*nl] in grid precision
  void *dF;
  // I[u-hat] of the step's markers [3][n*nl] in grid precision
  void *u0;
  // status and counters
  uint32_t *status;
  unsigned long long *counters;   // [0] directed contacts, [1] pp last, [2] wall last
  double *templ;                  // [nl][3]
  // marker offsets (R / h) t_l in node units: [nl][8] floats (rounded value
  // xyz, pad, remainder xyz, pad) and [nl][4] doubles (xyz, pad)
  float *tm32;
  double *tm64;
  // the same in the interpolation's lane order (entry i for marker
  // lane_order[i]), so a lane's offsets load without the order lookup
  float *tm32_lane;
  double *tm64_lane;
  int *lane_order;                // [nl]: marker handled by interpolation lane i
};

// Packed sphere state: sphere k's position (3 doubles) and its velocity and
// angular velocity (at +0 and +4) in an array of 12 n doubles.
#ifndef PRS_PK_SPLIT
#define PRS_PK_SPLIT 1
#endif
__host__ __device__ inline size_t pk_pos(size_t k, size_t n) { return PRS_PK_SPLIT ? 4 * k : 12 * k; }
__host__ __device__ inline size_t pk_vel(size_t k, size_t n) {
  return PRS_PK_SPLIT ? 4 * n + 8 * k : 12 * k + 4;
}

// Learned warm start: the network's device buffers and, for the feature
// pass, the output array and the sorted-to-caller permutation.
struct LearnArgs {
  const unsigned short *wbf;   // BF16 weights
  const float *master;         // FP32 master weights (biases)
  const float *norm;           // feature mean/std, target mean/std
  float *feat;                 // feature pass: [n][nl][16] in caller order
  const int *perm;             // sorted position -> caller index
  const float *gelu_tab;       // GELU table of the fused pass (float4 [kGeluTabN])
};

// Per-tile record of the spreading's candidate spheres and culled markers,
// reused by the later passes of a step (the spheres do not move between
// them).  Tile t's region items[t * cap ...]: ncand[t] sorted sphere indices,
// then count[t] markers as (candidate slot << 10 | marker); count -1: not
// recorded.
// mode 0: neither record nor replay; 1: record; 2: replay recorded tiles.
struct TileCache {
  int mode;
  int cap;
  unsigned *items;
  int *count;
  int *ncand;
  // nonzero: f holds stale values and is overwritten, every node of the
  // grid written once (zero where nothing is spread): clearing f fused into
  // the pass
  int overwrite = 0;
};

// ---- launchers (defined in the .hip files) ----
hipError_t launch_template(hipStream_t s, double *t, float *tm32, double *tm64, float *tm32_lane,
                           double *tm64_lane, int *lane_order,
                           int nl, double r_over_h);

hipError_t launch_sort(hipStream_t s, const Scratch &S, const Cells &C, const Geom &G,
                       const double *x_caller, int n, int nkeys_scan_levels);
hipError_t launch_gather_state(hipStream_t s, const Scratch &S, const Geom &G, const double *x,
                               const double *u, const double *om, const prs_history *H, int n);
hipError_t launch_gather_pos(hipStream_t s, const Scratch &S, const Geom &G, const double *x,
                             int n, const double *u, const double *om);
hipError_t launch_writeback(hipStream_t s, const Scratch &S, double *x, double *u, double *om,
                            const prs_history *H, double *Fh, double *Th, int n, int buf);
hipError_t launch_scan(hipStream_t s, int *data, int n, int *tmp);

int brick_edge(double R, double h);
// LDS bytes of one component's interpolation brick (x-rows padded to 16 bytes).
size_t brick_bytes(int nb, int esz);
// LDS of the interpolation's brick buffers (one or two bricks)
int interp_brick_buffers(int nb, int esz);
size_t interp_lds_bytes(int nb, int esz);
// Row pitch of the brick in elements: nb rounded up to 16 bytes, plus
// PRS_BRICK_PAD 16-byte vectors (a knob: padding by one or two vectors
// measured slower at D/h = 10 on MI355X).
#ifndef PRS_BRICK_PAD
#define PRS_BRICK_PAD 0
#endif
template <typename T>
__host__ __device__ constexpr int brick_pitch_c(int nb) {
  return ((nb + 16 / (int)sizeof(T) - 1) / (16 / (int)sizeof(T)) + PRS_BRICK_PAD) *
         (16 / (int)sizeof(T));
}
template <typename T>
hipError_t launch_interp_plain(hipStream_t s, const Geom &G, const Scratch &S, const T *gu,
                               const T *gv, const T *gw, const double *x, const double *up,
                               const double *om, int n, T *U, T *Ud);
template <typename T>
hipError_t launch_interp_mdf(hipStream_t s, const Geom &G, const Scratch &S, const T *uh[3],
                             const T *f[3], int n, double adt, int den_only);
template <typename T>
hipError_t launch_interp_feat(hipStream_t s, const Geom &G, const Scratch &S, const T *uh[3], int n,
                              float *feat);
template <typename T>
hipError_t launch_interp_learned(hipStream_t s, const Geom &G, const Scratch &S, const T *uh[3],
                                 int n, double adt, const LearnArgs &la);
template <typename T>
hipError_t launch_accum_target(hipStream_t s, const Geom &G, const Scratch &S, int n, double adt,
                               float *target);
// Dynamic LDS of the fused learned pass (bricks, network inputs, weights, table).
size_t learned_lds_bytes(int nl, int nb, int esz);
// Device buffers of a network (defined with the network).
void mlp_buffers(const prs_mlp *mlp, LearnArgs *la);

// Records of the spreading tiles (candidates and culled markers) for the
// passes of a step that replay them.
template <typename T>
hipError_t launch_tile_record(hipStream_t s, const Geom &G, const Cells &C, const Scratch &S,
                              int n);
template <typename T>
hipError_t launch_spread_tiles(hipStream_t s, const Geom &G, const Cells &C, const Scratch &S,
                               T *f[3], int n, const T *src_caller, TileCache tc = TileCache{});
// Nodes per axis of a spreading tile for fields of esz-byte elements.
int spread_tile_dim(int esz, int axis);
// Tiles of the spreading grid for fields of type T.
template <typename T>
int spread_tile_count(const Geom &G);
hipError_t launch_ft_commit(hipStream_t s, const Scratch &S, int n);
template <typename T>
hipError_t launch_sphere_vmax(hipStream_t s, const Geom &G, const Scratch &S, int n, const T *F);
template <typename T>
hipError_t launch_marker_sums(hipStream_t s, const Geom &G, const Scratch &S, int n, const T *F0);
hipError_t launch_copy_scalar(hipStream_t s, const double *src, double *dst);
hipError_t launch_ib_begin(hipStream_t s, const Scratch &S, int n);
hipError_t launch_slip_reduce(hipStream_t s, const Scratch &S, int n, int iter, int which);
hipError_t launch_ib_finish(hipStream_t s, const Scratch &S, const Geom &G, int n, double rho_f);
template <typename T>
hipError_t launch_fill_zero(hipStream_t s, T *p, size_t count);

hipError_t launch_candidates(hipStream_t s, const Scratch &S, const Cells &C, const Geom &G,
                             int n, double cut);
hipError_t launch_substep(hipStream_t s, const Scratch &S, const Geom &G, const Mech &M, int n,
                          int src, int last);
hipError_t launch_contact_list(hipStream_t s, const Scratch &S, const Cells &C, const Geom &G,
                               int n, int32_t *pairs, long long cap, int phase);
hipError_t launch_reset_status(hipStream_t s, const Scratch &S);
template <typename T>
hipError_t launch_inner_fluid(hipStream_t s, const Geom &G, const Scratch &S, const T *u[3],
                              const double *x, int n, double *inner);
template <typename T>
hipError_t launch_inner_step(hipStream_t s, const Geom &G, const Scratch &S, const T *uh[3],
                             const T *f[3], double adt, double rho_f, int n, const double *prev,
                             double *inner_out);
hipError_t launch_bed_seed(hipStream_t s, const Scratch &S, const Cells &C, const Geom &G, int n);
hipError_t launch_bed_pass(hipStream_t s, const Scratch &S, int n, unsigned long long *changed);
hipError_t launch_bed_out(hipStream_t s, const Scratch &S, int n, int8_t *flags,
                          unsigned long long *count);

}  // namespace prs
