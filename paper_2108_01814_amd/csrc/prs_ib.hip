// Immersed-boundary kernels: marker template, interpolation of the staggered
// fluid velocity at the Lagrangian markers with the direct-forcing
// correction, and diffusion (spreading) of marker forces back to the grid
// (sec. 3.3 and eq. 4 of the paper; the regularised delta function is the
// three-point kernel, the iteration is multi-direct forcing in Jacobi form).
//
// Interpolation: one workgroup per sphere, one lane per marker, so every
// workgroup carries the same number of markers however dense the bed is
// around it (the marker-based balancing of sec. 3.3 on one GPU).  The grid
// brick around the sphere is staged in LDS (one velocity component at a time
// unless all three fit in PRS_BRICK_ALL3_MAX_BYTES) with coalesced row loads,
// the next component's loads in flight while the current one is computed;
// the 27-point stencils then read LDS only.  Each pass loads one field: u-hat
// in the step's first pass (whose result is recorded per marker), f in the
// later ones (the recorded I[u-hat] added).
//
// Spreading: one workgroup per grid tile.  The tile gathers the spheres whose
// markers can reach it from the cell list (the step's first pass records
// them, the later passes replay the record), accumulates their contributions
// to the tile's own nodes with LDS atomics (32-bit fixed point for
// single-precision fields, double precision otherwise), and adds the tile to
// the force field with plain coalesced read-modify-writes (or stores every
// node, when the pass also clears the field).  Every grid node belongs to
// exactly one tile, so no global atomics are needed.
#include <algorithm>
#include <type_traits>

#include "prs_mlp.h"
#include "prs_stencil.h"

namespace prs {

// ---------------------------------------------------------------------------
// template
// ---------------------------------------------------------------------------
// Fibonacci sphere, pole along y.  The y-component 1 - (2l+1)/N decreases
// with l, which the spreading kernel uses to cull markers by height.
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

// Lane order of the interpolation workgroup: within every aligned chunk of
// 64 markers (a band of nearly equal height, the template's y-component being
// monotone in l) sort by azimuth, so the lanes of one wave handle neighbouring
// markers and their stencil reads from LDS mostly coincide or sit side by side.
__global__ void k_lane_order(const double *t, int nl, int *order) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nl) return;
  const int c0 = (l / 64) * 64, c1 = min(c0 + 64, nl);
  const double al = atan2(t[3 * l + 2], t[3 * l + 0]);
  int rank = 0;
  for (int m = c0; m < c1; ++m) {
    const double am = atan2(t[3 * m + 2], t[3 * m + 0]);
    if (am < al || (am == al && m < l)) ++rank;
  }
  order[c0 + rank] = l;
}

// Marker offsets in node units, (R / h) t_l: the double value, and its
// single-precision rounding plus the remainder (also rounded).
__global__ void k_marker_offsets(const double *t, int nl, double r_over_h, float *tm32,
                                 double *tm64) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nl) return;
  for (int a = 0; a < 3; ++a) {
    const double m = r_over_h * t[3 * l + a];
    const float hi = (float)m;
    tm32[8 * l + a] = hi;
    tm32[8 * l + 4 + a] = (float)(m - (double)hi);
    tm64[4 * l + a] = m;
  }
  tm32[8 * l + 3] = tm32[8 * l + 7] = 0.f;
  tm64[4 * l + 3] = 0.0;
}

// The offsets in the interpolation's lane order.
__global__ void k_lane_offsets(const int *order, const float *tm32, const double *tm64, int nl,
                               float *tm32_lane, double *tm64_lane) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl) return;
  const int l = order[i];
  for (int k = 0; k < 8; ++k) tm32_lane[8 * i + k] = tm32[8 * l + k];
  for (int k = 0; k < 4; ++k) tm64_lane[4 * i + k] = tm64[4 * l + k];
}

hipError_t launch_template(hipStream_t s, double *t, float *tm32, double *tm64, float *tm32_lane,
                           double *tm64_lane, int *lane_order, int nl, double r_over_h) {
  hipLaunchKernelGGL(k_template, dim3((nl + 255) / 256), dim3(256), 0, s, t, nl);
  hipLaunchKernelGGL(k_lane_order, dim3((nl + 255) / 256), dim3(256), 0, s, t, nl, lane_order);
  hipLaunchKernelGGL(k_marker_offsets, dim3((nl + 255) / 256), dim3(256), 0, s, t, nl, r_over_h,
                     tm32, tm64);
  hipLaunchKernelGGL(k_lane_offsets, dim3((nl + 255) / 256), dim3(256), 0, s, lane_order, tm32,
                     tm64, nl, tm32_lane, tm64_lane);
  return hipGetLastError();
}

int brick_edge(double R, double h) { return 2 * brick_reach(R, h) + 2; }

size_t brick_bytes(int nb, int esz) {
  return (size_t)nb * nb * (esz == 8 ? brick_pitch_c<double>(nb) : brick_pitch_c<float>(nb)) *
         esz;
}

// Interpolation brick chunks loaded straight into LDS (1) or through
// registers (0).
#ifndef PRS_INTERP_DMA
#define PRS_INTERP_DMA 1
#endif

// Brick chunks that no stencil of the sphere reads skipped (1) or loaded (0).
#ifndef PRS_INTERP_CULL
#define PRS_INTERP_CULL 1
#endif

static inline int block_for(int nl) { return ((nl + 63) / 64) * 64; }

// Brick buffers of the interpolation: two (the next component's brick loads
// while the current one's stencils run) when they take at most 32 KB of LDS,
// else one (the occupancy is worth more than the overlap).
int interp_brick_buffers(int nb, int esz) {
  return PRS_INTERP_DMA && 2 * brick_bytes(nb, esz) <= 32768 ? 2 : 1;
}

size_t interp_lds_bytes(int nb, int esz) { return brick_bytes(nb, esz) * interp_brick_buffers(nb, esz); }

// LDS of the fused learned pass: the brick buffers, later reused for the
// network's standardised inputs (BF16) and predictions (FP32) of the block's
// markers, then the forward weights and the GELU table (staged at the start,
// while the bricks load).
__host__ __device__ inline size_t learned_io_region(int block, size_t bricks) {
  const size_t io = ((size_t)block * (kMlpIn * sizeof(unsigned short) + kMlpUsed * sizeof(float)) +
                     15) & ~(size_t)15;
  return bricks > io ? bricks : io;
}

// (one brick buffer: the network's LDS and its occupancy matter more here
// than overlapping the brick loads)
size_t learned_lds_bytes(int nl, int nb, int esz) {
  return learned_io_region(block_for(nl), brick_bytes(nb, esz)) + kMlpFwdLdsBytes +
         kGeluTabN * sizeof(float4);
}

// ---------------------------------------------------------------------------
// interpolation with an LDS brick per sphere
// ---------------------------------------------------------------------------
enum { kInterpMDF = 0, kInterpDen = 1, kInterpPlain = 2, kInterpFeat = 3, kInterpLearned = 4 };

// MODE kInterpFeat   : like kInterpDen, and writes each marker's raw features
//                      (slip, normal, u_p, R omega_p, zero padding) to feat.
// MODE kInterpLearned: like kInterpDen, then evaluates the warm-start network
//                      on the features and writes the initial marker force
//                      F0 = prediction / (alpha dt) [3][M] and its per-sphere
//                      force/torque sums.


// MODE kInterpMDF  : sorted SoA state; u** = a + adt*b (b0 == NULL: a field
//                    known to be zero, not read); writes dF [3][M],
//                    the slip partial and the force/torque partials.
// MODE kInterpDen  : sorted SoA state; a only; writes the zero-forcing slip
//                    partial ||U_d - I[a]||^2.
// MODE kInterpPlain: caller-order AoS positions; a only; writes U [n][nl][3]
//                    and optionally U_d.
//
// The brick: nodes I_a - E .. I_a - E + nb - 1 along each axis a (I the
// sphere centre's node, E = brick_reach), the same origin for the three
// components (their staggering is in the stencil fractions).  Each
// component's brick is nb * nb x-rows of nb values, padded to P elements
// (16-byte chunks), loaded with one 16-byte load per chunk.  Rows outside the
// fluid (and the wall faces of v) are zero; chunks that cross the periodic x
// seam are loaded element by element.
//
// Chunk slots per lane of one component's brick: FP32 at D/h = 10 needs 3
// (784 chunks, 320 lanes).
#ifndef PRS_BRICK_SLOTS_F32
#define PRS_BRICK_SLOTS_F32 3
#endif
#ifndef PRS_BRICK_SLOTS_F64
#define PRS_BRICK_SLOTS_F64 5
#endif
template <typename T>
struct BrickSlots {
  static constexpr int value = sizeof(T) == 4 ? PRS_BRICK_SLOTS_F32 : PRS_BRICK_SLOTS_F64;
};

// NB: brick edge known at compile time (14 at D/h = 10, 20 at D/h = 16) or 0
// for the runtime edge nb.
// 16 bytes per lane from global memory straight into LDS: lane i of the wave
// writes at wave_base + 16 i (wave_base uniform across the wave).
__device__ inline void lds_load16(const void *src, void *wave_base) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)wave_base, 16,
                                   0, 0);
}
// 4 bytes per lane the same way: lane i writes at wave_base + 4 i.
__device__ inline void lds_load4(const void *src, void *wave_base) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)wave_base, 4,
                                   0, 0);
}
// Waits until this wave's memory operations have completed.
__device__ inline void wait_loads() { __builtin_amdgcn_s_waitcnt(0); }

// K: markers a lane.  With K = 2 (single-precision MDF passes only) lane t
// takes the lane slots t and t + blockDim: a sphere needs half the waves,
// so with one brick buffer about twice as many spheres are resident on a
// compute unit (a unit holds 32 waves; five-wave spheres left six of them
// in flight), and the per-sphere work is shared by twice the markers.  The
// second marker's terms are added in the lane before the wave sums.
constexpr int kSlotsK2 = 5;
#ifndef PRS_INTERP_K2
#define PRS_INTERP_K2 1
#endif
#ifndef PRS_INTERP_K2_WAVES
#define PRS_INTERP_K2_WAVES 6
#endif   // chunk slots a lane with K = 2 (784 chunks / 192 lanes at D/h = 10)
template <typename T, int MODE, int NB, int K = 1>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(K == 2 ? PRS_INTERP_K2_WAVES : 1)))
void k_interp(
    Geom G, const double *__restrict__ templ, const T *__restrict__ tm, const T *__restrict__ a0,
    const T *__restrict__ a1, const T *__restrict__ a2, const T *__restrict__ b0,
    const T *__restrict__ b1, const T *__restrict__ b2, double adt, double inv_adt,
    const double *__restrict__ xs, const double *__restrict__ us, const double *__restrict__ ws,
    int n, int nb, T *__restrict__ out, T *__restrict__ out2, double *__restrict__ slip_part,
    double *__restrict__ ft_part, const int *__restrict__ order, LearnArgs la,
    float *__restrict__ vmax_out, T *__restrict__ u0, int nbuf) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T *brick = reinterpret_cast<T *>(smem_raw);
  if (NB > 0) nb = NB;
  // the workgroup size and this wave's first thread, read once (blockDim is
  // otherwise reloaded from the dispatch packet, and that load's wait would
  // also wait for the brick loads in flight)
  const int bdim = (int)blockDim.x;
  const int wave_base = __builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~63;   // scalar
  const int p = xcd_item(blockIdx.x, n);
  if (p < 0) return;
  static_assert(K == 1 || (K == 2 && MODE == kInterpMDF && sizeof(T) == 4),
                "two markers a lane in the single-precision MDF pass only");
  const bool active = (int)threadIdx.x < G.nl;
  const int l = active ? order[threadIdx.x] : 0;
  // the second marker of the lane (K = 2)
  const bool active2 = K == 2 && (int)threadIdx.x + bdim < G.nl;
  const int l2 = active2 ? order[threadIdx.x + bdim] : 0;
  const size_t N = (size_t)n;

  // the sphere's node, staggered fractions and brick origin (the rest of
  // the sphere's state is read once the field is interpolated)
  int lo[3];
  T fo[3][2];
  const int E = brick_reach(G.R, G.h);
  {
    uint32_t fl = 0;
    for (int a = 0; a < 3; ++a) {
      const double xa = MODE == kInterpPlain
                            ? sane_coord(xs[3 * p + a], a == 0 ? G.Lx : (a == 1 ? G.Ly : G.Lz),
                                         a == 1, fl)
                            : xs[a * N + p];
      int Ia;
      sphere_axis<T>(xa, G.inv_h, Ia, fo[a]);
      lo[a] = Ia - E;
    }
  }
  const T tadt = (T)adt;
  // the correction r / (alpha dt) by multiplication (1 / (alpha dt) from the
  // host: a division here would be a per-lane FP64 sequence)
  const T inv_tadt = (T)inv_adt;
  // An MDF pass over a nonzero f interpolates f alone and adds the step's
  // recorded I[u-hat] (the interpolation is linear: I[u-hat + adt f] =
  // I[u-hat] + adt I[f]), so it loads one field instead of two; the passes
  // that interpolate u-hat record it in u0.
  const bool f_only = MODE == kInterpMDF && b0 != nullptr;
  T mhi[3] = {0, 0, 0}, mlo[3] = {0, 0, 0};
  if (active) MarkerOffset<T>::load(tm, threadIdx.x, mhi, mlo);   // tm in lane order
  T mhi2[3] = {0, 0, 0}, mlo2[3] = {0, 0, 0};
  if (K == 2 && active2) MarkerOffset<T>::load(tm, threadIdx.x + bdim, mhi2, mlo2);

  constexpr int VEC = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  const int P = brick_pitch_c<T>(nb);
  const int CPR = P / VEC;
  const int per_comp = nb * nb * CPR;
  // the fused learned pass: the network's weights and GELU table, staged now
  // so that their loads overlap the bricks'
  unsigned char *const learned_base =
      smem_raw + learned_io_region(bdim, (size_t)nbuf * per_comp * 16);
  // the reciprocals of the features' standard deviations (standardisation
  // by multiplication; within an FP64 rounding of the quotient)
  __shared__ double s_istd[kMlpFeat];
  if constexpr (MODE == kInterpLearned) {
    if ((int)threadIdx.x < kMlpFeat) s_istd[threadIdx.x] = 1.0 / (double)la.norm[kMlpIn + threadIdx.x];
    mlp_stage_fwd(*reinterpret_cast<MlpFwdLds *>(learned_base), la.wbf, la.master);
    float4 *gtab = reinterpret_cast<float4 *>(learned_base + kMlpFwdLdsBytes);
    for (int i = threadIdx.x; i < kGeluTabN; i += bdim)
      gtab[i] = reinterpret_cast<const float4 *>(la.gelu_tab)[i];
  }
  // this lane's chunk slots, the same for the three components (their
  // bricks share the origin), two registers each: the node plane k (wrapped)
  // with flags in the top bits (bit 28: row inside the fluid for u and w,
  // bit 29: for v, bit 30: the chunk crosses the periodic x seam, bit 31:
  // slot in use), and the chunk's element offset (k ny + j) nx + x0 in the
  // u and w arrays; in the v array (ny + 1 rows a plane) it is k nx more.
  // Element offsets fit 32 bits (a component holds fewer than 2^32 nodes).
  constexpr int kSlots = K == 1 ? BrickSlots<T>::value : kSlotsK2;
  constexpr unsigned kFuw = 1u << 28, kFv = 1u << 29, kFseam = 1u << 30, kFuse = 1u << 31;
  unsigned sK[kSlots];
  unsigned sOff[kSlots];
  // Chunks that no stencil of this sphere reads are not loaded (slot marked
  // unused): a stencil reads the nodes within 1.5 node of its marker along
  // each axis, and the markers lie on the sphere of radius R / h about the
  // centre, so a chunk is read only if the box of its nodes -- over the
  // three components' staggerings, widened by 1.5 -- meets that sphere:
  // nearest corner within and farthest corner beyond R / h (with a margin
  // for the rounding of the marker offsets).
  const float c_x = (float)E + (float)fo[0][0], c_y = (float)E + (float)fo[1][0],
              c_z = (float)E + (float)fo[2][0];
  const float rh = (float)(G.R * G.inv_h);
  const float r_in = (rh - 0.01f) * (rh - 0.01f), r_out = (rh + 0.01f) * (rh + 0.01f);
  auto chunk_read = [&](int bx0, int by, int bz) {
    auto axis = [](float c, float lo, float hi, float &near2, float &far2) {
      const float a = lo - c, b = c - hi;
      const float e = fmaxf(fmaxf(a, b), 0.0f), g = fmaxf(fabsf(a), fabsf(b));
      near2 = fmaf(e, e, near2);
      far2 = fmaf(g, g, far2);
    };
    float near2 = 0.0f, far2 = 0.0f;
    axis(c_x, (float)bx0 - 1.5f, (float)(bx0 + VEC - 1) + 2.0f, near2, far2);
    axis(c_y, (float)by - 1.5f, (float)by + 2.0f, near2, far2);
    axis(c_z, (float)bz - 1.5f, (float)bz + 2.0f, near2, far2);
    return near2 <= r_out && far2 >= r_in;
  };
#pragma unroll
  for (int u = 0; u < kSlots; ++u) {
    const int it = threadIdx.x + u * bdim;
    const int row = it / CPR, ch = it - row * CPR;
    const int bz = row / nb, by = row - bz * nb;
    const int j = lo[1] + by;
    const int x0 = lo[0] + ch * VEC;
    const bool read = !PRS_INTERP_CULL || chunk_read(ch * VEC, by, bz);
    sK[u] = (unsigned)wrap_once(lo[2] + bz, G.nz) | (j >= 0 && j <= G.ny - 1 ? kFuw : 0u) |
            (j >= 1 && j <= G.ny - 1 ? kFv : 0u) |
            (x0 < 0 || x0 + VEC > G.nx ? kFseam : 0u) | (it < per_comp && read ? kFuse : 0u);
    sOff[u] = (unsigned)wrap_once(lo[2] + bz, G.nz) * (unsigned)(G.ny * G.nx) +
              (unsigned)(j * G.nx + x0);
  }
  // rows per node plane of component c (v has ny + 1 rows)
  auto nyc = [&](int c) { return c == 1 ? G.ny + 1 : G.ny; };
  // element offset of slot u's chunk in component c's array (the plane
  // index is below 2^24, so k nx takes one 24-bit multiply)
  auto chunk_offset = [&](int c, int u) -> unsigned {
    return c == 1 ? sOff[u] + __umul24(sK[u] & (kFuw - 1u), (unsigned)G.nx)
                  : sOff[u];
  };
  auto load_slot = [&](int c, int u) {
    vec_t v = (vec_t)(T)0;
    const unsigned fl = sK[u];
    if ((fl & kFuse) && (fl & (c == 1 ? kFv : kFuw))) {
      const T *Sp = f_only ? (c == 0 ? b0 : (c == 1 ? b1 : b2)) : (c == 0 ? a0 : (c == 1 ? a1 : a2));
      if (!(fl & kFseam)) {
        __builtin_memcpy(&v, Sp + chunk_offset(c, u), sizeof(vec_t));
      } else {
        // the chunk crosses the seam: elements wrapped one by one
        const int it = threadIdx.x + u * bdim;
        const int row = it / CPR, ch = it - row * CPR;
        const int by = row - (row / nb) * nb;
        const size_t plane = (size_t)(fl & (kFuw - 1u)) * (size_t)nyc(c) * (size_t)G.nx;
        const T *rowp = Sp + plane + (size_t)(long)((lo[1] + by) * G.nx);
        const int x0 = lo[0] + ch * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = rowp[wrap_once(x0 + e, G.nx)];
      }
    }
    return v;
  };
  auto store_slot = [&](int u, vec_t v) {
    const int it = threadIdx.x + u * bdim;
    if (it < per_comp) {
      const int row = it / CPR, ch = it - row * CPR;
      *reinterpret_cast<vec_t *>(brick + row * P + ch * VEC) = v;
    }
  };
  T U[3] = {(T)0, (T)0, (T)0}, U2[3] = {(T)0, (T)0, (T)0};
  // Single-precision MDF passes over f read the recorded I[u-hat] through
  // LDS (loaded while the last stencils run) when the bricks are double
  // buffered.
  constexpr bool kU0Lds = sizeof(T) == 4 && MODE == kInterpMDF && PRS_INTERP_DMA != 0;
  const bool u0_in_lds =
      kU0Lds && f_only && u0 != nullptr && nbuf == 2 && per_comp <= kSlots * bdim;
  T u0_val[3] = {(T)0, (T)0, (T)0};
  // the field of component c that this pass interpolates
  auto field = [&](int c) {
    return f_only ? (c == 0 ? b0 : (c == 1 ? b1 : b2)) : (c == 0 ? a0 : (c == 1 ? a1 : a2));
  };
  // Component c's brick in buf, straight from memory (kDma): each chunk
  // inside the fluid and clear of the x seam goes into LDS without passing
  // through registers (global_load_lds_dwordx4: lane i of a wave writes the
  // 16 bytes at LDS base + 16 i, and chunk it = slot u * blockDim + wave * 64
  // + lane sits at byte 16 it of the brick); the other chunks are stored by
  // their lanes (zeros, or the wrapped elements at the seam).  Completes at
  // the caller's wait_loads.
  // The lanes' own stores come first (the seam chunks wait for their loads,
  // which would otherwise also wait for the direct loads in flight), then
  // the direct loads.
  auto dma_component = [&](int c, T *buf) {
    const T *Sp = field(c);
    const unsigned in_flag = c == 1 ? kFv : kFuw;
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      const unsigned fl = sK[u];
      if ((fl & kFuse) && !(fl & in_flag))
        *reinterpret_cast<vec_t *>(buf + (threadIdx.x + u * bdim) * VEC) = (vec_t)(T)0;
    }
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      const unsigned fl = sK[u];
      if ((fl & kFuse) && (fl & in_flag) && (fl & kFseam))
        *reinterpret_cast<vec_t *>(buf + (threadIdx.x + u * bdim) * VEC) = load_slot(c, u);
    }
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      const unsigned fl = sK[u];
      if ((fl & kFuse) && (fl & in_flag) && !(fl & kFseam)) {
        lds_load16(Sp + chunk_offset(c, u), buf + (u * bdim + wave_base) * VEC);
      }
    }
  };
  // Component c interpolated from its brick: the three axis stencils, then
  // the 27-point sum contracted separably (x, then y, then z).  Selects
  // rather than indexing by c keep the arrays in registers.
  auto stencil_one = [&](int c, const T *buf, const T mh[3], const T ml[3], T Uo[3]) {
    T wx[3], wy[3], wz[3];
    const T f0 = c == 0 ? fo[0][0] : fo[0][1];   // fo[0][stag(c, 0)]
    const T f1 = c == 1 ? fo[1][0] : fo[1][1];   // fo[1][stag(c, 1)]
    const T f2 = c == 2 ? fo[2][0] : fo[2][1];   // fo[2][stag(c, 2)]
    const int bx = min(max(stencil_axis<T>(f0, mh[0], ml[0], wx) - 1 + E, 0), nb - 3);
    const int by = min(max(stencil_axis<T>(f1, mh[1], ml[1], wy) - 1 + E, 0), nb - 3);
    const int bz = min(max(stencil_axis<T>(f2, mh[2], ml[2], wz) - 1 + E, 0), nb - 3);
    const T *bk = buf + ((bz * nb + by) * P + bx);
    T zsum = 0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      T ysum = 0;
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        const T *row = bk + (kk * nb + jj) * P;
        const T xsum = fma(row[2], wx[2], fma(row[1], wx[1], row[0] * wx[0]));
        ysum = fma(wy[jj], xsum, ysum);
      }
      zsum = fma(wz[kk], ysum, zsum);
    }
    Uo[0] = c == 0 ? zsum : Uo[0];
    Uo[1] = c == 1 ? zsum : Uo[1];
    Uo[2] = c == 2 ? zsum : Uo[2];
  };
  auto stencil_component = [&](int c, const T *buf) {
    if (active) stencil_one(c, buf, mhi, mlo, U);
    if (K == 2 && active2) stencil_one(c, buf, mhi2, mlo2, U2);
  };
  // When the lane's slots cover the brick: direct loads into two LDS
  // buffers, the next component's brick in flight while the current one's
  // stencils run (without direct loads, the next component's chunks wait in
  // registers meanwhile).  With few markers per sphere each component is
  // loaded in rounds of blockDim.
  const bool pipe = per_comp <= kSlots * bdim;
  constexpr bool kDma = PRS_INTERP_DMA != 0;
  if (pipe && kDma && nbuf == 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      __syncthreads();   // the previous component's brick is no longer read
      dma_component(c, brick);
      wait_loads();
      __syncthreads();
      stencil_component(c, brick);
    }
  } else if (pipe && kDma) {
    T *buf[2] = {brick, brick + per_comp * VEC};
    dma_component(0, buf[0]);
    wait_loads();
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // buf[(c + 1) & 1] was last read by component c - 1, before the
      // barrier that ended the previous round
      if (c < 2) {
        dma_component(c + 1, buf[(c + 1) & 1]);
      } else if (kU0Lds && u0_in_lds) {
        // the recorded I[u-hat] of this lane's marker, into the free buffer
        // while the last component's stencils run
        const size_t M = N * G.nl, m = (size_t)p * G.nl + l;
        if (active)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
            lds_load4(u0 + cc * M + m, buf[1] + cc * bdim + wave_base);
      }
      stencil_component(c, buf[c & 1]);
      if (c < 2) {
        wait_loads();
        __syncthreads();
      }
    }
    if (kU0Lds && u0_in_lds) {
      wait_loads();   // each lane reads the values its own wave loaded
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) u0_val[cc] = buf[1][cc * bdim + (int)threadIdx.x];
    }
  } else {
    vec_t nxt[kSlots];
    if (pipe) {
#pragma unroll
      for (int u = 0; u < kSlots; ++u) nxt[u] = load_slot(0, u);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      __syncthreads();   // the previous component's brick is no longer read
      if (pipe) {
#pragma unroll
        for (int u = 0; u < kSlots; ++u) store_slot(u, nxt[u]);
        if (c < 2) {
#pragma unroll
          for (int u = 0; u < kSlots; ++u) nxt[u] = load_slot(c + 1, u);
        }
      } else {
        const T *Sp = field(c);
        for (int it = threadIdx.x; it < per_comp; it += bdim) {
          const int row = it / CPR, ch = it - row * CPR;
          const int bz = row / nb, by = row - bz * nb;
          const int j = lo[1] + by, x0 = lo[0] + ch * VEC;
          vec_t v = (vec_t)(T)0;
          if (j >= (c == 1 ? 1 : 0) && j <= G.ny - 1) {
            const int k = wrap_once(lo[2] + bz, G.nz);
            const T *rowp = Sp + ((size_t)k * (size_t)nyc(c) + (size_t)j) * (size_t)G.nx;
            if (x0 >= 0 && x0 + VEC <= G.nx) {
              __builtin_memcpy(&v, rowp + x0, sizeof(vec_t));
            } else {
#pragma unroll
              for (int e = 0; e < VEC; ++e) v[e] = rowp[wrap_once(x0 + e, G.nx)];
            }
          }
          *reinterpret_cast<vec_t *>(brick + row * P + ch * VEC) = v;
        }
      }
      __syncthreads();
      stencil_component(c, brick);
    }
  }

  // the sphere's velocities and the marker's lever arm and rigid velocity
  double up[3] = {0, 0, 0}, wp[3] = {0, 0, 0};
  if (MODE == kInterpPlain) {
    if (out2)
      for (int a = 0; a < 3; ++a) {
        up[a] = us[3 * p + a];
        wp[a] = ws[3 * p + a];
      }
  } else {
    for (int a = 0; a < 3; ++a) {
      up[a] = us[a * N + p];
      wp[a] = ws[a * N + p];
    }
  }
  // the lever arm R t_l: in single precision from the marker offset in node
  // units already in registers, h (m_hi + m_lo), within a few FP64
  // roundings of R t_l (double precision, and the modes with the normal
  // among their features, read the template)
  double rl[3] = {0, 0, 0};
  if (active) {
    if (sizeof(T) == 8 || MODE == kInterpFeat || MODE == kInterpLearned)
      for (int a = 0; a < 3; ++a) rl[a] = G.R * templ[3 * l + a];
    else
      for (int a = 0; a < 3; ++a) rl[a] = G.h * ((double)mhi[a] + (double)mlo[a]);
  }
  const double Ud[3] = {up[0] + (wp[1] * rl[2] - wp[2] * rl[1]),
                        up[1] + (wp[2] * rl[0] - wp[0] * rl[2]),
                        up[2] + (wp[0] * rl[1] - wp[1] * rl[0])};
  double rl2[3] = {0, 0, 0};
  if (K == 2 && active2)
    for (int a = 0; a < 3; ++a) rl2[a] = G.h * ((double)mhi2[a] + (double)mlo2[a]);
  const double Ud2[3] = {up[0] + (wp[1] * rl2[2] - wp[2] * rl2[1]),
                         up[1] + (wp[2] * rl2[0] - wp[0] * rl2[2]),
                         up[2] + (wp[0] * rl2[1] - wp[1] * rl2[0])};

  if (MODE != kInterpPlain && active && u0) {
    const size_t M = N * G.nl, m = (size_t)p * G.nl + l;
    if (kU0Lds && u0_in_lds)
      for (int c = 0; c < 3; ++c) U[c] = u0_val[c] + tadt * U[c];
    else if (f_only)
      for (int c = 0; c < 3; ++c) U[c] = u0[c * M + m] + tadt * U[c];
    else
      for (int c = 0; c < 3; ++c) u0[c * M + m] = U[c];
  }
  if (K == 2 && active2 && u0) {
    const size_t M = N * G.nl, m2 = (size_t)p * G.nl + l2;
    if (f_only)
      for (int c = 0; c < 3; ++c) U2[c] = u0[c * M + m2] + tadt * U2[c];
    else
      for (int c = 0; c < 3; ++c) u0[c * M + m2] = U2[c];
  }

  if (MODE == kInterpPlain) {
    if (active) {
      const size_t m = (size_t)p * G.nl + l;
      for (int c = 0; c < 3; ++c) out[3 * m + c] = U[c];
      if (out2)
        for (int c = 0; c < 3; ++c) out2[3 * m + c] = (T)Ud[c];
    }
    return;
  }
  Red red;
  red_zero(red);
  unsigned vm = 0u;   // largest |value| this lane writes to out (MDF, learned), abs_bits
  // features of the learned warm start: slip, normal, u_p, R omega_p
  double featd[kMlpFeat];
  if (MODE == kInterpFeat || MODE == kInterpLearned) {
    for (int c = 0; c < 3; ++c) {
      featd[c] = Ud[c] - (double)U[c];
      featd[3 + c] = active ? templ[3 * l + c] : 0.0;
      featd[6 + c] = up[c];
      featd[9 + c] = G.R * wp[c];
    }
  }
  if (MODE == kInterpFeat && active) {
    float *dst = la.feat + ((size_t)la.perm[p] * G.nl + l) * kMlpIn;
    for (int k = 0; k < kMlpFeat; ++k) dst[k] = (float)featd[k];
    for (int k = kMlpFeat; k < kMlpIn; ++k) dst[k] = 0.f;
  }
  if constexpr (MODE == kInterpLearned) {
    // the network on the matrix cores: each wave evaluates its 64 markers as
    // four 16-marker tiles.  The brick's LDS is reused for the weights, the
    // standardised inputs (BF16) and the predictions (FP32).
    const MlpFwdLds &L = *reinterpret_cast<const MlpFwdLds *>(learned_base);
    const float4 *gtab = reinterpret_cast<const float4 *>(learned_base + kMlpFwdLdsBytes);
    // input fragments, tile-major: entry [tile][16 q + r] holds features
    // 4q .. 4q+3 of marker r of the tile (tile = 16 consecutive lanes)
    bf16x4 *fl = reinterpret_cast<bf16x4 *>(smem_raw);
    float *yl = reinterpret_cast<float *>(fl + bdim * (kMlpIn / 4));
    __syncthreads();   // the bricks are no longer read
    {
      const int tile = threadIdx.x >> 4, r = threadIdx.x & 15;
      for (int q = 0; q < kMlpIn / 4; ++q) {
        float v[4];
        for (int j = 0; j < 4; ++j) {
          const int k = 4 * q + j;
          v[j] = (active && k < kMlpFeat)
                     ? (float)((featd[k] - (double)la.norm[k]) * s_istd[k])
                     : 0.f;
        }
        fl[tile * 64 + 16 * q + r] = pack4(v[0], v[1], v[2], v[3]);
      }
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    for (int t = 0; t < 4; ++t) {
      const int tile = 4 * wave + t;
      MlpFwd s;
      mlp_forward_tile(L, fl[tile * 64 + lane], s, GeluTable{gtab});
      if (q == 0)
        for (int i = 0; i < kMlpUsed; ++i) yl[(16 * tile + r) * kMlpUsed + i] = s.y[i];
    }
    __syncthreads();
    if (active) {
      // de-standardise in FP64: F0 = (y std + mean) / (alpha dt)
      const size_t M = N * G.nl, m = (size_t)p * G.nl + l;
      double d[3];
      for (int c = 0; c < 3; ++c) {
        const double y = (double)yl[threadIdx.x * kMlpUsed + c];
        const T f0 = (T)((y * (double)la.norm[2 * kMlpIn + kMlpUsed + c] +
                          (double)la.norm[2 * kMlpIn + c]) * inv_adt);
        out[c * M + m] = f0;
        vm = max(vm, abs_bits((float)f0));
        d[c] = (double)f0;
      }
      red_set_ft(red, rl, d);
    }
  }
  if (active) {
    if (MODE == kInterpMDF) {
      const size_t M = N * G.nl, m = (size_t)p * G.nl + l;
      double d[3];
      for (int c = 0; c < 3; ++c) {
        const T res = (T)Ud[c] - U[c];
        const T corr = res * inv_tadt;
        out[c * M + m] = corr;
        vm = max(vm, abs_bits((float)corr));
        d[c] = (double)corr;
        red.v[kColSlip] += (double)res * (double)res;
      }
      red_set_ft(red, rl, d);
    } else {
      for (int c = 0; c < 3; ++c) {
        const double z = Ud[c] - (double)U[c];
        red.v[kColSlip0] += z * z;
      }
    }
  }
  if (K == 2 && active2) {
    // the lane's second marker (MDF), added to the first one's terms
    const size_t M = N * G.nl, m2 = (size_t)p * G.nl + l2;
    double d[3];
    for (int c = 0; c < 3; ++c) {
      const T res = (T)Ud2[c] - U2[c];
      const T corr = res * inv_tadt;
      out[c * M + m2] = corr;
      vm = max(vm, abs_bits((float)corr));
      d[c] = (double)corr;
      red.v[kColSlip] += (double)res * (double)res;
    }
    red_add_ft(red, rl2, d);
  }
  __shared__ float s_vmax[16];
  constexpr bool kForce = MODE == kInterpMDF || MODE == kInterpLearned;
  if (kForce) {
    vm = wave_max_last(vm);
    if ((threadIdx.x & 63) == 63) s_vmax[threadIdx.x >> 6] = __uint_as_float(vm);
  }
  constexpr unsigned kMask = (kForce ? 0x3Fu : 0u) |
                             (MODE == kInterpMDF ? 1u << kColSlip : 1u << kColSlip0);
  double rs, rc;
  block_reduce<kMask>(red, rs, rc);   // (its barrier also publishes s_vmax)
  const int t = threadIdx.x;
  if (kForce && t == 0 && vmax_out) {
    float m = 0.f;
    for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) m = nan_max(m, s_vmax[wv]);
    vmax_out[p] = m;
  }
  if (kForce && t < 6) {
    ft_part[(2 * t) * N + p] = rs;
    ft_part[(2 * t + 1) * N + p] = rc;
  }
  if (MODE == kInterpMDF && t == kColSlip) slip_part[p] = rs;
  if (MODE != kInterpMDF && t == kColSlip0) slip_part[N + p] = rs;
}

// Launch k_interp with the brick edge as a compile-time constant when it is
// one of the common sizes (D/h = 10 -> 14, D/h = 16 -> 20).
template <typename T, int MODE>
hipError_t launch_interp_any(hipStream_t s, const Geom &G, const Scratch &S, const T *a0,
                             const T *a1, const T *a2, const T *b0, const T *b1, const T *b2,
                             double adt, const double *xs, const double *us, const double *ws,
                             int n, T *out, T *out2, double *slip_part, double *ft_part,
                             const LearnArgs &la = LearnArgs{}, float *vmax_out = nullptr,
                             T *u0 = nullptr) {
  if (n == 0) return hipSuccess;
  const int nb = brick_edge(G.R, G.h);
  const dim3 grid(xcd_grid(n)), block(block_for(G.nl));
  const int nbuf = MODE == kInterpLearned ? 1 : interp_brick_buffers(nb, sizeof(T));
  size_t lds = brick_bytes(nb, sizeof(T)) * nbuf;
  if (MODE == kInterpLearned) lds = learned_lds_bytes(G.nl, nb, sizeof(T));
  // the marker offsets in lane order
  const T *tm = (const T *)(sizeof(T) == 4 ? (const void *)S.tm32_lane : (const void *)S.tm64_lane);
  const double inv_adt = adt != 0.0 ? 1.0 / adt : 0.0;
#define PRS_LAUNCH_INTERP(NBV)                                                                 \
  hipLaunchKernelGGL((k_interp<T, MODE, NBV>), grid, block, lds, s, G, S.templ, tm, a0, a1, a2, \
                     b0, b1, b2, adt, inv_adt, xs, us, ws, n, nb, out, out2, slip_part,        \
                     ft_part, S.lane_order, la, vmax_out, u0, nbuf)
  if (nb == 14)
    PRS_LAUNCH_INTERP(14);
  else if (nb == 20)
    PRS_LAUNCH_INTERP(20);
  else
    PRS_LAUNCH_INTERP(0);
#undef PRS_LAUNCH_INTERP
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interp_plain(hipStream_t s, const Geom &G, const Scratch &S, const T *gu,
                               const T *gv, const T *gw, const double *x, const double *up,
                               const double *om, int n, T *U, T *Ud) {
  return launch_interp_any<T, kInterpPlain>(s, G, S, gu, gv, gw, nullptr, nullptr, nullptr, 0.0,
                                            x, up, om, n, U, Ud, nullptr, nullptr);
}

template <typename T>
hipError_t launch_interp_mdf(hipStream_t s, const Geom &G, const Scratch &S, const T *uh[3],
                             const T *f[3], int n, double adt, int den_only) {
  if (den_only)
    return launch_interp_any<T, kInterpDen>(s, G, S, uh[0], uh[1], uh[2], nullptr, nullptr,
                                            nullptr, adt, S.xs[0], S.us[0], S.ws[0], n, nullptr,
                                            nullptr, S.slip_part, nullptr, LearnArgs{}, nullptr,
                                            (T *)S.u0);
  const int nb = brick_edge(G.R, G.h);
  if (PRS_INTERP_K2 && sizeof(T) == 4 && n > 0 && (nb == 14 || nb == 20)) {
    // two markers a lane, one brick buffer
    const int block = block_for((G.nl + 1) / 2);
    const int P = brick_pitch_c<T>(nb);
    if ((size_t)nb * nb * (P / (16 / sizeof(T))) <= (size_t)kSlotsK2 * block) {
      const size_t lds = brick_bytes(nb, sizeof(T));
      const T *tm = (const T *)S.tm32_lane;
      const double inv_adt = adt != 0.0 ? 1.0 / adt : 0.0;
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(xcd_grid(n)), dim3(block), lds, s, G, S.templ, tm, uh[0],
                           uh[1], uh[2], f[0], f[1], f[2], adt, inv_adt, S.xs[0], S.us[0],
                           S.ws[0], n, nb, (T *)S.dF, (T *)nullptr, S.slip_part, S.ft_part,
                           S.lane_order, LearnArgs{}, S.vmax, (T *)S.u0, 1);
        return hipGetLastError();
      };
      if constexpr (sizeof(T) == 4)
        return nb == 14 ? go(k_interp<float, kInterpMDF, 14, 2>)
                        : go(k_interp<float, kInterpMDF, 20, 2>);
    }
  }
  return launch_interp_any<T, kInterpMDF>(s, G, S, uh[0], uh[1], uh[2], f[0], f[1], f[2], adt,
                                          S.xs[0], S.us[0], S.ws[0], n, (T *)S.dF, nullptr,
                                          S.slip_part, S.ft_part, LearnArgs{}, S.vmax,
                                          (T *)S.u0);
}

template <typename T>
hipError_t launch_interp_feat(hipStream_t s, const Geom &G, const Scratch &S, const T *uh[3], int n,
                              float *feat) {
  LearnArgs la{};
  la.perm = S.perm;
  la.feat = feat;
  return launch_interp_any<T, kInterpFeat>(s, G, S, uh[0], uh[1], uh[2], nullptr, nullptr,
                                           nullptr, 0.0, S.xs[0], S.us[0], S.ws[0], n, nullptr,
                                           nullptr, S.slip_part, nullptr, la);
}

template <typename T>
hipError_t launch_interp_learned(hipStream_t s, const Geom &G, const Scratch &S, const T *uh[3],
                                 int n, double adt, const LearnArgs &la) {
  return launch_interp_any<T, kInterpLearned>(s, G, S, uh[0], uh[1], uh[2], nullptr, nullptr,
                                              nullptr, adt, S.xs[0], S.us[0], S.ws[0], n,
                                              (T *)S.dF, nullptr, S.slip_part, S.ft_part, la,
                                              S.vmax, (T *)S.u0);
}

// target[caller marker][c] += adt * dF[c][sorted marker]
template <typename T>
__global__ void k_accum_target(const T *__restrict__ dF, const int *__restrict__ perm, int n,
                               int nl, double adt, float *__restrict__ target) {
  const size_t M = (size_t)n * nl;
  const size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int p = (int)(m / nl), l = (int)(m - (size_t)p * nl);
  const size_t dst = ((size_t)perm[p] * nl + l) * 3;
  for (int c = 0; c < 3; ++c) target[dst + c] += (float)(adt * (double)dF[c * M + m]);
}

template <typename T>
hipError_t launch_accum_target(hipStream_t s, const Geom &G, const Scratch &S, int n, double adt,
                               float *target) {
  const size_t M = (size_t)n * G.nl;
  if (M == 0) return hipSuccess;
  hipLaunchKernelGGL(k_accum_target<T>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s,
                     (const T *)S.dF, S.perm, n, G.nl, adt, target);
  return hipGetLastError();
}

template hipError_t launch_interp_plain<float>(hipStream_t, const Geom &, const Scratch &,
                                               const float *, const float *, const float *,
                                               const double *, const double *, const double *,
                                               int, float *, float *);
template hipError_t launch_interp_plain<double>(hipStream_t, const Geom &, const Scratch &,
                                                const double *, const double *, const double *,
                                                const double *, const double *, const double *,
                                                int, double *, double *);
template hipError_t launch_interp_mdf<float>(hipStream_t, const Geom &, const Scratch &,
                                             const float *[3], const float *[3], int, double, int);
template hipError_t launch_interp_mdf<double>(hipStream_t, const Geom &, const Scratch &,
                                              const double *[3], const double *[3], int, double,
                                              int);
template hipError_t launch_interp_feat<float>(hipStream_t, const Geom &, const Scratch &,
                                              const float *[3], int, float *);
template hipError_t launch_interp_feat<double>(hipStream_t, const Geom &, const Scratch &,
                                               const double *[3], int, float *);
template hipError_t launch_interp_learned<float>(hipStream_t, const Geom &, const Scratch &,
                                                 const float *[3], int, double,
                                                 const LearnArgs &);
template hipError_t launch_interp_learned<double>(hipStream_t, const Geom &, const Scratch &,
                                                  const double *[3], int, double,
                                                  const LearnArgs &);
template hipError_t launch_accum_target<float>(hipStream_t, const Geom &, const Scratch &, int,
                                               double, float *);
template hipError_t launch_accum_target<double>(hipStream_t, const Geom &, const Scratch &, int,
                                                double, float *);

// ---------------------------------------------------------------------------
// spreading by grid tiles
// ---------------------------------------------------------------------------
// Tile shapes (nodes per axis) and workgroup size; compile-time tuning knobs.
#ifndef PRS_TILE_F32
#define PRS_TILE_F32 16, 8, 16
#endif
#ifndef PRS_TILE_F64
#define PRS_TILE_F64 16, 8, 8
#endif
#ifndef PRS_TILE_THREADS
#define PRS_TILE_THREADS 512
#endif

template <int TX_, int TY_, int TZ_>
struct Shape3 {
  static constexpr int X = TX_, Y = TY_, Z = TZ_;
};
template <typename T>
struct TileShape;
template <>
struct TileShape<float> : Shape3<PRS_TILE_F32> {};
template <>
struct TileShape<double> : Shape3<PRS_TILE_F64> {};

// Tile accumulators in LDS.  Double-precision fields: double, with the LDS
// double-precision atomic add.  Single-precision fields: 32-bit fixed point
// with a per-tile unit (block floating point), added with the LDS integer
// atomic -- on gfx950 it sustains about 1.5x the double-precision and 5x
// the single-precision floating-point atomic add in this access pattern.
// The unit is B / 2^30 with B a bound on any node's sum: wsum_bound (the
// largest weight sum one sphere's markers can give a node) times
// dV / h^3 times the sum over the tile's candidate spheres of their largest
// |marker value|, so no sum can overflow; each addend is rounded to the unit
// (about 22 bits relative to the tile's largest possible value, like FP32).
template <typename T>
struct TileAcc {
  using type = T;
};
template <>
struct TileAcc<float> {
  using type = int;
};

// Accumulator layout of a tile: per component TZ planes of TY x-rows, each
// row TX + 2 kGuard entries long.  A marker's component is accumulated when
// its 3-node stencil meets the tile along every axis; its rows outside the
// tile in y or z are skipped (one test per row), and along x the row carries
// a guard band of two nodes on each side, so the three adds of a row run
// without tests (the band's sums are discarded).  Only the tile's own rows
// take LDS, which keeps three tiles resident per compute unit.
constexpr int kGuard = 2;
// Padding of the accumulator's rows and planes in entries: the LDS bank of
// an entry follows its offset, and unpadded planes (160 entries in FP32)
// put the same node of different planes in one bank, so lanes adding at
// the same (x, y) of different planes conflict.  Eight entries a plane took
// the single-precision spreading pass from 15.8 to 14.5 ms at C3 (padding
// the rows instead, or the planes by 2 to 16 entries, gave 14.5 to 14.9 ms;
// 36 entries left two tiles per compute unit).
#ifndef PRS_ACC_ROW_PAD
#define PRS_ACC_ROW_PAD 0
#endif
#ifndef PRS_ACC_PLANE_PAD
#define PRS_ACC_PLANE_PAD 8
#endif
template <int TX, int TY, int TZ>
struct AccLayout {
  static constexpr int PX = TX + 2 * kGuard + PRS_ACC_ROW_PAD;   // row stride
  static constexpr int PZ = PX * TY + PRS_ACC_PLANE_PAD;         // plane stride
  static constexpr int NODES = PZ * TZ;   // per component
};

constexpr int kTileCand = 256;     // spheres gathered by one tile
constexpr int kTileThreads = PRS_TILE_THREADS;
constexpr int kTileList = 1024;    // culled markers buffered before accumulation
// Rounds of the block over a tile's recorded markers (a record holds at
// most kTileRecord entries: candidates, then markers).
constexpr int kReplayRounds = (kTileRecord + PRS_TILE_THREADS - 1) / PRS_TILE_THREADS;
static_assert(kTileThreads >= kTileCand && kTileCand % 64 == 0, "one scan lane per candidate");
static_assert(kTileList >= 2 * kTileThreads, "a round must fit after a flush check");
static_assert(kMaxMarkers <= 1024, "list code: candidate << 10 | marker");

// A candidate sphere of a tile: the offset of its centre node from the tile's
// first node plus the guard (periodic axes by minimum image about the tile
// centre), and its staggered fractions (sphere_axis).
template <typename T>
struct TileCand {
  int d[3];
  T fo[3][2];
};

template <typename T, int TX, int TY, int TZ>
__device__ inline void tile_cand(const Geom &G, double x, double y, double z, int i0, int j0,
                                 int k0, int d[3], T fo[3][2]) {
  int I[3];
  sphere_axis<T>(x, G.inv_h, I[0], fo[0]);
  sphere_axis<T>(y, G.inv_h, I[1], fo[1]);
  sphere_axis<T>(z, G.inv_h, I[2], fo[2]);
  const int n[3] = {G.nx, 0, G.nz}, t0[3] = {i0, j0, k0}, tl[3] = {TX, TY, TZ};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int dd = I[a] - t0[a];
    if (a != 1) {
      // minimum image about the tile centre
      const int rel2 = 2 * dd - tl[a];
      if (rel2 >= n[a]) dd -= n[a];
      else if (rel2 < -n[a]) dd += n[a];
    }
    d[a] = dd + kGuard;
  }
}

// Fixed-point rounding of one contribution: floor(x + 1/2) in one
// instruction (the sums stay exact integers, so their order does not matter;
// ties round up rather than to even).
__device__ inline int fixed_round(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Clears the tile accumulators with 16-byte stores.
template <typename A_t, int COUNT>
__device__ inline void acc_clear(A_t *acc) {
  static_assert((COUNT * sizeof(A_t)) % 16 == 0, "accumulators in 16-byte chunks");
  constexpr int kChunks = COUNT * sizeof(A_t) / 16;
  uint4 *p = reinterpret_cast<uint4 *>(acc);
  for (int q = threadIdx.x; q < kChunks; q += blockDim.x) p[q] = make_uint4(0, 0, 0, 0);
}

// One marker's contribution to a tile: the six axis stencils, and for each
// component whose stencil meets the tile, its 27 adds of
// value * weight * dV / h^3 into the guard-banded accumulator.
// scale: dV / h^3 (floating-point accumulators) or dV / h^3 / unit (fixed point).
// The marker's three values (marker l of sorted sphere k).
template <typename T, int SRC>
__device__ inline void marker_values(const Geom &G, const T *__restrict__ src,
                                     const int *__restrict__ perm, int k, int l, size_t M, T v[3]) {
  if (SRC == 0) {
    const size_t m = (size_t)k * G.nl + l;
    for (int c = 0; c < 3; ++c) v[c] = src[c * M + m];
  } else {
    const size_t m = (size_t)perm[k] * G.nl + l;
    for (int c = 0; c < 3; ++c) v[c] = src[3 * m + c];
  }
}

template <typename T, int SRC, int TX, int TY, int TZ>
__device__ inline void spread_visit(const Geom &G, const int d[3], const T fo[3][2],
                                    const T *__restrict__ tm, const T *__restrict__ src,
                                    const int *__restrict__ perm, int k, int l, size_t M, T scale,
                                    typename TileAcc<T>::type *acc);

// The same with the marker's values already loaded.
template <typename T, int TX, int TY, int TZ>
__device__ inline void spread_visit_v(const Geom &G, const int d[3], const T fo[3][2],
                                      const T *__restrict__ tm, const T v[3], int l, T scale,
                                      typename TileAcc<T>::type *acc) {
  using A_t = typename TileAcc<T>::type;
  constexpr int PX = AccLayout<TX, TY, TZ>::PX, PZ = AccLayout<TX, TY, TZ>::PZ,
                NODES = AccLayout<TX, TY, TZ>::NODES;
  T mhi[3], mlo[3];
  MarkerOffset<T>::load(tm, l, mhi, mlo);
  int b[3][2];
  T w[3][2][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < 2; ++o) b[a][o] = d[a] + stencil_axis<T>(fo[a][o], mhi[a], mlo[a], w[a][o]) - 1;
  constexpr unsigned lim[3] = {TX + 1, TY + 1, TZ + 1};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int ox = stag(c, 0), oy = stag(c, 1), oz = stag(c, 2);
    const int bx = b[0][ox], by = b[1][oy], bz = b[2][oz];
    // nodes b .. b + 2 (guard-banded index) meet the tile's b in [0, T + 1]
    if (!((unsigned)bx <= lim[0] && (unsigned)by <= lim[1] && (unsigned)bz <= lim[2])) continue;
    // the stencil's first row and plane in tile coordinates (-2 .. T - 1)
    const int y0 = by - kGuard, z0 = bz - kGuard;
    // the stencil's first row (it may lie outside the tile; only rows inside
    // are written): one multiply per component, the rows at constant offsets
    A_t *A0 = acc + c * NODES + bx + (z0 * PZ + y0 * PX);
    using W_t = typename std::conditional<std::is_integral<A_t>::value, T, A_t>::type;
    const W_t val = (W_t)(v[c] * scale);
    const T *wx = w[0][ox], *wy = w[1][oy], *wz = w[2][oz];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      if ((unsigned)(z0 + kk) >= (unsigned)TZ) continue;
      const W_t vz = val * (W_t)wz[kk];
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        if ((unsigned)(y0 + jj) >= (unsigned)TY) continue;
        const W_t vzy = vz * (W_t)wy[jj];
        A_t *row = A0 + (kk * PZ + jj * PX);   // constant offsets from A0
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          if constexpr (std::is_integral<A_t>::value)
            atomicAdd(row + ii, fixed_round(vzy * (W_t)wx[ii]));
          else
            atomicAdd(row + ii, vzy * (W_t)wx[ii]);
        }
      }
    }
  }
}

template <typename T, int SRC, int TX, int TY, int TZ>
__device__ inline void spread_visit(const Geom &G, const int d[3], const T fo[3][2],
                                    const T *__restrict__ tm, const T *__restrict__ src,
                                    const int *__restrict__ perm, int k, int l, size_t M, T scale,
                                    typename TileAcc<T>::type *acc) {
  T v[3];
  marker_values<T, SRC>(G, src, perm, k, l, M, v);
  spread_visit_v<T, TX, TY, TZ>(G, d, fo, tm, v, l, scale, acc);
}

// Accumulator unit of a tile: fixed point (single-precision fields) takes
// the smallest power of two >= B / 2^30 for the bound B on any node sum (a
// power of two keeps the unit, and so the sums, independent of the order in
// which B was summed); a non-finite bound poisons the tile.  Floating-point
// accumulators (double-precision fields) use dV / h^3 as the scale.
template <typename T, bool kFixed>
__device__ inline void tile_unit(double bound, double dvh, double &unit, bool &poison, T &scale) {
  unit = 1.0;
  poison = false;
  scale = (T)dvh;
  if (!kFixed) return;
  if (!(bound < INFINITY)) {
    poison = true;
    scale = (T)0;
    return;
  }
  if (!(bound > 0.0)) {
    scale = (T)0;   // every marker value is zero
    return;
  }
  int ex;
  frexp(bound * (1.0 / 1073741824.0), &ex);
  unit = ldexp(1.0, ex);
  scale = (T)(dvh / unit);
}

// Write-back of a tile: each owned node with a non-zero accumulator is added
// to the field once (plain read-modify-write; the tile owns its nodes), by
// x-rows: TX lanes per row, rows (component, z, y).  The wall faces of v
// (rows j = 0 and j = ny) take no part: they are skipped, or stored as zero
// when the pass overwrites.  A poisoned tile makes every node NaN and raises
// the status flag.
// Rows of f a lane reads before writing them back (loads in flight at once).
#ifndef PRS_FLUSH_BATCH
#define PRS_FLUSH_BATCH 12
#endif

// acc == nullptr: a tile with nothing to add (only written when overwriting).
// overwrite: every node of the tile is stored (zero where acc is), f is not
// read; otherwise only nonzero sums are added.
template <typename T, typename A_t, int TX, int TY, int TZ>
__device__ inline void tile_flush(const Geom &G, const A_t *acc, int i0, int j0, int k0,
                                  double unit, bool poison, bool overwrite, T *f0, T *f1, T *f2,
                                  uint32_t *status) {
  constexpr bool kFixed = std::is_integral<A_t>::value;
  constexpr int PX = AccLayout<TX, TY, TZ>::PX, PZ = AccLayout<TX, TY, TZ>::PZ,
                NODES = AccLayout<TX, TY, TZ>::NODES;
  static_assert((TX & (TX - 1)) == 0 && kTileThreads % TX == 0, "x-rows of the tile");
  constexpr int kRows = 3 * TZ * TY, kStep = kTileThreads / TX;
  constexpr int kPer = (kRows + kStep - 1) / kStep;   // rows per lane
  static_assert((TZ * TY) % kStep == 0 && kStep % TY == 0,
                "a round of rows stays within one component and starts a plane");
  // Row q of this lane: component c = q kStep / (TZ TY) and plane
  // lz0 + dz(q) are the same for every lane of the round, the y-row ly and
  // the first plane lz0 are the lane's own; so each row's field index is the
  // lane's base for its component plus a uniform multiple of the plane size.
  const int lx = threadIdx.x & (TX - 1), i = i0 + lx;
  const int r0 = threadIdx.x / TX, ly = r0 % TY, lz0 = r0 / TY;
  const int j = j0 + ly;
  const bool lane_ok = i < G.nx;
  const size_t base_uw = ((size_t)(k0 + lz0) * G.ny + j) * G.nx + i;
  const size_t base_v = ((size_t)(k0 + lz0) * (G.ny + 1) + j) * G.nx + i;
  auto row_of = [&](int q, int &c, int &dz) {
    c = (q * kStep) / (TZ * TY);
    dz = ((q * kStep) % (TZ * TY)) / TY;
  };
  // the lane's q-th row: false where it has nothing to write
  auto node = [&](int q, T *&Fp, size_t &g, A_t &a, bool &wall) {
    int c, dz;
    row_of(q, c, dz);
    const int nyc = G.ny + (c == 1 ? 1 : 0);
    const int lz = lz0 + dz;
    if (!lane_ok || j >= nyc || k0 + lz >= G.nz) return false;
    wall = c == 1 && (j == 0 || j == G.ny);
    a = (acc && !wall) ? acc[c * NODES + lz * PZ + ly * PX + lx + kGuard] : (A_t)0;
    if (wall ? !overwrite : (a == (A_t)0 && !poison && !overwrite)) return false;
    // the row's plane offset is the same for every lane (c and dz depend on
    // q only): it goes into the pointer, the lane's own base into the index
    g = c == 1 ? base_v : base_uw;
    Fp = (c == 0 ? f0 : (c == 1 ? f1 : f2)) + (size_t)dz * ((size_t)nyc * (size_t)G.nx);
    return true;
  };
  // the reads of f of a batch of the lane's rows first, so they are in
  // flight together, then their writes (each node belongs to one lane of
  // one tile)
  constexpr int kBatch = PRS_FLUSH_BATCH;
#pragma unroll
  for (int q0 = 0; q0 < kPer; q0 += kBatch) {
    T old[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      T *Fp;
      size_t g;
      A_t a;
      bool wall;
      old[b] = (T)0;
      if (!overwrite && q0 + b < kPer && node(q0 + b, Fp, g, a, wall)) old[b] = Fp[g];
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      T *Fp;
      size_t g;
      A_t a;
      bool wall;
      if (q0 + b >= kPer || !node(q0 + b, Fp, g, a, wall)) continue;
      if (wall) {
        Fp[g] = (T)0;
        continue;
      }
      const T v = poison ? (T)NAN : (kFixed ? (T)((double)a * unit) : (T)a);
      Fp[g] = old[b] + v;
    }
  }
  if (poison && threadIdx.x == 0) atomicOr(status, kFlagNonFinite);
}

// SRC 0: marker values from the correction buffer dF [3][n*nl] (sorted
//        spheres); SRC 1: caller-ordered [n][nl][3] values, sphere k of the
//        sorted order read at perm[k].
// Waves per SIMD the spreading kernel is compiled for: three 512-thread
// tiles per compute unit in single precision (about 47 KB of LDS each), two
// in double precision.
template <typename T>
struct TileWaves {
  static constexpr int value = (sizeof(T) == 4 ? 3 : 2) * kTileThreads / 256;
};
// The record-only form (no accumulators, 7 KB of LDS): 256-thread tiles,
// eight per compute unit (its code uses blockDim, and needs at least
// kTileCand threads for the scan and kTileList >= 2 blockDim).
constexpr int kRecordThreads = 256;
constexpr int kRecordWaves = 8 * kRecordThreads / 256;
static_assert(kRecordThreads >= kTileCand && kTileList >= 2 * kRecordThreads, "record-only tiles");

// kRecordOnly: only the first part, each tile's candidates and culled
// markers recorded for the spreading passes that follow (no accumulators,
// so many more tiles fit a compute unit; f untouched).
template <typename T, int SRC, bool kRecordOnly = false>
__global__ __launch_bounds__(kTileThreads)
__attribute__((amdgpu_waves_per_eu(kRecordOnly ? kRecordWaves : TileWaves<T>::value))) void k_spread_tiles(
    Geom G, Cells C, const int *__restrict__ start, const double *__restrict__ xs, int n,
    const double *__restrict__ templ, const T *__restrict__ tm, const T *__restrict__ src,
    const int *__restrict__ perm, const float *__restrict__ vmax, T *f0, T *f1, T *f2,
    uint32_t *status, TileCache tc) {
  constexpr int TX = TileShape<T>::X, TY = TileShape<T>::Y, TZ = TileShape<T>::Z;
  constexpr int NODES = AccLayout<TX, TY, TZ>::NODES;
  using A_t = typename TileAcc<T>::type;
  __shared__ __attribute__((aligned(16))) A_t acc[kRecordOnly ? 4 : 3 * NODES];
  __shared__ int c_idx[kTileCand];
  __shared__ int c_l0[kTileCand];
  __shared__ int c_pref[kTileCand + 1];
  __shared__ TileCand<T> c_geo[kRecordOnly ? 1 : kTileCand];
  __shared__ int c_n;
  __shared__ unsigned c_list[kTileList];   // culled (candidate << 10 | marker)
  __shared__ int c_list_n;

  const int ntx = (G.nx + TX - 1) / TX, nty = (G.ny + 1 + TY - 1) / TY,
            ntz = (G.nz + TZ - 1) / TZ;
  const int tile = xcd_item(blockIdx.x, ntx * nty * ntz);
  if (tile < 0) return;
  const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
  const int i0 = tx * TX, j0 = ty * TY, k0 = tz * TZ;
  const double h = G.h, R = G.R;
  const size_t N = (size_t)n;

  // Sphere centres whose markers can reach the tile's nodes: a marker reaches
  // node i of a component when |X/h - o - i| < 3/2, i.e. X/h in
  // (i0 - 3/2, i0 + T + 1) over the tile and both staggerings.
  const double lo[3] = {(i0 - 1.5) * h - R, (j0 - 1.5) * h - R, (k0 - 1.5) * h - R};
  const double hi[3] = {(i0 + TX + 1.0) * h + R, (j0 + TY + 1.0) * h + R,
                        (k0 + TZ + 1.0) * h + R};
  const double ctr[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
  const double hw[3] = {0.5 * (hi[0] - lo[0]) + 1e-9, 0.5 * (hi[1] - lo[1]) + 1e-9,
                        0.5 * (hi[2] - lo[2]) + 1e-9};
  // the same box for the markers themselves (no sphere radius), widened by
  // 1e-6 h for the single-precision stencil positions
  const double mctr[3] = {(i0 + 0.5 * (TX - 0.5)) * h, (j0 + 0.5 * (TY - 0.5)) * h,
                          (k0 + 0.5 * (TZ - 0.5)) * h};
  const double mhw[3] = {(0.5 * TX + 1.25 + 1e-6) * h, (0.5 * TY + 1.25 + 1e-6) * h,
                         (0.5 * TZ + 1.25 + 1e-6) * h};

  constexpr bool kFixed = std::is_integral<A_t>::value;
  const double dvh = G.dV * G.inv_h * G.inv_h * G.inv_h;
  const int nl = G.nl;
  const size_t M = N * nl;
  double vsum = 0.0;   // sum of the candidates' largest |marker value| (fixed point)
  double unit = 1.0;   // fixed point: the accumulators' unit
  bool poison = false;
  T scale = (T)dvh;

  // Replay: this step's earlier pass recorded the tile's candidates and
  // culled markers (the spheres have not moved since).
  const int cached = (!kRecordOnly && tc.mode == 2) ? tc.count[tile] : -1;   // uniform
  if (!kRecordOnly && cached >= 0) {
    if (cached == 0) {
      if (tc.overwrite)
        tile_flush<T, A_t, TX, TY, TZ>(G, nullptr, i0, j0, k0, 1.0, false, true, f0, f1, f2,
                                       status);
      return;
    }
    const unsigned *reg = tc.items + (size_t)tile * tc.cap;
    const int ncand = tc.ncand[tile];
    const unsigned *itm = reg + ncand;
    // the codes of this thread's listed markers (at most kReplayRounds),
    // loaded with the candidates
    unsigned code[kReplayRounds];
#pragma unroll
    for (int r = 0; r < kReplayRounds; ++r) {
      const int it = (int)threadIdx.x + r * (int)blockDim.x;
      code[r] = it < cached ? itm[it] : 0u;
    }
    for (int t = threadIdx.x; t < ncand; t += blockDim.x) {
      const int k = (int)reg[t];
      c_idx[t] = k;
      tile_cand<T, TX, TY, TZ>(G, xs[k], xs[N + k], xs[2 * N + k], i0, j0, k0, c_geo[t].d,
                               c_geo[t].fo);
    }
    if (kFixed) {
      __shared__ double r_wv[kTileThreads / 64];
      double vs = 0.0;
      for (int t = threadIdx.x; t < ncand; t += blockDim.x) vs += (double)vmax[reg[t]];
      vs = wave_sum_last(vs);
      if ((threadIdx.x & 63) == 63) r_wv[threadIdx.x >> 6] = vs;
      __syncthreads();
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) vsum += r_wv[w];
    }
    tile_unit<T, kFixed>(G.wsum_bound * dvh * vsum, dvh, unit, poison, scale);
    acc_clear<A_t, 3 * NODES>(acc);
    __syncthreads();
    // the listed markers, the next one's values loading while the current
    // one is accumulated
    T vc[3] = {(T)0, (T)0, (T)0};
    if ((int)threadIdx.x < cached)
      marker_values<T, SRC>(G, src, perm, c_idx[code[0] >> 10], (int)(code[0] & 1023u), M, vc);
#pragma unroll
    for (int r = 0; r < kReplayRounds; ++r) {
      const int it = (int)threadIdx.x + r * (int)blockDim.x;
      if (it >= cached) break;
      T vn[3] = {(T)0, (T)0, (T)0};
      if (r + 1 < kReplayRounds && it + (int)blockDim.x < cached)
        marker_values<T, SRC>(G, src, perm, c_idx[code[r + 1] >> 10],
                              (int)(code[r + 1] & 1023u), M, vn);
      const int sc = (int)(code[r] >> 10);
      spread_visit_v<T, TX, TY, TZ>(G, c_geo[sc].d, c_geo[sc].fo, tm, vc,
                                    (int)(code[r] & 1023u), scale, acc);
#pragma unroll
      for (int c = 0; c < 3; ++c) vc[c] = vn[c];
    }
    __syncthreads();
    tile_flush<T, A_t, TX, TY, TZ>(G, acc, i0, j0, k0, unit, poison, tc.overwrite, f0, f1, f2,
                                   status);
    return;
  }

  if (threadIdx.x == 0) {
    c_n = 0;
    c_list_n = 0;
  }
  __syncthreads();
  {
    const int cxl = (int)floor(lo[0] / C.csx), cxh = (int)floor(hi[0] / C.csx);
    const int czl = (int)floor(lo[2] / C.csz), czh = (int)floor(hi[2] / C.csz);
    const int cyl = max((int)floor(lo[1] / C.csy), 0), cyh = min((int)floor(hi[1] / C.csy), C.ncy - 1);
    const int nxc = min(cxh - cxl + 1, C.ncx), nzc = min(czh - czl + 1, C.ncz);
    const int nyc = cyh - cyl + 1;
    const int ncell = nyc > 0 ? nxc * nyc * nzc : 0;
    for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
      const int qx = q % nxc, qy = (q / nxc) % nyc, qz = q / (nxc * nyc);
      int cx = (cxl + qx) % C.ncx;
      if (cx < 0) cx += C.ncx;
      int cz = (czl + qz) % C.ncz;
      if (cz < 0) cz += C.ncz;
      const int key = cell_key(C, cx, cyl + qy, cz);
      const int e = start[key + 1];
      for (int k = start[key]; k < e; ++k) {
        const double px = xs[k], py = xs[N + k], pz = xs[2 * N + k];
        if (fabs(min_image(px - ctr[0], G.Lx)) > hw[0] || fabs(py - ctr[1]) > hw[1] ||
            fabs(min_image(pz - ctr[2], G.Lz)) > hw[2])
          continue;
        const int slot = atomicAdd(&c_n, 1);
        if (slot < kTileCand) {
          c_idx[slot] = k;
          if constexpr (!kRecordOnly)
            tile_cand<T, TX, TY, TZ>(G, px, py, pz, i0, j0, k0, c_geo[slot].d, c_geo[slot].fo);
        }
      }
    }
  }
  __syncthreads();
  int nc = c_n;
  const bool record = tc.mode == 1;
  if (nc == 0) {
    if (record && threadIdx.x == 0) tc.count[tile] = 0;
    if (!kRecordOnly && tc.overwrite)
      tile_flush<T, A_t, TX, TY, TZ>(G, nullptr, i0, j0, k0, 1.0, false, true, f0, f1, f2,
                                     status);
    return;
  }
  if (nc > kTileCand) {
    if (threadIdx.x == 0) atomicOr(status, kFlagCand);
    nc = kTileCand;
  }
  // recording: the candidates first, then the culled markers as
  // (candidate slot << 10 | marker); a tile whose list does not fit is not
  // recorded
  unsigned *reg = record ? tc.items + (size_t)tile * tc.cap : nullptr;
  __shared__ int r_len;   // entries recorded so far, -1 once out of room
  if (record) {
    if (threadIdx.x == 0) r_len = nc <= tc.cap ? nc : -1;
    if (nc <= tc.cap)
      for (int t = threadIdx.x; t < nc; t += blockDim.x) reg[t] = (unsigned)c_idx[t];
  }
  // markers of each sphere that can reach the tile: the template's
  // y-component 1 - (2l+1)/N_L is monotone in l, so the markers within the
  // tile's reach in y form one index range.  A centre a distance dx (dz)
  // outside the markers' reach box in x (z) needs |t_x| >= dx/R and |t_z| >=
  // dz/R, so t_x^2 + t_z^2 = 1 - t_y^2 >= (dx^2 + dz^2) / R^2: a band around
  // the equator, which narrows the range further.
  const double ylo = (j0 - 1.5) * h, yhi = (j0 + TY + 1.0) * h;
  for (int s = threadIdx.x; s < kTileCand; s += blockDim.x) {
    int cnt = 0, l0 = 0;
    if (s < nc) {
      const int k = c_idx[s];
      const double cx = xs[k], cy = xs[N + k], cz = xs[2 * N + k];
      double thi = (yhi - cy) / R, tlo = (ylo - cy) / R;
      const double dx = fmax(fabs(min_image(cx - mctr[0], G.Lx)) - mhw[0], 0.0);
      const double dz = fmax(fabs(min_image(cz - mctr[2], G.Lz)) - mhw[2], 0.0);
      const double tmax = sqrt(fmax(1.0 - (dx * dx + dz * dz) / (R * R), 0.0)) + 1e-6;
      thi = fmin(thi, tmax);
      tlo = fmax(tlo, -tmax);
      l0 = max((int)floor((nl * (1.0 - thi) - 1.0) * 0.5) - 1, 0);
      const int l1 = min((int)ceil((nl * (1.0 - tlo) - 1.0) * 0.5) + 1, nl - 1);
      cnt = l1 >= l0 ? l1 - l0 + 1 : 0;
    }
    c_l0[s] = l0;
    c_pref[s] = cnt;
  }
  if constexpr (!kRecordOnly) acc_clear<A_t, 3 * NODES>(acc);
  __syncthreads();
  if constexpr (kRecordOnly) {
    // Each wave walks whole candidates' marker ranges, 64 markers a round,
    // and appends the survivors straight to the tile's record (an LDS
    // counter places each wave's ballot): no search of the flattened
    // (candidate, marker) index and no block-wide rounds.  The entries'
    // order follows the waves' timing; the single-precision replay adds
    // fixed-point integers, whose sums do not depend on it.
    if (record && nc <= tc.cap) {
      const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
      for (int sidx = threadIdx.x >> 6; sidx < nc; sidx += nw) {
        const int cnt = c_pref[sidx], l0 = c_l0[sidx], k = c_idx[sidx];
        const double cx = xs[k], cy = xs[N + k], cz = xs[2 * N + k];
        for (int o = lane; o < ((cnt + 63) & ~63); o += 64) {
          bool pass = false;
          if (o < cnt) {
            const int l = l0 + o;
            const double X0 = cx + R * templ[3 * l], X1 = cy + R * templ[3 * l + 1],
                         X2 = cz + R * templ[3 * l + 2];
            pass = fabs(min_image(X0 - mctr[0], G.Lx)) <= mhw[0] &&
                   fabs(X1 - mctr[1]) <= mhw[1] && fabs(min_image(X2 - mctr[2], G.Lz)) <= mhw[2];
          }
          const unsigned long long ball = __ballot(pass);
          if (!ball) continue;
          int wbase = 0;
          if (lane == 0) wbase = atomicAdd(&r_len, __popcll(ball));
          wbase = __shfl(wbase, 0);
          const int pos = wbase + __popcll(ball & ((1ull << lane) - 1ull));
          if (pass && pos < tc.cap) reg[pos] = ((unsigned)sidx << 10) | (unsigned)(l0 + o);
        }
      }
    }
    __syncthreads();
    if (record && threadIdx.x == 0) {
      tc.count[tile] = (nc <= tc.cap && r_len <= tc.cap) ? r_len - nc : -1;
      tc.ncand[tile] = nc;
    }
    return;
  }
  // exclusive scan of the range lengths (kTileCand entries, one per lane of
  // the first kTileCand threads): shuffles inside each wave, then the wave
  // totals
  {
    __shared__ int c_wsum[kTileCand / 64];
    __shared__ double c_wvsum[kTileCand / 64];
    const int t = threadIdx.x, ln = t & 63;
    const int v = t < kTileCand ? c_pref[t] : 0;
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off);
      if (ln >= off) incl += y;
    }
    if (t < kTileCand && ln == 63) c_wsum[t >> 6] = incl;
    if (kFixed && !kRecordOnly) {
      double vs = t < nc ? (double)vmax[c_idx[t]] : 0.0;
      vs = wave_sum_last(vs);
      if (t < kTileCand && ln == 63) c_wvsum[t >> 6] = vs;
    }
    __syncthreads();
    if (kFixed && !kRecordOnly)
      for (int w = 0; w < kTileCand / 64; ++w) vsum += c_wvsum[w];
    if (t < kTileCand) {
      int base = 0;
      for (int w = 0; w < (t >> 6); ++w) base += c_wsum[w];
      c_pref[t] = base + incl - v;
      if (t == kTileCand - 1) c_pref[kTileCand] = base + incl;
    }
    __syncthreads();
  }
  const int total = c_pref[kTileCand];
  tile_unit<T, kFixed>(G.wsum_bound * dvh * vsum, dvh, unit, poison, scale);
  // Rounds of blockDim items (sphere, marker) of the y-bands: cull each item
  // by the tile's reach box and append the survivors to an LDS list (wave
  // ballot + one LDS atomic per wave); once the list could overflow, or at
  // the end, every lane takes one listed marker for the stencil and the LDS
  // atomics, so that work runs on full waves.
  const int lane = threadIdx.x & 63;
  for (int base0 = 0; base0 < total; base0 += blockDim.x) {
    const int item = base0 + threadIdx.x;
    bool pass = false;
    unsigned code = 0;
    if (item < total) {
      int a = 0, b = nc;   // largest s < nc with c_pref[s] <= item
      while (b - a > 1) {
        const int mid = (a + b) >> 1;
        if (c_pref[mid] <= item) a = mid; else b = mid;
      }
      const int l = c_l0[a] + (item - c_pref[a]);
      // a marker outside the tile's reach box touches none of its nodes
      // (conservative; the exact test is each component's stencil range)
      const int k = c_idx[a];
      const double X0 = xs[k] + R * templ[3 * l], X1 = xs[N + k] + R * templ[3 * l + 1],
                   X2 = xs[2 * N + k] + R * templ[3 * l + 2];
      pass = fabs(min_image(X0 - mctr[0], G.Lx)) <= mhw[0] && fabs(X1 - mctr[1]) <= mhw[1] &&
             fabs(min_image(X2 - mctr[2], G.Lz)) <= mhw[2];
      code = ((unsigned)a << 10) | (unsigned)l;
    }
    const unsigned long long ball = __ballot(pass);
    int wbase = 0;
    if (lane == 0 && ball) wbase = atomicAdd(&c_list_n, __popcll(ball));
    wbase = __shfl(wbase, 0);
    if (pass) c_list[wbase + __popcll(ball & ((1ull << lane) - 1ull))] = code;
    __syncthreads();
    const int listed = c_list_n;
    const bool flush = listed > kTileList - (int)blockDim.x || base0 + (int)blockDim.x >= total;
    __syncthreads();   // every lane has read the count before the next round appends
    if (flush) {
      const int rbase = record ? r_len : -1;
      const bool keep = rbase >= 0 && rbase + listed <= tc.cap;
      for (int it = threadIdx.x; it < listed; it += blockDim.x) {
        const unsigned cd = c_list[it];
        const int sc = (int)(cd >> 10), l = (int)(cd & 1023u);
        if (keep) reg[rbase + it] = cd;
        if constexpr (!kRecordOnly)
          spread_visit<T, SRC, TX, TY, TZ>(G, c_geo[sc].d, c_geo[sc].fo, tm, src, perm,
                                           c_idx[sc], l, M, scale, acc);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        c_list_n = 0;
        if (record) r_len = keep ? rbase + listed : -1;
      }
      __syncthreads();
    }
  }
  if (record && threadIdx.x == 0) {
    tc.count[tile] = r_len >= 0 ? r_len - nc : -1;
    tc.ncand[tile] = nc;
  }
  if constexpr (kRecordOnly) return;
  __syncthreads();
  tile_flush<T, A_t, TX, TY, TZ>(G, acc, i0, j0, k0, unit, poison, tc.overwrite, f0, f1, f2,
                                 status);
}


// vmax[p] = largest |component| of the caller-ordered marker values of
// sorted sphere p (NaN if any is NaN).
template <typename T>
__global__ __launch_bounds__(1024) void k_sphere_vmax(Geom G, const T *__restrict__ F,
                                                      const int *__restrict__ perm, int n,
                                                      float *vmax) {
  __shared__ float wm[16];
  const int p = xcd_item(blockIdx.x, n);
  if (p < 0) return;
  unsigned m = 0u;
  if ((int)threadIdx.x < G.nl) {
    const size_t q = ((size_t)perm[p] * G.nl + threadIdx.x) * 3;
    for (int c = 0; c < 3; ++c) m = max(m, abs_bits((float)F[q + c]));
  }
  m = wave_max_last(m);
  if ((threadIdx.x & 63) == 63) wm[threadIdx.x >> 6] = __uint_as_float(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    float mf = wm[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mf = nan_max(mf, wm[w]);
    vmax[p] = mf;
  }
}

template <typename T>
hipError_t launch_sphere_vmax(hipStream_t s, const Geom &G, const Scratch &S, int n, const T *F) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sphere_vmax<T>, dim3(xcd_grid(n)), dim3(block_for(G.nl)), 0, s, G, F,
                     S.perm, n, S.vmax);
  return hipGetLastError();
}
template hipError_t launch_sphere_vmax<float>(hipStream_t, const Geom &, const Scratch &, int,
                                              const float *);
template hipError_t launch_sphere_vmax<double>(hipStream_t, const Geom &, const Scratch &, int,
                                               const double *);

// The tiles' records alone (record-only form); the spreading passes that
// follow replay them.
template <typename T>
hipError_t launch_tile_record(hipStream_t s, const Geom &G, const Cells &C, const Scratch &S,
                              int n) {
  if (n == 0 || !S.tc_items) return hipSuccess;
  const int ntiles = spread_tile_count<T>(G);
  TileCache tc{1, S.tc_cap, S.tc_items, S.tc_count, S.tc_ncand};
  hipLaunchKernelGGL((k_spread_tiles<T, 0, true>), dim3(xcd_grid(ntiles)), dim3(kRecordThreads),
                     0, s, G, C, S.start, S.xs[0], n, S.templ,
                     (const T *)(sizeof(T) == 4 ? (const void *)S.tm32 : (const void *)S.tm64),
                     (const T *)S.dF, S.perm, S.vmax, nullptr, nullptr, nullptr, S.status, tc);
  return hipGetLastError();
}
template hipError_t launch_tile_record<float>(hipStream_t, const Geom &, const Cells &,
                                              const Scratch &, int);
template hipError_t launch_tile_record<double>(hipStream_t, const Geom &, const Cells &,
                                               const Scratch &, int);

template <typename T>
hipError_t launch_spread_tiles(hipStream_t s, const Geom &G, const Cells &C, const Scratch &S,
                               T *f[3], int n, const T *src_caller, TileCache tc) {
  if (n == 0) return hipSuccess;
  const int ntiles = spread_tile_count<T>(G);
  if (!tc.items) tc.mode = 0;
  if (tc.mode == 1) {
    // the records first, by the record-only form (more tiles resident), then
    // this pass replays them like the later ones
    hipLaunchKernelGGL((k_spread_tiles<T, 0, true>), dim3(xcd_grid(ntiles)), dim3(kRecordThreads),
                       0, s, G, C, S.start, S.xs[0], n, S.templ,
                       (const T *)(sizeof(T) == 4 ? (const void *)S.tm32 : (const void *)S.tm64),
                       (const T *)S.dF, S.perm, S.vmax, f[0], f[1], f[2], S.status, tc);
    tc.mode = 2;
  }
  const T *tm = (const T *)(sizeof(T) == 4 ? (const void *)S.tm32 : (const void *)S.tm64);
  // caller values: their per-sphere maxima first (the correction buffer's are
  // written by the interpolation pass that fills it)
  if (src_caller) {
    hipError_t e = launch_sphere_vmax<T>(s, G, S, n, src_caller);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_spread_tiles<T, 1>), dim3(xcd_grid(ntiles)), dim3(kTileThreads), 0, s,
                       G, C, S.start, S.xs[0], n, S.templ, tm, src_caller, S.perm, S.vmax, f[0],
                       f[1], f[2], S.status, tc);
  } else {
    hipLaunchKernelGGL((k_spread_tiles<T, 0>), dim3(xcd_grid(ntiles)), dim3(kTileThreads), 0, s,
                       G, C, S.start, S.xs[0], n, S.templ, tm, (const T *)S.dF, S.perm, S.vmax,
                       f[0], f[1], f[2], S.status, tc);
  }
  return hipGetLastError();
}

template <typename T>
int spread_tile_count(const Geom &G) {
  constexpr int TX = TileShape<T>::X, TY = TileShape<T>::Y, TZ = TileShape<T>::Z;
  return ((G.nx + TX - 1) / TX) * ((G.ny + 1 + TY - 1) / TY) * ((G.nz + TZ - 1) / TZ);
}
template int spread_tile_count<float>(const Geom &);

int spread_tile_dim(int esz, int axis) {
  if (esz == 4) return axis == 0 ? TileShape<float>::X : (axis == 1 ? TileShape<float>::Y : TileShape<float>::Z);
  return axis == 0 ? TileShape<double>::X : (axis == 1 ? TileShape<double>::Y : TileShape<double>::Z);
}
template int spread_tile_count<double>(const Geom &);

template hipError_t launch_spread_tiles<float>(hipStream_t, const Geom &, const Cells &,
                                               const Scratch &, float *[3], int, const float *,
                                               TileCache);
template hipError_t launch_spread_tiles<double>(hipStream_t, const Geom &, const Cells &,
                                                const Scratch &, double *[3], int,
                                                const double *, TileCache);

// ---------------------------------------------------------------------------
// per-sphere force/torque bookkeeping
// ---------------------------------------------------------------------------
// acc += part (compensated), for the iterations whose corrections are spread.
__global__ void k_ft_commit(double *acc, const double *part, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const size_t N = (size_t)n;
  for (int k = 0; k < 6; ++k) {
    double S = acc[(2 * k) * N + p], Cc = acc[(2 * k + 1) * N + p];
    comp_add(S, Cc, part[(2 * k) * N + p], part[(2 * k + 1) * N + p]);
    acc[(2 * k) * N + p] = S;
    acc[(2 * k + 1) * N + p] = Cc;
  }
}

hipError_t launch_ft_commit(hipStream_t s, const Scratch &S, int n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ft_commit, dim3((n + 255) / 256), dim3(256), 0, s, S.ft_acc, S.ft_part, n);
  return hipGetLastError();
}

// acc = compensated sums of a caller-ordered initial marker force F0.
template <typename T>
__global__ __launch_bounds__(1024) void k_marker_sums(Geom G, const double *__restrict__ templ,
                                                      const T *__restrict__ F0,
                                                      const int *__restrict__ perm, int n,
                                                      double *acc) {
  const int p = xcd_item(blockIdx.x, n);
  if (p < 0) return;
  const int l = threadIdx.x;
  Red red;
  red_zero(red);
  if (l < G.nl) {
    const double rl[3] = {G.R * templ[3 * l], G.R * templ[3 * l + 1], G.R * templ[3 * l + 2]};
    const size_t m = (size_t)perm[p] * G.nl + l;
    const double d[3] = {(double)F0[3 * m], (double)F0[3 * m + 1], (double)F0[3 * m + 2]};
    red_set_ft(red, rl, d);
  }
  double rs, rc;
  block_reduce<0x3Fu>(red, rs, rc);
  const int t = threadIdx.x;
  if (t < 6) {
    acc[(2 * t) * (size_t)n + p] = rs;
    acc[(2 * t + 1) * (size_t)n + p] = rc;
  }
}

template <typename T>
hipError_t launch_marker_sums(hipStream_t s, const Geom &G, const Scratch &S, int n, const T *F0) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_marker_sums<T>, dim3(xcd_grid(n)), dim3(block_for(G.nl)), 0, s, G,
                     S.templ, F0, S.perm, n, S.ft_acc);
  return hipGetLastError();
}

template hipError_t launch_marker_sums<float>(hipStream_t, const Geom &, const Scratch &, int,
                                              const float *);
template hipError_t launch_marker_sums<double>(hipStream_t, const Geom &, const Scratch &, int,
                                               const double *);

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

// Deterministic two-level reduction of the per-sphere slip partials of one
// pass into slip_hist[slot]: fixed chunks per block, then one block in order.
constexpr int kSlipBlocks = 256;

__global__ __launch_bounds__(256) void k_slip_partial(const double *part, int n, double *blocks) {
  __shared__ double lds[256];
  const int chunk = (n + kSlipBlocks - 1) / kSlipBlocks;
  const int b0 = blockIdx.x * chunk, b1 = min(b0 + chunk, n);
  double a = 0.0;
  for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) a += part[i];
  lds[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) blocks[blockIdx.x] = lds[0];
}

__global__ __launch_bounds__(256) void k_slip_final(const double *blocks, double *out) {
  __shared__ double lds[256];
  lds[threadIdx.x] = blocks[threadIdx.x];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = lds[0];
}

// which = 0: the slip of the pass just made -> slip_hist[iter];
// which = 1: the zero-forcing slip -> slip_hist[PRS_MAX_SLIP].
hipError_t launch_slip_reduce(hipStream_t s, const Scratch &S, int n, int iter, int which) {
  if (n == 0) return hipSuccess;
  const double *part = S.slip_part + (which ? (size_t)n : 0);
  double *blocks = S.slip_hist + PRS_MAX_SLIP + 1;
  double *dst = S.slip_hist + (which ? PRS_MAX_SLIP : iter);
  hipLaunchKernelGGL(k_slip_partial, dim3(kSlipBlocks), dim3(256), 0, s, part, n, blocks);
  hipLaunchKernelGGL(k_slip_final, dim3(1), dim3(256), 0, s, blocks, dst);
  return hipGetLastError();
}

__global__ void k_copy1(const double *src, double *dst) { *dst = *src; }

hipError_t launch_copy_scalar(hipStream_t s, const double *src, double *dst) {
  hipLaunchKernelGGL(k_copy1, dim3(1), dim3(1), 0, s, src, dst);
  return hipGetLastError();
}

__global__ void k_ib_finish(const double *acc, int n, double scale, double *fh, double *th) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const size_t N = (size_t)n;
  for (int a = 0; a < 3; ++a) {
    fh[a * N + p] = scale * (acc[(2 * a) * N + p] + acc[(2 * a + 1) * N + p]);
    th[a * N + p] = scale * (acc[(2 * (a + 3)) * N + p] + acc[(2 * (a + 3) + 1) * N + p]);
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
