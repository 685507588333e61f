/*
 * prs.h -- C ABI of the particle-phase step of the particle-resolved
 * sediment-transport method of Zhu, Hu, Lei, Shen and Zheng (arXiv
 * 2108.01814), built for AMD MI355X (gfx950).
 *
 * The step couples equal spheres to a fluid through a direct-forcing
 * immersed boundary (interpolation and diffusion through a regularised delta
 * function, sec. 3.3; forcing update eq. 4), resolves soft-sphere contacts
 * (collision force and torque, eqs. 9-10 and Appendix A, with the
 * fixed-capacity contact history of sec. 3.4) and advances the spheres by the
 * Newton-Euler equations (eqs. 7-8).
 *
 * Conventions shared by every call:
 *   - Units are those of the caller; the library never rescales.
 *   - Every array argument is DEVICE memory owned by the caller, contiguous,
 *     row-major, and is not retained after the call returns.  Host memory is
 *     used only where an argument says so (prs_template, stats, counts).
 *   - Particle vectors (positions x, velocities u, angular velocities omega,
 *     forces, torques) are double [n][3].
 *   - Grid fields use the staggered (MAC) layout of an nx*ny*nz box of
 *     spacing h, periodic in x and z, walls at y = 0 and y = ny*h:
 *       u: [nz][ny][nx]    at (i h, (j+1/2) h, (k+1/2) h)
 *       v: [nz][ny+1][nx]  at ((i+1/2) h, j h, (k+1/2) h)
 *       w: [nz][ny][nx]    at ((i+1/2) h, (j+1/2) h, k h)
 *     x fastest; element type float (PRS_F32) or double (PRS_F64) as chosen
 *     at prs_create.  Wall faces (v rows j = 0 and j = ny) never take part.
 *   - Per-marker vectors are [n][n_markers][3] in the grid element type.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is queued on that stream; calls that return counts or statistics
 *     synchronise with it before returning, as stated below.
 *   - Every call validates its arguments on the host before launching any
 *     work and returns a prs_status; prs_last_error() then describes it.
 *     Device-side conditions (capacity, non-finite state, a sphere leaving
 *     the domain) are reported through the status word at the next
 *     synchronising return.
 *   - One context per stream: a context's scratch memory is reused by every
 *     call, so calls on one context must not overlap.
 */
#ifndef PRS_H
#define PRS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum prs_status {
    PRS_OK = 0,
    PRS_EINVAL = 1,      /* invalid argument (detected on the host, nothing launched) */
    PRS_ECAPACITY = 2,   /* a fixed capacity was exceeded (see the call) */
    PRS_EDOMAIN = 3,     /* a sphere centre lies outside the box */
    PRS_ENONFINITE = 4,  /* a NaN or infinity in the particle state */
    PRS_EHIP = 5,        /* a HIP runtime call failed */
    PRS_ESKIN = 6        /* a sphere moved farther than skin/2 within one step */
} prs_status;

enum { PRS_F32 = 0, PRS_F64 = 1 };

#define PRS_SLOTS 14      /* contact slots per sphere: 12 spheres + 2 walls */
#define PRS_MAX_PP 12     /* equal spheres touch at most twelve others (sec. 3.4) */
#define PRS_WALL_BOTTOM (-1)
#define PRS_WALL_TOP (-2)
#define PRS_MAX_SLIP 64

typedef struct prs_params {
    /* Eulerian grid */
    int32_t nx, ny, nz;
    double h;
    /* spheres (all of radius `radius`) and fluid */
    double radius, rho_p, rho_f;
    double gravity[3];
    int32_t n_markers;   /* Lagrangian markers per sphere, 1 .. 1024 */
    /* immersed boundary: the forcing update uses alpha*dt_f (eq. 4) */
    double dt_f, alpha;
    int32_t n_iter;      /* multi-direct-forcing iterations when tol_mode = 0 */
    int32_t tol_mode;    /* 1: iterate until relative slip < tol or max_iter */
    double tol;
    int32_t max_iter;    /* <= PRS_MAX_SLIP - 1 */
    /* contacts and particle substeps (dt_p = dt_f / n_sub) */
    int32_t n_sub;
    double k_n, e_n, mu, kt_ratio, dt_ratio;
    double skin;         /* collision-search margin (>= 0), in length units */
    int32_t precision;   /* PRS_F32 or PRS_F64 */
    int32_t max_particles;
    /* contact coefficients (sec. 2.1, 4.1):
     *   PRS_CONTACT_FIXED: stiffness k_n, damping for restitution e_n with
     *     the pair's effective mass (m/2 sphere-sphere, m sphere-wall), and
     *     tangential k_t = kt_ratio k_n, d_t = dt_ratio d_n;
     *   PRS_CONTACT_COLLISION_TIME: every pair's coefficients calibrated so
     *     that a normal collision lasts t_c and restores e_n, and a sticking
     *     tangential contact (effective mass 2/7 of the pair's) oscillates
     *     with the same half-period and restores e_t: for mass m and
     *     restitution e, d = -2 m ln(e) / t_c, k = m (pi^2 + ln^2 e) / t_c^2
     *     (k_n, kt_ratio and dt_ratio unused). */
    int32_t contact_model;
    double t_c, e_t;
} prs_params;

enum { PRS_CONTACT_FIXED = 0, PRS_CONTACT_COLLISION_TIME = 1 };

typedef struct prs_ctx prs_ctx;

/* Contact history M_p of sec. 3.4, caller-owned device memory, slots of
 * sphere i at [i][0 .. cnt[i]-1]: partner index (another sphere, or
 * PRS_WALL_BOTTOM / PRS_WALL_TOP), tangential displacement delta_t (A.9-A.11)
 * and impact velocity u_in.  Slots are ordered by partner index ascending,
 * then the bottom wall, then the top wall; unused slots read zero on output.
 * An all-zero history means "no contacts yet". */
typedef struct prs_history {
    int32_t *partner;    /* [n][PRS_SLOTS] */
    double *delta_t;     /* [n][PRS_SLOTS][3] */
    double *u_in;        /* [n][PRS_SLOTS] */
    int8_t *count;       /* [n] */
} prs_history;

typedef struct prs_stats {
    int32_t iterations;                /* spreads performed (multi-direct forcing) */
    int32_t n_slip;                    /* entries of rel_slip filled */
    double rel_slip[PRS_MAX_SLIP];     /* ||U_d - I[u**]|| / ||U_d - I[u-hat]|| per interpolation */
    int64_t contacts;                  /* directed contacts summed over all substeps */
    int64_t pairs_last;                /* sphere-sphere pairs at the last substep */
    int64_t wall_last;                 /* sphere-wall contacts at the last substep */
    uint32_t flags;                    /* device status word (0 = clean) */
    int32_t rejected_learned;          /* 1: the learned warm start was rejected */
} prs_stats;

/* Create a context.  Checks the parameters, allocates the scratch memory for
 * up to p->max_particles spheres on the current device and builds the marker
 * template.  Returns PRS_EINVAL for inconsistent parameters (non-positive
 * sizes, n_markers outside 1..1024, a periodic box shorter than three
 * collision cells, ...), PRS_EHIP when allocation fails. */
int prs_create(const prs_params *p, prs_ctx **out);
void prs_destroy(prs_ctx *ctx);

/* Text of the last error on this context (never NULL). */
const char *prs_last_error(const prs_ctx *ctx);

/* Marker template (reading of sec. 3.5: one set of surface points shared by
 * every sphere): unit vectors t_l of a Fibonacci sphere with its pole along
 * y, and the marker volume dV = pi h (12 R^2 + h^2) / (3 n_markers).
 * t_host: HOST array double [n_markers][3]; dV: HOST double.  Synchronous. */
int prs_template(prs_ctx *ctx, double *t_host, double *dV);

/* Interpolation (sec. 3.3): for every marker X = x_p + R t_l of every sphere,
 * U_c = sum over the nodes of component c of g_c[node] * delta-kernel
 * weights (regularised three-point kernel, periodic in x and z, wall rule
 * above).  gu, gv, gw: grid fields; x, up, om: double [n][3];
 * U: [n][n_markers][3] out; Ud: optional [n][n_markers][3] out, the rigid
 * velocity u_p + omega_p x (R t_l) of each marker (NULL to skip).
 * Asynchronous.  PRS_EINVAL for n > max_particles or missing arrays. */
int prs_interpolate(prs_ctx *ctx, void *stream, const void *gu, const void *gv, const void *gw,
                    const double *x, const double *up, const double *om, int32_t n, void *U,
                    void *Ud);

/* Diffusion / spreading (sec. 3.3), the adjoint of prs_interpolate:
 * f_c[node] += F_c * weight * dV / h^3 for every marker.  F: [n][n_markers][3];
 * fu, fv, fw: grid fields, accumulated into (accumulate != 0) or
 * overwritten (accumulate == 0: every node stored, the entry values never
 * read).  FP64 fields accumulate with floating-point atomic
 * adds, so the summation order (and the last bits) may differ between runs;
 * FP32 fields accumulate in 32-bit fixed point per tile of the grid (each
 * addend rounded to 2^-30 of a bound on the tile's node sums), which is
 * deterministic.  Non-finite marker values make the reached nodes NaN.
 * Asynchronous. */
int prs_spread(prs_ctx *ctx, void *stream, const double *x, int32_t n, const void *F, void *fu,
               void *fv, void *fw, int accumulate);

/* Contact detection (Appendix A, (A.3)-(A.4)): every sphere pair with
 * minimum-image centre distance d, d^2 < (2R)^2, and every sphere with
 * y < R (bottom wall) or ny*h - y < R (top wall).  pairs: device int32
 * [cap][2] receiving rows (i, j), i < j for sphere pairs, j = PRS_WALL_BOTTOM
 * or PRS_WALL_TOP for walls, ordered by i, then j ascending, then bottom wall,
 * then top wall -- a canonical order independent of the device.  n_out: HOST
 * int64, the number of contacts.  When it exceeds cap, only the first cap
 * rows are written and PRS_ECAPACITY is returned; a sphere touching more
 * than PRS_MAX_PP spheres also gives PRS_ECAPACITY.  Positions must satisfy
 * 0 <= x < nx h, 0 <= y <= ny h, 0 <= z < nz h (else PRS_EDOMAIN /
 * PRS_ENONFINITE).  Synchronous. */
int prs_contacts(prs_ctx *ctx, void *stream, const double *x, int32_t n, int32_t *pairs,
                 int64_t cap, int64_t *n_out);

/* Bed and flying spheres (sec. 4.3.1, step (1)): a sphere in the bottom
 * layer (centre y < 2R) is a bed sphere, and so is every sphere in contact
 * with a bed sphere (A.3: d^2 < (2R)^2, minimum image in x and z), directly
 * or through a chain of contacts; all other spheres are flying.
 * x: device double [n][3]; flags: device int8 [n] out, caller order (1 bed,
 * 0 flying); n_bed: HOST int64 out, the number of bed spheres.  The same
 * position checks as prs_contacts (PRS_EDOMAIN / PRS_ENONFINITE), and
 * PRS_ECAPACITY when a sphere touches more than PRS_MAX_PP spheres.  The
 * result does not depend on the order of the device's updates.  Synchronous. */
int prs_bed_flags(prs_ctx *ctx, void *stream, const double *x, int32_t n, int8_t *flags,
                  int64_t *n_bed);

/* One particle-phase step (sec. 2.1 and 3): immersed-boundary forcing at the
 * current sphere state, then n_sub contact + Newton-Euler substeps of
 * dt_p = dt_f / n_sub with the hydrodynamic force and torque held fixed.
 *
 *   uhat  : 3 grid fields, the predicted fluid velocity u-hat (read only).
 *   f     : 3 grid fields, in/out.  On entry the initial forcing field
 *           (normally all zero; pass zero_f = 1 to have the call clear it:
 *           the entry values are then never read, whatever they hold, and
 *           the first spreading pass stores every node);
 *           on return the immersed-boundary force field.  The intermediate
 *           velocity of eq. 4 is u-tilde = u-hat + alpha dt_f f; it is never
 *           stored by the library.
 *   x, u, om : double [n][3] sphere state, advanced in place.  Written only
 *           at the very end and only when the step succeeded: on any error
 *           they (and the history) keep their input values.
 *   hist  : contact history, in/out (see prs_history).
 *   Fh, Th: double [n][3] out, hydrodynamic force and torque on each sphere,
 *           -rho_f dV sum_l F_l and -rho_f dV sum_l (R t_l) x F_l.
 *   F0    : optional [n][n_markers][3] initial marker force (warm start),
 *           spread before the first iteration; NULL for none.
 *   stats : HOST, optional, filled on return.
 * Synchronous on return.  Errors: PRS_EINVAL (arguments), PRS_ECAPACITY
 * (more than PRS_MAX_PP touching spheres, or more than 32 collision-search
 * candidates on one sphere), PRS_EDOMAIN, PRS_ENONFINITE, PRS_ESKIN (a sphere
 * moved more than skin/2 during the substeps; retry with a larger skin). */
int prs_step_particles(prs_ctx *ctx, void *stream, const void *const uhat[3], void *const f[3],
                       int zero_f, double *x, double *u, double *om, int32_t n,
                       const prs_history *hist, double *Fh, double *Th, const void *F0,
                       prs_stats *stats);

/* The step with the options of a Runge-Kutta coupling (eqs. 3-6): the
 * arguments of prs_step_particles in a struct, plus
 *   alpha      : > 0: this call's forcing coefficient alpha_k of the
 *                Runge-Kutta substep (the forcing uses alpha dt_f, eq. 4);
 *                0: the context's alpha;
 *   advance    : 0: the forcing only (F_h, T_h and f out; the spheres, their
 *                velocities and the history keep their values: a substep
 *                that is not the last); 1: the contact and Newton-Euler
 *                substeps follow, as in prs_step_particles;
 *   inner_prev : NULL, or [n][6] double: the previous call's integrals of
 *                the fluid inside the spheres (see prs_inner_fluid); then
 *                rho_f (I - I_prev) / (alpha dt_f) is added to F_h (first
 *                three) and T_h (last three), with I the integrals of
 *                u** = u-hat + alpha dt_f f after the forcing, over the spheres
 *                at the positions this call starts from;
 *   inner_out  : NULL, or [n][6] double out: I (required with inner_prev).
 * Reading (the paper does not say where the particle substeps fall in the
 * fluid's Runge-Kutta substeps): every substep forces the flow with its
 * alpha_k, the particles are advanced once, in the last one. */
typedef struct prs_step_args {
    const void *const *uhat;   /* 3 grid fields, read only */
    void *const *f;            /* 3 grid fields, in/out */
    int32_t zero_f;
    double *x, *u, *om;        /* [n][3] in/out */
    int32_t n;
    const prs_history *hist;
    double *Fh, *Th;           /* [n][3] out */
    const void *F0;            /* [n][n_markers][3] or NULL */
    double alpha;
    int32_t advance;
    const double *inner_prev;
    double *inner_out;
} prs_step_args;
int prs_step_particles_ex(prs_ctx *ctx, void *stream, const prs_step_args *args,
                          prs_stats *stats);

/* Fluid inside the spheres (the momentum term of the hydrodynamic force of
 * the direct-forcing method, eqs. 7-8): for every sphere, by the midpoint rule
 * over the staggered nodes inside it (|x_node - x_p| < R, minimum image in x
 * and z; wall faces and nodes outside the fluid excluded), each weighted h^3:
 *   inner[i][c]     = h^3 sum u_c[node]            (c = 0, 1, 2),
 *   inner[i][3 + a] = h^3 sum (r x e_c u_c[node])_a, r = x_node - x_p.
 * u: 3 grid fields; x: [n][3]; inner: device double [n][6] out.  Position
 * checks as prs_contacts.  Synchronous. */
int prs_inner_fluid(prs_ctx *ctx, void *stream, const void *const u[3], const double *x,
                    int32_t n, double *inner);

/* Per-phase device time of prs_step_particles, measured with HIP events
 * recorded on the caller's stream around each phase (milliseconds summed
 * over the steps since the last reset; launch counts alongside).  Phases:
 * clearing f, sorting into cells (+ state gather), interpolation passes,
 * spreading passes, the collision search, the particle substeps, the final
 * write-back.  Timing costs two event records per phase; it is off unless
 * enabled. */
typedef struct prs_timing {
    int64_t steps;
    double ms_zero_f, ms_sort, ms_interp, ms_spread, ms_search, ms_substep, ms_writeback;
    int64_t n_interp, n_spread, n_substep;
    double ms_learned;     /* the fused feature + network pass of a learned start */
    int64_t n_learned;
    double ms_record;      /* the spreading tiles' records (once per step, before the
                              first spreading pass) */
    int64_t n_record;
} prs_timing;

/* ---- learned warm start ------------------------------------------------
 * Not part of the paper: a small network predicts each marker's initial
 * forcing, after which the unchanged multi-direct forcing runs, so the plain
 * method stays both the fallback and the reference.  Network: 16 inputs (12
 * features zero-padded) -> 64 -> GELU -> 64 -> GELU -> 16 outputs (3 used),
 * exact-erf GELU, BF16 weights and activations on the matrix cores with FP32
 * accumulation, FP32 master weights trained by Adam (beta 0.9 / 0.999,
 * eps 1e-8) on the mean square error of standardised targets.
 * Parameter vector (FP32, PRS_MLP_PARAMS values, row-major out x in):
 *   W1[64][16], b1[64], W2[64][64], b2[64], W3[16][64], b3[16].
 * Normalisation vector (PRS_MLP_NORM values): feature mean[16], feature
 * std[16], target mean[3], target std[3] (std > 0).
 * Features of a marker (12, then 4 zeros): slip U_d - I[u-hat] (3), template
 * normal t_l (3), sphere velocity u_p (3), R omega_p (3).  Target (3): the
 * marker's total forcing after the plain iterations times alpha dt_f
 * (velocity units). */
#define PRS_MLP_PARAMS 6288
#define PRS_MLP_NORM 38
typedef struct prs_mlp prs_mlp;

/* Create a network on the current device from HOST arrays; Adam moments start
 * at zero.  PRS_EINVAL for non-finite values or non-positive std. */
int prs_mlp_create(const float *params, const float *norm, prs_mlp **out);
void prs_mlp_destroy(prs_mlp *mlp);
const char *prs_mlp_last_error(const prs_mlp *mlp);
/* Copy the FP32 master parameters / normalisation to HOST arrays (nullable). */
int prs_mlp_get(prs_mlp *mlp, float *params, float *norm);
/* Y [B][3] for inputs X [B][16] (device, FP32).  raw != 0: X are raw
 * features, standardised inside, and Y comes back in target units; raw == 0:
 * X and Y in standardised units.  Asynchronous. */
int prs_mlp_forward(prs_mlp *mlp, void *stream, const float *X, int32_t B, int raw, float *Y);
/* Backward pass: gradient of the loss (1/(3B)) sum (Y - T)^2 over the batch,
 * for standardised inputs X [B][16] and targets T [B][3] (device FP32).  The
 * forward pass is rerun inside (no activations are kept between calls); the
 * back-propagated errors are rounded to BF16 where they feed the matrix
 * cores, the bias gradients take them unrounded.  grad: device FP32
 * [PRS_MLP_PARAMS] (nullable: the network keeps the latest gradient for
 * prs_mlp_adam); loss: HOST (nullable; synchronises when given).  The batch
 * sums are reduced in a fixed order, so the result does not depend on the
 * launch. */
int prs_mlp_backward(prs_mlp *mlp, void *stream, const float *X, const float *T, int32_t B,
                     float *grad, double *loss);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected with the
 * network's step count) of the FP32 master weights with learning rate lr > 0
 * from grad (device FP32 [PRS_MLP_PARAMS]; NULL: the latest backward's
 * gradient); refreshes the BF16 copy.  Asynchronous. */
int prs_mlp_adam(prs_mlp *mlp, void *stream, const float *grad, float lr);
/* prs_mlp_backward followed by prs_mlp_adam on its gradient. */
int prs_mlp_train_step(prs_mlp *mlp, void *stream, const float *X, const float *T, int32_t B,
                       float lr, double *loss);
/* Loss (1/(3B)) sum (Y - T)^2 of standardised X [B][16], T [B][3] (device)
 * into *loss (HOST); forward pass only.  Synchronous. */
int prs_mlp_loss(prs_mlp *mlp, void *stream, const float *X, const float *T, int32_t B,
                 double *loss);
/* Standardise count raw samples with the network's statistics:
 * Xs = (X - mean) / std [count][16], Ts = (T - target mean) / target std
 * [count][3] (device FP32; T and Ts nullable together).  Asynchronous. */
int prs_mlp_standardize(prs_mlp *mlp, void *stream, const float *X, const float *T,
                        int64_t count, float *Xs, float *Ts);
/* Training-set statistics of count >= 2 raw samples X [count][16],
 * T [count][3] (device FP32) into norm (HOST, PRS_MLP_NORM values, the
 * layout prs_mlp_create takes): means and sample standard deviations
 * (denominator count - 1) in FP64, reduced in a fixed order; the four padding
 * features get mean 0 and std 1, a constant column std 1.  Allocates a small
 * scratch buffer.  Synchronous.  PRS_EINVAL for count < 2 or NULL arrays. */
int prs_mlp_fit_norm(void *stream, const float *X, const float *T, int64_t count, float *norm);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): prs_mlp_fit_norm
 * with the same arguments, results and errors, but no allocation of any
 * kind.  Its scratch (partial sums and statistics, 39,216 bytes) is a static
 * device array of the library, one instance per device, held until the
 * process ends; its size does not depend on count, so every count >= 2 is
 * accepted.  Calls that overlap on one device share that array and race:
 * issue them one at a time per device.  Synchronous. */
int prs_mlp_fit_norm_noalloc(void *stream, const float *X, const float *T, int64_t count,
                             float *norm);

/* Attach a network to a context (NULL detaches).  A step on a context with a
 * network starts the multi-direct forcing from the network's prediction: one
 * interpolation pass of u-hat computes each marker's features, evaluates the
 * network on them in the same kernel and writes F0 = prediction /
 * (alpha dt_f), which is spread before the first iteration.  The prediction
 * is rejected -- f cleared, the iteration restarted from zero forcing,
 * stats->rejected_learned = 1 -- when the first relative slip is >= 1 or the
 * slip grows from one iteration to the next.  Such steps need zero_f = 1 and
 * F0 = NULL (else PRS_EINVAL) and read the slip back after every iteration.
 * The context keeps the pointer: the network must outlive its use and must
 * not be trained concurrently with a step.  PRS_EINVAL when the pass does not
 * fit the device's LDS. */
int prs_set_learned(prs_ctx *ctx, const prs_mlp *mlp);

/* Training samples from the plain method: clears f, computes the features of
 * every marker of the spheres (x, u, om: double [n][3], device) against
 * u-hat, runs n_iter (1..PRS_MAX_SLIP-1) plain multi-direct-forcing
 * iterations (f on return: the resulting force field) and writes
 *   feat  : device float [n][n_markers][16], features (the last 4 zero),
 *   target: device float [n][n_markers][3], alpha dt_f times the marker's
 *           total forcing after the n_iter iterations,
 * both in caller order.  stats (HOST, nullable): iterations and relative
 * slips as for a step.  Synchronous. */
int prs_forcing_samples(prs_ctx *ctx, void *stream, const void *const uhat[3], void *const f[3],
                        const double *x, const double *u, const double *om, int32_t n,
                        int32_t n_iter, float *feat, float *target, prs_stats *stats);

/* Enable (1) or disable (0) phase timing on this context. */
int prs_timing_enable(prs_ctx *ctx, int enable);
/* Copy the accumulated phase times into *out (HOST); reset them if reset != 0. */
int prs_timing_read(prs_ctx *ctx, prs_timing *out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* PRS_H */
