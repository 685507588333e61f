/*
 * prs_oracle.c -- plain, slow, FP64 CPU oracle for the particle-phase step of
 * the particle-resolved sediment-transport method of Zhu, Hu, Lei, Shen and
 * Zheng, "Particle resolved simulation of sediment transport by a hybrid
 * parallel approach" (arXiv 2108.01814).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * reads this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or constant with the
 * HIP path.  Everything is double precision, single-threaded, and written as
 * the plain definition (loops in the order the method states them, no blocking,
 * no fusion).  Build: gcc -O2 -ffp-contract=off -fPIC -shared.
 *
 * Where the paper is silent the oracle follows a stated reading; every such
 * reading is marked "reading:" below.
 *
 * Layouts (all row-major, C order):
 *   particle vectors x, u, omega, F_h, T_h ........ [np][3]
 *   per-marker vectors (U, U_d, F) ................ [np][nl][3]
 *   staggered grid (window of the periodic grid) .. u, w: [wnz][ny][wnx],
 *                                                    v:    [wnz][ny+1][wnx]
 *   contact history ............................... partner [np][14] (int32),
 *        dt [np][14][3], uin [np][14], cnt [np] (int32)
 *
 * Return codes: 0 ok, 2 capacity exceeded, 3 particle outside the domain,
 * 4 non-finite value, 1 invalid argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ECAPACITY 2
#define OR_EDOMAIN 3
#define OR_ENONFINITE 4

#define OR_SLOTS 14   /* 12 particle partners + bottom wall + top wall */
#define OR_MAX_PP 12  /* equal spheres touch at most twelve others (sec. 3.4) */
#define OR_WALL_BOTTOM (-1)
#define OR_WALL_TOP (-2)

typedef struct {
    /* Eulerian grid: nx*ny*nz cells of spacing h; periodic in x and z, walls
     * at y = 0 and y = ny*h. */
    int32_t nx, ny, nz;
    double h;
    /* Stored window of the grid: global node columns i in [wi0, wi0+wnx) and
     * k in [wk0, wk0+wnz) (taken modulo nx, nz).  Nodes outside the window are
     * treated like nodes outside the domain: they take no part. */
    int32_t wi0, wnx, wk0, wnz;
    /* particles: equal spheres of radius R */
    double R, rho_p, rho_f;
    double g[3];
    int32_t nl;          /* Lagrangian markers per sphere */
    /* immersed boundary: forcing uses alpha*dt_f (eq. 4) */
    double dt_f, alpha;
    int32_t n_iter;      /* fixed number of multi-direct-forcing iterations */
    int32_t tol_mode;    /* 1: iterate until relative slip < tol or max_iter */
    double tol;
    int32_t max_iter;
    /* contacts */
    int32_t n_sub;       /* particle substeps per fluid step */
    double k_n, e_n, mu, kt_ratio, dt_ratio;
    int32_t use_cells;   /* 0: brute-force O(N^2) partner search; 1: cell list */
    /* contact coefficients: 0 = fixed linear law (k_n, e_n, kt_ratio,
     * dt_ratio); 1 = calibrated from the collision time t_c and the normal
     * and tangential restitution coefficients e_n, e_t (see contact_coeffs) */
    int32_t contact_model;
    double t_c, e_t;
} or_params;

/* ------------------------------------------------------------------------ */
/* Marker template.  Reading: one Fibonacci sphere shared by all particles,  */
/* pole along y, markers on the surface r = R; marker volume = volume of a   */
/* shell of thickness h around the surface divided by the number of markers. */
/* (The paper only states that the markers of one sphere are generated from  */
/* one set of points, sec. 3.5.)                                             */
/* ------------------------------------------------------------------------ */
void or_template(int32_t nl, double R, double h, double *t, double *dV)
{
    const double golden = M_PI * (3.0 - sqrt(5.0));
    for (int l = 0; l < nl; ++l) {
        double zp = 1.0 - (2.0 * l + 1.0) / nl;
        double rho = sqrt(1.0 - zp * zp);
        double th = l * golden;
        t[3 * l + 0] = rho * cos(th);
        t[3 * l + 1] = zp;
        t[3 * l + 2] = rho * sin(th);
    }
    *dV = M_PI * h * (12.0 * R * R + h * h) / (3.0 * nl);
}

/* ------------------------------------------------------------------------ */
/* Regularised delta function delta_d of the interpolation / diffusion      */
/* operations (sec. 3.3).  Reading: the three-point kernel of Roma, Peskin  */
/* and Berger, as a function of the distance in grid spacings.              */
/* ------------------------------------------------------------------------ */
double or_phi(double r)
{
    double a = fabs(r);
    if (a <= 0.5)
        return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
    if (a <= 1.5)
        return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * (1.0 - a) * (1.0 - a))) / 6.0;
    return 0.0;
}

/* Staggered (MAC) node offsets in units of h.  Reading: the x-velocity lives
 * on x-faces (i, j+1/2, k+1/2), y-velocity on y-faces, z-velocity on z-faces. */
static void stagger_offset(int comp, double o[3])
{
    o[0] = (comp == 0) ? 0.0 : 0.5;
    o[1] = (comp == 1) ? 0.0 : 0.5;
    o[2] = (comp == 2) ? 0.0 : 0.5;
}

static long wrap_index(long i, long n)
{
    long m = i % n;
    return m < 0 ? m + n : m;
}

/* Flat index of node (i, j, k) of component comp in the stored window, or -1
 * when the node takes no part.  Reading (wall rule): y-faces on the walls
 * (j = 0 and j = ny) and every node outside 0 <= y <= ny*h are dropped from
 * both interpolation and spreading, with no renormalisation. */
static long node_index(const or_params *P, int comp, long i, long j, long k)
{
    long nyc = (comp == 1) ? (long)P->ny + 1 : (long)P->ny;
    if (comp == 1) {
        if (j < 1 || j > P->ny - 1)
            return -1;
    } else {
        if (j < 0 || j > P->ny - 1)
            return -1;
    }
    long ig = wrap_index(i, P->nx);
    long kg = wrap_index(k, P->nz);
    long il = wrap_index(ig - P->wi0, P->nx);
    long kl = wrap_index(kg - P->wk0, P->nz);
    if (il >= P->wnx || kl >= P->wnz)
        return -1;
    return (kl * nyc + j) * (long)P->wnx + il;
}

/* Interpolation of one velocity component at point X (sec. 3.3):
 * U = sum_n u[n] phi((X-x_n)/h) phi(.) phi(.) over the nodes of that
 * component.  The 4x4x4 block below covers every node within 3/2 h in each
 * axis; nodes with zero weight contribute nothing. */
static double interp_point(const or_params *P, int comp, const double *g, const double X[3])
{
    double o[3], s[3];
    long b[3];
    stagger_offset(comp, o);
    for (int a = 0; a < 3; ++a) {
        s[a] = X[a] / P->h - o[a];
        b[a] = (long)floor(s[a]) - 1;
    }
    double acc = 0.0;
    for (int kk = 0; kk < 4; ++kk)
        for (int jj = 0; jj < 4; ++jj)
            for (int ii = 0; ii < 4; ++ii) {
                long i = b[0] + ii, j = b[1] + jj, k = b[2] + kk;
                double w = or_phi(s[0] - i) * or_phi(s[1] - j) * or_phi(s[2] - k);
                if (w == 0.0)
                    continue;
                long n = node_index(P, comp, i, j, k);
                if (n < 0)
                    continue;
                acc += g[n] * w;
            }
    return acc;
}

/* Diffusion ("spreading") of one component of a point value (sec. 3.3):
 * g[n] += val * phi phi phi, the transpose of interp_point. */
static void spread_point(const or_params *P, int comp, double *g, const double X[3], double val)
{
    double o[3], s[3];
    long b[3];
    stagger_offset(comp, o);
    for (int a = 0; a < 3; ++a) {
        s[a] = X[a] / P->h - o[a];
        b[a] = (long)floor(s[a]) - 1;
    }
    for (int kk = 0; kk < 4; ++kk)
        for (int jj = 0; jj < 4; ++jj)
            for (int ii = 0; ii < 4; ++ii) {
                long i = b[0] + ii, j = b[1] + jj, k = b[2] + kk;
                double w = or_phi(s[0] - i) * or_phi(s[1] - j) * or_phi(s[2] - k);
                if (w == 0.0)
                    continue;
                long n = node_index(P, comp, i, j, k);
                if (n < 0)
                    continue;
                g[n] += val * w;
            }
}

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Marker position X_pl = x_p + R t_l and desired (rigid-body) velocity
 * U_d = u_p + omega_p x (R t_l). */
static void marker(const or_params *P, const double *t, const double *x, const double *up,
                   const double *om, int p, int l, double X[3], double Ud[3])
{
    double r[3], wr[3];
    for (int a = 0; a < 3; ++a) {
        r[a] = P->R * t[3 * l + a];
        X[a] = x[3 * p + a] + r[a];
    }
    cross(&om[3 * p], r, wr);
    for (int a = 0; a < 3; ++a)
        Ud[a] = up[3 * p + a] + wr[a];
}

static long comp_size(const or_params *P, int comp)
{
    return (long)P->wnz * (long)(comp == 1 ? P->ny + 1 : P->ny) * (long)P->wnx;
}

/* Interpolate the three staggered components at every marker of every
 * particle.  U and Ud are [np][nl][3]; Ud may be NULL. */
int or_interpolate(const or_params *P, const double *gu, const double *gv, const double *gw,
                   int32_t np, const double *x, const double *up, const double *om,
                   double *U, double *Ud)
{
    double *t = malloc(sizeof(double) * 3 * P->nl), dV;
    const double *g[3] = {gu, gv, gw};
    or_template(P->nl, P->R, P->h, t, &dV);
    for (int p = 0; p < np; ++p)
        for (int l = 0; l < P->nl; ++l) {
            double X[3], ud[3];
            marker(P, t, x, up, om, p, l, X, ud);
            for (int c = 0; c < 3; ++c) {
                U[(3L * ((long)p * P->nl + l)) + c] = interp_point(P, c, g[c], X);
                if (Ud)
                    Ud[(3L * ((long)p * P->nl + l)) + c] = ud[c];
            }
        }
    free(t);
    return OR_OK;
}

/* Spread per-marker vectors F ([np][nl][3]) onto the three component grids:
 * f_c[n] += F_c * phi phi phi * dV/h^3 (accumulates into f). */
int or_spread(const or_params *P, int32_t np, const double *x, const double *F,
              double *fu, double *fv, double *fw)
{
    double *t = malloc(sizeof(double) * 3 * P->nl), dV;
    double *g[3] = {fu, fv, fw};
    or_template(P->nl, P->R, P->h, t, &dV);
    double scale = dV / (P->h * P->h * P->h);
    for (int p = 0; p < np; ++p)
        for (int l = 0; l < P->nl; ++l) {
            double X[3];
            for (int a = 0; a < 3; ++a)
                X[a] = x[3 * p + a] + P->R * t[3 * l + a];
            for (int c = 0; c < 3; ++c)
                spread_point(P, c, g[c], X, F[3L * ((long)p * P->nl + l) + c] * scale);
        }
    free(t);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Multi-direct-forcing immersed boundary step (sec. 2.1, eq. 4; the         */
/* iteration itself is the multi-direct forcing of the cited IB papers).     */
/* Reading (Jacobi form): each iteration interpolates the intermediate       */
/* velocity u** at all markers from the same field, sets the correction      */
/* dF = (U_d - U)/(alpha dt_f), adds it to the marker force, spreads it into */
/* the force field f and adds alpha dt_f times the spread to u**.            */
/*                                                                          */
/* Inputs: uh = the predicted velocity (u-hat, read only); f = the force     */
/* field, in/out: on entry the initial forcing (normally zero), on return    */
/* entry + spread of every correction.  The intermediate field starts as     */
/* u** = u-hat + alpha dt_f f(entry).  F0 (nullable, [np][nl][3]) is an     */
/* initial marker force, spread before the first iteration.                  */
/* Outputs: Fh, Th [np][3] hydrodynamic force and torque on each sphere:     */
/* Fh = -rho_f dV sum_l F_l, Th = -rho_f dV sum_l (R t_l) x F_l (reading,    */
/* the discrete counterpart of the surface integrals of eqs. 7-8);           */
/* slip[s] = ||U_d - I[u**(s)]|| / ||U_d - I[u-hat]|| for every             */
/* interpolation made; *iters = number of spreads; Fmark (nullable,         */
/* [np][nl][3]) the final marker force; ustar_out (nullable, 3 arrays) the   */
/* final u**.                                                                */
/* ------------------------------------------------------------------------ */
int or_ib_forcing(const or_params *P, const double *uhu, const double *uhv, const double *uhw,
                  double *fu, double *fv, double *fw, int32_t np, const double *x,
                  const double *up, const double *om, const double *F0, double *Fh, double *Th,
                  double *slip, int32_t *iters, double *Fmark, double *usu, double *usv,
                  double *usw)
{
    const int nl = P->nl;
    const long M = (long)np * nl;
    const double adt = P->alpha * P->dt_f;
    double *t = malloc(sizeof(double) * 3 * nl), dV;
    or_template(nl, P->R, P->h, t, &dV);
    const double scale = dV / (P->h * P->h * P->h);

    const double *uh[3] = {uhu, uhv, uhw};
    double *f[3] = {fu, fv, fw};
    double *us[3];
    for (int c = 0; c < 3; ++c) {
        long n = comp_size(P, c);
        us[c] = malloc(sizeof(double) * n);
        for (long i = 0; i < n; ++i)
            us[c][i] = uh[c][i] + adt * f[c][i];
    }
    double *X = malloc(sizeof(double) * 3 * M);
    double *Ud = malloc(sizeof(double) * 3 * M);
    double *F = calloc(3 * M, sizeof(double));
    double *r = malloc(sizeof(double) * 3 * M);
    for (int p = 0; p < np; ++p)
        for (int l = 0; l < nl; ++l)
            marker(P, t, x, up, om, p, l, &X[3 * ((long)p * nl + l)], &Ud[3 * ((long)p * nl + l)]);

    /* denominator of the relative slip: the slip of zero forcing, from u-hat */
    double den = 0.0;
    for (long m = 0; m < M; ++m)
        for (int c = 0; c < 3; ++c) {
            double d = Ud[3 * m + c] - interp_point(P, c, uh[c], &X[3 * m]);
            den += d * d;
        }
    den = sqrt(den);

    if (F0) {
        for (long m = 0; m < 3 * M; ++m)
            F[m] = F0[m];
        for (long m = 0; m < M; ++m)
            for (int c = 0; c < 3; ++c) {
                double v = F0[3 * m + c] * scale;
                spread_point(P, c, f[c], &X[3 * m], v);
                spread_point(P, c, us[c], &X[3 * m], adt * v);
            }
    }

    int s = 0;
    for (;;) {
        /* (i) interpolate u** at every marker from the same field */
        double num = 0.0;
        for (long m = 0; m < M; ++m)
            for (int c = 0; c < 3; ++c) {
                double d = Ud[3 * m + c] - interp_point(P, c, us[c], &X[3 * m]);
                r[3 * m + c] = d;
                num += d * d;
            }
        slip[s] = den > 0.0 ? sqrt(num) / den : 0.0;
        if (P->tol_mode) {
            if (slip[s] < P->tol || s >= P->max_iter)
                break;
        } else if (s >= P->n_iter) {
            break;
        }
        /* (ii) direct-forcing correction, (iii) spread it into f and u** */
        for (long m = 0; m < M; ++m)
            for (int c = 0; c < 3; ++c) {
                double dF = r[3 * m + c] / adt;
                F[3 * m + c] += dF;
                double v = dF * scale;
                spread_point(P, c, f[c], &X[3 * m], v);
                spread_point(P, c, us[c], &X[3 * m], adt * v);
            }
        ++s;
        if (!P->tol_mode && s >= P->n_iter)
            break;
    }
    *iters = s;

    for (int p = 0; p < np; ++p) {
        double sF[3] = {0, 0, 0}, sT[3] = {0, 0, 0};
        for (int l = 0; l < nl; ++l) {
            const double *Fl = &F[3 * ((long)p * nl + l)];
            double rl[3] = {P->R * t[3 * l], P->R * t[3 * l + 1], P->R * t[3 * l + 2]}, rxF[3];
            cross(rl, Fl, rxF);
            for (int a = 0; a < 3; ++a) {
                sF[a] += Fl[a];
                sT[a] += rxF[a];
            }
        }
        for (int a = 0; a < 3; ++a) {
            Fh[3 * p + a] = -P->rho_f * dV * sF[a];
            Th[3 * p + a] = -P->rho_f * dV * sT[a];
        }
    }
    if (Fmark)
        memcpy(Fmark, F, sizeof(double) * 3 * M);
    double *uso[3] = {usu, usv, usw};
    for (int c = 0; c < 3; ++c) {
        if (uso[c])
            memcpy(uso[c], us[c], sizeof(double) * comp_size(P, c));
        free(us[c]);
    }
    free(X);
    free(Ud);
    free(F);
    free(r);
    free(t);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Contact detection (plain definition).  Appendix A, eqs. (A.3)-(A.4): a    */
/* pair is in contact when the gap delta_n = |x_q - x_p| - 2R is negative,   */
/* i.e. d^2 < (2R)^2 with d the minimum-image separation in the periodic x   */
/* and z directions.  A sphere touches the bottom wall when y < R and the    */
/* top wall (reading) when L_y - y < R.                                      */
/* ------------------------------------------------------------------------ */
static double min_image(double d, double L)
{
    if (d > 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

static void separation(const or_params *P, const double *x, int p, int q, double d[3])
{
    double Lx = P->nx * P->h, Lz = P->nz * P->h;
    d[0] = min_image(x[3 * q + 0] - x[3 * p + 0], Lx);
    d[1] = x[3 * q + 1] - x[3 * p + 1];
    d[2] = min_image(x[3 * q + 2] - x[3 * p + 2], Lz);
}

static int in_contact(const or_params *P, const double *x, int p, int q)
{
    double d[3];
    separation(P, x, p, q, d);
    double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return d2 < (2.0 * P->R) * (2.0 * P->R);
}

/* A plain bucket grid for the cell-list partner search: cells of edge at
 * least 2R, so every partner lies in the 27 surrounding cells. */
typedef struct {
    int ncx, ncy, ncz;
    double cx, cy, cz;
    int *head, *next;
} or_cells;

static int cell_coord(double v, double c, int n)
{
    int i = (int)floor(v / c);
    if (i < 0)
        i = 0;
    if (i > n - 1)
        i = n - 1;
    return i;
}

static void cells_build(const or_params *P, int np, const double *x, or_cells *C)
{
    double Lx = P->nx * P->h, Ly = P->ny * P->h, Lz = P->nz * P->h, D = 2.0 * P->R;
    C->ncx = (int)floor(Lx / D);
    C->ncy = (int)floor(Ly / D);
    C->ncz = (int)floor(Lz / D);
    if (C->ncx < 1)
        C->ncx = 1;
    if (C->ncy < 1)
        C->ncy = 1;
    if (C->ncz < 1)
        C->ncz = 1;
    C->cx = Lx / C->ncx;
    C->cy = Ly / C->ncy;
    C->cz = Lz / C->ncz;
    long nc = (long)C->ncx * C->ncy * C->ncz;
    C->head = malloc(sizeof(int) * nc);
    C->next = malloc(sizeof(int) * (np > 0 ? np : 1));
    for (long i = 0; i < nc; ++i)
        C->head[i] = -1;
    for (int p = np - 1; p >= 0; --p) {
        int i = cell_coord(x[3 * p], C->cx, C->ncx);
        int j = cell_coord(x[3 * p + 1], C->cy, C->ncy);
        int k = cell_coord(x[3 * p + 2], C->cz, C->ncz);
        long c = ((long)k * C->ncy + j) * C->ncx + i;
        C->next[p] = C->head[c];
        C->head[c] = p;
    }
}

static void cells_free(or_cells *C)
{
    free(C->head);
    free(C->next);
}

/* Cells c - 1, c, c + 1 of a periodic axis of n cells, each listed once. */
static int neighbour_cells(int c, int n, int out[3])
{
    int k = 0;
    for (int d = -1; d <= 1; ++d) {
        int v = (int)wrap_index(c + d, n), seen = 0;
        for (int e = 0; e < k; ++e)
            seen |= out[e] == v;
        if (!seen)
            out[k++] = v;
    }
    return k;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Partners of particle p in canonical order: particle partners ascending,
 * then the bottom wall (-1), then the top wall (-2).  Returns the number of
 * partners, or -1 when more than twelve particles touch p. */
static int find_partners(const or_params *P, int np, const double *x, const or_cells *C, int p,
                         int *list)
{
    int n = 0;
    int buf[64];
    int nb = 0;
    if (!C) {
        for (int q = 0; q < np; ++q)
            if (q != p && in_contact(P, x, p, q)) {
                if (nb == 64)
                    return -1;
                buf[nb++] = q;
            }
    } else {
        int ci = cell_coord(x[3 * p], C->cx, C->ncx);
        int cj = cell_coord(x[3 * p + 1], C->cy, C->ncy);
        int ck = cell_coord(x[3 * p + 2], C->cz, C->ncz);
        /* the distinct neighbour columns along each periodic axis: with fewer
         * than three cells, ci - 1 and ci + 1 wrap onto the same cell, which
         * must be visited once */
        int xs[3], zs[3];
        int nxs = neighbour_cells(ci, C->ncx, xs), nzs = neighbour_cells(ck, C->ncz, zs);
        for (int a = 0; a < nzs; ++a)
            for (int dj = -1; dj <= 1; ++dj)
                for (int b = 0; b < nxs; ++b) {
                    int j = cj + dj;
                    if (j < 0 || j >= C->ncy)
                        continue;
                    int i = xs[b], k = zs[a];
                    for (int q = C->head[((long)k * C->ncy + j) * C->ncx + i]; q >= 0; q = C->next[q])
                        if (q != p && in_contact(P, x, p, q)) {
                            if (nb == 64)
                                return -1;
                            buf[nb++] = q;
                        }
                }
    }
    if (nb > OR_MAX_PP)
        return -1;
    qsort(buf, nb, sizeof(int), cmp_int);
    for (int i = 0; i < nb; ++i)
        list[n++] = buf[i];
    double Ly = P->ny * P->h;
    if (x[3 * p + 1] < P->R)
        list[n++] = OR_WALL_BOTTOM;
    if (Ly - x[3 * p + 1] < P->R)
        list[n++] = OR_WALL_TOP;
    return n;
}

static int check_domain(const or_params *P, int np, const double *x)
{
    double L[3] = {P->nx * P->h, P->ny * P->h, P->nz * P->h};
    for (int p = 0; p < np; ++p)
        for (int a = 0; a < 3; ++a) {
            double v = x[3 * p + a];
            if (!isfinite(v))
                return OR_ENONFINITE;
            if (a == 1 ? (v < 0.0 || v > L[1]) : (v < 0.0 || v >= L[a]))
                return OR_EDOMAIN;
        }
    return OR_OK;
}

/* Canonical contact list: one row (i, j) per contact with i < j for particle
 * pairs, and (i, -1) / (i, -2) for the bottom / top wall; rows ordered by i,
 * then particle partners ascending, then bottom wall, then top wall.  When
 * more than cap rows exist nothing beyond cap is written, *n_out receives
 * the full count and the return code is OR_ECAPACITY. */
int or_contacts(const or_params *P, int32_t np, const double *x, int32_t *pairs, int64_t cap,
                int64_t *n_out)
{
    int rc = check_domain(P, np, x);
    if (rc)
        return rc;
    or_cells C, *Cp = NULL;
    if (P->use_cells) {
        cells_build(P, np, x, &C);
        Cp = &C;
    }
    int64_t n = 0;
    int list[OR_SLOTS];
    for (int p = 0; p < np && rc == OR_OK; ++p) {
        int k = find_partners(P, np, x, Cp, p, list);
        if (k < 0) {
            rc = OR_ECAPACITY;
            break;
        }
        for (int s = 0; s < k; ++s) {
            if (list[s] >= 0 && list[s] < p)
                continue;
            if (n < cap) {
                pairs[2 * n] = p;
                pairs[2 * n + 1] = list[s];
            }
            ++n;
        }
    }
    if (Cp)
        cells_free(Cp);
    *n_out = n;
    if (rc == OR_OK && n > cap)
        rc = OR_ECAPACITY;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Bed and flying particles (sec. 4.3.1, step (1)).  A particle in the       */
/* bottom layer (centre below one diameter, y < 2R) is a bed particle, and   */
/* so is every particle in contact with a bed particle, directly or through  */
/* other bed particles; the rest are flying.  The detection is the paper's  */
/* iteration: sweep over the particles, marking each one that is in the     */
/* bottom layer or touches a particle already marked, and count the marks;  */
/* repeat until the count stops changing.  Contacts are those of (A.3), the */
/* partner lists of find_partners (the lists do not change during the      */
/* sweeps, so they are formed once).                                        */
/* flags[np] (out): 1 bed, 0 flying; *n_bed (out).  Return codes as         */
/* or_contacts.                                                              */
/* ------------------------------------------------------------------------ */
int or_bed_flags(const or_params *P, int32_t np, const double *x, int32_t *flags, int64_t *n_bed)
{
    int rc = check_domain(P, np, x);
    if (rc)
        return rc;
    or_cells C, *Cp = NULL;
    if (P->use_cells) {
        cells_build(P, np, x, &C);
        Cp = &C;
    }
    int32_t *part = malloc(sizeof(int32_t) * OR_SLOTS * (np > 0 ? np : 1));
    int32_t *npart = malloc(sizeof(int32_t) * (np > 0 ? np : 1));
    for (int p = 0; p < np && rc == OR_OK; ++p) {
        int k = find_partners(P, np, x, Cp, p, &part[OR_SLOTS * p]);
        if (k < 0)
            rc = OR_ECAPACITY;
        npart[p] = k;
    }
    if (Cp)
        cells_free(Cp);
    int64_t N_bed = 0, N_temp;
    if (rc == OR_OK) {
        for (int p = 0; p < np; ++p)
            flags[p] = 0;
        do {
            N_temp = N_bed;
            N_bed = 0;
            for (int i = 0; i < np; ++i) {
                int bed = x[3 * i + 1] < 2.0 * P->R;
                for (int s = 0; s < npart[i] && !bed; ++s) {
                    int q = part[OR_SLOTS * i + s];
                    if (q >= 0 && flags[q])
                        bed = 1;
                }
                flags[i] = bed;
                N_bed += bed;
            }
        } while (N_bed != N_temp);
    }
    *n_bed = N_bed;
    free(part);
    free(npart);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Contact history (sec. 3.4, memory optimisation).  M_temp holds the        */
/* partners of p at the previous (sub)step with their u_in and delta_t; M_p  */
/* the partners now.  For each partner now: if it is found in M_temp the     */
/* collision is an existing one (u_in inherited, delta_t advanced from the   */
/* stored value); otherwise it is new (u_in recorded, delta_t initialised).  */
/* Partners of M_temp that are not found now have finished: their data are   */
/* dropped (reset).  src[c] receives the M_temp slot of new partner c, or -1.*/
/* ------------------------------------------------------------------------ */
void or_history_match(int32_t n_old, const int32_t *old_id, int32_t n_new, const int32_t *new_id,
                      int32_t *src)
{
    for (int c = 0; c < n_new; ++c) {
        src[c] = -1;
        for (int s = 0; s < n_old; ++s)
            if (old_id[s] == new_id[c]) {
                src[c] = s;
                break;
            }
    }
}

/* Damping coefficient of the linear spring-dashpot giving restitution e for
 * effective mass m_eff (reading: the linear law with fixed stiffness). */
static double damping(double k, double e, double m_eff)
{
    double le = log(e);
    return -2.0 * le * sqrt(m_eff * k) / sqrt(M_PI * M_PI + le * le);
}

/* Coefficients of one contact of effective mass m_eff.
 * Model 0: the given stiffness k_n, d_n for restitution e_n, and the
 * tangential pair as fixed fractions of the normal one.
 * Model 1 (reading of the collision-time calibration of sec. 2.1 and 4.1,
 * T_c = 10 dt_f, for the linear spring-dashpot): m x'' + d x' + k x = 0 from
 * x = 0 with speed v lasts T_c = pi / sqrt(k/m - (d/2m)^2) and leaves with
 * speed e v, e = exp(-d T_c / (2m)), so
 *     d = -2 m ln(e) / T_c,   k = m (pi^2 + ln^2 e) / T_c^2,
 * with m = m_eff and e = e_n for the normal pair, and m = (2/7) m_eff (the
 * effective mass of a solid sphere's contact point under a tangential force)
 * and e = e_t for the tangential pair: a contact that sticks throughout
 * returns its tangential contact-point velocity with restitution e_t. */
static void contact_coeffs(const or_params *P, double m_eff, double *kn, double *dn, double *kt,
                           double *dt)
{
    if (P->contact_model == 1) {
        double Tc = P->t_c, ln_n = log(P->e_n), ln_t = log(P->e_t), mt = (2.0 / 7.0) * m_eff;
        *dn = -2.0 * m_eff * ln_n / Tc;
        *kn = m_eff * (M_PI * M_PI + ln_n * ln_n) / (Tc * Tc);
        *dt = -2.0 * mt * ln_t / Tc;
        *kt = mt * (M_PI * M_PI + ln_t * ln_t) / (Tc * Tc);
    } else {
        *kn = P->k_n;
        *dn = damping(P->k_n, P->e_n, m_eff);
        *kt = P->kt_ratio * *kn;
        *dt = P->dt_ratio * *dn;
    }
}

static double dot3(const double a[3], const double b[3])
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

/* Force and torque of one contact acting on particle p (Appendix A and eqs.
 * 9-10, without lubrication).  q >= 0: particle partner, -1 / -2: walls.
 * dprev: stored tangential displacement (zero for a new contact); on return
 * dnew holds the advanced displacement.  uin_out receives |u_cp . n|. */
static void contact_force(const or_params *P, const double *x, const double *u, const double *om,
                          int p, int q, const double dprev[3], double dnew[3], double F[3],
                          double T[3], double *uin_out)
{
    const double R = P->R;
    const double m = P->rho_p * (4.0 / 3.0) * M_PI * R * R * R;
    double n[3], xi, ucp[3], m_eff;
    if (q >= 0) {
        double d[3];
        separation(P, x, p, q, d);
        double dist = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
        for (int a = 0; a < 3; ++a)
            n[a] = d[a] / dist;                                   /* (A.1) */
        xi = 2.0 * R - dist;                                      /* -(A.3) */
        double ws[3], wxn[3];
        for (int a = 0; a < 3; ++a)
            ws[a] = om[3 * p + a] + om[3 * q + a];
        cross(ws, n, wxn);
        for (int a = 0; a < 3; ++a)                                /* (A.5) */
            ucp[a] = (u[3 * p + a] - u[3 * q + a]) + R * wxn[a];
        m_eff = 0.5 * m;
    } else {
        double Ly = P->ny * P->h;
        n[0] = 0.0;
        n[2] = 0.0;
        if (q == OR_WALL_BOTTOM) {
            n[1] = -1.0;                                           /* (A.2) */
            xi = R - x[3 * p + 1];                                 /* -(A.4) */
        } else {
            n[1] = 1.0;
            xi = R - (Ly - x[3 * p + 1]);
        }
        double wxn[3];
        cross(&om[3 * p], n, wxn);
        for (int a = 0; a < 3; ++a)                                /* (A.6) */
            ucp[a] = u[3 * p + a] + R * wxn[a];
        m_eff = m;
    }
    double un = dot3(ucp, n);                                      /* (A.7) */
    double ut[3];
    for (int a = 0; a < 3; ++a)                                    /* (A.8) */
        ut[a] = ucp[a] - un * n[a];
    *uin_out = fabs(un);

    double kn, dn, kt, dt;
    contact_coeffs(P, m_eff, &kn, &dn, &kt, &dt);
    const double dtp = P->dt_f / P->n_sub;

    /* tangential displacement: rotate the stored one onto the tangent plane
     * keeping its length, then advance with the tangential velocity
     * (A.9)-(A.11); a zero rotated vector stays zero. */
    double dn_ = dot3(dprev, n), dtil[3], dhat[3];
    for (int a = 0; a < 3; ++a)
        dtil[a] = dprev[a] - dn_ * n[a];
    double lt = sqrt(dot3(dtil, dtil)), lp = sqrt(dot3(dprev, dprev));
    for (int a = 0; a < 3; ++a)
        dhat[a] = lt > 0.0 ? (lp / lt) * dtil[a] : 0.0;
    for (int a = 0; a < 3; ++a)
        dnew[a] = dhat[a] + dtp * ut[a];

    /* linear spring-dashpot: normal force, tangential force, Coulomb cap */
    double fn = kn * xi + dn * un;
    double Fn[3], Ft[3];
    for (int a = 0; a < 3; ++a) {
        Fn[a] = -fn * n[a];
        Ft[a] = -kt * dnew[a] - dt * ut[a];
    }
    double FN = fn > 0.0 ? fn : 0.0;
    double lft = sqrt(dot3(Ft, Ft));
    if (lft > P->mu * FN) {
        double sc = lft > 0.0 ? P->mu * FN / lft : 0.0;
        for (int a = 0; a < 3; ++a) {
            Ft[a] = sc * Ft[a];
            dnew[a] = -(Ft[a] + dt * ut[a]) / kt;
        }
    }
    double nxF[3];
    cross(n, Ft, nxF);
    for (int a = 0; a < 3; ++a) {
        F[a] = Fn[a] + Ft[a];
        T[a] = R * nxF[a];                                         /* eq. 10 */
    }
}

/* ------------------------------------------------------------------------ */
/* Particle phase: n_sub substeps of dt_p = dt_f / n_sub (sec. 2.1).  Each  */
/* substep finds the contacts from the current positions, forms the contact  */
/* force and torque (eqs. 9-10), then advances every sphere by the Newton-   */
/* Euler equations (eqs. 7-8) with the hydrodynamic force and torque held    */
/* fixed over the step.  Reading: symplectic Euler (velocity first, then     */
/* position with the new velocity), buoyant weight (rho_p - rho_f) V g, and  */
/* x, z wrapped into [0, L).  Fc, Tc (nullable) receive the contact force    */
/* and torque of the last substep.                                           */
/* ------------------------------------------------------------------------ */
int or_dem(const or_params *P, int32_t np, double *x, double *u, double *om, const double *Fh,
           const double *Th, int32_t *hp, double *hd, double *hu, int32_t *hc, double *Fc_out,
           double *Tc_out)
{
    int rc = check_domain(P, np, x);
    if (rc)
        return rc;
    const double R = P->R;
    const double V = (4.0 / 3.0) * M_PI * R * R * R;
    const double m = P->rho_p * V, I = 0.4 * m * R * R;
    const double dtp = P->dt_f / P->n_sub;
    const double Lx = P->nx * P->h, Lz = P->nz * P->h;
    int32_t *np_id = malloc(sizeof(int32_t) * OR_SLOTS * (np > 0 ? np : 1));
    double *np_d = malloc(sizeof(double) * 3 * OR_SLOTS * (np > 0 ? np : 1));
    double *np_u = malloc(sizeof(double) * OR_SLOTS * (np > 0 ? np : 1));
    int32_t *np_c = malloc(sizeof(int32_t) * (np > 0 ? np : 1));
    double *Fc = malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
    double *Tc = malloc(sizeof(double) * 3 * (np > 0 ? np : 1));

    for (int sub = 0; sub < P->n_sub && rc == OR_OK; ++sub) {
        or_cells C, *Cp = NULL;
        if (P->use_cells) {
            cells_build(P, np, x, &C);
            Cp = &C;
        }
        for (int p = 0; p < np; ++p) {
            int list[OR_SLOTS], src[OR_SLOTS];
            int k = find_partners(P, np, x, Cp, p, list);
            if (k < 0) {
                rc = OR_ECAPACITY;
                break;
            }
            or_history_match(hc[p], &hp[OR_SLOTS * p], k, list, src);
            double sF[3] = {0, 0, 0}, sT[3] = {0, 0, 0};
            for (int c = 0; c < k; ++c) {
                double dprev[3] = {0, 0, 0}, dnew[3], F[3], T[3], uin;
                if (src[c] >= 0)
                    for (int a = 0; a < 3; ++a)
                        dprev[a] = hd[3 * (OR_SLOTS * p + src[c]) + a];
                contact_force(P, x, u, om, p, list[c], dprev, dnew, F, T, &uin);
                for (int a = 0; a < 3; ++a) {
                    sF[a] += F[a];
                    sT[a] += T[a];
                    np_d[3 * (OR_SLOTS * p + c) + a] = dnew[a];
                }
                np_id[OR_SLOTS * p + c] = list[c];
                np_u[OR_SLOTS * p + c] = src[c] >= 0 ? hu[OR_SLOTS * p + src[c]] : uin;
            }
            np_c[p] = k;
            for (int a = 0; a < 3; ++a) {
                Fc[3 * p + a] = sF[a];
                Tc[3 * p + a] = sT[a];
            }
        }
        if (Cp)
            cells_free(Cp);
        if (rc)
            break;
        for (int p = 0; p < np; ++p) {
            for (int a = 0; a < 3; ++a) {
                double Ftot = (Fh[3 * p + a] + (P->rho_p - P->rho_f) * V * P->g[a]) + Fc[3 * p + a];
                u[3 * p + a] += dtp * Ftot / m;
                om[3 * p + a] += dtp * (Th[3 * p + a] + Tc[3 * p + a]) / I;
                x[3 * p + a] += dtp * u[3 * p + a];
            }
            double L[3] = {Lx, 0.0, Lz};
            for (int a = 0; a < 3; a += 2) {
                if (x[3 * p + a] < 0.0)
                    x[3 * p + a] += L[a];
                if (x[3 * p + a] >= L[a])
                    x[3 * p + a] -= L[a];
            }
            /* M_temp <- M_p */
            hc[p] = np_c[p];
            for (int s = 0; s < OR_SLOTS; ++s) {
                int has = s < np_c[p];
                hp[OR_SLOTS * p + s] = has ? np_id[OR_SLOTS * p + s] : 0;
                hu[OR_SLOTS * p + s] = has ? np_u[OR_SLOTS * p + s] : 0.0;
                for (int a = 0; a < 3; ++a)
                    hd[3 * (OR_SLOTS * p + s) + a] = has ? np_d[3 * (OR_SLOTS * p + s) + a] : 0.0;
            }
        }
        rc = check_domain(P, np, x);
        for (int p = 0; p < np && rc == OR_OK; ++p)
            for (int a = 0; a < 3; ++a)
                if (!isfinite(u[3 * p + a]) || !isfinite(om[3 * p + a]))
                    rc = OR_ENONFINITE;
    }
    if (Fc_out)
        memcpy(Fc_out, Fc, sizeof(double) * 3 * np);
    if (Tc_out)
        memcpy(Tc_out, Tc, sizeof(double) * 3 * np);
    free(np_id);
    free(np_d);
    free(np_u);
    free(np_c);
    free(Fc);
    free(Tc);
    return rc;
}

/* One particle-phase step: immersed-boundary forcing at the current particle
 * state, then n_sub contact / Newton-Euler substeps with the hydrodynamic
 * force and torque held fixed. */
int or_step(const or_params *P, const double *uhu, const double *uhv, const double *uhw,
            double *fu, double *fv, double *fw, int32_t np, double *x, double *u, double *om,
            const double *F0, int32_t *hp, double *hd, double *hu, int32_t *hc, double *Fh,
            double *Th, double *slip, int32_t *iters)
{
    int rc = check_domain(P, np, x);
    if (rc)
        return rc;
    rc = or_ib_forcing(P, uhu, uhv, uhw, fu, fv, fw, np, x, u, om, F0, Fh, Th, slip, iters, NULL,
                       NULL, NULL, NULL);
    if (rc)
        return rc;
    return or_dem(P, np, x, u, om, Fh, Th, hp, hd, hu, hc, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Fluid inside the spheres.  Reading of the hydrodynamic force of the       */
/* direct-forcing method (sec. 2.1, eqs. 7-8): besides minus the marker       */
/* forces, the force on a sphere includes the rate of change of the momentum  */
/* of the fluid occupying its volume, rho_f d/dt int_{V_p} u dV (and         */
/* rho_f d/dt int_{V_p} r x u dV for the torque).  The integrals are taken   */
/* by the midpoint rule over the staggered nodes inside the sphere: node n   */
/* of component c (wall faces and nodes outside the fluid excluded) with     */
/* |x_n - x_p| < R (minimum image in x and z), each weighted h^3:            */
/*   inner[p][c]     = h^3 sum_n u_c[n],                                     */
/*   inner[p][3 + a] = h^3 sum_c sum_n eps_{a b c} r_b(x_n) u_c[n],          */
/* r = x_n - x_p.  inner: [np][6].                                            */
/* ------------------------------------------------------------------------ */
int or_inner_fluid(const or_params *P, const double *gu, const double *gv, const double *gw,
                   int32_t np, const double *x, double *inner)
{
    int rc = check_domain(P, np, x);
    if (rc)
        return rc;
    const double *g[3] = {gu, gv, gw};
    const double h = P->h, R = P->R, h3 = h * h * h;
    const double Lx = P->nx * h, Lz = P->nz * h;
    for (int p = 0; p < np; ++p) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int c = 0; c < 3; ++c) {
            double o[3];
            stagger_offset(c, o);
            long lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = (long)floor((x[3 * p + a] - R) / h - o[a]) - 1;
                hi[a] = (long)floor((x[3 * p + a] + R) / h - o[a]) + 1;
            }
            for (long k = lo[2]; k <= hi[2]; ++k)
                for (long j = lo[1]; j <= hi[1]; ++j)
                    for (long i = lo[0]; i <= hi[0]; ++i) {
                        double r[3];
                        r[0] = min_image((i + o[0]) * h - x[3 * p + 0], Lx);
                        r[1] = (j + o[1]) * h - x[3 * p + 1];
                        r[2] = min_image((k + o[2]) * h - x[3 * p + 2], Lz);
                        if (!((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2] < R * R))
                            continue;
                        long nidx = node_index(P, c, i, j, k);
                        if (nidx < 0)
                            continue;
                        double uc = g[c][nidx];
                        acc[c] += uc;
                        /* (r x e_c u_c): component a = eps_{a b c} r_b u_c */
                        if (c == 0) {
                            acc[4] += r[2] * uc;
                            acc[5] -= r[1] * uc;
                        } else if (c == 1) {
                            acc[3] -= r[2] * uc;
                            acc[5] += r[0] * uc;
                        } else {
                            acc[3] += r[1] * uc;
                            acc[4] -= r[0] * uc;
                        }
                    }
        }
        for (int k = 0; k < 6; ++k)
            inner[6 * p + k] = h3 * acc[k];
    }
    return OR_OK;
}

/* One step with the inner-fluid term and a per-call forcing coefficient
 * (the alpha_k of the Runge-Kutta substep, eq. 4): the forcing with alpha
 * dt_f; then F_h += rho_f (I_new - I_prev) / (alpha dt_f) and T_h likewise,
 * with I_new the integrals of u** = u-hat + alpha dt_f f (the field after the
 * forcing) over the spheres at their current positions and I_prev the
 * caller's integrals of the previous call (inner_prev, [np][6], NULL: no
 * inner-fluid term); inner_out (nullable) receives I_new.  advance = 0
 * stops after the forcing (the spheres and the history are not moved, as in
 * a Runge-Kutta substep that is not the last); otherwise the n_sub contact
 * and Newton-Euler substeps follow. */
int or_step_ex(const or_params *P0, double alpha, int advance, const double *uhu,
               const double *uhv, const double *uhw, double *fu, double *fv, double *fw,
               int32_t np, double *x, double *u, double *om, const double *F0, int32_t *hp,
               double *hd, double *hu, int32_t *hc, double *Fh, double *Th, double *slip,
               int32_t *iters, const double *inner_prev, double *inner_out)
{
    or_params P = *P0;
    P.alpha = alpha;
    int rc = check_domain(&P, np, x);
    if (rc)
        return rc;
    const long nu = (long)P.wnz * P.ny * P.wnx, nv = (long)P.wnz * (P.ny + 1) * P.wnx;
    double *us[3] = {NULL, NULL, NULL};
    if (inner_prev || inner_out) {
        us[0] = malloc(sizeof(double) * nu);
        us[1] = malloc(sizeof(double) * nv);
        us[2] = malloc(sizeof(double) * nu);
    }
    rc = or_ib_forcing(&P, uhu, uhv, uhw, fu, fv, fw, np, x, u, om, F0, Fh, Th, slip, iters, NULL,
                       us[0], us[1], us[2]);
    if (rc == OR_OK && (inner_prev || inner_out)) {
        double *inner = malloc(sizeof(double) * 6 * (np > 0 ? np : 1));
        rc = or_inner_fluid(&P, us[0], us[1], us[2], np, x, inner);
        const double adt = P.alpha * P.dt_f;
        for (int p = 0; p < np && rc == OR_OK && inner_prev; ++p)
            for (int a = 0; a < 3; ++a) {
                Fh[3 * p + a] += P.rho_f * (inner[6 * p + a] - inner_prev[6 * p + a]) / adt;
                Th[3 * p + a] += P.rho_f * (inner[6 * p + 3 + a] - inner_prev[6 * p + 3 + a]) / adt;
            }
        if (inner_out)
            memcpy(inner_out, inner, sizeof(double) * 6 * np);
        free(inner);
    }
    for (int c = 0; c < 3; ++c)
        free(us[c]);
    if (rc || !advance)
        return rc;
    return or_dem(&P, np, x, u, om, Fh, Th, hp, hd, hu, hc, NULL, NULL);
}

