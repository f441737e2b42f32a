/*
 * FP64 CPU oracle of the hybrid lattice-Boltzmann / immersed-boundary method of
 * Coclite, Pascazio, de Tullio and Decuzzi, "Predicting the vascular adhesion of
 * deformable drug carriers in narrow capillaries traversed by blood cells"
 * (arXiv 2210.06043).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header, table
 * or helper with the HIP library, and the HIP library never calls it.
 *
 * Everything is double precision with plain loops, in the order the method
 * states its steps:
 *   S1  pull streaming with halfway bounce-back walls            (Eq. 1; Sec. 2.2 walls)
 *   S2  pre-coupling moments, pressure, viscous stress per node   (Sec. 2.1 moments; Eqs. 5-6)
 *   S3  membrane geometry                                         (Sec. 2.3)
 *   S4  cosine-delta interpolation to vertices and probes         (Sec. 2.2, 2.6)
 *   S5  membrane, interaction, bond and load forces               (Eqs. 7-15)
 *   S6  structure integration                                     (Eqs. 16-20)
 *   S7  direct forcing and spreading                              (Sec. 2.2)
 *   S8  BGK collision with Guo forcing                            (Eqs. 1, 2, 4)
 *   S9  ligand-receptor bond kinetics                             (Sec. 2.5)
 *
 * Readings taken where the paper is silent or garbled are listed next to the
 * code they affect (walls instead of Zou-He ends, cosine delta instead of MLS,
 * direct forcing, probe clamping, bond-rate law).  Every function below is
 * pinned by the not-gpu tests except where its header says "parity unpinned".
 *
 * Populations are stored shifted, h_i = f_i - w_i, so that the rest state is
 * zero; this changes no arithmetic of the method.
 *
 * Loops whose iterations are independent (streaming, the per-node moments and
 * collision, the repulsion received by each vertex, the read-out) are split
 * over OpenMP threads; every value is still computed by the same expressions
 * in the same order, so the results do not depend on the thread count.  The
 * scatter of the spreading and all sums stay serial.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DEFORMABLE 0
#define ORC_RIGID 1
#define ORC_FIXED 2

/* ---- D2Q9 lattice, Eq. (3) and the weights given beneath it ---------------- */
/* Velocities in the order of Eq. (3): rest, the axis directions at angles
 * (i-1)*pi/2, the diagonals at angles (2i-9)*pi/4 with length sqrt(2).       */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WQ[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
/* index of the velocity opposite to i */
static int opposite(int i) {
    for (int k = 0; k < 9; k++)
        if (EX[k] == -EX[i] && EY[k] == -EY[i]) return k;
    return -1;
}

void orc_lattice_tables(int *ex, int *ey, double *w) {
    for (int i = 0; i < 9; i++) { ex[i] = EX[i]; ey[i] = EY[i]; w[i] = WQ[i]; }
}

/* ---- Equilibrium, Eq. (2), with c_s^2 = 1/3 ---------------------------------
 * f_eq = w rho [1 + e.u/cs2 + (e.u)^2/(2 cs2^2) - u^2/(2 cs2)], returned shifted
 * by w: with rho = 1 + drho, h_eq = f_eq - w = w [drho + rho (e.u/cs2 +
 * (e.u)^2/(2 cs2^2) - u^2/(2 cs2))], written so that the subtraction of w is
 * exact rather than rounded.                                                   */
void orc_heq(double drho, double ux, double uy, double *heq) {
    const double cs2 = 1.0 / 3.0;
    double rho = 1.0 + drho;
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy;
        heq[i] = WQ[i] * (drho + rho * (eu / cs2 + eu * eu / (2 * cs2 * cs2) - uu / (2 * cs2)));
    }
}

/* ---- Guo forcing term, Eq. (4) -----------------------------------------------
 * F_i = (1 - 1/(2 tau)) w_i [ (e_i - u)/cs2 + (e_i.u) e_i / cs2^2 ] . F        */
void orc_guo(double tau, double ux, double uy, double Fx, double Fy, double *Fi) {
    const double cs2 = 1.0 / 3.0;
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy;
        double ax = (EX[i] - ux) / cs2 + eu * EX[i] / (cs2 * cs2);
        double ay = (EY[i] - uy) / cs2 + eu * EY[i] / (cs2 * cs2);
        Fi[i] = (1.0 - 1.0 / (2.0 * tau)) * WQ[i] * (ax * Fx + ay * Fy);
    }
}

/* ---- 4-point cosine delta kernel ---------------------------------------------
 * phi(r) = (1 + cos(pi r / 2)) / 4 for |r| <= 2, else 0.  Used in place of the
 * moving-least-squares transfer the paper cites (Sec. 2.2).                    */
double orc_phi(double r) {
    if (fabs(r) >= 2.0) return 0.0;
    return 0.25 * (1.0 + cos(M_PI * r / 2.0));
}

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) -----------------------
 * Written from the published definition: ten rounds of two 32x32->64 bit
 * multiplications with the round constants of the paper, the key advanced by
 * the Weyl increments between rounds.                                          */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The uniform draw of bond site s at step n: word 0 of Philox4x32-10 with key
 * (seed low, seed high) and counter (n low, s, n high, 0), top 24 bits scaled
 * by 2^-24.                                                                    */
double orc_uniform(uint64_t seed, int64_t n, int32_t s) {
    uint32_t ctr[4] = {(uint32_t)((uint64_t)n & 0xffffffffu), (uint32_t)s,
                       (uint32_t)((uint64_t)n >> 32), 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    return (double)(o[0] >> 8) * (1.0 / 16777216.0);
}

/* ---- simulation state -------------------------------------------------------- */
typedef struct {
    int kind, n, tag;
    double ks, kb, ka, pref, rho_r;
    double *x, *y;        /* x^n */
    double *dxm, *dym;    /* x^n - x^{n-1} */
    double *l0, *th0;     /* rest element lengths, rest turning angles */
    double A0, P0;        /* rest area, initial perimeter */
    double vmass;         /* per-vertex mass of a deformable body */
    double mass, inertia; /* rigid body */
    double xc, yc, phi, ucx, ucy, ucx_m, ucy_m, om, om_m;
    double *rx0, *ry0;    /* rigid: vertex offsets from the centroid at t = 0 */
    /* per-step work */
    double *usx, *usy;                  /* u* at vertices (S4) */
    double *pp, *psxx, *psxy, *psyy;    /* pressure and viscous stress at probes (S4) */
    double *fx, *fy;                    /* total Lagrangian force (S5) */
    double *Ux, *Uy;                    /* target velocity U^{n+1} (S6) */
    double *xn, *yn;                    /* copy of x^n for spreading (S7) */
    /* bonds */
    int ns;
    int *host;
    double *frac;
    unsigned char *bound;
    double *anchor;
    double sigma, ycr, yeq, kf, kr0, lb;
    uint64_t seed;
} orc_body;

typedef struct {
    int nx, ny, walls;
    double tau, gx, gy;
    double *A;                 /* post-collision populations, [9][ny][nx] */
    double *h;                 /* streamed populations (S1) */
    double *drho, *j0x, *j0y;  /* S2 moments (j0 = sum h e, without forcing) */
    double *usx, *usy;         /* u* = (j0 + g/2)/rho */
    double *sxx, *sxy, *syy;   /* viscous stress -(1-1/2tau) Pi_neq */
    double *fibx, *fiby;       /* spread IB force (S7) */
    int nb, cap;
    orc_body *b;
    double rep_pref, rep_cut, rep_dmin, probe_dist;
    int velocity_wall;         /* 1: odd image across the walls (default); 0: wall nodes at rest */
    int64_t step;
    /* smallest |draw - P| / P over the bond decisions taken (P > 0), and
     * smallest |gap - y_cr| over the formation decisions that the gap
     * decided: a code that computes P or the gap with a smaller relative or
     * absolute error takes the same decisions */
    double min_margin_p, min_margin_gap;
    int64_t flips;   /* bond state changes so far */
    int flags; /* bit0: a vertex left the rows [-1, ny] */
} orc_sim;

#define IDX(s, q, j, i) (((size_t)(q) * (s)->ny + (size_t)(j)) * (s)->nx + (size_t)(i))

static double *dz(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

orc_sim *orc_create(int nx, int ny, double tau, double gx, double gy, int walls) {
    /* with walls a stencil's mirrored rows must be fluid rows: ny >= 4 */
    if (nx < 1 || ny < 1 || !(tau > 0.5) || (walls != 0 && walls != 3) || (walls && ny < 4)) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->nx = nx; s->ny = ny; s->tau = tau; s->gx = gx; s->gy = gy; s->walls = walls;
    size_t N = (size_t)nx * ny;
    s->A = dz(9 * N); s->h = dz(9 * N);
    s->drho = dz(N); s->j0x = dz(N); s->j0y = dz(N); s->usx = dz(N); s->usy = dz(N);
    s->sxx = dz(N); s->sxy = dz(N); s->syy = dz(N); s->fibx = dz(N); s->fiby = dz(N);
    s->cap = 16; s->b = (orc_body *)calloc(s->cap, sizeof(orc_body));
    /* interaction constants: Eq. (12) prefactor, minimum distance dx, probe 1.2 dx */
    s->rep_pref = 1.0e-4 / (8.0 * sqrt(2.0));
    s->rep_cut = 1.0; s->rep_dmin = 0.1; s->probe_dist = 1.2;
    s->velocity_wall = 1;
    s->min_margin_p = INFINITY;
    s->min_margin_gap = INFINITY;
    return s;
}

static void free_body(orc_body *b) {
    double **arrs[] = {&b->x, &b->y, &b->dxm, &b->dym, &b->l0, &b->th0, &b->rx0, &b->ry0,
                       &b->usx, &b->usy, &b->pp, &b->psxx, &b->psxy, &b->psyy, &b->fx, &b->fy,
                       &b->Ux, &b->Uy, &b->xn, &b->yn, &b->frac, &b->anchor};
    for (size_t k = 0; k < sizeof(arrs) / sizeof(arrs[0]); k++) free(*arrs[k]);
    free(b->host); free(b->bound);
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    free(s->A); free(s->h); free(s->drho); free(s->j0x); free(s->j0y); free(s->usx); free(s->usy);
    free(s->sxx); free(s->sxy); free(s->syy); free(s->fibx); free(s->fiby);
    for (int k = 0; k < s->nb; k++) free_body(&s->b[k]);
    free(s->b); free(s);
}

/* Reading of the velocity coupling at the walls: 1 = odd image (default),
 * 0 = rows beyond the wall are wall nodes at rest (earlier reading).       */
void orc_set_velocity_wall(orc_sim *s, int image) { s->velocity_wall = image ? 1 : 0; }

void orc_set_interactions(orc_sim *s, double rep_pref, double rep_cut, double probe_dist) {
    s->rep_pref = rep_pref; s->rep_cut = rep_cut; s->probe_dist = probe_dist;
}

/* Initial populations: equilibrium at drho = 0 and the given x-velocity per
 * row (NULL: fluid at rest).                                                   */
void orc_init_flow(orc_sim *s, const double *ux_of_y) {
    double heq[9];
    for (int j = 0; j < s->ny; j++) {
        orc_heq(0.0, ux_of_y ? ux_of_y[j] : 0.0, 0.0, heq);
        for (int i = 0; i < s->nx; i++)
            for (int q = 0; q < 9; q++) s->A[IDX(s, q, j, i)] = heq[q];
    }
}

void orc_get_populations(const orc_sim *s, double *out) {
    memcpy(out, s->A, sizeof(double) * 9 * (size_t)s->nx * s->ny);
}
void orc_set_populations(orc_sim *s, const double *in) {
    memcpy(s->A, in, sizeof(double) * 9 * (size_t)s->nx * s->ny);
}
int64_t orc_get_step(const orc_sim *s) { return s->step; }
double orc_min_margin(const orc_sim *s) {
    return s->min_margin_p < s->min_margin_gap ? s->min_margin_p : s->min_margin_gap;
}
void orc_margins(const orc_sim *s, double *out2) { out2[0] = s->min_margin_p; out2[1] = s->min_margin_gap; }
void orc_reset_margins(orc_sim *s) { s->min_margin_p = INFINITY; s->min_margin_gap = INFINITY; s->flips = 0; }
int64_t orc_bond_flips(const orc_sim *s) { return s->flips; }
void orc_set_step(orc_sim *s, int64_t n) { s->step = n; }
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }
int orc_flags(const orc_sim *s) { return s->flags; }

/* ---- S1: pull streaming, Eq. (1) ---------------------------------------------
 * h_i(x) = A_i(x - e_i); x is periodic; with walls a link that crosses y = -1/2
 * or y = ny - 1/2 is reflected in place: h_i(x) = A_opp(i)(x) (halfway
 * bounce-back, the no-slip wall of the capillary, Sec. 3.1).                  */
static void stream(const orc_sim *s, const double *A, double *h) {
    for (int q = 0; q < 9; q++) {
        int oq = opposite(q);
#pragma omp parallel for schedule(static)
        for (int j = 0; j < s->ny; j++)
            for (int i = 0; i < s->nx; i++) {
                int si = ((i - EX[q]) % s->nx + s->nx) % s->nx;
                int sj = j - EY[q];
                if (sj < 0 || sj >= s->ny) {
                    if (s->walls) { h[IDX(s, q, j, i)] = A[IDX(s, oq, j, i)]; continue; }
                    sj = (sj % s->ny + s->ny) % s->ny;
                }
                h[IDX(s, q, j, i)] = A[IDX(s, q, sj, si)];
            }
    }
}

/* ---- S2: moments of the streamed populations (Sec. 2.1, Eqs. 5-6) ------------
 * drho = sum h; j0 = sum h e; u* = (j0 + g/2)/rho (the fluid velocity before
 * the coupling force is known); p = cs2 drho; sigma = -(1 - 1/2tau) Pi_neq with
 * Pi_neq = sum e e (h - h_eq(drho, u*)).                                      */
static void node_moments(orc_sim *s) {
    const long N = (long)s->nx * s->ny;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < N; k++) {
        double hq[9], heq[9];
        double dr = 0, jx = 0, jy = 0;
        for (int q = 0; q < 9; q++) {
            hq[q] = s->h[(size_t)q * (size_t)N + (size_t)k];
            dr += hq[q]; jx += hq[q] * EX[q]; jy += hq[q] * EY[q];
        }
        double rho = 1.0 + dr;
        double ux = (jx + 0.5 * s->gx) / rho, uy = (jy + 0.5 * s->gy) / rho;
        orc_heq(dr, ux, uy, heq);
        double pxx = 0, pxy = 0, pyy = 0;
        for (int q = 0; q < 9; q++) {
            double d = hq[q] - heq[q];
            pxx += EX[q] * EX[q] * d; pxy += EX[q] * EY[q] * d; pyy += EY[q] * EY[q] * d;
        }
        double c = -(1.0 - 1.0 / (2.0 * s->tau));
        s->drho[k] = dr; s->j0x[k] = jx; s->j0y[k] = jy; s->usx[k] = ux; s->usy[k] = uy;
        s->sxx[k] = c * pxx; s->sxy[k] = c * pxy; s->syy[k] = c * pyy;
    }
}

/* ---- S4 helper: stencil of the cosine kernel -----------------------------------
 * Nodes i0..i0+3, j0..j0+3 with i0 = floor(X)-1, j0 = floor(Y)-1; weight
 * W = phi(X-i) phi(Y-j), divided by the sum of the weights.  With walls the
 * point's Y is clamped to [-1, ny] and rows beyond a wall are read in one of
 * two ways (the paper does not say how a stencil that crosses a wall is
 * treated):
 *   STEN_VELOCITY (interpolation of u* to vertices, spreading): the fluid
 *     velocity is continued across the no-slip wall as its odd image, so a
 *     row beyond the wall stands for the fluid row mirrored about the wall
 *     (row -1-j below y = -1/2, row 2 ny - 1 - j above y = ny - 1/2) with
 *     the sign reversed; spreading is the adjoint, so force that lands on a
 *     row beyond the wall reaches the mirrored fluid row negated.  The
 *     interpolated velocity then vanishes on the wall itself.  (The earlier
 *     reading, kept for the tests as velocity_wall = 0, counts the rows
 *     beyond the wall as wall nodes at rest: zero velocity and no force,
 *     with their weight kept in the normalising sum.  With it, the BDF2
 *     target of Eq. (18) and direct forcing amplify a mode of rows 0-1 that
 *     flips sign every step when deformable vertices sit between the wall
 *     and the first fluid row.)
 *   STEN_PROBE (pressure and stress at the probes): the rows beyond the wall
 *     are dropped and the remaining weights renormalised, i.e. the fluid
 *     field is extrapolated.
 * Returns the weights in w[b*4+a] (a along x), the wrapped node indices, and
 * jj[b] (the row a weight applies to; -1 for a dropped row).               */
enum { STEN_VELOCITY = 0, STEN_PROBE = 1 };
static void stencil(orc_sim *s, double X, double Y, int mode, int ii[4], int jj[4], double w[16]) {
    if (s->walls) {
        if (Y < -1.0) Y = -1.0;
        if (Y > (double)s->ny) Y = (double)s->ny;
    }
    int i0 = (int)floor(X) - 1, j0 = (int)floor(Y) - 1;
    double sum = 0;
    for (int b = 0; b < 4; b++) {
        int j = j0 + b;
        int valid = 1;      /* a fluid row */
        double sign = 1.0;
        if (j < 0 || j >= s->ny) {
            if (s->walls) {
                valid = 0;
                if (mode == STEN_VELOCITY && s->velocity_wall == 1) {
                    j = j < 0 ? -1 - j : 2 * s->ny - 1 - j;   /* mirror row across the wall */
                    sign = -1.0;
                }
            } else {
                j = ((j % s->ny) + s->ny) % s->ny;
            }
        }
        int used = valid || sign < 0;
        jj[b] = used ? j : -1;
        for (int a = 0; a < 4; a++) {
            int i = i0 + a;
            ii[a] = ((i % s->nx) + s->nx) % s->nx;
            double ww = orc_phi(X - (double)(i0 + a)) * orc_phi(Y - (double)(j0 + b));
            if (!valid && mode == STEN_PROBE) ww = 0.0;
            sum += ww;
            w[b * 4 + a] = used ? sign * ww : 0.0;
        }
    }
    for (int k = 0; k < 16; k++) w[k] /= sum;
}

/* exported for tests: weights and node indices of the stencil of (X, Y) */
void orc_stencil(orc_sim *s, double X, double Y, int mode, int *ii, int *jj, double *w) {
    stencil(s, X, Y, mode, ii, jj, w);
}

static double interp(orc_sim *s, const double *field, double X, double Y, int mode) {
    int ii[4], jj[4]; double w[16];
    stencil(s, X, Y, mode, ii, jj, w);
    double acc = 0;
    for (int b = 0; b < 4; b++) {
        if (jj[b] < 0) continue;
        for (int a = 0; a < 4; a++) acc += w[b * 4 + a] * field[(size_t)jj[b] * s->nx + ii[a]];
    }
    return acc;
}

/* exported for tests: interpolate a node field [ny][nx] at (X, Y) (mode: STEN_*) */
double orc_interp_field(orc_sim *s, const double *field, double X, double Y, int mode) {
    return interp(s, field, X, Y, mode);
}

/* spread: field(x) += W(x, X) * val, the transpose of the velocity interpolation */
static void spread(orc_sim *s, double *field, double X, double Y, double val) {
    int ii[4], jj[4]; double w[16];
    stencil(s, X, Y, STEN_VELOCITY, ii, jj, w);
    for (int b = 0; b < 4; b++) {
        if (jj[b] < 0) continue;
        for (int a = 0; a < 4; a++) field[(size_t)jj[b] * s->nx + ii[a]] += w[b * 4 + a] * val;
    }
}

/* ---- S3: membrane geometry (Sec. 2.3) --------------------------------------------
 * Element l joins vertex l to vertex l+1 (mod n); t_l = x_{l+1} - x_l, length
 * len_l, outward normal n_l = (t_y, -t_x)/len_l for a counter-clockwise body,
 * vertex normal n_v = normalise(n_{v-1} + n_v), turning angle
 * theta_v = atan2(t_{v-1} x t_v, t_{v-1} . t_v).  Area by Green's theorem
 * (shoelace, with the factor 1/2), taken relative to vertex 0.              */
typedef struct {
    double *tx, *ty, *len, *nlx, *nly, *nvx, *nvy, *th;
    double area, perim, cx, cy;
} geom;

static void geom_alloc(geom *g, int n) {
    g->tx = dz(n); g->ty = dz(n); g->len = dz(n); g->nlx = dz(n); g->nly = dz(n);
    g->nvx = dz(n); g->nvy = dz(n); g->th = dz(n);
}
static void geom_free(geom *g) {
    free(g->tx); free(g->ty); free(g->len); free(g->nlx); free(g->nly);
    free(g->nvx); free(g->nvy); free(g->th);
}

static void geometry(int n, const double *x, const double *y, geom *g) {
    for (int l = 0; l < n; l++) {
        int m = (l + 1) % n;
        g->tx[l] = x[m] - x[l]; g->ty[l] = y[m] - y[l];
        g->len[l] = sqrt(g->tx[l] * g->tx[l] + g->ty[l] * g->ty[l]);
        g->nlx[l] = g->ty[l] / g->len[l]; g->nly[l] = -g->tx[l] / g->len[l];
    }
    for (int v = 0; v < n; v++) {
        int p = (v + n - 1) % n;
        double ax = g->nlx[p] + g->nlx[v], ay = g->nly[p] + g->nly[v];
        double an = sqrt(ax * ax + ay * ay);
        g->nvx[v] = ax / an; g->nvy[v] = ay / an;
        double cr = g->tx[p] * g->ty[v] - g->ty[p] * g->tx[v];
        double dt = g->tx[p] * g->tx[v] + g->ty[p] * g->ty[v];
        g->th[v] = atan2(cr, dt);
    }
    double A = 0, P = 0, Sx = 0, Sy = 0;
    for (int l = 0; l < n; l++) {
        int m = (l + 1) % n;
        double xa = x[l] - x[0], ya = y[l] - y[0], xb = x[m] - x[0], yb = y[m] - y[0];
        double c = xa * yb - xb * ya;
        A += c; Sx += (xa + xb) * c; Sy += (ya + yb) * c;
        P += g->len[l];
    }
    A *= 0.5;
    g->area = A; g->perim = P;
    g->cx = x[0] + Sx / (6.0 * A); g->cy = y[0] + Sy / (6.0 * A);
}

/* polar second moment of area of a polygon about its own centroid */
static double polar_moment(int n, const double *x, const double *y, double cx, double cy) {
    double J = 0;
    for (int l = 0; l < n; l++) {
        int m = (l + 1) % n;
        double xa = x[l] - cx, ya = y[l] - cy, xb = x[m] - cx, yb = y[m] - cy;
        double c = xa * yb - xb * ya;
        J += c * (xa * xa + xa * xb + xb * xb + ya * ya + ya * yb + yb * yb);
    }
    return J / 12.0;
}

/* exported for tests: geometry of a polygon. out = {area, perimeter, cx, cy}
 * and per-vertex turning angle / vertex normal / element length & normal.   */
void orc_polygon(int n, const double *x, const double *y, double *out4, double *th,
                 double *nvx, double *nvy, double *len, double *nlx, double *nly) {
    geom g; geom_alloc(&g, n);
    geometry(n, x, y, &g);
    out4[0] = g.area; out4[1] = g.perim; out4[2] = g.cx; out4[3] = g.cy;
    for (int k = 0; k < n; k++) {
        if (th) th[k] = g.th[k];
        if (nvx) { nvx[k] = g.nvx[k]; nvy[k] = g.nvy[k]; }
        if (len) { len[k] = g.len[k]; nlx[k] = g.nlx[k]; nly[k] = g.nly[k]; }
    }
    geom_free(&g);
}
double orc_polar_moment(int n, const double *x, const double *y, double cx, double cy) {
    return polar_moment(n, x, y, cx, cy);
}

/* ---- bodies ----------------------------------------------------------------------- */
int orc_add_body(orc_sim *s, int kind, int n, const double *xy, const double *xy_rest,
                 double ks, double kb, double ka, double pref, double rho_r, int tag) {
    if (n < 3 || kind < 0 || kind > 2) return -1;
    if (s->nb == s->cap) {
        s->cap *= 2;
        s->b = (orc_body *)realloc(s->b, sizeof(orc_body) * s->cap);
    }
    orc_body *b = &s->b[s->nb];
    memset(b, 0, sizeof(*b));
    b->kind = kind; b->n = n; b->tag = tag;
    b->ks = ks; b->kb = kb; b->ka = ka; b->pref = pref; b->rho_r = rho_r;
    b->x = dz(n); b->y = dz(n); b->dxm = dz(n); b->dym = dz(n); b->l0 = dz(n); b->th0 = dz(n);
    b->rx0 = dz(n); b->ry0 = dz(n); b->usx = dz(n); b->usy = dz(n); b->pp = dz(n);
    b->psxx = dz(n); b->psxy = dz(n); b->psyy = dz(n); b->fx = dz(n); b->fy = dz(n);
    b->Ux = dz(n); b->Uy = dz(n); b->xn = dz(n); b->yn = dz(n);
    for (int v = 0; v < n; v++) { b->x[v] = xy[2 * v]; b->y[v] = xy[2 * v + 1]; }
    /* stress-free configuration: rest lengths, rest angles and rest area */
    double *rx = dz(n), *ry = dz(n);
    const double *r = xy_rest ? xy_rest : xy;
    for (int v = 0; v < n; v++) { rx[v] = r[2 * v]; ry[v] = r[2 * v + 1]; }
    geom g; geom_alloc(&g, n);
    geometry(n, rx, ry, &g);
    for (int v = 0; v < n; v++) { b->l0[v] = g.len[v]; b->th0[v] = g.th[v]; }
    b->A0 = g.area;
    geometry(n, b->x, b->y, &g);
    b->P0 = g.perim;
    /* membrane mass spread evenly over the vertices (Sec. 2.7): the enclosed
     * fluid-equivalent mass rho_r * A0 divided by n                          */
    b->vmass = rho_r * b->A0 / n;
    /* rigid body: mass, polar moment and vertex offsets from the centroid */
    b->xc = g.cx; b->yc = g.cy;
    b->mass = rho_r * g.area;
    b->inertia = rho_r * polar_moment(n, b->x, b->y, g.cx, g.cy);
    for (int v = 0; v < n; v++) { b->rx0[v] = b->x[v] - g.cx; b->ry0[v] = b->y[v] - g.cy; }
    geom_free(&g);
    free(rx); free(ry);
    return s->nb++;
}

/* Ligand sites on the elements of a body; receptors on the lower wall only.
 * A site is bound at t = 0 iff its gap to the wall is below y_cr (Sec. 2.5),
 * its anchor then sits straight below it.                                     */
int orc_add_bonds(orc_sim *s, int body, int ns, const int *host, const double *frac,
                  double sigma, double ycr, double yeq, double kf, double kr0, double lb,
                  uint64_t seed) {
    if (body < 0 || body >= s->nb) return -1;
    orc_body *b = &s->b[body];
    b->ns = ns; b->sigma = sigma; b->ycr = ycr; b->yeq = yeq; b->kf = kf; b->kr0 = kr0;
    b->lb = lb; b->seed = seed;
    b->host = (int *)calloc(ns ? ns : 1, sizeof(int));
    b->frac = dz(ns); b->anchor = dz(ns);
    b->bound = (unsigned char *)calloc(ns ? ns : 1, 1);
    for (int k = 0; k < ns; k++) {
        if (host[k] < 0 || host[k] >= b->n) return -1;
        b->host[k] = host[k]; b->frac[k] = frac[k];
        int e = host[k], m = (e + 1) % b->n;
        double xs = b->x[e] + frac[k] * (b->x[m] - b->x[e]);
        double ys = b->y[e] + frac[k] * (b->y[m] - b->y[e]);
        if (ys + 0.5 < ycr) { b->bound[k] = 1; b->anchor[k] = xs; }
    }
    return 0;
}

void orc_get_vertices(const orc_sim *s, int body, double *xy) {
    const orc_body *b = &s->b[body];
    for (int v = 0; v < b->n; v++) { xy[2 * v] = b->x[v]; xy[2 * v + 1] = b->y[v]; }
}
void orc_get_bonds(const orc_sim *s, int body, unsigned char *state, double *anchor) {
    const orc_body *b = &s->b[body];
    for (int k = 0; k < b->ns; k++) { state[k] = b->bound[k]; anchor[k] = b->anchor[k]; }
}
int orc_count_bound(const orc_sim *s, int body) {
    const orc_body *b = &s->b[body];
    int c = 0;
    for (int k = 0; k < b->ns; k++) c += b->bound[k];
    return c;
}
/* per-body data of the last step: u* at vertices, probe p and stress, force, target velocity */
void orc_get_body_work(const orc_sim *s, int body, double *usxy, double *probe4, double *fxy, double *Uxy) {
    const orc_body *b = &s->b[body];
    for (int v = 0; v < b->n; v++) {
        if (usxy) { usxy[2 * v] = b->usx[v]; usxy[2 * v + 1] = b->usy[v]; }
        if (probe4) {
            probe4[4 * v] = b->pp[v]; probe4[4 * v + 1] = b->psxx[v];
            probe4[4 * v + 2] = b->psxy[v]; probe4[4 * v + 3] = b->psyy[v];
        }
        if (fxy) { fxy[2 * v] = b->fx[v]; fxy[2 * v + 1] = b->fy[v]; }
        if (Uxy) { Uxy[2 * v] = b->Ux[v]; Uxy[2 * v + 1] = b->Uy[v]; }
    }
}
/* rigid state: {xc, yc, phi, ucx, ucy, om, mass, inertia} */
void orc_get_rigid(const orc_sim *s, int body, double *out8) {
    const orc_body *b = &s->b[body];
    out8[0] = b->xc; out8[1] = b->yc; out8[2] = b->phi; out8[3] = b->ucx;
    out8[4] = b->ucy; out8[5] = b->om; out8[6] = b->mass; out8[7] = b->inertia;
}
/* body diagnostics: {area, perimeter, cx, cy, A0, P0, bound count, vertex mass} */
void orc_body_diag(const orc_sim *s, int body, double *out8) {
    const orc_body *b = &s->b[body];
    geom g; geom_alloc(&g, b->n);
    geometry(b->n, b->x, b->y, &g);
    out8[0] = g.area; out8[1] = g.perim; out8[2] = g.cx; out8[3] = g.cy;
    out8[4] = b->A0; out8[5] = b->P0; out8[6] = orc_count_bound(s, body); out8[7] = b->vmass;
    geom_free(&g);
}

/* x-distance under the periodic x boundary (minimum image) */
static double min_image(const orc_sim *s, double dx) {
    double L = (double)s->nx;
    return dx - L * floor(dx / L + 0.5);
}

/* ---- S5: forces on the vertices of body k at x^n ----------------------------------
 * Deformable bodies: stretching springs (Eq. 8), bending (Eq. 10, with the
 * garbled "t" in its denominators read as "+"), area penalty (Eq. 11, with
 * p_ref = cs2), plus the external forces.  Rigid bodies: external forces only.
 * External: repulsion from vertices of other bodies closer than the minimum
 * distance (Eq. 12, along the inward vertex normal, distance floored at
 * rep_dmin), ligand-receptor springs along the outward normal of the host
 * element (Eq. 13), pressure and viscous loads from the element probes
 * (Eqs. 14-15).  Element forces are shared equally by the element's two
 * vertices.                                                                  */
static void body_forces(orc_sim *s, int k, const geom *G) {
    orc_body *b = &s->b[k];
    const geom *g = &G[k];
    int n = b->n;
    for (int v = 0; v < n; v++) { b->fx[v] = 0; b->fy[v] = 0; }
    if (b->kind == ORC_DEFORMABLE) {
        for (int l = 0; l < n; l++) {       /* Eq. (8) */
            int m = (l + 1) % n;
            double c = -b->ks * (g->len[l] - b->l0[l]) / g->len[l];
            double rx = b->x[l] - b->x[m], ry = b->y[l] - b->y[m];
            b->fx[l] += c * rx; b->fy[l] += c * ry;
            b->fx[m] -= c * rx; b->fy[m] -= c * ry;
        }
        for (int v = 0; v < n; v++) {       /* Eq. (10) */
            int p = (v + n - 1) % n, m = (v + 1) % n;
            double mag = b->kb * (g->th[v] - b->th0[v]);
            double ll = g->len[p], lr = g->len[v];
            b->fx[p] += mag * ll / (ll + lr) * g->nvx[v]; b->fy[p] += mag * ll / (ll + lr) * g->nvy[v];
            b->fx[v] -= mag * g->nvx[v];                  b->fy[v] -= mag * g->nvy[v];
            b->fx[m] += mag * lr / (ll + lr) * g->nvx[v]; b->fy[m] += mag * lr / (ll + lr) * g->nvy[v];
        }
        double cA = b->ka * (1.0 - g->area / b->A0) * b->pref;
        for (int l = 0; l < n; l++) {       /* Eq. (11): n^- = -n_l */
            int m = (l + 1) % n;
            double fx = -cA * (-g->nlx[l]) * g->len[l], fy = -cA * (-g->nly[l]) * g->len[l];
            b->fx[l] += 0.5 * fx; b->fy[l] += 0.5 * fy;
            b->fx[m] += 0.5 * fx; b->fy[m] += 0.5 * fy;
        }
    }
    if (b->kind == ORC_FIXED) return;
    /* Eq. (12) */
#pragma omp parallel for schedule(static)
    for (int v = 0; v < n; v++) {
        for (int c = 0; c < s->nb; c++) {
            if (c == k) continue;
            const orc_body *o = &s->b[c];
            for (int u = 0; u < o->n; u++) {
                double dx = min_image(s, b->x[v] - o->x[u]), dy = b->y[v] - o->y[u];
                double d = sqrt(dx * dx + dy * dy);
                if (d < s->rep_cut) {
                    double dd = d > s->rep_dmin ? d : s->rep_dmin;
                    double f = s->rep_pref * sqrt(1.0 / pow(dd, 5.0));
                    b->fx[v] += f * (-g->nvx[v]); b->fy[v] += f * (-g->nvy[v]);
                }
            }
        }
    }
    /* Eq. (13): bond length from the site to its anchor on the wall y = -1/2 */
    for (int q = 0; q < b->ns; q++) {
        if (!b->bound[q]) continue;
        int e = b->host[q], m = (e + 1) % n;
        double xs = b->x[e] + b->frac[q] * (b->x[m] - b->x[e]);
        double ys = b->y[e] + b->frac[q] * (b->y[m] - b->y[e]);
        double yl = sqrt((xs - b->anchor[q]) * (xs - b->anchor[q]) + (ys + 0.5) * (ys + 0.5));
        double f = b->sigma * (yl - b->yeq);
        b->fx[e] += 0.5 * f * g->nlx[e]; b->fy[e] += 0.5 * f * g->nly[e];
        b->fx[m] += 0.5 * f * g->nlx[e]; b->fy[m] += 0.5 * f * g->nly[e];
    }
    /* Eqs. (14)-(15) */
    for (int l = 0; l < n; l++) {
        int m = (l + 1) % n;
        double fx = (-b->pp[l] * g->nlx[l] + b->psxx[l] * g->nlx[l] + b->psxy[l] * g->nly[l]) * g->len[l];
        double fy = (-b->pp[l] * g->nly[l] + b->psxy[l] * g->nlx[l] + b->psyy[l] * g->nly[l]) * g->len[l];
        b->fx[l] += 0.5 * fx; b->fy[l] += 0.5 * fy;
        b->fx[m] += 0.5 * fx; b->fy[m] += 0.5 * fy;
    }
}

/* exported for tests: internal membrane forces (springs, bending, area) of a
 * free polygon against a rest polygon, f = {fx0, fy0, fx1, ...}             */
void orc_membrane_forces(int n, const double *xy, const double *xy_rest, double ks, double kb,
                         double ka, double pref, double *f) {
    orc_sim *s = orc_create(8, 8, 1.0, 0, 0, 0);
    orc_add_body(s, ORC_DEFORMABLE, n, xy, xy_rest, ks, kb, ka, pref, 1.0, 0);
    orc_body *b = &s->b[0];
    geom g; geom_alloc(&g, n);
    geometry(n, b->x, b->y, &g);
    b->kind = ORC_DEFORMABLE;
    /* no external forces: probes zero, no bonds, single body */
    body_forces(s, 0, &g);
    for (int v = 0; v < n; v++) { f[2 * v] = b->fx[v]; f[2 * v + 1] = b->fy[v]; }
    geom_free(&g);
    orc_destroy(s);
}

/* ---- S6: structure integration (Eqs. 16-20) ------------------------------------
 * Deformable: x^{n+1} = x^n + u* + F/(2 m_v) (Eq. 17, dt = 1), and the vertex
 * velocity from the second-order backward difference of Eq. (18), written as
 * U = 1.5 (x^{n+1}-x^n) - 0.5 (x^n - x^{n-1}).
 * Rigid: total force and moment about the centroid, the BDF2 updates of
 * Eqs. (19)-(20) for u and omega, then x_c += u, phi += omega and rigid
 * kinematics for the vertices.  Fixed: no motion, U = 0.                     */
static void integrate(orc_sim *s, int k) {
    orc_body *b = &s->b[k];
    int n = b->n;
    for (int v = 0; v < n; v++) { b->xn[v] = b->x[v]; b->yn[v] = b->y[v]; }
    if (b->kind == ORC_DEFORMABLE) {
        for (int v = 0; v < n; v++) {
            double dx = b->usx[v] + 0.5 * b->fx[v] / b->vmass;
            double dy = b->usy[v] + 0.5 * b->fy[v] / b->vmass;
            b->x[v] += dx; b->y[v] += dy;
            b->Ux[v] = 1.5 * dx - 0.5 * b->dxm[v];
            b->Uy[v] = 1.5 * dy - 0.5 * b->dym[v];
            b->dxm[v] = dx; b->dym[v] = dy;
        }
    } else if (b->kind == ORC_RIGID) {
        double Fx = 0, Fy = 0, M = 0;
        for (int v = 0; v < n; v++) {
            Fx += b->fx[v]; Fy += b->fy[v];
            M += (b->x[v] - b->xc) * b->fy[v] - (b->y[v] - b->yc) * b->fx[v];
        }
        double ux = (2.0 / 3.0) * (2.0 * b->ucx - 0.5 * b->ucx_m + Fx / b->mass);
        double uy = (2.0 / 3.0) * (2.0 * b->ucy - 0.5 * b->ucy_m + Fy / b->mass);
        double om = (2.0 / 3.0) * (2.0 * b->om - 0.5 * b->om_m + M / b->inertia);
        b->ucx_m = b->ucx; b->ucy_m = b->ucy; b->om_m = b->om;
        b->ucx = ux; b->ucy = uy; b->om = om;
        b->xc += ux; b->yc += uy; b->phi += om;
        double c = cos(b->phi), sn = sin(b->phi);
        for (int v = 0; v < n; v++) {
            b->x[v] = b->xc + c * b->rx0[v] - sn * b->ry0[v];
            b->y[v] = b->yc + sn * b->rx0[v] + c * b->ry0[v];
            b->Ux[v] = ux - om * (b->y[v] - b->yc);
            b->Uy[v] = uy + om * (b->x[v] - b->xc);
        }
    } else {
        for (int v = 0; v < n; v++) { b->Ux[v] = 0; b->Uy[v] = 0; }
    }
}

/* ---- S9: bond kinetics at x^{n+1} (Sec. 2.5, rates in Bell form) ---------------
 * Bound: P_r = 1 - exp(-k_r0 exp(|y_l - y_eq| / l_B)); the bond breaks if the
 * draw is below P_r.  Unbound with gap y_s + 1/2 < y_cr: P_f = 1 - exp(-k_f);
 * the bond forms, anchored straight below the site, if the draw is below P_f.
 * The smallest |draw - P| / P (and |gap - y_cr| where that decides) is recorded. */
static void bond_kinetics(orc_sim *s, int k) {
    orc_body *b = &s->b[k];
    int n = b->n;
    for (int q = 0; q < b->ns; q++) {
        int e = b->host[q], m = (e + 1) % n;
        double xs = b->x[e] + b->frac[q] * (b->x[m] - b->x[e]);
        double ys = b->y[e] + b->frac[q] * (b->y[m] - b->y[e]);
        double r = orc_uniform(b->seed, s->step, q);
        if (b->bound[q]) {
            double yl = sqrt((xs - b->anchor[q]) * (xs - b->anchor[q]) + (ys + 0.5) * (ys + 0.5));
            double P = 1.0 - exp(-b->kr0 * exp(fabs(yl - b->yeq) / b->lb));
            if (P > 0 && fabs(r - P) / P < s->min_margin_p) s->min_margin_p = fabs(r - P) / P;
            if (r < P) { b->bound[q] = 0; s->flips++; }
        } else {
            double gap = ys + 0.5;
            double P = 1.0 - exp(-b->kf);
            if (r < P && fabs(gap - b->ycr) < s->min_margin_gap) s->min_margin_gap = fabs(gap - b->ycr);
            if (gap < b->ycr) {
                if (P > 0 && fabs(r - P) / P < s->min_margin_p) s->min_margin_p = fabs(r - P) / P;
                if (r < P) { b->bound[q] = 1; b->anchor[q] = xs; s->flips++; }
            }
        }
    }
}

/* ---- one full time step ---------------------------------------------------------- */
static void one_step(orc_sim *s) {
    size_t N = (size_t)s->nx * s->ny;
    stream(s, s->A, s->h);                                   /* S1 */
    node_moments(s);                                         /* S2 */
    geom *G = (geom *)calloc(s->nb ? s->nb : 1, sizeof(geom));
    for (int k = 0; k < s->nb; k++) {                        /* S3, S4 */
        orc_body *b = &s->b[k];
        geom_alloc(&G[k], b->n);
        geometry(b->n, b->x, b->y, &G[k]);
        for (int v = 0; v < b->n; v++) {
            if (s->walls && (b->y[v] < -1.0 || b->y[v] > (double)s->ny)) s->flags |= 1;
            b->usx[v] = interp(s, s->usx, b->x[v], b->y[v], STEN_VELOCITY);
            b->usy[v] = interp(s, s->usy, b->x[v], b->y[v], STEN_VELOCITY);
        }
        for (int l = 0; l < b->n; l++) {
            int m = (l + 1) % b->n;
            double px = 0.5 * (b->x[l] + b->x[m]) + s->probe_dist * G[k].nlx[l];
            double py = 0.5 * (b->y[l] + b->y[m]) + s->probe_dist * G[k].nly[l];
            double pd = interp(s, s->drho, px, py, STEN_PROBE);
            b->pp[l] = pd / 3.0;
            b->psxx[l] = interp(s, s->sxx, px, py, STEN_PROBE);
            b->psxy[l] = interp(s, s->sxy, px, py, STEN_PROBE);
            b->psyy[l] = interp(s, s->syy, px, py, STEN_PROBE);
        }
    }
    for (int k = 0; k < s->nb; k++) body_forces(s, k, G);    /* S5 */
    for (int k = 0; k < s->nb; k++) integrate(s, k);         /* S6 */
    for (size_t c = 0; c < N; c++) { s->fibx[c] = 0; s->fiby[c] = 0; }
    for (int k = 0; k < s->nb; k++) {                        /* S7 */
        orc_body *b = &s->b[k];
        for (int v = 0; v < b->n; v++) {
            int p = (v + b->n - 1) % b->n;
            double dV = 0.5 * (G[k].len[p] + G[k].len[v]);
            double Fx = b->Ux[v] - b->usx[v], Fy = b->Uy[v] - b->usy[v];
            spread(s, s->fibx, b->xn[v], b->yn[v], dV * Fx);
            spread(s, s->fiby, b->xn[v], b->yn[v], dV * Fy);
        }
    }
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)N; c++) {                     /* S8 */
        double hq[9], heq[9], Fi[9];
        for (int q = 0; q < 9; q++) hq[q] = s->h[(size_t)q * N + c];
        double dr = s->drho[c], rho = 1.0 + dr;
        double Fx = s->gx + s->fibx[c], Fy = s->gy + s->fiby[c];
        double ux = (s->j0x[c] + 0.5 * Fx) / rho, uy = (s->j0y[c] + 0.5 * Fy) / rho;
        orc_heq(dr, ux, uy, heq);
        orc_guo(s->tau, ux, uy, Fx, Fy, Fi);
        for (int q = 0; q < 9; q++)
            s->A[(size_t)q * N + c] = hq[q] - (hq[q] - heq[q]) / s->tau + Fi[q];
    }
    for (int k = 0; k < s->nb; k++) bond_kinetics(s, k);     /* S9 */
    for (int k = 0; k < s->nb; k++) geom_free(&G[k]);
    free(G);
    s->step++;                                               /* S10 */
}

void orc_step(orc_sim *s, int nsteps) {
    for (int t = 0; t < nsteps; t++) one_step(s);
}

/* Macroscopic fields of the current state: the moments the next step starts
 * from, drho and u* = (sum h e + g/2)/rho of the streamed populations.       */
void orc_macro(orc_sim *s, double *drho, double *ux, double *uy) {
    size_t N = (size_t)s->nx * s->ny;
    stream(s, s->A, s->h);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)N; c++) {
        double dr = 0, jx = 0, jy = 0;
        for (int q = 0; q < 9; q++) {
            double v = s->h[(size_t)q * N + c];
            dr += v; jx += v * EX[q]; jy += v * EY[q];
        }
        drho[c] = dr;
        ux[c] = (jx + 0.5 * s->gx) / (1.0 + dr);
        uy[c] = (jy + 0.5 * s->gy) / (1.0 + dr);
    }
}

/* Node fields from the last step's S2 (stress) and S7 (spread force) */
void orc_node_fields(const orc_sim *s, double *sxx, double *sxy, double *syy, double *fibx, double *fiby) {
    size_t N = (size_t)s->nx * s->ny;
    if (sxx) memcpy(sxx, s->sxx, N * sizeof(double));
    if (sxy) memcpy(sxy, s->sxy, N * sizeof(double));
    if (syy) memcpy(syy, s->syy, N * sizeof(double));
    if (fibx) memcpy(fibx, s->fibx, N * sizeof(double));
    if (fiby) memcpy(fiby, s->fiby, N * sizeof(double));
}

/* Totals of the post-collision state: mass deviation sum(A) and momentum sum(A e) */
void orc_totals(const orc_sim *s, double *out3) {
    size_t N = (size_t)s->nx * s->ny;
    double m = 0, px = 0, py = 0;
    for (int q = 0; q < 9; q++)
        for (size_t c = 0; c < N; c++) {
            double v = s->A[(size_t)q * N + c];
            m += v; px += v * EX[q]; py += v * EY[q];
        }
    out3[0] = m; out3[1] = px; out3[2] = py;
}

/* ---- entry points for the unit pins of single steps ----------------------------- */

/* Overwrite the interpolated velocity and the total force of body k (the
 * inputs of S6), then run S6 alone on it.                                     */
void orc_set_body_work(orc_sim *s, int k, const double *usxy, const double *fxy) {
    orc_body *b = &s->b[k];
    for (int v = 0; v < b->n; v++) {
        if (usxy) { b->usx[v] = usxy[2 * v]; b->usy[v] = usxy[2 * v + 1]; }
        if (fxy) { b->fx[v] = fxy[2 * v]; b->fy[v] = fxy[2 * v + 1]; }
    }
}
void orc_integrate_body(orc_sim *s, int k) { integrate(s, k); }

/* ---- state transfer: restart the oracle from a state given in FP64 --------------
 * A run can be continued from another code's state (promoted to FP64): the
 * populations (orc_set_populations), the step index (orc_set_step, which
 * keys the bond draws), and per body the vertex positions x^n, the previous
 * increment x^n - x^{n-1} (deformable, the BDF2 history of Eq. 18), the
 * rigid state (centroid, angle, velocity and angular velocity at n and
 * n-1: the BDF2 history of Eqs. 19-20), and the bond states and anchors.
 * The rest shape, masses and rigid offsets stay those of the body as added. */
void orc_set_body_state(orc_sim *s, int k, const double *xy, const double *dxy_prev, const double *rigid9) {
    orc_body *b = &s->b[k];
    for (int v = 0; v < b->n; v++) {
        if (xy) { b->x[v] = xy[2 * v]; b->y[v] = xy[2 * v + 1]; }
        if (dxy_prev) { b->dxm[v] = dxy_prev[2 * v]; b->dym[v] = dxy_prev[2 * v + 1]; }
    }
    if (rigid9) {
        b->xc = rigid9[0]; b->yc = rigid9[1]; b->phi = rigid9[2];
        b->ucx = rigid9[3]; b->ucy = rigid9[4]; b->ucx_m = rigid9[5]; b->ucy_m = rigid9[6];
        b->om = rigid9[7]; b->om_m = rigid9[8];
    }
}
void orc_get_body_state(const orc_sim *s, int k, double *xy, double *dxy_prev, double *rigid9) {
    const orc_body *b = &s->b[k];
    for (int v = 0; v < b->n; v++) {
        if (xy) { xy[2 * v] = b->x[v]; xy[2 * v + 1] = b->y[v]; }
        if (dxy_prev) { dxy_prev[2 * v] = b->dxm[v]; dxy_prev[2 * v + 1] = b->dym[v]; }
    }
    if (rigid9) {
        rigid9[0] = b->xc; rigid9[1] = b->yc; rigid9[2] = b->phi;
        rigid9[3] = b->ucx; rigid9[4] = b->ucy; rigid9[5] = b->ucx_m; rigid9[6] = b->ucy_m;
        rigid9[7] = b->om; rigid9[8] = b->om_m;
    }
}
void orc_set_bonds(orc_sim *s, int k, const unsigned char *state, const double *anchor) {
    orc_body *b = &s->b[k];
    for (int q = 0; q < b->ns; q++) {
        b->bound[q] = state[q] ? 1 : 0;
        b->anchor[q] = anchor[q];
    }
}

/* Structure alone, fluid frozen at rest: repeat S3, S5 (internal forces only)
 * and S6 with u* = 0 on one deformable polygon.                               */
void orc_relax_membrane(int n, const double *xy, const double *xy_rest, double ks, double kb,
                        double ka, double pref, double rho_r, int nsteps, double *xy_out,
                        double *area_hist) {
    orc_sim *s = orc_create(8, 8, 1.0, 0, 0, 0);
    orc_add_body(s, ORC_DEFORMABLE, n, xy, xy_rest, ks, kb, ka, pref, rho_r, 0);
    orc_body *b = &s->b[0];
    geom g; geom_alloc(&g, n);
    for (int t = 0; t < nsteps; t++) {
        geometry(n, b->x, b->y, &g);
        if (area_hist) area_hist[t] = g.area;
        body_forces(s, 0, &g);
        integrate(s, 0);
    }
    for (int v = 0; v < n; v++) { xy_out[2 * v] = b->x[v]; xy_out[2 * v + 1] = b->y[v]; }
    geom_free(&g);
    orc_destroy(s);
}
