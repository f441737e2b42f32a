/*
 * FP64 CPU oracle of the lattice part of the three-dimensional extension of the
 * lattice-Boltzmann / immersed-boundary method of Coclite, Pascazio, de Tullio
 * and Decuzzi (arXiv 2210.06043), whose conclusions name 3D as the next step:
 * the BGK update of Eq. (1) with the equilibrium of Eq. (2), the Guo term of
 * Eq. (4) and the moments of Eqs. (5)-(6), written for the D3Q19 velocity set
 * instead of D2Q9, in a capillary tube with halfway bounce-back walls.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header, table
 * or helper with the HIP library, and the HIP library never calls it.
 *
 * Everything is double precision with plain loops:
 *   S1  pull streaming, periodic along x, halfway bounce-back on every link
 *       whose upstream node is solid                            (Eq. 1; walls as in 2D)
 *   S2  moments rho = sum f, rho u = sum f e + g/2               (Eqs. 5-6)
 *   S3  with fixed immersed bodies (triangulated surfaces): the velocity u*
 *       of S2 interpolated to every vertex with the cosine delta in 3D, the
 *       direct forcing F = (U - u*) dV with U = 0, spread back with the same
 *       delta                                                   (Sec. 2.2)
 *   S3' with deformable membranes (closed triangulated surfaces): u*
 *       interpolated as in S3; elastic forces at x^n from Skalak's strain
 *       energy of each triangle (Skalak et al. 1973), a bending energy
 *       k_b (1 - cos(theta - theta0)) of the dihedral angle at each edge, and
 *       penalties on the membrane's total area and enclosed volume (FP64
 *       sums); the vertex
 *       update of the 2D membranes, dx = u* + f/(2m), x^{n+1} = x^n + dx,
 *       U = 3/2 dx - 1/2 dx_prev; F = (U - u*) dV spread at x^n, dV a third
 *       of the adjacent triangles' area at x^n                  (Secs. 2.2-2.4 in 3D)
 *   S3" ligand-receptor bonds between sites on one membrane's triangles and
 *       the tube wall: a bound site pulls with sigma (y_l - y_eq) along its
 *       triangle's outward normal, a third on each corner (Eq. 13 in 3D);
 *       after the update, Bell-type kinetics at x^{n+1} with the 2D oracle's
 *       Philox draws: a bond breaks with P_r = 1 - exp(-k_r0 exp(|y_l - y_eq|
 *       / l_B)), an unbound site within y_cr of the wall binds with
 *       P_f = 1 - exp(-k_f), anchored on the wall radially outward (Sec. 2.5)
 *   S4  BGK collision towards the equilibrium with the Guo term for the
 *       total force g + f_ib, u = (sum f e + (g + f_ib)/2)/rho   (Eqs. 1, 2, 4-6)
 * Populations are stored shifted, h_i = f_i - w_i, as in the 2D oracle.
 *
 * Geometry (the fluid nodes; all others are solid and never updated):
 *   ORC3_TUBE  (y - (ny-1)/2)^2 + (z - (nz-1)/2)^2 < R^2, a circular tube along x
 *   ORC3_SLAB  every node, walls beyond z = 0 and z = nz - 1, periodic in y
 *   ORC3_BOX   every node, periodic in all three directions
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC3_TUBE 0
#define ORC3_SLAB 1
#define ORC3_BOX 2

/* ---- D3Q19: the rest velocity, the six axis directions, the twelve
 * face diagonals (Qian, d'Humieres and Lallemand 1992), opposite directions
 * adjacent; weights 1/3, 1/18, 1/36; c_s^2 = 1/3 as for D2Q9.               */
static const int E3[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                              {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                              {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight(int i) {
    const int n = abs(E3[i][0]) + abs(E3[i][1]) + abs(E3[i][2]);
    return n == 0 ? 1.0 / 3.0 : n == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
}

static int opposite3(int i) {
    for (int k = 0; k < 19; k++)
        if (E3[k][0] == -E3[i][0] && E3[k][1] == -E3[i][1] && E3[k][2] == -E3[i][2]) return k;
    return -1;
}

void orc3_lattice_tables(int *e, double *w) {
    for (int i = 0; i < 19; i++) {
        for (int a = 0; a < 3; a++) e[3 * i + a] = E3[i][a];
        w[i] = weight(i);
    }
}

/* Eq. (2) in three dimensions, shifted by w (h_eq = f_eq - w), with
 * rho = 1 + drho written so that the subtraction of w is exact.            */
void orc3_heq(double drho, double ux, double uy, double uz, double *heq) {
    const double cs2 = 1.0 / 3.0, rho = 1.0 + drho, uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < 19; i++) {
        const double eu = E3[i][0] * ux + E3[i][1] * uy + E3[i][2] * uz;
        heq[i] = weight(i) * (drho + rho * (eu / cs2 + eu * eu / (2 * cs2 * cs2) - uu / (2 * cs2)));
    }
}

/* Eq. (4) in three dimensions: F_i = (1 - 1/(2 tau)) w [(e - u)/cs2 + (e.u) e / cs2^2] . F */
void orc3_guo(double tau, double ux, double uy, double uz, double Fx, double Fy, double Fz, double *Fi) {
    const double cs2 = 1.0 / 3.0;
    for (int i = 0; i < 19; i++) {
        const double ex = E3[i][0], ey = E3[i][1], ez = E3[i][2];
        const double eu = ex * ux + ey * uy + ez * uz;
        const double gx = (ex - ux) / cs2 + eu * ex / (cs2 * cs2);
        const double gy = (ey - uy) / cs2 + eu * ey / (cs2 * cs2);
        const double gz = (ez - uz) / cs2 + eu * ez / (cs2 * cs2);
        Fi[i] = (1.0 - 0.5 / tau) * weight(i) * (gx * Fx + gy * Fy + gz * Fz);
    }
}

typedef struct {
    int nx, ny, nz, geom;
    double tau, gx, radius;
    long long n;            /* nodes nx*ny*nz */
    unsigned char *fluid;   /* [nz][ny] (the geometry does not depend on x) */
    double *A;              /* post-collision shifted populations [19][nz][ny][nx] */
    double *h;              /* streamed populations, same layout */
    long long step;
    int opp[19];            /* opposite direction of each velocity */
    int nv;                 /* vertices of the fixed immersed bodies */
    double *X;              /* [nv][3] positions */
    double *dV;             /* [nv] volume weight: a third of the adjacent triangles' area (unit thickness) */
    double *f;              /* [3][n] spread force of the current step */
    /* deformable membranes */
    int nm, mv, mt;         /* membranes, their vertices and triangles in all */
    int *m_v0, *m_nv, *m_t0, *m_nt;   /* [nm] vertex and triangle ranges */
    double *m_par;          /* [nm][6] G_s, C, k_A, k_V, vertex mass, k_b */
    int *m_e0, *m_ne;       /* [nm] edge ranges */
    int me;                 /* edges in all */
    int *Medge;             /* [me][4] x1, x2 (the edge), x3, x4 (opposite vertices) */
    double *Mth0;           /* [me] rest dihedral angle */
    /* bonds: sites on the triangles of membrane bm */
    int ns, bm;
    int *Stri;              /* [ns] triangle (global index) */
    double *Sbary;          /* [ns][2] barycentric coordinates (corners 1 and 2) */
    int *Sbound;            /* [ns] bound */
    double *Sanc;           /* [ns][3] anchor on the wall */
    double b_sigma, b_yeq, b_ycr, b_kf, b_kr0, b_lb;
    uint64_t b_seed;
    double min_margin_p, min_margin_gap;
    long long flips;
    double *m_A0, *m_V0;    /* [nm] rest area and enclosed volume */
    double *MX, *Mdxm;      /* [mv][3] positions, displacement of the previous step */
    double *Mus, *Mf, *MF;  /* [mv][3] u*, elastic force, spread force of the current step */
    int *Mtri;              /* [mt][3] membrane vertex indices */
    double *Mref;           /* [mt][7] rest shape-function gradients g0, g1, g2 (2 each) and rest area */
} orc3;

static long long idx(const orc3 *s, int x, int y, int z) { return ((long long)z * s->ny + y) * s->nx + x; }

static int is_fluid_yz(const orc3 *s, int y, int z) {
    if (s->geom == ORC3_TUBE) {
        if (y < 0 || y >= s->ny || z < 0 || z >= s->nz) return 0;
        const double dy = y - 0.5 * (s->ny - 1), dz = z - 0.5 * (s->nz - 1);
        return dy * dy + dz * dz < s->radius * s->radius;
    }
    if (s->geom == ORC3_SLAB) return z >= 0 && z < s->nz;
    return 1;
}

orc3 *orc3_create(int nx, int ny, int nz, double tau, double gx, int geom, double radius) {
    if (nx < 1 || ny < 1 || nz < 1 || !(tau > 0.5) || geom < 0 || geom > 2) return NULL;
    orc3 *s = (orc3 *)calloc(1, sizeof(orc3));
    s->nx = nx; s->ny = ny; s->nz = nz; s->tau = tau; s->gx = gx; s->geom = geom; s->radius = radius;
    s->n = (long long)nx * ny * nz;
    for (int i = 0; i < 19; i++) s->opp[i] = opposite3(i);
    s->fluid = (unsigned char *)calloc((size_t)ny * nz, 1);
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++) s->fluid[z * ny + y] = (unsigned char)is_fluid_yz(s, y, z);
    s->A = (double *)calloc((size_t)(19 * s->n), sizeof(double));
    s->h = (double *)calloc((size_t)(19 * s->n), sizeof(double));
    return s;
}

void orc3_destroy(orc3 *s) {
    if (!s) return;
    free(s->fluid); free(s->A); free(s->h); free(s->X); free(s->dV); free(s->f);
    free(s->m_v0); free(s->m_nv); free(s->m_t0); free(s->m_nt); free(s->m_par); free(s->m_A0); free(s->m_V0);
    free(s->MX); free(s->Mdxm); free(s->Mus); free(s->Mf); free(s->MF); free(s->Mtri); free(s->Mref);
    free(s->m_e0); free(s->m_ne); free(s->Medge); free(s->Mth0);
    free(s->Stri); free(s->Sbary); free(s->Sbound); free(s->Sanc);
    free(s);
}

/* The 4-point cosine delta, phi(r) = (1 + cos(pi r / 2)) / 4 for |r| <= 2. */
static double phi3(double r) {
    r = fabs(r);
    return r < 2.0 ? 0.25 * (1.0 + cos(M_PI * r / 2.0)) : 0.0;
}

/* The 4 x 4 x 4 stencil of a point: first node per axis (x wrapped later)
 * and the tensor-product weights.                                           */
static void stencil3(const double *X, int o[3], double w[3][4]) {
    for (int a = 0; a < 3; a++) {
        o[a] = (int)floor(X[a]) - 1;
        for (int k = 0; k < 4; k++) w[a][k] = phi3(X[a] - (o[a] + k));
    }
}

/* A fixed immersed body (the kind that does not move): nv vertices
 * (xyz, [nv][3], lattice coordinates) and ntri triangles (tri, [ntri][3]
 * vertex indices).  Every stencil node of every vertex must be fluid (the
 * body is away from the walls); returns the index of its first vertex, or
 * -1 if a stencil node is solid or outside the cross-section.             */
int orc3_add_fixed_body(orc3 *s, int nv, const double *xyz, int ntri, const int *tri) {
    for (int v = 0; v < nv; v++) {
        int o[3];
        double w[3][4];
        stencil3(xyz + 3 * v, o, w);
        if (o[1] < 0 || o[1] + 3 >= s->ny || o[2] < 0 || o[2] + 3 >= s->nz) return -1;
        for (int b = 0; b < 4; b++)
            for (int c = 0; c < 4; c++)
                if (!is_fluid_yz(s, o[1] + b, o[2] + c)) return -1;
    }
    const int v0 = s->nv;
    s->X = (double *)realloc(s->X, sizeof(double) * 3 * (s->nv + nv));
    s->dV = (double *)realloc(s->dV, sizeof(double) * (s->nv + nv));
    memcpy(s->X + 3 * v0, xyz, sizeof(double) * 3 * nv);
    for (int v = 0; v < nv; v++) s->dV[v0 + v] = 0.0;
    for (int t = 0; t < ntri; t++) {
        const double *a = xyz + 3 * tri[3 * t], *b = xyz + 3 * tri[3 * t + 1], *c = xyz + 3 * tri[3 * t + 2];
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double area = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        for (int k = 0; k < 3; k++) s->dV[v0 + tri[3 * t + k]] += area / 3.0;
    }
    s->nv += nv;
    if (!s->f) s->f = (double *)calloc((size_t)(3 * s->n), sizeof(double));
    return v0;
}

int orc3_is_fluid(const orc3 *s, int y, int z) { return s->fluid[z * s->ny + y]; }

/* Equilibrium at rho = 1 and u = (ux(y, z), 0, 0) on every fluid node
 * (ux_of_yz [nz][ny], may be NULL for rest).                               */
void orc3_init_flow(orc3 *s, const double *ux_of_yz) {
    memset(s->A, 0, sizeof(double) * 19 * s->n);
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++) {
            if (!s->fluid[z * s->ny + y]) continue;
            double heq[19];
            orc3_heq(0.0, ux_of_yz ? ux_of_yz[z * s->ny + y] : 0.0, 0.0, 0.0, heq);
            for (int x = 0; x < s->nx; x++)
                for (int i = 0; i < 19; i++) s->A[i * s->n + idx(s, x, y, z)] = heq[i];
        }
    s->step = 0;
}

void orc3_get_populations(const orc3 *s, double *out) { memcpy(out, s->A, sizeof(double) * 19 * s->n); }
void orc3_set_populations(orc3 *s, const double *in) { memcpy(s->A, in, sizeof(double) * 19 * s->n); }
long long orc3_get_step(const orc3 *s) { return s->step; }

/* S1: h_i(x) = A_i(x - e_i); a link whose upstream node is solid returns the
 * node's own post-collision population of the opposite direction.          */
static void stream3(orc3 *s) {
    const long long n = s->n;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++) {
            if (!s->fluid[z * s->ny + y]) continue;
            for (int x = 0; x < s->nx; x++) {
                const long long k = idx(s, x, y, z);
                for (int i = 0; i < 19; i++) {
                    int xs = x - E3[i][0], ys = y - E3[i][1], zs = z - E3[i][2];
                    xs = ((xs % s->nx) + s->nx) % s->nx;
                    if (s->geom != ORC3_TUBE) ys = ((ys % s->ny) + s->ny) % s->ny;
                    if (s->geom == ORC3_BOX) zs = ((zs % s->nz) + s->nz) % s->nz;
                    if (is_fluid_yz(s, ys, zs))
                        s->h[i * n + k] = s->A[i * n + idx(s, xs, ys, zs)];
                    else
                        s->h[i * n + k] = s->A[s->opp[i] * n + k];
                }
            }
        }
}

/* S2: rho = 1 + sum h, u = (sum h e + g/2) / rho of the streamed populations */
static void moments3(const orc3 *s, long long k, double *drho, double u[3]) {
    double d = 0, jx = 0, jy = 0, jz = 0;
    for (int i = 0; i < 19; i++) {
        const double v = s->h[i * s->n + k];
        d += v;
        jx += E3[i][0] * v; jy += E3[i][1] * v; jz += E3[i][2] * v;
    }
    const double rho = 1.0 + d;
    *drho = d;
    u[0] = (jx + 0.5 * s->gx) / rho; u[1] = jy / rho; u[2] = jz / rho;
}

/* S3: u* at every vertex, F = (U - u*) dV with U = 0, spread into s->f */
static void ib_force3(orc3 *s) {
    const long long n = s->n;
    for (int v = 0; v < s->nv; v++) {
        int o[3];
        double w[3][4], us[3] = {0, 0, 0};
        stencil3(s->X + 3 * v, o, w);
        for (int c = 0; c < 4; c++)
            for (int b = 0; b < 4; b++)
                for (int a = 0; a < 4; a++) {
                    const int x = ((o[0] + a) % s->nx + s->nx) % s->nx;
                    const long long k = idx(s, x, o[1] + b, o[2] + c);
                    double d, u[3];
                    moments3(s, k, &d, u);
                    const double W = w[0][a] * w[1][b] * w[2][c];
                    for (int q = 0; q < 3; q++) us[q] += W * u[q];
                }
        for (int c = 0; c < 4; c++)
            for (int b = 0; b < 4; b++)
                for (int a = 0; a < 4; a++) {
                    const int x = ((o[0] + a) % s->nx + s->nx) % s->nx;
                    const long long k = idx(s, x, o[1] + b, o[2] + c);
                    const double W = w[0][a] * w[1][b] * w[2][c];
                    for (int q = 0; q < 3; q++) s->f[q * n + k] += W * (0.0 - us[q]) * s->dV[v];
                }
    }
}

/* ---- deformable membranes ------------------------------------------------ */

static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* u* at a point: the streamed velocity with half the body force at the 64
 * nodes of its stencil, weighted by the cosine delta                        */
static void interp3(orc3 *s, const double *X, double us[3]) {
    int o[3];
    double w[3][4];
    stencil3(X, o, w);
    us[0] = us[1] = us[2] = 0.0;
    for (int c = 0; c < 4; c++)
        for (int b = 0; b < 4; b++)
            for (int a = 0; a < 4; a++) {
                const int x = ((o[0] + a) % s->nx + s->nx) % s->nx;
                double d, u[3];
                moments3(s, idx(s, x, o[1] + b, o[2] + c), &d, u);
                const double W = w[0][a] * w[1][b] * w[2][c];
                for (int q = 0; q < 3; q++) us[q] += W * u[q];
            }
}

/* F spread at the 64 nodes of X's stencil into s->f */
static void spread3(orc3 *s, const double *X, const double F[3]) {
    int o[3];
    double w[3][4];
    stencil3(X, o, w);
    for (int c = 0; c < 4; c++)
        for (int b = 0; b < 4; b++)
            for (int a = 0; a < 4; a++) {
                const int x = ((o[0] + a) % s->nx + s->nx) % s->nx;
                const long long k = idx(s, x, o[1] + b, o[2] + c);
                const double W = w[0][a] * w[1][b] * w[2][c];
                for (int q = 0; q < 3; q++) s->f[q * s->n + k] += W * F[q];
            }
}

/* Area and enclosed volume of membrane m at its current positions, summed
 * over its triangles in order (the volume about its first vertex).         */
static void membrane_totals(const orc3 *s, int m, double *A, double *V) {
    const double *r0 = s->MX + 3 * s->m_v0[m];
    double a = 0.0, v = 0.0;
    for (int t = s->m_t0[m]; t < s->m_t0[m] + s->m_nt[m]; t++) {
        const int *T = s->Mtri + 3 * t;
        double p[3], q[3], r[3], e1[3], e2[3], n[3], qr[3];
        sub3(s->MX + 3 * T[0], r0, p); sub3(s->MX + 3 * T[1], r0, q); sub3(s->MX + 3 * T[2], r0, r);
        sub3(q, p, e1); sub3(r, p, e2); cross3(e1, e2, n);
        a += 0.5 * sqrt(dot3(n, n));
        cross3(q, r, qr);
        v += dot3(p, qr) / 6.0;
    }
    *A = a;
    *V = v;
}

/* The deformation of triangle t: F = sum_a x_a g_a^T (3 x 2, g_a the rest
 * shape-function gradients in the triangle's own rest frame), the right
 * Cauchy-Green tensor C = F^T F, I1 = tr C - 2, I2 = det C - 1 (Skalak's
 * invariants); Skalak's energy per rest area
 *   w = G_s/4 (I1^2 + 2 I1 - 2 I2 + C I2^2)                                 */
static void triangle_state(const orc3 *s, int t, double F[3][2], double Cm[2][2], double *I1, double *I2) {
    const int *T = s->Mtri + 3 * t;
    const double *g = s->Mref + 7 * t;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 2; j++) F[i][j] = 0.0;
    for (int a = 0; a < 3; a++) {
        const double *x = s->MX + 3 * T[a];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 2; j++) F[i][j] += x[i] * g[2 * a + j];
    }
    for (int j = 0; j < 2; j++)
        for (int k = 0; k < 2; k++) Cm[j][k] = F[0][j] * F[0][k] + F[1][j] * F[1][k] + F[2][j] * F[2][k];
    *I1 = Cm[0][0] + Cm[1][1] - 2.0;
    *I2 = Cm[0][0] * Cm[1][1] - Cm[0][1] * Cm[1][0] - 1.0;
}

/* The dihedral angle at edge (x1, x2) between the triangles (x1, x2, x3)
 * and (x2, x1, x4), both counter-clockwise from outside: with n1, n2 their
 * unit normals and e the unit edge vector, theta = atan2((n1 x n2).e, n1.n2).
 * Its gradient with respect to the four vertices, l = |x2 - x1|,
 * N1 = (x2 - x1) x (x3 - x1), N2 = (x1 - x2) x (x4 - x2):
 *   g3 = -l N1 / |N1|^2, g4 = -l N2 / |N2|^2,
 *   g1 = ((x3 - x2).e / l^2) g3 + ((x4 - x2).e / l^2) g4 (e unnormalised),
 *   g2 = -(g1 + g3 + g4) (the angle does not change under translation).    */
static double dihedral(const double *x1, const double *x2, const double *x3, const double *x4, double g[4][3]) {
    double e[3], a[3], b[3], N1[3], N2[3];
    sub3(x2, x1, e);
    sub3(x3, x1, a);
    cross3(e, a, N1);
    double me[3];
    for (int i = 0; i < 3; i++) me[i] = -e[i];
    sub3(x4, x2, b);
    cross3(me, b, N2);
    const double l = sqrt(dot3(e, e)), q1 = dot3(N1, N1), q2 = dot3(N2, N2);
    double n1[3], n2[3], c12[3];
    for (int i = 0; i < 3; i++) { n1[i] = N1[i] / sqrt(q1); n2[i] = N2[i] / sqrt(q2); }
    cross3(n1, n2, c12);
    const double th = atan2(dot3(c12, e) / l, dot3(n1, n2));
    if (g) {
        double d32[3], d42[3];
        sub3(x3, x2, d32);
        sub3(x4, x2, d42);
        const double w3 = dot3(d32, e) / (l * l), w4 = dot3(d42, e) / (l * l);
        for (int i = 0; i < 3; i++) {
            g[2][i] = -l * N1[i] / q1;
            g[3][i] = -l * N2[i] / q2;
            g[0][i] = w3 * g[2][i] + w4 * g[3][i];
            g[1][i] = -(g[0][i] + g[2][i] + g[3][i]);
        }
    }
    return th;
}

/* Energies of membrane m (exported for the tests): Skalak, area penalty
 * k_A (A - A0)^2 / (2 A0), volume penalty k_V (V - V0)^2 / (2 V0), bending
 * k_b sum over edges of (1 - cos(theta - theta0)).                          */
void orc3_membrane_energy(const orc3 *s, int m, double *out4) {
    const double *P = s->m_par + 6 * m;
    double ws = 0.0;
    for (int t = s->m_t0[m]; t < s->m_t0[m] + s->m_nt[m]; t++) {
        double F[3][2], Cm[2][2], I1, I2;
        triangle_state(s, t, F, Cm, &I1, &I2);
        ws += s->Mref[7 * t + 6] * 0.25 * P[0] * (I1 * I1 + 2.0 * I1 - 2.0 * I2 + P[1] * I2 * I2);
    }
    double A, V;
    membrane_totals(s, m, &A, &V);
    double eb = 0.0;
    for (int k = s->m_e0[m]; k < s->m_e0[m] + s->m_ne[m]; k++) {
        const int *E = s->Medge + 4 * k;
        const double th = dihedral(s->MX + 3 * E[0], s->MX + 3 * E[1], s->MX + 3 * E[2], s->MX + 3 * E[3], NULL);
        eb += P[5] * (1.0 - cos(th - s->Mth0[k]));
    }
    out4[0] = ws;
    out4[1] = P[2] != 0.0 ? P[2] * (A - s->m_A0[m]) * (A - s->m_A0[m]) / (2.0 * s->m_A0[m]) : 0.0;
    out4[2] = P[3] != 0.0 ? P[3] * (V - s->m_V0[m]) * (V - s->m_V0[m]) / (2.0 * s->m_V0[m]) : 0.0;
    out4[3] = eb;
}

double orc_uniform(uint64_t seed, int64_t n, int32_t s);   /* the 2D oracle's bond draw */

/* Site q's position and its triangle's unit outward normal. */
static void site3(const orc3 *s, int q, double p[3], double n[3]) {
    const int *T = s->Mtri + 3 * s->Stri[q];
    const double *a = s->MX + 3 * T[0], *b = s->MX + 3 * T[1], *c = s->MX + 3 * T[2];
    const double b1 = s->Sbary[2 * q], b2 = s->Sbary[2 * q + 1];
    double e1[3], e2[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    for (int i = 0; i < 3; i++) p[i] = a[i] + b1 * e1[i] + b2 * e2[i];
    cross3(e1, e2, n);
    const double nn = sqrt(dot3(n, n));
    for (int i = 0; i < 3; i++) n[i] /= nn;
}

/* Elastic forces of membrane m into Mf, minus the gradients of its three
 * energies: for triangle t and its corner a,
 *   Skalak  -A0 [w1 2 F g_a + w2 2 det C F C^-1 g_a], w1 = dw/dI1, w2 = dw/dI2
 *   area    -k_A (A - A0)/A0 * n x (x_c - x_b) / 2
 *   volume  -k_V (V - V0)/V0 * (x_b - r0) x (x_c - r0) / 6
 * with (a, b, c) the triangle's corners in its own cyclic order from a.     */
static void membrane_forces(orc3 *s, int m) {
    const double *P = s->m_par + 6 * m;
    const int v0 = s->m_v0[m];
    for (int v = v0; v < v0 + s->m_nv[m]; v++) s->Mf[3 * v] = s->Mf[3 * v + 1] = s->Mf[3 * v + 2] = 0.0;
    double A, V;
    membrane_totals(s, m, &A, &V);
    /* a penalty with a zero modulus contributes nothing (an open surface has no volume) */
    const double ca = P[2] != 0.0 ? P[2] * (A - s->m_A0[m]) / s->m_A0[m] : 0.0;
    const double cv = P[3] != 0.0 ? P[3] * (V - s->m_V0[m]) / s->m_V0[m] : 0.0;
    const double *r0 = s->MX + 3 * v0;
    for (int t = s->m_t0[m]; t < s->m_t0[m] + s->m_nt[m]; t++) {
        const int *T = s->Mtri + 3 * t;
        const double *g = s->Mref + 7 * t, A0 = g[6];
        double F[3][2], Cm[2][2], I1, I2;
        triangle_state(s, t, F, Cm, &I1, &I2);
        const double w1 = 0.25 * P[0] * (2.0 * I1 + 2.0), w2 = 0.25 * P[0] * (-2.0 + 2.0 * P[1] * I2);
        const double det = Cm[0][0] * Cm[1][1] - Cm[0][1] * Cm[1][0];
        const double Ci[2][2] = {{Cm[1][1] / det, -Cm[0][1] / det}, {-Cm[1][0] / det, Cm[0][0] / det}};
        double e1[3], e2[3], n[3];
        sub3(s->MX + 3 * T[1], s->MX + 3 * T[0], e1);
        sub3(s->MX + 3 * T[2], s->MX + 3 * T[0], e2);
        cross3(e1, e2, n);
        const double nn = sqrt(dot3(n, n));
        for (int i = 0; i < 3; i++) n[i] /= nn;
        for (int a = 0; a < 3; a++) {
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            const double ga[2] = {g[2 * a], g[2 * a + 1]};
            const double Cg[2] = {Ci[0][0] * ga[0] + Ci[0][1] * ga[1], Ci[1][0] * ga[0] + Ci[1][1] * ga[1]};
            double fa[3];
            for (int i = 0; i < 3; i++) {
                const double Fg = F[i][0] * ga[0] + F[i][1] * ga[1];
                const double FCg = F[i][0] * Cg[0] + F[i][1] * Cg[1];
                fa[i] = -A0 * (w1 * 2.0 * Fg + w2 * 2.0 * det * FCg);
            }
            double cb[3], xb[3], xc[3], bc[3], nbc[3];
            sub3(s->MX + 3 * T[c], s->MX + 3 * T[b], cb);
            cross3(n, cb, nbc);
            sub3(s->MX + 3 * T[b], r0, xb);
            sub3(s->MX + 3 * T[c], r0, xc);
            cross3(xb, xc, bc);
            double *f = s->Mf + 3 * T[a];
            for (int i = 0; i < 3; i++) f[i] += fa[i] - ca * 0.5 * nbc[i] - cv * bc[i] / 6.0;
        }
    }
    /* bonds (Eq. 13 in 3D): sigma (y_l - y_eq) along the triangle's outward
     * normal, a third on each corner, site by site */
    if (s->ns && m == s->bm)
        for (int q = 0; q < s->ns; q++) {
            if (!s->Sbound[q]) continue;
            double ps[3], n[3], dl[3];
            site3(s, q, ps, n);
            sub3(ps, s->Sanc + 3 * q, dl);
            const double f = s->b_sigma * (sqrt(dot3(dl, dl)) - s->b_yeq);
            const int *T = s->Mtri + 3 * s->Stri[q];
            for (int k = 0; k < 3; k++)
                for (int i = 0; i < 3; i++) s->Mf[3 * T[k] + i] += f / 3.0 * n[i];
        }
    /* bending: -k_b sin(theta - theta0) grad theta, edge by edge */
    for (int k = s->m_e0[m]; k < s->m_e0[m] + s->m_ne[m]; k++) {
        const int *E = s->Medge + 4 * k;
        double g[4][3];
        const double th = dihedral(s->MX + 3 * E[0], s->MX + 3 * E[1], s->MX + 3 * E[2], s->MX + 3 * E[3], g);
        const double sb = -P[5] * sin(th - s->Mth0[k]);
        for (int r = 0; r < 4; r++)
            for (int i = 0; i < 3; i++) s->Mf[3 * E[r] + i] += sb * g[r][i];
    }
}

/* Bond kinetics at x^{n+1} (S3"): the draw of site q at step n is the 2D
 * oracle's; the wall is the tube's cylinder of radius R about the axis
 * ((ny-1)/2, (nz-1)/2); the gap of a site is R minus its distance from the
 * axis, a new bond's anchor the wall point radially outward of the site.
 * The smallest |draw - P| / P and |gap - y_cr| of the decisions are kept.   */
static void bonds3(orc3 *s) {
    const double yc = 0.5 * (s->ny - 1), zc = 0.5 * (s->nz - 1), R = s->radius;
    for (int q = 0; q < s->ns; q++) {
        double ps[3], n[3];
        site3(s, q, ps, n);
        const double r = orc_uniform(s->b_seed, s->step, q);
        if (s->Sbound[q]) {
            double dl[3];
            sub3(ps, s->Sanc + 3 * q, dl);
            const double yl = sqrt(dot3(dl, dl));
            const double P = 1.0 - exp(-s->b_kr0 * exp(fabs(yl - s->b_yeq) / s->b_lb));
            if (P > 0 && fabs(r - P) / P < s->min_margin_p) s->min_margin_p = fabs(r - P) / P;
            if (r < P) { s->Sbound[q] = 0; s->flips++; }
        } else {
            const double dy = ps[1] - yc, dz = ps[2] - zc, rho = sqrt(dy * dy + dz * dz), gap = R - rho;
            const double P = 1.0 - exp(-s->b_kf);
            if (r < P && fabs(gap - s->b_ycr) < s->min_margin_gap) s->min_margin_gap = fabs(gap - s->b_ycr);
            if (gap < s->b_ycr) {
                if (P > 0 && fabs(r - P) / P < s->min_margin_p) s->min_margin_p = fabs(r - P) / P;
                if (r < P) {
                    s->Sbound[q] = 1;
                    s->flips++;
                    s->Sanc[3 * q] = ps[0];
                    s->Sanc[3 * q + 1] = yc + R * dy / rho;
                    s->Sanc[3 * q + 2] = zc + R * dz / rho;
                }
            }
        }
    }
}

/* S3' for every membrane vertex (see the file header) */
static void membranes3(orc3 *s) {
    for (int v = 0; v < s->mv; v++) interp3(s, s->MX + 3 * v, s->Mus + 3 * v);
    for (int m = 0; m < s->nm; m++) membrane_forces(s, m);
    double *dV = (double *)calloc((size_t)s->mv, sizeof(double));
    for (int t = 0; t < s->mt; t++) {
        const int *T = s->Mtri + 3 * t;
        double e1[3], e2[3], n[3];
        sub3(s->MX + 3 * T[1], s->MX + 3 * T[0], e1);
        sub3(s->MX + 3 * T[2], s->MX + 3 * T[0], e2);
        cross3(e1, e2, n);
        const double area = 0.5 * sqrt(dot3(n, n));
        for (int k = 0; k < 3; k++) dV[T[k]] += area / 3.0;
    }
    for (int m = 0; m < s->nm; m++) {
        const double mass = s->m_par[6 * m + 4];
        for (int v = s->m_v0[m]; v < s->m_v0[m] + s->m_nv[m]; v++) {
            double Xn[3], F[3];
            for (int q = 0; q < 3; q++) {
                Xn[q] = s->MX[3 * v + q];
                const double dx = s->Mus[3 * v + q] + 0.5 * s->Mf[3 * v + q] / mass;
                const double U = 1.5 * dx - 0.5 * s->Mdxm[3 * v + q];
                s->MX[3 * v + q] += dx;
                s->Mdxm[3 * v + q] = dx;
                F[q] = (U - s->Mus[3 * v + q]) * dV[v];
            }
            for (int q = 0; q < 3; q++) s->MF[3 * v + q] = F[q];
            spread3(s, Xn, F);
        }
    }
    free(dV);
    if (s->ns) bonds3(s);
}

/* A deformable membrane: a closed triangulated surface (nv vertices xyz
 * [nv][3], ntri triangles tri [ntri][3] counter-clockwise seen from
 * outside), its rest shape the given one, with Skalak's G_s and C, the
 * area and volume penalties k_A, k_V and the vertex mass.  Every stencil
 * node must be fluid now; returns the index of its first vertex among the
 * membrane vertices, or -1.                                                 */
int orc3_add_membrane(orc3 *s, int nv, const double *xyz, int ntri, const int *tri, double gs, double c, double ka,
                      double kv, double mass, double kb) {
    for (int v = 0; v < nv; v++) {
        int o[3];
        double w[3][4];
        stencil3(xyz + 3 * v, o, w);
        if (o[1] < 0 || o[1] + 3 >= s->ny || o[2] < 0 || o[2] + 3 >= s->nz) return -1;
        for (int b = 0; b < 4; b++)
            for (int cc = 0; cc < 4; cc++)
                if (!is_fluid_yz(s, o[1] + b, o[2] + cc)) return -1;
    }
    const int m = s->nm, v0 = s->mv, t0 = s->mt;
    s->nm++; s->mv += nv; s->mt += ntri;
    s->m_v0 = (int *)realloc(s->m_v0, sizeof(int) * s->nm);
    s->m_nv = (int *)realloc(s->m_nv, sizeof(int) * s->nm);
    s->m_t0 = (int *)realloc(s->m_t0, sizeof(int) * s->nm);
    s->m_nt = (int *)realloc(s->m_nt, sizeof(int) * s->nm);
    s->m_par = (double *)realloc(s->m_par, sizeof(double) * 6 * s->nm);
    s->m_e0 = (int *)realloc(s->m_e0, sizeof(int) * s->nm);
    s->m_ne = (int *)realloc(s->m_ne, sizeof(int) * s->nm);
    s->m_A0 = (double *)realloc(s->m_A0, sizeof(double) * s->nm);
    s->m_V0 = (double *)realloc(s->m_V0, sizeof(double) * s->nm);
    s->MX = (double *)realloc(s->MX, sizeof(double) * 3 * s->mv);
    s->Mdxm = (double *)realloc(s->Mdxm, sizeof(double) * 3 * s->mv);
    s->Mus = (double *)realloc(s->Mus, sizeof(double) * 3 * s->mv);
    s->Mf = (double *)realloc(s->Mf, sizeof(double) * 3 * s->mv);
    s->MF = (double *)realloc(s->MF, sizeof(double) * 3 * s->mv);
    s->Mtri = (int *)realloc(s->Mtri, sizeof(int) * 3 * s->mt);
    s->Mref = (double *)realloc(s->Mref, sizeof(double) * 7 * s->mt);
    s->m_v0[m] = v0; s->m_nv[m] = nv; s->m_t0[m] = t0; s->m_nt[m] = ntri;
    const double par[6] = {gs, c, ka, kv, mass, kb};
    memcpy(s->m_par + 6 * m, par, sizeof par);
    memcpy(s->MX + 3 * v0, xyz, sizeof(double) * 3 * nv);
    memset(s->Mdxm + 3 * v0, 0, sizeof(double) * 3 * nv);
    memset(s->Mus + 3 * v0, 0, sizeof(double) * 3 * nv);
    memset(s->Mf + 3 * v0, 0, sizeof(double) * 3 * nv);
    memset(s->MF + 3 * v0, 0, sizeof(double) * 3 * nv);
    for (int t = 0; t < ntri; t++) {
        int *T = s->Mtri + 3 * (t0 + t);
        for (int k = 0; k < 3; k++) T[k] = v0 + tri[3 * t + k];
        /* the rest triangle in its own frame: X0 = 0, X1 = (l, 0), X2 = (p, q) */
        double e1[3], e2[3], n[3], u1[3], u2[3];
        sub3(xyz + 3 * tri[3 * t + 1], xyz + 3 * tri[3 * t], e1);
        sub3(xyz + 3 * tri[3 * t + 2], xyz + 3 * tri[3 * t], e2);
        cross3(e1, e2, n);
        const double l = sqrt(dot3(e1, e1)), nn = sqrt(dot3(n, n));
        for (int i = 0; i < 3; i++) { u1[i] = e1[i] / l; n[i] /= nn; }
        cross3(n, u1, u2);
        const double pp = dot3(e2, u1), qq = dot3(e2, u2);
        /* D = [X1 - X0, X2 - X0] = [[l, pp], [0, qq]]; the rows of D^-1 are g1 and g2 */
        double *g = s->Mref + 7 * (t0 + t);
        g[2] = 1.0 / l;  g[3] = -pp / (l * qq);
        g[4] = 0.0;      g[5] = 1.0 / qq;
        g[0] = -g[2] - g[4];
        g[1] = -g[3] - g[5];
        g[6] = 0.5 * nn;
    }
    double A, V;
    membrane_totals(s, m, &A, &V);
    s->m_A0[m] = A;
    s->m_V0[m] = V;
    /* the edges: each directed edge a -> b of a triangle with a < b, paired
     * with the triangle holding b -> a; x3 and x4 their opposite vertices
     * (edges in the order their first triangle and corner appear)           */
    s->m_e0[m] = s->me;
    s->m_ne[m] = 0;
    for (int t = 0; t < ntri; t++)
        for (int k = 0; k < 3; k++) {
            const int a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3], c3 = tri[3 * t + (k + 2) % 3];
            if (a >= b) continue;
            int c4 = -1;
            for (int u = 0; u < ntri && c4 < 0; u++)
                for (int j = 0; j < 3; j++)
                    if (tri[3 * u + j] == b && tri[3 * u + (j + 1) % 3] == a) { c4 = tri[3 * u + (j + 2) % 3]; break; }
            if (c4 < 0) continue;   /* a boundary edge: no dihedral angle */
            s->Medge = (int *)realloc(s->Medge, sizeof(int) * 4 * (s->me + 1));
            s->Mth0 = (double *)realloc(s->Mth0, sizeof(double) * (s->me + 1));
            int *E = s->Medge + 4 * s->me;
            E[0] = v0 + a; E[1] = v0 + b; E[2] = v0 + c3; E[3] = v0 + c4;
            s->Mth0[s->me] = dihedral(s->MX + 3 * E[0], s->MX + 3 * E[1], s->MX + 3 * E[2], s->MX + 3 * E[3], NULL);
            s->me++;
            s->m_ne[m]++;
        }
    if (!s->f) s->f = (double *)calloc((size_t)(3 * s->n), sizeof(double));
    return v0;
}

/* Bond sites on membrane m (tube geometry only): ns sites, each on the
 * membrane's triangle tri[q] (index among its triangles) at barycentric
 * coordinates bary[q] (weights of corners 1 and 2), all unbound, with the
 * spring sigma, y_eq, capture distance y_cr, rates k_f, k_r0, l_B and the
 * seed of the draws.  Returns 0, or -1 if refused (one set per simulation). */
int orc3_add_bonds(orc3 *s, int m, int ns, const int *tri, const double *bary, double sigma, double yeq, double ycr,
                   double kf, double kr0, double lb, uint64_t seed) {
    if (s->ns || m < 0 || m >= s->nm || ns < 1 || s->geom != ORC3_TUBE) return -1;
    for (int q = 0; q < ns; q++)
        if (tri[q] < 0 || tri[q] >= s->m_nt[m]) return -1;
    s->ns = ns;
    s->bm = m;
    s->Stri = (int *)malloc(sizeof(int) * ns);
    s->Sbary = (double *)malloc(sizeof(double) * 2 * ns);
    s->Sbound = (int *)calloc((size_t)ns, sizeof(int));
    s->Sanc = (double *)calloc((size_t)(3 * ns), sizeof(double));
    for (int q = 0; q < ns; q++) s->Stri[q] = s->m_t0[m] + tri[q];
    memcpy(s->Sbary, bary, sizeof(double) * 2 * ns);
    s->b_sigma = sigma; s->b_yeq = yeq; s->b_ycr = ycr; s->b_kf = kf; s->b_kr0 = kr0; s->b_lb = lb; s->b_seed = seed;
    s->min_margin_p = 1e300;
    s->min_margin_gap = 1e300;
    s->flips = 0;
    return 0;
}
/* bond states and anchors ([ns], [ns][3]); returns the bound count */
int orc3_bonds(const orc3 *s, int *bound, double *anchor) {
    int nb = 0;
    for (int q = 0; q < s->ns; q++) {
        if (bound) bound[q] = s->Sbound[q];
        if (anchor) memcpy(anchor + 3 * q, s->Sanc + 3 * q, sizeof(double) * 3);
        nb += s->Sbound[q];
    }
    return nb;
}
void orc3_set_bonds(orc3 *s, const int *bound, const double *anchor) {
    memcpy(s->Sbound, bound, sizeof(int) * s->ns);
    memcpy(s->Sanc, anchor, sizeof(double) * 3 * s->ns);
}
/* smallest decision margins so far (|draw - P| / P, |gap - y_cr|) and state changes */
void orc3_bond_margins(const orc3 *s, double *out3) {
    out3[0] = s->min_margin_p;
    out3[1] = s->min_margin_gap;
    out3[2] = (double)s->flips;
}

void orc3_membrane_vertices(const orc3 *s, double *out) { if (s->mv) memcpy(out, s->MX, sizeof(double) * 3 * s->mv); }
void orc3_membrane_set_vertices(orc3 *s, const double *in) { if (s->mv) memcpy(s->MX, in, sizeof(double) * 3 * s->mv); }
/* elastic forces of membrane m at the current positions, [nv][3] */
void orc3_membrane_forces(orc3 *s, int m, double *out) {
    membrane_forces(s, m);
    memcpy(out, s->Mf + 3 * s->m_v0[m], sizeof(double) * 3 * s->m_nv[m]);
}
/* the current dihedral angle at each edge of membrane m, and its rest value */
int orc3_membrane_dihedrals(const orc3 *s, int m, double *theta, double *theta0) {
    for (int k = 0; k < s->m_ne[m]; k++) {
        const int *E = s->Medge + 4 * (s->m_e0[m] + k);
        if (theta) theta[k] = dihedral(s->MX + 3 * E[0], s->MX + 3 * E[1], s->MX + 3 * E[2], s->MX + 3 * E[3], NULL);
        if (theta0) theta0[k] = s->Mth0[s->m_e0[m] + k];
    }
    return s->m_ne[m];
}
/* spread force F = (U - u*) dV of the last step at every membrane vertex, [mv][3] */
void orc3_membrane_spread_forces(const orc3 *s, double *out) { if (s->mv) memcpy(out, s->MF, sizeof(double) * 3 * s->mv); }
void orc3_membrane_totals(const orc3 *s, int m, double *out4) {
    membrane_totals(s, m, out4, out4 + 1);
    out4[2] = s->m_A0[m];
    out4[3] = s->m_V0[m];
}

/* S4: A = h - (h - h_eq)/tau + F_i(u, g + f_ib), u = (sum h e + (g + f_ib)/2)/rho */
static void collide3(orc3 *s) {
    const long long n = s->n;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++) {
            if (!s->fluid[z * s->ny + y]) continue;
            for (int x = 0; x < s->nx; x++) {
                const long long k = idx(s, x, y, z);
                double drho, u[3], heq[19], F[19];
                moments3(s, k, &drho, u);
                double Fx = s->gx, Fy = 0.0, Fz = 0.0;
                if (s->f) {
                    const double rho = 1.0 + drho;
                    Fx += s->f[k]; Fy = s->f[n + k]; Fz = s->f[2 * n + k];
                    u[0] += 0.5 * s->f[k] / rho; u[1] += 0.5 * Fy / rho; u[2] += 0.5 * Fz / rho;
                }
                orc3_heq(drho, u[0], u[1], u[2], heq);
                orc3_guo(s->tau, u[0], u[1], u[2], Fx, Fy, Fz, F);
                for (int i = 0; i < 19; i++) {
                    const double hv = s->h[i * n + k];
                    s->A[i * n + k] = hv - (hv - heq[i]) / s->tau + F[i];
                }
            }
        }
}

void orc3_step(orc3 *s, int nsteps) {
    for (int t = 0; t < nsteps; t++) {
        stream3(s);
        if (s->f) memset(s->f, 0, sizeof(double) * 3 * s->n);
        if (s->nv) ib_force3(s);
        if (s->nm) membranes3(s);
        collide3(s);
        s->step++;
    }
}

/* Moments the next step starts from: drho and u = (sum h e + g/2)/rho of the
 * streamed populations, [nz][ny][nx] each; zero on solid nodes.            */
void orc3_macro(orc3 *s, double *drho, double *ux, double *uy, double *uz) {
    stream3(s);
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++)
            for (int x = 0; x < s->nx; x++) {
                const long long k = idx(s, x, y, z);
                double d = 0, u[3] = {0, 0, 0};
                if (s->fluid[z * s->ny + y]) moments3(s, k, &d, u);
                drho[k] = d; ux[k] = u[0]; uy[k] = u[1]; uz[k] = u[2];
            }
}

/* Sums over the fluid nodes of the stored (post-collision) populations:
 * mass sum h and momentum sum h e.                                          */
void orc3_totals(const orc3 *s, double *out4) {
    double m = 0, px = 0, py = 0, pz = 0;
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++) {
            if (!s->fluid[z * s->ny + y]) continue;
            for (int x = 0; x < s->nx; x++) {
                const long long k = idx(s, x, y, z);
                for (int i = 0; i < 19; i++) {
                    const double v = s->A[i * s->n + k];
                    m += v; px += E3[i][0] * v; py += E3[i][1] * v; pz += E3[i][2] * v;
                }
            }
        }
    out4[0] = m; out4[1] = px; out4[2] = py; out4[3] = pz;
}

/* The spread force of the last step at every node, [3][nz][ny][nx]. */
void orc3_ib_force(const orc3 *s, double *out) {
    if (s->f) memcpy(out, s->f, sizeof(double) * 3 * s->n);
    else memset(out, 0, sizeof(double) * 3 * s->n);
}

/* The volume weight of every vertex, [nv]. */
void orc3_vertex_weights(const orc3 *s, double *out) { if (s->nv) memcpy(out, s->dV, sizeof(double) * s->nv); }
