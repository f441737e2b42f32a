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
    free(s->fluid); free(s->A); free(s->h); free(s->X); free(s->dV); free(s->f); free(s);
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
    memset(s->f, 0, sizeof(double) * 3 * n);
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
                if (s->nv) {
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
        if (s->nv) ib_force3(s);
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
