/*
 * capib3d — C-ABI of the lattice of the three-dimensional extension of the
 * lattice-Boltzmann / immersed-boundary method of Coclite, Pascazio, de
 * Tullio and Decuzzi (arXiv 2210.06043), which its conclusions name as the
 * next step: the BGK update of Eq. (1) with the equilibrium of Eq. (2), the
 * Guo term of Eq. (4) and the moments of Eqs. (5)-(6) on the D3Q19 velocity
 * set, in a capillary tube with no-slip walls (halfway bounce-back, as the
 * 2D channel's walls), driven by a uniform body force along the tube; and
 * fixed immersed bodies (triangulated surfaces that do not move) coupled as
 * in Sec. 2.2: the fluid velocity interpolated to every vertex with the
 * 4-point cosine delta in 3D, the direct force (U - u*) dV with U = 0,
 * spread back with the same delta; and deformable membranes (closed
 * triangulated surfaces with Skalak's strain energy per triangle and
 * penalties on their total area and enclosed volume, the 2D membranes'
 * vertex update of Secs. 2.2-2.4 carried to 3D).  A context holds fixed
 * bodies or membranes, not both.
 *
 * Conventions
 *   - Lattice units: dx = dt = 1, rho_0 = 1, c_s^2 = 1/3.
 *   - Nodes (x, y, z), x in [0, nx) along the tube (periodic), (y, z) the
 *     cross-section.  Geometry CAPIB3D_TUBE: fluid iff (y - (ny-1)/2)^2 +
 *     (z - (nz-1)/2)^2 < radius^2; CAPIB3D_SLAB: every node, walls half-way
 *     beyond z = 0 and z = nz - 1, periodic in y; CAPIB3D_BOX: periodic in
 *     all three directions.  A link whose upstream node is solid returns the
 *     node's own post-collision population of the opposite direction.
 *   - D3Q19 order: rest; +x, -x, +y, -y, +z, -z; (+1,+1,0), (-1,-1,0),
 *     (+1,-1,0), (-1,+1,0), (+1,0,+1), (-1,0,-1), (+1,0,-1), (-1,0,+1),
 *     (0,+1,+1), (0,-1,-1), (0,+1,-1), (0,-1,+1); weights 1/3, 1/18, 1/36.
 *   - Host arrays of node fields are [nz][ny][nx] doubles; population arrays
 *     [19][nz][ny][nx], stored shifted (h = f - w); solid nodes read as 0.
 *   - Storage: deviations from the equilibrium of the reference profile
 *     given to capib3d_init_flow (at rho = 1): CAPIB_FP32_SHIFTED stores
 *     them in FP32 with the collision evaluated in FP64 (one rounding per
 *     stored value); CAPIB_FP16_SHIFTED stores them in FP16 multiplied by
 *     fp16_scale, with FP32 arithmetic.
 *
 * Ownership, streams and errors as in capib.h: the caller owns the
 * workspace (capib3d_workspace_bytes(), 256-byte aligned, bound once); all
 * GPU work goes to the hip stream given at creation; calls marked "syncs"
 * wait for it; every call returns a capib_status, capib3d_last_error() gives
 * the message of the last failing call.  One context per host thread.
 */
#ifndef CAPIB3D_H
#define CAPIB3D_H

#include "capib.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { CAPIB3D_TUBE = 0, CAPIB3D_SLAB = 1, CAPIB3D_BOX = 2 };

/* The lattice and the tube.
 *   nx, ny, nz  nodes (each >= 1; nx * ny * nz < 2^31)
 *   tau         BGK relaxation time, > 1/2 (nu = (tau - 1/2)/3)
 *   gx          uniform driving body force per node along x
 *   geometry    CAPIB3D_TUBE, CAPIB3D_SLAB or CAPIB3D_BOX
 *   radius      tube radius in nodes (CAPIB3D_TUBE only, > 0)
 *   storage     CAPIB_FP32_SHIFTED or CAPIB_FP16_SHIFTED
 *   fp16_scale  power of two multiplying stored FP16 deviations (FP16 only)
 *   max_vertices  capacity for the vertices of fixed bodies (0: none)
 *   max_membranes, max_membrane_vertices, max_membrane_triangles
 *               capacity for deformable membranes (all 0, or all > 0)
 *   max_sites   capacity for ligand-receptor bond sites (needs membranes) */
typedef struct {
    int32_t nx, ny, nz;
    double tau, gx;
    int32_t geometry;
    double radius;
    int32_t storage;
    double fp16_scale;
    int32_t max_vertices;
    int32_t max_membranes, max_membrane_vertices, max_membrane_triangles;
    int32_t max_sites;
} capib3d_lattice;

/* A deformable membrane's constants (lattice units).
 *   gs    Skalak's shear modulus G_s: energy per rest area
 *         w = G_s/4 (I1^2 + 2 I1 - 2 I2 + C I2^2), I1 = tr C - 2,
 *         I2 = det C - 1 of the right Cauchy-Green tensor C of each triangle
 *   c     Skalak's C
 *   ka    penalty k_A (A - A0)^2 / (2 A0) on the total area
 *   kv    penalty k_V (V - V0)^2 / (2 V0) on the enclosed volume
 *   mass  vertex mass m of the update dx = u* + f/(2m)
 *   kb    bending k_b (1 - cos(theta - theta0)) at every interior edge,
 *         theta = atan2((n1 x n2).e, n1.n2) the angle between the adjacent
 *         faces' outward normals n1, n2 about the unit edge vector e         */
typedef struct {
    double gs, c, ka, kv, mass, kb;
} capib3d_membrane;

typedef struct capib3d_ctx capib3d_ctx;

/* Validates the lattice and creates a context (no device work). */
capib_status capib3d_create(const capib3d_lattice *lat, void *hip_stream, capib3d_ctx **out);
void capib3d_destroy(capib3d_ctx *ctx);

/* Bytes of device workspace the context needs. */
size_t capib3d_workspace_bytes(const capib3d_ctx *ctx);
/* Binds the caller's workspace (device pointer, 256-byte aligned, at least
 * capib3d_workspace_bytes()); uploads the geometry tables.  Syncs. */
capib_status capib3d_bind_workspace(capib3d_ctx *ctx, void *device_ptr, size_t bytes);

/* The initial state, Eq. (2) at rho = 1 and u = (ux(y, z), 0, 0) on every
 * fluid node, which is also the reference of the FP32 deviation storage
 * (ux_of_yz [nz][ny] host doubles, NULL = rest).  Syncs.                  */
capib_status capib3d_init_flow(capib3d_ctx *ctx, const double *ux_of_yz);

/* A fixed immersed body (Sec. 2.2 read in 3D; the body does not move): nv
 * vertices (xyz, [nv][3] host doubles, lattice coordinates: x along the
 * tube, wrapped periodically) and ntri triangles (tri, [ntri][3] vertex
 * indices).  Each vertex carries a third of the area of its triangles (unit
 * thickness) as its volume weight.  Every node of every vertex's 4 x 4 x 4
 * stencil must be a fluid node inside the cross-section (CAPIB_E_ARG
 * otherwise); more than max_vertices vertices in all gives
 * CAPIB_E_CAPACITY.  *first_vertex (may be NULL) receives the index of its
 * first vertex.  Syncs. */
capib_status capib3d_add_fixed_body(capib3d_ctx *ctx, int32_t nv, const double *xyz, int32_t ntri,
                                    const int32_t *tri, int32_t *first_vertex);

/* The force of the last step on the fluid at every vertex of the fixed
 * bodies, F = (U - u*) dV with U = 0, [vertices][3] host doubles in the
 * order the bodies were added; minus their sum is the hydrodynamic force on
 * the bodies (the spread weights of a vertex sum to one).  Syncs. */
capib_status capib3d_body_forces(capib3d_ctx *ctx, double *out);
/* Vertices of the fixed bodies added so far. */
int32_t capib3d_vertices(const capib3d_ctx *ctx);

/* A deformable membrane: nv vertices (xyz, [nv][3] host doubles, lattice
 * coordinates) and ntri triangles (tri, [ntri][3], counter-clockwise seen
 * from outside; nx >= 4), its rest shape the given one.  Each step:
 * u* interpolated at x^n (as for fixed bodies), the elastic force f at x^n
 * (Skalak, bending, area and volume terms, FP64), dx = u* + f/(2m), x^{n+1} =
 * x^n + dx, U = 3/2 dx - 1/2 dx_prev, F = (U - u*) dV spread at x^n with dV
 * a third of the adjacent triangles' area at x^n.  Every stencil node must
 * be fluid now (CAPIB_E_ARG; a node that leaves the fluid later raises
 * error flag 1 and contributes nothing; a work item, 64 nodes along x of
 * one column, lists at most 1024 vertices whose stencil touches it, beyond
 * which error flag 4 is raised), degenerate triangles or a
 * non-positive enclosed volume give CAPIB_E_ARG, capacity CAPIB_E_CAPACITY,
 * a context with fixed bodies CAPIB_E_STATE.  *first_vertex (may be NULL)
 * receives its first vertex among the membrane vertices.  Syncs. */
capib_status capib3d_add_membrane(capib3d_ctx *ctx, int32_t nv, const double *xyz, int32_t ntri,
                                  const int32_t *tri, const capib3d_membrane *par, int32_t *first_vertex);
/* Ligand-receptor bonds (Sec. 2.5 and Eq. 13 carried to 3D) between ns
 * sites on membrane m and the tube wall (CAPIB3D_TUBE only; one set of sites
 * per context, CAPIB_E_STATE for a second).
 *   sigma, yeq  spring constant and rest length: a bound site at distance y_l
 *               from its anchor pulls with sigma (y_l - yeq) along its
 *               triangle's outward normal, a third on each corner
 *   ycr         capture distance: an unbound site binds only while
 *               R - (its distance from the axis) < ycr
 *   kf          formation: P_f = 1 - exp(-kf) per step
 *   kr0, lb     rupture: P_r = 1 - exp(-kr0 exp(|y_l - yeq| / lb)) per step
 *   seed        key of the draws: site q's draw at step n is word 0 of
 *               Philox4x32-10 with key (seed low, high) and counter
 *               (n low, q, n high, 0), top 24 bits over 2^24 (as in capib.h)
 * tri [ns]: the triangle of each site among the membrane's triangles (the
 * order they were given in); bary [ns][2]: its barycentric weights of
 * corners 1 and 2 (>= 0, sum <= 1).  The decisions are taken after the
 * vertex update, at x^{n+1}; a new bond is anchored on the wall (radius R)
 * radially outward of its site.  All sites start unbound.  Syncs. */
typedef struct {
    double sigma, yeq, ycr, kf, kr0, lb;
    uint64_t seed;
} capib3d_bonds;
capib_status capib3d_add_bonds(capib3d_ctx *ctx, int32_t m, int32_t ns, const int32_t *tri, const double *bary,
                               const capib3d_bonds *par);
/* Bond states [ns] (may be NULL), anchors [ns][3] (may be NULL) and the
 * number bound (N_L, may be NULL); writing sets states and anchors.  Both
 * sync. */
capib_status capib3d_read_bonds(capib3d_ctx *ctx, int32_t *bound, double *anchor, int64_t *nbound);
capib_status capib3d_write_bonds(capib3d_ctx *ctx, const int32_t *bound, const double *anchor);

/* Membrane vertex positions, [membrane vertices][3] host doubles, in the
 * order the membranes were added (read and overwrite; the previous
 * displacement is kept).  Both sync. */
capib_status capib3d_read_membrane_vertices(capib3d_ctx *ctx, double *xyz);
capib_status capib3d_write_membrane_vertices(capib3d_ctx *ctx, const double *xyz);
/* The direct force F = (U - u*) dV of the last step at every membrane
 * vertex, [membrane vertices][3].  Syncs. */
capib_status capib3d_membrane_spread_forces(capib3d_ctx *ctx, double *out);
/* Membrane m's area and enclosed volume at the start of the last step (the
 * sums the step used: FP64 per wave of 64 triangles, the waves' sums added in
 * a fixed order), and its rest area and volume.  Syncs. */
capib_status capib3d_membrane_totals(capib3d_ctx *ctx, int32_t m, double *out4);
/* Error flags raised on the device since the workspace was bound: 1 a
 * membrane stencil node outside the fluid, 2 a spread contribution beyond
 * the fixed-point range (2^12) or not finite, 4 a work item's vertex list
 * full.  Syncs. */
capib_status capib3d_error_flags(capib3d_ctx *ctx, int32_t *flags);
/* Membranes, and their vertices in all. */
int32_t capib3d_membranes(const capib3d_ctx *ctx);
int32_t capib3d_membrane_vertex_count(const capib3d_ctx *ctx);

/* Schedule of a step with fixed bodies (three launches: the velocity at
 * every stencil node, the force at every vertex, the collision of the
 * stencil nodes): the shares, in percent of the work items, of the ordinary
 * sweep done in the first and in the second launch (defaults 0 and 0); the
 * rest is done in the third.  Any shares give the same result, bit for bit.
 * CAPIB_E_ARG if either is negative or their sum exceeds 100. */
capib_status capib3d_set_ib_schedule(capib3d_ctx *ctx, int32_t share_node_u, int32_t share_vertex);

/* nsteps steps of Eq. (1): pull streaming with bounce-back, moments of
 * Eqs. (5)-(6) with half the total force, BGK collision with the Guo term
 * of Eq. (4) for the body force plus the spread force of the fixed bodies
 * or membranes (interpolated, forced and spread from the streamed moments
 * at the start of the step; the membranes' spread contributions summed as
 * 64-bit fixed-point integers, 2^-50 units, so that every run gives the
 * same bits).  With bonds, every step ends with the sites' Bell-type
 * decisions at the new positions (Sec. 2.5 carried to 3D); the library
 * takes each step's decisions at the start of the next one, so the states
 * and anchors are current when the call's work completes.  Enqueued on the
 * context's stream; does not sync. */
capib_status capib3d_step(capib3d_ctx *ctx, int32_t nsteps);

/* The moments the next step starts from (Eqs. 5-6 of the streamed
 * populations with half the body force): drho, ux, uy, uz, [nz][ny][nx]
 * host doubles each (any may be NULL; zero on solid nodes).  Syncs. */
capib_status capib3d_read_macro(capib3d_ctx *ctx, double *drho, double *ux, double *uy, double *uz);

/* Stored (post-collision) populations, shifted h = f - w, [19][nz][ny][nx]
 * host doubles.  Writing rounds each to the storage type relative to the
 * reference (CAPIB_E_ARG if a scaled FP16 deviation would overflow); solid
 * nodes are ignored.  Both sync. */
capib_status capib3d_read_populations(capib3d_ctx *ctx, double *out);
capib_status capib3d_write_populations(capib3d_ctx *ctx, const double *in);

/* FP64 sums over the fluid nodes of the stored populations: out4 = {mass
 * sum h, momentum sum h e (x, y, z)}, the invariants of the update (mass
 * is conserved, momentum grows by the body force per node and step).
 * Also the step count.  Syncs. */
capib_status capib3d_diagnostics(capib3d_ctx *ctx, double *out4, int64_t *step);

/* Fluid nodes of the lattice. */
int64_t capib3d_fluid_nodes(const capib3d_ctx *ctx);

/* Message of the last failing call on this context (never NULL). */
const char *capib3d_last_error(const capib3d_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif
