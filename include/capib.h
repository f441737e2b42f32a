/*
 * capib — C-ABI of the MI355X (gfx950) implementation of the hybrid lattice
 * Boltzmann / immersed-boundary method of Coclite, Pascazio, de Tullio and
 * Decuzzi, "Predicting the vascular adhesion of deformable drug carriers in
 * narrow capillaries traversed by blood cells" (arXiv 2210.06043).
 *
 * The calls follow the paper's statement of the problem: a D2Q9 lattice with
 * capillary walls (Sec. 2.1-2.2, 3.1), immersed membranes (Sec. 2.2-2.3),
 * ligand-receptor bonds (Sec. 2.5) and a time step (Sec. 2.1-2.9: streaming
 * and collision, interpolation, membrane, interaction, bond and load forces,
 * integration, spreading).
 *
 * Conventions
 *   - Lattice units: dx = dt = 1, rho_0 = 1, c_s^2 = 1/3.
 *   - Fluid nodes (i, j), i in [0, nx), j in [0, ny); x is periodic.  With
 *     walls the no-slip walls sit half-way between nodes at y = -1/2 and
 *     y = ny - 1/2 (halfway bounce-back).
 *   - Host arrays of node fields are row-major [ny][nx] doubles; population
 *     arrays are [9][ny][nx] in the velocity order of Eq. (3): rest, +x, +y,
 *     -x, -y, (+1,+1), (-1,+1), (-1,-1), (+1,-1), stored shifted, h = f - w.
 *   - Membrane vertices are given counter-clockwise as interleaved (x, y)
 *     doubles in unwrapped lattice coordinates; element e joins vertex e to
 *     vertex e+1 (mod n).
 *
 * Ownership and memory
 *   - The caller owns all device memory: one workspace of
 *     capib_workspace_bytes() bytes (256-byte aligned), bound once with
 *     capib_bind_workspace().  The library never allocates or frees device
 *     memory.  Host arrays passed in are copied during the call.
 *   - All GPU work is enqueued on the hip stream given at creation (a
 *     hipStream_t passed as void*; NULL = the null stream).  Calls documented
 *     "syncs" wait for that stream before returning.  The library also keeps
 *     three streams of its own (created on the first capib_step, destroyed
 *     by capib_destroy): one for the far lattice tiles that run beside the
 *     immersed-boundary kernels on large lattices, joined back into the
 *     caller's stream within each step, and two on which HIP graphs are
 *     captured.  The caller sees ordinary stream order on its own stream.
 *
 * Errors
 *   - Every call returns a capib_status; capib_last_error() gives a message
 *     for the last failing call on that context.  Arguments are validated
 *     before any device work.  Numerical trouble detected on the device
 *     (non-finite values, |u| > 0.3 c_s, rho <= 0, a vertex outside the rows
 *     [-1, ny]) is sticky and is reported as CAPIB_E_UNSTABLE by
 *     capib_diagnostics().
 *
 * Threads: one context per host thread at a time; distinct contexts are
 * independent.
 */
#ifndef CAPIB_H
#define CAPIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CAPIB_OK = 0,
    CAPIB_E_ARG = -1,      /* invalid argument (message says which) */
    CAPIB_E_STATE = -2,    /* call out of order (e.g. no workspace bound) */
    CAPIB_E_HIP = -3,      /* HIP runtime error */
    CAPIB_E_UNSTABLE = -4, /* device error flag raised (see capib_diag.error_flags) */
    CAPIB_E_CAPACITY = -5  /* more bodies, vertices or sites than the capacities */
} capib_status;

/* population storage of the lattice sweep */
enum { CAPIB_FP32_SHIFTED = 0, CAPIB_FP16_SHIFTED = 1 };
/* membrane kinds: deformable (Eqs. 16-18), rigid (Eqs. 19-20), fixed (no motion) */
enum { CAPIB_DEFORMABLE = 0, CAPIB_RIGID = 1, CAPIB_FIXED = 2 };
/* device error flag bits */
enum {
    CAPIB_FLAG_VERTEX_OUT = 1,   /* a vertex left the rows [-1, ny] */
    CAPIB_FLAG_FLUID = 2,        /* non-finite population, rho <= 0 or |u| > 0.3 c_s */
    CAPIB_FLAG_NONFINITE_IB = 8  /* non-finite vertex force or position */
};

typedef struct capib_ctx capib_ctx;

/* The lattice of Sec. 2.1 and the channel of Sec. 3.1.
 *   nx, ny     nodes (nx >= 1; ny >= 2, and ny >= 4 with walls)
 *   tau        BGK relaxation time, > 1/2 (nu = (tau - 1/2)/3, Sec. 2.1)
 *   gx, gy     uniform driving body force per node (added to the Guo term)
 *   walls      3: bounce-back walls at both y ends; 0: periodic in y too
 *   storage    CAPIB_FP32_SHIFTED (collision arithmetic in FP64, one rounding
 *              per stored value) or CAPIB_FP16_SHIFTED (FP32 arithmetic)
 *   fp16_scale power of two multiplying stored FP16 deviations (ignored for FP32)
 *   max_*      capacities of the workspace; max_vertices counts all bodies,
 *              a single body holds at most 1024 vertices and 2048 sites     */
typedef struct {
    int32_t nx, ny;
    double tau, gx, gy;
    int32_t walls;
    int32_t storage;
    double fp16_scale;
    int32_t max_bodies, max_vertices, max_sites;
} capib_lattice;

/* An immersed membrane (Sec. 2.2-2.3).
 *   kind           CAPIB_DEFORMABLE | CAPIB_RIGID | CAPIB_FIXED
 *   n, xy          vertex count (3..1024) and 2n coordinates, counter-clockwise
 *   xy_rest        stress-free shape (2n) or NULL for xy (rest lengths, angles, A0)
 *   ks, kb, ka     spring (Eq. 8), bending (Eq. 10) and area (Eq. 11) constants
 *   p_ref          reference pressure of Eq. (11)
 *   density_ratio  rho_body / rho_0: vertex mass rho_r A0 / n (deformable),
 *                  mass rho_r A0 and inertia rho_r J0 (rigid)
 *   tag            free caller label
 *   band           ensemble member the membrane lives in (0 for a single
 *                  lattice); coordinates are local to the member, and
 *                  membranes are added in non-decreasing band order        */
typedef struct {
    int32_t kind;
    int32_t n;
    const double *xy;
    const double *xy_rest;
    double ks, kb, ka, p_ref, density_ratio;
    int32_t tag;
    int32_t band;
} capib_membrane;

/* Ligand sites on a body, receptors on the lower wall (Sec. 2.5).
 *   n_sites          0..2048 (CAPIB_E_CAPACITY beyond)
 *   host_elem, frac  site s sits on element host_elem[s] at fraction frac[s]
 *   sigma            bond spring constant of Eq. (13)
 *   y_cr, y_eq       critical gap for binding and equilibrium bond length
 *   k_f, k_r0        forward rate and unstressed reverse rate per step
 *   bell_len         Bell length: k_r = k_r0 exp(|y - y_eq| / bell_len)
 *   seed             key of the Philox4x32-10 stream of this body          */
typedef struct {
    int32_t n_sites;
    const int32_t *host_elem;
    const double *frac;
    double sigma, y_cr, y_eq, k_f, k_r0, bell_len;
    uint64_t seed;
} capib_bonds;

typedef struct {
    int64_t step;         /* completed steps */
    int32_t error_flags;  /* CAPIB_FLAG_* bits raised so far */
    int32_t n_bodies;
    double mass;          /* sum over nodes of drho, FP64 accumulation */
    double mom_x, mom_y;  /* sum over nodes of sum_i h_i e_i, FP64 accumulation */
    int32_t near_tiles;   /* 64x4 lattice tiles under membrane stencils for the next step
                             (0 until a capib_step call, of any count, has marked them) */
    int32_t tiles;        /* all lattice tiles */
} capib_diag;

typedef struct {
    double area, perimeter, cx, cy;  /* current polygon, FP64 sums (Green's theorem) */
    double area0, perimeter0;        /* rest area and initial perimeter */
    int32_t n_bound;                 /* engaged bonds N_L */
    int32_t kind;
    double xc, yc, phi, ucx, ucy, omega; /* rigid state (zero for other kinds) */
    int32_t n_bound0;                /* bonds engaged at t = 0 (N_L0, Sec. 3.1) */
    int32_t reserved;
} capib_body_diag;

/* Creates a context for the lattice; validates tau > 1/2, sizes, walls in
 * {0, 3}, storage, capacities.  hip_stream: hipStream_t or NULL.           */
capib_status capib_create(const capib_lattice *lat, void *hip_stream, capib_ctx **out);

/* Creates a context for an ensemble of nbands independent capillaries
 * advanced together (each step of the ensemble is one step of every member,
 * in the same launches).  Member k is a channel of widths[k] x lat->ny nodes
 * with the walls, tau, drive and storage of lat; lat->nx is ignored.  The
 * members are stacked as bands of rows in one workspace, so lat->ny must be
 * a multiple of 4 when nbands > 1.  The per-row calls (init_flow) take the
 * lat->ny rows of one member, shared by all; populations and macroscopic
 * fields are read and written as the stack [nbands * ny][max width], zero
 * beyond a member's width.  Membranes name their member (capib_membrane
 * band) and use coordinates local to it; bodies of different members never
 * interact.  max_* capacities count the whole ensemble.                   */
capib_status capib_create_ensemble(const capib_lattice *lat, int32_t nbands, const int32_t *widths,
                                   void *hip_stream, capib_ctx **out);

/* Bytes of device workspace the context needs (multiple of 256). */
size_t capib_workspace_bytes(const capib_ctx *ctx);

/* Binds caller-owned device memory (>= capib_workspace_bytes, 256-byte
 * aligned) and clears it on the stream.  Must precede every call below.   */
capib_status capib_bind_workspace(capib_ctx *ctx, void *device_ptr, size_t bytes);

/* Sets the populations to the equilibrium of Eq. (2) at drho = 0 and the
 * x-velocity ux_of_y[j] in row j (ny values; NULL = rest).  Enqueued.     */
capib_status capib_init_flow(capib_ctx *ctx, const double *ux_of_y);

/* Writes / reads the stored populations as [9][ny][nx] doubles (h = f - w),
 * rounding to the storage type on write.  With FP16 storage a deviation
 * from the row reference whose scaled value exceeds the FP16 range is
 * refused (CAPIB_E_ARG).  Syncs.                                            */
capib_status capib_write_populations(capib_ctx *ctx, const double *h);
capib_status capib_read_populations(capib_ctx *ctx, double *h);

/* Adds a membrane (Sec. 2.2-2.3); returns its index in *body_id.  Rest
 * lengths, angles, area and (rigid) mass and polar moment are computed from
 * the shape in FP64.  Fails with CAPIB_E_CAPACITY beyond the capacities.   */
capib_status capib_add_membrane(capib_ctx *ctx, const capib_membrane *m, int32_t *body_id);

/* Adds the ligand sites of one body (Sec. 2.5).  A site is engaged at the
 * start iff its gap to the wall y = -1/2 is below y_cr; its anchor is then
 * straight below it.  Once per body.                                       */
capib_status capib_add_bonds(capib_ctx *ctx, int32_t body_id, const capib_bonds *b);

/* Interaction constants: repulsion prefactor and range of Eq. (12) (defaults
 * 1e-4/(8 sqrt 2) and dx) and the probe length of Sec. 2.6 (default 1.2).  */
capib_status capib_set_interactions(capib_ctx *ctx, double rep_prefactor, double rep_cutoff,
                                    double probe_dist);

/* Advances nsteps full steps of the method (Sec. 2.1-2.9): interpolation of
 * the fluid velocity and of the probe pressure and stress (Sec. 2.2, 2.6),
 * membrane forces (Eqs. 7-11), repulsion (Eq. 12), bond springs (Eq. 13),
 * hydrodynamic loads (Eqs. 14-15), integration (Eqs. 16-20), spreading
 * (Sec. 2.2, 2.7), bond kinetics (Sec. 2.5) and the lattice sweep of
 * streaming, bounce-back and BGK collision with forcing (Eqs. 1-6).
 * Enqueued on the stream, returns immediately.  The
 * lattice tiles that receive no spread force are swept on a second stream
 * of the library concurrently with the immersed-boundary kernels; the step
 * is joined back into the caller's stream before the tiles under the
 * membranes are swept, so the caller sees ordinary stream order.          */
capib_status capib_step(capib_ctx *ctx, int32_t nsteps);

/* Replays the steps through captured HIP graphs of 16 (and 2) steps when
 * enable != 0 (results identical to plain launches).  The four graphs (both
 * starting parities) are captured and instantiated by this call when a
 * workspace is bound, and again by the first capib_step call of two or more
 * steps after any later set-up call; other calls only replay them.         */
capib_status capib_set_graph(capib_ctx *ctx, int32_t enable);

/* Launch configuration of the step (not a step of the method: every
 * configuration computes the same results, bit for bit).  Any field -1
 * keeps the library's own rule.
 *   split           1: the far lattice tiles (those no membrane stencil
 *                   covers) in a launch of their own, on a second stream
 *                   beside the immersed-boundary kernels; 0: one sweep after
 *                   the membrane phase, with a share of the far tiles swept
 *                   by the membrane launch.  Rule: 1 from 8192 tiles of
 *                   64 x 4 nodes.
 *   far_share_pct   with split 0, percent of the far tiles swept by the
 *                   membrane launch (rule: 65 FP32, 80 FP16).
 *   mark_pairs      1: the next step's near tiles marked with one (vertex,
 *                   stencil tile) pair per lane; 0: one vertex per lane
 *                   (rule: 1 below 16384 vertices).
 *   membrane_class  threads and LDS of the membrane kernel sized for
 *                   membranes of 256, 512 or 1024 vertices (at least the
 *                   largest membrane; rule: the smallest that holds it).   */
typedef struct {
    int32_t split, far_share_pct, mark_pairs, membrane_class;
} capib_tuning;
capib_status capib_set_tuning(capib_ctx *ctx, const capib_tuning *t);
/* The configuration the next step will launch with (rules resolved). */
capib_status capib_get_tuning(const capib_ctx *ctx, capib_tuning *t);

/* Picks the launch configuration for this context's workload by timing:
 * from the library's own configuration, a coordinate descent over the
 * schedule, the far share, the marking layout and the membrane class, each
 * candidate timed with HIP events over steps_per_trial steps (>= 16, twice,
 * the faster kept) on the context's stream, from the current state (saved
 * to host memory before the trials and restored after them, so the run
 * continues as if no trial had happened).  Graphs are used if enabled.  The
 * fastest configuration is applied and, with cache_path (a text file, may
 * be NULL), appended under a key of the device and the workload's shape;
 * a later call that finds the key there applies it without timing.
 * chosen and best_ms_per_step (may be NULL) receive the result.  Syncs.   */
capib_status capib_autotune(capib_ctx *ctx, int32_t steps_per_trial, const char *cache_path,
                            capib_tuning *chosen, double *best_ms_per_step);

/* Macroscopic fields of the current state, [ny][nx] each (any may be NULL):
 * drho = sum h and u* = (sum h e + g/2)/rho of the streamed populations
 * (the density and velocity moments of Sec. 2.1, Eqs. 5-6, before the
 * coupling force of the next step is known), the moments the next step
 * starts from.  Syncs.                                                     */
capib_status capib_read_macro(capib_ctx *ctx, double *drho, double *ux, double *uy);

/* Vertex positions x^n of a body, 2n doubles.  Syncs. */
capib_status capib_read_vertices(capib_ctx *ctx, int32_t body_id, double *xy);

/* Bond states (0/1) and anchor x of a body's sites in the order given to
 * capib_add_bonds (the ligand-receptor bonds of Sec. 2.5: a bond is engaged
 * or not, and an engaged bond is anchored on the lower wall where it
 * formed).  Syncs.                                                         */
capib_status capib_read_bonds(capib_ctx *ctx, int32_t body_id, uint8_t *state, double *anchor_x);

/* Per-vertex data of the last step of a body (any may be NULL): interpolated
 * u* (2n), probe pressure and viscous stress per element (4n: p, sxx, sxy,
 * syy), total Lagrangian force (2n), target velocity U^{n+1} (2n).  Syncs. */
capib_status capib_read_body_work(capib_ctx *ctx, int32_t body_id, double *ustar, double *probe,
                                  double *force, double *target);

/* Global FP64 sums and the sticky error flags; returns CAPIB_E_UNSTABLE if
 * any flag is set.  The sums are the invariants of the scheme: mass (sum
 * of drho, conserved by streaming, bounce-back and the collision, Sec. 2.1)
 * and momentum (sum of h e); the per-body quantities that Sec. 3.1 monitors
 * are in capib_body_diagnostics and capib_readout.  Syncs.                 */
capib_status capib_diagnostics(capib_ctx *ctx, capib_diag *out);

/* Per member (band) of the context (one for a single lattice), the
 * quantities the load/hazard surrogate (capib_mlp.h) learns from, at the
 * current state, into out_device[8 * band + 0..7] (device floats):
 *   0, 1  drag and lift: the hydrodynamic load of Eqs. (14)-(15) summed over
 *         the elements of the member's particle (its first body with tag
 *         particle_tag), from the last step's probes and element geometry
 *   2     hazard: mean Bell rupture probability of the particle's engaged
 *         bonds (Sec. 2.5) at the current positions (0 without bonds)
 *   3     r: distance from the particle's vertex mean to the nearest vertex
 *         mean of a body with tag cell_tag (periodic in x; 0 if none)
 *   4     dp: that cell's perimeter over its initial perimeter, minus one
 *   5     that cell's body id (-1 if none)
 *   6     wall shear rate du_x/dy at the lower wall, 2 u_x(row 0), two
 *         nodes upstream of the particle's leftmost vertex (0 without walls)
 *   7     N_L of the particle
 * A member without a particle gets zeros and -1.  Enqueued.               */
capib_status capib_sample_members(capib_ctx *ctx, int32_t particle_tag, int32_t cell_tag, float *out_device);

/* FP64 geometry of a body's current polygon (area and perimeter, Sec. 2.3;
 * polygon-area centroid, Sec. 3.1), N_L and N_L0 (Sec. 2.5, 3.1) and the
 * rigid state (Sec. 2.9).  Syncs.                                          */
capib_status capib_body_diagnostics(capib_ctx *ctx, int32_t body_id, capib_body_diag *out);

/* The three quantities Sec. 3.1 monitors over time, in FP64 from the
 * current state, into out3:
 *   0  delta_p = (p - p_0)/p_0, the cell's perimeter p over its initial
 *      perimeter p_0 minus one (cell membrane stretching);
 *   1  r, the distance between the polygon-area centroids of the cell and
 *      the particle (minimum image along the periodic x);
 *   2  N_L / N_L0, the particle's engaged bonds over those engaged at t = 0
 *      (0 if none were).
 * Both bodies must belong to the same member.  Syncs.                      */
capib_status capib_readout(capib_ctx *ctx, int32_t cell_body, int32_t particle_body, double *out3);

/* The state a run continues from, per body (any output may be NULL):
 * vertex positions x^n (2n doubles); the previous increment x^n - x^{n-1}
 * (2n, the history of the BDF2 target velocity of Eq. 18; zero for rigid
 * and fixed bodies); and for a rigid body {xc, yc, phi, ucx, ucy,
 * ucx_prev, ucy_prev, omega, omega_prev} (9 doubles: the centroid, the
 * rotation angle and the velocities at steps n and n-1 that Eqs. 19-20
 * advance; zero for other kinds).  Syncs.                                   */
capib_status capib_read_body_state(capib_ctx *ctx, int32_t body_id, double *xy, double *dxy_prev, double *rigid9);

/* Checkpoint: with host_buf == NULL stores the needed size in *bytes;
 * otherwise copies the whole device state (populations, bodies, bonds, step)
 * into host_buf (*bytes on input is its capacity).  Syncs.                  */
capib_status capib_save(capib_ctx *ctx, void *host_buf, size_t *bytes);

/* Restores a checkpoint written by capib_save on a context created with the
 * same lattice and capacities and the same bodies and bonds added.  Syncs.  */
capib_status capib_load(capib_ctx *ctx, const void *host_buf, size_t bytes);

/* Per-kernel timing with HIP events on the context's stream.  While enabled,
 * capib_step runs the launches of each step in sequence on the caller's
 * stream, each with a start/stop event pair stamped at its own start and
 * end, and synchronises at its end.  capib_read_timing returns the summed
 * milliseconds of {interpolation, membrane launch, far-tile launch, lattice
 * sweep after the membrane phase} (4 doubles), the number of steps timed
 * and, if nodes4 is not NULL, the summed number of lattice nodes each of
 * the four launches swept (the interpolation's is 0), then resets the sums.
 * On lattices of 8192 tiles of 64 x 4 nodes or more the far tiles have a
 * launch of their own (beside the membrane phase); on smaller ones the
 * membrane launch sweeps a share of the far tiles and the last sweep the
 * rest, and the third sums are 0.                                           */
capib_status capib_set_timing(capib_ctx *ctx, int32_t enable);
capib_status capib_read_timing(capib_ctx *ctx, double *ms4, int64_t *steps, int64_t *nodes4);

/* Device-to-device copy of `bytes` bytes with a plain streaming kernel of
 * this library (16-byte loads and stores), enqueued on hip_stream.  Not a
 * step of the method: it measures the bandwidth that a streaming kernel
 * reaches on the device, the practical ceiling beside the vendor's peak for
 * the memory-bound lattice sweep.  dst and src must be 16-byte aligned,
 * bytes a multiple of 16, and the ranges must not overlap.                  */
capib_status capib_copy_bandwidth(void *dst, const void *src, size_t bytes, void *hip_stream);

/* capib_diagnostics for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results, but the per-tile FP64 partial
 * sums are kept in a fixed array of CAPIB_NOALLOC_SCRATCH_BYTES inside the
 * library instead of the workspace, and the call allocates nothing.  The
 * array exists once per device and is held until the process ends; every
 * call on a device shares it, so calls that overlap on one device (from
 * several threads or streams) race and must be serialised by the caller.
 * Lattices of more than (CAPIB_NOALLOC_SCRATCH_BYTES / 8 - 3) / 3 tiles of
 * 64 x 4 nodes are refused with CAPIB_E_CAPACITY.  Syncs.                   */
#define CAPIB_NOALLOC_SCRATCH_BYTES ((size_t)4 << 20)
capib_status capib_diagnostics_noalloc(capib_ctx *ctx, capib_diag *out);

/* Message of the last failing call on this context (never NULL). */
const char *capib_last_error(const capib_ctx *ctx);

/* Frees the host-side context; the workspace stays the caller's.  Waits for
 * the stream.                                                               */
void capib_destroy(capib_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* CAPIB_H */
