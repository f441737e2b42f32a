// Device-side data layout and helpers shared by the kernels of libcapib.
// gfx950 only: wave64, LDS-resident membranes, spreading gathered per tile.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace capib {

// Lattice sweep tile: one wave per row segment of 64 nodes, four rows per
// workgroup.  The near-tile flags use the same tiling.
constexpr int TILE_X = 64;
constexpr int TILE_Y = 4;
constexpr int LAT_THREADS = TILE_X * TILE_Y;
constexpr int MAXV_BODY = 1024;    // vertices of one membrane held in LDS
constexpr int MAXS_BODY = 2048;    // ligand sites of one membrane held in LDS
constexpr int ARG_BODIES = 16;     // bodies whose index ranges travel with the kernel arguments
constexpr int INTERP_THREADS = 256;  // 16 lanes per interpolation point

enum { DEFORMABLE = 0, RIGID = 1, FIXED = 2 };
enum { FLAG_VERTEX_OUT = 1, FLAG_FLUID = 2, FLAG_NONFINITE_IB = 8 };

// Read-only description of a body.
struct BodyParams {
    int kind, n, vstart, tag;
    int site_start, n_sites;
    int band, band_b0;              // ensemble member, and its first body
    float ks, kb, ka, pref;
    float vmass, inv_mass, inv_inertia;
    int band_nb;                    // bodies of the member (contiguous from band_b0)
    double A0;
    float sigma, ycr, yeq, kf;
    float kr0, lb;
    uint32_t seed_lo, seed_hi;
    float c0xh, c0xl, c0yh, c0yl;   // rigid: centroid at t = 0 (hi + lo)
    float P0, pad3;                 // perimeter at t = 0
    // Eq. (13) in FP64: the stretch y_l - y_eq of a bond is a small
    // difference of lengths close to y_eq, and whether an open site binds
    // compares its gap with y_cr; both are formed in double
    double sigma64, yeq64, ycr64, pad4;
};

// Mutable per-body state.
struct BodyState {
    float dcxh, dcxl, dcyh, dcyl;   // rigid: centroid displacement (hi + lo)
    float phih, phil;               // rigid: rotation angle (hi + lo)
    float rot[2];                   // rigid: cos(phi) - 1 and sin(phi) of the stored angle
    // rigid: (u_x, u_y, omega) at steps n and n-1, FP64: the BDF2 recurrence
    // of Eqs. (19)-(20) has a root at one, so rounding the velocities to FP32
    // every step would accumulate (about 3e-5 of u over 1000 steps)
    double u[3], um[3];
    float bbox[2][4];               // xmin, xmax, ymin, ymax of the vertices, parity-indexed
    int n_bound, pad;
    double geo[4];                  // diagnostics: area, perimeter, cx, cy
    double pad2;                    // keeps arrays of the struct 16-byte aligned
};
// the membrane kernel reads the rigid state as two float4 and three double2
static_assert(sizeof(BodyState) % 16 == 0, "BodyState must keep 16-byte alignment in arrays");
static_assert(offsetof(BodyState, u) % 16 == 0, "rigid velocities on a 16-byte boundary");

// Everything a kernel needs, passed by value.
//
// The lattice is a stack of bands, each an independent capillary of
// band_rows rows (an ensemble member); band k has width band_nx[k], starts
// at row k * band_rows and wraps periodically at its own width.  A single
// lattice is one band.  nx is the widest band (the row pitch is sized from
// it) and ny the rows of all bands.  Membrane coordinates are local to their
// band: x in [0, band width), y in [0, band_rows).
struct Dev {
    int nx, ny, pitch, walls;
    int ntx, nty, storage, band_rows;
    long long qstride;              // ny * pitch elements per population
    float omega, fc, gx, gy;        // 1/tau, 1 - 1/(2 tau), body force
    float scale, inv_scale;         // FP16 storage scale
    void *pop[2];                   // populations, parity-indexed
    // Per-row reference: stored populations are deviations s_i = A_i - r_i(y)
    // from the equilibrium r_i(y) = h_eq(0, (u_ref(y), 0)) of the initial
    // channel profile.  rowref[16 y + i] (i < 9) is the constant that turns a
    // pulled stored value into h_i - r_i(y); rowref[16 y + 9] = u_ref(y).
    const float *rowref;
    // The same constants in FP64 (the FP32-storage sweep collides in FP64)
    const double *rowref64;
    double omega64, fc64, gx64, gy64;
    // Near tiles of a step: the 64x4 tiles that the stencils of the vertex
    // positions x^n cover, i.e. the only tiles that can receive spread force
    // in step n.  Double-buffered by step parity: tnear[p][tile] is 1 for a
    // near tile.  The covering vertices are recorded as two global index
    // ranges, one for the vertices in the first half of their membrane's
    // list and one for the second half (so that a tile under both ends of a
    // closed membrane does not span the whole membrane): tv[p][4 tile + 2 h]
    // = nverts - lo_h and tv[p][4 tile + 2 h + 1] = hi_h + 1 (0 = none; both
    // kept by max).  The near sweep clears both after reading them.
    int *tnear[2];
    int *tv[2];
    // On a large lattice the near sweep runs over a list of the near tiles
    // instead of over every tile: nlist[p][0 .. ncount[p]), appended once
    // per tile by the marking (whose flag exchange decides which caller
    // appends it).
    int *nlist[2];
    int *ncount;
    // The membrane kernel expands each entry of its step's list into
    // elist[p][2 k], [2 k + 1] = {tile, band width, lo0, n0}, {lo1, n1, 0, 0}:
    // the covering vertices as candidate positions u in [0, n0 + n1) (u < n0:
    // vertex lo0 + u, else lo1 + u - n0), the two ranges in index order and
    // merged when they overlap; the sweep then starts a near tile from one
    // load.
    int4 *elist[2];
    // immersed boundary
    int nbodies, nverts, nsites, nbands;
    // size class of the membrane kernel: the largest membrane of this run
    // has at most body_mv vertices and 2 body_mv ligand sites (256, 512 or
    // MAXV_BODY)
    int body_mv;
    // launch configuration of the step (host side; the library's rule or
    // the autotuner's choice): split = the far tiles in a launch of their
    // own beside the membrane phase (else one sweep after it, with
    // far_share percent of the far tiles swept by the membrane launch);
    // mark_pairs = near-tile marking with one (vertex, tile) pair per lane
    int split, far_share, mark_pairs;
    const int *band_nx;             // width of each band
    // tiles that hold fluid nodes of some band (with several bands of
    // different widths, the tiles beyond a band's width hold none), in
    // index order; the far sweep runs over these
    const int *live;
    int nlive;
    const int2 *band_bodies;        // (first body, body count) of each band
    int *vinfo;                     // 2 band + (1 in the second half of its membrane's list)
    // (first vertex, vertices, first site, sites) of the first ARG_BODIES
    // bodies, passed with the arguments so that the membrane kernel can
    // issue its loads without a round trip for its parameters
    int4 brange[ARG_BODIES];
    float rep_pref, rep_cut, rep_dmin, probe;
    BodyParams *bp;
    BodyState *bs;
    int *vnext;                     // next vertex of the same membrane (cyclic)
    float *pxh[2], *pxl[2], *pyh[2], *pyl[2];   // vertex positions, parity-indexed
    float *dxm, *dym;                           // previous increment x^n - x^{n-1}
    float *x0h, *x0l, *y0h, *y0l;               // positions at t = 0
    // rigid: offsets from the centroid at t = 0, FP64: a vertex moves by
    // (R(phi) - I) r0, and FP32 offsets (errors up to ~2e-6 at ~45 nodes)
    // would misplace it by phi times that once the body has turned
    double *r0x, *r0y;
    float *l0, *th0;                            // rest lengths and turning angles
    float2 *ustar;                              // u* at vertices
    float4 *probe4;                             // p, sxx, sxy, syy at element probes
    float4 *pprobe[2];                          // probe point of each element (x hi, lo, y hi, lo), parity-indexed
    float2 *force;                              // total Lagrangian force
    float2 *target;                             // U^{n+1}
    // spread records of the step, one per vertex (written by the membrane
    // kernel, gathered by the near-tile sweep): stencil origin, x and y
    // weights (x weights already divided by the normalising sum), and the
    // force dV (U - u*) to spread
    int2 *sp_org;
    float4 *sp_wx, *sp_wy;
    float2 *sp_f;
    int2 *srange;                               // sites [begin, end) per element
    int *s_host, *s_state, *s_orig;
    double *s_frac;                             // site position along its element (FP64, see BodyParams)
    float *s_anh, *s_anl;
    // scalars and scratch
    long long *counter;   // steps started
    int *err;             // sticky error flags
    double *red;          // reduction partials
    float *macro;         // [3][ny][nx] readout
};

// ---- small helpers -------------------------------------------------------------

// Band k of the stack: width, first global row, rows.
struct Band {
    int nx, y0, ny;
};
// (a single band is the whole lattice: no load of its width)
__device__ __forceinline__ Band band_of(const Dev &d, int k) {
    if (d.nbands == 1) return Band{d.nx, 0, d.band_rows};
    return Band{d.band_nx[k], k * d.band_rows, d.band_rows};
}
__device__ __forceinline__ Band band_of_row(const Dev &d, int j) { return band_of(d, j / d.band_rows); }
// The same with the kind of lattice fixed at compile time (ENS: several
// bands), for the kernels of the step: no load and no branch for a single
// band.
template <bool ENS>
__device__ __forceinline__ Band band_at(const Dev &d, int k) {
    if (!ENS) return Band{d.nx, 0, d.band_rows};
    return Band{d.band_nx[k], k * d.band_rows, d.band_rows};
}
template <bool ENS>
__device__ __forceinline__ Band band_at_row(const Dev &d, int j) {
    return band_at<ENS>(d, ENS ? j / d.band_rows : 0);
}

// Workgroup index -> tile index such that each XCD (workgroups are dealt
// round-robin to the 8 XCDs) receives one contiguous range of tiles, so that
// neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    // XCD x holds tiles [x q + min(x, r), (x + 1) q + min(x + 1, r))
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// The same contiguous run of XCD x among n far-tile candidates (in natural
// order: tile index, or index into the live-tile list), for launches whose
// far workgroups start at a block index that is a multiple of 8, so that
// blockIdx & 7 is their XCD.  On a small lattice the membrane launch sweeps
// the first far_share_len(len, pct) candidates of every run and the sweep
// the rest, each on the run's own XCD.
struct XcdRun {
    int start, len;
};
__host__ __device__ inline XcdRun xcd_run(int x, int n) {
    const int q = n >> 3, r = n & 7;
    return XcdRun{x * q + (x < r ? x : r), q + (x < r ? 1 : 0)};
}
__host__ __device__ inline int far_share_len(int len, int pct) { return (int)((long long)len * pct / 100); }
__host__ __device__ inline int round_up8(int n) { return (n + 7) & ~7; }

__device__ __forceinline__ int wrapi(int i, int n) {
    if ((unsigned)i < (unsigned)n) return i;   // the common case, without a division
    i %= n;
    return i < 0 ? i + n : i;
}

// Error-free sum of a float pair (hi, lo) and a float d, renormalised.
__device__ __forceinline__ void df_add(float &hi, float &lo, float d) {
    float s = hi + d;
    float bb = s - hi;
    float err = (hi - (s - bb)) + (d - bb);
    float l = lo + err;
    float h = s + l;
    lo = l - (h - s);
    hi = h;
}

// Cosine-kernel stencil of a point given as hi + lo: node offsets and the
// 4 + 4 one-dimensional weights phi(X - i), phi(Y - j) for i = ix0 .. ix0+3,
// j = iy0 .. iy0+3; 'inv' divides every product weight.  With walls, Y is
// clamped to [-1, ny].  For the velocity coupling (renorm = false) the rows
// beyond a wall are the odd image of the fluid rows mirrored about the wall
// (no slip): the weights are folded onto four fluid rows and iy0 is the
// first of them.  For the probe fields (renorm = true) the rows beyond the
// wall are dropped and the fluid rows renormalised to sum one.  Returns true
// when the unclamped Y left [-1, ny].
// Origin of the stencil of a point given as hi + lo: ix0 = floor(X) - 1,
// iy0 = floor(Y) - 1 and the fractions sx, sy.  With walls, Y is clamped to
// [-1, ny].  Non-finite or absurd coordinates are flagged and mapped to the
// origin so that every index stays in range.  Returns true when the point
// was moved (unclamped Y outside [-1, ny], or unusable coordinates).
__device__ __forceinline__ bool stencil_origin(const Dev &d, const Band &B, float xh, float xl, float yh, float yl,
                                               int &ix0, int &iy0, float &sx, float &sy) {
    bool out = false;
    if (!(fabsf(xh) < 1.0e8f) || !(fabsf(xl) < 1.0e4f)) { xh = 0.0f; xl = 0.0f; out = true; }
    if (!(fabsf(yh) < 1.0e8f) || !(fabsf(yl) < 1.0e4f)) { yh = 0.0f; yl = 0.0f; out = true; }
    int ix = (int)floorf(xh);
    sx = (xh - (float)ix) + xl;
    float kx = floorf(sx);
    ix += (int)kx;
    sx -= kx;
    if (d.walls) {
        const float Y = yh + yl;
        if (Y < -1.0f) { out = true; yh = -1.0f; yl = 0.0f; }
        if (Y > (float)B.ny) { out = true; yh = (float)B.ny; yl = 0.0f; }
    }
    int iy = (int)floorf(yh);
    sy = (yh - (float)iy) + yl;
    float ky = floorf(sy);
    iy += (int)ky;
    sy -= ky;
    ix0 = ix - 1;
    iy0 = iy - 1;
    return out;
}

__device__ __forceinline__ bool stencil(const Dev &d, const Band &B, float xh, float xl, float yh, float yl,
                                        bool renorm, int &ix0, int &iy0, float wx[4], float wy[4], float &inv) {
    float sx, sy;
    const bool out = stencil_origin(d, B, xh, xl, yh, yl, ix0, iy0, sx, sy);
    float cx, snx, cy, sny;
    sincospif(0.5f * sx, &snx, &cx);
    sincospif(0.5f * sy, &sny, &cy);
    // phi(1+s), phi(s), phi(s-1), phi(s-2) with phi(r) = (1 + cos(pi r/2))/4
    wx[0] = 0.25f * (1.0f - snx); wx[1] = 0.25f * (1.0f + cx);
    wx[2] = 0.25f * (1.0f + snx); wx[3] = 0.25f * (1.0f - cx);
    wy[0] = 0.25f * (1.0f - sny); wy[1] = 0.25f * (1.0f + cy);
    wy[2] = 0.25f * (1.0f + sny); wy[3] = 0.25f * (1.0f - cy);
    const float sxw = (wx[0] + wx[1]) + (wx[2] + wx[3]);
    const float syfull = (wy[0] + wy[1]) + (wy[2] + wy[3]);
    if (d.walls && renorm) {
#pragma unroll
        for (int b = 0; b < 4; b++) {
            int j = iy0 + b;
            if (j < 0 || j >= B.ny) wy[b] = 0.0f;
        }
    } else if (d.walls) {
        // velocity coupling: the fluid velocity continued across the no-slip
        // wall as its odd image, i.e. a row beyond the wall is the fluid row
        // mirrored about the wall with its sign reversed.  The four weights
        // are folded onto four fluid rows o .. o + 3 (a band has at least
        // four rows), in row order; away from the walls this is the identity.
        const int o = min(max(iy0, 0), B.ny - 4);
        float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f, f3 = 0.0f;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const int j = iy0 + b;
            const bool lo = j < 0, hi = j >= B.ny;
            const int t = (lo ? -1 - j : hi ? 2 * B.ny - 1 - j : j) - o;
            const float w = (lo || hi) ? -wy[b] : wy[b];
            f0 += t == 0 ? w : 0.0f;
            f1 += t == 1 ? w : 0.0f;
            f2 += t == 2 ? w : 0.0f;
            f3 += t == 3 ? w : 0.0f;
        }
        wy[0] = f0; wy[1] = f1; wy[2] = f2; wy[3] = f3;
        iy0 = o;
    }
    const float syw = renorm ? (wy[0] + wy[1]) + (wy[2] + wy[3]) : syfull;
    inv = 1.0f / (sxw * syw);
    return out;
}

// Streamed (pulled) populations at node (i, j): h_q(x) = A_q(x - e_q), with
// halfway bounce-back across the walls and periodic wrap otherwise.
template <typename T>
__device__ __forceinline__ float ldpop(const T *p, float inv_scale);
template <>
__device__ __forceinline__ float ldpop<float>(const float *p, float) { return *p; }
template <>
__device__ __forceinline__ float ldpop<_Float16>(const _Float16 *p, float inv_scale) {
    return (float)(*p) * inv_scale;
}

template <typename T>
__device__ __forceinline__ void pull9(const Dev &d, const T *__restrict__ A, int i, int j, const Band &B, float h[9]) {
    const long long Q = d.qstride;
    const int im = (i == 0) ? B.nx - 1 : i - 1;
    const int ip = (i == B.nx - 1) ? 0 : i + 1;
    const int jl = j - B.y0;
    const bool bot = (jl == 0), top = (jl == B.ny - 1);
    const int jm = bot ? j + B.ny - 1 : j - 1;
    const int jp = top ? j - B.ny + 1 : j + 1;
    const long long r0 = (long long)j * d.pitch, rm = (long long)jm * d.pitch, rp = (long long)jp * d.pitch;
    const float is = d.inv_scale;
    h[0] = ldpop(A + r0 + i, is);
    h[1] = ldpop(A + Q + r0 + im, is);
    h[3] = ldpop(A + 3 * Q + r0 + ip, is);
    if (d.walls && bot) {
        h[2] = ldpop(A + 4 * Q + r0 + i, is);
        h[5] = ldpop(A + 7 * Q + r0 + i, is);
        h[6] = ldpop(A + 8 * Q + r0 + i, is);
    } else {
        h[2] = ldpop(A + 2 * Q + rm + i, is);
        h[5] = ldpop(A + 5 * Q + rm + im, is);
        h[6] = ldpop(A + 6 * Q + rm + ip, is);
    }
    if (d.walls && top) {
        h[4] = ldpop(A + 2 * Q + r0 + i, is);
        h[7] = ldpop(A + 5 * Q + r0 + i, is);
        h[8] = ldpop(A + 6 * Q + r0 + i, is);
    } else {
        h[4] = ldpop(A + 4 * Q + rp + i, is);
        h[7] = ldpop(A + 7 * Q + rp + ip, is);
        h[8] = ldpop(A + 8 * Q + rp + im, is);
    }
}

// Pulled populations as deviations from the reference of (band-local) row
// jl: dh_i = h_i - r_i(y) = s_i(x - e_i) + rowref_i(jl).  Returns u_ref(y).
__device__ __forceinline__ float add_rowref(const Dev &d, int jl, float h[9]) {
    const float *R = d.rowref + 16 * jl;
    h[2] += R[2]; h[4] += R[4]; h[5] += R[5];
    h[6] += R[6]; h[7] += R[7]; h[8] += R[8];
    return R[9];
}

template <typename T>
__device__ __forceinline__ float pull_dev(const Dev &d, const T *__restrict__ A, int i, int j, const Band &B,
                                          float h[9]) {
    pull9<T>(d, A, i, j, B, h);
    return add_rowref(d, j - B.y0, h);
}

// Records that the stencil of vertex v (global index; list half h of its
// membrane) covers the tile, for the step of parity p: widens the tile's
// vertex range of that half.
__device__ __forceinline__ void note_cover(const Dev &d, int p, int tile, int v, int h) {
    int *t = d.tv[p] + 4 * tile + 2 * h;
    atomicMax(t + 1, v + 1);
    atomicMax(t, d.nverts - v);
}

// Equilibrium of Eq. (2) as a deviation from the row reference, with
// u = (uref + dux, duy):
//   h_eq_i(drho, u) - r_i = w [drho (1 - 1.5 u.u) - 1.5 du.(u + uref)
//                              + drho (3 e.u + 4.5 (e.u)^2) + 3 e.du
//                              + 4.5 (e.du)(e.u + e.uref)]
// Every term carries a deviation (drho or du), so nothing large is rounded.
// C is the arithmetic type (float, or double in the FP32-storage sweep).
template <typename C>
struct EqDevT {
    C drho, ux, uy, dux, duy, uref, c0;
    __device__ __forceinline__ EqDevT(C drho_, C uref_, C dux_, C duy_)
        : drho(drho_), ux(uref_ + dux_), uy(duy_), dux(dux_), duy(duy_), uref(uref_) {
        c0 = drho * (C(1) - C(1.5) * (ux * ux + uy * uy)) - C(1.5) * (dux * (ux + uref) + duy * uy);
    }
    __device__ __forceinline__ C operator()(C ex, C ey, C w) const {
        const C eu = ex * ux + ey * uy;
        const C edu = ex * dux + ey * duy;
        return w * (c0 + drho * (C(3) * eu + C(4.5) * eu * eu) + C(3) * edu + C(4.5) * edu * (eu + ex * uref));
    }
};
using EqDev = EqDevT<float>;

// The tiles covered by the velocity-coupling stencil of a point of band B
// (local coordinates): its four rows (with walls the four fluid rows its
// weights are folded onto, wrapped within the band without) and four
// columns (wrapped at the
// band's width).  Four consecutive wrapped rows or columns can meet three
// tiles when the last tile of a band is narrower than the stencil.  Returns
// the count (at most 9) and writes the tile indices.
__device__ __forceinline__ int stencil_tiles(const Dev &d, const Band &B, float xh, float xl, float yh, float yl,
                                             int tiles[9]) {
    int ix0, iy0;
    float sx, sy;
    stencil_origin(d, B, xh, xl, yh, yl, ix0, iy0, sx, sy);
    // with walls, the four fluid rows the velocity stencil is folded onto
    if (d.walls) iy0 = min(max(iy0, 0), B.ny - 4);
    int ty[3], nty = 0;
#pragma unroll
    for (int b = 0; b < 4; b++) {
        int j = iy0 + b;
        if (d.walls) {
            if (j < 0 || j >= B.ny) continue;
        } else {
            j = wrapi(j, B.ny);
        }
        const int t = (B.y0 + j) / TILE_Y;
        bool seen = false;
        for (int k = 0; k < nty; k++) seen |= (ty[k] == t);
        if (!seen && nty < 3) ty[nty++] = t;
    }
    int tx[3], ntx = 0;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const int t = wrapi(ix0 + a, B.nx) / TILE_X;
        bool seen = false;
        for (int k = 0; k < ntx; k++) seen |= (tx[k] == t);
        if (!seen && ntx < 3) tx[ntx++] = t;
    }
    int c = 0;
    for (int a = 0; a < nty; a++)
        for (int b = 0; b < ntx; b++) tiles[c++] = ty[a] * d.ntx + tx[b];
    return c;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// Value of another lane of the same row of 16 through the DPP modifier (a
// register move, no LDS round trip).  CTRL: 0xB1 = lane i ^ 1, 0x4E = lane
// i ^ 2 (quad permutations), 0x141 = lane 7 - i within each 8 (row half
// mirror), 0x140 = lane 15 - i (row mirror).  Every lane must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum (or min, max) over each row of 16 lanes, in every lane of the row: the
// partner lanes i ^ 1, i ^ 2, then the mirrors.  Once a quad (an 8) holds one
// value in all its lanes, its mirror partner is the same as lane i ^ 4 (i ^ 8),
// so this takes the additions of the xor butterfly 1, 2, 4, 8 in its order.
template <typename Op>
__device__ __forceinline__ float row16_reduce(float v, Op op) {
    v = op(v, dpp_f<0xB1>(v));
    v = op(v, dpp_f<0x4E>(v));
    v = op(v, dpp_f<0x141>(v));
    return op(v, dpp_f<0x140>(v));
}

// The same over the whole wave, (row 0 + row 1) + (row 2 + row 3), from
// the rows' first lanes (register reads, no LDS round trip); the same in
// every lane.  Every lane must be active.
template <typename Op>
__device__ __forceinline__ float wave_total(float v, Op op) {
    v = row16_reduce(v, op);
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return op(op(r0, r1), op(r2, r3));
}

// FP64 sum over the wave in the same order, in every lane.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_total_d(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

struct OpAdd { __device__ float operator()(float a, float b) const { return a + b; } };
struct OpMin { __device__ float operator()(float a, float b) const { return fminf(a, b); } };
struct OpMax { __device__ float operator()(float a, float b) const { return fmaxf(a, b); } };

// Probe point of the element from vertex (xh + xl, yh + yl) to the next
// vertex (nxh + nxl, nyh + nyl): its midpoint moved by the probe distance
// along the element's outward normal (Sec. 2.6), as a hi/lo pair.
__device__ __forceinline__ float4 probe_point(const Dev &d, float xh, float xl, float yh, float yl, float nxh,
                                              float nxl, float nyh, float nyl) {
    const float tx = (nxh - xh) + (nxl - xl);
    const float ty = (nyh - yh) + (nyl - yl);
    const float len = sqrtf(tx * tx + ty * ty);
    return make_float4(xh, xl + (0.5f * tx + d.probe * (ty / len)), yh, yl + (0.5f * ty - d.probe * (tx / len)));
}

// Counter-based generator: Philox4x32-10 (Salmon et al., SC'11), word 0.
__device__ __forceinline__ uint32_t philox_w0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        // both halves of each 32 x 32 product from one 64-bit multiply
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
    }
    return c0;
}

}  // namespace capib
