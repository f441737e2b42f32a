// Per-node device code of the lattice sweep (Eqs. 1-6 with the Guo term of
// Eq. 4), shared by the sweep kernels and by the membrane launch that also
// sweeps a share of the far tiles.
//
// Layout: structure of arrays pop[q][j][i], i fastest, row pitch a multiple
// of 64 elements, two buffers swapped every step.  Populations are stored as
// deviations h = f - w from the rest state, FP32 or FP16 (scaled).
#pragma once
#include "capib_dev.hpp"

namespace capib {

template <typename T>
__device__ __forceinline__ T stpop(float v, float scale);
template <>
__device__ __forceinline__ float stpop<float>(float v, float) { return v; }
template <>
__device__ __forceinline__ _Float16 stpop<_Float16>(float v, float scale) { return (_Float16)(v * scale); }

// Node (i, j) of a 64x4 tile for thread t of the tile's 256: i runs along
// the wave, j is wave-uniform (one wave per row, so the row reference is
// read once per wave).
__device__ __forceinline__ void tile_node(const Dev &d, int tile, int &i, int &j, int t = threadIdx.x) {
    const int ty = tile / d.ntx;
    const int tx = tile - ty * d.ntx;
    i = tx * TILE_X + (t & (TILE_X - 1));
    j = __builtin_amdgcn_readfirstlane(ty * TILE_Y + t / TILE_X);
}

// Arithmetic of the collision.  FP32 storage collides in FP64, so that a
// stored population carries one rounding, at the store: in a nearly steady
// flow the same FP32 roundings of the arithmetic recur step after step at a
// node (the rounded weights 1/9, 1/36, 4/9 among them) and their momentum
// adds up, which a single rounding of the stored value does not.  FP16
// storage, whose own rounding is far coarser, collides in FP32.
template <typename T> struct Arith { using type = float; };
template <> struct Arith<float> { using type = double; };

__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }   // hardware, 1 ulp
__device__ __forceinline__ double recip(double x) {
    // the FP32 hardware reciprocal refined by one Newton step, which squares
    // its relative error (1e-7 -> 1e-14): 1/rho only scales deviation-sized
    // terms, so the error it leaves is far below one FP32 ulp of them
    const double r = (double)__builtin_amdgcn_rcpf((float)x);
    return r * (2.0 - x * r);
}
__device__ __forceinline__ void coll_consts(const Dev &d, float &om, float &fc) { om = d.omega; fc = d.fc; }
__device__ __forceinline__ void coll_consts(const Dev &d, double &om, double &fc) { om = d.omega64; fc = d.fc64; }
__device__ __forceinline__ void body_force(const Dev &d, float &gx, float &gy) { gx = d.gx; gy = d.gy; }
__device__ __forceinline__ void body_force(const Dev &d, double &gx, double &gy) { gx = d.gx64; gy = d.gy64; }

// The constants of band-local row jl in the arithmetic type C: the terms
// that turn pulled stored values of directions 2, 4, 5, 6, 7, 8 into
// deviations from the row's reference, and u_ref.  Every caller sweeps one
// row per wave (jl is wave-uniform), and loads them before any store of its
// own, so that they come from scalar loads.
template <typename C>
struct RowRef {
    C r2, r4, r5, r6, r7, r8, uref;
};
__device__ __forceinline__ void load_rowref(const Dev &d, int jl, RowRef<float> &c) {
    const float *R = d.rowref + 16 * __builtin_amdgcn_readfirstlane(jl);
    c.r2 = R[2]; c.r4 = R[4]; c.r5 = R[5]; c.r6 = R[6]; c.r7 = R[7]; c.r8 = R[8]; c.uref = R[9];
}
__device__ __forceinline__ void load_rowref(const Dev &d, int jl, RowRef<double> &c) {
    const double *R = d.rowref64 + 16 * __builtin_amdgcn_readfirstlane(jl);
    c.r2 = R[2]; c.r4 = R[4]; c.r5 = R[5]; c.r6 = R[6]; c.r7 = R[7]; c.r8 = R[8]; c.uref = R[9];
}
template <typename T>
using RowRefOf = RowRef<typename Arith<T>::type>;

// Pulled stored values hp as deviations from the row's reference, in the
// arithmetic type: h_i = hp_i + rowref_i.
template <typename C>
__device__ __forceinline__ void row_dev(const RowRef<C> &c, const float hp[9], C h[9]) {
#pragma unroll
    for (int q = 0; q < 9; q++) h[q] = C(hp[q]);
    h[2] += c.r2; h[4] += c.r4; h[5] += c.r5;
    h[6] += c.r6; h[7] += c.r7; h[8] += c.r8;
}

// Collision of one node from its pulled deviations h (Eq. 1 with the Guo
// term of Eq. 4), for the total force (Fx, Fy) = g + f_ib: the post-collision
// deviations out[9], in the arithmetic type C.
template <typename C>
__device__ __forceinline__ void collide_core(const Dev &d, const C h[9], C uref, C Fx, C Fy, C out[9]) {
    // moments of the streamed deviations: drho, and j - u_ref x
    const C drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const C jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
    const C jy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);

    const C rho = C(1) + drho;
    const C irho = recip(rho);
    // u = (j + F/2)/rho written as u_ref + du with du from deviations only
    const C dux = (jx + C(0.5) * Fx - drho * uref) * irho;
    const C duy = (jy + C(0.5) * Fy) * irho;
    const EqDevT<C> E(drho, uref, dux, duy);
    const C ux = E.ux, uy = E.uy;
    const C uu = ux * ux + uy * uy;
    if (!(rho > C(0)) || !(uu < C(0.03))) atomicOr(d.err, FLAG_FLUID);  // NaN fails both tests

    // s'_i = (1 - omega) dh_i + omega (h_eq_i - r_i) + F_i with the Guo term
    // F_i = (1 - omega/2) w [3 (e - u).F + 9 (e.u)(e.F)]
    C om, fc;
    coll_consts(d, om, fc);
    const C om1 = C(1) - om;
    const C uF = ux * Fx + uy * Fy;
    const C fb = C(-3) * uF;                     // 3 (-u).F
    {
        const C w = C(4) / C(9);
        out[0] = om1 * h[0] + om * E(C(0), C(0), w) + fc * w * fb;
    }
    // The other directions in opposite pairs (e, -e).  With eu = e.u,
    // edu = e.du and eF = e.F, h_eq - r splits into w S, even in e, with
    // S = c0 + 4.5 drho eu^2 + 4.5 edu (eu + e.u_ref), and w A, odd in e,
    // with A = 3 (drho eu + edu); the Guo term into fc w (fb + 9 eu eF), even,
    // and fc w 3 eF, odd.  So s'_{+-e} = (1 - omega) dh + w (P +- M).
#define CAPIB_PAIR(q, qb, ex, ey, w)                                                         \
    {                                                                                        \
        const C eu = C(ex) * ux + C(ey) * uy;                                                \
        const C edu = C(ex) * E.dux + C(ey) * E.duy;                                         \
        const C eF = C(ex) * Fx + C(ey) * Fy;                                                \
        const C S = E.c0 + C(4.5) * (drho * eu * eu + edu * (eu + C(ex) * uref));            \
        const C A = C(3) * (drho * eu + edu);                                                \
        const C P = om * S + fc * (fb + C(9) * eu * eF);                                     \
        const C M = om * A + fc * (C(3) * eF);                                               \
        out[q] = om1 * h[q] + (w) * (P + M);                                                 \
        out[qb] = om1 * h[qb] + (w) * (P - M);                                               \
    }
    CAPIB_PAIR(1, 3, 1, 0, C(1) / C(9))
    CAPIB_PAIR(2, 4, 0, 1, C(1) / C(9))
    CAPIB_PAIR(5, 7, 1, 1, C(1) / C(36))
    CAPIB_PAIR(6, 8, -1, 1, C(1) / C(36))
#undef CAPIB_PAIR
}

// Collision and store of node (i, j), with its row's constants rr, from its
// pulled stored values hp, for the immersed-boundary force (ax, ay) (the body
// force is added here).  NT: streaming (non-temporal) stores,
// for lattices much larger than the L2 caches, where the next step finds
// nothing of this step's output there anyway and keeping it only evicts
// lines that are still to be read (256-member ensemble: 5 % faster step).
// On a lattice of a few tens of MB the next step's far tiles, mapped to the
// same XCD every step, find much of it in that XCD's L2 (3840 x 240 FP32:
// 9 % slower with streaming stores).
template <typename T, bool NT = false>
__device__ __forceinline__ void lattice_collide(const Dev &d, int par, int i, int j, const RowRefOf<T> &rr,
                                                const float hp[9], float ax, float ay) {
    using C = typename Arith<T>::type;
    T *__restrict__ B = (T *)d.pop[par ^ 1];
    const long long node = (long long)j * d.pitch + i;
    C h[9], out[9], gx, gy;
    row_dev(rr, hp, h);
    body_force(d, gx, gy);
    collide_core<C>(d, h, rr.uref, gx + C(ax), gy + C(ay), out);
    const long long Q = d.qstride;
#pragma unroll
    for (int q = 0; q < 9; q++) {
        const T v = stpop<T>((float)out[q], d.scale);
        if (NT)
            __builtin_nontemporal_store(v, &B[q * Q + node]);
        else
            B[q * Q + node] = v;
    }
}

// A far tile: one that is not near in this step (its flag is clear), swept
// with the body force alone by the 256 threads t of a workgroup (or of its
// half).  b is the candidate in natural order: the tile (with several bands,
// the index into the list of tiles that hold fluid nodes).
template <typename T, int PAR, bool ENS>
__device__ __forceinline__ void far_tile(const Dev &d, int b, int t = threadIdx.x) {
    const int tile = ENS ? d.live[b] : b;
    if (d.tnear[PAR][tile]) return;
    int i, j;
    tile_node(d, tile, i, j, t);
    if (j >= d.ny) return;
    const Band B = band_at_row<ENS>(d, j);   // wave-uniform
    if (i >= B.nx) return;
    RowRefOf<T> rr;
    load_rowref(d, j - B.y0, rr);
    float h[9];
    pull9<T>(d, (const T *)d.pop[PAR], i, j, B, h);
    lattice_collide<T>(d, PAR, i, j, rr, h, 0.0f, 0.0f);
}

}  // namespace capib
