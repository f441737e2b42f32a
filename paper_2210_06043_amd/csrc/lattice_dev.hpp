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

// Collision of one node from its pulled deviations h (Eq. 1 with the Guo
// term of Eq. 4), for the total force (Fx, Fy) = g + f_ib: the post-collision
// deviations out[9].
__device__ __forceinline__ void collide_core(const Dev &d, const float h[9], float uref, float Fx, float Fy,
                                             float out[9]) {
    // moments of the streamed deviations: drho, and j - u_ref x
    const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const float jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
    const float jy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);

    const float rho = 1.0f + drho;
    const float irho = __builtin_amdgcn_rcpf(rho);   // hardware reciprocal (1 ulp)
    // u = (j + F/2)/rho written as u_ref + du with du from deviations only
    const float dux = (jx + 0.5f * Fx - drho * uref) * irho;
    const float duy = (jy + 0.5f * Fy) * irho;
    const EqDev E(drho, uref, dux, duy);
    const float ux = E.ux, uy = E.uy;
    const float uu = ux * ux + uy * uy;
    if (!(rho > 0.0f) || !(uu < 0.03f)) atomicOr(d.err, FLAG_FLUID);  // NaN fails both tests

    // s'_i = (1 - omega) dh_i + omega (h_eq_i - r_i) + F_i with the Guo term
    // F_i = (1 - omega/2) w [3 (e - u).F + 9 (e.u)(e.F)]
    const float om = d.omega, om1 = 1.0f - d.omega, fc = d.fc;
    const float uF = ux * Fx + uy * Fy;
    const float fb = -3.0f * uF;                 // 3 (-u).F
    {
        const float w = 4.0f / 9.0f;
        out[0] = om1 * h[0] + om * E(0.0f, 0.0f, w) + fc * w * fb;
    }
    // The other directions in opposite pairs (e, -e).  With eu = e.u,
    // edu = e.du and eF = e.F, h_eq - r splits into w S, even in e, with
    // S = c0 + 4.5 drho eu^2 + 4.5 edu (eu + e.u_ref), and w A, odd in e,
    // with A = 3 (drho eu + edu); the Guo term into fc w (fb + 9 eu eF), even,
    // and fc w 3 eF, odd.  So s'_{+-e} = (1 - omega) dh + w (P +- M).
#define CAPIB_PAIR(q, qb, ex, ey, w)                                                         \
    {                                                                                        \
        const float eu = (ex) * ux + (ey) * uy;                                              \
        const float edu = (ex) * E.dux + (ey) * E.duy;                                       \
        const float eF = (ex) * Fx + (ey) * Fy;                                              \
        const float S = E.c0 + 4.5f * (drho * eu * eu + edu * (eu + (ex) * uref));           \
        const float A = 3.0f * (drho * eu + edu);                                            \
        const float P = om * S + fc * (fb + 9.0f * eu * eF);                                 \
        const float M = om * A + fc * (3.0f * eF);                                           \
        out[q] = om1 * h[q] + (w) * (P + M);                                                 \
        out[qb] = om1 * h[qb] + (w) * (P - M);                                               \
    }
    CAPIB_PAIR(1, 3, 1.0f, 0.0f, 1.0f / 9.0f)
    CAPIB_PAIR(2, 4, 0.0f, 1.0f, 1.0f / 9.0f)
    CAPIB_PAIR(5, 7, 1.0f, 1.0f, 1.0f / 36.0f)
    CAPIB_PAIR(6, 8, -1.0f, 1.0f, 1.0f / 36.0f)
#undef CAPIB_PAIR
}

// Collision and store of node (i, j).  NT: streaming (non-temporal) stores,
// for lattices much larger than the L2 caches, where the next step finds
// nothing of this step's output there anyway and keeping it only evicts
// lines that are still to be read (256-member ensemble: 5 % faster step).
// On a lattice of a few tens of MB the next step's far tiles, mapped to the
// same XCD every step, find much of it in that XCD's L2 (3840 x 240 FP32:
// 9 % slower with streaming stores).
template <typename T, bool NT = false>
__device__ __forceinline__ void lattice_collide(const Dev &d, int par, int i, int j, const float h[9], float uref,
                                                float Fx, float Fy) {
    T *__restrict__ B = (T *)d.pop[par ^ 1];
    const long long node = (long long)j * d.pitch + i;
    float out[9];
    collide_core(d, h, uref, Fx, Fy, out);
    const long long Q = d.qstride;
#pragma unroll
    for (int q = 0; q < 9; q++) {
        if (NT)
            __builtin_nontemporal_store(stpop<T>(out[q], d.scale), &B[q * Q + node]);
        else
            B[q * Q + node] = stpop<T>(out[q], d.scale);
    }
}

// A far tile: one that is not near in this step (its flag is clear), swept
// with the body force alone by the 256 threads t of a workgroup (or of its
// half).  b indexes the far-tile candidates, mapped in XCD-contiguous order
// to every tile (with several bands: to every tile that holds fluid nodes).
template <typename T, int PAR, bool ENS>
__device__ __forceinline__ void far_tile(const Dev &d, int b, int t = threadIdx.x) {
    const int tile = ENS ? d.live[xcd_tile(b, d.nlive)] : xcd_tile(b, d.ntx * d.nty);
    if (d.tnear[PAR][tile]) return;
    int i, j;
    tile_node(d, tile, i, j, t);
    if (j >= d.ny) return;
    const Band B = band_at_row<ENS>(d, j);   // wave-uniform
    if (i >= B.nx) return;
    float h[9];
    const float uref = pull_dev<T>(d, (const T *)d.pop[PAR], i, j, B, h);
    lattice_collide<T>(d, PAR, i, j, h, uref, d.gx, d.gy);
}

}  // namespace capib
