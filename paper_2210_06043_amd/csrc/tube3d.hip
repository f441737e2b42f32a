// The lattice of the 3D extension (C-ABI include/capib3d.h): the BGK update of
// Eq. (1) with the equilibrium of Eq. (2), the Guo term of Eq. (4) and the
// moments of Eqs. (5)-(6) on the D3Q19 velocity set, in a capillary tube with
// halfway bounce-back walls, driven by a body force along the tube.
//
// Layout and schedule.  The geometry does not depend on x (the tube's axis),
// so every decision about a link is one of its cross-section column (y, z):
// whether the upstream node is solid (bounce-back) and, if not, which column
// it lies in.  One wave sweeps 64 consecutive x of one fluid column; its
// column's tables (19 source rows, 19 deviation constants and u_ref, FP64)
// are wave-uniform scalar loads, and solid columns are never visited.
// Populations are SoA pop[q][z][y][x] (x fastest, pitch a multiple of 64) as
// deviations s = h - r(y, z) from the equilibrium of the reference profile:
// FP32 with the collision evaluated in FP64 and each stored value rounded
// once, or FP16 scaled by a power of two with FP32 arithmetic (as the 2D
// storage modes).  Work items (column, 64-wide x segment) are ordered column-major, so
// that a contiguous range of items (one XCD's share of the workgroups) holds
// every segment of a run of neighbouring columns and their shifted pulls
// share its L2.
//
// Fixed immersed bodies (Sec. 2.2 in 3D, bodies that do not move).  Their
// stencils and weights never change, so the host lays the coupling out once:
// the slots (work items holding stencil nodes), per vertex the slot lane of
// each of its 64 stencil nodes and their weights, and per stencil node a
// contiguous range of the spread contributions W (-u*) dV that reach it, in
// vertex order.  A node lies in the stencils of some twenty vertices, so its
// velocity is computed once.  A step is three launches: k3_node_u (a wave
// per slot: the velocity of every stencil node), k3_vertex (a wave per
// vertex, a lane per stencil node: weighted wave sum to u*, and each lane's
// contribution stored at its node's place), k3_sweep_ib (a wave per slot:
// each lane sums its node's contributions in vertex order, no atomics, the
// same order on every run, and collides; then the ordinary items).  The
// first two may also take shares of the ordinary items (a schedule knob).
//
// Deformable membranes (closed triangulated surfaces: Skalak elements,
// dihedral bending, penalties on total area and enclosed volume, Secs.
// 2.2-2.4 read in 3D).  Their stencils move, so the coupling is rebuilt every
// step on the device, and every sum is taken in an order the launch fixes or
// in 64-bit fixed point (integer adds are exact, so the order does not
// matter): every run gives the same bits.  A step is three launches.
// k3_m_first: a wave per work item under the stencils (u* of its nodes,
// once per node although a node lies in some 50 stencils), a lane per
// triangle (its corner terms; the area and volume, summed per wave) and a
// lane per edge (its bending forces).  k3_m_patch: a workgroup per patch of
// 32 vertices (the host numbers each membrane's vertices by recursive
// bisection of their rest positions, so a patch is compact): each vertex's
// u* gathered from its stencil's nodes and its force from its terms, the
// vertex update and the direct force, the work items under the next step's
// stencils flagged, the patch's stencil contributions summed
// in an LDS box in 2^-50 units and added to a global force field with one
// atomic per node and component, its work items flagged.  The sweep reads and
// clears the field on flagged items.  Ligand-receptor bonds between sites on
// one membrane's triangles and the tube wall: a bound site's spring force
// (along its triangle's normal, a third per corner) joins the triangle terms.
// Each site's Bell-type decision at x^{n+1} of step n (the same Philox draw
// as the 2D library) is taken by its triangle's lane at the start of step
// n + 1, just before that lane adds the site's spring, and by k3_m_bonds
// after the last step of a call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/capib3d.h"
#include "capib_dev.hpp"

namespace tube3d {

constexpr int Q = 19;
constexpr int WAVES = 4;   // waves (work items) per workgroup
// D3Q19 in the order of the header: rest, the six axis directions, the twelve
// face diagonals, each followed by its opposite
constexpr int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__host__ __device__ constexpr double wq(int q) { return q == 0 ? 1.0 / 3.0 : q < 7 ? 1.0 / 18.0 : 1.0 / 36.0; }
__host__ __device__ constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }

struct Dev3 {
    int nx, ny, nz, pitch, ncol, nseg;
    long long qstride;          // nz * ny * pitch elements per population
    double omega, fc, gx;
    float scale, inv_scale;     // FP16 storage scale (1 for FP32)
    void *pop[2];
    const int *crow;            // [ncol][20]: own row (z ny + y), then the source row of each q (-1: bounce-back)
    const double *cK;           // [ncol][20]: deviation constant of each q, then u_ref
    double *macro;              // [4][nz][ny][nx]
    double *part;               // [nblocks][4] partial sums
    // fixed immersed bodies
    int nv, nslot;              // vertices; work items holding stencil nodes
    const int *vnode;           // [nv][64] stencil node of each lane: slot * 64 + x % 64
    const double *vW;           // [nv][64] its weight phi phi phi
    const double *vdV;          // [nv] volume weight
    const int *vpos;            // [nv][64] place of the lane's contribution in the ranges
    double *vF;                 // [nv][3] -u* of the current step
    double *contrib;            // [nv * 64][3] spread contributions, grouped by node
    double *unode;              // [3][ucap] velocity of every stencil node (slot * 64 + lane)
    long long ucap;
    const int *islot;           // [ncol * nseg] slot of a work item holding stencil nodes, -1 none
    const int *fitem;           // [nslot] work item of each slot
    const int *sbeg;            // [nslot][65] per lane, first contribution of its node
    // deformable membranes
    int nm, mv;                 // membranes, their vertices in all
    long long ms;               // stride of the coordinate planes of the vertex arrays
    long long fs;               // stride of the force field's planes: nz * ny * pitch
    double *MX[2];              // [3][ms] positions, by parity
    double *Mdxm, *MF;          // [3][ms] previous displacement, spread force
    const int *Mtri;            // [mt][3] membrane vertex indices
    const double *Mref;         // [mt][8] rest gradients g0, g1, g2 (2 each), rest area
    const int *vtb, *tslot;     // [mv + 1] starts of each vertex's corner slots; [mt][3] slot of each corner
    const int *mv0, *mnv, *mt0, *mnt;   // [nm] first vertex, vertices, first triangle, triangles
    const double *mpar;         // [nm][8] G_s, C, k_A, k_V, vertex mass, rest area, rest volume, k_b
    const int *Medge;           // [me][4] edge (x1, x2) and its opposite vertices x3, x4
    const double *Mth0;         // [me] rest dihedral angle
    const int *veb, *eslot;     // [mv + 1] starts of each vertex's edge slots; [me][4] slot of each role
    double *mtot;               // [nm][2] area and volume at the start of the last step
    const int *twave;           // [ntw][2] membrane and first triangle of each triangle wave
    const int *ewave;           // [new_][2] membrane and first edge of each edge wave
    const int *me0, *mne;       // [nm] first edge, edges
    int ntw, new_, mcap;        // triangle waves, edge waves; capacity of membranes
    double *tpart;              // [ntw][2] area and volume of each triangle wave
    // per corner slot (a vertex's slots are consecutive, its incident
    // triangles in ascending order): Skalak force, area gradient, volume
    // gradient, area / 3
    double *tcf;                // [3 mt][10]
    double *ecf;                // [4 me][3] bending force on one of an edge's four vertices
    const int *ptab;            // [npatch][5] first vertex, vertices, membrane, its first triangle wave, its waves
    unsigned long long *mforce; // [3][fs] spread force, fixed point (2^-50)
    int *mflag;                 // [ncol * nseg] work item with spread force
    double *Mu;                 // [fs][4] u* of the nodes under this step's stencils (x, y, z, unused)
    int *uflag;                 // [ncol * nseg] work item holding nodes under this step's stencils
    // bonds
    int ns;                     // sites
    const int *Stri;            // [ns] triangle (global)
    const double *Sbary;        // [ns][2] barycentric weights of corners 1 and 2
    int *Sbound;                // [ns] bound
    double *Sanc;               // [ns][3] anchor
    const int *tsb, *tsl;       // sites of each triangle: [mt + 1] starts, site indices
    double b_sigma, b_yeq, b_ycr, b_kf, b_kr0, b_lb, radius;
    unsigned long long b_seed;
    const int *colof;           // [nz][ny] column of a row, -1 solid
    int *err;                   // error flags
};

constexpr double FIX_ONE = 1125899906842624.0;   // 2^50, spread contributions
constexpr int ERR_STENCIL = 1, ERR_FORCE = 2;

// Workgroup b -> work item such that each XCD (workgroups dealt round-robin
// to the 8 XCDs) holds one contiguous range of items.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// Arithmetic of the collision: FP64 for FP32 storage, FP32 for FP16.
template <typename T> struct Arith3 { using type = float; };
template <> struct Arith3<float> { using type = double; };
__device__ __forceinline__ float ld3(const float *p, float) { return *p; }
__device__ __forceinline__ float ld3(const _Float16 *p, float is) { return (float)(*p) * is; }
__device__ __forceinline__ void st3(float *p, float v, float) { *p = v; }
__device__ __forceinline__ void st3(_Float16 *p, float v, float sc) { *p = (_Float16)(v * sc); }

// The wave's work item: its column c and x of this lane; false past the end.
__device__ __forceinline__ bool item_of(const Dev3 &d, int &c, int &x, int &item) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    item = __builtin_amdgcn_readfirstlane(b * WAVES + (int)(threadIdx.x >> 6));
    if (item >= d.ncol * d.nseg) return false;
    c = item / d.nseg;
    const int seg = item - c * d.nseg;
    x = seg * 64 + (int)(threadIdx.x & 63);
    return true;
}
__device__ __forceinline__ bool item_of(const Dev3 &d, int &c, int &x) {
    int item;
    return item_of(d, c, x, item);
}

// Pulled populations of node x of column c as deviations from its column's
// reference, in the arithmetic type C: dh_q = s_q(source) + K_q.  Returns u_ref.
template <typename T, typename C, int PAR>
__device__ __forceinline__ C pull_t(const Dev3 &d, const int *crow, const double *cK, int c, int x, C dh[Q],
                                    long long &own) {
    const int *R = crow + 20 * c;
    const double *K = cK + 20 * c;
    const T *A = (const T *)d.pop[PAR];
    own = (long long)R[0] * d.pitch + x;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int rs = R[1 + q];
        float v;
        if (rs < 0) {
            v = ld3(A + opp(q) * d.qstride + own, d.inv_scale);
        } else {
            int xs = x - EX[q];
            xs = xs < 0 ? xs + d.nx : xs >= d.nx ? xs - d.nx : xs;
            v = ld3(A + q * d.qstride + (long long)rs * d.pitch + xs, d.inv_scale);
        }
        dh[q] = (C)v + (C)K[q];
    }
    return (C)K[19];
}
template <typename T, typename C, int PAR>
__device__ __forceinline__ C pull(const Dev3 &d, int c, int x, C dh[Q], long long &own) {
    return pull_t<T, C, PAR>(d, d.crow, d.cK, c, x, dh, own);
}
// The same for a latency-bound caller with a wave-uniform column c and
// read-only tables: every table entry read before any population, so the
// entries' loads go out together, then the 19 loads.
template <typename T, typename C, int PAR>
__device__ __forceinline__ C pull_u(const Dev3 &d, const int *__restrict__ crow, const double *__restrict__ cK, int c,
                                    int x, C dh[Q], long long &own) {
    int R[20];
    double K[20];
#pragma unroll
    for (int q = 0; q < 20; q++) {
        R[q] = crow[20 * c + q];
        K[q] = cK[20 * c + q];
    }
    const T *A = (const T *)d.pop[PAR];
    own = (long long)R[0] * d.pitch + x;
    float v[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int rs = R[1 + q];
        int xs = x - EX[q];
        xs = xs < 0 ? xs + d.nx : xs >= d.nx ? xs - d.nx : xs;
        v[q] = ld3(A + (rs < 0 ? opp(q) * d.qstride + own : q * d.qstride + (long long)rs * d.pitch + xs), d.inv_scale);
    }
#pragma unroll
    for (int q = 0; q < Q; q++) dh[q] = (C)v[q] + (C)K[q];
    return (C)K[19];
}

// One work item (wave-uniform): pull, moments, BGK collision with the Guo
// term for the body force plus, on a slot (an item holding stencil nodes of
// the fixed bodies), the spread force of each lane's node.
// MODE 0: body force only; 1: a slot of fixed bodies (spread force from its
// contribution ranges); 2: the membranes' fixed-point field, read and cleared
// on flagged items.
template <typename T, int PAR, int MODE>
__device__ __forceinline__ void sweep_item(const Dev3 &d, int item, int slot) {
    using C = typename Arith3<T>::type;
    const int c = item / d.nseg;
    const int x = (item - c * d.nseg) * 64 + (int)(threadIdx.x & 63);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (x >= d.nx) return;
    if (MODE == 1) {
        const int *sb = d.sbeg + 65 * slot + (threadIdx.x & 63);
        const int k1 = sb[1];
#pragma unroll 4
        for (int k = sb[0]; k < k1; k++) {
            const double *p = d.contrib + 3 * (long long)k;
            fx += p[0];
            fy += p[1];
            fz += p[2];
        }
    }
    C h[Q];
    long long own;
    const C ur = pull<T, C, PAR>(d, c, x, h, own);
    // the membranes' field, read (and cleared) on flagged items after the
    // pulls are issued, so that the flag does not hold them back
    if (MODE == 2 && d.mflag[item]) {
        unsigned long long *p = d.mforce + own;
        fx = (double)(long long)p[0] / FIX_ONE;
        fy = (double)(long long)p[d.fs] / FIX_ONE;
        fz = (double)(long long)p[2 * d.fs] / FIX_ONE;
        p[0] = 0;
        p[d.fs] = 0;
        p[2 * d.fs] = 0;
        if ((threadIdx.x & 63) == 0) d.mflag[item] = 0;
    }
    const C Fx = (C)d.gx + (C)fx, Fy = (C)fy, Fz = (C)fz;
    // moments of the deviations: drho, and j - (u_ref, 0, 0)
    C drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        drho += h[q];
        jx += (C)EX[q] * h[q];
        jy += (C)EY[q] * h[q];
        jz += (C)EZ[q] * h[q];
    }
    const C rho = C(1) + drho;
    // 1/rho: the FP32 hardware reciprocal, refined by one Newton step in FP64
    // (relative error ~1e-14; it only scales deviation-sized terms)
    C ir = (C)__builtin_amdgcn_rcpf((float)rho);
    if (sizeof(C) == 8) ir = ir * (C(2) - rho * ir);
    const C dux = (jx + C(0.5) * Fx - drho * ur) * ir, duy = (jy + C(0.5) * Fy) * ir, duz = (jz + C(0.5) * Fz) * ir;
    const C ux = ur + dux, uy = duy, uz = duz;
    const C uu = ux * ux + uy * uy + uz * uz;
    // Eq. (2) as a deviation from the reference, every term carrying drho or du:
    // h_eq - r = w [c0 + drho (3 eu + 4.5 eu^2) + 3 edu + 4.5 edu (eu + e.u_ref)]
    const C c0 = drho * (C(1) - C(1.5) * uu) - C(1.5) * (dux * (ux + ur) + duy * uy + duz * uz);
    const C om = (C)d.omega, om1 = C(1) - om, fc = (C)d.fc;
    const C fb = C(-3) * (ux * Fx + uy * Fy + uz * Fz);   // 3 (-u).F
    T *B = (T *)d.pop[PAR ^ 1];
    st3(B + own, (float)(om1 * h[0] + om * (C)wq(0) * c0 + fc * (C)wq(0) * fb), d.scale);
    // opposite pairs (q, q + 1): even part S, odd part M, as in the 2D sweep
#pragma unroll
    for (int q = 1; q < Q; q += 2) {
        const C eu = (C)EX[q] * ux + (C)EY[q] * uy + (C)EZ[q] * uz;
        const C edu = (C)EX[q] * dux + (C)EY[q] * duy + (C)EZ[q] * duz;
        const C eF = (C)EX[q] * Fx + (C)EY[q] * Fy + (C)EZ[q] * Fz;
        const C S = c0 + C(4.5) * (drho * eu * eu + edu * (eu + (C)EX[q] * ur));
        const C A = C(3) * (drho * eu + edu);
        const C P = om * S + fc * (fb + C(9) * eu * eF);
        const C M = om * A + fc * (C(3) * eF);
        st3(B + q * d.qstride + own, (float)(om1 * h[q] + (C)wq(q) * (P + M)), d.scale);
        st3(B + (q + 1) * d.qstride + own, (float)(om1 * h[q + 1] + (C)wq(q) * (P - M)), d.scale);
    }
}


template <typename T, int PAR, int MODE>
__global__ __launch_bounds__(64 * WAVES) void k3_sweep(Dev3 d) {
    int c, x, item;
    if (!item_of(d, c, x, item)) return;
    sweep_item<T, PAR, MODE>(d, item, -1);
}

// The ordinary part of a launch with fixed bodies: workgroups from nfront on
// (nfront a multiple of 8, so each keeps its XCD) sweep the items [lo, hi)
// that hold no stencil node.
template <typename T, int PAR>
__device__ __forceinline__ void sweep_share(const Dev3 &d, int nfront, int lo, int hi) {
    const int b = xcd_block((int)blockIdx.x - nfront, (int)gridDim.x - nfront);
    const int item = __builtin_amdgcn_readfirstlane(lo + b * WAVES + (int)(threadIdx.x >> 6));
    if (item >= hi || d.islot[item] >= 0) return;
    sweep_item<T, PAR, 0>(d, item, -1);
}

// First launch of a step with fixed bodies: workgroups [0, nfb) give every
// slot a wave that stores the velocity of the streamed populations with half
// the body force (FP64) at its nodes; the rest sweep the items [0, s1).
template <typename T, int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_node_u(Dev3 d, int nfb, int s1) {
    if ((int)blockIdx.x >= nfb) {
        sweep_share<T, PAR>(d, nfb, 0, s1);
        return;
    }
    const int slot = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WAVES + (int)(threadIdx.x >> 6));
    if (slot >= d.nslot) return;
    const int item = d.fitem[slot], c = item / d.nseg, lane = (int)(threadIdx.x & 63);
    const int x = (item - c * d.nseg) * 64 + lane;
    if (x >= d.nx) return;
    double h[Q];
    long long own;
    const double ur = pull<T, double, PAR>(d, c, x, h, own);
    double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int q = 0; q < Q; q++) {
        drho += h[q];
        jx += EX[q] * h[q];
        jy += EY[q] * h[q];
        jz += EZ[q] * h[q];
    }
    const double rho = 1.0 + drho;
    const long long k = 64LL * slot + lane;
    d.unode[k] = ur + (jx + 0.5 * d.gx - drho * ur) / rho;
    d.unode[d.ucap + k] = jy / rho;
    d.unode[2 * d.ucap + k] = jz / rho;
}

// Second launch: workgroups [0, nvb) give every vertex a wave, a lane per
// stencil node: u* is the weighted wave sum of the nodes' velocities; stores
// -u* and each lane's contribution W (-u*) dV.  The rest sweep [s1, s2).
template <typename T, int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_vertex(Dev3 d, int nvb, int s1, int s2) {
    if ((int)blockIdx.x >= nvb) {
        sweep_share<T, PAR>(d, nvb, s1, s2);
        return;
    }
    const int v = blockIdx.x * WAVES + (int)(threadIdx.x >> 6);
    if (v >= d.nv) return;
    const int l = 64 * v + (int)(threadIdx.x & 63);
    const long long k = d.vnode[l];
    const double W = d.vW[l];
    double ux = W * d.unode[k], uy = W * d.unode[d.ucap + k], uz = W * d.unode[2 * d.ucap + k];
    for (int o = 32; o >= 1; o >>= 1) {
        ux += __shfl_xor(ux, o);
        uy += __shfl_xor(uy, o);
        uz += __shfl_xor(uz, o);
    }
    if ((threadIdx.x & 63) == 0) {
        d.vF[3 * v] = -ux;
        d.vF[3 * v + 1] = -uy;
        d.vF[3 * v + 2] = -uz;
    }
    const double dV = d.vdV[v];
    double *p = d.contrib + 3 * (long long)d.vpos[l];
    p[0] = W * -ux * dV;
    p[1] = W * -uy * dV;
    p[2] = W * -uz * dV;
}

// Third launch: workgroups [0, nfb) sweep the slots with their spread force,
// the rest the items [s2, ncol * nseg).
template <typename T, int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_sweep_ib(Dev3 d, int nfb, int s2) {
    if ((int)blockIdx.x >= nfb) {
        sweep_share<T, PAR>(d, nfb, s2, d.ncol * d.nseg);
        return;
    }
    const int slot = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WAVES + (int)(threadIdx.x >> 6));
    if (slot >= d.nslot) return;
    sweep_item<T, PAR, 1>(d, d.fitem[slot], slot);
}

// ---- deformable membranes --------------------------------------------------

__device__ __forceinline__ double phi_cos(double r) {
    r = fabs(r);
    return r < 2.0 ? 0.25 * (1.0 + cos(M_PI * r / 2.0)) : 0.0;
}

__device__ __forceinline__ void cross(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Bond kinetics of site q at the end of step n, at its position ps at
// x^{n+1}.  The draw is word 0 of Philox4x32-10 with key (seed low, seed high)
// and counter (n low, site, n high, 0), top 24 bits over 2^24.  Bound: it
// breaks if the draw is below 1 - exp(-k_r0 exp(|y_l - y_eq| / l_B)).
// Unbound within y_cr of the wall (R minus the site's distance from the
// axis): it binds if the draw is below 1 - exp(-k_f), anchored on the wall
// radially outward of the site.
__device__ __forceinline__ void bond_decide(const Dev3 &d, int q, const double ps[3], long long step) {
    const uint32_t w0 = capib::philox_w0((uint32_t)((unsigned long long)step & 0xffffffffu), (uint32_t)q,
                                         (uint32_t)((unsigned long long)step >> 32), 0u,
                                         (uint32_t)(d.b_seed & 0xffffffffu), (uint32_t)(d.b_seed >> 32));
    const double r = (double)(w0 >> 8) * (1.0 / 16777216.0);
    if (d.Sbound[q]) {
        double dl2 = 0.0;
        for (int u = 0; u < 3; u++) {
            const double dl = ps[u] - d.Sanc[3 * q + u];
            dl2 += dl * dl;
        }
        const double P = 1.0 - exp(-d.b_kr0 * exp(fabs(sqrt(dl2) - d.b_yeq) / d.b_lb));
        if (r < P) d.Sbound[q] = 0;
    } else {
        const double yc = 0.5 * (d.ny - 1), zc = 0.5 * (d.nz - 1);
        const double dy = ps[1] - yc, dz = ps[2] - zc, rho = sqrt(dy * dy + dz * dz);
        const double P = 1.0 - exp(-d.b_kf);
        if (d.radius - rho < d.b_ycr && r < P) {
            d.Sbound[q] = 1;
            d.Sanc[3 * q] = ps[0];
            d.Sanc[3 * q + 1] = yc + d.radius * dy / rho;
            d.Sanc[3 * q + 2] = zc + d.radius * dz / rho;
        }
    }
}

// The bond kinetics of step n at x^{n+1} (positions of parity mp), a thread
// per site: after the last step of a call (the steps before it leave theirs
// to the next step's triangle lanes).
__global__ __launch_bounds__(256) void k3_m_bonds(Dev3 d, int mp, long long step) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= d.ns) return;
    const int *T = d.Mtri + 3 * d.Stri[q];
    const double *X = d.MX[mp];
    const double b1 = d.Sbary[2 * q], b2 = d.Sbary[2 * q + 1];
    double ps[3];
    for (int u = 0; u < 3; u++) {
        const double xa = X[u * d.ms + T[0]];
        ps[u] = xa + b1 * (X[u * d.ms + T[1]] - xa) + b2 * (X[u * d.ms + T[2]] - xa);
    }
    bond_decide(d, q, ps, step);
}

// u* = (j + g/2) / rho (the velocity of the streamed populations with half
// the body force) at every node of the flagged work items, into Mu, and the
// flags cleared.  Wave w < nw of the launch takes the items w, w + nw, ...,
// their flags loaded together, one lane each.
template <typename T, int PAR>
__device__ __forceinline__ void nodeu_waves(const Dev3 &d, const int *__restrict__ crow,
                                            const double *__restrict__ cK, int nw, int blk) {
    const int w = __builtin_amdgcn_readfirstlane(blk * WAVES + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (w >= nw) return;   // the grid's last workgroup may hold more waves
    const int nitem = d.ncol * d.nseg;
    const int mine = w + lane * nw;
    const bool on = lane * nw < nitem && mine < nitem && d.uflag[mine];
    for (unsigned long long m = __ballot(on); m; m &= m - 1ull) {
        const int k = __ffsll((long long)m) - 1;
        const int item = __builtin_amdgcn_readfirstlane(w + k * nw);
        const int c = item / d.nseg, x = (item - c * d.nseg) * 64 + lane;
        if (x < d.nx) {
            double h[Q];
            long long own;
            // the column tables come in as read-only kernel arguments, so
            // that their wave-uniform entries are scalar loads issued
            // together rather than a vector load and a wait per population
            const double ur = pull_u<T, double, PAR>(d, crow, cK, c, x, h, own);
            double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
            for (int q = 0; q < Q; q++) {
                drho += h[q];
                jx += EX[q] * h[q];
                jy += EY[q] * h[q];
                jz += EZ[q] * h[q];
            }
            const double rho = 1.0 + drho;
            double4 *o = (double4 *)d.Mu + own;
            *o = make_double4(ur + (jx + 0.5 * d.gx - drho * ur) / rho, jy / rho, jz / rho, 0.0);
        }
    }
    if (on) d.uflag[mine] = 0;
}

// First launch of a step with membranes (positions x^n of parity mp).
// Workgroups [0, ntb): a wave per 64 triangles of one membrane, a lane per triangle: for each
// corner a, the Skalak force -A0 [w1 2 F g_a + w2 2 det C F C^-1 g_a], the
// area gradient n x (x_c - x_b) / 2 and the volume gradient
// (x_b - r0) x (x_c - r0) / 6 ((a, b, c) in the triangle's cyclic order),
// and a third of the area; the area and volume terms (about the membrane's
// first vertex r0) summed over the wave into the wave's own pair of partial
// sums.  [ntb, nte): a wave per 64 edges of one membrane, a lane per edge:
// the bending force -k_b sin(theta - theta0) grad theta on its four
// vertices.  The rest: nodeu_waves over nuw waves (dispatched last: the
// triangle and edge waves have the longer chains).
// The three parts are independent latency chains, so they share a launch.
template <typename T, int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_m_first(Dev3 d, const int *__restrict__ crow,
                                                         const double *__restrict__ cK, int mp, int nte, int nuw,
                                                         int ntb, long long kstep) {
    if ((int)blockIdx.x >= nte) {
        nodeu_waves<T, PAR>(d, crow, cK, nuw, (int)blockIdx.x - nte);
        return;
    }
    const int lane = threadIdx.x & 63;
    const double *X = d.MX[mp];
    const int bx = (int)blockIdx.x;
    if (bx >= ntb) {
        const int ew = (bx - ntb) * WAVES + (int)(threadIdx.x >> 6);
        if (ew >= d.new_) return;
        const int m = d.ewave[2 * ew], k = d.ewave[2 * ew + 1] + lane;
        if (k >= d.me0[m] + d.mne[m]) return;
        // theta = atan2((n1 x n2).e, n1.n2) at edge (x1, x2) between the faces
        // (x1, x2, x3) and (x2, x1, x4): l = |e|, e = x2 - x1,
        // N1 = e x (x3 - x1), N2 = -e x (x4 - x2), g3 = -l N1/|N1|^2,
        // g4 = -l N2/|N2|^2, g1 = ((x3 - x2).e/l^2) g3 + ((x4 - x2).e/l^2) g4,
        // g2 = -(g1 + g3 + g4)
        const int *E = d.Medge + 4 * k;
        const int es[4] = {d.eslot[4 * k], d.eslot[4 * k + 1], d.eslot[4 * k + 2], d.eslot[4 * k + 3]};
        double y[4][3];
        for (int s = 0; s < 4; s++)
            for (int u = 0; u < 3; u++) y[s][u] = X[u * d.ms + E[s]];
        const double e[3] = {y[1][0] - y[0][0], y[1][1] - y[0][1], y[1][2] - y[0][2]};
        const double me[3] = {-e[0], -e[1], -e[2]};
        const double a3[3] = {y[2][0] - y[0][0], y[2][1] - y[0][1], y[2][2] - y[0][2]};
        const double b4[3] = {y[3][0] - y[1][0], y[3][1] - y[1][1], y[3][2] - y[1][2]};
        double N1[3], N2[3], n1[3], n2[3], c12[3];
        cross(e, a3, N1);
        cross(me, b4, N2);
        const double l2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2], l = sqrt(l2);
        const double q1 = N1[0] * N1[0] + N1[1] * N1[1] + N1[2] * N1[2];
        const double q2 = N2[0] * N2[0] + N2[1] * N2[1] + N2[2] * N2[2];
        const double r1 = sqrt(q1), r2 = sqrt(q2);
        for (int u = 0; u < 3; u++) {
            n1[u] = N1[u] / r1;
            n2[u] = N2[u] / r2;
        }
        cross(n1, n2, c12);
        const double th = atan2((c12[0] * e[0] + c12[1] * e[1] + c12[2] * e[2]) / l,
                                n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2]);
        const double sb = -d.mpar[8 * m + 7] * sin(th - d.Mth0[k]);
        const double w3 = ((y[2][0] - y[1][0]) * e[0] + (y[2][1] - y[1][1]) * e[1] + (y[2][2] - y[1][2]) * e[2]) / l2;
        const double w4 = ((y[3][0] - y[1][0]) * e[0] + (y[3][1] - y[1][1]) * e[1] + (y[3][2] - y[1][2]) * e[2]) / l2;
        // into the slots of the four vertices' edge terms
        double *o1 = d.ecf + 3 * (long long)es[0], *o2 = d.ecf + 3 * (long long)es[1];
        double *o3 = d.ecf + 3 * (long long)es[2], *o4 = d.ecf + 3 * (long long)es[3];
        for (int u = 0; u < 3; u++) {
            const double g3 = -l * N1[u] / q1, g4 = -l * N2[u] / q2, g1 = w3 * g3 + w4 * g4;
            o1[u] = sb * g1;
            o2[u] = sb * -(g1 + g3 + g4);
            o3[u] = sb * g3;
            o4[u] = sb * g4;
        }
        return;
    }
    {
        const int tw = bx * WAVES + (int)(threadIdx.x >> 6);
        if (tw >= d.ntw) return;
        const int m = d.twave[2 * tw], t = d.twave[2 * tw + 1] + lane;
        double A = 0.0, V = 0.0;
        if (t < d.mt0[m] + d.mnt[m]) {
            const double *P = d.mpar + 8 * m;
            const int *tv = d.Mtri + 3 * t;
            const int ts[3] = {d.tslot[3 * t], d.tslot[3 * t + 1], d.tslot[3 * t + 2]};
            const double *g = d.Mref + 8 * t;
            const int r0 = d.mv0[m];
            double x[3][3], xr[3][3];
            for (int s = 0; s < 3; s++)
                for (int u = 0; u < 3; u++) {
                    x[s][u] = X[u * d.ms + tv[s]];
                    xr[s][u] = x[s][u] - X[u * d.ms + r0];
                }
            double F[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
            for (int s = 0; s < 3; s++)
                for (int u = 0; u < 3; u++) {
                    F[u][0] += x[s][u] * g[2 * s];
                    F[u][1] += x[s][u] * g[2 * s + 1];
                }
            double Cm[2][2];
            for (int r = 0; r < 2; r++)
                for (int w = 0; w < 2; w++) Cm[r][w] = F[0][r] * F[0][w] + F[1][r] * F[1][w] + F[2][r] * F[2][w];
            const double I1 = Cm[0][0] + Cm[1][1] - 2.0, I2 = Cm[0][0] * Cm[1][1] - Cm[0][1] * Cm[1][0] - 1.0;
            const double w1 = 0.25 * P[0] * (2.0 * I1 + 2.0), w2 = 0.25 * P[0] * (-2.0 + 2.0 * P[1] * I2);
            const double det = Cm[0][0] * Cm[1][1] - Cm[0][1] * Cm[1][0];
            const double Ci[2][2] = {{Cm[1][1] / det, -Cm[0][1] / det}, {-Cm[1][0] / det, Cm[0][0] / det}};
            const double e1[3] = {x[1][0] - x[0][0], x[1][1] - x[0][1], x[1][2] - x[0][2]};
            const double e2[3] = {x[2][0] - x[0][0], x[2][1] - x[0][1], x[2][2] - x[0][2]};
            double n[3];
            cross(e1, e2, n);
            const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            for (int u = 0; u < 3; u++) n[u] /= nn;
            double fc[3][3];   // each corner's force, stored after the bond springs are added
            for (int a = 0; a < 3; a++) {
                double *out = d.tcf + 10 * (long long)ts[a];   // corner a's slot
                const int b = a == 2 ? 0 : a + 1, c = a == 0 ? 2 : a - 1;
                const double ga[2] = {g[2 * a], g[2 * a + 1]};
                const double Cg[2] = {Ci[0][0] * ga[0] + Ci[0][1] * ga[1], Ci[1][0] * ga[0] + Ci[1][1] * ga[1]};
                double pb[3], pc[3], rb[3], rc[3];
                for (int u = 0; u < 3; u++) {
                    pb[u] = b == 0 ? x[0][u] : b == 1 ? x[1][u] : x[2][u];
                    pc[u] = c == 0 ? x[0][u] : c == 1 ? x[1][u] : x[2][u];
                    rb[u] = b == 0 ? xr[0][u] : b == 1 ? xr[1][u] : xr[2][u];
                    rc[u] = c == 0 ? xr[0][u] : c == 1 ? xr[1][u] : xr[2][u];
                }
                const double cb[3] = {pc[0] - pb[0], pc[1] - pb[1], pc[2] - pb[2]};
                double nbc[3], bc[3];
                cross(n, cb, nbc);
                cross(rb, rc, bc);
                for (int u = 0; u < 3; u++) {
                    const double Fg = F[u][0] * ga[0] + F[u][1] * ga[1];
                    const double FCg = F[u][0] * Cg[0] + F[u][1] * Cg[1];
                    fc[a][u] = -g[6] * (w1 * 2.0 * Fg + w2 * 2.0 * det * FCg);
                    out[3 + u] = 0.5 * nbc[u];
                    out[6 + u] = bc[u] / 6.0;
                }
                out[9] = 0.5 * nn / 3.0;
            }
            // the sites on this triangle: first (kstep >= 0) the previous
            // step's bond kinetics at these positions, x^{n+1} of that step;
            // then for every bound site sigma (y_l - y_eq) along n, a third
            // per corner
            for (int k = d.ns > 0 ? d.tsb[t] : 0; d.ns > 0 && k < d.tsb[t + 1]; k++) {
                const int q = d.tsl[k];
                const double b1 = d.Sbary[2 * q], b2 = d.Sbary[2 * q + 1];
                double ps[3];
                for (int u = 0; u < 3; u++) ps[u] = x[0][u] + b1 * e1[u] + b2 * e2[u];
                if (kstep >= 0) bond_decide(d, q, ps, kstep);
                if (!d.Sbound[q]) continue;
                double dl2 = 0.0;
                for (int u = 0; u < 3; u++) {
                    const double dl = ps[u] - d.Sanc[3 * q + u];
                    dl2 += dl * dl;
                }
                const double f = d.b_sigma * (sqrt(dl2) - d.b_yeq);
                for (int a = 0; a < 3; a++)
                    for (int u = 0; u < 3; u++) fc[a][u] += f / 3.0 * n[u];
            }
            for (int a = 0; a < 3; a++)
                for (int u = 0; u < 3; u++) d.tcf[10 * (long long)ts[a] + u] = fc[a][u];
            A = 0.5 * nn;
            // the volume term about r0, from the corners relative to r0
            double qr[3];
            cross(xr[1], xr[2], qr);
            V = (xr[0][0] * qr[0] + xr[0][1] * qr[1] + xr[0][2] * qr[2]) / 6.0;
        }
        for (int o = 32; o >= 1; o >>= 1) {
            A += __shfl_xor(A, o);
            V += __shfl_xor(V, o);
        }
        if (lane == 0) {
            d.tpart[2 * tw] = A;
            d.tpart[2 * tw + 1] = V;
        }
    }
}

// Flags the work items that hold the stencil nodes of vertex position X
// (columns outside the fluid are left to the spreading's check): plain
// stores of 1, so that any number of writers agree.  b, c: the stencil's y
// and z offsets.
__device__ __forceinline__ int stencil_col(const Dev3 &d, int oy, int oz, int b, int c) {
    const int y = oy + b, z = oz + c;
    return (y >= 0 && y < d.ny && z >= 0 && z < d.nz) ? d.colof[z * d.ny + y] : -1;
}
__device__ __forceinline__ void flag_col_items(const Dev3 &d, int col, int ox) {
    const int x0 = (ox % d.nx + d.nx) % d.nx, x3 = ((ox + 3) % d.nx + d.nx) % d.nx;
    d.uflag[col * d.nseg + x0 / 64] = 1;
    d.uflag[col * d.nseg + x3 / 64] = 1;   // the stencil's 4 nodes span at most two items
}
__device__ __forceinline__ void flag_stencil_items(const Dev3 &d, int ox, int oy, int oz, int b, int c) {
    const int col = stencil_col(d, oy, oz, b, c);
    if (col >= 0) flag_col_items(d, col, ox);
}

// The items under the stencils of positions mp, for a step whose positions
// the previous step did not write (new membranes, positions set from the
// host): a thread per (vertex, stencil column).
__global__ __launch_bounds__(256) void k3_m_umark(Dev3 d, int mp) {
    const int i = blockIdx.x * 256 + threadIdx.x, v = i >> 4;
    if (v >= d.mv) return;
    const double *X = d.MX[mp];
    const int ox = (int)floor(X[v]) - 1, oy = (int)floor(X[d.ms + v]) - 1, oz = (int)floor(X[2 * d.ms + v]) - 1;
    flag_stencil_items(d, ox, oy, oz, i & 3, (i >> 2) & 3);
}

constexpr int PATCH_THREADS = 256;
constexpr int PATCH_V = 32;   // vertices of a patch (the host's numbering makes them compact)
// a vertex's gathers are split PATCH_THREADS / PATCH_V ways: its u* by z
// layer and by PATCH_ROWS groups of stencil rows, its terms into PATCH_FR parts
constexpr int PATCH_FR = PATCH_THREADS / PATCH_V, PATCH_ROWS = PATCH_FR / 4;
static_assert(PATCH_FR % 4 == 0 && 4 % PATCH_ROWS == 0, "whole layers and rows per thread");
constexpr int NODEU_WAVES = 16384;   // waves of nodeu_waves below 64 x 16384 items (one item each below 16384)
constexpr int BOX = 12;   // edge of the LDS box of a patch's stencils

// Second launch: a workgroup per patch (up to 32 consecutive vertices of one
// membrane, numbered by the host so that a patch is compact).  The first wave
// adds the membrane's triangle waves' area and volume (lane k the waves k,
// k + 64, ..., then across the lanes) while the second and third put each
// vertex's stencil at x^n (origin and weights, four threads per vertex)
// into LDS and the fourth its fluid mask.  Vertex v = first + j: u*
// interpolated from its stencil's nodes (the cosine delta of the coupling),
// its force gathered from the corner terms of its triangles (Skalak
// - (k_A (A - A0)/A0) area gradient - (k_V (V - V0)/V0) volume gradient) and
// the bending terms of its edges, dV the sum of the thirds of their areas,
// the terms split eight ways (part r the entries r, r + 8, ...; the eight
// parts added in order); then thread j: dx = u* + f/(2m),
// x^{n+1} = x^n + dx, U = 3/2 dx - 1/2 dx_prev, F = (U - u*) dV, and the
// work items under the stencil of x^{n+1} flagged for the next step's u*.
// Then the patch's 32 x 64 contributions W F are added in 2^-50 units into
// an LDS box over its stencils (integer adds: the order does not matter),
// and the box is added to the global field with one integer atomic per node
// and component, flagging each node's work item; a patch whose box exceeds
// BOX^3 adds its contributions to the field directly.
__global__ __launch_bounds__(PATCH_THREADS) void k3_m_patch(Dev3 d, int mp) {
    __shared__ double sw[PATCH_V][12];
    __shared__ double sF[PATCH_V][3];
    __shared__ int so[PATCH_V][3];
    __shared__ int sbox[6];
    __shared__ unsigned long long box[BOX * BOX * BOX][3];
    __shared__ double sp[PATCH_FR][PATCH_V][4];
    __shared__ double stot[2];
    __shared__ int sno[PATCH_V][3];   // stencil origins of x^{n+1}
    __shared__ double sus[PATCH_ROWS][4][PATCH_V][3];   // u* of each vertex, by row group and z layer
    __shared__ int smask[PATCH_V];          // bit b + 4 c: column (b, c) of the stencil at x^n is fluid
    const int t = threadIdx.x, p = blockIdx.x;
    const int pv0 = d.ptab[5 * p], pn = d.ptab[5 * p + 1], m = d.ptab[5 * p + 2];
    const int tw0 = d.ptab[5 * p + 3], ntw = d.ptab[5 * p + 4];
    const double *X = d.MX[mp];
    static_assert(4 * PATCH_V <= 128, "four threads per vertex in the second and third waves");
    if (t >= 64 && t < 64 + 4 * pn) {
        // the stencil of x^n of vertex pv0 + (t - 64) / 4: its origin, and
        // the weights of stencil offset k4 = (t - 64) % 4 along each axis
        const int j = (t - 64) >> 2, k4 = (t - 64) & 3, v = pv0 + j;
        for (int u = 0; u < 3; u++) {
            const double xu = X[u * d.ms + v];
            const int o = (int)floor(xu) - 1;
            if (k4 == 0) so[j][u] = o;
            sw[j][4 * u + k4] = phi_cos(xu - (o + k4));
        }
    } else if (t >= 192 && t < 192 + pn) {
        // which of the 16 columns of the same stencil are fluid (the loads
        // issued together); a stencil that reaches outside the fluid raises
        // the error flag
        const int j = t - 192, v = pv0 + j;
        const int oy = (int)floor(X[d.ms + v]) - 1, oz = (int)floor(X[2 * d.ms + v]) - 1;
        int cl[16];
#pragma unroll
        for (int k = 0; k < 16; k++) cl[k] = stencil_col(d, oy, oz, k & 3, k >> 2);
        int mask = 0;
#pragma unroll
        for (int k = 0; k < 16; k++) mask |= (cl[k] >= 0 ? 1 : 0) << k;
        smask[j] = mask;
        if (mask != 0xFFFF) atomicOr(d.err, ERR_STENCIL);
    }
    if (t < 64) {
        // the membrane's area and volume: its triangle waves' sums added over
        // the lanes in a fixed order
        double a = 0.0, b = 0.0;
        for (int k = t; k < ntw; k += 64) {
            a += d.tpart[2 * (tw0 + k)];
            b += d.tpart[2 * (tw0 + k) + 1];
        }
        for (int o = 32; o >= 1; o >>= 1) {
            a += __shfl_xor(a, o);
            b += __shfl_xor(b, o);
        }
        if (t == 0) {
            stot[0] = a;
            stot[1] = b;
        }
    }
    __syncthreads();
    // each vertex's u*: thread (j, c, h) sums W u* over the nodes of layer c
    // of vertex j's stencil in row group h (y offset b, then x offset a),
    // the groups and the four layers added in order below.  The nodes' u* were stored by nodeu_waves; a
    // node outside the fluid reads the +0 of the field's solid rows, which
    // nothing writes (the spreading below flags such a stencil)
    {
        const int j = t % PATCH_V, c = (t / PATCH_V) & 3, hb = t / (4 * PATCH_V);
        constexpr int NR = 4 / PATCH_ROWS;   // stencil rows per thread
        double su[3] = {0.0, 0.0, 0.0};
        const int z = j < pn ? so[j][2] + c : -1;
        if (z >= 0 && z < d.nz) {
            const int x0 = (so[j][0] % d.nx + d.nx) % d.nx;
            const double wz = sw[j][8 + c];
#pragma unroll
            for (int b = NR * hb; b < NR * hb + NR; b++) {
                const int y = so[j][1] + b;
                if (y < 0 || y >= d.ny) continue;
                const long long row = (long long)(z * d.ny + y) * d.pitch;
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    const double W = sw[j][a] * sw[j][4 + b] * wz;
                    const int x = x0 + a < d.nx ? x0 + a : x0 + a - d.nx;
                    const double4 m = ((const double4 *)d.Mu)[row + x];
                    su[0] += W * m.x;
                    su[1] += W * m.y;
                    su[2] += W * m.z;
                }
            }
        }
        for (int u = 0; u < 3; u++) sus[hb][c][j][u] = su[u];
    }
    // each vertex's force and dV, its terms split PATCH_FR ways (part r takes
    // the entries r, r + PATCH_FR, ...; the parts are added in order)
    const double *P = d.mpar + 8 * m;
    const double A = stot[0], V = stot[1];
    const double ca = P[2] * (A - P[5]) / P[5], cv = P[3] * (V - P[6]) / P[6];
    {
        const int j = t % PATCH_V, r = t / PATCH_V;
        double f[3] = {0.0, 0.0, 0.0}, dV = 0.0;
        if (j < pn) {
            const int v = pv0 + j;
            for (int k = d.vtb[v] + r; k < d.vtb[v + 1]; k += PATCH_FR) {
                const double *q = d.tcf + 10 * (long long)k;
                for (int u = 0; u < 3; u++) f[u] += q[u] - ca * q[3 + u] - cv * q[6 + u];
                dV += q[9];
            }
            for (int k = d.veb[v] + r; k < d.veb[v + 1]; k += PATCH_FR) {
                const double *q = d.ecf + 3 * (long long)k;
                for (int u = 0; u < 3; u++) f[u] += q[u];
            }
        }
        for (int u = 0; u < 3; u++) sp[r][j][u] = f[u];
        sp[r][j][3] = dV;
    }
    __syncthreads();
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
    if (t < pn) {
        const int v = pv0 + t;
        if (v == d.mv0[m]) {
            d.mtot[2 * m] = A;
            d.mtot[2 * m + 1] = V;
        }
        double f[3], dV;
        for (int u = 0; u < 3; u++) {
            f[u] = 0.0;
            for (int r = 0; r < PATCH_FR; r++) f[u] += sp[r][t][u];
        }
        dV = 0.0;
        for (int r = 0; r < PATCH_FR; r++) dV += sp[r][t][3];
        for (int u = 0; u < 3; u++) {
            const long long k = u * d.ms + v;
            const double xn = X[k];
            double us = 0.0;
            for (int c = 0; c < 4; c++) {
                double lc = 0.0;
                for (int h = 0; h < PATCH_ROWS; h++) lc += sus[h][c][t][u];
                us += lc;
            }
            const double dx = us + 0.5 * f[u] / P[4];
            const double U = 1.5 * dx - 0.5 * d.Mdxm[k];
            const double Fs = (U - us) * dV;
            d.MX[mp ^ 1][k] = xn + dx;
            sno[t][u] = (int)floor(xn + dx) - 1;
            d.Mdxm[k] = dx;
            d.MF[k] = Fs;
            sF[t][u] = Fs;
            lo[u] = so[t][u];
            hi[u] = so[t][u];
        }
    }
    if (t < 64) {
        // the patch's vertices are the first wave: its box by lane reductions
        for (int k = 32; k >= 1; k >>= 1)
            for (int u = 0; u < 3; u++) {
                lo[u] = min(lo[u], __shfl_xor(lo[u], k));
                hi[u] = max(hi[u], __shfl_xor(hi[u], k));
            }
        if (t == 0)
            for (int u = 0; u < 3; u++) {
                sbox[u] = lo[u];
                sbox[3 + u] = (int)min((long long)hi[u] - lo[u] + 4, (long long)INT_MAX);
            }
    }
    __syncthreads();
    const int lx = sbox[0], ly = sbox[1], lz = sbox[2], ex = sbox[3], ey = sbox[4], ez = sbox[5];
    const bool inbox = ex >= 4 && ex <= BOX && ey >= 4 && ey <= BOX && ez >= 4 && ez <= BOX;
    const int nb = inbox ? ex * ey * ez : 0;
    for (int i = t; i < nb; i += PATCH_THREADS) box[i][0] = box[i][1] = box[i][2] = 0;
    __syncthreads();
    // the work items under the next step's stencils: thread t takes the
    // (vertex, column) pairs t + 256 r, their columns loaded together here
    // and the flags stored after the spreading, which hides the loads
    static_assert(16 * 64 <= 4 * PATCH_THREADS, "four pairs per thread");
    int fc[4];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int i = t + r * PATCH_THREADS, j = i >> 4;
        fc[r] = i < 16 * pn ? stencil_col(d, sno[j][1], sno[j][2], i & 3, (i >> 2) & 3) : -1;
    }
    // lane l of wave r: node (l & 3, (l >> 2) & 3, l >> 4) of the stencils of
    // vertices r, r + 4, ...  In the box, the next vertex's inputs are read
    // from LDS before this one's three atomics go out, so that no wait for
    // an LDS read also waits for the atomics.
    {
        const int l = t & 63, a = l & 3, b = (l >> 2) & 3, c = l >> 4;
        struct In {
            int o[3], m;
            double w, f[3];
        };
        auto take = [&](int j) {
            In q;
            for (int u = 0; u < 3; u++) q.o[u] = so[j][u];
            q.m = (smask[j] >> (l >> 2)) & 1;
            q.w = sw[j][a] * sw[j][4 + b] * sw[j][8 + c];
            for (int u = 0; u < 3; u++) q.f[u] = sF[j][u];
            return q;
        };
        int j = t >> 6;
        if (inbox) {
            // every pass issues the same LDS operations (the next vertex's
            // eight reads, then three atomics; a solid node or a rejected
            // value adds 0 inside the box), so that the wait before the
            // next pass can leave the atomics in flight
            In cur = take(min(j, pn - 1));
            for (; j < pn; j += PATCH_THREADS / 64) {
                const In nxt = take(min(j + PATCH_THREADS / 64, pn - 1));
                const int y = cur.o[1] + b, z = cur.o[2] + c, xu = cur.o[0] + a;
                unsigned long long iv[3];
                bool ok = true;
                for (int u = 0; u < 3; u++) {
                    const double cq = cur.w * cur.f[u] * FIX_ONE;
                    const bool oku = fabs(cq) < 4.0e18;
                    ok = ok && oku;
                    iv[u] = cur.m && oku ? (unsigned long long)__double2ll_rn(cq) : 0ull;
                }
                if (cur.m && !ok) atomicOr(d.err, ERR_FORCE);
                unsigned long long *q = box[((z - lz) * ey + (y - ly)) * ex + (xu - lx)];
                atomicAdd(q, iv[0]);
                atomicAdd(q + 1, iv[1]);
                atomicAdd(q + 2, iv[2]);
                cur = nxt;
            }
        } else {
            for (; j < pn; j += PATCH_THREADS / 64) {
                const In cur = take(j);
                if (!cur.m) continue;   // outside the fluid (flagged above)
                const int y = cur.o[1] + b, z = cur.o[2] + c, xu = cur.o[0] + a;   // xu unwrapped
                const int xw = (xu % d.nx + d.nx) % d.nx;
                bool ok = true;
                for (int u = 0; u < 3; u++) {
                    const double cq = cur.w * cur.f[u] * FIX_ONE;
                    if (!(fabs(cq) < 4.0e18)) {
                        ok = false;
                        continue;
                    }
                    atomicAdd(d.mforce + u * d.fs + (long long)(z * d.ny + y) * d.pitch + xw,
                              (unsigned long long)__double2ll_rn(cq));
                }
                if (!ok) atomicOr(d.err, ERR_FORCE);
                d.mflag[d.colof[z * d.ny + y] * d.nseg + xw / 64] = 1;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; r++)
        if (fc[r] >= 0) flag_col_items(d, fc[r], sno[(t + r * PATCH_THREADS) >> 4][0]);
    __syncthreads();
    for (int i = t; i < nb; i += PATCH_THREADS) {
        const unsigned long long v0 = box[i][0], v1 = box[i][1], v2 = box[i][2];
        if ((v0 | v1 | v2) == 0) continue;
        const int ix = i % ex, iy = (i / ex) % ey, iz = i / (ex * ey);
        const int y = ly + iy, z = lz + iz, xw = ((lx + ix) % d.nx + d.nx) % d.nx;
        const int col = d.colof[z * d.ny + y];   // fluid: only fluid nodes received contributions
        const long long node = (long long)(z * d.ny + y) * d.pitch + xw;
        if (v0) atomicAdd(d.mforce + node, v0);
        if (v1) atomicAdd(d.mforce + d.fs + node, v1);
        if (v2) atomicAdd(d.mforce + 2 * d.fs + node, v2);
        d.mflag[col * d.nseg + xw / 64] = 1;
    }
}

// Moments the next step starts from, FP64, into d.macro (fluid nodes).
template <typename T, int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_macro(Dev3 d) {
    int c, x;
    if (!item_of(d, c, x) || x >= d.nx) return;
    double h[Q];
    long long own;
    const double ur = pull<T, double, PAR>(d, c, x, h, own);
    double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int q = 0; q < Q; q++) {
        drho += h[q];
        jx += EX[q] * h[q];
        jy += EY[q] * h[q];
        jz += EZ[q] * h[q];
    }
    const double rho = 1.0 + drho;
    const long long n = (long long)d.nx * d.ny * d.nz, k = (long long)d.crow[20 * c] * d.nx + x;
    d.macro[k] = drho;
    d.macro[n + k] = ur + (jx + 0.5 * d.gx - drho * ur) / rho;
    d.macro[2 * n + k] = jy / rho;
    d.macro[3 * n + k] = jz / rho;
}

// Per-workgroup FP64 sums of the stored populations: mass and momentum
// (the reference's own momentum, (u_ref, 0, 0) per node, added exactly).
template <typename T, int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_diag(Dev3 d) {
    __shared__ double s[WAVES][4];
    int c = 0, x = 0;
    double m = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    if (item_of(d, c, x) && x < d.nx) {
        const long long own = (long long)d.crow[20 * c] * d.pitch + x;
        const T *A = (const T *)d.pop[PAR];
        for (int q = 0; q < Q; q++) {
            const double v = ld3(A + q * d.qstride + own, d.inv_scale);
            m += v;
            px += EX[q] * v;
            py += EY[q] * v;
            pz += EZ[q] * v;
        }
        px += d.cK[20 * c + 19];
    }
    for (int o = 32; o >= 1; o >>= 1) {
        m += __shfl_xor(m, o);
        px += __shfl_xor(px, o);
        py += __shfl_xor(py, o);
        pz += __shfl_xor(pz, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { s[w][0] = m; s[w][1] = px; s[w][2] = py; s[w][3] = pz; }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int k = 0; k < WAVES; k++) t += s[k][threadIdx.x];
        d.part[4 * blockIdx.x + threadIdx.x] = t;
    }
}

}  // namespace tube3d

using namespace tube3d;

// ---- host side ------------------------------------------------------------------------------

struct capib3d_ctx {
    capib3d_lattice lat{};
    hipStream_t stream = nullptr;
    int pitch = 0, ncol = 0, nseg = 0, nblk = 0, par = 0, esize = 4;
    long long step = 0;
    std::vector<int> crow;        // [ncol][20]
    std::vector<double> cK;       // [ncol][20]
    std::vector<double> ref;      // [nz][ny][19]: r_q(y, z) of the reference profile
    std::vector<double> uref;     // [nz][ny]
    std::vector<unsigned char> fluid;   // [nz][ny]
    std::vector<int> colof;             // [nz][ny]: column index of a fluid row, -1 solid
    // fixed immersed bodies, host copies of the device maps
    int nv = 0, nslot = 0, nslot_max = 0, share_u = 0, share_v = 0;
    bool umarks = false;   // the items under the membranes' current stencils are flagged
    std::vector<int> vcol, vxs;         // [nv][64]
    std::vector<double> vW, vdV;        // [nv][64], [nv]
    // deformable membranes, host copies
    int nm = 0, mvn = 0, mtn = 0, mpar = 0, mmaxv = 0;   // counts, positions' parity, largest membrane
    std::vector<int> m_v0, m_nv, m_t0, m_nt, mtri;       // ranges, [mt][3]
    std::vector<double> mref, mparam;                    // [mt][8], [nm][8]
    std::vector<int> medge;                              // [me][4]
    std::vector<double> mth0;                            // [me]
    char *base = nullptr;
    size_t off_pop[2]{}, off_crow = 0, off_cK = 0, off_macro = 0, off_part = 0, ws = 0;
    size_t off_vnode = 0, off_vW = 0, off_vdV = 0, off_vpos = 0, off_vF = 0, off_contrib = 0, off_unode = 0,
           off_islot = 0, off_fitem = 0, off_sbeg = 0;
    size_t off_MX[2]{}, off_Mdxm = 0, off_MF = 0, off_Mtri = 0, off_Mref = 0, off_vtb = 0, off_tslot = 0,
           off_mv0 = 0, off_mnv = 0, off_mt0 = 0, off_mnt = 0, off_mpar = 0, off_mtot = 0, off_ewave = 0,
           off_me0 = 0, off_mne = 0, off_tcf = 0, off_ecf = 0, off_ptab = 0, off_mforce = 0, off_mflag = 0, off_Mu = 0, off_uflag = 0,
           off_twave = 0, off_tpart = 0, off_colof = 0, off_stri = 0, off_sbary = 0, off_sbound = 0, off_sanc = 0,
           off_tsb = 0, off_tsl = 0,
           off_err = 0, off_medge = 0, off_mth0 = 0, off_veb = 0, off_eslot = 0;
    int ntw = 0, new_ = 0;                // triangle waves, edge waves
    std::vector<int> perm;                // internal vertex -> the caller's vertex
    std::vector<int> ptab;                // [npatch][3]
    std::vector<int> m_e0, m_ne;          // edge ranges
    int nsite = 0;                        // bond sites
    Dev3 d{};
    std::string err = "no error";
};

static capib_status fail3(capib3d_ctx *c, capib_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIP3(c, call)                                                                                     \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return fail3(c, CAPIB_E_HIP, "%s: %s", #call, hipGetErrorString(e_));         \
    } while (0)

static size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

static bool fluid_yz(const capib3d_lattice &L, int y, int z) {
    if (L.geometry == CAPIB3D_TUBE) {
        if (y < 0 || y >= L.ny || z < 0 || z >= L.nz) return false;
        const double dy = y - 0.5 * (L.ny - 1), dz = z - 0.5 * (L.nz - 1);
        return dy * dy + dz * dz < L.radius * L.radius;
    }
    if (L.geometry == CAPIB3D_SLAB) return z >= 0 && z < L.nz;
    return true;
}

// r_q(y, z) = h_eq(rho = 1, (u, 0, 0)) - w, Eq. (2), FP64
static void ref_pops(double u, double *r) {
    for (int q = 0; q < Q; q++) {
        const double eu = EX[q] * u;
        r[q] = wq(q) * (3.0 * eu + 4.5 * eu * eu - 1.5 * u * u);
    }
}

// Column tables from the geometry and the reference profile.
static void build_tables(capib3d_ctx *c) {
    const capib3d_lattice &L = c->lat;
    c->ref.assign((size_t)L.ny * L.nz * Q, 0.0);
    for (int z = 0; z < L.nz; z++)
        for (int y = 0; y < L.ny; y++) ref_pops(c->uref[(size_t)z * L.ny + y], &c->ref[((size_t)z * L.ny + y) * Q]);
    c->crow.clear();
    c->cK.clear();
    for (int z = 0; z < L.nz; z++)
        for (int y = 0; y < L.ny; y++) {
            if (!c->fluid[(size_t)z * L.ny + y]) continue;
            const double *r = &c->ref[((size_t)z * L.ny + y) * Q];
            c->crow.push_back(z * L.ny + y);
            double K[20];
            int rows[Q];
            for (int q = 0; q < Q; q++) {
                int ys = y - EY[q], zs = z - EZ[q];
                if (L.geometry != CAPIB3D_TUBE) ys = ((ys % L.ny) + L.ny) % L.ny;
                if (L.geometry == CAPIB3D_BOX) zs = ((zs % L.nz) + L.nz) % L.nz;
                if (fluid_yz(L, ys, zs)) {
                    rows[q] = zs * L.ny + ys;
                    K[q] = c->ref[((size_t)zs * L.ny + ys) * Q + q] - r[q];
                } else {
                    rows[q] = -1;
                    K[q] = r[opp(q)] - r[q];   // the node's own opposite population
                }
            }
            K[19] = c->uref[(size_t)z * L.ny + y];
            for (int q = 0; q < Q; q++) c->crow.push_back(rows[q]);
            for (int q = 0; q < 20; q++) c->cK.push_back(K[q]);
        }
}

extern "C" {

capib_status capib3d_create(const capib3d_lattice *lat, void *hip_stream, capib3d_ctx **out) {
    if (!lat || !out) return CAPIB_E_ARG;
    *out = nullptr;
    const capib3d_lattice &L = *lat;
    if (L.nx < 1 || L.ny < 1 || L.nz < 1 || (long long)L.nx * L.ny * L.nz >= (1LL << 31)) return CAPIB_E_ARG;
    if (!(L.tau > 0.5) || !std::isfinite(L.gx)) return CAPIB_E_ARG;
    if (L.geometry < CAPIB3D_TUBE || L.geometry > CAPIB3D_BOX) return CAPIB_E_ARG;
    if (L.geometry == CAPIB3D_TUBE && !(L.radius > 0.0)) return CAPIB_E_ARG;
    if (L.storage != CAPIB_FP32_SHIFTED && L.storage != CAPIB_FP16_SHIFTED) return CAPIB_E_ARG;
    if (L.storage == CAPIB_FP16_SHIFTED) {
        int ex = 0;
        if (!(L.fp16_scale > 0.0) || std::frexp(L.fp16_scale, &ex) != 0.5) return CAPIB_E_ARG;   // a power of two
    }
    if (L.max_vertices < 0 || L.max_vertices > (1 << 24)) return CAPIB_E_ARG;
    if (L.max_sites < 0 || (L.max_sites > 0 && L.max_membranes == 0)) return CAPIB_E_ARG;
    if (L.max_membranes < 0 || L.max_membrane_vertices < 0 || L.max_membrane_triangles < 0 ||
        L.max_membrane_vertices > (1 << 24) || L.max_membrane_triangles > (1 << 25) ||
        (L.max_membrane_vertices > 0) != (L.max_membranes > 0) ||
        (L.max_membrane_vertices > 0) != (L.max_membrane_triangles > 0))
        return CAPIB_E_ARG;
    capib3d_ctx *c = new capib3d_ctx();
    c->lat = L;
    c->stream = (hipStream_t)hip_stream;
    c->pitch = (L.nx + 63) / 64 * 64;
    c->esize = L.storage == CAPIB_FP16_SHIFTED ? 2 : 4;
    c->nseg = c->pitch / 64;
    c->fluid.assign((size_t)L.ny * L.nz, 0);
    for (int z = 0; z < L.nz; z++)
        for (int y = 0; y < L.ny; y++) c->fluid[(size_t)z * L.ny + y] = fluid_yz(L, y, z) ? 1 : 0;
    c->colof.assign((size_t)L.ny * L.nz, -1);
    for (size_t k = 0; k < c->fluid.size(); k++)
        if (c->fluid[k]) c->colof[k] = c->ncol++;
    if (c->ncol == 0) {
        delete c;
        return CAPIB_E_ARG;
    }
    c->nblk = (c->ncol * c->nseg + WAVES - 1) / WAVES;
    c->uref.assign((size_t)L.ny * L.nz, 0.0);
    const size_t N = (size_t)c->pitch * L.ny * L.nz;
    size_t o = 0;
    for (int p = 0; p < 2; p++) { c->off_pop[p] = o; o = al256(o + (size_t)Q * N * c->esize); }
    c->off_crow = o; o = al256(o + (size_t)c->ncol * 20 * 4);
    c->off_cK = o; o = al256(o + (size_t)c->ncol * 20 * 8);
    c->off_macro = o; o = al256(o + (size_t)4 * L.nx * L.ny * L.nz * 8);
    c->off_part = o; o = al256(o + (size_t)c->nblk * 4 * 8);
    const size_t M = (size_t)L.max_vertices, nitem = (size_t)c->ncol * c->nseg;
    c->nslot_max = (int)std::min(nitem, 64 * M);
    c->off_vnode = o; o = al256(o + M * 64 * 4);
    c->off_vW = o; o = al256(o + M * 64 * 8);
    c->off_vdV = o; o = al256(o + M * 8);
    c->off_vpos = o; o = al256(o + M * 64 * 4);
    c->off_vF = o; o = al256(o + M * 3 * 8);
    c->off_contrib = o; o = al256(o + M * 64 * 3 * 8);
    c->off_unode = o; o = al256(o + (size_t)c->nslot_max * 64 * 3 * 8);
    c->off_islot = o; o = al256(o + (M ? nitem * 4 : 0));
    c->off_fitem = o; o = al256(o + (size_t)c->nslot_max * 4);
    c->off_sbeg = o; o = al256(o + (size_t)c->nslot_max * 65 * 4);
    const size_t MM = (size_t)L.max_membranes, MV = (size_t)L.max_membrane_vertices, MT = (size_t)L.max_membrane_triangles;
    const size_t fs = (size_t)L.nz * L.ny * c->pitch;
    for (int p = 0; p < 2; p++) { c->off_MX[p] = o; o = al256(o + 3 * MV * 8); }
    c->off_Mdxm = o; o = al256(o + 3 * MV * 8);
    c->off_MF = o; o = al256(o + 3 * MV * 8);
    c->off_Mtri = o; o = al256(o + MT * 3 * 4);
    c->off_Mref = o; o = al256(o + MT * 8 * 8);
    c->off_vtb = o; o = al256(o + (MV ? MV + 1 : 0) * 4);
    c->off_tslot = o; o = al256(o + 3 * MT * 4);
    c->off_mv0 = o; o = al256(o + MM * 4);
    c->off_mnv = o; o = al256(o + MM * 4);
    c->off_mt0 = o; o = al256(o + MM * 4);
    c->off_mnt = o; o = al256(o + MM * 4);
    c->off_mpar = o; o = al256(o + MM * 8 * 8);
    c->off_mtot = o; o = al256(o + MM * 2 * 8);
    (void)fs;
    c->off_ewave = o; o = al256(o + ((3 * MT) / 2 / 64 + MM + 1) * 2 * 4);
    c->off_me0 = o; o = al256(o + MM * 4);
    c->off_mne = o; o = al256(o + MM * 4);
    c->off_tcf = o; o = al256(o + 3 * MT * 10 * 8);
    c->off_ecf = o; o = al256(o + ((3 * MT) / 2 + 1) * 4 * 3 * 8);
    c->off_ptab = o; o = al256(o + (MV / PATCH_V + MM) * 5 * 4);
    c->off_mforce = o; o = al256(o + (MV ? 3 * fs * 8 : 0));
    c->off_mflag = o; o = al256(o + (MV ? nitem * 4 : 0));
    c->off_Mu = o; o = al256(o + (MV ? 4 * fs * 8 : 0));
    c->off_uflag = o; o = al256(o + (MV ? nitem * 4 : 0));
    const size_t MSITE = (size_t)L.max_sites;
    c->off_stri = o; o = al256(o + MSITE * 4);
    c->off_sbary = o; o = al256(o + MSITE * 2 * 8);
    c->off_sbound = o; o = al256(o + MSITE * 4);
    c->off_sanc = o; o = al256(o + MSITE * 3 * 8);
    c->off_tsb = o; o = al256(o + (MSITE ? MT + 1 : 0) * 4);
    c->off_tsl = o; o = al256(o + MSITE * 4);
    const size_t ME = (3 * MT) / 2 + 1;   // interior edges of the triangles at most
    c->off_medge = o; o = al256(o + ME * 4 * 4);
    c->off_mth0 = o; o = al256(o + ME * 8);
    c->off_veb = o; o = al256(o + (MV ? MV + 1 : 0) * 4);
    c->off_eslot = o; o = al256(o + ME * 4 * 4);
    c->off_twave = o; o = al256(o + (MT / 64 + MM) * 2 * 4);
    c->off_tpart = o; o = al256(o + (MT / 64 + MM) * 2 * 8);

    c->off_colof = o; o = al256(o + (size_t)L.ny * L.nz * 4);
    c->off_err = o; o = al256(o + 4);
    c->ws = o;
    *out = c;
    return CAPIB_OK;
}

void capib3d_destroy(capib3d_ctx *c) { delete c; }

size_t capib3d_workspace_bytes(const capib3d_ctx *c) { return c ? c->ws : 0; }

int64_t capib3d_fluid_nodes(const capib3d_ctx *c) { return c ? (int64_t)c->ncol * c->lat.nx : 0; }

const char *capib3d_last_error(const capib3d_ctx *c) { return c ? c->err.c_str() : "null context"; }

static capib_status upload_tables(capib3d_ctx *c) {
    build_tables(c);
    HIP3(c, hipMemcpyAsync(c->base + c->off_colof, c->colof.data(), c->colof.size() * 4, hipMemcpyHostToDevice,
                           c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_crow, c->crow.data(), c->crow.size() * 4, hipMemcpyHostToDevice,
                           c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_cK, c->cK.data(), c->cK.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    return CAPIB_OK;
}

capib_status capib3d_bind_workspace(capib3d_ctx *c, void *ptr, size_t bytes) {
    if (!c) return CAPIB_E_ARG;
    if (!ptr || ((uintptr_t)ptr & 255)) return fail3(c, CAPIB_E_ARG, "workspace must be a 256-byte aligned device pointer");
    if (bytes < c->ws) return fail3(c, CAPIB_E_ARG, "workspace of %zu bytes, %zu needed", bytes, c->ws);
    c->base = (char *)ptr;
    const capib3d_lattice &L = c->lat;
    Dev3 &d = c->d;
    d.nx = L.nx; d.ny = L.ny; d.nz = L.nz; d.pitch = c->pitch; d.ncol = c->ncol; d.nseg = c->nseg;
    d.qstride = (long long)c->pitch * L.ny * L.nz;
    d.omega = 1.0 / L.tau;
    d.fc = 1.0 - 0.5 / L.tau;
    d.gx = L.gx;
    d.scale = L.storage == CAPIB_FP16_SHIFTED ? (float)L.fp16_scale : 1.0f;
    d.inv_scale = L.storage == CAPIB_FP16_SHIFTED ? (float)(1.0 / L.fp16_scale) : 1.0f;
    for (int p = 0; p < 2; p++) d.pop[p] = c->base + c->off_pop[p];
    d.crow = (const int *)(c->base + c->off_crow);
    d.cK = (const double *)(c->base + c->off_cK);
    d.macro = (double *)(c->base + c->off_macro);
    d.part = (double *)(c->base + c->off_part);
    d.nv = 0;
    d.nslot = 0;
    d.vnode = (const int *)(c->base + c->off_vnode);
    d.vW = (const double *)(c->base + c->off_vW);
    d.vdV = (const double *)(c->base + c->off_vdV);
    d.vpos = (const int *)(c->base + c->off_vpos);
    d.vF = (double *)(c->base + c->off_vF);
    d.contrib = (double *)(c->base + c->off_contrib);
    d.unode = (double *)(c->base + c->off_unode);
    d.ucap = (long long)c->nslot_max * 64;
    d.islot = (const int *)(c->base + c->off_islot);
    d.fitem = (const int *)(c->base + c->off_fitem);
    d.sbeg = (const int *)(c->base + c->off_sbeg);
    c->nv = 0;
    c->nslot = 0;
    d.nm = 0;
    d.mv = 0;
    d.ms = L.max_membrane_vertices;
    d.fs = (long long)L.nz * L.ny * c->pitch;
    for (int p = 0; p < 2; p++) d.MX[p] = (double *)(c->base + c->off_MX[p]);
    d.Mdxm = (double *)(c->base + c->off_Mdxm);
    d.MF = (double *)(c->base + c->off_MF);
    d.Mtri = (const int *)(c->base + c->off_Mtri);
    d.Mref = (const double *)(c->base + c->off_Mref);
    d.vtb = (const int *)(c->base + c->off_vtb);
    d.tslot = (const int *)(c->base + c->off_tslot);
    d.mv0 = (const int *)(c->base + c->off_mv0);
    d.mnv = (const int *)(c->base + c->off_mnv);
    d.mt0 = (const int *)(c->base + c->off_mt0);
    d.mnt = (const int *)(c->base + c->off_mnt);
    d.mpar = (const double *)(c->base + c->off_mpar);
    d.mtot = (double *)(c->base + c->off_mtot);
    d.ewave = (const int *)(c->base + c->off_ewave);
    d.me0 = (const int *)(c->base + c->off_me0);
    d.mne = (const int *)(c->base + c->off_mne);
    d.new_ = 0;
    d.tcf = (double *)(c->base + c->off_tcf);
    d.ecf = (double *)(c->base + c->off_ecf);
    d.ptab = (const int *)(c->base + c->off_ptab);
    d.mforce = (unsigned long long *)(c->base + c->off_mforce);
    d.mflag = (int *)(c->base + c->off_mflag);
    d.Mu = (double *)(c->base + c->off_Mu);
    d.uflag = (int *)(c->base + c->off_uflag);
    d.ns = 0;
    d.Stri = (const int *)(c->base + c->off_stri);
    d.Sbary = (const double *)(c->base + c->off_sbary);
    d.Sbound = (int *)(c->base + c->off_sbound);
    d.Sanc = (double *)(c->base + c->off_sanc);
    d.tsb = (const int *)(c->base + c->off_tsb);
    d.tsl = (const int *)(c->base + c->off_tsl);
    d.radius = L.radius;
    c->nsite = 0;
    c->new_ = 0;
    c->perm.clear();
    c->ptab.clear();
    c->m_e0.clear();
    c->m_ne.clear();
    d.Medge = (const int *)(c->base + c->off_medge);
    d.Mth0 = (const double *)(c->base + c->off_mth0);
    d.veb = (const int *)(c->base + c->off_veb);
    d.eslot = (const int *)(c->base + c->off_eslot);
    d.twave = (const int *)(c->base + c->off_twave);
    d.ntw = 0;
    d.mcap = L.max_membranes;
    d.tpart = (double *)(c->base + c->off_tpart);

    c->ntw = 0;
    d.colof = (const int *)(c->base + c->off_colof);
    d.err = (int *)(c->base + c->off_err);
    c->nm = c->mvn = c->mtn = c->mpar = c->mmaxv = 0;
    c->umarks = false;
    c->m_v0.clear(); c->m_nv.clear(); c->m_t0.clear(); c->m_nt.clear(); c->mtri.clear(); c->mref.clear();
    c->mparam.clear(); c->medge.clear(); c->mth0.clear();
    c->vcol.clear(); c->vxs.clear(); c->vW.clear(); c->vdV.clear();
    HIP3(c, hipMemsetAsync(c->base, 0, c->ws, c->stream));
    return upload_tables(c);
}

static capib_status need_ws(capib3d_ctx *c) {
    if (!c) return CAPIB_E_ARG;
    if (!c->base) return fail3(c, CAPIB_E_STATE, "no workspace bound");
    return CAPIB_OK;
}

capib_status capib3d_init_flow(capib3d_ctx *c, const double *ux_of_yz) {
    capib_status s = need_ws(c);
    if (s) return s;
    const capib3d_lattice &L = c->lat;
    for (size_t k = 0; k < c->uref.size(); k++) {
        const double u = ux_of_yz ? ux_of_yz[k] : 0.0;
        if (!std::isfinite(u) || std::fabs(u) > 0.1) return fail3(c, CAPIB_E_ARG, "reference velocity %g at %zu", u, k);
        c->uref[k] = c->fluid[k] ? u : 0.0;
    }
    if ((s = upload_tables(c))) return s;
    const size_t N = (size_t)c->pitch * L.ny * L.nz;
    for (int p = 0; p < 2; p++)
        HIP3(c, hipMemsetAsync(c->base + c->off_pop[p], 0, (size_t)Q * N * c->esize, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    c->par = 0;
    c->step = 0;
    return CAPIB_OK;
}

capib_status capib3d_step(capib3d_ctx *c, int32_t nsteps) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (nsteps < 0) return fail3(c, CAPIB_E_ARG, "negative step count");
    const bool h16 = c->lat.storage == CAPIB_FP16_SHIFTED, ib = c->nv > 0;
    const dim3 blk(64 * WAVES);
    // with bodies: vertex workgroups and slot workgroups rounded up to a
    // multiple of 8, so the sweep workgroups after them keep their XCD; the
    // ordinary items split in three shares
    const int nitem = c->ncol * c->nseg;
    const int s1 = (int)((long long)nitem * c->share_u / 100), s2 = (int)((long long)nitem * (c->share_u + c->share_v) / 100);
    const int nvb = ((c->nv + WAVES - 1) / WAVES + 7) / 8 * 8, nfb = ((c->nslot + WAVES - 1) / WAVES + 7) / 8 * 8;
    const dim3 g1(nfb + (s1 + WAVES - 1) / WAVES), g2(nvb + (s2 - s1 + WAVES - 1) / WAVES),
        g3(nfb + (nitem - s2 + WAVES - 1) / WAVES);
    // waves of nodeu_waves: lane l of wave w scans item w + l nuw, so at
    // least nitem / 64 of them reach every item
    const int nuw = std::max(std::min(nitem, NODEU_WAVES), (nitem + 63) / 64), nub = (nuw + WAVES - 1) / WAVES;
    const int ntb = (c->ntw + WAVES - 1) / WAVES;
    const int nte = ntb + (c->new_ + WAVES - 1) / WAVES;   // triangle and edge workgroups
    const dim3 gf(nte + nub), gp((unsigned)(c->ptab.size() / 3));
    for (int t = 0; t < nsteps && c->nm > 0; t++) {
        const int mp = c->mpar;
        if (!c->umarks) {
            hipLaunchKernelGGL(k3_m_umark, dim3((unsigned)((16LL * c->mvn + 255) / 256)), dim3(256), 0, c->stream, c->d, mp);
            c->umarks = true;
        }
        // the previous step's bond kinetics in this step's triangle lanes
        const long long kstep = t > 0 && c->nsite > 0 ? c->step - 1 : -1;
        if (c->par)
            hipLaunchKernelGGL((h16 ? k3_m_first<_Float16, 1> : k3_m_first<float, 1>), gf, blk, 0, c->stream, c->d,
                               c->d.crow, c->d.cK, mp, nte, nuw, ntb, kstep);
        else
            hipLaunchKernelGGL((h16 ? k3_m_first<_Float16, 0> : k3_m_first<float, 0>), gf, blk, 0, c->stream, c->d,
                               c->d.crow, c->d.cK, mp, nte, nuw, ntb, kstep);
        hipLaunchKernelGGL(k3_m_patch, gp, dim3(PATCH_THREADS), 0, c->stream, c->d, mp);
        if (c->par)
            hipLaunchKernelGGL((h16 ? k3_sweep<_Float16, 1, 2> : k3_sweep<float, 1, 2>), dim3(c->nblk), blk, 0,
                               c->stream, c->d);
        else
            hipLaunchKernelGGL((h16 ? k3_sweep<_Float16, 0, 2> : k3_sweep<float, 0, 2>), dim3(c->nblk), blk, 0,
                               c->stream, c->d);
        HIP3(c, hipGetLastError());
        c->par ^= 1;
        c->mpar ^= 1;
        c->step++;
    }
    if (nsteps > 0 && c->nm > 0 && c->nsite > 0) {
        // the last step's bond kinetics, so that the states are current
        // when the call returns
        hipLaunchKernelGGL(k3_m_bonds, dim3((c->nsite + 255) / 256), dim3(256), 0, c->stream, c->d, c->mpar,
                           c->step - 1);
        HIP3(c, hipGetLastError());
    }
    for (int t = 0; t < nsteps && c->nm == 0; t++) {
        if (ib && c->par) {
            hipLaunchKernelGGL((h16 ? k3_node_u<_Float16, 1> : k3_node_u<float, 1>), g1, blk, 0, c->stream, c->d, nfb, s1);
            hipLaunchKernelGGL((h16 ? k3_vertex<_Float16, 1> : k3_vertex<float, 1>), g2, blk, 0, c->stream, c->d, nvb, s1,
                               s2);
            hipLaunchKernelGGL((h16 ? k3_sweep_ib<_Float16, 1> : k3_sweep_ib<float, 1>), g3, blk, 0, c->stream, c->d, nfb,
                               s2);
        } else if (ib) {
            hipLaunchKernelGGL((h16 ? k3_node_u<_Float16, 0> : k3_node_u<float, 0>), g1, blk, 0, c->stream, c->d, nfb, s1);
            hipLaunchKernelGGL((h16 ? k3_vertex<_Float16, 0> : k3_vertex<float, 0>), g2, blk, 0, c->stream, c->d, nvb, s1,
                               s2);
            hipLaunchKernelGGL((h16 ? k3_sweep_ib<_Float16, 0> : k3_sweep_ib<float, 0>), g3, blk, 0, c->stream, c->d, nfb,
                               s2);
        } else if (c->par) {
            hipLaunchKernelGGL((h16 ? k3_sweep<_Float16, 1, 0> : k3_sweep<float, 1, 0>), dim3(c->nblk), blk, 0,
                               c->stream, c->d);
        } else {
            hipLaunchKernelGGL((h16 ? k3_sweep<_Float16, 0, 0> : k3_sweep<float, 0, 0>), dim3(c->nblk), blk, 0,
                               c->stream, c->d);
        }
        HIP3(c, hipGetLastError());
        c->par ^= 1;
        c->step++;
    }
    return CAPIB_OK;
}

capib_status capib3d_read_macro(capib3d_ctx *c, double *drho, double *ux, double *uy, double *uz) {
    capib_status s = need_ws(c);
    if (s) return s;
    const capib3d_lattice &L = c->lat;
    const size_t n = (size_t)L.nx * L.ny * L.nz;
    HIP3(c, hipMemsetAsync(c->base + c->off_macro, 0, 4 * n * 8, c->stream));
    const bool h16 = c->lat.storage == CAPIB_FP16_SHIFTED;
    if (c->par)
        hipLaunchKernelGGL((h16 ? k3_macro<_Float16, 1> : k3_macro<float, 1>), dim3(c->nblk), dim3(64 * WAVES), 0,
                           c->stream, c->d);
    else
        hipLaunchKernelGGL((h16 ? k3_macro<_Float16, 0> : k3_macro<float, 0>), dim3(c->nblk), dim3(64 * WAVES), 0,
                           c->stream, c->d);
    HIP3(c, hipGetLastError());
    double *outs[4] = {drho, ux, uy, uz};
    for (int k = 0; k < 4; k++)
        if (outs[k])
            HIP3(c, hipMemcpyAsync(outs[k], c->base + c->off_macro + k * n * 8, n * 8, hipMemcpyDeviceToHost,
                                   c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    return CAPIB_OK;
}

capib_status capib3d_read_populations(capib3d_ctx *c, double *out) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!out) return fail3(c, CAPIB_E_ARG, "null output");
    const capib3d_lattice &L = c->lat;
    const size_t N = (size_t)c->pitch * L.ny * L.nz, n = (size_t)L.nx * L.ny * L.nz;
    std::vector<unsigned char> raw((size_t)Q * N * c->esize);
    HIP3(c, hipMemcpyAsync(raw.data(), c->base + c->off_pop[c->par], raw.size(), hipMemcpyDeviceToHost, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    const bool h16 = c->lat.storage == CAPIB_FP16_SHIFTED;
    const double inv = h16 ? 1.0 / c->lat.fp16_scale : 1.0;
    for (int q = 0; q < Q; q++)
        for (int z = 0; z < L.nz; z++)
            for (int y = 0; y < L.ny; y++) {
                const size_t col = (size_t)z * L.ny + y;
                const bool fl = c->fluid[col];
                const double r = c->ref[col * Q + q];
                for (int x = 0; x < L.nx; x++) {
                    const size_t k = q * N + col * c->pitch + x;
                    const double sv = h16 ? (double)((const _Float16 *)raw.data())[k] * inv
                                          : (double)((const float *)raw.data())[k];
                    out[q * n + col * L.nx + x] = fl ? sv + r : 0.0;
                }
            }
    return CAPIB_OK;
}

capib_status capib3d_write_populations(capib3d_ctx *c, const double *in) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!in) return fail3(c, CAPIB_E_ARG, "null input");
    const capib3d_lattice &L = c->lat;
    const size_t N = (size_t)c->pitch * L.ny * L.nz, n = (size_t)L.nx * L.ny * L.nz;
    const bool h16 = c->lat.storage == CAPIB_FP16_SHIFTED;
    const double sc = h16 ? c->lat.fp16_scale : 1.0;
    std::vector<unsigned char> raw((size_t)Q * N * c->esize, 0);
    for (int q = 0; q < Q; q++)
        for (int z = 0; z < L.nz; z++)
            for (int y = 0; y < L.ny; y++) {
                const size_t col = (size_t)z * L.ny + y;
                if (!c->fluid[col]) continue;
                const double r = c->ref[col * Q + q];
                for (int x = 0; x < L.nx; x++) {
                    const double v = in[q * n + col * L.nx + x];
                    if (!std::isfinite(v)) return fail3(c, CAPIB_E_ARG, "non-finite population");
                    const size_t k = q * N + col * c->pitch + x;
                    if (h16) {
                        const double sv = (v - r) * sc;
                        if (std::fabs(sv) > 65504.0)
                            return fail3(c, CAPIB_E_ARG, "deviation %g overflows FP16 at scale %g", v - r, sc);
                        ((_Float16 *)raw.data())[k] = (_Float16)(float)sv;
                    } else {
                        ((float *)raw.data())[k] = (float)(v - r);
                    }
                }
            }
    HIP3(c, hipMemcpyAsync(c->base + c->off_pop[c->par], raw.data(), raw.size(), hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    return CAPIB_OK;
}

// The contributions of every stencil node of every vertex, grouped by node
// with the vertices in ascending order (each lane's place in that order, the
// ranges per lane of a slot, the slot of every item); uploads the maps.
static capib_status upload_bodies(capib3d_ctx *c, int v0) {
    const size_t nitem = (size_t)c->ncol * c->nseg, ne = (size_t)c->nv * 64;
    std::vector<long long> node(ne);
    std::vector<int> order(ne);
    for (size_t k = 0; k < ne; k++) {
        node[k] = (long long)c->vcol[k] * c->pitch + c->vxs[k];
        order[k] = (int)k;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return node[a] < node[b]; });
    std::vector<int> vpos(ne), vnode(ne), islot(nitem, -1), fitem, sbeg;
    for (size_t j = 0; j < ne; j++) vpos[order[j]] = (int)j;
    for (size_t k = 0; k < ne;) {
        const long long item = node[order[k]] / 64;   // column * nseg + x / 64: the pitch is nseg * 64
        const int slot = (int)fitem.size();
        if (slot >= c->nslot_max) return fail3(c, CAPIB_E_CAPACITY, "stencil slots exhausted");
        islot[item] = slot;
        fitem.push_back((int)item);
        sbeg.resize(sbeg.size() + 65);
        int *sb = &sbeg[65 * (size_t)slot];
        size_t j = k;
        for (int l = 0; l < 64; l++) {
            sb[l] = (int)j;
            while (j < ne && node[order[j]] == item * 64 + l) j++;
        }
        sb[64] = (int)j;
        k = j;
    }
    for (size_t k = 0; k < ne; k++) vnode[k] = islot[node[k] / 64] * 64 + (int)(node[k] % 64);
    const size_t nv = c->nv, a = (size_t)v0;
    HIP3(c, hipMemcpyAsync(c->base + c->off_vnode, vnode.data(), ne * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_vW + a * 512, &c->vW[a * 64], (nv - a) * 512, hipMemcpyHostToDevice,
                           c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_vdV + a * 8, &c->vdV[a], (nv - a) * 8, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_vpos, vpos.data(), ne * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_islot, islot.data(), nitem * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_fitem, fitem.data(), fitem.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_sbeg, sbeg.data(), sbeg.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    c->nslot = (int)fitem.size();
    return CAPIB_OK;
}

static double phi3(double r) {
    r = std::fabs(r);
    return r < 2.0 ? 0.25 * (1.0 + std::cos(M_PI * r / 2.0)) : 0.0;
}

capib_status capib3d_add_fixed_body(capib3d_ctx *c, int32_t nv, const double *xyz, int32_t ntri, const int32_t *tri,
                                    int32_t *first_vertex) {
    capib_status s = need_ws(c);
    if (s) return s;
    const capib3d_lattice &L = c->lat;
    if (nv < 1 || ntri < 0 || !xyz || (ntri > 0 && !tri)) return fail3(c, CAPIB_E_ARG, "bad body arrays");
    if (c->nm > 0) return fail3(c, CAPIB_E_STATE, "fixed bodies and membranes do not share a context");
    if ((long long)c->nv + nv > L.max_vertices)
        return fail3(c, CAPIB_E_CAPACITY, "%d + %d vertices exceed the capacity of %d", c->nv, nv, L.max_vertices);
    for (int k = 0; k < 3 * ntri; k++)
        if (tri[k] < 0 || tri[k] >= nv) return fail3(c, CAPIB_E_ARG, "triangle vertex %d out of range", tri[k]);
    std::vector<int> vcol((size_t)nv * 64), vxs((size_t)nv * 64);
    std::vector<double> vW((size_t)nv * 64), vdV(nv, 0.0);
    for (int v = 0; v < nv; v++) {
        const double *X = xyz + 3 * v;
        if (!std::isfinite(X[0]) || !std::isfinite(X[1]) || !std::isfinite(X[2]) || std::fabs(X[0]) > 1e9)
            return fail3(c, CAPIB_E_ARG, "vertex %d not finite", v);
        int o[3];
        double w[3][4];
        for (int a = 0; a < 3; a++) {
            o[a] = (int)std::floor(X[a]) - 1;
            for (int k = 0; k < 4; k++) w[a][k] = phi3(X[a] - (o[a] + k));
        }
        if (o[1] < 0 || o[1] + 3 >= L.ny || o[2] < 0 || o[2] + 3 >= L.nz)
            return fail3(c, CAPIB_E_ARG, "vertex %d: stencil outside the cross-section", v);
        for (int zc = 0; zc < 4; zc++)
            for (int yb = 0; yb < 4; yb++) {
                const int col = c->colof[(size_t)(o[2] + zc) * L.ny + o[1] + yb];
                if (col < 0) return fail3(c, CAPIB_E_ARG, "vertex %d: stencil node on a solid column", v);
                for (int xa = 0; xa < 4; xa++) {
                    const int l = xa + 4 * yb + 16 * zc;
                    vcol[64 * (size_t)v + l] = col;
                    vxs[64 * (size_t)v + l] = (int)((((long long)o[0] + xa) % L.nx + L.nx) % L.nx);
                    vW[64 * (size_t)v + l] = w[0][xa] * w[1][yb] * w[2][zc];
                }
            }
    }
    // a third of the area of every triangle to each of its vertices
    for (int t = 0; t < ntri; t++) {
        const double *a = xyz + 3 * tri[3 * t], *b = xyz + 3 * tri[3 * t + 1], *e = xyz + 3 * tri[3 * t + 2];
        const double p[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, r[3] = {e[0] - a[0], e[1] - a[1], e[2] - a[2]};
        const double n[3] = {p[1] * r[2] - p[2] * r[1], p[2] * r[0] - p[0] * r[2], p[0] * r[1] - p[1] * r[0]};
        const double area = 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; k++) vdV[tri[3 * t + k]] += area / 3.0;
    }
    const int v0 = c->nv;
    c->vcol.insert(c->vcol.end(), vcol.begin(), vcol.end());
    c->vxs.insert(c->vxs.end(), vxs.begin(), vxs.end());
    c->vW.insert(c->vW.end(), vW.begin(), vW.end());
    c->vdV.insert(c->vdV.end(), vdV.begin(), vdV.end());
    c->nv += nv;
    if ((s = upload_bodies(c, v0))) {
        c->nv = v0;
        c->vcol.resize((size_t)v0 * 64); c->vxs.resize((size_t)v0 * 64); c->vW.resize((size_t)v0 * 64);
        c->vdV.resize(v0);
        return s;
    }
    c->d.nv = c->nv;
    c->d.nslot = c->nslot;
    if (first_vertex) *first_vertex = v0;
    return CAPIB_OK;
}

capib_status capib3d_body_forces(capib3d_ctx *c, double *out) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!out) return fail3(c, CAPIB_E_ARG, "null output");
    if (c->nv == 0) return CAPIB_OK;
    std::vector<double> f((size_t)c->nv * 3);
    HIP3(c, hipMemcpyAsync(f.data(), c->base + c->off_vF, f.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    for (int v = 0; v < c->nv; v++)
        for (int k = 0; k < 3; k++) out[3 * v + k] = f[3 * (size_t)v + k] * c->vdV[v];
    return CAPIB_OK;
}

int32_t capib3d_vertices(const capib3d_ctx *c) { return c ? c->nv : 0; }

capib_status capib3d_set_ib_schedule(capib3d_ctx *c, int32_t share_node_u, int32_t share_vertex) {
    if (!c) return CAPIB_E_ARG;
    if (share_node_u < 0 || share_vertex < 0 || share_node_u + share_vertex > 100)
        return fail3(c, CAPIB_E_ARG, "shares %d + %d outside [0, 100]", share_node_u, share_vertex);
    c->share_u = share_node_u;
    c->share_v = share_vertex;
    return CAPIB_OK;
}

static void sub3h(const double *a, const double *b, double *o) {
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static void cross3h(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3h(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

capib_status capib3d_add_membrane(capib3d_ctx *c, int32_t nv, const double *xyz, int32_t ntri, const int32_t *tri,
                                  const capib3d_membrane *par, int32_t *first_vertex) {
    capib_status s = need_ws(c);
    if (s) return s;
    const capib3d_lattice &L = c->lat;
    if (nv < 3 || ntri < 1 || !xyz || !tri || !par) return fail3(c, CAPIB_E_ARG, "bad membrane arrays");
    if (c->nv > 0) return fail3(c, CAPIB_E_STATE, "fixed bodies and membranes do not share a context");
    if (L.nx < 4) return fail3(c, CAPIB_E_ARG, "membranes need nx >= 4");
    if (c->nm >= L.max_membranes || (long long)c->mvn + nv > L.max_membrane_vertices ||
        (long long)c->mtn + ntri > L.max_membrane_triangles)
        return fail3(c, CAPIB_E_CAPACITY, "membrane capacity exceeded");
    const double pv[6] = {par->gs, par->c, par->ka, par->kv, par->mass, par->kb};
    for (double x : pv)
        if (!std::isfinite(x)) return fail3(c, CAPIB_E_ARG, "non-finite membrane parameter");
    if (par->gs < 0 || par->ka < 0 || par->kv < 0 || par->kb < 0 || !(par->mass > 0))
        return fail3(c, CAPIB_E_ARG, "membrane moduli must be >= 0 and the mass > 0");
    for (int k = 0; k < 3 * ntri; k++)
        if (tri[k] < 0 || tri[k] >= nv) return fail3(c, CAPIB_E_ARG, "triangle vertex %d out of range", tri[k]);
    for (int v = 0; v < nv; v++) {
        const double *X = xyz + 3 * v;
        if (!std::isfinite(X[0]) || !std::isfinite(X[1]) || !std::isfinite(X[2]) || std::fabs(X[0]) > 1e9)
            return fail3(c, CAPIB_E_ARG, "vertex %d not finite", v);
        const int oy = (int)std::floor(X[1]) - 1, oz = (int)std::floor(X[2]) - 1;
        if (oy < 0 || oy + 3 >= L.ny || oz < 0 || oz + 3 >= L.nz)
            return fail3(c, CAPIB_E_ARG, "vertex %d: stencil outside the cross-section", v);
        for (int zc = 0; zc < 4; zc++)
            for (int yb = 0; yb < 4; yb++)
                if (c->colof[(size_t)(oz + zc) * L.ny + oy + yb] < 0)
                    return fail3(c, CAPIB_E_ARG, "vertex %d: stencil node on a solid column", v);
    }
    // internal numbering: recursive bisection of the rest positions along the
    // longest extent, splitting at a multiple of PATCH_V, so that every
    // PATCH_V consecutive vertices (a patch) lie close together;
    // pp[internal] = the caller's index, ip[caller's] = internal
    std::vector<int> pp(nv), ip(nv);
    {
        for (int v = 0; v < nv; v++) pp[v] = v;
        std::vector<std::pair<int, int>> todo{{0, nv}};
        while (!todo.empty()) {
            const auto [b0, b1] = todo.back();
            todo.pop_back();
            if (b1 - b0 <= PATCH_V) continue;
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
            for (int k = b0; k < b1; k++)
                for (int u = 0; u < 3; u++) {
                    lo[u] = std::min(lo[u], xyz[3 * pp[k] + u]);
                    hi[u] = std::max(hi[u], xyz[3 * pp[k] + u]);
                }
            int ax = 0;
            for (int u = 1; u < 3; u++)
                if (hi[u] - lo[u] > hi[ax] - lo[ax]) ax = u;
            std::stable_sort(pp.begin() + b0, pp.begin() + b1,
                             [&](int a, int b) { return xyz[3 * a + ax] < xyz[3 * b + ax]; });
            const int half = std::min(b1 - b0, ((b1 - b0 + 1) / 2 + PATCH_V - 1) / PATCH_V * PATCH_V);
            todo.push_back({b0 + half, b1});
            todo.push_back({b0, b0 + half});
        }
        for (int k = 0; k < nv; k++) ip[pp[k]] = k;
    }
    // rest data of every triangle: the rest triangle in its own frame,
    // X0 = 0, X1 = (l, 0), X2 = (p, q); the rows of [X1 - X0, X2 - X0]^-1 are
    // the gradients g1, g2, and g0 = -g1 - g2
    const int v0 = c->mvn, t0 = c->mtn;
    std::vector<double> ref((size_t)ntri * 8, 0.0);
    for (int t = 0; t < ntri; t++) {
        double e1[3], e2[3], n[3], u1[3], u2[3];
        sub3h(xyz + 3 * tri[3 * t + 1], xyz + 3 * tri[3 * t], e1);
        sub3h(xyz + 3 * tri[3 * t + 2], xyz + 3 * tri[3 * t], e2);
        cross3h(e1, e2, n);
        const double l = std::sqrt(dot3h(e1, e1)), nn = std::sqrt(dot3h(n, n));
        if (!(l > 0) || !(nn > 1e-12 * l * l)) return fail3(c, CAPIB_E_ARG, "triangle %d is degenerate", t);
        for (int i = 0; i < 3; i++) { u1[i] = e1[i] / l; n[i] /= nn; }
        cross3h(n, u1, u2);
        const double pp = dot3h(e2, u1), qq = dot3h(e2, u2);
        double *g = &ref[8 * (size_t)t];
        g[2] = 1.0 / l;  g[3] = -pp / (l * qq);
        g[4] = 0.0;      g[5] = 1.0 / qq;
        g[0] = -g[2] - g[4];
        g[1] = -g[3] - g[5];
        g[6] = 0.5 * nn;
    }
    // rest area and volume, triangle by triangle, the volume about the first vertex
    double A0 = 0.0, V0 = 0.0;
    for (int t = 0; t < ntri; t++) {
        double p[3], q[3], r[3], e1[3], e2[3], n[3], qr[3];
        sub3h(xyz + 3 * tri[3 * t], xyz, p);
        sub3h(xyz + 3 * tri[3 * t + 1], xyz, q);
        sub3h(xyz + 3 * tri[3 * t + 2], xyz, r);
        sub3h(q, p, e1);
        sub3h(r, p, e2);
        cross3h(e1, e2, n);
        A0 += 0.5 * std::sqrt(dot3h(n, n));
        cross3h(q, r, qr);
        V0 += dot3h(p, qr) / 6.0;
    }
    if (!(A0 > 0) || !(V0 > 0)) return fail3(c, CAPIB_E_ARG, "membrane must enclose a positive volume (counter-clockwise from outside)");
    c->m_v0.push_back(v0); c->m_nv.push_back(nv); c->m_t0.push_back(t0); c->m_nt.push_back(ntri);
    for (int k = 0; k < 3 * ntri; k++) c->mtri.push_back(v0 + ip[tri[k]]);
    c->mref.insert(c->mref.end(), ref.begin(), ref.end());
    // interior edges: each directed edge a -> b (a < b) of a triangle, paired
    // with the triangle holding b -> a; in the order of first appearance
    std::vector<int> edges;
    std::vector<double> th0;
    {
        std::map<std::pair<int, int>, int> opp;   // directed edge -> opposite vertex
        for (int t = 0; t < ntri; t++)
            for (int k = 0; k < 3; k++) opp[{tri[3 * t + k], tri[3 * t + (k + 1) % 3]}] = tri[3 * t + (k + 2) % 3];
        for (int t = 0; t < ntri; t++)
            for (int k = 0; k < 3; k++) {
                const int a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3], c3 = tri[3 * t + (k + 2) % 3];
                if (a >= b) continue;
                auto it = opp.find({b, a});
                if (it == opp.end()) continue;
                const int E[4] = {a, b, c3, it->second};
                for (int r = 0; r < 4; r++) edges.push_back(v0 + ip[E[r]]);
                // rest dihedral angle, atan2((n1 x n2).e, n1.n2)
                double e[3], me[3], a3[3], b4[3], N1[3], N2[3], c12[3];
                sub3h(xyz + 3 * b, xyz + 3 * a, e);
                for (int i = 0; i < 3; i++) me[i] = -e[i];
                sub3h(xyz + 3 * c3, xyz + 3 * a, a3);
                sub3h(xyz + 3 * it->second, xyz + 3 * b, b4);
                cross3h(e, a3, N1);
                cross3h(me, b4, N2);
                const double r1 = std::sqrt(dot3h(N1, N1)), r2 = std::sqrt(dot3h(N2, N2)), l = std::sqrt(dot3h(e, e));
                double n1[3], n2[3];
                for (int i = 0; i < 3; i++) { n1[i] = N1[i] / r1; n2[i] = N2[i] / r2; }
                cross3h(n1, n2, c12);
                th0.push_back(std::atan2(dot3h(c12, e) / l, dot3h(n1, n2)));
            }
    }
    if (c->medge.size() / 4 + th0.size() > (3 * (size_t)L.max_membrane_triangles) / 2 + 1)
        return fail3(c, CAPIB_E_CAPACITY, "edge capacity exceeded");
    const double mp8[8] = {par->gs, par->c, par->ka, par->kv, par->mass, A0, V0, par->kb};
    c->mparam.insert(c->mparam.end(), mp8, mp8 + 8);
    c->nm++;
    c->umarks = false;
    c->mvn += nv;
    c->mtn += ntri;
    c->mmaxv = std::max(c->mmaxv, nv);
    c->medge.insert(c->medge.end(), edges.begin(), edges.end());
    c->mth0.insert(c->mth0.end(), th0.begin(), th0.end());
    // incident triangles of every vertex, ascending: the slot of each corner
    std::vector<int> vtb(c->mvn + 1, 0), tslot(3 * (size_t)c->mtn);
    for (int k = 0; k < 3 * c->mtn; k++) vtb[c->mtri[k] + 1]++;
    for (int v = 0; v < c->mvn; v++) vtb[v + 1] += vtb[v];
    // the edge terms of every vertex: its role in each edge, ascending
    const int me = (int)c->mth0.size();
    std::vector<int> veb(c->mvn + 1, 0), eslot(4 * (size_t)me);
    for (int k = 0; k < 4 * me; k++) veb[c->medge[k] + 1]++;
    for (int v = 0; v < c->mvn; v++) veb[v + 1] += veb[v];
    {
        std::vector<int> fe(veb.begin(), veb.end() - 1);
        for (int k = 0; k < me; k++)
            for (int r = 0; r < 4; r++) eslot[4 * k + r] = fe[c->medge[4 * k + r]]++;
    }
    std::vector<int> fill(vtb.begin(), vtb.end() - 1);
    for (int t = 0; t < c->mtn; t++)
        for (int a = 0; a < 3; a++) tslot[3 * t + a] = fill[c->mtri[3 * t + a]]++;
    // the membrane of each vertex, and the totals waves (64 triangles of one membrane each)
    // the caller's index of every internal vertex; the patches, triangle waves and edge waves
    for (int k = 0; k < nv; k++) c->perm.push_back(v0 + pp[k]);
    for (int k0 = 0; k0 < nv; k0 += PATCH_V) {
        c->ptab.push_back(v0 + k0);
        c->ptab.push_back(std::min(PATCH_V, nv - k0));
        c->ptab.push_back(c->nm - 1);
    }
    c->m_e0.push_back(me - (int)th0.size());
    c->m_ne.push_back((int)th0.size());
    std::vector<int> twave, ewave, mtw;
    for (int k = 0; k < c->nm; k++) {
        mtw.push_back((int)(twave.size() / 2));
        for (int t = c->m_t0[k]; t < c->m_t0[k] + c->m_nt[k]; t += 64) {
            twave.push_back(k);
            twave.push_back(t);
        }
        mtw.push_back((int)(twave.size() / 2) - mtw.back());
        for (int e = c->m_e0[k]; e < c->m_e0[k] + c->m_ne[k]; e += 64) {
            ewave.push_back(k);
            ewave.push_back(e);
        }
    }
    // the patch table with each patch's membrane's triangle waves (the
    // area and volume partials it adds)
    std::vector<int> pt5;
    for (size_t q = 0; q < c->ptab.size(); q += 3) {
        const int m = c->ptab[q + 2];
        pt5.insert(pt5.end(), {c->ptab[q], c->ptab[q + 1], m, mtw[2 * m], mtw[2 * m + 1]});
    }
    HIP3(c, hipMemcpyAsync(c->base + c->off_ptab, pt5.data(), pt5.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_me0, c->m_e0.data(), c->nm * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_mne, c->m_ne.data(), c->nm * 4, hipMemcpyHostToDevice, c->stream));
    if (!ewave.empty())
        HIP3(c, hipMemcpyAsync(c->base + c->off_ewave, ewave.data(), ewave.size() * 4, hipMemcpyHostToDevice,
                               c->stream));
    c->new_ = (int)(ewave.size() / 2);
    c->d.new_ = c->new_;
    if (me > 0) {
        HIP3(c, hipMemcpyAsync(c->base + c->off_medge, c->medge.data(), c->medge.size() * 4, hipMemcpyHostToDevice,
                               c->stream));
        HIP3(c, hipMemcpyAsync(c->base + c->off_mth0, c->mth0.data(), c->mth0.size() * 8, hipMemcpyHostToDevice,
                               c->stream));
        HIP3(c, hipMemcpyAsync(c->base + c->off_eslot, eslot.data(), eslot.size() * 4, hipMemcpyHostToDevice, c->stream));
    }
    HIP3(c, hipMemcpyAsync(c->base + c->off_veb, veb.data(), veb.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_twave, twave.data(), twave.size() * 4, hipMemcpyHostToDevice, c->stream));
    c->ntw = (int)(twave.size() / 2);
    c->d.ntw = c->ntw;
    // upload: the new positions into the current parity, the tables whole
    const size_t MS = (size_t)L.max_membrane_vertices;
    std::vector<double> plane(nv);
    for (int u = 0; u < 3; u++) {
        for (int k = 0; k < nv; k++) plane[k] = xyz[3 * pp[k] + u];
        HIP3(c, hipMemcpyAsync(c->base + c->off_MX[c->mpar] + (u * MS + v0) * 8, plane.data(), nv * 8,
                               hipMemcpyHostToDevice, c->stream));
        HIP3(c, hipMemsetAsync(c->base + c->off_Mdxm + (u * MS + v0) * 8, 0, nv * 8, c->stream));
        HIP3(c, hipMemsetAsync(c->base + c->off_MF + (u * MS + v0) * 8, 0, nv * 8, c->stream));
    }
    HIP3(c, hipMemcpyAsync(c->base + c->off_Mtri, c->mtri.data(), c->mtri.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_Mref, c->mref.data(), c->mref.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_vtb, vtb.data(), vtb.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_tslot, tslot.data(), tslot.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_mv0, c->m_v0.data(), c->nm * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_mnv, c->m_nv.data(), c->nm * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_mt0, c->m_t0.data(), c->nm * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_mnt, c->m_nt.data(), c->nm * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_mpar, c->mparam.data(), c->mparam.size() * 8, hipMemcpyHostToDevice,
                           c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    c->d.nm = c->nm;
    c->d.mv = c->mvn;
    if (first_vertex) *first_vertex = v0;
    return CAPIB_OK;
}

// positions of parity mpar <-> [mv][3] host doubles
static capib_status membrane_planes(capib3d_ctx *c, size_t off, double *out, const double *in) {
    const size_t MS = (size_t)c->lat.max_membrane_vertices, n = c->mvn;
    std::vector<double> pl(3 * n);
    if (in) {
        for (size_t v = 0; v < n; v++)
            for (int u = 0; u < 3; u++) pl[u * n + v] = in[3 * (size_t)c->perm[v] + u];
        for (int u = 0; u < 3; u++)
            HIP3(c, hipMemcpyAsync(c->base + off + u * MS * 8, &pl[u * n], n * 8, hipMemcpyHostToDevice, c->stream));
        HIP3(c, hipStreamSynchronize(c->stream));
        return CAPIB_OK;
    }
    for (int u = 0; u < 3; u++)
        HIP3(c, hipMemcpyAsync(&pl[u * n], c->base + off + u * MS * 8, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    for (size_t v = 0; v < n; v++)
        for (int u = 0; u < 3; u++) out[3 * (size_t)c->perm[v] + u] = pl[u * n + v];
    return CAPIB_OK;
}

capib_status capib3d_read_membrane_vertices(capib3d_ctx *c, double *xyz) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!xyz) return fail3(c, CAPIB_E_ARG, "null output");
    return c->mvn ? membrane_planes(c, c->off_MX[c->mpar], xyz, nullptr) : CAPIB_OK;
}

capib_status capib3d_write_membrane_vertices(capib3d_ctx *c, const double *xyz) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!xyz) return fail3(c, CAPIB_E_ARG, "null input");
    for (long long k = 0; k < 3LL * c->mvn; k++)
        if (!std::isfinite(xyz[k])) return fail3(c, CAPIB_E_ARG, "non-finite vertex");
    c->umarks = false;
    return c->mvn ? membrane_planes(c, c->off_MX[c->mpar], nullptr, xyz) : CAPIB_OK;
}

capib_status capib3d_membrane_spread_forces(capib3d_ctx *c, double *out) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!out) return fail3(c, CAPIB_E_ARG, "null output");
    return c->mvn ? membrane_planes(c, c->off_MF, out, nullptr) : CAPIB_OK;
}

capib_status capib3d_membrane_totals(capib3d_ctx *c, int32_t m, double *out4) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!out4 || m < 0 || m >= c->nm) return fail3(c, CAPIB_E_ARG, "no membrane %d", m);
    double t[2];
    HIP3(c, hipMemcpyAsync(t, c->base + c->off_mtot + 16 * (size_t)m, 16, hipMemcpyDeviceToHost, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    out4[0] = t[0];
    out4[1] = t[1];
    out4[2] = c->mparam[8 * (size_t)m + 5];
    out4[3] = c->mparam[8 * (size_t)m + 6];
    return CAPIB_OK;
}

capib_status capib3d_add_bonds(capib3d_ctx *c, int32_t m, int32_t ns, const int32_t *tri, const double *bary,
                               const capib3d_bonds *par) {
    capib_status s = need_ws(c);
    if (s) return s;
    const capib3d_lattice &L = c->lat;
    if (c->nsite > 0) return fail3(c, CAPIB_E_STATE, "the context already holds its bond sites");
    if (L.geometry != CAPIB3D_TUBE) return fail3(c, CAPIB_E_ARG, "bonds need the tube geometry");
    if (m < 0 || m >= c->nm) return fail3(c, CAPIB_E_ARG, "no membrane %d", m);
    if (ns < 1 || !tri || !bary || !par) return fail3(c, CAPIB_E_ARG, "bad bond arrays");
    if (ns > L.max_sites) return fail3(c, CAPIB_E_CAPACITY, "%d sites exceed the capacity of %d", ns, L.max_sites);
    const double pv[6] = {par->sigma, par->yeq, par->ycr, par->kf, par->kr0, par->lb};
    for (double x : pv)
        if (!std::isfinite(x)) return fail3(c, CAPIB_E_ARG, "non-finite bond parameter");
    if (par->kf < 0 || par->kr0 < 0 || !(par->lb > 0)) return fail3(c, CAPIB_E_ARG, "rates must be >= 0 and l_B > 0");
    std::vector<int> st(ns);
    for (int q = 0; q < ns; q++) {
        if (tri[q] < 0 || tri[q] >= c->m_nt[m]) return fail3(c, CAPIB_E_ARG, "site %d: triangle out of range", q);
        const double b1 = bary[2 * q], b2 = bary[2 * q + 1];
        if (!(b1 >= 0) || !(b2 >= 0) || !(b1 + b2 <= 1)) return fail3(c, CAPIB_E_ARG, "site %d: not inside its triangle", q);
        st[q] = c->m_t0[m] + tri[q];
    }
    // the sites of every triangle
    std::vector<int> tsb(c->mtn + 1, 0), tsl(ns);
    for (int q = 0; q < ns; q++) tsb[st[q] + 1]++;
    for (int t = 0; t < c->mtn; t++) tsb[t + 1] += tsb[t];
    {
        std::vector<int> f(tsb.begin(), tsb.end() - 1);
        for (int q = 0; q < ns; q++) tsl[f[st[q]]++] = q;
    }
    HIP3(c, hipMemcpyAsync(c->base + c->off_stri, st.data(), ns * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_sbary, bary, ns * 16, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemsetAsync(c->base + c->off_sbound, 0, ns * 4, c->stream));
    HIP3(c, hipMemsetAsync(c->base + c->off_sanc, 0, ns * 24, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_tsb, tsb.data(), tsb.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipMemcpyAsync(c->base + c->off_tsl, tsl.data(), ns * 4, hipMemcpyHostToDevice, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    Dev3 &d = c->d;
    d.b_sigma = par->sigma; d.b_yeq = par->yeq; d.b_ycr = par->ycr; d.b_kf = par->kf; d.b_kr0 = par->kr0;
    d.b_lb = par->lb; d.b_seed = par->seed;
    d.ns = ns;
    c->nsite = ns;
    return CAPIB_OK;
}

capib_status capib3d_read_bonds(capib3d_ctx *c, int32_t *bound, double *anchor, int64_t *nbound) {
    capib_status s = need_ws(c);
    if (s) return s;
    std::vector<int> b(c->nsite);
    if (c->nsite) {
        HIP3(c, hipMemcpyAsync(b.data(), c->base + c->off_sbound, c->nsite * 4, hipMemcpyDeviceToHost, c->stream));
        if (anchor)
            HIP3(c, hipMemcpyAsync(anchor, c->base + c->off_sanc, c->nsite * 24, hipMemcpyDeviceToHost, c->stream));
        HIP3(c, hipStreamSynchronize(c->stream));
    }
    int64_t n = 0;
    for (int q = 0; q < c->nsite; q++) {
        if (bound) bound[q] = b[q];
        n += b[q];
    }
    if (nbound) *nbound = n;
    return CAPIB_OK;
}

capib_status capib3d_write_bonds(capib3d_ctx *c, const int32_t *bound, const double *anchor) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!bound || !anchor) return fail3(c, CAPIB_E_ARG, "null input");
    for (int q = 0; q < c->nsite; q++)
        if ((bound[q] != 0 && bound[q] != 1) || !std::isfinite(anchor[3 * q]) || !std::isfinite(anchor[3 * q + 1]) ||
            !std::isfinite(anchor[3 * q + 2]))
            return fail3(c, CAPIB_E_ARG, "site %d: bad state", q);
    if (c->nsite) {
        HIP3(c, hipMemcpyAsync(c->base + c->off_sbound, bound, c->nsite * 4, hipMemcpyHostToDevice, c->stream));
        HIP3(c, hipMemcpyAsync(c->base + c->off_sanc, anchor, c->nsite * 24, hipMemcpyHostToDevice, c->stream));
        HIP3(c, hipStreamSynchronize(c->stream));
    }
    return CAPIB_OK;
}

capib_status capib3d_error_flags(capib3d_ctx *c, int32_t *flags) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!flags) return fail3(c, CAPIB_E_ARG, "null output");
    HIP3(c, hipMemcpyAsync(flags, c->base + c->off_err, 4, hipMemcpyDeviceToHost, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    return CAPIB_OK;
}

int32_t capib3d_membranes(const capib3d_ctx *c) { return c ? c->nm : 0; }
int32_t capib3d_membrane_vertex_count(const capib3d_ctx *c) { return c ? c->mvn : 0; }

capib_status capib3d_diagnostics(capib3d_ctx *c, double *out4, int64_t *step) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!out4) return fail3(c, CAPIB_E_ARG, "null output");
    const bool h16 = c->lat.storage == CAPIB_FP16_SHIFTED;
    if (c->par)
        hipLaunchKernelGGL((h16 ? k3_diag<_Float16, 1> : k3_diag<float, 1>), dim3(c->nblk), dim3(64 * WAVES), 0,
                           c->stream, c->d);
    else
        hipLaunchKernelGGL((h16 ? k3_diag<_Float16, 0> : k3_diag<float, 0>), dim3(c->nblk), dim3(64 * WAVES), 0,
                           c->stream, c->d);
    HIP3(c, hipGetLastError());
    std::vector<double> p((size_t)c->nblk * 4);
    HIP3(c, hipMemcpyAsync(p.data(), c->base + c->off_part, p.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    double t[4] = {0, 0, 0, 0};
    for (int b = 0; b < c->nblk; b++)
        for (int k = 0; k < 4; k++) t[k] += p[4 * (size_t)b + k];
    for (int k = 0; k < 4; k++) out4[k] = t[k];
    if (step) *step = c->step;
    return CAPIB_OK;
}

}  // extern "C"
