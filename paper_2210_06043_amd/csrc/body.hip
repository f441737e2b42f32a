// Per-membrane phase of the LBM-IB step: one workgroup per membrane, the
// membrane resident in LDS.
//
//   geometry and the FP64 Green's-theorem area (Sec. 2.3)
//   springs (Eq. 8), bending (Eq. 10), area penalty (Eq. 11)
//   repulsion (Eq. 12), ligand-receptor springs (Eq. 13),
//   pressure and viscous loads from the element probes (Eqs. 14-15)
//   Verlet position update (Eq. 17) and BDF2 vertex velocity (Eq. 18), or the
//   rigid BDF2 updates (Eqs. 19-20) with rigid kinematics
//   direct forcing U - u*: spread records for the near-tile sweep
//   bond kinetics with one Philox4x32-10 draw per site (Sec. 2.5)
//   the near tiles of the next step (tiles under the stencils of x^{n+1})
//
// The kernel is latency-bound (a few thousand vertices per step against a
// lattice of a million nodes), so every per-vertex global load is issued in
// one batch at entry and the membrane then lives in LDS; reductions combine
// their operands to keep the number of barriers low.
#include "capib_dev.hpp"
#include "capib_kernels.hpp"

namespace capib {

constexpr int BT = BODY_THREADS;
constexpr int VPT = MAXV_BODY / BT;   // vertices per thread
constexpr int MAX_BOX = 64;           // bounding boxes cached in LDS

// (ah, al) += (bh, bl), renormalised.
__device__ __forceinline__ void df_add2(float &ah, float &al, float bh, float bl) {
    float s = ah + bh;
    float bb = s - ah;
    float e = (ah - (s - bb)) + (bh - bb);
    e += al + bl;
    float h = s + e;
    al = e - (h - s);
    ah = h;
}

constexpr int TILE_SLOTS = 512;       // distinct 64x4 tiles per membrane in the LDS table
constexpr int HASH_PROBES = 64;       // linear-probe limit of the LDS table
constexpr int NEW_SLOTS = 1024;       // newly marked tiles listed per workgroup
constexpr int EMPTY_KEY = -1;

__device__ __forceinline__ unsigned hash_slot(int key, int slots) {
    return ((unsigned)key * 2654435761u) >> (32 - __builtin_ctz((unsigned)slots));
}

// Marks a tile as near for the step of parity p: flag and list entry, once.
// Within a workgroup an LDS table (stile, may be null) filters repeats before
// they reach global memory; across workgroups the flag's exchange does.  New
// tiles go to the workgroup's LDS list (snew/snum) when one is given, so that
// the global list is extended with a single counter update per workgroup
// (a counter that every vertex incremented would serialise the kernel).
__device__ __forceinline__ void mark_tile(const Dev &d, int p, int tile, int *stile, int *snew, int *snum) {
    if (stile) {
        unsigned t = hash_slot(tile, TILE_SLOTS);
        for (int q = 0; q < HASH_PROBES; q++) {
            int k = stile[t];
            if (k == EMPTY_KEY) k = atomicCAS(&stile[t], EMPTY_KEY, tile);
            if (k == EMPTY_KEY) break;   // first time in this workgroup
            if (k == tile) return;       // this workgroup has marked it already
            t = (t + 1) & (TILE_SLOTS - 1);
        }
    }
    if (atomicExch(&d.tnear[p][tile], 1) == 0) {
        if (snew) {
            const int k = atomicAdd(snum, 1);
            if (k < NEW_SLOTS) {
                snew[k] = tile;
                return;
            }
        }
        const int slot = atomicAdd(&d.ncount[p], 1);
        d.nlist[p][slot] = tile;
    }
}

// Spread record of vertex g at x^n: the stencil of the velocity coupling and
// the force dV (U - u*) to spread; the near-tile sweep gathers these records
// (spreading as a gather: no atomics, sums in vertex order).
__device__ __forceinline__ void write_spread(const Dev &d, int g, float xh, float xl, float yh, float yl, float fx,
                                             float fy) {
    int ix0, iy0;
    float wx[4], wy[4], inv;
    stencil(d, xh, xl, yh, yl, false, ix0, iy0, wx, wy, inv);
    // columns wrapped into [0, nx); rows too when y is periodic
    d.sp_org[g] = make_int2(wrapi(ix0, d.nx), d.walls ? iy0 : wrapi(iy0, d.ny));
    d.sp_wx[g] = make_float4(wx[0] * inv, wx[1] * inv, wx[2] * inv, wx[3] * inv);
    d.sp_wy[g] = make_float4(wy[0], wy[1], wy[2], wy[3]);
    d.sp_f[g] = make_float2(fx, fy);
}

__global__ __launch_bounds__(BT) void k_body(Dev d, int par) {
    __shared__ float sxh[MAXV_BODY], sxl[MAXV_BODY], syh[MAXV_BODY], syl[MAXV_BODY];
    __shared__ float slen[MAXV_BODY], snlx[MAXV_BODY], snly[MAXV_BODY];
    __shared__ float snvx[MAXV_BODY], snvy[MAXV_BODY], sbend[MAXV_BODY];
    __shared__ float sSx[MAXV_BODY], sSy[MAXV_BODY];   // spring force k (l - l0) t_hat of each element
    __shared__ float sHx[MAXV_BODY], sHy[MAXV_BODY];   // half of the element's area, bond and load force
    __shared__ float sbox[MAX_BOX][4];
    __shared__ double shd[BT / 64];
    __shared__ float shf[BT / 64][5];
    __shared__ float srig[8];
    __shared__ int stile[TILE_SLOTS];
    __shared__ int snew[NEW_SLOTS];
    __shared__ int snum, snbase;

    const int b = blockIdx.x, tid = threadIdx.x;
    if (tid == 0) snum = 0;
    for (int h = tid; h < TILE_SLOTS; h += BT) stile[h] = EMPTY_KEY;
    const BodyParams P = d.bp[b];
    const int n = P.n, v0 = P.vstart, npar = par ^ 1;
    const long long step = *d.counter - 1;
    const bool deform = P.kind == DEFORMABLE, rigid = P.kind == RIGID;

    // ---- every per-vertex global load of the step, issued together -------------
    float rxh[VPT], rxl[VPT], ryh[VPT], ryl[VPT], rl0[VPT], rth0[VPT], rdxm[VPT], rdym[VPT];
    float2 rus[VPT];
    float4 rpr[VPT];
    int2 rsr[VPT];
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BT;
        if (v >= n) continue;
        const int g = v0 + v;
        rxh[k] = d.pxh[par][g]; rxl[k] = d.pxl[par][g];
        ryh[k] = d.pyh[par][g]; ryl[k] = d.pyl[par][g];
        rl0[k] = d.l0[g]; rth0[k] = d.th0[g];
        rus[k] = d.ustar[g];
        rpr[k] = d.probe4[g];
        rdxm[k] = d.dxm[g]; rdym[k] = d.dym[g];
        rsr[k] = P.n_sites ? d.srange[g] : make_int2(0, 0);
    }
    if (tid < d.nbodies && tid < MAX_BOX)
        for (int c = 0; c < 4; c++) sbox[tid][c] = d.bs[tid].bbox[par][c];
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BT;
        if (v >= n) continue;
        sxh[v] = rxh[k]; sxl[v] = rxl[k]; syh[v] = ryh[k]; syl[v] = ryl[k];
    }
    __syncthreads();

    // ---- elements: length, outward normal, FP64 area, spring and external forces
    double apart = 0.0;
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int l = tid + k * BT;
        if (l >= n) continue;
        const int m = (l + 1 == n) ? 0 : l + 1;
        const float tx = (sxh[m] - rxh[k]) + (sxl[m] - rxl[k]);
        const float ty = (syh[m] - ryh[k]) + (syl[m] - ryl[k]);
        const float len = sqrtf(tx * tx + ty * ty);
        const float nx = ty / len, ny = -tx / len;
        slen[l] = len; snlx[l] = nx; snly[l] = ny;
        const double xa = ((double)rxh[k] - (double)sxh[0]) + ((double)rxl[k] - (double)sxl[0]);
        const double ya = ((double)ryh[k] - (double)syh[0]) + ((double)ryl[k] - (double)syl[0]);
        const double xb = ((double)sxh[m] - (double)sxh[0]) + ((double)sxl[m] - (double)sxl[0]);
        const double yb = ((double)syh[m] - (double)syh[0]) + ((double)syl[m] - (double)syl[0]);
        apart += xa * yb - xb * ya;
        // Eq. (8): the element pulls its ends together along t_hat = (-ny, nx)
        const float ks = deform ? P.ks * (len - rl0[k]) : 0.0f;
        sSx[l] = -ks * ny;
        sSy[l] = ks * nx;
        // Eq. (13): engaged bonds of this element, along its outward normal
        float bm = 0.0f;
        for (int s = rsr[k].x; s < rsr[k].y; s++) {
            if (!d.s_state[s]) continue;
            const float f = d.s_frac[s];
            const float dx = (rxh[k] - d.s_anh[s]) + ((rxl[k] - d.s_anl[s]) + f * tx);
            const float dy = (ryh[k] + 0.5f) + (ryl[k] + f * ty);
            bm += P.sigma * (sqrtf(dx * dx + dy * dy) - P.yeq);
        }
        // Eqs. (14)-(15): (-p n + sigma . n) l from the element's probe
        const float4 q = rpr[k];
        const float Lx = ((q.y - q.x) * nx + q.z * ny) * len;
        const float Ly = (q.z * nx + (q.w - q.x) * ny) * len;
        sHx[l] = 0.5f * (bm * nx + Lx);
        sHy[l] = 0.5f * (bm * ny + Ly);
    }
    apart = wave_sum(apart);
    if ((tid & 63) == 0) shd[tid >> 6] = apart;
    __syncthreads();
    double asum = 0.0;
#pragma unroll
    for (int w = 0; w < BT / 64; w++) asum += shd[w];
    const double area = 0.5 * asum;

    // ---- vertices: outward normal, bending magnitude; area penalty per element
    const float cA = deform ? (float)((double)P.ka * (1.0 - area / P.A0) * (double)P.pref) : 0.0f;
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BT;
        if (v >= n) continue;
        const int p = (v == 0) ? n - 1 : v - 1;
        const float ax = snlx[p] + snlx[v], ay = snly[p] + snly[v];
        const float an = sqrtf(ax * ax + ay * ay);
        snvx[v] = ax / an;
        snvy[v] = ay / an;
        // turning angle from the unit tangents (-nly, nlx) of elements p and v
        const float cr = snlx[p] * snly[v] - snly[p] * snlx[v];
        const float dt = snly[p] * snly[v] + snlx[p] * snlx[v];
        sbend[v] = deform ? P.kb * (atan2f(cr, dt) - rth0[k]) : 0.0f;
        // Eq. (11): k_a (1 - A/A0) p_ref l n_l, half to each end (element v)
        sHx[v] += 0.5f * cA * slen[v] * snlx[v];
        sHy[v] += 0.5f * cA * slen[v] * snly[v];
    }
    __syncthreads();

    // ---- total force per vertex ---------------------------------------------------------
    float fvx[VPT], fvy[VPT];
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        fvx[k] = 0.0f;
        fvy[k] = 0.0f;
        const int v = tid + k * BT;
        if (v >= n || P.kind == FIXED) continue;
        const int p = (v == 0) ? n - 1 : v - 1;
        const int m = (v + 1 == n) ? 0 : v + 1;
        // springs of both elements, half of the element forces of both elements
        float fx = (sSx[v] - sSx[p]) + (sHx[v] + sHx[p]);
        float fy = (sSy[v] - sSy[p]) + (sHy[v] + sHy[p]);
        if (deform) {
            // Eq. (10): own term and the neighbour shares l_left/(l_left + l_right)
            const int pp = (p == 0) ? n - 1 : p - 1;
            const float sp = slen[p] / (slen[pp] + slen[p]);
            const float sm = slen[v] / (slen[v] + slen[m]);
            fx += -sbend[v] * snvx[v] + sbend[p] * sp * snvx[p] + sbend[m] * sm * snvx[m];
            fy += -sbend[v] * snvy[v] + sbend[p] * sp * snvy[p] + sbend[m] * sm * snvy[m];
        }
        // Eq. (12): repulsion from vertices of other bodies within the cut-off
        const float myx = rxh[k] + rxl[k], myy = ryh[k] + ryl[k];
        const float L = (float)d.nx;
        const float cut2 = d.rep_cut * d.rep_cut;
        for (int c = 0; c < d.nbodies; c++) {
            if (c == b) continue;
            float bb0, bb1, bb2, bb3;
            if (c < MAX_BOX) { bb0 = sbox[c][0]; bb1 = sbox[c][1]; bb2 = sbox[c][2]; bb3 = sbox[c][3]; }
            else { const float *bb = d.bs[c].bbox[par]; bb0 = bb[0]; bb1 = bb[1]; bb2 = bb[2]; bb3 = bb[3]; }
            float dxc = myx - 0.5f * (bb0 + bb1);
            dxc -= L * rintf(dxc / L);
            if (fabsf(dxc) > 0.5f * (bb1 - bb0) + d.rep_cut + 0.5f) continue;
            if (myy < bb2 - d.rep_cut - 0.5f || myy > bb3 + d.rep_cut + 0.5f) continue;
            const int cs = d.bp[c].vstart, cn = d.bp[c].n;
            for (int u = cs; u < cs + cn; u++) {
                float ddx = (rxh[k] - d.pxh[par][u]) + (rxl[k] - d.pxl[par][u]);
                ddx -= L * rintf(ddx / L);
                const float ddy = (ryh[k] - d.pyh[par][u]) + (ryl[k] - d.pyl[par][u]);
                const float r2 = ddx * ddx + ddy * ddy;
                if (r2 < cut2) {
                    const float dd = fmaxf(sqrtf(r2), d.rep_dmin);
                    const float f = d.rep_pref / (dd * dd * sqrtf(dd));
                    fx -= f * snvx[v];
                    fy -= f * snvy[v];
                }
            }
        }
        fvx[k] = fx;
        fvy[k] = fy;
        d.force[v0 + v] = make_float2(fx, fy);
    }

    // ---- integration (Eqs. 16-20), direct forcing and spreading at x^n -----------------
    float nxh[VPT], nxl[VPT], nyh[VPT], nyl[VPT];
    if (rigid) {
        const float phin = d.bs[b].phih + d.bs[b].phil;
        const float shalf = sinf(0.5f * phin);
        const float c1 = -2.0f * shalf * shalf, sphi = sinf(phin);
        float Fx = 0.0f, Fy = 0.0f, M = 0.0f;
#pragma unroll
        for (int k = 0; k < VPT; k++) {
            const int v = tid + k * BT;
            if (v >= n) continue;
            const float rx = d.r0x[v0 + v], ry = d.r0y[v0 + v];
            const float armx = rx + (c1 * rx - sphi * ry), army = ry + (sphi * rx + c1 * ry);
            Fx += fvx[k];
            Fy += fvy[k];
            M += armx * fvy[k] - army * fvx[k];
        }
        Fx = wave_sum(Fx);
        Fy = wave_sum(Fy);
        M = wave_sum(M);
        if ((tid & 63) == 0) { shf[tid >> 6][0] = Fx; shf[tid >> 6][1] = Fy; shf[tid >> 6][2] = M; }
        __syncthreads();
        if (tid == 0) {
            Fx = 0.0f; Fy = 0.0f; M = 0.0f;
            for (int w = 0; w < BT / 64; w++) { Fx += shf[w][0]; Fy += shf[w][1]; M += shf[w][2]; }
            BodyState &S = d.bs[b];
            const float ux = (2.0f / 3.0f) * (2.0f * S.ucx - 0.5f * S.ucxm + Fx * P.inv_mass);
            const float uy = (2.0f / 3.0f) * (2.0f * S.ucy - 0.5f * S.ucym + Fy * P.inv_mass);
            const float om = (2.0f / 3.0f) * (2.0f * S.om - 0.5f * S.omm + M * P.inv_inertia);
            S.ucxm = S.ucx; S.ucym = S.ucy; S.omm = S.om;
            S.ucx = ux; S.ucy = uy; S.om = om;
            df_add(S.dcxh, S.dcxl, ux);
            df_add(S.dcyh, S.dcyl, uy);
            df_add(S.phih, S.phil, om);
            srig[0] = ux; srig[1] = uy; srig[2] = om;
            srig[3] = S.dcxh; srig[4] = S.dcxl; srig[5] = S.dcyh; srig[6] = S.dcyl;
            srig[7] = S.phih + S.phil;
        }
        __syncthreads();
        const float ph = srig[7];
        const float sh2 = sinf(0.5f * ph);
        const float c1n = -2.0f * sh2 * sh2, sn = sinf(ph);
#pragma unroll
        for (int k = 0; k < VPT; k++) {
            const int v = tid + k * BT;
            if (v >= n) continue;
            const float rx = d.r0x[v0 + v], ry = d.r0y[v0 + v];
            const float drx = c1n * rx - sn * ry, dry = sn * rx + c1n * ry;
            float xh = d.x0h[v0 + v], xl = d.x0l[v0 + v], yh = d.y0h[v0 + v], yl = d.y0l[v0 + v];
            df_add2(xh, xl, srig[3], srig[4]);
            df_add2(yh, yl, srig[5], srig[6]);
            df_add(xh, xl, drx);
            df_add(yh, yl, dry);
            nxh[k] = xh; nxl[k] = xl; nyh[k] = yh; nyl[k] = yl;
            const float Ux = srig[0] - srig[2] * (ry + dry);
            const float Uy = srig[1] + srig[2] * (rx + drx);
            d.target[v0 + v] = make_float2(Ux, Uy);
            const int p = (v == 0) ? n - 1 : v - 1;
            const float dV = 0.5f * (slen[p] + slen[v]);
            write_spread(d, v0 + v, rxh[k], rxl[k], ryh[k], ryl[k], dV * (Ux - rus[k].x), dV * (Uy - rus[k].y));
        }
    } else {
        bool bad = false;
#pragma unroll
        for (int k = 0; k < VPT; k++) {
            const int v = tid + k * BT;
            if (v >= n) continue;
            float Ux = 0.0f, Uy = 0.0f;
            nxh[k] = rxh[k]; nxl[k] = rxl[k]; nyh[k] = ryh[k]; nyl[k] = ryl[k];
            if (deform) {
                const float dx = rus[k].x + 0.5f * fvx[k] / P.vmass;
                const float dy = rus[k].y + 0.5f * fvy[k] / P.vmass;
                Ux = 1.5f * dx - 0.5f * rdxm[k];
                Uy = 1.5f * dy - 0.5f * rdym[k];
                d.dxm[v0 + v] = dx;
                d.dym[v0 + v] = dy;
                df_add(nxh[k], nxl[k], dx);
                df_add(nyh[k], nyl[k], dy);
                bad |= !isfinite(dx) || !isfinite(dy);
            }
            d.target[v0 + v] = make_float2(Ux, Uy);
            const int p = (v == 0) ? n - 1 : v - 1;
            const float dV = 0.5f * (slen[p] + slen[v]);
            write_spread(d, v0 + v, rxh[k], rxl[k], ryh[k], ryl[k], dV * (Ux - rus[k].x), dV * (Uy - rus[k].y));
        }
        if (bad) atomicOr(d.err, FLAG_NONFINITE_IB);
    }
    __syncthreads();   // every thread has read x^n from LDS

    // near tiles of the next step: the tiles under the stencils of x^{n+1}
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BT;
        if (v >= n) continue;
        int tl[9];
        const int c = stencil_tiles(d, nxh[k], nxl[k], nyh[k], nyl[k], tl);
        for (int q = 0; q < c; q++) mark_tile(d, npar, tl[q], stile, snew, &snum);
    }
    __syncthreads();
    if (tid == 0) {
        const int m = min(snum, NEW_SLOTS);
        snbase = m ? atomicAdd(&d.ncount[npar], m) : 0;
    }
    __syncthreads();
    for (int k = tid; k < min(snum, NEW_SLOTS); k += BT) d.nlist[npar][snbase + k] = snew[k];
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BT;
        if (v >= n) continue;
        sxh[v] = nxh[k]; sxl[v] = nxl[k]; syh[v] = nyh[k]; syl[v] = nyl[k];
        d.pxh[npar][v0 + v] = nxh[k];
        d.pxl[npar][v0 + v] = nxl[k];
        d.pyh[npar][v0 + v] = nyh[k];
        d.pyl[npar][v0 + v] = nyl[k];
    }
    __syncthreads();

    // ---- bond kinetics at x^{n+1} --------------------------------------------------------
    int cnt = 0;
    for (int s = P.site_start + tid; s < P.site_start + P.n_sites; s += BT) {
        const int e = d.s_host[s] - v0;
        const int m = (e + 1 == n) ? 0 : e + 1;
        const float f = d.s_frac[s];
        const float tx = (sxh[m] - sxh[e]) + (sxl[m] - sxl[e]);
        const float ty = (syh[m] - syh[e]) + (syl[m] - syl[e]);
        const float xsh = sxh[e], xsl = sxl[e] + f * tx;
        const float ysh = syh[e], ysl = syl[e] + f * ty;
        const uint32_t w = philox_w0((uint32_t)step, (uint32_t)d.s_orig[s], (uint32_t)((unsigned long long)step >> 32),
                                     0u, P.seed_lo, P.seed_hi);
        const float r = (float)(w >> 8) * (1.0f / 16777216.0f);
        int st = d.s_state[s];
        if (st) {
            const float dx = (xsh - d.s_anh[s]) + (xsl - d.s_anl[s]);
            const float dy = (ysh + 0.5f) + ysl;
            const float yl = sqrtf(dx * dx + dy * dy);
            const float Pr = -expm1f(-P.kr0 * expf(fabsf(yl - P.yeq) / P.lb));
            if (r < Pr) st = 0;
        } else {
            const float gap = (ysh + 0.5f) + ysl;
            if (gap < P.ycr) {
                const float Pf = -expm1f(-P.kf);
                if (r < Pf) {
                    st = 1;
                    const float ah = xsh + xsl;
                    d.s_anh[s] = ah;
                    d.s_anl[s] = xsl - (ah - xsh);
                }
            }
        }
        d.s_state[s] = st;
        cnt += st;
    }

    // ---- N_L and the bounding box of x^{n+1} (for next step's repulsion culling) ----------
    float xmin = 3.0e38f, xmax = -3.0e38f, ymin = 3.0e38f, ymax = -3.0e38f;
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BT;
        if (v >= n) continue;
        const float x = nxh[k] + nxl[k], y = nyh[k] + nyl[k];
        xmin = fminf(xmin, x); xmax = fmaxf(xmax, x);
        ymin = fminf(ymin, y); ymax = fmaxf(ymax, y);
    }
    float fc = (float)cnt;
#pragma unroll
    for (int msk = 32; msk >= 1; msk >>= 1) {
        fc += __shfl_xor(fc, msk);
        xmin = fminf(xmin, __shfl_xor(xmin, msk));
        xmax = fmaxf(xmax, __shfl_xor(xmax, msk));
        ymin = fminf(ymin, __shfl_xor(ymin, msk));
        ymax = fmaxf(ymax, __shfl_xor(ymax, msk));
    }
    if ((tid & 63) == 0) {
        const int w = tid >> 6;
        shf[w][0] = fc; shf[w][1] = xmin; shf[w][2] = xmax; shf[w][3] = ymin; shf[w][4] = ymax;
    }
    __syncthreads();
    if (tid == 0) {
        float c = 0.0f, a0 = 3.0e38f, a1 = -3.0e38f, a2 = 3.0e38f, a3 = -3.0e38f;
        for (int w = 0; w < BT / 64; w++) {
            c += shf[w][0];
            a0 = fminf(a0, shf[w][1]); a1 = fmaxf(a1, shf[w][2]);
            a2 = fminf(a2, shf[w][3]); a3 = fmaxf(a3, shf[w][4]);
        }
        BodyState &S = d.bs[b];
        S.n_bound = (int)c;
        S.bbox[npar][0] = a0; S.bbox[npar][1] = a1;
        S.bbox[npar][2] = a2; S.bbox[npar][3] = a3;
    }
}

// Near tiles of the current positions (before the first step, after a
// checkpoint is loaded or membranes are added).  The flags and the count of
// parity par must be clear.
__global__ __launch_bounds__(256) void k_mark(Dev d, int par) {
    const int v = blockIdx.x * 256 + threadIdx.x;
    if (v >= d.nverts) return;
    int tl[9];
    const int c = stencil_tiles(d, d.pxh[par][v], d.pxl[par][v], d.pyh[par][v], d.pyl[par][v], tl);
    for (int q = 0; q < c; q++) mark_tile(d, par, tl[q], nullptr, nullptr, nullptr);
}

hipError_t launch_mark(const Dev &d, int par, hipStream_t st) {
    if (d.nverts == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark, dim3((d.nverts + 255) / 256), dim3(256), 0, st, d, par);
    return hipGetLastError();
}

hipError_t launch_body(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (d.nbodies == 0) {
        // keep the event pair meaningful for callers that time every phase
        if (e0) { hipError_t e = hipEventRecord(e0, st); if (e != hipSuccess) return e; }
        if (e1) return hipEventRecord(e1, st);
        return hipSuccess;
    }
    hipExtLaunchKernelGGL(k_body, dim3(d.nbodies), dim3(BT), 0, st, e0, e1, 0, d, par);
    return hipGetLastError();
}

}  // namespace capib
