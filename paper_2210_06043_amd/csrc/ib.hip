// Immersed-boundary phase of the LBM-IB step.
//
// k_interp: cosine-delta interpolation (Sec. 2.2) of the pre-coupling fluid
//   velocity u* = (sum h e + g/2)/rho to every membrane vertex, and of the
//   pressure c_s^2 drho and viscous stress -(1 - 1/2tau) Pi_neq to the probe
//   of every element, 1.2 dx along its outward normal (Sec. 2.6).  Sixteen
//   lanes serve one point, one stencil node each, and reduce with shuffles.
// k_body: one workgroup per membrane with the membrane resident in LDS:
//   geometry and the FP64 Green's-theorem area (Sec. 2.3), springs (Eq. 8),
//   bending (Eq. 10), area penalty (Eq. 11), repulsion (Eq. 12), bonds
//   (Eq. 13), pressure and viscous loads (Eqs. 14-15), Verlet + BDF2
//   (Eqs. 16-18) or rigid BDF2 (Eqs. 19-20), direct forcing and spreading
//   into an int64 fixed-point force field (deterministic), and the bond
//   kinetics with a Philox4x32-10 draw per site (Sec. 2.5).
#include "capib_dev.hpp"
#include "capib_kernels.hpp"

namespace capib {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// Fixed-order sum over a 256-thread workgroup (4 waves).
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *sh) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

template <bool MAX>
__device__ __forceinline__ float block_ext(float v, float *sh) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        float o = __shfl_xor(v, m);
        v = MAX ? fmaxf(v, o) : fminf(v, o);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return MAX ? fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]))
               : fminf(fminf(sh[0], sh[1]), fminf(sh[2], sh[3]));
}

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

// ---- interpolation ----------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void node_moments(const Dev &d, const T *A, int i, int j, bool stress, float out[4]) {
    float h[9];
    const float uref = pull_dev<T>(d, A, i, j, h);   // deviations from the row reference
    const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const float jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
    const float jy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);
    const float rho = 1.0f + drho;
    const float dux = (jx + 0.5f * d.gx - drho * uref) / rho;
    const float duy = (jy + 0.5f * d.gy) / rho;
    if (!stress) {
        out[0] = uref + dux;
        out[1] = duy;
        return;
    }
    // non-equilibrium momentum flux h - h_eq(drho, u*) (Eq. 2); the row
    // reference cancels between the two terms
    const EqDev E(drho, uref, dux, duy);
    float neq[9];
    const float ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const float ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
    for (int q = 0; q < 9; q++) {
        const float w = q == 0 ? 4.0f / 9.0f : (q < 5 ? 1.0f / 9.0f : 1.0f / 36.0f);
        neq[q] = h[q] - E(ex[q], ey[q], w);
    }
    const float pxx = (neq[1] + neq[3]) + ((neq[5] + neq[6]) + (neq[7] + neq[8]));
    const float pyy = (neq[2] + neq[4]) + ((neq[5] + neq[6]) + (neq[7] + neq[8]));
    const float pxy = (neq[5] - neq[6]) + (neq[7] - neq[8]);
    out[0] = drho * (1.0f / 3.0f);
    out[1] = -d.fc * pxx;
    out[2] = -d.fc * pxy;
    out[3] = -d.fc * pyy;
}

__global__ __launch_bounds__(INTERP_THREADS) void k_interp(Dev d, int par) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *d.counter += 1;   // steps started
    const int gid = blockIdx.x * INTERP_THREADS + threadIdx.x;
    const int p = gid >> 4, lane = gid & 15;
    if (p >= 2 * d.nverts) return;    // whole groups of 16 leave together
    const bool probe = p >= d.nverts;
    const int v = probe ? p - d.nverts : p;
    const int b = d.vbody[v];
    const int vs = d.bp[b].vstart, n = d.bp[b].n;
    const int vn = (v + 1 - vs == n) ? vs : v + 1;
    float xh = d.pxh[par][v], xl = d.pxl[par][v], yh = d.pyh[par][v], yl = d.pyl[par][v];
    if (probe) {
        const float tx = (d.pxh[par][vn] - xh) + (d.pxl[par][vn] - xl);
        const float ty = (d.pyh[par][vn] - yh) + (d.pyl[par][vn] - yl);
        const float len = sqrtf(tx * tx + ty * ty);
        xl += 0.5f * tx + d.probe * (ty / len);
        yl += 0.5f * ty - d.probe * (tx / len);
    }
    int ix0, iy0;
    float wx[4], wy[4], inv;
    const bool out = stencil(d, xh, xl, yh, yl, probe, ix0, iy0, wx, wy, inv);
    if (out && !probe && lane == 0) atomicOr(d.err, FLAG_VERTEX_OUT);
    const int a = lane & 3, bb = lane >> 2;
    const float W = wx[a] * wy[bb] * inv;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int j = iy0 + bb;
    if (!d.walls) j = wrapi(j, d.ny);
    if (W != 0.0f && j >= 0 && j < d.ny) {
        const int i = wrapi(ix0 + a, d.nx);
        float m[4];
        if (d.storage == 0)
            node_moments<float>(d, (const float *)d.pop[par], i, j, probe, m);
        else
            node_moments<_Float16>(d, (const _Float16 *)d.pop[par], i, j, probe, m);
        acc[0] = W * m[0];
        acc[1] = W * m[1];
        if (probe) {
            acc[2] = W * m[2];
            acc[3] = W * m[3];
        }
    }
#pragma unroll
    for (int c = 0; c < 4; c++) {
        float s = acc[c];
        s += __shfl_xor(s, 1, 16);
        s += __shfl_xor(s, 2, 16);
        s += __shfl_xor(s, 4, 16);
        s += __shfl_xor(s, 8, 16);
        acc[c] = s;
    }
    if (lane == 0) {
        if (probe)
            d.probe4[v] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        else
            d.ustar[v] = make_float2(acc[0], acc[1]);
    }
}

// ---- spreading -------------------------------------------------------------------------------

__device__ __forceinline__ void spread(const Dev &d, float xh, float xl, float yh, float yl, float vx, float vy,
                                       uint32_t tag) {
    int ix0, iy0;
    float wx[4], wy[4], inv;
    stencil(d, xh, xl, yh, yl, false, ix0, iy0, wx, wy, inv);
#pragma unroll
    for (int b = 0; b < 4; b++) {
        if (wy[b] == 0.0f) continue;
        int j = iy0 + b;
        if (!d.walls) j = wrapi(j, d.ny);
        if (j < 0 || j >= d.ny) continue;
#pragma unroll
        for (int a = 0; a < 4; a++) {
            const float W = wx[a] * wy[b] * inv;
            if (W == 0.0f) continue;
            const int i = wrapi(ix0 + a, d.nx);
            const float cx = W * vx, cy = W * vy;
            if (!(fabsf(cx) <= FIX_LIMIT) || !(fabsf(cy) <= FIX_LIMIT)) {
                atomicOr(d.err, FLAG_FORCE_RANGE);
                continue;
            }
            const long long qx = __float2ll_rn(cx * FIX_ONE);
            const long long qy = __float2ll_rn(cy * FIX_ONE);
            unsigned long long *f = (unsigned long long *)(d.fib + 2 * ((long long)j * d.pitch + i));
            if (qx) atomicAdd(f, (unsigned long long)qx);
            if (qy) atomicAdd(f + 1, (unsigned long long)qy);
            d.tflag[(j / TILE_Y) * d.ntx + i / TILE_X] = tag;
        }
    }
}

// ---- per-membrane phase ------------------------------------------------------------------------

constexpr int VPT = MAXV_BODY / BODY_THREADS;   // vertices per thread

__global__ __launch_bounds__(BODY_THREADS) void k_body(Dev d, int par) {
    __shared__ float sxh[MAXV_BODY], sxl[MAXV_BODY], syh[MAXV_BODY], syl[MAXV_BODY];
    __shared__ float slen[MAXV_BODY], snlx[MAXV_BODY], snly[MAXV_BODY];
    __shared__ float snvx[MAXV_BODY], snvy[MAXV_BODY], sbend[MAXV_BODY], sbond[MAXV_BODY];
    __shared__ double shd[4];
    __shared__ float shf[4];
    __shared__ int shi[4];
    __shared__ float srig[10];

    const int b = blockIdx.x, tid = threadIdx.x;
    const BodyParams P = d.bp[b];
    const int n = P.n, v0 = P.vstart, npar = par ^ 1;
    const long long step = *d.counter - 1;
    const uint32_t tag = (uint32_t)(step + 1);

    for (int v = tid; v < n; v += BODY_THREADS) {
        sxh[v] = d.pxh[par][v0 + v];
        sxl[v] = d.pxl[par][v0 + v];
        syh[v] = d.pyh[par][v0 + v];
        syl[v] = d.pyl[par][v0 + v];
    }
    __syncthreads();

    // elements: length, outward normal, FP64 area, bond tension per element
    double apart = 0.0;
    for (int l = tid; l < n; l += BODY_THREADS) {
        const int m = (l + 1 == n) ? 0 : l + 1;
        const float tx = (sxh[m] - sxh[l]) + (sxl[m] - sxl[l]);
        const float ty = (syh[m] - syh[l]) + (syl[m] - syl[l]);
        const float len = sqrtf(tx * tx + ty * ty);
        slen[l] = len;
        snlx[l] = ty / len;
        snly[l] = -tx / len;
        const double xa = ((double)sxh[l] - (double)sxh[0]) + ((double)sxl[l] - (double)sxl[0]);
        const double ya = ((double)syh[l] - (double)syh[0]) + ((double)syl[l] - (double)syl[0]);
        const double xb = ((double)sxh[m] - (double)sxh[0]) + ((double)sxl[m] - (double)sxl[0]);
        const double yb = ((double)syh[m] - (double)syh[0]) + ((double)syl[m] - (double)syl[0]);
        apart += xa * yb - xb * ya;
        float bm = 0.0f;
        if (P.n_sites) {
            const int2 sr = d.srange[v0 + l];
            for (int s = sr.x; s < sr.y; s++) {
                if (!d.s_state[s]) continue;
                const float f = d.s_frac[s];
                const float dx = (sxh[l] - d.s_anh[s]) + ((sxl[l] - d.s_anl[s]) + f * tx);
                const float dy = (syh[l] + 0.5f) + (syl[l] + f * ty);
                bm += P.sigma * (sqrtf(dx * dx + dy * dy) - P.yeq);
            }
        }
        sbond[l] = bm;
    }
    const double area = 0.5 * block_sum(apart, shd);

    // vertices: outward vertex normal and bending magnitude k_b (theta - theta0)
    for (int v = tid; v < n; v += BODY_THREADS) {
        const int p = (v == 0) ? n - 1 : v - 1;
        const float ax = snlx[p] + snlx[v], ay = snly[p] + snly[v];
        const float an = sqrtf(ax * ax + ay * ay);
        snvx[v] = ax / an;
        snvy[v] = ay / an;
        // unit tangents are (-nly, nlx)
        const float cr = snlx[p] * snly[v] - snly[p] * snlx[v];
        const float dt = snly[p] * snly[v] + snlx[p] * snlx[v];
        sbend[v] = (P.kind == DEFORMABLE) ? P.kb * (atan2f(cr, dt) - d.th0[v0 + v]) : 0.0f;
    }
    __syncthreads();

    // total force on each vertex
    const float cA = (float)((double)P.ka * (1.0 - area / P.A0) * (double)P.pref);
    float fvx[VPT], fvy[VPT];
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        fvx[k] = 0.0f;
        fvy[k] = 0.0f;
        const int v = tid + k * BODY_THREADS;
        if (v >= n || P.kind == FIXED) continue;
        const int p = (v == 0) ? n - 1 : v - 1;
        const int m = (v + 1 == n) ? 0 : v + 1;
        float fx = 0.0f, fy = 0.0f;
        if (P.kind == DEFORMABLE) {
            const float kv = P.ks * (slen[v] - d.l0[v0 + v]);
            const float kp = P.ks * (slen[p] - d.l0[v0 + p]);
            fx += kv * (-snly[v]) - kp * (-snly[p]);
            fy += kv * snlx[v] - kp * snlx[p];
            const int pp = (p == 0) ? n - 1 : p - 1;
            const float sp = slen[p] / (slen[pp] + slen[p]);
            const float sm = slen[v] / (slen[v] + slen[m]);
            fx += -sbend[v] * snvx[v] + sbend[p] * sp * snvx[p] + sbend[m] * sm * snvx[m];
            fy += -sbend[v] * snvy[v] + sbend[p] * sp * snvy[p] + sbend[m] * sm * snvy[m];
            fx += 0.5f * cA * (slen[p] * snlx[p] + slen[v] * snlx[v]);
            fy += 0.5f * cA * (slen[p] * snly[p] + slen[v] * snly[v]);
        }
        // ligand-receptor springs along the host element's outward normal
        fx += 0.5f * (sbond[p] * snlx[p] + sbond[v] * snlx[v]);
        fy += 0.5f * (sbond[p] * snly[p] + sbond[v] * snly[v]);
        // pressure and viscous loads of the two adjacent elements
        const float4 qp = d.probe4[v0 + p], qv = d.probe4[v0 + v];
        fx += 0.5f * slen[p] * ((qp.y - qp.x) * snlx[p] + qp.z * snly[p]) +
              0.5f * slen[v] * ((qv.y - qv.x) * snlx[v] + qv.z * snly[v]);
        fy += 0.5f * slen[p] * (qp.z * snlx[p] + (qp.w - qp.x) * snly[p]) +
              0.5f * slen[v] * (qv.z * snlx[v] + (qv.w - qv.x) * snly[v]);
        // repulsion from vertices of other bodies closer than the cut-off
        const float myx = sxh[v] + sxl[v], myy = syh[v] + syl[v];
        const float L = (float)d.nx;
        const float cut2 = d.rep_cut * d.rep_cut;
        for (int c = 0; c < d.nbodies; c++) {
            if (c == b) continue;
            const float *bb = d.bs[c].bbox[par];
            float dxc = myx - 0.5f * (bb[0] + bb[1]);
            dxc -= L * rintf(dxc / L);
            if (fabsf(dxc) > 0.5f * (bb[1] - bb[0]) + d.rep_cut + 0.5f) continue;
            if (myy < bb[2] - d.rep_cut - 0.5f || myy > bb[3] + d.rep_cut + 0.5f) continue;
            const int cs = d.bp[c].vstart, cn = d.bp[c].n;
            for (int u = cs; u < cs + cn; u++) {
                float ddx = (sxh[v] - d.pxh[par][u]) + (sxl[v] - d.pxl[par][u]);
                ddx -= L * rintf(ddx / L);
                const float ddy = (syh[v] - d.pyh[par][u]) + (syl[v] - d.pyl[par][u]);
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

    // integration (Eqs. 16-20), direct forcing and spreading at x^n
    float nxh[VPT], nxl[VPT], nyh[VPT], nyl[VPT];
    if (P.kind == RIGID) {
        const float phin = d.bs[b].phih + d.bs[b].phil;
        const float shalf = sinf(0.5f * phin);
        const float c1 = -2.0f * shalf * shalf, sphi = sinf(phin);
        float Fx = 0.0f, Fy = 0.0f, M = 0.0f;
#pragma unroll
        for (int k = 0; k < VPT; k++) {
            const int v = tid + k * BODY_THREADS;
            if (v >= n) continue;
            const float rx = d.r0x[v0 + v], ry = d.r0y[v0 + v];
            const float armx = rx + (c1 * rx - sphi * ry), army = ry + (sphi * rx + c1 * ry);
            Fx += fvx[k];
            Fy += fvy[k];
            M += armx * fvy[k] - army * fvx[k];
        }
        Fx = block_sum(Fx, shf);
        Fy = block_sum(Fy, shf);
        M = block_sum(M, shf);
        if (tid == 0) {
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
            const int v = tid + k * BODY_THREADS;
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
            const float2 us = d.ustar[v0 + v];
            const int p = (v == 0) ? n - 1 : v - 1;
            const float dV = 0.5f * (slen[p] + slen[v]);
            spread(d, sxh[v], sxl[v], syh[v], syl[v], dV * (Ux - us.x), dV * (Uy - us.y), tag);
        }
    } else {
        bool bad = false;
#pragma unroll
        for (int k = 0; k < VPT; k++) {
            const int v = tid + k * BODY_THREADS;
            if (v >= n) continue;
            const float2 us = d.ustar[v0 + v];
            float Ux = 0.0f, Uy = 0.0f;
            nxh[k] = sxh[v]; nxl[k] = sxl[v]; nyh[k] = syh[v]; nyl[k] = syl[v];
            if (P.kind == DEFORMABLE) {
                const float dx = us.x + 0.5f * fvx[k] / P.vmass;
                const float dy = us.y + 0.5f * fvy[k] / P.vmass;
                Ux = 1.5f * dx - 0.5f * d.dxm[v0 + v];
                Uy = 1.5f * dy - 0.5f * d.dym[v0 + v];
                d.dxm[v0 + v] = dx;
                d.dym[v0 + v] = dy;
                df_add(nxh[k], nxl[k], dx);
                df_add(nyh[k], nyl[k], dy);
                bad |= !isfinite(dx) || !isfinite(dy);
            }
            d.target[v0 + v] = make_float2(Ux, Uy);
            const int p = (v == 0) ? n - 1 : v - 1;
            const float dV = 0.5f * (slen[p] + slen[v]);
            spread(d, sxh[v], sxl[v], syh[v], syl[v], dV * (Ux - us.x), dV * (Uy - us.y), tag);
        }
        if (bad) atomicOr(d.err, FLAG_NONFINITE_IB);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BODY_THREADS;
        if (v >= n) continue;
        sxh[v] = nxh[k]; sxl[v] = nxl[k]; syh[v] = nyh[k]; syl[v] = nyl[k];
        d.pxh[npar][v0 + v] = nxh[k];
        d.pxl[npar][v0 + v] = nxl[k];
        d.pyh[npar][v0 + v] = nyh[k];
        d.pyl[npar][v0 + v] = nyl[k];
    }
    __syncthreads();

    // bond kinetics at x^{n+1}
    int cnt = 0;
    for (int s = P.site_start + tid; s < P.site_start + P.n_sites; s += BODY_THREADS) {
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
    cnt = block_sum(cnt, shi);

    // bounding box of x^{n+1} for next step's repulsion culling
    float xmin = 3.0e38f, xmax = -3.0e38f, ymin = 3.0e38f, ymax = -3.0e38f;
    for (int v = tid; v < n; v += BODY_THREADS) {
        const float x = sxh[v] + sxl[v], y = syh[v] + syl[v];
        xmin = fminf(xmin, x); xmax = fmaxf(xmax, x);
        ymin = fminf(ymin, y); ymax = fmaxf(ymax, y);
    }
    xmin = block_ext<false>(xmin, shf);
    xmax = block_ext<true>(xmax, shf);
    ymin = block_ext<false>(ymin, shf);
    ymax = block_ext<true>(ymax, shf);
    if (tid == 0) {
        BodyState &S = d.bs[b];
        S.n_bound = cnt;
        S.bbox[npar][0] = xmin; S.bbox[npar][1] = xmax;
        S.bbox[npar][2] = ymin; S.bbox[npar][3] = ymax;
    }
}

// FP64 geometry of the current polygon of each body (diagnostics).
__global__ __launch_bounds__(BODY_THREADS) void k_body_geom(Dev d, int par) {
    __shared__ double shd[4];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int n = d.bp[b].n, v0 = d.bp[b].vstart;
    auto X = [&](int v) { return (double)d.pxh[par][v0 + v] + (double)d.pxl[par][v0 + v]; };
    auto Y = [&](int v) { return (double)d.pyh[par][v0 + v] + (double)d.pyl[par][v0 + v]; };
    const double x0 = X(0), y0 = Y(0);
    double a = 0, p = 0, sx = 0, sy = 0;
    for (int l = tid; l < n; l += BODY_THREADS) {
        const int m = (l + 1 == n) ? 0 : l + 1;
        const double xa = X(l) - x0, ya = Y(l) - y0, xb = X(m) - x0, yb = Y(m) - y0;
        const double c = xa * yb - xb * ya;
        a += c;
        sx += (xa + xb) * c;
        sy += (ya + yb) * c;
        p += sqrt((xb - xa) * (xb - xa) + (yb - ya) * (yb - ya));
    }
    a = block_sum(a, shd);
    p = block_sum(p, shd);
    sx = block_sum(sx, shd);
    sy = block_sum(sy, shd);
    if (tid == 0) {
        d.bs[b].geo[0] = 0.5 * a;
        d.bs[b].geo[1] = p;
        d.bs[b].geo[2] = x0 + sx / (3.0 * a);
        d.bs[b].geo[3] = y0 + sy / (3.0 * a);
    }
}

// ---- host launchers --------------------------------------------------------------------------------

hipError_t launch_interp(const Dev &d, int par, hipStream_t st) {
    const int pts = 2 * d.nverts;
    int nb = (pts * 16 + INTERP_THREADS - 1) / INTERP_THREADS;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_interp, dim3(nb), dim3(INTERP_THREADS), 0, st, d, par);
    return hipGetLastError();
}

hipError_t launch_body(const Dev &d, int par, hipStream_t st) {
    if (d.nbodies == 0) return hipSuccess;
    hipLaunchKernelGGL(k_body, dim3(d.nbodies), dim3(BODY_THREADS), 0, st, d, par);
    return hipGetLastError();
}

hipError_t launch_body_geom(const Dev &d, int par, hipStream_t st) {
    if (d.nbodies == 0) return hipSuccess;
    hipLaunchKernelGGL(k_body_geom, dim3(d.nbodies), dim3(BODY_THREADS), 0, st, d, par);
    return hipGetLastError();
}

}  // namespace capib
