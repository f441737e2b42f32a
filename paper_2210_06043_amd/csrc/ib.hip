// Immersed-boundary phase of the LBM-IB step.
//
// k_interp: cosine-delta interpolation (Sec. 2.2) of the pre-coupling fluid
//   velocity u* = (sum h e + g/2)/rho to every membrane vertex, and of the
//   pressure c_s^2 drho and viscous stress -(1 - 1/2tau) Pi_neq to the probe
//   of every element, 1.2 dx along its outward normal (Sec. 2.6).  Sixteen
//   lanes serve one point, one stencil node each, and reduce with DPP moves.
// k_body_geom: FP64 geometry of each membrane for the diagnostics.
// (The per-membrane phase of the step is in body.hip.)
#include "capib_dev.hpp"
#include "capib_kernels.hpp"

namespace capib {

constexpr int GEOM_THREADS = 256;

// Fixed-order sum over a 256-thread workgroup (4 waves).
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *sh) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// ---- interpolation ----------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void node_moments(const Dev &d, const T *A, int i, int j, const Band &B, bool stress,
                                             float out[4]) {
    float h[9];
    const float uref = pull_dev<T>(d, A, i, j, B, h);   // deviations from the row reference
    const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const float jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
    const float jy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);
    const float rho = 1.0f + drho;
    const float dux = (jx + 0.5f * d.gx - drho * uref) / rho;
    const float duy = (jy + 0.5f * d.gy) / rho;
    if (!stress) {
        out[0] = uref + dux;
        out[1] = duy;
        out[2] = 0.0f;
        out[3] = 0.0f;
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

template <int PAR, bool ENS>
__device__ __forceinline__ void interp_point(const Dev &d, int gid) {
    const int p = gid >> 4, lane = gid & 15;
    if (p >= 2 * d.nverts) return;    // whole groups of 16 leave together
    const bool probe = p >= d.nverts;
    const int v = probe ? p - d.nverts : p;
    // the loads that need only v, issued together
    const int info = d.vinfo[v];
    float xh, xl, yh, yl;
    if (probe) {
        const float4 q = d.pprobe[PAR][v];
        xh = q.x; xl = q.y; yh = q.z; yl = q.w;
    } else {
        xh = d.pxh[PAR][v]; xl = d.pxl[PAR][v]; yh = d.pyh[PAR][v]; yl = d.pyl[PAR][v];
    }
    const Band B = band_at<ENS>(d, info >> 1);
    int ix0, iy0;
    float wx[4], wy[4], inv;
    const bool out = stencil(d, B, xh, xl, yh, yl, probe, ix0, iy0, wx, wy, inv);
    if (out && !probe && lane == 0) atomicOr(d.err, FLAG_VERTEX_OUT);
    const int a = lane & 3, bb = lane >> 2;
    // lane-dependent picks as selects (an indexed register array would spill)
    const float wxa = a == 0 ? wx[0] : a == 1 ? wx[1] : a == 2 ? wx[2] : wx[3];
    const float wyb = bb == 0 ? wy[0] : bb == 1 ? wy[1] : bb == 2 ? wy[2] : wy[3];
    const float W = wxa * wyb * inv;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int j = iy0 + bb;   // band-local row
    if (!d.walls) j = wrapi(j, B.ny);
    if (W != 0.0f && j >= 0 && j < B.ny) {
        const int i = wrapi(ix0 + a, B.nx);
        float m[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (d.storage == 0)
            node_moments<float>(d, (const float *)d.pop[PAR], i, B.y0 + j, B, probe, m);
        else
            node_moments<_Float16>(d, (const _Float16 *)d.pop[PAR], i, B.y0 + j, B, probe, m);
        acc[0] = W * m[0];
        acc[1] = W * m[1];
        if (probe) {
            acc[2] = W * m[2];
            acc[3] = W * m[3];
        }
    }
#pragma unroll
    for (int c = 0; c < 4; c++) acc[c] = row16_reduce(acc[c], OpAdd());
    if (lane == 0) {
        if (probe)
            d.probe4[v] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        else
            d.ustar[v] = make_float2(acc[0], acc[1]);
    }
}

// The interpolation, and the clearing of the flags and vertex ranges of the
// previous step's near tiles (parity PAR ^ 1), whose sweep has used them,
// before this step's sweep marks that parity again.  That list holds at
// most 9 tiles per vertex, fewer than the 32 threads per vertex of this
// grid, so one entry per thread covers it; its entries are loaded with the
// interpolation's first loads.
template <int PAR, bool ENS>
__global__ __launch_bounds__(INTERP_THREADS) void k_interp(Dev d) {
    const int gid = blockIdx.x * INTERP_THREADS + threadIdx.x;
    const int cnt = d.ncount[PAR ^ 1];
    const int prev = gid < d.ntx * d.nty ? d.nlist[PAR ^ 1][gid] : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *d.counter += 1;   // steps started
    interp_point<PAR, ENS>(d, gid);
    if (gid < cnt) {
        d.tnear[PAR ^ 1][prev] = 0;
        ((int4 *)d.tv[PAR ^ 1])[prev] = make_int4(0, 0, 0, 0);
    }
}

// ---- per-member sample for the surrogate -----------------------------------------------

// One workgroup per band (ensemble member): for its particle (first body
// with tag ptag) and its cells (bodies with tag ctag), at the current state
// (positions x^{n+1} of parity par; the last step's probe values belong to
// x^n, parity par ^ 1), out[8 k ..] = drag, lift (the hydrodynamic load of
// Eqs. 14-15 summed over the particle's elements), hazard (mean Bell
// rupture probability of the engaged bonds, Sec. 2.5), r (distance from the
// particle's vertex mean to the nearest cell's, periodic in x), dp (that
// cell's perimeter over its initial perimeter, minus one), the cell's body
// id (-1: none), the wall shear rate du_x/dy = u_x(row 0) / (1/2) two nodes
// upstream of the particle's leftmost vertex, and N_L.
template <typename T>
__global__ __launch_bounds__(GEOM_THREADS) void k_sample(Dev d, int par, int ptag, int ctag, float *out) {
    __shared__ double shd[GEOM_THREADS / 64];
    const int k = blockIdx.x, tid = threadIdx.x;
    const Band B = band_of(d, k);
    const int2 bb = d.band_bodies[k];
    float *o = out + 8 * (long long)k;
    int part = -1;
    for (int b = bb.x; b < bb.x + bb.y; b++)
        if (d.bp[b].tag == ptag) { part = b; break; }
    if (part < 0) {
        if (tid < 8) o[tid] = tid == 5 ? -1.0f : 0.0f;
        return;
    }
    const BodyParams P = d.bp[part];
    const int n = P.n, v0 = P.vstart, pp = par ^ 1;
    double sx = 0.0, sy = 0.0, fx = 0.0, fy = 0.0;
    for (int l = tid; l < n; l += GEOM_THREADS) {
        sx += (double)d.pxh[par][v0 + l] + (double)d.pxl[par][v0 + l];
        sy += (double)d.pyh[par][v0 + l] + (double)d.pyl[par][v0 + l];
        const int m = (l + 1 == n) ? 0 : l + 1;
        const float tx = (d.pxh[pp][v0 + m] - d.pxh[pp][v0 + l]) + (d.pxl[pp][v0 + m] - d.pxl[pp][v0 + l]);
        const float ty = (d.pyh[pp][v0 + m] - d.pyh[pp][v0 + l]) + (d.pyl[pp][v0 + m] - d.pyl[pp][v0 + l]);
        const float len = sqrtf(tx * tx + ty * ty);
        const float nx = ty / len, ny = -tx / len;
        const float4 q = d.probe4[v0 + l];
        fx += (double)(((q.y - q.x) * nx + q.z * ny) * len);
        fy += (double)((q.z * nx + (q.w - q.x) * ny) * len);
    }
    sx = block_sum(sx, shd);
    sy = block_sum(sy, shd);
    fx = block_sum(fx, shd);
    fy = block_sum(fy, shd);
    const double cx = sx / n, cy = sy / n;
    double hz = 0.0, nl = 0.0;
    for (int q = tid; q < P.n_sites; q += GEOM_THREADS) {
        const int s = P.site_start + q;
        if (!d.s_state[s]) continue;
        const int e = d.s_host[s] - v0;
        const int m = (e + 1 == n) ? 0 : e + 1;
        const float f = (float)d.s_frac[s];
        const float xh = d.pxh[par][v0 + e], xl = d.pxl[par][v0 + e] + f * ((d.pxh[par][v0 + m] - xh) +
                                                                          (d.pxl[par][v0 + m] - d.pxl[par][v0 + e]));
        const float yh = d.pyh[par][v0 + e], yl = d.pyl[par][v0 + e] + f * ((d.pyh[par][v0 + m] - yh) +
                                                                          (d.pyl[par][v0 + m] - d.pyl[par][v0 + e]));
        const float dx = (xh - d.s_anh[s]) + (xl - d.s_anl[s]);
        const float dy = (yh + 0.5f) + yl;
        const float len = sqrtf(dx * dx + dy * dy);
        hz += (double)(-expm1f(-P.kr0 * expf(fabsf(len - P.yeq) / P.lb)));
        nl += 1.0;
    }
    hz = block_sum(hz, shd);
    nl = block_sum(nl, shd);
    double best = 1.0e300, bdp = 0.0;
    int bi = -1;
    for (int c = bb.x; c < bb.x + bb.y; c++) {
        const BodyParams C = d.bp[c];
        if (C.tag != ctag || c == part) continue;
        double ax = 0.0, ay = 0.0, per = 0.0;
        for (int l = tid; l < C.n; l += GEOM_THREADS) {
            const int g = C.vstart + l, gm = C.vstart + ((l + 1 == C.n) ? 0 : l + 1);
            ax += (double)d.pxh[par][g] + (double)d.pxl[par][g];
            ay += (double)d.pyh[par][g] + (double)d.pyl[par][g];
            const double tx = ((double)d.pxh[par][gm] - d.pxh[par][g]) + ((double)d.pxl[par][gm] - d.pxl[par][g]);
            const double ty = ((double)d.pyh[par][gm] - d.pyh[par][g]) + ((double)d.pyl[par][gm] - d.pyl[par][g]);
            per += sqrt(tx * tx + ty * ty);
        }
        ax = block_sum(ax, shd);
        ay = block_sum(ay, shd);
        per = block_sum(per, shd);
        double dx = ax / C.n - cx;
        dx -= B.nx * rint(dx / B.nx);
        const double dy = ay / C.n - cy;
        const double dist = sqrt(dx * dx + dy * dy);
        if (dist < best) {
            best = dist;
            bi = c;
            bdp = per / (double)C.P0 - 1.0;
        }
    }
    if (tid == 0) {
        float shear = 0.0f;
        if (d.walls) {
            const int i = wrapi((int)floorf(d.bs[part].bbox[par][0]) - 2, B.nx);
            float h[9];
            const float uref = pull_dev<T>(d, (const T *)d.pop[par], i, B.y0, B, h);
            const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
            const float jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
            const float ux = uref + (jx + 0.5f * d.gx - drho * uref) / (1.0f + drho);
            shear = 2.0f * ux;
        }
        o[0] = (float)fx;
        o[1] = (float)fy;
        o[2] = nl > 0.0 ? (float)(hz / nl) : 0.0f;
        o[3] = bi >= 0 ? (float)best : 0.0f;
        o[4] = (float)bdp;
        o[5] = (float)bi;
        o[6] = shear;
        o[7] = (float)nl;
    }
}

hipError_t launch_sample(const Dev &d, int par, int ptag, int ctag, float *out, hipStream_t st) {
    if (d.storage == 0)
        hipLaunchKernelGGL(k_sample<float>, dim3(d.nbands), dim3(GEOM_THREADS), 0, st, d, par, ptag, ctag, out);
    else
        hipLaunchKernelGGL(k_sample<_Float16>, dim3(d.nbands), dim3(GEOM_THREADS), 0, st, d, par, ptag, ctag, out);
    return hipGetLastError();
}

// FP64 geometry of the current polygon of each body (diagnostics).
__global__ __launch_bounds__(GEOM_THREADS) void k_body_geom(Dev d, int par) {
    __shared__ double shd[4];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int n = d.bp[b].n, v0 = d.bp[b].vstart;
    auto X = [&](int v) { return (double)d.pxh[par][v0 + v] + (double)d.pxl[par][v0 + v]; };
    auto Y = [&](int v) { return (double)d.pyh[par][v0 + v] + (double)d.pyl[par][v0 + v]; };
    const double x0 = X(0), y0 = Y(0);
    double a = 0, p = 0, sx = 0, sy = 0;
    for (int l = tid; l < n; l += GEOM_THREADS) {
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

hipError_t launch_interp(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const int pts = 2 * d.nverts;
    int nb = (pts * 16 + INTERP_THREADS - 1) / INTERP_THREADS;
    if (nb < 1) nb = 1;
    const bool ens = d.nbands > 1;
    // instantiated per step parity and kind of lattice (no dependent loads
    // for the parity-indexed pointers and the band)
    if (par)
        hipExtLaunchKernelGGL(ens ? k_interp<1, true> : k_interp<1, false>, dim3(nb), dim3(INTERP_THREADS), 0, st,
                              e0, e1, 0, d);
    else
        hipExtLaunchKernelGGL(ens ? k_interp<0, true> : k_interp<0, false>, dim3(nb), dim3(INTERP_THREADS), 0, st,
                              e0, e1, 0, d);
    return hipGetLastError();
}

hipError_t launch_body_geom(const Dev &d, int par, hipStream_t st) {
    if (d.nbodies == 0) return hipSuccess;
    hipLaunchKernelGGL(k_body_geom, dim3(d.nbodies), dim3(GEOM_THREADS), 0, st, d, par);
    return hipGetLastError();
}

}  // namespace capib
