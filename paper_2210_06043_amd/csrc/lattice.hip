// Lattice sweep of the LBM-IB step: pull streaming with halfway bounce-back
// walls (Eq. 1; no-slip capillary walls of Sec. 3.1), moments (Sec. 2.1,
// Eqs. 5-6), the Hermite equilibrium (Eq. 2) and the BGK collision with the
// Guo forcing term (Eq. 4) for the total force g + f_ib, fused in one pass
// that reads 9 and writes 9 populations per node.
//
// Layout: structure of arrays pop[q][j][i], i fastest, row pitch a multiple
// of 64 elements, two buffers swapped every step.  Populations are stored as
// deviations h = f - w from the rest state, FP32 or FP16 (scaled).
#include "capib_dev.hpp"
#include "capib_kernels.hpp"

namespace capib {

template <typename T>
__device__ __forceinline__ T stpop(float v, float scale);
template <>
__device__ __forceinline__ float stpop<float>(float v, float) { return v; }
template <>
__device__ __forceinline__ _Float16 stpop<_Float16>(float v, float scale) { return (_Float16)(v * scale); }

// One node of one 64x4 tile.  FORCED: the tile is a near tile of this step
// and (ax, ay) is the IB force spread onto this node.
template <typename T, bool FORCED>
__device__ __forceinline__ void lattice_node(const Dev &d, int par, int tile, float ax = 0.0f, float ay = 0.0f) {
    const T *__restrict__ A = (const T *)d.pop[par];
    T *__restrict__ B = (T *)d.pop[par ^ 1];
    const int ty = tile / d.ntx;
    const int tx = tile - ty * d.ntx;
    const int i = tx * TILE_X + (threadIdx.x & (TILE_X - 1));
    // one wave per row: the row index (and the row reference) is wave-uniform
    const int j = __builtin_amdgcn_readfirstlane(ty * TILE_Y + (int)(threadIdx.x / TILE_X));
    if (i >= d.nx || j >= d.ny) return;
    float h[9];
    const float uref = pull_dev<T>(d, A, i, j, h);

    // moments of the streamed deviations: drho, and j - u_ref x
    const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const float jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
    const float jy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);

    // total force: uniform drive plus the spread IB force of this step
    float Fx = d.gx, Fy = d.gy;
    const long long node = (long long)j * d.pitch + i;
    if (FORCED) {
        Fx += ax;
        Fy += ay;
    }

    const float rho = 1.0f + drho;
    const float irho = 1.0f / rho;
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
    float out[9];
    {
        const float w = 4.0f / 9.0f;
        out[0] = om1 * h[0] + om * E(0.0f, 0.0f, w) + fc * w * fb;
    }
#define CAPIB_DIR(q, ex, ey, w)                                                              \
    {                                                                                        \
        const float eu = (ex) * ux + (ey) * uy;                                              \
        const float eF = (ex) * Fx + (ey) * Fy;                                              \
        const float Fi = fc * (w) * (fb + 3.0f * eF + 9.0f * eu * eF);                       \
        out[q] = om1 * h[q] + om * E((ex), (ey), (w)) + Fi;                                  \
    }
    CAPIB_DIR(1, 1.0f, 0.0f, 1.0f / 9.0f)
    CAPIB_DIR(2, 0.0f, 1.0f, 1.0f / 9.0f)
    CAPIB_DIR(3, -1.0f, 0.0f, 1.0f / 9.0f)
    CAPIB_DIR(4, 0.0f, -1.0f, 1.0f / 9.0f)
    CAPIB_DIR(5, 1.0f, 1.0f, 1.0f / 36.0f)
    CAPIB_DIR(6, -1.0f, 1.0f, 1.0f / 36.0f)
    CAPIB_DIR(7, -1.0f, -1.0f, 1.0f / 36.0f)
    CAPIB_DIR(8, 1.0f, -1.0f, 1.0f / 36.0f)
#undef CAPIB_DIR
    const long long Q = d.qstride;
#pragma unroll
    for (int q = 0; q < 9; q++) B[q * Q + node] = stpop<T>(out[q], d.scale);
}

// Far tiles: every tile of the lattice except this step's near tiles, in
// XCD-contiguous order.  Runs concurrently with the immersed-boundary phase.
template <typename T>
__global__ __launch_bounds__(LAT_THREADS) void k_lattice_far(Dev d, int par) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (d.tnear[par][tile]) return;
    lattice_node<T, false>(d, par, tile);
}

// Does a 4-wide stencil starting at o (wrapped into [0, n)) meet the range
// [t0, t0 + w) of a periodic axis of length n?
__device__ __forceinline__ bool meets_periodic(int o, int t0, int w, int n) {
    int r = o - t0;
    if (r < 0) r += n;
    return r < w || r + 3 >= n;
}

// Near tiles of this step, after the membrane kernel: grid-stride over the
// list.  Spreading (Sec. 2.2) is done here as a gather: for each tile the
// workgroup scans the membranes whose bounding box (of x^n, widened by the
// stencil reach) meets the tile, 256 vertices at a time, compacts the
// vertices whose stencil covers the tile into LDS in vertex order, and every
// node sums W f over them in that order, so the result does not depend on
// scheduling.  Each tile's flag is cleared for the next step of the same
// parity.
template <typename T>
__global__ __launch_bounds__(LAT_THREADS) void k_lattice_near(Dev d, int par) {
    __shared__ int2 sorg[LAT_THREADS];
    __shared__ float sw[LAT_THREADS][10];   // x weights (normalised), y weights, force
    __shared__ int swave[LAT_THREADS / 64];
    const int cnt = d.ncount[par];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = blockIdx.x; k < cnt; k += gridDim.x) {
        const int tile = d.nlist[par][k];
        const int ty = tile / d.ntx, tx = tile - ty * d.ntx;
        const int x0 = tx * TILE_X, y0 = ty * TILE_Y;
        const int tw = min(TILE_X, d.nx - x0), th = min(TILE_Y, d.ny - y0);
        const int i = x0 + lane, j = y0 + wv;
        float ax = 0.0f, ay = 0.0f;
        for (int b = 0; b < d.nbodies; b++) {
            const float bx0 = d.bs[b].bbox[par][0], bx1 = d.bs[b].bbox[par][1];
            const float by0 = d.bs[b].bbox[par][2], by1 = d.bs[b].bbox[par][3];
            bool meet = true;   // an unusable box (non-finite, huge) meets every tile
            if (fabsf(bx0) < 1.0e8f && fabsf(bx1) < 1.0e8f && bx1 - bx0 < (float)(d.nx - 8)) {
                const int lo = wrapi((int)floorf(bx0) - 3, d.nx);
                const int wd = (int)ceilf(bx1) - (int)floorf(bx0) + 6;
                int r = lo - x0;
                if (r < 0) r += d.nx;
                meet = r < tw || r + wd >= d.nx;
            }
            if (meet && fabsf(by0) < 1.0e8f && fabsf(by1) < 1.0e8f) {
                const int lo = (int)floorf(d.walls ? fminf(fmaxf(by0, -1.0f), (float)d.ny) : by0) - 3;
                const int hi = (int)ceilf(d.walls ? fminf(fmaxf(by1, -1.0f), (float)d.ny) : by1) + 3;
                if (d.walls) {
                    meet = hi >= y0 && lo < y0 + th;
                } else if (hi - lo < d.ny) {
                    int r = wrapi(lo, d.ny) - y0;
                    if (r < 0) r += d.ny;
                    meet = r < th || r + (hi - lo) >= d.ny;
                }
            }
            if (!meet) continue;
            const int vs = d.bp[b].vstart, n = d.bp[b].n;
            for (int c0 = 0; c0 < n; c0 += LAT_THREADS) {
                const int v = c0 + (int)threadIdx.x;
                bool hit = false;
                int2 o = make_int2(0, 0);
                if (v < n) {
                    o = d.sp_org[vs + v];
                    const bool hx = meets_periodic(o.x, x0, tw, d.nx);
                    const bool hy = d.walls ? (o.y + 3 >= y0 && o.y < y0 + th) : meets_periodic(o.y, y0, th, d.ny);
                    hit = hx && hy;
                }
                const unsigned long long m = __ballot(hit);
                if (lane == 0) swave[wv] = __popcll(m);
                __syncthreads();
                int base = 0, tot = 0;
#pragma unroll
                for (int w = 0; w < LAT_THREADS / 64; w++) {
                    base += (w < wv) ? swave[w] : 0;
                    tot += swave[w];
                }
                if (hit) {
                    const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
                    const float4 wx = d.sp_wx[vs + v], wy = d.sp_wy[vs + v];
                    const float2 f = d.sp_f[vs + v];
                    sorg[slot] = o;
                    sw[slot][0] = wx.x; sw[slot][1] = wx.y; sw[slot][2] = wx.z; sw[slot][3] = wx.w;
                    sw[slot][4] = wy.x; sw[slot][5] = wy.y; sw[slot][6] = wy.z; sw[slot][7] = wy.w;
                    sw[slot][8] = f.x; sw[slot][9] = f.y;
                }
                __syncthreads();
                for (int h = 0; h < tot; h++) {
                    int a = i - sorg[h].x;
                    if (a < 0) a += d.nx;
                    int c = j - sorg[h].y;
                    if (!d.walls && c < 0) c += d.ny;
                    if (a < 4 && (unsigned)c < 4u) {
                        const float w = sw[h][a] * sw[h][4 + c];
                        ax += w * sw[h][8];
                        ay += w * sw[h][9];
                    }
                }
                __syncthreads();
            }
        }
        if (threadIdx.x == 0) d.tnear[par][tile] = 0;
        lattice_node<T, true>(d, par, tile, ax, ay);
    }
}

// Moments of the current state for read-out: drho and u* = (j + g/2)/rho.
template <typename T>
__global__ __launch_bounds__(LAT_THREADS) void k_macro(Dev d, int par) {
    const T *__restrict__ A = (const T *)d.pop[par];
    const int i = blockIdx.x * TILE_X + (threadIdx.x & (TILE_X - 1));
    const int j = blockIdx.y * TILE_Y + (threadIdx.x / TILE_X);
    if (i >= d.nx || j >= d.ny) return;
    float h[9];
    const float uref = pull_dev<T>(d, A, i, j, h);
    const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const float jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
    const float jy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);
    const float irho = 1.0f / (1.0f + drho);
    const long long N = (long long)d.nx * d.ny, k = (long long)j * d.nx + i;
    d.macro[k] = drho;
    d.macro[N + k] = uref + (jx + 0.5f * d.gx - drho * uref) * irho;
    d.macro[2 * N + k] = (jy + 0.5f * d.gy) * irho;
}

// Initial state: the equilibrium at drho = 0 and the reference profile,
// i.e. zero deviation everywhere.
template <typename T>
__global__ __launch_bounds__(LAT_THREADS) void k_init_flow(Dev d, int par) {
    T *__restrict__ A = (T *)d.pop[par];
    const int i = blockIdx.x * TILE_X + (threadIdx.x & (TILE_X - 1));
    const int j = blockIdx.y * TILE_Y + (threadIdx.x / TILE_X);
    if (i >= d.nx || j >= d.ny) return;
    const long long node = (long long)j * d.pitch + i;
    for (int q = 0; q < 9; q++) A[q * d.qstride + node] = stpop<T>(0.0f, d.scale);
}

// FP64 partial sums per tile of the stored populations: sum h, sum h e.
template <typename T>
__global__ __launch_bounds__(LAT_THREADS) void k_diag_partial(Dev d, int par) {
    const T *__restrict__ A = (const T *)d.pop[par];
    const int i = blockIdx.x * TILE_X + (threadIdx.x & (TILE_X - 1));
    const int j = blockIdx.y * TILE_Y + (threadIdx.x / TILE_X);
    double m = 0, px = 0, py = 0;
    if (i < d.nx && j < d.ny) {
        const long long node = (long long)j * d.pitch + i;
        double h[9];
        for (int q = 0; q < 9; q++) h[q] = (double)ldpop<T>(A + q * d.qstride + node, d.inv_scale);
        m = h[0] + h[1] + h[2] + h[3] + h[4] + h[5] + h[6] + h[7] + h[8];
        px = h[1] - h[3] + h[5] - h[6] - h[7] + h[8];
        py = h[2] - h[4] + h[5] + h[6] - h[7] - h[8];
    }
    __shared__ double sm[3][LAT_THREADS];
    sm[0][threadIdx.x] = m;
    sm[1][threadIdx.x] = px;
    sm[2][threadIdx.x] = py;
    __syncthreads();
    for (int s = LAT_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 3; c++) sm[c][threadIdx.x] += sm[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
        d.red[3 * blk + threadIdx.x] = sm[threadIdx.x][0];
    }
}

// Fixed-order final sum of the partials into red[3 * nblk .. +2].
__global__ __launch_bounds__(256) void k_diag_final(Dev d, int nblk) {
    __shared__ double sm[3][256];
    double a[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256)
        for (int c = 0; c < 3; c++) a[c] += d.red[3 * b + c];
    for (int c = 0; c < 3; c++) sm[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 3; c++) sm[c][threadIdx.x] += sm[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) d.red[3 * (long long)nblk + threadIdx.x] = sm[threadIdx.x][0];
}

// ---- host launchers ---------------------------------------------------------------

hipError_t launch_lattice_far(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const int nb = d.ntx * d.nty;
    if (d.storage == 0)
        hipExtLaunchKernelGGL(k_lattice_far<float>, dim3(nb), dim3(LAT_THREADS), 0, st, e0, e1, 0, d, par);
    else
        hipExtLaunchKernelGGL(k_lattice_far<_Float16>, dim3(nb), dim3(LAT_THREADS), 0, st, e0, e1, 0, d, par);
    return hipGetLastError();
}

hipError_t launch_lattice_near(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    // enough workgroups for the near tiles of a few thousand vertices; the
    // grid-stride loop covers any count
    const int nt = d.ntx * d.nty;
    const int nb = nt < 1024 ? nt : 1024;
    if (d.storage == 0)
        hipExtLaunchKernelGGL(k_lattice_near<float>, dim3(nb), dim3(LAT_THREADS), 0, st, e0, e1, 0, d, par);
    else
        hipExtLaunchKernelGGL(k_lattice_near<_Float16>, dim3(nb), dim3(LAT_THREADS), 0, st, e0, e1, 0, d, par);
    return hipGetLastError();
}

hipError_t launch_macro(const Dev &d, int par, hipStream_t st) {
    dim3 g(d.ntx, d.nty);
    if (d.storage == 0)
        hipLaunchKernelGGL(k_macro<float>, g, dim3(LAT_THREADS), 0, st, d, par);
    else
        hipLaunchKernelGGL(k_macro<_Float16>, g, dim3(LAT_THREADS), 0, st, d, par);
    return hipGetLastError();
}

hipError_t launch_init_flow(const Dev &d, int par, hipStream_t st) {
    dim3 g(d.ntx, d.nty);
    if (d.storage == 0)
        hipLaunchKernelGGL(k_init_flow<float>, g, dim3(LAT_THREADS), 0, st, d, par);
    else
        hipLaunchKernelGGL(k_init_flow<_Float16>, g, dim3(LAT_THREADS), 0, st, d, par);
    return hipGetLastError();
}

hipError_t launch_diag(const Dev &d, int par, hipStream_t st) {
    dim3 g(d.ntx, d.nty);
    if (d.storage == 0)
        hipLaunchKernelGGL(k_diag_partial<float>, g, dim3(LAT_THREADS), 0, st, d, par);
    else
        hipLaunchKernelGGL(k_diag_partial<_Float16>, g, dim3(LAT_THREADS), 0, st, d, par);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, st, d, d.ntx * d.nty);
    return hipGetLastError();
}

}  // namespace capib
