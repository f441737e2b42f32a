// Lattice sweep of the LBM-IB step: pull streaming with halfway bounce-back
// walls (Eq. 1; no-slip capillary walls of Sec. 3.1), moments (Sec. 2.1,
// Eqs. 5-6), the Hermite equilibrium (Eq. 2) and the BGK collision with the
// Guo forcing term (Eq. 4) for the total force g + f_ib, fused in one pass
// that reads 9 and writes 9 populations per node (the per-node code is in
// lattice_dev.hpp).
#include "capib_dev.hpp"
#include "capib_kernels.hpp"
#include "lattice_dev.hpp"

namespace capib {

// A far tile's inputs, loaded ahead of its collision.
template <typename T>
struct FarIn {
    int i, j;
    bool go;          // a far tile and a fluid node
    RowRefOf<T> rr;   // the row's constants
    float h[9];       // pulled stored values
};

template <typename T, int PAR, bool ENS>
__device__ __forceinline__ void far_load(const Dev &d, int c, FarIn<T> &f) {
    const int tile = ENS ? d.live[c] : c;
    const int flag = d.tnear[PAR][tile];
    tile_node(d, tile, f.i, f.j);
    const Band B = band_at_row<ENS>(d, f.j < d.ny ? f.j : 0);
    f.go = !flag && f.j < d.ny && f.i < B.nx;
    load_rowref(d, f.j < d.ny ? f.j - B.y0 : 0, f.rr);   // wave-uniform, before any store
    if (f.go) pull9<T>(d, (const T *)d.pop[PAR], f.i, f.j, B, f.h);
}

// Far tiles on a large lattice, concurrently with the immersed-boundary
// phase: two consecutive candidates per workgroup (pairs in XCD-contiguous
// order), both tiles' loads in flight together, streaming stores.
template <typename T, int PAR, bool ENS>
__global__ __launch_bounds__(LAT_THREADS) void k_lattice_far(Dev d, int n) {
    const int c0 = 2 * xcd_tile(blockIdx.x, gridDim.x);
    FarIn<T> f0, f1;
    f1.go = false;
    far_load<T, PAR, ENS>(d, c0, f0);
    if (c0 + 1 < n) far_load<T, PAR, ENS>(d, c0 + 1, f1);
    if (f0.go) lattice_collide<T, true>(d, PAR, f0.i, f0.j, f0.rr, f0.h, 0.0f, 0.0f);
    if (f1.go) lattice_collide<T, true>(d, PAR, f1.i, f1.j, f1.rr, f1.h, 0.0f, 0.0f);
}

// Does a 4-wide stencil starting at o (wrapped into [0, n)) meet the range
// [t0, t0 + w) of a periodic axis of length n?
__device__ __forceinline__ bool meets_periodic(int o, int t0, int w, int n) {
    int r = o - t0;
    if (r < 0) r += n;
    return r < w || r + 3 >= n;
}

// The lattice sweep after the membrane kernel, one launch in three parts.
// The first nmark workgroups mark the near tiles of the next step: the
// tiles under the stencils of x^{n+1}, which the membrane kernel has
// written, with one range update and flag exchange per distinct tile of a
// wave (see mark_next).  The next nlb workgroups sweep this step's near tiles from the list that the
// previous step's marking built (grid-stride, one workgroup per tile while
// there are enough).  On a lattice of fewer than SPLIT_MIN_TILES tiles the
// last part is the far tiles that the membrane launch (k_body_far) left
// (all but the first pct percent of each XCD's run of candidates), one
// workgroup each on the run's own XCD, dispatched after the near
// tiles so that their longer latency chains start first: there, far tiles
// in the membrane launch and in this sweep cost less than far tiles run
// beside the membrane phase on a second stream, whose cross-stream
// dependencies cost more than the far tiles themselves.  On a larger
// lattice the far tiles are swept beside the membrane phase instead
// (k_lattice_far).
//
// Spreading (Sec. 2.2) is done as a gather: each wave of a near tile's
// workgroup (one tile row) loads the spread records of the tile's vertex
// ranges (64 per pass, one per lane), keeps those whose stencil reaches its
// row, in index order, and every node sums W f over them in that order, so
// the result does not depend on scheduling.  The first records are loaded
// before the node's populations, whose latency then overlaps the gather.
// The flags and ranges of this step's near tiles are cleared by the next
// step's interpolation kernel (the far tiles of this launch read the flags).

// One pass over a wave's (vertex v, tile) pairs, one distinct tile at a
// time: the lowest pending lane leads and alone widens the tile's vertex
// ranges to the highest and lowest covering vertex of each half over the
// lanes with that tile.  Neighbouring vertices share their tiles, so a wave
// makes a few range updates per tile instead of one per pair.  LANEV: the
// vertex of lane l is vb + l, so those bounds are the first and last lane of
// a ballot; otherwise the wave reduces them with shuffles.  Returns whether
// this lane led.
template <int NPAR, bool LANEV>
__device__ __forceinline__ bool mark_pass(const Dev &d, bool pend, int tile, int half, int v, int vb) {
    const int lane = threadIdx.x & 63;
    bool led = false;
    for (unsigned long long m = __ballot(pend); m; m = __ballot(pend)) {
        const int lead = __ffsll((long long)m) - 1;
        const int lt = __shfl(tile, lead);
        const bool same = pend && tile == lt;
        int hi0, lo0, hi1, lo1;
        if (LANEV) {
            const unsigned long long m0 = __ballot(same && half == 0), m1 = __ballot(same && half == 1);
            hi0 = m0 ? vb + 63 - __clzll((long long)m0) : -1;
            lo0 = vb + __ffsll((long long)m0) - 1;
            hi1 = m1 ? vb + 63 - __clzll((long long)m1) : -1;
            lo1 = vb + __ffsll((long long)m1) - 1;
        } else {
            hi0 = (same && half == 0) ? v : -1;
            lo0 = (same && half == 0) ? v : INT_MAX;
            hi1 = (same && half == 1) ? v : -1;
            lo1 = (same && half == 1) ? v : INT_MAX;
#pragma unroll
            for (int sh = 32; sh >= 1; sh >>= 1) {
                hi0 = max(hi0, __shfl_xor(hi0, sh));
                lo0 = min(lo0, __shfl_xor(lo0, sh));
                hi1 = max(hi1, __shfl_xor(hi1, sh));
                lo1 = min(lo1, __shfl_xor(lo1, sh));
            }
        }
        if (lane == lead) {
            int *t = d.tv[NPAR] + 4 * lt;
            if (hi0 >= 0) {
                atomicMax(t + 1, hi0 + 1);
                atomicMax(t, d.nverts - lo0);
            }
            if (hi1 >= 0) {
                atomicMax(t + 3, hi1 + 1);
                atomicMax(t + 2, d.nverts - lo1);
            }
            led = true;
        }
        pend = pend && !same;
    }
    return led;
}

// The leaders' flag exchanges (all in flight together: a returned value kept
// across the loops of mark_pass would hold each iteration until the previous
// one returned), then one list-counter update per workgroup for its fresh
// tiles (the counter is a single address that every marking workgroup
// updates: one update per wave kept it busy for tens of microseconds).
// Called by every thread of the workgroup.
template <int NPAR, int NP>
__device__ __forceinline__ void mark_append(const Dev &d, const bool (&led)[NP], const int (&tl)[NP]) {
    constexpr int NW = LAT_THREADS / 64;
    __shared__ int swave[NW], sbase;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    bool fresh[NP];
#pragma unroll
    for (int r = 0; r < NP; r++) fresh[r] = led[r] && atomicExch(&d.tnear[NPAR][tl[r]], 1) == 0;
    unsigned long long fm[NP];
    int total = 0;
#pragma unroll
    for (int r = 0; r < NP; r++) {
        fm[r] = __ballot(fresh[r]);
        total += __popcll(fm[r]);
    }
    if (lane == 0) swave[wv] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) t += swave[w];
        sbase = t ? atomicAdd(&d.ncount[NPAR], t) : 0;
    }
    __syncthreads();
    if (total) {
        int base = sbase;
#pragma unroll
        for (int w = 0; w < NW; w++) base += w < wv ? swave[w] : 0;
        const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
        for (int r = 0; r < NP; r++) {
            if (fresh[r]) d.nlist[NPAR][base + __popcll(fm[r] & below)] = tl[r];
            base += __popcll(fm[r]);
        }
    }
}

// Marking workgroup mb.  On a small lattice (PAIRS): one (vertex, stencil
// tile) pair per lane, 28 vertices per workgroup, so that the marking's
// chains are short and spread over many workgroups.  On a large one: one
// vertex per lane and a pass per stencil tile, so that far fewer waves
// contend for the list counter.
template <bool PAIRS>
constexpr int mark_verts() { return PAIRS ? LAT_THREADS / 9 : LAT_THREADS; }

template <int NPAR, bool ENS, bool PAIRS>
__device__ __forceinline__ void mark_next(const Dev &d, int mb) {
    constexpr int MV = mark_verts<PAIRS>();
    if constexpr (PAIRS) {
        const int v = mb * MV + (int)threadIdx.x / 9, q = (int)threadIdx.x % 9;
        bool pend = false;
        int tile[1] = {0}, half = 0;
        if ((int)threadIdx.x < MV * 9 && v < d.nverts) {
            int tl[9];
            const int info = d.vinfo[v];
            const Band B = band_at<ENS>(d, info >> 1);
            const int c = stencil_tiles(d, B, d.pxh[NPAR][v], d.pxl[NPAR][v], d.pyh[NPAR][v], d.pyl[NPAR][v], tl);
#pragma unroll
            for (int r = 0; r < 9; r++)
                if (r == q) tile[0] = tl[r];
            pend = q < c;
            half = info & 1;
        }
        const bool led[1] = {mark_pass<NPAR, false>(d, pend, tile[0], half, v, 0)};
        mark_append<NPAR>(d, led, tile);
    } else {
        const int v = mb * MV + (int)threadIdx.x;
        int tl[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, c = 0, half = 0;
        if (v < d.nverts) {
            const int info = d.vinfo[v];
            const Band B = band_at<ENS>(d, info >> 1);
            c = stencil_tiles(d, B, d.pxh[NPAR][v], d.pxl[NPAR][v], d.pyh[NPAR][v], d.pyl[NPAR][v], tl);
            half = info & 1;
        }
        const int vb = mb * MV + ((int)threadIdx.x & ~63);   // vertex of the wave's lane 0
        bool led[9];
#pragma unroll
        for (int r = 0; r < 9; r++) led[r] = mark_pass<NPAR, true>(d, r < c, tl[r], half, v, vb);
        mark_append<NPAR>(d, led, tl);
    }
}

// The spread record of the candidate at position u of a tile's vertex
// ranges, as stored by the membrane kernel (zero past the end).
struct Cand {
    int2 o;
    float4 wx, wy;
    float2 f;
};

__device__ __forceinline__ Cand load_cand(const Dev &d, int u, int nv, int lo0, int n0, int lo1) {
    Cand c;
    c.o = make_int2(0, -(1 << 30));
    c.wx = c.wy = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    c.f = make_float2(0.0f, 0.0f);
    if (u < nv) {
        const int v = u < n0 ? lo0 + u : lo1 + (u - n0);
        c.o = d.sp_org[v];
        c.wx = d.sp_wx[v];
        c.wy = d.sp_wy[v];
        c.f = d.sp_f[v];
    }
    return c;
}

// One near tile from its expanded list entry e0, e1: the tile, its band's
// width and its covering vertices as candidate positions u in [0, n0 + n1)
// (u < n0: vertex lo0 + u, else lo1 + u - n0).  Each wave holds one row of
// the tile and gathers the spread force of its nodes by itself, with no
// barrier: its lanes load 64 candidates at a time, the candidates whose
// stencil reaches the row (and the tile's columns) go to the wave's own LDS
// rows in candidate order, with the y weight of the row already chosen, and
// every lane then reads each record in turn (broadcast); a node adds
// w_x w_y f of the vertices whose stencil holds it, in candidate order.
template <typename T, int PAR, bool NT>
__device__ __forceinline__ void near_tile(const Dev &d, const int4 e0, const int4 e1) {
    const int tile = e0.x, lo0 = e0.z, n0 = e0.w, lo1 = e1.x, nv = n0 + e1.y;
    const int tyi = tile / d.ntx, txi = tile - tyi * d.ntx;
    const int x0 = txi * TILE_X, y0 = tyi * TILE_Y;
    const Band B{e0.y, y0 - y0 % d.band_rows, d.band_rows};   // tiles never straddle bands
    const int lane = threadIdx.x & 63;
    const int tw = min(TILE_X, B.nx - x0);
    int i, j;
    tile_node(d, tile, i, j);
    if (j >= B.y0 + B.ny) return;   // the whole wave lies beyond the band
    const bool valid = i < B.nx;
    // the first candidates' loads go out before the pulls: the gather then
    // waits for them alone
    Cand c = load_cand(d, lane, nv, lo0, n0, lo1);
    float h[9];
    if (valid) pull9<T>(d, (const T *)d.pop[PAR], i, j, B, h);
    // each wave's own records: (origin x, w_y of its row, fx, fy) and w_x
    __shared__ float4 srec[LAT_THREADS / 64][66][2];
    float4(*R)[2] = srec[threadIdx.x >> 6];
    float ax = 0.0f, ay = 0.0f;
    for (int c0 = 0; c0 < nv; c0 += 64) {
        if (c0 > 0) c = load_cand(d, c0 + lane, nv, lo0, n0, lo1);
        int e = j - c.o.y;
        if (!d.walls && e < 0) e += B.ny;
        const bool t = c0 + lane < nv && (unsigned)e < 4u && meets_periodic(c.o.x, x0, tw, B.nx);
        const float we = e == 0 ? c.wy.x : e == 1 ? c.wy.y : e == 2 ? c.wy.z : c.wy.w;
        const float4 r0 = make_float4(__int_as_float(c.o.x), we, c.f.x, c.f.y), r1 = c.wx;
        const unsigned long long m = __ballot(t);
        const int nt = __popcll(m);
        if (t) {
            const int k = __popcll(m & ((1ull << lane) - 1ull));   // keeps candidate order
            R[k][0] = r0;
            R[k][1] = r1;
        }
        // pad to an even count with a record that reaches no node
        if (lane < (nt & 1)) {
            R[nt + lane][0] = make_float4(__int_as_float(-(1 << 30)), 0.0f, 0.0f, 0.0f);
            R[nt + lane][1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int k0 = 0; k0 < nt; k0 += 2)
#pragma unroll
        for (int k = k0; k < k0 + 2; k++) {
            const float4 q0 = R[k][0], q1 = R[k][1];   // broadcast reads
            int a = i - __float_as_int(q0.x);
            if (a < 0) a += B.nx;
            // w = 0 off the stencil; adding 0 f leaves a sum as it is (the
            // sums start at +0, so they are never -0): no branch
            const float wl = (a & 1) ? q1.y : q1.x, wh = (a & 1) ? q1.w : q1.z;
            const float w = (unsigned)a < 4u ? ((a & 2) ? wh : wl) * q0.y : 0.0f;
            ax += w * q0.z;
            ay += w * q0.w;
        }
        __builtin_amdgcn_wave_barrier();   // the next batch overwrites the records
    }
    if (valid) {
        RowRefOf<T> rr;
        load_rowref(d, j - B.y0, rr);
        lattice_collide<T, NT>(d, PAR, i, j, rr, h, ax, ay);
    }
}

template <typename T, int PAR, bool ENS, bool FULL, bool PAIRS>
__global__ __launch_bounds__(LAT_THREADS) void k_lattice_sweep(Dev d, int nmark, int nlb, int pct) {
    if ((int)blockIdx.x < nmark) {
        mark_next<PAR ^ 1, ENS, PAIRS>(d, blockIdx.x);
        return;
    }
    const int bid = blockIdx.x - nmark;
    if (bid < nlb) {
        // near tiles, grid-stride over the expanded list; the first entry is
        // loaded with the count (nlb does not exceed the list's capacity)
        const int4 *E = d.elist[PAR];
        int4 e0 = E[2 * bid], e1 = E[2 * bid + 1];
        const int cnt = d.ncount[PAR];
        for (int k = bid; k < cnt; k += nlb) {
            if (k != bid) {
                e0 = E[2 * k];
                e1 = E[2 * k + 1];
            }
            near_tile<T, PAR, !FULL>(d, e0, e1);   // streaming stores on a large lattice
        }
        return;
    }
    if (FULL) {
        // from the first multiple of 8 at or after block nmark + nlb: the
        // candidates of each XCD's run that the membrane launch left, on the
        // run's own XCD (the few blocks before it have nothing to do)
        const int g0 = round_up8(nmark + nlb);
        if ((int)blockIdx.x < g0) return;
        const int ncand = ENS ? d.nlive : d.ntx * d.nty;
        const XcdRun run = xcd_run(blockIdx.x & 7, ncand);
        const int c = far_share_len(run.len, pct) + (((int)blockIdx.x - g0) >> 3);
        if (c < run.len) far_tile<T, PAR, ENS>(d, run.start + c);
    }
}

// Moments of the current state for read-out: drho and u* = (j + g/2)/rho
// ([3][ny][nx]; zero beyond the width of a band).
template <typename T>
__global__ __launch_bounds__(LAT_THREADS) void k_macro(Dev d, int par) {
    const T *__restrict__ A = (const T *)d.pop[par];
    const int i = blockIdx.x * TILE_X + (threadIdx.x & (TILE_X - 1));
    const int j = blockIdx.y * TILE_Y + (threadIdx.x / TILE_X);
    if (i >= d.nx || j >= d.ny) return;
    const long long N = (long long)d.nx * d.ny, k = (long long)j * d.nx + i;
    const Band B = band_of_row(d, j);
    if (i >= B.nx) {
        d.macro[k] = 0.0f;
        d.macro[N + k] = 0.0f;
        d.macro[2 * N + k] = 0.0f;
        return;
    }
    float h[9];
    const float uref = pull_dev<T>(d, A, i, j, B, h);
    const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const float jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
    const float jy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);
    const float irho = 1.0f / (1.0f + drho);
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
    if (i < d.nx && j < d.ny && i < band_of_row(d, j).nx) {
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

// The step kernels are instantiated per step parity and per kind of
// lattice (one band or several), so that their parity-indexed pointers and
// the band geometry need no dependent loads.
template <typename T, int P, bool E>
static void go_far(const Dev &d, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const int n = E ? d.nlive : d.ntx * d.nty;
    hipExtLaunchKernelGGL((k_lattice_far<T, P, E>), dim3((n + 1) / 2), dim3(LAT_THREADS), 0, st, e0, e1, 0, d, n);
}
template <typename T>
static void far_of(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const bool ens = d.nbands > 1;
    if (par) ens ? go_far<T, 1, true>(d, st, e0, e1) : go_far<T, 1, false>(d, st, e0, e1);
    else ens ? go_far<T, 0, true>(d, st, e0, e1) : go_far<T, 0, false>(d, st, e0, e1);
}

hipError_t launch_lattice_far(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (d.storage == 0)
        far_of<float>(d, par, st, e0, e1);
    else
        far_of<_Float16>(d, par, st, e0, e1);
    return hipGetLastError();
}

// Grid of the sweep: the marking workgroups; about one workgroup per near
// tile, which number a fraction of the vertices (the list's grid-stride
// loop covers any count); on a small lattice one workgroup per far-tile
// candidate.
constexpr int SPLIT_MIN_TILES = 8192;

bool default_split(int tiles) { return tiles >= SPLIT_MIN_TILES; }
bool lattice_split(const Dev &d) { return d.split != 0; }

// marking layout: pairs per lane below this many vertices (see mark_next)
constexpr int PAIRS_MAX_VERTS = 16384;

bool default_mark_pairs(int nverts) { return nverts < PAIRS_MAX_VERTS; }

template <typename T, int P, bool E, bool PA>
static void go_sweep(const Dev &d, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int pct) {
    constexpr int mv = mark_verts<PA>();
    const int nmark = (d.nverts + mv - 1) / mv;
    const int nt = d.ntx * d.nty;
    const int want = d.nverts / 8 > 1024 ? d.nverts / 8 : 1024;
    const int nlb = nt < want ? nt : want;
    if (!lattice_split(d)) {
        // the far workgroups start at the first multiple of 8 after the near
        // ones; each XCD's run needs at most len - share of them
        const int ncand = E ? d.nlive : nt;
        const int len = xcd_run(0, ncand).len;
        const int most = len - far_share_len(len, pct);
        hipExtLaunchKernelGGL((k_lattice_sweep<T, P, E, true, PA>), dim3(round_up8(nmark + nlb) + 8 * most),
                              dim3(LAT_THREADS), 0, st, e0, e1, 0, d, nmark, nlb, pct);
    } else
        hipExtLaunchKernelGGL((k_lattice_sweep<T, P, E, false, PA>), dim3(nmark + nlb), dim3(LAT_THREADS), 0, st, e0,
                              e1, 0, d, nmark, nlb, 0);
}
template <typename T, int P, bool E>
static void go_sweep(const Dev &d, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int pct) {
    if (d.mark_pairs)
        go_sweep<T, P, E, true>(d, st, e0, e1, pct);
    else
        go_sweep<T, P, E, false>(d, st, e0, e1, pct);
}
template <typename T>
static void sweep_of(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int pct) {
    const bool ens = d.nbands > 1;
    if (par) ens ? go_sweep<T, 1, true>(d, st, e0, e1, pct) : go_sweep<T, 1, false>(d, st, e0, e1, pct);
    else ens ? go_sweep<T, 0, true>(d, st, e0, e1, pct) : go_sweep<T, 0, false>(d, st, e0, e1, pct);
}

hipError_t launch_lattice_sweep(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int pct) {
    if (d.storage == 0)
        sweep_of<float>(d, par, st, e0, e1, pct);
    else
        sweep_of<_Float16>(d, par, st, e0, e1, pct);
    return hipGetLastError();
}

// Nodes swept by the lattice launches of a step, for the timing accounting:
// out[0] += far-tile nodes among the first far_share_len(len, pct)
// candidates of each XCD's run (swept by the membrane launch), out[1] +=
// the other far-tile nodes, out[2] += near-tile nodes.  One thread per
// candidate tile.
template <bool ENS>
__global__ __launch_bounds__(256) void k_census(Dev d, int par, int pct, unsigned long long *out) {
    const int ncand = ENS ? d.nlive : d.ntx * d.nty;
    const int b = blockIdx.x * 256 + threadIdx.x;
    int c[3] = {0, 0, 0};
    if (b < ncand) {
        const int tile = ENS ? d.live[b] : b;
        int x = 7;
        while (x > 0 && xcd_run(x, ncand).start > b) x--;
        const XcdRun run = xcd_run(x, ncand);
        const bool membrane_launch = b - run.start < far_share_len(run.len, pct);
        const int ty = tile / d.ntx, tx = tile - ty * d.ntx;
        const int x0 = tx * TILE_X, y0 = ty * TILE_Y;
        const Band B = band_at_row<ENS>(d, y0);   // a tile lies in one band
        const int n = max(0, min(TILE_X, B.nx - x0)) * max(0, min(TILE_Y, d.ny - y0));
        c[d.tnear[par][tile] ? 2 : membrane_launch ? 0 : 1] = n;
    }
    for (int k = 0; k < 3; k++) {
        const int s = wave_sum(c[k]);
        if ((threadIdx.x & 63) == 0 && s) atomicAdd(out + k, (unsigned long long)s);
    }
}

hipError_t launch_census(const Dev &d, int par, int pct, unsigned long long *out, hipStream_t st) {
    const int ncand = d.nbands > 1 ? d.nlive : d.ntx * d.nty;
    if (d.nbands > 1)
        hipLaunchKernelGGL(k_census<true>, dim3((ncand + 255) / 256), dim3(256), 0, st, d, par, pct, out);
    else
        hipLaunchKernelGGL(k_census<false>, dim3((ncand + 255) / 256), dim3(256), 0, st, d, par, pct, out);
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
