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
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/capib3d.h"

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
};

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
__device__ __forceinline__ bool item_of(const Dev3 &d, int &c, int &x) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int item = __builtin_amdgcn_readfirstlane(b * WAVES + (int)(threadIdx.x >> 6));
    if (item >= d.ncol * d.nseg) return false;
    c = item / d.nseg;
    const int seg = item - c * d.nseg;
    x = seg * 64 + (int)(threadIdx.x & 63);
    return true;
}

// Pulled populations of node x of column c as deviations from its column's
// reference, in the arithmetic type C: dh_q = s_q(source) + K_q.  Returns u_ref.
template <typename T, typename C, int PAR>
__device__ __forceinline__ C pull(const Dev3 &d, int c, int x, C dh[Q], long long &own) {
    const int *R = d.crow + 20 * c;
    const double *K = d.cK + 20 * c;
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

template <typename T, int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_sweep(Dev3 d) {
    using C = typename Arith3<T>::type;
    int c, x;
    if (!item_of(d, c, x) || x >= d.nx) return;
    C h[Q];
    long long own;
    const C ur = pull<T, C, PAR>(d, c, x, h, own);
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
    const C Fx = (C)d.gx;
    const C dux = (jx + C(0.5) * Fx - drho * ur) * ir, duy = jy * ir, duz = jz * ir;
    const C ux = ur + dux, uy = duy, uz = duz;
    const C uu = ux * ux + uy * uy + uz * uz;
    // Eq. (2) as a deviation from the reference, every term carrying drho or du:
    // h_eq - r = w [c0 + drho (3 eu + 4.5 eu^2) + 3 edu + 4.5 edu (eu + e.u_ref)]
    const C c0 = drho * (C(1) - C(1.5) * uu) - C(1.5) * (dux * (ux + ur) + duy * uy + duz * uz);
    const C om = (C)d.omega, om1 = C(1) - om, fc = (C)d.fc;
    const C fb = C(-3) * (ux * Fx);   // 3 (-u).F with F = (gx, 0, 0)
    T *B = (T *)d.pop[PAR ^ 1];
    st3(B + own, (float)(om1 * h[0] + om * (C)wq(0) * c0 + fc * (C)wq(0) * fb), d.scale);
    // opposite pairs (q, q + 1): even part S, odd part M, as in the 2D sweep
#pragma unroll
    for (int q = 1; q < Q; q += 2) {
        const C eu = (C)EX[q] * ux + (C)EY[q] * uy + (C)EZ[q] * uz;
        const C edu = (C)EX[q] * dux + (C)EY[q] * duy + (C)EZ[q] * duz;
        const C eF = (C)EX[q] * Fx;
        const C S = c0 + C(4.5) * (drho * eu * eu + edu * (eu + (C)EX[q] * ur));
        const C A = C(3) * (drho * eu + edu);
        const C P = om * S + fc * (fb + C(9) * eu * eF);
        const C M = om * A + fc * (C(3) * eF);
        st3(B + q * d.qstride + own, (float)(om1 * h[q] + (C)wq(q) * (P + M)), d.scale);
        st3(B + (q + 1) * d.qstride + own, (float)(om1 * h[q + 1] + (C)wq(q) * (P - M)), d.scale);
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
    char *base = nullptr;
    size_t off_pop[2]{}, off_crow = 0, off_cK = 0, off_macro = 0, off_part = 0, ws = 0;
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
    capib3d_ctx *c = new capib3d_ctx();
    c->lat = L;
    c->stream = (hipStream_t)hip_stream;
    c->pitch = (L.nx + 63) / 64 * 64;
    c->esize = L.storage == CAPIB_FP16_SHIFTED ? 2 : 4;
    c->nseg = c->pitch / 64;
    c->fluid.assign((size_t)L.ny * L.nz, 0);
    for (int z = 0; z < L.nz; z++)
        for (int y = 0; y < L.ny; y++) c->fluid[(size_t)z * L.ny + y] = fluid_yz(L, y, z) ? 1 : 0;
    for (unsigned char f : c->fluid) c->ncol += f;
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
    const bool h16 = c->lat.storage == CAPIB_FP16_SHIFTED;
    for (int t = 0; t < nsteps; t++) {
        if (c->par)
            hipLaunchKernelGGL((h16 ? k3_sweep<_Float16, 1> : k3_sweep<float, 1>), dim3(c->nblk), dim3(64 * WAVES), 0,
                               c->stream, c->d);
        else
            hipLaunchKernelGGL((h16 ? k3_sweep<_Float16, 0> : k3_sweep<float, 0>), dim3(c->nblk), dim3(64 * WAVES), 0,
                               c->stream, c->d);
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
