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
// FP32 deviations s = h - r(y, z) from the equilibrium of the reference
// profile; the collision is evaluated in FP64 and each stored value rounded
// once.  Work items (column, 64-wide x segment) are ordered column-major, so
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
    float *pop[2];
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

// Pulled populations of node x of column c as FP64 deviations from its
// column's reference: dh_q = s_q(source) + K_q.  Returns u_ref.
template <int PAR>
__device__ __forceinline__ double pull(const Dev3 &d, int c, int x, double dh[Q], long long &own) {
    const int *R = d.crow + 20 * c;
    const double *K = d.cK + 20 * c;
    const float *A = d.pop[PAR];
    own = (long long)R[0] * d.pitch + x;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int rs = R[1 + q];
        float v;
        if (rs < 0) {
            v = A[opp(q) * d.qstride + own];
        } else {
            int xs = x - EX[q];
            xs = xs < 0 ? xs + d.nx : xs >= d.nx ? xs - d.nx : xs;
            v = A[q * d.qstride + (long long)rs * d.pitch + xs];
        }
        dh[q] = (double)v + K[q];
    }
    return K[19];
}

template <int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_sweep(Dev3 d) {
    int c, x;
    if (!item_of(d, c, x) || x >= d.nx) return;
    double h[Q];
    long long own;
    const double ur = pull<PAR>(d, c, x, h, own);
    // moments of the deviations: drho, and j - (u_ref, 0, 0)
    double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        drho += h[q];
        jx += EX[q] * h[q];
        jy += EY[q] * h[q];
        jz += EZ[q] * h[q];
    }
    const double rho = 1.0 + drho;
    // 1/rho: the FP32 hardware reciprocal and one Newton step (relative
    // error ~1e-14; it only scales deviation-sized terms)
    double ir = (double)__builtin_amdgcn_rcpf((float)rho);
    ir = ir * (2.0 - rho * ir);
    const double Fx = d.gx;
    const double dux = (jx + 0.5 * Fx - drho * ur) * ir, duy = jy * ir, duz = jz * ir;
    const double ux = ur + dux, uy = duy, uz = duz;
    const double uu = ux * ux + uy * uy + uz * uz;
    // Eq. (2) as a deviation from the reference, every term carrying drho or du:
    // h_eq - r = w [c0 + drho (3 eu + 4.5 eu^2) + 3 edu + 4.5 edu (eu + e.u_ref)]
    const double c0 = drho * (1.0 - 1.5 * uu) - 1.5 * (dux * (ux + ur) + duy * uy + duz * uz);
    const double om = d.omega, om1 = 1.0 - om, fc = d.fc;
    const double fb = -3.0 * (ux * Fx);   // 3 (-u).F with F = (gx, 0, 0)
    float *B = d.pop[PAR ^ 1];
    B[own] = (float)(om1 * h[0] + om * wq(0) * c0 + fc * wq(0) * fb);
    // opposite pairs (q, q + 1): even part S, odd part M, as in the 2D sweep
#pragma unroll
    for (int q = 1; q < Q; q += 2) {
        const double eu = EX[q] * ux + EY[q] * uy + EZ[q] * uz;
        const double edu = EX[q] * dux + EY[q] * duy + EZ[q] * duz;
        const double eF = EX[q] * Fx;
        const double S = c0 + 4.5 * (drho * eu * eu + edu * (eu + EX[q] * ur));
        const double A = 3.0 * (drho * eu + edu);
        const double P = om * S + fc * (fb + 9.0 * eu * eF);
        const double M = om * A + fc * (3.0 * eF);
        B[q * d.qstride + own] = (float)(om1 * h[q] + wq(q) * (P + M));
        B[(q + 1) * d.qstride + own] = (float)(om1 * h[q + 1] + wq(q) * (P - M));
    }
}

// Moments the next step starts from, FP64, into d.macro (fluid nodes).
template <int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_macro(Dev3 d) {
    int c, x;
    if (!item_of(d, c, x) || x >= d.nx) return;
    double h[Q];
    long long own;
    const double ur = pull<PAR>(d, c, x, h, own);
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
template <int PAR>
__global__ __launch_bounds__(64 * WAVES) void k3_diag(Dev3 d) {
    __shared__ double s[WAVES][4];
    int c = 0, x = 0;
    double m = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    if (item_of(d, c, x) && x < d.nx) {
        const long long own = (long long)d.crow[20 * c] * d.pitch + x;
        const float *A = d.pop[PAR];
        for (int q = 0; q < Q; q++) {
            const double v = A[q * d.qstride + own];
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
    int pitch = 0, ncol = 0, nseg = 0, nblk = 0, par = 0;
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
    capib3d_ctx *c = new capib3d_ctx();
    c->lat = L;
    c->stream = (hipStream_t)hip_stream;
    c->pitch = (L.nx + 63) / 64 * 64;
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
    for (int p = 0; p < 2; p++) { c->off_pop[p] = o; o = al256(o + (size_t)Q * N * 4); }
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
    for (int p = 0; p < 2; p++) d.pop[p] = (float *)(c->base + c->off_pop[p]);
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
    for (int p = 0; p < 2; p++) HIP3(c, hipMemsetAsync(c->base + c->off_pop[p], 0, (size_t)Q * N * 4, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    c->par = 0;
    c->step = 0;
    return CAPIB_OK;
}

capib_status capib3d_step(capib3d_ctx *c, int32_t nsteps) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (nsteps < 0) return fail3(c, CAPIB_E_ARG, "negative step count");
    for (int t = 0; t < nsteps; t++) {
        if (c->par)
            hipLaunchKernelGGL(k3_sweep<1>, dim3(c->nblk), dim3(64 * WAVES), 0, c->stream, c->d);
        else
            hipLaunchKernelGGL(k3_sweep<0>, dim3(c->nblk), dim3(64 * WAVES), 0, c->stream, c->d);
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
    if (c->par)
        hipLaunchKernelGGL(k3_macro<1>, dim3(c->nblk), dim3(64 * WAVES), 0, c->stream, c->d);
    else
        hipLaunchKernelGGL(k3_macro<0>, dim3(c->nblk), dim3(64 * WAVES), 0, c->stream, c->d);
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
    std::vector<float> buf((size_t)Q * N);
    HIP3(c, hipMemcpyAsync(buf.data(), c->base + c->off_pop[c->par], buf.size() * 4, hipMemcpyDeviceToHost,
                           c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    for (int q = 0; q < Q; q++)
        for (int z = 0; z < L.nz; z++)
            for (int y = 0; y < L.ny; y++) {
                const size_t col = (size_t)z * L.ny + y;
                const bool fl = c->fluid[col];
                const double r = c->ref[col * Q + q];
                for (int x = 0; x < L.nx; x++)
                    out[q * n + col * L.nx + x] = fl ? (double)buf[q * N + col * c->pitch + x] + r : 0.0;
            }
    return CAPIB_OK;
}

capib_status capib3d_write_populations(capib3d_ctx *c, const double *in) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!in) return fail3(c, CAPIB_E_ARG, "null input");
    const capib3d_lattice &L = c->lat;
    const size_t N = (size_t)c->pitch * L.ny * L.nz, n = (size_t)L.nx * L.ny * L.nz;
    std::vector<float> buf((size_t)Q * N, 0.0f);
    for (int q = 0; q < Q; q++)
        for (int z = 0; z < L.nz; z++)
            for (int y = 0; y < L.ny; y++) {
                const size_t col = (size_t)z * L.ny + y;
                if (!c->fluid[col]) continue;
                const double r = c->ref[col * Q + q];
                for (int x = 0; x < L.nx; x++) {
                    const double v = in[q * n + col * L.nx + x];
                    if (!std::isfinite(v)) return fail3(c, CAPIB_E_ARG, "non-finite population");
                    buf[q * N + col * c->pitch + x] = (float)(v - r);
                }
            }
    HIP3(c, hipMemcpyAsync(c->base + c->off_pop[c->par], buf.data(), buf.size() * 4, hipMemcpyHostToDevice,
                           c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    return CAPIB_OK;
}

capib_status capib3d_diagnostics(capib3d_ctx *c, double *out4, int64_t *step) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!out4) return fail3(c, CAPIB_E_ARG, "null output");
    if (c->par)
        hipLaunchKernelGGL(k3_diag<1>, dim3(c->nblk), dim3(64 * WAVES), 0, c->stream, c->d);
    else
        hipLaunchKernelGGL(k3_diag<0>, dim3(c->nblk), dim3(64 * WAVES), 0, c->stream, c->d);
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
