// C-ABI of libcapib: context, workspace layout, set-up of membranes and
// bonds (FP64 on the host, once), the step loop and read-outs.  Every step
// of the method runs in the kernels of lattice.hip and ib.hip.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/capib.h"
#include "capib_dev.hpp"
#include "capib_kernels.hpp"

using namespace capib;

namespace {

struct BodyHost {
    int kind, n, vstart, band = 0;
    int site_start = 0, n_sites = 0, n_bound0 = 0;
    bool has_bonds = false;
    double A0, P0;
    std::vector<double> xy;        // shape at creation
    std::vector<int> perm;         // sorted site k -> caller's site index
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

void split(double x, float &hi, float &lo) {
    hi = (float)x;
    lo = (float)(x - (double)hi);
}

}  // namespace

// steps captured in one HIP graph (even: a graph starts and ends on the
// same population parity); more steps per graph amortise the launch of the
// graph itself
constexpr int GRAPH_STEPS = 16;

struct capib_ctx {
    capib_lattice lat;
    int device = -1;               // HIP device current at creation (or at binding)
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    Dev d{};
    int pitch = 0, ntx = 0, nty = 0;
    size_t esize = 4;
    // workspace layout
    size_t ws_bytes = 0;
    size_t off_pop[2]{}, off_sp = 0, off_near = 0, off_red = 0, off_macro = 0, off_rowref = 0, off_rowref64 = 0, off_scal = 0;
    size_t off_ib = 0, ib_bytes = 0;
    size_t off_bp = 0, off_bs = 0, off_vnext = 0, off_pos[8]{}, off_dxm = 0, off_dym = 0, off_x0[4]{};
    size_t off_r0x = 0, off_r0y = 0, off_l0 = 0, off_th0 = 0, off_ustar = 0, off_probe = 0, off_force = 0;
    size_t off_target = 0, off_srange = 0, off_shost = 0, off_sstate = 0, off_sorig = 0, off_sfrac = 0;
    size_t off_sanh = 0, off_sanl = 0;
    char *base = nullptr;
    bool bound = false;
    int par = 0;
    long long step = 0;
    int nbodies = 0, nverts = 0, nsites = 0;
    std::vector<BodyHost> bodies;
    std::vector<double> ref_u;     // reference x-velocity per band-local row (FP64)
    // bands of the stack (ensemble members); a single lattice is one band
    int nbands = 1, band_rows = 0;
    std::vector<int> band_nx;
    std::vector<int> band_b0, band_nb;   // first body and body count per band
    size_t off_band = 0, off_vinfo = 0, off_live = 0;
    int nlive = 0;
    std::string err = "no error";
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    double ms[4] = {0, 0, 0, 0};
    long long nodes[4] = {0, 0, 0, 0};   // lattice nodes swept per phase
    long long tsteps = 0;
    // graphs
    bool use_graph = false;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};    // GRAPH_STEPS steps, by starting parity
    hipGraphExec_t gexec2[2] = {nullptr, nullptr};   // two steps
    // fork/join of the immersed-boundary phase with the far lattice tiles
    hipStream_t side = nullptr, cap_side = nullptr;
    hipEvent_t ev_fork[GRAPH_STEPS] = {}, ev_join[GRAPH_STEPS] = {};
    bool marks_valid = false;
    // launch configuration asked for (-1: the library's rule), see capib_tuning
    capib_tuning tune{-1, -1, -1, -1};
};

static capib_status fail(capib_ctx *c, capib_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIPCHK(c, call)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail((c), CAPIB_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// near-tile bookkeeping, per parity: the two vertex ranges of every tile
// (16 bytes), the flags, the list, the expanded list (32 bytes per entry);
// then the two list counts
static size_t near_bytes(const capib_ctx *c) { return 2 * 56 * (size_t)c->ntx * c->nty + 64; }

static void layout(capib_ctx *c) {
    const capib_lattice &L = c->lat;
    size_t o = 0;
    const size_t N = (size_t)c->pitch * L.ny;
    for (int p = 0; p < 2; p++) { c->off_pop[p] = o; o = align256(o + 9 * N * c->esize); }
    // near-tile flags and lists (two parities each) and their two counts
    c->off_near = o; o = align256(o + near_bytes(c));
    c->off_red = o; o = align256(o + (3 * (size_t)c->ntx * c->nty + 3) * 8);
    c->off_macro = o; o = align256(o + 3 * (size_t)L.nx * L.ny * 4);
    c->off_rowref = o; o = align256(o + (size_t)c->band_rows * 16 * 4);
    c->off_rowref64 = o; o = align256(o + (size_t)c->band_rows * 16 * 8);
    c->off_band = o; o = align256(o + (size_t)c->nbands * 12);   // widths, then (first body, count)
    c->off_live = o; o = align256(o + (size_t)c->ntx * c->nty * 4);
    c->off_scal = o; o = align256(o + 64);
    // spread records (rewritten every step, not checkpointed): origin, x and y
    // weights, force per vertex
    c->off_sp = o; o = align256(o + (size_t)std::max(1, L.max_vertices) * (8 + 16 + 16 + 8 + 32));
    // IB region: one contiguous block (checkpointed whole)
    const size_t B = (size_t)std::max(1, L.max_bodies), V = (size_t)std::max(1, L.max_vertices),
                 S = (size_t)std::max(1, L.max_sites);
    c->off_ib = o;
    c->off_bp = o; o = align256(o + B * sizeof(BodyParams));
    c->off_bs = o; o = align256(o + B * sizeof(BodyState));
    c->off_vnext = o; o = align256(o + V * 4);
    c->off_vinfo = o; o = align256(o + V * 4);
    for (int k = 0; k < 8; k++) { c->off_pos[k] = o; o = align256(o + V * 4); }
    c->off_dxm = o; o = align256(o + V * 4);
    c->off_dym = o; o = align256(o + V * 4);
    for (int k = 0; k < 4; k++) { c->off_x0[k] = o; o = align256(o + V * 4); }
    c->off_r0x = o; o = align256(o + V * 8);
    c->off_r0y = o; o = align256(o + V * 8);
    c->off_l0 = o; o = align256(o + V * 4);
    c->off_th0 = o; o = align256(o + V * 4);
    c->off_ustar = o; o = align256(o + V * 8);
    c->off_probe = o; o = align256(o + V * 16);
    c->off_force = o; o = align256(o + V * 8);
    c->off_target = o; o = align256(o + V * 8);
    c->off_srange = o; o = align256(o + V * 8);
    c->off_shost = o; o = align256(o + S * 4);
    c->off_sstate = o; o = align256(o + S * 4);
    c->off_sorig = o; o = align256(o + S * 4);
    c->off_sfrac = o; o = align256(o + S * 8);
    c->off_sanh = o; o = align256(o + S * 4);
    c->off_sanl = o; o = align256(o + S * 4);
    c->ib_bytes = o - c->off_ib;
    c->ws_bytes = o;
}

static void fill_dev(capib_ctx *c) {
    Dev &d = c->d;
    const capib_lattice &L = c->lat;
    char *b = c->base;
    d.nx = L.nx; d.ny = L.ny; d.pitch = c->pitch; d.walls = L.walls;
    d.ntx = c->ntx; d.nty = c->nty; d.storage = L.storage; d.band_rows = c->band_rows;
    d.qstride = (long long)c->pitch * L.ny;
    d.omega = (float)(1.0 / L.tau);
    d.fc = (float)(1.0 - 0.5 / L.tau);
    d.gx = (float)L.gx; d.gy = (float)L.gy;
    d.omega64 = 1.0 / L.tau;
    d.fc64 = 1.0 - 0.5 / L.tau;
    d.gx64 = L.gx; d.gy64 = L.gy;
    d.scale = L.storage ? (float)L.fp16_scale : 1.0f;
    d.inv_scale = L.storage ? (float)(1.0 / L.fp16_scale) : 1.0f;
    for (int p = 0; p < 2; p++) d.pop[p] = b + c->off_pop[p];
    {
        const size_t V = (size_t)std::max(1, L.max_vertices);
        char *q = b + c->off_sp;
        d.sp_wx = (float4 *)q;
        d.sp_wy = (float4 *)(q + 16 * V);
        d.sp_org = (int2 *)(q + 32 * V);
        d.sp_f = (float2 *)(q + 40 * V);
        d.pprobe[0] = (float4 *)(q + 48 * V);
        d.pprobe[1] = (float4 *)(q + 64 * V);
    }
    {
        const size_t nt = (size_t)c->ntx * c->nty;
        int *nb = (int *)(b + c->off_near);
        d.tv[0] = nb;
        d.tv[1] = nb + 4 * nt;
        d.tnear[0] = nb + 8 * nt;
        d.tnear[1] = nb + 9 * nt;
        d.nlist[0] = nb + 10 * nt;
        d.nlist[1] = nb + 11 * nt;
        d.ncount = nb + 12 * nt;
        d.elist[0] = (int4 *)(b + c->off_near + 48 * nt + 64);
        d.elist[1] = d.elist[0] + 2 * nt;
    }
    d.red = (double *)(b + c->off_red);
    d.macro = (float *)(b + c->off_macro);
    d.rowref = (const float *)(b + c->off_rowref);
    d.rowref64 = (const double *)(b + c->off_rowref64);
    d.counter = (long long *)(b + c->off_scal);
    d.err = (int *)(b + c->off_scal + 8);
    d.nbodies = c->nbodies; d.nverts = c->nverts; d.nsites = c->nsites; d.nbands = c->nbands;
    d.body_mv = 256;
    for (const BodyHost &bh : c->bodies) {
        const int need = std::max(bh.n, (bh.n_sites + 1) / 2);
        while (d.body_mv < need) d.body_mv *= 2;
    }
    // launch configuration: the tuning asked for, else the library's rules
    if (c->tune.membrane_class > d.body_mv) d.body_mv = c->tune.membrane_class;
    d.split = c->tune.split >= 0 ? c->tune.split : default_split(c->ntx * c->nty);
    d.far_share = c->tune.far_share_pct >= 0 ? c->tune.far_share_pct : default_far_share(L.storage);
    d.mark_pairs = c->tune.mark_pairs >= 0 ? c->tune.mark_pairs : default_mark_pairs(c->nverts);
    d.band_nx = (const int *)(b + c->off_band);
    d.band_bodies = (const int2 *)(b + c->off_band + 4 * (size_t)c->nbands);
    d.live = (const int *)(b + c->off_live);
    d.nlive = c->nlive;
    d.vinfo = (int *)(b + c->off_vinfo);
    for (int k = 0; k < ARG_BODIES; k++) {
        if (k < c->nbodies) {
            const BodyHost &bh = c->bodies[k];
            d.brange[k] = make_int4(bh.vstart, bh.n, bh.site_start, bh.n_sites);
        } else {
            d.brange[k] = make_int4(0, 0, 0, 0);
        }
    }
    d.bp = (BodyParams *)(b + c->off_bp);
    d.bs = (BodyState *)(b + c->off_bs);
    d.vnext = (int *)(b + c->off_vnext);
    for (int p = 0; p < 2; p++) {
        d.pxh[p] = (float *)(b + c->off_pos[4 * p + 0]);
        d.pxl[p] = (float *)(b + c->off_pos[4 * p + 1]);
        d.pyh[p] = (float *)(b + c->off_pos[4 * p + 2]);
        d.pyl[p] = (float *)(b + c->off_pos[4 * p + 3]);
    }
    d.dxm = (float *)(b + c->off_dxm); d.dym = (float *)(b + c->off_dym);
    d.x0h = (float *)(b + c->off_x0[0]); d.x0l = (float *)(b + c->off_x0[1]);
    d.y0h = (float *)(b + c->off_x0[2]); d.y0l = (float *)(b + c->off_x0[3]);
    d.r0x = (double *)(b + c->off_r0x); d.r0y = (double *)(b + c->off_r0y);
    d.l0 = (float *)(b + c->off_l0); d.th0 = (float *)(b + c->off_th0);
    d.ustar = (float2 *)(b + c->off_ustar);
    d.probe4 = (float4 *)(b + c->off_probe);
    d.force = (float2 *)(b + c->off_force);
    d.target = (float2 *)(b + c->off_target);
    d.srange = (int2 *)(b + c->off_srange);
    d.s_host = (int *)(b + c->off_shost); d.s_state = (int *)(b + c->off_sstate);
    d.s_orig = (int *)(b + c->off_sorig); d.s_frac = (double *)(b + c->off_sfrac);
    d.s_anh = (float *)(b + c->off_sanh); d.s_anl = (float *)(b + c->off_sanl);
}

static void drop_graphs(capib_ctx *c) {
    for (int p = 0; p < 2; p++) {
        if (c->gexec[p]) { (void)hipGraphExecDestroy(c->gexec[p]); c->gexec[p] = nullptr; }
        if (c->gexec2[p]) { (void)hipGraphExecDestroy(c->gexec2[p]); c->gexec2[p] = nullptr; }
    }
}

static capib_status need_ws(capib_ctx *c) {
    if (!c) return CAPIB_E_ARG;
    if (!c->bound) return fail(c, CAPIB_E_STATE, "no workspace bound");
    return CAPIB_OK;
}

static capib_status h2d(capib_ctx *c, size_t off, const void *src, size_t bytes) {
    if (!bytes) return CAPIB_OK;
    HIPCHK(c, hipMemcpyAsync(c->base + off, src, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CAPIB_OK;
}

static capib_status d2h(capib_ctx *c, void *dst, size_t off, size_t bytes) {
    if (!bytes) return CAPIB_OK;
    HIPCHK(c, hipMemcpyAsync(dst, c->base + off, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CAPIB_OK;
}

// D2Q9 in the order of Eq. (3)
static const int EXq[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EYq[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPPq[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double Wq[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// Reference population of band-local row y: h_eq(drho = 0, u = (u_ref(y), 0)), FP64.
static double ref_pop(const capib_ctx *c, int y, int q) {
    const double u = c->ref_u[y], eu = EXq[q] * u;
    return Wq[q] * (3.0 * eu + 4.5 * eu * eu - 1.5 * u * u);
}

// Per-row constants of the deviation storage (see Dev::rowref), from FP64.
static capib_status upload_ref(capib_ctx *c) {
    const int ny = c->band_rows;
    std::vector<double> t((size_t)ny * 16, 0.0);
    for (int y = 0; y < ny; y++) {
        for (int q = 0; q < 9; q++) {
            int ys = y - EYq[q];
            if (ys < 0 || ys >= ny) {
                if (c->lat.walls) {
                    t[16 * y + q] = ref_pop(c, y, OPPq[q]) - ref_pop(c, y, q);   // bounce-back from the node itself
                    continue;
                }
                ys = (ys + ny) % ny;
            }
            t[16 * y + q] = ref_pop(c, ys, q) - ref_pop(c, y, q);
        }
        t[16 * y + 9] = c->ref_u[y];
    }
    // FP32 for the FP16-storage sweep and the read-outs, FP64 for the
    // FP32-storage sweep
    std::vector<float> tf(t.size());
    for (size_t k = 0; k < t.size(); k++) tf[k] = (float)t[k];
    capib_status s = h2d(c, c->off_rowref, tf.data(), tf.size() * 4);
    if (s) return s;
    return h2d(c, c->off_rowref64, t.data(), t.size() * 8);
}

extern "C" {

// A stack of nbands bands of lat->ny rows each, band k of width widths[k].
static capib_status create_stack(const capib_lattice *lat, int nbands, const int32_t *widths, void *hip_stream,
                                 capib_ctx **out) {
    if (!lat || !out || nbands < 1 || !widths) return CAPIB_E_ARG;
    *out = nullptr;
    capib_lattice L = *lat;
    int wmax = 0;
    for (int k = 0; k < nbands; k++) {
        if (widths[k] < 1) return CAPIB_E_ARG;
        wmax = std::max(wmax, (int)widths[k]);
    }
    // bands are whole tile rows, so that no tile straddles two of them
    if (nbands > 1 && L.ny % TILE_Y != 0) return CAPIB_E_ARG;
    if (L.ny < 2 || (long long)wmax * L.ny * nbands > (1LL << 31)) return CAPIB_E_ARG;
    // with walls the velocity stencil folds onto four fluid rows
    if (L.walls && L.ny < 4) return CAPIB_E_ARG;
    if (!(L.tau > 0.5) || !std::isfinite(L.tau) || !std::isfinite(L.gx) || !std::isfinite(L.gy)) return CAPIB_E_ARG;
    if (L.walls != 0 && L.walls != 3) return CAPIB_E_ARG;
    if (L.storage != CAPIB_FP32_SHIFTED && L.storage != CAPIB_FP16_SHIFTED) return CAPIB_E_ARG;
    if (L.storage == CAPIB_FP16_SHIFTED) {
        int ex;
        double m = std::frexp(L.fp16_scale, &ex);
        if (!(L.fp16_scale > 0) || m != 0.5) return CAPIB_E_ARG;   // a power of two
    }
    if (L.max_bodies < 0 || L.max_vertices < 0 || L.max_sites < 0) return CAPIB_E_ARG;
    int dev = -1;   // unknown until a device is present (set again when the workspace is bound)
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    capib_ctx *c = new capib_ctx();
    c->device = dev;
    c->nbands = nbands;
    c->band_rows = L.ny;
    c->band_nx.assign(widths, widths + nbands);
    c->band_b0.assign(nbands, 0);
    c->band_nb.assign(nbands, 0);
    L.nx = wmax;
    L.ny = L.ny * nbands;
    c->lat = L;
    c->stream = (hipStream_t)hip_stream;
    c->esize = L.storage == CAPIB_FP32_SHIFTED ? 4 : 2;
    c->pitch = (L.nx + TILE_X - 1) / TILE_X * TILE_X;
    c->ntx = (L.nx + TILE_X - 1) / TILE_X;
    c->nty = (L.ny + TILE_Y - 1) / TILE_Y;
    // Eq. (12) prefactor, minimum allowed distance dx, distance floor, probe 1.2 dx
    c->d.rep_pref = (float)(1.0e-4 / (8.0 * std::sqrt(2.0)));
    c->d.rep_cut = 1.0f;
    c->d.rep_dmin = 0.1f;
    c->d.probe = 1.2f;
    layout(c);
    *out = c;
    return CAPIB_OK;
}

capib_status capib_create(const capib_lattice *lat, void *hip_stream, capib_ctx **out) {
    if (!lat) return CAPIB_E_ARG;
    if (lat->nx < 1) return CAPIB_E_ARG;
    const int32_t w = lat->nx;
    return create_stack(lat, 1, &w, hip_stream, out);
}

capib_status capib_create_ensemble(const capib_lattice *lat, int32_t nbands, const int32_t *widths, void *hip_stream,
                                   capib_ctx **out) {
    return create_stack(lat, nbands, widths, hip_stream, out);
}

size_t capib_workspace_bytes(const capib_ctx *c) { return c ? c->ws_bytes : 0; }

capib_status capib_bind_workspace(capib_ctx *c, void *ptr, size_t bytes) {
    if (!c) return CAPIB_E_ARG;
    if (!ptr || bytes < c->ws_bytes) return fail(c, CAPIB_E_ARG, "workspace of %zu bytes needs %zu", bytes, c->ws_bytes);
    if (((uintptr_t)ptr & 255) != 0) return fail(c, CAPIB_E_ARG, "workspace not 256-byte aligned");
    drop_graphs(c);
    if (c->device < 0) HIPCHK(c, hipGetDevice(&c->device));
    c->base = (char *)ptr;
    c->bound = true;
    c->marks_valid = false;
    c->par = 0;
    c->step = 0;
    c->nbodies = c->nverts = c->nsites = 0;
    c->bodies.clear();
    fill_dev(c);
    c->ref_u.assign(c->band_rows, 0.0);
    c->band_b0.assign(c->nbands, 0);
    c->band_nb.assign(c->nbands, 0);
    HIPCHK(c, hipMemsetAsync(c->base, 0, c->ws_bytes, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    capib_status s = h2d(c, c->off_band, c->band_nx.data(), (size_t)c->nbands * 4);
    if (s) return s;
    // the tiles that hold fluid nodes, in index order
    std::vector<int> live;
    for (int t = 0; t < c->ntx * c->nty; t++) {
        const int row = (t / c->ntx) * TILE_Y, x0 = (t % c->ntx) * TILE_X;
        if (row < c->lat.ny && x0 < c->band_nx[row / c->band_rows]) live.push_back(t);
    }
    c->nlive = (int)live.size();
    c->d.nlive = c->nlive;
    return h2d(c, c->off_live, live.data(), live.size() * 4);
}

capib_status capib_init_flow(capib_ctx *c, const double *ux) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (c->step != 0) return fail(c, CAPIB_E_STATE, "the flow is initialised before the first step");
    if (ux)
        for (int j = 0; j < c->band_rows; j++)
            if (!std::isfinite(ux[j]) || std::fabs(ux[j]) > 0.1) return fail(c, CAPIB_E_ARG, "bad velocity in row %d", j);
    // the initial profile becomes the reference of the deviation storage
    for (int j = 0; j < c->band_rows; j++) c->ref_u[j] = ux ? ux[j] : 0.0;
    if ((s = upload_ref(c))) return s;
    HIPCHK(c, launch_init_flow(c->d, c->par, c->stream));
    return CAPIB_OK;
}

capib_status capib_write_populations(capib_ctx *c, const double *h) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!h) return fail(c, CAPIB_E_ARG, "null populations");
    const capib_lattice &L = c->lat;
    const size_t N = (size_t)c->pitch * L.ny;
    std::vector<char> buf(9 * N * c->esize, 0);
    for (int q = 0; q < 9; q++)
        for (int j = 0; j < L.ny; j++)
            for (int i = 0; i < L.nx; i++) {
                const double hv = h[((size_t)q * L.ny + j) * L.nx + i];
                if (!std::isfinite(hv)) return fail(c, CAPIB_E_ARG, "non-finite population");
                const double v = hv - ref_pop(c, j % c->band_rows, q);
                const size_t k = q * N + (size_t)j * c->pitch + i;
                if (c->esize == 4) {
                    ((float *)buf.data())[k] = (float)v;
                } else {
                    const double sv = v * L.fp16_scale;
                    if (!(std::fabs(sv) <= 65504.0))
                        return fail(c, CAPIB_E_ARG, "population deviation %g beyond FP16 at scale %g", v, L.fp16_scale);
                    ((_Float16 *)buf.data())[k] = (_Float16)(float)sv;
                }
            }
    return h2d(c, c->off_pop[c->par], buf.data(), buf.size());
}

capib_status capib_read_populations(capib_ctx *c, double *h) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!h) return fail(c, CAPIB_E_ARG, "null output");
    const capib_lattice &L = c->lat;
    const size_t N = (size_t)c->pitch * L.ny;
    std::vector<char> buf(9 * N * c->esize);
    if ((s = d2h(c, buf.data(), c->off_pop[c->par], buf.size()))) return s;
    for (int q = 0; q < 9; q++)
        for (int j = 0; j < L.ny; j++)
            for (int i = 0; i < L.nx; i++) {
                const size_t k = q * N + (size_t)j * c->pitch + i;
                h[((size_t)q * L.ny + j) * L.nx + i] =
                    ref_pop(c, j % c->band_rows, q) + (c->esize == 4 ? (double)((float *)buf.data())[k]
                                                       : (double)(float)((_Float16 *)buf.data())[k] / L.fp16_scale);
            }
    return CAPIB_OK;
}

capib_status capib_add_membrane(capib_ctx *c, const capib_membrane *m, int32_t *body_id) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!m || !m->xy) return fail(c, CAPIB_E_ARG, "null membrane");
    if (m->kind < 0 || m->kind > 2) return fail(c, CAPIB_E_ARG, "bad membrane kind %d", m->kind);
    const int n = m->n;
    if (n < 3 || n > MAXV_BODY) return fail(c, CAPIB_E_CAPACITY, "membrane of %d vertices (3..%d)", n, MAXV_BODY);
    if (c->nbodies + 1 > c->lat.max_bodies) return fail(c, CAPIB_E_CAPACITY, "more than %d bodies", c->lat.max_bodies);
    if (c->nverts + n > c->lat.max_vertices)
        return fail(c, CAPIB_E_CAPACITY, "more than %d vertices", c->lat.max_vertices);
    if (c->step != 0) return fail(c, CAPIB_E_STATE, "membranes are added before the first step");
    const int band = m->band;
    if (band < 0 || band >= c->nbands) return fail(c, CAPIB_E_ARG, "bad band %d", band);
    if (c->nbodies > 0 && band < c->bodies.back().band)
        return fail(c, CAPIB_E_ARG, "membranes are added in band order (band %d after %d)", band, c->bodies.back().band);
    const double params[] = {m->ks, m->kb, m->ka, m->p_ref, m->density_ratio};
    for (double p : params)
        if (!std::isfinite(p)) return fail(c, CAPIB_E_ARG, "non-finite membrane parameter");
    if (!(m->density_ratio > 0)) return fail(c, CAPIB_E_ARG, "density ratio must be > 0");
    const double *xy = m->xy, *rs = m->xy_rest ? m->xy_rest : m->xy;
    for (int k = 0; k < 2 * n; k++)
        if (!std::isfinite(xy[k]) || !std::isfinite(rs[k])) return fail(c, CAPIB_E_ARG, "non-finite vertex");
    for (int v = 0; v < n; v++) {
        const double y = xy[2 * v + 1];
        if (c->lat.walls && (y < -0.5 || y > c->band_rows - 0.5)) return fail(c, CAPIB_E_ARG, "vertex %d outside the fluid", v);
    }
    // FP64 geometry of a polygon
    auto geo = [n](const double *p, std::vector<double> &len, std::vector<double> &th, double &A, double &P,
                   double &cx, double &cy) {
        len.assign(n, 0); th.assign(n, 0);
        std::vector<double> tx(n), ty(n);
        for (int l = 0; l < n; l++) {
            const int q = (l + 1) % n;
            tx[l] = p[2 * q] - p[2 * l]; ty[l] = p[2 * q + 1] - p[2 * l + 1];
            len[l] = std::sqrt(tx[l] * tx[l] + ty[l] * ty[l]);
        }
        for (int v = 0; v < n; v++) {
            const int q = (v + n - 1) % n;
            th[v] = std::atan2(tx[q] * ty[v] - ty[q] * tx[v], tx[q] * tx[v] + ty[q] * ty[v]);
        }
        A = 0; P = 0;
        double sx = 0, sy = 0;
        for (int l = 0; l < n; l++) {
            const int q = (l + 1) % n;
            const double xa = p[2 * l] - p[0], ya = p[2 * l + 1] - p[1], xb = p[2 * q] - p[0], yb = p[2 * q + 1] - p[1];
            const double cr = xa * yb - xb * ya;
            A += cr; sx += (xa + xb) * cr; sy += (ya + yb) * cr;
            P += len[l];
        }
        A *= 0.5;
        cx = p[0] + sx / (6 * A);
        cy = p[1] + sy / (6 * A);
    };
    std::vector<double> l0, th0, len, th;
    double A0, P0r, cxr, cyr, A, P, cx, cy;
    geo(rs, l0, th0, A0, P0r, cxr, cyr);
    geo(xy, len, th, A, P, cx, cy);
    if (!(A > 0) || !(A0 > 0)) return fail(c, CAPIB_E_ARG, "membrane is not counter-clockwise");
    for (int l = 0; l < n; l++)
        if (!(l0[l] > 0) || !(len[l] > 0)) return fail(c, CAPIB_E_ARG, "degenerate element %d", l);
    double J = 0;
    for (int l = 0; l < n; l++) {
        const int q = (l + 1) % n;
        const double xa = xy[2 * l] - cx, ya = xy[2 * l + 1] - cy, xb = xy[2 * q] - cx, yb = xy[2 * q + 1] - cy;
        const double cr = xa * yb - xb * ya;
        J += cr * (xa * xa + xa * xb + xb * xb + ya * ya + ya * yb + yb * yb);
    }
    J /= 12.0;

    const int b = c->nbodies, v0 = c->nverts;
    BodyParams bp{};
    bp.kind = m->kind; bp.n = n; bp.vstart = v0; bp.tag = m->tag;
    // bodies of a band are numbered contiguously (they are added in band order)
    if (c->band_nb[band] == 0) c->band_b0[band] = b;
    bp.band = band;
    bp.band_b0 = c->band_b0[band];
    bp.band_nb = c->band_nb[band] + 1;
    bp.ks = (float)m->ks; bp.kb = (float)m->kb; bp.ka = (float)m->ka; bp.pref = (float)m->p_ref;
    bp.vmass = (float)(m->density_ratio * A0 / n);
    bp.inv_mass = (float)(1.0 / (m->density_ratio * A));
    bp.inv_inertia = (float)(1.0 / (m->density_ratio * J));
    bp.A0 = A0;
    bp.P0 = (float)P;
    split(cx, bp.c0xh, bp.c0xl);
    split(cy, bp.c0yh, bp.c0yl);
    BodyState bs{};
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    std::vector<float> xh(n), xl(n), yh(n), yl(n), fl0(n), fth0(n);
    std::vector<double> r0x(n), r0y(n);
    std::vector<int> vnx(n), vinf(n);
    for (int v = 0; v < n; v++) {
        split(xy[2 * v], xh[v], xl[v]);
        split(xy[2 * v + 1], yh[v], yl[v]);
        vnx[v] = v0 + (v + 1) % n;
        vinf[v] = 2 * band + (v >= n / 2);
        r0x[v] = xy[2 * v] - cx;
        r0y[v] = xy[2 * v + 1] - cy;
        fl0[v] = (float)l0[v];
        fth0[v] = (float)th0[v];
        xmin = std::min(xmin, xy[2 * v]); xmax = std::max(xmax, xy[2 * v]);
        ymin = std::min(ymin, xy[2 * v + 1]); ymax = std::max(ymax, xy[2 * v + 1]);
    }
    for (int p = 0; p < 2; p++) {
        bs.bbox[p][0] = (float)xmin; bs.bbox[p][1] = (float)xmax;
        bs.bbox[p][2] = (float)ymin; bs.bbox[p][3] = (float)ymax;
    }
    const size_t fo = (size_t)v0 * 4;
    const int pp = c->par;
    if ((s = h2d(c, c->off_bp + b * sizeof(BodyParams), &bp, sizeof bp))) return s;
    if ((s = h2d(c, c->off_bs + b * sizeof(BodyState), &bs, sizeof bs))) return s;
    if ((s = h2d(c, c->off_vnext + fo, vnx.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_vinfo + fo, vinf.data(), n * 4))) return s;
    // the band's earlier bodies see one more neighbour
    for (int e = c->band_b0[band]; e < b; e++)
        if ((s = h2d(c, c->off_bp + e * sizeof(BodyParams) + offsetof(BodyParams, band_nb), &bp.band_nb, 4))) return s;
    if ((s = h2d(c, c->off_pos[4 * pp + 0] + fo, xh.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_pos[4 * pp + 1] + fo, xl.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_pos[4 * pp + 2] + fo, yh.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_pos[4 * pp + 3] + fo, yl.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_x0[0] + fo, xh.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_x0[1] + fo, xl.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_x0[2] + fo, yh.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_x0[3] + fo, yl.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_r0x + (size_t)v0 * 8, r0x.data(), n * 8))) return s;
    if ((s = h2d(c, c->off_r0y + (size_t)v0 * 8, r0y.data(), n * 8))) return s;
    if ((s = h2d(c, c->off_l0 + fo, fl0.data(), n * 4))) return s;
    if ((s = h2d(c, c->off_th0 + fo, fth0.data(), n * 4))) return s;
    BodyHost bh;
    bh.kind = m->kind; bh.n = n; bh.vstart = v0; bh.band = band; bh.A0 = A0; bh.P0 = P;
    bh.xy.assign(xy, xy + 2 * n);
    c->bodies.push_back(bh);
    c->band_nb[band]++;
    {
        const int2 r = make_int2(c->band_b0[band], c->band_nb[band]);
        if ((s = h2d(c, c->off_band + 4 * (size_t)c->nbands + 8 * (size_t)band, &r, 8))) return s;
    }
    c->nbodies++;
    c->nverts += n;
    c->marks_valid = false;
    drop_graphs(c);
    fill_dev(c);
    if (body_id) *body_id = b;
    return CAPIB_OK;
}

capib_status capib_add_bonds(capib_ctx *c, int32_t body_id, const capib_bonds *bd) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!bd || body_id < 0 || body_id >= c->nbodies) return fail(c, CAPIB_E_ARG, "bad body id %d", body_id);
    BodyHost &bh = c->bodies[body_id];
    if (bh.has_bonds) return fail(c, CAPIB_E_STATE, "body %d already has bonds", body_id);
    if (c->step != 0) return fail(c, CAPIB_E_STATE, "bonds are added before the first step");
    const int ns = bd->n_sites;
    if (ns < 0 || (ns > 0 && (!bd->host_elem || !bd->frac))) return fail(c, CAPIB_E_ARG, "bad site arrays");
    if (c->nsites + ns > c->lat.max_sites) return fail(c, CAPIB_E_CAPACITY, "more than %d sites", c->lat.max_sites);
    if (ns > MAXS_BODY) return fail(c, CAPIB_E_CAPACITY, "more than %d sites on one body", MAXS_BODY);
    const double pr[] = {bd->sigma, bd->y_cr, bd->y_eq, bd->k_f, bd->k_r0, bd->bell_len};
    for (double p : pr)
        if (!std::isfinite(p)) return fail(c, CAPIB_E_ARG, "non-finite bond parameter");
    if (!(bd->bell_len > 0) || bd->k_f < 0 || bd->k_r0 < 0) return fail(c, CAPIB_E_ARG, "bad bond rates");
    for (int k = 0; k < ns; k++)
        if (bd->host_elem[k] < 0 || bd->host_elem[k] >= bh.n || !(bd->frac[k] >= 0 && bd->frac[k] <= 1))
            return fail(c, CAPIB_E_ARG, "bad site %d", k);
    std::vector<int> perm(ns);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
        return bd->host_elem[a] != bd->host_elem[b] ? bd->host_elem[a] < bd->host_elem[b] : bd->frac[a] < bd->frac[b];
    });
    const int s0 = c->nsites, n = bh.n;
    std::vector<int> host(ns), state(ns), orig(ns);
    std::vector<double> frac(ns);
    std::vector<float> anh(ns, 0), anl(ns, 0);
    std::vector<int2> sr(n, make_int2(s0, s0));
    int nb = 0;
    for (int k = 0; k < ns; k++) {
        const int q = perm[k];
        const int e = bd->host_elem[q], mm = (e + 1) % n;
        host[k] = bh.vstart + e;
        frac[k] = bd->frac[q];
        orig[k] = q;
        const double xs = bh.xy[2 * e] + bd->frac[q] * (bh.xy[2 * mm] - bh.xy[2 * e]);
        const double ys = bh.xy[2 * e + 1] + bd->frac[q] * (bh.xy[2 * mm + 1] - bh.xy[2 * e + 1]);
        state[k] = (ys + 0.5 < bd->y_cr) ? 1 : 0;
        if (state[k]) split(xs, anh[k], anl[k]);
        nb += state[k];
    }
    for (int k = 0; k < ns; k++) {
        const int e = host[k] - bh.vstart;
        if (sr[e].x == s0 && sr[e].y == s0) sr[e] = make_int2(s0 + k, s0 + k + 1);
        else sr[e].y = s0 + k + 1;
    }
    // elements without sites get an empty range
    for (int e = 0; e < n; e++)
        if (sr[e].y == s0) sr[e] = make_int2(s0, s0);
    BodyParams bp{};
    if ((s = d2h(c, &bp, c->off_bp + body_id * sizeof(BodyParams), sizeof bp))) return s;
    bp.site_start = s0; bp.n_sites = ns;
    bp.sigma = (float)bd->sigma; bp.ycr = (float)bd->y_cr; bp.yeq = (float)bd->y_eq;
    bp.sigma64 = bd->sigma; bp.yeq64 = bd->y_eq; bp.ycr64 = bd->y_cr;
    bp.kf = (float)bd->k_f; bp.kr0 = (float)bd->k_r0; bp.lb = (float)bd->bell_len;
    bp.seed_lo = (uint32_t)(bd->seed & 0xffffffffu);
    bp.seed_hi = (uint32_t)(bd->seed >> 32);
    BodyState bs{};
    if ((s = d2h(c, &bs, c->off_bs + body_id * sizeof(BodyState), sizeof bs))) return s;
    bs.n_bound = nb;
    const size_t so = (size_t)s0 * 4;
    if ((s = h2d(c, c->off_bp + body_id * sizeof(BodyParams), &bp, sizeof bp))) return s;
    if ((s = h2d(c, c->off_bs + body_id * sizeof(BodyState), &bs, sizeof bs))) return s;
    if ((s = h2d(c, c->off_shost + so, host.data(), ns * 4))) return s;
    if ((s = h2d(c, c->off_sstate + so, state.data(), ns * 4))) return s;
    if ((s = h2d(c, c->off_sorig + so, orig.data(), ns * 4))) return s;
    if ((s = h2d(c, c->off_sfrac + (size_t)s0 * 8, frac.data(), ns * 8))) return s;
    if ((s = h2d(c, c->off_sanh + so, anh.data(), ns * 4))) return s;
    if ((s = h2d(c, c->off_sanl + so, anl.data(), ns * 4))) return s;
    if ((s = h2d(c, c->off_srange + (size_t)bh.vstart * 8, sr.data(), n * 8))) return s;
    bh.has_bonds = true;
    bh.n_bound0 = nb;
    bh.site_start = s0;
    bh.n_sites = ns;
    bh.perm = perm;
    c->nsites += ns;
    drop_graphs(c);
    fill_dev(c);
    return CAPIB_OK;
}

capib_status capib_set_interactions(capib_ctx *c, double pref, double cut, double probe) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!std::isfinite(pref) || !(cut >= 0) || !std::isfinite(cut) || !std::isfinite(probe))
        return fail(c, CAPIB_E_ARG, "bad interaction constants");
    c->d.rep_pref = (float)pref;
    c->d.rep_cut = (float)cut;
    c->d.probe = (float)probe;
    drop_graphs(c);
    return CAPIB_OK;
}

// Streams and events of the fork/join step, created once.
static capib_status ensure_streams(capib_ctx *c) {
    if (!c->side) HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (!c->cap_side) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_side, hipStreamNonBlocking));
    for (int k = 0; k < GRAPH_STEPS; k++) {
        if (!c->ev_fork[k]) HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork[k], hipEventDisableTiming));
        if (!c->ev_join[k]) HIPCHK(c, hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming));
    }
    return CAPIB_OK;
}

// Near tiles of the current positions, needed before a step when the
// previous step did not mark them (start, new membranes, loaded checkpoint).
static capib_status ensure_marks(capib_ctx *c) {
    if (c->marks_valid) return CAPIB_OK;
    HIPCHK(c, hipMemsetAsync(c->base + c->off_near, 0, near_bytes(c), c->stream));
    HIPCHK(c, launch_mark(c->d, c->par, c->stream));
    c->marks_valid = true;
    return CAPIB_OK;
}

// One step.  On a small lattice: interpolation, membrane kernel and the
// sweep of every tile, in sequence on the main stream.  On a large lattice
// the far tiles run on the main stream while the interpolation, the
// membrane kernel and the sweep of the near tiles run on the side stream:
// the two sweeps write the new populations of disjoint tiles, both only
// read the current ones, and the far tiles read this step's near-tile
// flags, which the marking leaves alone (it marks the other parity).  The
// step ends at the join.  main/side are the streams to enqueue on, k
// selects the event pair (so that several steps can be captured in one
// graph).
static capib_status one_step(capib_ctx *c, int par, hipStream_t main, hipStream_t side, int k) {
    if (!lattice_split(c->d)) {
        HIPCHK(c, launch_interp(c->d, par, main));
        HIPCHK(c, launch_body_far(c->d, par, main));
        HIPCHK(c, launch_lattice_sweep(c->d, par, main, nullptr, nullptr, body_far_share(c->d)));
        return CAPIB_OK;
    }
    HIPCHK(c, hipEventRecord(c->ev_fork[k], main));
    HIPCHK(c, hipStreamWaitEvent(side, c->ev_fork[k], 0));
    HIPCHK(c, launch_interp(c->d, par, side));
    HIPCHK(c, launch_body(c->d, par, side));
    HIPCHK(c, launch_lattice_sweep(c->d, par, side));
    HIPCHK(c, launch_lattice_far(c->d, par, main));
    HIPCHK(c, hipEventRecord(c->ev_join[k], side));
    HIPCHK(c, hipStreamWaitEvent(main, c->ev_join[k], 0));
    return CAPIB_OK;
}

static capib_status make_graph(capib_ctx *c, int par, int nsteps, hipGraphExec_t *out) {
    capib_status s = ensure_streams(c);
    if (s) return s;
    hipGraph_t g;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < nsteps && !s; k++) s = one_step(c, par ^ (k & 1), c->cap_stream, c->cap_side, k);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (s) return s;
    if (e != hipSuccess) return fail(c, CAPIB_E_HIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, CAPIB_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
    return CAPIB_OK;
}

// All four executables (16 and 2 steps, both starting parities), captured
// and instantiated together, so that no later call builds a graph between
// replays.
static capib_status build_graphs(capib_ctx *c) {
    capib_status s;
    for (int p = 0; p < 2; p++) {
        if (!c->gexec[p] && (s = make_graph(c, p, GRAPH_STEPS, &c->gexec[p]))) return s;
        if (!c->gexec2[p] && (s = make_graph(c, p, 2, &c->gexec2[p]))) return s;
    }
    return CAPIB_OK;
}

capib_status capib_step(capib_ctx *c, int32_t nsteps) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (nsteps < 0) return fail(c, CAPIB_E_ARG, "negative step count");
    if ((s = ensure_streams(c))) return s;
    if ((s = ensure_marks(c))) return s;
    if (c->timing) {
        // kernels in sequence on the main stream, each launched with a
        // start/stop event pair stamped at its own start and end
        const size_t need = 8 * (size_t)nsteps;
        while (c->ev.size() < need) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
        // the nodes each lattice launch sweeps, counted after every step
        // (untimed) from that step's near-tile flags
        const bool split = lattice_split(c->d);
        const int pct = split ? 0 : body_far_share(c->d);
        unsigned long long *cens = (unsigned long long *)(c->base + c->off_scal + 32);
        HIPCHK(c, hipMemsetAsync(cens, 0, 24, c->stream));
        for (int t = 0; t < nsteps; t++) {
            hipEvent_t *e = &c->ev[8 * t];
            HIPCHK(c, launch_interp(c->d, c->par, c->stream, e[0], e[1]));
            if (split) {
                HIPCHK(c, launch_body(c->d, c->par, c->stream, e[2], e[3]));
                HIPCHK(c, launch_lattice_far(c->d, c->par, c->stream, e[4], e[5]));
            } else {
                HIPCHK(c, launch_body_far(c->d, c->par, c->stream, e[2], e[3]));
            }
            HIPCHK(c, launch_lattice_sweep(c->d, c->par, c->stream, e[6], e[7], pct));
            HIPCHK(c, launch_census(c->d, c->par, pct, cens, c->stream));
            c->par ^= 1;
            c->step++;
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));
        unsigned long long cn[3];
        capib_status s2 = d2h(c, cn, c->off_scal + 32, sizeof cn);
        if (s2) return s2;
        c->nodes[1] += (long long)cn[0];
        c->nodes[split ? 2 : 3] += (long long)cn[1];
        c->nodes[3] += (long long)cn[2];
        for (int t = 0; t < nsteps; t++) {
            hipEvent_t *e = &c->ev[8 * t];
            for (int k = 0; k < 4; k++) {
                if (k == 2 && !split) continue;   // no far-tile launch
                float ms = 0;
                HIPCHK(c, hipEventElapsedTime(&ms, e[2 * k], e[2 * k + 1]));
                c->ms[k] += ms;
            }
        }
        c->tsteps += nsteps;
        return CAPIB_OK;
    }
    int t = 0;
    if (c->use_graph && nsteps >= 2) {
        if ((s = build_graphs(c))) return s;
        for (; t + GRAPH_STEPS <= nsteps; t += GRAPH_STEPS) {
            HIPCHK(c, hipGraphLaunch(c->gexec[c->par], c->stream));
            c->step += GRAPH_STEPS;
        }
        for (; t + 2 <= nsteps; t += 2) {
            HIPCHK(c, hipGraphLaunch(c->gexec2[c->par], c->stream));
            c->step += 2;
        }
    }
    for (; t < nsteps; t++) {
        if ((s = one_step(c, c->par, c->stream, c->side, 0))) return s;
        c->par ^= 1;
        c->step++;
    }
    return CAPIB_OK;
}

capib_status capib_set_graph(capib_ctx *c, int32_t enable) {
    if (!c) return CAPIB_E_ARG;
    c->use_graph = enable != 0;
    if (!c->use_graph) {
        drop_graphs(c);
        return CAPIB_OK;
    }
    // with a workspace bound, instantiate the graphs now
    return c->bound ? build_graphs(c) : CAPIB_OK;
}

// ---- launch configuration and its autotuner ---------------------------------------

capib_status capib_set_tuning(capib_ctx *c, const capib_tuning *t) {
    if (!c || !t) return CAPIB_E_ARG;
    if (t->split < -1 || t->split > 1 || t->mark_pairs < -1 || t->mark_pairs > 1 || t->far_share_pct < -1 ||
        t->far_share_pct > 100 || !(t->membrane_class == -1 || t->membrane_class == 256 ||
                                    t->membrane_class == 512 || t->membrane_class == MAXV_BODY))
        return fail(c, CAPIB_E_ARG, "bad tuning {%d, %d, %d, %d}", t->split, t->far_share_pct, t->mark_pairs,
                    t->membrane_class);
    c->tune = *t;
    drop_graphs(c);
    if (c->bound) fill_dev(c);
    return CAPIB_OK;
}

capib_status capib_get_tuning(const capib_ctx *c, capib_tuning *t) {
    if (!c || !t) return CAPIB_E_ARG;
    // resolved as the next step will launch (with the bodies added so far)
    t->split = c->tune.split >= 0 ? c->tune.split : (c->bound ? c->d.split : default_split(c->ntx * c->nty));
    t->far_share_pct = c->tune.far_share_pct >= 0 ? c->tune.far_share_pct
                                                  : (c->bound ? c->d.far_share : default_far_share(c->lat.storage));
    t->mark_pairs = c->tune.mark_pairs >= 0 ? c->tune.mark_pairs
                                            : (c->bound ? c->d.mark_pairs : default_mark_pairs(c->nverts));
    t->membrane_class = c->bound ? c->d.body_mv : (c->tune.membrane_class > 0 ? c->tune.membrane_class : 256);
    return CAPIB_OK;
}

// Workload signature of the cache: device, lattice shape and storage, the
// bands, the membranes and the sites (their counts and the largest membrane).
static std::string tune_key(const capib_ctx *c) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (c->device >= 0 && hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    uint64_t h = 1469598103934665603ULL;   // FNV-1a of the band widths
    for (int w : c->band_nx) {
        h ^= (uint64_t)(uint32_t)w;
        h *= 1099511628211ULL;
    }
    int big = 0;
    for (const BodyHost &bh : c->bodies) big = std::max(big, bh.n);
    char buf[512];
    snprintf(buf, sizeof buf, "%s|rows=%d|bands=%d|widths=%016llx|storage=%d|walls=%d|bodies=%d|verts=%d|sites=%d|"
             "largest=%d|graph=%d", arch.c_str(), c->band_rows, c->nbands, (unsigned long long)h, c->lat.storage,
             c->lat.walls, c->nbodies, c->nverts, c->nsites, big, c->use_graph ? 1 : 0);
    return buf;
}

static bool tune_cache_lookup(const char *path, const std::string &key, capib_tuning *t, double *ms) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char *tab = strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        if (key != line) continue;
        capib_tuning r;
        double m;
        if (sscanf(tab + 1, "%d %d %d %d %lf", &r.split, &r.far_share_pct, &r.mark_pairs, &r.membrane_class, &m) == 5) {
            *t = r;   // the last matching line wins
            *ms = m;
            found = true;
        }
    }
    fclose(f);
    return found;
}

capib_status capib_autotune(capib_ctx *c, int32_t steps, const char *cache_path, capib_tuning *chosen,
                            double *best_ms) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (steps < 16) return fail(c, CAPIB_E_ARG, "at least 16 steps per trial");
    const std::string key = tune_key(c);
    capib_tuning best = c->tune;
    double best_t = 0.0;
    if (cache_path && tune_cache_lookup(cache_path, key, &best, &best_t)) {
        if ((s = capib_set_tuning(c, &best))) return s;
        if (chosen) *chosen = best;
        if (best_ms) *best_ms = best_t;
        return CAPIB_OK;
    }
    // the state every trial starts from, restored at the end
    size_t bytes = 0;
    if ((s = capib_save(c, nullptr, &bytes))) return s;
    std::vector<char> ck(bytes);
    if ((s = capib_save(c, ck.data(), &bytes))) return s;
    const capib_tuning asked = c->tune;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    auto trial = [&](const capib_tuning &t, double &ms) -> capib_status {
        capib_status r;
        if ((r = capib_set_tuning(c, &t))) return r;
        if ((r = capib_load(c, ck.data(), ck.size()))) return r;
        if ((r = capib_step(c, GRAPH_STEPS))) return r;   // warm-up: marks, graphs
        ms = 1e30;
        for (int rep = 0; rep < 2; rep++) {
            HIPCHK(c, hipEventRecord(e0, c->stream));
            if ((r = capib_step(c, steps))) return r;
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            float el = 0.0f;
            HIPCHK(c, hipEventElapsedTime(&el, e0, e1));
            ms = std::min(ms, (double)el / steps);
        }
        return CAPIB_OK;
    };
    // coordinate descent from the library's own configuration: the
    // schedule, then (one sweep after the membrane phase) the far share of
    // the membrane launch, the marking layout, the membrane class
    capib_tuning cur;
    if ((s = capib_get_tuning(c, &cur))) return s;
    double cur_t = 0.0;
    auto better = [&](capib_tuning t) -> capib_status {
        double m;
        capib_status r = trial(t, m);
        if (r) return r;
        if (m < cur_t) { cur = t; cur_t = m; }
        return CAPIB_OK;
    };
    if ((s = trial(cur, cur_t))) goto done;
    {
        capib_tuning t = cur;
        t.split = 1 - cur.split;
        if ((s = better(t))) goto done;
    }
    if (cur.split == 0)
        for (int share : {20, 35, 50, 65, 80, 95}) {
            if (share == cur.far_share_pct) continue;
            capib_tuning t = cur;
            t.far_share_pct = share;
            if ((s = better(t))) goto done;
        }
    {
        capib_tuning t = cur;
        t.mark_pairs = 1 - cur.mark_pairs;
        if ((s = better(t))) goto done;
    }
    for (int cls : {256, 512, MAXV_BODY}) {
        if (cls <= cur.membrane_class) continue;
        capib_tuning t = cur;
        t.membrane_class = cls;
        if ((s = better(t))) goto done;
    }
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) {
        // leave the context as it was asked for, with its state
        c->tune = asked;
        fill_dev(c);
        drop_graphs(c);
        (void)capib_load(c, ck.data(), ck.size());
        return s;
    }
    best = cur;
    best_t = cur_t;
    if ((s = capib_set_tuning(c, &best))) return s;
    if ((s = capib_load(c, ck.data(), ck.size()))) return s;
    if (c->use_graph && (s = build_graphs(c))) return s;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s\t%d %d %d %d %.6f\n", key.c_str(), best.split, best.far_share_pct, best.mark_pairs,
                    best.membrane_class, best_t);
            fclose(f);
        }
    }
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = best_t;
    return CAPIB_OK;
}

capib_status capib_read_macro(capib_ctx *c, double *drho, double *ux, double *uy) {
    capib_status s = need_ws(c);
    if (s) return s;
    HIPCHK(c, launch_macro(c->d, c->par, c->stream));
    const size_t N = (size_t)c->lat.nx * c->lat.ny;
    std::vector<float> buf(3 * N);
    if ((s = d2h(c, buf.data(), c->off_macro, buf.size() * 4))) return s;
    for (size_t k = 0; k < N; k++) {
        if (drho) drho[k] = buf[k];
        if (ux) ux[k] = buf[N + k];
        if (uy) uy[k] = buf[2 * N + k];
    }
    return CAPIB_OK;
}

static capib_status check_body(capib_ctx *c, int32_t b) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (b < 0 || b >= c->nbodies) return fail(c, CAPIB_E_ARG, "bad body id %d", b);
    return CAPIB_OK;
}

capib_status capib_read_vertices(capib_ctx *c, int32_t b, double *xy) {
    capib_status s = check_body(c, b);
    if (s) return s;
    if (!xy) return fail(c, CAPIB_E_ARG, "null output");
    const BodyHost &bh = c->bodies[b];
    const int n = bh.n;
    std::vector<float> a(4 * n);
    for (int k = 0; k < 4; k++)
        if ((s = d2h(c, a.data() + k * n, c->off_pos[4 * c->par + k] + (size_t)bh.vstart * 4, n * 4))) return s;
    for (int v = 0; v < n; v++) {
        xy[2 * v] = (double)a[v] + (double)a[n + v];
        xy[2 * v + 1] = (double)a[2 * n + v] + (double)a[3 * n + v];
    }
    return CAPIB_OK;
}

capib_status capib_read_bonds(capib_ctx *c, int32_t b, uint8_t *state, double *anchor) {
    capib_status s = check_body(c, b);
    if (s) return s;
    const BodyHost &bh = c->bodies[b];
    const int ns = bh.n_sites;
    std::vector<int> st(ns);
    std::vector<float> ah(ns), al(ns);
    const size_t so = (size_t)bh.site_start * 4;
    if ((s = d2h(c, st.data(), c->off_sstate + so, ns * 4))) return s;
    if ((s = d2h(c, ah.data(), c->off_sanh + so, ns * 4))) return s;
    if ((s = d2h(c, al.data(), c->off_sanl + so, ns * 4))) return s;
    for (int k = 0; k < ns; k++) {
        const int q = bh.perm[k];
        if (state) state[q] = (uint8_t)st[k];
        if (anchor) anchor[q] = (double)ah[k] + (double)al[k];
    }
    return CAPIB_OK;
}

capib_status capib_read_body_work(capib_ctx *c, int32_t b, double *ustar, double *probe, double *force, double *target) {
    capib_status s = check_body(c, b);
    if (s) return s;
    const BodyHost &bh = c->bodies[b];
    const int n = bh.n;
    std::vector<float> f(4 * n);
    const size_t v0 = bh.vstart;
    struct { double *dst; size_t off; int w; } items[] = {
        {ustar, c->off_ustar + v0 * 8, 2}, {probe, c->off_probe + v0 * 16, 4},
        {force, c->off_force + v0 * 8, 2}, {target, c->off_target + v0 * 8, 2}};
    for (auto &it : items) {
        if (!it.dst) continue;
        if ((s = d2h(c, f.data(), it.off, (size_t)n * it.w * 4))) return s;
        for (int k = 0; k < n * it.w; k++) it.dst[k] = f[k];
    }
    return CAPIB_OK;
}

// The FP64 totals r[3] (sums of the stored deviations) completed with the
// reference part, the step counter and the error flags.
static capib_status diag_finish(capib_ctx *c, const double r[3], capib_diag *out) {
    capib_status s;
    const size_t nblk = (size_t)c->ntx * c->nty;
    long long cnt;
    int err;
    if ((s = d2h(c, &cnt, c->off_scal, 8))) return s;
    if ((s = d2h(c, &err, c->off_scal + 8, 4))) return s;
    // add the reference part of the stored deviations (FP64, host)
    double rm = 0, rx = 0, width = 0;
    for (int y = 0; y < c->band_rows; y++)
        for (int q = 0; q < 9; q++) {
            rm += ref_pop(c, y, q);
            rx += ref_pop(c, y, q) * EXq[q];
        }
    for (int k = 0; k < c->nbands; k++) width += c->band_nx[k];
    out->step = c->step;
    out->error_flags = err;
    out->n_bodies = c->nbodies;
    out->mass = r[0] + width * rm;
    out->mom_x = r[1] + width * rx;
    out->mom_y = r[2];
    out->tiles = c->ntx * c->nty;
    out->near_tiles = 0;
    if (c->marks_valid) {
        // tiles of the current parity with a non-empty covering vertex range
        std::vector<int> tv(4 * nblk);
        if ((s = d2h(c, tv.data(), c->off_near + 16 * nblk * c->par, 16 * nblk))) return s;
        for (size_t t = 0; t < nblk; t++) out->near_tiles += (tv[4 * t + 1] | tv[4 * t + 3]) != 0;
    }
    if (cnt != c->step) return fail(c, CAPIB_E_STATE, "device step counter %lld != %lld", cnt, c->step);
    if (err) return fail(c, CAPIB_E_UNSTABLE, "device error flags 0x%x", err);
    return CAPIB_OK;
}

capib_status capib_diagnostics(capib_ctx *c, capib_diag *out) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!out) return fail(c, CAPIB_E_ARG, "null output");
    HIPCHK(c, launch_diag(c->d, c->par, c->stream));
    double r[3];
    const size_t nblk = (size_t)c->ntx * c->nty;
    if ((s = d2h(c, r, c->off_red + 3 * nblk * 8, 24))) return s;
    return diag_finish(c, r, out);
}

// ---- diagnostics without the workspace's reduction region --------------------------
// The per-tile FP64 partials of capib_diagnostics live in a fixed array in
// device memory of the library itself.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is handed to kernels and copies.
static __device__ __align__(256) double scratch[CAPIB_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[MAX_DEVICES] = {};

static capib_status scratch_on_device(capib_ctx *c, double **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device < 0 || c->device >= MAX_DEVICES) return fail(c, CAPIB_E_ARG, "device %d out of range", c->device);
    if (!g_scratch_ptr[c->device]) {
        int cur = 0;
        HIPCHK(c, hipGetDevice(&cur));
        if (cur != c->device) HIPCHK(c, hipSetDevice(c->device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != c->device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(c, CAPIB_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", c->device,
                        hipGetErrorString(e));
        g_scratch_ptr[c->device] = (double *)p;
    }
    *out = g_scratch_ptr[c->device];
    return CAPIB_OK;
}

capib_status capib_diagnostics_noalloc(capib_ctx *c, capib_diag *out) {
    if (!c) return CAPIB_E_ARG;
    const size_t nblk = (size_t)c->ntx * c->nty;
    const size_t need = (3 * nblk + 3) * sizeof(double);
    if (need > CAPIB_NOALLOC_SCRATCH_BYTES)
        return fail(c, CAPIB_E_CAPACITY, "lattice of %zu tiles needs %zu bytes of reduction scratch, above the %zu of "
                    "the allocation-free diagnostics (at most %zu tiles of 64x4 nodes)", nblk, need,
                    (size_t)CAPIB_NOALLOC_SCRATCH_BYTES, (size_t)(CAPIB_NOALLOC_SCRATCH_BYTES / sizeof(double) - 3) / 3);
    capib_status s = need_ws(c);
    if (s) return s;
    if (!out) return fail(c, CAPIB_E_ARG, "null output");
    double *ptr = nullptr;
    if ((s = scratch_on_device(c, &ptr))) return s;
    // the same kernels as capib_diagnostics, with the partials in the fixed
    // array (every partial and the total are rewritten by each call)
    Dev d = c->d;
    d.red = ptr;
    HIPCHK(c, launch_diag(d, c->par, c->stream));
    double r[3];
    HIPCHK(c, hipMemcpyAsync(r, ptr + 3 * nblk, sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return diag_finish(c, r, out);
}

capib_status capib_sample_members(capib_ctx *c, int32_t particle_tag, int32_t cell_tag, float *out_device) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!out_device) return fail(c, CAPIB_E_ARG, "null output");
    HIPCHK(c, launch_sample(c->d, c->par, particle_tag, cell_tag, out_device, c->stream));
    return CAPIB_OK;
}

capib_status capib_body_diagnostics(capib_ctx *c, int32_t b, capib_body_diag *out) {
    capib_status s = check_body(c, b);
    if (s) return s;
    if (!out) return fail(c, CAPIB_E_ARG, "null output");
    HIPCHK(c, launch_body_geom(c->d, c->par, c->stream));
    BodyState bs;
    if ((s = d2h(c, &bs, c->off_bs + b * sizeof(BodyState), sizeof bs))) return s;
    const BodyHost &bh = c->bodies[b];
    out->area = bs.geo[0];
    out->perimeter = bs.geo[1];
    out->cx = bs.geo[2];
    out->cy = bs.geo[3];
    out->area0 = bh.A0;
    out->perimeter0 = bh.P0;
    out->n_bound = bs.n_bound;
    out->n_bound0 = bh.n_bound0;
    out->kind = bh.kind;
    if (bh.kind == CAPIB_RIGID) {
        BodyParams bp;
        if ((s = d2h(c, &bp, c->off_bp + b * sizeof(BodyParams), sizeof bp))) return s;
        out->xc = ((double)bp.c0xh + bp.c0xl) + ((double)bs.dcxh + bs.dcxl);
        out->yc = ((double)bp.c0yh + bp.c0yl) + ((double)bs.dcyh + bs.dcyl);
        out->phi = (double)bs.phih + bs.phil;
        out->ucx = bs.u[0]; out->ucy = bs.u[1]; out->omega = bs.u[2];
    } else {
        out->xc = out->yc = out->phi = out->ucx = out->ucy = out->omega = 0;
    }
    return CAPIB_OK;
}

capib_status capib_read_body_state(capib_ctx *c, int32_t b, double *xy, double *dxy_prev, double *rigid9) {
    capib_status s = check_body(c, b);
    if (s) return s;
    const BodyHost &bh = c->bodies[b];
    const int n = bh.n;
    if (xy && (s = capib_read_vertices(c, b, xy))) return s;
    if (dxy_prev) {
        std::vector<float> a(2 * n);
        if ((s = d2h(c, a.data(), c->off_dxm + (size_t)bh.vstart * 4, n * 4))) return s;
        if ((s = d2h(c, a.data() + n, c->off_dym + (size_t)bh.vstart * 4, n * 4))) return s;
        for (int v = 0; v < n; v++) {
            dxy_prev[2 * v] = bh.kind == CAPIB_DEFORMABLE ? (double)a[v] : 0.0;
            dxy_prev[2 * v + 1] = bh.kind == CAPIB_DEFORMABLE ? (double)a[n + v] : 0.0;
        }
    }
    if (rigid9) {
        for (int k = 0; k < 9; k++) rigid9[k] = 0.0;
        if (bh.kind == CAPIB_RIGID) {
            BodyParams bp;
            BodyState bs;
            if ((s = d2h(c, &bp, c->off_bp + b * sizeof(BodyParams), sizeof bp))) return s;
            if ((s = d2h(c, &bs, c->off_bs + b * sizeof(BodyState), sizeof bs))) return s;
            rigid9[0] = ((double)bp.c0xh + bp.c0xl) + ((double)bs.dcxh + bs.dcxl);
            rigid9[1] = ((double)bp.c0yh + bp.c0yl) + ((double)bs.dcyh + bs.dcyl);
            rigid9[2] = (double)bs.phih + bs.phil;
            rigid9[3] = bs.u[0]; rigid9[4] = bs.u[1]; rigid9[5] = bs.um[0]; rigid9[6] = bs.um[1];
            rigid9[7] = bs.u[2]; rigid9[8] = bs.um[2];
        }
    }
    return CAPIB_OK;
}

capib_status capib_readout(capib_ctx *c, int32_t cell, int32_t particle, double *out3) {
    capib_status s = check_body(c, cell);
    if (s) return s;
    if ((s = check_body(c, particle))) return s;
    if (!out3) return fail(c, CAPIB_E_ARG, "null output");
    if (cell == particle) return fail(c, CAPIB_E_ARG, "the cell and the particle are the same body");
    const BodyHost &bc = c->bodies[cell], &bpart = c->bodies[particle];
    if (bc.band != bpart.band) return fail(c, CAPIB_E_ARG, "bodies %d and %d are in different members", cell, particle);
    capib_body_diag dc, dp;
    if ((s = capib_body_diagnostics(c, cell, &dc))) return s;
    if ((s = capib_body_diagnostics(c, particle, &dp))) return s;
    const double L = c->band_nx[bc.band];
    double dx = dc.cx - dp.cx;
    dx -= L * std::floor(dx / L + 0.5);   // minimum image: x is periodic
    const double dy = dc.cy - dp.cy;
    out3[0] = dc.perimeter / dc.perimeter0 - 1.0;
    out3[1] = std::sqrt(dx * dx + dy * dy);
    out3[2] = dp.n_bound0 > 0 ? (double)dp.n_bound / dp.n_bound0 : 0.0;
    return CAPIB_OK;
}

// checkpoint: header, current populations, IB region, scalars
struct CkptHeader {
    uint64_t magic;
    int32_t nx, ny, pitch, storage, nbodies, nverts, nsites, par;
    int64_t step;
    uint64_t pop_bytes, ib_bytes;
};
static const uint64_t CKPT_MAGIC = 0x31424950414331ULL;

capib_status capib_save(capib_ctx *c, void *buf, size_t *bytes) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!bytes) return fail(c, CAPIB_E_ARG, "null size");
    const size_t pop_bytes = 9 * (size_t)c->pitch * c->lat.ny * c->esize;
    const size_t total = sizeof(CkptHeader) + pop_bytes + c->ib_bytes + 16 + (size_t)c->band_rows * 8 +
                         (size_t)c->nbands * 4;
    if (!buf) { *bytes = total; return CAPIB_OK; }
    if (*bytes < total) return fail(c, CAPIB_E_ARG, "checkpoint buffer of %zu bytes needs %zu", *bytes, total);
    CkptHeader h{CKPT_MAGIC, c->lat.nx, c->lat.ny, c->pitch, c->lat.storage, c->nbodies, c->nverts, c->nsites,
                  c->par, c->step, pop_bytes, c->ib_bytes};
    char *p = (char *)buf;
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    if ((s = d2h(c, p, c->off_pop[c->par], pop_bytes))) return s;
    p += pop_bytes;
    if ((s = d2h(c, p, c->off_ib, c->ib_bytes))) return s;
    p += c->ib_bytes;
    if ((s = d2h(c, p, c->off_scal, 16))) return s;
    p += 16;
    std::memcpy(p, c->ref_u.data(), (size_t)c->band_rows * 8);
    p += (size_t)c->band_rows * 8;
    std::memcpy(p, c->band_nx.data(), (size_t)c->nbands * 4);
    *bytes = total;
    return CAPIB_OK;
}

capib_status capib_load(capib_ctx *c, const void *buf, size_t bytes) {
    capib_status s = need_ws(c);
    if (s) return s;
    if (!buf || bytes < sizeof(CkptHeader)) return fail(c, CAPIB_E_ARG, "checkpoint too short");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof h);
    const size_t pop_bytes = 9 * (size_t)c->pitch * c->lat.ny * c->esize;
    if (h.magic != CKPT_MAGIC || h.nx != c->lat.nx || h.ny != c->lat.ny || h.pitch != c->pitch ||
        h.storage != c->lat.storage || h.nbodies != c->nbodies || h.nverts != c->nverts || h.nsites != c->nsites ||
        h.pop_bytes != pop_bytes || h.ib_bytes != c->ib_bytes || (h.par != 0 && h.par != 1))
        return fail(c, CAPIB_E_ARG, "checkpoint does not match this context");
    const size_t tail = 16 + (size_t)c->band_rows * 8 + (size_t)c->nbands * 4;
    if (bytes < sizeof h + pop_bytes + c->ib_bytes + tail) return fail(c, CAPIB_E_ARG, "checkpoint truncated");
    const char *p = (const char *)buf + sizeof h;
    if (std::memcmp(p + pop_bytes + c->ib_bytes + 16 + (size_t)c->band_rows * 8, c->band_nx.data(),
                    (size_t)c->nbands * 4) != 0)
        return fail(c, CAPIB_E_ARG, "checkpoint band widths do not match this context");
    // reject non-finite populations before touching the device
    if (c->esize == 4) {
        const float *f = (const float *)p;
        for (size_t k = 0; k < pop_bytes / 4; k++)
            if (!std::isfinite(f[k])) return fail(c, CAPIB_E_ARG, "checkpoint holds a non-finite population");
    } else {
        const _Float16 *f = (const _Float16 *)p;
        for (size_t k = 0; k < pop_bytes / 2; k++)
            if (!std::isfinite((float)f[k])) return fail(c, CAPIB_E_ARG, "checkpoint holds a non-finite population");
    }
    drop_graphs(c);
    c->par = h.par;
    c->step = h.step;
    if ((s = h2d(c, c->off_pop[c->par], p, pop_bytes))) return s;
    p += pop_bytes;
    if ((s = h2d(c, c->off_ib, p, c->ib_bytes))) return s;
    p += c->ib_bytes;
    if ((s = h2d(c, c->off_scal, p, 16))) return s;
    p += 16;
    std::memcpy(c->ref_u.data(), p, (size_t)c->band_rows * 8);
    if ((s = upload_ref(c))) return s;
    // near tiles are marked afresh
    c->marks_valid = false;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CAPIB_OK;
}

capib_status capib_set_timing(capib_ctx *c, int32_t enable) {
    if (!c) return CAPIB_E_ARG;
    c->timing = enable != 0;
    return CAPIB_OK;
}

capib_status capib_read_timing(capib_ctx *c, double *ms4, int64_t *steps, int64_t *nodes4) {
    if (!c || !ms4) return CAPIB_E_ARG;
    for (int k = 0; k < 4; k++) {
        ms4[k] = c->ms[k];
        if (nodes4) nodes4[k] = c->nodes[k];
        c->ms[k] = 0;
        c->nodes[k] = 0;
    }
    if (steps) *steps = c->tsteps;
    c->tsteps = 0;
    return CAPIB_OK;
}

const char *capib_last_error(const capib_ctx *c) { return c ? c->err.c_str() : "null context"; }

void capib_destroy(capib_ctx *c) {
    if (!c) return;
    if (c->bound) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (int k = 0; k < GRAPH_STEPS; k++) {
        if (c->ev_fork[k]) (void)hipEventDestroy(c->ev_fork[k]);
        if (c->ev_join[k]) (void)hipEventDestroy(c->ev_join[k]);
    }
    if (c->side) { (void)hipStreamSynchronize(c->side); (void)hipStreamDestroy(c->side); }
    if (c->cap_side) (void)hipStreamDestroy(c->cap_side);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

}  // extern "C"
