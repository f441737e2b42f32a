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
//
// The kernel is latency-bound (a few thousand vertices per step against a
// lattice of a million nodes), so every per-vertex global load is issued in
// one batch at entry and the membrane then lives in LDS; reductions combine
// their operands to keep the number of barriers low.
#include "capib_dev.hpp"
#include "capib_kernels.hpp"
#include "lattice_dev.hpp"

namespace capib {

constexpr int MAX_BOX = 64;   // bounding boxes of the band's bodies cached in LDS

// Workgroup shape of the membrane kernel for membranes of at most MV
// vertices and 2 MV ligand sites: the LDS it holds scales with MV, so a run
// of small membranes keeps several workgroups resident per compute unit.
template <int MV>
struct BodyShape {
    static constexpr int MAXV = MV, MAXS = 2 * MV;
    static constexpr int BT = MV < 512 ? MV : 512;   // threads
    static constexpr int VPT = MAXV / BT;            // vertices per thread
    static constexpr int SPT = MAXS / BT;            // ligand sites per thread
};
static_assert(BodyShape<MAXV_BODY>::MAXS == MAXS_BODY, "site capacity of the largest class");

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

// Spread record of vertex g at x^n: the stencil of the velocity coupling and
// the force dV (U - u*) to spread; the near-tile sweep gathers these records
// (spreading as a gather: no atomics, sums in vertex order).
__device__ __forceinline__ void write_spread(const Dev &d, const Band &B, int g, float xh, float xl, float yh, float yl,
                                             float fx, float fy) {
    int ix0, iy0;
    float wx[4], wy[4], inv;
    stencil(d, B, xh, xl, yh, yl, false, ix0, iy0, wx, wy, inv);
    // global row of the origin; columns wrapped into the band's width, rows
    // into the band's rows when y is periodic
    d.sp_org[g] = make_int2(wrapi(ix0, B.nx), B.y0 + (d.walls ? iy0 : wrapi(iy0, B.ny)));
    d.sp_wx[g] = make_float4(wx[0] * inv, wx[1] * inv, wx[2] * inv, wx[3] * inv);
    d.sp_wy[g] = make_float4(wy[0], wy[1], wy[2], wy[3]);
    d.sp_f[g] = make_float2(fx, fy);
}

template <int PAR, bool ENS, int MV>
__device__ __forceinline__ void body_run(const Dev &d, const int b) {
    constexpr int MAXV = BodyShape<MV>::MAXV, MAXS = BodyShape<MV>::MAXS;
    constexpr int BT = BodyShape<MV>::BT, VPT = BodyShape<MV>::VPT, SPT = BodyShape<MV>::SPT;
    __shared__ float sxh[MAXV], sxl[MAXV], syh[MAXV], syl[MAXV];
    __shared__ float slen[MAXV], snlx[MAXV], snly[MAXV];
    __shared__ float snvx[MAXV], snvy[MAXV], sbend[MAXV];
    __shared__ float sSx[MAXV], sSy[MAXV];   // spring force k (l - l0) t_hat of each element
    __shared__ float sHx[MAXV], sHy[MAXV];   // half of the element's area, bond and load force
    __shared__ float sbox[MAX_BOX][4];
    __shared__ float sqxh[MAXV], sqxl[MAXV], sqyh[MAXV], sqyl[MAXV];   // another body, staged
    __shared__ double ss_bond[MAXS];  // Eq. (13) magnitude of each engaged bond (0 if free), FP64
    // rigid bodies: half of each element's bond and load force in FP64.  The
    // body's net force and moment are small residuals of large element
    // forces (side bonds pull the two sides apart along their normals), so
    // FP32 element or vertex forces would round into its motion
    __shared__ double sHd[2][MAXV];
    __shared__ double shd[BT / 64];
    __shared__ float shf[BT / 64][5];
    __shared__ double shr[BT / 64][3];

    const int tid = threadIdx.x;
    // the next step's near tiles are listed from zero by this step's sweep
    // (the interpolation has read the old count)
    if (b == 0 && tid == 0) d.ncount[PAR ^ 1] = 0;
    // this step's near-tile list, expanded for the sweep at the end of this
    // kernel: its first loads go out with the kernel's own (stale entries
    // beyond the count are valid tile indices too)
    const int nt = d.ntx * d.nty, gt = b * BT + tid;
    const int ecnt = d.ncount[PAR];
    const int etile = d.nlist[PAR][gt < nt ? gt : 0];
    const BodyParams P = d.bp[b];
    const int4 rg = b < ARG_BODIES ? d.brange[b] : make_int4(P.vstart, P.n, P.site_start, P.n_sites);
    const int n = rg.y, v0 = rg.x, ns = rg.w, s0 = rg.z, npar = PAR ^ 1;
    const long long step = *d.counter - 1;
    const bool deform = P.kind == DEFORMABLE, rigid = P.kind == RIGID;
    const Band BB = band_at<ENS>(d, P.band);
    // rigid state (centroid displacement, angle, velocities), read up front
    const float4 RS0 = *(const float4 *)&d.bs[b].dcxh;   // dcxh, dcxl, dcyh, dcyl
    const float4 RS1 = *(const float4 *)&d.bs[b].phih;   // phih, phil, cos(phi) - 1, sin(phi)
    const double2 RU0 = *(const double2 *)&d.bs[b].u[0];  // u_x, u_y at n
    const double2 RU1 = *(const double2 *)&d.bs[b].u[2];  // omega at n, u_x at n-1
    const double2 RU2 = *(const double2 *)&d.bs[b].um[1]; // u_y, omega at n-1

    // ---- every per-vertex and per-site global load of the step, issued together --
    float rxh[VPT], rxl[VPT], ryh[VPT], ryl[VPT], rl0[VPT], rth0[VPT], rdxm[VPT], rdym[VPT];
    float2 rus[VPT];
    float4 rpr[VPT];
    int2 rsr[VPT];
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BT;
        if (v >= n) continue;
        const int g = v0 + v;
        rxh[k] = d.pxh[PAR][g]; rxl[k] = d.pxl[PAR][g];
        ryh[k] = d.pyh[PAR][g]; ryl[k] = d.pyl[PAR][g];
        rl0[k] = d.l0[g]; rth0[k] = d.th0[g];
        rus[k] = d.ustar[g];
        rpr[k] = d.probe4[g];
        rdxm[k] = d.dxm[g]; rdym[k] = d.dym[g];
        rsr[k] = ns ? d.srange[g] : make_int2(0, 0);
    }
    // rigid: offsets from the centroid and positions at t = 0
    double rr0x[VPT], rr0y[VPT];
    float rx0h[VPT], rx0l[VPT], ry0h[VPT], ry0l[VPT];
    if (rigid) {
#pragma unroll
        for (int k = 0; k < VPT; k++) {
            const int v = tid + k * BT;
            if (v >= n) continue;
            const int g = v0 + v;
            rr0x[k] = d.r0x[g]; rr0y[k] = d.r0y[g];
            rx0h[k] = d.x0h[g]; rx0l[k] = d.x0l[g]; ry0h[k] = d.y0h[g]; ry0l[k] = d.y0l[g];
        }
    }
    // sites: host element, draw index, state, fraction and anchor of this
    // thread's own
    int rsh[SPT], rso[SPT], rst[SPT];
    double rsf[SPT];
    float rsah[SPT], rsal[SPT];
#pragma unroll
    for (int k = 0; k < SPT; k++) {
        const int q = tid + k * BT;
        if (q >= ns) continue;
        const int g = s0 + q;
        rsh[k] = d.s_host[g]; rso[k] = d.s_orig[g]; rst[k] = d.s_state[g];
        rsf[k] = d.s_frac[g]; rsah[k] = d.s_anh[g]; rsal[k] = d.s_anl[g];
    }
    if (tid < P.band_nb && tid < MAX_BOX)
        for (int c = 0; c < 4; c++) sbox[tid][c] = d.bs[P.band_b0 + tid].bbox[PAR][c];
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BT;
        if (v >= n) continue;
        sxh[v] = rxh[k]; sxl[v] = rxl[k]; syh[v] = ryh[k]; syl[v] = ryl[k];
    }
    const int4 erange = ((const int4 *)d.tv[PAR])[etile];   // used at the end
    __syncthreads();

    // ---- Eq. (13): bond spring magnitude of every engaged site, one site per
    // thread, so that an element's sum below reads them in site order
    if (ns) {
#pragma unroll
        for (int k = 0; k < SPT; k++) {
            const int q = tid + k * BT;
            if (q >= ns) continue;
            double bf = 0.0;
            if (rst[k]) {
                // FP64 from the hi/lo positions: the stretch is a small
                // difference of lengths close to y_eq
                const int e = rsh[k] - v0;
                const int m = (e + 1 == n) ? 0 : e + 1;
                const double xe = (double)sxh[e] + (double)sxl[e], ye = (double)syh[e] + (double)syl[e];
                const double xm = (double)sxh[m] + (double)sxl[m], ym = (double)syh[m] + (double)syl[m];
                const double f = rsf[k];
                const double dx = (xe + f * (xm - xe)) - ((double)rsah[k] + (double)rsal[k]);
                const double dy = (ye + f * (ym - ye)) + 0.5;
                bf = P.sigma64 * (sqrt(dx * dx + dy * dy) - P.yeq64);
            }
            ss_bond[q] = bf;
        }
        __syncthreads();
    }

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
        double bmd = 0.0;
        for (int s = rsr[k].x - s0; s < rsr[k].y - s0; s++) bmd += ss_bond[s];
        const float bm = (float)bmd;
        // Eqs. (14)-(15): (-p n + sigma . n) l from the element's probe
        const float4 q = rpr[k];
        const float Lx = ((q.y - q.x) * nx + q.z * ny) * len;
        const float Ly = (q.z * nx + (q.w - q.x) * ny) * len;
        sHx[l] = 0.5f * (bm * nx + Lx);
        sHy[l] = 0.5f * (bm * ny + Ly);
        if (rigid) {
            // the same in FP64, from the hi/lo positions
            const double txd = ((double)sxh[m] - (double)rxh[k]) + ((double)sxl[m] - (double)rxl[k]);
            const double tyd = ((double)syh[m] - (double)ryh[k]) + ((double)syl[m] - (double)ryl[k]);
            const double lend = sqrt(txd * txd + tyd * tyd), il = 1.0 / lend;
            const double nxd = tyd * il, nyd = -txd * il;
            const double Lxd = (((double)q.y - (double)q.x) * nxd + (double)q.z * nyd) * lend;
            const double Lyd = ((double)q.z * nxd + ((double)q.w - (double)q.x) * nyd) * lend;
            sHd[0][l] = 0.5 * (bmd * nxd + Lxd);
            sHd[1][l] = 0.5 * (bmd * nyd + Lyd);
        }
    }
    apart = wave_total_d(apart);
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

    // ---- Eq. (12): repulsion from the vertices of other bodies within the cut-off -------
    // A body whose box (of x^n) comes within the cut-off of this body's box is
    // staged in LDS; every vertex near that box then scans it.  rep[k] is the
    // summed magnitude, applied along the vertex normal.
    float rep[VPT];
#pragma unroll
    for (int k = 0; k < VPT; k++) rep[k] = 0.0f;
    if (P.kind != FIXED) {
        // only bodies of the same band interact; they are numbered
        // contiguously from P.band_b0
        const float L = (float)BB.nx, cut = d.rep_cut, cut2 = cut * cut;
        float ob[4];
        for (int q = 0; q < 4; q++) ob[q] = b - P.band_b0 < MAX_BOX ? sbox[b - P.band_b0][q] : d.bs[b].bbox[PAR][q];
        const int cend = P.band_b0 + P.band_nb;
        for (int c0 = P.band_b0; c0 < cend; c0 += 64) {
            // candidate bodies, one lane each; every wave forms the same mask
            const int cl = c0 + (tid & 63);
            bool close = false;
            if (cl < cend && cl != b) {
                float bq[4];
                for (int q = 0; q < 4; q++) bq[q] = cl - P.band_b0 < MAX_BOX ? sbox[cl - P.band_b0][q] : d.bs[cl].bbox[PAR][q];
                float dcc = 0.5f * (ob[0] + ob[1]) - 0.5f * (bq[0] + bq[1]);
                dcc -= L * rintf(dcc / L);
                // NaN boxes fail both distance tests and are scanned
                close = !(fabsf(dcc) > 0.5f * (ob[1] - ob[0]) + 0.5f * (bq[1] - bq[0]) + cut + 1.0f) &&
                        !(ob[3] < bq[2] - cut - 1.0f || ob[2] > bq[3] + cut + 1.0f);
            }
            unsigned long long mm = __ballot(close);
            while (mm) {
                const int c = c0 + __ffsll((long long)mm) - 1;
                mm &= mm - 1ull;
                float bb[4];
                for (int q = 0; q < 4; q++) bb[q] = c - P.band_b0 < MAX_BOX ? sbox[c - P.band_b0][q] : d.bs[c].bbox[PAR][q];
                const int cs = d.bp[c].vstart, cn = d.bp[c].n;
                __syncthreads();   // the staging arrays are free
                for (int u = tid; u < cn; u += BT) {
                    sqxh[u] = d.pxh[PAR][cs + u]; sqxl[u] = d.pxl[PAR][cs + u];
                    sqyh[u] = d.pyh[PAR][cs + u]; sqyl[u] = d.pyl[PAR][cs + u];
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < VPT; k++) {
                    const int v = tid + k * BT;
                    if (v >= n) continue;
                    const float myx = rxh[k] + rxl[k], myy = ryh[k] + ryl[k];
                    float dxc = myx - 0.5f * (bb[0] + bb[1]);
                    dxc -= L * rintf(dxc / L);
                    if (fabsf(dxc) > 0.5f * (bb[1] - bb[0]) + cut + 0.5f) continue;
                    if (myy < bb[2] - cut - 0.5f || myy > bb[3] + cut + 0.5f) continue;
                    for (int u = 0; u < cn; u++) {
                        float ddx = (rxh[k] - sqxh[u]) + (rxl[k] - sqxl[u]);
                        ddx -= L * rintf(ddx / L);
                        const float ddy = (ryh[k] - sqyh[u]) + (ryl[k] - sqyl[u]);
                        const float r2 = ddx * ddx + ddy * ddy;
                        if (r2 < cut2) {
                            const float dd = fmaxf(sqrtf(r2), d.rep_dmin);
                            rep[k] += d.rep_pref / (dd * dd * sqrtf(dd));
                        }
                    }
                }
            }
        }
    }

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
        fx -= rep[k] * snvx[v];
        fy -= rep[k] * snvy[v];
        fvx[k] = fx;
        fvy[k] = fy;
        d.force[v0 + v] = make_float2(fx, fy);
    }

    // ---- integration (Eqs. 16-20), direct forcing and spreading at x^n -----------------
    float nxh[VPT], nxl[VPT], nyh[VPT], nyl[VPT];
    if (rigid) {
        const double c1 = RS1.z, sphi = RS1.w;   // rotation by the stored angle
        // total force and moment about the centroid in FP64: each vertex's
        // force from the FP64 element forces (half of each adjacent
        // element's) and its repulsion, its arm R(phi) r0 from the FP64 offsets
        double Fx = 0.0, Fy = 0.0, M = 0.0;
#pragma unroll
        for (int k = 0; k < VPT; k++) {
            const int v = tid + k * BT;
            if (v >= n) continue;
            const int p = (v == 0) ? n - 1 : v - 1;
            const double fx = (sHd[0][v] + sHd[0][p]) - (double)rep[k] * (double)snvx[v];
            const double fy = (sHd[1][v] + sHd[1][p]) - (double)rep[k] * (double)snvy[v];
            const double armx = rr0x[k] + (c1 * rr0x[k] - sphi * rr0y[k]);
            const double army = rr0y[k] + (sphi * rr0x[k] + c1 * rr0y[k]);
            Fx += fx;
            Fy += fy;
            M += armx * fy - army * fx;
        }
        Fx = wave_total_d(Fx);
        Fy = wave_total_d(Fy);
        M = wave_total_d(M);
        if ((tid & 63) == 0) { shr[tid >> 6][0] = Fx; shr[tid >> 6][1] = Fy; shr[tid >> 6][2] = M; }
        __syncthreads();
        // every thread sums the wave partials in the same order and takes
        // the same rigid update (no second barrier); thread 0 stores it.
        // Waves past the last vertex hold +0 and are left out.
        const int nw = min(BT / 64, (n + 63) / 64);
        Fx = 0.0; Fy = 0.0; M = 0.0;
        for (int w = 0; w < nw; w++) { Fx += shr[w][0]; Fy += shr[w][1]; M += shr[w][2]; }
        // Eqs. (19)-(20) in FP64: u^{n+1} = 2/3 (2 u^n - u^{n-1}/2 + F/m)
        const double uxd = (2.0 / 3.0) * (2.0 * RU0.x - 0.5 * RU1.y + Fx * (double)P.inv_mass);
        const double uyd = (2.0 / 3.0) * (2.0 * RU0.y - 0.5 * RU2.x + Fy * (double)P.inv_mass);
        const double omd = (2.0 / 3.0) * (2.0 * RU1.x - 0.5 * RU2.y + M * (double)P.inv_inertia);
        const float ux = (float)uxd, uy = (float)uyd, om = (float)omd;
        float dcxh = RS0.x, dcxl = RS0.y, dcyh = RS0.z, dcyl = RS0.w, phih = RS1.x, phil = RS1.y;
        df_add(dcxh, dcxl, ux);
        df_add(dcyh, dcyl, uy);
        df_add(phih, phil, om);
        if (tid == 0) {
            BodyState &S = d.bs[b];
            *(float4 *)&S.dcxh = make_float4(dcxh, dcxl, dcyh, dcyl);
            S.phih = phih;
            S.phil = phil;
            *(double2 *)&S.u[0] = make_double2(uxd, uyd);
            *(double2 *)&S.u[2] = make_double2(omd, RU0.x);   // omega, then u_x of the step before
            *(double2 *)&S.um[1] = make_double2(RU0.y, RU1.x);
        }
        const float srig[7] = {ux, uy, om, dcxh, dcxl, dcyh, dcyl};
        const float ph = phih + phil;
        // cos(ph) - 1 = -2 sin^2(ph/2) (no cancellation at small angles) and
        // sin(ph) = 2 sin(ph/2) cos(ph/2), kept for the next step
        float sh2, ch2;
        sincosf(0.5f * ph, &sh2, &ch2);
        const float c1n = -2.0f * sh2 * sh2, sn = 2.0f * sh2 * ch2;
        if (tid == 0) *(float2 *)&d.bs[b].rot = make_float2(c1n, sn);
#pragma unroll
        for (int k = 0; k < VPT; k++) {
            const int v = tid + k * BT;
            if (v >= n) continue;
            // (R - I) r0 from the FP64 offsets: its size is phi |r0|, so the
            // offsets' own rounding must stay far below phi's
            const float rx = (float)rr0x[k], ry = (float)rr0y[k];
            const float drx = (float)((double)c1n * rr0x[k] - (double)sn * rr0y[k]);
            const float dry = (float)((double)sn * rr0x[k] + (double)c1n * rr0y[k]);
            float xh = rx0h[k], xl = rx0l[k], yh = ry0h[k], yl = ry0l[k];
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
            write_spread(d, BB, v0 + v, rxh[k], rxl[k], ryh[k], ryl[k], dV * (Ux - rus[k].x), dV * (Uy - rus[k].y));
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
            write_spread(d, BB, v0 + v, rxh[k], rxl[k], ryh[k], ryl[k], dV * (Ux - rus[k].x), dV * (Uy - rus[k].y));
        }
        if (bad) atomicOr(d.err, FLAG_NONFINITE_IB);
    }
    __syncthreads();   // every thread has read x^n from LDS

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

    // ---- probe points of x^{n+1} for the next step's interpolation ------------------------
#pragma unroll
    for (int k = 0; k < VPT; k++) {
        const int v = tid + k * BT;
        if (v >= n) continue;
        const int m = (v + 1 == n) ? 0 : v + 1;
        d.pprobe[npar][v0 + v] = probe_point(d, nxh[k], nxl[k], nyh[k], nyl[k], sxh[m], sxl[m], syh[m], syl[m]);
    }

    // ---- bond kinetics at x^{n+1} --------------------------------------------------------
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < SPT; k++) {
        const int q = tid + k * BT;
        if (q >= ns) continue;
        const int e = rsh[k] - v0;
        const int m = (e + 1 == n) ? 0 : e + 1;
        // the site at x^{n+1}, FP64 from the hi/lo positions (its gap and
        // stretch are small differences)
        const double xe = (double)sxh[e] + (double)sxl[e], ye = (double)syh[e] + (double)syl[e];
        const double xm = (double)sxh[m] + (double)sxl[m], ym = (double)syh[m] + (double)syl[m];
        const double f = rsf[k];
        const double xs = xe + f * (xm - xe), ys = ye + f * (ym - ye);
        const uint32_t w = philox_w0((uint32_t)step, (uint32_t)rso[k], (uint32_t)((unsigned long long)step >> 32),
                                     0u, P.seed_lo, P.seed_hi);
        const float r = (float)(w >> 8) * (1.0f / 16777216.0f);
        int st = rst[k];
        if (st) {
            const double dx = xs - ((double)rsah[k] + (double)rsal[k]);
            const double dy = ys + 0.5;
            const float stretch = (float)fabs(sqrt(dx * dx + dy * dy) - P.yeq64);
            const float Pr = -expm1f(-P.kr0 * expf(stretch / P.lb));
            if (r < Pr) st = 0;
        } else {
            if (ys + 0.5 < P.ycr64) {
                const float Pf = -expm1f(-P.kf);
                if (r < Pf) {
                    st = 1;
                    const float ah = (float)xs;
                    d.s_anh[s0 + q] = ah;
                    d.s_anl[s0 + q] = (float)(xs - (double)ah);
                }
            }
        }
        if (st != rst[k]) d.s_state[s0 + q] = st;
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
    const float fc = wave_total((float)cnt, OpAdd());
    xmin = wave_total(xmin, OpMin());
    xmax = wave_total(xmax, OpMax());
    ymin = wave_total(ymin, OpMin());
    ymax = wave_total(ymax, OpMax());
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

    // ---- expanded near-tile list of this step (see Dev::elist) ----------------------------
    for (int k = gt; k < ecnt; k += d.nbodies * BT) {
        const int tile = k == gt ? etile : d.nlist[PAR][k];
        const int4 r = k == gt ? erange : ((const int4 *)d.tv[PAR])[tile];
        // the ranges [lo, hi] of the two halves (hi = -1: none) in index
        // order, merged when they overlap
        int lo0 = d.nverts - r.x, hi0 = r.y - 1, lo1 = d.nverts - r.z, hi1 = r.w - 1;
        if (hi1 >= 0 && (hi0 < 0 || lo1 < lo0)) {
            const int x = lo0, y = hi0;
            lo0 = lo1; hi0 = hi1; lo1 = x; hi1 = y;
        }
        if (hi1 >= 0 && lo1 <= hi0) {
            hi0 = max(hi0, hi1);
            hi1 = -1;
        }
        const int nx = band_at<ENS>(d, ENS ? (tile / d.ntx) * TILE_Y / d.band_rows : 0).nx;
        d.elist[PAR][2 * k] = make_int4(tile, nx, lo0, hi0 - lo0 + 1);
        d.elist[PAR][2 * k + 1] = make_int4(lo1, hi1 >= 0 ? hi1 - lo1 + 1 : 0, 0, 0);
    }
}

// Near tiles of the current positions (before the first step, after a
// checkpoint is loaded or membranes are added): flags, vertex ranges and
// list of parity par, which must be clear.
__global__ __launch_bounds__(256) void k_mark(Dev d, int par) {
    const int v = blockIdx.x * 256 + threadIdx.x;
    if (v >= d.nverts) return;
    int tl[9];
    const int info = d.vinfo[v];
    const Band B = band_of(d, info >> 1);
    const int c = stencil_tiles(d, B, d.pxh[par][v], d.pxl[par][v], d.pyh[par][v], d.pyl[par][v], tl);
    const int vn = d.vnext[v];
    d.pprobe[par][v] = probe_point(d, d.pxh[par][v], d.pxl[par][v], d.pyh[par][v], d.pyl[par][v], d.pxh[par][vn],
                                   d.pxl[par][vn], d.pyh[par][vn], d.pyl[par][vn]);
    for (int q = 0; q < c; q++) {
        note_cover(d, par, tl[q], v, info & 1);
        if (atomicExch(&d.tnear[par][tl[q]], 1) == 0) d.nlist[par][atomicAdd(&d.ncount[par], 1)] = tl[q];
    }
}

hipError_t launch_mark(const Dev &d, int par, hipStream_t st) {
    if (d.nverts == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark, dim3((d.nverts + 255) / 256), dim3(256), 0, st, d, par);
    return hipGetLastError();
}

template <int PAR, bool ENS, int MV>
__global__ __launch_bounds__(BodyShape<MV>::BT) void k_body(Dev d) {
    body_run<PAR, ENS, MV>(d, blockIdx.x);
}

// The membrane workgroups first, then (from the next multiple of 8, so that
// blockIdx & 7 is a far workgroup's XCD) BT / 256 far-tile candidates per
// workgroup: the first far_share_len(len, pct) of each XCD's run of ncand
// candidates, in order.  On a lattice small enough that one sweep after the
// membrane phase beats a second stream, these far tiles stream on the
// compute units that the few membrane workgroups leave idle.
template <typename T, int PAR, bool ENS, int MV>
__global__ __launch_bounds__(BodyShape<MV>::BT) void k_body_far(Dev d, int ncand, int pct) {
    const int f0 = round_up8(d.nbodies);
    if ((int)blockIdx.x < f0) {
        if ((int)blockIdx.x < d.nbodies) body_run<PAR, ENS, MV>(d, blockIdx.x);
        return;
    }
    constexpr int TPW = BodyShape<MV>::BT / LAT_THREADS;
    const XcdRun run = xcd_run(blockIdx.x & 7, ncand);
    const int c = (((int)blockIdx.x - f0) >> 3) * TPW + (int)(threadIdx.x / LAT_THREADS);
    if (c < far_share_len(run.len, pct)) far_tile<T, PAR, ENS>(d, run.start + c, threadIdx.x % LAT_THREADS);
}

// Default share of the far-tile candidates swept by the membrane launch, in
// percent (measured on 3840 x 240, step time against the share in steps of
// 5-10 %: the membrane kernel's 8-10 us hide about this much streaming; FP16
// tiles cost half the bytes); the autotuner picks it per workload.
constexpr int FAR_SHARE_FP32 = 65, FAR_SHARE_FP16 = 80;

int default_far_share(int storage) { return storage == 0 ? FAR_SHARE_FP32 : FAR_SHARE_FP16; }

int body_far_share(const Dev &d) { return d.far_share; }

template <typename T, int MV>
static void go_body_far(const Dev &d, int par, bool ens, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    constexpr int TPW = BodyShape<MV>::BT / LAT_THREADS;
    const int ncand = ens ? d.nlive : d.ntx * d.nty;
    const int pct = body_far_share(d);
    // the longest run's share (runs differ by at most one candidate)
    const int most = far_share_len(xcd_run(0, ncand).len, pct);
    const dim3 g(std::max(1, round_up8(d.nbodies) + 8 * ((most + TPW - 1) / TPW))), t(BodyShape<MV>::BT);
    if (par)
        hipExtLaunchKernelGGL(ens ? k_body_far<T, 1, true, MV> : k_body_far<T, 1, false, MV>, g, t, 0, st, e0, e1, 0,
                              d, ncand, pct);
    else
        hipExtLaunchKernelGGL(ens ? k_body_far<T, 0, true, MV> : k_body_far<T, 0, false, MV>, g, t, 0, st, e0, e1, 0,
                              d, ncand, pct);
}

template <typename T>
static void body_far_of(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const bool ens = d.nbands > 1;
    if (d.body_mv <= 256)
        go_body_far<T, 256>(d, par, ens, st, e0, e1);
    else if (d.body_mv <= 512)
        go_body_far<T, 512>(d, par, ens, st, e0, e1);
    else
        go_body_far<T, MAXV_BODY>(d, par, ens, st, e0, e1);
}

hipError_t launch_body_far(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (d.storage == 0)
        body_far_of<float>(d, par, st, e0, e1);
    else
        body_far_of<_Float16>(d, par, st, e0, e1);
    return hipGetLastError();
}

template <int MV>
static void go_body(const Dev &d, int par, bool ens, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const dim3 g(d.nbodies), t(BodyShape<MV>::BT);
    if (par)
        hipExtLaunchKernelGGL(ens ? k_body<1, true, MV> : k_body<1, false, MV>, g, t, 0, st, e0, e1, 0, d);
    else
        hipExtLaunchKernelGGL(ens ? k_body<0, true, MV> : k_body<0, false, MV>, g, t, 0, st, e0, e1, 0, d);
}

hipError_t launch_body(const Dev &d, int par, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (d.nbodies == 0) {
        // keep the event pair meaningful for callers that time every phase
        if (e0) { hipError_t e = hipEventRecord(e0, st); if (e != hipSuccess) return e; }
        if (e1) return hipEventRecord(e1, st);
        return hipSuccess;
    }
    // instantiated per step parity, kind of lattice and membrane size class
    const bool ens = d.nbands > 1;
    if (d.body_mv <= 256)
        go_body<256>(d, par, ens, st, e0, e1);
    else if (d.body_mv <= 512)
        go_body<512>(d, par, ens, st, e0, e1);
    else
        go_body<MAXV_BODY>(d, par, ens, st, e0, e1);
    return hipGetLastError();
}

}  // namespace capib
