// The load/hazard surrogate: a 37 -> 4 x 256 (GELU) -> 3 perceptron with
// bfloat16 operands and FP32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_32x32x16_bf16), its backward pass and the Adam update.
//
// Every matrix product of the forward and backward pass is one tiled GEMM
// kernel, C[M][N] = sum_k A(m, k) B(n, k), with each operand either
// k-contiguous or m/n-contiguous in memory (staging transposes through LDS
// as needed), and a fused epilogue:
//   forward hidden layer   z = acc + b (kept in FP32), a = bf16(GELU(z))
//   forward output layer   y = acc + b
//   backward through GELU  dz = bf16(acc * GELU'(z))
//   weight gradient        FP32 partial sums over a slice of the batch,
//                          reduced afterwards in a fixed order
// Internally the input is padded to 64 features and the output to 64 rows
// of W4 (zeros), batches to a multiple of 128 (zero rows masked out of the
// loss), so every GEMM dimension is a multiple of its block tile (128 x 128
// for the batch-sized products, 64 x 64 for the weight gradients).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/capib_mlp.h"

namespace capib_mlp_impl {

constexpr int KIN = CAPIB_MLP_IN, H = CAPIB_MLP_HIDDEN, KOUT = CAPIB_MLP_OUT;
constexpr int K0P = 64;            // padded input width
constexpr int NOP = 64;            // padded output rows of W4
constexpr int NL = 5;              // layers
constexpr int BT = 128;            // batch padding: a multiple of the largest block tile
constexpr int BK = 32;             // reduction step per stage
constexpr int LDS_ROW = BK + 8;    // padded LDS row (80 bytes: 16-byte aligned rows, fewer bank conflicts)
constexpr int KSPLIT = 32;         // batch slices of the weight-gradient GEMMs

// layer shapes in the padded layout: W_l is [NP[l]][KP[l]]
constexpr int KP[NL] = {K0P, H, H, H, H};
constexpr int NP[NL] = {H, H, H, H, NOP};
constexpr int KR[NL] = {KIN, H, H, H, H};   // true widths
constexpr int NR[NL] = {H, H, H, H, KOUT};

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

enum { EPI_GELU = 0, EPI_LINEAR = 1, EPI_DGELU = 2, EPI_PARTIAL = 3 };

struct GemmArgs {
    int M, N, K;                  // C is M x N; reduction over [0, K)
    const __bf16 *A;
    long long a_m, a_k;           // A(m, k) = A[m * a_m + k * a_k]
    const __bf16 *B;
    long long b_n, b_k;           // B(n, k) = B[n * b_n + k * b_k]
    int kchunk;                   // reduction length of one blockIdx.z slice
    const float *bias;            // [N] (GELU, LINEAR)
    float *cf;                    // FP32 output [M][ldc] (z, y, or partial slice z at cf + z * M * ldc)
    __bf16 *cb;                   // bfloat16 output [M][ldc] (activation or dz)
    const float *zin;             // pre-activation [M][ldc] (DGELU)
    long long ldc;
};

// erf by the rational-exponential approximation 7.1.26 of Abramowitz and
// Stegun (|error| <= 1.5e-7, far below the bfloat16 rounding that follows
// it), about a third of the instructions of a full-precision erff: the
// GELU of every hidden activation is the inference kernel's vector work.
__device__ __forceinline__ float erf_as(float x) {
    const float a = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * a);
    const float p = ((((1.061405429f * t - 1.453152027f) * t + 1.421413741f) * t - 0.284496736f) * t + 0.254829592f) * t;
    const float y = 1.0f - p * __expf(-a * a);
    return copysignf(y, x);
}
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_prime(float z) {
    return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) + z * __expf(-0.5f * z * z) * 0.39894228040143268f;
}

// One ROWS x BK operand tile: global -> registers (NV 16-byte vectors per
// thread) -> LDS as [row][k].  KC: the operand is k-contiguous (vectors
// along k); otherwise it is row-contiguous (vectors along the rows,
// scattered into LDS).
template <int ROWS, bool KC>
struct Tile {
    static constexpr int NV = ROWS * BK / 8 / 256;
    u32x4 v[NV];
    __device__ __forceinline__ void load(const __bf16 *P, long long s_row, long long s_k, int r0, int k0) {
#pragma unroll
        for (int u = 0; u < NV; u++) {
            const int e = (int)threadIdx.x + 256 * u;
            if constexpr (KC) {
                const int row = e >> 2, kq = (e & 3) * 8;
                v[u] = *(const u32x4 *)(P + (long long)(r0 + row) * s_row + (k0 + kq));
            } else {
                const int k = e / (ROWS / 8), rq = (e % (ROWS / 8)) * 8;
                v[u] = *(const u32x4 *)(P + (long long)(r0 + rq) + (long long)(k0 + k) * s_k);
            }
        }
    }
    __device__ __forceinline__ void store(__bf16 (*S)[LDS_ROW]) const {
#pragma unroll
        for (int u = 0; u < NV; u++) {
            const int e = (int)threadIdx.x + 256 * u;
            if constexpr (KC) {
                const int row = e >> 2, kq = (e & 3) * 8;
                *(u32x4 *)&S[row][kq] = v[u];
            } else {
                const int k = e / (ROWS / 8), rq = (e % (ROWS / 8)) * 8;
                const uint32_t w4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                for (int i = 0; i < 8; i++)
                    S[rq + i][k] = __builtin_bit_cast(__bf16, (unsigned short)(w4[i >> 1] >> (16 * (i & 1))));
            }
        }
    }
};

// 256 threads = 4 waves in a 2 x 2 arrangement; each wave owns a
// (BM/2) x (BN/2) block of 32 x 32 FP32 accumulators.  Two LDS buffers:
// the next k-slice is loaded into registers while the current one feeds
// the matrix cores, then stored into the other buffer.
template <int BM, int BN, bool A_KC, bool B_KC, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 32, FN = WN / 32;
    __shared__ __bf16 As[2][BM][LDS_ROW];
    __shared__ __bf16 Bs[2][BN][LDS_ROW];
    const int bm = blockIdx.x * BM, bn = blockIdx.y * BN;
    const int kbeg = blockIdx.z * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w & 1, wn = w >> 1;
    const long long a_row = A_KC ? g.a_m : 1, a_k = A_KC ? 1 : g.a_k;
    const long long b_row = B_KC ? g.b_n : 1, b_k = B_KC ? 1 : g.b_k;
    floatx16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int j = 0; j < FN; j++) acc[i][j] = floatx16{};
    Tile<BM, A_KC> ta;
    Tile<BN, B_KC> tb;
    if (kbeg < kend) {
        ta.load(g.A, a_row, a_k, bm, kbeg);
        tb.load(g.B, b_row, b_k, bn, kbeg);
        ta.store(As[0]);
        tb.store(Bs[0]);
    }
    __syncthreads();
    int cur = 0;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        const bool more = k0 + BK < kend;
        if (more) {
            ta.load(g.A, a_row, a_k, bm, k0 + BK);
            tb.load(g.B, b_row, b_k, bn, k0 + BK);
        }
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            // lane l supplies row (l mod 32) and k = 8 (l / 32) .. +7 of each 32 x 16 slice
            // (named fragments: at most two per operand)
            static_assert(FM <= 2 && FN <= 2, "at most 2 x 2 fragments per wave");
            const int r = lane & 31, kq = kk + 8 * (lane >> 5);
            const bf16x8 a0 = *(const bf16x8 *)&As[cur][WM * wm + r][kq];
            const bf16x8 b0 = *(const bf16x8 *)&Bs[cur][WN * wn + r][kq];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
            if constexpr (FN > 1) {
                const bf16x8 b1 = *(const bf16x8 *)&Bs[cur][WN * wn + 32 + r][kq];
                acc[0][FN - 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][FN - 1], 0, 0, 0);
                if constexpr (FM > 1) {
                    const bf16x8 a1 = *(const bf16x8 *)&As[cur][WM * wm + 32 + r][kq];
                    acc[FM - 1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[FM - 1][0], 0, 0, 0);
                    acc[FM - 1][FN - 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[FM - 1][FN - 1], 0, 0, 0);
                }
            } else if constexpr (FM > 1) {
                const bf16x8 a1 = *(const bf16x8 *)&As[cur][WM * wm + 32 + r][kq];
                acc[FM - 1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[FM - 1][0], 0, 0, 0);
            }
        }
        if (more) {
            ta.store(As[cur ^ 1]);
            tb.store(Bs[cur ^ 1]);
        }
        __syncthreads();
        cur ^= 1;
    }
    // accumulator element e of lane l: row 8 (e / 4) + 4 (l / 32) + (e mod 4), column l mod 32
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int j = 0; j < FN; j++) {
            const int col = bn + WN * wn + 32 * j + (lane & 31);
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int row = bm + WM * wm + 32 * i + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const long long o = (long long)row * g.ldc + col;
                const float v = acc[i][j][e];
                if (EPI == EPI_GELU) {
                    const float z = v + g.bias[col];
                    g.cf[o] = z;
                    g.cb[o] = (__bf16)gelu(z);
                } else if (EPI == EPI_LINEAR) {
                    g.cf[o] = v + g.bias[col];
                } else if (EPI == EPI_DGELU) {
                    g.cb[o] = (__bf16)(v * gelu_prime(g.zin[o]));
                } else {
                    g.cf[(long long)blockIdx.z * g.M * g.ldc + o] = v;
                }
            }
        }
}

// Inference in one kernel: a block takes 128 rows of the batch through all
// five layers with the activations resident in LDS (bfloat16, written back
// in place once every wave has read the layer's input), the weights read
// from L2, and only the input and the 3 outputs touching HBM.  Each wave
// takes all 128 rows x 64 columns (4 x 2 accumulators) of each hidden
// layer, so every weight is read from L2 once per block (a 2 x 2
// arrangement read each twice: 101 against 85 us per 65,536 rows); the
// output layer's first 32 rows of W4, 32 batch rows per wave.  Same
// rounding points as the layer-by-layer path.
constexpr int IB = 128;             // batch rows per block
constexpr int ILD = H + 8;          // LDS row stride (bfloat16 elements)

struct InferArgs {
    const float *x;
    int n;
    const __bf16 *w[NL];            // bfloat16 weights [NP][KP]
    const float *b[NL];             // FP32 biases
    float *y;
};

// One hidden layer's products for a wave: all 128 rows x 64 columns of
// S (LDS, bfloat16) times W^T (global, [256][K]); the four waves split the
// columns, so each weight is read from L2 once per block.  The weight
// fragments of the next D k-steps are in flight while the current one is
// multiplied (their L2 latency is several times one step's matrix work).
template <int K>
__device__ __forceinline__ void hidden_layer(const __bf16 (*S)[ILD], const __bf16 *W, floatx16 (&acc)[4][2], int wn,
                                             int lane) {
    constexpr int NI = K / 16, D = 6;
    const int r = lane & 31, kh = 8 * (lane >> 5);
    const __bf16 *w0 = W + (long long)(64 * wn + r) * K + kh;
    bf16x8 pb[D][2];
#pragma unroll
    for (int p = 0; p < D && p < NI; p++)
#pragma unroll
        for (int j = 0; j < 2; j++) pb[p][j] = *(const bf16x8 *)(w0 + (long long)32 * j * K + 16 * p);
#pragma unroll
    for (int it = 0; it < NI; it++) {
        const int slot = it % D;
        const bf16x8 b0 = pb[slot][0], b1 = pb[slot][1];
        if (it + D < NI) {
#pragma unroll
            for (int j = 0; j < 2; j++) pb[slot][j] = *(const bf16x8 *)(w0 + (long long)32 * j * K + 16 * (it + D));
        }
        const int kq = 16 * it + kh;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const bf16x8 a = *(const bf16x8 *)&S[32 * i + r][kq];
            acc[i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc[i][0], 0, 0, 0);
            acc[i][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc[i][1], 0, 0, 0);
        }
    }
}

__global__ __launch_bounds__(256, 2) void k_mlp_infer(InferArgs g) {
    __shared__ __bf16 S[IB][ILD];
    const int r0 = blockIdx.x * IB;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 31;
    for (int e = threadIdx.x; e < IB * K0P; e += 256) {
        const int rr = e / K0P, c = e % K0P;
        S[rr][c] = (__bf16)((r0 + rr < g.n && c < KIN) ? g.x[(long long)(r0 + rr) * KIN + c] : 0.0f);
    }
    __syncthreads();
    for (int l = 0; l < NL - 1; l++) {
        floatx16 acc[4][2];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 2; j++) acc[i][j] = floatx16{};
        if (l == 0)
            hidden_layer<K0P>(S, g.w[0], acc, w, lane);
        else
            hidden_layer<H>(S, g.w[l], acc, w, lane);
        __syncthreads();   // every wave has read this layer's input
        const float *bias = g.b[l];
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int col = 64 * w + 32 * j + r;
            const float bc = bias[col];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int e = 0; e < 16; e++) {
                    const int row = 32 * i + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                    S[row][col] = (__bf16)gelu(acc[i][j][e] + bc);
                }
        }
        __syncthreads();
    }
    // output layer
    const __bf16 *W4 = g.w[NL - 1];
    floatx16 o = floatx16{};
    for (int kk = 0; kk < H; kk += 16) {
        const int kq = kk + 8 * (lane >> 5);
        const bf16x8 a = *(const bf16x8 *)&S[32 * w + r][kq];
        const bf16x8 b = *(const bf16x8 *)(W4 + (long long)r * H + kq);
        o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, o, 0, 0, 0);
    }
    if (r < KOUT) {
        const float bc = g.b[NL - 1][r];
#pragma unroll
        for (int e = 0; e < 16; e++) {
            const int row = r0 + 32 * w + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
            if (row < g.n) g.y[(long long)row * KOUT + r] = o[e] + bc;
        }
    }
}

// x [n][37] FP32 -> X0 [np][64] bfloat16, zero padding.
__global__ void k_stage_input(const float *x, int n, int np, __bf16 *X0) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)np * K0P) return;
    const int r = (int)(i / K0P), c = (int)(i % K0P);
    X0[i] = (__bf16)((r < n && c < KIN) ? x[(long long)r * KIN + c] : 0.0f);
}

// dY = bf16(2 (y - t) / (3 n)) on the valid rows and outputs (zero
// elsewhere); per-block FP64 partial sums of (y - t)^2.
__global__ __launch_bounds__(256) void k_loss(const float *Y, const float *t, int n, int np, __bf16 *dY,
                                              double *part) {
    __shared__ double sh[256];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    double sq = 0.0;
    if (i < (long long)np * NOP) {
        const int r = (int)(i / NOP), c = (int)(i % NOP);
        float gv = 0.0f;
        if (r < n && c < KOUT) {
            const float d = Y[i] - t[(long long)r * KOUT + c];
            sq = (double)d * (double)d;
            gv = 2.0f * d / (float)(3 * n);
        }
        dY[i] = (__bf16)gv;
    }
    sh[threadIdx.x] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Fixed-order sum of nparts FP64 partials into out[0], divided by `div`.
__global__ void k_sum_parts(const double *part, int nparts, double div, double *out) {
    __shared__ double sh[256];
    double a = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) a += part[k];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] / div;
}

// out[i] = sum over z of part[z][i] (fixed order), i < count.
__global__ void k_reduce_slices(const float *part, int nz, long long count, float *out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float a = 0.0f;
    for (int z = 0; z < nz; z++) a += part[(long long)z * count + i];
    out[i] = a;
}

// Column sums of dz [rows][ncol] over row slices: part[z][c].
__global__ void k_colsum(const __bf16 *dz, int rows, int ncol, int rchunk, float *part) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    const int r0 = blockIdx.y * rchunk, r1 = min(rows, r0 + rchunk);
    float a = 0.0f;
    for (int r = r0; r < r1; r++) a += (float)dz[(long long)r * ncol + c];
    part[(long long)blockIdx.y * ncol + c] = a;
}

// Adam on the FP32 master parameters; bfloat16 copies of the weights.
__global__ void k_adam(float *p, const float *g, float *m, float *v, long long count, float lr, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

__global__ void k_to_bf16(const float *src, __bf16 *dst, long long count) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = (__bf16)src[i];
}

}  // namespace capib_mlp_impl

using namespace capib_mlp_impl;

struct capib_mlp {
    hipStream_t stream = nullptr;
    int max_batch = 0, max_np = 0;
    char *base = nullptr;
    size_t ws = 0;
    // FP32 parameter regions (padded layout) and their offsets
    size_t off_p = 0, off_g = 0, off_m = 0, off_v = 0, nparam = 0;
    size_t woff[NL]{}, boff[NL]{};        // float offsets of W_l and b_l within a parameter region
    size_t off_wb = 0, wboff[NL]{};       // bfloat16 weights
    size_t off_x0 = 0, off_z[4]{}, off_a[4]{}, off_y = 0, off_dy = 0, off_dz[2]{}, off_part = 0, off_cpart = 0;
    size_t off_lpart = 0, off_loss = 0;
    int adam_t = 0;
    bool have_grad = false;
    std::string err = "no error";
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

capib_status fail(capib_mlp *m, capib_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (m) m->err = buf;
    return s;
}

#define MLPCHK(m, call)                                                                                \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail((m), CAPIB_E_HIP, "%s: %s", #call, hipGetErrorString(e_));   \
    } while (0)

float *P(capib_mlp *m, size_t off) { return (float *)(m->base + off); }
__bf16 *Bf(capib_mlp *m, size_t off) { return (__bf16 *)(m->base + off); }

template <int BM, int BN, bool A_KC, bool B_KC, int EPI>
hipError_t gemm(capib_mlp *m, const GemmArgs &g, int nz) {
    hipLaunchKernelGGL((k_gemm<BM, BN, A_KC, B_KC, EPI>), dim3(g.M / BM, g.N / BN, nz), dim3(256), 0, m->stream, g);
    return hipGetLastError();
}

int padded(int n) { return (n + BT - 1) / BT * BT; }

// forward pass over np rows (X0 staged); keeps z and activations
capib_status forward(capib_mlp *m, int np) {
    const __bf16 *in = Bf(m, m->off_x0);
    for (int l = 0; l < NL; l++) {
        GemmArgs g{};
        g.M = np; g.N = NP[l]; g.K = KP[l];
        g.A = in; g.a_m = KP[l]; g.a_k = 1;
        g.B = Bf(m, m->off_wb + 2 * m->wboff[l]); g.b_n = KP[l]; g.b_k = 1;
        g.kchunk = KP[l];
        g.bias = P(m, m->off_p) + m->boff[l];
        if (l < NL - 1) {
            g.cf = P(m, m->off_z[l]); g.cb = Bf(m, m->off_a[l]); g.ldc = H;
            MLPCHK(m, (gemm<128, 128, true, true, EPI_GELU>(m, g, 1)));
            in = Bf(m, m->off_a[l]);
        } else {
            g.cf = P(m, m->off_y); g.ldc = NOP;
            MLPCHK(m, (gemm<128, 64, true, true, EPI_LINEAR>(m, g, 1)));
        }
    }
    return CAPIB_OK;
}

capib_status check_batch(capib_mlp *m, int n) {
    if (!m) return CAPIB_E_ARG;
    if (!m->base) return fail(m, CAPIB_E_STATE, "no workspace bound");
    if (n < 1 || n > m->max_batch) return fail(m, CAPIB_E_ARG, "batch of %d (1..%d)", n, m->max_batch);
    return CAPIB_OK;
}

capib_status refresh_bf16(capib_mlp *m) {
    const long long cnt = (long long)m->nparam;
    // the whole parameter region is converted (biases too: unused as bf16, harmless)
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, m->stream, P(m, m->off_p),
                       Bf(m, m->off_wb), cnt);
    MLPCHK(m, hipGetLastError());
    return CAPIB_OK;
}

}  // namespace

extern "C" {

capib_status capib_mlp_create(int32_t max_batch, void *hip_stream, capib_mlp **out) {
    if (!out) return CAPIB_E_ARG;
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1 << 24)) return CAPIB_E_ARG;
    capib_mlp *m = new capib_mlp();
    m->stream = (hipStream_t)hip_stream;
    m->max_batch = max_batch;
    m->max_np = padded(max_batch);
    // parameter layout (floats), padded shapes
    size_t o = 0;
    for (int l = 0; l < NL; l++) {
        m->woff[l] = o; o += (size_t)NP[l] * KP[l];
        m->boff[l] = o; o += NP[l];
    }
    m->nparam = o;
    for (int l = 0; l < NL; l++) m->wboff[l] = m->woff[l];   // bf16 copy mirrors the float layout
    const size_t np = m->max_np;
    const int nz = std::min(KSPLIT, (int)(np / BT));
    size_t w = 0;
    m->off_p = w; w = a256(w + 4 * o);
    m->off_g = w; w = a256(w + 4 * o);
    m->off_m = w; w = a256(w + 4 * o);
    m->off_v = w; w = a256(w + 4 * o);
    m->off_wb = w; w = a256(w + 2 * o);
    m->off_x0 = w; w = a256(w + 2 * np * K0P);
    for (int l = 0; l < 4; l++) { m->off_z[l] = w; w = a256(w + 4 * np * H); }
    for (int l = 0; l < 4; l++) { m->off_a[l] = w; w = a256(w + 2 * np * H); }
    m->off_y = w; w = a256(w + 4 * np * NOP);
    m->off_dy = w; w = a256(w + 2 * np * NOP);
    for (int l = 0; l < 2; l++) { m->off_dz[l] = w; w = a256(w + 2 * np * H); }
    m->off_part = w; w = a256(w + 4 * (size_t)(nz + 1) * H * H);
    m->off_cpart = w; w = a256(w + 4 * (size_t)(nz + 1) * H);
    m->off_lpart = w; w = a256(w + 8 * (np * NOP / 256 + 1));
    m->off_loss = w; w = a256(w + 8);
    m->ws = w;
    *out = m;
    return CAPIB_OK;
}

size_t capib_mlp_workspace_bytes(const capib_mlp *m) { return m ? m->ws : 0; }

capib_status capib_mlp_bind_workspace(capib_mlp *m, void *ptr, size_t bytes) {
    if (!m) return CAPIB_E_ARG;
    if (!ptr || bytes < m->ws) return fail(m, CAPIB_E_ARG, "workspace of %zu bytes needs %zu", bytes, m->ws);
    if (((uintptr_t)ptr & 255) != 0) return fail(m, CAPIB_E_ARG, "workspace not 256-byte aligned");
    m->base = (char *)ptr;
    m->adam_t = 0;
    m->have_grad = false;
    MLPCHK(m, hipMemsetAsync(m->base, 0, m->ws, m->stream));
    MLPCHK(m, hipStreamSynchronize(m->stream));
    return CAPIB_OK;
}

capib_status capib_mlp_set_params(capib_mlp *m, const float *params) {
    if (!m || !params) return CAPIB_E_ARG;
    if (!m->base) return fail(m, CAPIB_E_STATE, "no workspace bound");
    for (size_t i = 0; i < CAPIB_MLP_PARAMS; i++)
        if (!std::isfinite(params[i])) return fail(m, CAPIB_E_ARG, "non-finite parameter %zu", i);
    std::vector<float> pad(m->nparam, 0.0f);
    size_t src = 0;
    for (int l = 0; l < NL; l++) {
        for (int r = 0; r < NR[l]; r++)
            for (int c = 0; c < KR[l]; c++) pad[m->woff[l] + (size_t)r * KP[l] + c] = params[src++];
        for (int r = 0; r < NR[l]; r++) pad[m->boff[l] + r] = params[src++];
    }
    MLPCHK(m, hipMemcpyAsync(m->base + m->off_p, pad.data(), 4 * m->nparam, hipMemcpyHostToDevice, m->stream));
    MLPCHK(m, hipMemsetAsync(m->base + m->off_m, 0, 4 * m->nparam, m->stream));
    MLPCHK(m, hipMemsetAsync(m->base + m->off_v, 0, 4 * m->nparam, m->stream));
    m->adam_t = 0;
    m->have_grad = false;
    capib_status s = refresh_bf16(m);
    if (s) return s;
    MLPCHK(m, hipStreamSynchronize(m->stream));
    return CAPIB_OK;
}

static capib_status unpad(capib_mlp *m, size_t off, float *out) {
    std::vector<float> pad(m->nparam);
    MLPCHK(m, hipMemcpyAsync(pad.data(), m->base + off, 4 * m->nparam, hipMemcpyDeviceToHost, m->stream));
    MLPCHK(m, hipStreamSynchronize(m->stream));
    size_t dst = 0;
    for (int l = 0; l < NL; l++) {
        for (int r = 0; r < NR[l]; r++)
            for (int c = 0; c < KR[l]; c++) out[dst++] = pad[m->woff[l] + (size_t)r * KP[l] + c];
        for (int r = 0; r < NR[l]; r++) out[dst++] = pad[m->boff[l] + r];
    }
    return CAPIB_OK;
}

capib_status capib_mlp_get_params(capib_mlp *m, float *params) {
    if (!m || !params) return CAPIB_E_ARG;
    if (!m->base) return fail(m, CAPIB_E_STATE, "no workspace bound");
    return unpad(m, m->off_p, params);
}

capib_status capib_mlp_forward(capib_mlp *m, const float *x, int32_t n, float *y) {
    capib_status s = check_batch(m, n);
    if (s) return s;
    if (!x || !y) return fail(m, CAPIB_E_ARG, "null array");
    InferArgs g{};
    g.x = x;
    g.n = n;
    g.y = y;
    for (int l = 0; l < NL; l++) {
        g.w[l] = Bf(m, m->off_wb + 2 * m->wboff[l]);
        g.b[l] = P(m, m->off_p) + m->boff[l];
    }
    hipLaunchKernelGGL(k_mlp_infer, dim3((n + IB - 1) / IB), dim3(256), 0, m->stream, g);
    MLPCHK(m, hipGetLastError());
    return CAPIB_OK;
}

capib_status capib_mlp_loss_grad(capib_mlp *m, const float *x, const float *t, int32_t n, double *loss, float *grads) {
    capib_status s = check_batch(m, n);
    if (s) return s;
    if (!x || !t) return fail(m, CAPIB_E_ARG, "null array");
    const int np = padded(n);
    hipLaunchKernelGGL(k_stage_input, dim3((np * K0P + 255) / 256), dim3(256), 0, m->stream, x, n, np,
                       Bf(m, m->off_x0));
    MLPCHK(m, hipGetLastError());
    if ((s = forward(m, np))) return s;
    const int nlb = (np * NOP + 255) / 256;
    hipLaunchKernelGGL(k_loss, dim3(nlb), dim3(256), 0, m->stream, P(m, m->off_y), t, n, np, Bf(m, m->off_dy),
                       (double *)(m->base + m->off_lpart));
    MLPCHK(m, hipGetLastError());
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, m->stream, (const double *)(m->base + m->off_lpart), nlb,
                       (double)n * KOUT, (double *)(m->base + m->off_loss));
    MLPCHK(m, hipGetLastError());
    // batch slices of the weight-gradient GEMMs: multiples of the reduction step
    const int nz = std::min(KSPLIT, np / BT);
    const int kchunk = ((np + nz - 1) / nz + BK - 1) / BK * BK;
    const int nzz = (np + kchunk - 1) / kchunk;
    const __bf16 *dz = Bf(m, m->off_dy);   // gradient at the pre-activation of layer l
    int nb = NOP;                            // its width
    for (int l = NL - 1; l >= 0; l--) {
        const __bf16 *ain = l == 0 ? Bf(m, m->off_x0) : Bf(m, m->off_a[l - 1]);
        // dW_l = dz^T ain: M = NP[l], N = KP[l], reduction over the batch
        GemmArgs g{};
        g.M = NP[l]; g.N = KP[l]; g.K = np;
        g.A = dz; g.a_m = 1; g.a_k = nb;
        g.B = ain; g.b_n = 1; g.b_k = KP[l];
        g.kchunk = kchunk;
        g.cf = P(m, m->off_part); g.ldc = KP[l];
        MLPCHK(m, (gemm<64, 64, false, false, EPI_PARTIAL>(m, g, nzz)));
        const long long cnt = (long long)NP[l] * KP[l];
        hipLaunchKernelGGL(k_reduce_slices, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, m->stream,
                           P(m, m->off_part), nzz, cnt, P(m, m->off_g) + m->woff[l]);
        MLPCHK(m, hipGetLastError());
        // db_l = column sums of dz
        hipLaunchKernelGGL(k_colsum, dim3((NP[l] + 255) / 256, nzz), dim3(256), 0, m->stream, dz, np, NP[l], kchunk,
                           P(m, m->off_cpart));
        MLPCHK(m, hipGetLastError());
        hipLaunchKernelGGL(k_reduce_slices, dim3((NP[l] + 255) / 256), dim3(256), 0, m->stream, P(m, m->off_cpart),
                           nzz, (long long)NP[l], P(m, m->off_g) + m->boff[l]);
        MLPCHK(m, hipGetLastError());
        if (l == 0) break;
        // dz_{l-1} = bf16((dz W_l) * GELU'(z_{l-1})): C[m][k] = sum_n dz[m][n] W_l[n][k]
        __bf16 *dzn = Bf(m, m->off_dz[l & 1]);
        GemmArgs h{};
        h.M = np; h.N = KP[l]; h.K = NP[l];
        h.A = dz; h.a_m = nb; h.a_k = 1;
        h.B = Bf(m, m->off_wb + 2 * m->wboff[l]); h.b_n = 1; h.b_k = KP[l];
        h.kchunk = NP[l];
        h.cb = dzn; h.zin = P(m, m->off_z[l - 1]); h.ldc = H;
        MLPCHK(m, (gemm<128, 128, true, false, EPI_DGELU>(m, h, 1)));
        dz = dzn;
        nb = H;
    }
    m->have_grad = true;
    if (loss) MLPCHK(m, hipMemcpyAsync(loss, m->base + m->off_loss, 8, hipMemcpyDeviceToHost, m->stream));
    if (grads) {
        if ((s = unpad(m, m->off_g, grads))) return s;
    } else if (loss) {
        MLPCHK(m, hipStreamSynchronize(m->stream));
    }
    return CAPIB_OK;
}

capib_status capib_mlp_adam_step(capib_mlp *m, float lr) {
    if (!m) return CAPIB_E_ARG;
    if (!m->base) return fail(m, CAPIB_E_STATE, "no workspace bound");
    if (!m->have_grad) return fail(m, CAPIB_E_STATE, "no gradients computed");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(m, CAPIB_E_ARG, "bad learning rate");
    m->adam_t++;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, m->adam_t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, m->adam_t)));
    const long long cnt = (long long)m->nparam;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, m->stream, P(m, m->off_p),
                       P(m, m->off_g), P(m, m->off_m), P(m, m->off_v), cnt, lr, c1, c2);
    MLPCHK(m, hipGetLastError());
    return refresh_bf16(m);
}

const char *capib_mlp_last_error(const capib_mlp *m) { return m ? m->err.c_str() : "null surrogate"; }

void capib_mlp_destroy(capib_mlp *m) { delete m; }

}  // extern "C"
