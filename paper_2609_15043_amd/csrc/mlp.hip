// Surrogate network of the coil-plasma response: three GELU hidden layers
// of width H between 32-column (padded) inputs and outputs.  BF16 weights
// and activations on the matrix cores (gfx950's v_mfma_f32_16x16x32_bf16,
// FP32 accumulation), FP32 master weights, Adam (Kingma & Ba) in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/phasorpic.h"

namespace {

constexpr int PAD = 32;        // padded input / output width
constexpr int TM = 64, TN = 64, TK = 32, KP = 40;   // GEMM tile and LDS row pitch (bf16 elements)
constexpr int SPLITK = 16;     // K splits of the weight-gradient products

// MFMA operands: eight BF16 values along K per lane (lane l holds row or
// column l % 16 and the K octet l / 16 of a 32-wide slice; A and B take the
// same K order, so the dot products do not depend on it)
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

template <typename T> __device__ __forceinline__ uint16_t to_bf(T v);
template <> __device__ __forceinline__ uint16_t to_bf<uint16_t>(uint16_t v) { return v; }
template <> __device__ __forceinline__ uint16_t to_bf<float>(float v) { return f2bf(v); }

enum Epi { EPI_GELU = 0, EPI_LINEAR = 1, EPI_DGELU = 2, EPI_STORE = 3 };

// C = A B with A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn]; both
// operands are rounded to BF16 when staged (FP32 sources) and multiplied
// on the matrix cores with FP32 accumulation.
struct GemmArgs {
    int M, N, K;
    const void *A;
    int64_t sam, sak;
    const void *B;
    int64_t sbk, sbn;
    const float *bias;     // EPI_GELU, EPI_LINEAR
    float *C;              // FP32 result (or K-split partials for EPI_STORE)
    int64_t ldc;
    uint16_t *Abf;         // EPI_GELU: BF16 activation
    int64_t ldabf;
    const float *Zin;      // EPI_DGELU: pre-activation
    int64_t ldz;
    int ksplit;            // EPI_STORE: number of K splits (grid.z); partial z at C + z * M * ldc
};

// Store of a wave's 32 x 32 accumulators (2 x 2 MFMA blocks) at (r0, c0)
// with the fused epilogue.  D of a 16x16 block: lane l holds rows
// 4 (l / 16) + r, column l % 16.
template <int EPI> __device__ __forceinline__ void gemm_epilogue(const GemmArgs &g, const floatx4 (&acc)[2][2], int r0,
                                                                 int c0, int lane)
{
    float *C = g.C;
    if (EPI == EPI_STORE && g.ksplit > 1) C += (int64_t)blockIdx.z * g.M * g.ldc;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + 16 * i + 4 * (lane >> 4) + r;
                const int col = c0 + 16 * j + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                const float v = acc[i][j][r];
                if (EPI == EPI_GELU) {
                    const float z = v + g.bias[col];
                    C[(int64_t)row * g.ldc + col] = z;
                    g.Abf[(int64_t)row * g.ldabf + col] = f2bf(gelu(z));
                } else if (EPI == EPI_LINEAR) {
                    C[(int64_t)row * g.ldc + col] = v + g.bias[col];
                } else if (EPI == EPI_DGELU) {
                    C[(int64_t)row * g.ldc + col] = v * gelu_grad(g.Zin[(int64_t)row * g.ldz + col]);
                } else {
                    C[(int64_t)row * g.ldc + col] = v;
                }
            }
}

template <typename TA, typename TB, int EPI> __global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[TM * KP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN * KP];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    int kb = 0, ke = g.K;
    if (EPI == EPI_STORE && g.ksplit > 1) {
        const int per = (g.K + g.ksplit - 1) / g.ksplit;
        kb = blockIdx.z * per;
        ke = min(g.K, kb + per);
    }
    const TA *A = static_cast<const TA *>(g.A);
    const TB *B = static_cast<const TB *>(g.B);
    floatx4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bool a_mfast = g.sam == 1, b_nfast = g.sbn == 1;
    for (int k0 = kb; k0 < ke; k0 += TK) {
        for (int e = t; e < TM * TK; e += 256) {
            const int mm = a_mfast ? e % TM : e / TK, kk = a_mfast ? e / TM : e % TK;
            const int m = m0 + mm, k = k0 + kk;
            As[mm * KP + kk] = (m < g.M && k < ke) ? to_bf<TA>(A[(int64_t)m * g.sam + (int64_t)k * g.sak]) : 0;
        }
        for (int e = t; e < TN * TK; e += 256) {
            const int nn = b_nfast ? e % TN : e / TK, kk = b_nfast ? e / TN : e % TK;
            const int n = n0 + nn, k = k0 + kk;
            Bs[nn * KP + kk] = (n < g.N && k < ke) ? to_bf<TB>(B[(int64_t)k * g.sbk + (int64_t)n * g.sbn]) : 0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; kk += 32) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x8 *>(&As[(wm + 16 * i + (lane & 15)) * KP + kk + 8 * (lane >> 4)]);
                b[i] = *reinterpret_cast<const bf16x8 *>(&Bs[(wn + 16 * i + (lane & 15)) * KP + kk + 8 * (lane >> 4)]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    gemm_epilogue<EPI>(g, acc, m0 + wm, n0 + wn, lane);
}

// Tile kernel with vector staging, for operands contiguous along K (A: the
// activations or the FP32 gradient; B: the weights, contiguous along K in
// the forward products and along N in the activation gradients).  Each
// thread moves 16-byte vectors (8 BF16 values; FP32 sources are rounded to
// BF16 as in k_gemm), the K slice is VTK wide, and the next slice's loads
// are issued before the current slice's products, so a hidden layer takes
// two dependent memory round trips instead of eight.  Same products and
// epilogues as k_gemm.
constexpr int VTK = 128, VKP = VTK + 8;
template <typename TA> __device__ __forceinline__ uint4 load8_bf(const TA *p);
template <> __device__ __forceinline__ uint4 load8_bf<uint16_t>(const uint16_t *p)
{
    return *reinterpret_cast<const uint4 *>(p);
}
template <> __device__ __forceinline__ uint4 load8_bf<float>(const float *p)
{
    const float4 a = *reinterpret_cast<const float4 *>(p), b = *reinterpret_cast<const float4 *>(p + 4);
    uint4 r;
    r.x = (uint32_t)f2bf(a.x) | ((uint32_t)f2bf(a.y) << 16);
    r.y = (uint32_t)f2bf(a.z) | ((uint32_t)f2bf(a.w) << 16);
    r.z = (uint32_t)f2bf(b.x) | ((uint32_t)f2bf(b.y) << 16);
    r.w = (uint32_t)f2bf(b.z) | ((uint32_t)f2bf(b.w) << 16);
    return r;
}

template <typename TA, int EPI, bool AK, bool BK> __global__ __launch_bounds__(256) void k_gemm_v(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[TM * VKP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN * VKP];
    constexpr int NV = TM * VTK / 8 / 256;   // vectors per thread and operand
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const TA *A = static_cast<const TA *>(g.A);
    const uint16_t *B = static_cast<const uint16_t *>(g.B);
    const uint4 zero{0u, 0u, 0u, 0u};
    // K range: the whole of K, or this block's split of it
    int kb = 0, ke = g.K;
    if (EPI == EPI_STORE && g.ksplit > 1) {
        const int per = (g.K + g.ksplit - 1) / g.ksplit;
        kb = blockIdx.z * per;
        ke = min(g.K, kb + per);
    }
    uint4 ra[NV], rb[NV];
    auto load = [&](int k0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = t + 256 * v;
            if (AK) {
                const int r = e / (VTK / 8), k8 = (e % (VTK / 8)) * 8;
                const int m = m0 + r, k = k0 + k8;
                ra[v] = (m < g.M && k < ke) ? load8_bf<TA>(A + (int64_t)m * g.sam + k) : zero;
            } else {
                const int kk = e / (TM / 8), m8 = (e % (TM / 8)) * 8;
                const int m = m0 + m8, k = k0 + kk;
                ra[v] = (m < g.M && k < ke) ? load8_bf<TA>(A + (int64_t)k * g.sak + m) : zero;
            }
            if (BK) {
                const int r = e / (VTK / 8), k8 = (e % (VTK / 8)) * 8;
                const int n = n0 + r, k = k0 + k8;
                rb[v] = (n < g.N && k < ke) ? load8_bf<uint16_t>(B + (int64_t)n * g.sbn + k) : zero;
            } else {
                const int kk = e / (TN / 8), n8 = (e % (TN / 8)) * 8;
                const int n = n0 + n8, k = k0 + kk;
                rb[v] = (n < g.N && k < ke) ? load8_bf<uint16_t>(B + (int64_t)k * g.sbk + n) : zero;
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = t + 256 * v;
            const int r = e / (VTK / 8), k8 = (e % (VTK / 8)) * 8;
            if (AK) {
                *reinterpret_cast<uint4 *>(&As[r * VKP + k8]) = ra[v];
            } else {
                const int kk = e / (TM / 8), m8 = (e % (TM / 8)) * 8;
                const uint32_t w[4] = {ra[v].x, ra[v].y, ra[v].z, ra[v].w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    As[(m8 + 2 * q) * VKP + kk] = (uint16_t)(w[q] & 0xFFFFu);
                    As[(m8 + 2 * q + 1) * VKP + kk] = (uint16_t)(w[q] >> 16);
                }
            }
            if (BK) {
                *reinterpret_cast<uint4 *>(&Bs[r * VKP + k8]) = rb[v];
            } else {
                const int kk = e / (TN / 8), n8 = (e % (TN / 8)) * 8;
                const uint32_t w[4] = {rb[v].x, rb[v].y, rb[v].z, rb[v].w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    Bs[(n8 + 2 * q) * VKP + kk] = (uint16_t)(w[q] & 0xFFFFu);
                    Bs[(n8 + 2 * q + 1) * VKP + kk] = (uint16_t)(w[q] >> 16);
                }
            }
        }
    };
    floatx4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    load(kb);
    for (int k0 = kb; k0 < ke; k0 += VTK) {
        store();
        __syncthreads();
        if (k0 + VTK < ke) load(k0 + VTK);
        const int kend = ke - k0;   // K blocks past the end hold zeros only
#pragma unroll
        for (int kk = 0; kk < VTK; kk += 32) {
            if (kk >= kend) break;
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x8 *>(&As[(wm + 16 * i + (lane & 15)) * VKP + kk + 8 * (lane >> 4)]);
                b[i] = *reinterpret_cast<const bf16x8 *>(&Bs[(wn + 16 * i + (lane & 15)) * VKP + kk + 8 * (lane >> 4)]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    gemm_epilogue<EPI>(g, acc, m0 + wm, n0 + wn, lane);
}

// Products with a few rows (inference inside the surrogate-assisted period
// update, batch 1): the tile kernel would stream K in eight dependent slices
// for one useful row.  One workgroup per row stages the BF16 activations in
// LDS as floats; each thread takes one output column and reads its weight
// row (contiguous, W[n][k]) in 16-byte loads.  Products of BF16 values are
// exact in FP32 and accumulate in FP32, as on the matrix cores (in another
// order).  Same epilogues as k_gemm (GELU, linear).
constexpr int GEMV_MAX_K = 1024;
constexpr int GEMV_MAX_M = 8;
template <int EPI> __global__ __launch_bounds__(256) void k_gemv(GemmArgs g)
{
    __shared__ float a[GEMV_MAX_K];
    const int m = blockIdx.y;
    const uint16_t *A = static_cast<const uint16_t *>(g.A);
    for (int k = threadIdx.x; k < g.K; k += blockDim.x) a[k] = bf2f(A[(int64_t)m * g.sam + k]);
    __syncthreads();
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const uint16_t *w = static_cast<const uint16_t *>(g.B) + (int64_t)n * g.sbn;
    float acc = 0.f;
    int k = 0;
    for (; k + 8 <= g.K; k += 8) {
        const uint4 v = *reinterpret_cast<const uint4 *>(w + k);
        const uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            acc += bf2f((uint16_t)(q[e] & 0xFFFFu)) * a[k + 2 * e];
            acc += bf2f((uint16_t)(q[e] >> 16)) * a[k + 2 * e + 1];
        }
    }
    for (; k < g.K; ++k) acc += bf2f(w[k]) * a[k];
    if (EPI == EPI_GELU) {
        const float z = acc + g.bias[n];
        g.C[(int64_t)m * g.ldc + n] = z;
        g.Abf[(int64_t)m * g.ldabf + n] = f2bf(gelu(z));
    } else {
        g.C[(int64_t)m * g.ldc + n] = acc + g.bias[n];
    }
}

// sum of the K-split partials in split order
__global__ void k_splitk_sum(const float *part, int splits, int64_t count, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * count + i];
    out[i] = s;
}

// standardised, padded BF16 input rows
__global__ void k_input(const float *x, int B, int n_in, const float *mean, const float *stdv, uint16_t *X)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * PAD) return;
    const int b = e / PAD, i = e % PAD;
    X[e] = i < n_in ? f2bf((x[(int64_t)b * n_in + i] - mean[i]) / stdv[i]) : (uint16_t)0;
}

// de-standardised outputs
__global__ void k_output(const float *Y, int B, int n_out, const float *mean, const float *stdv, float *y)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * n_out) return;
    const int b = e / n_out, o = e % n_out;
    y[e] = Y[(int64_t)b * PAD + o] * stdv[o] + mean[o];
}

// mean-squared error on standardised targets: dY = 2 (Y - T) / (B n_out) on
// the real columns (0 on the padding), per-block partial sums of (Y - T)^2
__global__ __launch_bounds__(256) void k_loss(const float *Y, const float *t, int B, int n_out, const float *mean,
                                              const float *stdv, float *dY, float *partial)
{
    __shared__ float red[256];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.f;
    if (e < B * PAD) {
        const int b = e / PAD, o = e % PAD;
        float d = 0.f;
        if (o < n_out) d = Y[e] - (t[(int64_t)b * n_out + o] - mean[o]) / stdv[o];
        dY[e] = 2.0f * d / (float)(B * n_out);
        sq = d * d;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_fold(const float *partial, int np, float scale, float *out)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < np; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// bias gradient: column sums of the BF16-rounded output gradient, in two
// passes (row chunks, then chunks in order)
constexpr int COLSUM_CHUNKS = 32;
__global__ __launch_bounds__(256) void k_colsum(const float *G, int B, int N, int64_t ld, float *partial)
{
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), grp = threadIdx.x >> 6;
    const int per = (B + COLSUM_CHUNKS - 1) / COLSUM_CHUNKS;
    const int r0 = blockIdx.y * per, r1 = min(B, r0 + per);
    float s = 0.f;
    if (c < N)
        for (int r = r0 + grp; r < r1; r += 4) s += bf2f(f2bf(G[(int64_t)r * ld + c]));
    red[grp][threadIdx.x & 63] = s;
    __syncthreads();
    if (grp == 0 && c < N)
        partial[(int64_t)blockIdx.y * N + c] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                                               red[3][threadIdx.x];
}

__global__ void k_colsum_fold(const float *partial, int N, float *out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    float s = 0.f;
    for (int z = 0; z < COLSUM_CHUNKS; ++z) s += partial[(int64_t)z * N + c];
    out[c] = s;
}

// Adam on the FP32 master parameters; refreshes the BF16 copy
__global__ void k_adam(float *p, const float *gr, float *m, float *v, uint16_t *pbf, int64_t n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float x = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = x;
    pbf[i] = f2bf(x);
}

__global__ void k_to_bf16(const float *p, uint16_t *q, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = f2bf(p[i]);
}

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct Carver {
    uint8_t *base;
    size_t off = 0;
    template <typename U> U *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        U *p = base ? reinterpret_cast<U *>(base + off) : nullptr;
        off += count * sizeof(U);
        return p;
    }
};

// Inference scratch of mlp_forward_noalloc: a file-scope device array, so
// that entry point needs no device memory from anyone.  Layout (byte
// offsets, each a multiple of 256): X [64 x 32] BF16, A_l [64 x 256] BF16 for
// the three hidden layers, Z_l [64 x 256] FP32, Y [64 x 32] FP32.  Every
// device the library runs on holds its own copy until the process ends.
constexpr int NOALLOC_MAX_BATCH = 64, NOALLOC_MAX_HIDDEN = 256;
constexpr size_t NA_X = 0, NA_A = NA_X + (size_t)NOALLOC_MAX_BATCH * PAD * 2,
                 NA_Z = NA_A + 3 * (size_t)NOALLOC_MAX_BATCH * NOALLOC_MAX_HIDDEN * 2,
                 NA_Y = NA_Z + 3 * (size_t)NOALLOC_MAX_BATCH * NOALLOC_MAX_HIDDEN * 4,
                 NOALLOC_BYTES = NA_Y + (size_t)NOALLOC_MAX_BATCH * PAD * 4;
static_assert(NA_A % 256 == 0 && NA_Z % 256 == 0 && NA_Y % 256 == 0, "scratch offsets must stay 256-aligned");

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Device address of `scratch` on device dev (in host code the array's name
// is a host-side stand-in, not a device address): looked up once per device
// with that device current, then kept.
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[MAX_DEVICES] = {};

hipError_t scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

struct mlp_ctx {
    mlp_config cfg{};
    hipStream_t stream = nullptr;
    std::string err;
    int H = 0, maxB = 0;
    void *scratch = nullptr;   // this device's static inference scratch (mlp_forward_noalloc)
    int64_t P = 0;
    // parameter layout offsets (floats)
    int64_t oW[4]{}, ob[4]{};
    float *p = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *pbf = nullptr;
    float *norm = nullptr;   // in_mean[32], in_std[32], out_mean[32], out_std[32]
    uint16_t *X = nullptr, *A[3]{};
    float *Z[3]{}, *Y = nullptr, *dY = nullptr, *D[2]{}, *part = nullptr, *colpart = nullptr, *lpart = nullptr,
          *loss = nullptr;
    int64_t step = 0;
};

namespace {

pic_status mfail(mlp_ctx *c, pic_status s, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define MCHK(ctx, expr)                                                                                \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return mfail(ctx, PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

void mlp_layout(mlp_ctx &c, Carver &cv)
{
    const int H = c.H, B = c.maxB;
    int64_t o = 0;
    const int64_t wsz[4] = {(int64_t)H * PAD, (int64_t)H * H, (int64_t)H * H, (int64_t)PAD * H};
    const int64_t bsz[4] = {H, H, H, PAD};
    for (int l = 0; l < 4; ++l) {
        c.oW[l] = o;
        o += wsz[l];
        c.ob[l] = o;
        o += bsz[l];
    }
    c.P = o;
    c.p = cv.take<float>(c.P);
    c.grad = cv.take<float>(c.P);
    c.m = cv.take<float>(c.P);
    c.v = cv.take<float>(c.P);
    c.pbf = cv.take<uint16_t>(c.P);
    c.norm = cv.take<float>(4 * PAD);
    c.X = cv.take<uint16_t>((size_t)B * PAD);
    for (int l = 0; l < 3; ++l) {
        c.A[l] = cv.take<uint16_t>((size_t)B * H);
        c.Z[l] = cv.take<float>((size_t)B * H);
    }
    c.Y = cv.take<float>((size_t)B * PAD);
    c.dY = cv.take<float>((size_t)B * PAD);
    c.D[0] = cv.take<float>((size_t)B * H);
    c.D[1] = cv.take<float>((size_t)B * H);
    c.part = cv.take<float>((size_t)SPLITK * H * H);
    c.colpart = cv.take<float>((size_t)COLSUM_CHUNKS * H);
    c.lpart = cv.take<float>(nb((int64_t)B * PAD, 256));
    c.loss = cv.take<float>(1);
}

template <typename TA, typename TB, int EPI> void gemm(mlp_ctx &c, GemmArgs g)
{
    // a few rows of a forward product (BF16 operands, weight rows contiguous
    // and 16-byte aligned): one workgroup per row
    if constexpr ((EPI == EPI_GELU || EPI == EPI_LINEAR) && sizeof(TA) == 2 && sizeof(TB) == 2) {
        if (g.M <= GEMV_MAX_M && g.K <= GEMV_MAX_K && g.sak == 1 && g.sbk == 1 && g.sbn % 8 == 0 &&
            reinterpret_cast<uintptr_t>(g.B) % 16 == 0) {
            hipLaunchKernelGGL((k_gemv<EPI>), dim3(nb(g.N, 256), g.M), dim3(256), 0, c.stream, g);
            return;
        }
    }
    // vector staging: each operand contiguous along K or along its other
    // dimension (multiple of 8), rows 16-byte aligned
    if constexpr (sizeof(TB) == 2) {
        const bool al = reinterpret_cast<uintptr_t>(g.A) % 16 == 0 && reinterpret_cast<uintptr_t>(g.B) % 16 == 0;
        const bool ak = g.sak == 1 && g.K % 8 == 0 && (g.sam * (int64_t)sizeof(TA)) % 16 == 0;
        const bool am = g.sam == 1 && g.M % 8 == 0 && (g.sak * (int64_t)sizeof(TA)) % 16 == 0;
        const bool bk = g.sbk == 1 && g.K % 8 == 0 && (g.sbn * 2) % 16 == 0;
        const bool bn = g.sbn == 1 && g.N % 8 == 0 && (g.sbk * 2) % 16 == 0;
        const dim3 grid(nb(g.N, TN), nb(g.M, TM), EPI == EPI_STORE ? g.ksplit : 1);
        if (al && ak && bk) {
            hipLaunchKernelGGL((k_gemm_v<TA, EPI, true, true>), grid, dim3(256), 0, c.stream, g);
            return;
        }
        if (al && ak && bn) {
            hipLaunchKernelGGL((k_gemm_v<TA, EPI, true, false>), grid, dim3(256), 0, c.stream, g);
            return;
        }
        if (al && am && bn) {
            hipLaunchKernelGGL((k_gemm_v<TA, EPI, false, false>), grid, dim3(256), 0, c.stream, g);
            return;
        }
    }
    dim3 grid(nb(g.N, TN), nb(g.M, TM), EPI == EPI_STORE ? g.ksplit : 1);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, c.stream, g);
}

// weight gradient dW[M x N] = sum_b G[b, m] Act[b, n] (K = batch), split-K
template <typename TB> void weight_grad(mlp_ctx &c, const float *G, int ldg, const TB *Act, int lda, int M, int N,
                                        int B, float *out)
{
    GemmArgs g{};
    g.M = M;
    g.N = N;
    g.K = B;
    g.A = G;
    g.sam = 1;
    g.sak = ldg;
    g.B = Act;
    g.sbk = lda;
    g.sbn = 1;
    g.C = c.part;
    g.ldc = N;
    g.ksplit = std::max(1, std::min(SPLITK, (B + TK - 1) / TK));
    gemm<float, TB, EPI_STORE>(c, g);
    const int64_t cnt = (int64_t)M * N;
    hipLaunchKernelGGL(k_splitk_sum, dim3(nb(cnt, 256)), dim3(256), 0, c.stream, c.part, g.ksplit, cnt, out);
}

void bias_grad(mlp_ctx &c, const float *G, int ld, int B, int N, float *out)
{
    hipLaunchKernelGGL(k_colsum, dim3(nb(N, 64), COLSUM_CHUNKS), dim3(256), 0, c.stream, G, B, N, (int64_t)ld,
                       c.colpart);
    hipLaunchKernelGGL(k_colsum_fold, dim3(nb(N, 256)), dim3(256), 0, c.stream, c.colpart, N, out);
}

// Activation buffers of one forward pass: padded BF16 input X [B x 32],
// per hidden layer the pre-activation Z (FP32) and the BF16 activation A
// [B x H], the FP32 output Y [B x 32].
struct Acts {
    uint16_t *X, *A[3];
    float *Z[3], *Y;
};

void forward(mlp_ctx &c, int B, const Acts &a)
{
    const int H = c.H;
    const uint16_t *in = a.X;
    int K = PAD;
    for (int l = 0; l < 3; ++l) {
        GemmArgs g{};
        g.M = B;
        g.N = H;
        g.K = K;
        g.A = in;
        g.sam = K;
        g.sak = 1;
        g.B = c.pbf + c.oW[l];
        g.sbk = 1;
        g.sbn = K;
        g.bias = c.p + c.ob[l];
        g.C = a.Z[l];
        g.ldc = H;
        g.Abf = a.A[l];
        g.ldabf = H;
        gemm<uint16_t, uint16_t, EPI_GELU>(c, g);
        in = a.A[l];
        K = H;
    }
    GemmArgs g{};
    g.M = B;
    g.N = PAD;
    g.K = H;
    g.A = a.A[2];
    g.sam = H;
    g.sak = 1;
    g.B = c.pbf + c.oW[3];
    g.sbk = 1;
    g.sbn = H;
    g.bias = c.p + c.ob[3];
    g.C = a.Y;
    g.ldc = PAD;
    gemm<uint16_t, uint16_t, EPI_LINEAR>(c, g);
}

Acts ctx_acts(const mlp_ctx &c) { return Acts{c.X, {c.A[0], c.A[1], c.A[2]}, {c.Z[0], c.Z[1], c.Z[2]}, c.Y}; }

void backward(mlp_ctx &c, int B)
{
    const int H = c.H;
    float *gr = c.grad;
    // output layer
    weight_grad<uint16_t>(c, c.dY, PAD, c.A[2], H, PAD, H, B, gr + c.oW[3]);
    bias_grad(c, c.dY, PAD, B, PAD, gr + c.ob[3]);
    // dZ3 = (dY W4) * GELU'(Z3)
    const float *G = c.dY;
    int ldG = PAD, Kin = PAD;
    int buf = 0;
    for (int l = 2; l >= 0; --l) {
        GemmArgs g{};
        g.M = B;
        g.N = H;
        g.K = Kin;
        g.A = G;
        g.sam = ldG;
        g.sak = 1;
        g.B = c.pbf + c.oW[l + 1];
        g.sbk = H;   // W_{l+1} rows = outputs (Kin), columns = H inputs
        g.sbn = 1;
        g.C = c.D[buf];
        g.ldc = H;
        g.Zin = c.Z[l];
        g.ldz = H;
        gemm<float, uint16_t, EPI_DGELU>(c, g);
        // dW_l = dZ_l^T A_{l-1}, db_l
        if (l > 0)
            weight_grad<uint16_t>(c, c.D[buf], H, c.A[l - 1], H, H, H, B, gr + c.oW[l]);
        else
            weight_grad<uint16_t>(c, c.D[buf], H, c.X, PAD, H, PAD, B, gr + c.oW[0]);
        bias_grad(c, c.D[buf], H, B, H, gr + c.ob[l]);
        G = c.D[buf];
        ldG = H;
        Kin = H;
        buf ^= 1;
    }
}

}  // namespace

extern "C" pic_status mlp_workspace_bytes(const mlp_config *cfg, size_t *bytes)
{
    if (!cfg || !bytes) return PIC_EINVAL;
    if (cfg->n_in < 1 || cfg->n_in > PAD || cfg->n_out < 1 || cfg->n_out > PAD || cfg->hidden < 64 ||
        cfg->hidden % 64 != 0 || cfg->max_batch < 1)
        return PIC_EINVAL;
    mlp_ctx c;
    c.H = cfg->hidden;
    c.maxB = cfg->max_batch;
    Carver cv{nullptr};
    mlp_layout(c, cv);
    *bytes = cv.off + 256;
    return PIC_OK;
}

extern "C" pic_status mlp_init(const mlp_config *cfg, void *workspace, size_t bytes, void *stream, mlp_ctx **out)
{
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    size_t need = 0;
    pic_status st = mlp_workspace_bytes(cfg, &need);
    if (st) return st;
    if (!workspace || bytes < need) return PIC_ENOMEM;
    mlp_ctx *c = new mlp_ctx();
    c->cfg = *cfg;
    c->H = cfg->hidden;
    c->maxB = cfg->max_batch;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    Carver cv{reinterpret_cast<uint8_t *>(workspace)};
    mlp_layout(*c, cv);
    // the static inference scratch of the current device (the stream's)
    {
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = scratch_address(dev, &c->scratch);
        if (e != hipSuccess) {
            delete c;
            return PIC_EDEVICE;
        }
    }
    std::vector<float> nrm(4 * PAD, 0.0f);
    for (int i = 0; i < PAD; ++i) nrm[PAD + i] = nrm[3 * PAD + i] = 1.0f;
    for (int i = 0; i < cfg->n_in; ++i) {
        if (cfg->in_mean) nrm[i] = cfg->in_mean[i];
        if (cfg->in_std) nrm[PAD + i] = cfg->in_std[i];
    }
    for (int i = 0; i < cfg->n_out; ++i) {
        if (cfg->out_mean) nrm[2 * PAD + i] = cfg->out_mean[i];
        if (cfg->out_std) nrm[3 * PAD + i] = cfg->out_std[i];
    }
    hipError_t e = hipMemcpyAsync(c->norm, nrm.data(), nrm.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->p, 0, c->P * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->pbf, 0, c->P * 2, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->m, 0, c->P * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->v, 0, c->P * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->grad, 0, c->P * 4, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return PIC_EDEVICE;
    }
    *out = c;
    return PIC_OK;
}

extern "C" pic_status mlp_param_count(const mlp_ctx *c, int64_t *n)
{
    if (!c || !n) return PIC_EINVAL;
    *n = c->P;
    return PIC_OK;
}

extern "C" pic_status mlp_set_params(mlp_ctx *c, const float *host)
{
    if (!c || !host) return PIC_EINVAL;
    MCHK(c, hipMemcpyAsync(c->p, host, c->P * 4, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_to_bf16, dim3(nb(c->P, 256)), dim3(256), 0, c->stream, c->p, c->pbf, c->P);
    MCHK(c, hipMemsetAsync(c->m, 0, c->P * 4, c->stream));
    MCHK(c, hipMemsetAsync(c->v, 0, c->P * 4, c->stream));
    c->step = 0;
    MCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

extern "C" pic_status mlp_get_params(mlp_ctx *c, float *host)
{
    if (!c || !host) return PIC_EINVAL;
    MCHK(c, hipMemcpyAsync(host, c->p, c->P * 4, hipMemcpyDeviceToHost, c->stream));
    MCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

extern "C" pic_status mlp_get_grads(mlp_ctx *c, float *host)
{
    if (!c || !host) return PIC_EINVAL;
    MCHK(c, hipMemcpyAsync(host, c->grad, c->P * 4, hipMemcpyDeviceToHost, c->stream));
    MCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

extern "C" pic_status mlp_forward(mlp_ctx *c, const float *x, int32_t batch, float *y)
{
    if (!c || !x || !y) return PIC_EINVAL;
    if (batch < 1 || batch > c->maxB) return mfail(c, PIC_EINVAL, "batch %d outside 1..%d", batch, c->maxB);
    const mlp_config &f = c->cfg;
    hipLaunchKernelGGL(k_input, dim3(nb((int64_t)batch * PAD, 256)), dim3(256), 0, c->stream, x, batch, f.n_in, c->norm,
                       c->norm + PAD, c->X);
    forward(*c, batch, ctx_acts(*c));
    hipLaunchKernelGGL(k_output, dim3(nb((int64_t)batch * f.n_out, 256)), dim3(256), 0, c->stream, c->Y, batch,
                       f.n_out, c->norm + 2 * PAD, c->norm + 3 * PAD, y);
    return hipGetLastError() == hipSuccess ? PIC_OK : mfail(c, PIC_EDEVICE, "kernel launch failed");
}

extern "C" pic_status mlp_forward_noalloc(mlp_ctx *c, const float *x, int32_t batch, float *y)
{
    if (!c || !x || !y) return PIC_EINVAL;
    if (batch < 1 || batch > NOALLOC_MAX_BATCH)
        return mfail(c, PIC_EINVAL, "batch %d outside 1..%d (static inference scratch)", batch, NOALLOC_MAX_BATCH);
    if (c->H > NOALLOC_MAX_HIDDEN)
        return mfail(c, PIC_EINVAL, "hidden width %d above %d (static inference scratch)", c->H, NOALLOC_MAX_HIDDEN);
    if (!c->scratch) return mfail(c, PIC_EDEVICE, "static inference scratch not available on this device");
    uint8_t *s = reinterpret_cast<uint8_t *>(c->scratch);
    const size_t la = (size_t)NOALLOC_MAX_BATCH * NOALLOC_MAX_HIDDEN;
    Acts a{};
    a.X = reinterpret_cast<uint16_t *>(s + NA_X);
    for (int l = 0; l < 3; ++l) {
        a.A[l] = reinterpret_cast<uint16_t *>(s + NA_A) + l * la;
        a.Z[l] = reinterpret_cast<float *>(s + NA_Z) + l * la;
    }
    a.Y = reinterpret_cast<float *>(s + NA_Y);
    const mlp_config &f = c->cfg;
    hipLaunchKernelGGL(k_input, dim3(nb((int64_t)batch * PAD, 256)), dim3(256), 0, c->stream, x, batch, f.n_in, c->norm,
                       c->norm + PAD, a.X);
    forward(*c, batch, a);
    hipLaunchKernelGGL(k_output, dim3(nb((int64_t)batch * f.n_out, 256)), dim3(256), 0, c->stream, a.Y, batch,
                       f.n_out, c->norm + 2 * PAD, c->norm + 3 * PAD, y);
    return hipGetLastError() == hipSuccess ? PIC_OK : mfail(c, PIC_EDEVICE, "kernel launch failed");
}

extern "C" pic_status mlp_train_step(mlp_ctx *c, const float *x, const float *t, int32_t batch, float *loss)
{
    if (!c || !x || !t) return PIC_EINVAL;
    if (batch < 1 || batch > c->maxB) return mfail(c, PIC_EINVAL, "batch %d outside 1..%d", batch, c->maxB);
    const mlp_config &f = c->cfg;
    hipLaunchKernelGGL(k_input, dim3(nb((int64_t)batch * PAD, 256)), dim3(256), 0, c->stream, x, batch, f.n_in, c->norm,
                       c->norm + PAD, c->X);
    forward(*c, batch, ctx_acts(*c));
    const unsigned nl = nb((int64_t)batch * PAD, 256);
    hipLaunchKernelGGL(k_loss, dim3(nl), dim3(256), 0, c->stream, c->Y, t, batch, f.n_out, c->norm + 2 * PAD,
                       c->norm + 3 * PAD, c->dY, c->lpart);
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(256), 0, c->stream, c->lpart, (int)nl, 1.0f / (float)(batch * f.n_out),
                       c->loss);
    backward(*c, batch);
    c->step += 1;
    const double bc1 = 1.0 - std::pow(f.beta1, (double)c->step), bc2 = 1.0 - std::pow(f.beta2, (double)c->step);
    hipLaunchKernelGGL(k_adam, dim3(nb(c->P, 256)), dim3(256), 0, c->stream, c->p, c->grad, c->m, c->v, c->pbf, c->P,
                       (float)f.lr, (float)f.beta1, (float)f.beta2, (float)f.eps, (float)bc1, (float)bc2);
    if (hipGetLastError() != hipSuccess) return mfail(c, PIC_EDEVICE, "kernel launch failed");
    if (loss) {
        MCHK(c, hipMemcpyAsync(loss, c->loss, 4, hipMemcpyDeviceToHost, c->stream));
        MCHK(c, hipStreamSynchronize(c->stream));
    }
    return PIC_OK;
}

extern "C" pic_status mlp_sync(mlp_ctx *c)
{
    if (!c) return PIC_EINVAL;
    MCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

extern "C" void mlp_destroy(mlp_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

extern "C" const char *mlp_last_error(const mlp_ctx *c) { return c ? c->err.c_str() : "null context"; }

namespace pic {
// input / output widths and stream of a network (for the circuit update)
void mlp_shape(const mlp_ctx *c, int *n_in, int *n_out, void **stream)
{
    *n_in = c->cfg.n_in;
    *n_out = c->cfg.n_out;
    *stream = c->stream;
}
}  // namespace pic
