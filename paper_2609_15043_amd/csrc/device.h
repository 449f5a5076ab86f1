// Device-side building blocks of the phasorpic kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
// ten rounds, each two 32x32 -> 64-bit products of counter words 0 and 2
// with fixed multipliers, outputs mixed with words 1, 3 and the round key;
// the key advances by the two Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo_a = 0xD2511F53u * c.x;
        const uint32_t hi_a = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo_b = 0xCD9E8D57u * c.z;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, c.z);
        c = U4{hi_b ^ c.y ^ k0, lo_b, hi_a ^ c.w ^ k1, lo_a};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// uniform on (0, 1): (x + 1/2) / 2^32, evaluated in FP64
__device__ __forceinline__ double unit(uint32_t x) { return ((double)x + 0.5) * 2.3283064365386963e-10; }

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Wave total in lane 63: in-row shift-add scan (1, 2, 4, 8), then the row
// broadcasts 15 and 31.  Lanes outside a shifted row read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}

__device__ __forceinline__ float wave_total(float v)
{
    v += dpp_f32<0x111, 0xF>(v);
    v += dpp_f32<0x112, 0xF>(v);
    v += dpp_f32<0x114, 0xF>(v);
    v += dpp_f32<0x118, 0xF>(v);
    v += dpp_f32<0x142, 0xA>(v);
    v += dpp_f32<0x143, 0xC>(v);
    return v;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_total(double v)
{
    v += dpp_f64<0x111, 0xF>(v);
    v += dpp_f64<0x112, 0xF>(v);
    v += dpp_f64<0x114, 0xF>(v);
    v += dpp_f64<0x118, 0xF>(v);
    v += dpp_f64<0x142, 0xA>(v);
    v += dpp_f64<0x143, 0xC>(v);
    return v;
}

// a / b: hardware reciprocal in FP32 (about 1 ulp), IEEE division in FP64
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double quot(double a, double b) { return a / b; }

// square root: the hardware instruction in FP32 (about 1 ulp; the correctly
// rounded form adds a dozen instructions of range scaling and refinement),
// IEEE in FP64
__device__ __forceinline__ float root(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double root(double x) { return sqrt(x); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// ---------------------------------------------------------------------------
// Exact fixed-point accumulation.  Deposits are summed as signed 64-bit
// integers (value * 2^k rounded once per contribution), so the node sums do
// not depend on the order of the atomics.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long to_fixed(double v, double scale) { return __double2ll_rn(v * scale); }

// round(v * scale) for a power-of-two scale, fast path of the particle
// deposits: for |x| < 2^51, x + 1.5 * 2^52 rounds x to an integer (half to
// even, as the conversion above) and leaves it in the low significand bits,
// so the integer is the difference of the two bit patterns.  Larger values
// take the library conversion.  The FP32 overload is exact in the same way
// (the product of an FP32 value and a power of two is exact in FP64).
__device__ __forceinline__ long long to_fixed_fast(double v, double scale)
{
    constexpr double magic = 6755399441055744.0;   // 1.5 * 2^52
    const double x = v * scale;
    const bool big = !(fabs(x) < 0x1p51);
    long long f = __double_as_longlong(x + magic) - __double_as_longlong(magic);
    // the library conversion behind a wave-uniform branch: short divergent
    // blocks are issued with the lanes masked off rather than skipped, and
    // this one would cost every conversion six more instructions
    if (__builtin_expect(__ballot(big) != 0, 0))
        if (big) f = __double2ll_rn(x);
    return f;
}
__device__ __forceinline__ long long to_fixed_fast(float v, float scale)
{
    return to_fixed_fast((double)v, (double)scale);
}

__device__ __forceinline__ void atomic_add_i64(long long *p, long long v)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
}

// Packed field of one node for the gather: (E_r, E_z, E_theta, unused).
template <typename T> struct Field4;
template <> struct Field4<float> {
    using type = float4;
};
template <> struct Field4<double> {
    using type = double4;
};
// RF magnetic field of one node for the gather: (B_r, B_z).
template <typename T> struct Field2;
template <> struct Field2<float> {
    using type = float2;
};
template <> struct Field2<double> {
    using type = double2;
};

// Structure-of-arrays particle store of one species.
template <typename T> struct Parts {
    int32_t *cell;   // linear cell index i * nr + j, -1 once absorbed
    T *dr;           // radial offset in the cell, R = (j + dr) dR, in [0, 1)
    T *dz;           // axial offset, z = (i + dz) dz, in [0, 1)
    T *vr, *vt, *vz; // velocity in the local (r, theta, z) frame (m/s)
    uint32_t *id;    // particle id (Philox counter word 0)
    int32_t *next;   // step of the next null-collision candidate
    // direct-implicit update only (else null): the D1 filter's running
    // electrostatic half kick (dt/2) abar in the local frame (m/s)
    T *fr, *ft, *fz;
};

}  // namespace pic
