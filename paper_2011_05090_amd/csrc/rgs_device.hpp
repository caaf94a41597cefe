// Device-side building blocks of librgs (gfx950, wave64).
//
//  * Philox4x32-10 (Salmon et al., SC'11) -- the seeded generator that lets any
//    block of the sketch be regenerated on the fly (Sec. 2.1 of Balabanov &
//    Grigori; Sec. 2.4 on seeded generation without storage/communication).
//  * Gaussian sketch entries: Box-Muller on Philox words, N(0,1) before the
//    1/sqrt(k) scale (Sec. 2.1, Gaussian / Rademacher family).
//  * In-wave Walsh-Hadamard transform of 1024 points (the H factor of the
//    P-SRHT, Sec. 2.1), one wave64 holding 16 values per lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgs {

constexpr int kWG = 256;       // threads per workgroup (4 x wave64)
constexpr int kWave = 64;
constexpr int kTile = 1024;    // rows per wave tile = in-wave FWHT order
constexpr int kBlock = 4096;   // rows per workgroup block (4 wave tiles)
constexpr int kSlice = 64;     // sketch-space rows per workgroup
constexpr int kKptMax = 16;    // sketch rows per thread: k <= 16 * 256
constexpr int kProjWaves = 8;  // wave tiles per workgroup of the projection kernel
// Step 3 sums the terms coef_c q_c of kProjGroup consecutive columns in a fresh
// accumulator before subtracting them from w: fewer roundings of the large
// running vector (fp32 accumulation throughout).
constexpr int kProjGroup = 8;
constexpr int kProjRows = kProjWaves * kTile;

// The dispatcher sends workgroup b of a launch to XCD b mod kXcd, each XCD
// with its own L2.  xcd_block maps b to a logical block so that every XCD
// gets one contiguous range of the G blocks: blocks that read each other's
// rows (the neighbour planes of a stencil) then share an L2.  A bijection of
// [0, G); only cache reuse depends on it.
constexpr int kXcd = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
    const int64_t x = b % kXcd, slot = b / kXcd, q = G / kXcd, r = G % kXcd;
    return x * q + (x < r ? x : r) + slot;
}

constexpr uint32_t kTagSigns = 0xFFFFFFFFu;  // counter word 1 of the SRHT sign draws
constexpr uint32_t kTagRows = 0xFFFFFFFEu;   // counter word 1 of the SRHT row draws

// Philox4x32-10: 10 rounds of (M0*c0, M1*c2) multiply-xor with a Weyl key
// schedule.  Host and device share this definition inside the library.
__host__ __device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                       uint32_t c3, uint32_t k0, uint32_t k1,
                                                       uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// fp64 -> bfloat16 bits, rounded to nearest (ties to even) in one step.
// For finite values in the float range (the rounded value, 8 significant
// bits with a float exponent, converts to float exactly).
__device__ __forceinline__ uint32_t bf16_rne_f64(double x) {
    uint64_t u = (uint64_t)__double_as_longlong(x);
    u = ((u + ((1ull << 44) - 1) + ((u >> 45) & 1ull)) >> 45) << 45;
    return __float_as_uint((float)__longlong_as_double((long long)u)) >> 16;
}

// The bf16 Gaussian table (unscaled entries): group o of sketch row j holds
// z(j, 8o .. 8o+7) as one 16-byte word.
typedef uint32_t tabw_t __attribute__((ext_vector_type(4)));
constexpr int kTabDepth = 16;   // table groups a thread keeps in flight

__device__ __forceinline__ tabw_t tab_load(const uint16_t* __restrict__ table, int k, int64_t o, int j) {
    return __builtin_nontemporal_load(reinterpret_cast<const tabw_t*>(table + (o * k + j) * 8));
}

template <typename T>
__device__ __forceinline__ void tab_unpack(const tabw_t w, T z[8]) {
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        z[2 * t] = (T)__uint_as_float(ws[t] << 16);
        z[2 * t + 1] = (T)__uint_as_float(ws[t] & 0xFFFF0000u);
    }
}

template <typename T>
__device__ __forceinline__ void tab8(const uint16_t* __restrict__ table, int k, int64_t o, int j, T z[8]) {
    tab_unpack<T>(tab_load(table, k, o, j), z);
}

// Rademacher sketch (entries +-1/sqrt(k)): the signs of row j at the 128
// columns 128 b .. 128 b + 127 are the bits of one Philox call at counter
// (b, j, sketch_id, instance); bit l % 32 of word (l % 128) / 32 set means -1.
__device__ __forceinline__ void rad_words(uint32_t b, uint32_t j, uint32_t sid, uint32_t inst, uint32_t k0,
                                          uint32_t k1, uint32_t w[4]) {
    philox4x32_10(b, j, sid, inst, k0, k1, w);
}

// +1 or -1 (bit r of wd set) in T, built from the bit without a branch.
template <typename T>
__device__ __forceinline__ T rad_sign(uint32_t wd, int r);
template <>
__device__ __forceinline__ float rad_sign<float>(uint32_t wd, int r) {
    return __uint_as_float(0x3F800000u | ((wd << (31 - r)) & 0x80000000u));
}
template <>
__device__ __forceinline__ double rad_sign<double>(uint32_t wd, int r) {
    return __hiloint2double((int)(0x3FF00000u | ((wd << (31 - r)) & 0x80000000u)), 0);
}

// Four standard normals z(j, 4q .. 4q+3) from one Philox call at counter
// (q, j, sketch_id, instance).  Uniforms: u1 = ((x_a >> 9) + 1/2) 2^-23 in (0,1),
// u2 = (x_b >> 8) 2^-24 in [0,1), both exact in fp32 and fp64;
// z_a = sqrt(-2 ln u1) cos(2 pi u2), z_b = sqrt(-2 ln u1) sin(2 pi u2).
// fp64: libm log and sincospi in double.
__device__ __forceinline__ void gauss4(uint32_t q, uint32_t j, uint32_t sid, uint32_t inst,
                                       uint32_t k0, uint32_t k1, double z[4]) {
    uint32_t x[4];
    philox4x32_10(q, j, sid, inst, k0, k1, x);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double u1 = ((double)(x[2 * h] >> 9) + 0.5) * 0x1p-23;
        const double u2 = (double)(x[2 * h + 1] >> 8) * 0x1p-24;
        const double rho = sqrt(-2.0 * log(u1));
        double s, c;
        sincospi(2.0 * u2, &s, &c);
        z[2 * h] = rho * c;
        z[2 * h + 1] = rho * s;
    }
}

// Correctly rounded sqrt of a positive normal float: the hardware square root
// (within 1 ulp) corrected by the signs of x - y^2 at the neighbouring floats,
// each an exact fma residual.  This is the correctly rounded sqrtf's own
// sequence without its denormal scaling and zero / infinity / NaN handling,
// which the Box-Muller radius never needs (its argument lies in
// [2.4e-7, 33.3]); over every float of [2^-23, 34] it gives sqrtf's bits.
__device__ __forceinline__ float sqrt_pos_normal(float x) {
    float y = __builtin_amdgcn_sqrtf(x);
    const float ym = __uint_as_float(__float_as_uint(y) - 1u), yp = __uint_as_float(__float_as_uint(y) + 1u);
    const float rm = __builtin_fmaf(-ym, y, x), rp = __builtin_fmaf(-yp, y, x);
    y = (rm <= 0.f) ? ym : y;
    y = (rp > 0.f) ? yp : y;
    return y;
}

// fp32: hardware log2, sqrt, and sine/cosine (whose argument is in revolutions,
// so cos(2 pi u2) is the instruction applied to u2 itself).
__device__ __forceinline__ void gauss4(uint32_t q, uint32_t j, uint32_t sid, uint32_t inst,
                                       uint32_t k0, uint32_t k1, float z[4]) {
    uint32_t x[4];
    philox4x32_10(q, j, sid, inst, k0, k1, x);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float u1 = ((float)(x[2 * h] >> 9) + 0.5f) * 0x1p-23f;
        const float u2 = (float)(x[2 * h + 1] >> 8) * 0x1p-24f;
        // -2 ln u1 = -2 ln(2) log2(u1): in [2.4e-7, 33.3] for u1 in [2^-24, 1 - 2^-24]
        const float rho = sqrt_pos_normal(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
        z[2 * h] = rho * __builtin_amdgcn_cosf(u2);
        z[2 * h + 1] = rho * __builtin_amdgcn_sinf(u2);
    }
}

// Unnormalised Walsh-Hadamard transform (Sylvester order) of the 1024 values
// held by one wave: lane L holds v[4e + r] = x[256 e + 4 L + r], e, r in 0..3.
// Index bits 0-1 and 8-9 live in registers, bits 2-7 across lanes.
template <typename T>
__device__ __forceinline__ void fwht1024_wave(T v[16], int lane) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const T a0 = v[4 * e], a1 = v[4 * e + 1], a2 = v[4 * e + 2], a3 = v[4 * e + 3];
        const T b0 = a0 + a1, b1 = a0 - a1, b2 = a2 + a3, b3 = a2 - a3;
        v[4 * e] = b0 + b2;
        v[4 * e + 1] = b1 + b3;
        v[4 * e + 2] = b0 - b2;
        v[4 * e + 3] = b1 - b3;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const T a0 = v[r], a1 = v[4 + r], a2 = v[8 + r], a3 = v[12 + r];
        const T b0 = a0 + a1, b1 = a0 - a1, b2 = a2 + a3, b3 = a2 - a3;
        v[r] = b0 + b2;
        v[4 + r] = b1 + b3;
        v[8 + r] = b0 - b2;
        v[12 + r] = b1 - b3;
    }
#pragma unroll
    for (int msk = 1; msk < 64; msk <<= 1) {
        const bool upper = (lane & msk) != 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const T o = __shfl_xor(v[t], msk);
            v[t] = upper ? (o - v[t]) : (v[t] + o);
        }
    }
}

}  // namespace rgs
