// Block-level building blocks shared by the projection kernel (rgs_kernels.hip)
// and the Arnoldi mat-vec kernel (rgs_gmres.hip): the streaming loads/stores
// of a lane's 16 rows and the per-block sketch of Sec. 2.1 (P-SRHT through the
// Kronecker split of H_s, or the on-the-fly Gaussian).
#pragma once

#include "rgs_device.hpp"
#include "rgs_types.hpp"

namespace rgs {

// ---------------------------------------------------------------------------
// Loads/stores of the 16 rows a lane owns in a wave tile:
// rows row0[e] .. row0[e] + 3, e = 0..3 (row0[e] is a multiple of 4).
// Full tiles use nontemporal vector accesses: every column of W and Q is
// touched once per pass and the basis is far larger than any cache level.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// SK_TABX: group o of sketch row j holds the 8 entries z(j, 8o .. 8o+7) in the
// working type T as W = 8 sizeof(T) / 16 words of 16 bytes; word w of every
// sketch row of the group sits in one run, at 16-byte index (o W + w) k + j,
// so the lanes of a wave (consecutive j) read one contiguous kilobyte per load.
template <typename T>
struct TabxGroup;
template <>
struct TabxGroup<float> {
    f32x4 a, b;
};
template <>
struct TabxGroup<double> {
    f64x2 a, b, c, d;
};
__device__ __forceinline__ TabxGroup<float> tabx_load(const float* __restrict__ t, int k, int64_t o, int j) {
    const f32x4* p = reinterpret_cast<const f32x4*>(t) + 2 * o * k + j;
    return {__builtin_nontemporal_load(p), __builtin_nontemporal_load(p + k)};
}
__device__ __forceinline__ TabxGroup<double> tabx_load(const double* __restrict__ t, int k, int64_t o, int j) {
    const f64x2* p = reinterpret_cast<const f64x2*>(t) + 4 * o * k + j;
    return {__builtin_nontemporal_load(p), __builtin_nontemporal_load(p + k), __builtin_nontemporal_load(p + 2 * k),
            __builtin_nontemporal_load(p + 3 * k)};
}
__device__ __forceinline__ void tabx_unpack(const TabxGroup<float>& g, float z[8]) {
    z[0] = g.a.x; z[1] = g.a.y; z[2] = g.a.z; z[3] = g.a.w;
    z[4] = g.b.x; z[5] = g.b.y; z[6] = g.b.z; z[7] = g.b.w;
}
__device__ __forceinline__ void tabx_unpack(const TabxGroup<double>& g, double z[8]) {
    z[0] = g.a.x; z[1] = g.a.y; z[2] = g.b.x; z[3] = g.b.y;
    z[4] = g.c.x; z[5] = g.c.y; z[6] = g.d.x; z[7] = g.d.y;
}
// groups a thread keeps in flight: 256 bytes, as kTabDepth bf16 groups
template <typename T>
constexpr int tabx_depth() {
    return 256 / (8 * (int)sizeof(T));
}

// `vec` (aligned columns) lets a partial tile still load its complete 4-row
// groups as vectors; the group that straddles n is read element by element.
template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ p, T v[4]) {
    if constexpr (sizeof(T) == 4) {
        const f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    } else {
        const f64x2 a = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
        const f64x2 b = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p + 2));
        v[0] = a.x;
        v[1] = a.y;
        v[2] = b.x;
        v[3] = b.y;
    }
}

template <typename T>
__device__ __forceinline__ void load16(const T* __restrict__ p, const int64_t row0[4], int64_t n,
                                       bool full, T v[16], bool vec = false) {
    if (!full && vec) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (row0[e] + 4 <= n) {
                load4(p + row0[e], v + 4 * e);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) v[4 * e + r] = (row0[e] + r < n) ? p[row0[e] + r] : T(0);
            }
        }
        return;
    }
    if (full) {
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p + row0[e]));
                v[4 * e] = t.x;
                v[4 * e + 1] = t.y;
                v[4 * e + 2] = t.z;
                v[4 * e + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const f64x2 a = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p + row0[e]));
                const f64x2 b = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p + row0[e] + 2));
                v[4 * e] = a.x;
                v[4 * e + 1] = a.y;
                v[4 * e + 2] = b.x;
                v[4 * e + 3] = b.y;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) v[4 * e + r] = (row0[e] + r < n) ? p[row0[e] + r] : T(0);
    }
}

template <typename T>
__device__ __forceinline__ void store16(T* __restrict__ p, const int64_t row0[4], int64_t n,
                                        bool full, const T v[16]) {
    if (full) {
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const f32x4 t = {v[4 * e], v[4 * e + 1], v[4 * e + 2], v[4 * e + 3]};
                __builtin_nontemporal_store(t, reinterpret_cast<f32x4*>(p + row0[e]));
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const f64x2 a = {v[4 * e], v[4 * e + 1]};
                const f64x2 b = {v[4 * e + 2], v[4 * e + 3]};
                __builtin_nontemporal_store(a, reinterpret_cast<f64x2*>(p + row0[e]));
                __builtin_nontemporal_store(b, reinterpret_cast<f64x2*>(p + row0[e] + 2));
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (row0[e] + r < n) p[row0[e] + r] = v[4 * e + r];
    }
}

// ---------------------------------------------------------------------------
// bfloat16 storage of the basis: round to nearest even on store, exact on load.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t float_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void load16(const bf16* __restrict__ p, const int64_t row0[4], int64_t n, bool full,
                                       float v[16], bool vec = false) {
    if (!full && vec) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (row0[e] + 4 <= n) {
                const u32x2 t = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p + row0[e]));
                v[4 * e] = __uint_as_float(t.x << 16);
                v[4 * e + 1] = __uint_as_float(t.x & 0xFFFF0000u);
                v[4 * e + 2] = __uint_as_float(t.y << 16);
                v[4 * e + 3] = __uint_as_float(t.y & 0xFFFF0000u);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    v[4 * e + r] = (row0[e] + r < n) ? bf16_to_float(p[row0[e] + r].bits) : 0.f;
            }
        }
        return;
    }
    if (full) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const u32x2 t = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p + row0[e]));
            v[4 * e] = __uint_as_float(t.x << 16);
            v[4 * e + 1] = __uint_as_float(t.x & 0xFFFF0000u);
            v[4 * e + 2] = __uint_as_float(t.y << 16);
            v[4 * e + 3] = __uint_as_float(t.y & 0xFFFF0000u);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) v[4 * e + r] = (row0[e] + r < n) ? bf16_to_float(p[row0[e] + r].bits) : 0.f;
    }
}

// Stores fl_bf16(v) and replaces v by the stored values.
__device__ __forceinline__ void store16(bf16* __restrict__ p, const int64_t row0[4], int64_t n, bool full,
                                        float v[16]) {
    uint16_t h[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        h[t] = float_to_bf16(v[t]);
        v[t] = bf16_to_float(h[t]);
    }
    if (full) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const u32x2 t = {(uint32_t)h[4 * e] | ((uint32_t)h[4 * e + 1] << 16),
                             (uint32_t)h[4 * e + 2] | ((uint32_t)h[4 * e + 3] << 16)};
            __builtin_nontemporal_store(t, reinterpret_cast<u32x2*>(p + row0[e]));
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (row0[e] + r < n) p[row0[e] + r].bits = h[4 * e + r];
    }
}

// Rows of this lane in block blk of a workgroup with NW wave tiles.
template <int NW>
__device__ __forceinline__ void lane_rows(int64_t blk, int64_t row0[4]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 4; ++e) row0[e] = blk * (NW * kTile) + wave * kTile + 256 * e + 4 * lane;
}

// ---------------------------------------------------------------------------
// Sketch of one block of NW * 1024 rows held in registers (v = this lane's 16
// rows), accumulated into acc[u] for the sketch rows j = threadIdx.x + 64 NW u.
// The 1/sqrt(k) scale is applied later, in fp64.
//
// SRHT: with s = 2^a T (T = 1024 the in-wave FWHT order) the Sylvester
// Hadamard matrix factors as H_s = H_{s/T} (x) H_T, so for a sampled row
// rho = alpha T + beta and the tile index t of rows [tT, (t+1)T):
//   (H_s D x)[rho] = sum_t (-1)^popcount(alpha & t) (H_T D x_t)[beta].
// Each wave transforms its tile in registers; the block's NW tiles are then
// combined per sampled row through LDS (tile t = NW blk + w, and since the
// bits of w and NW blk are disjoint the sign factors into both parts).
// Gaussian: theta_{j,l} generated on the fly, 4 entries per Philox call.
// Rademacher: the signs of 128 entries of a row per Philox call, applied as
// fma(+-1, x, acc).  Table (bf16 Gaussian): 8 entries per 16-byte load.
// ---------------------------------------------------------------------------
template <typename T, typename PT, int SK, int NW>
__device__ __forceinline__ void block_sketch(T v[16], int64_t blk, int64_t n, const SketchArgs& sk,
                                             PT acc[kKptMax], T* __restrict__ lds) {
    constexpr int NT = NW * kWave;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int kpt = (sk.k + NT - 1) / NT;
    if constexpr (SK == SK_SRHT) {
        int64_t row0[4];
        lane_rows<NW>(blk, row0);
        // the sign words and the sampled rows are read from valid (clamped)
        // addresses without a condition, so the loads issue together; a load
        // under a condition would be a branch and a wait each
        uint32_t words[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) words[e] = sk.signs[min(row0[e], n - 1) >> 5];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (row0[e] < n) {
                const int sh = (int)(row0[e] & 31);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if ((words[e] >> (sh + r)) & 1u) v[4 * e + r] = -v[4 * e + r];
            }
        }
        fwht1024_wave<T>(v, lane);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[wave * kTile + 256 * e + 4 * lane + r] = v[4 * e + r];
        __syncthreads();
        const uint32_t tb = (uint32_t)(blk * NW);  // tile index of wave 0
#pragma unroll
        for (int u0 = 0; u0 < kKptMax; u0 += 4) {
            if (u0 >= kpt) break;
            uint32_t rows[4];   // four sampled rows per round trip
#pragma unroll
            for (int d = 0; d < 4; ++d) rows[d] = (uint32_t)sk.rows[min(t + NT * (u0 + d), sk.k - 1)];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int u = u0 + d, j = t + NT * u;
                if (u < kpt && j < sk.k) {
                    const uint32_t alpha = rows[d] >> 10, beta = rows[d] & 1023u;
                    T tot = T(0);
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        const T z = lds[w * kTile + beta];
                        tot = (__popc(alpha & (uint32_t)w) & 1) ? tot - z : tot + z;
                    }
                    if (__popc(alpha & tb) & 1) tot = -tot;
                    acc[u] += (PT)tot;
                }
            }
        }
        __syncthreads();
    } else if constexpr (SK == SK_GAUSS) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[wave * kTile + 256 * e + 4 * lane + r] = v[4 * e + r];
        __syncthreads();
        const int64_t rem = n - blk * (NW * kTile);
        const int nq = rem >= NW * kTile ? NW * kTile / 4 : (int)((rem + 3) / 4);
        const uint32_t q0 = (uint32_t)(blk * (NW * kTile / 4));
        for (int q = 0; q < nq; ++q) {
            const T x0 = lds[4 * q], x1 = lds[4 * q + 1], x2 = lds[4 * q + 2], x3 = lds[4 * q + 3];
#pragma unroll
            for (int u = 0; u < kKptMax; ++u) {
                const int j = t + NT * u;
                if (u < kpt && j < sk.k) {
                    T z[4];
                    gauss4(q0 + (uint32_t)q, (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z);
                    acc[u] += (PT)(z[0] * x0 + z[1] * x1 + z[2] * x2 + z[3] * x3);
                }
            }
        }
        __syncthreads();
    } else if constexpr (SK == SK_TABLE) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[wave * kTile + 256 * e + 4 * lane + r] = v[4 * e + r];
        __syncthreads();
        const int64_t rem = n - blk * (NW * kTile);
        const int no = rem >= NW * kTile ? NW * kTile / 8 : (int)((rem + 7) / 8);
        const int64_t o0 = blk * (NW * kTile / 8);
        // each thread streams its sketch rows through the block's table groups,
        // kTabDepth 16-byte loads in flight; x comes from LDS (broadcast reads)
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) {
            const int j = t + NT * u;
            if (u < kpt && j < sk.k) {
                PT a = acc[u];
                for (int o = 0; o < no; o += kTabDepth) {
                    tabw_t w[kTabDepth];
#pragma unroll
                    for (int d = 0; d < kTabDepth; ++d)
                        if (o + d < no) w[d] = tab_load(sk.table, sk.k, o0 + o + d, j);
#pragma unroll
                    for (int d = 0; d < kTabDepth; ++d) {
                        if (o + d < no) {
                            T z[8];
                            tab_unpack<T>(w[d], z);
                            const T* x = lds + 8 * (o + d);
                            a += (PT)(z[0] * x[0] + z[1] * x[1] + z[2] * x[2] + z[3] * x[3]);
                            a += (PT)(z[4] * x[4] + z[5] * x[5] + z[6] * x[6] + z[7] * x[7]);
                        }
                    }
                }
                acc[u] = a;
            }
        }
        __syncthreads();
    } else if constexpr (SK == SK_TABX) {   // the SK_TABLE pass with the entries in T
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[wave * kTile + 256 * e + 4 * lane + r] = v[4 * e + r];
        __syncthreads();
        const T* tab = static_cast<const T*>(sk.tabx);
        constexpr int D = tabx_depth<T>();
        const int64_t rem = n - blk * (NW * kTile);
        const int no = rem >= NW * kTile ? NW * kTile / 8 : (int)((rem + 7) / 8);
        const int64_t o0 = blk * (NW * kTile / 8);
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) {
            const int j = t + NT * u;
            if (u < kpt && j < sk.k) {
                PT a = acc[u];
                for (int o = 0; o < no; o += D) {
                    TabxGroup<T> w[D];
#pragma unroll
                    for (int d = 0; d < D; ++d)
                        if (o + d < no) w[d] = tabx_load(tab, sk.k, o0 + o + d, j);
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        if (o + d < no) {
                            T z[8];
                            tabx_unpack(w[d], z);
                            const T* x = lds + 8 * (o + d);
                            a += (PT)(z[0] * x[0] + z[1] * x[1] + z[2] * x[2] + z[3] * x[3]);
                            a += (PT)(z[4] * x[4] + z[5] * x[5] + z[6] * x[6] + z[7] * x[7]);
                        }
                    }
                }
                acc[u] = a;
            }
        }
        __syncthreads();
    } else if constexpr (SK == SK_RADEM) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[wave * kTile + 256 * e + 4 * lane + r] = v[4 * e + r];
        __syncthreads();
        // rows past n hold zeros, so only whole 128-row groups up to n are visited
        const int64_t rem = n - blk * (NW * kTile);
        const int ng = rem >= NW * kTile ? NW * kTile / 128 : (int)((rem + 127) / 128);
        const uint32_t g0 = (uint32_t)(blk * (NW * kTile / 128));
        for (int g = 0; g < ng; ++g) {
#pragma unroll
            for (int u = 0; u < kKptMax; ++u) {
                const int j = t + NT * u;
                if (u < kpt && j < sk.k) {
                    uint32_t wd[4];
                    rad_words(g0 + (uint32_t)g, (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, wd);
                    PT a = acc[u];
#pragma unroll
                    for (int c4 = 0; c4 < 4; ++c4) {
                        const T* xs = lds + 128 * g + 32 * c4;
#pragma unroll
                        for (int r = 0; r < 32; ++r) a = fma((PT)rad_sign<T>(wd[c4], r), (PT)xs[r], a);
                    }
                    acc[u] = a;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Rademacher sketch of one fp32 block (NW = kProjWaves wave tiles, v = this
// lane's 16 rows) through signed-sum tables: for every aligned 4-row chunk c
// of the block and every 4-bit sign pattern m, T[c][m] = sum_r (-1)^{m_r} x_{4c+r}
// (bit r of m set meaning -1).  The block's rows are the same for all k sketch
// rows, so the tables are built once and each sketch row then adds one table
// entry per 4 rows, indexed by the nibble of its Philox sign word that covers
// them (the bit layout of rad_words / rad_sign), instead of applying 4 signs.
// The tables of half a block (NW/2 wave tiles: 1024 chunks x 16 floats =
// 64 KiB of LDS, kRadNibLds floats) are built and consumed at a time.  Within
// a 128-row group the 32 entries are added in row order; the result differs
// from the sign-by-sign sum only by fp32 rounding.
// ---------------------------------------------------------------------------
constexpr int kRadNibLds = (kProjWaves / 2) * kTile / 4 * 16;

template <typename PT, int NW>
__device__ __forceinline__ void block_sketch_rad_nib(const float v[16], int64_t blk, int64_t n, const SketchArgs& sk,
                                                     PT acc[kKptMax], float* __restrict__ lds) {
    static_assert(NW == kProjWaves, "table layout of a kProjWaves block");
    constexpr int NT = NW * kWave;
    constexpr int HW = NW / 2;                 // wave tiles per half
    constexpr int GH = HW * kTile / 128;       // 128-row groups per half
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int kpt = (sk.k + NT - 1) / NT;
    const int64_t rem = n - blk * (NW * kTile);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t rem_h = rem - (int64_t)h * HW * kTile;
        if (rem_h <= 0) break;                 // workgroup-uniform
        if (wave / HW == h) {                  // this half's waves build the tables of their chunks
            const int wl = wave - h * HW;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float x0 = v[4 * e], x1 = v[4 * e + 1], x2 = v[4 * e + 2], x3 = v[4 * e + 3];
                const float p[4] = {x0 + x1, -x0 + x1, x0 - x1, -x0 - x1};   // pattern bits 0-1
                const float q[4] = {x2 + x3, -x2 + x3, x2 - x3, -x2 - x3};   // pattern bits 2-3
                float* dst = lds + (wl * (kTile / 4) + 64 * e + lane) * 16;
#pragma unroll
                for (int m2 = 0; m2 < 4; ++m2) {
                    const f32x4 o = {p[0] + q[m2], p[1] + q[m2], p[2] + q[m2], p[3] + q[m2]};
                    *reinterpret_cast<f32x4*>(dst + 4 * m2) = o;
                }
            }
        }
        __syncthreads();
        const int ng = rem_h >= HW * kTile ? GH : (int)((rem_h + 127) / 128);
        const uint32_t g0 = (uint32_t)(blk * (NW * kTile / 128) + h * GH);
        for (int g = 0; g < ng; ++g) {
#pragma unroll
            for (int u = 0; u < kKptMax; ++u) {
                const int j = t + NT * u;
                if (u < kpt && j < sk.k) {
                    uint32_t wd[4];
                    rad_words(g0 + (uint32_t)g, (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, wd);
                    const float* tg = lds + 32 * g * 16;   // the group's 32 chunks
                    PT a = acc[u];
#pragma unroll
                    for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            a += (PT)tg[(8 * c4 + i) * 16 + ((wd[c4] >> (4 * i)) & 15u)];
                    acc[u] = a;
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace rgs
