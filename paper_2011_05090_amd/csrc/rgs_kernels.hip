// HIP kernels of librgs for gfx950 (MI355X).
//
// Randomized Gram-Schmidt, Algorithm 2 of Balabanov & Grigori (Sec. 2.3), one
// column i at a time:
//   step 1  p_i = Theta w_i                 -> k_sketch_cols (SRHT) / k_gauss_cols (Gaussian)
//                                              + k_reduce, all columns at once
//   step 2  y = argmin ||S_{i-1} y - p_i||  -> k_ls1, k_ls2, k_ls3 (Householder, compact WY)
//   step 3  q'_i = w_i - Q_{i-1} y          -> k_project (rgs_project.hip): one coalesced pass
//   step 4  s'_i = Theta q'_i               -> fused into k_project as per-block partials
//                                              (k_gauss_cols on the stored column for small n)
//   steps 5-6  r_ii = ||s'_i||, s_i = s'_i / r_ii, and the Householder append of s_i
//                                           -> k_qa .. k_qd
//   step 7  q_i = q'_i / r_ii               -> done in the next column's k_project pass
//                                              (k_scale_col for the last column)
//
// Sketch-space state (fp64), for j columns factorised so far:
//   S_j = U_j [R_S; 0],  U_j = H_0 ... H_{j-1} = I - V Wm^T with Wm = V T
//   (compact WY; V unit lower trapezoidal), and X = R_S^{-1} kept explicitly.
//   V and Wm are stored twice: column-major (k x m) for row-parallel products
//   and row-major (k rows of m) for the column-parallel dot products.
// All cross-workgroup sums are taken in a fixed order, so results are
// bitwise reproducible run to run.

#include <algorithm>
#include <type_traits>

#include "rgs_map.hpp"
#include "rgs_step.hpp"

namespace rgs {

// SRHT diagonal D as a bit table: bit b of word w is set iff d_{32w+b} = -1.
// Word w comes from word (w mod 4) of Philox(w/4, 0xFFFFFFFF, sketch_id, instance).
__device__ __forceinline__ void srht_signs_body(uint32_t* __restrict__ signs, int64_t nwords, uint32_t k0,
                                                uint32_t k1, uint32_t sid, uint32_t inst, int64_t b) {
    if (4 * b >= nwords) return;
    uint32_t x[4];
    philox4x32_10((uint32_t)b, kTagSigns, sid, inst, k0, k1, x);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (4 * b + t < nwords) signs[4 * b + t] = x[t];
}

__global__ void k_srht_signs(uint32_t* __restrict__ signs, int64_t nwords, uint32_t k0, uint32_t k1,
                             uint32_t sid, uint32_t inst) {
    srht_signs_body(signs, nwords, k0, k1, sid, inst, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// The k sampled rows of the P-SRHT (partial Fisher-Yates over [0, s), the
// same draws and swaps as the host's draw: draw t uses Philox(t, 0xFFFFFFFE,
// sketch_id, instance) and swaps position t with t + floor((x1 2^32 + x0)
// (s - t) / 2^64); rows kept in draw order), for callers that cannot copy a
// host table.  One workgroup: the draws of 256 consecutive t are made in
// parallel, the swaps -- a sequential chain -- by one lane, on positions < k
// held directly and positions >= k (at most k of them are ever touched) in an
// open-addressing table, both in LDS (k <= kRowsDevMax).
constexpr int kRowsHashBits = 13;   // 8192 slots: load factor <= 1/2 for k <= 4096

__global__ __launch_bounds__(256) void k_srht_rows(int* __restrict__ rows, int64_t s, int k, uint32_t k0,
                                                   uint32_t k1, uint32_t sid, uint32_t inst) {
    __shared__ uint32_t low[kRowsDevMax];                       // value at position p < k
    __shared__ unsigned long long slot[1 << kRowsHashBits];     // (p + 1) << 32 | value for p >= k; 0 = empty
    __shared__ uint32_t draw[256];
    for (int p = threadIdx.x; p < k; p += 256) low[p] = (uint32_t)p;
    for (int p = threadIdx.x; p < (1 << kRowsHashBits); p += 256) slot[p] = 0ull;
    __syncthreads();
    for (int t0 = 0; t0 < k; t0 += 256) {
        const int t = t0 + (int)threadIdx.x;
        if (t < k) {
            uint32_t x[4];
            philox4x32_10((uint32_t)t, kTagRows, sid, inst, k0, k1, x);
            const uint64_t r64 = ((uint64_t)x[1] << 32) | x[0];
            draw[threadIdx.x] = (uint32_t)((uint64_t)t + __umul64hi(r64, (uint64_t)(s - t)));
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int nt = min(256, k - t0);
            for (int j = 0; j < nt; ++j) {
                const uint32_t tt = (uint32_t)(t0 + j), ii = draw[j];
                const uint32_t at = low[tt];
                uint32_t ai;
                if (ii < (uint32_t)k) {
                    ai = low[ii];
                    low[ii] = at;
                } else {
                    uint32_t h = (ii * 2654435761u) >> (32 - kRowsHashBits);
                    const unsigned long long key = (unsigned long long)(ii + 1u) << 32;
                    while (slot[h] != 0ull && (slot[h] & 0xFFFFFFFF00000000ull) != key)
                        h = (h + 1) & ((1u << kRowsHashBits) - 1);
                    ai = slot[h] == 0ull ? ii : (uint32_t)slot[h];
                    slot[h] = key | at;
                }
                low[tt] = ai;
                rows[tt] = (int)ai;
            }
        }
        __syncthreads();
    }
}

// Batched: map blocks are (factorisation, 256 groups of 4 sign words).
__global__ void kb_srht_signs(const BatchItem* __restrict__ items, BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    srht_signs_body(const_cast<uint32_t*>(it.sk.signs), (it.n + 31) / 32, it.sk.k0, it.sk.k1, it.sk.sid,
                    it.sk.inst, (int64_t)bm.y * blockDim.x + threadIdx.x);
}

// 16 rows of a lane loaded as T (a float or bf16 column widened to double: the
// step-1 sketches of the fp32 paths accumulate in fp64).
template <typename T, typename TX>
__device__ __forceinline__ void load16_as(const TX* __restrict__ p, const int64_t row0[4], int64_t n, bool full,
                                          T v[16]) {
    if constexpr (std::is_same<TX, T>::value) {
        load16(p, row0, n, full, v);
    } else {
        float t[16];   // TX is float or bf16 here
        load16(p, row0, n, full, t);
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = (T)t[e];
    }
}

// Partial sketches of ncols columns of X: workgroup (g, col) covers row blocks
// g, g + G, ... (NW * 1024 rows each) and writes partials[(col * G + g) * k + j].
// TX: element type of X (float, double or bf16); T: arithmetic and partial type.
// NW = 4 (256 threads) for k <= 4096, NW = 8 (512 threads) for k <= 8192.
template <typename TX, typename T, int SK, int NW = 4>
__device__ __forceinline__ void sketch_cols_body(const TX* __restrict__ X, int64_t ldx, int64_t n, int64_t nblk,
                                                 int G, const SketchArgs& sk, T* __restrict__ partials, int g,
                                                 int col, T* __restrict__ lds) {
    constexpr int NT = NW * kWave;
    const TX* x = X + (int64_t)col * ldx;
    T acc[kKptMax];
#pragma unroll
    for (int u = 0; u < kKptMax; ++u) acc[u] = T(0);
    const bool vec_ok = ((reinterpret_cast<uintptr_t>(x) & 15) == 0);
    for (int64_t blk = g; blk < nblk; blk += G) {
        int64_t row0[4];
        lane_rows<NW>(blk, row0);
        const bool full = vec_ok && (blk + 1) * (NW * kTile) <= n;
        T v[16];
        load16_as<T>(x, row0, n, full, v);
        block_sketch<T, T, SK, NW>(v, blk, n, sk, acc, lds);
    }
    T* out = partials + ((int64_t)col * G + g) * sk.k;
    const int kpt = (sk.k + NT - 1) / NT;
#pragma unroll
    for (int u = 0; u < kKptMax; ++u) {
        const int j = threadIdx.x + NT * u;
        if (u < kpt && j < sk.k) out[j] = acc[u];
    }
}

template <typename TX, typename T, int SK, int NW>
__global__ __launch_bounds__(NW * kWave) void k_sketch_cols(const TX* __restrict__ X, int64_t ldx, int64_t n,
                                                            int64_t nblk, int G, SketchArgs sk,
                                                            T* __restrict__ partials) {
    __shared__ T lds[NW * kTile];
    sketch_cols_body<TX, T, SK, NW>(X, ldx, n, nblk, G, sk, partials, blockIdx.x, blockIdx.y, lds);
}

// Batched step 1 (SRHT): map blocks are (factorisation, g + G_P * column).
// TA: accumulation type (fp64 on the fp32 path, as its single-factorisation
// step 1; the working precision on the bf16-basis path).
template <typename T, typename TA, int SK>
__global__ __launch_bounds__(kWG) void kb_sketch_cols(const BatchItem* __restrict__ items, BlockMap map) {
    __shared__ TA lds[kBlock];
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    sketch_cols_body<T, TA, SK>(static_cast<const T*>(it.W), it.ldw, it.n, (it.n + kBlock - 1) / kBlock, it.G_P,
                                it.sk, static_cast<TA*>(it.partP), bm.y % it.G_P, bm.y / it.G_P, lds);
}

// Gaussian sketch of ncols columns with every entry of Theta generated once
// per workgroup and applied to C columns (instead of once per column).
// Workgroup (g, jc, cc): sketch rows j = 256 jc + threadIdx.x, columns
// [C cc, C cc + C), row sub-blocks sb = g, g + G, ... of kGSub rows.  The
// sub-block of the C columns is staged in LDS column by column, so rows
// 4q..4q+3 of a column are one vector read; z(j, 4q..4q+3) comes from one
// Philox call.  Writes partials[(col * G + g) * k + j] (the k_reduce layout).
// TX: element type of X (float, double or bf16); T: arithmetic type.
constexpr int kGSub = 256;

__device__ __forceinline__ float elem_real(float v) { return v; }
__device__ __forceinline__ double elem_real(double v) { return v; }
__device__ __forceinline__ float elem_real(bf16 v) { return bf16_to_float(v.bits); }

template <typename TX, typename T, typename TA, int C, int SUB = kGSub>
__device__ __forceinline__ void gauss_cols_body(const TX* __restrict__ X, int64_t ldx, int64_t n, int ncols, int G,
                                                const SketchArgs& sk, TA* __restrict__ partials, int g, int jc,
                                                int cc, TA (*w)[SUB]) {
    const int j = jc * kWG + threadIdx.x;
    const int c0 = cc * C;
    const int nc = min(C, ncols - c0);
    TA acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = TA(0);
    const int64_t nsub = (n + SUB - 1) / SUB;
    for (int64_t sb = g; sb < nsub; sb += G) {
        const int64_t r0 = sb * SUB;
        for (int t = threadIdx.x; t < SUB; t += kWG) {
            const int64_t l = r0 + t;
#pragma unroll
            for (int c = 0; c < C; ++c) {   // clamped loads, masked after: no branch per load
                const TA x = (TA)elem_real(X[(int64_t)(c0 + min(c, nc - 1)) * ldx + min(l, n - 1)]);
                w[c][t] = (c < nc && l < n) ? x : TA(0);
            }
        }
        __syncthreads();
        if (j < sk.k) {
            const int64_t rem = n - r0;
            const int nq = rem >= SUB ? SUB / 4 : (int)((rem + 3) / 4);
            const uint32_t q0 = (uint32_t)(r0 / 4);
            for (int q = 0; q < nq; ++q) {
                T z[4];
                gauss4(q0 + (uint32_t)q, (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const TA x0 = w[c][4 * q], x1 = w[c][4 * q + 1], x2 = w[c][4 * q + 2], x3 = w[c][4 * q + 3];
                    acc[c] += (TA)z[0] * x0 + (TA)z[1] * x1 + (TA)z[2] * x2 + (TA)z[3] * x3;
                }
            }
        }
        __syncthreads();
    }
    if (j < sk.k) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c < nc) partials[((int64_t)(c0 + c) * G + g) * sk.k + j] = acc[c];
    }
}

template <typename TX, typename T, typename TA, int C, int SUB>
__global__ __launch_bounds__(kWG) void k_gauss_cols(const TX* __restrict__ X, int64_t ldx, int64_t n, int ncols,
                                                    int G, SketchArgs sk, TA* __restrict__ partials) {
    __shared__ __attribute__((aligned(16))) TA w[C][SUB];
    gauss_cols_body<TX, T, TA, C, SUB>(X, ldx, n, ncols, G, sk, partials, blockIdx.x, blockIdx.y, blockIdx.z, w);
}

// Rademacher counterpart of gauss_cols_body (same workgroup and partials
// layout): each Philox call gives the signs of 128 rows of sketch row j,
// applied to the C staged columns.  SUB is a multiple of 128.
template <typename TX, typename T, typename TA, int C, int SUB>
__device__ __forceinline__ void rad_cols_body(const TX* __restrict__ X, int64_t ldx, int64_t n, int ncols, int G,
                                              const SketchArgs& sk, TA* __restrict__ partials, int g, int jc, int cc,
                                              TA (*w)[SUB]) {
    static_assert(SUB % 128 == 0, "whole 128-row sign groups per sub-block");
    const int j = jc * kWG + threadIdx.x;
    const int c0 = cc * C;
    const int nc = min(C, ncols - c0);
    TA acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = TA(0);
    const int64_t nsub = (n + SUB - 1) / SUB;
    for (int64_t sb = g; sb < nsub; sb += G) {
        const int64_t r0 = sb * SUB;
        for (int t = threadIdx.x; t < SUB; t += kWG) {
            const int64_t l = r0 + t;
#pragma unroll
            for (int c = 0; c < C; ++c) {   // clamped loads, masked after: no branch per load
                const TA x = (TA)elem_real(X[(int64_t)(c0 + min(c, nc - 1)) * ldx + min(l, n - 1)]);
                w[c][t] = (c < nc && l < n) ? x : TA(0);
            }
        }
        __syncthreads();
        if (j < sk.k) {
            const int64_t rem = n - r0;
            const int ng = rem >= SUB ? SUB / 128 : (int)((rem + 127) / 128);
            const uint32_t b0 = (uint32_t)(r0 / 128);
            for (int q = 0; q < ng; ++q) {
                uint32_t wd[4];
                rad_words(b0 + (uint32_t)q, (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, wd);
#pragma unroll
                for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll 8
                    for (int r = 0; r < 32; ++r) {
                        const TA sg = rad_sign<TA>(wd[c4], r);
                        const int t = 128 * q + 32 * c4 + r;
#pragma unroll
                        for (int c = 0; c < C; ++c) acc[c] = fma(sg, w[c][t], acc[c]);
                    }
            }
        }
        __syncthreads();
    }
    if (j < sk.k) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c < nc) partials[((int64_t)(c0 + c) * G + g) * sk.k + j] = acc[c];
    }
}

template <typename TX, typename T, typename TA, int C, int SUB>
__global__ __launch_bounds__(kWG) void k_rad_cols(const TX* __restrict__ X, int64_t ldx, int64_t n, int ncols,
                                                  int G, SketchArgs sk, TA* __restrict__ partials) {
    __shared__ __attribute__((aligned(16))) TA w[C][SUB];
    rad_cols_body<TX, T, TA, C, SUB>(X, ldx, n, ncols, G, sk, partials, blockIdx.x, blockIdx.y, blockIdx.z, w);
}

// Register-blocked form of k_rad_cols for many columns (step 1, the
// certificate's sketches): a thread takes J sketch rows
// j = (jc J + jj) kWG + threadIdx.x and the workgroup's C staged columns, so
// each staged value read from LDS (the same address in every lane) feeds J
// fused multiply-adds and each sign feeds C.  Every (j, column) accumulator
// takes its products in the row order of rad_cols_body, so the partials are
// the same bits.  SUB is a multiple of 128.
template <typename TX, typename T, typename TA, int J, int C, int SUB>
__global__ __launch_bounds__(kWG) void k_rad_cols_rb(const TX* __restrict__ X, int64_t ldx, int64_t n, int ncols,
                                                     int G, SketchArgs sk, TA* __restrict__ partials) {
    static_assert(SUB % 128 == 0, "whole 128-row sign groups per sub-block");
    __shared__ __attribute__((aligned(16))) TA w[C][SUB];
    const int g = blockIdx.x, c0 = blockIdx.z * C;
    const int nc = min(C, ncols - c0);
    int jr[J];
#pragma unroll
    for (int jj = 0; jj < J; ++jj) jr[jj] = (blockIdx.y * J + jj) * kWG + threadIdx.x;
    TA acc[J][C];
#pragma unroll
    for (int jj = 0; jj < J; ++jj)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[jj][c] = TA(0);
    const int64_t nsub = (n + SUB - 1) / SUB;
    for (int64_t sb = g; sb < nsub; sb += G) {
        const int64_t r0 = sb * SUB;
        for (int e = threadIdx.x; e < C * SUB; e += kWG) {   // column-major staging: coalesced per column
            const int c = e / SUB, t = e - c * SUB;
            const int64_t l = r0 + t;
            const TA x = (TA)elem_real(X[(int64_t)(c0 + min(c, nc - 1)) * ldx + min(l, n - 1)]);
            w[c][t] = (c < nc && l < n) ? x : TA(0);
        }
        __syncthreads();
        const int64_t rem = n - r0;
        const int ng = rem >= SUB ? SUB / 128 : (int)((rem + 127) / 128);
        const uint32_t b0 = (uint32_t)(r0 / 128);
        for (int q = 0; q < ng; ++q) {
            uint32_t wd[J][4];
#pragma unroll
            for (int jj = 0; jj < J; ++jj)   // rows past k draw signs that are never stored
                rad_words(b0 + (uint32_t)q, (uint32_t)jr[jj], sk.sid, sk.inst, sk.k0, sk.k1, wd[jj]);
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll 4
                for (int r = 0; r < 32; ++r) {
                    const int t = 128 * q + 32 * c4 + r;
                    TA xv[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) xv[c] = w[c][t];
#pragma unroll
                    for (int jj = 0; jj < J; ++jj) {
                        const TA sg = rad_sign<TA>(wd[jj][c4], r);
#pragma unroll
                        for (int c = 0; c < C; ++c) acc[jj][c] = fma(sg, xv[c], acc[jj][c]);
                    }
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int jj = 0; jj < J; ++jj)
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (jr[jj] < sk.k && c < nc) partials[((int64_t)(c0 + c) * G + g) * sk.k + jr[jj]] = acc[jj][c];
}

// Table of the Gaussian sketch with bf16 entries: thread (o, j) draws
// z(j, 8o .. 8o+7) with the fp64 Box-Muller of two Philox quads, rounds each
// once to bf16 and writes the group as one 16-byte store at (o k + j) 8
// (rows past n hold 0).
__global__ void k_theta_table(SketchArgs sk, int64_t n, int64_t ngroups, uint16_t* __restrict__ table) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ngroups * sk.k) return;
    const int64_t o = idx / sk.k;
    const int j = (int)(idx - o * sk.k);
    double z[8];
    gauss4((uint32_t)(2 * o), (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z);
    gauss4((uint32_t)(2 * o + 1), (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z + 4);
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t l = 8 * o + 2 * t;
        const uint32_t lo = l < n ? bf16_rne_f64(z[2 * t]) : 0u;
        const uint32_t hi = l + 1 < n ? bf16_rne_f64(z[2 * t + 1]) : 0u;
        w[t] = lo | (hi << 16);
    }
    typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
    u32x4_t v;
    v.x = w[0];
    v.y = w[1];
    v.z = w[2];
    v.w = w[3];
    *reinterpret_cast<u32x4_t*>(table + idx * 8) = v;
}

// Exact table of the Gaussian sketch (SK_TABX): thread (o, j) draws
// z(j, 8o .. 8o+7) with the Box-Muller of the working type T -- the values the
// drawn pass computes -- and writes the group's 16-byte words at 16-byte
// indices (o W + w) k + j, W = 8 sizeof(T) / 16 (rows past n hold 0).
template <typename T>
__global__ void k_theta_tabx(SketchArgs sk, int64_t n, int64_t ngroups, T* __restrict__ table) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ngroups * sk.k) return;
    const int64_t o = idx / sk.k;
    const int j = (int)(idx - o * sk.k);
    T z[8];
    gauss4((uint32_t)(2 * o), (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z);
    gauss4((uint32_t)(2 * o + 1), (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z + 4);
#pragma unroll
    for (int r = 0; r < 8; ++r)
        if (8 * o + r >= n) z[r] = T(0);
    if constexpr (sizeof(T) == 4) {
        f32x4* p = reinterpret_cast<f32x4*>(table) + 2 * o * sk.k + j;
        f32x4 a, b;
        a.x = z[0]; a.y = z[1]; a.z = z[2]; a.w = z[3];
        b.x = z[4]; b.y = z[5]; b.z = z[6]; b.w = z[7];
        p[0] = a;
        p[sk.k] = b;
    } else {
        f64x2* p = reinterpret_cast<f64x2*>(table) + 4 * o * sk.k + j;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            f64x2 v;
            v.x = z[2 * h];
            v.y = z[2 * h + 1];
            p[h * sk.k] = v;
        }
    }
}

// Table counterpart of gauss_cols_body (same workgroup and partials layout):
// each 16-byte table load serves 8 rows of sketch row j for the C staged
// columns (EXACT: the SK_TABX table of the entries in T, 8 rows per 32- or
// 64-byte group).  SUB is a multiple of 8.
template <typename TX, typename T, typename TA, int C, int SUB, bool EXACT = false>
__device__ __forceinline__ void table_cols_body(const TX* __restrict__ X, int64_t ldx, int64_t n, int ncols, int G,
                                                const SketchArgs& sk, TA* __restrict__ partials, int g, int jc,
                                                int cc, TA (*w)[SUB]) {
    static_assert(SUB % 8 == 0, "whole 8-row table groups per sub-block");
    const int j = jc * kWG + threadIdx.x;
    const int c0 = cc * C;
    const int nc = min(C, ncols - c0);
    TA acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = TA(0);
    const int64_t nsub = (n + SUB - 1) / SUB;
    for (int64_t sb = g; sb < nsub; sb += G) {
        const int64_t r0 = sb * SUB;
        for (int t = threadIdx.x; t < SUB; t += kWG) {
            const int64_t l = r0 + t;
#pragma unroll
            for (int c = 0; c < C; ++c) {   // clamped loads, masked after: no branch per load
                const TA x = (TA)elem_real(X[(int64_t)(c0 + min(c, nc - 1)) * ldx + min(l, n - 1)]);
                w[c][t] = (c < nc && l < n) ? x : TA(0);
            }
        }
        __syncthreads();
        if (j < sk.k) {
            const int64_t rem = n - r0;
            const int no = rem >= SUB ? SUB / 8 : (int)((rem + 7) / 8);
            const int64_t o0 = r0 / 8;
            for (int o = 0; o < no; ++o) {
                TA z[8];
                if constexpr (EXACT) {
                    T ze[8];
                    tabx_unpack(tabx_load(static_cast<const T*>(sk.tabx), sk.k, o0 + o, j), ze);
#pragma unroll
                    for (int r = 0; r < 8; ++r) z[r] = (TA)ze[r];
                } else {
                    tab8<TA>(sk.table, sk.k, o0 + o, j, z);
                }
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const TA* x = w[c] + 8 * o;
                    acc[c] += z[0] * x[0] + z[1] * x[1] + z[2] * x[2] + z[3] * x[3];
                    acc[c] += z[4] * x[4] + z[5] * x[5] + z[6] * x[6] + z[7] * x[7];
                }
            }
        }
        __syncthreads();
    }
    if (j < sk.k) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c < nc) partials[((int64_t)(c0 + c) * G + g) * sk.k + j] = acc[c];
    }
}

template <typename TX, typename T, typename TA, int C, int SUB, bool EXACT = false>
__global__ __launch_bounds__(kWG) void k_table_cols(const TX* __restrict__ X, int64_t ldx, int64_t n, int ncols,
                                                    int G, SketchArgs sk, TA* __restrict__ partials) {
    __shared__ __attribute__((aligned(16))) TA w[C][SUB];
    table_cols_body<TX, T, TA, C, SUB, EXACT>(X, ldx, n, ncols, G, sk, partials, blockIdx.x, blockIdx.y, blockIdx.z,
                                              w);
}

// Batched step 1 (Gaussian): map blocks are (factorisation, g + G_P (jc + njc cc)).
template <typename T>
__global__ __launch_bounds__(kWG) void kb_gauss_cols(const BatchItem* __restrict__ items, BlockMap map) {
    __shared__ __attribute__((aligned(16))) T w[kGaussCols][kGSub];
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const int njc = (it.k + kWG - 1) / kWG;
    const int rest = bm.y / it.G_P;
    gauss_cols_body<T, T, T, kGaussCols>(static_cast<const T*>(it.W), it.ldw, it.n, it.m, it.G_P, it.sk,
                                      static_cast<T*>(it.partP), bm.y % it.G_P, rest % njc, rest / njc, w);
}

// ---------------------------------------------------------------------------
// The batched Gaussian sketch as dense products with the shared master matrix
// Z (instance 0; item b uses Z[0:k_b, 0:n_b] / sqrt(k_b)): for a tile of up to
// 64 operand columns x (each a column of some item's W or Q) and a chunk of
// `rows` rows, partial[x, j] = sum over the chunk's rows l of Z[j, l] x[l] --
// a (sketch rows) x (rows) times (rows) x (columns) product, done with fp32
// MFMA 32x32x2 (fp32 inputs: Z exact in fp32, x exact from bf16 or fp32;
// fp32 accumulation, as the VALU sketches).  Z is generated in registers, each
// entry once per work unit: wave w owns sketch rows 128 jt + 32 w + (0..31);
// lane L (jr = L % 32, kk = L / 32) draws the Philox quad of rows r + 4 kk ..
// r + 4 kk + 3 for sketch row jr, which is exactly its A operand for the four
// k-steps over rows r .. r + 7 (k-slot kk of step t is row r + 4 kk + t).  Its
// B operand for column x = L % 32 of each 32-column sub-tile is the same 4 rows
// of that column; the next 8 rows are loaded while the current ones are used.
// Accumulator t of the 32x32 result is sketch row 8 (t / 4) + 4 kk + t % 4 of
// column L % 32.  A wave whose 32 sketch rows all lie at or past the largest
// k of the unit's items has nothing to store and returns at once.
//   STEP4: the columns are column i of the listed items' Q (step 4 of the
//   column step; partial of chunk blk -> part[blk k_b + j]);
//   otherwise columns of W (step 1; partial of chunk blk of column c ->
//   partP[(c G_P + blk) k_b + j]).
// ---------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Rows r .. r+3 of a column (zeros past n); one 8-byte (bf16) or 16-byte
// (fp32) load when they are all present and the column is aligned.
template <typename TB>
__device__ __forceinline__ void ld4_rows(const TB* __restrict__ col, int64_t r, int64_t n, bool vec, float v[4]) {
    if constexpr (sizeof(TB) == 2) {
        const bf16* c = reinterpret_cast<const bf16*>(col);
        if (vec && r + 4 <= n) {
            const u32x2 t = *reinterpret_cast<const u32x2*>(c + r);
            v[0] = __uint_as_float(t.x << 16);
            v[1] = __uint_as_float(t.x & 0xFFFF0000u);
            v[2] = __uint_as_float(t.y << 16);
            v[3] = __uint_as_float(t.y & 0xFFFF0000u);
            return;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = (r + t < n) ? bf16_to_float(c[r + t].bits) : 0.f;
    } else {
        if (vec && r + 4 <= n) {
            const f32x4 t = *reinterpret_cast<const f32x4*>(col + r);
            v[0] = t.x;
            v[1] = t.y;
            v[2] = t.z;
            v[3] = t.w;
            return;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = (r + t < n) ? (float)col[r + t] : 0.f;
    }
}

// TABX: the entries are read from the exact fp32 table of the master matrix
// (RGS_FLAG_THETA_EXACT; the SK_TABX layout, whose 16-byte word q tk + j holds
// z(j, 4q .. 4q+3), made by the same fp32 Box-Muller) instead of drawn: the
// same A operands, so the same bits.
template <typename TB, bool STEP4, int NSUB, bool TABX = false>
__global__ __launch_bounds__(256) void kb_gauss_gemm(const BatchItem* __restrict__ items,
                                                     const GemmUnit* __restrict__ units, const int2* __restrict__ cols,
                                                     int rows, const float* __restrict__ tabx = nullptr, int tk = 0) {
    const GemmUnit un = units[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int jr = lane & 31, kk = lane >> 5;
    const int j = un.jt * 128 + wave * 32 + jr;   // this lane's sketch row (A operand)
    const TB* col[NSUB];
    int64_t nb[NSUB];
    bool vec[NSUB];
#pragma unroll
    for (int s2 = 0; s2 < NSUB; ++s2) {   // B operand: column x = lane % 32 of each 32-column sub-tile
        const int c = s2 * 32 + jr;
        col[s2] = nullptr;
        nb[s2] = 0;
        vec[s2] = false;
        if (c < un.count) {
            const int2 ic = cols[un.first + c];
            const BatchItem& it = items[ic.x];
            col[s2] = STEP4 ? static_cast<const TB*>(it.Q) + (int64_t)ic.y * it.ldq
                            : static_cast<const TB*>(it.W) + (int64_t)ic.y * it.ldw;
            nb[s2] = it.n;
            vec[s2] = it.vec_ok != 0;
        }
    }
    int kmax = 0;
    int64_t nmax = 0;
    for (int c = 0; c < un.count; ++c) {
        const BatchItem& it = items[cols[un.first + c].x];
        kmax = max(kmax, it.k);
        nmax = max(nmax, it.n);
    }
    if (un.jt * 128 + wave * 32 >= kmax) return;   // wave-uniform; the kernel has no barrier
    const SketchArgs& sk = items[cols[un.first].x].sk;   // seed, sketch id, instance: shared
    const int64_t r_begin = (int64_t)un.blk * rows;
    const int64_t r_end = min(r_begin + (int64_t)rows, nmax);
    f32x16 acc[NSUB];
    float b[NSUB][4];
#pragma unroll
    for (int s2 = 0; s2 < NSUB; ++s2) {
        acc[s2] = f32x16{0};
        ld4_rows(col[s2], r_begin + 4 * kk, col[s2] ? nb[s2] : 0, vec[s2], b[s2]);
    }
    for (int64_t r = r_begin; r < r_end; r += 8) {
        float z[4] = {0.f, 0.f, 0.f, 0.f};
        if (j < kmax) {
            if constexpr (TABX) {
                const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(tabx) +
                                                           (r / 4 + kk) * tk + j);
                z[0] = v.x;
                z[1] = v.y;
                z[2] = v.z;
                z[3] = v.w;
            } else {
                gauss4((uint32_t)(r / 4 + kk), (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z);
            }
        }
        float c[NSUB][4];
#pragma unroll
        for (int s2 = 0; s2 < NSUB; ++s2)
#pragma unroll
            for (int t = 0; t < 4; ++t) c[s2][t] = b[s2][t];
        if (r + 8 < r_end) {   // next 8 rows while these are used
#pragma unroll
            for (int s2 = 0; s2 < NSUB; ++s2)
                ld4_rows(col[s2], r + 8 + 4 * kk, col[s2] ? nb[s2] : 0, vec[s2], b[s2]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int s2 = 0; s2 < NSUB; ++s2)
                acc[s2] = __builtin_amdgcn_mfma_f32_32x32x2f32(z[t], c[s2][t], acc[s2], 0, 0, 0);
    }
#pragma unroll
    for (int s2 = 0; s2 < NSUB; ++s2) {
        const int c = s2 * 32 + jr;
        if (c >= un.count) continue;
        const int2 ic = cols[un.first + c];
        const BatchItem& it = items[ic.x];
        if (r_begin >= it.n) continue;
        float* out = STEP4 ? static_cast<float*>(it.part) + (int64_t)un.blk * it.k
                           : static_cast<float*>(it.partP) + ((int64_t)ic.y * it.G_P + un.blk) * it.k;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int jj = un.jt * 128 + wave * 32 + 8 * (t / 4) + 4 * kk + (t % 4);
            if (jj < it.k) out[jj] = acc[s2][t];
        }
    }
}

// The drawn products over 128-column tiles as a 128 x 128 output tile per
// workgroup: the four waves take the tile's four 32-column sub-tiles and share
// the unit's 128 sketch rows, whose entries the workgroup draws once per
// super-step of 32 rows into LDS (each of the 256 threads makes 4 Philox calls,
// 16 entries; double-buffered) instead of every wave drawing its own 32 sketch
// rows for its own columns: a quarter of the draws per column of the 32-column
// tiles.  Each output sees the k-steps of kb_gauss_gemm in the same order
// (k-step t of the 8-row step at r pairs rows r + t and r + 4 + t), so the
// partials are the same bits.
template <typename TB, bool STEP4, bool TABX = false>
__global__ __launch_bounds__(256) void kb_gauss_gemm_t128(const BatchItem* __restrict__ items,
                                                          const GemmUnit* __restrict__ units,
                                                          const int2* __restrict__ cols, int rows,
                                                          const float* __restrict__ tabx = nullptr, int tk = 0) {
    constexpr int R = 32;                            // rows per super-step
    __shared__ float zbuf[2][R][128];
    const GemmUnit un = units[blockIdx.x];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int jr = lane & 31, kk = lane >> 5;
    int kmax = 0;
    int64_t nmax = 0;
    for (int c = 0; c < un.count; ++c) {
        const BatchItem& it = items[cols[un.first + c].x];
        kmax = max(kmax, it.k);
        nmax = max(nmax, it.n);
    }
    if (un.jt * 128 >= kmax) return;                // workgroup-uniform: before any barrier
    const int nq = min(4, (kmax - un.jt * 128 + 31) / 32);
    const SketchArgs& sk = items[cols[un.first].x].sk;   // seed, sketch id, instance: shared
    const int c = wave * 32 + jr;
    const TB* col = nullptr;
    int64_t nb = 0;
    bool vec = false;
    if (c < un.count) {
        const int2 ic = cols[un.first + c];
        const BatchItem& it = items[ic.x];
        col = STEP4 ? static_cast<const TB*>(it.Q) + (int64_t)ic.y * it.ldq
                    : static_cast<const TB*>(it.W) + (int64_t)ic.y * it.ldw;
        nb = it.n;
        vec = it.vec_ok != 0;
    }
    const bool wave_has_cols = wave * 32 < un.count;   // wave-uniform
    const int64_t r_begin = (int64_t)un.blk * rows;     // rows is a multiple of R
    const int64_t r_end = min(r_begin + (int64_t)rows, nmax);
    // draw e = t + 256 p: Philox call for rows r + 4 (e >> 7) .. + 3 of sketch row 128 jt + (e & 127)
    auto draw = [&](int64_t r, float z[4][4]) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int e = t + 256 * p, jl = e & 127;
            const int j = un.jt * 128 + jl;
            z[p][0] = z[p][1] = z[p][2] = z[p][3] = 0.f;
            if (j < kmax) {
                if constexpr (TABX) {   // (kb_gauss_gemm: the table's word for the same Philox call)
                    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(tabx) +
                                                               (r / 4 + (e >> 7)) * tk + j);
                    z[p][0] = v.x;
                    z[p][1] = v.y;
                    z[p][2] = v.z;
                    z[p][3] = v.w;
                } else {
                    gauss4((uint32_t)(r / 4 + (e >> 7)), (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z[p]);
                }
            }
        }
    };
    auto store = [&](int buf, const float z[4][4]) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int e = t + 256 * p, q4 = e >> 7, jl = e & 127;
#pragma unroll
            for (int u = 0; u < 4; ++u) zbuf[buf][4 * q4 + u][jl] = z[p][u];
        }
    };
    f32x16 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f32x16{0};
    float b[R / 8][4];
    float z[4][4];
    draw(r_begin, z);
#pragma unroll
    for (int u = 0; u < R / 8; ++u) ld4_rows(col, r_begin + 8 * u + 4 * kk, col ? nb : 0, vec, b[u]);
    store(0, z);
    __syncthreads();
    int cur = 0;
    for (int64_t r = r_begin; r < r_end; r += R) {
        float cb[R / 8][4];
#pragma unroll
        for (int u = 0; u < R / 8; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) cb[u][v] = b[u][v];
        const int64_t rn = r + R;
        const bool more = rn < r_end;                  // workgroup-uniform
        if (more) {
#pragma unroll
            for (int u = 0; u < R / 8; ++u) ld4_rows(col, rn + 8 * u + 4 * kk, col ? nb : 0, vec, b[u]);
        }
        if (wave_has_cols) {
#pragma unroll
            for (int u = 0; u < R / 8; ++u) {
                if (r + 8 * u >= r_end) break;
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (q < nq)
                            acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(zbuf[cur][8 * u + 4 * kk + tt][32 * q + jr],
                                                                          cb[u][tt], acc[q], 0, 0, 0);
            }
        }
        if (more) {   // the next super-step's entries, drawn while the loads above are in flight
            draw(rn, z);
            store(cur ^ 1, z);
        }
        __syncthreads();
        cur ^= 1;
    }
    if (c >= un.count) return;
    const int2 ic = cols[un.first + c];
    const BatchItem& it = items[ic.x];
    if (r_begin >= it.n) return;
    float* out = STEP4 ? static_cast<float*>(it.part) + (int64_t)un.blk * it.k
                       : static_cast<float*>(it.partP) + ((int64_t)ic.y * it.G_P + un.blk) * it.k;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= nq) break;
#pragma unroll
        for (int tt = 0; tt < 16; ++tt) {
            const int jj = un.jt * 128 + 32 * q + 8 * (tt / 4) + 4 * kk + (tt % 4);
            if (jj < it.k) out[jj] = acc[q][tt];
        }
    }
}

// The same products with the bf16 Gaussian entries read from a table
// (RGS_FLAG_THETA_BF16: theta = bf16(z) / sqrt(k_b), the table holding the
// unscaled bf16(z) of the master matrix, group (o, j) of 8 columns at
// ((o tk) + j) 8) instead of drawn: bf16 MFMA 32x32x16 with fp32
// accumulation.  A bf16 column (the stored q'_i of the bf16 basis) is its own
// B operand, so every product theta x is exact before the fp32 accumulation;
// an fp32 column x is split exactly into three bf16 parts,
// x = hi + mid + lo (hi its leading 8 significand bits, mid the next 8, lo the
// last 8), and takes three MFMAs with the same A -- again exact products.
//
// The rows are walked in super-steps of 16 S rows (S k-steps of 16 rows; S = 4
// for bf16 columns, 2 for fp32).  The sum over rows does not care which rows
// form which k-step, so lane L (jr = L % 32, kk = L / 32) of wave w takes
// rows r + 8 S kk + 8 s .. + 7 as its k-slots of k-step s: its B operand for
// the whole super-step is 8 S contiguous rows of column jr of each 32-column
// sub-tile (the two kk lanes of a column together read 16 S contiguous rows,
// 128 bytes, one cache line), loaded one super-step ahead; its A operand for
// k-step s is table group r / 8 + S kk + s of sketch row
// j = 128 jt + 32 w + jr (16 bytes; the 32 lanes of one kk read 512
// contiguous bytes).  Accumulator t is sketch row 8 (t / 4) + 4 kk + t % 4 of
// column L % 32 (as for the fp32 MFMA), and the partials go where
// kb_gauss_gemm puts them.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));

// 8 S contiguous rows r .. r + 8 S - 1 of a column, raw: S u32x4v of 8 bf16
// (bf16 column) or 2 S of 4 fp32 bit patterns (fp32 column); zeros past n.
// The split into bf16 parts (split8) is left to the point of use, so the
// loads stay in flight meanwhile.
template <typename TB, int S>
struct RawRows {
    u32x4v w[sizeof(TB) == 2 ? S : 2 * S];
};

template <typename TB, int S>
__device__ __forceinline__ void ld_rows(const TB* __restrict__ col, int64_t r, int64_t n, bool vec,
                                        RawRows<TB, S>& out) {
    if constexpr (sizeof(TB) == 2) {
        const uint16_t* c = reinterpret_cast<const uint16_t*>(col);
        if (vec && r + 8 * S <= n) {   // columns start 8-byte aligned (ld a multiple of 4)
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const u32x2 lo = *reinterpret_cast<const u32x2*>(c + r + 8 * q);
                const u32x2 hi = *reinterpret_cast<const u32x2*>(c + r + 8 * q + 4);
                out.w[q] = u32x4v{lo.x, lo.y, hi.x, hi.y};
            }
            return;
        }
#pragma unroll
        for (int q = 0; q < S; ++q) {
            uint32_t w[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) w[t] = (r + 8 * q + t < n) ? (uint32_t)c[r + 8 * q + t] : 0u;
            out.w[q] = u32x4v{w[0] | (w[1] << 16), w[2] | (w[3] << 16), w[4] | (w[5] << 16), w[6] | (w[7] << 16)};
        }
    } else {
        if (vec && r + 8 * S <= n) {   // 16-byte aligned: ld a multiple of 4, r a multiple of 8
#pragma unroll
            for (int q = 0; q < 2 * S; ++q) out.w[q] = *reinterpret_cast<const u32x4v*>(col + r + 4 * q);
            return;
        }
#pragma unroll
        for (int q = 0; q < 2 * S; ++q) {
            uint32_t w[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) w[t] = (r + 4 * q + t < n) ? __float_as_uint((float)col[r + 4 * q + t]) : 0u;
            out.w[q] = u32x4v{w[0], w[1], w[2], w[3]};
        }
    }
}

// The B operands of k-step s of a super-step: the 8 bf16 words themselves, or
// the exact split of each of the 8 fp32 values x into hi + mid + lo (leading 8
// significand bits, the next 8, the last 8), three bf16x8 operands.
template <typename TB, int S>
__device__ __forceinline__ void split8(const RawRows<TB, S>& raw, int s, u32x4v parts[3]) {
    if constexpr (sizeof(TB) == 2) {
        parts[0] = raw.w[s];
    } else {
        uint32_t h[8], m[8], l[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const uint32_t bx = raw.w[2 * s + t / 4][t % 4];
            h[t] = bx >> 16;
            const float rem = __uint_as_float(bx) - __uint_as_float(bx & 0xFFFF0000u);   // exact
            const uint32_t bm = __float_as_uint(rem);
            m[t] = bm >> 16;
            l[t] = __float_as_uint(rem - __uint_as_float(bm & 0xFFFF0000u)) >> 16;   // exact: the last 8 bits
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            parts[0][q] = h[2 * q] | (h[2 * q + 1] << 16);
            parts[1][q] = m[2 * q] | (m[2 * q + 1] << 16);
            parts[2][q] = l[2 * q] | (l[2 * q + 1] << 16);
        }
    }
}

template <typename TB, bool STEP4, int NSUB>
__global__ __launch_bounds__(256) void kb_table_gemm(const BatchItem* __restrict__ items,
                                                     const GemmUnit* __restrict__ units, const int2* __restrict__ cols,
                                                     int rows, const uint16_t* __restrict__ table, int tk,
                                                     int64_t tgroups) {
    constexpr int NP = sizeof(TB) == 2 ? 1 : 3;   // bf16 parts per operand column
    constexpr int S = sizeof(TB) == 2 ? 4 : 2;    // k-steps per super-step
    const GemmUnit un = units[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int jr = lane & 31, kk = lane >> 5;
    const int j = un.jt * 128 + wave * 32 + jr;
    const TB* col[NSUB];
    int64_t nb[NSUB];
    bool vec[NSUB];
#pragma unroll
    for (int s2 = 0; s2 < NSUB; ++s2) {
        const int c = s2 * 32 + jr;
        col[s2] = nullptr;
        nb[s2] = 0;
        vec[s2] = false;
        if (c < un.count) {
            const int2 ic = cols[un.first + c];
            const BatchItem& it = items[ic.x];
            col[s2] = STEP4 ? static_cast<const TB*>(it.Q) + (int64_t)ic.y * it.ldq
                            : static_cast<const TB*>(it.W) + (int64_t)ic.y * it.ldw;
            nb[s2] = it.n;
            vec[s2] = it.vec_ok != 0;
        }
    }
    int kmax = 0;
    int64_t nmax = 0;
    for (int c = 0; c < un.count; ++c) {
        const BatchItem& it = items[cols[un.first + c].x];
        kmax = max(kmax, it.k);
        nmax = max(nmax, it.n);
    }
    if (un.jt * 128 + wave * 32 >= kmax) return;   // wave-uniform; the kernel has no barrier
    const bool jok = j < tk;
    // rows is a multiple of 16 S, so a super-step never crosses into the next
    // chunk; rows at or past nmax read zero columns (and zero table groups past
    // the table), so the last super-step may run past nmax
    const int64_t r_begin = (int64_t)un.blk * rows;
    const int64_t r_end = min(r_begin + (int64_t)rows, nmax);
    const uint16_t* trow = table + (int64_t)j * 8;
    auto load_a = [&](int64_t o) {
        return (jok && o < tgroups) ? *reinterpret_cast<const u32x4v*>(trow + o * tk * 8) : u32x4v{0u, 0u, 0u, 0u};
    };
    f32x16 acc[NSUB];
#pragma unroll
    for (int s2 = 0; s2 < NSUB; ++s2) acc[s2] = f32x16{0};
    RawRows<TB, S> b[NSUB];
    u32x4v a[S];
#pragma unroll
    for (int s2 = 0; s2 < NSUB; ++s2) ld_rows<TB, S>(col[s2], r_begin + 8 * S * kk, col[s2] ? nb[s2] : 0, vec[s2], b[s2]);
#pragma unroll
    for (int s = 0; s < S; ++s) a[s] = load_a(r_begin / 8 + S * kk + s);
    for (int64_t r = r_begin; r < r_end; r += 16 * S) {
        RawRows<TB, S> cb[NSUB];
        u32x4v ca[S];
#pragma unroll
        for (int s2 = 0; s2 < NSUB; ++s2) cb[s2] = b[s2];
#pragma unroll
        for (int s = 0; s < S; ++s) ca[s] = a[s];
        const int64_t rn = r + 16 * S;
        if (rn < r_end) {   // the next super-step's operands while these are used
#pragma unroll
            for (int s2 = 0; s2 < NSUB; ++s2)
                ld_rows<TB, S>(col[s2], rn + 8 * S * kk, col[s2] ? nb[s2] : 0, vec[s2], b[s2]);
#pragma unroll
            for (int s = 0; s < S; ++s) a[s] = load_a(rn / 8 + S * kk + s);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8_t av = __builtin_bit_cast(bf16x8_t, ca[s]);
#pragma unroll
            for (int s2 = 0; s2 < NSUB; ++s2) {
                u32x4v parts[3];
                split8<TB, S>(cb[s2], s, parts);
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    acc[s2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8_t, parts[p]),
                                                                      acc[s2], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int s2 = 0; s2 < NSUB; ++s2) {
        const int c = s2 * 32 + jr;
        if (c >= un.count) continue;
        const int2 ic = cols[un.first + c];
        const BatchItem& it = items[ic.x];
        if (r_begin >= it.n) continue;
        float* out = STEP4 ? static_cast<float*>(it.part) + (int64_t)un.blk * it.k
                           : static_cast<float*>(it.partP) + ((int64_t)ic.y * it.G_P + un.blk) * it.k;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int jj = un.jt * 128 + wave * 32 + 8 * (t / 4) + 4 * kk + (t % 4);
            if (jj < it.k) out[jj] = acc[s2][t];
        }
    }
}

// The table products over 128-column tiles as a 128 x 128 output tile per
// workgroup: the four waves take the tile's four 32-column sub-tiles, and all
// four share the unit's 128 sketch rows.  Per super-step the workgroup loads
// the table slice of those 128 sketch rows (2 S groups of 8 rows: 4 KiB per
// k-step pair, 16 KiB at S = 4) into LDS once, with 16-byte loads of whole
// contiguous rows of the table, double-buffered; each wave reads its A
// operands there (sketch sub-block q: table group r / 8 + S kk + s of sketch
// row 128 jt + 32 q + jr, as kb_table_gemm) and streams its own columns as B
// (the same contiguous row runs).  The table slice is so read once per 128
// columns instead of once per 32; the arithmetic per output (the same exact
// products, fp32 accumulation over the same k-steps in the same order) is that
// of kb_table_gemm, so the partials are the same bits.
template <typename TB, bool STEP4>
__global__ __launch_bounds__(256) void kb_table_gemm_t128(const BatchItem* __restrict__ items,
                                                          const GemmUnit* __restrict__ units,
                                                          const int2* __restrict__ cols, int rows,
                                                          const uint16_t* __restrict__ table, int tk, int64_t tgroups) {
    constexpr int NP = sizeof(TB) == 2 ? 1 : 3;
    constexpr int S = sizeof(TB) == 2 ? 4 : 2;
    constexpr int GS = 2 * S;                       // table groups (8 rows each) per super-step
    __shared__ u32x4v abuf[2][GS * 128];            // [buffer][group][sketch row], 16 bytes each
    const GemmUnit un = units[blockIdx.x];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int jr = lane & 31, kk = lane >> 5;
    int kmax = 0;
    int64_t nmax = 0;
    for (int c = 0; c < un.count; ++c) {
        const BatchItem& it = items[cols[un.first + c].x];
        kmax = max(kmax, it.k);
        nmax = max(nmax, it.n);
    }
    if (un.jt * 128 >= kmax) return;                // workgroup-uniform: before any barrier
    const int nq = min(4, (kmax - un.jt * 128 + 31) / 32);   // sketch sub-blocks with rows below kmax
    // this wave's column (B operand) of sub-tile `wave`
    const int c = wave * 32 + jr;
    const TB* col = nullptr;
    int64_t nb = 0;
    bool vec = false;
    if (c < un.count) {
        const int2 ic = cols[un.first + c];
        const BatchItem& it = items[ic.x];
        col = STEP4 ? static_cast<const TB*>(it.Q) + (int64_t)ic.y * it.ldq
                    : static_cast<const TB*>(it.W) + (int64_t)ic.y * it.ldw;
        nb = it.n;
        vec = it.vec_ok != 0;
    }
    const bool wave_has_cols = wave * 32 < un.count;   // wave-uniform
    const int64_t r_begin = (int64_t)un.blk * rows;     // rows is a multiple of 16 S
    const int64_t r_end = min(r_begin + (int64_t)rows, nmax);
    // cooperative A load: entry e = t + 256 p of the super-step's GS x 128 (group, sketch row) entries
    constexpr int AP = GS * 128 / 256;
    auto load_a = [&](int64_t r, u32x4v v[AP]) {
#pragma unroll
        for (int p = 0; p < AP; ++p) {
            const int e = t + 256 * p, g = e >> 7, jl = e & 127;
            const int64_t o = r / 8 + g;
            const int j = un.jt * 128 + jl;
            v[p] = (j < tk && o < tgroups) ? *reinterpret_cast<const u32x4v*>(table + (o * tk + j) * 8)
                                           : u32x4v{0u, 0u, 0u, 0u};
        }
    };
    f32x16 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f32x16{0};
    u32x4v av[AP];
    RawRows<TB, S> b;
    load_a(r_begin, av);
    ld_rows<TB, S>(col, r_begin + 8 * S * kk, col ? nb : 0, vec, b);
#pragma unroll
    for (int p = 0; p < AP; ++p) abuf[0][t + 256 * p] = av[p];
    __syncthreads();
    int cur = 0;
    for (int64_t r = r_begin; r < r_end; r += 16 * S) {
        const RawRows<TB, S> cb = b;
        const int64_t rn = r + 16 * S;
        const bool more = rn < r_end;                  // workgroup-uniform
        if (more) {   // the next super-step's operands while these are used
            load_a(rn, av);
            ld_rows<TB, S>(col, rn + 8 * S * kk, col ? nb : 0, vec, b);
        }
        if (wave_has_cols) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                u32x4v parts[3];
                split8<TB, S>(cb, s, parts);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q < nq) {
                        const bf16x8_t a_op = __builtin_bit_cast(bf16x8_t, abuf[cur][(S * kk + s) * 128 + 32 * q + jr]);
#pragma unroll
                        for (int pp = 0; pp < NP; ++pp)
                            acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                a_op, __builtin_bit_cast(bf16x8_t, parts[pp]), acc[q], 0, 0, 0);
                    }
                }
            }
        }
        if (more) {
#pragma unroll
            for (int p = 0; p < AP; ++p) abuf[cur ^ 1][t + 256 * p] = av[p];
        }
        __syncthreads();
        cur ^= 1;
    }
    if (c >= un.count) return;
    const int2 ic = cols[un.first + c];
    const BatchItem& it = items[ic.x];
    if (r_begin >= it.n) return;
    float* out = STEP4 ? static_cast<float*>(it.part) + (int64_t)un.blk * it.k
                       : static_cast<float*>(it.partP) + ((int64_t)ic.y * it.G_P + un.blk) * it.k;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= nq) break;
#pragma unroll
        for (int tt = 0; tt < 16; ++tt) {
            const int jj = un.jt * 128 + 32 * q + 8 * (tt / 4) + 4 * kk + (tt % 4);
            if (jj < it.k) out[jj] = acc[q][tt];
        }
    }
}

// out[j + col*ldo] = scale * sum_{g=0}^{G-1} partials[(col*G + g)*k + j], in fp64 and
// in a fixed order: 8 contiguous g-ranges summed by 8 threads, then combined in order.
// TR: the arithmetic of the sums (fp64; float32 for the unique-precision model,
// whose results are float32 values stored in the fp64 output).
template <typename PT, typename TR = double>
__device__ __forceinline__ void reduce_body(const PT* __restrict__ partials, int G, int k, double scale,
                                            double* __restrict__ out, int64_t ldo, int jb, int col) {
    __shared__ TR red[8][32];
    const int jl = threadIdx.x & 31, part = threadIdx.x >> 5;
    const int j = jb * 32 + jl;
    const int g0 = (int)((int64_t)G * part / 8), g1 = (int)((int64_t)G * (part + 1) / 8);
    TR s = TR(0);
    if (j < k) {
        const PT* p = partials + (int64_t)col * G * k + j;
        for (int g = g0; g < g1; ++g) s += (TR)p[(int64_t)g * k];
    }
    red[part][jl] = s;
    __syncthreads();
    if (part == 0 && j < k) {
        TR tot = TR(0);
#pragma unroll
        for (int t = 0; t < 8; ++t) tot += red[t][jl];
        out[j + (int64_t)col * ldo] = tot * (TR)scale;
    }
}

template <typename PT, typename TR = double>
__global__ __launch_bounds__(kWG) void k_reduce(const PT* __restrict__ partials, int G, int k,
                                                double scale, double* __restrict__ out, int64_t ldo) {
    reduce_body<PT, TR>(partials, G, k, scale, out, ldo, blockIdx.x, blockIdx.y);
}

// Batched: map blocks are (factorisation, 32-row chunk + ceil(k/32) * column) of P.
template <typename PT>
__global__ __launch_bounds__(kWG) void kb_reduce(const BatchItem* __restrict__ items, BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const int nj = (it.k + 31) / 32;
    reduce_body<PT>(static_cast<const PT*>(it.partP), it.G_P, it.k, it.sketch_scale, it.P, it.k, bm.y % nj,
                    bm.y / nj);
}

// Final step 7 for the last column: q = q' / r (fp64 reciprocal, rounded to T).
template <typename T>
__global__ void k_scale_col(T* __restrict__ q, int64_t n, const double* __restrict__ invr,
                            const int* __restrict__ status) {
    RGS_EXIT_IF_FAILED(status);
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n) q[l] = (T)((double)q[l] * invr[0]);
}

// Step 7 for bf16 storage, all columns at the end: q_c = fl_bf16(fl32(q'_c / r_cc)).
// Rows l0 .. l0+3 (l0 a multiple of 4) of every column; one 8-byte access per
// column when the columns are aligned (vec) and the 4 rows are all below n.
__device__ __forceinline__ void scale_cols_bf16_body(bf16* __restrict__ Q, int64_t ldq, int64_t n, int m,
                                                     const double* __restrict__ invr, int64_t l0, bool vec) {
    if (l0 >= n) return;
    auto scale = [](uint32_t h, double ir) -> uint32_t {
        return float_to_bf16((float)((double)bf16_to_float((uint16_t)h) * ir));
    };
    if (vec && l0 + 4 <= n) {
        for (int c = 0; c < m; ++c) {
            u32x2* p = reinterpret_cast<u32x2*>(Q + l0 + (int64_t)c * ldq);
            const double ir = invr[c];
            const u32x2 t = *p;
            u32x2 o;
            o.x = scale(t.x & 0xFFFFu, ir) | (scale(t.x >> 16, ir) << 16);
            o.y = scale(t.y & 0xFFFFu, ir) | (scale(t.y >> 16, ir) << 16);
            *p = o;
        }
        return;
    }
    for (int c = 0; c < m; ++c)
        for (int r = 0; r < 4 && l0 + r < n; ++r) {
            bf16* p = Q + l0 + r + (int64_t)c * ldq;
            p->bits = (uint16_t)scale(p->bits, invr[c]);
        }
}

__global__ void k_scale_cols_bf16(bf16* __restrict__ Q, int64_t ldq, int64_t n, int m,
                                  const double* __restrict__ invr, int vec, const int* __restrict__ status) {
    RGS_EXIT_IF_FAILED(status);
    scale_cols_bf16_body(Q, ldq, n, m, invr, 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x), vec != 0);
}

// Batched end of step 7: map blocks are (factorisation, block of 1024 rows),
// 4 rows per thread.
template <typename TQ, bool DEFER>
__global__ void kb_scale(const BatchItem* __restrict__ items, BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    RGS_EXIT_IF_FAILED(it.sa.status);
    const int64_t l0 = 4 * ((int64_t)bm.y * blockDim.x + threadIdx.x);
    if constexpr (DEFER) {
        scale_cols_bf16_body(static_cast<bf16*>(it.Q), it.ldq, it.n, it.m, it.sa.invr, l0, it.vec_ok != 0);
    } else {
        TQ* q = static_cast<TQ*>(it.Q) + (int64_t)(it.m - 1) * it.ldq;
        for (int r = 0; r < 4; ++r)
            if (l0 + r < it.n) q[l0 + r] = (TQ)((double)q[l0 + r] * it.sa.invr[it.m - 1]);
    }
}

// Batched: zero R and reset the status word of every factorisation.
__global__ void kb_init(const BatchItem* __restrict__ items, int nitems) {
    const int b = blockIdx.y;
    if (b >= nitems) return;
    const BatchItem& it = items[b];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (int64_t)it.m * it.m) it.R[idx % it.m + (idx / it.m) * it.ldr] = 0.0;
    if (idx < 4) it.sa.status[idx] = 0;
}

// Step 2 for a right-hand side p known only now (Arnoldi): part 1, per-slice
// partials of c = Wm_i^T p (c < i) and of ||p||^2 (slot i).
__global__ __launch_bounds__(kGW) void k_ls1(const double* __restrict__ p, int k, int i,
                                             const double* __restrict__ Wr, int mcap, double* __restrict__ pd) {
    __shared__ double xs[kSlice];
    const int s = blockIdx.x, r0 = s * kSlice;
    if (threadIdx.x < kSlice) xs[threadIdx.x] = (r0 + threadIdx.x < k) ? p[r0 + threadIdx.x] : 0.0;
    __syncthreads();
    double* out = pd + (int64_t)s * (mcap + 1);
    for (int c = threadIdx.x; c <= i; c += kGW) out[c] = (c < i) ? slice_dot(Wr, mcap, r0, k, xs, c) : slice_sq(xs);
}

template <typename TS = double>
__global__ __launch_bounds__(kGW) void k_ls2(const TS* __restrict__ p, int k, int i, int nsl,
                                             const TS* __restrict__ Vc, int mcap, const TS* __restrict__ pd,
                                             TS* __restrict__ uh, TS* __restrict__ pnorm) {
    extern __shared__ double cp_raw[];  // [i + 1]
    ls2_body<kGW, TS>(p, k, i, nsl, Vc, mcap, pd, uh, pnorm, blockIdx.x, reinterpret_cast<TS*>(cp_raw));
}

// The single-factorisation column-step kernels.  TS is the arithmetic of the
// sketch-space state: fp64, or float32 for the unique-precision model (the
// workspace buffers are sized for fp64 and hold TS values); R, S, rr and invr
// are fp64 arrays either way.  Dynamic LDS is sized by the launcher in fp64
// elements.
template <typename T, int NT = kGW, typename TS = double>
__global__ __launch_bounds__(NT) void k_ls3(int nr, int col, const TS* __restrict__ X, int mcap,
                                            const TS* __restrict__ uh, double* __restrict__ R,
                                            int64_t ldr, T* __restrict__ coef, const double* __restrict__ cscale) {
    extern __shared__ double us_raw[];  // [nr]
    ls3_body<T, NT, TS>(nr, col, X, mcap, uh, R, ldr, coef, cscale, blockIdx.x, reinterpret_cast<TS*>(us_raw));
}

template <typename PT, int NT = kGW, typename TS = double>
__global__ __launch_bounds__(NT) void k_qa(const PT* __restrict__ partials, int G, double scale,
                                           const double* __restrict__ src, int k, int i,
                                           const TS* __restrict__ Wr, int mcap, TS* __restrict__ sp,
                                           TS* __restrict__ pd, const double* __restrict__ scale2,
                                           int pstride = 0) {
    qa_body<PT, NT, TS>(partials, G, scale, src, k, i, Wr, mcap, sp, pd, blockIdx.x, scale2, pstride);
}

template <int NT = kGW, typename TS = double>
__global__ __launch_bounds__(NT) void k_qb(int k, int i, int nsl, const TS* __restrict__ sp,
                                            const TS* __restrict__ Vc, int mcap,
                                            const TS* __restrict__ pd, TS* __restrict__ u,
                                            TS* __restrict__ pd2, double* __restrict__ S, int64_t lds,
                                            double* __restrict__ R, int64_t ldr, double* __restrict__ rr,
                                            double* __restrict__ invr, const TS* __restrict__ pnorm,
                                            int* __restrict__ status) {
    extern __shared__ double c1_raw[];  // [i + 1]
    qb_body<NT, TS>(k, i, nsl, sp, Vc, mcap, pd, u, pd2, S, lds, R, ldr, rr, invr, pnorm, status, blockIdx.x,
                    reinterpret_cast<TS*>(c1_raw));
}

template <int NT = kGW, typename TS = double>
__global__ __launch_bounds__(NT) void k_qc(int k, int i, int nsl, const TS* __restrict__ u,
                                            const TS* __restrict__ pd2, const double* __restrict__ pn,
                                            TS* __restrict__ v, TS* __restrict__ Vc,
                                            TS* __restrict__ Vr, const TS* __restrict__ Wr, int mcap,
                                            TS* __restrict__ pd, TS* __restrict__ pdb,
                                            TS* __restrict__ tau_a, TS* __restrict__ beta_a,
                                            int* __restrict__ status) {
    qc_body<NT, TS>(k, i, nsl, u, pd2, pn, v, Vc, Vr, Wr, mcap, pd, pdb, tau_a, beta_a, status, blockIdx.x);
}

template <int NT = kGW, typename TS = double>
__global__ __launch_bounds__(NT) void k_qd(int k, int i, int nsl, const TS* __restrict__ v,
                                            const TS* __restrict__ u, const double* __restrict__ pn,
                                            TS* __restrict__ Wc, TS* __restrict__ Wr,
                                            const TS* __restrict__ Vc, int mcap, const TS* __restrict__ pd,
                                            const TS* __restrict__ pdb, TS* __restrict__ X,
                                            TS* __restrict__ uh, TS* __restrict__ pnorm,
                                            const TS* __restrict__ tau_a, const TS* __restrict__ beta_a) {
    extern __shared__ double dyn_raw[];  // [3 (i + 2)]
    qd_body<NT, TS>(k, i, nsl, v, u, pn, Wc, Wr, Vc, mcap, pd, pdb, X, uh, pnorm, tau_a, beta_a, blockIdx.x,
                    reinterpret_cast<TS*>(dyn_raw));
}

// ---------------------------------------------------------------------------
// Batched column steps: workgroup -> (factorisation, local block) through map.
// Every factorisation in the map is at column i.  pnext is P(:, i+1) when the
// factorisation has a column i+1, and nothing otherwise.
// ---------------------------------------------------------------------------
// TS: the sketch-space arithmetic (fp64, or float32 for the unique-precision
// GMRES systems); the workspace buffers hold TS values, R, S, rr and invr are fp64
template <typename PT, typename TS = double>
__global__ __launch_bounds__(kGWB) void kb_qa(const BatchItem* __restrict__ items, BlockMap map, int i) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    const bool from_p = (i == 0 && !it.defer && it.P != nullptr);   // GMRES systems carry no P
    qa_body<PT, kGWB, TS>(static_cast<const PT*>(it.part), it.npart, it.sketch_scale, from_p ? it.P : nullptr, a.k,
                          i, ws_as<TS>(a.Wr), a.mcap, ws_as<TS>(a.sp), ws_as<TS>(a.pd), bm.y);
}

template <typename TS = double>
__global__ __launch_bounds__(kGWB) void kb_qb(const BatchItem* __restrict__ items, BlockMap map, int i) {
    extern __shared__ double c1[];
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    qb_body<kGWB, TS>(a.k, i, it.nsl, ws_as<TS>(a.sp), ws_as<TS>(a.Vc), a.mcap, ws_as<TS>(a.pd), ws_as<TS>(a.u),
                      ws_as<TS>(a.pd2), it.S, it.lds, it.R, it.ldr, a.rr, a.invr, ws_as<TS>(a.pnorm), a.status, bm.y,
                      ws_as<TS>(c1));
}

template <typename TS = double>
__global__ __launch_bounds__(kGWB) void kb_qc(const BatchItem* __restrict__ items, BlockMap map, int i) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    const double* pn = (i + 1 < it.m && it.P) ? it.P + (int64_t)(i + 1) * a.k : nullptr;
    qc_body<kGWB, TS>(a.k, i, it.nsl, ws_as<TS>(a.u), ws_as<TS>(a.pd2), pn, ws_as<TS>(a.v), ws_as<TS>(a.Vc),
                      ws_as<TS>(a.Vr), ws_as<TS>(a.Wr), a.mcap, ws_as<TS>(a.pd), ws_as<TS>(a.pdb), ws_as<TS>(a.tau),
                      ws_as<TS>(a.beta), a.status, bm.y);
}

template <typename TS = double>
__global__ __launch_bounds__(kGWB) void kb_qd(const BatchItem* __restrict__ items, BlockMap map, int i) {
    extern __shared__ double dyn[];
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    const double* pn = (i + 1 < it.m && it.P) ? it.P + (int64_t)(i + 1) * a.k : nullptr;
    qd_body<kGWB, TS>(a.k, i, it.nsl, ws_as<TS>(a.v), ws_as<TS>(a.u), pn, ws_as<TS>(a.Wc), ws_as<TS>(a.Wr),
                      ws_as<TS>(a.Vc), a.mcap, ws_as<TS>(a.pd), ws_as<TS>(a.pdb), ws_as<TS>(a.X), ws_as<TS>(a.uh),
                      ws_as<TS>(a.pnorm), ws_as<TS>(a.tau), ws_as<TS>(a.beta), bm.y, ws_as<TS>(dyn));
}

template <typename TW>
__global__ __launch_bounds__(kGWB) void kb_ls3(const BatchItem* __restrict__ items, BlockMap map, int i) {
    extern __shared__ double us[];
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    ls3_body<TW, kGWB>(i + 1, i + 1, a.X, a.mcap, a.uh, it.R, it.ldr, static_cast<TW*>(it.coef),
                       it.defer ? a.invr : nullptr, bm.y, us);
}

// Step 2 by Richardson sweeps on the normal equations (remark on the
// least-squares solver, Sec. 2.3): the bodies and kGW-thread shape of the
// single-factorisation kernels, so a batched factorisation keeps the bits of a
// separate one.  The column step: s' and the slice partials of ||s'||^2 ...
template <typename PT>
__global__ __launch_bounds__(kGW) void kb_rqa(const BatchItem* __restrict__ items, BlockMap map, int i) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    const bool from_p = (i == 0 && !it.defer);
    qa_body<PT, kGW>(static_cast<const PT*>(it.part), it.npart, it.sketch_scale, from_p ? it.P : nullptr, a.k, 0,
                     a.Wr, a.mcap, a.sp, a.pd, bm.y);
}

// ... r_ii, s_i (both layouts), the breakdown test and, for a factorisation
// with a column i+1, the slice partials of S^T p_{i+1} and ||p_{i+1}||^2 ...
__global__ __launch_bounds__(kGW) void kb_rb(const BatchItem* __restrict__ items, BlockMap map, int i) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    const double* pn = (i + 1 < it.m) ? it.P + (int64_t)(i + 1) * a.k : nullptr;
    rb_body(a.k, i, it.nsl, a.sp, a.pd, a.mcap, it.S, it.lds, a.Wr, it.R, it.ldr, a.rr, a.invr, a.pnorm, a.status,
            pn, a.pdb, bm.y);
}

// ... the sums of a sweep (y, then R(0:i+1, i+1) and the coefficients of
// column i+1 after the last) ...
template <typename TW>
__global__ __launch_bounds__(kGW) void kb_rsum(const BatchItem* __restrict__ items, BlockMap map, int i,
                                              int accumulate, int last) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    rsum_body<TW>(i, it.nsl, a.mcap, a.pdb, a.uh, accumulate, last, a.pnorm, it.R, it.ldr,
                  static_cast<TW*>(it.coef), it.defer ? a.invr : nullptr, bm.y);
}

// ... and the residual partials of one more sweep.
__global__ __launch_bounds__(kGW) void kb_rres(const BatchItem* __restrict__ items, BlockMap map, int i) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    rres_body(a.k, i, a.mcap, it.S, it.lds, a.Wr, it.P + (int64_t)(i + 1) * a.k, a.uh, a.pdb, bm.y);
}

__global__ void k_zero_mat(double* __restrict__ A, int64_t rows, int64_t cols, int64_t lda) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    const int64_t r = idx % rows, c = idx / rows;
    A[r + c * lda] = 0.0;
}

// Dense block of Theta as the device generates it (test hook).
template <typename T, int SK>
__global__ void k_materialize(SketchArgs sk, int64_t j0, int64_t j1, int64_t l0, int64_t l1,
                              double rsk, double* __restrict__ out, int64_t ldo) {
    const int64_t nj = j1 - j0, nl = l1 - l0;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nj * nl) return;
    const int64_t jj = idx % nj, ll = idx / nj;
    const int64_t j = j0 + jj, l = l0 + ll;
    double val;
    if constexpr (SK == SK_GAUSS) {
        T z[4];
        gauss4((uint32_t)(l >> 2), (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z);
        val = (double)z[l & 3] * rsk;
    } else if constexpr (SK == SK_TABLE) {
        T z[8];
        tab8<T>(sk.table, sk.k, l >> 3, (int)j, z);
        val = (double)z[l & 7] * rsk;
    } else if constexpr (SK == SK_RADEM) {
        uint32_t wd[4];
        rad_words((uint32_t)(l >> 7), (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, wd);
        val = ((wd[(l >> 5) & 3] >> (l & 31)) & 1u) ? -rsk : rsk;
    } else if constexpr (SK == SK_SRHT) {
        const uint32_t rho = (uint32_t)sk.rows[j];
        const int par = __popcll((uint64_t)rho & (uint64_t)l) & 1;
        const int neg = (sk.signs[l >> 5] >> (l & 31)) & 1;
        val = ((par ^ neg) ? -1.0 : 1.0) * rsk;
    } else {
        val = (j == l) ? 1.0 : 0.0;
    }
    out[jj + ll * ldo] = val;
}

// Small fp64 product of the certification (Prop. 3.7): C = op(A) B with
// op(A) = A (M x K, column-major, lda) or A^T (A stored K x M), B K x N (ldb),
// C M x N (ldc).  64 x 64 output tile per workgroup, 16-deep slices of both
// operands staged in LDS; each thread owns a 4 x 4 block of the tile.
template <bool TA>
__global__ __launch_bounds__(kWG) void k_dgemm(int M, int N, int K, const double* __restrict__ A, int64_t lda,
                                               const double* __restrict__ B, int64_t ldb, double* __restrict__ C,
                                               int64_t ldc) {
    constexpr int TM = 64, TN = 64, TK = 16;
    __shared__ double As[TK][TM + 1];
    __shared__ double Bs[TK][TN + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < K; k0 += TK) {
        for (int e = threadIdx.x; e < TK * TM; e += kWG) {
            // consecutive threads walk the contiguous index of A
            const int kk = TA ? e % TK : e / TM, mm = TA ? e / TK : e % TM;
            const int gm = m0 + mm, gk = k0 + kk;
            double v = 0.0;
            if (gm < M && gk < K) v = TA ? A[gk + (int64_t)gm * lda] : A[gm + (int64_t)gk * lda];
            As[kk][mm] = v;
        }
        for (int e = threadIdx.x; e < TK * TN; e += kWG) {
            const int kk = e % TK, nn = e / TK;
            const int gn = n0 + nn, gk = k0 + kk;
            Bs[kk][nn] = (gn < N && gk < K) ? B[gk + (int64_t)gn * ldb] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
            if (gm < M && gn < N) C[gm + (int64_t)gn * ldc] = acc[i][j];
        }
}

// Step 8 diagnostics: per column a of S, sum_b (S^T S - I)_{ab}^2.
__global__ void k_diag_gram(const double* __restrict__ S, int64_t lds, int k, int m,
                            double* __restrict__ outcol) {
    __shared__ double red[kWG];
    const int a = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < m; b += kWG) {
        double g = 0.0;
        for (int r = 0; r < k; ++r) g = fma(S[r + (int64_t)a * lds], S[r + (int64_t)b * lds], g);
        if (a == b) g -= 1.0;
        acc += g * g;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kWG; ++q) t += red[q];
        outcol[a] = t;
    }
}

// Step 8 diagnostics: per column c, sum_r (P - S R)_{rc}^2 and sum_r P_{rc}^2.
__global__ void k_diag_resid(const double* __restrict__ P, int64_t ldp, const double* __restrict__ S,
                             int64_t lds, const double* __restrict__ R, int64_t ldr, int k, int m,
                             double* __restrict__ outcol) {
    __shared__ double red[2][kWG];
    const int c = blockIdx.x;
    double e2 = 0.0, p2 = 0.0;
    for (int r = threadIdx.x; r < k; r += kWG) {
        double acc = P[r + (int64_t)c * ldp];
        p2 += acc * acc;
        for (int a = 0; a <= c; ++a) acc -= S[r + (int64_t)a * lds] * R[a + (int64_t)c * ldr];
        e2 += acc * acc;
    }
    red[0][threadIdx.x] = e2;
    red[1][threadIdx.x] = p2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int q = 0; q < kWG; ++q) {
            t0 += red[0][q];
            t1 += red[1][q];
        }
        outcol[2 * c] = t0;
        outcol[2 * c + 1] = t1;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
#define RGS_LAUNCH_CHECK()                                   \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return false;   \
    } while (0)

static inline unsigned nblocks(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

bool launch_srht_signs(hipStream_t st, uint32_t* signs, int64_t nwords, const SketchArgs& sk) {
    const int64_t nthr = (nwords + 3) / 4;
    hipLaunchKernelGGL(k_srht_signs, dim3(nblocks(nthr, 256)), dim3(256), 0, st, signs, nwords, sk.k0,
                       sk.k1, sk.sid, sk.inst);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_srht_rows(hipStream_t st, int* rows, int64_t s, const SketchArgs& sk) {
    if (sk.k < 1 || sk.k > kRowsDevMax || s < sk.k || s > ((int64_t)1 << 31)) return false;
    hipLaunchKernelGGL(k_srht_rows, dim3(1), dim3(256), 0, st, rows, s, sk.k, sk.k0, sk.k1, sk.sid, sk.inst);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T, typename PT>
bool launch_sketch_cols(hipStream_t st, const T* X, int64_t ldx, int64_t n, int ncols, int G,
                        const SketchArgs& sk, PT* partials) {
    dim3 grid(G, ncols);
    if (sk.k > kKptMax * kWG) {   // 512 threads, 8192-row blocks
        const int64_t nblk = (n + kProjRows - 1) / kProjRows;
        if (sk.sketch == SK_SRHT)
            hipLaunchKernelGGL((k_sketch_cols<T, PT, SK_SRHT, kProjWaves>), grid, dim3(kProjWaves * kWave), 0, st, X,
                               ldx, n, nblk, G, sk, partials);
        else
            hipLaunchKernelGGL((k_sketch_cols<T, PT, SK_GAUSS, kProjWaves>), grid, dim3(kProjWaves * kWave), 0, st,
                               X, ldx, n, nblk, G, sk, partials);
    } else {
        const int64_t nblk = (n + kBlock - 1) / kBlock;
        if (sk.sketch == SK_SRHT)
            hipLaunchKernelGGL((k_sketch_cols<T, PT, SK_SRHT, 4>), grid, dim3(kWG), 0, st, X, ldx, n, nblk, G, sk,
                               partials);
        else
            hipLaunchKernelGGL((k_sketch_cols<T, PT, SK_GAUSS, 4>), grid, dim3(kWG), 0, st, X, ldx, n, nblk, G, sk,
                               partials);
    }
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TX, typename T, typename TA>
bool launch_gauss_cols(hipStream_t st, const TX* X, int64_t ldx, int64_t n, int ncols, int G, const SketchArgs& sk,
                       TA* partials) {
    const unsigned jc = nblocks(sk.k, kWG);
    const dim3 g1(G, jc, 1), gc(G, jc, nblocks(ncols, kGaussCols));
    // columns staged in LDS in TA: 32 x kGSub fp32 or 32 x kGSub/2 fp64 (32 KB)
    constexpr int SUBC = sizeof(TA) > sizeof(float) && sizeof(T) == sizeof(float) ? kGSub / 2 : kGSub;
    if (sk.sketch == SK_TABX) {
        if (ncols == 1)
            hipLaunchKernelGGL((k_table_cols<TX, T, TA, 1, kGSubCol, true>), g1, dim3(kWG), 0, st, X, ldx, n, 1, G, sk,
                               partials);
        else
            hipLaunchKernelGGL((k_table_cols<TX, T, TA, kGaussCols, SUBC, true>), gc, dim3(kWG), 0, st, X, ldx, n,
                               ncols, G, sk, partials);
    } else if (sk.sketch == SK_TABLE) {
        if (ncols == 1)
            hipLaunchKernelGGL((k_table_cols<TX, T, TA, 1, kGSubCol>), g1, dim3(kWG), 0, st, X, ldx, n, 1, G, sk,
                               partials);
        else
            hipLaunchKernelGGL((k_table_cols<TX, T, TA, kGaussCols, SUBC>), gc, dim3(kWG), 0, st, X, ldx, n, ncols,
                               G, sk, partials);
    } else if (sk.sketch == SK_RADEM) {
        if (ncols == 1)
            hipLaunchKernelGGL((k_rad_cols<TX, T, TA, 1, 128>), g1, dim3(kWG), 0, st, X, ldx, n, 1, G, sk, partials);
        else   // register-blocked: 4 sketch rows x 8 columns per thread (same bits as k_rad_cols)
            hipLaunchKernelGGL((k_rad_cols_rb<TX, T, TA, 4, 8, SUBC>),
                               dim3(G, nblocks(sk.k, 4 * kWG), nblocks(ncols, 8)), dim3(kWG), 0, st, X, ldx, n,
                               ncols, G, sk, partials);
    } else if (ncols == 1) {   // the single-column sketch of a small-n step: 64-row sub-blocks
        hipLaunchKernelGGL((k_gauss_cols<TX, T, TA, 1, kGSubCol>), g1, dim3(kWG), 0, st, X, ldx, n, 1, G, sk,
                           partials);
    } else {
        hipLaunchKernelGGL((k_gauss_cols<TX, T, TA, kGaussCols, SUBC>), gc, dim3(kWG), 0, st, X, ldx, n, ncols, G,
                           sk, partials);
    }
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TB, bool STEP4>
bool launch_batch_table_gemm(hipStream_t st, const BatchItem* items, const GemmUnit* units, int nunits,
                             const int2* cols, int rows, int tile, const uint16_t* table, int tk, int64_t tgroups) {
    if (nunits <= 0) return true;
    if (rows % 64 != 0) return false;   // whole super-steps per chunk
    if (tile <= 32)
        hipLaunchKernelGGL((kb_table_gemm<TB, STEP4, 1>), dim3(nunits), dim3(256), 0, st, items, units, cols, rows,
                           table, tk, tgroups);
    else if (tile <= 64)
        hipLaunchKernelGGL((kb_table_gemm<TB, STEP4, 2>), dim3(nunits), dim3(256), 0, st, items, units, cols, rows,
                           table, tk, tgroups);
    else if (tile <= 128)
        hipLaunchKernelGGL((kb_table_gemm_t128<TB, STEP4>), dim3(nunits), dim3(256), 0, st, items, units, cols, rows,
                           table, tk, tgroups);
    else
        return false;
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TB, bool STEP4>
bool launch_batch_gauss_gemm(hipStream_t st, const BatchItem* items, const GemmUnit* units, int nunits,
                             const int2* cols, int rows, int tile, const float* tabx, int tk) {
    if (nunits == 0) return true;
    if (tabx) {
        if (tile <= 32)
            hipLaunchKernelGGL((kb_gauss_gemm<TB, STEP4, 1, true>), dim3(nunits), dim3(256), 0, st, items, units,
                               cols, rows, tabx, tk);
        else if (tile <= 64)
            hipLaunchKernelGGL((kb_gauss_gemm<TB, STEP4, 2, true>), dim3(nunits), dim3(256), 0, st, items, units,
                               cols, rows, tabx, tk);
        else if (tile <= 128 && rows % 32 == 0)
            hipLaunchKernelGGL((kb_gauss_gemm_t128<TB, STEP4, true>), dim3(nunits), dim3(256), 0, st, items, units,
                               cols, rows, tabx, tk);
        else
            return false;
    } else if (tile <= 32) {
        hipLaunchKernelGGL((kb_gauss_gemm<TB, STEP4, 1>), dim3(nunits), dim3(256), 0, st, items, units, cols, rows,
                           nullptr, 0);
    } else if (tile <= 64) {
        hipLaunchKernelGGL((kb_gauss_gemm<TB, STEP4, 2>), dim3(nunits), dim3(256), 0, st, items, units, cols, rows,
                           nullptr, 0);
    } else if (tile <= 128 && rows % 32 == 0) {
        hipLaunchKernelGGL((kb_gauss_gemm_t128<TB, STEP4>), dim3(nunits), dim3(256), 0, st, items, units, cols, rows,
                           nullptr, 0);
    } else {
        return false;
    }
    RGS_LAUNCH_CHECK();
    return true;
}

// Step 1 for every factorisation of a batch: sign tables (SRHT), block
// partials of P_b = Theta_b W_b, and their reduction into P_b.
template <typename T>
bool launch_batch_sketch_p(hipStream_t st, int sketch, const BatchItem* items, const BlockMap& map_signs,
                           int64_t n_signs, const BlockMap& map_part, int64_t n_part, const BlockMap& map_red,
                           int64_t n_red, bool acc64) {
    const bool srht64 = sketch == SK_SRHT && acc64;
    if (sketch == SK_SRHT) {
        if (n_signs > 0) hipLaunchKernelGGL(kb_srht_signs, dim3(n_signs), dim3(256), 0, st, items, map_signs);
        RGS_LAUNCH_CHECK();
        if (n_part > 0 && srht64)
            hipLaunchKernelGGL((kb_sketch_cols<T, double, SK_SRHT>), dim3(n_part), dim3(kWG), 0, st, items, map_part);
        else if (n_part > 0)
            hipLaunchKernelGGL((kb_sketch_cols<T, T, SK_SRHT>), dim3(n_part), dim3(kWG), 0, st, items, map_part);
    } else if (n_part > 0) {
        hipLaunchKernelGGL(kb_gauss_cols<T>, dim3(n_part), dim3(kWG), 0, st, items, map_part);
    }
    RGS_LAUNCH_CHECK();
    if (n_red > 0) {
        if (srht64)
            hipLaunchKernelGGL(kb_reduce<double>, dim3(n_red), dim3(kWG), 0, st, items, map_red);
        else
            hipLaunchKernelGGL(kb_reduce<T>, dim3(n_red), dim3(kWG), 0, st, items, map_red);
    }
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename PT, typename TR>
bool launch_reduce(hipStream_t st, const PT* partials, int G, int k, int ncols, double scale, double* out,
                   int64_t ldo) {
    hipLaunchKernelGGL((k_reduce<PT, TR>), dim3(nblocks(k, 32), ncols), dim3(kWG), 0, st, partials, G, k, scale,
                       out, ldo);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T>
bool launch_scale_col(hipStream_t st, T* q, int64_t n, const double* invr, const int* status) {
    hipLaunchKernelGGL(k_scale_col<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, q, n, invr, status);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_scale_cols_bf16(hipStream_t st, bf16* Q, int64_t ldq, int64_t n, int m, const double* invr, int vec,
                            const int* status) {
    hipLaunchKernelGGL(k_scale_cols_bf16, dim3(nblocks(n, 1024)), dim3(256), 0, st, Q, ldq, n, m, invr, vec, status);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T>
bool launch_ls(hipStream_t st, const SpaceArgs& a, const double* p, int i, double* R, int64_t ldr, T* coef) {
    const int nsl = (a.k + kSlice - 1) / kSlice;
    hipLaunchKernelGGL(k_ls1, dim3(nsl), dim3(kGW), 0, st, p, a.k, i, a.Wr, a.mcap, a.pd);
    RGS_LAUNCH_CHECK();
    const unsigned nrb = nblocks(i, 64);
    hipLaunchKernelGGL(k_ls2<double>, dim3(nrb), dim3(kGW), (i + 1) * sizeof(double), st, p, a.k, i, nsl, a.Vc,
                       a.mcap, a.pd, a.uh, a.pnorm);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ls3<T>, dim3(nrb), dim3(kGW), (i + 1) * sizeof(double), st, i, i, a.X, a.mcap, a.uh, R,
                       ldr, coef, (const double*)nullptr);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T, typename PT, typename TS>
bool launch_ls_partials(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale, int i,
                        double* R, int64_t ldr, T* coef, const double* cscale, const double* scale2) {
    const int nsl = (a.k + kSlice - 1) / kSlice;
    auto ws = [](double* p) { return reinterpret_cast<TS*>(p); };   // the workspace in the sketch-space type
    hipLaunchKernelGGL((k_qa<PT, kGW, TS>), dim3(nsl), dim3(kGW), 0, st, partials, G, scale, (const double*)nullptr,
                       a.k, i, ws(a.Wr), a.mcap, ws(a.pbuf), ws(a.pd), scale2, 0);
    RGS_LAUNCH_CHECK();
    const unsigned nrb = nblocks(i, 64);
    hipLaunchKernelGGL(k_ls2<TS>, dim3(nrb), dim3(kGW), (i + 1) * sizeof(double), st, ws(a.pbuf), a.k, i, nsl,
                       ws(a.Vc), a.mcap, ws(a.pd), ws(a.uh), ws(a.pnorm));
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_ls3<T, kGW, TS>), dim3(nrb), dim3(kGW), (i + 1) * sizeof(double), st, i, i, ws(a.X),
                       a.mcap, ws(a.uh), R, ldr, coef, cscale);
    RGS_LAUNCH_CHECK();
    return true;
}

__global__ __launch_bounds__(kGW) void k_rb(int k, int i, int nsl, const double* __restrict__ sp,
                                            const double* __restrict__ pd, int mcap, double* __restrict__ S,
                                            int64_t lds, double* __restrict__ Sr, double* __restrict__ R, int64_t ldr,
                                            double* __restrict__ rr, double* __restrict__ invr,
                                            const double* __restrict__ pnorm, int* __restrict__ status,
                                            const double* __restrict__ pn, double* __restrict__ pdb) {
    rb_body(k, i, nsl, sp, pd, mcap, S, lds, Sr, R, ldr, rr, invr, pnorm, status, pn, pdb, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kGW) void k_rsum(int i, int nsl, int mcap, const double* __restrict__ pdb,
                                              double* __restrict__ y, int accumulate, int last,
                                              double* __restrict__ pnorm, double* __restrict__ R, int64_t ldr,
                                              T* __restrict__ coef, const double* __restrict__ cscale) {
    rsum_body<T>(i, nsl, mcap, pdb, y, accumulate, last, pnorm, R, ldr, coef, cscale, blockIdx.x);
}

__global__ __launch_bounds__(kGW) void k_rres(int k, int i, int mcap, const double* __restrict__ Sc, int64_t lds,
                                              const double* __restrict__ Sr, const double* __restrict__ pn,
                                              const double* __restrict__ y, double* __restrict__ pdb) {
    rres_body(k, i, mcap, Sc, lds, Sr, pn, y, pdb, blockIdx.x);
}

// Step 2 for the Arnoldi right-hand side p_i (block partials of the mat-vec
// kernel, times scale2[0] when given) by `sweeps` Richardson iterations on the
// normal equations with S_i (kept row-major in Wr by the Richardson column
// step): p_i into pbuf with the slice partials of S_i^T p_i and ||p_i||^2 in
// one pass, then the sweeps as in the QR chain (y = S^T p, y += S^T (p - S y)).
template <typename T, typename PT>
bool launch_ls_partials_richardson(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale, int i,
                                   double* S, int64_t lds, double* R, int64_t ldr, T* coef, const double* cscale,
                                   const double* scale2, int sweeps) {
    if (i < 1 || sweeps < 1) return false;
    const int nsl = (a.k + kSlice - 1) / kSlice;
    hipLaunchKernelGGL(k_qa<PT>, dim3(nsl), dim3(kGW), 0, st, partials, G, scale, (const double*)nullptr, a.k, i,
                       a.Wr, a.mcap, a.pbuf, a.pdb, scale2, a.mcap + 2);
    RGS_LAUNCH_CHECK();
    const unsigned nb = nblocks(i, kGW);
    for (int sw = 0; sw < sweeps; ++sw) {
        const int last = sw + 1 == sweeps;
        hipLaunchKernelGGL(k_rsum<T>, dim3(nb), dim3(kGW), 0, st, i - 1, nsl, a.mcap, a.pdb, a.uh, sw > 0 ? 1 : 0,
                           last, a.pnorm, R, ldr, coef, cscale);
        RGS_LAUNCH_CHECK();
        if (!last) {
            hipLaunchKernelGGL(k_rres, dim3(nsl), dim3(kGW), 0, st, a.k, i - 1, a.mcap, S, lds, a.Wr, a.pbuf, a.uh,
                               a.pdb);
            RGS_LAUNCH_CHECK();
        }
    }
    return true;
}

// The column step with step 2 by `sweeps` Richardson iterations (sweeps >= 1).
template <typename T, typename PT>
bool launch_column_richardson(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale,
                              const double* src, int i, double* S, int64_t lds, double* R, int64_t ldr,
                              const double* pnext, T* coef, const double* cscale, int sweeps) {
    const int nsl = (a.k + kSlice - 1) / kSlice;
    // s' and the slice partials of ||s'||^2 (slot 0)
    hipLaunchKernelGGL(k_qa<PT>, dim3(nsl), dim3(kGW), 0, st, partials, G, scale, src, a.k, 0, a.Wr, a.mcap, a.sp,
                       a.pd, (const double*)nullptr);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rb, dim3(nsl), dim3(kGW), 0, st, a.k, i, nsl, a.sp, a.pd, a.mcap, S, lds, a.Wr, R, ldr, a.rr,
                       a.invr, a.pnorm, a.status, pnext, a.pdb);
    RGS_LAUNCH_CHECK();
    if (!pnext) return true;
    const unsigned nb = nblocks(i + 1, kGW);
    for (int sw = 0; sw < sweeps; ++sw) {
        const int last = sw + 1 == sweeps;
        hipLaunchKernelGGL(k_rsum<T>, dim3(nb), dim3(kGW), 0, st, i, nsl, a.mcap, a.pdb, a.uh, sw > 0 ? 1 : 0, last,
                           a.pnorm, R, ldr, coef, cscale);
        RGS_LAUNCH_CHECK();
        if (!last) {
            hipLaunchKernelGGL(k_rres, dim3(nsl), dim3(kGW), 0, st, a.k, i, a.mcap, S, lds, a.Wr, pnext, a.uh, a.pdb);
            RGS_LAUNCH_CHECK();
        }
    }
    return true;
}

template <typename T, typename PT, typename TS>
bool launch_column(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale,
                   const double* src, int i, double* S, int64_t lds, double* R, int64_t ldr,
                   const double* pnext, T* coef, const double* cscale) {
    const int nsl = (a.k + kSlice - 1) / kSlice;
    constexpr int NT = kGWS;
    auto ws = [](double* p) { return reinterpret_cast<TS*>(p); };   // the workspace in the sketch-space type
    hipLaunchKernelGGL((k_qa<PT, NT, TS>), dim3(nsl), dim3(NT), 0, st, partials, G, scale, src, a.k, i, ws(a.Wr),
                       a.mcap, ws(a.sp), ws(a.pd), (const double*)nullptr, 0);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_qb<NT, TS>), dim3(nsl), dim3(NT), (i + 1) * sizeof(double), st, a.k, i, nsl, ws(a.sp),
                       ws(a.Vc), a.mcap, ws(a.pd), ws(a.u), ws(a.pd2), S, lds, R, ldr, a.rr, a.invr, ws(a.pnorm),
                       a.status);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_qc<NT, TS>), dim3(nsl), dim3(NT), 0, st, a.k, i, nsl, ws(a.u), ws(a.pd2), pnext, ws(a.v),
                       ws(a.Vc), ws(a.Vr), ws(a.Wr), a.mcap, ws(a.pd), ws(a.pdb), ws(a.tau), ws(a.beta), a.status);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_qd<NT, TS>), dim3(nsl + nblocks(i + 1, 64)), dim3(NT), 3 * (i + 2) * sizeof(double), st,
                       a.k, i, nsl, ws(a.v), ws(a.u), pnext, ws(a.Wc), ws(a.Wr), ws(a.Vc), a.mcap, ws(a.pd),
                       ws(a.pdb), ws(a.X), ws(a.uh), ws(a.pnorm), ws(a.tau), ws(a.beta));
    RGS_LAUNCH_CHECK();
    if (pnext) {
        hipLaunchKernelGGL((k_ls3<T, NT, TS>), dim3(nblocks(i + 1, 64)), dim3(NT), (i + 1) * sizeof(double), st,
                           i + 1, i + 1, ws(a.X), a.mcap, ws(a.uh), R, ldr, coef, cscale);
        RGS_LAUNCH_CHECK();
    }
    return true;
}

// ---- batched launchers: one launch per column step for every factorisation in the map ----
bool launch_batch_init(hipStream_t st, const BatchItem* items, int nitems, int64_t max_m2) {
    hipLaunchKernelGGL(kb_init, dim3(nblocks(std::max<int64_t>(max_m2, 4), 256), nitems), dim3(256), 0, st, items,
                       nitems);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TW, typename TS>
bool launch_batch_column(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t n_sl,
                         const BlockMap& map_qd, int64_t n_qd, const BlockMap& map_ls, int64_t n_ls, int i) {
    if (!std::is_same<TS, double>::value && n_ls > 0) return false;   // kb_ls3 reads an fp64 workspace
    if (n_sl > 0) {
        hipLaunchKernelGGL((kb_qa<TW, TS>), dim3(n_sl), dim3(kGWB), 0, st, items, map_sl, i);
        RGS_LAUNCH_CHECK();
        hipLaunchKernelGGL(kb_qb<TS>, dim3(n_sl), dim3(kGWB), (i + 1) * sizeof(double), st, items, map_sl, i);
        RGS_LAUNCH_CHECK();
        hipLaunchKernelGGL(kb_qc<TS>, dim3(n_sl), dim3(kGWB), 0, st, items, map_sl, i);
        RGS_LAUNCH_CHECK();
    }
    if (n_qd > 0) {
        hipLaunchKernelGGL(kb_qd<TS>, dim3(n_qd), dim3(kGWB), 3 * (i + 2) * sizeof(double), st, items, map_qd, i);
        RGS_LAUNCH_CHECK();
    }
    if (n_ls > 0) {
        hipLaunchKernelGGL(kb_ls3<TW>, dim3(n_ls), dim3(kGWB), (i + 1) * sizeof(double), st, items, map_ls, i);
        RGS_LAUNCH_CHECK();
    }
    return true;
}

template <typename TW>
bool launch_batch_column_richardson(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t n_sl,
                                    const BlockMap& map_next, int64_t n_next, const BlockMap& map_rs, int64_t n_rs,
                                    int i, int sweeps) {
    if (sweeps < 1) return false;
    if (n_sl > 0) {
        hipLaunchKernelGGL(kb_rqa<TW>, dim3(n_sl), dim3(kGW), 0, st, items, map_sl, i);
        RGS_LAUNCH_CHECK();
        hipLaunchKernelGGL(kb_rb, dim3(n_sl), dim3(kGW), 0, st, items, map_sl, i);
        RGS_LAUNCH_CHECK();
    }
    if (n_rs == 0) return true;   // no factorisation has a column i+1
    for (int sw = 0; sw < sweeps; ++sw) {
        const int last = sw + 1 == sweeps;
        hipLaunchKernelGGL(kb_rsum<TW>, dim3(n_rs), dim3(kGW), 0, st, items, map_rs, i, sw > 0 ? 1 : 0, last);
        RGS_LAUNCH_CHECK();
        if (!last) {
            hipLaunchKernelGGL(kb_rres, dim3(n_next), dim3(kGW), 0, st, items, map_next, i);
            RGS_LAUNCH_CHECK();
        }
    }
    return true;
}

template <typename TQ, bool DEFER>
bool launch_batch_scale(hipStream_t st, const BatchItem* items, const BlockMap& map, int64_t nblk) {
    if (nblk == 0) return true;
    hipLaunchKernelGGL((kb_scale<TQ, DEFER>), dim3(nblk), dim3(256), 0, st, items, map);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_zero_mat(hipStream_t st, double* A, int64_t rows, int64_t cols, int64_t lda) {
    if (rows * cols == 0) return true;
    hipLaunchKernelGGL(k_zero_mat, dim3(nblocks(rows * cols, 256)), dim3(256), 0, st, A, rows, cols, lda);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T>
bool launch_materialize(hipStream_t st, const SketchArgs& sk, int64_t j0, int64_t j1, int64_t l0, int64_t l1,
                        double rsk, double* out, int64_t ldo) {
    const int64_t cnt = (j1 - j0) * (l1 - l0);
    if (cnt == 0) return true;
    const dim3 g(nblocks(cnt, 256)), b(256);
    if (sk.sketch == SK_GAUSS)
        hipLaunchKernelGGL((k_materialize<T, SK_GAUSS>), g, b, 0, st, sk, j0, j1, l0, l1, rsk, out, ldo);
    else if (sk.sketch == SK_RADEM)
        hipLaunchKernelGGL((k_materialize<T, SK_RADEM>), g, b, 0, st, sk, j0, j1, l0, l1, rsk, out, ldo);
    else if (sk.sketch == SK_TABLE)
        hipLaunchKernelGGL((k_materialize<T, SK_TABLE>), g, b, 0, st, sk, j0, j1, l0, l1, rsk, out, ldo);
    else if (sk.sketch == SK_SRHT)
        hipLaunchKernelGGL((k_materialize<T, SK_SRHT>), g, b, 0, st, sk, j0, j1, l0, l1, rsk, out, ldo);
    else
        hipLaunchKernelGGL((k_materialize<T, SK_IDENT>), g, b, 0, st, sk, j0, j1, l0, l1, rsk, out, ldo);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_theta_table(hipStream_t st, const SketchArgs& sk, int64_t n, uint16_t* table) {
    const int64_t ngroups = (n + 7) / 8;
    const int64_t work = ngroups * sk.k;
    hipLaunchKernelGGL(k_theta_table, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, sk, n, ngroups, table);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T>
bool launch_theta_tabx(hipStream_t st, const SketchArgs& sk, int64_t n, T* table) {
    const int64_t ngroups = (n + 7) / 8;
    const int64_t work = ngroups * sk.k;
    hipLaunchKernelGGL(k_theta_tabx<T>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, sk, n, ngroups,
                       table);
    RGS_LAUNCH_CHECK();
    return true;
}
template bool launch_theta_tabx<float>(hipStream_t, const SketchArgs&, int64_t, float*);
template bool launch_theta_tabx<double>(hipStream_t, const SketchArgs&, int64_t, double*);

bool launch_dgemm(hipStream_t st, bool transA, int M, int N, int K, const double* A, int64_t lda, const double* B,
                  int64_t ldb, double* C, int64_t ldc) {
    if (M <= 0 || N <= 0) return true;
    const dim3 grid(nblocks(M, 64), nblocks(N, 64));
    if (transA)
        hipLaunchKernelGGL(k_dgemm<true>, grid, dim3(kWG), 0, st, M, N, K, A, lda, B, ldb, C, ldc);
    else
        hipLaunchKernelGGL(k_dgemm<false>, grid, dim3(kWG), 0, st, M, N, K, A, lda, B, ldb, C, ldc);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_diagnostics(hipStream_t st, const double* P, int64_t ldp, const double* S, int64_t lds,
                        const double* R, int64_t ldr, int k, int m, double* gram_out, double* resid_out) {
    hipLaunchKernelGGL(k_diag_gram, dim3(m), dim3(kWG), 0, st, S, lds, k, m, gram_out);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_diag_resid, dim3(m), dim3(kWG), 0, st, P, ldp, S, lds, R, ldr, k, m, resid_out);
    RGS_LAUNCH_CHECK();
    return true;
}

// explicit instantiations
template bool launch_sketch_cols<float, float>(hipStream_t, const float*, int64_t, int64_t, int, int,
                                               const SketchArgs&, float*);
template bool launch_sketch_cols<double, double>(hipStream_t, const double*, int64_t, int64_t, int, int,
                                                 const SketchArgs&, double*);
template bool launch_sketch_cols<bf16, float>(hipStream_t, const bf16*, int64_t, int64_t, int, int,
                                              const SketchArgs&, float*);
template bool launch_sketch_cols<float, double>(hipStream_t, const float*, int64_t, int64_t, int, int,
                                                const SketchArgs&, double*);
template bool launch_sketch_cols<bf16, double>(hipStream_t, const bf16*, int64_t, int64_t, int, int,
                                               const SketchArgs&, double*);
template bool launch_gauss_cols<float, float, float>(hipStream_t, const float*, int64_t, int64_t, int, int,
                                                     const SketchArgs&, float*);
template bool launch_gauss_cols<double, double, double>(hipStream_t, const double*, int64_t, int64_t, int, int,
                                                        const SketchArgs&, double*);
template bool launch_gauss_cols<bf16, float, float>(hipStream_t, const bf16*, int64_t, int64_t, int, int,
                                                    const SketchArgs&, float*);
template bool launch_gauss_cols<float, float, double>(hipStream_t, const float*, int64_t, int64_t, int, int,
                                                      const SketchArgs&, double*);
template bool launch_gauss_cols<bf16, float, double>(hipStream_t, const bf16*, int64_t, int64_t, int, int,
                                                     const SketchArgs&, double*);
template bool launch_reduce<float>(hipStream_t, const float*, int, int, int, double, double*, int64_t);
template bool launch_reduce<float, float>(hipStream_t, const float*, int, int, int, double, double*, int64_t);
template bool launch_reduce<double>(hipStream_t, const double*, int, int, int, double, double*, int64_t);
template bool launch_scale_col<float>(hipStream_t, float*, int64_t, const double*, const int*);
template bool launch_scale_col<double>(hipStream_t, double*, int64_t, const double*, const int*);
template bool launch_ls<float>(hipStream_t, const SpaceArgs&, const double*, int, double*, int64_t, float*);
template bool launch_ls<double>(hipStream_t, const SpaceArgs&, const double*, int, double*, int64_t, double*);
template bool launch_ls_partials<float, float>(hipStream_t, const SpaceArgs&, const float*, int, double, int,
                                               double*, int64_t, float*, const double*, const double*);
template bool launch_ls_partials<double, double>(hipStream_t, const SpaceArgs&, const double*, int, double, int,
                                                 double*, int64_t, double*, const double*, const double*);
template bool launch_ls_partials<float, float, float>(hipStream_t, const SpaceArgs&, const float*, int, double, int,
                                                      double*, int64_t, float*, const double*, const double*);
template bool launch_ls_partials_richardson<float, float>(hipStream_t, const SpaceArgs&, const float*, int, double,
                                                          int, double*, int64_t, double*, int64_t, float*,
                                                          const double*, const double*, int);
template bool launch_ls_partials_richardson<double, double>(hipStream_t, const SpaceArgs&, const double*, int, double,
                                                            int, double*, int64_t, double*, int64_t, double*,
                                                            const double*, const double*, int);
template bool launch_column_richardson<float, float>(hipStream_t, const SpaceArgs&, const float*, int, double,
                                                     const double*, int, double*, int64_t, double*, int64_t,
                                                     const double*, float*, const double*, int);
template bool launch_column_richardson<double, double>(hipStream_t, const SpaceArgs&, const double*, int, double,
                                                       const double*, int, double*, int64_t, double*, int64_t,
                                                       const double*, double*, const double*, int);
template bool launch_column<float, float>(hipStream_t, const SpaceArgs&, const float*, int, double, const double*,
                                          int, double*, int64_t, double*, int64_t, const double*, float*,
                                          const double*);
template bool launch_column<double, double>(hipStream_t, const SpaceArgs&, const double*, int, double,
                                            const double*, int, double*, int64_t, double*, int64_t, const double*,
                                            double*, const double*);
template bool launch_column<float, float, float>(hipStream_t, const SpaceArgs&, const float*, int, double,
                                                 const double*, int, double*, int64_t, double*, int64_t,
                                                 const double*, float*, const double*);
template bool launch_batch_table_gemm<float, true>(hipStream_t, const BatchItem*, const GemmUnit*, int, const int2*,
                                                   int, int, const uint16_t*, int, int64_t);
template bool launch_batch_table_gemm<bf16, true>(hipStream_t, const BatchItem*, const GemmUnit*, int, const int2*,
                                                  int, int, const uint16_t*, int, int64_t);
template bool launch_batch_table_gemm<float, false>(hipStream_t, const BatchItem*, const GemmUnit*, int, const int2*,
                                                    int, int, const uint16_t*, int, int64_t);
template bool launch_batch_gauss_gemm<float, true>(hipStream_t, const BatchItem*, const GemmUnit*, int, const int2*,
                                                   int, int, const float*, int);
template bool launch_batch_gauss_gemm<bf16, true>(hipStream_t, const BatchItem*, const GemmUnit*, int, const int2*, int,
                                                  int, const float*, int);
template bool launch_batch_gauss_gemm<float, false>(hipStream_t, const BatchItem*, const GemmUnit*, int, const int2*,
                                                    int, int, const float*, int);
template bool launch_batch_sketch_p<float>(hipStream_t, int, const BatchItem*, const BlockMap&, int64_t,
                                          const BlockMap&, int64_t, const BlockMap&, int64_t, bool);
template bool launch_batch_column<float>(hipStream_t, const BatchItem*, const BlockMap&, int64_t, const BlockMap&,
                                         int64_t, const BlockMap&, int64_t, int);
template bool launch_batch_column<float, float>(hipStream_t, const BatchItem*, const BlockMap&, int64_t,
                                                const BlockMap&, int64_t, const BlockMap&, int64_t, int);
template bool launch_batch_column<double>(hipStream_t, const BatchItem*, const BlockMap&, int64_t, const BlockMap&,
                                         int64_t, const BlockMap&, int64_t, int);
template bool launch_batch_column_richardson<float>(hipStream_t, const BatchItem*, const BlockMap&, int64_t,
                                                     const BlockMap&, int64_t, const BlockMap&, int64_t, int, int);
template bool launch_batch_scale<float, false>(hipStream_t, const BatchItem*, const BlockMap&, int64_t);
template bool launch_batch_scale<bf16, true>(hipStream_t, const BatchItem*, const BlockMap&, int64_t);
template bool launch_materialize<float>(hipStream_t, const SketchArgs&, int64_t, int64_t, int64_t, int64_t,
                                        double, double*, int64_t);
template bool launch_materialize<double>(hipStream_t, const SketchArgs&, int64_t, int64_t, int64_t, int64_t,
                                         double, double*, int64_t);

}  // namespace rgs
