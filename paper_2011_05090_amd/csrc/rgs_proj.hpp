// Device body of the fused projection + sketch pass (steps 3, 4 and 7 of
// Algorithm 2) over one row block, shared by the QR kernels and the GMRES
// kernels.
#pragma once

#include "rgs_block.hpp"
#include "rgs_device.hpp"
#include "rgs_types.hpp"

namespace rgs {

// LDS elements (of TW) a workgroup running project_body with sketch SK must
// provide: one block of rows, or the signed-sum tables of the fp32
// Rademacher sketch.
template <typename TW, int SK>
constexpr int proj_lds_size() {
    return (SK == SK_RADEM && sizeof(TW) == 4) ? kRadNibLds : kProjWaves * kTile;
}

// Workgroup-uniform early exit once an earlier step has flagged a breakdown:
// one thread reads the status word, the whole workgroup takes the same branch.
#define RGS_EXIT_IF_FAILED(status)                      \
    do {                                                \
        __shared__ int rgs_stop_;                       \
        if (threadIdx.x == 0) rgs_stop_ = (status)[0] | (status)[2]; \
        __syncthreads();                                \
        if (rgs_stop_ != 0) return;                     \
    } while (0)

// Step 3 (+ step 4 partials, + step 7 of the previous column), for row block
// blk of kProjWaves * 1024 rows:
//   q'_i = w_i - sum_{c<j} coef[c] q_c        (working precision TW; the terms of
//   each group of kProjGroup columns are summed by an fma chain in c order, then
//   subtracted)
// If normalize_last, column j-1 still holds q'_{i-1} and is first scaled to
// q_{i-1} = q'_{i-1} / r_{i-1,i-1} (fp64 multiply by the reciprocal, rounded
// to the storage type) and written back.  q'_i is stored in column j, then the
// block's sketch partials of the stored q'_i are written (or q'_i itself for
// Theta = I).  DEFER (bf16 storage): columns stay unnormalised, the
// coefficients already carry 1/r_cc, and the sketch is taken of the rounded,
// stored q'_i.  WSCALE: w_i arrives unscaled and is first multiplied by
// wscale[0] when wscale is given (fp64 multiply, rounded to TW) -- the Arnoldi
// vector A q'_{i-1} of the fused-sketch GMRES step, whose 1/r_{i-1,i-1} is
// known only now.
template <typename TW, typename TQ, typename PT, int SK, bool DEFER, bool WSCALE = false>
__device__ __forceinline__ void project_body(const TW* __restrict__ w, TQ* __restrict__ Q, int64_t ldq, int64_t n,
                                             int j, const TW* __restrict__ coef, const double* __restrict__ invr,
                                             int normalize_last, int do_sketch, int vec_ok, const SketchArgs& sk,
                                             PT* __restrict__ partials, int64_t blk, TW* __restrict__ lds,
                                             const double* __restrict__ wscale = nullptr) {
    constexpr int NW = kProjWaves;
    int64_t row0[4];
    lane_rows<NW>(blk, row0);
    const bool full = vec_ok && (blk + 1) * (NW * kTile) <= n;
    TW v[16];
    load16(w, row0, n, full, v, vec_ok);
    if constexpr (WSCALE) {
        if (wscale) {   // none at the first column of a cycle (w_1 = r_0)
            const double ws = wscale[0];
#pragma unroll
            for (int t = 0; t < 16; ++t) v[t] = (TW)((double)v[t] * ws);
        }
    }
    const int jl = (!DEFER && normalize_last) ? j - 1 : j;
    for (int c0 = 0; c0 < jl; c0 += kProjGroup) {
        const int c1 = min(c0 + kProjGroup, jl);
        TW g[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) g[t] = TW(0);
        for (int c = c0; c < c1; ++c) {
            const TW a = coef[c];
            TW q[16];
            load16(Q + (int64_t)c * ldq, row0, n, full, q, vec_ok);
#pragma unroll
            for (int t = 0; t < 16; ++t) g[t] = fma(a, q[t], g[t]);
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] -= g[t];
    }
    if constexpr (!DEFER) {
        if (normalize_last) {
            const int c = j - 1;
            const TW a = coef[c];
            const double ir = invr[0];
            TW q[16];
            TQ* qc = Q + (int64_t)c * ldq;
            load16(qc, row0, n, full, q);
#pragma unroll
            for (int t = 0; t < 16; ++t) q[t] = (TW)((double)q[t] * ir);
            store16(qc, row0, n, full, q);
#pragma unroll
            for (int t = 0; t < 16; ++t) v[t] = fma(-a, q[t], v[t]);
        }
    }
    store16(Q + (int64_t)j * ldq, row0, n, full, v);   // bf16: v becomes the stored value
    if (!do_sketch) return;
    if constexpr (SK == SK_IDENT) {
        store16(partials, row0, n, false, v);   // Theta = I: the "sketch" is q' itself
    } else {
        PT acc[kKptMax];
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) acc[u] = PT(0);
        if constexpr (SK == SK_RADEM && sizeof(TW) == 4)   // lds holds kRadNibLds floats here
            block_sketch_rad_nib<PT, NW>(v, blk, n, sk, acc, lds);
        else
            block_sketch<TW, PT, SK, NW>(v, blk, n, sk, acc, lds);
        PT* out = partials + blk * sk.k;
        constexpr int NT = NW * kWave;
        const int kpt = (sk.k + NT - 1) / NT;
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) {
            const int jj = threadIdx.x + NT * u;
            if (u < kpt && jj < sk.k) out[jj] = acc[u];
        }
    }
}

}  // namespace rgs
