// The fused projection + sketch kernel of librgs for gfx950 (MI355X): steps
// 3, 4 and 7 of Algorithm 2 (Sec. 2.3 of Balabanov & Grigori) in one
// coalesced pass over the basis, for one factorisation (k_project) or for
// every factorisation of a batched call at the same column (kb_project).  It
// is the kernel that bounds the factorisation (one read of Q_{i-1} per
// column), so it sits in a translation unit of its own.

#include "rgs_internal.hpp"
#include "rgs_map.hpp"
#include "rgs_proj.hpp"

namespace rgs {

template <typename TW, typename TQ, typename PT, int SK, bool DEFER>
__global__ __launch_bounds__(kProjWaves * kWave) void k_project(
    const TW* __restrict__ w, TQ* __restrict__ Q, int64_t ldq, int64_t n, int j, const TW* __restrict__ coef,
    const double* __restrict__ invr, int normalize_last, int do_sketch, int vec_ok, SketchArgs sk,
    PT* __restrict__ partials, const int* __restrict__ status) {
    __shared__ TW lds[proj_lds_size<TW, SK>()];
    RGS_EXIT_IF_FAILED(status);
    project_body<TW, TQ, PT, SK, DEFER>(w, Q, ldq, n, j, coef, invr, normalize_last, do_sketch, vec_ok, sk,
                                        partials, blockIdx.x, lds);
}

// The same pass with w_i scaled by wscale[0] on load (fused-sketch GMRES step;
// the sketch of q'_i is taken elsewhere, so none here).
template <typename TW, typename TQ, bool DEFER>
__global__ __launch_bounds__(kProjWaves * kWave) void k_project_ws(
    const TW* __restrict__ w, TQ* __restrict__ Q, int64_t ldq, int64_t n, int j, const TW* __restrict__ coef,
    const double* __restrict__ invr, int normalize_last, int vec_ok, const double* __restrict__ wscale,
    const int* __restrict__ status) {
    __shared__ TW lds[kProjWaves * kTile];
    RGS_EXIT_IF_FAILED(status);
    SketchArgs none{};
    project_body<TW, TQ, TW, SK_GAUSS, DEFER, true>(w, Q, ldq, n, j, coef, invr, normalize_last, 0, vec_ok, none,
                                                    nullptr, blockIdx.x, lds, wscale);
}

// Batched: workgroup -> (factorisation, row block) through the implicit map;
// column i of every factorisation listed in it.
template <typename TW, typename TQ, typename PT, int SK, bool DEFER>
__global__ __launch_bounds__(kProjWaves * kWave) void kb_project(const BatchItem* __restrict__ items, BlockMap map,
                                                                 int i) {
    __shared__ TW lds[proj_lds_size<TW, SK>()];
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    RGS_EXIT_IF_FAILED(it.sa.status);
    const TW* W = static_cast<const TW*>(it.W);
    project_body<TW, TQ, PT, SK, DEFER>(W + (int64_t)i * it.ldw, static_cast<TQ*>(it.Q), it.ldq, it.n, i,
                                        static_cast<const TW*>(it.coef), i > 0 ? it.sa.invr + (i - 1) : nullptr,
                                        (!DEFER && i > 0) ? 1 : 0, ((DEFER || i > 0) && !it.gemm_sketch) ? 1 : 0,
                                        it.vec_ok, it.sk,
                                        static_cast<PT*>(it.part), bm.y, lds);
}

// The same step 3 (+ step 7 of the previous column) without a sketch, 4 rows
// per lane and one wave per workgroup (256 rows), for factorisations too
// small to fill the device with kProjWaves-tile blocks; their column sketch is
// a launch of its own.  Per-element arithmetic as in project_body, so the
// stored q'_i is the same.
template <typename TW, typename TQ, bool DEFER>
__global__ __launch_bounds__(64) void k_project_rows(const TW* __restrict__ w, TQ* __restrict__ Q, int64_t ldq,
                                                     int64_t n, int j, const TW* __restrict__ coef,
                                                     const double* __restrict__ invr, int normalize_last,
                                                     const int* __restrict__ status) {
    RGS_EXIT_IF_FAILED(status);
    const int64_t r0 = ((int64_t)blockIdx.x * 64 + threadIdx.x) * 4;
    if (r0 >= n) return;
    auto load = [&](const auto* p, TW v[4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if constexpr (sizeof(*p) == 2)
                v[r] = (r0 + r < n) ? (TW)bf16_to_float(p[r0 + r].bits) : TW(0);
            else
                v[r] = (r0 + r < n) ? (TW)p[r0 + r] : TW(0);
        }
    };
    TW v[4];
    load(w, v);
    const int jl = (!DEFER && normalize_last) ? j - 1 : j;
    for (int c0 = 0; c0 < jl; c0 += kProjGroup) {
        const int c1 = min(c0 + kProjGroup, jl);
        TW g[4] = {TW(0), TW(0), TW(0), TW(0)};
        for (int c = c0; c < c1; ++c) {
            const TW a = coef[c];
            TW q[4];
            load(Q + (int64_t)c * ldq, q);
#pragma unroll
            for (int t = 0; t < 4; ++t) g[t] = fma(a, q[t], g[t]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] -= g[t];
    }
    if constexpr (!DEFER) {
        if (normalize_last) {
            const int c = j - 1;
            const TW a = coef[c];
            const double ir = invr[0];
            TQ* qc = Q + (int64_t)c * ldq;
            TW q[4];
            load(qc, q);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                q[t] = (TW)((double)q[t] * ir);
                if (r0 + t < n) qc[r0 + t] = q[t];
                v[t] = fma(-a, q[t], v[t]);
            }
        }
    }
    TQ* qj = Q + (int64_t)j * ldq;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (r0 + t >= n) break;
        if constexpr (sizeof(TQ) == 2)
            qj[r0 + t].bits = float_to_bf16((float)v[t]);
        else
            qj[r0 + t] = v[t];
    }
}

#define RGS_LAUNCH_CHECK()                                   \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return false;   \
    } while (0)

static inline unsigned nblocks(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

template <typename TW, typename TQ, bool DEFER>
bool launch_project(hipStream_t st, const TW* w, TQ* Q, int64_t ldq, int64_t n, int j, const TW* coef,
                    const double* invr, int normalize_last, int do_sketch, int vec_ok, const SketchArgs& sk,
                    TW* partials, const int* status) {
    const unsigned nblk = nblocks(n, kProjRows);
    const dim3 thr(kProjWaves * kWave);
    switch (sk.sketch) {
        case SK_SRHT:
            hipLaunchKernelGGL((k_project<TW, TQ, TW, SK_SRHT, DEFER>), dim3(nblk), thr, 0, st, w, Q, ldq, n, j,
                               coef, invr, normalize_last, do_sketch, vec_ok, sk, partials, status);
            break;
        case SK_GAUSS:
            hipLaunchKernelGGL((k_project<TW, TQ, TW, SK_GAUSS, DEFER>), dim3(nblk), thr, 0, st, w, Q, ldq, n, j,
                               coef, invr, normalize_last, do_sketch, vec_ok, sk, partials, status);
            break;
        case SK_RADEM:
            hipLaunchKernelGGL((k_project<TW, TQ, TW, SK_RADEM, DEFER>), dim3(nblk), thr, 0, st, w, Q, ldq, n, j,
                               coef, invr, normalize_last, do_sketch, vec_ok, sk, partials, status);
            break;
        case SK_TABLE:
            hipLaunchKernelGGL((k_project<TW, TQ, TW, SK_TABLE, DEFER>), dim3(nblk), thr, 0, st, w, Q, ldq, n, j,
                               coef, invr, normalize_last, do_sketch, vec_ok, sk, partials, status);
            break;
        case SK_TABX:
            hipLaunchKernelGGL((k_project<TW, TQ, TW, SK_TABX, DEFER>), dim3(nblk), thr, 0, st, w, Q, ldq, n, j,
                               coef, invr, normalize_last, do_sketch, vec_ok, sk, partials, status);
            break;
        default:
            hipLaunchKernelGGL((k_project<TW, TQ, TW, SK_IDENT, DEFER>), dim3(nblk), thr, 0, st, w, Q, ldq, n, j,
                               coef, invr, normalize_last, do_sketch, vec_ok, sk, partials, status);
    }
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TW, typename TQ, bool DEFER>
bool launch_project_rows(hipStream_t st, const TW* w, TQ* Q, int64_t ldq, int64_t n, int j, const TW* coef,
                         const double* invr, int normalize_last, const int* status) {
    hipLaunchKernelGGL((k_project_rows<TW, TQ, DEFER>), dim3(nblocks(n, 256)), dim3(64), 0, st, w, Q, ldq, n, j, coef,
                       invr, normalize_last, status);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TW, typename TQ, bool DEFER>
bool launch_project_ws(hipStream_t st, const TW* w, TQ* Q, int64_t ldq, int64_t n, int j, const TW* coef,
                       const double* invr, int normalize_last, int vec_ok, const double* wscale, const int* status) {
    hipLaunchKernelGGL((k_project_ws<TW, TQ, DEFER>), dim3(nblocks(n, kProjRows)), dim3(kProjWaves * kWave), 0, st,
                       w, Q, ldq, n, j, coef, invr, normalize_last, vec_ok, wscale, status);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TW, typename TQ, bool DEFER>
bool launch_batch_project(hipStream_t st, int sketch, const BatchItem* items, const BlockMap& map, int64_t nblk,
                          int i) {
    if (nblk == 0) return true;
    const dim3 thr(kProjWaves * kWave);
    if (sketch == SK_SRHT)
        hipLaunchKernelGGL((kb_project<TW, TQ, TW, SK_SRHT, DEFER>), dim3(nblk), thr, 0, st, items, map, i);
    else
        hipLaunchKernelGGL((kb_project<TW, TQ, TW, SK_GAUSS, DEFER>), dim3(nblk), thr, 0, st, items, map, i);
    RGS_LAUNCH_CHECK();
    return true;
}

// explicit instantiations
template bool launch_project_rows<float, float, false>(hipStream_t, const float*, float*, int64_t, int64_t, int,
                                                       const float*, const double*, int, const int*);
template bool launch_project_rows<double, double, false>(hipStream_t, const double*, double*, int64_t, int64_t, int,
                                                         const double*, const double*, int, const int*);
template bool launch_project_rows<float, bf16, true>(hipStream_t, const float*, bf16*, int64_t, int64_t, int,
                                                     const float*, const double*, int, const int*);
template bool launch_project_ws<float, float, false>(hipStream_t, const float*, float*, int64_t, int64_t, int,
                                                     const float*, const double*, int, int, const double*,
                                                     const int*);
template bool launch_project_ws<double, double, false>(hipStream_t, const double*, double*, int64_t, int64_t, int,
                                                       const double*, const double*, int, int, const double*,
                                                       const int*);
template bool launch_project_ws<float, bf16, true>(hipStream_t, const float*, bf16*, int64_t, int64_t, int,
                                                   const float*, const double*, int, int, const double*,
                                                   const int*);
template bool launch_project<float, float, false>(hipStream_t, const float*, float*, int64_t, int64_t, int,
                                                  const float*, const double*, int, int, int, const SketchArgs&,
                                                  float*, const int*);
template bool launch_project<double, double, false>(hipStream_t, const double*, double*, int64_t, int64_t, int,
                                                    const double*, const double*, int, int, int,
                                                    const SketchArgs&, double*, const int*);
template bool launch_project<float, bf16, true>(hipStream_t, const float*, bf16*, int64_t, int64_t, int,
                                                const float*, const double*, int, int, int, const SketchArgs&,
                                                float*, const int*);
template bool launch_batch_project<float, float, false>(hipStream_t, int, const BatchItem*, const BlockMap&, int64_t,
                                                        int);
template bool launch_batch_project<float, bf16, true>(hipStream_t, int, const BatchItem*, const BlockMap&, int64_t, int);

}  // namespace rgs
