// HIP kernels of librgs for gfx950 (MI355X).
//
// Randomized Gram-Schmidt, Algorithm 2 of Balabanov & Grigori (Sec. 2.3), one
// column i at a time:
//   step 1  p_i = Theta w_i                 -> k_sketch_cols + k_reduce (all columns at once)
//   step 2  y = argmin ||S_{i-1} y - p_i||  -> k_ls1, k_ls2, k_ls3 (Householder, compact WY)
//   step 3  q'_i = w_i - Q_{i-1} y          -> k_project (one coalesced pass over Q_{i-1})
//   step 4  s'_i = Theta q'_i               -> fused into k_project as per-block partials
//   steps 5-6  r_ii = ||s'_i||, s_i = s'_i / r_ii, and the Householder append of s_i
//                                           -> k_ap1 .. k_ap4
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

#include "rgs_device.hpp"
#include "rgs_internal.hpp"

namespace rgs {

// Workgroup-uniform early exit once an earlier step has flagged a breakdown:
// one thread reads the status word, the whole workgroup takes the same branch.
#define RGS_EXIT_IF_FAILED(status)                      \
    do {                                                \
        __shared__ int rgs_stop_;                       \
        if (threadIdx.x == 0) rgs_stop_ = (status)[0];  \
        __syncthreads();                                \
        if (rgs_stop_ != 0) return;                     \
    } while (0)

// ---------------------------------------------------------------------------
// Loads/stores of the 16 rows a lane owns in a wave tile:
// rows row0[e] .. row0[e] + 3, e = 0..3 (row0[e] is a multiple of 4).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void load16(const T* __restrict__ p, const int64_t row0[4], int64_t n,
                                       bool full, T v[16]) {
    if (full) {
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float4 t = *reinterpret_cast<const float4*>(p + row0[e]);
                v[4 * e] = t.x;
                v[4 * e + 1] = t.y;
                v[4 * e + 2] = t.z;
                v[4 * e + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double2 a = *reinterpret_cast<const double2*>(p + row0[e]);
                const double2 b = *reinterpret_cast<const double2*>(p + row0[e] + 2);
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
            for (int e = 0; e < 4; ++e)
                *reinterpret_cast<float4*>(p + row0[e]) =
                    make_float4(v[4 * e], v[4 * e + 1], v[4 * e + 2], v[4 * e + 3]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                *reinterpret_cast<double2*>(p + row0[e]) = make_double2(v[4 * e], v[4 * e + 1]);
                *reinterpret_cast<double2*>(p + row0[e] + 2) = make_double2(v[4 * e + 2], v[4 * e + 3]);
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

__device__ __forceinline__ void lane_rows(int64_t blk, int64_t row0[4]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 4; ++e) row0[e] = blk * kBlock + wave * kTile + 256 * e + 4 * lane;
}

// ---------------------------------------------------------------------------
// Sketch of one 4096-row block held in registers (v = this lane's 16 rows),
// accumulated into acc[u] for the sketch rows j = threadIdx.x + 256 u.
// The 1/sqrt(k) scale is applied later, in fp64.
//
// SRHT: with s = 2^a T (T = 1024 the in-wave FWHT order) the Sylvester
// Hadamard matrix factors as H_s = H_{s/T} (x) H_T, so for a sampled row
// rho = alpha T + beta and the tile index t of rows [tT, (t+1)T):
//   (H_s D x)[rho] = sum_t (-1)^popcount(alpha & t) (H_T D x_t)[beta].
// Each wave transforms its tile in registers; the block's four tiles are then
// combined per sampled row through LDS.
// Gaussian: theta_{j,l} generated on the fly, 4 entries per Philox call.
// ---------------------------------------------------------------------------
template <typename T, typename PT, int SK>
__device__ __forceinline__ void block_sketch(T v[16], int64_t blk, int64_t n, const SketchArgs& sk,
                                             PT acc[kKptMax], T* __restrict__ lds) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int kpt = (sk.k + kWG - 1) / kWG;
    if constexpr (SK == SK_SRHT) {
        int64_t row0[4];
        lane_rows(blk, row0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (row0[e] < n) {
                const uint32_t word = sk.signs[row0[e] >> 5];
                const int sh = (int)(row0[e] & 31);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if ((word >> (sh + r)) & 1u) v[4 * e + r] = -v[4 * e + r];
            }
        }
        fwht1024_wave<T>(v, lane);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[wave * kTile + 256 * e + 4 * lane + r] = v[4 * e + r];
        __syncthreads();
        const uint32_t tb = (uint32_t)(blk * 4);  // tile index of wave 0
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) {
            const int j = t + kWG * u;
            if (u < kpt && j < sk.k) {
                const uint32_t rho = (uint32_t)sk.rows[j];
                const uint32_t alpha = rho >> 10, beta = rho & 1023u;
                const T z0 = lds[beta], z1 = lds[kTile + beta];
                const T z2 = lds[2 * kTile + beta], z3 = lds[3 * kTile + beta];
                const T s01 = (alpha & 1u) ? z0 - z1 : z0 + z1;
                const T s23 = (alpha & 1u) ? z2 - z3 : z2 + z3;
                T tot = (alpha & 2u) ? s01 - s23 : s01 + s23;
                if (__popc(alpha & tb) & 1) tot = -tot;
                acc[u] += (PT)tot;
            }
        }
        __syncthreads();
    } else if constexpr (SK == SK_GAUSS) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[wave * kTile + 256 * e + 4 * lane + r] = v[4 * e + r];
        __syncthreads();
        const int64_t rem = n - blk * kBlock;
        const int nq = rem >= kBlock ? kBlock / 4 : (int)((rem + 3) / 4);
        const uint32_t q0 = (uint32_t)(blk * (kBlock / 4));
        for (int q = 0; q < nq; ++q) {
            const T x0 = lds[4 * q], x1 = lds[4 * q + 1], x2 = lds[4 * q + 2], x3 = lds[4 * q + 3];
#pragma unroll
            for (int u = 0; u < kKptMax; ++u) {
                const int j = t + kWG * u;
                if (u < kpt && j < sk.k) {
                    T z[4];
                    gauss4(q0 + (uint32_t)q, (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z);
                    acc[u] += (PT)(z[0] * x0 + z[1] * x1 + z[2] * x2 + z[3] * x3);
                }
            }
        }
        __syncthreads();
    }
}

// SRHT diagonal D as a bit table: bit b of word w is set iff d_{32w+b} = -1.
// Word w comes from word (w mod 4) of Philox(w/4, 0xFFFFFFFF, sketch_id, instance).
__global__ void k_srht_signs(uint32_t* __restrict__ signs, int64_t nwords, uint32_t k0, uint32_t k1,
                             uint32_t sid, uint32_t inst) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * b >= nwords) return;
    uint32_t x[4];
    philox4x32_10((uint32_t)b, kTagSigns, sid, inst, k0, k1, x);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (4 * b + t < nwords) signs[4 * b + t] = x[t];
}

// Partial sketches of ncols columns of X: workgroup (g, col) covers row blocks
// g, g + G, ... and writes partials[(col * G + g) * k + j].
template <typename T, typename PT, int SK>
__global__ __launch_bounds__(kWG) void k_sketch_cols(const T* __restrict__ X, int64_t ldx, int64_t n,
                                                     int64_t nblk, int G, SketchArgs sk,
                                                     PT* __restrict__ partials) {
    __shared__ T lds[kBlock];
    const int g = blockIdx.x, col = blockIdx.y;
    const T* x = X + (int64_t)col * ldx;
    PT acc[kKptMax];
#pragma unroll
    for (int u = 0; u < kKptMax; ++u) acc[u] = PT(0);
    const bool vec_ok = ((reinterpret_cast<uintptr_t>(x) & 15) == 0);
    for (int64_t blk = g; blk < nblk; blk += G) {
        int64_t row0[4];
        lane_rows(blk, row0);
        const bool full = vec_ok && (blk + 1) * kBlock <= n;
        T v[16];
        load16(x, row0, n, full, v);
        block_sketch<T, PT, SK>(v, blk, n, sk, acc, lds);
    }
    PT* out = partials + ((int64_t)col * G + g) * sk.k;
    const int kpt = (sk.k + kWG - 1) / kWG;
#pragma unroll
    for (int u = 0; u < kKptMax; ++u) {
        const int j = threadIdx.x + kWG * u;
        if (u < kpt && j < sk.k) out[j] = acc[u];
    }
}

// out[j + col*ldo] = scale * sum_{g=0}^{G-1} partials[(col*G + g)*k + j], in fp64 and
// in a fixed order: 8 contiguous g-ranges summed by 8 threads, then combined in order.
template <typename PT>
__global__ __launch_bounds__(kWG) void k_reduce(const PT* __restrict__ partials, int G, int k,
                                                double scale, double* __restrict__ out, int64_t ldo) {
    __shared__ double red[8][32];
    const int col = blockIdx.y;
    const int jl = threadIdx.x & 31, part = threadIdx.x >> 5;
    const int j = blockIdx.x * 32 + jl;
    const int g0 = (int)((int64_t)G * part / 8), g1 = (int)((int64_t)G * (part + 1) / 8);
    double s = 0.0;
    if (j < k) {
        const PT* p = partials + (int64_t)col * G * k + j;
        for (int g = g0; g < g1; ++g) s += (double)p[(int64_t)g * k];
    }
    red[part][jl] = s;
    __syncthreads();
    if (part == 0 && j < k) {
        double tot = 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) tot += red[t][jl];
        out[j + (int64_t)col * ldo] = tot * scale;
    }
}

// Step 3 (+ step 4 partials, + step 7 of the previous column):
//   q'_i = w_i - sum_{c<j} coef[c] q_c           (working precision T, fma chain in c order)
// where, if normalize_last, column j-1 still holds q'_{i-1} and is first
// scaled to q_{i-1} = q'_{i-1} / r_{i-1,i-1} (fp64 multiply by the reciprocal,
// rounded to T) and written back.  q'_i is stored in column j.  Then the
// block's sketch partials of q'_i are written (or q'_i itself for Theta = I).
template <typename T, typename PT, int SK>
__global__ __launch_bounds__(kWG) void k_project(const T* __restrict__ w, T* __restrict__ Q, int64_t ldq,
                                                 int64_t n, int j, const T* __restrict__ coef,
                                                 const double* __restrict__ invr, int normalize_last,
                                                 int do_sketch, int vec_ok, SketchArgs sk,
                                                 PT* __restrict__ partials,
                                                 const int* __restrict__ status) {
    __shared__ T lds[kBlock];
    RGS_EXIT_IF_FAILED(status);
    const int64_t blk = blockIdx.x;
    int64_t row0[4];
    lane_rows(blk, row0);
    const bool full = vec_ok && (blk + 1) * kBlock <= n;
    T v[16];
    load16(w, row0, n, full, v);
    const int jl = normalize_last ? j - 1 : j;
#pragma unroll 2
    for (int c = 0; c < jl; ++c) {
        const T a = coef[c];
        T q[16];
        load16(Q + (int64_t)c * ldq, row0, n, full, q);
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] = fma(-a, q[t], v[t]);
    }
    if (normalize_last) {
        const int c = j - 1;
        const T a = coef[c];
        const double ir = invr[0];
        T q[16];
        T* qc = Q + (int64_t)c * ldq;
        load16(qc, row0, n, full, q);
#pragma unroll
        for (int t = 0; t < 16; ++t) q[t] = (T)((double)q[t] * ir);
        store16(qc, row0, n, full, q);
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] = fma(-a, q[t], v[t]);
    }
    store16(Q + (int64_t)j * ldq, row0, n, full, v);
    if (!do_sketch) return;
    if constexpr (SK == SK_IDENT) {
        store16(partials, row0, n, false, v);   // Theta = I: the "sketch" is q' itself
    } else {
        PT acc[kKptMax];
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) acc[u] = PT(0);
        block_sketch<T, PT, SK>(v, blk, n, sk, acc, lds);
        PT* out = partials + blk * sk.k;
        const int kpt = (sk.k + kWG - 1) / kWG;
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) {
            const int jj = threadIdx.x + kWG * u;
            if (u < kpt && jj < sk.k) out[jj] = acc[u];
        }
    }
}

// Final step 7 for the last column: q = q' / r (fp64 reciprocal, rounded to T).
template <typename T>
__global__ void k_scale_col(T* __restrict__ q, int64_t n, const double* __restrict__ invr,
                            const int* __restrict__ status) {
    RGS_EXIT_IF_FAILED(status);
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n) q[l] = (T)((double)q[l] * invr[0]);
}

// ---------------------------------------------------------------------------
// Sketch-space kernels (fp64).  i = 0-based index of the current column,
// j = i columns are already factorised.  SL = 64 rows per workgroup slice,
// pd = per-slice partial dot products, row stride m1 = mcap + 1.
// ---------------------------------------------------------------------------

// Step 2, part 1: per-slice partials of c = Wm_i^T p (c < i) and of ||p||^2 (slot i).
__global__ __launch_bounds__(kWG) void k_ls1(const double* __restrict__ p, int k, int i,
                                             const double* __restrict__ Wr, int mcap,
                                             double* __restrict__ pd, const int* __restrict__ status) {
    RGS_EXIT_IF_FAILED(status);
    const int s = blockIdx.x, r0 = s * kSlice, r1 = min(k, r0 + kSlice);
    for (int c = threadIdx.x; c <= i; c += kWG) {
        double acc = 0.0;
        if (c < i) {
            for (int r = r0; r < r1; ++r) acc = fma(Wr[(int64_t)r * mcap + c], p[r], acc);
        } else {
            for (int r = r0; r < r1; ++r) acc = fma(p[r], p[r], acc);
        }
        pd[(int64_t)s * (mcap + 1) + c] = acc;
    }
}

// Step 2, part 2: c = sum of slice partials; head of U_i^T p:
//   uh[r] = p[r] - sum_{c <= r} V[r, c] c[c],  r < i.
__global__ __launch_bounds__(kWG) void k_ls2(const double* __restrict__ p, int k, int i, int nsl,
                                             const double* __restrict__ Vc, int mcap,
                                             const double* __restrict__ pd, double* __restrict__ uh,
                                             double* __restrict__ pnorm, const int* __restrict__ status) {
    extern __shared__ double cp[];  // [i + 1]
    __shared__ double red[4][64];
    RGS_EXIT_IF_FAILED(status);
    for (int c = threadIdx.x; c <= i; c += kWG) {
        double acc = 0.0;
        for (int s = 0; s < nsl; ++s) acc += pd[(int64_t)s * (mcap + 1) + c];
        cp[c] = acc;
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) pnorm[i] = sqrt(cp[i]);
    const int rl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int r = blockIdx.x * 64 + rl;
    double part = 0.0;
    if (r < i) {
        const int cmax = min(r, i - 1);
        for (int c = q; c <= cmax; c += 4) part = fma(Vc[r + (int64_t)c * k], cp[c], part);
    }
    red[q][rl] = part;
    __syncthreads();
    if (q == 0 && r < i) uh[r] = p[r] - (((red[0][rl] + red[1][rl]) + red[2][rl]) + red[3][rl]);
}

// Step 2, part 3: y = R_S^{-1} uh with X = R_S^{-1} (upper triangular):
//   y[r] = sum_{c >= r} X[r, c] uh[c].  Writes R(0:i, i), and coef (working precision).
template <typename T>
__global__ __launch_bounds__(kWG) void k_ls3(int i, const double* __restrict__ X, int mcap,
                                             const double* __restrict__ uh, double* __restrict__ R,
                                             int64_t ldr, T* __restrict__ coef,
                                             const int* __restrict__ status) {
    extern __shared__ double us[];  // [i]
    __shared__ double red[4][64];
    RGS_EXIT_IF_FAILED(status);
    for (int c = threadIdx.x; c < i; c += kWG) us[c] = uh[c];
    __syncthreads();
    const int rl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int r = blockIdx.x * 64 + rl;
    double part = 0.0;
    if (r < i) {
        for (int c = r + ((q - r) & 3); c < i; c += 4) part = fma(X[r + (int64_t)c * mcap], us[c], part);
    }
    red[q][rl] = part;
    __syncthreads();
    if (q == 0 && r < i) {
        const double y = ((red[0][rl] + red[1][rl]) + red[2][rl]) + red[3][rl];
        R[r + (int64_t)i * ldr] = y;
        coef[r] = (T)y;
    }
}

// Append, part 1: s' = scale * (sum of block partials) for this slice (or a copy
// of src when src != nullptr), stored in sp; per-slice partials of
// c1 = Wm_i^T s' (c < i) and of ||s'||^2 (slot i).
template <typename PT>
__global__ __launch_bounds__(kWG) void k_ap1(const PT* __restrict__ partials, int G, double scale,
                                             const double* __restrict__ src, int k, int i,
                                             const double* __restrict__ Wr, int mcap,
                                             double* __restrict__ sp, double* __restrict__ pd,
                                             const int* __restrict__ status) {
    __shared__ double red[4][64];
    __shared__ double ss[64];
    RGS_EXIT_IF_FAILED(status);
    const int s = blockIdx.x, r0 = s * kSlice, r1 = min(k, r0 + kSlice);
    const int rl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int r = r0 + rl;
    if (src) {
        if (q == 0 && r < k) {
            ss[rl] = src[r];
            sp[r] = src[r];
        }
    } else {
        const int g0 = (int)((int64_t)G * q / 4), g1 = (int)((int64_t)G * (q + 1) / 4);
        double acc = 0.0;
        if (r < k)
            for (int g = g0; g < g1; ++g) acc += (double)partials[(int64_t)g * k + r];
        red[q][rl] = acc;
        __syncthreads();
        if (q == 0 && r < k) {
            const double val = ((((red[0][rl] + red[1][rl]) + red[2][rl]) + red[3][rl])) * scale;
            ss[rl] = val;
            sp[r] = val;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c <= i; c += kWG) {
        double acc = 0.0;
        if (c < i) {
            for (int rr = r0; rr < r1; ++rr) acc = fma(Wr[(int64_t)rr * mcap + c], ss[rr - r0], acc);
        } else {
            for (int rr = r0; rr < r1; ++rr) acc = fma(ss[rr - r0], ss[rr - r0], acc);
        }
        pd[(int64_t)s * (mcap + 1) + c] = acc;
    }
}

// Append, part 2: steps 5-6.  r_ii = ||s'||, S(:, i) = s'/r_ii, breakdown test,
// u = U_i^T s_i = (s' - V c1) / r_ii, per-slice partials of ||u(i+1:k)||^2.
__global__ __launch_bounds__(kWG) void k_ap2(int k, int i, int nsl, const double* __restrict__ sp,
                                             const double* __restrict__ Vc, int mcap,
                                             const double* __restrict__ pd, double* __restrict__ u,
                                             double* __restrict__ pd2, double* __restrict__ S, int64_t lds,
                                             double* __restrict__ R, int64_t ldr,
                                             double* __restrict__ rr, double* __restrict__ invr,
                                             const double* __restrict__ pnorm, int* __restrict__ status) {
    extern __shared__ double c1[];  // [i + 1]
    __shared__ double red[4][64];
    __shared__ double tl[64];
    RGS_EXIT_IF_FAILED(status);
    for (int c = threadIdx.x; c <= i; c += kWG) {
        double acc = 0.0;
        for (int s = 0; s < nsl; ++s) acc += pd[(int64_t)s * (mcap + 1) + c];
        c1[c] = acc;
    }
    __syncthreads();
    const double rii = sqrt(c1[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rr[i] = rii;
        invr[i] = 1.0 / rii;
        R[i + (int64_t)i * ldr] = rii;
        const double pn = (i == 0) ? rii : pnorm[i];
        if (!isfinite(rii) || !isfinite(pn)) {
            status[1] = i;
            status[0] = kStatusNonfinite;
        } else if (rii == 0.0 || rii <= 0x1p-50 * pn) {
            status[1] = i;
            status[0] = kStatusBreakdown;
        }
    }
    const int s = blockIdx.x, rl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int r = s * kSlice + rl;
    double part = 0.0;
    if (r < k)
        for (int c = q; c < i; c += 4) part = fma(Vc[r + (int64_t)c * k], c1[c], part);
    red[q][rl] = part;
    __syncthreads();
    if (q == 0) {
        double t2 = 0.0;
        if (r < k) {
            const double spr = sp[r];
            const double val = (spr - (((red[0][rl] + red[1][rl]) + red[2][rl]) + red[3][rl])) / rii;
            u[r] = val;
            S[r + (int64_t)i * lds] = spr / rii;
            if (r > i) t2 = val * val;
        }
        tl[rl] = t2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int t = 0; t < 64; ++t) acc += tl[t];
        pd2[s] = acc;
    }
}

// Append, part 3: Householder reflector of u(i:k) (dlarfg convention):
// beta = -sign(u_i) ||u(i:k)||, tau = (beta - u_i)/beta, v = [0; 1; u(i+1:k)/(u_i - beta)].
// Stores v as column i of V (both layouts); per-slice partials of d = V_i^T v.
__global__ __launch_bounds__(kWG) void k_ap3(int k, int i, int nsl, const double* __restrict__ u,
                                             const double* __restrict__ pd2, double* __restrict__ v,
                                             double* __restrict__ Vc, double* __restrict__ Vr, int mcap,
                                             double* __restrict__ pd, double* __restrict__ tau_a,
                                             double* __restrict__ beta_a, int* __restrict__ status) {
    __shared__ double vs[64];
    __shared__ double hh[3];
    RGS_EXIT_IF_FAILED(status);
    if (threadIdx.x == 0) {
        double tail2 = 0.0;
        for (int s = 0; s < nsl; ++s) tail2 += pd2[s];
        const double x1 = u[i];
        double beta, tau, scal;
        if (tail2 == 0.0) {
            beta = x1;
            tau = 0.0;
            scal = 0.0;
        } else {
            beta = -copysign(sqrt(x1 * x1 + tail2), x1);
            tau = (beta - x1) / beta;
            scal = 1.0 / (x1 - beta);
        }
        hh[0] = beta;
        hh[1] = tau;
        hh[2] = scal;
        if (blockIdx.x == 0) {
            tau_a[i] = tau;
            beta_a[i] = beta;
            if (!(fabs(beta) > 0x1p-50)) {   // s_i in span(S_{i-1}) in sketch space
                status[1] = i;
                status[0] = kStatusBreakdown;
            }
        }
    }
    __syncthreads();
    const int s = blockIdx.x, r0 = s * kSlice, r1 = min(k, r0 + kSlice);
    const int t = threadIdx.x;
    if (t < 64) {
        const int r = r0 + t;
        double val = 0.0;
        if (r < k) {
            val = (r < i) ? 0.0 : (r == i ? 1.0 : u[r] * hh[2]);
            v[r] = val;
            Vc[r + (int64_t)i * k] = val;
            Vr[(int64_t)r * mcap + i] = val;
        }
        vs[t] = val;
    }
    __syncthreads();
    for (int c = t; c < i; c += kWG) {
        double acc = 0.0;
        for (int r = max(r0, c); r < r1; ++r) acc = fma(Vr[(int64_t)r * mcap + c], vs[r - r0], acc);
        pd[(int64_t)s * (mcap + 1) + c] = acc;
    }
}

// Append, part 4.  Blocks [0, nsl): Wm(:, i) = tau (v - Wm_i d), d = sum of slice partials.
// Blocks [nsl, nsl + ceil(i/64)): column i of X = R_S^{-1}:
//   X(r, i) = -(sum_{c=r}^{i-1} X(r, c) u(c)) / beta  (u(0:i) is R_S(0:i, i)),  X(i, i) = 1/beta.
__global__ __launch_bounds__(kWG) void k_ap4(int k, int i, int nsl, const double* __restrict__ v,
                                             const double* __restrict__ u, double* __restrict__ Wc,
                                             double* __restrict__ Wr, int mcap, const double* __restrict__ pd,
                                             double* __restrict__ X, const double* __restrict__ tau_a,
                                             const double* __restrict__ beta_a, const int* __restrict__ status) {
    extern __shared__ double dsh[];  // [i]
    __shared__ double red[4][64];
    RGS_EXIT_IF_FAILED(status);
    const int rl = threadIdx.x & 63, q = threadIdx.x >> 6;
    if ((int)blockIdx.x < nsl) {
        for (int c = threadIdx.x; c < i; c += kWG) {
            double acc = 0.0;
            for (int s = 0; s < nsl; ++s) acc += pd[(int64_t)s * (mcap + 1) + c];
            dsh[c] = acc;
        }
        __syncthreads();
        const int r = blockIdx.x * kSlice + rl;
        double part = 0.0;
        if (r < k)
            for (int c = q; c < i; c += 4) part = fma(Wc[r + (int64_t)c * k], dsh[c], part);
        red[q][rl] = part;
        __syncthreads();
        if (q == 0 && r < k) {
            const double val = tau_a[i] * (v[r] - (((red[0][rl] + red[1][rl]) + red[2][rl]) + red[3][rl]));
            Wc[r + (int64_t)i * k] = val;
            Wr[(int64_t)r * mcap + i] = val;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) X[i + (int64_t)i * mcap] = 1.0 / beta_a[i];
    } else {
        for (int c = threadIdx.x; c < i; c += kWG) dsh[c] = u[c];
        __syncthreads();
        const int r = (blockIdx.x - nsl) * 64 + rl;
        double part = 0.0;
        if (r < i)
            for (int c = r + ((q - r) & 3); c < i; c += 4) part = fma(X[r + (int64_t)c * mcap], dsh[c], part);
        red[q][rl] = part;
        __syncthreads();
        if (q == 0 && r < i)
            X[r + (int64_t)i * mcap] = -((((red[0][rl] + red[1][rl]) + red[2][rl]) + red[3][rl])) / beta_a[i];
    }
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

template <typename T, typename PT>
bool launch_sketch_cols(hipStream_t st, const T* X, int64_t ldx, int64_t n, int ncols, int G,
                        const SketchArgs& sk, PT* partials) {
    const int64_t nblk = (n + kBlock - 1) / kBlock;
    dim3 grid(G, ncols);
    if (sk.sketch == SK_SRHT)
        hipLaunchKernelGGL((k_sketch_cols<T, PT, SK_SRHT>), grid, dim3(kWG), 0, st, X, ldx, n, nblk, G, sk,
                           partials);
    else
        hipLaunchKernelGGL((k_sketch_cols<T, PT, SK_GAUSS>), grid, dim3(kWG), 0, st, X, ldx, n, nblk, G, sk,
                           partials);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename PT>
bool launch_reduce(hipStream_t st, const PT* partials, int G, int k, int ncols, double scale, double* out,
                   int64_t ldo) {
    hipLaunchKernelGGL(k_reduce<PT>, dim3(nblocks(k, 32), ncols), dim3(kWG), 0, st, partials, G, k, scale,
                       out, ldo);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T, typename PT>
bool launch_project(hipStream_t st, const T* w, T* Q, int64_t ldq, int64_t n, int j, const T* coef,
                    const double* invr, int normalize_last, int do_sketch, int vec_ok, const SketchArgs& sk,
                    PT* partials, const int* status) {
    const unsigned nblk = nblocks(n, kBlock);
    switch (sk.sketch) {
        case SK_SRHT:
            hipLaunchKernelGGL((k_project<T, PT, SK_SRHT>), dim3(nblk), dim3(kWG), 0, st, w, Q, ldq, n, j, coef,
                               invr, normalize_last, do_sketch, vec_ok, sk, partials, status);
            break;
        case SK_GAUSS:
            hipLaunchKernelGGL((k_project<T, PT, SK_GAUSS>), dim3(nblk), dim3(kWG), 0, st, w, Q, ldq, n, j,
                               coef, invr, normalize_last, do_sketch, vec_ok, sk, partials, status);
            break;
        default:
            hipLaunchKernelGGL((k_project<T, PT, SK_IDENT>), dim3(nblk), dim3(kWG), 0, st, w, Q, ldq, n, j,
                               coef, invr, normalize_last, do_sketch, vec_ok, sk, partials, status);
    }
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T>
bool launch_scale_col(hipStream_t st, T* q, int64_t n, const double* invr, const int* status) {
    hipLaunchKernelGGL(k_scale_col<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, q, n, invr, status);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T>
bool launch_ls(hipStream_t st, const SpaceArgs& a, const double* p, int i, double* R, int64_t ldr, T* coef) {
    const int nsl = (a.k + kSlice - 1) / kSlice;
    hipLaunchKernelGGL(k_ls1, dim3(nsl), dim3(kWG), 0, st, p, a.k, i, a.Wr, a.mcap, a.pd, a.status);
    RGS_LAUNCH_CHECK();
    const unsigned nrb = nblocks(i, 64);
    hipLaunchKernelGGL(k_ls2, dim3(nrb), dim3(kWG), (i + 1) * sizeof(double), st, p, a.k, i, nsl, a.Vc, a.mcap,
                       a.pd, a.uh, a.pnorm, a.status);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ls3<T>, dim3(nrb), dim3(kWG), (i + 1) * sizeof(double), st, i, a.X, a.mcap, a.uh, R,
                       ldr, coef, a.status);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename PT>
bool launch_append(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale,
                   const double* src, int i, double* S, int64_t lds, double* R, int64_t ldr) {
    const int nsl = (a.k + kSlice - 1) / kSlice;
    hipLaunchKernelGGL(k_ap1<PT>, dim3(nsl), dim3(kWG), 0, st, partials, G, scale, src, a.k, i, a.Wr, a.mcap,
                       a.sp, a.pd, a.status);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ap2, dim3(nsl), dim3(kWG), (i + 1) * sizeof(double), st, a.k, i, nsl, a.sp, a.Vc,
                       a.mcap, a.pd, a.u, a.pd2, S, lds, R, ldr, a.rr, a.invr, a.pnorm, a.status);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ap3, dim3(nsl), dim3(kWG), 0, st, a.k, i, nsl, a.u, a.pd2, a.v, a.Vc, a.Vr, a.mcap,
                       a.pd, a.tau, a.beta, a.status);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ap4, dim3(nsl + nblocks(i, 64)), dim3(kWG), (i + 1) * sizeof(double), st, a.k, i, nsl,
                       a.v, a.u, a.Wc, a.Wr, a.mcap, a.pd, a.X, a.tau, a.beta, a.status);
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
    else if (sk.sketch == SK_SRHT)
        hipLaunchKernelGGL((k_materialize<T, SK_SRHT>), g, b, 0, st, sk, j0, j1, l0, l1, rsk, out, ldo);
    else
        hipLaunchKernelGGL((k_materialize<T, SK_IDENT>), g, b, 0, st, sk, j0, j1, l0, l1, rsk, out, ldo);
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
template bool launch_reduce<float>(hipStream_t, const float*, int, int, int, double, double*, int64_t);
template bool launch_reduce<double>(hipStream_t, const double*, int, int, int, double, double*, int64_t);
template bool launch_project<float, float>(hipStream_t, const float*, float*, int64_t, int64_t, int,
                                           const float*, const double*, int, int, int, const SketchArgs&,
                                           float*, const int*);
template bool launch_project<double, double>(hipStream_t, const double*, double*, int64_t, int64_t, int,
                                             const double*, const double*, int, int, int, const SketchArgs&,
                                             double*, const int*);
template bool launch_scale_col<float>(hipStream_t, float*, int64_t, const double*, const int*);
template bool launch_scale_col<double>(hipStream_t, double*, int64_t, const double*, const int*);
template bool launch_ls<float>(hipStream_t, const SpaceArgs&, const double*, int, double*, int64_t, float*);
template bool launch_ls<double>(hipStream_t, const SpaceArgs&, const double*, int, double*, int64_t, double*);
template bool launch_append<float>(hipStream_t, const SpaceArgs&, const float*, int, double, const double*, int,
                                   double*, int64_t, double*, int64_t);
template bool launch_append<double>(hipStream_t, const SpaceArgs&, const double*, int, double, const double*,
                                    int, double*, int64_t, double*, int64_t);
template bool launch_materialize<float>(hipStream_t, const SketchArgs&, int64_t, int64_t, int64_t, int64_t,
                                        double, double*, int64_t);
template bool launch_materialize<double>(hipStream_t, const SketchArgs&, int64_t, int64_t, int64_t, int64_t,
                                         double, double*, int64_t);

}  // namespace rgs
