// Randomized GMRES kernels (Sec. 4 of Balabanov & Grigori) for gfx950.
//
// RGS-Arnoldi (Algorithm 3) builds the Krylov basis with the RGS column step:
// w_1 = r_0, then w_i = A q_{i-1}.  Here A is a constant-coefficient 7-point
// operator applied matrix-free, and the sketch p_i = Theta w_i of step 1 is
// fused into the mat-vec (same per-block partials as the projection kernel).
// The Hessenberg matrix is H = R(1:i, 2:i) (Sec. 4.1); its least-squares
// problem min ||H y - r_11 e_1|| is solved by Givens rotations in fp64
// (Sec. 4.2), with |g_{i+1}| the sketched residual ||Theta (b - A x_i)||.
// x and the restart residual b - A x are kept in fp64.
//
// Status word (shared with the QR kernels): [0] breakdown / non-finite,
// [1] failed column, [2] "cycle done" (converged or lucky breakdown): once it
// is set the remaining launches of the cycle return immediately.

#include "rgs_block.hpp"
#include "rgs_device.hpp"
#include "rgs_internal.hpp"

namespace rgs {

namespace {

__device__ __forceinline__ bool cycle_stopped(const int* status) { return status[0] != 0 || status[2] != 0; }

#define RGS_EXIT_IF_STOPPED(status)                                   \
    do {                                                              \
        __shared__ int rgs_stop_;                                     \
        if (threadIdx.x == 0) rgs_stop_ = cycle_stopped(status);      \
        __syncthreads();                                              \
        if (rgs_stop_) return;                                        \
    } while (0)

struct Grid3 {
    int nx, ny, nz;
    double c0, cxm, cxp, cym, cyp, czm, czp;
};

// (A u)_l for one row l, u read through `ld` (a functor giving u at an index).
template <typename T, typename Load>
__device__ __forceinline__ T stencil_row(const Grid3& g, int64_t l, const Load& ld) {
    const uint32_t nxy = (uint32_t)g.nx * (uint32_t)g.ny;
    const uint32_t lu = (uint32_t)l;
    const uint32_t z = lu / nxy;
    const uint32_t rem = lu - z * nxy;
    const uint32_t y = rem / (uint32_t)g.nx;
    const uint32_t x = rem - y * (uint32_t)g.nx;
    // same association as a left-to-right sum: c0 u + xm + xp + ym + yp + zm + zp
    T acc = (T)g.c0 * ld(l);
    acc = acc + (x > 0 ? (T)g.cxm * ld(l - 1) : T(0));
    acc = acc + (x + 1 < (uint32_t)g.nx ? (T)g.cxp * ld(l + 1) : T(0));
    acc = acc + (y > 0 ? (T)g.cym * ld(l - g.nx) : T(0));
    acc = acc + (y + 1 < (uint32_t)g.ny ? (T)g.cyp * ld(l + g.nx) : T(0));
    acc = acc + (z > 0 ? (T)g.czm * ld(l - (int64_t)nxy) : T(0));
    acc = acc + (z + 1 < (uint32_t)g.nz ? (T)g.czp * ld(l + (int64_t)nxy) : T(0));
    return acc;
}

}  // namespace

// Step 3 of Algorithm 3 (+ step 1 of Algorithm 2): w = A q with q = q' / r
// normalised on the fly (fp64 reciprocal, rounded to T, exactly as the next
// projection pass will store it), then the block's sketch partials of w.
// Block layout identical to k_project (kProjWaves wave tiles of 1024 rows).
template <typename T, typename PT, int SK>
__global__ __launch_bounds__(kProjWaves * kWave) void k_stencil_sketch(
    const T* __restrict__ qp, const double* __restrict__ invr, Grid3 g, int64_t n, T* __restrict__ w,
    int do_sketch, SketchArgs sk, PT* __restrict__ partials, const int* __restrict__ status) {
    constexpr int NW = kProjWaves;
    __shared__ T lds[NW * kTile];
    RGS_EXIT_IF_STOPPED(status);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t blk = blockIdx.x;
    const double ir = invr ? invr[0] : 1.0;
    auto ld = [&](int64_t idx) -> T { return invr ? (T)((double)qp[idx] * ir) : qp[idx]; };
    T v[16];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t r0 = blk * (NW * kTile) + wave * kTile + 256 * e + 4 * lane;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t l = r0 + r;
            v[4 * e + r] = (l < n) ? stencil_row<T>(g, l, ld) : T(0);
            if (l < n) w[l] = v[4 * e + r];
        }
    }
    if (!do_sketch) return;
    PT acc[kKptMax];
#pragma unroll
    for (int u = 0; u < kKptMax; ++u) acc[u] = PT(0);
    if constexpr (SK == SK_IDENT) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r0 = blk * (NW * kTile) + wave * kTile + 256 * e + 4 * lane;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r0 + r < n) partials[r0 + r] = (PT)v[4 * e + r];
        }
    } else {
        block_sketch<T, PT, SK, NW>(v, blk, n, sk, acc, lds);
        constexpr int NT = NW * kWave;
        const int kpt = (sk.k + NT - 1) / NT;
        PT* out = partials + blk * sk.k;
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) {
            const int jj = threadIdx.x + NT * u;
            if (u < kpt && jj < sk.k) out[jj] = acc[u];
        }
    }
}

// r = b - A x in fp64, and per-block partial sums of ||r||^2 (one per workgroup of 256 rows).
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ b, const double* __restrict__ x,
                                                  Grid3 g, int64_t n, double* __restrict__ r,
                                                  double* __restrict__ part) {
    __shared__ double red[256];
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double val = 0.0;
    if (l < n) {
        auto ld = [&](int64_t idx) -> double { return x[idx]; };
        val = b[l] - stencil_row<double>(g, l, ld);
        r[l] = val;
    }
    red[threadIdx.x] = val * val;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = sqrt(sum of G partials), fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_norm_finish(const double* __restrict__ part, int64_t G,
                                                     double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    const int64_t per = (G + 255) / 256;
    const int64_t g0 = threadIdx.x * per, g1 = min(G, g0 + per);
    for (int64_t gi = g0; gi < g1; ++gi) acc += part[gi];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

template <typename T>
__global__ void k_cast(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n) dst[l] = (T)src[l];
}

// One Givens step for Hessenberg column c-1 (0-based basis column c >= 1):
// h = R(0:c, c) (RGS R column, h_c = r_cc), apply the c-1 previous rotations,
// form rotation c-1 that zeroes h_c, update g; record |g_c| / ||b|| in the
// history and stop the cycle when it is <= tol or at a lucky breakdown
// (status[0] = breakdown at column c: h_c = 0).  One thread: at most
// `restart` rotations of 2-vectors.
__global__ void k_givens(int c, const double* __restrict__ R, int mcap, double* __restrict__ Hr,
                         double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ gv,
                         double bnorm, double tol, double* __restrict__ hist, int* __restrict__ status,
                         int* __restrict__ used) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (status[2] != 0) return;
    bool lucky = false;
    if (status[0] != 0) {
        if (status[0] == kStatusBreakdown && status[1] == c) {
            lucky = true;          // w_c numerically in span(Q_c): exact Krylov space reached
        } else {
            return;                // non-finite data: the host reports it
        }
    }
    double* h = Hr + (int64_t)(c - 1) * mcap;   // rotated column c-1 of H
    for (int t = 0; t < c; ++t) h[t] = R[t + (int64_t)c * mcap];
    h[c] = lucky ? 0.0 : R[c + (int64_t)c * mcap];
    for (int t = 0; t < c - 1; ++t) {
        const double a = h[t], bb = h[t + 1];
        h[t] = cs[t] * a + sn[t] * bb;
        h[t + 1] = -sn[t] * a + cs[t] * bb;
    }
    const double a = h[c - 1], bb = h[c];
    double co = 1.0, si = 0.0, rho = a;
    if (bb != 0.0) {
        rho = hypot(a, bb);
        co = a / rho;
        si = bb / rho;
    }
    cs[c - 1] = co;
    sn[c - 1] = si;
    h[c - 1] = rho;
    h[c] = 0.0;
    gv[c] = -si * gv[c - 1];
    gv[c - 1] = co * gv[c - 1];
    const double est = fabs(gv[c]) / bnorm;
    hist[c - 1] = est;
    used[0] = c;
    if (lucky) status[0] = 0;       // a lucky breakdown is not an error in GMRES
    if (lucky || est <= tol) status[2] = 1;
}

// g(0) = r_11 = R(0, 0) at the start of a cycle.
__global__ void k_givens_init(const double* __restrict__ R, double* __restrict__ gv, int* __restrict__ used) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        gv[0] = R[0];
        used[0] = 0;
    }
}

// y = Hr(0:u, 0:u)^{-1} g(0:u), u = used[0]: back substitution (one thread).
__global__ void k_backsub(const double* __restrict__ Hr, int mcap, const double* __restrict__ gv,
                          const int* __restrict__ used, double* __restrict__ y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int u = used[0];
    for (int r = u - 1; r >= 0; --r) {
        double acc = gv[r];
        for (int c = r + 1; c < u; ++c) acc -= Hr[r + (int64_t)c * mcap] * y[c];
        y[r] = acc / Hr[r + (int64_t)r * mcap];
    }
}

// x += Q(:, 0:u) y in fp64 (u = used[0]; columns in ascending order).
template <typename T>
__global__ __launch_bounds__(256) void k_xupdate(double* __restrict__ x, const T* __restrict__ Q, int64_t ldq,
                                                 int64_t n, const int* __restrict__ used,
                                                 const double* __restrict__ y) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= n) return;
    const int u = used[0];
    double acc = x[l];
    for (int c = 0; c < u; ++c) acc += (double)Q[l + (int64_t)c * ldq] * y[c];
    x[l] = acc;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define RGS_LAUNCH_CHECK()                                   \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return false;   \
    } while (0)

static inline unsigned nblk_of(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

static Grid3 grid3(const StencilArgs& a) {
    Grid3 g;
    g.nx = (int)a.nx;
    g.ny = (int)a.ny;
    g.nz = (int)a.nz;
    g.c0 = a.c[0];
    g.cxm = a.c[1];
    g.cxp = a.c[2];
    g.cym = a.c[3];
    g.cyp = a.c[4];
    g.czm = a.c[5];
    g.czp = a.c[6];
    return g;
}

template <typename T, typename PT>
bool launch_stencil_sketch(hipStream_t st, const StencilArgs& A, const T* qp, const double* invr, T* w,
                           int do_sketch, const SketchArgs& sk, PT* partials, const int* status) {
    const int64_t n = A.nx * A.ny * A.nz;
    const Grid3 g = grid3(A);
    const dim3 grid(nblk_of(n, kProjRows)), thr(kProjWaves * kWave);
    if (sk.sketch == SK_SRHT)
        hipLaunchKernelGGL((k_stencil_sketch<T, PT, SK_SRHT>), grid, thr, 0, st, qp, invr, g, n, w, do_sketch, sk,
                           partials, status);
    else if (sk.sketch == SK_GAUSS)
        hipLaunchKernelGGL((k_stencil_sketch<T, PT, SK_GAUSS>), grid, thr, 0, st, qp, invr, g, n, w, do_sketch,
                           sk, partials, status);
    else
        hipLaunchKernelGGL((k_stencil_sketch<T, PT, SK_IDENT>), grid, thr, 0, st, qp, invr, g, n, w, do_sketch,
                           sk, partials, status);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_residual(hipStream_t st, const StencilArgs& A, const double* b, const double* x, double* r,
                     double* part, double* norm_out) {
    const int64_t n = A.nx * A.ny * A.nz;
    const unsigned G = nblk_of(n, 256);
    hipLaunchKernelGGL(k_residual, dim3(G), dim3(256), 0, st, b, x, grid3(A), n, r, part);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(256), 0, st, part, (int64_t)G, norm_out);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T>
bool launch_cast(hipStream_t st, const double* src, T* dst, int64_t n) {
    hipLaunchKernelGGL(k_cast<T>, dim3(nblk_of(n, 256)), dim3(256), 0, st, src, dst, n);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_givens_init(hipStream_t st, const double* R, double* gv, int* used) {
    hipLaunchKernelGGL(k_givens_init, dim3(1), dim3(64), 0, st, R, gv, used);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_givens(hipStream_t st, int c, const double* R, int mcap, double* Hr, double* cs, double* sn,
                   double* gv, double bnorm, double tol, double* hist, int* status, int* used) {
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, st, c, R, mcap, Hr, cs, sn, gv, bnorm, tol, hist, status,
                       used);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T>
bool launch_update_x(hipStream_t st, const double* Hr, int mcap, const double* gv, const int* used, double* y,
                     double* x, const T* Q, int64_t ldq, int64_t n) {
    hipLaunchKernelGGL(k_backsub, dim3(1), dim3(64), 0, st, Hr, mcap, gv, used, y);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_xupdate<T>, dim3(nblk_of(n, 256)), dim3(256), 0, st, x, Q, ldq, n, used, y);
    RGS_LAUNCH_CHECK();
    return true;
}

template bool launch_stencil_sketch<float, float>(hipStream_t, const StencilArgs&, const float*, const double*,
                                                  float*, int, const SketchArgs&, float*, const int*);
template bool launch_stencil_sketch<double, double>(hipStream_t, const StencilArgs&, const double*, const double*,
                                                    double*, int, const SketchArgs&, double*, const int*);
template bool launch_cast<float>(hipStream_t, const double*, float*, int64_t);
template bool launch_cast<double>(hipStream_t, const double*, double*, int64_t);
template bool launch_update_x<float>(hipStream_t, const double*, int, const double*, const int*, double*, double*,
                                     const float*, int64_t, int64_t);
template bool launch_update_x<double>(hipStream_t, const double*, int, const double*, const int*, double*,
                                      double*, const double*, int64_t, int64_t);

}  // namespace rgs
