// Device bodies of the RGS column step shared by the QR kernels
// (rgs_kernels.hip) and the randomized GMRES kernels (rgs_gmres.hip): the
// fp64 sketch-space work of one column (least squares on the compact-WY Householder
// factorisation of S, r_ii, and the append of s_i).  Each __global__ wrapper
// passes its block index; single-factorisation and batched wrappers call the
// same bodies, so both produce the same bits.
#pragma once

#include "rgs_internal.hpp"
#include "rgs_proj.hpp"

namespace rgs {

// ---------------------------------------------------------------------------
// Sketch-space kernels (fp64).  i = 0-based index of the current column;
// i columns are already factorised.  A "slice" is 64 consecutive sketch rows
// (one workgroup); pd buffers hold per-slice partial dot products.  These
// kernels are latency-bound, so every loop over global memory issues its
// loads in batches (independent loads first, then the fixed-order sums) to
// keep the number of dependent round trips per kernel at two or three.
// Column-parallel dot products run one thread per column over a slice;
// row-parallel products run 64 rows x 16 column groups.  The bodies are
// written for NT threads per workgroup (kGW, or kGWB in the batched kernels,
// which share the GPU with other launches and so use smaller workgroups);
// with NT < kGW a thread takes the column groups q, q + NT/64, ... and the
// fixed-shape reductions keep the kGW-thread shape, so every NT gives the
// same bits.
// ---------------------------------------------------------------------------
constexpr int kGW = 1024;   // threads of the sketch-space kernels
constexpr int kGWB = 256;   // threads of the batched sketch-space kernels
// threads of the single-factorisation column-step kernels: alone on the device
// the 1024-thread shape is faster (each thread one column group); 256 threads
// cost ≈ 8 µs per column at k = 2048
constexpr int kGWS = kGW;
// the sketch-space workspace (buffers sized for fp64) viewed in the
// sketch-space type TS
template <typename TS>
__device__ __forceinline__ TS* ws_as(double* p) {
    return reinterpret_cast<TS*>(p);
}
constexpr int kGQ = 16;     // column groups of the row-parallel products
constexpr int kBatch = 16;  // loads issued back to back per thread
constexpr int kSliceBatch = 32;   // the same in the column-parallel slice products

// sum_{s < nsl} pd[s * stride + c] (fixed order in s)
template <typename TS>
__device__ __forceinline__ TS sum_col(const TS* __restrict__ pd, int nsl, int stride, int c) {
    TS acc = TS(0);
    for (int s0 = 0; s0 < nsl; s0 += kBatch) {
        TS t[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) t[u] = (s0 + u < nsl) ? pd[(int64_t)(s0 + u) * stride + c] : TS(0);
#pragma unroll
        for (int u = 0; u < kBatch; ++u) acc += t[u];
    }
    return acc;
}

template <typename TS>
__device__ __forceinline__ void sum_slices(const TS* __restrict__ pd, int nsl, int stride, int cnt,
                                           TS* __restrict__ out) {
    for (int c = threadIdx.x; c < cnt; c += blockDim.x) out[c] = sum_col(pd, nsl, stride, c);
}

// sum_{rr < 64} M[row(rr), c] * xs[rr], M row-major with row stride mcap; rows
// past k are clamped (xs is 0 there).
template <typename TS>
__device__ __forceinline__ TS slice_dot(const TS* __restrict__ Mr, int mcap, int r0, int k,
                                        const TS* __restrict__ xs, int c) {
    TS acc = TS(0);
#pragma unroll 1
    for (int b = 0; b < kSlice; b += kSliceBatch) {
        TS t[kSliceBatch];
#pragma unroll
        for (int u = 0; u < kSliceBatch; ++u) t[u] = Mr[(int64_t)min(r0 + b + u, k - 1) * mcap + c];
#pragma unroll
        for (int u = 0; u < kSliceBatch; ++u) acc = fma(t[u], xs[b + u], acc);
    }
    return acc;
}

template <typename TS>
__device__ __forceinline__ TS slice_sq(const TS* __restrict__ xs) {
    TS acc = TS(0);
    for (int rr = 0; rr < kSlice; ++rr) acc = fma(xs[rr], xs[rr], acc);
    return acc;
}

template <typename TS>
__device__ __forceinline__ TS slice_xy(const TS* __restrict__ xs, const TS* __restrict__ ys) {
    TS acc = TS(0);
    for (int rr = 0; rr < kSlice; ++rr) acc = fma(xs[rr], ys[rr], acc);
    return acc;
}

// Row-parallel partial: sum over c in [c0, c1) with c = q (mod kGQ), ascending,
// of M[r, c] * xl[c]; M column-major with leading dimension ld.
template <typename TS>
__device__ __forceinline__ TS row_part(const TS* __restrict__ Mc, int64_t ld, int r, int c0, int c1,
                                       const TS* __restrict__ xl, int q) {
    TS acc = TS(0);
    for (int c = c0 + ((q - c0) % kGQ + kGQ) % kGQ; c < c1; c += kGQ * kBatch) {
        TS t[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int cc = c + kGQ * u;
            t[u] = (cc < c1) ? Mc[r + (int64_t)cc * ld] : TS(0);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int cc = c + kGQ * u;
            if (cc < c1) acc = fma(t[u], xl[cc], acc);
        }
    }
    return acc;
}

template <typename TS>
__device__ __forceinline__ TS combine16(TS (*red)[64], int rl) {
    TS t = TS(0);
#pragma unroll
    for (int q = 0; q < kGQ; ++q) t += red[q][rl];
    return t;
}

// Step 2, part 2: c = sum of slice partials; head of U_i^T p:
//   uh[r] = p[r] - sum_{c <= r} V[r, c] c[c],  r < i.
template <int NT = kGW, typename TS = double>
__device__ __forceinline__ void ls2_body(const TS* __restrict__ p, int k, int i, int nsl,
                                         const TS* __restrict__ Vc, int mcap, const TS* __restrict__ pd,
                                         TS* __restrict__ uh, TS* __restrict__ pnorm, int bid,
                                         TS* __restrict__ cp) {
    __shared__ TS red[kGQ][64];
    sum_slices(pd, nsl, mcap + 1, i + 1, cp);
    __syncthreads();
    if (bid == 0 && threadIdx.x == 0) pnorm[i] = sqrt(cp[i]);
    const int rl = threadIdx.x & 63, q0 = threadIdx.x >> 6;
    const int r = bid * 64 + rl;
    for (int q = q0; q < kGQ; q += NT / 64)
        red[q][rl] = (r < i) ? row_part(Vc, k, r, 0, min(r, i - 1) + 1, cp, q) : TS(0);
    __syncthreads();
    if (q0 == 0 && r < i) uh[r] = p[r] - combine16(red, rl);
}

// Step 2, last part: y = R_S^{-1} uh with X = R_S^{-1} (upper triangular, nr x nr):
//   y[r] = sum_{c >= r} X[r, c] uh[c].  Writes R(0:nr, col) and the working-
// precision coefficients coef[r] = y[r] (times cscale[r] = 1/r_rr when the
// basis is kept unnormalised).  bid = row block of 64.
template <typename T, int NT = kGW, typename TS = double>
__device__ __forceinline__ void ls3_body(int nr, int col, const TS* __restrict__ X, int mcap,
                                         const TS* __restrict__ uh, double* __restrict__ R, int64_t ldr,
                                         T* __restrict__ coef, const double* __restrict__ cscale, int bid,
                                         TS* __restrict__ us) {
    __shared__ TS red[kGQ][64];
    for (int c = threadIdx.x; c < nr; c += NT) us[c] = uh[c];
    __syncthreads();
    const int rl = threadIdx.x & 63, q0 = threadIdx.x >> 6;
    const int r = bid * 64 + rl;
    for (int q = q0; q < kGQ; q += NT / 64) red[q][rl] = (r < nr) ? row_part(X, mcap, r, r, nr, us, q) : 0.0;
    __syncthreads();
    if (q0 == 0 && r < nr) {
        const TS y = combine16(red, rl);
        R[r + (int64_t)col * ldr] = y;
        coef[r] = (T)(cscale ? y * (TS)cscale[r] : y);
    }
}

// Column step A: s' = scale * (sum of the projection kernel's block partials)
// (times scale2[0] when given: the 1/r_ii of an Arnoldi vector sketched before
// its normalisation was known) for slice bid (or a copy of src), stored in sp;
// per-slice partials of c1 = Wm_i^T s' (c < i) and of ||s'||^2 (slot i), at
// stride pstride per slice (mcap + 1 when 0).
template <typename PT, int NT = kGW, typename TS = double>
__device__ __forceinline__ void qa_body(const PT* __restrict__ partials, int G, double scale,
                                        const double* __restrict__ src, int k, int i,
                                        const TS* __restrict__ Wr, int mcap, TS* __restrict__ sp,
                                        TS* __restrict__ pd, int bid,
                                        const double* __restrict__ scale2 = nullptr, int pstride = 0) {
    __shared__ TS red[kGQ][64];
    __shared__ TS xs[kSlice];
    const int s = bid, r0 = s * kSlice, rl = threadIdx.x & 63, q0 = threadIdx.x >> 6;
    const int r = r0 + rl;
    if (src) {
        if (q0 == 0) {
            const TS val = (r < k) ? (TS)src[r] : TS(0);
            xs[rl] = val;
            if (r < k) sp[r] = val;
        }
    } else {
        // group q sums the block partials g in [G q / 16, G (q+1) / 16), in order
        for (int q = q0; q < kGQ; q += NT / 64) {
            const int g0 = (int)((int64_t)G * q / kGQ), g1 = (int)((int64_t)G * (q + 1) / kGQ);
            TS acc = TS(0);
            if (r < k) {
                for (int g = g0; g < g1; g += 32) {
                    // clamped addresses, masked after: loads under a per-element
                    // condition came out as a branch and a wait per element
                    PT t[32];
#pragma unroll
                    for (int u = 0; u < 32; ++u) t[u] = partials[(int64_t)min(g + u, g1 - 1) * k + r];
#pragma unroll
                    for (int u = 0; u < 32; ++u) acc += (g + u < g1) ? (TS)t[u] : TS(0);
                }
            }
            red[q][rl] = acc;
        }
        __syncthreads();
        if (q0 == 0) {
            TS val = (r < k) ? combine16(red, rl) * (TS)scale : TS(0);
            if (scale2) val *= (TS)scale2[0];
            xs[rl] = val;
            if (r < k) sp[r] = val;
        }
    }
    __syncthreads();
    TS* out = pd + (int64_t)s * (pstride ? pstride : mcap + 1);
    for (int c = threadIdx.x; c <= i; c += NT) out[c] = (c < i) ? slice_dot(Wr, mcap, r0, k, xs, c) : slice_sq(xs);
}

// Column step B (steps 5-6): r_ii = ||s'||, S(:, i) = s'/r_ii, breakdown test,
// u = U_i^T s_i = (s' - V c1) / r_ii, per-slice partials of ||u(i+1:k)||^2.
template <int NT = kGW, typename TS = double>
__device__ __forceinline__ void qb_body(int k, int i, int nsl, const TS* __restrict__ sp,
                                        const TS* __restrict__ Vc, int mcap, const TS* __restrict__ pd,
                                        TS* __restrict__ u, TS* __restrict__ pd2, double* __restrict__ S,
                                        int64_t lds, double* __restrict__ R, int64_t ldr, double* __restrict__ rr,
                                        double* __restrict__ invr, const TS* __restrict__ pnorm,
                                        int* __restrict__ status, int bid, TS* __restrict__ c1) {
    __shared__ TS red[kGQ][64];
    __shared__ TS tl[64];
    sum_slices(pd, nsl, mcap + 1, i + 1, c1);
    __syncthreads();
    const TS rii = sqrt(c1[i]);
    if (bid == 0 && threadIdx.x == 0) {
        rr[i] = rii;
        invr[i] = TS(1) / rii;   // the step-7 factor, in the arithmetic of the sketch space
        R[i + (int64_t)i * ldr] = rii;
        const TS pn = (i == 0) ? rii : pnorm[i];
        if (status[0] == 0 && status[2] == 0) {
            if (!isfinite(rii) || !isfinite(pn)) {
                status[1] = i;
                status[0] = kStatusNonfinite;
            } else if (rii == TS(0) || rii <= TS(0x1p-50) * pn) {
                status[1] = i;
                status[0] = kStatusBreakdown;
            }
        }
    }
    const int s = bid, rl = threadIdx.x & 63, q0 = threadIdx.x >> 6;
    const int r = s * kSlice + rl;
    for (int q = q0; q < kGQ; q += NT / 64) red[q][rl] = (r < k) ? row_part(Vc, k, r, 0, i, c1, q) : TS(0);
    __syncthreads();
    if (q0 == 0) {
        TS t2 = TS(0);
        if (r < k) {
            const TS spr = sp[r];
            const TS val = (spr - combine16(red, rl)) / rii;
            u[r] = val;
            S[r + (int64_t)i * lds] = spr / rii;
            if (r > i) t2 = val * val;
        }
        tl[rl] = t2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        TS acc = TS(0);
        for (int t = 0; t < 64; ++t) acc += tl[t];
        pd2[s] = acc;
    }
}

// Column step C: Householder reflector of u(i:k) (dlarfg convention):
// beta = -sign(u_i) ||u(i:k)||, tau = (beta - u_i)/beta, v = [0; 1; u(i+1:k)/(u_i - beta)],
// stored as column i of V (both layouts).  Per-slice partials of d = V_i^T v
// (pd, stride mcap+1) and, when the next right-hand side pn = p_{i+1} is given,
// of e = Wm_i^T pn, v.pn and ||pn||^2 (pdb, stride mcap+2, slots [0,i), i, i+1).
template <int NT = kGW, typename TS = double>
__device__ __forceinline__ void qc_body(int k, int i, int nsl, const TS* __restrict__ u,
                                        const TS* __restrict__ pd2, const double* __restrict__ pn,
                                        TS* __restrict__ v, TS* __restrict__ Vc, TS* __restrict__ Vr,
                                        const TS* __restrict__ Wr, int mcap, TS* __restrict__ pd,
                                        TS* __restrict__ pdb, TS* __restrict__ tau_a,
                                        TS* __restrict__ beta_a, int* __restrict__ status, int bid) {
    __shared__ TS vs[kSlice], ps[kSlice];
    __shared__ TS hh[3];
    if (threadIdx.x == 0) {
        const TS tail2 = sum_col(pd2, nsl, 1, 0);   // ascending s, loads in batches
        const TS x1 = u[i];
        TS beta, tau, scal;
        if (tail2 == TS(0)) {
            beta = x1;
            tau = TS(0);
            scal = TS(0);
        } else {
            beta = -copysign(sqrt(x1 * x1 + tail2), x1);
            tau = (beta - x1) / beta;
            scal = TS(1) / (x1 - beta);
        }
        hh[0] = beta;
        hh[1] = tau;
        hh[2] = scal;
        if (bid == 0) {
            tau_a[i] = tau;
            beta_a[i] = beta;
            if (status[0] == 0 && status[2] == 0 && !(fabs(beta) > TS(0x1p-50))) {   // s_i in span(S_{i-1})
                status[1] = i;
                status[0] = kStatusBreakdown;
            }
        }
    }
    __syncthreads();
    const int s = bid, r0 = s * kSlice;
    if (threadIdx.x < kSlice) {
        const int r = r0 + threadIdx.x;
        TS val = TS(0);
        if (r < k) {
            val = (r < i) ? TS(0) : (r == i ? TS(1) : u[r] * hh[2]);
            v[r] = val;
            Vc[r + (int64_t)i * k] = val;
            Vr[(int64_t)r * mcap + i] = val;
        }
        vs[threadIdx.x] = val;
        ps[threadIdx.x] = (pn && r < k) ? (TS)pn[r] : TS(0);
    }
    __syncthreads();
    const int ntot = pn ? 2 * i + 2 : i;
    TS* outd = pd + (int64_t)s * (mcap + 1);
    TS* oute = pdb + (int64_t)s * (mcap + 2);
    for (int c = threadIdx.x; c < ntot; c += NT) {
        const bool isd = c < i;
        const int ce = isd ? c : c - i;
        TS val;
        if (isd || ce < i) {
            val = slice_dot(isd ? Vr : Wr, mcap, r0, k, isd ? vs : ps, ce);
        } else {
            val = (ce == i) ? slice_xy(vs, ps) : slice_sq(ps);
        }
        if (isd) outd[c] = val;
        else oute[ce] = val;
    }
}

// Column step D.  Blocks [0, nsl): Wm(:, i) = tau (v - Wm_i d), d = sum of the slice partials.
// Blocks [nsl, ...), rows r of [64 b, 64 b + 64):
//   column i of X = R_S^{-1}: X(r, i) = -(sum_{c=r}^{i-1} X(r, c) u(c)) / beta for r < i
//   (u(0:i) is R_S(0:i, i)), X(i, i) = 1/beta;
//   when pn is given, the head of U_{i+1}^T pn for the next column's least squares:
//   cp = Wm_{i+1}^T pn = [e; tau (v.pn - d.e)],  uh(r) = pn(r) - sum_{c <= min(r,i)} V(r, c) cp(c), r <= i.
template <int NT = kGW, typename TS = double>
__device__ __forceinline__ void qd_body(int k, int i, int nsl, const TS* __restrict__ v,
                                        const TS* __restrict__ u, const double* __restrict__ pn,
                                        TS* __restrict__ Wc, TS* __restrict__ Wr,
                                        const TS* __restrict__ Vc, int mcap, const TS* __restrict__ pd,
                                        const TS* __restrict__ pdb, TS* __restrict__ X,
                                        TS* __restrict__ uh, TS* __restrict__ pnorm,
                                        const TS* __restrict__ tau_a, const TS* __restrict__ beta_a,
                                        int bid, TS* __restrict__ dyn) {
    __shared__ TS red[kGQ][64];
    __shared__ TS tree[NT];
    const int rl = threadIdx.x & 63, q0 = threadIdx.x >> 6;
    const TS tau = tau_a[i];
    if (bid < nsl) {
        TS* dsh = dyn;
        sum_slices(pd, nsl, mcap + 1, i, dsh);
        __syncthreads();
        const int r = bid * kSlice + rl;
        for (int q = q0; q < kGQ; q += NT / 64) red[q][rl] = (r < k) ? row_part(Wc, k, r, 0, i, dsh, q) : TS(0);
        __syncthreads();
        if (q0 == 0 && r < k) {
            const TS val = tau * (v[r] - combine16(red, rl));
            Wc[r + (int64_t)i * k] = val;
            Wr[(int64_t)r * mcap + i] = val;
        }
        if (bid == 0 && threadIdx.x == 0) X[i + (int64_t)i * mcap] = TS(1) / beta_a[i];
        return;
    }
    TS* ush = dyn;            // u(0:i)
    TS* dsh = dyn + (i + 1);  // d
    TS* csh = dsh + (i + 1);  // cp
    for (int c = threadIdx.x; c < i; c += NT) ush[c] = u[c];
    if (pn) {
        for (int c = threadIdx.x; c < 2 * i + 2; c += NT) {
            if (c < i) dsh[c] = sum_col(pd, nsl, mcap + 1, c);
            else csh[c - i] = sum_col(pdb, nsl, mcap + 2, c - i);   // e, then v.pn at i, ||pn||^2 at i+1
        }
    }
    __syncthreads();
    const int r = (bid - nsl) * 64 + rl;
    for (int q = q0; q < kGQ; q += NT / 64) red[q][rl] = (r < i) ? row_part(X, mcap, r, r, i, ush, q) : TS(0);
    __syncthreads();
    if (q0 == 0 && r < i) X[r + (int64_t)i * mcap] = -combine16(red, rl) / beta_a[i];
    if (!pn) return;
    // d.e by a fixed-shape tree over kGW leaves (leaf t: the products c = t
    // (mod kGW), ascending), then cp(i) = tau (v.pn - d.e).  A thread holds
    // the leaves threadIdx.x + NT j; the levels wider than NT are summed in
    // its registers, the rest in LDS.
    constexpr int V = kGW / NT;
    TS part[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        part[j] = TS(0);
        for (int c = threadIdx.x + NT * j; c < i; c += kGW) part[j] = fma(dsh[c], csh[c], part[j]);
    }
#pragma unroll
    for (int w = kGW / 2; w >= NT; w >>= 1)
#pragma unroll
        for (int j = 0; j < w / NT; ++j) part[j] += part[j + w / NT];
    tree[threadIdx.x] = part[0];
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) tree[threadIdx.x] += tree[threadIdx.x + w];
        __syncthreads();
    }
    const TS vp = csh[i], pp = csh[i + 1];
    __syncthreads();
    if (threadIdx.x == 0) csh[i] = tau * (vp - tree[0]);
    if (bid == nsl && threadIdx.x == 0) pnorm[i + 1] = sqrt(pp);
    __syncthreads();
    for (int q = q0; q < kGQ; q += NT / 64) red[q][rl] = (r <= i) ? row_part(Vc, k, r, 0, min(r, i) + 1, csh, q) : TS(0);
    __syncthreads();
    if (q0 == 0 && r <= i) uh[r] = (TS)pn[r] - combine16(red, rl);
}

// ---------------------------------------------------------------------------
// Step 2 by Richardson iterations on the normal equations (remark on the
// least-squares solver in Sec. 2.3): y = S^T p, then y <- y + S^T (p - S y)
// per further sweep; one sweep is the sketched classical Gram-Schmidt.  S is
// kept row-major as well (stride mcap, in the Wr buffer, unused by this
// solver otherwise) for the column-parallel dot products.  Steps 5-6 are as
// in the Householder chain (qa_body run with i = 0 gives s' and the slice
// partials of ||s'||^2).
// ---------------------------------------------------------------------------

// Column step B (Richardson): r_ii = ||s'||, S(:, i) = s'/r_ii in both
// layouts, breakdown test as qb_body (without the Householder beta test), and,
// when the next right-hand side pn is given, the slice partials of S_{i+1}^T pn
// (slots 0..i) and ||pn||^2 (slot i+1), stride mcap + 2.
__device__ __forceinline__ void rb_body(int k, int i, int nsl, const double* __restrict__ sp,
                                        const double* __restrict__ pd, int mcap, double* __restrict__ S, int64_t lds,
                                        double* __restrict__ Sr, double* __restrict__ R, int64_t ldr,
                                        double* __restrict__ rr, double* __restrict__ invr,
                                        const double* __restrict__ pnorm, int* __restrict__ status,
                                        const double* __restrict__ pn, double* __restrict__ pdb, int bid) {
    __shared__ double ss[kSlice], ps[kSlice];
    __shared__ double rii_s;
    if (threadIdx.x == 0) rii_s = sqrt(sum_col(pd, nsl, mcap + 1, 0));
    __syncthreads();
    const double rii = rii_s;
    if (bid == 0 && threadIdx.x == 0) {
        rr[i] = rii;
        invr[i] = 1.0 / rii;
        R[i + (int64_t)i * ldr] = rii;
        const double pnv = (i == 0) ? rii : pnorm[i];
        if (status[0] == 0 && status[2] == 0) {
            if (!isfinite(rii) || !isfinite(pnv)) {
                status[1] = i;
                status[0] = kStatusNonfinite;
            } else if (rii == 0.0 || rii <= 0x1p-50 * pnv) {
                status[1] = i;
                status[0] = kStatusBreakdown;
            }
        }
    }
    const int r0 = bid * kSlice;
    if (threadIdx.x < kSlice) {
        const int r = r0 + threadIdx.x;
        double sv = 0.0, pv = 0.0;
        if (r < k) {
            sv = sp[r] / rii;
            S[r + (int64_t)i * lds] = sv;
            Sr[(int64_t)r * mcap + i] = sv;
            if (pn) pv = pn[r];
        }
        ss[threadIdx.x] = sv;
        ps[threadIdx.x] = pv;
    }
    __syncthreads();
    if (!pn) return;
    double* out = pdb + (int64_t)bid * (mcap + 2);
    // column i from shared memory: this workgroup's own writes of Sr are not read back
    for (int c = threadIdx.x; c <= i + 1; c += kGW)
        out[c] = (c < i) ? slice_dot(Sr, mcap, r0, k, ps, c) : (c == i ? slice_xy(ss, ps) : slice_sq(ps));
}

// Richardson: y[c] = (y[c] +) sum of the slice partials (c <= i); the first
// sweep also sets pnorm[i+1] from slot i+1; the last writes R(0:i+1, i+1) = y
// and the working-precision coefficients (times cscale[c] when given).
template <typename T>
__device__ __forceinline__ void rsum_body(int i, int nsl, int mcap, const double* __restrict__ pdb,
                                          double* __restrict__ y, int accumulate, int last,
                                          double* __restrict__ pnorm, double* __restrict__ R, int64_t ldr,
                                          T* __restrict__ coef, const double* __restrict__ cscale, int bid) {
    const int c = bid * kGW + threadIdx.x;
    if (c <= i) {
        double v = sum_col(pdb, nsl, mcap + 2, c);
        if (accumulate) v += y[c];
        y[c] = v;
        if (last) {
            R[c + (int64_t)(i + 1) * ldr] = v;
            coef[c] = (T)(cscale ? v * cscale[c] : v);
        }
    }
    if (!accumulate && bid == 0 && threadIdx.x == 0) pnorm[i + 1] = sqrt(sum_col(pdb, nsl, mcap + 2, i + 1));
}

// Richardson, one more sweep: t = pn - S y on the slice's rows (row-parallel),
// then the slice partials of S^T t (slots 0..i, stride mcap + 2).
__device__ __forceinline__ void rres_body(int k, int i, int mcap, const double* __restrict__ Sc, int64_t lds,
                                          const double* __restrict__ Sr, const double* __restrict__ pn,
                                          const double* __restrict__ y, double* __restrict__ pdb, int bid) {
    __shared__ double red[kGQ][64];
    __shared__ double ts[kSlice];
    const int rl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int r = bid * kSlice + rl;
    red[q][rl] = (r < k) ? row_part(Sc, lds, r, 0, i + 1, y, q) : 0.0;
    __syncthreads();
    if (q == 0) ts[rl] = (r < k) ? pn[r] - combine16(red, rl) : 0.0;
    __syncthreads();
    double* out = pdb + (int64_t)bid * (mcap + 2);
    for (int c = threadIdx.x; c <= i; c += kGW) out[c] = slice_dot(Sr, mcap, bid * kSlice, k, ts, c);
}

}  // namespace rgs
