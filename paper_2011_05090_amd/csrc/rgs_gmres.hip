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
// Every kernel is a thin wrapper around a device body.  The single-system
// wrappers take explicit arguments; the batched ("kg_") wrappers map their
// workgroup to (system, local block) through a host-built table and read the
// system's pointers from its BatchItem (column-step state) and GmresItem
// (operator, x, residual, Givens state).  Both call the same bodies, so a
// batched solve reproduces separate solves bit for bit.
//
// Status word (shared with the QR kernels): [0] breakdown / non-finite,
// [1] failed column, [2] "cycle done" (converged, lucky breakdown or the
// cycle's step limit): once it is set the remaining launches of the cycle
// return immediately.

#include "rgs_map.hpp"
#include "rgs_step.hpp"

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

__host__ __device__ inline Grid3 grid3(const StencilArgs& a) {
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

__device__ __forceinline__ double to_double(float v) { return (double)v; }
__device__ __forceinline__ double to_double(double v) { return v; }
__device__ __forceinline__ double to_double(bf16 v) { return (double)bf16_to_float(v.bits); }

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

// p + i; with a 32-bit index, as a 32-bit byte offset from p (the caller has
// checked that the column spans less than 4 GiB), which the loads take as one
// register instead of a 64-bit address.
template <typename TQ, typename I>
__device__ __forceinline__ const TQ* at(const TQ* p, I i) {
    if constexpr (std::is_same<I, uint32_t>::value)
        return reinterpret_cast<const TQ*>(reinterpret_cast<const char*>(p) + i * (uint32_t)sizeof(TQ));
    else
        return p + i;
}

// Four stored values at rows l .. l+3 (l % 4 == 0, 16-byte aligned fp32 /
// 8-byte bf16 / 2 x 16-byte fp64 vector loads), widened to double.
template <typename I>
__device__ __forceinline__ void ld4_raw(const float* __restrict__ p, I l, double o[4]) {
    const f32x4 t = *reinterpret_cast<const f32x4*>(at(p, l));
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
}
template <typename I>
__device__ __forceinline__ void ld4_raw(const double* __restrict__ p, I l, double o[4]) {
    const f64x2 a = *reinterpret_cast<const f64x2*>(at(p, l)), b = *reinterpret_cast<const f64x2*>(at(p, l + 2));
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}
template <typename I>
__device__ __forceinline__ void ld4_raw(const bf16* __restrict__ p, I l, double o[4]) {
    const u32x2 t = *reinterpret_cast<const u32x2*>(at(p, l));
    o[0] = __uint_as_float(t.x << 16);
    o[1] = __uint_as_float(t.x & 0xFFFF0000u);
    o[2] = __uint_as_float(t.y << 16);
    o[3] = __uint_as_float(t.y & 0xFFFF0000u);
}

// Rows l0 .. l0+3 (l0 % 4 == 0) of w = A u, u = (T)(stored * ir) when SCALE,
// else (T)stored; out[r] = 0 past n, cen[r] = u at row l0 + r.  Same per-row
// association as stencil_row, so the same bits.  With vec (nx % 4 == 0 and an
// aligned column) the four rows share y and z: the centre and each of the
// four y/z neighbour planes are one vector load, plus the two x neighbours
// outside the group, addressed by 32-bit offsets when O32 (n sizeof(TQ) <
// 2^32).  Otherwise the rows are stepped from one coordinate division and
// read element by element.  TC: the arithmetic of the products with A (T, or
// fp64 for the configuration of Sec. 5.3, the result rounded once to T).
template <typename T, typename TQ, bool SCALE, bool O32, typename TC = T>
__device__ __forceinline__ void stencil4(const Grid3& g, const TQ* __restrict__ qs, double ir, bool vec, int64_t l0,
                                         int64_t n, T out[4], T cen[4]) {
    const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny, nz = (uint32_t)g.nz, nxy = nx * ny;
    const uint32_t lu = (uint32_t)l0;
    uint32_t z = lu / nxy;
    const uint32_t rem = lu - z * nxy;
    uint32_t y = rem / nx;
    uint32_t x = rem - y * nx;
    auto cv = [&](double d) -> T {
        if constexpr (SCALE)
            return (T)(d * ir);
        else
            return (T)d;
    };
    auto ld1 = [&](auto idx) -> T { return cv(to_double(*at(qs, idx))); };
    // results in local arrays with one store sequence at the end: stores
    // through out/cen on several paths keep the caller's array out of registers
    T ro[4], rc[4];
    if (vec) {
        if (l0 >= n) {   // n is a multiple of 4 here: whole groups only
#pragma unroll
            for (int r = 0; r < 4; ++r) ro[r] = rc[r] = T(0);
        } else {
            // every load reads a valid address (a missing neighbour reads the
            // centre group) and the value is dropped afterwards: loads under a
            // condition would each be a branch and a wait
            using I = typename std::conditional<O32, uint32_t, int64_t>::type;
            const I lc = (I)l0;
            double a[4], am[4], ap[4], bm[4], bp[4];
            T u[4], ym[4], yp[4], zm[4], zp[4];
            const bool hxm = x > 0, hxp = x + 4 < nx, hym = y > 0, hyp = y + 1 < ny, hzm = z > 0, hzp = z + 1 < nz;
            ld4_raw(qs, lc, a);
            ld4_raw(qs, hym ? lc - (I)nx : lc, am);
            ld4_raw(qs, hyp ? lc + (I)nx : lc, ap);
            ld4_raw(qs, hzm ? lc - (I)nxy : lc, bm);
            ld4_raw(qs, hzp ? lc + (I)nxy : lc, bp);
            const T xm0 = ld1(hxm ? lc - 1 : lc), xp0 = ld1(hxp ? lc + 4 : lc);
            const T xm = hxm ? xm0 : T(0), xp = hxp ? xp0 : T(0);
            // a missing y / z neighbour's value (read from the centre) is dropped by
            // the term's own condition below
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                u[r] = cv(a[r]);
                ym[r] = cv(am[r]);
                yp[r] = cv(ap[r]);
                zm[r] = cv(bm[r]);
                zp[r] = cv(bp[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                TC acc = (TC)g.c0 * (TC)u[r];
                acc = acc + (x + r > 0 ? (TC)g.cxm * (TC)(r > 0 ? u[r - 1] : xm) : TC(0));
                acc = acc + (x + r + 1 < nx ? (TC)g.cxp * (TC)(r < 3 ? u[r + 1] : xp) : TC(0));
                acc = acc + (y > 0 ? (TC)g.cym * (TC)ym[r] : TC(0));
                acc = acc + (y + 1 < ny ? (TC)g.cyp * (TC)yp[r] : TC(0));
                acc = acc + (z > 0 ? (TC)g.czm * (TC)zm[r] : TC(0));
                acc = acc + (z + 1 < nz ? (TC)g.czp * (TC)zp[r] : TC(0));
                ro[r] = (T)acc;
                rc[r] = u[r];
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // as in the vector path: valid addresses always (a row past n reads
            // row n - 1, a missing neighbour the row itself), values dropped after
            const int64_t l = l0 + r;
            const bool live = l < n;
            const int64_t lc = live ? l : n - 1;
            const bool hxm = live && x > 0, hxp = live && x + 1 < nx, hym = live && y > 0,
                       hyp = live && y + 1 < ny, hzm = live && z > 0, hzp = live && z + 1 < nz;
            const T c = ld1(lc);
            const T vxm = ld1(hxm ? lc - 1 : lc), vxp = ld1(hxp ? lc + 1 : lc);
            const T vym = ld1(hym ? lc - nx : lc), vyp = ld1(hyp ? lc + nx : lc);
            const T vzm = ld1(hzm ? lc - (int64_t)nxy : lc), vzp = ld1(hzp ? lc + (int64_t)nxy : lc);
            TC acc = (TC)g.c0 * (TC)c;
            acc = acc + (hxm ? (TC)g.cxm * (TC)vxm : TC(0));
            acc = acc + (hxp ? (TC)g.cxp * (TC)vxp : TC(0));
            acc = acc + (hym ? (TC)g.cym * (TC)vym : TC(0));
            acc = acc + (hyp ? (TC)g.cyp * (TC)vyp : TC(0));
            acc = acc + (hzm ? (TC)g.czm * (TC)vzm : TC(0));
            acc = acc + (hzp ? (TC)g.czp * (TC)vzp : TC(0));
            ro[r] = live ? (T)acc : T(0);
            rc[r] = live ? c : T(0);
            if (++x == nx) {
                x = 0;
                if (++y == ny) {
                    y = 0;
                    ++z;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out[r] = ro[r];
        cen[r] = rc[r];
    }
}

// Stores 4 values at rows l0 .. l0+3 (rows past n skipped): one vector store
// when the group is whole and aligned.
template <typename T>
__device__ __forceinline__ void st4(T* __restrict__ w, int64_t l0, int64_t n, bool vec, const T v[4]) {
    if (vec && l0 + 4 <= n) {
        if constexpr (sizeof(T) == 4) {
            f32x4 t;
            t.x = v[0];
            t.y = v[1];
            t.z = v[2];
            t.w = v[3];
            *reinterpret_cast<f32x4*>(w + l0) = t;
        } else {
            typedef double f64x2 __attribute__((ext_vector_type(2)));
            f64x2 a, b;
            a.x = v[0];
            a.y = v[1];
            b.x = v[2];
            b.y = v[3];
            *reinterpret_cast<f64x2*>(w + l0) = a;
            *reinterpret_cast<f64x2*>(w + l0 + 2) = b;
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (l0 + r < n) w[l0 + r] = v[r];
}

template <typename TQ, typename T>
__device__ __forceinline__ bool stencil_vec_ok(const Grid3& g, const TQ* qs, const T* w) {
    return (g.nx % 4 == 0) && ((reinterpret_cast<uintptr_t>(qs) & (4 * sizeof(TQ) - 1)) == 0) &&
           ((reinterpret_cast<uintptr_t>(w) & (4 * sizeof(T) - 1)) == 0);
}

// ---------------------------------------------------------------------------
// Device bodies
// ---------------------------------------------------------------------------

// Step 3 of Algorithm 3 (+ step 1 of Algorithm 2): w = A q with q = qs * invr
// (qs the stored column, invr its fp64 reciprocal scale; the product rounded
// to T exactly as a normalising projection pass stores it), then the block's
// sketch partials of w.  Block layout identical to the projection kernel
// (kProjWaves wave tiles of 1024 rows).
template <typename TQ, typename T, typename PT, int SK, typename TC = T>
__device__ __forceinline__ void stencil_sketch_body(const TQ* __restrict__ qs, const double* __restrict__ invr,
                                                    const Grid3& g, int64_t n, T* __restrict__ w, int do_sketch,
                                                    const SketchArgs& sk, PT* __restrict__ partials, int64_t blk,
                                                    T* __restrict__ lds) {
    constexpr int NW = kProjWaves;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double ir = invr ? invr[0] : 1.0;
    const bool vec = stencil_vec_ok(g, qs, w);
    T v[16];
    auto pass = [&](auto scale, auto o32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r0 = blk * (NW * kTile) + wave * kTile + 256 * e + 4 * lane;
            T c[4];
            stencil4<T, TQ, decltype(scale)::value, decltype(o32)::value, TC>(g, qs, ir, vec, r0, n, v + 4 * e, c);
            st4<T>(w, r0, n, vec, v + 4 * e);
        }
    };
    const bool o32 = (uint64_t)n * sizeof(TQ) < ((uint64_t)1 << 32);
    if (invr) {
        if (o32)
            pass(std::true_type{}, std::true_type{});
        else
            pass(std::true_type{}, std::false_type{});
    } else if (o32) {
        pass(std::false_type{}, std::true_type{});
    } else {
        pass(std::false_type{}, std::false_type{});
    }
    if (!do_sketch) return;
    if constexpr (SK == SK_IDENT) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r0 = blk * (NW * kTile) + wave * kTile + 256 * e + 4 * lane;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r0 + r < n) partials[r0 + r] = (PT)v[4 * e + r];
        }
    } else {
        PT acc[kKptMax];
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) acc[u] = PT(0);
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

// Gaussian sketch only.  For the stored column x (unscaled): t = A x, stored
// in t_out, and the block's sketch partials of both x and t from one
// generation of Theta's entries (the two sketches of an Arnoldi step, s'_i of
// q'_i and p_{i+1} of A q'_i, share every draw; the normalisation 1/r_ii is
// applied to both later, when it is known).  Same row mapping and summation
// order per vector as stencil_sketch_body.
// TAB: the entries come from the bf16 table (SK_TABLE), 8 rows per load;
// EXACT (with TAB): from the table of the entries in T (SK_TABX), 8 rows per
// 32- or 64-byte group.
// Segments per sketch row of the drawn dual sketch: with one row per thread,
// k < NT leaves NT - k lanes idle (k = 400 of 512: one SIMD in four half
// loaded; k = 200: half the waves idle).  Splitting each row's quads of the
// block into S segments gives k S (row, segment) tasks over ceil(k S / NT)
// rounds; S is the smallest count that keeps 95 % of the lanes busy (else the
// best up to kKptMax), and 1 when k already does.  Uniform over the grid.
__device__ __forceinline__ int dual_segments(int k, int nt) {
    if (k >= nt || 20 * k >= 19 * nt) return 1;
    int best = 1;
    int64_t bnum = k, bden = nt;   // busy lanes / lane slots of the best count so far
    for (int S = 2; S <= kKptMax; ++S) {
        const int64_t tasks = (int64_t)k * S, slots = (tasks + nt - 1) / nt * nt;
        if (slots / nt > kKptMax) break;
        if (20 * tasks >= 19 * slots) return S;
        if (tasks * bden > bnum * slots) {
            best = S;
            bnum = tasks;
            bden = slots;
        }
    }
    return best;
}

template <typename TQ, typename T, bool TAB = false, int DEPTH = kTabDepth, bool EXACT = false, typename TC = T>
__device__ __forceinline__ void stencil_dual_body(const TQ* __restrict__ xs, const Grid3& g, int64_t n,
                                                  T* __restrict__ t_out, const SketchArgs& sk,
                                                  T* __restrict__ part_x, T* __restrict__ part_t, int64_t blk,
                                                  T* __restrict__ lds) {
    constexpr int NW = kProjWaves, NT = NW * kWave, RB = NW * kTile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool vec = stencil_vec_ok(g, xs, t_out);
    auto pass = [&](auto o32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int local = wave * kTile + 256 * e + 4 * lane;
            const int64_t r0 = blk * RB + local;
            T tv[4], xv[4];
            stencil4<T, TQ, false, decltype(o32)::value, TC>(g, xs, 1.0, vec, r0, n, tv, xv);
            st4<T>(t_out, r0, n, vec, tv);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                lds[local + r] = xv[r];
                lds[RB + local + r] = tv[r];
            }
        }
    };
    if ((uint64_t)n * sizeof(TQ) < ((uint64_t)1 << 32))
        pass(std::true_type{});
    else
        pass(std::false_type{});
    __syncthreads();
    const int kpt = (sk.k + NT - 1) / NT;
    T ax[kKptMax], at[kKptMax];
#pragma unroll
    for (int u = 0; u < kKptMax; ++u) ax[u] = at[u] = T(0);
    const int64_t rem = n - blk * RB;
    if constexpr (TAB) {
        const int no = rem >= RB ? RB / 8 : (int)((rem + 7) / 8);
        const int64_t o0 = blk * (RB / 8);
        // per sketch row, the block's table groups with DEPTH loads in flight
#pragma unroll
        for (int u = 0; u < kKptMax; ++u) {
            const int j = threadIdx.x + NT * u;
            if (u < kpt && j < sk.k) {
                T sx = ax[u], st = at[u];
                for (int o = 0; o < no; o += DEPTH) {
                    using group_t = std::conditional_t<EXACT, TabxGroup<T>, tabw_t>;
                    group_t w[DEPTH];
#pragma unroll
                    for (int d = 0; d < DEPTH; ++d) {
                        if (o + d < no) {
                            if constexpr (EXACT)
                                w[d] = tabx_load(static_cast<const T*>(sk.tabx), sk.k, o0 + o + d, j);
                            else
                                w[d] = tab_load(sk.table, sk.k, o0 + o + d, j);
                        }
                    }
#pragma unroll
                    for (int d = 0; d < DEPTH; ++d) {
                        if (o + d < no) {
                            T z[8];
                            if constexpr (EXACT)
                                tabx_unpack(w[d], z);
                            else
                                tab_unpack<T>(w[d], z);
                            const T* x = lds + 8 * (o + d);
                            const T* tt = lds + RB + 8 * (o + d);
                            sx += z[0] * x[0] + z[1] * x[1] + z[2] * x[2] + z[3] * x[3];
                            sx += z[4] * x[4] + z[5] * x[5] + z[6] * x[6] + z[7] * x[7];
                            st += z[0] * tt[0] + z[1] * tt[1] + z[2] * tt[2] + z[3] * tt[3];
                            st += z[4] * tt[4] + z[5] * tt[5] + z[6] * tt[6] + z[7] * tt[7];
                        }
                    }
                }
                ax[u] = sx;
                at[u] = st;
            }
        }
    } else {
        const int nq = rem >= RB ? RB / 4 : (int)((rem + 3) / 4);
        const uint32_t q0 = (uint32_t)(blk * (RB / 4));
        const int S = dual_segments(sk.k, NT);
        if (S == 1) {
            for (int q = 0; q < nq; ++q) {
                const T x0 = lds[4 * q], x1 = lds[4 * q + 1], x2 = lds[4 * q + 2], x3 = lds[4 * q + 3];
                const T t0 = lds[RB + 4 * q], t1 = lds[RB + 4 * q + 1], t2 = lds[RB + 4 * q + 2],
                        t3 = lds[RB + 4 * q + 3];
#pragma unroll
                for (int u = 0; u < kKptMax; ++u) {
                    const int j = threadIdx.x + NT * u;
                    if (u < kpt && j < sk.k) {
                        T z[4];
                        gauss4(q0 + (uint32_t)q, (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z);
                        ax[u] += z[0] * x0 + z[1] * x1 + z[2] * x2 + z[3] * x3;
                        at[u] += z[0] * t0 + z[1] * t1 + z[2] * t2 + z[3] * t3;
                    }
                }
            }
        } else {
            // k < NT: task tau = s k + j sums row j over segment s of the block's
            // quads, so that the k S tasks keep every lane busy; then row j adds
            // its S segment sums in segment order
            const int ntask = sk.k * S;
#pragma unroll
            for (int u = 0; u < kKptMax; ++u) {
                const int tau = threadIdx.x + NT * u;
                if (tau < ntask) {
                    const int j = tau % sk.k, sg = tau / sk.k;
                    const int qa = (int)((int64_t)nq * sg / S), qb = (int)((int64_t)nq * (sg + 1) / S);
                    T sx = T(0), st = T(0);
                    for (int q = qa; q < qb; ++q) {
                        T z[4];
                        gauss4(q0 + (uint32_t)q, (uint32_t)j, sk.sid, sk.inst, sk.k0, sk.k1, z);
                        sx += z[0] * lds[4 * q] + z[1] * lds[4 * q + 1] + z[2] * lds[4 * q + 2] +
                              z[3] * lds[4 * q + 3];
                        st += z[0] * lds[RB + 4 * q] + z[1] * lds[RB + 4 * q + 1] + z[2] * lds[RB + 4 * q + 2] +
                              z[3] * lds[RB + 4 * q + 3];
                    }
                    ax[u] = sx;
                    at[u] = st;
                }
            }
            __syncthreads();   // every task has read x and t: their LDS takes the segment sums
#pragma unroll
            for (int u = 0; u < kKptMax; ++u) {
                const int tau = threadIdx.x + NT * u;
                if (tau < ntask) {
                    lds[tau] = ax[u];
                    lds[RB + tau] = at[u];
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kKptMax; ++u) ax[u] = at[u] = T(0);
            const int j = threadIdx.x;   // kpt == 1
            if (j < sk.k) {
                T sx = lds[j], st = lds[RB + j];
                for (int sg = 1; sg < S; ++sg) {
                    sx += lds[sg * sk.k + j];
                    st += lds[RB + sg * sk.k + j];
                }
                ax[0] = sx;
                at[0] = st;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kKptMax; ++u) {
        const int j = threadIdx.x + NT * u;
        if (u < kpt && j < sk.k) {
            part_x[blk * sk.k + j] = ax[u];
            part_t[blk * sk.k + j] = at[u];
        }
    }
}

// P-SRHT / Rademacher counterpart of stencil_dual_body (the lagged Arnoldi
// step, RGS_FLAG_LAG): for the stored column x (unscaled q'_i), t = A x is
// stored in t_out, and the block's sketch partials of x and of t are taken in
// the same pass by two applications of the block sketch (the block transform
// of the projection kernel) -- so the two sketches of the step, s'_i of q'_i
// and p_{i+1} of A q'_i, come out of one reduction, r_ii and the 1/r_ii of
// p_{i+1} and w_{i+1} being applied when known.  Rows and their order per
// vector as in stencil_sketch_body.
template <typename TQ, typename T, int SK, typename TC = T>
__device__ __forceinline__ void stencil_dual_sk_body(const TQ* __restrict__ xs, const Grid3& g, int64_t n,
                                                     T* __restrict__ t_out, const SketchArgs& sk,
                                                     T* __restrict__ part_x, T* __restrict__ part_t, int64_t blk,
                                                     T* __restrict__ lds) {
    constexpr int NW = kProjWaves, NT = NW * kWave;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool vec = stencil_vec_ok(g, xs, t_out);
    T xv[16], tv[16];
    auto pass = [&](auto o32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r0 = blk * (NW * kTile) + wave * kTile + 256 * e + 4 * lane;
            stencil4<T, TQ, false, decltype(o32)::value, TC>(g, xs, 1.0, vec, r0, n, tv + 4 * e, xv + 4 * e);
            st4<T>(t_out, r0, n, vec, tv + 4 * e);
        }
    };
    if ((uint64_t)n * sizeof(TQ) < ((uint64_t)1 << 32))
        pass(std::true_type{});
    else
        pass(std::false_type{});
    T ax[kKptMax], at[kKptMax];
#pragma unroll
    for (int u = 0; u < kKptMax; ++u) ax[u] = at[u] = T(0);
    block_sketch<T, T, SK, NW>(xv, blk, n, sk, ax, lds);   // transforms xv, tv in place
    block_sketch<T, T, SK, NW>(tv, blk, n, sk, at, lds);
    const int kpt = (sk.k + NT - 1) / NT;
#pragma unroll
    for (int u = 0; u < kKptMax; ++u) {
        const int j = threadIdx.x + NT * u;
        if (u < kpt && j < sk.k) {
            part_x[blk * sk.k + j] = ax[u];
            part_t[blk * sk.k + j] = at[u];
        }
    }
}

// r = b - A x in fp64 for the 256 rows of block blk (256 threads), and the
// block's partial sum of ||r||^2.
__device__ __forceinline__ void residual_body(const double* __restrict__ b, const double* __restrict__ x,
                                              const Grid3& g, int64_t n, double* __restrict__ r,
                                              double* __restrict__ part, int64_t blk) {
    __shared__ double red[256];
    const int64_t l = blk * 256 + threadIdx.x;
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
    if (threadIdx.x == 0) part[blk] = red[0];
}

// out[0] = sqrt(sum of G partials), fixed order (one workgroup of 256).
__device__ __forceinline__ void norm_finish_body(const double* __restrict__ part, int64_t G,
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

// One Givens step for Hessenberg column c-1 (0-based basis column c >= 1):
// h = R(0:c, c) (RGS R column, h_c = r_cc), apply the c-1 previous rotations,
// form rotation c-1 that zeroes h_c, update g; record |g_c| / ||b|| in the
// history and stop the cycle when it is <= tol, at a lucky breakdown
// (status[0] = breakdown at column c: h_c = 0) or once c reaches `limit`.
// Called by every thread of one wave: the column is loaded into LDS (hs, at
// least c + 1 doubles) in parallel, one thread runs the chain of rotations
// with the running entry in a register and the rotations read 16 at a time,
// and the rotated column is written back in parallel.
__device__ __forceinline__ void givens_body(int c, const double* __restrict__ R, int mcap,
                                            double* __restrict__ Hr, double* __restrict__ cs,
                                            double* __restrict__ sn, double* __restrict__ gv, double bnorm,
                                            double tol, double* __restrict__ hist, int* __restrict__ status,
                                            int* __restrict__ used, int limit, double* __restrict__ hs) {
    __shared__ int mode;   // 0: skip, 1: normal step, 2: lucky breakdown
    if (threadIdx.x == 0) {
        int md = 1;
        if (status[2] != 0) {
            md = 0;
        } else if (status[0] != 0) {
            // w_c numerically in span(Q_c): exact Krylov space reached; otherwise non-finite data
            md = (status[0] == kStatusBreakdown && status[1] == c) ? 2 : 0;
        }
        mode = md;
    }
    __syncthreads();
    if (mode == 0) return;
    const bool lucky = mode == 2;
    for (int t = threadIdx.x; t <= c; t += blockDim.x)
        hs[t] = (t == c && lucky) ? 0.0 : R[t + (int64_t)c * mcap];
    __syncthreads();
    if (threadIdx.x == 0) {
        double cur = hs[0];   // entry t of the column, already rotated by rotations < t
        for (int t0 = 0; t0 < c - 1; t0 += 16) {
            double cv[16], sv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                cv[u] = (t0 + u < c - 1) ? cs[t0 + u] : 0.0;
                sv[u] = (t0 + u < c - 1) ? sn[t0 + u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int t = t0 + u;
                if (t < c - 1) {
                    const double a = cur, bb = hs[t + 1];
                    hs[t] = cv[u] * a + sv[u] * bb;
                    cur = -sv[u] * a + cv[u] * bb;
                }
            }
        }
        const double a = cur, bb = hs[c];
        double co = 1.0, si = 0.0, rho = a;
        if (bb != 0.0) {
            rho = hypot(a, bb);
            co = a / rho;
            si = bb / rho;
        }
        cs[c - 1] = co;
        sn[c - 1] = si;
        hs[c - 1] = rho;
        hs[c] = 0.0;
        gv[c] = -si * gv[c - 1];
        gv[c - 1] = co * gv[c - 1];
        const double est = fabs(gv[c]) / bnorm;
        hist[c - 1] = est;
        used[0] = c;
        if (lucky) status[0] = 0;       // a lucky breakdown is not an error in GMRES
        if (lucky || est <= tol || c >= limit) status[2] = 1;
    }
    __syncthreads();
    double* h = Hr + (int64_t)(c - 1) * mcap;   // rotated column c-1 of H
    for (int t = threadIdx.x; t <= c; t += blockDim.x) h[t] = hs[t];
}

// y = Hr(0:u, 0:u)^{-1} g(0:u), u = used[0]: back substitution (one thread).
// With an unnormalised stored basis (invr given) y_c is then scaled by 1/r_cc
// so that x += sum_c qs_c y_c.
__device__ __forceinline__ void backsub_body(const double* __restrict__ Hr, int mcap, const double* __restrict__ gv,
                                             const int* __restrict__ used, double* __restrict__ y,
                                             const double* __restrict__ invr) {
    const int u = used[0];
    for (int r = u - 1; r >= 0; --r) {
        double acc = gv[r];
        for (int c = r + 1; c < u; ++c) acc -= Hr[r + (int64_t)c * mcap] * y[c];
        y[r] = acc / Hr[r + (int64_t)r * mcap];
    }
    if (invr)
        for (int r = 0; r < u; ++r) y[r] = y[r] * invr[r];
}

// x_l += sum_{c < u} Q(l, c) y_c in fp64, columns in ascending order.
template <typename TQ>
__device__ __forceinline__ void xupdate_body(double* __restrict__ x, const TQ* __restrict__ Q, int64_t ldq,
                                             int64_t n, const int* __restrict__ used, const double* __restrict__ y,
                                             int64_t l) {
    if (l >= n) return;
    const int u = used[0];
    double acc = x[l];
    for (int c = 0; c < u; ++c) acc += to_double(Q[l + (int64_t)c * ldq]) * y[c];
    x[l] = acc;
}

}  // namespace

// ---------------------------------------------------------------------------
// Single-system kernels
// ---------------------------------------------------------------------------
// (fp32: at most 80 registers, 6 waves per SIMD: 28.3 instead of 30.6 us per
// launch at 192^3; the dual kernels are faster without the cap, and fp64 blocks
// are held to fewer waves by their LDS anyway)
template <typename TQ, typename T, typename PT, int SK, typename TC = T>
__global__ __launch_bounds__(kProjWaves * kWave, sizeof(T) == 4 ? 6 : 1) void k_stencil_sketch(
    const TQ* __restrict__ qs, const double* __restrict__ invr, Grid3 g, int64_t n, T* __restrict__ w,
    int do_sketch, SketchArgs sk, PT* __restrict__ partials, const int* __restrict__ status) {
    __shared__ T lds[kProjWaves * kTile];
    RGS_EXIT_IF_STOPPED(status);
    stencil_sketch_body<TQ, T, PT, SK, TC>(qs, invr, g, n, w, do_sketch, sk, partials,
                                           xcd_block(blockIdx.x, gridDim.x), lds);
}

template <typename TQ, typename T, bool TAB, bool EXACT = false, typename TC = T>
__global__ __launch_bounds__(kProjWaves * kWave) void k_stencil_dual(
    const TQ* __restrict__ xs, Grid3 g, int64_t n, T* __restrict__ t_out, SketchArgs sk, T* __restrict__ part_x,
    T* __restrict__ part_t, const int* __restrict__ status) {
    __shared__ T lds[2 * kProjWaves * kTile];
    RGS_EXIT_IF_STOPPED(status);
    // one system: k <= 512 threads stream the table with 4 loads in flight
    // (16 measured slower here; the batched row-block launch uses 16)
    // (the exact table: 256 bytes in flight per thread)
    stencil_dual_body<TQ, T, TAB, EXACT ? tabx_depth<T>() : 4, EXACT, TC>(xs, g, n, t_out, sk, part_x, part_t,
                                                                        xcd_block(blockIdx.x, gridDim.x), lds);
}

template <typename TQ, typename T, int SK, typename TC = T>
__global__ __launch_bounds__(kProjWaves * kWave) void k_stencil_dual_sk(
    const TQ* __restrict__ xs, Grid3 g, int64_t n, T* __restrict__ t_out, SketchArgs sk, T* __restrict__ part_x,
    T* __restrict__ part_t, const int* __restrict__ status) {
    __shared__ T lds[kProjWaves * kTile];
    RGS_EXIT_IF_STOPPED(status);
    stencil_dual_sk_body<TQ, T, SK, TC>(xs, g, n, t_out, sk, part_x, part_t, xcd_block(blockIdx.x, gridDim.x), lds);
}

__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ b, const double* __restrict__ x,
                                                  Grid3 g, int64_t n, double* __restrict__ r,
                                                  double* __restrict__ part) {
    residual_body(b, x, g, n, r, part, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_norm_finish(const double* __restrict__ part, int64_t G,
                                                     double* __restrict__ out) {
    norm_finish_body(part, G, out);
}

template <typename T>
__global__ void k_cast(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n) dst[l] = (T)src[l];
}

__global__ __launch_bounds__(64) void k_givens(int c, const double* __restrict__ R, int mcap,
                                               double* __restrict__ Hr, double* __restrict__ cs,
                                               double* __restrict__ sn, double* __restrict__ gv, double bnorm,
                                               double tol, double* __restrict__ hist, int* __restrict__ status,
                                               int* __restrict__ used, int limit) {
    extern __shared__ double hs_dyn[];
    givens_body(c, R, mcap, Hr, cs, sn, gv, bnorm, tol, hist, status, used, limit, hs_dyn);
}

// g(0) = r_11 = R(0, 0) at the start of a cycle.
__global__ void k_givens_init(const double* __restrict__ R, double* __restrict__ gv, int* __restrict__ used) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        gv[0] = R[0];
        used[0] = 0;
    }
}

__global__ void k_backsub(const double* __restrict__ Hr, int mcap, const double* __restrict__ gv,
                          const int* __restrict__ used, double* __restrict__ y, const double* __restrict__ invr) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    backsub_body(Hr, mcap, gv, used, y, invr);
}

template <typename TQ>
__global__ __launch_bounds__(256) void k_xupdate(double* __restrict__ x, const TQ* __restrict__ Q, int64_t ldq,
                                                 int64_t n, const int* __restrict__ used,
                                                 const double* __restrict__ y) {
    xupdate_body<TQ>(x, Q, ldq, n, used, y, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Batched kernels: workgroup -> (system, local block) through map.
// ---------------------------------------------------------------------------

// Start of a cycle: clear the status word (a kernel, not a memset, so that the
// cycle can be captured in a graph).
__global__ void kg_reset(const BatchItem* __restrict__ items, BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    if (threadIdx.x < 3) items[bm.x].sa.status[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void kg_zero_x(const GmresItem* __restrict__ gi, BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    const GmresItem& g = gi[bm.x];
    const int64_t l = (int64_t)bm.y * 256 + threadIdx.x;
    if (l < g.n) g.x[l] = 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void kg_cast(const GmresItem* __restrict__ gi, BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    const GmresItem& g = gi[bm.x];
    const int64_t l = (int64_t)bm.y * 256 + threadIdx.x;
    if (l < g.n) static_cast<T*>(g.w)[l] = (T)g.r[l];
}

// TC: the arithmetic of the product with A (T, or fp64 from the float32 basis
// vector in the unique-precision model)
template <typename TQ, typename T, int SK, typename TC = T>
__global__ __launch_bounds__(kProjWaves * kWave) void kg_stencil(const BatchItem* __restrict__ items,
                                                                 const GmresItem* __restrict__ gi,
                                                                 BlockMap map, int i) {
    __shared__ T lds[proj_lds_size<T, SK>()];
    const int2 bm = locate(map, xcd_block(blockIdx.x, gridDim.x));
    const BatchItem& it = items[bm.x];
    RGS_EXIT_IF_STOPPED(it.sa.status);
    const GmresItem& g = gi[bm.x];
    stencil_sketch_body<TQ, T, T, SK, TC>(static_cast<const TQ*>(it.Q) + (int64_t)(i - 1) * it.ldq,
                                      it.sa.invr + (i - 1), grid3(g.A), it.n, static_cast<T*>(g.w), 1, it.sk,
                                      static_cast<T*>(it.part), bm.y, lds);
}

template <typename TQ, typename T, bool TAB, typename TC = T>
__global__ __launch_bounds__(kProjWaves * kWave) void kg_stencil_dual(const BatchItem* __restrict__ items,
                                                                      const GmresItem* __restrict__ gi,
                                                                      BlockMap map, int i) {
    __shared__ T lds[2 * kProjWaves * kTile];
    const int2 bm = locate(map, xcd_block(blockIdx.x, gridDim.x));
    const BatchItem& it = items[bm.x];
    RGS_EXIT_IF_STOPPED(it.sa.status);
    const GmresItem& g = gi[bm.x];
    stencil_dual_body<TQ, T, TAB, kTabDepth, false, TC>(static_cast<const TQ*>(it.Q) + (int64_t)i * it.ldq,
                                                        grid3(g.A), it.n,
                             static_cast<T*>(g.w), it.sk, static_cast<T*>(it.part), static_cast<T*>(it.part2), bm.y,
                             lds);
}

// The lagged P-SRHT step (RGS_FLAG_LAG): t = A q'_i and the block partials of
// both sketches, the body of k_stencil_dual_sk.
template <typename TQ, typename T, typename TC = T>
__global__ __launch_bounds__(kProjWaves * kWave) void kg_stencil_dual_sk(const BatchItem* __restrict__ items,
                                                                         const GmresItem* __restrict__ gi,
                                                                         BlockMap map, int i) {
    __shared__ T lds[kProjWaves * kTile];
    const int2 bm = locate(map, xcd_block(blockIdx.x, gridDim.x));
    const BatchItem& it = items[bm.x];
    RGS_EXIT_IF_STOPPED(it.sa.status);
    const GmresItem& g = gi[bm.x];
    stencil_dual_sk_body<TQ, T, SK_SRHT, TC>(static_cast<const TQ*>(it.Q) + (int64_t)i * it.ldq, grid3(g.A), it.n,
                                         static_cast<T*>(g.w), it.sk, static_cast<T*>(it.part),
                                         static_cast<T*>(it.part2), bm.y, lds);
}

// The bf16-table variant with the L2 in mind: workgroup b -> (row block r,
// system) from a host-built list.  The table's entries do not depend on the
// system, so every system with a row block r reads the same k x kProjRows
// slice of it; the list gives the pairs of row block r to the workgroups that
// the round-robin dispatch sends to XCD r mod 8, in r order, so the workgroups
// resident on one XCD share one slice, which its L2 then serves after one read
// from HBM.  An entry with r < 0 is an idle slot.  Same body per (system,
// block) as kg_stencil_dual, so the same bits.
template <typename TQ, typename T, typename TC = T>
__global__ __launch_bounds__(kProjWaves * kWave) void kg_stencil_dual_rows(const BatchItem* __restrict__ items,
                                                                           const GmresItem* __restrict__ gi,
                                                                           const int2* __restrict__ pairs, int i) {
    __shared__ T lds[2 * kProjWaves * kTile];
    const int2 p = pairs[blockIdx.x];   // (row block, system)
    if (p.x < 0) return;
    const BatchItem& it = items[p.y];
    RGS_EXIT_IF_STOPPED(it.sa.status);
    const GmresItem& g = gi[p.y];
    stencil_dual_body<TQ, T, true, kTabDepth, false, TC>(static_cast<const TQ*>(it.Q) + (int64_t)i * it.ldq,
                                                         grid3(g.A), it.n,
                                   static_cast<T*>(g.w), it.sk, static_cast<T*>(it.part), static_cast<T*>(it.part2),
                                   p.x, lds);
}

// The projection of the fused-sketch Gaussian step: w_i = (A q'_{i-1}) / r_{i-1,i-1}
// scaled on load, no sketch (taken by kg_stencil_dual afterwards).
template <typename T, typename TQ, bool DEFER>
__global__ __launch_bounds__(kProjWaves * kWave) void kg_project_ws(const BatchItem* __restrict__ items,
                                                                    const GmresItem* __restrict__ gi,
                                                                    BlockMap map, int i) {
    __shared__ T lds[kProjWaves * kTile];
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    RGS_EXIT_IF_STOPPED(it.sa.status);
    const GmresItem& g = gi[bm.x];
    SketchArgs none{};
    project_body<T, TQ, T, SK_GAUSS, DEFER, true>(static_cast<const T*>(g.w), static_cast<TQ*>(it.Q), it.ldq, it.n,
                                                  i, static_cast<const T*>(it.coef),
                                                  i > 0 ? it.sa.invr + (i - 1) : nullptr, (!DEFER && i > 0) ? 1 : 0,
                                                  0, it.vec_ok, none, nullptr, bm.y, lds,
                                                  i > 0 ? it.sa.invr + (i - 1) : nullptr);
}

template <typename T, typename TQ, int SK, bool DEFER>
__global__ __launch_bounds__(kProjWaves * kWave) void kg_project(const BatchItem* __restrict__ items,
                                                                 const GmresItem* __restrict__ gi,
                                                                 BlockMap map, int i) {
    __shared__ T lds[kProjWaves * kTile];
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    RGS_EXIT_IF_STOPPED(it.sa.status);
    const GmresItem& g = gi[bm.x];
    project_body<T, TQ, T, SK, DEFER>(static_cast<const T*>(g.w), static_cast<TQ*>(it.Q), it.ldq, it.n, i,
                                      static_cast<const T*>(it.coef), i > 0 ? it.sa.invr + (i - 1) : nullptr,
                                      (!DEFER && i > 0) ? 1 : 0, 1, it.vec_ok, it.sk, static_cast<T*>(it.part),
                                      bm.y, lds);
}

// Step 2 for the Arnoldi right-hand side p_i (block partials of the mat-vec
// kernel): reduce to pbuf with the per-slice partials of Wm^T p, then the head
// of U^T p, then y = R_S^{-1} uh -> R(0:i, i) and the projection coefficients.
// TS: the sketch-space arithmetic (fp64, or float32 in the unique-precision model)
template <typename PT, typename TS = double>
__global__ __launch_bounds__(kGWB) void kg_lsa(const BatchItem* __restrict__ items, BlockMap map,
                                              int i, int dual) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    // dual: p_i arrives as the sketch of A q'_{i-1} (part2), scaled by 1/r_{i-1,i-1} here
    qa_body<PT, kGWB, TS>(static_cast<const PT*>(dual ? it.part2 : it.part), it.nproj, it.sketch_scale, nullptr, a.k,
                          i, ws_as<TS>(a.Wr), a.mcap, ws_as<TS>(a.pbuf), ws_as<TS>(a.pd), bm.y,
                          dual ? a.invr + (i - 1) : nullptr);
}

template <typename TS = double>
__global__ __launch_bounds__(kGWB) void kg_ls2(const BatchItem* __restrict__ items, BlockMap map,
                                              int i) {
    extern __shared__ double cp[];  // [i + 1]
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    ls2_body<kGWB, TS>(ws_as<TS>(a.pbuf), a.k, i, it.nsl, ws_as<TS>(a.Vc), a.mcap, ws_as<TS>(a.pd), ws_as<TS>(a.uh),
                       ws_as<TS>(a.pnorm), bm.y, ws_as<TS>(cp));
}

template <typename T, typename TS = double>
__global__ __launch_bounds__(kGWB) void kg_ls3(const BatchItem* __restrict__ items, BlockMap map,
                                              int i) {
    extern __shared__ double us[];  // [i]
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    ls3_body<T, kGWB, TS>(i, i, ws_as<TS>(a.X), a.mcap, ws_as<TS>(a.uh), it.R, it.ldr, static_cast<T*>(it.coef),
                          it.defer ? a.invr : nullptr, bm.y, ws_as<TS>(us));
}

// Step 2 by Richardson sweeps on the normal equations (ls_sweeps > 0; the
// bodies and workgroup size of the single-system kernels, so a batched solve
// keeps the bits of separate ones): the reduction of kg_lsa into the slice
// partials of S^T p and ||p||^2 (stride mcap + 2), ...
template <typename PT>
__global__ __launch_bounds__(kGW) void kg_lsr(const BatchItem* __restrict__ items, BlockMap map, int i, int dual) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    qa_body<PT, kGW>(static_cast<const PT*>(dual ? it.part2 : it.part), it.nproj, it.sketch_scale, nullptr, a.k, i,
                     a.Wr, a.mcap, a.pbuf, a.pdb, bm.y, dual ? a.invr + (i - 1) : nullptr, a.mcap + 2);
}

// ... the sums of a sweep (y, R(0:i+1, i+1) and the coefficients after the last) ...
template <typename T>
__global__ __launch_bounds__(kGW) void kg_rsum(const BatchItem* __restrict__ items, BlockMap map, int i,
                                              int accumulate, int last) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    rsum_body<T>(i, it.nsl, a.mcap, a.pdb, a.uh, accumulate, last, a.pnorm, it.R, it.ldr, static_cast<T*>(it.coef),
                 it.defer ? a.invr : nullptr, bm.y);
}

// ... the residual partials of one more sweep ...
__global__ __launch_bounds__(kGW) void kg_rres(const BatchItem* __restrict__ items, BlockMap map, int i) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    rres_body(a.k, i, a.mcap, it.S, it.lds, a.Wr, a.pbuf, a.uh, a.pdb, bm.y);
}

// ... and the column step: s' and the slice partials of ||s'||^2, then r_ii,
// s_i (both layouts) and the breakdown test.
template <typename PT>
__global__ __launch_bounds__(kGW) void kg_rqa(const BatchItem* __restrict__ items, BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    qa_body<PT, kGW>(static_cast<const PT*>(it.part), it.npart, it.sketch_scale, nullptr, a.k, 0, a.Wr, a.mcap, a.sp,
                     a.pd, bm.y);
}

__global__ __launch_bounds__(kGW) void kg_rb(const BatchItem* __restrict__ items, BlockMap map, int i) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const SpaceArgs& a = it.sa;
    rb_body(a.k, i, it.nsl, a.sp, a.pd, a.mcap, it.S, it.lds, a.Wr, it.R, it.ldr, a.rr, a.invr, a.pnorm, a.status,
            nullptr, a.pdb, bm.y);
}

__global__ void kg_givens_init(const BatchItem* __restrict__ items, const GmresItem* __restrict__ gi,
                               BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    if (threadIdx.x != 0) return;
    const GmresItem& g = gi[bm.x];
    g.gv[0] = items[bm.x].R[0];
    g.used[0] = 0;
}

__global__ __launch_bounds__(64) void kg_givens(const BatchItem* __restrict__ items, const GmresItem* __restrict__ gi,
                                                BlockMap map, int c) {
    extern __shared__ double hs_dyn[];
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const GmresItem& g = gi[bm.x];
    givens_body(c, it.R, it.sa.mcap, g.Hr, g.cs, g.sn, g.gv, g.bnorm, g.tol, g.hist, it.sa.status, g.used,
                g.limit[0], hs_dyn);
}

__global__ void kg_backsub(const BatchItem* __restrict__ items, const GmresItem* __restrict__ gi,
                           BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    if (threadIdx.x != 0) return;
    const BatchItem& it = items[bm.x];
    const GmresItem& g = gi[bm.x];
    backsub_body(g.Hr, it.sa.mcap, g.gv, g.used, g.y, it.defer ? it.sa.invr : nullptr);
}

template <typename TQ>
__global__ __launch_bounds__(256) void kg_xupdate(const BatchItem* __restrict__ items,
                                                  const GmresItem* __restrict__ gi, BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    const BatchItem& it = items[bm.x];
    const GmresItem& g = gi[bm.x];
    xupdate_body<TQ>(g.x, static_cast<const TQ*>(it.Q), it.ldq, g.n, g.used, g.y,
                     (int64_t)bm.y * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void kg_residual(const GmresItem* __restrict__ gi, BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    const GmresItem& g = gi[bm.x];
    residual_body(g.b, g.x, grid3(g.A), g.n, g.r, g.rpart, bm.y);
}

__global__ __launch_bounds__(256) void kg_norm_finish(const GmresItem* __restrict__ gi,
                                                      BlockMap map) {
    const int2 bm = locate(map, blockIdx.x);
    const GmresItem& g = gi[bm.x];
    norm_finish_body(g.rpart, (g.n + 255) / 256, g.norm);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define RGS_LAUNCH_CHECK()                                   \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return false;   \
    } while (0)

static inline unsigned nblk_of(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

template <typename TQ, typename T, typename TC>
bool launch_stencil_sketch(hipStream_t st, const StencilArgs& A, const TQ* qs, const double* invr, T* w,
                           int do_sketch, const SketchArgs& sk, T* partials, const int* status) {
    const int64_t n = A.nx * A.ny * A.nz;
    const Grid3 g = grid3(A);
    const dim3 grid(nblk_of(n, kProjRows)), thr(kProjWaves * kWave);
    if (sk.sketch == SK_SRHT)
        hipLaunchKernelGGL((k_stencil_sketch<TQ, T, T, SK_SRHT, TC>), grid, thr, 0, st, qs, invr, g, n, w, do_sketch,
                           sk, partials, status);
    else if (sk.sketch == SK_GAUSS)
        hipLaunchKernelGGL((k_stencil_sketch<TQ, T, T, SK_GAUSS, TC>), grid, thr, 0, st, qs, invr, g, n, w, do_sketch,
                           sk, partials, status);
    else if (sk.sketch == SK_RADEM)
        hipLaunchKernelGGL((k_stencil_sketch<TQ, T, T, SK_RADEM, TC>), grid, thr, 0, st, qs, invr, g, n, w, do_sketch,
                           sk, partials, status);
    else
        hipLaunchKernelGGL((k_stencil_sketch<TQ, T, T, SK_IDENT, TC>), grid, thr, 0, st, qs, invr, g, n, w, do_sketch,
                           sk, partials, status);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TQ, typename T, typename TC>
bool launch_stencil_dual(hipStream_t st, const StencilArgs& A, const TQ* xs, T* t_out, const SketchArgs& sk,
                         T* part_x, T* part_t, const int* status) {
    const int64_t n = A.nx * A.ny * A.nz;
    const dim3 grid(nblk_of(n, kProjRows)), thr(kProjWaves * kWave);
    if (sk.sketch == SK_TABX)
        hipLaunchKernelGGL((k_stencil_dual<TQ, T, true, true, TC>), grid, thr, 0, st, xs, grid3(A), n, t_out, sk, part_x,
                           part_t, status);
    else if (sk.sketch == SK_TABLE)
        hipLaunchKernelGGL((k_stencil_dual<TQ, T, true, false, TC>), grid, thr, 0, st, xs, grid3(A), n, t_out, sk, part_x, part_t,
                           status);
    else if (sk.sketch == SK_GAUSS)
        hipLaunchKernelGGL((k_stencil_dual<TQ, T, false, false, TC>), grid, thr, 0, st, xs, grid3(A), n, t_out, sk, part_x,
                           part_t, status);
    else if (sk.sketch == SK_SRHT)
        hipLaunchKernelGGL((k_stencil_dual_sk<TQ, T, SK_SRHT, TC>), grid, thr, 0, st, xs, grid3(A), n, t_out, sk, part_x,
                           part_t, status);
    else if (sk.sketch == SK_RADEM)
        hipLaunchKernelGGL((k_stencil_dual_sk<TQ, T, SK_RADEM, TC>), grid, thr, 0, st, xs, grid3(A), n, t_out, sk,
                           part_x, part_t, status);
    else
        return false;
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
                   double* gv, double bnorm, double tol, double* hist, int* status, int* used, int limit) {
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), (c + 1) * sizeof(double), st, c, R, mcap, Hr, cs, sn, gv,
                       bnorm, tol, hist, status, used, limit);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TQ>
bool launch_update_x(hipStream_t st, const double* Hr, int mcap, const double* gv, const int* used, double* y,
                     double* x, const TQ* Q, int64_t ldq, int64_t n, const double* invr) {
    hipLaunchKernelGGL(k_backsub, dim3(1), dim3(64), 0, st, Hr, mcap, gv, used, y, invr);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_xupdate<TQ>, dim3(nblk_of(n, 256)), dim3(256), 0, st, x, Q, ldq, n, used, y);
    RGS_LAUNCH_CHECK();
    return true;
}

// ---- batched ----
bool launch_gbatch_reset(hipStream_t st, const BatchItem* items, const BlockMap& map_sys, int64_t nsys) {
    if (nsys == 0) return true;
    hipLaunchKernelGGL(kg_reset, dim3(nsys), dim3(64), 0, st, items, map_sys);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_gbatch_zero_x(hipStream_t st, const GmresItem* gi, const BlockMap& map_row, int64_t nrow) {
    if (nrow == 0) return true;
    hipLaunchKernelGGL(kg_zero_x, dim3(nrow), dim3(256), 0, st, gi, map_row);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T>
bool launch_gbatch_cast(hipStream_t st, const GmresItem* gi, const BlockMap& map_row, int64_t nrow) {
    if (nrow == 0) return true;
    hipLaunchKernelGGL(kg_cast<T>, dim3(nrow), dim3(256), 0, st, gi, map_row);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T, typename TQ, typename TC>
bool launch_gbatch_stencil(hipStream_t st, int sketch, const BatchItem* items, const GmresItem* gi,
                           const BlockMap& map_proj, int64_t nproj, int i) {
    if (nproj == 0) return true;
    const dim3 thr(kProjWaves * kWave);
    if (sketch == SK_SRHT)
        hipLaunchKernelGGL((kg_stencil<TQ, T, SK_SRHT, TC>), dim3(nproj), thr, 0, st, items, gi, map_proj, i);
    else
        hipLaunchKernelGGL((kg_stencil<TQ, T, SK_GAUSS, TC>), dim3(nproj), thr, 0, st, items, gi, map_proj, i);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T, typename TQ, typename TC>
bool launch_gbatch_stencil_dual(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_proj,
                                int64_t nproj, int i, bool table, bool lag_srht) {
    if (nproj == 0) return true;
    if (lag_srht)
        hipLaunchKernelGGL((kg_stencil_dual_sk<TQ, T, TC>), dim3(nproj), dim3(kProjWaves * kWave), 0, st, items, gi,
                           map_proj, i);
    else if (table)
        hipLaunchKernelGGL((kg_stencil_dual<TQ, T, true, TC>), dim3(nproj), dim3(kProjWaves * kWave), 0, st, items,
                           gi, map_proj, i);
    else
        hipLaunchKernelGGL((kg_stencil_dual<TQ, T, false, TC>), dim3(nproj), dim3(kProjWaves * kWave), 0, st, items,
                           gi, map_proj, i);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T, typename TQ, typename TC>
bool launch_gbatch_stencil_dual_rows(hipStream_t st, const BatchItem* items, const GmresItem* gi, const int2* pairs,
                                     int64_t npairs, int i) {
    if (npairs == 0) return true;
    hipLaunchKernelGGL((kg_stencil_dual_rows<TQ, T, TC>), dim3(npairs), dim3(kProjWaves * kWave), 0, st, items, gi,
                       pairs, i);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T, typename TQ, bool DEFER>
bool launch_gbatch_project_ws(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_proj,
                              int64_t nproj, int i) {
    if (nproj == 0) return true;
    hipLaunchKernelGGL((kg_project_ws<T, TQ, DEFER>), dim3(nproj), dim3(kProjWaves * kWave), 0, st, items, gi,
                       map_proj, i);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T, typename TQ, bool DEFER>
bool launch_gbatch_project(hipStream_t st, int sketch, const BatchItem* items, const GmresItem* gi,
                           const BlockMap& map_proj, int64_t nproj, int i) {
    if (nproj == 0) return true;
    const dim3 thr(kProjWaves * kWave);
    if (sketch == SK_SRHT)
        hipLaunchKernelGGL((kg_project<T, TQ, SK_SRHT, DEFER>), dim3(nproj), thr, 0, st, items, gi, map_proj, i);
    else
        hipLaunchKernelGGL((kg_project<T, TQ, SK_GAUSS, DEFER>), dim3(nproj), thr, 0, st, items, gi, map_proj, i);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename T, typename TS>
bool launch_gbatch_ls(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t nsl, const BlockMap& map_rb,
                      int64_t nrb, int i, int dual) {
    if (nsl > 0) {
        hipLaunchKernelGGL((kg_lsa<T, TS>), dim3(nsl), dim3(kGWB), 0, st, items, map_sl, i, dual);
        RGS_LAUNCH_CHECK();
    }
    if (nrb > 0) {
        hipLaunchKernelGGL(kg_ls2<TS>, dim3(nrb), dim3(kGWB), (i + 1) * sizeof(double), st, items, map_rb, i);
        RGS_LAUNCH_CHECK();
        hipLaunchKernelGGL((kg_ls3<T, TS>), dim3(nrb), dim3(kGWB), (i + 1) * sizeof(double), st, items, map_rb, i);
        RGS_LAUNCH_CHECK();
    }
    return true;
}

static_assert(kRsumCoefs == kGW, "a kg_rsum workgroup sums kGW coefficients");

template <typename T>
bool launch_gbatch_ls_richardson(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t nsl,
                                 const BlockMap& map_rs, int64_t nrs, int i, int dual, int sweeps) {
    if (nsl == 0) return true;
    if (i < 1 || sweeps < 1) return false;
    hipLaunchKernelGGL(kg_lsr<T>, dim3(nsl), dim3(kGW), 0, st, items, map_sl, i, dual);
    RGS_LAUNCH_CHECK();
    for (int sw = 0; sw < sweeps; ++sw) {
        const int last = sw + 1 == sweeps;
        hipLaunchKernelGGL(kg_rsum<T>, dim3(nrs), dim3(kGW), 0, st, items, map_rs, i - 1, sw > 0 ? 1 : 0, last);
        RGS_LAUNCH_CHECK();
        if (!last) {
            hipLaunchKernelGGL(kg_rres, dim3(nsl), dim3(kGW), 0, st, items, map_sl, i - 1);
            RGS_LAUNCH_CHECK();
        }
    }
    return true;
}

template <typename T>
bool launch_gbatch_column_richardson(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t nsl,
                                     int i) {
    if (nsl == 0) return true;
    hipLaunchKernelGGL(kg_rqa<T>, dim3(nsl), dim3(kGW), 0, st, items, map_sl);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(kg_rb, dim3(nsl), dim3(kGW), 0, st, items, map_sl, i);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_gbatch_givens_init(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_sys,
                               int64_t nsys) {
    if (nsys == 0) return true;
    hipLaunchKernelGGL(kg_givens_init, dim3(nsys), dim3(64), 0, st, items, gi, map_sys);
    RGS_LAUNCH_CHECK();
    return true;
}

bool launch_gbatch_givens(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_sys,
                          int64_t nsys, int c) {
    if (nsys == 0) return true;
    hipLaunchKernelGGL(kg_givens, dim3(nsys), dim3(64), (c + 1) * sizeof(double), st, items, gi, map_sys, c);
    RGS_LAUNCH_CHECK();
    return true;
}

template <typename TQ>
bool launch_gbatch_finish(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_sys,
                          int64_t nsys, const BlockMap& map_row, int64_t nrow) {
    if (nsys == 0) return true;
    hipLaunchKernelGGL(kg_backsub, dim3(nsys), dim3(64), 0, st, items, gi, map_sys);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(kg_xupdate<TQ>, dim3(nrow), dim3(256), 0, st, items, gi, map_row);
    RGS_LAUNCH_CHECK();
    return launch_gbatch_residual(st, gi, map_sys, nsys, map_row, nrow);
}

bool launch_gbatch_residual(hipStream_t st, const GmresItem* gi, const BlockMap& map_sys, int64_t nsys,
                            const BlockMap& map_row, int64_t nrow) {
    if (nsys == 0) return true;
    hipLaunchKernelGGL(kg_residual, dim3(nrow), dim3(256), 0, st, gi, map_row);
    RGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(kg_norm_finish, dim3(nsys), dim3(256), 0, st, gi, map_sys);
    RGS_LAUNCH_CHECK();
    return true;
}

template bool launch_stencil_sketch<float, float, float>(hipStream_t, const StencilArgs&, const float*,
                                                         const double*, float*, int, const SketchArgs&, float*,
                                                         const int*);
template bool launch_stencil_sketch<float, float, double>(hipStream_t, const StencilArgs&, const float*,
                                                          const double*, float*, int, const SketchArgs&, float*,
                                                          const int*);
template bool launch_stencil_sketch<double, double, double>(hipStream_t, const StencilArgs&, const double*,
                                                            const double*, double*, int, const SketchArgs&,
                                                            double*, const int*);
template bool launch_stencil_sketch<bf16, float, float>(hipStream_t, const StencilArgs&, const bf16*, const double*,
                                                        float*, int, const SketchArgs&, float*, const int*);
template bool launch_cast<float>(hipStream_t, const double*, float*, int64_t);
template bool launch_cast<double>(hipStream_t, const double*, double*, int64_t);
template bool launch_update_x<float>(hipStream_t, const double*, int, const double*, const int*, double*, double*,
                                     const float*, int64_t, int64_t, const double*);
template bool launch_update_x<double>(hipStream_t, const double*, int, const double*, const int*, double*,
                                      double*, const double*, int64_t, int64_t, const double*);
template bool launch_update_x<bf16>(hipStream_t, const double*, int, const double*, const int*, double*, double*,
                                    const bf16*, int64_t, int64_t, const double*);
template bool launch_gbatch_cast<float>(hipStream_t, const GmresItem*, const BlockMap&, int64_t);
template bool launch_gbatch_cast<double>(hipStream_t, const GmresItem*, const BlockMap&, int64_t);
template bool launch_gbatch_stencil<float, float>(hipStream_t, int, const BatchItem*, const GmresItem*, const BlockMap&, int64_t, int);
template bool launch_gbatch_stencil<float, float, double>(hipStream_t, int, const BatchItem*, const GmresItem*,
                                                          const BlockMap&, int64_t, int);
template bool launch_gbatch_stencil<double, double>(hipStream_t, int, const BatchItem*, const GmresItem*,
                                                    const BlockMap&, int64_t, int);
template bool launch_gbatch_stencil<float, bf16>(hipStream_t, int, const BatchItem*, const GmresItem*, const BlockMap&, int64_t, int);
template bool launch_gbatch_project<float, float, false>(hipStream_t, int, const BatchItem*, const GmresItem*,
                                                         const BlockMap&, int64_t, int);
template bool launch_gbatch_project<double, double, false>(hipStream_t, int, const BatchItem*, const GmresItem*,
                                                           const BlockMap&, int64_t, int);
template bool launch_gbatch_project<float, bf16, true>(hipStream_t, int, const BatchItem*, const GmresItem*,
                                                       const BlockMap&, int64_t, int);
template bool launch_gbatch_ls<float>(hipStream_t, const BatchItem*, const BlockMap&, int64_t, const BlockMap&, int64_t, int, int);
template bool launch_gbatch_ls<float, float>(hipStream_t, const BatchItem*, const BlockMap&, int64_t, const BlockMap&,
                                             int64_t, int, int);
template bool launch_gbatch_ls_richardson<float>(hipStream_t, const BatchItem*, const BlockMap&, int64_t,
                                                 const BlockMap&, int64_t, int, int, int);
template bool launch_gbatch_ls_richardson<double>(hipStream_t, const BatchItem*, const BlockMap&, int64_t,
                                                  const BlockMap&, int64_t, int, int, int);
template bool launch_gbatch_column_richardson<float>(hipStream_t, const BatchItem*, const BlockMap&, int64_t, int);
template bool launch_gbatch_column_richardson<double>(hipStream_t, const BatchItem*, const BlockMap&, int64_t, int);
template bool launch_gbatch_ls<double>(hipStream_t, const BatchItem*, const BlockMap&, int64_t, const BlockMap&, int64_t, int, int);
template bool launch_stencil_dual<float, float, float>(hipStream_t, const StencilArgs&, const float*, float*,
                                                       const SketchArgs&, float*, float*, const int*);
template bool launch_stencil_dual<float, float, double>(hipStream_t, const StencilArgs&, const float*, float*,
                                                        const SketchArgs&, float*, float*, const int*);
template bool launch_stencil_dual<double, double, double>(hipStream_t, const StencilArgs&, const double*, double*,
                                                          const SketchArgs&, double*, double*, const int*);
template bool launch_stencil_dual<bf16, float, float>(hipStream_t, const StencilArgs&, const bf16*, float*,
                                                      const SketchArgs&, float*, float*, const int*);
template bool launch_gbatch_stencil_dual<float, float>(hipStream_t, const BatchItem*, const GmresItem*, const BlockMap&, int64_t, int, bool, bool);
template bool launch_gbatch_stencil_dual<float, float, double>(hipStream_t, const BatchItem*, const GmresItem*,
                                                               const BlockMap&, int64_t, int, bool, bool);
template bool launch_gbatch_stencil_dual<double, double>(hipStream_t, const BatchItem*, const GmresItem*,
                                                         const BlockMap&, int64_t, int, bool, bool);
template bool launch_gbatch_stencil_dual<float, bf16>(hipStream_t, const BatchItem*, const GmresItem*, const BlockMap&, int64_t, int, bool, bool);
template bool launch_gbatch_stencil_dual_rows<float, float>(hipStream_t, const BatchItem*, const GmresItem*,
                                                            const int2*, int64_t, int);
template bool launch_gbatch_stencil_dual_rows<float, float, double>(hipStream_t, const BatchItem*, const GmresItem*,
                                                                    const int2*, int64_t, int);
template bool launch_gbatch_stencil_dual_rows<double, double>(hipStream_t, const BatchItem*, const GmresItem*,
                                                              const int2*, int64_t, int);
template bool launch_gbatch_stencil_dual_rows<float, bf16>(hipStream_t, const BatchItem*, const GmresItem*,
                                                           const int2*, int64_t, int);
template bool launch_gbatch_project_ws<float, float, false>(hipStream_t, const BatchItem*, const GmresItem*,
                                                            const BlockMap&, int64_t, int);
template bool launch_gbatch_project_ws<double, double, false>(hipStream_t, const BatchItem*, const GmresItem*,
                                                              const BlockMap&, int64_t, int);
template bool launch_gbatch_project_ws<float, bf16, true>(hipStream_t, const BatchItem*, const GmresItem*,
                                                          const BlockMap&, int64_t, int);
template bool launch_gbatch_finish<float>(hipStream_t, const BatchItem*, const GmresItem*, const BlockMap&, int64_t,
                                          const BlockMap&, int64_t);
template bool launch_gbatch_finish<double>(hipStream_t, const BatchItem*, const GmresItem*, const BlockMap&, int64_t,
                                           const BlockMap&, int64_t);
template bool launch_gbatch_finish<bf16>(hipStream_t, const BatchItem*, const GmresItem*, const BlockMap&, int64_t,
                                         const BlockMap&, int64_t);

}  // namespace rgs
