// Internal declarations shared by the kernels (rgs_kernels.hip, rgs_gmres.hip)
// and the host C ABI (rgs_api.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgs {

enum { SK_GAUSS = 0, SK_SRHT = 1, SK_IDENT = 2 };
enum { kStatusOk = 0, kStatusBreakdown = 1, kStatusNonfinite = 2 };

// Everything a kernel needs to regenerate Theta (k x n) on the fly.
struct SketchArgs {
    int sketch;             // SK_*
    int k;
    uint32_t k0, k1;        // Philox key (seed low / high word)
    uint32_t sid, inst;     // counter words 2 and 3
    const uint32_t* signs;  // SRHT: bit table of D
    const int* rows;        // SRHT: sampled rows of H_s
};

// The 7-point operator: (A u)_l = c[0] u_l + c[1] u_{x-1} + c[2] u_{x+1} + c[3] u_{y-1}
// + c[4] u_{y+1} + c[5] u_{z-1} + c[6] u_{z+1}, Dirichlet 0 outside the box.
struct StencilArgs {
    int64_t nx, ny, nz;
    double c[7];
};

// bfloat16 storage element of the basis (round to nearest even).
struct bf16 {
    uint16_t bits;
};

// Device pointers of the sketch-space state (all fp64).
struct SpaceArgs {
    int k, mcap;
    double *Vc, *Vr;        // reflectors, column-major (k x mcap) and row-major (k rows of mcap)
    double *Wc, *Wr;        // Wm = V T, same two layouts
    double* X;              // R_S^{-1}, mcap x mcap column-major
    double *sp, *u, *v;     // k-vectors: s', U^T s, current reflector
    double *uh;             // mcap: head of U^T p
    double *pd, *pd2;       // per-slice partial sums: nsl x (mcap+1), nsl
    double* pdb;            // per-slice partials for the next right-hand side: nsl x (mcap+2)
    double *rr, *invr, *pnorm, *tau, *beta;  // per-column scalars (mcap each)
    double* pbuf;           // k: sketch of the current Arnoldi vector
    int* status;            // [0] = kStatus*, [1] = failed column, [2] = cycle done
};

// One factorisation of a batched call, as the batched kernels see it.
struct BatchItem {
    int64_t n;
    int m, k, nproj, nsl;
    const void* W;
    int64_t ldw;
    void* Q;
    int64_t ldq;
    double* R;
    int64_t ldr;
    double* S;
    int64_t lds;
    double* P;            // k x m: sketches of the columns of W
    void* part;           // nproj x k block partials (working precision)
    void* coef;           // m coefficients of the projection (working precision)
    double sketch_scale;  // 1 / sqrt(k)
    int vec_ok, defer;
    SpaceArgs sa;
    SketchArgs sk;
};

// One system of a batched GMRES call, beside its BatchItem (the column-step
// view: basis, sketch-space state, R, S).
struct GmresItem {
    int64_t n;
    StencilArgs A;
    const double* b;
    double* x;
    double* r;            // n: restart residual b - A x (fp64)
    void* w;              // n: the current Arnoldi vector (working precision)
    double* rpart;        // per 256-row block partial sums of ||r||^2
    double* norm;         // [0] = ||r||
    double bnorm, tol;
    double *Hr, *cs, *sn, *gv, *y, *hist;   // Givens state (mcap each; gv mcap + 1)
    int* used;            // inner steps done in the current cycle
    const int* limit;     // inner steps allowed in the current cycle
};

bool launch_srht_signs(hipStream_t st, uint32_t* signs, int64_t nwords, const SketchArgs& sk);
template <typename T, typename PT>
bool launch_sketch_cols(hipStream_t st, const T* X, int64_t ldx, int64_t n, int ncols, int G,
                        const SketchArgs& sk, PT* partials);
template <typename PT>
bool launch_reduce(hipStream_t st, const PT* partials, int G, int k, int ncols, double scale, double* out,
                   int64_t ldo);
template <typename TW, typename TQ, bool DEFER>
bool launch_project(hipStream_t st, const TW* w, TQ* Q, int64_t ldq, int64_t n, int j, const TW* coef,
                    const double* invr, int normalize_last, int do_sketch, int vec_ok, const SketchArgs& sk,
                    TW* partials, const int* status);
template <typename T>
bool launch_scale_col(hipStream_t st, T* q, int64_t n, const double* invr, const int* status);
template <typename T>
bool launch_ls(hipStream_t st, const SpaceArgs& a, const double* p, int i, double* R, int64_t ldr, T* coef);
template <typename T, typename PT>
bool launch_column(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale,
                   const double* src, int i, double* S, int64_t lds, double* R, int64_t ldr,
                   const double* pnext, T* coef, const double* cscale);
bool launch_zero_mat(hipStream_t st, double* A, int64_t rows, int64_t cols, int64_t lda);
bool launch_scale_cols_bf16(hipStream_t st, bf16* Q, int64_t ldq, int64_t n, int m, const double* invr,
                            const int* status);
bool launch_batch_init(hipStream_t st, const BatchItem* items, int nitems, int64_t max_m2);
template <typename TW, typename TQ, bool DEFER>
bool launch_batch_project(hipStream_t st, int sketch, const BatchItem* items, const int2* map, int count, int i);
template <typename TW>
bool launch_batch_column(hipStream_t st, const BatchItem* items, const int2* map_sl, int n_sl, const int2* map_qd,
                         int n_qd, const int2* map_ls, int n_ls, int i);
template <typename TQ, bool DEFER>
bool launch_batch_scale(hipStream_t st, const BatchItem* items, const int2* map, int count);
template <typename T>
bool launch_materialize(hipStream_t st, const SketchArgs& sk, int64_t j0, int64_t j1, int64_t l0, int64_t l1,
                        double rsk, double* out, int64_t ldo);
bool launch_diagnostics(hipStream_t st, const double* P, int64_t ldp, const double* S, int64_t lds,
                        const double* R, int64_t ldr, int k, int m, double* gram_out, double* resid_out);

template <typename TQ, typename T>
bool launch_stencil_sketch(hipStream_t st, const StencilArgs& A, const TQ* qs, const double* invr, T* w,
                           int do_sketch, const SketchArgs& sk, T* partials, const int* status);
bool launch_residual(hipStream_t st, const StencilArgs& A, const double* b, const double* x, double* r,
                     double* part, double* norm_out);
template <typename T>
bool launch_cast(hipStream_t st, const double* src, T* dst, int64_t n);
bool launch_givens_init(hipStream_t st, const double* R, double* gv, int* used);
bool launch_givens(hipStream_t st, int c, const double* R, int mcap, double* Hr, double* cs, double* sn,
                   double* gv, double bnorm, double tol, double* hist, int* status, int* used, int limit);
template <typename TQ>
bool launch_update_x(hipStream_t st, const double* Hr, int mcap, const double* gv, const int* used, double* y,
                     double* x, const TQ* Q, int64_t ldq, int64_t n, const double* invr);
// Step 2 when the right-hand side arrives as block partials (Arnoldi): reduce to
// a.pbuf, then the least-squares solve of column i (R(0:i, i) and coef).
template <typename T, typename PT>
bool launch_ls_partials(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale, int i,
                        double* R, int64_t ldr, T* coef, const double* cscale);

// Batched GMRES: every launch covers the systems listed in its map
// (map_sys: one entry per system, map_row: 256-row blocks, map_proj: blocks
// of kProjRows rows, map_sl: 64-row sketch slices, map_rb: 64-row blocks of
// the i x i least-squares solve).
bool launch_gbatch_reset(hipStream_t st, const BatchItem* items, const int2* map_sys, int nsys);
bool launch_gbatch_zero_x(hipStream_t st, const GmresItem* gi, const int2* map_row, int nrow);
template <typename T>
bool launch_gbatch_cast(hipStream_t st, const GmresItem* gi, const int2* map_row, int nrow);
template <typename T, typename TQ>
bool launch_gbatch_stencil(hipStream_t st, int sketch, const BatchItem* items, const GmresItem* gi,
                           const int2* map_proj, int nproj, int i);
template <typename T, typename TQ, bool DEFER>
bool launch_gbatch_project(hipStream_t st, int sketch, const BatchItem* items, const GmresItem* gi,
                           const int2* map_proj, int nproj, int i);
template <typename T>
bool launch_gbatch_ls(hipStream_t st, const BatchItem* items, const int2* map_sl, int nsl, const int2* map_rb,
                      int nrb, int i);
bool launch_gbatch_givens_init(hipStream_t st, const BatchItem* items, const GmresItem* gi, const int2* map_sys,
                               int nsys);
bool launch_gbatch_givens(hipStream_t st, const BatchItem* items, const GmresItem* gi, const int2* map_sys,
                          int nsys, int c);
template <typename TQ>
bool launch_gbatch_finish(hipStream_t st, const BatchItem* items, const GmresItem* gi, const int2* map_sys,
                          int nsys, const int2* map_row, int nrow);
bool launch_gbatch_residual(hipStream_t st, const GmresItem* gi, const int2* map_sys, int nsys,
                            const int2* map_row, int nrow);

}  // namespace rgs
