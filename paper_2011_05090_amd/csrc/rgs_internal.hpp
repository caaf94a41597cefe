// Launchers of the device code (rgs_project.hip, rgs_kernels.hip, rgs_gmres.hip)
// called by the host C ABI (rgs_api.cpp).  Not part of the public interface.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rgs_types.hpp"

namespace rgs {

bool launch_srht_signs(hipStream_t st, uint32_t* signs, int64_t nwords, const SketchArgs& sk);
// The P-SRHT's k sampled rows of [0, s) drawn on the device (one workgroup),
// equal to the host draw; k <= kRowsDevMax, s <= 2^31.
constexpr int kRowsDevMax = 4096;
bool launch_srht_rows(hipStream_t st, int* rows, int64_t s, const SketchArgs& sk);
template <typename T, typename PT>
bool launch_sketch_cols(hipStream_t st, const T* X, int64_t ldx, int64_t n, int ncols, int G,
                        const SketchArgs& sk, PT* partials);
// Gaussian sketch partials of ncols columns (k_reduce layout, G row groups of
// 256-row sub-blocks), each entry of Theta generated once per kGaussCols columns.
constexpr int kGaussCols = 32;
constexpr int kGSubCol = 64;   // rows per sub-block of the single-column Gaussian sketch
// Gaussian (drawn or bf16 table) / Rademacher sketches of ncols columns: T the
// entry and staging type, TA the accumulation and partials type.
template <typename TX, typename T, typename TA = T>
bool launch_gauss_cols(hipStream_t st, const TX* X, int64_t ldx, int64_t n, int ncols, int G, const SketchArgs& sk,
                       TA* partials);
template <typename PT, typename TR = double>   // TR: arithmetic of the sums
bool launch_reduce(hipStream_t st, const PT* partials, int G, int k, int ncols, double scale, double* out,
                   int64_t ldo);
template <typename TW, typename TQ, bool DEFER>
bool launch_project(hipStream_t st, const TW* w, TQ* Q, int64_t ldq, int64_t n, int j, const TW* coef,
                    const double* invr, int normalize_last, int do_sketch, int vec_ok, const SketchArgs& sk,
                    TW* partials, const int* status);
// launch_project without a sketch, on small row blocks (small factorisations
// whose column sketch is launched separately).
template <typename TW, typename TQ, bool DEFER>
bool launch_project_rows(hipStream_t st, const TW* w, TQ* Q, int64_t ldq, int64_t n, int j, const TW* coef,
                         const double* invr, int normalize_last, const int* status);
// launch_project with w_i multiplied by wscale[0] on load and no sketch (the
// fused-sketch GMRES step).
template <typename TW, typename TQ, bool DEFER>
bool launch_project_ws(hipStream_t st, const TW* w, TQ* Q, int64_t ldq, int64_t n, int j, const TW* coef,
                       const double* invr, int normalize_last, int vec_ok, const double* wscale, const int* status);
template <typename T>
bool launch_scale_col(hipStream_t st, T* q, int64_t n, const double* invr, const int* status);
template <typename T>
bool launch_ls(hipStream_t st, const SpaceArgs& a, const double* p, int i, double* R, int64_t ldr, T* coef);
// Step 2 of an Arnoldi step (right-hand side from block partials) by `sweeps`
// Richardson iterations on the normal equations (with the Richardson column step).
template <typename T, typename PT>
bool launch_ls_partials_richardson(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale, int i,
                                   double* S, int64_t lds, double* R, int64_t ldr, T* coef, const double* cscale,
                                   const double* scale2, int sweeps);
// The column step with step 2 by `sweeps` Richardson iterations on the normal equations.
template <typename T, typename PT>
bool launch_column_richardson(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale,
                              const double* src, int i, double* S, int64_t lds, double* R, int64_t ldr,
                              const double* pnext, T* coef, const double* cscale, int sweeps);
// TS: arithmetic of the sketch-space state (fp64; float32 for the unique-precision model).
template <typename T, typename PT, typename TS = double>
bool launch_column(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale,
                   const double* src, int i, double* S, int64_t lds, double* R, int64_t ldr,
                   const double* pnext, T* coef, const double* cscale);
bool launch_zero_mat(hipStream_t st, double* A, int64_t rows, int64_t cols, int64_t lda);
bool launch_scale_cols_bf16(hipStream_t st, bf16* Q, int64_t ldq, int64_t n, int m, const double* invr, int vec,
                            const int* status);
bool launch_batch_init(hipStream_t st, const BatchItem* items, int nitems, int64_t max_m2);
template <typename T>
bool launch_batch_sketch_p(hipStream_t st, int sketch, const BatchItem* items, const BlockMap& map_signs,
                           int64_t n_signs, const BlockMap& map_part, int64_t n_part, const BlockMap& map_red,
                           int64_t n_red, bool acc64);
// Batched Gaussian sketch products with the shared master matrix, one
// workgroup per GemmUnit over the (item, column) list `cols` (tile: 32, 64 or 128
// columns per unit, as the units were built): STEP4, column i
// of Q (partials per `rows`-row chunk into part); otherwise columns of W
// (partials per chunk into partP, G_P chunks per column).
constexpr int kGemmRows = 2048;      // row chunk of the step-4 product
constexpr int kGemmRowsP = 16384;    // row chunk of the step-1 product
// tabx (RGS_FLAG_THETA_EXACT): the entries read from the exact fp32 table of
// the master matrix (tk rows, SK_TABX layout) instead of drawn, same bits.
template <typename TB, bool STEP4>
bool launch_batch_gauss_gemm(hipStream_t st, const BatchItem* items, const GemmUnit* units, int nunits,
                             const int2* cols, int rows, int tile, const float* tabx = nullptr, int tk = 0);
// The same products with the bf16 Gaussian entries read from the table
// (tk rows, tgroups groups of 8 columns, the k_theta_table layout) through
// bf16 MFMA; rows a multiple of 16.
template <typename TB, bool STEP4>
bool launch_batch_table_gemm(hipStream_t st, const BatchItem* items, const GemmUnit* units, int nunits,
                             const int2* cols, int rows, int tile, const uint16_t* table, int tk, int64_t tgroups);
template <typename TW, typename TQ, bool DEFER>
bool launch_batch_project(hipStream_t st, int sketch, const BatchItem* items, const BlockMap& map, int64_t nblk,
                          int i);
template <typename TW, typename TS = double>
bool launch_batch_column(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t n_sl,
                         const BlockMap& map_qd, int64_t n_qd, const BlockMap& map_ls, int64_t n_ls, int i);
// step 2 by `sweeps` Richardson sweeps: the column step of every factorisation in
// map_sl (its slices), the sweeps over those with a column i+1 (map_next: their
// slices; map_rs: their blocks of kRsumCoefs coefficients)
template <typename TW>
bool launch_batch_column_richardson(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t n_sl,
                                    const BlockMap& map_next, int64_t n_next, const BlockMap& map_rs, int64_t n_rs,
                                    int i, int sweeps);
template <typename TQ, bool DEFER>
bool launch_batch_scale(hipStream_t st, const BatchItem* items, const BlockMap& map, int64_t nblk);
template <typename T>
bool launch_materialize(hipStream_t st, const SketchArgs& sk, int64_t j0, int64_t j1, int64_t l0, int64_t l1,
                        double rsk, double* out, int64_t ldo);
bool launch_diagnostics(hipStream_t st, const double* P, int64_t ldp, const double* S, int64_t lds,
                        const double* R, int64_t ldr, int k, int m, double* gram_out, double* resid_out);
// Table of the Gaussian sketch with bf16 entries ((n + 7) / 8 * 8 * k entries, SK_TABLE layout).
bool launch_theta_table(hipStream_t st, const SketchArgs& sk, int64_t n, uint16_t* table);
// Table of the Gaussian sketch with its entries in T, exactly those the drawn
// sketch computes ((n + 7) / 8 * 8 * k entries, SK_TABX layout).
template <typename T>
bool launch_theta_tabx(hipStream_t st, const SketchArgs& sk, int64_t n, T* table);
// C = op(A) B in fp64 (op(A) = A^T when transA), the small products of the certification.
bool launch_dgemm(hipStream_t st, bool transA, int M, int N, int K, const double* A, int64_t lda, const double* B,
                  int64_t ldb, double* C, int64_t ldc);

// TC: the arithmetic of the product with A (T; fp64 for the configuration of
// Sec. 5.3, the result rounded once to T).
template <typename TQ, typename T, typename TC = T>
bool launch_stencil_sketch(hipStream_t st, const StencilArgs& A, const TQ* qs, const double* invr, T* w,
                           int do_sketch, const SketchArgs& sk, T* partials, const int* status);
// Gaussian, fused-sketch Arnoldi step: t = A xs and the block partials of both
// sketches (xs: part_x, t: part_t) from one generation of Theta.
template <typename TQ, typename T, typename TC = T>
bool launch_stencil_dual(hipStream_t st, const StencilArgs& A, const TQ* xs, T* t_out, const SketchArgs& sk,
                         T* part_x, T* part_t, const int* status);
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
// TS: the arithmetic of the sketch space (fp64; float32 for the unique-precision model).
template <typename T, typename PT, typename TS = double>
bool launch_ls_partials(hipStream_t st, const SpaceArgs& a, const PT* partials, int G, double scale, int i,
                        double* R, int64_t ldr, T* coef, const double* cscale, const double* scale2);

// Batched GMRES: every launch covers the systems listed in its map
// (map_sys: one entry per system, map_row: 256-row blocks, map_proj: blocks
// of kProjRows rows, map_sl: 64-row sketch slices, map_rb: 64-row blocks of
// the i x i least-squares solve).
bool launch_gbatch_reset(hipStream_t st, const BatchItem* items, const BlockMap& map_sys, int64_t nsys);
bool launch_gbatch_zero_x(hipStream_t st, const GmresItem* gi, const BlockMap& map_row, int64_t nrow);
template <typename T>
bool launch_gbatch_cast(hipStream_t st, const GmresItem* gi, const BlockMap& map_row, int64_t nrow);
template <typename T, typename TQ, typename TC = T>
bool launch_gbatch_stencil(hipStream_t st, int sketch, const BatchItem* items, const GmresItem* gi,
                           const BlockMap& map_proj, int64_t nproj, int i);
template <typename T, typename TQ, bool DEFER>
bool launch_gbatch_project(hipStream_t st, int sketch, const BatchItem* items, const GmresItem* gi,
                           const BlockMap& map_proj, int64_t nproj, int i);
template <typename T, typename TS = double>
bool launch_gbatch_ls(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t nsl, const BlockMap& map_rb,
                      int64_t nrb, int i, int dual);
// The same step, and the column step, with the least squares by `sweeps`
// Richardson iterations on the normal equations (map_rs: blocks of
// kRsumCoefs coefficients per system).
constexpr int kRsumCoefs = 1024;
template <typename T>
bool launch_gbatch_ls_richardson(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t nsl,
                                 const BlockMap& map_rs, int64_t nrs, int i, int dual, int sweeps);
template <typename T>
bool launch_gbatch_column_richardson(hipStream_t st, const BatchItem* items, const BlockMap& map_sl, int64_t nsl,
                                     int i);
template <typename T, typename TQ, typename TC = T>
// (lag_srht: the lagged P-SRHT step of RGS_FLAG_LAG instead of the Gaussian one)
bool launch_gbatch_stencil_dual(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_proj,
                                int64_t nproj, int i, bool table, bool lag_srht = false);
template <typename T, typename TQ, typename TC = T>
bool launch_gbatch_stencil_dual_rows(hipStream_t st, const BatchItem* items, const GmresItem* gi, const int2* pairs,
                                     int64_t npairs, int i);
template <typename T, typename TQ, bool DEFER>
bool launch_gbatch_project_ws(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_proj,
                              int64_t nproj, int i);
bool launch_gbatch_givens_init(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_sys,
                               int64_t nsys);
bool launch_gbatch_givens(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_sys,
                          int64_t nsys, int c);
template <typename TQ>
bool launch_gbatch_finish(hipStream_t st, const BatchItem* items, const GmresItem* gi, const BlockMap& map_sys,
                          int64_t nsys, const BlockMap& map_row, int64_t nrow);
bool launch_gbatch_residual(hipStream_t st, const GmresItem* gi, const BlockMap& map_sys, int64_t nsys,
                            const BlockMap& map_row, int64_t nrow);

}  // namespace rgs
