// Data structures shared by the device code and the host driver: sketch
// descriptors, the operator, the bf16 storage element and the per-system
// views of batched calls.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgs {

// SK_TABLE: the Gaussian sketch with bf16 entries, read from a table made by
// k_theta_table (entry (j, l) at ((l / 8) k + j) 8 + l % 8, unscaled).
// SK_TABX: the Gaussian sketch itself, its entries drawn once into a table of
// the working type T (float or double; same layout) by k_theta_tabx and read
// back by every application instead of being drawn again.
enum { SK_GAUSS = 0, SK_SRHT = 1, SK_IDENT = 2, SK_RADEM = 3, SK_TABLE = 4, SK_TABX = 5 };
enum { kStatusOk = 0, kStatusBreakdown = 1, kStatusNonfinite = 2 };

// Everything a kernel needs to regenerate Theta (k x n) on the fly.
struct SketchArgs {
    int sketch;             // SK_*
    int k;
    uint32_t k0, k1;        // Philox key (seed low / high word)
    uint32_t sid, inst;     // counter words 2 and 3
    const uint32_t* signs;  // SRHT: bit table of D
    const int* rows;        // SRHT: sampled rows of H_s
    const uint16_t* table;  // SK_TABLE: bf16 entries
    const void* tabx;       // SK_TABX: the entries in the working type
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
    int npart;            // block partials of step 4 reduced by the column step (nproj, or the
                          // 2048-row chunks of the batched Gaussian sketch product)
    const void* W;
    int64_t ldw;
    void* Q;
    int64_t ldq;
    double* R;
    int64_t ldr;
    double* S;
    int64_t lds;
    double* P;            // k x m: sketches of the columns of W
    void* partP;          // batched step 1: G_P x k x m block partials of P
    int G_P;              // row groups of step 1
    void* part;           // nproj x k block partials (working precision)
    void* part2;          // GMRES, Gaussian: block partials of the next Arnoldi vector's sketch
    void* coef;           // m coefficients of the projection (working precision)
    double sketch_scale;  // 1 / sqrt(k)
    int vec_ok, defer;
    int gemm_sketch;      // batched Gaussian: step 4 by the shared-Theta MFMA kernel, not in the projection
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

// Implicit launch map of a batched call: the grid is the concatenation of the
// block ranges of the listed items.  Listed position p owns blocks
// [first(p), first(p + 1)), first(p) = base[p] + uniform * p (base: prefix sums
// of per-item block counts, or none), and names item ids[p] (or item p).
struct BlockMap {
    const int64_t* base;
    const int* ids;
    int count;
    int uniform;
};

// One work unit of the batched Gaussian sketch product: the operand columns
// at positions [first, first + count) of the launch's (item, column) list (at
// most 64), row chunk blk, sketch rows [128 jt, 128 jt + 128).
struct GemmUnit {
    int first, count, blk, jt;
};

}  // namespace rgs
