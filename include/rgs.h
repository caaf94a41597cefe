/*
 * rgs.h -- C ABI of librgs: randomized Gram-Schmidt (RGS) and randomized
 * GMRES on one AMD Instinct MI355X (gfx950).
 *
 * Method: O. Balabanov, L. Grigori, "Randomized Gram-Schmidt process with
 * application to GMRES", arXiv:2011.05090.
 *   - RGS column step: Algorithm 2 (Sec. 2.3).
 *   - RGS-Arnoldi: Algorithm 3 (Sec. 4.1); randomized GMRES: Sec. 4.2.
 *   - Sketching operators (Gaussian, Rademacher, P-SRHT) and seeded generation: Sec. 2.1.
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major with an explicit leading dimension (in
 *     elements).  Vectors are contiguous.
 *   - Every array argument is DEVICE memory owned by the caller, unless the
 *     parameter comment says "host".  The library never frees caller memory;
 *     its own scratch lives in the handle and is grown on demand.
 *   - The element type of W, Q and X is fixed by the precision field:
 *       RGS_P_FP64       -> double
 *       RGS_P_FP32_LS64  -> float   (step 3 in fp32; sketches, least
 *                                    squares and normalisation in fp64)
 *       RGS_P_BF16Q_FP32_LS64 -> W and X float, Q bfloat16 (raw 16-bit
 *                                    words): the basis is stored in bf16,
 *                                    step 3 computes in fp32
 *     R, S, P, b, x and histories are always double.
 *   - Work is ordered on the handle's stream.  Calls that return a report
 *     synchronise that stream before returning.  Some calls also run part of
 *     their work on an auxiliary stream the handle creates (default
 *     priority): rgs_qr (step-1 chunks after the first), rgs_qr_batched and
 *     rgs_gmres_batched (the second half of the batch).  That work is forked
 *     from the handle's stream and joined back into it with events within
 *     the call, so the ordering on the handle's stream is unchanged.
 *   - Errors are negative rgs_status codes; nothing is thrown across the ABI
 *     (a host allocation failure inside a call returns RGS_ENOMEM).
 *     Argument errors are detected before any device work is enqueued.
 *   - A handle is not thread-safe: use one handle per host thread.
 */
#ifndef RGS_H
#define RGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RGS_ABI_VERSION 7

typedef struct rgs_handle rgs_handle;  /* opaque */
typedef void *rgs_stream;              /* a hipStream_t; NULL = the null stream */

typedef enum {
    RGS_OK = 0,
    RGS_EINVAL = -1,      /* bad argument (sizes, pointers, leading dims, enums) */
    RGS_ENOMEM = -2,      /* device scratch or host memory allocation failed */
    RGS_EDEVICE = -3,     /* a HIP runtime call or a kernel launch failed, or the
                             host runtime did (e.g. a worker thread could not start) */
    RGS_EBREAKDOWN = -4,  /* r_ii = 0 or r_ii <= 2^-50 ||p_i||: w_i numerically in
                             span(Q_{i-1}); columns before report.failed_column are valid */
    RGS_ENONFINITE = -5,  /* a sketch p_i or s'_i is not finite (NaN/Inf in the input) */
    RGS_ENOCONV = -6,     /* GMRES hit max_iters; x holds the last iterate */
    RGS_ESCRATCH = -7     /* rgs_qr_noalloc: the problem does not fit its fixed scratch */
} rgs_status;

typedef enum {
    RGS_SKETCH_GAUSSIAN = 0, /* entries N(0,1/k), Philox4x32-10 + Box-Muller, generated on the fly */
    RGS_SKETCH_SRHT = 1,     /* P-SRHT: k^-1/2 Rows H_s D on the zero-padded input */
    RGS_SKETCH_IDENTITY = 2, /* test sketch: k = n, Theta = I */
    RGS_SKETCH_RADEMACHER = 3 /* entries +-1/sqrt(k) (Sec. 2.1), generated on the fly: the signs of
                                 columns 128b..128b+127 of row j are the 128 bits of one Philox4x32-10
                                 call at counter (b, j, sketch_id, instance), bit l%32 of word
                                 (l%128)/32 set meaning -1.  rgs_qr, rgs_gmres, rgs_sketch_apply and
                                 rgs_sketch_materialize; not the batched calls */
} rgs_sketch;

typedef enum {
    RGS_P_FP64 = 0,            /* u_crs = u_fine = fp64 */
    RGS_P_FP32_LS64 = 1,       /* multi-precision model: u_crs = fp32, u_fine = fp64 */
    RGS_P_BF16Q_FP32_LS64 = 2, /* as FP32_LS64 with the basis stored in bfloat16 (round to nearest
                                  even): columns are kept unnormalised with an fp64 scale 1/r_ii,
                                  step 4 sketches the stored column, the coefficients of step 3
                                  carry the scales, and the returned Q is bf16(q'_i / r_ii) */
    RGS_P_FP32 = 3             /* unique precision u_crs = u_fine = fp32 (the comparison of
                                  Sec. 5.1): every step of Algorithm 2 in float32 arithmetic --
                                  the sketches of steps 1 and 4 (block partials and their sums),
                                  the Householder least squares of step 2, r_ii, s_i and step 7
                                  (q'_i times the float32 reciprocal of r_ii); R and S receive
                                  float32 values.  rgs_qr, rgs_qr_noalloc (Householder solver
                                  only: ls_sweeps must be 0) and rgs_sketch_apply (float32
                                  arithmetic); rgs_gmres: the configuration of the GMRES
                                  experiment of Sec. 5.3 -- this RGS as the Arnoldi step, the
                                  products with A in fp64 from the float32 basis vector (rounded
                                  once to float32), Givens rotations, x and the restart residual
                                  in fp64 (ls_sweeps 0), and rgs_gmres_batched the same, every
                                  system bit for bit a separate rgs_gmres call; not
                                  rgs_qr_batched(_ex) (EINVAL) */
} rgs_precision;

/* Flags for rgs_qr_desc.flags / rgs_gmres_desc.flags */
#define RGS_FLAG_DIAGNOSTICS 1u  /* compute step 8 of Algorithm 2 (Delta_m, tilde Delta_m) */
#define RGS_FLAG_TIME_KERNELS 2u /* time every projection+sketch launch with events */
#define RGS_FLAG_GRAPH 4u        /* rgs_gmres_batched: capture a restart cycle once as a HIP graph
                                    and replay it while the set of running systems is unchanged.
                                    rgs_qr_batched_ex: see there.
                                    rgs_qr: capture the factorisation's device work (all columns) once
                                    as a HIP graph, kept in the handle, and replay it on later calls
                                    with the same descriptor, pointers and leading dimensions (the
                                    contents of W may change); step 1 then runs on the handle's
                                    stream only.  Not with RGS_FLAG_TIME_KERNELS (EINVAL). */
#define RGS_FLAG_CERTIFY 8u      /* rgs_qr: a-posteriori certification of Theta (Prop. 3.7, Sec. 3)
                                    for V = Q and V = W with a second sketch Phi of the same kind and
                                    size, independent of Theta (counter word 2 = sketch_id + 1) and
                                    used for nothing else; results in rgs_report.cert_*.  Costs three
                                    sketches of n x m matrices (Theta Q, Phi Q, Phi W), a few k x m x m
                                    fp64 products and O(m^3) host work.  Not with IDENTITY (EINVAL).
                                    With RGS_FLAG_THETA_BF16, Phi is the Gaussian sketch (not its
                                    bf16 variant).
                                    rgs_gmres: the certificate (Phi with counter word 2 = 1, which no
                                    cycle's Theta uses) of the last cycle's Theta for V = its basis
                                    vectors that the last update of x used, in rgs_report.cert_smin_q,
                                    cert_smax_q, cert_cond_phi_q (the W pair stays NaN: the Arnoldi
                                    vectors are not kept); Sec. 5.3 reports omega for this basis. */
#define RGS_FLAG_THETA_BF16 16u  /* GAUSSIAN only (rgs_qr, rgs_qr_batched_ex, rgs_gmres, rgs_gmres_batched,
                                    rgs_sketch_apply, rgs_sketch_materialize): the Gaussian sketch
                                    with bf16 entries,
                                    theta = bf16(z)/sqrt(k), z the fp64 Box-Muller value of the
                                    Gaussian sketch rounded once to nearest even; the entries are
                                    made once per Theta into a table of 2 k ceil(n/8)*8 bytes in the
                                    handle's scratch and read by every later sketch instead of being
                                    drawn again.  A different (still i.i.d., entries within 2^-8
                                    relative of N(0,1/k)) sketch from the GAUSSIAN one */

#define RGS_FLAG_LAG 32u         /* rgs_gmres with SRHT or RADEMACHER, rgs_gmres_batched with SRHT:
                                    the lagged Arnoldi step (the lagged normalisation of Sec. 2.4)
                                    -- the mat-vec kernel computes
                                    t = A q'_i from the stored, unnormalised q'_i and sketches q'_i
                                    and t in the same pass, so r_ii = ||Theta q'_i|| and
                                    p_{i+1} = Theta t / r_ii come out of one reduction, and the
                                    projection no longer sketches; w_{i+1} = t / r_ii is applied on
                                    load.  Equal to Algorithm 3 in exact arithmetic.  The GAUSSIAN
                                    sketch always takes this step (its two sketches share draws). */
#define RGS_FLAG_THETA_EXACT 64u /* GAUSSIAN only (rgs_qr, rgs_gmres, rgs_sketch_apply; rgs_qr_batched_ex:
                                    see there; EINVAL with RGS_FLAG_THETA_BF16 and on the other
                                    calls): the same sketch
                                    (Sec. 2.1), its entries made once per Theta -- by the Box-Muller
                                    of the working precision, as every drawn sketch makes them --
                                    into a table of sizeof(T) k ceil(n/8)*8 bytes (T: double for
                                    RGS_P_FP64, else float) in the handle's scratch, and read from it
                                    by every later sketch instead of being drawn again: a sketch
                                    becomes a memory stream instead of a Philox call and a
                                    Box-Muller per four entries.  Results agree with the drawn sketch
                                    up to the order of the sums.  For k n small enough to keep
                                    (11.3 GB at k = 400, n = 192^3, float). */
/* rgs_qr_batched_ex only: step 2 of every factorisation of the call by s = 1..8
 * Richardson sweeps on the normal equations, exactly as rgs_qr_desc.ls_sweeps = s
 * gives rgs_qr (remark on the least-squares solver, Sec. 2.3); s = 0 keeps the
 * Householder QR of S.  The count sits in bits 24..27 of flags; EINVAL above 8. */
#define RGS_FLAG_LS_SWEEPS(s) (((uint32_t)(s)&15u) << 24)
#define RGS_FLAG_LS_SWEEPS_MASK (15u << 24)

/* Describes one RGS factorisation and its sketch Theta (k x n).
 * Theta is defined by (sketch, k, seed, sketch_id, instance) alone, so it is
 * regenerated on demand and not stored (Sec. 2.1, seeded generation), except
 * for the tables that RGS_FLAG_THETA_BF16 and RGS_FLAG_THETA_EXACT ask for. */
typedef struct {
    int64_t n;           /* rows of W (high dimension), n >= 1 */
    int64_t m;           /* columns of W, 1 <= m <= k */
    int64_t k;           /* sketch rows; k <= 2^ceil(log2 n) for SRHT, k = n for IDENTITY */
    uint64_t seed;       /* Philox key */
    uint32_t sketch_id;  /* counter word 2: independent sketches from one seed */
    uint32_t instance;   /* counter word 3 */
    int32_t sketch;      /* rgs_sketch */
    int32_t prec;        /* rgs_precision */
    uint32_t flags;      /* RGS_FLAG_* */
    uint32_t ls_sweeps;  /* step 2 solver of rgs_qr (ignored by the sketch hooks): 0 = Householder QR of S in
                            compact-WY form; 1..8 = that many Richardson iterations on the normal
                            equations, y = S^T p then y += S^T (p - S y) (remark on the least-squares
                            solver, Sec. 2.3): 1 is the sketched classical Gram-Schmidt, 2 its
                            re-orthogonalised form; EINVAL above 8 */
} rgs_qr_desc;

/* Constant-coefficient 7-point operator on an nx*ny*nz box, Dirichlet 0,
 * lexicographic order with x fastest (l = x + nx*(y + ny*z)):
 * (A u)_l = c0 u_l + cxm u_{x-1} + cxp u_{x+1} + cym u_{y-1} + cyp u_{y+1}
 *                  + czm u_{z-1} + czp u_{z+1}.  It is the Arnoldi mat-vec
 * w_i = A q_{i-1} of Algorithm 3 (Sec. 4.1). */
typedef struct {
    int64_t nx, ny, nz;
    double c0, cxm, cxp, cym, cyp, czm, czp;
} rgs_stencil7;

/* Restarted randomized GMRES (Sec. 4.2). */
typedef struct {
    int64_t restart;    /* inner steps per cycle (basis of restart+1 vectors), 1 <= restart < k */
    int64_t max_iters;  /* cap on the total number of inner steps (mat-vecs) */
    int64_t k;          /* sketch rows */
    double tol;         /* stop when ||b - A x||_2 / ||b||_2 <= tol (fp64) */
    uint64_t seed;
    int32_t sketch;     /* rgs_sketch (GAUSSIAN, SRHT or RADEMACHER; batched: GAUSSIAN or SRHT) */
    int32_t prec;       /* rgs_precision of the basis, mat-vec and projection */
    int32_t reuse_theta;/* 0: cycle c uses sketch_id 2+c (fresh Theta); 1: always sketch_id 2 */
    uint32_t flags;     /* rgs_gmres: RGS_FLAG_THETA_BF16, RGS_FLAG_THETA_EXACT, RGS_FLAG_LAG and
                           RGS_FLAG_CERTIFY (other bits: EINVAL);
                           rgs_gmres_batched: RGS_FLAG_GRAPH, RGS_FLAG_THETA_BF16, RGS_FLAG_LAG */
    uint32_t ls_sweeps; /* rgs_gmres: step 2 of every Arnoldi step (Alg. 3 on RGS, Sec. 2.3's remark on the
                           least-squares solver): 0 = Householder QR of S; 1..8 = that many Richardson
                           iterations on the normal equations, y = S^T p then y += S^T (p - S y), the first
                           being the sketched classical Gram-Schmidt; EINVAL above 8.  rgs_gmres_batched:
                           the same (every system, with the single solver's bits) */
} rgs_gmres_desc;

typedef struct {
    int64_t failed_column;  /* first invalid column on BREAKDOWN/NONFINITE, else -1 */
    int64_t iters;          /* GMRES: total inner steps; QR: m on success */
    int64_t cycles;         /* GMRES restart cycles */
    double delta_F;         /* ||I - S^T S||_F      (step 8; NaN unless requested) */
    double delta_tilde_F;   /* ||P - S R||_F/||P||_F (step 8; NaN unless requested) */
    double true_relres;     /* GMRES: ||b - A x||_2 / ||b||_2 at exit (fp64) */
    double seconds;         /* host wall time of the call, including the final sync */
    double proj_kernel_ms;  /* with RGS_FLAG_TIME_KERNELS: summed duration of the
                               projection+sketch launches, else 0 */
    int64_t proj_launches;  /* number of projection+sketch launches */
    /* RGS_FLAG_CERTIFY (Prop. 3.7): for V = Q (the returned basis) and V = W, the smallest and
     * largest singular values of (Theta V) X, X any matrix with (Phi V) X orthonormal; NaN when
     * not requested, when the factorisation failed, or when Phi V is numerically rank deficient.
     * rgs_omega_bar turns a pair into the bound omega_bar. */
    double cert_smin_q, cert_smax_q;
    double cert_smin_w, cert_smax_w;
    double cert_cond_phi_q; /* cond_2(Phi Q); u_crs times it bounds the rounding error of the
                               computed omega_bar for V = Q (Prop. 3.9) */
} rgs_report;

/* One factorisation of a batched call (all pointers device memory, as in rgs_qr). */
typedef struct {
    int64_t n, m, k;      /* 1 <= m <= k, per factorisation */
    const void *W;        /* n x m, ldw >= n, float */
    int64_t ldw;
    void *Q;              /* n x m, ldq >= n, float or bf16 per the batch precision */
    int64_t ldq;
    double *R;            /* m x m, ldr >= m */
    int64_t ldr;
    double *S;            /* k x m, lds >= k */
    int64_t lds;
} rgs_qr_item;

/* One system of a batched GMRES call (b and x device memory, res_hist host). */
typedef struct {
    rgs_stencil7 A;       /* operator of this system (its own grid and coefficients) */
    const double *b;      /* [n], n = nx*ny*nz */
    double *x;            /* [n] output, x0 = 0 */
    double *res_hist;     /* host, hist_cap entries, may be NULL when hist_cap == 0 */
    int64_t hist_cap;
} rgs_gmres_item;

/* Library version of this header (RGS_ABI_VERSION). */
int rgs_abi_version(void);

/* Prop. 3.7: omega_bar = max(1 - (1 - eps_star) smin^2, (1 + eps_star) smax^2 - 1), from the
 * rgs_report.cert_* pair of one V.  If omega_bar < 1 and Phi is an (eps_star, delta*, 1)
 * oblivious subspace embedding, Theta is an omega_bar-embedding of range(V) with probability at
 * least 1 - delta*.  NaN if smin or smax is NaN.  Pure host function. */
double rgs_omega_bar(double smin, double smax, double eps_star);

/* Static English description of a status code.  Never NULL. */
const char *rgs_status_string(rgs_status s);

/* Create a handle bound to HIP device `device` and stream `stream`.
 * *h receives the handle.  EINVAL: h == NULL or bad device; EDEVICE: HIP
 * failure.  The handle owns all scratch memory. */
rgs_status rgs_create(rgs_handle **h, int device, rgs_stream stream);

/* Release the handle and its scratch (synchronises its streams first). */
rgs_status rgs_destroy(rgs_handle *h);

/* Re-bind the handle to another stream of the same device. */
rgs_status rgs_set_stream(rgs_handle *h, rgs_stream stream);

/* Autotuner of the batched Gaussian sketch product (rgs_qr_batched and
 * rgs_qr_batched_ex with the Gaussian sketch).  Its schedules -- 64, 32 or
 * 128 operand columns per work unit; units in plain order, grouped so that
 * the units reading the same columns share an XCD, or with every unit of one
 * row chunk on one XCD -- give identical results; with mode 0 (default) the
 * handle times the nine on the first column step of the first call for a
 * batch signature (precision, sketch entries and every (n, m, k)) and keeps
 * the fastest for later calls with that signature; mode 1..9 always uses that
 * schedule (1: 64/plain, 2: 64/XCD, 3: 32/plain, 4: 32/XCD, 5: 64/chunk,
 * 6: 32/chunk, 7: 128/plain, 8: 128/XCD, 9: 128/chunk).  EINVAL otherwise. */
rgs_status rgs_set_tuning(rgs_handle *h, int32_t mode);

/* The schedule (1..9) the last batched Gaussian QR on this handle used, 0 if none. */
int32_t rgs_last_tuning(const rgs_handle *h);

/* RGS QR factorisation, Algorithm 2 (Sec. 2.3), W = Q R.
 *   W  [n x m, ldw >= n] input, element type per desc->prec.
 *   Q  [n x m, ldq >= n] output, same element type; Q = W R^-1 is orthonormal
 *      in the sketched inner product <Theta ., Theta .> (not in l2).
 *   R  [m x m, ldr >= m] output, upper triangular, r_ii > 0 (strict lower part
 *      is zeroed).
 *   S  [k x m, lds >= k] output, S = Theta Q as computed in steps 4-6.
 *   rep (host, may be NULL) receives the report.
 * Step 2 uses a Householder QR of S kept in compact-WY form (Sec. 2.3; the
 * solver of the experiments, Sec. 5).  W and Q must not overlap.
 * Returns OK, EINVAL, ENOMEM, EDEVICE, EBREAKDOWN or ENONFINITE. */
rgs_status rgs_qr(rgs_handle *h, const rgs_qr_desc *desc,
                  const void *W, int64_t ldw, void *Q, int64_t ldq,
                  double *R, int64_t ldr, double *S, int64_t lds, rgs_report *rep);

/* rgs_qr without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and status codes as rgs_qr --
 * the same kernels in the same order, so Q, R and S equal rgs_qr's bit for
 * bit -- except:
 *   - the library's scratch is a fixed 64 MiB device array per device (one
 *     copy on each device, held from the library's load until the process
 *     ends); its address is looked up when a handle is created on the device.
 *     No hipMalloc, hipFree, event or stream is created by the call, and no
 *     host table is copied (the P-SRHT rows are drawn on the device);
 *   - RGS_ESCRATCH (before any device work) when the factorisation does not
 *     fit that array: it holds five k x m fp64 matrices (P, the compact-WY
 *     factors twice), k x ceil(n/8192) partial sums of the working precision,
 *     at least one column of step-1 partials (64 x k fp64) and O(k + m^2 + n/32)
 *     more; e.g. k = 2048, m = 512 fits up to n = 2^23 in every precision; P-SRHT also needs
 *     k <= 4096;
 *   - desc->flags must be 0 (EINVAL): diagnostics, kernel timing,
 *     certification and the bf16 table need memory of their own;
 *   - step 1 runs on the handle's stream only (no auxiliary stream).
 * Every call on a device shares that device's array and leaves its contents
 * behind (each call initialises what it reads): calls that overlap in time on
 * one device -- two host threads, or two streams -- race and corrupt each
 * other's results.  Serialise them.
 * Returns OK, EINVAL, ESCRATCH, EDEVICE, EBREAKDOWN or ENONFINITE. */
rgs_status rgs_qr_noalloc(rgs_handle *h, const rgs_qr_desc *desc,
                          const void *W, int64_t ldw, void *Q, int64_t ldq,
                          double *R, int64_t ldr, double *S, int64_t lds, rgs_report *rep);

/* A batch of independent RGS QR factorisations (Algorithm 2, Sec. 2.3) of
 * uneven sizes, advanced in lockstep: each column step is one launch of each
 * kernel covering every factorisation that still has that column, so small
 * factorisations fill the device together.
 *   items (host array of `batch` <= 65535 entries) describe device buffers as in rgs_qr.
 *   prec: RGS_P_FP32_LS64 or RGS_P_BF16Q_FP32_LS64.
 *   Sketches: SRHT -- factorisation b uses counter word 3 (instance) = b;
 *   GAUSSIAN -- every factorisation uses the leading k_b x n_b block of one
 *   master Gaussian matrix (instance 0, entries scaled by 1/sqrt(k_b)).
 *   item_status / failed_column (host arrays of `batch`, may be NULL) receive
 *   each factorisation's status (RGS_OK, RGS_EBREAKDOWN, RGS_ENONFINITE) and
 *   first invalid column (-1 if none).
 * Returns RGS_OK when every factorisation succeeded, the first failing
 * status otherwise, or EINVAL / ENOMEM / EDEVICE. */
rgs_status rgs_qr_batched(rgs_handle *h, int64_t batch, const rgs_qr_item *items, int32_t sketch,
                          int32_t prec, uint64_t seed, uint32_t sketch_id, int32_t *item_status,
                          int64_t *failed_column, rgs_report *rep);

/* rgs_qr_batched with flags, any combination of:
 *   RGS_FLAG_THETA_BF16 (GAUSSIAN sketch only) -- the master matrix with bf16
 *     entries, bf16(z)/sqrt(k_b) (the entries the flag gives rgs_qr), made once
 *     per call into a table of 2 max(k_b) * 16 ceil(max(n_b)/16) bytes of the
 *     handle's scratch; the products of steps 1 and 4 then read it through
 *     bf16 matrix-core instructions (exact products: fp32 columns are split
 *     into three bf16 parts, bf16-basis columns are exact; fp32 accumulation)
 *     instead of drawing the entries;
 *   RGS_FLAG_THETA_EXACT (GAUSSIAN sketch only, not with THETA_BF16) -- the
 *     master matrix's fp32 entries, exactly those the drawn products make,
 *     made once per call into a table of 4 max(k_b) (32 ceil(max(n_b)/32) + 32)
 *     bytes of the handle's scratch and read by the fp32 matrix-core products
 *     of steps 1 and 4 instead of being drawn: results bitwise those of the
 *     call without the flag;
 *   RGS_FLAG_GRAPH -- each of the two streams' kernel sequences (every column
 *     of its share of the batch) is captured once as a HIP graph, kept in the
 *     handle, and replayed on later calls with the same items (sizes,
 *     pointers, leading dimensions; the contents of W may change), sketch,
 *     seed, sketch_id, precision and flags, while the handle's scratch has not
 *     moved.  The launch tables are still copied per call, before the graphs
 *     run.  With the GAUSSIAN sketch, a call whose product schedule is not yet
 *     tuned for this batch (the first, unless rgs_set_tuning forces one) runs
 *     eagerly and tunes it.  Results are bitwise those of an eager call.
 *   RGS_FLAG_LS_SWEEPS(s), s = 1..8 -- step 2 by s Richardson sweeps instead
 *     of the Householder QR of S (the kernels of rgs_qr with ls_sweeps = s:
 *     with the SRHT sketch every factorisation is bitwise that of a separate
 *     rgs_qr call with instance b and ls_sweeps = s).
 * EINVAL for any other flag, THETA_BF16 or THETA_EXACT with another sketch, both, or more than
 * 8 sweeps. */
rgs_status rgs_qr_batched_ex(rgs_handle *h, int64_t batch, const rgs_qr_item *items, int32_t sketch,
                             int32_t prec, uint64_t seed, uint32_t sketch_id, uint32_t flags,
                             int32_t *item_status, int64_t *failed_column, rgs_report *rep);

/* Y = Theta X for ncols columns (the sketch of steps 1 and 4 of Algorithm 2).
 *   X [n x ncols, ldx >= n], element type per desc->prec; Y [k x ncols, ldy >= k].
 * desc->m is ignored.  Synchronous.  Returns OK, EINVAL, ENOMEM or EDEVICE. */
rgs_status rgs_sketch_apply(rgs_handle *h, const rgs_qr_desc *desc, const void *X,
                            int64_t ldx, int64_t ncols, double *Y, int64_t ldy);

/* Dense block Theta[j0:j1, l0:l1] (0-based, half-open) into out
 * [(j1-j0) x (l1-l0), ldo >= j1-j0], as the device generates it in the working
 * precision of desc->prec (fp32 entries are widened).  Test hook for the
 * on-the-fly generation of Sec. 2.1.  Synchronous. */
rgs_status rgs_sketch_materialize(rgs_handle *h, const rgs_qr_desc *desc, int64_t j0,
                                  int64_t j1, int64_t l0, int64_t l1, double *out,
                                  int64_t ldo);

/* Restarted randomized GMRES (Sec. 4.2) on the 7-point operator A, built on
 * RGS-Arnoldi (Algorithm 3): H = R(1:i, 2:i), Givens rotations in fp64, x kept
 * in fp64, x0 = 0.
 *   b  [n] input (device, double), n = nx*ny*nz.
 *   x  [n] output (device, double).
 *   res_hist (host, may be NULL) receives |g_i|/||b||_2 after each inner step,
 *      up to hist_cap entries (the sketched residual ||Theta(b - A x_i)||, Sec. 4.2).
 *   rep (host, may be NULL).
 * desc->prec: FP64, FP32_LS64, BF16Q_FP32_LS64 (basis stored unnormalised in
 * bf16 with fp64 scales; the mat-vec input is fl32(stored column / r_ii)) or
 * FP32 (the configuration of Sec. 5.3, see rgs_precision).
 * Returns OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE or ENOCONV. */
rgs_status rgs_gmres(rgs_handle *h, const rgs_stencil7 *A, const rgs_gmres_desc *desc,
                     const double *b, double *x, double *res_hist, int64_t hist_cap,
                     rgs_report *rep);

/* A batch of independent restarted randomized GMRES solves (Sec. 4.2, on
 * RGS-Arnoldi, Algorithm 3) of uneven sizes, sharing one descriptor (restart,
 * k, tol, max_iters, sketch, precision).  The systems advance in lockstep, one
 * restart cycle at a time: each inner step is one launch of each kernel over
 * every system still running; a system stops itself on the device when its
 * sketched residual reaches tol (or at a lucky breakdown), and drops out of
 * later cycles once its true residual ||b - A x||/||b|| <= tol (fp64).
 *   items (host array of `batch` <= 65535 entries); every system's sketch is
 *   the one a separate rgs_gmres call with the same descriptor would use
 *   (instance 0, its own n), so each system's x, history and counts equal
 *   those of a separate call.
 *   desc->sketch: GAUSSIAN or SRHT.  desc->flags: RGS_FLAG_GRAPH, RGS_FLAG_THETA_BF16 (one
 *   table over the largest n per cycle serves every system).
 *   item_status (host, `batch` entries, may be NULL): RGS_OK, RGS_ENONFINITE or
 *   RGS_ENOCONV per system; reps (host, `batch` entries, may be NULL): per
 *   system iters, cycles, true_relres (seconds = the whole call).
 * Returns RGS_OK when every system converged, the first failing system's
 * status otherwise, or EINVAL / ENOMEM / EDEVICE. */
rgs_status rgs_gmres_batched(rgs_handle *h, int64_t batch, const rgs_gmres_item *items,
                             const rgs_gmres_desc *desc, int32_t *item_status, rgs_report *reps);

/* w = A u for the 7-point operator (the mat-vec of Algorithm 3, step 3), in
 * the working precision of `prec` (u, w: float for FP32_LS64, double for FP64;
 * FP32: float u and w with the arithmetic in fp64, the mat-vec of RGS_P_FP32
 * GMRES).  Test hook.  Synchronous. */
rgs_status rgs_stencil_apply(rgs_handle *h, const rgs_stencil7 *A, int32_t prec,
                             const void *u, void *w);

#ifdef __cplusplus
}
#endif

#endif /* RGS_H */
