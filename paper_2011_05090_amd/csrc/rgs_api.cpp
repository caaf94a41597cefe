// Host side of librgs: the C ABI declared in include/rgs.h.
//
// rgs_qr drives Algorithm 2 (Sec. 2.3 of Balabanov & Grigori) column by column
// with no host synchronisation inside the loop: every step's scalars (r_ii,
// 1/r_ii, the Householder tau/beta, the breakdown status) stay in device
// memory and the host only enqueues launches on the handle's stream.  The
// stream is synchronised once, at the end, to read the status word.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "rgs.h"
#include "rgs_dense.hpp"
#include "rgs_device.hpp"
#include "rgs_internal.hpp"

using namespace rgs;

struct rgs_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;   // created on first use: graph capture needs a non-null stream
    hipStream_t aux = nullptr;       // created on first use: the second share of a batched QR call
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    std::vector<hipEvent_t> chunk_ev;   // step-1 chunks of a QR on the auxiliary stream
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::vector<hipEvent_t> events;
    // autotuner of the batched Gaussian sketch product: schedule chosen per
    // batch signature (1-based index into kGemmSchedules), tuning mode
    std::unordered_map<uint64_t, int> gemm_tuned;
    int tune_mode = 0;        // 0: tune on first use, s > 0: always schedule s
    int last_schedule = 0;    // schedule used by the last batched Gaussian call
    // RGS_FLAG_GRAPH on rgs_qr: the device work of the last captured call and
    // the signature (every argument, the arena's address and size) it was captured for
    hipGraph_t qr_graph = nullptr;
    hipGraphExec_t qr_exec = nullptr;
    std::vector<uint64_t> qr_key;
    // RGS_FLAG_GRAPH on rgs_qr_batched_ex: one captured kernel sequence per
    // share of the last captured batch, and its signature
    hipGraph_t qrb_graph[2] = {nullptr, nullptr};
    hipGraphExec_t qrb_exec[2] = {nullptr, nullptr};
    std::vector<uint64_t> qrb_key;
};

// Fixed device scratch of rgs_qr_noalloc, for callers that cannot allocate.
// One copy per device, held from the library's load until the process ends.
// In host code `scratch` only names the symbol: its device address (different
// on every device) comes from hipGetSymbolAddress, taken once per device when
// a handle is created on it (bind_scratch) and used everywhere after that.
static constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr size_t kAlign = 256;

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxScratchDevices] = {};

// With `device` current: looks up (once per device) the device address of
// this device's copy of `scratch`.
rgs_status bind_scratch(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return RGS_OK;   // rgs_qr_noalloc then reports EDEVICE
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return RGS_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        return RGS_EDEVICE;
    }
    g_scratch_ptr[device] = static_cast<char*>(ptr);
    return RGS_OK;
}

char* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

struct Carver {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count) {
        off = (off + kAlign - 1) / kAlign * kAlign;
        const size_t at = off;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return at;
    }
};

rgs_status ensure_arena(rgs_handle* h, size_t bytes) {
    if (h->arena_bytes >= bytes) return RGS_OK;
    if (h->arena) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) return RGS_EDEVICE;
        if (h->aux && hipStreamSynchronize(h->aux) != hipSuccess) return RGS_EDEVICE;
        (void)hipFree(h->arena);
        h->arena = nullptr;
        h->arena_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return RGS_ENOMEM;
    }
    h->arena = static_cast<char*>(p);
    h->arena_bytes = bytes;
    return RGS_OK;
}

rgs_status ensure_events(rgs_handle* h, size_t count) {
    while (h->events.size() < count) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return RGS_EDEVICE;
        h->events.push_back(e);
    }
    return RGS_OK;
}

// The handle's auxiliary stream (default priority) and its fork / join
// events: work put on it is forked from the handle's stream and joined back
// into it with events, so every call stays ordered on the handle's stream.
rgs_status ensure_aux(rgs_handle* h) {
    if (!h->aux && hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess) return RGS_EDEVICE;
    for (hipEvent_t* e : {&h->fork_ev, &h->join_ev})
        if (!*e && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return RGS_EDEVICE;
    return RGS_OK;
}

// Untimed events that mark the step-1 chunks done on the auxiliary stream.
rgs_status ensure_chunk_events(rgs_handle* h, size_t count) {
    while (h->chunk_ev.size() < count) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return RGS_EDEVICE;
        h->chunk_ev.push_back(e);
    }
    return RGS_OK;
}

int64_t srht_order(int64_t n) {
    int64_t s = 1;
    while (s < n) s <<= 1;
    return s;
}

// k distinct rows of [0, s) by a partial Fisher-Yates shuffle; draw t uses
// Philox(t, 0xFFFFFFFE, sketch_id, instance) and swaps position t with
// t + floor((x1 2^32 + x0) (s - t) / 2^64).  Rows are kept in draw order.
void srht_rows_host(int64_t s, int k, const SketchArgs& sk, std::vector<int>& rows) {
    std::unordered_map<uint64_t, uint64_t> perm;
    perm.reserve(2 * (size_t)k + 1);
    rows.resize(k);
    for (int t = 0; t < k; ++t) {
        uint32_t x[4];
        philox4x32_10((uint32_t)t, kTagRows, sk.sid, sk.inst, sk.k0, sk.k1, x);
        const uint64_t r64 = ((uint64_t)x[1] << 32) | x[0];
        const uint64_t span = (uint64_t)(s - t);
        const uint64_t off = (uint64_t)(((unsigned __int128)r64 * span) >> 64);
        const uint64_t idx = (uint64_t)t + off;
        auto it_t = perm.find((uint64_t)t);
        auto it_i = perm.find(idx);
        const uint64_t at = it_t == perm.end() ? (uint64_t)t : it_t->second;
        const uint64_t ai = it_i == perm.end() ? idx : it_i->second;
        perm[(uint64_t)t] = ai;
        perm[idx] = at;
        rows[t] = (int)ai;
    }
}

SketchArgs make_sketch(int sketch, int64_t k, uint64_t seed, uint32_t sid, uint32_t inst) {
    SketchArgs sk{};
    sk.sketch = sketch;
    sk.k = (int)k;
    sk.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    sk.k1 = (uint32_t)(seed >> 32);
    sk.sid = sid;
    sk.inst = inst;
    return sk;
}

constexpr uint32_t kMaxSweeps = 8;   // Richardson sweeps of step 2 accepted by rgs_qr
// Sketch rows of a single call: kKptMax rows per thread of a 512-thread
// workgroup (the batched calls keep 256-thread kernels: kKptMax * kWG).
constexpr int64_t kMaxK = (int64_t)kKptMax * kProjWaves * kWave;

int sketch_kind(int32_t sketch) {
    switch (sketch) {
        case RGS_SKETCH_GAUSSIAN: return SK_GAUSS;
        case RGS_SKETCH_SRHT: return SK_SRHT;
        case RGS_SKETCH_RADEMACHER: return SK_RADEM;
        default: return SK_IDENT;
    }
}

// Sketches generated entry by entry from Philox (no transform).
bool dense_sketch(int sk_kind) {
    return sk_kind == SK_GAUSS || sk_kind == SK_RADEM || sk_kind == SK_TABLE || sk_kind == SK_TABX;
}

bool valid_desc(const rgs_qr_desc* d, bool need_m) {
    if (!d) return false;
    if (d->n < 1 || d->k < 1) return false;
    if (need_m && (d->m < 1 || d->m > d->k)) return false;
    if (d->prec != RGS_P_FP64 && d->prec != RGS_P_FP32_LS64 && d->prec != RGS_P_BF16Q_FP32_LS64 &&
        d->prec != RGS_P_FP32)
        return false;
    if (d->ls_sweeps > kMaxSweeps) return false;
    if (d->prec == RGS_P_FP32 && d->ls_sweeps != 0) return false;   // the float32 chain is Householder only
    switch (d->sketch) {
        case RGS_SKETCH_GAUSSIAN:
            if (d->k > kMaxK) return false;
            if (d->n > ((int64_t)1 << 34)) return false;   // counter word 0 holds l/4
            break;
        case RGS_SKETCH_RADEMACHER:
            if (d->k > kMaxK) return false;
            if (d->n > ((int64_t)1 << 38)) return false;   // counter word 0 holds l/128
            break;
        case RGS_SKETCH_SRHT:
            if (d->k > kMaxK) return false;
            if (d->k > srht_order(d->n)) return false;
            if (d->n > ((int64_t)1 << 31)) return false;
            break;
        case RGS_SKETCH_IDENTITY:
            if (d->k != d->n) return false;
            if (d->n > ((int64_t)1 << 24)) return false;
            break;
        default:
            return false;
    }
    return true;
}

// Prepares the sketch tables (SRHT sign bits, sampled rows) in `sk`.
// device_rows: draw the sampled rows on the device (no host table, no copy,
// no synchronisation) instead of on the host.
rgs_status setup_sketch(rgs_handle* h, SketchArgs& sk, int64_t n, uint32_t* signs_dev, int* rows_dev,
                        bool device_rows = false) {
    if (sk.sketch != SK_SRHT) return RGS_OK;
    const int64_t nwords = (n + 31) / 32;
    if (!launch_srht_signs(h->stream, signs_dev, nwords, sk)) return RGS_EDEVICE;
    if (device_rows) {
        if (!launch_srht_rows(h->stream, rows_dev, srht_order(n), sk)) return RGS_EDEVICE;
        sk.signs = signs_dev;
        sk.rows = rows_dev;
        return RGS_OK;
    }
    std::vector<int> rows;
    srht_rows_host(srht_order(n), sk.k, sk, rows);
    if (hipMemcpyAsync(rows_dev, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice, h->stream) !=
        hipSuccess)
        return RGS_EDEVICE;
    // rows lives on the host stack frame: wait for the copy before returning
    if (hipStreamSynchronize(h->stream) != hipSuccess) return RGS_EDEVICE;
    sk.signs = signs_dev;
    sk.rows = rows_dev;
    return RGS_OK;
}

// Layout of the scratch arena for one factorisation.
struct QrPlan {
    size_t signs, rows, part_proj, part_P, P, Vc, Vr, Wc, Wr, X, sp, u, v, uh, pd, pd2, pdb, pbuf;
    size_t rr, invr, pnorm, tau, beta, status, coef, diag, cert, table;
    size_t total;
    int G_P, G_col, cc;
    int64_t nblk, nproj;
};

// Below this many rows the fused projection + Gaussian sketch has too few row
// blocks to fill the device, so the column's sketch gets a launch of its own
// spread over up to 256 row groups x k/256 row chunks of Theta.
constexpr int64_t kSplitRows = (int64_t)128 * kProjRows;

// part_budget: bytes for the step-1 partials of the columns sketched together
// (at least one column's worth is always planned).
// table: bytes per entry of a table of Theta (0: none; 2: the bf16 table;
// sizeof(T): the exact table).
QrPlan plan_qr(int64_t n, int64_t m, int64_t k, int sketch, size_t tsize, bool certify = false,
               size_t table = 0, size_t part_budget = (size_t)64 << 20) {
    QrPlan p{};
    Carver c;
    p.nblk = (n + kBlock - 1) / kBlock;
    p.nproj = (n + kProjRows - 1) / kProjRows;
    const int64_t nsl = (k + kSlice - 1) / kSlice;
    const int64_t nsub = (n + 255) / 256;
    // row groups of P = Theta W: 4096-row blocks (SRHT), 256-row sub-blocks (Gaussian)
    p.G_P = (int)std::min<int64_t>(dense_sketch(sketch) ? nsub : p.nblk, 64);
    // Gaussian / Rademacher sketch of a single column in its own launch (below kSplitRows rows)
    p.G_col = (dense_sketch(sketch) && n < kSplitRows)
                  ? (int)std::min<int64_t>((n + kGSubCol - 1) / kGSubCol, 256)
                  : 0;
    const size_t per_col = (size_t)p.G_P * k * sizeof(double);   // step-1 partials accumulate in fp64
    p.cc = (int)std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)(part_budget / std::max<size_t>(per_col, 1))));
    p.signs = c.take<uint32_t>((n + 31) / 32 + 4);
    p.rows = c.take<int>(k);
    p.part_proj = c.take<char>(
        (sketch == SK_IDENT ? (size_t)n : (size_t)std::max<int64_t>(p.nproj, p.G_col) * k) * tsize);
    p.part_P = c.take<char>(per_col * p.cc);
    p.P = c.take<double>(k * m);
    p.Vc = c.take<double>(k * m);
    p.Vr = c.take<double>(k * m);
    p.Wc = c.take<double>(k * m);
    p.Wr = c.take<double>(k * m);
    p.X = c.take<double>(m * m);
    p.sp = c.take<double>(k);
    p.u = c.take<double>(k);
    p.v = c.take<double>(k);
    p.uh = c.take<double>(m + 1);
    p.pd = c.take<double>(nsl * (m + 1));
    p.pd2 = c.take<double>(nsl);
    p.pdb = c.take<double>(nsl * (m + 2));
    p.pbuf = c.take<double>(k);
    p.rr = c.take<double>(m);
    p.invr = c.take<double>(m);
    p.pnorm = c.take<double>(m);
    p.tau = c.take<double>(m);
    p.beta = c.take<double>(m);
    p.status = c.take<int>(4);
    p.coef = c.take<char>(m * tsize);
    p.diag = c.take<double>(3 * m);
    // certification (Prop. 3.7): six k x m and four m x m fp64 matrices
    p.cert = certify ? c.take<double>(6 * k * m + 4 * m * m) : 0;
    // table of the Gaussian sketch: (n + 7) / 8 groups of 8 entries per sketch row
    p.table = table ? c.take<char>((size_t)((n + 7) / 8) * 8 * k * table) : 0;
    p.total = c.off + kAlign;
    return p;
}

SpaceArgs space_args(char* A, const QrPlan& pl, int64_t k, int64_t m) {
    SpaceArgs sa{};
    sa.k = (int)k;
    sa.mcap = (int)m;
    sa.Vc = reinterpret_cast<double*>(A + pl.Vc);
    sa.Vr = reinterpret_cast<double*>(A + pl.Vr);
    sa.Wc = reinterpret_cast<double*>(A + pl.Wc);
    sa.Wr = reinterpret_cast<double*>(A + pl.Wr);
    sa.X = reinterpret_cast<double*>(A + pl.X);
    sa.sp = reinterpret_cast<double*>(A + pl.sp);
    sa.u = reinterpret_cast<double*>(A + pl.u);
    sa.v = reinterpret_cast<double*>(A + pl.v);
    sa.uh = reinterpret_cast<double*>(A + pl.uh);
    sa.pd = reinterpret_cast<double*>(A + pl.pd);
    sa.pd2 = reinterpret_cast<double*>(A + pl.pd2);
    sa.pdb = reinterpret_cast<double*>(A + pl.pdb);
    sa.pbuf = reinterpret_cast<double*>(A + pl.pbuf);
    sa.rr = reinterpret_cast<double*>(A + pl.rr);
    sa.invr = reinterpret_cast<double*>(A + pl.invr);
    sa.pnorm = reinterpret_cast<double*>(A + pl.pnorm);
    sa.tau = reinterpret_cast<double*>(A + pl.tau);
    sa.beta = reinterpret_cast<double*>(A + pl.beta);
    sa.status = reinterpret_cast<int*>(A + pl.status);
    return sa;
}

// RGS_FLAG_THETA_BF16: fills the bf16 table of the Gaussian sketch sk (in
// stream order) and switches sk to read it.
rgs_status use_table(rgs_handle* h, SketchArgs& sk, int64_t n, uint16_t* table) {
    if (!launch_theta_table(h->stream, sk, n, table)) return RGS_EDEVICE;
    sk.sketch = SK_TABLE;
    sk.table = table;
    return RGS_OK;
}

// RGS_FLAG_THETA_EXACT: fills the table of the Gaussian sketch sk with its
// entries in T (in stream order) and switches sk to read it.
template <typename T>
rgs_status use_tabx(rgs_handle* h, SketchArgs& sk, int64_t n, T* table) {
    if (!launch_theta_tabx<T>(h->stream, sk, n, table)) return RGS_EDEVICE;
    sk.sketch = SK_TABX;
    sk.tabx = table;
    return RGS_OK;
}

// Bytes per entry of the table of Theta that desc flags ask for (T: the
// working type of the sketches).
size_t table_entry(uint32_t flags, size_t tsize) {
    if (flags & RGS_FLAG_THETA_BF16) return 2;
    if (flags & RGS_FLAG_THETA_EXACT) return tsize;
    return 0;
}

// Y = Theta X for ncols columns of X (element type TX; Theta's entries and
// the staging in T; accumulation and block partials in TA, fp64 for step 1 and
// the certificate, as the paper's multi-precision model computes sketches at
// u_fine; reduction in TR: fp64, or float32 with TA for the unique-precision
// model), cc columns per pass.
template <typename TX, typename T, typename TA, typename TR = double>
rgs_status sketch_matrix(rgs_handle* h, const SketchArgs& sk, const TX* X, int64_t ldx, int64_t n, int64_t ncols,
                         int G, int cc, TA* part, double* out, int64_t ldo, hipStream_t stream = nullptr) {
    hipStream_t st = stream ? stream : h->stream;
    const double scale = sk.sketch == SK_IDENT ? 1.0 : 1.0 / std::sqrt((double)sk.k);
    for (int64_t c0 = 0; c0 < ncols; c0 += cc) {
        const int nc = (int)std::min<int64_t>(cc, ncols - c0);
        if (sk.sketch == SK_IDENT) {
            if constexpr (std::is_same<TX, T>::value) {
                // Theta = I: the sketch of a column is the column (reduce over G = 1 partial)
                for (int c = 0; c < nc; ++c)
                    if (!launch_reduce<T>(st, X + (c0 + c) * ldx, 1, (int)n, 1, 1.0, out + (c0 + c) * ldo,
                                          ldo))
                        return RGS_EDEVICE;
                continue;
            } else {
                return RGS_EINVAL;
            }
        }
        if (dense_sketch(sk.sketch)) {
            if (!launch_gauss_cols<TX, T, TA>(st, X + c0 * ldx, ldx, n, nc, G, sk, part)) return RGS_EDEVICE;
        } else if (!launch_sketch_cols<TX, TA>(st, X + c0 * ldx, ldx, n, nc, G, sk, part)) {
            return RGS_EDEVICE;
        }
        if (!launch_reduce<TA, TR>(st, part, G, sk.k, nc, scale, out + c0 * ldo, ldo)) return RGS_EDEVICE;
    }
    return RGS_OK;
}

void report_defaults(rgs_report* r) {
    r->failed_column = -1;
    r->iters = 0;
    r->cycles = 0;
    r->delta_F = NAN;
    r->delta_tilde_F = NAN;
    r->true_relres = NAN;
    r->seconds = 0.0;
    r->proj_kernel_ms = 0.0;
    r->proj_launches = 0;
    r->cert_smin_q = r->cert_smax_q = NAN;
    r->cert_smin_w = r->cert_smax_w = NAN;
    r->cert_cond_phi_q = NAN;
}

// A-posteriori certification of Theta (Prop. 3.7) for V = Q (the returned
// basis) and V = W: the extreme singular values of (Theta V) X with X such
// that (Phi V) X is orthonormal.  Phi is a second sketch of the same kind and
// size, independent of Theta (counter word 2 = sketch_id + 1); as the paper
// suggests, it is used for nothing else.  Theta Q is a fresh sketch of the
// returned Q, Theta W is P from step 1.  For V = W both sketches are first
// multiplied by R^-1: the range, hence the singular values, is unchanged, and
// the Gram matrices formed next stay well conditioned however ill-conditioned
// W is.  With Z_Phi = (Phi V) M, Z_Theta = (Theta V) M (M = I or R^-1):
// Z_Phi^T Z_Phi = T^T T (Cholesky), X = M T^-1, and the squared singular
// values are the eigenvalues of Y^T Y with Y = Z_Theta T^-1.  The k x m
// products run on the device, the m x m factorisations, inverses and
// eigenvalue extremes on the host, all in fp64.
template <typename T, typename TQ>
rgs_status certify(rgs_handle* h, const rgs_qr_desc* d, const QrPlan& pl, const SketchArgs& theta, const T* W,
                   int64_t ldw, const TQ* Q, int64_t ldq, const double* R, int64_t ldr, rgs_report* rep) {
    const int64_t n = d->n, m = d->m, k = d->k;
    const int mi = (int)m, ki = (int)k;
    hipStream_t s = h->stream;
    char* A = h->arena;
    const double* P = reinterpret_cast<const double*>(A + pl.P);
    double* thQ = reinterpret_cast<double*>(A + pl.cert);
    double* phQ = thQ + k * m;
    double* phW = phQ + k * m;
    double* Z1 = phW + k * m;   // P R^-1
    double* Z2 = Z1 + k * m;    // (Phi W) R^-1
    double* Y = Z2 + k * m;
    double* Md = Y + k * m;     // two m x m right factors
    double* Gd = Md + 2 * m * m;   // two m x m Gram matrices
    double* part = reinterpret_cast<double*>(A + pl.part_P);
    const size_t mm = (size_t)m * m;
    auto both = [](auto f) {   // f(0) and f(1) on two host threads; an exception of either is rethrown here
        std::exception_ptr e1;
        std::thread t1([&]() {
            try {
                f(1);
            } catch (...) {
                e1 = std::current_exception();
            }
        });
        try {
            f(0);
        } catch (...) {
            t1.join();
            throw;
        }
        t1.join();
        if (e1) std::rethrow_exception(e1);
    };

    std::vector<double> Rh(mm);
    if (hipMemcpy2DAsync(Rh.data(), m * sizeof(double), R, ldr * sizeof(double), m * sizeof(double), m,
                         hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return RGS_EDEVICE;
    rgs_status st = sketch_matrix<TQ, T, double>(h, theta, Q, ldq, n, m, pl.G_P, pl.cc, part, thQ, k);
    if (st != RGS_OK) return st;
    // Phi of a bf16-table Theta is the Gaussian sketch generated on the fly
    const int phi_kind = (theta.sketch == SK_TABLE || theta.sketch == SK_TABX) ? SK_GAUSS : theta.sketch;
    SketchArgs phi = make_sketch(phi_kind, k, d->seed, d->sketch_id + 1u, d->instance);
    // Theta's tables are no longer read: Phi's overwrite them in stream order
    st = setup_sketch(h, phi, n, reinterpret_cast<uint32_t*>(A + pl.signs), reinterpret_cast<int*>(A + pl.rows));
    if (st != RGS_OK) return st;
    st = sketch_matrix<TQ, T, double>(h, phi, Q, ldq, n, m, pl.G_P, pl.cc, part, phQ, k);
    if (st != RGS_OK) return st;
    st = sketch_matrix<T, T, double>(h, phi, W, ldw, n, m, pl.G_P, pl.cc, part, phW, k);
    if (st != RGS_OK) return st;
    const std::vector<double> Rinv = dense::upper_inverse(Rh, mi);   // overlaps the sketches
    if (hipMemcpyAsync(Md, Rinv.data(), mm * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return RGS_EDEVICE;
    if (!launch_dgemm(s, false, ki, mi, mi, P, k, Md, m, Z1, k) ||
        !launch_dgemm(s, false, ki, mi, mi, phW, k, Md, m, Z2, k) ||
        !launch_dgemm(s, true, mi, mi, ki, phQ, k, phQ, k, Gd, m) ||
        !launch_dgemm(s, true, mi, mi, ki, Z2, k, Z2, k, Gd + mm, m))
        return RGS_EDEVICE;
    std::vector<double> Gh(2 * mm);
    if (hipMemcpyAsync(Gh.data(), Gd, 2 * mm * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return RGS_EDEVICE;

    // host: Cholesky factors of both Gram matrices and their inverses; cond(Phi Q)
    // on a third thread that runs on through the second device phase
    std::vector<double> Tq(Gh.begin(), Gh.begin() + mm), Tw(Gh.begin() + mm, Gh.end());
    bool ok[2] = {false, false}, ok_c = false;
    double gq_min = NAN, gq_max = NAN;
    std::vector<double> Tinv(2 * mm);
    std::thread tc([&]() {   // reads Gh, which nothing writes from here on
        try {
            ok_c = dense::sym_eig_extremes(std::vector<double>(Gh.begin(), Gh.begin() + mm), mi, gq_min, gq_max);
        } catch (...) {
            ok_c = false;   // cond(Phi Q) stays NaN
        }
    });
    struct Joiner {
        std::thread& t;
        ~Joiner() {
            if (t.joinable()) t.join();
        }
    } join_tc{tc};   // every return below waits for it
    both([&](int b) {
        std::vector<double>& Tm = b == 0 ? Tq : Tw;
        ok[b] = dense::cholesky_upper(Tm, mi);
        if (ok[b]) {
            const std::vector<double> inv = dense::upper_inverse(Tm, mi);
            std::copy(inv.begin(), inv.end(), Tinv.begin() + b * mm);
        }
    });
    if (hipMemcpyAsync(Md, Tinv.data(), 2 * mm * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return RGS_EDEVICE;
    if (!launch_dgemm(s, false, ki, mi, mi, thQ, k, Md, m, Y, k) ||
        !launch_dgemm(s, true, mi, mi, ki, Y, k, Y, k, Gd, m) ||
        !launch_dgemm(s, false, ki, mi, mi, Z1, k, Md + mm, m, Y, k) ||
        !launch_dgemm(s, true, mi, mi, ki, Y, k, Y, k, Gd + mm, m))
        return RGS_EDEVICE;
    std::vector<double> Ch(2 * mm);
    if (hipMemcpyAsync(Ch.data(), Gd, 2 * mm * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return RGS_EDEVICE;
    double lo[2] = {NAN, NAN}, hi[2] = {NAN, NAN};
    bool ok_e[2] = {false, false};
    both([&](int b) {
        if (!ok[b]) return;
        ok_e[b] = dense::sym_eig_extremes(std::vector<double>(Ch.begin() + b * mm, Ch.begin() + (b + 1) * mm), mi,
                                          lo[b], hi[b]);
    });
    if (ok_e[0]) {
        rep->cert_smin_q = std::sqrt(std::max(lo[0], 0.0));
        rep->cert_smax_q = std::sqrt(std::max(hi[0], 0.0));
    }
    if (ok_e[1]) {
        rep->cert_smin_w = std::sqrt(std::max(lo[1], 0.0));
        rep->cert_smax_w = std::sqrt(std::max(hi[1], 0.0));
    }
    tc.join();
    if (ok_c && gq_min > 0) rep->cert_cond_phi_q = std::sqrt(gq_max / gq_min);
    return RGS_OK;
}

// The certificate of Prop. 3.7 for one basis V (n x m, leading dimension ldv,
// element TQ): the extreme singular values of (Theta V) X with (Phi V) X
// orthonormal, and cond_2(Phi V).  Any column scaling of V gives the same
// values (V -> V M leaves them unchanged), so unnormalised stored columns are
// certified as they are.  Phi's tables overwrite Theta's (signs, rows): V is
// sketched with Theta first.  ws: 3 k m + 2 m^2 doubles; part: the plan's
// step-1 partials.  The values stay NaN where a factorisation fails.
template <typename TQ, typename T>
rgs_status certify_basis(rgs_handle* h, const QrPlan& pl, const SketchArgs& theta, const SketchArgs& phi,
                         const TQ* V, int64_t ldv, int64_t n, int m, int k, double* ws, double* part,
                         uint32_t* signs, int* rows, double* smin, double* smax, double* cond_phi) {
    hipStream_t s = h->stream;
    const size_t mm = (size_t)m * m;
    double* thV = ws;
    double* phV = thV + (size_t)k * m;
    double* Y = phV + (size_t)k * m;
    double* Md = Y + (size_t)k * m;
    double* Gd = Md + mm;
    rgs_status st = sketch_matrix<TQ, T, double>(h, theta, V, ldv, n, m, pl.G_P, pl.cc, part, thV, k);
    if (st != RGS_OK) return st;
    SketchArgs ph = phi;
    if ((st = setup_sketch(h, ph, n, signs, rows)) != RGS_OK) return st;
    if ((st = sketch_matrix<TQ, T, double>(h, ph, V, ldv, n, m, pl.G_P, pl.cc, part, phV, k)) != RGS_OK) return st;
    if (!launch_dgemm(s, true, m, m, k, phV, k, phV, k, Gd, m)) return RGS_EDEVICE;
    std::vector<double> G(mm);
    if (hipMemcpyAsync(G.data(), Gd, mm * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return RGS_EDEVICE;
    double gmin = NAN, gmax = NAN;
    if (dense::sym_eig_extremes(G, m, gmin, gmax) && gmin > 0) *cond_phi = std::sqrt(gmax / gmin);
    std::vector<double> Tm = G;
    if (!dense::cholesky_upper(Tm, m)) return RGS_OK;   // Phi V rank-deficient: no certificate
    const std::vector<double> Tinv = dense::upper_inverse(Tm, m);
    if (hipMemcpyAsync(Md, Tinv.data(), mm * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
        !launch_dgemm(s, false, k, m, m, thV, k, Md, m, Y, k) || !launch_dgemm(s, true, m, m, k, Y, k, Y, k, Gd, m))
        return RGS_EDEVICE;
    std::vector<double> C(mm);
    if (hipMemcpyAsync(C.data(), Gd, mm * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)   // Tinv and C stay alive till here
        return RGS_EDEVICE;
    double lo = NAN, hi = NAN;
    if (dense::sym_eig_extremes(C, m, lo, hi)) {
        *smin = std::sqrt(std::max(lo, 0.0));
        *smax = std::sqrt(std::max(hi, 0.0));
    }
    return RGS_OK;
}

// fixed != nullptr: the factorisation runs in the caller-independent fixed
// buffer `fixed` of fixed_bytes (the no-allocation entry point) instead of
// the handle's arena: nothing is allocated, no event or auxiliary stream is
// used, step 1 runs chunk by chunk on the handle's stream just before the
// columns that read each chunk, and the SRHT rows are drawn on the device.
// Flags that need memory of their own are rejected by the caller.
// TS: arithmetic of the sketch space, steps 1-2 and 4-6 (fp64; float32 for
// the unique-precision model RGS_P_FP32, whose step-1 partials and their
// reduction are float32 too).
template <typename T, typename TQ, bool DEFER, typename TS = double>
rgs_status run_qr(rgs_handle* h, const rgs_qr_desc* d, const T* W, int64_t ldw, TQ* Q, int64_t ldq, double* R,
                  int64_t ldr, double* S, int64_t lds, rgs_report* rep, char* fixed = nullptr,
                  size_t fixed_bytes = 0) {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = d->n, m = d->m, k = d->k;
    const int sk_kind = sketch_kind(d->sketch);
    const bool want_cert = (d->flags & RGS_FLAG_CERTIFY) != 0 && rep != nullptr;
    const bool tab = (d->flags & RGS_FLAG_THETA_BF16) != 0;
    const bool tabx = (d->flags & RGS_FLAG_THETA_EXACT) != 0;
    QrPlan pl = plan_qr(n, m, k, sk_kind, sizeof(T), want_cert, table_entry(d->flags, sizeof(T)));
    rgs_status st = RGS_OK;
    char* A = nullptr;
    if (fixed) {
        // as many step-1 columns per chunk as the fixed buffer leaves room for
        const size_t per_col = (size_t)pl.G_P * k * sizeof(double);
        pl = plan_qr(n, m, k, sk_kind, sizeof(T), false, 0, per_col);
        if (pl.total > fixed_bytes) return RGS_ESCRATCH;
        const size_t more = (fixed_bytes - pl.total) / std::max<size_t>(per_col, 1);
        pl = plan_qr(n, m, k, sk_kind, sizeof(T), false, 0, per_col * (1 + more));
        while (pl.total > fixed_bytes && pl.cc > 1)   // alignment padding
            pl = plan_qr(n, m, k, sk_kind, sizeof(T), false, 0, per_col * (size_t)(pl.cc - 1));
        if (pl.total > fixed_bytes) return RGS_ESCRATCH;
        A = fixed;
    } else {
        st = ensure_arena(h, pl.total);
        if (st != RGS_OK) return st;
        A = h->arena;
    }
    SketchArgs sk = make_sketch(sk_kind, k, d->seed, d->sketch_id, d->instance);
    st = setup_sketch(h, sk, n, reinterpret_cast<uint32_t*>(A + pl.signs), reinterpret_cast<int*>(A + pl.rows),
                      fixed != nullptr);
    if (st != RGS_OK) return st;
    if (tab && (st = use_table(h, sk, n, reinterpret_cast<uint16_t*>(A + pl.table))) != RGS_OK) return st;
    if (tabx && (st = use_tabx<T>(h, sk, n, reinterpret_cast<T*>(A + pl.table))) != RGS_OK) return st;

    SpaceArgs sa = space_args(A, pl, k, m);
    double* P = reinterpret_cast<double*>(A + pl.P);
    T* coef = reinterpret_cast<T*>(A + pl.coef);
    T* part = reinterpret_cast<T*>(A + pl.part_proj);
    // step 1 accumulates in fp64 (R-2), except on the bf16-basis path whose rounding dominates
    // and in the unique-precision model (float32 throughout)
    constexpr bool kUnique = std::is_same<TS, float>::value;
    using TP = typename std::conditional<DEFER || kUnique, T, double>::type;
    TP* partP = reinterpret_cast<TP*>(A + pl.part_P);

    hipStream_t s = h->stream;
    if (h->aux &&   // anything a failed call left on the auxiliary stream comes first
        (hipEventRecord(h->join_ev, h->aux) != hipSuccess || hipStreamWaitEvent(s, h->join_ev, 0) != hipSuccess))
        return RGS_EDEVICE;
    const bool graph = fixed == nullptr && (d->flags & RGS_FLAG_GRAPH) != 0;
    const bool timed = (d->flags & RGS_FLAG_TIME_KERNELS) != 0;   // never with a graph (rejected by the caller)
    if (timed && ensure_events(h, 2 * (size_t)m) != RGS_OK) return RGS_EDEVICE;
    const bool vec_ok = (ldq % 4 == 0) && (ldw % 4 == 0) && ((reinterpret_cast<uintptr_t>(Q) & 15) == 0) &&
                        ((reinterpret_cast<uintptr_t>(W) & 15) == 0);
    const double scale = sk_kind == SK_IDENT ? 1.0 : 1.0 / std::sqrt((double)k);
    const bool split = pl.G_col > 0;
    const int Gp = sk_kind == SK_IDENT ? 1 : (split ? pl.G_col : (int)pl.nproj);

    // The factorisation's device work, enqueued on stream q.  With `one`
    // (fixed scratch, or a graph being captured) everything runs on q: the
    // status words are cleared by a kernel (no memset node) and step 1 runs
    // chunk by chunk on q just before the column that first reads each chunk.
    auto enqueue = [&](hipStream_t q, bool one) -> rgs_status {
        if (one) {   // the status words: four ints
            if (!launch_zero_mat(q, reinterpret_cast<double*>(sa.status), 2, 1, 2)) return RGS_EDEVICE;
        } else if (hipMemsetAsync(sa.status, 0, 4 * sizeof(int), q) != hipSuccess) {
            return RGS_EDEVICE;
        }
        if (!launch_zero_mat(q, R, m, m, ldr)) return RGS_EDEVICE;

        // Step 1 for every column at once: P = Theta W, in chunks of pl.cc columns.
        // The first chunk runs on q; the others run on the auxiliary stream
        // beside the first columns' steps, whose latency-bound sketch-space
        // chains leave the device mostly idle.  Chunk c signals chunk_ev[c],
        // which the column loop waits for before the least squares that first
        // reads one of its columns.  The chunks share one partials buffer, so
        // the auxiliary stream starts after the first chunk.
        const int64_t nchunk = (m + pl.cc - 1) / pl.cc;
        rgs_status r1 = sketch_matrix<T, T, TP, TS>(h, sk, W, ldw, n, std::min<int64_t>(m, pl.cc), pl.G_P, pl.cc, partP, P,
                                                k, q);
        if (r1 != RGS_OK) return r1;
        if (nchunk > 1 && !one) {
            if (ensure_aux(h) != RGS_OK || ensure_chunk_events(h, (size_t)nchunk) != RGS_OK ||
                hipEventRecord(h->fork_ev, q) != hipSuccess || hipStreamWaitEvent(h->aux, h->fork_ev, 0) != hipSuccess)
                return RGS_EDEVICE;
            for (int64_t c = 1; c < nchunk; ++c) {
                const int64_t c0 = c * pl.cc;
                r1 = sketch_matrix<T, T, TP, TS>(h, sk, W + c0 * ldw, ldw, n, std::min<int64_t>(m - c0, pl.cc), pl.G_P,
                                             pl.cc, partP, P + c0 * k, k, h->aux);
                if (r1 != RGS_OK) return r1;
                if (hipEventRecord(h->chunk_ev[c], h->aux) != hipSuccess) return RGS_EDEVICE;
            }
        }

        for (int64_t i = 0; i < m; ++i) {
            // column i: step 3 (+4, + step 7 of column i-1) with the coefficients solved at the end
            // of column i-1, then steps 5-6, the Householder append of s_i and step 2 for column i+1
            const double* pnext = (i + 1 < m) ? P + (i + 1) * k : nullptr;
            if (timed) (void)hipEventRecord(h->events[2 * i], q);
            const bool sketch_col = DEFER || i > 0;
            if (split) {
                if (!launch_project_rows<T, TQ, DEFER>(q, W + i * ldw, Q, ldq, n, (int)i, coef,
                                                       i > 0 ? sa.invr + (i - 1) : nullptr,
                                                       (!DEFER && i > 0) ? 1 : 0, sa.status))
                    return RGS_EDEVICE;
            } else if (!launch_project<T, TQ, DEFER>(q, W + i * ldw, Q, ldq, n, (int)i, coef,
                                                     i > 0 ? sa.invr + (i - 1) : nullptr, (!DEFER && i > 0) ? 1 : 0,
                                                     sketch_col ? 1 : 0, vec_ok ? 1 : 0, sk, part, sa.status)) {
                return RGS_EDEVICE;
            }
            if (split && sketch_col && !launch_gauss_cols<TQ, T>(q, Q + i * ldq, ldq, n, 1, pl.G_col, sk, part))
                return RGS_EDEVICE;
            if (timed) (void)hipEventRecord(h->events[2 * i + 1], q);
            if (i + 1 < m && (i + 1) % pl.cc == 0) {   // the next column opens a chunk of P
                if (one) {
                    const int64_t c0 = i + 1;
                    r1 = sketch_matrix<T, T, TP, TS>(h, sk, W + c0 * ldw, ldw, n, std::min<int64_t>(m - c0, pl.cc),
                                                 pl.G_P, pl.cc, partP, P + c0 * k, k, q);
                    if (r1 != RGS_OK) return r1;
                } else if (hipStreamWaitEvent(q, h->chunk_ev[(i + 1) / pl.cc], 0) != hipSuccess) {
                    return RGS_EDEVICE;
                }
            }
            const double* src0 = (i == 0 && !DEFER) ? P : nullptr;
            const bool ok = d->ls_sweeps > 0
                                ? launch_column_richardson<T, T>(q, sa, part, Gp, scale, src0, (int)i, S, lds, R, ldr,
                                                                 pnext, coef, DEFER ? sa.invr : nullptr,
                                                                 (int)d->ls_sweeps)
                                : launch_column<T, T, TS>(q, sa, part, Gp, scale, src0, (int)i, S, lds, R, ldr, pnext,
                                                      coef, DEFER ? sa.invr : nullptr);
            if (!ok) return RGS_EDEVICE;
        }
        if constexpr (DEFER) {
            if (!launch_scale_cols_bf16(q, Q, ldq, n, (int)m, sa.invr, vec_ok ? 1 : 0, sa.status)) return RGS_EDEVICE;
        } else {
            if (!launch_scale_col<T>(q, Q + (m - 1) * ldq, n, sa.invr + (m - 1), sa.status)) return RGS_EDEVICE;
        }
        return RGS_OK;
    };

    if (graph) {
        // replay the captured work when every argument, the arena and its plan
        // are those it was captured for; otherwise capture it anew
        const std::vector<uint64_t> key = {
            (uint64_t)n, (uint64_t)m, (uint64_t)k, d->seed, d->sketch_id, d->instance, (uint64_t)d->sketch,
            (uint64_t)d->prec, d->flags, d->ls_sweeps, (uint64_t)(uintptr_t)W, (uint64_t)ldw,
            (uint64_t)(uintptr_t)Q, (uint64_t)ldq, (uint64_t)(uintptr_t)R, (uint64_t)ldr, (uint64_t)(uintptr_t)S,
            (uint64_t)lds, (uint64_t)(uintptr_t)A, (uint64_t)pl.total};
        if (!h->qr_exec || h->qr_key != key) {
            if (h->qr_exec) (void)hipGraphExecDestroy(h->qr_exec);
            if (h->qr_graph) (void)hipGraphDestroy(h->qr_graph);
            h->qr_exec = nullptr;
            h->qr_graph = nullptr;
            h->qr_key.clear();
            if (!h->capture && hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking) != hipSuccess)
                return RGS_EDEVICE;
            if (hipStreamBeginCapture(h->capture, hipStreamCaptureModeRelaxed) != hipSuccess) return RGS_EDEVICE;
            const rgs_status est = enqueue(h->capture, true);
            hipGraph_t gr = nullptr;
            const bool ended = hipStreamEndCapture(h->capture, &gr) == hipSuccess;
            if (est != RGS_OK || !ended || hipGraphInstantiate(&h->qr_exec, gr, nullptr, nullptr, 0) != hipSuccess) {
                if (gr) (void)hipGraphDestroy(gr);
                h->qr_exec = nullptr;
                (void)hipGetLastError();
                return est != RGS_OK ? est : RGS_EDEVICE;
            }
            h->qr_graph = gr;
            h->qr_key = key;
        }
        if (hipGraphLaunch(h->qr_exec, s) != hipSuccess) return RGS_EDEVICE;
    } else if ((st = enqueue(s, fixed != nullptr)) != RGS_OK) {
        return st;
    }

    double* diag = reinterpret_cast<double*>(A + pl.diag);
    const bool want_diag = (d->flags & RGS_FLAG_DIAGNOSTICS) != 0;
    if (want_diag && !launch_diagnostics(s, P, k, S, lds, R, ldr, (int)k, (int)m, diag, diag + m))
        return RGS_EDEVICE;

    int status[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(status, sa.status, sizeof(status), hipMemcpyDeviceToHost, s) != hipSuccess)
        return RGS_EDEVICE;
    std::vector<double> dh;
    if (want_diag) {
        dh.resize(3 * m);
        if (hipMemcpyAsync(dh.data(), diag, 3 * m * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
            return RGS_EDEVICE;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return RGS_EDEVICE;
    if (rep) report_defaults(rep);
    if (want_cert && status[0] == 0) {
        const rgs_status cs = certify<T, TQ>(h, d, pl, sk, W, ldw, Q, ldq, R, ldr, rep);
        if (cs != RGS_OK) return cs;
    }
    const auto t1 = std::chrono::steady_clock::now();
    if (rep) {
        rep->failed_column = status[0] ? status[1] : -1;
        rep->iters = status[0] ? status[1] : m;
        if (want_diag && status[0] == 0) {
            double g = 0, e = 0, p2 = 0;
            for (int64_t c = 0; c < m; ++c) {
                g += dh[c];
                e += dh[m + 2 * c];
                p2 += dh[m + 2 * c + 1];
            }
            rep->delta_F = std::sqrt(g);
            rep->delta_tilde_F = std::sqrt(e / p2);
        }
        rep->seconds = std::chrono::duration<double>(t1 - t0).count();
        rep->proj_launches = m;
        rep->proj_kernel_ms = 0.0;
        if (timed) {
            double tot = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, h->events[2 * i], h->events[2 * i + 1]);
                tot += ms;
            }
            rep->proj_kernel_ms = tot;
        }
    }
    if (status[0] == kStatusBreakdown) return RGS_EBREAKDOWN;
    if (status[0] == kStatusNonfinite) return RGS_ENONFINITE;
    return RGS_OK;
}


StencilArgs stencil_args(const rgs_stencil7* A) {
    StencilArgs s{};
    s.nx = A->nx;
    s.ny = A->ny;
    s.nz = A->nz;
    s.c[0] = A->c0;
    s.c[1] = A->cxm;
    s.c[2] = A->cxp;
    s.c[3] = A->cym;
    s.c[4] = A->cyp;
    s.c[5] = A->czm;
    s.c[6] = A->czp;
    return s;
}

// Restarted randomized GMRES (Sec. 4.2) driven from the host: one restart
// cycle is enqueued in full (its inner steps stop themselves on the device
// once converged), then the host synchronises once to read the true residual.
// TS: the arithmetic of the sketch space (fp64; float32 for the configuration
// of Sec. 5.3, unique-precision RGS, whose products with A are then computed
// in fp64 and rounded once to float32).
template <typename T, typename TQ, bool DEFER, typename TS = double>
rgs_status run_gmres(rgs_handle* h, const rgs_stencil7* Ad, const rgs_gmres_desc* d, const double* b, double* x,
                     double* res_hist, int64_t hist_cap, rgs_report* rep) {
    const auto t0 = std::chrono::steady_clock::now();
    const StencilArgs A = stencil_args(Ad);
    const int64_t n = A.nx * A.ny * A.nz, mcap = d->restart + 1, k = d->k;
    const int sk_kind = sketch_kind(d->sketch);
    const bool tab = (d->flags & RGS_FLAG_THETA_BF16) != 0;
    const bool tabx = (d->flags & RGS_FLAG_THETA_EXACT) != 0;
    const QrPlan pl = plan_qr(n, mcap, k, sk_kind, sizeof(T), false, table_entry(d->flags, sizeof(T)));
    Carver c;
    c.off = pl.total;
    const int64_t ldq = (n + 3) / 4 * 4;   // 16-byte aligned columns: every full block takes vector loads
    const size_t oQ = c.take<TQ>((size_t)ldq * mcap), oW = c.take<T>(n), oR = c.take<double>(mcap * mcap);
    const size_t oS = c.take<double>(k * mcap), oHr = c.take<double>(mcap * mcap), ocs = c.take<double>(mcap);
    const size_t osn = c.take<double>(mcap), ogv = c.take<double>(mcap + 1), oy = c.take<double>(mcap);
    const size_t ohist = c.take<double>(mcap), oused = c.take<int>(4), or_ = c.take<double>(n);
    const size_t opart = c.take<double>((n + 255) / 256), onorm = c.take<double>(4);
    // Gaussian: the two sketches of an Arnoldi step share their draws (the
    // mat-vec kernel sketches q'_i and A q'_i together), second partials buffer;
    // P-SRHT / Rademacher with RGS_FLAG_LAG: the same lagged step
    const bool dual = sk_kind == SK_GAUSS ||
                      ((d->flags & RGS_FLAG_LAG) != 0 && (sk_kind == SK_SRHT || sk_kind == SK_RADEM));
    const size_t opart2 = c.take<T>(dual ? pl.nproj * k : 1);
    // RGS_FLAG_CERTIFY: the certificate of the last cycle's basis
    const bool want_cert = (d->flags & RGS_FLAG_CERTIFY) != 0 && rep != nullptr;
    const size_t ocert = c.take<double>(want_cert ? 3 * k * mcap + 2 * mcap * mcap : 1);
    rgs_status st = ensure_arena(h, c.off + kAlign);
    if (st != RGS_OK) return st;
    char* Ar = h->arena;
    T* part2 = reinterpret_cast<T*>(Ar + opart2);
    SpaceArgs sa = space_args(Ar, pl, k, mcap);
    TQ* Q = reinterpret_cast<TQ*>(Ar + oQ);
    T* wbuf = reinterpret_cast<T*>(Ar + oW);
    double* R = reinterpret_cast<double*>(Ar + oR);
    double* S = reinterpret_cast<double*>(Ar + oS);
    double* Hr = reinterpret_cast<double*>(Ar + oHr);
    double* cs = reinterpret_cast<double*>(Ar + ocs);
    double* sn = reinterpret_cast<double*>(Ar + osn);
    double* gv = reinterpret_cast<double*>(Ar + ogv);
    double* y = reinterpret_cast<double*>(Ar + oy);
    double* hist = reinterpret_cast<double*>(Ar + ohist);
    int* used = reinterpret_cast<int*>(Ar + oused);
    double* r = reinterpret_cast<double*>(Ar + or_);
    double* rpart = reinterpret_cast<double*>(Ar + opart);
    double* norm = reinterpret_cast<double*>(Ar + onorm);
    T* coef = reinterpret_cast<T*>(Ar + pl.coef);
    T* part = reinterpret_cast<T*>(Ar + pl.part_proj);
    hipStream_t s = h->stream;
    const double scale = sk_kind == SK_IDENT ? 1.0 : 1.0 / std::sqrt((double)k);
    const int Gp = sk_kind == SK_IDENT ? 1 : (int)pl.nproj;
    const bool vec_ok = true;   // ldq % 4 == 0 and the arena is 256-byte aligned
    // step 2 of an Arnoldi step (Householder QR of S, or ls_sweeps Richardson
    // iterations on the normal equations) and steps 5-6 with the append of s_i
    const int sweeps = (int)d->ls_sweeps;
    auto ls_rhs = [&](const T* partials, int i, const double* scale2) {
        return sweeps > 0 ? launch_ls_partials_richardson<T, T>(s, sa, partials, Gp, scale, i, S, k, R, mcap, coef,
                                                                DEFER ? sa.invr : nullptr, scale2, sweeps)
                          : launch_ls_partials<T, T, TS>(s, sa, partials, Gp, scale, i, R, mcap, coef,
                                                         DEFER ? sa.invr : nullptr, scale2);
    };
    auto column = [&](int i) {
        return sweeps > 0 ? launch_column_richardson<T, T>(s, sa, part, Gp, scale, nullptr, i, S, k, R, mcap, nullptr,
                                                           coef, nullptr, sweeps)
                          : launch_column<T, T, TS>(s, sa, part, Gp, scale, nullptr, i, S, k, R, mcap, nullptr,
                                                    coef, nullptr);
    };
    // the arithmetic of the products with A
    using TC = typename std::conditional<std::is_same<TS, float>::value, double, T>::type;

    // x0 = 0, r0 = b, ||b||
    if (hipMemsetAsync(x, 0, n * sizeof(double), s) != hipSuccess) return RGS_EDEVICE;
    if (!launch_residual(s, A, b, x, r, rpart, norm)) return RGS_EDEVICE;
    double bnorm = 0.0;
    if (hipMemcpyAsync(&bnorm, norm, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return RGS_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return RGS_EDEVICE;
    int64_t iters = 0, cycles = 0, nhist = 0;
    double relres = bnorm > 0 ? 1.0 : 0.0;
    rgs_status result = RGS_OK;
    std::vector<double> hh((size_t)mcap);
    SketchArgs sk_last{};   // the last cycle's Theta and the basis vectors its update used
    int u_last = 0;
    while (bnorm > 0 && std::isfinite(bnorm)) {
        if (iters >= d->max_iters) {
            result = RGS_ENOCONV;
            break;
        }
        const uint32_t sid = d->reuse_theta ? 2u : (uint32_t)(2 + cycles);
        SketchArgs sk = make_sketch(sk_kind, k, d->seed, sid, 0);
        st = setup_sketch(h, sk, n, reinterpret_cast<uint32_t*>(Ar + pl.signs), reinterpret_cast<int*>(Ar + pl.rows));
        if (st != RGS_OK) return st;
        if (tab) {   // a fresh table per cycle, unless the cycles share Theta
            uint16_t* table = reinterpret_cast<uint16_t*>(Ar + pl.table);
            if (cycles == 0 || !d->reuse_theta) {
                if ((st = use_table(h, sk, n, table)) != RGS_OK) return st;
            } else {
                sk.sketch = SK_TABLE;
                sk.table = table;
            }
        } else if (tabx) {
            T* table = reinterpret_cast<T*>(Ar + pl.table);
            if (cycles == 0 || !d->reuse_theta) {
                if ((st = use_tabx<T>(h, sk, n, table)) != RGS_OK) return st;
            } else {
                sk.sketch = SK_TABX;
                sk.tabx = table;
            }
        }
        if (hipMemsetAsync(sa.status, 0, 4 * sizeof(int), s) != hipSuccess) return RGS_EDEVICE;
        // RGS step 1 of Algorithm 3: w_1 = r_0
        if (!launch_cast<T>(s, r, wbuf, n)) return RGS_EDEVICE;
        if (!launch_project<T, TQ, DEFER>(s, wbuf, Q, ldq, n, 0, coef, nullptr, 0, dual ? 0 : 1, vec_ok ? 1 : 0, sk,
                                          part, sa.status))
            return RGS_EDEVICE;
        // dual: t_1 = A q'_0 with the sketches of q'_0 (part) and t_1 (part2)
        if (dual && !launch_stencil_dual<TQ, T, TC>(s, A, Q, wbuf, sk, part, part2, sa.status)) return RGS_EDEVICE;
        if (!column(0)) return RGS_EDEVICE;
        if (!launch_givens_init(s, R, gv, used)) return RGS_EDEVICE;
        const int64_t steps = std::min<int64_t>(d->restart, d->max_iters - iters);
        for (int64_t ci = 1; ci <= steps; ++ci) {
            const int i = (int)ci;
            if (dual) {
                // p_i = Theta (A q'_{i-1}) / r_{i-1,i-1} and w_i = (A q'_{i-1}) / r_{i-1,i-1}
                if (!ls_rhs(part2, i, sa.invr + (i - 1))) return RGS_EDEVICE;
                if (!launch_project_ws<T, TQ, DEFER>(s, wbuf, Q, ldq, n, i, coef, sa.invr + (i - 1), DEFER ? 0 : 1,
                                                     vec_ok ? 1 : 0, sa.invr + (i - 1), sa.status))
                    return RGS_EDEVICE;
                if (!launch_stencil_dual<TQ, T, TC>(s, A, Q + i * ldq, wbuf, sk, part, part2, sa.status))
                    return RGS_EDEVICE;
            } else {
                // w_i = A q_{i-1}, sketched: p_i (step 3 of Algorithm 3, step 1 of Algorithm 2)
                if (!launch_stencil_sketch<TQ, T, TC>(s, A, Q + (i - 1) * ldq, sa.invr + (i - 1), wbuf, 1, sk,
                                                      part, sa.status))
                    return RGS_EDEVICE;
                if (!ls_rhs(part, i, nullptr)) return RGS_EDEVICE;
                if (!launch_project<T, TQ, DEFER>(s, wbuf, Q, ldq, n, i, coef, sa.invr + (i - 1), DEFER ? 0 : 1, 1,
                                                  vec_ok ? 1 : 0, sk, part, sa.status))
                    return RGS_EDEVICE;
            }
            if (!column(i)) return RGS_EDEVICE;
            if (!launch_givens(s, i, R, (int)mcap, Hr, cs, sn, gv, bnorm, d->tol, hist, sa.status, used,
                               (int)steps))
                return RGS_EDEVICE;
        }
        if (!launch_update_x<TQ>(s, Hr, (int)mcap, gv, used, y, x, Q, ldq, n, DEFER ? sa.invr : nullptr))
            return RGS_EDEVICE;
        if (!launch_residual(s, A, b, x, r, rpart, norm)) return RGS_EDEVICE;
        int stat[4] = {0, 0, 0, 0};
        int u = 0;
        double rn = 0.0;
        if (hipMemcpyAsync(stat, sa.status, sizeof(stat), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&u, used, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&rn, norm, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(hh.data(), hist, mcap * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
            return RGS_EDEVICE;
        if (hipStreamSynchronize(s) != hipSuccess) return RGS_EDEVICE;
        ++cycles;
        iters += u;
        sk_last = sk;
        u_last = u;
        for (int t = 0; t < u && nhist < hist_cap && res_hist; ++t) res_hist[nhist++] = hh[t];
        relres = rn / bnorm;
        if (stat[0] == kStatusNonfinite || !std::isfinite(rn)) {
            result = RGS_ENONFINITE;
            break;
        }
        if (relres <= d->tol) break;
        if (u == 0) {             // no inner step could run: breakdown of the very first column
            result = RGS_ENOCONV;
            break;
        }
    }
    if (!(bnorm > 0) && std::isfinite(bnorm)) relres = 0.0;
    if (!std::isfinite(bnorm)) result = RGS_ENONFINITE;
    const auto t1 = std::chrono::steady_clock::now();
    if (rep) {
        report_defaults(rep);
        rep->failed_column = -1;
        rep->iters = iters;
        rep->cycles = cycles;
        rep->delta_F = NAN;
        rep->delta_tilde_F = NAN;
        rep->true_relres = relres;
        rep->seconds = std::chrono::duration<double>(t1 - t0).count();
        rep->proj_kernel_ms = 0.0;
        rep->proj_launches = iters;
        if (want_cert && u_last > 0 && result != RGS_ENONFINITE) {
            // Phi: the same kind and size, counter word 2 = 1, which no cycle's Theta
            // uses (they take 2 + c); the Gaussian sketch for a bf16-table Theta
            const int phi_kind =
                (sk_last.sketch == SK_TABLE || sk_last.sketch == SK_TABX) ? SK_GAUSS : sk_last.sketch;
            const SketchArgs phi = make_sketch(phi_kind, k, d->seed, 1u, 0);
            st = certify_basis<TQ, T>(h, pl, sk_last, phi, Q, ldq, n, u_last, (int)k,
                                      reinterpret_cast<double*>(Ar + ocert), reinterpret_cast<double*>(Ar + pl.part_P),
                                      reinterpret_cast<uint32_t*>(Ar + pl.signs), reinterpret_cast<int*>(Ar + pl.rows),
                                      &rep->cert_smin_q, &rep->cert_smax_q, &rep->cert_cond_phi_q);
            if (st != RGS_OK) return st;
            rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
    }
    return result;
}

// ---------------------------------------------------------------------------
// Batched QR: every factorisation gets its own scratch; per column step the
// host-built maps list (factorisation, local block) for each launch.
// ---------------------------------------------------------------------------
bool valid_item(const rgs_qr_item& it, int sk_kind) {
    if (it.n < 1 || it.m < 1 || it.k < it.m || !it.W || !it.Q || !it.R || !it.S) return false;
    if (it.ldw < it.n || it.ldq < it.n || it.ldr < it.m || it.lds < it.k) return false;
    if (it.k > (int64_t)kKptMax * kWG || it.m > 4096) return false;
    if (sk_kind == SK_SRHT && (it.k > srht_order(it.n) || it.n > ((int64_t)1 << 31))) return false;
    if (sk_kind == SK_GAUSS && it.n > ((int64_t)1 << 34)) return false;
    return true;
}

// Prefix sums (count + 1 entries) of per-position block counts.
template <typename F>
std::vector<int64_t> prefix_of(int64_t count, F blocks) {
    std::vector<int64_t> p((size_t)count + 1, 0);
    for (int64_t q = 0; q < count; ++q) p[q + 1] = p[q] + blocks(q);
    return p;
}

// Runs f(b) for b in [0, count) on a few host threads (independent items).
// Joins every thread it started before returning or rethrowing the first
// exception of any of them.
template <typename F>
void parallel_for(int64_t count, F f) {
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(16, std::min<int64_t>(count / 64 + 1,
                                                                 (int64_t)std::thread::hardware_concurrency())));
    std::vector<std::exception_ptr> err((size_t)nt);
    auto body = [&](int64_t t) {
        try {
            for (int64_t b = t; b < count; b += nt) f(b);
        } catch (...) {
            err[(size_t)t] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    th.reserve((size_t)nt);
    try {
        for (int64_t t = 1; t < nt; ++t) th.emplace_back(body, t);
    } catch (...) {
        for (auto& x : th) x.join();
        throw;
    }
    body(0);
    for (auto& x : th) x.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

// Schedules of the batched Gaussian sketch product that the autotuner picks
// from: columns per work unit, and the order of the units in the launch --
// plain; XCD-grouped (xcd 1: the units of one (column tile, row chunk) pair,
// which read the same operand columns, are placed 8 apart so that the
// round-robin dispatch over the 8 XCDs puts them on the same L2); or
// chunk-affine (xcd 2: every unit of row chunk b goes to XCD b mod 8, chunk by
// chunk, tile by tile, so one L2 holds a chunk's sketch entries -- the bf16
// table's slice -- for all the column tiles that read it, and each tile's
// columns for all its sketch-row tiles).  Every schedule gives the same bits:
// each partial is one unit's fixed-order sum.
struct GemmSchedule {
    int tile, xcd;
};
constexpr int kNumSchedules = 9;
constexpr GemmSchedule kGemmSchedules[kNumSchedules] = {{64, 0},  {64, 1},  {32, 0},  {32, 1}, {64, 2},
                                                        {32, 2}, {128, 0}, {128, 1}, {128, 2}};
// Column-tile widths of the step-4 unit lists; unit list of a schedule's tile.
constexpr int kNumWidths = 3;
constexpr int kTileWidths[kNumWidths] = {64, 32, 128};
constexpr int width_index(int tile) { return tile == 64 ? 0 : tile == 32 ? 1 : 2; }

// Streams a batched QR call spreads its factorisations over, and a batched
// GMRES call its systems.
constexpr int kQrShares = 2;
constexpr int kGmresShares = 2;

// XCDs of the device: the dispatcher sends workgroup b of a launch to XCD
// b mod kXcds (a launch order built on it only affects cache reuse).
constexpr int kXcds = 8;

void order_units(const std::vector<GemmUnit>& in, size_t a, size_t b, int xcd, std::vector<GemmUnit>& out) {
    if (!xcd) {
        out.insert(out.end(), in.begin() + a, in.begin() + b);
        return;
    }
    std::vector<std::vector<GemmUnit>> q(8);
    if (xcd == 2) {   // queue = row chunk mod 8, ordered by chunk, then (as built) tile and sketch-row tile
        for (size_t u = a; u < b; ++u) q[in[u].blk % 8].push_back(in[u]);
        for (auto& qq : q)
            std::stable_sort(qq.begin(), qq.end(), [](const GemmUnit& x, const GemmUnit& y) { return x.blk < y.blk; });
    } else {   // group = consecutive units with the same (first, blk); queue = group index mod 8
        int g = -1;
        for (size_t u = a; u < b; ++u) {
            if (u == a || in[u].first != in[u - 1].first || in[u].blk != in[u - 1].blk) ++g;
            q[g % 8].push_back(in[u]);
        }
    }
    std::vector<size_t> pos(8, 0);
    for (size_t done = 0; done < b - a;)
        for (int x = 0; x < 8; ++x)
            if (pos[x] < q[x].size()) {
                out.push_back(q[x][pos[x]++]);
                ++done;
            }
}

// Workspace offsets of one factorisation of a batched QR call.
struct QrItemOff {
    size_t signs, part, partP, P, Vc, Vr, Wc, Wr, X, sp, u, v, pbuf, uh, pd, pdb, pd2, rr, invr, pnorm, tau, beta,
        coef;
};

// One stream's share of a batched QR call.  The call's factorisations are
// ordered by m (descending) and dealt out round-robin, so each share is in
// that order too: the factorisations of a share that still have a column i
// are a prefix of it, and every launch map is implicit.  The shares run the
// same per-column launch sequence on their own streams, so the latency-bound
// sketch-space kernels of one share overlap the HBM-bound projection of the
// other; each factorisation's arithmetic does not depend on the split.
struct QrGroup {
    std::vector<int64_t> order;   // indices into the caller's items
    int64_t max_m = 0;
    int64_t rows_p = 0;           // row chunk of the step-1 Gaussian product
    int tile_p = 0;               // operand columns per work unit of the step-1 Gaussian product
    std::vector<int> active;      // active[i]: factorisations with a column i
    std::vector<int64_t> pre_proj, pre_sl, pre_row, pre_sign, pre_part, pre_red;
    std::vector<QrItemOff> off;
    size_t o_rows = 0, o_status = 0, o_items = 0, o_pre = 0, o_gcols = 0, o_gunits_p = 0, o_gunits = 0,
           o_gtune = 0;
    // Gaussian: the step-1 product over (item, column) tiles, and per column the
    // active items ordered by n (descending) in tiles of 64, 32 or 128; each tile is
    // split into work units of one row chunk and 128 sketch rows
    std::vector<int2> g_cols;
    std::vector<GemmUnit> g_units_p;   // step 1
    std::vector<GemmUnit> g_units[kNumWidths];  // step 4, tile widths kTileWidths, all columns
    std::vector<size_t> g_at[kNumWidths];       // per column offsets into g_units[w]
    std::vector<BatchItem> bi;
    std::vector<int> rows_all;
    std::vector<int64_t> pre_all;
    std::vector<GemmUnit> sched_units;  // staged for an asynchronous copy: alive until the final synchronisation
    std::vector<int> stat;              // 4 status words per factorisation, read back at the end
};

// step-1 row groups: 4096-row blocks (SRHT, at most 16 groups), 16384-row
// chunks of the Gaussian product
int64_t qr_group_gp(int64_t n, int sk_kind, int64_t rows_p) {
    return sk_kind == SK_GAUSS ? (n + rows_p - 1) / rows_p : std::min<int64_t>((n + kBlock - 1) / kBlock, 16);
}

// step-4 block partials per column
int64_t qr_group_npart(int64_t n, int sk_kind) {
    return sk_kind == SK_GAUSS ? (n + kGemmRows - 1) / kGemmRows : (n + kProjRows - 1) / kProjRows;
}

// Launch tables and workspace layout of one share (g.order already set).
// table: the Gaussian products read the bf16 table; step 1 then runs over
// kGemmRows-row chunks in chunk-affine order (a chunk's table slice for every
// sketch-row tile fits one L2 beside a tile's columns), otherwise over
// kGemmRowsP-row chunks in the order built; both on 128-column tiles.
void plan_qr_group(QrGroup& g, const rgs_qr_item* items, int sk_kind, bool table, Carver& c) {
    g.rows_p = table ? kGemmRows : kGemmRowsP;
    g.tile_p = 128;   // 128 x 128 output tiles (kb_table_gemm_t128 / kb_gauss_gemm_t128)
    typedef float T;
    const int64_t cnt = (int64_t)g.order.size();
    auto it_of = [&](int64_t q) -> const rgs_qr_item& { return items[g.order[q]]; };
    g.max_m = it_of(0).m;
    g.active.assign((size_t)g.max_m + 1, 0);
    for (int64_t i = 0; i <= g.max_m; ++i)
        g.active[i] = (int)(std::upper_bound(g.order.begin(), g.order.end(), i,
                                             [&](int64_t v, int64_t b) { return v >= items[b].m; }) -
                            g.order.begin());
    g.pre_proj = prefix_of(cnt, [&](int64_t q) { return (it_of(q).n + kProjRows - 1) / kProjRows; });
    g.pre_sl = prefix_of(cnt, [&](int64_t q) { return (it_of(q).k + kSlice - 1) / kSlice; });
    g.pre_row = prefix_of(cnt, [&](int64_t q) { return (it_of(q).n + 1023) / 1024; });
    g.pre_sign = prefix_of(cnt, [&](int64_t q) { return ((it_of(q).n + 31) / 32 + 1023) / 1024; });
    g.pre_part = prefix_of(
        cnt, [&](int64_t q) { return sk_kind == SK_GAUSS ? 0 : qr_group_gp(it_of(q).n, sk_kind, g.rows_p) * it_of(q).m; });
    g.pre_red = prefix_of(cnt, [&](int64_t q) { return ((it_of(q).k + 31) / 32) * it_of(q).m; });
    g.off.resize((size_t)cnt);
    int64_t ktot = 0;
    for (int64_t q = 0; q < cnt; ++q) {
        const rgs_qr_item& it = it_of(q);
        const int64_t n = it.n, m = it.m, k = it.k;
        const int64_t nproj = (n + kProjRows - 1) / kProjRows, nsl = (k + kSlice - 1) / kSlice;
        QrItemOff& o = g.off[q];
        o.signs = c.take<uint32_t>(sk_kind == SK_SRHT ? (n + 31) / 32 + 4 : 1);
        o.part = c.take<T>(std::max<int64_t>(nproj, qr_group_npart(n, sk_kind)) * k);
        o.partP = c.take<double>(qr_group_gp(n, sk_kind, g.rows_p) * k * m);   // fp64 for SRHT, T for the Gaussian sketch
        o.P = c.take<double>(k * m);
        o.Vc = c.take<double>(k * m);
        o.Vr = c.take<double>(k * m);
        o.Wc = c.take<double>(k * m);
        o.Wr = c.take<double>(k * m);
        o.X = c.take<double>(m * m);
        o.sp = c.take<double>(k);
        o.u = c.take<double>(k);
        o.v = c.take<double>(k);
        o.pbuf = c.take<double>(k);
        o.uh = c.take<double>(m + 1);
        o.pd = c.take<double>(nsl * (m + 1));
        o.pdb = c.take<double>(nsl * (m + 2));
        o.pd2 = c.take<double>(nsl);
        o.rr = c.take<double>(m);
        o.invr = c.take<double>(m);
        o.pnorm = c.take<double>(m);
        o.tau = c.take<double>(m);
        o.beta = c.take<double>(m);
        o.coef = c.take<T>(m);
        ktot += k;
    }
    g.o_rows = c.take<int>(sk_kind == SK_SRHT ? ktot : 1);
    g.o_status = c.take<int>(4 * cnt);
    g.o_items = c.take<BatchItem>(cnt);
    g.o_pre = c.take<int64_t>(6 * (cnt + 1));
    if (sk_kind == SK_GAUSS) {
        auto add_tile = [&](std::vector<GemmUnit>& out, int first, int tcnt, int64_t rows) {
            int64_t nmax = 0, kmax = 0;
            for (int c2 = 0; c2 < tcnt; ++c2) {
                const rgs_qr_item& it = it_of(g.g_cols[first + c2].x);
                nmax = std::max<int64_t>(nmax, it.n);
                kmax = std::max<int64_t>(kmax, it.k);
            }
            for (int64_t blk = 0; blk < (nmax + rows - 1) / rows; ++blk)
                for (int64_t jt = 0; jt < (kmax + 127) / 128; ++jt)
                    out.push_back(GemmUnit{first, tcnt, (int)blk, (int)jt});
        };
        // Items in a tile share its draws of Z and its MFMA work, which runs over
        // the largest k (in steps of 32 sketch rows: one wave each) and the largest
        // n of the tile: tiles are cut from an order by k class, then n (descending)
        auto by_class = [&](int64_t kstep) {
            return [&, kstep](int64_t x, int64_t y) {
                const rgs_qr_item &a = it_of(x), &b = it_of(y);
                const int64_t ca = (a.k + kstep - 1) / kstep, cb = (b.k + kstep - 1) / kstep;
                return ca != cb ? ca > cb : a.n > b.n;
            };
        };
        {   // step 1: the columns of every W in tiles of tile_p that may span items
            std::vector<int64_t> ord((size_t)cnt);
            for (int64_t q = 0; q < cnt; ++q) ord[q] = q;
            std::stable_sort(ord.begin(), ord.end(), by_class(32));
            const int first0 = (int)g.g_cols.size();
            for (int64_t q : ord)
                for (int64_t c2 = 0; c2 < it_of(q).m; ++c2) g.g_cols.push_back(make_int2((int)q, (int)c2));
            const int total = (int)g.g_cols.size() - first0;
            for (int t0 = 0; t0 < total; t0 += g.tile_p)
                add_tile(g.g_units_p, first0 + t0, std::min(g.tile_p, total - t0), g.rows_p);
            if (table) {
                std::vector<GemmUnit> ord_units;
                order_units(g.g_units_p, 0, g.g_units_p.size(), 2, ord_units);
                g.g_units_p.swap(ord_units);
            }
        }
        std::vector<int> act;
        for (int w = 0; w < kNumWidths; ++w) g.g_at[w].assign((size_t)g.max_m + 1, 0);
        for (int64_t i = 0; i < g.max_m; ++i) {   // step 4 of column i: active items by k class of 128, then n
            const int a = g.active[i];
            act.resize((size_t)a);
            for (int q = 0; q < a; ++q) act[q] = q;
            std::stable_sort(act.begin(), act.end(), by_class(128));
            const int base = (int)g.g_cols.size();
            for (int q = 0; q < a; ++q) g.g_cols.push_back(make_int2(act[q], (int)i));
            for (int w = 0; w < kNumWidths; ++w) {
                const int tile = kTileWidths[w];
                for (int t0 = 0; t0 < a; t0 += tile) add_tile(g.g_units[w], base + t0, std::min(tile, a - t0), kGemmRows);
                g.g_at[w][i + 1] = g.g_units[w].size();
            }
        }
    }
    size_t n_units_max = 0, n_units_col1 = 0;   // all columns; the first two columns (the tuning step)
    for (int w = 0; w < kNumWidths; ++w) {
        n_units_max = std::max(n_units_max, g.g_units[w].size());
        n_units_col1 = std::max(n_units_col1, g.g_at[w].size() > 2 ? g.g_at[w][2] : (size_t)0);
    }
    g.o_gcols = c.take<int2>(std::max<size_t>(g.g_cols.size(), 1));
    g.o_gunits_p = c.take<GemmUnit>(std::max<size_t>(g.g_units_p.size(), 1));
    g.o_gunits = c.take<GemmUnit>(std::max<size_t>(n_units_max, 1));
    size_t tune_units = 1;
    if (sk_kind == SK_GAUSS)
        tune_units = kNumSchedules * std::max<size_t>(1, n_units_col1);
    g.o_gtune = c.take<GemmUnit>(tune_units);
}

// Device-side descriptors of one share's factorisations (arena at A).
template <bool DEFER>
void bind_qr_group(QrGroup& g, const rgs_qr_item* items, int sk_kind, uint64_t seed, uint32_t sid, char* A) {
    const int64_t cnt = (int64_t)g.order.size();
    const bool gemm = sk_kind == SK_GAUSS;
    g.bi.assign((size_t)cnt, BatchItem{});
    std::vector<int64_t> rpos((size_t)cnt + 1, 0);
    for (int64_t q = 0; q < cnt; ++q) rpos[q + 1] = rpos[q] + items[g.order[q]].k;
    g.rows_all.assign(sk_kind == SK_SRHT ? (size_t)rpos[cnt] : 0, 0);
    parallel_for(cnt, [&](int64_t q) {
        const rgs_qr_item& it = items[g.order[q]];
        const QrItemOff& o = g.off[q];
        BatchItem& x = g.bi[q];
        x.n = it.n;
        x.m = (int)it.m;
        x.k = (int)it.k;
        x.nproj = (int)((it.n + kProjRows - 1) / kProjRows);
        x.npart = (int)qr_group_npart(it.n, sk_kind);
        x.nsl = (int)((it.k + kSlice - 1) / kSlice);
        x.W = it.W;
        x.ldw = it.ldw;
        x.Q = it.Q;
        x.ldq = it.ldq;
        x.R = it.R;
        x.ldr = it.ldr;
        x.S = it.S;
        x.lds = it.lds;
        x.P = reinterpret_cast<double*>(A + o.P);
        x.partP = A + o.partP;
        x.G_P = (int)qr_group_gp(it.n, sk_kind, g.rows_p);
        x.part = A + o.part;
        x.coef = A + o.coef;
        x.sketch_scale = 1.0 / std::sqrt((double)it.k);
        x.vec_ok = (it.ldq % 4 == 0) && (it.ldw % 4 == 0) && ((reinterpret_cast<uintptr_t>(it.Q) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(it.W) & 15) == 0);
        x.defer = DEFER ? 1 : 0;
        x.gemm_sketch = gemm ? 1 : 0;
        SpaceArgs& a = x.sa;
        a.k = (int)it.k;
        a.mcap = (int)it.m;
        a.Vc = reinterpret_cast<double*>(A + o.Vc);
        a.Vr = reinterpret_cast<double*>(A + o.Vr);
        a.Wc = reinterpret_cast<double*>(A + o.Wc);
        a.Wr = reinterpret_cast<double*>(A + o.Wr);
        a.X = reinterpret_cast<double*>(A + o.X);
        a.sp = reinterpret_cast<double*>(A + o.sp);
        a.u = reinterpret_cast<double*>(A + o.u);
        a.v = reinterpret_cast<double*>(A + o.v);
        a.pbuf = reinterpret_cast<double*>(A + o.pbuf);
        a.uh = reinterpret_cast<double*>(A + o.uh);
        a.pd = reinterpret_cast<double*>(A + o.pd);
        a.pdb = reinterpret_cast<double*>(A + o.pdb);
        a.pd2 = reinterpret_cast<double*>(A + o.pd2);
        a.rr = reinterpret_cast<double*>(A + o.rr);
        a.invr = reinterpret_cast<double*>(A + o.invr);
        a.pnorm = reinterpret_cast<double*>(A + o.pnorm);
        a.tau = reinterpret_cast<double*>(A + o.tau);
        a.beta = reinterpret_cast<double*>(A + o.beta);
        a.status = reinterpret_cast<int*>(A + g.o_status) + 4 * q;
        // Theta of factorisation b: SRHT per factorisation (instance b, the
        // caller's index); Gaussian: the leading k_b x n_b block of one master
        // matrix (instance 0)
        x.sk = make_sketch(sk_kind, it.k, seed, sid, sk_kind == SK_SRHT ? (uint32_t)g.order[q] : 0u);
        if (sk_kind == SK_SRHT) {
            std::vector<int> rows;
            srht_rows_host(srht_order(it.n), (int)it.k, x.sk, rows);
            std::copy(rows.begin(), rows.end(), g.rows_all.begin() + rpos[q]);
            x.sk.signs = reinterpret_cast<uint32_t*>(A + o.signs);
            x.sk.rows = reinterpret_cast<int*>(A + g.o_rows) + rpos[q];
        }
    });
    g.pre_all.clear();
    g.pre_all.reserve(6 * (cnt + 1));
    for (const auto* v : {&g.pre_proj, &g.pre_sl, &g.pre_row, &g.pre_sign, &g.pre_part, &g.pre_red})
        g.pre_all.insert(g.pre_all.end(), v->begin(), v->end());
}

// Enqueues one share's factorisations on its stream: begin() uploads the
// tables and runs step 1, step(i) the launches of column i, end() the final
// scaling.  The caller interleaves the shares column by column, so both
// streams are fed from the start; nothing here waits for the device (a copy
// into pageable host memory would), except the schedule timing of the
// Gaussian product.
template <typename TQ, bool DEFER>
struct QrGroupLauncher {
    typedef float T;
    rgs_handle* h;
    QrGroup& g;
    int sk_kind;
    char* A;
    hipStream_t s;
    bool gemm = false;
    int nb = 0;
    int uploaded = 0;   // schedule whose unit order sits in d_units
    const BatchItem* itd = nullptr;
    const int64_t *d_proj = nullptr, *d_sl = nullptr, *d_row = nullptr, *d_sign = nullptr, *d_part = nullptr,
                  *d_red = nullptr;
    GemmUnit *d_units = nullptr, *d_tune = nullptr;
    const int2* d_cols = nullptr;
    // RGS_FLAG_THETA_BF16: the master matrix's bf16 entries (tk rows, tgroups groups of 8 columns);
    // RGS_FLAG_THETA_EXACT: its exact fp32 entries (tk rows, SK_TABX layout)
    const uint16_t* table = nullptr;
    const float* tabx = nullptr;
    int tk = 0;
    int64_t tgroups = 0;
    int sweeps = 0;   // step 2: 0 = Householder QR of S, else Richardson sweeps

    QrGroupLauncher(rgs_handle* h_, QrGroup& g_, int sk, char* A_, hipStream_t s_)
        : h(h_), g(g_), sk_kind(sk), A(A_), s(s_) {}

    // one product of the Gaussian sketch: drawn or exact-table entries (fp32 MFMA) or bf16 table entries
    // (bf16 MFMA)
    template <typename TB, bool STEP4>
    bool product(const GemmUnit* units, int nunits, int rows, int tile) {
        if (table)
            return launch_batch_table_gemm<TB, STEP4>(s, itd, units, nunits, d_cols, rows, tile, table, tk, tgroups);
        return launch_batch_gauss_gemm<TB, STEP4>(s, itd, units, nunits, d_cols, rows, tile, tabx, tk);
    }

    bool upload_schedule(int sc) {
        const int w = width_index(kGemmSchedules[sc - 1].tile);
        g.sched_units.clear();
        for (int64_t i = 0; i < g.max_m; ++i)
            order_units(g.g_units[w], g.g_at[w][i], g.g_at[w][i + 1], kGemmSchedules[sc - 1].xcd, g.sched_units);
        uploaded = sc;
        return hipMemcpyAsync(d_units, g.sched_units.data(), g.sched_units.size() * sizeof(GemmUnit),
                              hipMemcpyHostToDevice, s) == hipSuccess;
    }

    rgs_status begin(int sched) {
        const rgs_status st = upload(sched);
        return st != RGS_OK ? st : launch_first();
    }

    // The share's launch tables (host -> device copies, on stream s).
    rgs_status upload(int sched) {
        gemm = sk_kind == SK_GAUSS;
        nb = (int)g.order.size();
        if ((sk_kind == SK_SRHT && hipMemcpyAsync(A + g.o_rows, g.rows_all.data(), g.rows_all.size() * sizeof(int),
                                                  hipMemcpyHostToDevice, s) != hipSuccess) ||
            hipMemcpyAsync(A + g.o_items, g.bi.data(), g.bi.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(A + g.o_pre, g.pre_all.data(), g.pre_all.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                           s) != hipSuccess ||
            (gemm && (hipMemcpyAsync(A + g.o_gcols, g.g_cols.data(), g.g_cols.size() * sizeof(int2),
                                     hipMemcpyHostToDevice, s) != hipSuccess ||
                      hipMemcpyAsync(A + g.o_gunits_p, g.g_units_p.data(), g.g_units_p.size() * sizeof(GemmUnit),
                                     hipMemcpyHostToDevice, s) != hipSuccess)))
            return RGS_EDEVICE;
        itd = reinterpret_cast<const BatchItem*>(A + g.o_items);
        const int64_t* pre_dev = reinterpret_cast<const int64_t*>(A + g.o_pre);
        d_proj = pre_dev;
        d_sl = pre_dev + (nb + 1);
        d_row = pre_dev + 2 * (nb + 1);
        d_sign = pre_dev + 3 * (nb + 1);
        d_part = pre_dev + 4 * (nb + 1);
        d_red = pre_dev + 5 * (nb + 1);
        d_units = reinterpret_cast<GemmUnit*>(A + g.o_gunits);
        d_tune = reinterpret_cast<GemmUnit*>(A + g.o_gtune);
        d_cols = reinterpret_cast<const int2*>(A + g.o_gcols);
        // the copies come before the first launch: a copy from pageable host
        // memory can hold the host until the stream has drained
        if (gemm && sched > 0 && !upload_schedule(sched)) return RGS_EDEVICE;
        return RGS_OK;
    }

    // The launches before the first column: initialisation and step 1.
    rgs_status launch_first() {
        if (!launch_batch_init(s, itd, nb, g.max_m * g.max_m)) return RGS_EDEVICE;
        // step 1 for every column of every factorisation: P_b = Theta_b W_b (and the SRHT signs)
        if (gemm && !product<T, false>(reinterpret_cast<const GemmUnit*>(A + g.o_gunits_p), (int)g.g_units_p.size(),
                                       (int)g.rows_p, g.tile_p))
            return RGS_EDEVICE;
        if (!launch_batch_sketch_p<T>(s, sk_kind, itd, BlockMap{d_sign, nullptr, nb, 0}, g.pre_sign[nb],
                                      BlockMap{d_part, nullptr, nb, 0}, g.pre_part[nb],
                                      BlockMap{d_red, nullptr, nb, 0}, g.pre_red[nb], !DEFER))
            return RGS_EDEVICE;
        return RGS_OK;
    }

    // Column i (i < g.max_m).  sched: the Gaussian step-4 schedule; 0 = time
    // the six on this column's product (the first column that needs it),
    // keep the fastest and record it under sig.
    rgs_status step(int64_t i, int& sched, uint64_t sig) {
        const int a = g.active[i], a1 = g.active[i + 1];
        const int rb = (int)((i + 1 + 63) / 64);
        const int64_t i_tune = DEFER ? 0 : 1;
        if (!launch_batch_project<T, TQ, DEFER>(s, sk_kind, itd, BlockMap{d_proj, nullptr, a, 0}, g.pre_proj[a],
                                                (int)i))
            return RGS_EDEVICE;
        if (gemm && sched == 0 && i == i_tune) {
            std::vector<GemmUnit> tu[kNumSchedules];
            size_t off_t[kNumSchedules + 1] = {};
            for (int sc = 1; sc <= kNumSchedules; ++sc) {
                const int w = width_index(kGemmSchedules[sc - 1].tile);
                order_units(g.g_units[w], g.g_at[w][i], g.g_at[w][i + 1], kGemmSchedules[sc - 1].xcd, tu[sc - 1]);
                off_t[sc] = off_t[sc - 1] + tu[sc - 1].size();
                if (hipMemcpyAsync(d_tune + off_t[sc - 1], tu[sc - 1].data(), tu[sc - 1].size() * sizeof(GemmUnit),
                                   hipMemcpyHostToDevice, s) != hipSuccess)
                    return RGS_EDEVICE;
            }
            if (ensure_events(h, 2 * kNumSchedules) != RGS_OK) return RGS_EDEVICE;
            for (int rep2 = 0; rep2 < 2; ++rep2)   // the first round warms the caches
                for (int sc = 1; sc <= kNumSchedules; ++sc) {
                    (void)hipEventRecord(h->events[2 * sc - 2], s);
                    if (!product<TQ, true>(d_tune + off_t[sc - 1], (int)tu[sc - 1].size(), (int)kGemmRows,
                                           kGemmSchedules[sc - 1].tile))
                        return RGS_EDEVICE;
                    (void)hipEventRecord(h->events[2 * sc - 1], s);
                }
            if (hipStreamSynchronize(s) != hipSuccess) return RGS_EDEVICE;   // tu stays alive till here
            float best = 0.f;
            for (int sc = 1; sc <= kNumSchedules; ++sc) {
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, h->events[2 * sc - 2], h->events[2 * sc - 1]);
                if (sched == 0 || ms < best) {
                    best = ms;
                    sched = sc;
                }
            }
            h->gemm_tuned[sig] = sched;
        }
        if (gemm && (DEFER || i > 0)) {
            if (uploaded != sched && !upload_schedule(sched)) return RGS_EDEVICE;
            const int w = width_index(kGemmSchedules[sched - 1].tile);
            if (!product<TQ, true>(d_units + g.g_at[w][i], (int)(g.g_at[w][i + 1] - g.g_at[w][i]), (int)kGemmRows,
                                   kGemmSchedules[sched - 1].tile))
                return RGS_EDEVICE;
        }
        if (sweeps > 0) {
            const int rs = (int)((i + 1 + kRsumCoefs - 1) / kRsumCoefs);
            return launch_batch_column_richardson<T>(s, itd, BlockMap{d_sl, nullptr, a, 0}, g.pre_sl[a],
                                                     BlockMap{d_sl, nullptr, a1, 0}, g.pre_sl[a1],
                                                     BlockMap{nullptr, nullptr, a1, rs}, (int64_t)rs * a1, (int)i,
                                                     sweeps)
                       ? RGS_OK
                       : RGS_EDEVICE;
        }
        if (!launch_batch_column<T>(s, itd, BlockMap{d_sl, nullptr, a, 0}, g.pre_sl[a],
                                    BlockMap{d_sl, nullptr, a, rb}, g.pre_sl[a] + (int64_t)rb * a,
                                    BlockMap{nullptr, nullptr, a1, rb}, (int64_t)rb * a1, (int)i))
            return RGS_EDEVICE;
        return RGS_OK;
    }

    rgs_status end() {
        return launch_batch_scale<TQ, DEFER>(s, itd, BlockMap{d_row, nullptr, nb, 0}, g.pre_row[nb]) ? RGS_OK
                                                                                                     : RGS_EDEVICE;
    }
};

template <typename TQ, bool DEFER>
rgs_status run_qr_batched(rgs_handle* h, int64_t batch, const rgs_qr_item* items, int sk_kind, uint64_t seed,
                          uint32_t sid, bool use_table, bool use_tabx, int sweeps, bool want_graph,
                          int32_t* item_status, int64_t* failed_column, rgs_report* rep) {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<int64_t> order((size_t)batch);
    for (int64_t b = 0; b < batch; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return items[a].m > items[b].m; });
    const int ng = batch >= 2 ? kQrShares : 1;
    std::vector<QrGroup> grp((size_t)ng);
    for (int64_t q = 0; q < batch; ++q) grp[q % ng].order.push_back(order[q]);
    Carver c;
    for (QrGroup& g : grp) plan_qr_group(g, items, sk_kind, use_table, c);
    // RGS_FLAG_THETA_BF16: one table of the master matrix's bf16 entries,
    // rows 0 .. max k - 1, columns padded to whole 16-row k-steps of the product
    int tk = 0;
    int64_t tgroups = 0;
    size_t o_table = 0;
    if (use_table) {
        int64_t nmax = 0;
        for (int64_t b = 0; b < batch; ++b) {
            tk = std::max<int>(tk, (int)items[b].k);
            nmax = std::max<int64_t>(nmax, items[b].n);
        }
        tgroups = 2 * ((nmax + 15) / 16);
        o_table = c.take<uint16_t>((size_t)tgroups * 8 * (size_t)tk);
    }
    // RGS_FLAG_THETA_EXACT: the master matrix's fp32 entries, rows 0 .. max k - 1,
    // columns to the last 4-row draw any product reads (a 32-row super-step past n)
    int64_t tcols = 0;
    if (use_tabx) {
        int64_t nmax = 0;
        for (int64_t b = 0; b < batch; ++b) {
            tk = std::max<int>(tk, (int)items[b].k);
            nmax = std::max<int64_t>(nmax, items[b].n);
        }
        tcols = (nmax + 31) / 32 * 32 + 32;
        o_table = c.take<float>((size_t)tcols * (size_t)tk);
    }
    // the batch signature of the tuning cache: precision, sketch entries, shares and every (n, m, k)
    uint64_t sig = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { sig = (sig ^ v) * 1099511628211ull; };
    mix((uint64_t)DEFER);
    mix((uint64_t)use_table);
    mix((uint64_t)use_tabx);
    mix((uint64_t)ng);
    for (int64_t q = 0; q < batch; ++q) {
        mix((uint64_t)items[order[q]].n);
        mix((uint64_t)items[order[q]].m);
        mix((uint64_t)items[order[q]].k);
    }
    rgs_status st = ensure_arena(h, c.off + kAlign);
    if (st != RGS_OK) return st;
    char* A = h->arena;
    for (QrGroup& g : grp) bind_qr_group<DEFER>(g, items, sk_kind, seed, sid, A);
    const bool gemm = sk_kind == SK_GAUSS;
    // step-4 schedule: forced, cached for this batch signature, or tuned by the
    // first share at the first column that needs the product (the schedules
    // give the same bits, so the timing launches leave nothing behind)
    int sched = 0;
    if (gemm) {
        if (h->tune_mode > 0) sched = h->tune_mode;
        else if (h->gemm_tuned.count(sig)) sched = h->gemm_tuned[sig];
    }
    std::vector<QrGroupLauncher<TQ, DEFER>> run;
    for (int gi = 0; gi < ng; ++gi) {
        run.emplace_back(h, grp[gi], sk_kind, A, h->stream);
        run.back().sweeps = sweeps;
        if (use_table) {
            run.back().table = reinterpret_cast<const uint16_t*>(A + o_table);
            run.back().tk = tk;
            run.back().tgroups = tgroups;
        }
        if (use_tabx) {
            run.back().tabx = reinterpret_cast<const float*>(A + o_table);
            run.back().tk = tk;
        }
    }
    // RGS_FLAG_GRAPH: every share's kernel sequence (from its initialisation
    // to the closing scale pass) is captured once as a graph for this batch
    // signature, arena and schedule, and replayed on its stream; the launch
    // tables of both shares are copied eagerly, on the handle's stream, before
    // the first launch of the call.  A call whose Gaussian schedule is not
    // tuned yet runs eagerly (and tunes it).
    const bool use_graph = want_graph && (!gemm || sched > 0);
    for (int gi = 0; gi < ng && use_graph; ++gi)
        if ((st = run[gi].upload(sched)) != RGS_OK) return st;
    // the table is made on the handle's stream before the shares fork from it
    if (use_table && !launch_theta_table(h->stream, make_sketch(SK_GAUSS, tk, seed, sid, 0u), tgroups * 8,
                                         reinterpret_cast<uint16_t*>(A + o_table)))
        return RGS_EDEVICE;
    if (use_tabx && !launch_theta_tabx<float>(h->stream, make_sketch(SK_GAUSS, tk, seed, sid, 0u), tcols,
                                              reinterpret_cast<float*>(A + o_table)))
        return RGS_EDEVICE;
    static_assert(kQrShares == 2, "the shares past the first run on the one auxiliary stream");
    hipStream_t ss[kQrShares] = {h->stream, h->stream};
    if (ng > 1) {
        if (ensure_aux(h) != RGS_OK) return RGS_EDEVICE;
        ss[1] = h->aux;
        run[1].s = h->aux;
        if (hipEventRecord(h->fork_ev, h->stream) != hipSuccess || hipStreamWaitEvent(h->aux, h->fork_ev, 0) != hipSuccess)
            return RGS_EDEVICE;
    }
    rgs_status est = RGS_OK;
    if (use_graph) {
        std::vector<uint64_t> key = {sig, (uint64_t)sched, (uint64_t)(uintptr_t)A, (uint64_t)h->arena_bytes,
                                     (uint64_t)sk_kind, seed, sid, (uint64_t)use_table, (uint64_t)use_tabx,
                                     (uint64_t)sweeps, (uint64_t)ng};
        for (int64_t b = 0; b < batch; ++b) {
            const rgs_qr_item& it = items[b];
            for (uint64_t v : {(uint64_t)it.n, (uint64_t)it.m, (uint64_t)it.k, (uint64_t)(uintptr_t)it.W,
                               (uint64_t)it.ldw, (uint64_t)(uintptr_t)it.Q, (uint64_t)it.ldq,
                               (uint64_t)(uintptr_t)it.R, (uint64_t)it.ldr, (uint64_t)(uintptr_t)it.S,
                               (uint64_t)it.lds})
                key.push_back(v);
        }
        if (h->qrb_key != key) {
            for (int gi = 0; gi < 2; ++gi) {
                if (h->qrb_exec[gi]) (void)hipGraphExecDestroy(h->qrb_exec[gi]);
                if (h->qrb_graph[gi]) (void)hipGraphDestroy(h->qrb_graph[gi]);
                h->qrb_exec[gi] = nullptr;
                h->qrb_graph[gi] = nullptr;
            }
            h->qrb_key.clear();
            if (!h->capture && hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking) != hipSuccess)
                est = RGS_EDEVICE;
            for (int gi = 0; gi < ng && est == RGS_OK; ++gi) {
                QrGroupLauncher<TQ, DEFER>& L = run[gi];
                L.s = h->capture;
                if (hipStreamBeginCapture(h->capture, hipStreamCaptureModeRelaxed) != hipSuccess) {
                    est = RGS_EDEVICE;
                    break;
                }
                est = L.launch_first();
                for (int64_t i = 0; i < grp[gi].max_m && est == RGS_OK; ++i) est = L.step(i, sched, sig);
                if (est == RGS_OK) est = L.end();
                L.s = ss[gi];
                hipGraph_t gr = nullptr;
                const bool ended = hipStreamEndCapture(h->capture, &gr) == hipSuccess;
                if (est == RGS_OK &&
                    (!ended || hipGraphInstantiate(&h->qrb_exec[gi], gr, nullptr, nullptr, 0) != hipSuccess))
                    est = RGS_EDEVICE;
                h->qrb_graph[gi] = gr;
                if (est != RGS_OK) (void)hipGetLastError();
            }
            if (est == RGS_OK) h->qrb_key = key;
        }
        for (int gi = 0; gi < ng && est == RGS_OK; ++gi)
            if (hipGraphLaunch(h->qrb_exec[gi], ss[gi]) != hipSuccess) est = RGS_EDEVICE;
    } else {
        est = run[0].begin(sched);
    // an untuned Gaussian product: share 0 (it holds the largest m) runs alone
    // up to the column whose product it times, so the timing sees no other work
    int64_t done0 = 0;
    if (gemm && sched == 0)
        for (const int64_t i_tune = DEFER ? 0 : 1; done0 <= i_tune && done0 < grp[0].max_m && est == RGS_OK; ++done0)
            est = run[0].step(done0, sched, sig);
    for (int gi = 1; gi < ng && est == RGS_OK; ++gi) est = run[gi].begin(sched);
    // then column by column over the shares
    for (int64_t i = 0; i < grp[0].max_m && est == RGS_OK; ++i)
        for (int gi = 0; gi < ng && est == RGS_OK; ++gi)
            if (i < grp[gi].max_m && (gi > 0 || i >= done0)) est = run[gi].step(i, sched, sig);
    for (int gi = 0; gi < ng && est == RGS_OK; ++gi) est = run[gi].end();
    }
    if (ng > 1) {   // join (also after a failed enqueue, so no work is left behind unordered)
        if (hipEventRecord(h->join_ev, h->aux) != hipSuccess || hipStreamWaitEvent(h->stream, h->join_ev, 0) != hipSuccess)
            est = RGS_EDEVICE;
    }
    for (QrGroup& g : grp) {   // the status words, once every share has finished
        g.stat.assign(4 * g.order.size(), 0);
        if (est == RGS_OK && hipMemcpyAsync(g.stat.data(), A + g.o_status, g.stat.size() * sizeof(int),
                                            hipMemcpyDeviceToHost, h->stream) != hipSuccess)
            est = RGS_EDEVICE;
    }
    // host staging vectors stay alive till here
    if (hipStreamSynchronize(h->stream) != hipSuccess) return RGS_EDEVICE;
    if (est != RGS_OK) return est;
    std::vector<rgs_status> sb((size_t)batch, RGS_OK);
    std::vector<int64_t> fc((size_t)batch, -1);
    for (const QrGroup& g : grp)
        for (size_t q = 0; q < g.order.size(); ++q) {
            const int code = g.stat[4 * q];
            sb[g.order[q]] = code == kStatusBreakdown   ? RGS_EBREAKDOWN
                             : code == kStatusNonfinite ? RGS_ENONFINITE
                                                        : RGS_OK;
            if (code) fc[g.order[q]] = g.stat[4 * q + 1];
        }
    rgs_status result = RGS_OK;
    for (int64_t b = 0; b < batch; ++b) {
        if (item_status) item_status[b] = sb[b];
        if (failed_column) failed_column[b] = fc[b];
        if (sb[b] != RGS_OK && result == RGS_OK) result = sb[b];
    }
    if (gemm) h->last_schedule = sched;
    const auto t1 = std::chrono::steady_clock::now();
    if (rep) {
        report_defaults(rep);
        rep->failed_column = -1;
        rep->iters = items[order[0]].m;
        rep->cycles = 0;
        rep->delta_F = NAN;
        rep->delta_tilde_F = NAN;
        rep->true_relres = NAN;
        rep->seconds = std::chrono::duration<double>(t1 - t0).count();
        rep->proj_kernel_ms = 0.0;
        rep->proj_launches = items[order[0]].m;
    }
    return result;
}

// ---------------------------------------------------------------------------
// Batched randomized GMRES.  The systems advance in lockstep, one restart
// cycle at a time: a cycle is one launch sequence over the systems still
// running (optionally captured once as a HIP graph and replayed while that set
// does not change).  Inside a cycle each system stops itself on the device
// (converged, lucky breakdown, or its step limit); between cycles the host
// reads every system's status, step count and true residual.  Every system
// uses the sketch instance 0 with its own n, exactly as a separate rgs_gmres
// call on it, so the batched solve reproduces separate solves bit for bit.
// ---------------------------------------------------------------------------
bool grid_size(const rgs_stencil7& A, int64_t* n) {
    if (A.nx < 1 || A.ny < 1 || A.nz < 1) return false;
    const double nd = (double)A.nx * (double)A.ny * (double)A.nz;
    if (!(nd <= (double)(((int64_t)1 << 31) - 1))) return false;
    *n = A.nx * A.ny * A.nz;
    return true;
}

// The tables of Theta: GAUSSIAN only, at most one of the two.
bool valid_table_flags(uint32_t flags, int32_t sketch) {
    const uint32_t t = flags & (RGS_FLAG_THETA_BF16 | RGS_FLAG_THETA_EXACT);
    if (t == 0) return true;
    return sketch == RGS_SKETCH_GAUSSIAN && t != (RGS_FLAG_THETA_BF16 | RGS_FLAG_THETA_EXACT);
}

bool valid_gmres_desc(const rgs_gmres_desc* d) {
    if (!d) return false;
    if (d->restart < 1 || d->restart + 1 > d->k || d->restart > 4000 || d->max_iters < 1 || !(d->tol >= 0))
        return false;
    if (d->ls_sweeps > kMaxSweeps) return false;
    // the unique-precision float32 chain is Householder only
    if (d->prec == RGS_P_FP32) return d->ls_sweeps == 0;
    return d->prec == RGS_P_FP64 || d->prec == RGS_P_FP32_LS64 || d->prec == RGS_P_BF16Q_FP32_LS64;
}

// Implicit launch maps of the systems still running (ids = their indices):
// per-system 256-row blocks and projection blocks as prefix sums; the other
// launches have the same number of blocks for every system.
struct GmresMaps {
    std::vector<int> ids;
    std::vector<int64_t> row, proj;   // prefix sums over the listed systems
    // the (row block, system) pairs of the projection blocks, for the launch
    // whose systems share a row block's data: pairs[j kXcds + x] is the j-th
    // pair, in r order, of the row blocks r with r mod kXcds = x, so each row
    // block stays on one XCD; (-1, -1) marks an idle slot
    std::vector<int2> pairs;
    int nsl = 0;
    int count() const { return (int)ids.size(); }
};

void build_gmres_maps(GmresMaps& g, const std::vector<int64_t>& active, const std::vector<int64_t>& ns, int64_t k) {
    g.ids.assign(active.begin(), active.end());
    g.row = prefix_of((int64_t)active.size(), [&](int64_t p) { return (ns[active[p]] + 255) / 256; });
    g.proj = prefix_of((int64_t)active.size(), [&](int64_t p) { return (ns[active[p]] + kProjRows - 1) / kProjRows; });
    std::vector<std::vector<int2>> lane((size_t)kXcds);
    for (int64_t r = 0;; ++r) {
        bool any = false;
        for (int64_t b : active)
            if (r * kProjRows < ns[b]) {
                lane[r % kXcds].push_back(make_int2((int)r, (int)b));
                any = true;
            }
        if (!any) break;
    }
    size_t len = 0;
    for (const auto& l : lane) len = std::max(len, l.size());
    g.pairs.assign(len * kXcds, make_int2(-1, -1));
    for (int x = 0; x < kXcds; ++x)
        for (size_t j = 0; j < lane[x].size(); ++j) g.pairs[j * kXcds + x] = lane[x][j];
    g.nsl = (int)((k + kSlice - 1) / kSlice);
}

// TS: the sketch-space arithmetic, fp64, or float32 in the unique-precision
// model (RGS_P_FP32), whose products with A run in fp64 (TC) from the float32
// basis vectors, as in rgs_gmres
template <typename T, typename TQ, bool DEFER, typename TS = double>
rgs_status run_gmres_batched(rgs_handle* h, int64_t batch, const rgs_gmres_item* items, const rgs_gmres_desc* d,
                             int32_t* item_status, rgs_report* reps) {
    using TC = typename std::conditional<std::is_same<TS, float>::value, double, T>::type;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = h->stream;
    const int sk_kind = sketch_kind(d->sketch);
    const int64_t restart = d->restart, mcap = restart + 1, k = d->k;
    const int64_t nsl = (k + kSlice - 1) / kSlice;
    const bool use_graph = (d->flags & RGS_FLAG_GRAPH) != 0;
    // Gaussian sketch with bf16 entries: entry (j, l) does not depend on n, so
    // one table over the largest n serves every system of the cycle
    const bool tab = (d->flags & RGS_FLAG_THETA_BF16) != 0;
    // RGS_FLAG_LAG with the P-SRHT: the lagged step (the Gaussian sketch takes it anyway)
    const bool lag = (d->flags & RGS_FLAG_LAG) != 0 && sk_kind == SK_SRHT;
    std::vector<int64_t> ns((size_t)batch);
    for (int64_t b = 0; b < batch; ++b) grid_size(items[b].A, &ns[b]);
    const int64_t nmax = *std::max_element(ns.begin(), ns.end());

    // scratch of every system, carved from the handle's arena
    struct Off {
        size_t Q, w, r, rpart, R, S, part, part2, coef, Vc, Vr, Wc, Wr, X, sp, u, v, pbuf, uh, pd, pdb, pd2, rr, invr, pnorm,
            tau, beta, Hr, cs, sn, gv, y, signs;
    };
    std::vector<Off> off((size_t)batch);
    Carver c;
    for (int64_t b = 0; b < batch; ++b) {
        const int64_t n = ns[b], nproj = (n + kProjRows - 1) / kProjRows;
        Off& o = off[b];
        o.Q = c.take<TQ>((size_t)((n + 3) / 4 * 4) * mcap);
        o.w = c.take<T>(n);
        o.r = c.take<double>(n);
        o.rpart = c.take<double>((n + 255) / 256);
        o.R = c.take<double>(mcap * mcap);
        o.S = c.take<double>(k * mcap);
        o.part = c.take<T>(nproj * k);
        o.part2 = c.take<T>(sk_kind == SK_GAUSS || lag ? nproj * k : 1);
        o.coef = c.take<T>(mcap);
        o.Vc = c.take<double>(k * mcap);
        o.Vr = c.take<double>(k * mcap);
        o.Wc = c.take<double>(k * mcap);
        o.Wr = c.take<double>(k * mcap);
        o.X = c.take<double>(mcap * mcap);
        o.sp = c.take<double>(k);
        o.u = c.take<double>(k);
        o.v = c.take<double>(k);
        o.pbuf = c.take<double>(k);
        o.uh = c.take<double>(mcap + 1);
        o.pd = c.take<double>(nsl * (mcap + 1));
        o.pdb = c.take<double>(nsl * (mcap + 2));
        o.pd2 = c.take<double>(nsl);
        o.rr = c.take<double>(mcap);
        o.invr = c.take<double>(mcap);
        o.pnorm = c.take<double>(mcap);
        o.tau = c.take<double>(mcap);
        o.beta = c.take<double>(mcap);
        o.Hr = c.take<double>(mcap * mcap);
        o.cs = c.take<double>(mcap);
        o.sn = c.take<double>(mcap);
        o.gv = c.take<double>(mcap + 1);
        o.y = c.take<double>(mcap);
        o.signs = sk_kind == SK_SRHT ? c.take<uint32_t>((n + 31) / 32 + 4) : 0;
    }
    const size_t o_rows = c.take<int>(sk_kind == SK_SRHT ? k * batch : 1);
    const size_t o_status = c.take<int>(4 * batch), o_used = c.take<int>(batch), o_limit = c.take<int>(batch);
    const size_t o_norm = c.take<double>(batch), o_hist = c.take<double>(batch * mcap);
    const size_t o_items = c.take<BatchItem>(batch), o_gitems = c.take<GmresItem>(batch);
    const size_t o_table = c.take<uint16_t>(tab ? (size_t)((nmax + 7) / 8) * 8 * k : 1);
    std::vector<int64_t> all((size_t)batch);
    for (int64_t b = 0; b < batch; ++b) all[b] = b;
    GmresMaps gm;
    build_gmres_maps(gm, all, ns, k);
    const size_t o_ids = c.take<int>(batch), o_mrow = c.take<int64_t>(batch + 1);
    const size_t o_mproj = c.take<int64_t>(batch + 1);
    // pair list: at most kXcds x (the blocks of the XCD with the most)
    const size_t o_pairs = c.take<int2>((size_t)kXcds * (gm.proj[gm.count()] + (nmax + kProjRows - 1) / kProjRows));
    // the running systems of a cycle are dealt out, by n, into two shares that
    // run their launch sequences on two streams (the handle's and the
    // auxiliary one): one share's latency-bound sketch-space kernels then run
    // beside the other's HBM-bound passes.  Each system's arithmetic does not
    // depend on the split.
    struct GShare {
        GmresMaps gm;
        size_t o_ids = 0, o_mrow = 0, o_mproj = 0, o_pairs = 0;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        std::vector<int64_t> active;
    };
    GShare sh[kGmresShares];
    for (GShare& g : sh) {
        g.o_ids = c.take<int>(batch);
        g.o_mrow = c.take<int64_t>(batch + 1);
        g.o_mproj = c.take<int64_t>(batch + 1);
        g.o_pairs = c.take<int2>((size_t)kXcds * (gm.proj[gm.count()] + (nmax + kProjRows - 1) / kProjRows));
    }
    rgs_status st = ensure_arena(h, c.off + kAlign);
    if (st != RGS_OK) return st;
    char* A = h->arena;

    std::vector<BatchItem> bi((size_t)batch);
    std::vector<GmresItem> gi((size_t)batch);
    for (int64_t b = 0; b < batch; ++b) {
        const Off& o = off[b];
        const int64_t n = ns[b];
        BatchItem& x = bi[b];
        x = BatchItem{};
        x.n = n;
        x.m = (int)mcap;
        x.k = (int)k;
        x.nproj = (int)((n + kProjRows - 1) / kProjRows);
        x.npart = x.nproj;
        x.nsl = (int)nsl;
        x.Q = A + o.Q;
        x.ldq = (n + 3) / 4 * 4;   // 16-byte aligned columns
        x.R = reinterpret_cast<double*>(A + o.R);
        x.ldr = mcap;
        x.S = reinterpret_cast<double*>(A + o.S);
        x.lds = k;
        x.P = nullptr;
        x.part = A + o.part;
        x.part2 = A + o.part2;
        x.coef = A + o.coef;
        x.sketch_scale = 1.0 / std::sqrt((double)k);
        x.vec_ok = 1;
        x.defer = DEFER ? 1 : 0;
        SpaceArgs& a = x.sa;
        a.k = (int)k;
        a.mcap = (int)mcap;
        a.Vc = reinterpret_cast<double*>(A + o.Vc);
        a.Vr = reinterpret_cast<double*>(A + o.Vr);
        a.Wc = reinterpret_cast<double*>(A + o.Wc);
        a.Wr = reinterpret_cast<double*>(A + o.Wr);
        a.X = reinterpret_cast<double*>(A + o.X);
        a.sp = reinterpret_cast<double*>(A + o.sp);
        a.u = reinterpret_cast<double*>(A + o.u);
        a.v = reinterpret_cast<double*>(A + o.v);
        a.pbuf = reinterpret_cast<double*>(A + o.pbuf);
        a.uh = reinterpret_cast<double*>(A + o.uh);
        a.pd = reinterpret_cast<double*>(A + o.pd);
        a.pdb = reinterpret_cast<double*>(A + o.pdb);
        a.pd2 = reinterpret_cast<double*>(A + o.pd2);
        a.rr = reinterpret_cast<double*>(A + o.rr);
        a.invr = reinterpret_cast<double*>(A + o.invr);
        a.pnorm = reinterpret_cast<double*>(A + o.pnorm);
        a.tau = reinterpret_cast<double*>(A + o.tau);
        a.beta = reinterpret_cast<double*>(A + o.beta);
        a.status = reinterpret_cast<int*>(A + o_status) + 4 * b;
        x.sk = make_sketch(sk_kind, k, d->seed, 2, 0);
        if (tab) {
            x.sk.sketch = SK_TABLE;
            x.sk.table = reinterpret_cast<uint16_t*>(A + o_table);
        }
        if (sk_kind == SK_SRHT) {
            x.sk.signs = reinterpret_cast<uint32_t*>(A + o.signs);
            x.sk.rows = reinterpret_cast<int*>(A + o_rows) + b * k;
        }
        GmresItem& g = gi[b];
        g = GmresItem{};
        g.n = n;
        g.A = stencil_args(&items[b].A);
        g.b = items[b].b;
        g.x = items[b].x;
        g.r = reinterpret_cast<double*>(A + o.r);
        g.w = A + o.w;
        g.rpart = reinterpret_cast<double*>(A + o.rpart);
        g.norm = reinterpret_cast<double*>(A + o_norm) + b;
        g.tol = d->tol;
        g.Hr = reinterpret_cast<double*>(A + o.Hr);
        g.cs = reinterpret_cast<double*>(A + o.cs);
        g.sn = reinterpret_cast<double*>(A + o.sn);
        g.gv = reinterpret_cast<double*>(A + o.gv);
        g.y = reinterpret_cast<double*>(A + o.y);
        g.hist = reinterpret_cast<double*>(A + o_hist) + b * mcap;
        g.used = reinterpret_cast<int*>(A + o_used) + b;
        g.limit = reinterpret_cast<int*>(A + o_limit) + b;
    }
    BatchItem* itd = reinterpret_cast<BatchItem*>(A + o_items);
    GmresItem* gid = reinterpret_cast<GmresItem*>(A + o_gitems);
    // maps of a set of systems (gm at arena offsets o): their ids, 256-row
    // blocks, projection blocks and (row block, system) pairs
    struct MapAt {
        const GmresMaps& gm;
        const int* ids;
        const int64_t *row, *proj;
        const int2* pairs;
    };
    auto map_at = [&](const GmresMaps& m, size_t oi, size_t orow, size_t oproj, size_t opairs) {
        return MapAt{m, reinterpret_cast<const int*>(A + oi), reinterpret_cast<const int64_t*>(A + orow),
                     reinterpret_cast<const int64_t*>(A + oproj), reinterpret_cast<const int2*>(A + opairs)};
    };
    auto upload = [&](const GmresMaps& m, size_t oi, size_t orow, size_t oproj, size_t opairs) -> bool {
        return hipMemcpyAsync(A + oi, m.ids.data(), m.ids.size() * sizeof(int), hipMemcpyHostToDevice, s) ==
                   hipSuccess &&
               hipMemcpyAsync(A + opairs, m.pairs.data(), m.pairs.size() * sizeof(int2), hipMemcpyHostToDevice, s) ==
                   hipSuccess &&
               hipMemcpyAsync(A + orow, m.row.data(), m.row.size() * sizeof(int64_t), hipMemcpyHostToDevice, s) ==
                   hipSuccess &&
               hipMemcpyAsync(A + oproj, m.proj.data(), m.proj.size() * sizeof(int64_t), hipMemcpyHostToDevice, s) ==
                   hipSuccess;
    };
    // launch maps over a set of systems: one block per system, 256-row blocks,
    // projection blocks, sketch slices (+ rb row blocks of the least squares)
    auto m_sys = [](const MapAt& M) { return BlockMap{nullptr, M.ids, M.gm.count(), 1}; };
    auto m_row = [](const MapAt& M) { return BlockMap{M.row, M.ids, M.gm.count(), 0}; };
    auto m_proj = [](const MapAt& M) { return BlockMap{M.proj, M.ids, M.gm.count(), 0}; };
    auto m_uni = [](const MapAt& M, int per) { return BlockMap{nullptr, M.ids, M.gm.count(), per}; };
    auto n_row = [](const MapAt& M) { return M.gm.row[M.gm.count()]; };
    auto n_proj = [](const MapAt& M) { return M.gm.proj[M.gm.count()]; };
    auto n_uni = [](const MapAt& M, int per) { return (int64_t)per * M.gm.count(); };
    const MapAt every = map_at(gm, o_ids, o_mrow, o_mproj, o_pairs);
    if (hipMemcpyAsync(A + o_gitems, gi.data(), gi.size() * sizeof(GmresItem), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        !upload(gm, o_ids, o_mrow, o_mproj, o_pairs))
        return RGS_EDEVICE;
    // x0 = 0, r0 = b, ||b|| of every system
    if (!launch_gbatch_zero_x(s, gid, m_row(every), n_row(every)) ||
        !launch_gbatch_residual(s, gid, m_sys(every), gm.count(), m_row(every), n_row(every)))
        return RGS_EDEVICE;
    std::vector<double> bn((size_t)batch), rn((size_t)batch), hh((size_t)(batch * mcap));
    if (hipMemcpyAsync(bn.data(), A + o_norm, batch * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
        return RGS_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return RGS_EDEVICE;   // host vectors above stay alive till here
    for (int64_t b = 0; b < batch; ++b) gi[b].bnorm = bn[b];
    if (hipMemcpyAsync(A + o_gitems, gi.data(), gi.size() * sizeof(GmresItem), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return RGS_EDEVICE;

    std::vector<int64_t> iters((size_t)batch, 0), cycles((size_t)batch, 0), nhist((size_t)batch, 0);
    std::vector<double> relres((size_t)batch, 1.0);
    std::vector<rgs_status> res((size_t)batch, RGS_OK);
    std::vector<char> done((size_t)batch, 0);
    for (int64_t b = 0; b < batch; ++b) {
        if (!std::isfinite(bn[b])) {
            res[b] = RGS_ENONFINITE;
            done[b] = 1;
        } else if (!(bn[b] > 0)) {
            relres[b] = 0.0;
            done[b] = 1;
        }
    }
    std::vector<int> lim((size_t)batch, 0), stat((size_t)(4 * batch)), usedh((size_t)batch);
    std::vector<int> rows_all;
    std::vector<int64_t> active, prev_active;
    auto drop_graph = [](GShare& g) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        g.exec = nullptr;
        g.graph = nullptr;
    };
    auto drop_graphs = [&]() {
        for (GShare& g : sh) drop_graph(g);
    };
    // the two sketches of an Arnoldi step in the mat-vec pass: the Gaussian sketch
    // (they share their draws), or the P-SRHT with the lagged step
    const bool dual = sk_kind == SK_GAUSS || lag;
    // the dual mat-vec + sketch step: with the bf16 table in row-block-major
    // order (the systems share the table's entries), else system by system
    auto dual_step = [&](hipStream_t q, const MapAt& M, int ii) -> bool {
        return tab ? launch_gbatch_stencil_dual_rows<T, TQ, TC>(q, itd, gid, M.pairs, (int64_t)M.gm.pairs.size(),
                                                                ii)
                   : launch_gbatch_stencil_dual<T, TQ, TC>(q, itd, gid, m_proj(M), n_proj(M), ii, false, lag);
    };
    // step 2: Householder (the compact-WY chain) or ls_sweeps Richardson sweeps
    const int sweeps = (int)d->ls_sweeps;
    auto enqueue_cycle = [&](hipStream_t q, const MapAt& M) -> bool {
        const int nsl = M.gm.nsl, cnt = M.gm.count();
        const BlockMap none{nullptr, nullptr, 0, 0};
        auto ls_step = [&](int ii, int dualflag) {
            const int rbl = (ii + 63) / 64, rbs = (ii + kRsumCoefs - 1) / kRsumCoefs;
            return sweeps > 0 ? launch_gbatch_ls_richardson<T>(q, itd, m_uni(M, nsl), n_uni(M, nsl), m_uni(M, rbs),
                                                               n_uni(M, rbs), ii, dualflag, sweeps)
                              : launch_gbatch_ls<T, TS>(q, itd, m_uni(M, nsl), n_uni(M, nsl), m_uni(M, rbl),
                                                    n_uni(M, rbl), ii, dualflag);
        };
        auto column_step = [&](int ii) {
            const int rbq = (ii + 1 + 63) / 64;   // column-step blocks beyond the slices
            return sweeps > 0 ? launch_gbatch_column_richardson<T>(q, itd, m_uni(M, nsl), n_uni(M, nsl), ii)
                              : launch_batch_column<T, TS>(q, itd, m_uni(M, nsl), n_uni(M, nsl), m_uni(M, nsl + rbq),
                                                       n_uni(M, nsl + rbq), none, 0, ii);
        };
        if (!launch_gbatch_reset(q, itd, m_sys(M), cnt)) return false;
        if (!launch_gbatch_cast<T>(q, gid, m_row(M), n_row(M))) return false;
        if (dual) {
            if (!launch_gbatch_project_ws<T, TQ, DEFER>(q, itd, gid, m_proj(M), n_proj(M), 0) || !dual_step(q, M, 0))
                return false;
        } else if (!launch_gbatch_project<T, TQ, DEFER>(q, sk_kind, itd, gid, m_proj(M), n_proj(M), 0)) {
            return false;
        }
        if (!column_step(0)) return false;
        if (!launch_gbatch_givens_init(q, itd, gid, m_sys(M), cnt)) return false;
        for (int64_t i = 1; i <= restart; ++i) {
            const int ii = (int)i;
            if (dual) {
                if (!ls_step(ii, 1) || !launch_gbatch_project_ws<T, TQ, DEFER>(q, itd, gid, m_proj(M), n_proj(M), ii) ||
                    !dual_step(q, M, ii))
                    return false;
            } else {
                if (!launch_gbatch_stencil<T, TQ, TC>(q, sk_kind, itd, gid, m_proj(M), n_proj(M), ii)) return false;
                if (!ls_step(ii, 0)) return false;
                if (!launch_gbatch_project<T, TQ, DEFER>(q, sk_kind, itd, gid, m_proj(M), n_proj(M), ii))
                    return false;
            }
            if (!column_step(ii)) return false;
            if (!launch_gbatch_givens(q, itd, gid, m_sys(M), cnt, ii)) return false;
        }
        return launch_gbatch_finish<TQ>(q, itd, gid, m_sys(M), cnt, m_row(M), n_row(M));
    };
    rgs_status fail = RGS_OK;
    for (int64_t cycle = 0;; ++cycle) {
        active.clear();
        for (int64_t b = 0; b < batch; ++b) {
            if (done[b]) continue;
            if (iters[b] >= d->max_iters) {
                res[b] = RGS_ENOCONV;
                done[b] = 1;
                continue;
            }
            active.push_back(b);
        }
        if (active.empty()) break;
        for (int64_t b : active) lim[b] = (int)std::min<int64_t>(restart, d->max_iters - iters[b]);
        // the cycle's sketch: sketch_id 2 (+ cycle unless reused), instance 0, per-system n
        if (cycle == 0 || !d->reuse_theta) {
            const uint32_t sid = d->reuse_theta ? 2u : (uint32_t)(2 + cycle);
            bool ok = true;
            if (sk_kind == SK_SRHT) rows_all.assign((size_t)(k * batch), 0);
            for (int64_t b : active) {
                bi[b].sk.sid = sid;
                if (sk_kind == SK_SRHT) {
                    ok = ok && launch_srht_signs(s, const_cast<uint32_t*>(bi[b].sk.signs), (ns[b] + 31) / 32,
                                                 bi[b].sk);
                    std::vector<int> rows;
                    srht_rows_host(srht_order(ns[b]), (int)k, bi[b].sk, rows);
                    std::copy(rows.begin(), rows.end(), rows_all.begin() + b * k);
                }
            }
            ok = ok && (sk_kind != SK_SRHT || hipMemcpyAsync(A + o_rows, rows_all.data(), rows_all.size() * sizeof(int),
                                                             hipMemcpyHostToDevice, s) == hipSuccess);
            ok = ok && (!tab || launch_theta_table(s, make_sketch(SK_GAUSS, k, d->seed, sid, 0), nmax,
                                                   reinterpret_cast<uint16_t*>(A + o_table)));
            ok = ok && hipMemcpyAsync(A + o_items, bi.data(), bi.size() * sizeof(BatchItem), hipMemcpyHostToDevice,
                                      s) == hipSuccess;
            if (!ok) {
                drop_graphs();
                return RGS_EDEVICE;
            }
        }
        if (active != prev_active) {
            // deal the running systems, by n (descending), into the shares
            std::vector<int64_t> by_n(active);
            std::stable_sort(by_n.begin(), by_n.end(), [&](int64_t a, int64_t b) { return ns[a] > ns[b]; });
            for (GShare& g : sh) g.active.clear();
            for (size_t q = 0; q < by_n.size(); ++q) sh[q % kGmresShares].active.push_back(by_n[q]);
            for (GShare& g : sh) {
                std::sort(g.active.begin(), g.active.end());
                drop_graph(g);
                if (g.active.empty()) continue;
                build_gmres_maps(g.gm, g.active, ns, k);
                if (!upload(g.gm, g.o_ids, g.o_mrow, g.o_mproj, g.o_pairs)) {
                    drop_graphs();
                    return RGS_EDEVICE;
                }
            }
            prev_active = active;
        }
        if (hipMemcpyAsync(A + o_limit, lim.data(), batch * sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess) {
            drop_graphs();
            return RGS_EDEVICE;
        }
        const bool two = !sh[1].active.empty();
        if (two && (ensure_aux(h) != RGS_OK || hipEventRecord(h->fork_ev, s) != hipSuccess ||
                    hipStreamWaitEvent(h->aux, h->fork_ev, 0) != hipSuccess)) {
            drop_graphs();
            return RGS_EDEVICE;
        }
        bool ok = true;
        for (int si = 0; si < kGmresShares && ok; ++si) {
            GShare& g = sh[si];
            if (g.active.empty()) continue;
            const hipStream_t q = si == 0 ? s : h->aux;
            const MapAt M = map_at(g.gm, g.o_ids, g.o_mrow, g.o_mproj, g.o_pairs);
            if (use_graph) {
                if (!g.exec) {
                    if (!h->capture && hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking) != hipSuccess) {
                        ok = false;
                        break;
                    }
                    if (hipStreamBeginCapture(h->capture, hipStreamCaptureModeRelaxed) != hipSuccess) {
                        ok = false;
                        break;
                    }
                    const bool enq = enqueue_cycle(h->capture, M);
                    const bool ended = hipStreamEndCapture(h->capture, &g.graph) == hipSuccess;
                    if (!enq || !ended || hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) != hipSuccess) {
                        ok = false;
                        break;
                    }
                }
                ok = hipGraphLaunch(g.exec, q) == hipSuccess;
            } else {
                ok = enqueue_cycle(q, M);
            }
        }
        if (two && (hipEventRecord(h->join_ev, h->aux) != hipSuccess ||
                    hipStreamWaitEvent(s, h->join_ev, 0) != hipSuccess))
            ok = false;
        if (!ok ||
            hipMemcpyAsync(stat.data(), A + o_status, stat.size() * sizeof(int), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipMemcpyAsync(usedh.data(), A + o_used, batch * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(rn.data(), A + o_norm, batch * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(hh.data(), A + o_hist, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) {
            (void)hipStreamSynchronize(s);
            if (h->aux) (void)hipStreamSynchronize(h->aux);
            drop_graphs();
            return RGS_EDEVICE;
        }
        if (hipStreamSynchronize(s) != hipSuccess) {
            drop_graphs();
            return RGS_EDEVICE;
        }
        for (int64_t b : active) {
            const int u = usedh[b];
            ++cycles[b];
            iters[b] += u;
            const rgs_gmres_item& it = items[b];
            for (int t = 0; t < u && nhist[b] < it.hist_cap && it.res_hist; ++t)
                it.res_hist[nhist[b]++] = hh[b * mcap + t];
            relres[b] = rn[b] / bn[b];
            if (stat[4 * b] == kStatusNonfinite || !std::isfinite(rn[b])) {
                res[b] = RGS_ENONFINITE;
                done[b] = 1;
            } else if (relres[b] <= d->tol) {
                done[b] = 1;
            } else if (u == 0) {   // no inner step could run: breakdown of the very first column
                res[b] = RGS_ENOCONV;
                done[b] = 1;
            }
        }
    }
    drop_graphs();
    const auto t1 = std::chrono::steady_clock::now();
    for (int64_t b = 0; b < batch; ++b) {
        if (item_status) item_status[b] = res[b];
        if (res[b] != RGS_OK && fail == RGS_OK) fail = res[b];
        if (reps) {
            rgs_report& r = reps[b];
            report_defaults(&r);
            r.failed_column = -1;
            r.iters = iters[b];
            r.cycles = cycles[b];
            r.delta_F = NAN;
            r.delta_tilde_F = NAN;
            r.true_relres = relres[b];
            r.seconds = std::chrono::duration<double>(t1 - t0).count();
            r.proj_kernel_ms = 0.0;
            r.proj_launches = iters[b];
        }
    }
    return fail;
}
}  // namespace

extern "C" {

int rgs_abi_version(void) { return RGS_ABI_VERSION; }

double rgs_omega_bar(double smin, double smax, double eps_star) {
    const double lo = 1.0 - (1.0 - eps_star) * smin * smin, hi = (1.0 + eps_star) * smax * smax - 1.0;
    if (std::isnan(lo) || std::isnan(hi)) return NAN;
    return lo > hi ? lo : hi;
}

const char* rgs_status_string(rgs_status s) {
    switch (s) {
        case RGS_OK: return "success";
        case RGS_EINVAL: return "invalid argument";
        case RGS_ENOMEM: return "memory allocation failed (device scratch or host)";
        case RGS_EDEVICE: return "HIP runtime, kernel launch or host runtime failure";
        case RGS_EBREAKDOWN: return "breakdown: column numerically in the span of the previous ones";
        case RGS_ENONFINITE: return "non-finite sketch (NaN or Inf in the input)";
        case RGS_ENOCONV: return "GMRES did not converge within max_iters";
        case RGS_ESCRATCH:
            return "problem larger than the fixed scratch of the no-allocation entry point "
                   "(64 MiB per device; P-SRHT k <= 4096)";
    }
    return "unknown status";
}

rgs_status rgs_create(rgs_handle** h, int device, rgs_stream stream) try {
    if (!h) return RGS_EINVAL;
    *h = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) {
        (void)hipGetLastError();
        return RGS_EDEVICE;
    }
    if (device < 0 || device >= count) return RGS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return RGS_EDEVICE;
    if (bind_scratch(device) != RGS_OK) return RGS_EDEVICE;
    rgs_handle* p = new rgs_handle();
    p->device = device;
    p->stream = static_cast<hipStream_t>(stream);
    *h = p;
    return RGS_OK;
} catch (const std::bad_alloc&) {
    return RGS_ENOMEM;
} catch (...) {
    return RGS_EDEVICE;
}

rgs_status rgs_destroy(rgs_handle* h) {
    if (!h) return RGS_EINVAL;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    if (h->aux) (void)hipStreamSynchronize(h->aux);
    for (hipEvent_t e : {h->fork_ev, h->join_ev})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->chunk_ev) (void)hipEventDestroy(e);
    if (h->qr_exec) (void)hipGraphExecDestroy(h->qr_exec);
    if (h->qr_graph) (void)hipGraphDestroy(h->qr_graph);
    for (int gi = 0; gi < 2; ++gi) {
        if (h->qrb_exec[gi]) (void)hipGraphExecDestroy(h->qrb_exec[gi]);
        if (h->qrb_graph[gi]) (void)hipGraphDestroy(h->qrb_graph[gi]);
    }
    if (h->capture) (void)hipStreamDestroy(h->capture);
    if (h->aux) (void)hipStreamDestroy(h->aux);
    if (h->arena) (void)hipFree(h->arena);
    delete h;
    return RGS_OK;
}

rgs_status rgs_set_tuning(rgs_handle* h, int32_t mode) {
    if (!h || mode < 0 || mode > kNumSchedules) return RGS_EINVAL;
    h->tune_mode = mode;
    return RGS_OK;
}

int32_t rgs_last_tuning(const rgs_handle* h) { return h ? h->last_schedule : 0; }

rgs_status rgs_set_stream(rgs_handle* h, rgs_stream stream) {
    if (!h) return RGS_EINVAL;
    h->stream = static_cast<hipStream_t>(stream);
    return RGS_OK;
}

rgs_status rgs_qr(rgs_handle* h, const rgs_qr_desc* d, const void* W, int64_t ldw, void* Q, int64_t ldq,
                  double* R, int64_t ldr, double* S, int64_t lds, rgs_report* rep) try {
    if (!h || !valid_desc(d, true) || !W || !Q || !R || !S) return RGS_EINVAL;
    if (ldw < d->n || ldq < d->n || ldr < d->m || lds < d->k) return RGS_EINVAL;
    if ((d->flags & ~(RGS_FLAG_DIAGNOSTICS | RGS_FLAG_TIME_KERNELS | RGS_FLAG_CERTIFY | RGS_FLAG_THETA_BF16 |
                      RGS_FLAG_GRAPH | RGS_FLAG_THETA_EXACT)) != 0)
        return RGS_EINVAL;
    if (!valid_table_flags(d->flags, d->sketch)) return RGS_EINVAL;
    // kernel timing records events between the launches, which a replayed graph does not have
    if ((d->flags & RGS_FLAG_GRAPH) && (d->flags & RGS_FLAG_TIME_KERNELS)) return RGS_EINVAL;
    // Phi = Theta = I would certify nothing
    if ((d->flags & RGS_FLAG_CERTIFY) && d->sketch == RGS_SKETCH_IDENTITY) return RGS_EINVAL;
    if (d->m > 4096) return RGS_EINVAL;   // dynamic LDS of the sketch-space kernels
    if (hipSetDevice(h->device) != hipSuccess) return RGS_EDEVICE;
    if (d->prec == RGS_P_FP64)
        return run_qr<double, double, false>(h, d, static_cast<const double*>(W), ldw, static_cast<double*>(Q), ldq,
                                             R, ldr, S, lds, rep);
    if (d->prec == RGS_P_BF16Q_FP32_LS64)
        return run_qr<float, bf16, true>(h, d, static_cast<const float*>(W), ldw, static_cast<bf16*>(Q), ldq, R,
                                         ldr, S, lds, rep);
    if (d->prec == RGS_P_FP32)
        return run_qr<float, float, false, float>(h, d, static_cast<const float*>(W), ldw, static_cast<float*>(Q),
                                                  ldq, R, ldr, S, lds, rep);
    return run_qr<float, float, false>(h, d, static_cast<const float*>(W), ldw, static_cast<float*>(Q), ldq, R,
                                       ldr, S, lds, rep);
} catch (const std::bad_alloc&) {
    return RGS_ENOMEM;
} catch (...) {
    return RGS_EDEVICE;
}

rgs_status rgs_qr_noalloc(rgs_handle* h, const rgs_qr_desc* d, const void* W, int64_t ldw, void* Q, int64_t ldq,
                          double* R, int64_t ldr, double* S, int64_t lds, rgs_report* rep) try {
    if (!h || !valid_desc(d, true) || !W || !Q || !R || !S) return RGS_EINVAL;
    if (ldw < d->n || ldq < d->n || ldr < d->m || lds < d->k) return RGS_EINVAL;
    if (d->flags != 0) return RGS_EINVAL;   // every flag needs memory or events of its own
    if (d->m > 4096) return RGS_EINVAL;     // dynamic LDS of the sketch-space kernels
    if (d->sketch == RGS_SKETCH_SRHT && d->k > kRowsDevMax) return RGS_ESCRATCH;   // device row draw
    char* buf = scratch_ptr(h->device);
    if (!buf) return RGS_EDEVICE;
    if (hipSetDevice(h->device) != hipSuccess) return RGS_EDEVICE;
    if (d->prec == RGS_P_FP64)
        return run_qr<double, double, false>(h, d, static_cast<const double*>(W), ldw, static_cast<double*>(Q), ldq,
                                             R, ldr, S, lds, rep, buf, kScratchBytes);
    if (d->prec == RGS_P_BF16Q_FP32_LS64)
        return run_qr<float, bf16, true>(h, d, static_cast<const float*>(W), ldw, static_cast<bf16*>(Q), ldq, R,
                                         ldr, S, lds, rep, buf, kScratchBytes);
    if (d->prec == RGS_P_FP32)
        return run_qr<float, float, false, float>(h, d, static_cast<const float*>(W), ldw, static_cast<float*>(Q),
                                                  ldq, R, ldr, S, lds, rep, buf, kScratchBytes);
    return run_qr<float, float, false>(h, d, static_cast<const float*>(W), ldw, static_cast<float*>(Q), ldq, R,
                                       ldr, S, lds, rep, buf, kScratchBytes);
} catch (...) {
    return RGS_EDEVICE;
}

rgs_status rgs_sketch_apply(rgs_handle* h, const rgs_qr_desc* d, const void* X, int64_t ldx, int64_t ncols,
                            double* Y, int64_t ldy) try {
    if (!h || !valid_desc(d, false) || !X || !Y || ncols < 1 || ldx < d->n || ldy < d->k) return RGS_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return RGS_EDEVICE;
    const int sk_kind = sketch_kind(d->sketch);
    const bool tab = (d->flags & RGS_FLAG_THETA_BF16) != 0;
    const bool tabx = (d->flags & RGS_FLAG_THETA_EXACT) != 0;
    if (!valid_table_flags(d->flags, d->sketch)) return RGS_EINVAL;
    const size_t tsize = d->prec == RGS_P_FP64 ? sizeof(double) : sizeof(float);
    // W and X are float on the bf16 path
    const QrPlan pl = plan_qr(d->n, ncols, d->k, sk_kind, tsize, false, table_entry(d->flags, tsize));
    rgs_status st = ensure_arena(h, pl.total);
    if (st != RGS_OK) return st;
    char* A = h->arena;
    SketchArgs sk = make_sketch(sk_kind, d->k, d->seed, d->sketch_id, d->instance);
    st = setup_sketch(h, sk, d->n, reinterpret_cast<uint32_t*>(A + pl.signs), reinterpret_cast<int*>(A + pl.rows));
    if (st != RGS_OK) return st;
    if (tab && (st = use_table(h, sk, d->n, reinterpret_cast<uint16_t*>(A + pl.table))) != RGS_OK) return st;
    if (tabx) {
        st = d->prec == RGS_P_FP64 ? use_tabx<double>(h, sk, d->n, reinterpret_cast<double*>(A + pl.table))
                                   : use_tabx<float>(h, sk, d->n, reinterpret_cast<float*>(A + pl.table));
        if (st != RGS_OK) return st;
    }
    if (d->prec == RGS_P_FP64)
        st = sketch_matrix<double, double, double>(h, sk, static_cast<const double*>(X), ldx, d->n, ncols, pl.G_P,
                                                   pl.cc, reinterpret_cast<double*>(A + pl.part_P), Y, ldy);
    else if (d->prec == RGS_P_FP32)   // float32 arithmetic throughout (unique-precision model)
        st = sketch_matrix<float, float, float, float>(h, sk, static_cast<const float*>(X), ldx, d->n, ncols,
                                                       pl.G_P, pl.cc, reinterpret_cast<float*>(A + pl.part_P), Y,
                                                       ldy);
    else
        st = sketch_matrix<float, float, double>(h, sk, static_cast<const float*>(X), ldx, d->n, ncols, pl.G_P,
                                                 pl.cc, reinterpret_cast<double*>(A + pl.part_P), Y, ldy);
    if (st != RGS_OK) return st;
    return hipStreamSynchronize(h->stream) == hipSuccess ? RGS_OK : RGS_EDEVICE;
} catch (const std::bad_alloc&) {
    return RGS_ENOMEM;
} catch (...) {
    return RGS_EDEVICE;
}

rgs_status rgs_sketch_materialize(rgs_handle* h, const rgs_qr_desc* d, int64_t j0, int64_t j1, int64_t l0,
                                  int64_t l1, double* out, int64_t ldo) try {
    if (!h || !valid_desc(d, false) || !out) return RGS_EINVAL;
    if (j0 < 0 || j1 < j0 || j1 > d->k || l0 < 0 || l1 < l0 || l1 > d->n || ldo < std::max<int64_t>(1, j1 - j0))
        return RGS_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return RGS_EDEVICE;
    const int sk_kind = sketch_kind(d->sketch);
    const bool tab = (d->flags & RGS_FLAG_THETA_BF16) != 0;
    if (tab && sk_kind != SK_GAUSS) return RGS_EINVAL;
    if (d->flags & RGS_FLAG_THETA_EXACT) return RGS_EINVAL;   // the entries are those of the GAUSSIAN sketch
    const QrPlan pl = plan_qr(d->n, 1, d->k, sk_kind, sizeof(double), false, tab ? 2 : 0);
    rgs_status st = ensure_arena(h, pl.total);
    if (st != RGS_OK) return st;
    char* A = h->arena;
    SketchArgs sk = make_sketch(sk_kind, d->k, d->seed, d->sketch_id, d->instance);
    st = setup_sketch(h, sk, d->n, reinterpret_cast<uint32_t*>(A + pl.signs), reinterpret_cast<int*>(A + pl.rows));
    if (st != RGS_OK) return st;
    if (tab && (st = use_table(h, sk, d->n, reinterpret_cast<uint16_t*>(A + pl.table))) != RGS_OK) return st;
    const double rsk = sk_kind == SK_IDENT ? 1.0 : 1.0 / std::sqrt((double)d->k);
    const bool ok = d->prec == RGS_P_FP64
                        ? launch_materialize<double>(h->stream, sk, j0, j1, l0, l1, rsk, out, ldo)
                        : launch_materialize<float>(h->stream, sk, j0, j1, l0, l1, rsk, out, ldo);
    if (!ok) return RGS_EDEVICE;
    return hipStreamSynchronize(h->stream) == hipSuccess ? RGS_OK : RGS_EDEVICE;
} catch (const std::bad_alloc&) {
    return RGS_ENOMEM;
} catch (...) {
    return RGS_EDEVICE;
}

rgs_status rgs_gmres(rgs_handle* h, const rgs_stencil7* A, const rgs_gmres_desc* d, const double* b, double* x,
                     double* res_hist, int64_t hist_cap, rgs_report* rep) try {
    if (!h || !A || !b || !x || hist_cap < 0 || (hist_cap > 0 && !res_hist) || !valid_gmres_desc(d))
        return RGS_EINVAL;
    int64_t n = 0;
    if (!grid_size(*A, &n)) return RGS_EINVAL;
    rgs_qr_desc q{};
    q.n = n;
    q.m = d->restart + 1;
    q.k = d->k;
    q.sketch = d->sketch;
    q.prec = d->prec;
    if (!valid_desc(&q, true)) return RGS_EINVAL;
    if ((d->flags & ~(RGS_FLAG_THETA_BF16 | RGS_FLAG_THETA_EXACT | RGS_FLAG_LAG | RGS_FLAG_CERTIFY)) != 0)
        return RGS_EINVAL;
    if (!valid_table_flags(d->flags, d->sketch)) return RGS_EINVAL;
    if ((d->flags & RGS_FLAG_CERTIFY) && d->sketch == RGS_SKETCH_IDENTITY) return RGS_EINVAL;   // Phi = Theta = I
    if (hipSetDevice(h->device) != hipSuccess) return RGS_EDEVICE;
    if (d->prec == RGS_P_FP64) return run_gmres<double, double, false>(h, A, d, b, x, res_hist, hist_cap, rep);
    if (d->prec == RGS_P_BF16Q_FP32_LS64) return run_gmres<float, bf16, true>(h, A, d, b, x, res_hist, hist_cap, rep);
    if (d->prec == RGS_P_FP32)   // the configuration of Sec. 5.3
        return run_gmres<float, float, false, float>(h, A, d, b, x, res_hist, hist_cap, rep);
    return run_gmres<float, float, false>(h, A, d, b, x, res_hist, hist_cap, rep);
} catch (const std::bad_alloc&) {
    return RGS_ENOMEM;
} catch (...) {
    return RGS_EDEVICE;
}

rgs_status rgs_stencil_apply(rgs_handle* h, const rgs_stencil7* Ad, int32_t prec, const void* u, void* w) try {
    if (!h || !Ad || !u || !w) return RGS_EINVAL;
    if (Ad->nx < 1 || Ad->ny < 1 || Ad->nz < 1) return RGS_EINVAL;
    if (Ad->nx * Ad->ny * Ad->nz > ((int64_t)1 << 31) - 1) return RGS_EINVAL;
    if (prec != RGS_P_FP64 && prec != RGS_P_FP32_LS64 && prec != RGS_P_FP32) return RGS_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return RGS_EDEVICE;
    rgs_status st = ensure_arena(h, 4096);
    if (st != RGS_OK) return st;
    int* status = reinterpret_cast<int*>(h->arena);
    if (hipMemsetAsync(status, 0, 4 * sizeof(int), h->stream) != hipSuccess) return RGS_EDEVICE;
    const StencilArgs A = stencil_args(Ad);
    SketchArgs sk{};
    bool ok;
    if (prec == RGS_P_FP64)
        ok = launch_stencil_sketch<double, double>(h->stream, A, static_cast<const double*>(u), nullptr,
                                                   static_cast<double*>(w), 0, sk, nullptr, status);
    else if (prec == RGS_P_FP32)   // float32 vectors, the product in fp64 (Sec. 5.3)
        ok = launch_stencil_sketch<float, float, double>(h->stream, A, static_cast<const float*>(u), nullptr,
                                                         static_cast<float*>(w), 0, sk, nullptr, status);
    else
        ok = launch_stencil_sketch<float, float>(h->stream, A, static_cast<const float*>(u), nullptr,
                                                 static_cast<float*>(w), 0, sk, nullptr, status);
    if (!ok) return RGS_EDEVICE;
    return hipStreamSynchronize(h->stream) == hipSuccess ? RGS_OK : RGS_EDEVICE;
} catch (const std::bad_alloc&) {
    return RGS_ENOMEM;
} catch (...) {
    return RGS_EDEVICE;
}

rgs_status rgs_qr_batched_ex(rgs_handle* h, int64_t batch, const rgs_qr_item* items, int32_t sketch, int32_t prec,
                             uint64_t seed, uint32_t sketch_id, uint32_t flags, int32_t* item_status,
                             int64_t* failed_column, rgs_report* rep) try {
    if (!h || batch < 1 || batch > 65535 || !items) return RGS_EINVAL;
    if (sketch != RGS_SKETCH_GAUSSIAN && sketch != RGS_SKETCH_SRHT) return RGS_EINVAL;
    if (prec != RGS_P_FP32_LS64 && prec != RGS_P_BF16Q_FP32_LS64) return RGS_EINVAL;
    if ((flags & ~(RGS_FLAG_THETA_BF16 | RGS_FLAG_THETA_EXACT | RGS_FLAG_GRAPH | RGS_FLAG_LS_SWEEPS_MASK)) != 0)
        return RGS_EINVAL;
    const uint32_t sweeps = (flags & RGS_FLAG_LS_SWEEPS_MASK) >> 24;
    if (sweeps > kMaxSweeps) return RGS_EINVAL;
    const bool tab = (flags & RGS_FLAG_THETA_BF16) != 0;
    const bool tabx = (flags & RGS_FLAG_THETA_EXACT) != 0;
    const bool graph = (flags & RGS_FLAG_GRAPH) != 0;
    if (!valid_table_flags(flags, sketch)) return RGS_EINVAL;
    const int sk_kind = sketch_kind(sketch);
    for (int64_t b = 0; b < batch; ++b)
        if (!valid_item(items[b], sk_kind)) return RGS_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return RGS_EDEVICE;
    if (prec == RGS_P_BF16Q_FP32_LS64)
        return run_qr_batched<bf16, true>(h, batch, items, sk_kind, seed, sketch_id, tab, tabx, (int)sweeps, graph,
                                          item_status, failed_column, rep);
    return run_qr_batched<float, false>(h, batch, items, sk_kind, seed, sketch_id, tab, tabx, (int)sweeps, graph,
                                        item_status, failed_column, rep);
} catch (const std::bad_alloc&) {
    return RGS_ENOMEM;
} catch (...) {
    return RGS_EDEVICE;
}

rgs_status rgs_qr_batched(rgs_handle* h, int64_t batch, const rgs_qr_item* items, int32_t sketch, int32_t prec,
                          uint64_t seed, uint32_t sketch_id, int32_t* item_status, int64_t* failed_column,
                          rgs_report* rep) {
    return rgs_qr_batched_ex(h, batch, items, sketch, prec, seed, sketch_id, 0u, item_status, failed_column, rep);
}

rgs_status rgs_gmres_batched(rgs_handle* h, int64_t batch, const rgs_gmres_item* items, const rgs_gmres_desc* d,
                             int32_t* item_status, rgs_report* reps) try {
    if (!h || batch < 1 || batch > 65535 || !items || !valid_gmres_desc(d)) return RGS_EINVAL;
    if (d->sketch != RGS_SKETCH_GAUSSIAN && d->sketch != RGS_SKETCH_SRHT) return RGS_EINVAL;
    if ((d->flags & ~(RGS_FLAG_GRAPH | RGS_FLAG_THETA_BF16 | RGS_FLAG_LAG)) != 0) return RGS_EINVAL;
    if ((d->flags & RGS_FLAG_THETA_BF16) && d->sketch != RGS_SKETCH_GAUSSIAN) return RGS_EINVAL;
    for (int64_t b = 0; b < batch; ++b) {
        const rgs_gmres_item& it = items[b];
        int64_t n = 0;
        if (!it.b || !it.x || it.hist_cap < 0 || (it.hist_cap > 0 && !it.res_hist)) return RGS_EINVAL;
        if (!grid_size(it.A, &n)) return RGS_EINVAL;
        rgs_qr_desc q{};
        q.n = n;
        q.m = d->restart + 1;
        q.k = d->k;
        q.sketch = d->sketch;
        q.prec = d->prec;
        if (!valid_desc(&q, true)) return RGS_EINVAL;
    }
    if (hipSetDevice(h->device) != hipSuccess) return RGS_EDEVICE;
    if (d->prec == RGS_P_FP64) return run_gmres_batched<double, double, false>(h, batch, items, d, item_status, reps);
    if (d->prec == RGS_P_BF16Q_FP32_LS64)
        return run_gmres_batched<float, bf16, true>(h, batch, items, d, item_status, reps);
    if (d->prec == RGS_P_FP32)
        return run_gmres_batched<float, float, false, float>(h, batch, items, d, item_status, reps);
    return run_gmres_batched<float, float, false>(h, batch, items, d, item_status, reps);
} catch (const std::bad_alloc&) {
    return RGS_ENOMEM;
} catch (...) {
    return RGS_EDEVICE;
}

}  // extern "C"
