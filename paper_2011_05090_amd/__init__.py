"""Python binding of librgs (randomized Gram-Schmidt / randomized GMRES on MI355X).

Argument marshalling only: every step of the method runs in the HIP kernels of
``librgs.so`` (built in-tree by ``python -m paper_2011_05090_amd.build``).  The
functions carry the names of the C entry points declared in ``include/rgs.h``
and take torch tensors for device memory; torch is used for allocation and
streams, nothing else.  If the library is missing, importing works but every
call raises -- there is no fallback path.

Matrices are column-major: an n x m matrix is a tensor of shape (n, m) with
stride(0) == 1 (``colmajor`` allocates one).
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librgs.so")

(RGS_OK, RGS_EINVAL, RGS_ENOMEM, RGS_EDEVICE, RGS_EBREAKDOWN, RGS_ENONFINITE, RGS_ENOCONV,
 RGS_ESCRATCH) = 0, -1, -2, -3, -4, -5, -6, -7
SKETCH = {"gaussian": 0, "srht": 1, "identity": 2, "rademacher": 3}
PREC = {"fp64": 0, "fp32": 1, "bf16q": 2, "fp32u": 3}
FLAG_DIAGNOSTICS = 1
FLAG_TIME_KERNELS = 2
FLAG_GRAPH = 4
FLAG_CERTIFY = 8
FLAG_THETA_BF16 = 16
FLAG_LAG = 32
FLAG_THETA_EXACT = 64


class RgsError(RuntimeError):
    def __init__(self, status, where):
        super().__init__("%s failed: %s (%d)" % (where, status_string(status), status))
        self.status = status


class QrDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("k", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("sketch_id", ctypes.c_uint32), ("instance", ctypes.c_uint32),
                ("sketch", ctypes.c_int32), ("prec", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("ls_sweeps", ctypes.c_uint32)]


class Stencil7(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("c0", ctypes.c_double), ("cxm", ctypes.c_double), ("cxp", ctypes.c_double),
                ("cym", ctypes.c_double), ("cyp", ctypes.c_double), ("czm", ctypes.c_double),
                ("czp", ctypes.c_double)]


class GmresDesc(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int64), ("max_iters", ctypes.c_int64), ("k", ctypes.c_int64),
                ("tol", ctypes.c_double), ("seed", ctypes.c_uint64), ("sketch", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("reuse_theta", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("ls_sweeps", ctypes.c_uint32)]


class QrItem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("k", ctypes.c_int64),
                ("W", ctypes.c_void_p), ("ldw", ctypes.c_int64), ("Q", ctypes.c_void_p), ("ldq", ctypes.c_int64),
                ("R", ctypes.c_void_p), ("ldr", ctypes.c_int64), ("S", ctypes.c_void_p), ("lds", ctypes.c_int64)]


class GmresItem(ctypes.Structure):
    _fields_ = [("A", Stencil7), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p), ("res_hist", ctypes.c_void_p),
                ("hist_cap", ctypes.c_int64)]


class Report(ctypes.Structure):
    _fields_ = [("failed_column", ctypes.c_int64), ("iters", ctypes.c_int64), ("cycles", ctypes.c_int64),
                ("delta_F", ctypes.c_double), ("delta_tilde_F", ctypes.c_double),
                ("true_relres", ctypes.c_double), ("seconds", ctypes.c_double),
                ("proj_kernel_ms", ctypes.c_double), ("proj_launches", ctypes.c_int64),
                ("cert_smin_q", ctypes.c_double), ("cert_smax_q", ctypes.c_double),
                ("cert_smin_w", ctypes.c_double), ("cert_smax_w", ctypes.c_double),
                ("cert_cond_phi_q", ctypes.c_double)]

    status = RGS_OK

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["status"] = self.status
        return d


# C entry points declared in include/rgs.h: name -> (restype, argtypes)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_DESCP = ctypes.POINTER(QrDesc)
SIGNATURES = {
    "rgs_abi_version": (ctypes.c_int, []),
    "rgs_omega_bar": (ctypes.c_double, [ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "rgs_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rgs_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P]),
    "rgs_destroy": (ctypes.c_int, [_P]),
    "rgs_set_stream": (ctypes.c_int, [_P, _P]),
    "rgs_set_tuning": (ctypes.c_int, [_P, ctypes.c_int32]),
    "rgs_last_tuning": (ctypes.c_int32, [_P]),
    "rgs_qr": (ctypes.c_int, [_P, _DESCP, _P, _I64, _P, _I64, _P, _I64, _P, _I64, ctypes.POINTER(Report)]),
    "rgs_qr_noalloc": (ctypes.c_int, [_P, _DESCP, _P, _I64, _P, _I64, _P, _I64, _P, _I64, ctypes.POINTER(Report)]),
    "rgs_sketch_apply": (ctypes.c_int, [_P, _DESCP, _P, _I64, _I64, _P, _I64]),
    "rgs_sketch_materialize": (ctypes.c_int, [_P, _DESCP, _I64, _I64, _I64, _I64, _P, _I64]),
    "rgs_gmres": (ctypes.c_int, [_P, ctypes.POINTER(Stencil7), ctypes.POINTER(GmresDesc), _P, _P, _P, _I64,
                                 ctypes.POINTER(Report)]),
    "rgs_stencil_apply": (ctypes.c_int, [_P, ctypes.POINTER(Stencil7), ctypes.c_int32, _P, _P]),
    "rgs_qr_batched": (ctypes.c_int, [_P, _I64, ctypes.POINTER(QrItem), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(Report)]),
    "rgs_qr_batched_ex": (ctypes.c_int, [_P, _I64, ctypes.POINTER(QrItem), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(Report)]),
    "rgs_gmres_batched": (ctypes.c_int, [_P, _I64, ctypes.POINTER(GmresItem), ctypes.POINTER(GmresDesc),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Report)]),
}

_lib = None


def lib():
    """Load librgs.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librgs.so is not built (run: python -m paper_2011_05090_amd.build); "
                               "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status):
    try:
        return lib().rgs_status_string(int(status)).decode()
    except Exception:   # library unavailable: still produce a message
        return "status %d" % status


def rgs_abi_version():
    return lib().rgs_abi_version()


def rgs_omega_bar(smin, smax, eps_star):
    """Prop. 3.7 bound from one pair of rgs_report.cert_* values."""
    return lib().rgs_omega_bar(smin, smax, eps_star)


def _check(status, where, allow=()):
    if status != RGS_OK and status not in allow:
        raise RgsError(status, where)
    return status


def colmajor(n, m, dtype, device="cuda", pad=True):
    """Uninitialised column-major n x m tensor (shape (n, m), stride (1, ld)).
    With pad, ld = n rounded up to a multiple of 4: every column then starts
    16-byte aligned (8-byte for bf16), which the library's vectorised loads need."""
    import torch
    ld = (n + 3) // 4 * 4 if pad else n
    return torch.empty((m, ld), dtype=dtype, device=device).t()[:n]


def _ld(t, rows):
    if t.dim() == 1:
        return max(rows, 1)
    if t.stride(0) != 1 and t.shape[0] > 1:
        raise ValueError("matrix arguments must be column-major (stride(0) == 1)")
    return max(t.stride(1), rows) if t.shape[1] > 1 else max(rows, 1)


def _dev(t, name, dtype=None):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s" % (name, dtype))
    return ctypes.c_void_p(t.data_ptr())


def _torch_dtype(prec):
    import torch
    return torch.float64 if PREC[prec] == 0 else torch.float32


def _dtypes(prec_code):
    """(W dtype, Q dtype) of a precision code."""
    import torch
    if prec_code == 0:
        return torch.float64, torch.float64
    if prec_code == 2:
        return torch.float32, torch.bfloat16
    return torch.float32, torch.float32


class Handle:
    """rgs_create / rgs_destroy.  Bound to a device and a stream (default: torch's current)."""

    def __init__(self, device=0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().rgs_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream.cuda_stream)), "rgs_create")
        self._h = h

    @property
    def ptr(self):
        return self._h

    def set_stream(self, stream):
        self.stream = stream
        _check(lib().rgs_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)), "rgs_set_stream")

    def close(self):
        if self._h:
            lib().rgs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qr_desc(n, m, k, sketch="srht", prec="fp32", seed=42, sketch_id=0, instance=0, flags=0, ls_sweeps=0):
    """prec: 'fp64', 'fp32' (fp32 projection, fp64 least squares), 'bf16q' (bf16 basis) or
    'fp32u' (unique precision: every step in float32).
    ls_sweeps: 0 = Householder least squares, s > 0 = s Richardson sweeps."""
    return QrDesc(n=n, m=m, k=k, seed=seed, sketch_id=sketch_id, instance=instance,
                  sketch=SKETCH[sketch], prec=PREC[prec], flags=flags, ls_sweeps=ls_sweeps)


def _qr_call(name, handle, desc, W, Q, R, S, allow):
    import torch
    dw, dq = _dtypes(desc.prec)
    n, m, k = desc.n, desc.m, desc.k
    if tuple(W.shape) != (n, m) or tuple(Q.shape) != (n, m) or tuple(R.shape) != (m, m) or tuple(S.shape) != (k, m):
        raise ValueError("shape mismatch")
    rep = Report()
    st = getattr(lib(), name)(handle.ptr, ctypes.byref(desc), _dev(W, "W", dw), _ld(W, n), _dev(Q, "Q", dq),
                              _ld(Q, n), _dev(R, "R", torch.float64), _ld(R, m), _dev(S, "S", torch.float64),
                              _ld(S, k), ctypes.byref(rep))
    _check(st, name, allow)
    rep.status = st
    return rep


def rgs_qr(handle, desc, W, Q, R, S, allow=(RGS_EBREAKDOWN, RGS_ENONFINITE)):
    """Algorithm 2 on W -> Q, R, S (all preallocated device tensors).  Returns the Report."""
    return _qr_call("rgs_qr", handle, desc, W, Q, R, S, allow)


def rgs_qr_noalloc(handle, desc, W, Q, R, S, allow=(RGS_EBREAKDOWN, RGS_ENONFINITE)):
    """rgs_qr in the library's fixed per-device scratch: allocates nothing (RGS_ESCRATCH if the
    factorisation does not fit it; flags must be 0).  Returns the Report."""
    return _qr_call("rgs_qr_noalloc", handle, desc, W, Q, R, S, allow)


def flag_ls_sweeps(s):
    """RGS_FLAG_LS_SWEEPS(s): rgs_qr_batched_ex's step 2 by s Richardson sweeps."""
    return (int(s) & 15) << 24


def rgs_qr_batched(handle, items, sketch="srht", prec="fp32", seed=42, sketch_id=0,
                   allow=(RGS_EBREAKDOWN, RGS_ENONFINITE), flags=0, ls_sweeps=0):
    """A batch of factorisations; items = list of (W, Q, R, S, k) device tensors.
    flags: 0 (rgs_qr_batched), or FLAG_THETA_BF16 or FLAG_THETA_EXACT (Gaussian sketch only)
    and/or FLAG_GRAPH (rgs_qr_batched_ex); ls_sweeps > 0 adds flag_ls_sweeps(ls_sweeps).
    Returns (Report, per-item statuses, per-item failed columns)."""
    import torch
    flags |= flag_ls_sweeps(ls_sweeps)
    dw, dq = _dtypes(PREC[prec])
    arr = (QrItem * len(items))()
    for b, (W, Q, R, S, k) in enumerate(items):
        n, m = W.shape
        if tuple(Q.shape) != (n, m) or tuple(R.shape) != (m, m) or tuple(S.shape) != (k, m):
            raise ValueError("shape mismatch in item %d" % b)
        arr[b] = QrItem(n=n, m=m, k=k, W=_dev(W, "W", dw), ldw=_ld(W, n), Q=_dev(Q, "Q", dq), ldq=_ld(Q, n),
                        R=_dev(R, "R", torch.float64), ldr=_ld(R, m), S=_dev(S, "S", torch.float64), lds=_ld(S, k))
    stat = (ctypes.c_int32 * len(items))()
    fcol = (ctypes.c_int64 * len(items))()
    rep = Report()
    if flags:
        st = lib().rgs_qr_batched_ex(handle.ptr, len(items), arr, SKETCH[sketch], PREC[prec], seed, sketch_id, flags,
                                     stat, fcol, ctypes.byref(rep))
    else:
        st = lib().rgs_qr_batched(handle.ptr, len(items), arr, SKETCH[sketch], PREC[prec], seed, sketch_id, stat,
                                  fcol, ctypes.byref(rep))
    _check(st, "rgs_qr_batched", allow)
    rep.status = st
    return rep, list(stat), list(fcol)


def rgs_set_tuning(handle, mode):
    """0: autotune the batched Gaussian sketch product per batch signature; 1..9: force a schedule."""
    _check(lib().rgs_set_tuning(handle.ptr, int(mode)), "rgs_set_tuning")


def rgs_last_tuning(handle):
    return int(lib().rgs_last_tuning(handle.ptr))


def rgs_sketch_apply(handle, desc, X, Y):
    """Y = Theta X (X: n x ncols column-major in the working precision; Y: k x ncols fp64)."""
    import torch
    dt = _dtypes(desc.prec)[0]
    Xm = X if X.dim() == 2 else X.reshape(-1, 1)
    Ym = Y if Y.dim() == 2 else Y.reshape(-1, 1)
    ncols = Xm.shape[1]
    st = lib().rgs_sketch_apply(handle.ptr, ctypes.byref(desc), _dev(Xm, "X", dt), _ld(Xm, desc.n), ncols,
                                _dev(Ym, "Y", torch.float64), _ld(Ym, desc.k))
    _check(st, "rgs_sketch_apply")


def rgs_sketch_materialize(handle, desc, j0, j1, l0, l1, out):
    import torch
    st = lib().rgs_sketch_materialize(handle.ptr, ctypes.byref(desc), j0, j1, l0, l1,
                                      _dev(out, "out", torch.float64), _ld(out, j1 - j0))
    _check(st, "rgs_sketch_materialize")


def stencil7(dims, coeffs):
    nx, ny, nz = dims
    c0, cxm, cxp, cym, cyp, czm, czp = coeffs
    return Stencil7(nx=nx, ny=ny, nz=nz, c0=c0, cxm=cxm, cxp=cxp, cym=cym, cyp=cyp, czm=czm, czp=czp)


def gmres_desc(restart, k, tol, max_iters=100000, sketch="gaussian", prec="fp32", seed=42, reuse_theta=False,
               flags=0, ls_sweeps=0):
    """ls_sweeps: 0 = Householder least squares in every Arnoldi step, s > 0 = s Richardson sweeps."""
    return GmresDesc(restart=restart, max_iters=max_iters, k=k, tol=tol, seed=seed, sketch=SKETCH[sketch],
                     prec=PREC[prec], reuse_theta=1 if reuse_theta else 0, flags=flags, ls_sweeps=ls_sweeps)


def rgs_gmres(handle, A, desc, b, x, res_hist=None, allow=(RGS_ENOCONV,)):
    """Randomized GMRES on the 7-point operator.  Returns (Report, history as a list)."""
    import torch
    n = A.nx * A.ny * A.nz
    if b.numel() != n or x.numel() != n:
        raise ValueError("b and x must have nx*ny*nz entries")
    cap = 0 if res_hist is None else int(res_hist)
    hist = (ctypes.c_double * max(cap, 1))()
    rep = Report()
    st = lib().rgs_gmres(handle.ptr, ctypes.byref(A), ctypes.byref(desc), _dev(b, "b", torch.float64),
                         _dev(x, "x", torch.float64), hist if cap else None, cap, ctypes.byref(rep))
    _check(st, "rgs_gmres", allow)
    rep.status = st
    used = min(cap, rep.iters)
    return rep, [hist[i] for i in range(used)]


def rgs_gmres_batched(handle, systems, desc, hist_cap=0, allow=(RGS_ENOCONV, RGS_ENONFINITE)):
    """Batched randomized GMRES.  systems: list of (Stencil7, b, x) with b, x
    float64 device tensors of nx*ny*nz entries.  Returns (status, per-system
    statuses, per-system Reports, per-system histories)."""
    import torch
    B = len(systems)
    arr = (GmresItem * B)()
    hists = []
    for i, (A, b, x) in enumerate(systems):
        n = A.nx * A.ny * A.nz
        if b.numel() != n or x.numel() != n:
            raise ValueError("system %d: b and x must have nx*ny*nz entries" % i)
        h = (ctypes.c_double * max(int(hist_cap), 1))()
        hists.append(h)
        arr[i] = GmresItem(A=A, b=_dev(b, "b", torch.float64), x=_dev(x, "x", torch.float64),
                           res_hist=ctypes.cast(h, ctypes.c_void_p) if hist_cap else None, hist_cap=int(hist_cap))
    stat = (ctypes.c_int32 * B)()
    reps = (Report * B)()
    st = lib().rgs_gmres_batched(handle.ptr, B, arr, ctypes.byref(desc), stat, reps)
    _check(st, "rgs_gmres_batched", allow)
    out = []
    for i in range(B):
        reps[i].status = stat[i]
        out.append(reps[i])
    return st, list(stat), out, [[hists[i][t] for t in range(min(int(hist_cap), out[i].iters))] for i in range(B)]


def rgs_stencil_apply(handle, A, prec, u, w):
    dt = _torch_dtype(prec)
    st = lib().rgs_stencil_apply(handle.ptr, ctypes.byref(A), PREC[prec], _dev(u, "u", dt), _dev(w, "w", dt))
    _check(st, "rgs_stencil_apply")
