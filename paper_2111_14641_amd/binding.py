"""Thin ctypes binding of the C ABI declared in include/rbgs.h.

Only argument marshalling happens here: every step of the computation runs in
the HIP kernels of librbgs.so.  PyTorch supplies device memory and the stream.
If the library has not been built, importing functions from here raises
immediately; there is no fallback implementation.
"""
import atexit
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librbgs.so")

# rbgs_status
RBGS_OK, RBGS_EINVAL, RBGS_ENOMEM, RBGS_EDEVICE, RBGS_EBREAKDOWN, RBGS_ENOTCONV, RBGS_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
# rbgs_store / rbgs_math / rbgs_sketch_kind / rbgs_variant
STORE = {"f64": 0, "f32": 1}
MATH = {"f64": 0, "f32": 1, "bf16x3": 2}
RBGS_BATCH_GRAPH, RBGS_BATCH_PERSISTENT = 1, 2   # flags of rbgs_qr_batched
SKETCH = {"gaussian": 0, "sparse": 1, "identity": 2, "rademacher": 3, "srht": 4}
VARIANT = {"plain": 0, "lowsync": 1, "twice": 2, "l2qr": 3}
PROFILE = {"update": 0, "sketch": 1, "reduce": 2, "small": 3, "trsm": 4}


class rbgs_sketch(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("zeta", ctypes.c_int32), ("k", ctypes.c_int64),
                ("seed", ctypes.c_uint64)]


class rbgs_opts(ctypes.Structure):
    _fields_ = [("store", ctypes.c_int32), ("math", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("ls_iters", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class rbgs_cert(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("delta_tilde", ctypes.c_double),
                ("breakdown_col", ctypes.c_int64), ("nonfinite", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class rbgs_problem(ctypes.Structure):
    _fields_ = [("W", ctypes.c_void_p), ("ldw", ctypes.c_int64), ("n", ctypes.c_int64),
                ("m", ctypes.c_int64), ("Q", ctypes.c_void_p), ("ldq", ctypes.c_int64),
                ("R", ctypes.c_void_p), ("ldr", ctypes.c_int64), ("p", ctypes.c_int64),
                ("k", ctypes.c_int64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class rbgs_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class RbgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SIGNATURES = {
    "rbgs_create": ([ctypes.POINTER(_P), ctypes.c_int], ctypes.c_int),
    "rbgs_destroy": ([_P], ctypes.c_int),
    "rbgs_qr": ([_P, _P, _I64, _I64, _I64, _I64, ctypes.POINTER(rbgs_sketch),
                 ctypes.POINTER(rbgs_opts), _P, _I64, _P, _I64, _P, ctypes.POINTER(rbgs_cert)],
                ctypes.c_int),
    "rbgs_qr_noalloc": ([_P, _P, _I64, _I64, _I64, _I64, ctypes.POINTER(rbgs_sketch),
                         ctypes.POINTER(rbgs_opts), _P, _I64, _P, _I64, _P], ctypes.c_int),
    "rbgs_qr_batched": ([_P, _I64, ctypes.POINTER(rbgs_problem), ctypes.POINTER(rbgs_sketch),
                         ctypes.POINTER(rbgs_opts), _I32], ctypes.c_int),
    "rbgs_autotune": ([_P, _I64, _I64, ctypes.POINTER(rbgs_sketch), ctypes.POINTER(rbgs_opts),
                       ctypes.POINTER(_I64), ctypes.POINTER(_I64)], ctypes.c_int),
    "rbgs_spmm": ([_P, ctypes.POINTER(rbgs_csr), _I32, _P, _I64, _I64, ctypes.c_double,
                   ctypes.c_double, _P, _I64, _I32, _P, _I64, _P], ctypes.c_int),
    "rbgs_block_arnoldi": ([_P, ctypes.POINTER(rbgs_csr), _P, _I64, _I64, _I64,
                            ctypes.POINTER(rbgs_sketch), ctypes.POINTER(rbgs_opts), _P, _I64, _P,
                            _I64, ctypes.POINTER(rbgs_cert)], ctypes.c_int),
    "rbgs_block_gmres": ([_P, ctypes.POINTER(rbgs_csr), _P, _P, _I64, _I64, _I64, ctypes.c_double,
                          ctypes.POINTER(rbgs_sketch), ctypes.POINTER(rbgs_opts),
                          ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "rbgs_sketch_apply": ([_P, ctypes.POINTER(rbgs_sketch), _I32, _P, _I64, _I64, _I64, _I64, _P,
                           _I64, _P], ctypes.c_int),
    "rbgs_theta_dense": ([_P, ctypes.POINTER(rbgs_sketch), _I64, _I64, _P, _P], ctypes.c_int),
    "rbgs_cholqr_post": ([_P, _I32, _P, _I64, _I64, _I64, _P, _I64, _P, _P], ctypes.c_int),
    "rbgs_profile_enable": ([_P, _I32], ctypes.c_int),
    "rbgs_profile_get": ([_P, _I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64),
                          ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "rbgs_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "rbgs_last_error": ([_P], ctypes.c_char_p),
}


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2111_14641_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


class Library:
    """Process-wide library and one handle per device."""
    _inst = None

    def __init__(self):
        self.lib = load_library()
        self.handles = {}
        # Free every handle (workspace, events, streams, graphs) while the HIP
        # runtime is still fully loaded, before interpreter and library teardown.
        atexit.register(self.close)

    def close(self):
        """rbgs_destroy on every handle (it waits for the device first)."""
        handles, self.handles = self.handles, {}
        for h in handles.values():
            self.lib.rbgs_destroy(h)

    @classmethod
    def get(cls):
        if cls._inst is None:
            cls._inst = Library()
        return cls._inst

    def handle(self, device=0):
        if device not in self.handles:
            h = _P()
            st = self.lib.rbgs_create(ctypes.byref(h), device)
            if st != RBGS_OK:
                raise RbgsError(st, "rbgs_create failed")
            self.handles[device] = h
        return self.handles[device]

    def check(self, st, h):
        if st != RBGS_OK:
            msg = self.lib.rbgs_last_error(h).decode() or self.lib.rbgs_status_string(st).decode()
            raise RbgsError(st, msg)

    # -- raw C ABI (same names) -------------------------------------------
    def rbgs_qr(self, h, W, ldw, n, m, p, sk, opts, Q, ldq, R, ldr, S_out, cert):
        return self.lib.rbgs_qr(h, W, ldw, n, m, p, ctypes.byref(sk), ctypes.byref(opts), Q, ldq,
                                R, ldr, S_out, ctypes.byref(cert) if cert is not None else None)

    def rbgs_qr_noalloc(self, h, W, ldw, n, m, p, sk, opts, Q, ldq, R, ldr, S_out):
        return self.lib.rbgs_qr_noalloc(h, W, ldw, n, m, p, ctypes.byref(sk), ctypes.byref(opts), Q,
                                        ldq, R, ldr, S_out)

    def rbgs_qr_batched(self, h, count, probs, sk, opts, graph):
        return self.lib.rbgs_qr_batched(h, count, probs, ctypes.byref(sk), ctypes.byref(opts), graph)

    def rbgs_autotune(self, h, n, m, sk, opts):
        p, k = _I64(), _I64()
        st = self.lib.rbgs_autotune(h, n, m, ctypes.byref(sk), ctypes.byref(opts), ctypes.byref(p),
                                    ctypes.byref(k))
        return st, p.value, k.value

    def rbgs_sketch_apply(self, h, sk, store, X, ldx, n, c, row0, out, ldo, stream):
        return self.lib.rbgs_sketch_apply(h, ctypes.byref(sk), store, X, ldx, n, c, row0, out,
                                          ldo, stream)

    def rbgs_theta_dense(self, h, sk, n, row0, out, stream):
        return self.lib.rbgs_theta_dense(h, ctypes.byref(sk), n, row0, out, stream)

    def rbgs_cholqr_post(self, h, store, Q, ldq, n, m, R, ldr, breakdown, stream):
        return self.lib.rbgs_cholqr_post(h, store, Q, ldq, n, m, R, ldr, breakdown, stream)

    def rbgs_profile_enable(self, h, enable):
        return self.lib.rbgs_profile_enable(h, int(enable))

    def rbgs_profile_get(self, h, which):
        ms, cnt, by = ctypes.c_double(), _I64(), ctypes.c_double()
        st = self.lib.rbgs_profile_get(h, which, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(by))
        return st, ms.value, cnt.value, by.value


# ---------------------------------------------------------------------------
# torch-facing helpers (allocation and stream plumbing only)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def colmajor(n, m, dtype, device="cuda"):
    """An n x m column-major tensor (stride (1, n))."""
    torch = _torch()
    return torch.empty((m, n), dtype=dtype, device=device).t()


def as_colmajor(X):
    """(pointer, ld) of a 2-D column-major tensor; raises if X is not one."""
    if X.dim() != 2 or X.stride(0) != 1 or (X.shape[1] > 1 and X.stride(1) < X.shape[0]):
        raise ValueError("expected a column-major 2-D tensor (stride (1, ld), ld >= rows)")
    return X.data_ptr(), max(X.stride(1), X.shape[0])


def _stream_ptr(X):
    torch = _torch()
    return torch.cuda.current_stream(X.device).cuda_stream


def make_sketch(kind, k, seed, zeta=None):
    """zeta: nonzeros per column (sparse sign, default 8) or log2 of the SRHT
    transform size (default 0: derived from the row count)."""
    if zeta is None:
        zeta = 0 if kind == "srht" else 8
    return rbgs_sketch(SKETCH[kind], int(zeta), int(k), int(seed) & 0xFFFFFFFFFFFFFFFF)


def rbgs_qr(W, p, kind="sparse", k=None, seed=0, zeta=None, variant="lowsync", ls_iters=4,
            Q=None, R=None, want_S=False, want_cert=False, math="f64", noalloc=False):
    """RBGS QR of a column-major CUDA tensor W (n x m, float32 or float64).

    math: arithmetic of the update (step 3): "f64" (default, any storage) or
    "f32" (FP32 storage only).
    noalloc: call rbgs_qr_noalloc (the library's fixed device scratch array
    instead of its workspace; no certificate).

    Returns (Q, R, S, cert): Q like W (or the given Q, e.g. W itself for an
    in-place factorization), R (m x m float64, column-major), S (k x m float64)
    or None, and a dict with the certificates or None.
    """
    torch = _torch()
    lib = Library.get()
    n, m = W.shape
    if W.dtype == torch.float64:
        store = "f64"
    elif W.dtype == torch.float32:
        store = "f32"
    else:
        raise TypeError("W must be float32 or float64")
    if k is None:
        raise ValueError("sketch dimension k is required")
    dev = W.device.index or 0
    h = lib.handle(dev)
    if Q is None:
        Q = colmajor(n, m, W.dtype, W.device)
    if R is None:
        R = colmajor(m, m, torch.float64, W.device)
    S = colmajor(k, m, torch.float64, W.device) if want_S else None
    wp, ldw = as_colmajor(W)
    qp, ldq = as_colmajor(Q)
    rp, ldr = as_colmajor(R)
    sk = make_sketch(kind, k, seed, zeta)
    opts = rbgs_opts(STORE[store], MATH[math], VARIANT[variant], int(ls_iters), _stream_ptr(W))
    cert = rbgs_cert() if want_cert else None
    if noalloc:
        if want_cert:
            raise ValueError("rbgs_qr_noalloc computes no certificate")
        st = lib.rbgs_qr_noalloc(h, wp, ldw, n, m, p, sk, opts, qp, ldq, rp, ldr,
                                 S.data_ptr() if S is not None else None)
        lib.check(st, h)
        return Q, R, S, None
    st = lib.rbgs_qr(h, wp, ldw, n, m, p, sk, opts, qp, ldq, rp, ldr,
                     S.data_ptr() if S is not None else None, cert)
    if st == RBGS_EBREAKDOWN and cert is not None:
        return Q, R, S, dict(delta=cert.delta, delta_tilde=cert.delta_tilde,
                             breakdown_col=cert.breakdown_col, nonfinite=cert.nonfinite,
                             status=st)
    lib.check(st, h)
    cd = None
    if cert is not None:
        cd = dict(delta=cert.delta, delta_tilde=cert.delta_tilde,
                  breakdown_col=cert.breakdown_col, nonfinite=cert.nonfinite, status=st)
    return Q, R, S, cd


def rbgs_qr_batched(Ws, ps=None, ks=None, kind="sparse", seed=0, zeta=None, variant="lowsync",
                    ls_iters=4, Qs=None, Rs=None, math="f64", graph=False, persistent=False):
    """Independent RBGS QRs of column-major CUDA tensors Ws (same dtype and
    device) in one call; problem i uses sketch seed `seed + i`.  ps / ks: block
    widths and sketch sizes per problem (None or 0 = autotuned).  persistent:
    the problems the persistent queue takes run in one launch (the call then
    waits for the device).

    Returns (Qs, Rs, ps, ks) with the block widths and sketch sizes used."""
    torch = _torch()
    lib = Library.get()
    count = len(Ws)
    if count == 0:
        raise ValueError("empty batch")
    dt = Ws[0].dtype
    store = {torch.float64: "f64", torch.float32: "f32"}.get(dt)
    if store is None or any(W.dtype != dt for W in Ws):
        raise TypeError("all W must be float32 or all float64")
    dev = Ws[0].device
    h = lib.handle(dev.index or 0)
    Qs = list(Qs) if Qs is not None else [colmajor(W.shape[0], W.shape[1], dt, dev) for W in Ws]
    Rs = list(Rs) if Rs is not None else [colmajor(W.shape[1], W.shape[1], torch.float64, dev)
                                          for W in Ws]
    arr = (rbgs_problem * count)()
    for i, (W, Q, R) in enumerate(zip(Ws, Qs, Rs)):
        wp, ldw = as_colmajor(W)
        qp, ldq = as_colmajor(Q)
        rp, ldr = as_colmajor(R)
        p = int(ps[i]) if ps is not None and ps[i] else 0
        k = int(ks[i]) if ks is not None and ks[i] else 0
        arr[i] = rbgs_problem(wp, ldw, W.shape[0], W.shape[1], qp, ldq, rp, ldr, p, k, 0, 0)
    sk = make_sketch(kind, 0, seed, zeta)
    opts = rbgs_opts(STORE[store], MATH[math], VARIANT[variant], int(ls_iters), _stream_ptr(Ws[0]))
    st = lib.rbgs_qr_batched(h, count, arr, sk, opts,
                             (RBGS_BATCH_GRAPH if graph else 0) |
                             (RBGS_BATCH_PERSISTENT if persistent else 0))
    lib.check(st, h)
    return Qs, Rs, [arr[i].p for i in range(count)], [arr[i].k for i in range(count)]


def autotune(n, m, kind="sparse", store="f32", math="f64", variant="lowsync", ls_iters=4, zeta=None,
             device=0):
    """(p, k) the library's autotuner picks for an n x m problem."""
    lib = Library.get()
    h = lib.handle(device)
    sk = make_sketch(kind, 0, 0, zeta)
    import torch
    opts = rbgs_opts(STORE[store], MATH[math], VARIANT[variant], int(ls_iters),
                     torch.cuda.current_stream(device).cuda_stream)
    st, p, k = lib.rbgs_autotune(h, n, m, sk, opts)
    lib.check(st, h)
    return p, k


class CSR:
    """A square CSR matrix on the device (int64 row pointers, int32 columns,
    FP64 values), kept alive with its C descriptor."""

    def __init__(self, indptr, indices, data, device="cuda"):
        torch = _torch()
        self.row_ptr = torch.as_tensor(indptr, dtype=torch.int64).to(device)
        self.col_idx = torch.as_tensor(indices, dtype=torch.int32).to(device)
        self.val = torch.as_tensor(data, dtype=torch.float64).to(device)
        self.n = int(self.row_ptr.numel() - 1)
        self.device = self.val.device

    def struct(self):
        return rbgs_csr(self.n, int(self.val.numel()), self.row_ptr.data_ptr(),
                        self.col_idx.data_ptr(), self.val.data_ptr())


def spmm(A, X, alpha=1.0, beta=0.0, Y0=None, out_dtype=None):
    """alpha A X + beta Y0 for a column-major block X (n x bs) on the device."""
    torch = _torch()
    lib = Library.get()
    h = lib.handle(A.device.index or 0)
    n, bs = X.shape
    dt = out_dtype or X.dtype
    Y = colmajor(n, bs, dt, X.device)
    xp, ldx = as_colmajor(X)
    yp, ldy = as_colmajor(Y)
    y0p, ldy0 = as_colmajor(Y0) if Y0 is not None else (None, n)
    st = lib.lib.rbgs_spmm(h, ctypes.byref(A.struct()), STORE[_store_of(X.dtype)], xp, ldx, bs,
                           float(alpha), float(beta), y0p, ldy0, STORE[_store_of(dt)], yp, ldy,
                           _stream_ptr(X))
    lib.check(st, h)
    return Y


def _store_of(dtype):
    torch = _torch()
    if dtype == torch.float64:
        return "f64"
    if dtype == torch.float32:
        return "f32"
    raise TypeError("expected float32 or float64")


def block_arnoldi(A, B, nblocks, kind="sparse", k=None, seed=0, zeta=None, variant="lowsync",
                  ls_iters=4, math="f64", want_cert=False):
    """RBGS-Arnoldi from the block B (n x bs, column-major, FP32 or FP64).
    Returns (Q, R, cert): H = R[:, bs:] is the block Hessenberg matrix."""
    torch = _torch()
    lib = Library.get()
    h = lib.handle(A.device.index or 0)
    n, bs = B.shape
    m = nblocks * bs
    Q = colmajor(n, m, B.dtype, B.device)
    R = colmajor(m, m, torch.float64, B.device)
    bp, ldb = as_colmajor(B)
    opts = rbgs_opts(STORE[_store_of(B.dtype)], MATH[math], VARIANT[variant], int(ls_iters),
                     _stream_ptr(B))
    cert = rbgs_cert() if want_cert else None
    st = lib.lib.rbgs_block_arnoldi(h, ctypes.byref(A.struct()), bp, ldb, bs, nblocks,
                                    ctypes.byref(make_sketch(kind, k, seed, zeta)),
                                    ctypes.byref(opts), Q.data_ptr(), n, R.data_ptr(), m,
                                    ctypes.byref(cert) if cert is not None else None)
    lib.check(st, h)
    cd = None
    if cert is not None:
        cd = dict(delta=cert.delta, delta_tilde=cert.delta_tilde,
                  breakdown_col=cert.breakdown_col, nonfinite=cert.nonfinite)
    return Q, R, cd


def block_gmres(A, B, X0=None, blocks_per_cycle=40, max_cycles=10, tol=1e-8, kind="sparse",
                k=None, seed=0, zeta=None, store="f32", variant="lowsync", ls_iters=4, math="f64"):
    """Restarted randomized block GMRES for A X = B (B: n x bs FP64 on the
    device).  Returns (X, block iterations, final relative residual, history,
    converged)."""
    torch = _torch()
    lib = Library.get()
    h = lib.handle(A.device.index or 0)
    n, bs = B.shape
    Bc = colmajor(n, bs, torch.float64, B.device)
    Bc.copy_(B)
    X = colmajor(n, bs, torch.float64, B.device)
    if X0 is None:
        X.zero_()
    else:
        X.copy_(X0)
    opts = rbgs_opts(STORE[store], MATH[math], VARIANT[variant], int(ls_iters), _stream_ptr(B))
    iters, rel = _I64(), ctypes.c_double()
    hist = (ctypes.c_double * (max_cycles + 1))()
    st = lib.lib.rbgs_block_gmres(h, ctypes.byref(A.struct()), Bc.data_ptr(), X.data_ptr(), bs,
                                  blocks_per_cycle, max_cycles, float(tol),
                                  ctypes.byref(make_sketch(kind, k, seed, zeta)), ctypes.byref(opts),
                                  ctypes.byref(iters), ctypes.byref(rel), hist)
    if st not in (RBGS_OK, RBGS_ENOTCONV):
        lib.check(st, h)
    history = [v for v in hist if v >= 0.0]
    return X, iters.value, rel.value, history, st == RBGS_OK


def cholqr_post(Q, R, check=True):
    """Cholesky-QR post-processing in place: Q <- Q R'^{-1}, R <- R' R with
    R'^T R' = Q^T Q.  With check=True waits and raises on a breakdown."""
    torch = _torch()
    lib = Library.get()
    n, m = Q.shape
    store = "f64" if Q.dtype == torch.float64 else "f32"
    h = lib.handle(Q.device.index or 0)
    qp, ldq = as_colmajor(Q)
    rp, ldr = as_colmajor(R)
    bc = ctypes.c_int64(-1)
    st = lib.rbgs_cholqr_post(h, STORE[store], qp, ldq, n, m, rp, ldr,
                              ctypes.byref(bc) if check else None, _stream_ptr(Q))
    lib.check(st, h)
    return Q, R


def sketch_apply(X, kind, k, seed, zeta=None, row0=0, out=None):
    """Theta[:, row0:row0+n] X for a column-major CUDA tensor X (n x c)."""
    torch = _torch()
    lib = Library.get()
    n, c = X.shape
    store = "f64" if X.dtype == torch.float64 else "f32"
    h = lib.handle(X.device.index or 0)
    if out is None:
        out = colmajor(k, c, torch.float64, X.device)
    xp, ldx = as_colmajor(X)
    op, ldo = as_colmajor(out)
    st = lib.rbgs_sketch_apply(h, make_sketch(kind, k, seed, zeta), STORE[store], xp, ldx, n, c,
                               row0, op, ldo, _stream_ptr(X))
    lib.check(st, h)
    return out


def theta_dense(kind, k, seed, n, row0=0, zeta=None, device="cuda"):
    """Explicit unscaled Theta[:, row0:row0+n] (k x n float32, column-major)."""
    torch = _torch()
    lib = Library.get()
    dev = torch.device(device)
    h = lib.handle(dev.index or 0)
    out = colmajor(k, n, torch.float32, dev)
    st = lib.rbgs_theta_dense(h, make_sketch(kind, k, seed, zeta), n, row0, out.data_ptr(),
                              torch.cuda.current_stream(dev).cuda_stream)
    lib.check(st, h)
    return out


def profile_enable(enable=True, device=0, classes=None):
    """Record kernel timings: all classes, or only those named in `classes`."""
    lib = Library.get()
    h = lib.handle(device)
    if not enable:
        mask = 0
    elif classes is None:
        mask = -1
    else:
        mask = sum(1 << PROFILE[c] for c in classes)
    lib.check(lib.rbgs_profile_enable(h, mask), h)


def profile_get(which, device=0):
    """(milliseconds, launches, algorithmic bytes) summed over the recorded launches."""
    lib = Library.get()
    h = lib.handle(device)
    st, ms, cnt, by = lib.rbgs_profile_get(h, PROFILE[which])
    lib.check(st, h)
    return ms, cnt, by
