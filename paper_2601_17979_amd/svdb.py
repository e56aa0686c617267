"""Python binding of the C ABI in include/svdb.h (ctypes; argument marshalling
only -- every step of the SVD runs in the HIP kernels of libsvdb.so).

Tensors are torch tensors on the GPU; a batch of column-major m x n matrices
is a tensor of shape (batch, m, n) with strides (strideA, 1, lda), e.g.
``torch.empty(batch, n, m).transpose(1, 2)``.  `col_major(x)` converts.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsvdb.so")

R32, R64, C64, C128 = 0, 1, 2, 3
PATH_AUTO, PATH_PLAIN, PATH_RESIDENT, PATH_BLOCKED = 0, 1, 2, 3
ERR_UNSUPPORTED, ERR_HIP = -200, -100

_DTYPES = {torch.float32: R32, torch.float64: R64, torch.complex64: C64, torch.complex128: C128}
_REAL = {torch.float32: torch.float32, torch.float64: torch.float64,
         torch.complex64: torch.float32, torch.complex128: torch.float64}
_PATHS = {"auto": PATH_AUTO, "plain": PATH_PLAIN, "resident": PATH_RESIDENT,
          "blocked": PATH_BLOCKED}


class Opts(C.Structure):
    _fields_ = [("max_sweeps", C.c_int), ("path", C.c_int), ("nb", C.c_int),
                ("masking", C.c_int), ("precision", C.c_int), ("sweeps", C.c_void_p),
                ("waves", C.c_int), ("precondition", C.c_int), ("inner_sweeps", C.c_int),
                ("persistent", C.c_int), ("inner_tol_start", C.c_double),
                ("inner_tol_rate", C.c_double)]


class SvdbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"svdb error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libsvdb.so.  Raises if the library has not been built: there
    is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                               "`python -m paper_2601_17979_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I, D, LL, SZ = C.c_void_p, C.c_int, C.c_double, C.c_longlong, C.c_size_t
        L.svdb_opts_default.argtypes = [C.POINTER(Opts)]
        L.svdb_last_error.restype = C.c_char_p
        L.svdb_version.restype = C.c_char_p
        L.svdb_plan.argtypes = [I, I, I, C.POINTER(Opts), C.POINTER(I), C.POINTER(I),
                                C.POINTER(I)]
        L.svdb_plan.restype = I
        L.svdb_workspace_size.argtypes = [I, I, I, I, C.POINTER(Opts)]
        L.svdb_workspace_size.restype = SZ
        L.svdb_batched_workspace_size.argtypes = [I, I, P, P, C.POINTER(Opts)]
        L.svdb_batched_workspace_size.restype = SZ
        L.svdb_svd_strided_batched.argtypes = [I, I, I, I, P, I, LL, P, LL, P, I, LL, P, I, LL,
                                               D, P, P, SZ, C.POINTER(Opts), P]
        L.svdb_svd_strided_batched.restype = I
        L.svdb_svd_strided_batched_noalloc.argtypes = [I, I, I, I, P, I, LL, P, LL, P, I, LL,
                                                       P, I, LL, D, P, C.POINTER(Opts), P]
        L.svdb_svd_strided_batched_noalloc.restype = I
        L.svdb_noalloc_scratch_bytes.argtypes = []
        L.svdb_noalloc_scratch_bytes.restype = SZ
        L.svdb_svd_batched.argtypes = [I, I, P, P, P, P, P, P, P, P, P, D, P, P, SZ,
                                       C.POINTER(Opts), P]
        L.svdb_svd_batched.restype = I
        L.svdb_server_create.argtypes = [C.POINTER(P), SZ, I, C.POINTER(Opts)]
        L.svdb_server_create.restype = I
        L.svdb_server_submit.argtypes = [P, I, I, I, P, I, P, P, I, P, I, D, P, P]
        L.svdb_server_submit.restype = LL
        L.svdb_server_poll.argtypes = [P, P, P, P, I, I]
        L.svdb_server_poll.restype = I
        L.svdb_server_stats.argtypes = [P, C.POINTER(LL), C.POINTER(LL), C.POINTER(I),
                                        C.POINTER(I), C.POINTER(SZ)]
        L.svdb_server_stats.restype = I
        L.svdb_server_error.argtypes = [P]
        L.svdb_server_error.restype = C.c_char_p
        L.svdb_server_destroy.argtypes = [P]
        L.svdb_server_destroy.restype = I
        L.svdb_server_clock.argtypes = []
        L.svdb_server_clock.restype = D
        _lib = L
    return _lib


def last_error() -> str:
    return lib().svdb_last_error().decode()


def version() -> str:
    return lib().svdb_version().decode()


def make_opts(max_sweeps=100, path="auto", nb=0, masking=True, precision=0, sweeps=None,
              waves=0, precondition=-1, inner_sweeps=0, persistent=False, inner_tol=None):
    o = Opts()
    lib().svdb_opts_default(C.byref(o))
    o.max_sweeps = int(max_sweeps)
    o.path = _PATHS[path] if isinstance(path, str) else int(path)
    o.nb = int(nb)
    o.masking = 1 if masking else 0
    o.precision = int(precision)
    o.sweeps = sweeps.data_ptr() if sweeps is not None else None
    o.waves = int(waves)
    o.precondition = int(precondition)
    o.inner_sweeps = int(inner_sweeps)
    o.persistent = 1 if persistent else 0
    if inner_tol is not None:   # (start, rate) of the dynamic inner tolerance
        o.inner_tol_start, o.inner_tol_rate = float(inner_tol[0]), float(inner_tol[1])
    return o


def dtype_code(dt: torch.dtype) -> int:
    if dt not in _DTYPES:
        raise TypeError(f"unsupported dtype {dt}")
    return _DTYPES[dt]


def plan(dtype: torch.dtype, m: int, n: int, **kw):
    """(path, nb, threads) the library would use for one m x n matrix."""
    o = make_opts(**kw)
    p, nb, th = C.c_int(), C.c_int(), C.c_int()
    rc = lib().svdb_plan(dtype_code(dtype), m, n, C.byref(o), C.byref(p), C.byref(nb),
                         C.byref(th))
    if rc:
        raise SvdbError(rc, last_error())
    return p.value, nb.value, th.value


def col_major(A: torch.Tensor) -> torch.Tensor:
    """Copy of a (batch, m, n) tensor laid out column-major per matrix."""
    b, m, n = A.shape
    out = torch.empty((b, n, m), dtype=A.dtype, device=A.device).transpose(1, 2)
    out.copy_(A)
    return out


def empty_col_major(b, m, n, dtype, device):
    return torch.empty((b, n, m), dtype=dtype, device=device).transpose(1, 2)


def _check_cm(x: torch.Tensor, name: str):
    if x.dim() != 3:
        raise ValueError(f"{name} must be (batch, rows, cols)")
    if x.shape[1] > 1 and x.stride(1) != 1:
        raise ValueError(f"{name} must be column-major per matrix (stride(1) == 1)")


def svd(A: torch.Tensor, tol: float = 0.0, max_sweeps: int = 100, path="auto", nb: int = 0,
        compute_u: bool = True, compute_v: bool = True, masking: bool = True,
        precision: int = 0, want_sweeps: bool = True, stream=None, out=None, waves: int = 0,
        precondition: int = -1, inner_sweeps: int = 0, persistent: bool = False,
        inner_tol=None):
    """Batched reduced SVD of a (batch, m, n) column-major GPU tensor:
    A = U diag(S) V^H with k = min(m, n) singular values, U (m x k), V (n x k)
    (a wide matrix, m < n, is solved through its conjugate transpose).

    Returns (S, U, V, info, sweeps); U/V are None when not requested, sweeps
    is None unless want_sweeps.  Enqueued on `stream` (default: torch's
    current stream); synchronise before reading results on the host.
    """
    _check_cm(A, "A")
    if stream is not None:
        # outputs and workspace belong to the stream the kernels run on, so
        # that torch's caching allocator does not hand their memory to another
        # stream while the kernels still use it
        with torch.cuda.stream(stream):
            return svd(A, tol, max_sweeps, path, nb, compute_u, compute_v, masking, precision,
                       want_sweeps, None, out, waves, precondition, inner_sweeps, persistent,
                       inner_tol)
    b, m, n = A.shape
    k = min(m, n)
    dev = A.device
    code = dtype_code(A.dtype)
    if out is not None:
        S, U, V, info, sweeps = out
    else:
        S = torch.empty((b, k), dtype=_REAL[A.dtype], device=dev)
        U = empty_col_major(b, m, k, A.dtype, dev) if compute_u else None
        V = empty_col_major(b, n, k, A.dtype, dev) if compute_v else None
        info = torch.empty(b, dtype=torch.int32, device=dev)
        sweeps = torch.empty(b, dtype=torch.int32, device=dev) if want_sweeps else None
    o = make_opts(max_sweeps, path, nb, masking, precision, sweeps, waves, precondition,
                  inner_sweeps, persistent, inner_tol)
    st = (stream or torch.cuda.current_stream(dev)).cuda_stream
    lda = max(A.stride(2), 1) if n > 1 else max(m, 1)
    ldu = (U.stride(2) if k > 1 else max(m, 1)) if U is not None else 1
    ldv = (V.stride(2) if k > 1 else max(n, 1)) if V is not None else 1
    ws_bytes = lib().svdb_workspace_size(code, b, m, n, C.byref(o))
    if ws_bytes == C.c_size_t(-1).value:
        raise SvdbError(-1, last_error() or "invalid arguments")
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev) if ws_bytes else None
    rc = lib().svdb_svd_strided_batched(
        code, b, m, n, A.data_ptr(), lda, A.stride(0), S.data_ptr(), S.stride(0),
        U.data_ptr() if U is not None else None, ldu, U.stride(0) if U is not None else 0,
        V.data_ptr() if V is not None else None, ldv, V.stride(0) if V is not None else 0,
        float(tol), info.data_ptr(), ws.data_ptr() if ws is not None else None, ws_bytes,
        C.byref(o), st)
    if rc:
        raise SvdbError(rc, last_error())
    return S, U, V, info, sweeps


def svd_noalloc(A: torch.Tensor, out, tol: float = 0.0, max_sweeps: int = 100, path="auto",
                waves: int = 0, precondition: int = -1, stream=None):
    """svd() through svdb_svd_strided_batched_noalloc: no workspace, the
    library's static scratch instead.  `out` = (S, U, V, info, sweeps) as
    svd() returns them (U, V or sweeps may be None); nothing is allocated
    here or in the library.  Returns `out`."""
    _check_cm(A, "A")
    b, m, n = A.shape
    k = min(m, n)
    S, U, V, info, sweeps = out
    o = make_opts(max_sweeps, path, 0, True, 0, sweeps, waves, precondition)
    st = (stream or torch.cuda.current_stream(A.device)).cuda_stream
    lda = max(A.stride(2), 1) if n > 1 else max(m, 1)
    ldu = (U.stride(2) if k > 1 else max(m, 1)) if U is not None else 1
    ldv = (V.stride(2) if k > 1 else max(n, 1)) if V is not None else 1
    rc = lib().svdb_svd_strided_batched_noalloc(
        dtype_code(A.dtype), b, m, n, A.data_ptr(), lda, A.stride(0), S.data_ptr(), S.stride(0),
        U.data_ptr() if U is not None else None, ldu, U.stride(0) if U is not None else 0,
        V.data_ptr() if V is not None else None, ldv, V.stride(0) if V is not None else 0,
        float(tol), info.data_ptr(), C.byref(o), st)
    if rc:
        raise SvdbError(rc, last_error())
    return out


class BatchedCall:
    """A prepared svdb_svd_batched call: outputs, pointer arrays and the
    workspace are built once; calling the object enqueues the SVD of every
    matrix of `mats` (a list of column-major (m_b, n_b) GPU tensors of one
    dtype, any shapes) and returns (S, U, V, info, sweeps) (lists for S, U,
    V, with k_b = min(m_b, n_b) columns)."""

    def __init__(self, mats, tol: float = 0.0, max_sweeps: int = 100, compute_u: bool = True,
                 compute_v: bool = True, masking: bool = True, precision: int = 0,
                 inner_sweeps: int = 0, persistent: bool = False, inner_tol=None):
        dt = mats[0].dtype
        dev = mats[0].device
        self.code = dtype_code(dt)
        bsz = len(mats)
        self.bsz = bsz
        for x in mats:
            if x.dtype != dt or x.dim() != 2 or (x.shape[0] > 1 and x.stride(0) != 1):
                raise ValueError("every matrix must be a 2-D column-major tensor of one dtype")
        self.ms = (C.c_int * bsz)(*[int(x.shape[0]) for x in mats])
        self.ns = (C.c_int * bsz)(*[int(x.shape[1]) for x in mats])
        ks = [min(int(x.shape[0]), int(x.shape[1])) for x in mats]
        self.S = [torch.empty(k, dtype=_REAL[dt], device=dev) for k in ks]
        self.U = [torch.empty((k, int(x.shape[0])), dtype=dt, device=dev).t()
                  for x, k in zip(mats, ks)] if compute_u else None
        self.V = [torch.empty((k, int(x.shape[1])), dtype=dt, device=dev).t()
                  for x, k in zip(mats, ks)] if compute_v else None
        self.info = torch.empty(bsz, dtype=torch.int32, device=dev)
        self.sweeps = torch.empty(bsz, dtype=torch.int32, device=dev)
        P = C.c_void_p * bsz
        I = C.c_int * bsz

        def ld(x, rows):
            return max(x.stride(1), rows, 1) if x.shape[1] > 1 else max(rows, 1)
        self.mats = mats
        self.Ap = P(*[x.data_ptr() for x in mats])
        self.lda = I(*[ld(x, x.shape[0]) for x in mats])
        self.Sp = P(*[t.data_ptr() for t in self.S])
        self.Up = P(*[u.data_ptr() for u in self.U]) if self.U is not None else None
        self.ldu = I(*[ld(u, u.shape[0]) for u in self.U]) if self.U is not None else None
        self.Vp = P(*[v.data_ptr() for v in self.V]) if self.V is not None else None
        self.ldv = I(*[ld(v, v.shape[0]) for v in self.V]) if self.V is not None else None
        self.opts = make_opts(max_sweeps, "auto", 0, masking, precision, self.sweeps,
                              inner_sweeps=inner_sweeps, persistent=persistent,
                              inner_tol=inner_tol)
        self.tol = float(tol)
        self.ws_bytes = lib().svdb_batched_workspace_size(self.code, bsz, self.ms, self.ns,
                                                          C.byref(self.opts))
        if self.ws_bytes == C.c_size_t(-1).value:
            raise SvdbError(-1, last_error() or "invalid arguments")
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)

    def __call__(self, stream=None):
        if stream is not None:
            # the workspace and outputs are in use on `stream` until its work
            # has finished
            for t in [self.ws, self.info, self.sweeps, *self.S, *(self.U or []),
                      *(self.V or [])]:
                t.record_stream(stream)
        st = (stream or torch.cuda.current_stream(self.info.device)).cuda_stream
        rc = lib().svdb_svd_batched(self.code, self.bsz, self.ms, self.ns, self.Ap, self.lda,
                                    self.Sp, self.Up, self.ldu, self.Vp, self.ldv, self.tol,
                                    self.info.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                                    C.byref(self.opts), st)
        if rc:
            raise SvdbError(rc, last_error())
        return self.S, self.U, self.V, self.info, self.sweeps


def svd_batched(mats, tol: float = 0.0, max_sweeps: int = 100, path="auto", nb: int = 0,
                compute_u: bool = True, compute_v: bool = True, masking: bool = True,
                precision: int = 0, stream=None, inner_sweeps: int = 0,
                persistent: bool = False, inner_tol=None):
    """Mixed-shape batch: `mats` is a list of (m_b, n_b) column-major GPU
    tensors of one dtype.  Returns lists (S, U, V) and tensors (info, sweeps).
    (path and nb are accepted for symmetry with svd(); uneven batches always
    run the block method with nb = 16.)"""
    if not mats:
        return [], [], [], None, None
    call = BatchedCall(mats, tol, max_sweeps, compute_u, compute_v, masking, precision,
                       inner_sweeps, persistent, inner_tol)
    return call(stream)


class Server:
    """Continuous-batching SVD server (svdb_server_* of the C ABI).

    ``submit(A)`` takes one column-major (m, n) GPU tensor whose values are
    final (synchronise the stream that produced it first: the server reads
    it on its own stream), allocates the outputs
    and returns a request id; ``poll()`` returns completed requests as
    (id, t_submit, t_done, (S, U, V, info, sweeps)).  The server keeps every
    tensor of a request alive until it completes."""

    def __init__(self, budget_bytes: int, max_requests: int = 1024, max_sweeps: int = 100,
                 device=None, precondition: int = -1):
        self._dev = torch.device(device or "cuda")
        o = make_opts(max_sweeps=max_sweeps, precondition=precondition)
        h = C.c_void_p()
        rc = lib().svdb_server_create(C.byref(h), int(budget_bytes), int(max_requests),
                                      C.byref(o))
        if rc:
            raise SvdbError(rc, "svdb_server_create failed")
        self._h = h
        self._live = {}

    def submit(self, A: torch.Tensor, compute_u: bool = True, compute_v: bool = True):
        if A.dim() != 2 or (A.shape[0] > 1 and A.stride(0) != 1):
            raise ValueError("A must be a 2-D column-major tensor")
        m, n = int(A.shape[0]), int(A.shape[1])
        k = min(m, n)
        dt = A.dtype
        S = torch.empty(k, dtype=_REAL[dt], device=A.device)
        U = torch.empty((k, m), dtype=dt, device=A.device).t() if compute_u else None
        V = torch.empty((k, n), dtype=dt, device=A.device).t() if compute_v else None
        info = torch.empty(1, dtype=torch.int32, device=A.device)
        sweeps = torch.empty(1, dtype=torch.int32, device=A.device)
        lda = max(A.stride(1), m, 1) if n > 1 else max(m, 1)
        rid = lib().svdb_server_submit(
            self._h, dtype_code(dt), m, n, A.data_ptr() if k else None, lda,
            S.data_ptr() if k else None, U.data_ptr() if U is not None and k else None,
            max(m, 1), V.data_ptr() if V is not None and k else None, max(n, 1), 0.0,
            info.data_ptr(), sweeps.data_ptr())
        if rid < 0:
            raise SvdbError(int(rid), self.error() or "svdb_server_submit failed")
        self._live[int(rid)] = (A, S, U, V, info, sweeps)
        return int(rid)

    def poll(self, timeout_ms: int = 0, cap: int = 4096):
        ids = (C.c_longlong * cap)()
        ts = (C.c_double * cap)()
        td = (C.c_double * cap)()
        k = lib().svdb_server_poll(self._h, ids, ts, td, cap, int(timeout_ms))
        if k < 0:
            raise SvdbError(k, self.error())
        out = []
        for i in range(k):
            A, S, U, V, info, sweeps = self._live.pop(int(ids[i]))
            out.append((int(ids[i]), ts[i], td[i], (S, U, V, info, sweeps)))
        return out

    def stats(self):
        sub, com, act, q, used = C.c_longlong(), C.c_longlong(), C.c_int(), C.c_int(), C.c_size_t()
        rc = lib().svdb_server_stats(self._h, C.byref(sub), C.byref(com), C.byref(act),
                                     C.byref(q), C.byref(used))
        if rc:
            raise SvdbError(rc, self.error())
        return {"submitted": sub.value, "completed": com.value, "active": act.value,
                "queued": q.value, "bytes_in_use": used.value}

    def error(self) -> str:
        return lib().svdb_server_error(self._h).decode() if self._h else ""

    @staticmethod
    def clock() -> float:
        return lib().svdb_server_clock()

    def close(self):
        if self._h:
            lib().svdb_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
