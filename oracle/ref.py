"""ctypes front end of the CPU oracle (``jacobi_ref.c``).

TEST INFRASTRUCTURE ONLY: the GPU library never imports this module.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark use it.

All arrays cross the boundary as column-major FP64 / complex128 numpy arrays;
FP32 inputs are up-cast (the oracle always computes in FP64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi_ref.c")
_LIB = os.path.join(_HERE, "libjacobi_ref.so")

EPS64 = 2.0 ** -53          # unit roundoff u of FP64 ("Algorithmic Background", u = 2^-s)
EPS32 = 2.0 ** -24


def default_tol(dtype) -> float:
    """k*u with k = 30, the paper's test threshold (subsections "Performance of the
    Baseline Implementation" and "Numerical Accuracy")."""
    return 30.0 * (EPS32 if np.dtype(dtype) in (np.float32, np.complex64) else EPS64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load(path: str):
    """Open a compiled oracle library and declare its signatures.

    Its OpenMP threads wait passively between parallel regions (unless the
    caller chose otherwise): the oracle shares the host with the GPU
    library's threads, which must not compete with spinning idle workers."""
    os.environ.setdefault("OMP_WAIT_POLICY", "passive")
    L = C.CDLL(path)
    P, I, D, L_ = C.c_void_p, C.c_int, C.c_double, C.c_long
    L.oracle_round_robin.argtypes = [I, P]
    L.oracle_round_robin.restype = I
    L.oracle_row_cyclic.argtypes = [I, P]
    L.oracle_gesvj_d.argtypes = [I, I, P, I, D, I, I, P, P, I, P, I, P]
    L.oracle_gesvj_d.restype = I
    L.oracle_gesvj_z.argtypes = [I, I, P, I, D, I, I, P, P, I, P, I, P]
    L.oracle_gesvj_z.restype = I
    L.oracle_heevj_z.argtypes = [I, P, P, D, I, I, P, P]
    L.oracle_heevj_z.restype = L_
    L.oracle_block_iter_z.argtypes = [I, I, I, I, P, P, I, D, I]
    L.oracle_block_iter_z.restype = L_
    L.oracle_block_gesvj_z.argtypes = [I, I, I, P, I, D, I, I, P, P, I, P, I, P]
    L.oracle_block_gesvj_z.restype = I
    L.oracle_block_gesvj_dyn_z.argtypes = [I, I, I, P, I, D, I, I, D, D, P, P, I, P, I, P]
    L.oracle_block_gesvj_dyn_z.restype = I
    L.oracle_num_threads.restype = I
    L.oracle_set_num_threads.argtypes = [I]
    L.oracle_gesvj_strided_d.argtypes = [I, I, I, P, I, L_, D, I, I, P, L_, P, I, L_,
                                         P, I, L_, P, P]
    L.oracle_gesvj_strided_z.argtypes = [I, I, I, P, I, L_, D, I, I, P, L_, P, I, L_,
                                         P, I, L_, P, P]
    return L


_lib = None
_override = None


def lib():
    """The active oracle library (a test may swap in another build with
    `use_library`)."""
    global _lib
    if _override is not None:
        return _override
    if _lib is None:
        build()
        _lib = load(_LIB)
    return _lib


def use_library(L) -> None:
    """Route every oracle call to library handle L (None restores the default).
    Used by the tests that plant mistakes in a copy of the oracle."""
    global _override
    _override = L


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(t: int) -> None:
    lib().oracle_set_num_threads(int(t))


def round_robin(l: int) -> np.ndarray:
    """Brent-Luk round robin: array (l-1, l/2, 2) of pairs (i < j)."""
    out = np.zeros(((l - 1) * (l // 2), 2), dtype=np.int32)
    if lib().oracle_round_robin(l, _p(out)) != 0:
        raise ValueError("l must be even and >= 2")
    return out.reshape(l - 1, l // 2, 2)


def row_cyclic(n: int) -> np.ndarray:
    out = np.zeros((n * (n - 1) // 2, 2), dtype=np.int32)
    lib().oracle_row_cyclic(n, _p(out))
    return out


def _is_complex(a) -> bool:
    return np.iscomplexobj(a)


def gesvj(A, tol=None, max_sweeps=100, order=0, want_u=True, want_v=True):
    """Alg. 2 on one m x n matrix (m >= n).  Returns (S, U, V, sweeps, info)."""
    A = np.asarray(A)
    m, n = A.shape
    if m < n:
        raise ValueError("oracle requires m >= n")
    cplx = _is_complex(A)
    dt = np.complex128 if cplx else np.float64
    if tol is None:
        tol = default_tol(A.dtype)
    Af = np.asfortranarray(A.astype(dt))
    S = np.zeros(n, dtype=np.float64)
    U = np.zeros((m, n), dtype=dt, order="F") if want_u else None
    V = np.zeros((n, n), dtype=dt, order="F") if want_v else None
    sw = C.c_int(0)
    f = lib().oracle_gesvj_z if cplx else lib().oracle_gesvj_d
    info = f(m, n, _p(Af), max(m, 1), float(tol), int(max_sweeps), int(order), _p(S),
             _p(U), max(m, 1), _p(V), max(n, 1), C.byref(sw))
    return S, U, V, sw.value, info


def gesvj_batch(A, tol=None, max_sweeps=100, order=0, threads=None):
    """Alg. 2 over a uniform batch A of shape (batch, m, n), OpenMP over the
    batch.  Returns (S (b,n), U (b,m,n), V (b,n,n), sweeps (b,), info (b,))."""
    A = np.asarray(A)
    b, m, n = A.shape
    cplx = _is_complex(A)
    dt = np.complex128 if cplx else np.float64
    if tol is None:
        tol = default_tol(A.dtype)
    if threads:
        set_num_threads(threads)
    # per-matrix column major: (b, n, m) C-contiguous
    At = np.ascontiguousarray(A.astype(dt).transpose(0, 2, 1))
    S = np.zeros((b, n), dtype=np.float64)
    Ut = np.zeros((b, n, m), dtype=dt)
    Vt = np.zeros((b, n, n), dtype=dt)
    sweeps = np.zeros(b, dtype=np.int32)
    info = np.zeros(b, dtype=np.int32)
    f = lib().oracle_gesvj_strided_z if cplx else lib().oracle_gesvj_strided_d
    f(b, m, n, _p(At), max(m, 1), m * n, float(tol), int(max_sweeps), int(order),
      _p(S), n, _p(Ut), max(m, 1), m * n, _p(Vt), max(n, 1), n * n, _p(sweeps), _p(info))
    return S, Ut.transpose(0, 2, 1), Vt.transpose(0, 2, 1), sweeps, info


def precond_gesvj(A, tol=None, max_sweeps=100, order=1, pivot=True):
    """Alg. 2 preconditioned after Drmac and Veselic, as the section
    "Algorithmic Background" (paragraph "Efficient implementations") cites
    them: the iteration on the transposed triangular factor of a
    column-pivoted QR, here after a second, unpivoted QR of that factor (one
    real m x n matrix, m >= n; each factorisation a library step):
        A P = Q1 R1      column-pivoted QR (LAPACK xGEQP3 through scipy)
        R1^T = Q2 R2     unpivoted QR (LAPACK xGEQRF through numpy)
        X = R2^T,  X J = U_x diag(S)   Alg. 2 on X (its U is U_x, its V is J)
        A = (Q1 U_x) diag(S) (P Q2 J)^T.
    pivot=False takes the first QR without pivoting (P = I), as the QR step
    of the section "Other Performance Considerations" does.
    Returns (S, U, V, sweeps, info), sweeps being those of Alg. 2 on X."""
    import scipy.linalg as sl
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("oracle requires m >= n")
    if not np.all(np.isfinite(A)):
        return np.zeros(n), None, None, 0, 2
    if pivot:
        Q1, R1, piv = sl.qr(A, mode="economic", pivoting=True)   # A[:, piv] = Q1 R1
    else:
        Q1, R1 = np.linalg.qr(A)
        piv = np.arange(n)
    Q2, R2 = np.linalg.qr(R1.T)
    S, Ux, J, sw, info = gesvj(R2.T, tol, max_sweeps, order)
    U = Q1 @ Ux
    V = np.empty_like(J)
    V[piv, :] = Q2 @ J                                       # P e_k = e_piv[k]
    return S, U, V, sw, info


def precond_gesvj_batch(A, tol=None, max_sweeps=100, order=1, pivot=True):
    """precond_gesvj over a batch (batch, m, n); same returns as gesvj_batch."""
    A = np.asarray(A)
    out = [precond_gesvj(a, tol, max_sweeps, order, pivot) for a in A]
    b, m, n = A.shape
    S = np.stack([o[0] for o in out])
    U = np.stack([o[1] if o[1] is not None else np.full((m, n), np.nan) for o in out])
    V = np.stack([o[2] if o[2] is not None else np.full((n, n), np.nan) for o in out])
    return (S, U, V, np.array([o[3] for o in out], dtype=np.int32),
            np.array([o[4] for o in out], dtype=np.int32))


def heevj(G, tol=None, max_sweeps=100, order=1):
    """Alg. 1 on a Hermitian G.  Returns (G_out, J, n_rotations, sweeps, converged)."""
    G = np.asfortranarray(np.asarray(G, dtype=np.complex128))
    n = G.shape[0]
    J = np.zeros((n, n), dtype=np.complex128, order="F")
    if tol is None:
        tol = default_tol(np.float64)
    sw, cv = C.c_int(0), C.c_int(0)
    nrot = lib().oracle_heevj_z(n, _p(G), _p(J), float(tol), int(max_sweeps), int(order),
                                C.byref(sw), C.byref(cv))
    return G, J, int(nrot), sw.value, bool(cv.value)


def block_iter(W, V, l, nb, it, tol=None, inner_sweeps=1):
    """One round-robin iteration of the block method, in place on complex
    Fortran-ordered W (m x l*nb) and V (nv x l*nb).  Returns rotations."""
    assert W.dtype == np.complex128 and W.flags.f_contiguous
    assert V.dtype == np.complex128 and V.flags.f_contiguous
    if tol is None:
        tol = default_tol(np.float64)
    return int(lib().oracle_block_iter_z(W.shape[0], V.shape[0], l, nb, _p(W), _p(V), it,
                                         float(tol), int(inner_sweeps)))


def block_gesvj(A, nb, tol=None, max_sweeps=100, inner_sweeps=1, tol_start=0.0,
                tol_rate=0.0):
    """Blocked one-sided Jacobi ("Algorithmic Background" to "Inexact Hermitian
    Eigendecomposition").  Returns (S, U, V, sweeps, info);
    U and V are real when A is real.  tol_start > tol selects the dynamic
    inner tolerance: outer sweep s uses max(tol, tol_start * tol_rate^s)."""
    A = np.asarray(A)
    m, n = A.shape
    cplx = _is_complex(A)
    if tol is None:
        tol = default_tol(A.dtype)
    Af = np.asfortranarray(A.astype(np.complex128))
    S = np.zeros(n, dtype=np.float64)
    U = np.zeros((m, n), dtype=np.complex128, order="F")
    V = np.zeros((n, n), dtype=np.complex128, order="F")
    sw = C.c_int(0)
    if tol_start > tol:
        info = lib().oracle_block_gesvj_dyn_z(m, n, nb, _p(Af), max(m, 1), float(tol),
                                              int(max_sweeps), int(inner_sweeps),
                                              float(tol_start), float(tol_rate), _p(S), _p(U),
                                              max(m, 1), _p(V), max(n, 1), C.byref(sw))
    else:
        info = lib().oracle_block_gesvj_z(m, n, nb, _p(Af), max(m, 1), float(tol),
                                          int(max_sweeps), int(inner_sweeps), _p(S), _p(U),
                                          max(m, 1), _p(V), max(n, 1), C.byref(sw))
    if not cplx:
        U, V = U.real.copy(), V.real.copy()
    return S, U, V, sw.value, info
