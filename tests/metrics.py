"""Error measures used by the tests.

The tolerances of the build: normwise sigma error max_i |s_i - s_i^ref| / s_1^ref
<= 1e-12 (FP64) / 1e-5 (FP32); ||A - U S V^H||_F / ||A||_F <= 1e-13 n and
||U^H U - I||_F, ||V^H V - I||_F <= 1e-13 n (FP64); FP32 uses 30 u_32 n.
The paper's e1-e4 (subsection "Numerical Accuracy") are computed for reporting.
"""
import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def sigma_err(S, Sref):
    """Normwise: max_i |s_i - ref_i| / ref_1."""
    S, Sref = np.asarray(S, np.float64), np.asarray(Sref, np.float64)
    if Sref.size == 0 or Sref[0] == 0:
        return float(np.abs(S - Sref).max(initial=0.0))
    return float(np.abs(S - Sref).max() / Sref[0])


def recon_err(A, S, U, V):
    A = np.asarray(A, np.complex128 if np.iscomplexobj(A) else np.float64)
    R = A - (U * S[None, :]) @ V.conj().T
    na = np.linalg.norm(A)
    return float(np.linalg.norm(R) / (na if na > 0 else 1.0))


def orth_err(Q):
    k = Q.shape[1]
    return float(np.linalg.norm(Q.conj().T @ Q - np.eye(k)))


def paper_errors(A, S, U, V, Sref):
    """e1..e4 of the subsection "Numerical Accuracy" (1-norms)."""
    m, n = A.shape
    e1 = np.linalg.norm(A - (U * S) @ V.conj().T, 1) / (n * max(np.linalg.norm(A, 1), 1e-300))
    e2 = np.linalg.norm(np.eye(n) - U.conj().T @ U, 1) / m
    e3 = np.linalg.norm(np.eye(n) - V.conj().T @ V, 1) / n
    e4 = np.linalg.norm(S - Sref) / (min(m, n) * max(np.linalg.norm(Sref), 1e-300))
    return e1, e2, e3, e4


def tolerances(dtype, n):
    """(sigma, reconstruction, orthogonality) bounds for a result of width n."""
    if np.dtype(dtype) in (np.float32, np.complex64):
        t = 30 * U32 * max(n, 1)
        return 1e-5, t, t
    return 1e-12, 1e-13 * max(n, 1), 1e-13 * max(n, 1)
