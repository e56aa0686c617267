"""Helpers of the GPU tests: move seeded numpy batches to the GPU in the
library's layout, run the C ABI, and compare results with the oracle."""
import sys

import numpy as np

import oracle
from metrics import orth_err, recon_err, sigma_err, tolerances


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_gpu(A, dtype=None):
    import torch
    from paper_2601_17979_amd import svdb
    t = torch.from_numpy(np.ascontiguousarray(A))
    if dtype is not None:
        t = t.to(dtype)
    return svdb.col_major(t.to("cuda"))


def run_gpu(A, **kw):
    """A: numpy (b, m, n).  Returns numpy S, U, V, info, sweeps."""
    import torch
    from paper_2601_17979_amd import svdb
    dtype = kw.pop("dtype", None)
    Ag = to_gpu(A, dtype)
    S, U, V, info, sw = svdb.svd(Ag, **kw)
    torch.cuda.synchronize()
    out = [x.cpu().numpy() if x is not None else None for x in (S, U, V, info, sw)]
    return out


def compare_with_oracle(A, S, U, V, info, Sref, inforef, dtype=np.float64, label=""):
    """Tolerance checks of one batch against oracle singular values."""
    b, m, n = A.shape
    tol_s, tol_r, tol_o = tolerances(dtype, n)
    worst = [0.0, 0.0, 0.0, 0.0]
    for k in range(b):
        assert info[k] == inforef[k], (label, k, info[k], inforef[k])
        if info[k] == 2:
            continue
        es = sigma_err(S[k], Sref[k])
        er = recon_err(A[k], S[k], U[k], V[k])
        eu, ev = orth_err(U[k]), orth_err(V[k])
        worst = [max(worst[0], es), max(worst[1], er), max(worst[2], eu), max(worst[3], ev)]
        assert es <= tol_s, (label, k, "sigma", es)
        assert er <= tol_r, (label, k, "recon", er)
        assert eu <= tol_o and ev <= tol_o, (label, k, "orth", eu, ev)
        assert np.all(np.diff(S[k]) <= 0), (label, k, "not sorted")
    say(f"  {label}: worst sigma {worst[0]:.2e} recon {worst[1]:.2e} "
        f"orthU {worst[2]:.2e} orthV {worst[3]:.2e}")
    return worst


def aligned_vector_err(S, U, V, Sref, Uref, Vref, min_gap=1e-6):
    """Largest difference of singular vectors of well-separated singular
    values after aligning each pair's sign/phase; gap-scaled."""
    n = S.shape[0]
    if n == 0 or Sref[0] == 0:
        return 0.0
    worst = 0.0
    for k in range(n):
        gaps = [abs(Sref[k] - Sref[j]) for j in (k - 1, k + 1) if 0 <= j < n]
        gap = min(gaps) / Sref[0] if gaps else 1.0
        if gap < min_gap or Sref[k] == 0:
            continue
        d = np.vdot(Vref[:, k], V[:, k])
        ph = d / abs(d) if abs(d) > 0 else 1.0
        e = max(np.abs(V[:, k] - ph * Vref[:, k]).max(), np.abs(U[:, k] - ph * Uref[:, k]).max())
        worst = max(worst, e * gap)
    return worst


def oracle_batch(A, tol=None, max_sweeps=100, order=0):
    return oracle.gesvj_batch(A, tol=tol, max_sweeps=max_sweeps, order=order)
