"""GPU accuracy on the singular-value families of the paper's accuracy study
(Table "svd_dist", subsection "Numerical Accuracy"): random (uniform [0, 1]
entries), arith, cluster0, cluster1, logrand and geo, at the paper's
condition numbers (1e10 for FP64 and complex128, 1e5 for FP32 and
complex64), in every precision and through every path that serves the
shape.

Each result meets the tolerances of the build against the oracle (sigma
normwise, reconstruction, orthogonality).  The paper's own measures e1-e4
(1-norm residual, the two orthogonality defects, and the sigma error) are
reported for every family, and each must stay within the paper's threshold
k u (k = 30), or within twice what the oracle itself attains on the same
matrix where the oracle does not meet that threshold either (the paper
reports e3 above it for logrand and geo in FP64).
"""
import numpy as np
import pytest

import oracle
from metrics import U32, U64, paper_errors
from workloads import gen
from gpu_util import compare_with_oracle, run_gpu, say

pytestmark = pytest.mark.gpu

FAMILIES = ("random", "arith", "cluster0", "cluster1", "logrand", "geo")

CASES = [
    # (label, numpy dtype, torch dtype name, shape, run_gpu options)
    ("f64 auto", np.float64, "float64", (64, 64), {}),
    ("f64 resident", np.float64, "float64", (48, 40), dict(path="resident", precondition=0)),
    ("f64 blocked", np.float64, "float64", (200, 160), dict(path="blocked", precondition=0)),
    ("f64 precond wide", np.float64, "float64", (200, 160), {}),
    ("f32 blocked", np.float32, "float32", (96, 80), dict(path="blocked", precondition=0)),
    ("f32 auto", np.float32, "float32", (64, 64), {}),
    ("c128 blocked", np.complex128, "complex128", (100, 70), {}),
    ("c64 blocked", np.complex64, "complex64", (64, 48), {}),
]


@pytest.mark.parametrize("label,npdt,tdt,shape,kw", CASES, ids=[c[0] for c in CASES])
def test_paper_families(label, npdt, tdt, shape, kw):
    import torch
    m, n = shape
    single = npdt in (np.float32, np.complex64)
    cx = npdt in (np.complex64, np.complex128)
    kappa = 1e5 if single else 1e10
    thr = 30 * (U32 if single else U64)
    A = np.stack([gen.family(gen.rng_for(8800 + 7 * n, k), fam, m, n, kappa, complex_=cx)
                  for k, fam in enumerate(FAMILIES)]).astype(npdt)
    wide = np.complex128 if cx else np.float64
    A64 = A.astype(wide)
    say(f"[families {label} {m}x{n}]")
    S, U, V, info, sw = run_gpu(A, dtype=getattr(torch, tdt), **kw)
    Sr, Ur, Vr, swr, infor = oracle.gesvj_batch(A64)
    compare_with_oracle(A64, S.astype(np.float64), U.astype(wide), V.astype(wide), info, Sr,
                        infor, dtype=npdt, label=label)
    Sl = np.linalg.svd(A64, compute_uv=False)
    for k, fam in enumerate(FAMILIES):
        e = paper_errors(A64[k], S[k].astype(np.float64), U[k].astype(wide), V[k].astype(wide),
                         Sl[k])
        eo = paper_errors(A64[k], Sr[k], Ur[k], Vr[k], Sl[k])
        say(f"  {fam:8s} gpu e1..e4 " + " ".join(f"{x:.1e}" for x in e) +
            "   oracle " + " ".join(f"{x:.1e}" for x in eo))
        for j in range(4):
            assert e[j] <= max(thr, 2 * eo[j]), (label, fam, f"e{j + 1}", e[j], eo[j], thr)
