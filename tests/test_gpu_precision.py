"""GPU parity of the FP32 working precision and of the mixed mode (FP32
sweeps, then an FP64 refinement), through the C ABI, against the FP64 oracle.

FP32 input is judged against the oracle run on the upcast input with the FP32
tolerances (normwise sigma error <= 1e-5, reconstruction and orthogonality
<= 30 u32 n).  The mixed mode takes FP64 input and must meet the FP64
tolerances (sigma <= 1e-12, the rest <= 1e-13 n).
"""
import numpy as np
import pytest

from workloads import gen
from gpu_util import compare_with_oracle, oracle_batch, run_gpu, say

pytestmark = pytest.mark.gpu


def _batch(shape, count, seed, kinds=("gauss", "geo", "cluster1"), kappa=1e6):
    m, n = shape
    return np.stack([gen.family(gen.rng_for(seed, k), kinds[k % len(kinds)], m, n, kappa)
                     for k in range(count)])


SHAPES = [(1, 1), (7, 3), (24, 16), (33, 17), (64, 64), (128, 32), (100, 100), (130, 65),
          (200, 130)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_fp32_blocked_vs_oracle(m, n):
    import torch
    A = _batch((m, n), 6, seed=4000 + 13 * m + n).astype(np.float32)
    say(f"[fp32 {m}x{n}]")
    S, U, V, info, sw = run_gpu(A, dtype=torch.float32, path="blocked")
    assert S.dtype == np.float32 and U.dtype == np.float32
    A64 = A.astype(np.float64)
    Sr, _, _, _, infor = oracle_batch(A64)
    compare_with_oracle(A64, S.astype(np.float64), U.astype(np.float64), V.astype(np.float64),
                        info, Sr, infor, dtype=np.float32, label=f"fp32 {m}x{n}")
    say(f"  sweeps {np.bincount(sw)}")


@pytest.mark.parametrize("m,n", [(7, 3), (33, 17), (64, 64), (128, 32), (130, 65), (200, 130)])
def test_mixed_mode_vs_oracle(m, n):
    A = _batch((m, n), 6, seed=5000 + 17 * m + n, kappa=1e8)
    say(f"[mixed {m}x{n}]")
    S, U, V, info, sw = run_gpu(A, path="blocked", precision=1)
    Sr, _, _, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"mixed {m}x{n}")
    say(f"  sweeps {sw.tolist()} oracle {swr.tolist()}")


@pytest.mark.parametrize("kappa_index", [0, 1])
def test_mixed_mode_square256_sample(kappa_index):
    """Matrices of the 256 x 256 workload (geometric spectra, kappa 1e2 and
    1e8): mixed mode and FP64 blocked both meet the FP64 tolerances."""
    idx = [0, 1] if kappa_index == 0 else [2000, 2001]
    grp = gen.square256(batch=4000, indices=idx)[0]
    A = grp.A
    say(f"[square256 {grp.kinds[0]}] mixed and fp64")
    Sr, _, _, swr, infor = oracle_batch(A)
    for prec in (1, 0):
        S, U, V, info, sw = run_gpu(A, path="blocked", precision=prec)
        compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"square256 prec={prec}")
        say(f"  prec={prec} sweeps {sw.tolist()} oracle {swr.tolist()}")


@pytest.mark.parametrize("mode", ["fp32", "mixed"])
def test_precision_edge_cases(mode):
    import torch
    m, n = 40, 24
    A = _batch((m, n), 5, seed=6100)
    A[0] = 0.0
    A[1][:, 3] = 0.0
    A[1][:, 7] = A[1][:, 5]
    A[2][2, 2] = np.nan
    A[3][0, 1] = np.inf
    A[4] *= 2.0 ** 100
    kw = dict(path="blocked")
    if mode == "fp32":
        A = A.astype(np.float32)
        kw["dtype"] = torch.float32
    else:
        kw["precision"] = 1
    say(f"[edge {mode}]")
    S, U, V, info, sw = run_gpu(A, **kw)
    assert info[2] == 2 and info[3] == 2
    keep = [0, 1, 4]
    A64 = A.astype(np.float64)[keep]
    Sr, _, _, _, infor = oracle_batch(A64)
    dt = np.float32 if mode == "fp32" else np.float64
    compare_with_oracle(A64, S[keep].astype(np.float64), U[keep].astype(np.float64),
                        V[keep].astype(np.float64), info[keep], Sr, infor, dtype=dt,
                        label=f"edge {mode}")
    assert np.all(S[0] == 0.0)


def test_masking_off_gives_the_same_result():
    """Without masks a converged matrix keeps being swept, but its inner
    solves rotate nothing, so every output is bitwise the same (section "Masked Batch Operations")."""
    A = _batch((96, 80), 8, seed=6200)
    S1, U1, V1, i1, s1 = run_gpu(A, path="blocked", masking=True)
    S0, U0, V0, i0, s0 = run_gpu(A, path="blocked", masking=False)
    say(f"[masking] sweeps {s1.tolist()}")
    assert np.array_equal(i0, i1) and np.array_equal(s0, s1)
    assert np.array_equal(S0, S1) and np.array_equal(U0, U1) and np.array_equal(V0, V1)


@pytest.mark.parametrize("m,n", [(100, 100), (130, 65), (200, 130), (256, 256)])
def test_mixed_mode_on_the_preconditioned_path(m, n):
    """AUTO with precision 1 on FP64 input wider than 64 columns: the QR
    pre-processing, FP32 sweeps on R2^T, then the FP64 refinement; the FP64
    tolerances hold, at kappa 1e8 and kappa 1e2."""
    import torch
    from paper_2601_17979_amd import svdb
    assert svdb.plan(torch.float64, m, n, precision=1)[0] == svdb.PATH_BLOCKED
    for kappa in (1e8, 1e2):
        A = _batch((m, n), 4, seed=5600 + m + n + int(kappa > 1e3), kinds=("geo", "gauss"),
                   kappa=kappa)
        say(f"[qr + mixed {m}x{n} kappa {kappa:g}]")
        S, U, V, info, sw = run_gpu(A, precision=1)
        Sr, _, _, swr, infor = oracle_batch(A)
        compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"qr+mixed {m}x{n}")
        say(f"  sweeps {sw.tolist()} (oracle on A: {swr.tolist()})")
