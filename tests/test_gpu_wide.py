"""GPU parity of wide matrices (m < n) through the C ABI.  The library solves
them through A^H = V S U^H (section "Pre-processing the SVD using a QR
Factorization", the case m < n); each result is checked as the SVD of the
tall matrix A^H against the oracle run on A^H, with the tolerances of that
tall problem, and for A = U S V^H itself."""
import numpy as np
import pytest

from workloads import gen
from gpu_util import compare_with_oracle, oracle_batch, run_gpu, say, to_gpu
from metrics import orth_err, recon_err, tolerances

pytestmark = pytest.mark.gpu


def _wide(m, n, count, seed, complex_=False, kinds=("gauss", "geo", "cluster1"), kappa=1e6):
    """count wide m x n matrices: conjugate transposes of tall n x m ones."""
    return np.stack([gen.family(gen.rng_for(seed, k), kinds[k % len(kinds)], n, m, kappa,
                                complex_).conj().T for k in range(count)])


def _check(A, S, U, V, info, dt, label):
    b, m, n = A.shape
    assert S.shape == (b, m) and U.shape == (b, m, m) and V.shape == (b, n, m), label
    At = np.ascontiguousarray(A.conj().transpose(0, 2, 1))
    Sr, _, _, _, infor = oracle_batch(At)
    # the tall problem A^H = V S U^H
    compare_with_oracle(At, S.astype(np.float64), V.astype(At.dtype), U.astype(At.dtype), info,
                        Sr, infor, dtype=dt, label=label)
    tol_r = tolerances(dt, m)[1]
    for k in range(b):
        if info[k] != 2:
            assert recon_err(A[k], S[k], U[k], V[k]) <= tol_r, (label, k)


FP64_SHAPES = [(1, 3), (5, 9), (16, 40), (24, 64), (32, 33), (64, 128), (40, 130), (70, 200),
               (100, 300)]


@pytest.mark.parametrize("m,n", FP64_SHAPES)
def test_wide_fp64_auto(m, n):
    import torch
    from paper_2601_17979_amd import svdb
    A = _wide(m, n, 6, seed=9100 + m + 7 * n)
    say(f"[wide fp64 {m}x{n}] plan {svdb.plan(torch.float64, m, n)}")
    S, U, V, info, sw = run_gpu(A)
    _check(A, S, U, V, info, np.float64, f"wide fp64 {m}x{n}")
    say(f"  sweeps {sw.tolist()}")


@pytest.mark.parametrize("path", ["plain", "resident", "blocked"])
def test_wide_fp64_forced_paths(path):
    m, n = 20, 48
    A = _wide(m, n, 5, seed=9200)
    say(f"[wide fp64 {m}x{n} {path}]")
    S, U, V, info, sw = run_gpu(A, path=path, precondition=0)
    _check(A, S, U, V, info, np.float64, f"wide {path}")


@pytest.mark.parametrize("dt,m,n", [("f32", 16, 40), ("f32", 30, 100), ("c128", 10, 30),
                                    ("c128", 24, 70), ("c64", 12, 33)])
def test_wide_other_dtypes(dt, m, n):
    import torch
    tdt = {"f32": torch.float32, "c128": torch.complex128, "c64": torch.complex64}[dt]
    cx = dt.startswith("c")
    A = _wide(m, n, 4, seed=9300 + m + n, complex_=cx)
    A = A.astype({"f32": np.float32, "c128": np.complex128, "c64": np.complex64}[dt])
    say(f"[wide {dt} {m}x{n}]")
    S, U, V, info, sw = run_gpu(A, dtype=tdt)
    A64 = A.astype(np.complex128 if cx else np.float64)
    low = dt in ("f32", "c64")
    _check(A64, S.astype(np.float64), U.astype(A64.dtype), V.astype(A64.dtype), info,
           np.float32 if low else np.float64, f"wide {dt} {m}x{n}")


def test_wide_optional_outputs():
    m, n = 12, 30
    A = _wide(m, n, 3, seed=9400)
    At = np.ascontiguousarray(A.conj().transpose(0, 2, 1))
    Sr = oracle_batch(At)[0]
    for cu, cv in ((True, False), (False, True), (False, False)):
        S, U, V, info, sw = run_gpu(A, compute_u=cu, compute_v=cv)
        assert (U is None) != cu and (V is None) != cv
        assert np.all(info == 0)
        assert max(np.abs(S[k] - Sr[k]).max() / Sr[k][0] for k in range(3)) <= 1e-12
        if U is not None:
            assert max(orth_err(U[k]) for k in range(3)) <= 1e-13 * m
        if V is not None:
            assert max(orth_err(V[k]) for k in range(3)) <= 1e-13 * m


@pytest.mark.parametrize("dt", ["f64", "c128"])
def test_wide_in_an_uneven_batch(dt):
    """Tall and wide matrices in one uneven call: every wide one is read
    transposed into its working copy, with U and V exchanged."""
    import torch
    from paper_2601_17979_amd import svdb
    cx = dt == "c128"
    shapes = [(40, 20), (20, 40), (7, 3), (3, 7), (64, 64), (33, 90), (90, 33), (1, 5), (16, 16)]
    mats = []
    for k, (m, n) in enumerate(shapes):
        if m >= n:
            a = gen.family(gen.rng_for(9500, k), ("gauss", "geo")[k % 2], m, n, 1e6, cx)
        else:
            a = gen.family(gen.rng_for(9500, k), ("gauss", "geo")[k % 2], n, m, 1e6, cx).conj().T
        mats.append(np.ascontiguousarray(a))
    tdt = torch.complex128 if cx else torch.float64
    gm = [to_gpu(a[None], tdt)[0] for a in mats]
    say(f"[wide uneven {dt}] {shapes}")
    S, U, V, info, sw = svdb.svd_batched(gm)
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    for k, a in enumerate(mats):
        s, u, v = S[k].cpu().numpy(), U[k].cpu().numpy(), V[k].cpu().numpy()
        m, n = a.shape
        kk = min(m, n)
        assert s.shape == (kk,) and u.shape == (m, kk) and v.shape == (n, kk)
        if m >= n:
            Sr, _, _, _, infor = oracle_batch(a[None])
            compare_with_oracle(a[None], s[None], u[None], v[None], info[k:k + 1], Sr, infor,
                                label=f"tall {m}x{n}")
        else:
            _check(a[None], s[None], u[None], v[None], info[k:k + 1], np.float64,
                   f"wide {m}x{n}")
