"""GPU parity of the complex types (complex128 and complex64) on the block
path, through the C ABI, against the complex FP64 oracle.

complex128 meets the FP64 tolerances (normwise sigma error <= 1e-12,
reconstruction and orthogonality <= 1e-13 n); complex64 is judged against
the oracle on the upcast input with the FP32 ones (1e-5, 30 u32 n).
"""
import numpy as np
import pytest

from workloads import gen
from gpu_util import aligned_vector_err, compare_with_oracle, oracle_batch, run_gpu, say

pytestmark = pytest.mark.gpu


def _cbatch(shape, count, seed, kinds=("gauss", "geo", "cluster1", "random"), kappa=1e6):
    m, n = shape
    return np.stack([gen.family(gen.rng_for(seed, k), kinds[k % len(kinds)], m, n, kappa,
                                complex_=True) for k in range(count)])


SHAPES = [(1, 1), (3, 2), (9, 9), (24, 16), (33, 17), (40, 40), (64, 64), (100, 70), (130, 65),
          (160, 96)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_complex128_vs_oracle(m, n):
    import torch
    A = _cbatch((m, n), 6, seed=7000 + 11 * m + n)
    say(f"[c128 {m}x{n}]")
    S, U, V, info, sw = run_gpu(A, dtype=torch.complex128, path="blocked")
    assert S.dtype == np.float64 and U.dtype == np.complex128
    Sr, Ur, Vr, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, dtype=np.complex128, label=f"c128 {m}x{n}")
    # vectors of well-separated singular values, phase-aligned and gap-scaled;
    # U is compared as U diag(S) / s_1 (a column of a tiny singular value is
    # only determined to about u s_1 / s_k)
    worst = max(aligned_vector_err(S[k], U[k] * S[k] / S[k][0], V[k], Sr[k],
                                   Ur[k] * Sr[k] / Sr[k][0], Vr[k]) for k in range(6))
    assert worst <= 1e-12, worst
    say(f"  sweeps gpu {sw.tolist()} oracle {swr.tolist()}")


@pytest.mark.parametrize("m,n", [(3, 2), (24, 16), (64, 64), (130, 65)])
def test_complex64_vs_oracle(m, n):
    import torch
    A = _cbatch((m, n), 6, seed=7500 + 11 * m + n).astype(np.complex64)
    say(f"[c64 {m}x{n}]")
    S, U, V, info, sw = run_gpu(A, dtype=torch.complex64, path="blocked")
    assert S.dtype == np.float32 and U.dtype == np.complex64
    A128 = A.astype(np.complex128)
    Sr, _, _, _, infor = oracle_batch(A128)
    compare_with_oracle(A128, S.astype(np.float64), U.astype(np.complex128),
                        V.astype(np.complex128), info, Sr, infor, dtype=np.complex64,
                        label=f"c64 {m}x{n}")


def test_complex_one_sweep_elementwise():
    """After one sweep the complex iterate matches the complex block oracle
    (same round-robin order, one inner sweep, rotation R1) element by
    element, within ten times the oracle's own response to one-ulp
    perturbations of A."""
    import oracle
    import torch
    for m, n in [(24, 16), (40, 32)]:
        A = _cbatch((m, n), 6, seed=7900 + n, kinds=("gauss",))
        S, U, V, info, sw = run_gpu(A, dtype=torch.complex128, path="blocked", max_sweeps=1,
                                    inner_sweeps=1)
        ref = [oracle.block_gesvj(A[k], 16, max_sweeps=1) for k in range(6)]
        r = np.random.default_rng(3)
        for k in range(6):
            Sr, Ur, Vr = ref[k][0], ref[k][1], ref[k][2]
            Ap = A[k] * (1 + 2.0 ** -52 * (r.standard_normal(A[k].shape) +
                                           1j * r.standard_normal(A[k].shape)))
            Sp, Up, Vp, _, _ = oracle.block_gesvj(Ap, 16, max_sweeps=1)
            amax = np.abs(A[k]).max()
            sens = np.abs(Up * Sp - Ur * Sr).max() / amax
            tol = max(1e-13, 10 * sens)
            ew = np.abs(U[k] * S[k] - Ur * Sr).max() / amax
            ev = np.abs(V[k] - Vr).max()
            say(f"  {m}x{n} #{k}: W diff {ew:.2e} (bound {tol:.2e}) V diff {ev:.2e}")
            assert info[k] == 1 and ref[k][4] == 1
            assert ew <= tol, (m, n, k, ew, tol)
            assert ev <= max(1e-12, 10 * np.abs(Vp - Vr).max()), (m, n, k, ev)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_complex_edge_cases(prec):
    import torch
    m, n = 40, 24
    A = _cbatch((m, n), 5, seed=7800)
    A[0] = 0.0
    A[1][:, 3] = 0.0
    A[1][:, 7] = 1j * A[1][:, 5]
    A[2][2, 2] = complex(np.nan, 0.0)
    A[3][0, 1] = complex(0.0, np.inf)
    A[4] *= 2.0 ** -90
    dt, npdt = (torch.complex128, np.complex128) if prec == "c128" else \
        (torch.complex64, np.complex64)
    A = A.astype(npdt)
    S, U, V, info, sw = run_gpu(A, dtype=dt, path="blocked")
    assert info[2] == 2 and info[3] == 2
    keep = [0, 1, 4]
    A128 = A.astype(np.complex128)[keep]
    Sr, _, _, _, infor = oracle_batch(A128)
    compare_with_oracle(A128, S[keep].astype(np.float64), U[keep].astype(np.complex128),
                        V[keep].astype(np.complex128), info[keep], Sr, infor, dtype=npdt,
                        label=f"edge {prec}")
    assert np.all(S[0] == 0.0)


def test_uneven_complex_workload_sample():
    """Shapes drawn from the uneven complex128 workload (n ~ U{8..256},
    m ~ U{n..2n}): a few of each size class."""
    import torch
    groups = gen.uneven_complex(batch=400)
    picked = [g for g in groups if g.n <= 200][:: max(1, len(groups) // 8)][:8]
    for g in picked:
        A = g.A[:2]
        say(f"[uneven {g.m}x{g.n}]")
        S, U, V, info, sw = run_gpu(A, dtype=torch.complex128)
        Sr, _, _, _, infor = oracle_batch(A)
        compare_with_oracle(A, S, U, V, info, Sr, infor, dtype=np.complex128,
                            label=f"uneven {g.m}x{g.n}")


@pytest.mark.parametrize("m,n", [(256, 256), (512, 256), (480, 240), (300, 250)])
def test_complex128_upper_range(m, n):
    """The top of the uneven complex128 range (n up to 256, m up to 2n),
    through the uniform-shape call and through the mixed-shape call; the two
    run the same block method (nb = 16) on the same schedule, so they agree
    bit for bit."""
    import torch
    from paper_2601_17979_amd import svdb
    A = _cbatch((m, n), 2, seed=7600 + m + n, kinds=("gauss", "geo"))
    say(f"[c128 upper {m}x{n}]")
    S, U, V, info, sw = run_gpu(A, dtype=torch.complex128)
    Sr, _, _, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, dtype=np.complex128,
                        label=f"c128 {m}x{n} strided")
    gm = [svdb.col_major(torch.from_numpy(A[k])[None].cuda())[0] for k in range(2)]
    Sb, Ub, Vb, infob, swb = svdb.svd_batched(gm)
    torch.cuda.synchronize()
    for k in range(2):
        assert int(infob[k]) == int(info[k])
        assert np.array_equal(Sb[k].cpu().numpy(), S[k])
        assert np.array_equal(Ub[k].cpu().numpy(), U[k])
        assert np.array_equal(Vb[k].cpu().numpy(), V[k])
    say(f"  sweeps gpu {sw.tolist()} oracle {swr.tolist()}")


def test_complex128_upper_range_mixed_batch():
    """One mixed-shape call over shapes from the whole uneven range, largest
    ones included (n = 256, m = 512), against the oracle."""
    import torch
    from paper_2601_17979_amd import svdb
    shapes = [(512, 256), (256, 256), (300, 241), (17, 9), (64, 33), (130, 128), (8, 8)]
    mats = [gen.family(gen.rng_for(7700, k), "gauss", m, n, 1.0, complex_=True)
            for k, (m, n) in enumerate(shapes)]
    gm = [svdb.col_major(torch.from_numpy(a)[None].cuda())[0] for a in mats]
    S, U, V, info, sw = svdb.svd_batched(gm)
    torch.cuda.synchronize()
    import oracle
    for k, A in enumerate(mats):
        Sk, _, _, _, ik = oracle.gesvj(A)
        compare_with_oracle(A[None], S[k].cpu().numpy()[None], U[k].cpu().numpy()[None],
                            V[k].cpu().numpy()[None], info[k:k + 1].cpu().numpy(), Sk[None],
                            np.array([ik]), dtype=np.complex128, label=f"mixed #{k} {A.shape}")
