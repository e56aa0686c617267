"""GPU parity: the HIP paths against the FP64 oracle, through the C ABI.

Sizes are chosen so that the oracle finishes in seconds while spanning several
lane groups and ragged tails (m, n not multiples of the group widths); the
full-size workloads are checked on sampled matrices.  Tolerances: normwise
sigma error <= 1e-12, ||A - U S V^H||_F / ||A||_F <= 1e-13 n and
||U^H U - I||_F, ||V^H V - I||_F <= 1e-13 n (FP64).
"""
import numpy as np
import pytest

from workloads import gen
from gpu_util import aligned_vector_err, compare_with_oracle, oracle_batch, run_gpu, say

pytestmark = pytest.mark.gpu

PATHS = ["plain", "resident", "blocked"]


def _supported(path, m, n):
    import torch
    from paper_2601_17979_amd import svdb
    try:
        svdb.plan(torch.float64, m, n, path=path)
        return True
    except svdb.SvdbError:
        return False


def _batch(shape_list, seed, kind="gauss", kappa=1e6):
    out = []
    for k, (m, n) in enumerate(shape_list):
        r = gen.rng_for(seed, k)
        out.append(gen.family(r, kind, m, n, kappa))
    return np.stack(out)


@pytest.mark.parametrize("path", PATHS)
def test_small16_workload(path):
    """1000 x (16 x 16) FP64, A = U diag(s) V^T, s log-uniform [1e-3, 1],
    tol 1e-14: every matrix against the oracle."""
    A = gen.small16(batch=1000)[0].A
    say(f"[small16 {path}] batch {A.shape}")
    S, U, V, info, sw = run_gpu(A, tol=1e-14, path=path)
    Sr, Ur, Vr, swr, infor = oracle_batch(A, tol=1e-14)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"small16/{path}")
    worst = max(aligned_vector_err(S[k], U[k], V[k], Sr[k], Ur[k], Vr[k]) for k in range(100))
    assert worst <= 1e-13, worst
    say(f"  sweeps gpu {np.bincount(sw)} oracle {np.bincount(swr)}")


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("m,n", [(1, 1), (5, 1), (2, 2), (7, 3), (9, 9), (17, 9), (33, 17),
                                 (40, 40), (65, 31), (64, 64), (128, 32), (100, 100)])
def test_shapes_vs_oracle(path, m, n):
    """Ragged and odd shapes (phantom column for odd n), up to the LDS limit."""
    if not _supported(path, m, n):
        pytest.skip(f"{path} does not cover {m}x{n}")
    A = _batch([(m, n)] * 6, seed=100 + m * 7 + n, kind="gauss")
    A[1] = _batch([(m, n)], seed=200 + m, kind="geo", kappa=1e6)[0]
    A[2] = _batch([(m, n)], seed=300 + m, kind="cluster1", kappa=1e8)[0]
    say(f"[shape {m}x{n} {path}]")
    S, U, V, info, sw = run_gpu(A, path=path)
    Sr, Ur, Vr, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"{m}x{n}/{path}")


def _block_oracle(A, nb, max_sweeps=100, tol=None):
    import oracle
    out = [oracle.block_gesvj(A[k], nb, tol=tol, max_sweeps=max_sweeps, inner_sweeps=1)
           for k in range(A.shape[0])]
    return (np.stack([o[0] for o in out]), np.stack([o[1] for o in out]),
            np.stack([o[2] for o in out]), np.array([o[3] for o in out]),
            np.array([o[4] for o in out]))


def _one_sweep_oracle(A, path):
    if path == "blocked":
        return _block_oracle(A, 16, max_sweeps=1)
    return oracle_batch(A, max_sweeps=1, order=1)


def _one_sweep_sensitivity(A, path, trials=3, seed=7):
    """How far the oracle's own one-sweep iterate moves when every entry of A
    is perturbed by about one unit roundoff: each rotation angle follows
    (g_ii - g_jj) / (2 |g_ij|) (eq. sin-cos), which is ill-conditioned for
    nearly tied diagonal entries, so rounding-order differences between two
    correct implementations are bounded by this response, not by u.
    Returns (max over W = U S relative to max|A|, max over V, max over S
    relative to its largest entry)."""
    S, U, V, _, _ = _one_sweep_oracle(A, path)
    r = np.random.default_rng(seed)
    dw = dv = ds = 0.0
    for _ in range(trials):
        Ap = A * (1.0 + 2.0 ** -52 * r.standard_normal(A.shape))
        S2, U2, V2, _, _ = _one_sweep_oracle(Ap, path)
        dw = max(dw, float(np.max(np.abs(U2 * S2[:, None, :] - U * S[:, None, :]) /
                                  np.abs(A).max(axis=(1, 2), keepdims=True))))
        dv = max(dv, float(np.abs(V2 - V).max()))
        ds = max(ds, float(np.abs(S2 - S).max() / S.max()))
    return dw, dv, ds


@pytest.mark.parametrize("path", PATHS)
def test_one_sweep_elementwise(path):
    """After exactly one sweep (max_sweeps = 1, info = 1) the GPU iterate
    matches the oracle run in the same round-robin order element by element:
    this pins the pair schedule, the rotation and its orientation (for the
    block path: the block pairs, the Gram matrix, the inner sweep of Alg. 1
    and the update by J).  A wrong schedule or orientation moves the iterate
    by O(1); the bound (on S, W and V) is 1e-13 (V: 1e-12) or ten times the
    oracle's own response to perturbations of A of one unit roundoff,
    whichever is larger."""
    for m, n in [(24, 16), (40, 32), (64, 64)]:
        A = _batch([(m, n)] * 8, seed=400 + n)
        S, U, V, info, sw = run_gpu(A, path=path, max_sweeps=1, inner_sweeps=1)
        Sr, Ur, Vr, swr, infor = _one_sweep_oracle(A, path)
        dw, dv, ds = _one_sweep_sensitivity(A, path)
        tol_w, tol_v, tol_s = max(1e-13, 10 * dw), max(1e-12, 10 * dv), max(1e-13, 10 * ds)
        assert np.all(info == 1) and np.all(infor == 1) and np.all(sw == 1)
        assert np.abs(S - Sr).max() <= tol_s * Sr.max(), (m, n, np.abs(S - Sr).max() / Sr.max())
        # the iterate W = A V = U diag(S), element by element, relative to max|A|
        W, Wr = U * S[:, None, :], Ur * Sr[:, None, :]
        ew = float(np.max(np.abs(W - Wr) / np.abs(A).max(axis=(1, 2), keepdims=True)))
        ev = float(np.abs(V - Vr).max())
        say(f"  {m}x{n} {path}: W diff {ew:.2e} (bound {tol_w:.2e}), "
            f"V diff {ev:.2e} (bound {tol_v:.2e})")
        assert ew <= tol_w, (m, n, ew, tol_w)
        assert ev <= tol_v, (m, n, ev, tol_v)


@pytest.mark.parametrize("path", PATHS)
def test_sweep_counts_match_round_robin_oracle(path):
    """Same ordering, same threshold: the sweep counts agree (within one
    sweep, since rounding can move the last decision)."""
    A = _batch([(32, 32)] * 16, seed=500, kind="geo", kappa=1e6)
    S, U, V, info, sw = run_gpu(A, path=path, inner_sweeps=1)
    if path == "blocked":
        Sr, Ur, Vr, swr, infor = _block_oracle(A, 16)
    else:
        Sr, Ur, Vr, swr, infor = oracle_batch(A, order=1)
    assert np.all(np.abs(sw - swr) <= 1), (sw, swr)


@pytest.mark.parametrize("path", PATHS)
def test_edge_cases(path):
    """Zero matrix, exactly rank-1 with a zero column (orthonormal
    completion of U), a NaN (info 2), Inf (info 2), max_sweeps = 1 (info 1)."""
    m, n = 12, 7
    A = _batch([(m, n)] * 6, seed=600)
    A[0] = 0.0
    x, y = gen.gaussian(gen.rng_for(601, 0), m, 1), gen.gaussian(gen.rng_for(601, 1), 1, n)
    y[0, 3] = 0.0
    A[1] = x @ y
    A[2, 4, 5] = np.nan
    A[3, 0, 0] = np.inf
    S, U, V, info, sw = run_gpu(A, path=path)
    Sr, Ur, Vr, swr, infor = oracle_batch(A)
    assert list(info) == [0, 0, 2, 2, 0, 0]
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"edge/{path}")
    S1, U1, V1, info1, sw1 = run_gpu(A[4:], path=path, max_sweeps=1)
    assert np.all(info1 == 1) and np.all(sw1 == 1)


@pytest.mark.parametrize("path", PATHS)
def test_deterministic(path):
    """Two runs give bitwise identical results (no races in LDS)."""
    A = _batch([(64, 64)] * 32, seed=700, kind="geo")
    r1 = run_gpu(A, path=path)
    r2 = run_gpu(A, path=path)
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("path", PATHS)
def test_scale_extremes(path):
    """Entries near the overflow and underflow limits: the power-of-two
    pre-scaling makes the result the scaled result of a unit-size matrix."""
    A = _batch([(20, 10)] * 3, seed=800)
    A[0] *= 2.0 ** 900
    A[1] *= 2.0 ** -900
    S, U, V, info, sw = run_gpu(A, path=path)
    Sr, Ur, Vr, swr, infor = oracle_batch(A / np.array([2.0 ** 900, 2.0 ** -900, 1.0])[:, None, None])
    assert np.all(info == 0)
    scales = np.array([2.0 ** 900, 2.0 ** -900, 1.0])
    for k in range(3):
        assert np.abs(S[k] / scales[k] - Sr[k]).max() <= 1e-13 * Sr[k][0]


def test_full_mixed_workload_sampled():
    """10000 FP64 matrices (5000 of 64 x 64, 5000 of 128 x 32, half geometric
    kappa = 1e6, half Gaussian) through the default path, exactly as the
    benchmark launches them; 120 sampled matrices per shape against the
    oracle, and invariants on every matrix."""
    import torch
    from metrics import orth_err, recon_err
    groups = gen.mixed_64_128x32()
    rng = np.random.default_rng(1)
    for g in groups:
        say(f"[full mixed] {g.m}x{g.n} batch {g.A.shape[0]}")
        S, U, V, info, sw = run_gpu(g.A, path="auto")
        assert np.all(info == 0)
        idx = np.sort(rng.choice(g.A.shape[0], 120, replace=False))
        Sr, Ur, Vr, swr, infor = oracle_batch(g.A[idx])
        compare_with_oracle(g.A[idx], S[idx], U[idx], V[idx], info[idx], Sr, infor,
                            label=f"full {g.m}x{g.n}")
        # invariants on all matrices (cheap, vectorised)
        R = g.A - np.einsum("bij,bj,bkj->bik", U, S, V)
        rel = np.linalg.norm(R, axis=(1, 2)) / np.linalg.norm(g.A, axis=(1, 2))
        assert rel.max() <= 1e-13 * g.n, rel.max()
        assert np.all(np.diff(S, axis=1) <= 0)
        say(f"  sweeps histogram {np.bincount(sw)}")
        del S, U, V
        torch.cuda.empty_cache()


@pytest.mark.parametrize("nb", [16, 32])
@pytest.mark.parametrize("m,n", [(96, 80), (130, 65), (200, 130), (256, 256)])
def test_blocked_larger_shapes(nb, m, n):
    """Block path beyond the register-resident sizes: several block pairs per
    iteration, padded block columns (n not a multiple of nb), ragged row
    chunks (m not a multiple of 64)."""
    A = _batch([(m, n)] * 3, seed=900 + m + n, kind="gauss")
    A[1] = _batch([(m, n)], seed=950 + m, kind="geo", kappa=1e8)[0]
    say(f"[blocked {m}x{n} nb {nb}]")
    S, U, V, info, sw = run_gpu(A, path="blocked", nb=nb)
    Sr, Ur, Vr, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"blocked {m}x{n} nb{nb}")
    say(f"  sweeps gpu {list(sw)} oracle {list(swr)}")


@pytest.mark.parametrize("m,n", [(3, 0), (0, 0), (0, 3)])
def test_no_singular_values(m, n):
    """min(m, n) = 0 in every dtype: nothing to factor, info 0 and sweeps 0
    for every matrix of the batch."""
    import torch
    from paper_2601_17979_amd import svdb
    for dt in (torch.float32, torch.float64, torch.complex64, torch.complex128):
        A = torch.zeros((4, m, n), dtype=dt, device="cuda")
        S, U, V, info, sw = svdb.svd(A)
        torch.cuda.synchronize()
        assert S.shape == (4, 0) and U.shape == (4, m, 0) and V.shape == (4, n, 0)
        assert info.cpu().tolist() == [0] * 4 and sw.cpu().tolist() == [0] * 4
