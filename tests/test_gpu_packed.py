"""GPU checks of the packed register layout of the resident kernel (m <= 32,
n <= 32: W rows in lanes 0..31 and V rows in lanes 32..63 of one register
slot).  Appending a zero row to A (m + 1 rows, past 32) moves the same
problem to the unpacked layout, where every Gram entry and norm gains only
exact zero terms and every rotation the same operands: the two runs must
agree bit for bit (the one-sided Jacobi method of Alg. 2 on [A; 0] performs
the rotations of A itself).  Both are also checked against the oracle."""
import numpy as np
import pytest

from workloads import gen
from gpu_util import compare_with_oracle, oracle_batch, run_gpu, say

pytestmark = pytest.mark.gpu


def _batch(m, n, count, seed):
    kinds = ("gauss", "geo", "cluster1", "cluster0")
    return np.stack([gen.family(gen.rng_for(seed, k), kinds[k % len(kinds)], m, n, 1e6)
                     for k in range(count)])


@pytest.mark.parametrize("m,n,waves", [(32, 32, 0), (32, 32, 2), (32, 32, 4), (25, 20, 0),
                                       (16, 16, 0), (16, 16, 2), (30, 12, 0), (1, 1, 0),
                                       (7, 3, 0), (32, 17, 0)])
def test_packed_equals_unpacked_on_zero_padded_copy(m, n, waves):
    from paper_2601_17979_amd import svdb
    import torch
    A = _batch(m, n, 24, seed=9600 + 33 * m + n)
    Ap = np.concatenate([A, np.zeros((A.shape[0], 33 - m, n))], axis=1)
    say(f"[packed {m}x{n} waves {waves}] plans {svdb.plan(torch.float64, m, n, path='resident')}"
        f" / {svdb.plan(torch.float64, 33, n, path='resident')}")
    S, U, V, info, sw = run_gpu(A, path="resident", precondition=0, waves=waves)
    S2, U2, V2, info2, sw2 = run_gpu(Ap, path="resident", precondition=0, waves=waves)
    assert np.array_equal(info, info2) and np.array_equal(sw, sw2)
    assert np.array_equal(S, S2)
    assert np.array_equal(V, V2)
    assert np.array_equal(U, U2[:, :m])
    assert not np.any(U2[:, m:])
    Sr, _, _, _, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"packed {m}x{n}")


def test_packed_edge_cases():
    """Zero matrix, rank one with a zero column (orthonormal completion of
    U), a NaN (info 2), entries near the overflow and underflow limits and
    max_sweeps = 1 on the packed layout: bitwise equal to the zero-padded
    unpacked run, and the finite ones against the oracle."""
    m, n = 24, 20
    A = _batch(m, n, 7, seed=9700)
    A[0] = 0.0
    x, y = gen.gaussian(gen.rng_for(9701, 0), m, 1), gen.gaussian(gen.rng_for(9701, 1), 1, n)
    y[0, 3] = 0.0
    A[1] = x @ y
    A[2, 4, 5] = np.nan
    A[3] *= 2.0 ** 900
    A[4] *= 2.0 ** -900
    Ap = np.concatenate([A, np.zeros((A.shape[0], 33 - m, n))], axis=1)
    for ms in (100, 1):
        S, U, V, info, sw = run_gpu(A, path="resident", precondition=0, max_sweeps=ms)
        S2, U2, V2, info2, sw2 = run_gpu(Ap, path="resident", precondition=0, max_sweeps=ms)
        assert info[2] == 2 and np.array_equal(info, info2) and np.array_equal(sw, sw2)
        ok = info != 2
        assert np.array_equal(S[ok], S2[ok]) and np.array_equal(V[ok], V2[ok])
        assert np.array_equal(U[ok], U2[ok][:, :m])
        if ms == 1:
            assert info[0] == 0 and np.all(info[[1, 3, 4, 5, 6]] == 1)
            continue
        assert np.all(info[ok] == 0)
        sc = np.array([1.0, 1.0, 1.0, 2.0 ** 900, 2.0 ** -900, 1.0, 1.0])[ok]
        As = A[ok] / sc[:, None, None]
        Sr, _, _, _, infor = oracle_batch(As)
        compare_with_oracle(As, S[ok] / sc[:, None], U[ok], V[ok], info[ok], Sr, infor,
                            label="packed edge")
