"""GPU parity of uneven batches (svdb_svd_batched: one pointer and one shape
per matrix) against the oracle, through the C ABI.

Every matrix runs the block method on its own round-robin schedule, so a
matrix's result does not depend on the rest of the batch: checked bitwise
(alone vs. in a mixed batch, and against the uniform-shape block path)."""
import numpy as np
import pytest

import oracle
from workloads import gen
from gpu_util import compare_with_oracle, say

pytestmark = pytest.mark.gpu


def _run_batched(mats, dtype, **kw):
    import torch
    from paper_2601_17979_amd import svdb
    gm = [svdb.col_major(torch.from_numpy(np.ascontiguousarray(a))[None].to(dtype).cuda())[0]
          for a in mats]
    S, U, V, info, sw = svdb.svd_batched(gm, **kw)
    torch.cuda.synchronize()
    return ([s.cpu().numpy() for s in S], [u.cpu().numpy() for u in U],
            [v.cpu().numpy() for v in V], info.cpu().numpy(), sw.cpu().numpy())


def _check(mats, S, U, V, info, dtype, label):
    for k, A in enumerate(mats):
        A64 = A.astype(np.complex128 if np.iscomplexobj(A) else np.float64)
        if A.shape[1] == 0:
            assert info[k] == 0
            continue
        Sr, _, _, _, infor = oracle.gesvj(A64)
        compare_with_oracle(A64[None], S[k][None].astype(np.float64), U[k][None].astype(A64.dtype),
                            V[k][None].astype(A64.dtype), info[k:k + 1], Sr[None],
                            np.array([infor]), dtype=dtype, label=f"{label} #{k} {A.shape}")


SHAPES = [(1, 1), (5, 0), (7, 3), (16, 16), (17, 16), (40, 33), (64, 64), (128, 32), (90, 47),
          (33, 33), (200, 130), (2, 2), (150, 120)]


@pytest.mark.parametrize("dt", ["f64", "f32", "c128", "c64"])
def test_uneven_shapes_vs_oracle(dt):
    import torch
    cx = dt.startswith("c")
    kinds = ("gauss", "geo", "random")
    mats = [gen.family(gen.rng_for(9100, k), kinds[k % 3], m, n, 1e6, complex_=cx)
            if n > 0 else np.zeros((m, 0), np.complex128 if cx else np.float64)
            for k, (m, n) in enumerate(SHAPES)]
    npdt = {"f64": np.float64, "f32": np.float32, "c128": np.complex128, "c64": np.complex64}[dt]
    tdt = {"f64": torch.float64, "f32": torch.float32, "c128": torch.complex128,
           "c64": torch.complex64}[dt]
    mats = [a.astype(npdt) for a in mats]
    say(f"[uneven {dt}] {len(mats)} matrices")
    S, U, V, info, sw = _run_batched(mats, tdt)
    _check(mats, S, U, V, info, npdt, f"uneven {dt}")
    say(f"  sweeps {sw.tolist()}")


def test_uneven_complex_workload_sample():
    """60 matrices of the uneven complex128 workload recipe (n ~ U{8..160},
    m ~ U{n..2n}, complex Gaussian entries) in one call."""
    import torch
    groups = gen.uneven_complex(batch=60, nmax=160)
    mats = [g.A[k] for g in groups for k in range(g.A.shape[0])]
    say(f"[uneven complex workload] {len(mats)} matrices, {len(groups)} shapes")
    S, U, V, info, sw = _run_batched(mats, torch.complex128)
    _check(mats, S, U, V, info, np.complex128, "uneven cplx")
    say(f"  sweeps min {sw.min()} max {sw.max()}")


def test_result_independent_of_the_batch():
    """A matrix alone and inside a mixed batch gives bitwise the same
    outputs; so does the uniform-shape block path with nb = 16."""
    import torch
    from paper_2601_17979_amd import svdb
    mats = [gen.gaussian(gen.rng_for(9200, k), m, n) for k, (m, n) in
            enumerate([(70, 50), (20, 9), (130, 100), (64, 64)])]
    S, U, V, info, sw = _run_batched(mats, torch.float64)
    for k, A in enumerate(mats):
        S1, U1, V1, i1, s1 = _run_batched([A], torch.float64)
        assert np.array_equal(S1[0], S[k]) and np.array_equal(U1[0], U[k])
        assert np.array_equal(V1[0], V[k]) and i1[0] == info[k] and s1[0] == sw[k]
        Ag = svdb.col_major(torch.from_numpy(A)[None].cuda())
        S2, U2, V2, i2, s2 = svdb.svd(Ag, path="blocked", nb=16)
        torch.cuda.synchronize()
        assert np.array_equal(S2.cpu().numpy()[0], S[k]), k
        assert np.array_equal(U2.cpu().numpy()[0], U[k]), k
        assert np.array_equal(V2.cpu().numpy()[0], V[k]), k
        assert int(s2.cpu()[0]) == sw[k]


def test_uneven_edge_cases():
    import torch
    mats = [gen.gaussian(gen.rng_for(9300, k), 30, 20) for k in range(4)]
    mats[0][:] = 0.0
    mats[1][3, 4] = np.nan
    mats[2][:, 5] = 0.0
    S, U, V, info, sw = _run_batched(mats, torch.float64)
    assert info[1] == 2
    assert np.all(S[0] == 0.0) and info[0] == 0
    keep = [0, 2, 3]
    _check([mats[k] for k in keep], [S[k] for k in keep], [U[k] for k in keep],
           [V[k] for k in keep], info[keep], np.float64, "uneven edge")
