"""GPU parity of the QR-preconditioned paths against the FP64 oracle, through
the C ABI.  Resident path (n <= 64): A P = Q1 R1 (pivoted), R1^T = Q2 R2, the
Jacobi on R2^T, U = Q1 U_x, V = P Q2 J.  Wide path: A = Q R, the block Jacobi
on R^T, U = Q J.  FP64 tolerances: normwise sigma error <= 1e-12,
reconstruction and orthogonality <= 1e-13 n."""
import numpy as np
import pytest

from workloads import gen
from gpu_util import aligned_vector_err, compare_with_oracle, oracle_batch, run_gpu, say

pytestmark = pytest.mark.gpu


def _batch(shape, count, seed, kinds=("gauss", "geo", "cluster1", "random"), kappa=1e6):
    m, n = shape
    return np.stack([gen.family(gen.rng_for(seed, k), kinds[k % len(kinds)], m, n, kappa)
                     for k in range(count)])


SHAPES = [(1, 1), (2, 2), (7, 3), (16, 16), (17, 9), (40, 24), (64, 64), (65, 31), (100, 50),
          (128, 32), (128, 64), (256, 32)]


@pytest.mark.parametrize("path", ["auto", "resident"])
@pytest.mark.parametrize("m,n", SHAPES)
def test_precond_vs_oracle(m, n, path):
    A = _batch((m, n), 8, seed=8100 + 7 * m + n)
    A[3] = _batch((m, n), 1, seed=8200 + m, kinds=("geo",), kappa=1e12)[0]
    say(f"[precond {m}x{n} {path}]")
    S, U, V, info, sw = run_gpu(A, path=path, precondition=1)
    Sr, Ur, Vr, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"precond {m}x{n}")
    worst = max(aligned_vector_err(S[k], U[k] * S[k] / S[k][0], V[k], Sr[k],
                                   Ur[k] * Sr[k] / Sr[k][0], Vr[k]) for k in range(8))
    assert worst <= 1e-12, worst
    say(f"  sweeps gpu {sw.tolist()} oracle {swr.tolist()}")


@pytest.mark.parametrize("m,n", [(1, 1), (2, 2), (7, 3), (16, 16), (17, 9), (30, 20), (32, 32),
                                 (40, 24), (50, 37), (64, 64), (64, 40)])
def test_precond_pivoted_vs_oracle(m, n):
    """Column pivoting at every n (precondition 2); up to 64 rows the pivoted
    QR runs one wave per matrix with one column per lane (every row-block
    count), beyond it the register QR of 16-lane groups."""
    A = _batch((m, n), 8, seed=8300 + 7 * m + n)
    A[3] = _batch((m, n), 1, seed=8400 + m, kinds=("geo",), kappa=1e12)[0]
    say(f"[precond pivoted {m}x{n}]")
    S, U, V, info, sw = run_gpu(A, precondition=2)
    Sr, Ur, Vr, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"pivoted {m}x{n}")


def test_precond_is_the_auto_default_and_saves_sweeps():
    """AUTO uses the preconditioned path where it applies; on graded
    (geometric kappa 1e6) matrices it needs fewer sweeps than the iteration
    on A itself."""
    import torch
    from paper_2601_17979_amd import svdb
    path, nb, thr = svdb.plan(torch.float64, 64, 64)
    assert path == svdb.PATH_RESIDENT
    A = _batch((64, 64), 16, seed=8300, kinds=("geo",))
    _, _, _, _, sw_pc = run_gpu(A)
    _, _, _, _, sw_a = run_gpu(A, precondition=0)
    say(f"[precond sweeps] R^T {sw_pc.mean():.2f} vs A {sw_a.mean():.2f}")
    assert sw_pc.mean() < 0.8 * sw_a.mean()


@pytest.mark.parametrize("want", [(True, False), (False, True), (False, False)])
def test_precond_optional_outputs(want):
    cu, cv = want
    A = _batch((48, 32), 4, seed=8400)
    S, U, V, info, sw = run_gpu(A, compute_u=cu, compute_v=cv, precondition=1)
    Sr, Ur, Vr, _, infor = oracle_batch(A)
    assert np.all(info == 0)
    assert (U is None) != cu and (V is None) != cv
    assert max(np.abs(S[k] - Sr[k]).max() / Sr[k][0] for k in range(4)) <= 1e-12
    for k in range(4):
        if U is not None:
            assert np.linalg.norm(U[k].T @ U[k] - np.eye(32)) <= 1e-13 * 32
        if V is not None:
            assert np.linalg.norm(V[k].T @ V[k] - np.eye(32)) <= 1e-13 * 32


@pytest.mark.parametrize("m,n,pc", [(40, 24, 1), (40, 24, 2), (64, 64, 1), (100, 64, 2)])
def test_precond_edge_cases(m, n, pc):
    """Zero and rank-deficient matrices, extreme scales, and non-finite input
    (info 2, outputs untouched), through the unpivoted and both pivoted QR
    kernels."""
    import torch
    from paper_2601_17979_amd import svdb
    A = _batch((m, n), 6, seed=8500 + m + n)
    A[0] = 0.0
    A[1][:, 3] = 0.0
    A[1][:, 7] = A[1][:, 5]
    A[2][4, 4] = np.nan
    A[3][1, 2] = -np.inf
    A[4] *= 2.0 ** 600
    A[5] *= 2.0 ** -600
    Ag = svdb.col_major(torch.from_numpy(A).cuda())
    out = (torch.full((6, n), 7.0, dtype=torch.float64, device="cuda"),
           svdb.empty_col_major(6, m, n, torch.float64, "cuda").fill_(7.0),
           svdb.empty_col_major(6, n, n, torch.float64, "cuda").fill_(7.0),
           torch.empty(6, dtype=torch.int32, device="cuda"),
           torch.empty(6, dtype=torch.int32, device="cuda"))
    say(f"[precond edge {m}x{n} pc {pc}]")
    svdb.svd(Ag, out=out, precondition=pc)
    torch.cuda.synchronize()
    S, U, V, info, sw = (x.cpu().numpy() for x in out)
    assert info[2] == 2 and info[3] == 2
    for k in (2, 3):
        assert np.all(U[k] == 7.0) and np.all(V[k] == 7.0)
    keep = [0, 1, 4, 5]
    # the oracle runs unscaled (its Gram sums would overflow at 2^600):
    # compare the scaled results with the scaled oracle
    scales = np.array([1.0, 1.0, 2.0 ** 600, 2.0 ** -600])
    A0 = A[keep] / scales[:, None, None]
    Sr, _, _, _, infor = oracle_batch(A0)
    compare_with_oracle(A0, S[keep] / scales[:, None], U[keep], V[keep], info[keep], Sr, infor,
                        label="precond edge")
    assert np.all(S[0] == 0.0)


def test_precond_mixed_workload_sample():
    """Matrices of the 64 x 64 / 128 x 32 workload through AUTO."""
    groups = gen.mixed_64_128x32(batch=400)
    for g in groups:
        A = g.A[::10]
        S, U, V, info, sw = run_gpu(A)
        Sr, _, _, swr, infor = oracle_batch(A)
        compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"auto {g.m}x{g.n}")
        say(f"  {g.m}x{g.n}: sweeps gpu {sw.mean():.2f} oracle on A {swr.mean():.2f}")


@pytest.mark.parametrize("pc", [-1, 2])
def test_precond_sweeps_match_the_oracle_pipeline(pc):
    """The resident path follows the oracle's preconditioned driver (QR,
    with column pivoting for 32 < n <= 64 and, with precondition 2, at every
    n, second QR, Alg. 2 on R2^T): same SVD, and sweep counts within one of
    the oracle's on every matrix of a workload sample (rounding can move a
    pair across the threshold, never the whole schedule)."""
    import oracle
    groups = gen.mixed_64_128x32(batch=400)
    for g in groups:
        A = g.A[::8]
        S, U, V, info, sw = run_gpu(A, precondition=pc)
        pivot = pc == 2 or 32 < g.n <= 64
        Sr, Ur, Vr, swr, infor = oracle.precond_gesvj_batch(A, pivot=pivot)
        compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"pipeline {g.m}x{g.n} pc {pc}")
        say(f"  {g.m}x{g.n} pc {pc}: sweeps gpu {sw.mean():.2f} oracle pipeline {swr.mean():.2f}")
        assert np.all(np.abs(sw - swr) <= 1), (sw.tolist(), swr.tolist())


@pytest.mark.parametrize("pc", [1, 2])
@pytest.mark.parametrize("m,n", [(33, 33), (48, 40), (64, 64), (100, 64), (160, 50)])
def test_precond_v_from_triangular_solve(m, n, pc):
    """For 32 < n <= 64 the Jacobi on X = R2^T accumulates no rotations:
    J = X^-1 U_x diag(S) comes from a triangular solve, and only matrices
    whose J fails the orthogonality check run the Jacobi again with J
    accumulated.  The batch holds matrices that pass (well and badly
    conditioned, graded) and ones that fail (X singular: repeated and zero
    columns), all compared with the oracle; S and U are the same bits
    whether V is asked for or not (the Jacobi on W does not depend on J)."""
    A = _batch((m, n), 10, seed=8700 + m + n)
    A[2] = _batch((m, n), 1, seed=8800 + m, kinds=("geo",), kappa=1e12)[0]
    A[3] = _batch((m, n), 1, seed=8810 + m, kinds=("random",), kappa=1e14)[0]
    A[4][:, 5] = A[4][:, 9]
    A[5][:, 1] = 0.0
    A[5][:, n - 1] = 0.0
    A[6][:, :] = np.outer(A[6][:, 0], np.arange(1, n + 1))   # rank one
    A[7][:, n // 2:] = A[7][:, :n - n // 2] * 3.0             # rank n - n // 2
    say(f"[precond nv {m}x{n} pc {pc}]")
    S, U, V, info, sw = run_gpu(A, precondition=pc)
    Sr, Ur, Vr, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"precond nv {m}x{n}")
    S1, U1, V1, info1, sw1 = run_gpu(A, precondition=pc, compute_v=False)
    assert V1 is None
    assert np.array_equal(S, S1) and np.array_equal(U, U1)
    assert np.array_equal(info, info1) and np.array_equal(sw, sw1)


@pytest.mark.parametrize("m,n,count", [(96, 65, 4), (130, 96, 4), (200, 130, 3), (256, 256, 2),
                                       (1000, 100, 2)])
def test_precond_wide_vs_oracle(m, n, count):
    """n > 64: QR in global memory, the block Jacobi on R^T, U = Q J."""
    import torch
    from paper_2601_17979_amd import svdb
    assert svdb.plan(torch.float64, m, n)[0] == svdb.PATH_BLOCKED
    A = _batch((m, n), count, seed=8600 + m + n, kinds=("geo", "gauss", "cluster1"), kappa=1e8)
    say(f"[precond wide {m}x{n}]")
    S, U, V, info, sw = run_gpu(A)
    Sr, Ur, Vr, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"precond wide {m}x{n}")
    _, _, _, _, sw0 = run_gpu(A, path="blocked", nb=16 if n <= 96 else 32)
    say(f"  sweeps on R^T {sw.tolist()} on A {sw0.tolist()} oracle {swr.tolist()}")


def test_precond_wide_edge_cases():
    import torch
    from paper_2601_17979_amd import svdb
    m, n = 150, 100
    A = _batch((m, n), 4, seed=8700)
    A[0] = 0.0
    A[1][:, 10] = 0.0
    A[1][:, 20] = A[1][:, 30]
    A[2][5, 5] = np.nan
    Ag = svdb.col_major(torch.from_numpy(A).cuda())
    out = (torch.full((4, n), 7.0, dtype=torch.float64, device="cuda"),
           svdb.empty_col_major(4, m, n, torch.float64, "cuda").fill_(7.0),
           svdb.empty_col_major(4, n, n, torch.float64, "cuda").fill_(7.0),
           torch.empty(4, dtype=torch.int32, device="cuda"),
           torch.empty(4, dtype=torch.int32, device="cuda"))
    svdb.svd(Ag, out=out)
    torch.cuda.synchronize()
    S, U, V, info, sw = (x.cpu().numpy() for x in out)
    assert info[2] == 2 and np.all(U[2] == 7.0)
    keep = [0, 1, 3]
    Sr, _, _, _, infor = oracle_batch(A[keep])
    compare_with_oracle(A[keep], S[keep], U[keep], V[keep], info[keep], Sr, infor,
                        label="precond wide edge")


@pytest.mark.parametrize("m,n,count", [(257, 16, 4), (512, 16, 4), (1000, 16, 3), (2000, 16, 2),
                                       (4096, 16, 2), (1000, 40, 2), (300, 64, 3), (4000, 7, 2),
                                       (600, 1, 2)])
def test_precond_tall_vs_oracle(m, n, count):
    """Tall matrices with few columns beyond the register QR (the paper's
    tall-skinny experiment, n = 16 and m up to 2000): QR in global memory,
    the resident Jacobi on R^T, U = Q J by one wave per column."""
    import torch
    from paper_2601_17979_amd import svdb
    # AUTO takes the tall path up to m = 1024; precondition = 1 up to 4096
    assert (svdb.plan(torch.float64, m, n)[0] == svdb.PATH_RESIDENT) == (m <= 1024)
    assert svdb.plan(torch.float64, m, n, precondition=1)[0] == svdb.PATH_RESIDENT
    A = _batch((m, n), count, seed=8700 + m + n, kinds=("geo", "gauss", "random"), kappa=1e8)
    say(f"[precond tall {m}x{n}]")
    S, U, V, info, sw = run_gpu(A, precondition=1)
    Sr, Ur, Vr, swr, infor = oracle_batch(A)
    compare_with_oracle(A, S, U, V, info, Sr, infor, label=f"precond tall {m}x{n}")
    say(f"  sweeps on R^T {sw.tolist()} oracle on A {swr.tolist()}")


def test_precond_tall_edge_cases_and_outputs():
    """Zero and rank-deficient tall matrices, non-finite input (info 2,
    outputs untouched), and each optional output."""
    import torch
    from paper_2601_17979_amd import svdb
    m, n = 700, 12
    A = _batch((m, n), 5, seed=8800)
    A[0] = 0.0
    A[1][:, 3] = 0.0
    A[1][:, 7] = A[1][:, 5]
    A[2][4, 4] = np.nan
    A[3] *= 2.0 ** 400
    Ag = svdb.col_major(torch.from_numpy(A).cuda())
    out = (torch.full((5, n), 7.0, dtype=torch.float64, device="cuda"),
           svdb.empty_col_major(5, m, n, torch.float64, "cuda").fill_(7.0),
           svdb.empty_col_major(5, n, n, torch.float64, "cuda").fill_(7.0),
           torch.empty(5, dtype=torch.int32, device="cuda"),
           torch.empty(5, dtype=torch.int32, device="cuda"))
    svdb.svd(Ag, out=out)
    torch.cuda.synchronize()
    S, U, V, info, sw = (x.cpu().numpy() for x in out)
    assert info[2] == 2 and np.all(U[2] == 7.0) and np.all(V[2] == 7.0)
    keep = [0, 1, 3, 4]
    scales = np.array([1.0, 1.0, 2.0 ** 400, 1.0])
    A0 = A[keep] / scales[:, None, None]
    Sr, _, _, _, infor = oracle_batch(A0)
    compare_with_oracle(A0, S[keep] / scales[:, None], U[keep], V[keep], info[keep], Sr, infor,
                        label="precond tall edge")
    assert np.all(S[0] == 0.0)
    B = A[[0, 1, 4]]
    Sr = oracle_batch(B)[0]
    for cu, cv in ((True, False), (False, True)):
        S, U, V, info, sw = run_gpu(B, compute_u=cu, compute_v=cv)
        assert np.all(info == 0)
        assert np.abs(S - Sr).max() <= 1e-12 * max(Sr.max(), 1.0)
        if U is not None:
            assert max(np.linalg.norm(U[k].T @ U[k] - np.eye(n)) for k in (1, 2)) <= 1e-13 * n
        if V is not None:
            assert max(np.linalg.norm(V[k].T @ V[k] - np.eye(n)) for k in range(3)) <= 1e-13 * n


@pytest.mark.parametrize("m,n", [(64, 64), (128, 32), (40, 24), (256, 256), (200, 130),
                                 (1000, 16), (700, 40)])
def test_precond_fp32_input_runs_in_fp64(m, n):
    """FP32 input on the QR-preconditioned paths: A is widened, the FP64
    kernels run with the FP32 threshold (30 u of FP32), and S, U, V are
    narrowed; judged against the oracle on the widened input with the FP32
    tolerances, and against the FP32 block method without QR (which it
    matches in sigma to FP32 accuracy, in far fewer sweeps)."""
    import torch
    from paper_2601_17979_amd import svdb
    assert svdb.plan(torch.float32, m, n) == svdb.plan(torch.float64, m, n)
    count = 2 if m * n > 20000 else 5
    A = _batch((m, n), count, seed=8900 + m + n, kinds=("geo", "gauss"), kappa=1e4)
    A32 = A.astype(np.float32)
    say(f"[precond fp32 {m}x{n}]")
    S, U, V, info, sw = run_gpu(A32, dtype=torch.float32)
    assert S.dtype == np.float32 and U.dtype == np.float32 and V.dtype == np.float32
    A64 = A32.astype(np.float64)
    Sr, _, _, _, infor = oracle_batch(A64)
    compare_with_oracle(A64, S.astype(np.float64), U.astype(np.float64), V.astype(np.float64),
                        info, Sr, infor, dtype=np.float32, label=f"precond fp32 {m}x{n}")
    _, _, _, _, sw0 = run_gpu(A32, dtype=torch.float32, precondition=0)
    say(f"  sweeps {sw.tolist()} without QR (FP32 block) {sw0.tolist()}")


def test_precond_fp32_edge_cases():
    """Zero and rank-deficient FP32 input; a NaN gives info 2 with the FP32
    outputs untouched."""
    import torch
    from paper_2601_17979_amd import svdb
    m, n = 48, 32
    A = _batch((m, n), 4, seed=8950).astype(np.float32)
    A[0] = 0.0
    A[1][:, 3] = 0.0
    A[2][5, 6] = np.nan
    Ag = svdb.col_major(torch.from_numpy(A).cuda())
    out = (torch.full((4, n), 7.0, dtype=torch.float32, device="cuda"),
           svdb.empty_col_major(4, m, n, torch.float32, "cuda").fill_(7.0),
           svdb.empty_col_major(4, n, n, torch.float32, "cuda").fill_(7.0),
           torch.empty(4, dtype=torch.int32, device="cuda"),
           torch.empty(4, dtype=torch.int32, device="cuda"))
    svdb.svd(Ag, out=out)
    torch.cuda.synchronize()
    S, U, V, info, sw = (x.cpu().numpy() for x in out)
    assert info[2] == 2
    assert np.all(S[2] == 7.0) and np.all(U[2] == 7.0) and np.all(V[2] == 7.0)
    keep = [0, 1, 3]
    A64 = A[keep].astype(np.float64)
    Sr, _, _, _, infor = oracle_batch(A64)
    compare_with_oracle(A64, S[keep].astype(np.float64), U[keep].astype(np.float64),
                        V[keep].astype(np.float64), info[keep], Sr, infor, dtype=np.float32,
                        label="precond fp32 edge")
    assert np.all(S[0] == 0.0)


@pytest.mark.parametrize("m,n", [(1024, 1024), (1024, 520)])
def test_precond_wide_at_the_maximum_size(m, n):
    """The largest wide preconditioned shapes (m = 1024): the oracle would
    take minutes here, so the result is judged by properties that hold at
    any size (reconstruction, orthogonality, ordering) and by LAPACK's
    singular values (numpy.linalg.svd) at the FP64 tolerances."""
    from metrics import orth_err, recon_err, tolerances
    A = _batch((m, n), 1, seed=9000 + n, kinds=("geo",), kappa=1e6)
    say(f"[precond wide max {m}x{n}]")
    S, U, V, info, sw = run_gpu(A)
    ref = np.linalg.svd(A[0], compute_uv=False)
    tol_s, tol_r, tol_o = tolerances(np.float64, n)
    assert info[0] == 0
    assert np.abs(S[0] - ref).max() / ref[0] <= tol_s
    assert recon_err(A[0], S[0], U[0], V[0]) <= tol_r
    assert orth_err(U[0]) <= tol_o and orth_err(V[0]) <= tol_o
    assert np.all(np.diff(S[0]) <= 0)
    say(f"  sweeps {sw.tolist()}")


@pytest.mark.parametrize("m,n,qr", [(16, 16, False), (100, 16, False), (127, 16, False),
                                    (128, 16, True), (63, 8, False), (64, 8, True),
                                    (17, 17, True), (40, 24, True)])
def test_auto_skips_qr_for_few_columns(m, n, qr):
    """AUTO leaves out the QR pre-processing for FP64 with n <= 16 and
    m < 8 n (where it costs more than the sweeps it saves): its result is
    bit for bit that of precondition 0 there, and of precondition 1 elsewhere."""
    A = _batch((m, n), 6, seed=9800 + m + n, kinds=("gauss", "geo", "random"))
    auto = run_gpu(A)
    ref = run_gpu(A, precondition=1 if qr else 0)
    for x, y in zip(auto, ref):
        assert np.array_equal(x, y)
    Sr, _, _, _, infor = oracle_batch(A)
    compare_with_oracle(A, auto[0], auto[1], auto[2], auto[3], Sr, infor, label=f"auto {m}x{n}")


@pytest.mark.parametrize("m,n,pc", [(64, 64, 1), (128, 32, 1), (48, 40, 2), (40, 24, 1)])
def test_precond_ignores_stale_workspace(m, n, pc):
    """The kernels of the preconditioned path hand each other triangular
    factors and reflectors written and read only from the diagonal down; the
    rest of the workspace is never read.  A workspace full of NaN bytes from
    an earlier use must give the same bits as a zeroed one (rank-deficient
    matrices included, whose V comes from the V-accumulating rerun)."""
    import ctypes as C
    import torch
    from paper_2601_17979_amd import svdb
    A = _batch((m, n), 6, seed=8600 + m + n)
    A[2][:, 5] = 0.0
    A[2][:, 7] = A[2][:, 6]
    Ag = svdb.col_major(torch.from_numpy(A).cuda())
    L = svdb.lib()
    b, k = A.shape[0], min(m, n)
    o = svdb.make_opts(precondition=pc)
    ws_bytes = L.svdb_workspace_size(svdb.dtype_code(Ag.dtype), b, m, n, C.byref(o))
    assert ws_bytes > 0
    outs = []
    for fill in (0, 255):
        S = torch.empty((b, k), dtype=torch.float64, device="cuda")
        U = svdb.empty_col_major(b, m, k, torch.float64, "cuda")
        V = svdb.empty_col_major(b, n, k, torch.float64, "cuda")
        info = torch.empty(b, dtype=torch.int32, device="cuda")
        ws = torch.full((ws_bytes,), fill, dtype=torch.uint8, device="cuda")
        say(f"[stale workspace {m}x{n} pc {pc} fill {fill}]")
        rc = L.svdb_svd_strided_batched(
            svdb.dtype_code(Ag.dtype), b, m, n, Ag.data_ptr(), Ag.stride(2), Ag.stride(0),
            S.data_ptr(), S.stride(0), U.data_ptr(), U.stride(2), U.stride(0), V.data_ptr(),
            V.stride(2), V.stride(0), 0.0, info.data_ptr(), ws.data_ptr(), ws_bytes, C.byref(o),
            torch.cuda.current_stream().cuda_stream)
        assert rc == 0, svdb.last_error()
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in (S, U, V, info)])
    for x0, x1 in zip(*outs):
        assert np.array_equal(x0, x1)
    assert np.all(outs[0][3] == 0)
    Sr, _, _, _, infor = oracle_batch(A)
    compare_with_oracle(A, outs[0][0], outs[0][1], outs[0][2], outs[0][3], Sr, infor,
                        label=f"stale workspace {m}x{n}")
