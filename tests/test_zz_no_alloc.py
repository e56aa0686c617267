"""The allocation-free entry point svdb_svd_strided_batched_noalloc, on the
GPU through the C ABI: two calls in a row (the second on a smaller input),
each equal bit for bit to svdb_svd_strided_batched on the same input, which
runs the same kernels with a caller-provided workspace."""
import numpy as np
import pytest

from workloads import gen
from gpu_util import say, to_gpu

pytestmark = pytest.mark.gpu


def _batch(m, n, count, seed):
    """count matrices m x n (a wide one is the transpose of a tall draw)."""
    kinds = ("gauss", "geo")
    mt, nt = max(m, n), min(m, n)
    A = np.stack([gen.family(gen.rng_for(seed, k), kinds[k % 2], mt, nt, 1e6)
                  for k in range(count)])
    return A if m >= n else np.ascontiguousarray(A.transpose(0, 2, 1))


def _outputs(b, m, n, dtype):
    import torch
    from paper_2601_17979_amd import svdb
    k = min(m, n)
    real = torch.float32 if dtype in (torch.float32, torch.complex64) else torch.float64
    return (torch.full((b, k), float("nan"), dtype=real, device="cuda"),
            svdb.empty_col_major(b, m, k, dtype, "cuda").fill_(float("nan")),
            svdb.empty_col_major(b, n, k, dtype, "cuda").fill_(float("nan")),
            torch.full((b,), -7, dtype=torch.int32, device="cuda"),
            torch.full((b,), -7, dtype=torch.int32, device="cuda"))


# (rows, cols, batch, dtype name, options): the first call the largest
CALLS = [(64, 64, 250, "float64", {}),            # QR-preconditioned resident path
         (128, 32, 120, "float64", {}),           # smaller: the second call
         (40, 24, 37, "float32", {}),             # FP32 input on the FP64 path
         (24, 40, 19, "float64", {}),             # wide: A^H staged in the scratch
         (48, 48, 9, "float64", dict(precondition=0))]   # resident on A: no scratch


def test_noalloc_equals_the_workspace_call_on_consecutive_calls():
    import torch
    from paper_2601_17979_amd import svdb
    assert svdb.lib().svdb_noalloc_scratch_bytes() == 64 << 20
    for j, (m, n, b, dt, kw) in enumerate(CALLS):
        dtype = getattr(torch, dt)
        A = _batch(m, n, b, 9100 + j)
        Ag = to_gpu(A, dtype)
        say(f"[noalloc call {j}] {b} x {m}x{n} {dt} {kw}")
        ref = svdb.svd(Ag, **kw)
        out = _outputs(b, m, n, dtype)
        got = svdb.svd_noalloc(Ag, out, **kw)
        torch.cuda.synchronize()
        for name, r, g in zip(("S", "U", "V", "info", "sweeps"), ref, got):
            r, g = r.cpu().numpy(), g.cpu().numpy()
            assert np.array_equal(r, g), (j, name, np.nanmax(np.abs(r - g)))
        assert np.all(got[3].cpu().numpy() == 0), j
        say(f"  equal bit for bit; sweeps {got[4].cpu().numpy().min()}-"
            f"{got[4].cpu().numpy().max()}")
