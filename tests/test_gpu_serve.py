"""GPU tests of the serving runtime (svdb_server_*): continuous batching
with admission by an HBM budget, early retirement and mixed dtypes.  Every
completed request is checked against the oracle."""
import time

import numpy as np
import pytest

import oracle
from workloads import gen
from gpu_util import compare_with_oracle, say

pytestmark = pytest.mark.gpu


def _mat(seed, k, m, n, dtype, kappa=1e4):
    A = gen.from_spectrum(gen.rng_for(seed, k), m, n, gen.spectrum("geo", n, kappa))
    return A.astype(dtype)


def _to_dev(A):
    import torch
    return torch.from_numpy(np.asfortranarray(A)).cuda().t().contiguous().t()


def _drain(srv, count, timeout_s=120.0):
    got = {}
    t0 = time.time()
    while len(got) < count:
        assert time.time() - t0 < timeout_s, f"only {len(got)} of {count} completed"
        for rid, ts, td, out in srv.poll(timeout_ms=200):
            got[rid] = (ts, td, out)
    return got


def _check(A, out, label):
    S, U, V, info, sw = (x.cpu().numpy() if x is not None else None for x in out)
    A64 = A.astype(np.float64)
    dt = np.float32 if A.dtype == np.float32 else np.float64
    Sr, _, _, _, infor = oracle.gesvj(A64)
    compare_with_oracle(A64[None], S[None].astype(np.float64), U[None].astype(np.float64),
                        V[None].astype(np.float64), info, Sr[None], np.array([infor]), dtype=dt,
                        label=label)


def test_server_mixed_requests_vs_oracle():
    import torch
    from paper_2601_17979_amd import svdb
    shapes = [(16, 16), (32, 16), (32, 32), (64, 32), (64, 64), (128, 64), (128, 128),
              (256, 128)]
    reqs = []
    for k in range(48):
        m, n = shapes[k % len(shapes)]
        dt = np.float64 if k % 2 == 0 else np.float32
        reqs.append(_mat(9500, k, m, n, dt))
    dev = [_to_dev(A) for A in reqs]
    torch.cuda.synchronize()
    srv = svdb.Server(budget_bytes=256 << 20, max_requests=64)
    ids = {srv.submit(x): k for k, x in enumerate(dev)}
    got = _drain(srv, len(reqs))
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["active"] == 0 and st["bytes_in_use"] == 0
    lat = sorted(td - ts for ts, td, _ in got.values())
    say(f"[serve mix] {len(reqs)} requests, latency p50 {lat[len(lat) // 2] * 1e3:.2f} ms "
        f"max {lat[-1] * 1e3:.2f} ms")
    for rid, (ts, td, out) in got.items():
        k = ids[rid]
        _check(reqs[k], out, f"serve #{k} {reqs[k].shape} {reqs[k].dtype}")


@pytest.mark.parametrize("precondition", [-1, 0])
def test_server_alone_equals_in_mix(precondition):
    """A request's outputs do not depend on what else is being served (with
    the default QR preconditioning, whose wide QRs are batched by shape, and
    without)."""
    import torch
    from paper_2601_17979_amd import svdb
    probe = _mat(9600, 0, 96, 80, np.float64)
    others = [_mat(9600, k, 200, 150, np.float64) for k in range(1, 9)]
    torch.cuda.synchronize()

    def run(mats):
        dev = [_to_dev(A) for A in mats]
        torch.cuda.synchronize()
        srv = svdb.Server(budget_bytes=128 << 20, max_requests=16, precondition=precondition)
        ids = [srv.submit(x) for x in dev]
        got = _drain(srv, len(mats))
        srv.close()
        return [tuple(t.cpu().numpy() for t in got[i][2][:3]) for i in ids]

    alone = run([probe])[0]
    mixed = run(others[:4] + [probe] + others[4:])[4]
    # the same shape as the probe in the mix: one blocked-QR launch for both
    twin = run([_mat(9600, 9, 96, 80, np.float64), probe])[1]
    for a, b, c in zip(alone, mixed, twin):
        assert np.array_equal(a, b) and np.array_equal(a, c)


def test_server_budget_admission():
    """A budget that holds only two working sets at a time still serves a
    longer queue; the arena never exceeds the budget.  (Without QR
    preconditioning, so that a working set is W (m x np) and V (np x np).)"""
    import torch
    from paper_2601_17979_amd import svdb
    m, n = 128, 96
    need = (m * 96 + 96 * 96) * 8            # np = 96 for nb = 16 (l = 6)
    budget = 2 * need + 1024
    mats = [_mat(9700, k, m, n, np.float64) for k in range(10)]
    dev = [_to_dev(A) for A in mats]
    torch.cuda.synchronize()
    srv = svdb.Server(budget_bytes=budget, max_requests=8, precondition=0)
    ids = {srv.submit(x): k for k, x in enumerate(dev)}
    got = {}
    peak = 0
    t0 = time.time()
    while len(got) < len(mats):
        assert time.time() - t0 < 120
        st = srv.stats()
        peak = max(peak, st["bytes_in_use"])
        for rid, ts, td, out in srv.poll(timeout_ms=5):
            got[rid] = out
    srv.close()
    say(f"[serve budget] peak arena {peak} of {budget} bytes")
    assert 0 < peak <= budget
    for rid, out in got.items():
        _check(mats[ids[rid]], out, f"budget #{ids[rid]}")
    with pytest.raises(svdb.SvdbError):
        srv2 = svdb.Server(budget_bytes=4096, max_requests=2, precondition=0)
        try:
            srv2.submit(dev[0])
        finally:
            srv2.close()


@pytest.mark.parametrize("precondition", [0, 1])
def test_server_precondition_modes(precondition):
    """FP64 and FP32 requests with and without QR preconditioning (FP32
    requests are then solved in FP64 and returned in FP32)."""
    import torch
    from paper_2601_17979_amd import svdb
    shapes = [(48, 40), (130, 96), (300, 200), (64, 64)]
    reqs = [_mat(9800, k, m, n, np.float64 if k % 2 else np.float32, kappa=1e6)
            for k, (m, n) in enumerate(shapes * 2)]
    dev = [_to_dev(A) for A in reqs]
    torch.cuda.synchronize()
    srv = svdb.Server(budget_bytes=512 << 20, max_requests=32,
                      precondition=1 if precondition else 0)
    ids = {srv.submit(x): k for k, x in enumerate(dev)}
    got = _drain(srv, len(reqs))
    srv.close()
    for rid, (ts, td, out) in got.items():
        k = ids[rid]
        assert out[0].dtype == (torch.float64 if reqs[k].dtype == np.float64 else torch.float32)
        _check(reqs[k], out, f"precondition={precondition} #{k} {reqs[k].shape}")


def test_server_wide_requests():
    """Wide requests (m < n) run as A^H, read transposed, with U and V
    exchanged; each is checked as the SVD of the tall matrix A^H."""
    import torch
    from paper_2601_17979_amd import svdb
    shapes = [(16, 40), (40, 16), (30, 64), (64, 30), (1, 9), (100, 200)]
    reqs = []
    for k, (m, n) in enumerate(shapes):
        dt = np.float64 if k % 2 == 0 else np.float32
        reqs.append(_mat(9700, k, n, m, dt).T.copy() if m < n else _mat(9700, k, m, n, dt))
    dev = [_to_dev(A) for A in reqs]
    torch.cuda.synchronize()
    srv = svdb.Server(budget_bytes=64 << 20, max_requests=16)
    ids = {srv.submit(x): k for k, x in enumerate(dev)}
    got = _drain(srv, len(reqs))
    srv.close()
    for rid, (ts, td, out) in got.items():
        k = ids[rid]
        A = reqs[k]
        m, n = A.shape
        S, U, V = out[0], out[1], out[2]
        assert S.shape == (min(m, n),) and U.shape == (m, min(m, n)) and V.shape == (n, min(m, n))
        if m >= n:
            _check(A, out, f"serve tall {A.shape}")
        else:   # A^H = V S U^H
            _check(A.T.copy(), (out[0], out[2], out[1], out[3], out[4]), f"serve wide {A.shape}")


def test_server_precondition_wide_qr():
    """Preconditioned requests with more than 64 columns take the blocked QR
    (request by request on the wide QR lane), up to m = 1024; FP32 requests
    are widened into the reflector buffer first."""
    import torch
    from paper_2601_17979_amd import svdb
    shapes = [(700, 300, np.float64), (700, 300, np.float32), (1024, 128, np.float64),
              (256, 256, np.float32), (90, 65, np.float64)]
    reqs = [_mat(9900, k, m, n, dt, kappa=1e8) for k, (m, n, dt) in enumerate(shapes)]
    dev = [_to_dev(A) for A in reqs]
    torch.cuda.synchronize()
    srv = svdb.Server(budget_bytes=1 << 30, max_requests=8, precondition=1)
    ids = {srv.submit(x): k for k, x in enumerate(dev)}
    got = _drain(srv, len(reqs))
    srv.close()
    for rid, (ts, td, out) in got.items():
        k = ids[rid]
        say(f"  wide QR {reqs[k].shape} {reqs[k].dtype}: sweeps {int(out[4].item())}, "
            f"{(td - ts) * 1e3:.1f} ms")
        _check(reqs[k], out, f"precond wide #{k} {reqs[k].shape}")


@pytest.mark.parametrize("precondition", [-1, 0])
def test_server_late_admission_bitwise(precondition):
    """A request submitted while others are already on the GPU (admitted and
    sweeping, none finished) joins the running launches with its own
    schedule; its outputs equal those of the same request served alone, bit
    for bit, and match the oracle.  With QR preconditioning the probe also
    has to wait for, and pass through, the QR lanes while the others'
    applications of Q are queued."""
    import torch
    from paper_2601_17979_amd import svdb
    probe = _mat(9650, 0, 96, 80, np.float64, kappa=1e6)
    big = [_mat(9650, k, 1024, 512, np.float64, kappa=1e8) for k in range(1, 5)]
    dev_probe = _to_dev(probe)
    dev_big = [_to_dev(A) for A in big]
    torch.cuda.synchronize()

    srv = svdb.Server(budget_bytes=512 << 20, max_requests=16, precondition=precondition)
    pid = srv.submit(dev_probe)
    alone = _drain(srv, 1)[pid][2]
    alone = tuple(t.cpu().numpy() for t in alone[:3])
    srv.close()

    srv = svdb.Server(budget_bytes=512 << 20, max_requests=16, precondition=precondition)
    ids = [srv.submit(x) for x in dev_big]
    t0 = time.time()
    while srv.stats()["active"] < len(big):
        assert time.time() - t0 < 30
        time.sleep(0.0005)
    time.sleep(0.01)   # let the admitted requests run a few launches
    st = srv.stats()
    pid = srv.submit(dev_probe)
    say(f"[late admission pc={precondition}] probe submitted with {st['active']} active, "
        f"{st['completed']} completed")
    assert st["completed"] == 0 and st["active"] == len(big)
    got = _drain(srv, len(big) + 1)
    srv.close()
    mixed = tuple(t.cpu().numpy() for t in got[pid][2][:3])
    for a, b in zip(alone, mixed):
        assert np.array_equal(a, b)
    _check(probe, got[pid][2], f"late probe pc={precondition}")
    assert got[pid][1] < max(got[i][1] for i in ids), "the probe should finish first"
