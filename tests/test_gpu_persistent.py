"""Sweep control on the device (svdb_opts_t.persistent = 1): the block
method queues the launches of every sweep up to max_sweeps, the count of
unconverged matrices stays on the device, and the launches after the sweep
that leaves none return at once.  svdb_svd_strided_batched and
svdb_svd_batched then return before the work is done, and the strided call
can be captured into a HIP graph (a capturing stream selects this form by
itself).

The queued form takes the same convergence decisions as the host-closed
loop (persistent = 0), so the two agree bit for bit; both are checked
against the oracle as well.
"""
import time

import numpy as np
import pytest

import oracle
from workloads import gen
from gpu_util import compare_with_oracle, run_gpu, say

pytestmark = pytest.mark.gpu

def _batch(m, n, count, seed, cx=False, kinds=("gauss", "geo", "random")):
    return np.stack([gen.family(gen.rng_for(seed, k), kinds[k % len(kinds)], m, n, 1e6,
                                complex_=cx) for k in range(count)])


CASES = [
    # (label, numpy dtype, torch dtype, shape, nb, extra options)
    ("f64 nb16", np.float64, "float64", (200, 130), 16, {}),
    ("f64 nb32", np.float64, "float64", (130, 96), 32, {}),
    ("f64 nb8", np.float64, "float64", (72, 40), 8, {}),
    ("f64 l2", np.float64, "float64", (90, 30), 16, {}),
    ("f64 no masking", np.float64, "float64", (96, 80), 16, dict(masking=False)),
    ("f64 mixed", np.float64, "float64", (130, 96), 16, dict(precision=1)),
    ("f32", np.float32, "float32", (150, 100), 16, {}),
    ("c128", np.complex128, "complex128", (100, 70), 16, {}),
    ("c64", np.complex64, "complex64", (64, 48), 16, {}),
    ("f64 capped", np.float64, "float64", (96, 96), 16, dict(max_sweeps=3)),
]


@pytest.mark.parametrize("label,npdt,tdt,shape,nb,kw", CASES, ids=[c[0] for c in CASES])
def test_queued_equals_host_closed_sweeps(label, npdt, tdt, shape, nb, kw):
    import torch
    m, n = shape
    cx = npdt in (np.complex64, np.complex128)
    A = _batch(m, n, 7, 6100 + m + n, cx=cx).astype(npdt)
    A[3] *= 0.0   # a zero matrix converges at once and is retired early
    say(f"[queued {label} {m}x{n}]")
    common = dict(dtype=getattr(torch, tdt), path="blocked", nb=nb, precondition=0, **kw)
    P = run_gpu(A, persistent=True, **common)
    H = run_gpu(A, persistent=False, **common)
    for a, b, name in zip(P, H, ("S", "U", "V", "info", "sweeps")):
        assert np.array_equal(a, b), (label, name)
    say(f"  sweeps {P[4].tolist()} info {P[3].tolist()}")
    if kw.get("max_sweeps"):
        assert np.all(P[3][np.arange(7) != 3] == 1) and P[3][3] == 0
        return
    wide = np.complex128 if cx else np.float64
    A64 = A.astype(wide)
    Sr, _, _, _, infor = oracle.gesvj_batch(A64)
    compare_with_oracle(A64, P[0].astype(np.float64), P[1].astype(wide), P[2].astype(wide),
                        P[3], Sr, infor, dtype=npdt, label=label)


@pytest.mark.parametrize("dt", ["f64", "c128", "f32"])
def test_uneven_queued_equals_host_closed_sweeps(dt):
    import torch
    from paper_2601_17979_amd import svdb
    cx = dt == "c128"
    npdt = {"f64": np.float64, "c128": np.complex128, "f32": np.float32}[dt]
    shapes = [(5, 0), (1, 1), (7, 3), (40, 33), (130, 128), (300, 256), (64, 16), (16, 40),
              (200, 130), (33, 33)]
    mats = [np.zeros((m, 0), npdt) if n == 0 else
            gen.family(gen.rng_for(6200, k), "gauss", m, n, 1.0, complex_=cx).astype(npdt)
            for k, (m, n) in enumerate(shapes)]
    gm = [svdb.col_major(torch.from_numpy(np.ascontiguousarray(a))[None].cuda())[0]
          for a in mats]
    out = {}
    for pers in (True, False):
        S, U, V, info, sw = svdb.svd_batched(gm, persistent=pers)
        torch.cuda.synchronize()
        out[pers] = ([s.cpu().numpy() for s in S], [u.cpu().numpy() for u in U],
                     [v.cpu().numpy() for v in V], info.cpu().numpy(), sw.cpu().numpy())
    for k in range(len(mats)):
        for j in range(3):
            assert np.array_equal(out[True][j][k], out[False][j][k]), (dt, k, j)
    assert np.array_equal(out[True][3], out[False][3])
    assert np.array_equal(out[True][4], out[False][4])
    say(f"[uneven queued {dt}] sweeps {out[True][4].tolist()}")
    for k, A in enumerate(mats):
        if min(A.shape) == 0:
            assert out[True][3][k] == 0
            continue
        wide = np.complex128 if cx else np.float64
        m, n = A.shape
        At = A.astype(wide) if m >= n else A.astype(wide).conj().T
        Sr, _, _, _, ir = oracle.gesvj(At)
        U_, V_ = (out[True][1][k], out[True][2][k]) if m >= n else \
            (out[True][2][k], out[True][1][k])
        compare_with_oracle(At[None], out[True][0][k][None].astype(np.float64),
                            U_[None].astype(wide), V_[None].astype(wide),
                            out[True][3][k:k + 1], Sr[None], np.array([ir]), dtype=npdt,
                            label=f"uneven {dt} #{k} {A.shape}")


def test_calls_return_before_the_work_is_done():
    """The strided and the mixed-shape calls only enqueue work: each returns
    long before its stream has finished (the per-iteration form waits on the
    host after every sweep)."""
    import torch
    from paper_2601_17979_amd import svdb
    A = _batch(256, 256, 64, 6300, kinds=("geo",))
    Ag = svdb.col_major(torch.from_numpy(np.repeat(A, 16, axis=0)).cuda())
    mats = [Ag[k] for k in range(256)]
    call = svdb.BatchedCall(mats, persistent=True)
    for label, fn in (("strided", lambda: svdb.svd(Ag, path="blocked", precondition=0,
                                                   persistent=True)),
                      ("batched", call)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        t_host = time.perf_counter() - t0
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t0
        say(f"[async {label}] call returned after {t_host * 1e3:.2f} ms, work done after "
            f"{t_all * 1e3:.2f} ms")
        assert t_all > 0.02 and t_host < 0.25 * t_all, (label, t_host, t_all)


def test_strided_call_replays_from_a_graph():
    """The whole strided call (workspace clears by kernels, init, the queued
    sweeps, finalisation) captured in a HIP graph: every replay, with other
    work and a new input in between, equals the eager call (which closes its
    sweeps on the host)."""
    import torch
    from paper_2601_17979_amd import svdb
    m, n, b = 130, 96, 24
    A0 = _batch(m, n, b, 6400)
    A1 = _batch(m, n, b, 6401)
    Ag = svdb.col_major(torch.from_numpy(A0).cuda())
    out = (torch.empty((b, n), dtype=torch.float64, device="cuda"),
           svdb.empty_col_major(b, m, n, torch.float64, "cuda"),
           svdb.empty_col_major(b, n, n, torch.float64, "cuda"),
           torch.empty(b, dtype=torch.int32, device="cuda"),
           torch.empty(b, dtype=torch.int32, device="cuda"))
    kw = dict(path="blocked", precondition=0, out=out)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        svdb.svd(Ag, **kw)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref = {}
    for key, A in ((0, A0), (1, A1)):
        Ag.copy_(svdb.col_major(torch.from_numpy(A).cuda()))
        svdb.svd(Ag, **kw)
        torch.cuda.synchronize()
        ref[key] = [t.cpu().numpy() for t in out]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        svdb.svd(Ag, **kw)
    for rep, key in enumerate((0, 1, 0, 1)):
        Ag.copy_(svdb.col_major(torch.from_numpy(A0 if key == 0 else A1).cuda()))
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        for t in out:
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in out]
        for a, r in zip(got, ref[key]):
            assert np.array_equal(a, r), (rep, key)
        say(f"[graph] replay {rep} (input {key}) equals the eager call; junk {float(junk):.2f}")
