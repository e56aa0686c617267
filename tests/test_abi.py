"""The C-ABI library on the host: it loads, exports every function declared in
include/svdb.h, and rejects invalid arguments with the documented codes before
anything reaches the GPU (no GPU is needed for these checks)."""
import ctypes as C
import os
import re

import pytest
import torch

from paper_2601_17979_amd import svdb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(svdb_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = svdb.lib()
    names = _declared()
    assert "svdb_svd_strided_batched" in names and "svdb_svd_batched" in names
    for name in sorted(names):
        assert hasattr(L, name), name


def test_version_and_defaults():
    assert "gfx950" in svdb.version()
    o = svdb.Opts()
    svdb.lib().svdb_opts_default(C.byref(o))
    assert o.max_sweeps == 100 and o.path == svdb.PATH_AUTO and o.masking == 1


def _call(**kw):
    args = dict(dtype=svdb.R64, batch=2, m=8, n=4, A=0x1000, lda=8, sA=32, S=0x2000, sS=4,
                U=0x3000, ldu=8, sU=32, V=0x4000, ldv=4, sV=16, tol=0.0, info=0x5000,
                ws=None, wsb=0, opts=None, stream=None)
    args.update(kw)
    o = C.byref(args["opts"]) if args["opts"] is not None else None
    return svdb.lib().svdb_svd_strided_batched(
        args["dtype"], args["batch"], args["m"], args["n"], args["A"], args["lda"], args["sA"],
        args["S"], args["sS"], args["U"], args["ldu"], args["sU"], args["V"], args["ldv"],
        args["sV"], args["tol"], args["info"], args["ws"], args["wsb"], o, args["stream"])


@pytest.mark.parametrize("kw,code", [
    (dict(dtype=9), -1),
    (dict(batch=-1), -2),
    (dict(m=-1), -3),
    (dict(n=-1), -4),
    # wide (m < n): k = min(m, n) = 4 columns of U (4 x 4) and V (8 x 4)
    (dict(m=4, n=8, lda=3, sA=32, sS=4, ldu=4, sU=16, ldv=8, sV=32), -6),
    (dict(m=4, n=8, lda=4, sA=32, sS=3, ldu=4, sU=16, ldv=8, sV=32), -9),
    (dict(m=4, n=8, lda=4, sA=32, sS=4, ldu=4, sU=15, ldv=8, sV=32), -12),
    (dict(m=4, n=8, lda=4, sA=32, sS=4, ldu=4, sU=16, ldv=7, sV=32), -14),
    (dict(m=4, n=8, lda=4, sA=32, sS=4, ldu=4, sU=16, ldv=8, sV=31), -15),
    (dict(m=4, n=8, lda=4, sA=32, sS=4, ldu=4, sU=16, ldv=8, sV=32), -19),   # A^H copy
    (dict(A=None), -5),
    (dict(lda=7), -6),
    (dict(sA=31), -7),
    (dict(S=None), -8),
    (dict(sS=3), -9),
    (dict(ldu=7), -11),
    (dict(sU=31), -12),
    (dict(ldv=3), -14),
    (dict(sV=15), -15),
    (dict(tol=float("nan")), -16),
    (dict(info=None), -17),
])
def test_argument_errors(kw, code):
    assert _call(**kw) == code
    assert svdb.last_error() != ""


def test_empty_batch_is_a_noop():
    # nothing is launched for an empty batch, so this runs without a GPU
    assert _call(batch=0) == 0
    assert _call(batch=0, A=None, S=None, info=None) == 0


@pytest.mark.parametrize("m,n", [(3, 0), (0, 0), (0, 3)])
def test_no_singular_values_is_accepted(m, n):
    """min(m, n) = 0: no workspace, NULL A and S accepted, and the call only
    sets info (a small kernel, so without a GPU it can fail only in the HIP
    runtime, never as an unsupported shape)."""
    L = svdb.lib()
    for code in (svdb.R32, svdb.R64, svdb.C64, svdb.C128):
        assert L.svdb_workspace_size(code, 5, m, n, None) == 0
        rc = _call(dtype=code, batch=5, m=m, n=n, A=None, lda=max(m, 1), sA=0, S=None, sS=0,
                   U=None, ldu=max(m, 1), sU=0, V=None, ldv=max(n, 1), sV=0)
        assert rc in (0, svdb.ERR_HIP), (code, rc, svdb.last_error())


def test_plan_and_workspace():
    p, nb, th = svdb.plan(svdb.torch.float64, 16, 16)
    assert p in (svdb.PATH_PLAIN, svdb.PATH_RESIDENT, svdb.PATH_BLOCKED)
    L = svdb.lib()
    assert L.svdb_workspace_size(svdb.R64, 10, -1, 8, None) == C.c_size_t(-1).value
    # a wide matrix runs the plan of A^H, with the A^H copy added to the workspace
    for dt, code, es in ((svdb.torch.float64, svdb.R64, 8), (svdb.torch.complex64, svdb.C64, 8),
                         (svdb.torch.float32, svdb.R32, 4)):
        for m, n in ((4, 8), (24, 100), (40, 64)):
            assert svdb.plan(dt, m, n) == svdb.plan(dt, n, m)
            tall = L.svdb_workspace_size(code, 10, n, m, None)
            wide = L.svdb_workspace_size(code, 10, m, n, None)
            assert wide == tall + (10 * m * n * es + 255) // 256 * 256


def test_batched_argument_errors():
    L = svdb.lib()
    m = (C.c_int * 2)(8, 4)
    n = (C.c_int * 2)(4, 6)                # second matrix is wide
    P = C.c_void_p * 2
    I = C.c_int * 2
    A = P(0x1000, 0x2000)
    lda = I(8, 4)
    S = P(0x3000, 0x4000)
    info = 0x5000
    rc = L.svdb_svd_batched(svdb.R64, 2, m, n, A, lda, S, None, None, None, None, 0.0, info,
                            None, 0, None, None)
    assert rc == -14                       # wide matrices are accepted; no workspace given
    # the workspace of a wide matrix is that of its (tall) conjugate transpose
    wide = L.svdb_batched_workspace_size(svdb.R64, 2, m, n, None)
    mt, nt = (C.c_int * 2)(8, 6), (C.c_int * 2)(4, 4)
    assert wide == L.svdb_batched_workspace_size(svdb.R64, 2, mt, nt, None)
    n[1] = -1
    rc = L.svdb_svd_batched(svdb.R64, 2, m, n, A, lda, S, None, None, None, None, 0.0, info,
                            None, 0, None, None)
    assert rc == -4
    n[1] = 2
    lda[0] = 7
    rc = L.svdb_svd_batched(svdb.R64, 2, m, n, A, lda, S, None, None, None, None, 0.0, info,
                            None, 0, None, None)
    assert rc == -6


def test_server_argument_errors():
    """Argument checks of the serving entry points that run before any
    device call."""
    h = C.c_void_p()
    lib = svdb.lib()
    assert lib.svdb_server_create(None, 1 << 20, 4, None) == -1
    assert lib.svdb_server_create(C.byref(h), 0, 4, None) == -2
    assert lib.svdb_server_create(C.byref(h), 1 << 20, 0, None) == -3
    o = svdb.make_opts(precision=1)
    assert lib.svdb_server_create(C.byref(h), 1 << 20, 4, C.byref(o)) == svdb.ERR_UNSUPPORTED
    o = svdb.make_opts(precondition=2)   # the server's QR does not pivot
    assert lib.svdb_server_create(C.byref(h), 1 << 20, 4, C.byref(o)) == svdb.ERR_UNSUPPORTED
    assert lib.svdb_server_submit(None, svdb.R64, 8, 4, 0x1000, 8, 0x2000, None, 8, None, 4,
                                  0.0, 0x3000, None) == -1
    assert lib.svdb_server_poll(None, None, None, None, 0, 0) == -1
    assert lib.svdb_server_stats(None, None, None, None, None, None) == -1
    assert lib.svdb_server_destroy(None) == -1
    assert lib.svdb_server_clock() > 0.0


def test_precondition_option_in_plan():
    """AUTO plans the QR-preconditioned resident path for FP64 n <= 64 and
    the preconditioned block path for wider matrices; precondition = 0 turns
    both off, and 1 is refused where it does not apply."""
    p_auto = svdb.plan(torch.float64, 64, 64)
    assert p_auto[0] == svdb.PATH_RESIDENT
    assert svdb.plan(torch.float64, 256, 256)[0] == svdb.PATH_BLOCKED
    assert svdb.plan(torch.float64, 64, 64, precondition=0)[0] == svdb.PATH_RESIDENT
    with pytest.raises(svdb.SvdbError):
        svdb.plan(torch.complex128, 64, 64, precondition=1)
    with pytest.raises(svdb.SvdbError):
        svdb.plan(torch.float64, 2048, 100, precondition=1)
    # column pivoting (precondition 2) only where the register QR runs
    assert svdb.plan(torch.float64, 64, 64, precondition=2)[0] == svdb.PATH_RESIDENT
    assert svdb.plan(torch.float32, 100, 40, precondition=2)[0] == svdb.PATH_RESIDENT
    for dt, m, n in [(torch.float64, 256, 256), (torch.float64, 1000, 16),
                     (torch.complex128, 64, 64)]:
        with pytest.raises(svdb.SvdbError) as e:
            svdb.plan(dt, m, n, precondition=2)
        assert e.value.code == svdb.ERR_UNSUPPORTED
    with pytest.raises(svdb.SvdbError):
        svdb.plan(torch.float64, 64, 64, precondition=3)
    # waves per matrix the register layout of 64 columns cannot take are
    # refused by the plan, before any launch
    assert svdb.plan(torch.float64, 64, 64, waves=4)[2] == 256
    with pytest.raises(svdb.SvdbError) as e:
        svdb.plan(torch.float64, 64, 64, waves=1)
    assert e.value.code == svdb.ERR_UNSUPPORTED and "waves" in str(e.value)
    ws_pc = svdb.lib().svdb_workspace_size(svdb.R64, 10, 64, 64, C.byref(svdb.make_opts()))
    ws_no = svdb.lib().svdb_workspace_size(svdb.R64, 10, 64, 64,
                                           C.byref(svdb.make_opts(precondition=0)))
    assert ws_pc > 0 and ws_no == 0



def test_queued_sweep_control_is_an_option():
    """The block method's sweep control: the host-closed loop is the default
    and the queued form (persistent = 1) is accepted on every path of the
    plan, uniform and uneven."""
    o = svdb.Opts()
    svdb.lib().svdb_opts_default(C.byref(o))
    assert o.persistent == 0
    assert svdb.plan(torch.float64, 256, 256)[0] == svdb.PATH_BLOCKED
    assert svdb.plan(torch.float64, 256, 256, persistent=True) == svdb.plan(torch.float64, 256,
                                                                            256)
    assert svdb.plan(torch.complex64, 40, 30, persistent=True)[0] == svdb.PATH_BLOCKED
    ms, ns = (C.c_int * 2)(8, 40), (C.c_int * 2)(4, 30)
    assert svdb.lib().svdb_batched_workspace_size(
        svdb.C128, 2, ms, ns, C.byref(svdb.make_opts(persistent=True))) > 0


def test_noalloc_refusals_before_any_launch():
    """The allocation-free call refuses, on the host, a batch whose workspace
    exceeds its static scratch (-2) and a request planned on the block method
    (unsupported); neither touches the device."""
    L = svdb.lib()
    cap = L.svdb_noalloc_scratch_bytes()
    assert cap == 64 << 20
    big = 20000
    assert L.svdb_workspace_size(svdb.R64, big, 64, 64, None) > cap

    def call(batch, m, n):
        return L.svdb_svd_strided_batched_noalloc(
            svdb.R64, batch, m, n, 0x1000, m, m * n, 0x2000, n, 0x3000, m, m * n, 0x4000, n,
            n * n, 0.0, 0x5000, None, None)
    assert call(big, 64, 64) == -2 and "static maximum" in svdb.last_error()
    assert call(8, 256, 256) == svdb.ERR_UNSUPPORTED and "block method" in svdb.last_error()
    assert call(0, 64, 64) == 0


def test_plan_reads_the_tuned_table():
    """With nb left open, the block method's width is the measured table's
    (csrc/tuned.inc) for each of its (dtype, n class, tall) rows."""
    import re
    txt = open(os.path.join(ROOT, "paper_2601_17979_amd", "csrc", "tuned.inc")).read()
    blk = txt[txt.index("kTunedBlock"):txt.index("kTunedResident")]
    rows = [tuple(int(x) for x in r.groups()) for r in
            re.finditer(r"\{\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(-?\d+),", blk)]
    assert rows, "the table is empty"
    lower = {32: 16, 64: 32, 128: 64, 256: 128, 512: 256}
    dts = {0: torch.float32, 1: torch.float64, 2: torch.complex64, 3: torch.complex128}
    for dt, nmax, tall, nb, _ in rows:
        n = lower[nmax] + 5
        m = 3 * n if tall else n
        assert svdb.plan(dts[dt], m, n, path="blocked", precondition=0)[1] == nb, (dt, nmax, tall)
