"""Autotuner of the launch configuration: measures, on the GPU it runs on,
every choice the library leaves open for each shape class, and writes the
table the library's plan reads (csrc/tuned.inc, compiled in).

    python -m paper_2601_17979_amd.tune [--out FILE] [--quick]

Choices and classes:
  * block method (every dtype; FP64 and FP32 real, complex128 and complex64),
    per (n class, tall or not): the block width nb (8, 16 or 32 for real
    data; complex keeps 16, whose 2nb x 2nb complex Gram matrix and J fill
    the LDS budget of two resident workgroups) and the inner solve of a
    block pair ("Inexact Hermitian Eigendecomposition"): one sweep, two
    sweeps, the converged solve, or the converged solve under the dynamic
    tolerance (start 1e-1, shrinking by 1e-2 per outer sweep);
  * register-resident unblocked path (FP64, n <= 64), per (N, rows per
    lane): the wavefronts per matrix (1, 2 or 4).
Each choice is timed on a batch of seeded matrices (half Gaussian, half with
a geometric spectrum, kappa 1e6), through the C ABI; a choice whose results fail the accuracy check (every info 0, sigma
against LAPACK within 1e-12 normwise, 1e-5 in single precision) is never
chosen.  The fastest admissible choice wins.
"""
from __future__ import annotations

import argparse
import datetime
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "tuned.inc")

# n classes of the block method: (upper bound of the class, representative n)
N_CLASSES = [(32, 28), (64, 56), (128, 112), (256, 224), (512, 448)]
DTYPES = {"f32": 0, "f64": 1, "c64": 2, "c128": 3}
INNER = {"1": (1, None), "2": (2, None), "conv": (-1, None), "dyn": (-1, (1e-1, 1e-2))}
DYN_START, DYN_RATE = 1e-1, 1e-2
RES_CLASSES = [(16, 16), (16, 64), (16, 128), (16, 192), (16, 256), (32, 32), (32, 64),
               (32, 128), (32, 192), (32, 256), (64, 64), (64, 128), (64, 192), (64, 256)]


def _inputs(m, n, batch, cx, seed):
    from workloads import gen
    kinds = ("gauss", "geo")
    return np.stack([gen.family(gen.rng_for(seed, k), kinds[k % 2], m, n, 1e6, complex_=cx)
                     for k in range(batch)])


def _batch_for(m, n, cx):
    """Batch size of about 2^28 flops per sweep of Alg. 2 (at least 64)."""
    per = (4 if cx else 1) * n * n * (12 * m + 6 * n) / 2
    return int(max(64, min(4000, 2 ** 28 / per)))


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best, out


def _admissible(out, Sref, single):
    S, info = out[0].cpu().numpy(), out[3].cpu().numpy()
    if np.any(info != 0):
        return False
    k = Sref.shape[0]
    err = np.max(np.abs(S[:k] - Sref) / Sref[:, :1])
    return err <= (1e-5 if single else 1e-12)


def tune_block(quick, log):
    import torch
    from paper_2601_17979_amd import svdb
    tdt = {"f32": torch.float32, "f64": torch.float64, "c64": torch.complex64,
           "c128": torch.complex128}
    rows = []
    for dname, code in DTYPES.items():
        cx = dname.startswith("c")
        single = dname in ("f32", "c64")
        nbs = (16,) if cx else (8, 16, 32)
        for nmax, n in N_CLASSES:
            if quick and n > 256:
                continue
            for tall in (0, 1):
                m = 3 * n if tall else n
                b = _batch_for(m, n, cx)
                A = _inputs(m, n, b, cx, 17000 + n + m)
                Sref = np.linalg.svd(A[:4].astype(np.complex128 if cx else np.float64),
                                     compute_uv=False)
                Ag = svdb.col_major(torch.from_numpy(A).to(tdt[dname]).cuda())
                best = None
                for nb in nbs:
                    for iname, (inner, dyn) in INNER.items():
                        def call(nb=nb, inner=inner, dyn=dyn):
                            return svdb.svd(Ag, path="blocked", nb=nb, precondition=0,
                                            inner_sweeps=inner, inner_tol=dyn)
                        t, out = _time(call, 1 if quick else 2)
                        ok = _admissible(out, Sref, single)
                        log(f"block {dname} {m}x{n} x{b}: nb {nb} inner {iname}: "
                            f"{b / t:10.1f} SVDs/s {'ok' if ok else 'REJECTED'}")
                        if ok and (best is None or t < best[0]):
                            best = (t, nb, inner, dyn)
                if best is not None:
                    t, nb, inner, dyn = best
                    rows.append((code, nmax, tall, nb, inner, dyn[0] if dyn else 0.0,
                                 dyn[1] if dyn else 0.0, f"{dname} {m}x{n}: {b / t:.1f} SVDs/s"))
    return rows


def tune_resident(quick, log):
    import torch
    from paper_2601_17979_amd import svdb
    rows = []
    for nn, m in RES_CLASSES:
        n = nn - nn // 8 if nn > 16 else nn
        if m < n:
            continue
        rw = 0 if (m <= 32 and nn <= 32) else -(-m // 64)
        b = 4000
        A = _inputs(m, n, b, False, 18000 + nn + m)
        Sref = np.linalg.svd(A[:4], compute_uv=False)
        Ag = svdb.col_major(torch.from_numpy(A).cuda())
        best = None
        for waves in (1, 2, 4):
            try:
                svdb.plan(torch.float64, m, n, path="resident", waves=waves, precondition=0)
            except svdb.SvdbError:
                continue
            t, out = _time(lambda w=waves: svdb.svd(Ag, path="resident", waves=w,
                                                    precondition=0), 1 if quick else 3)
            ok = _admissible(out, Sref, False)
            log(f"resident {m}x{n} (N {nn}, rows/lane {rw}) waves {waves}: {b / t:10.1f} "
                f"SVDs/s {'ok' if ok else 'REJECTED'}")
            if ok and (best is None or t < best[0]):
                best = (t, waves)
        if best is not None:
            rows.append((nn, rw, best[1], f"{m}x{n}: {b / best[0]:.1f} SVDs/s"))
    return rows


def write_table(path, blk, res, device):
    lines = [
        "// tuned.inc -- launch choices measured by paper_2601_17979_amd/tune.py",
        f"// on {device}, {datetime.date.today().isoformat()}.  Regenerate with",
        "//     python -m paper_2601_17979_amd.tune",
        "// rather than editing by hand.",
        "//",
        "// Block method: the first row with the request's dtype, n <= nmax and",
        "// tall == (m >= 2 n) gives nb and the inner solve (inner sweeps k > 0, or",
        "// -1 for the converged solve; tol_start > 0 adds the dynamic tolerance).",
        "// Resident path: wavefronts per matrix for (N, rows per lane).",
        "static const TunedBlock kTunedBlock[] = {",
    ]
    for code, nmax, tall, nb, inner, t0, rate, note in blk:
        lines.append(f"    {{{code}, {nmax}, {tall}, {nb}, {inner}, {t0!r}, {rate!r}}},   // {note}")
    lines.append("};")
    lines.append("static const TunedResident kTunedResident[] = {")
    for nn, rw, waves, note in res:
        lines.append(f"    {{{nn}, {rw}, {waves}}},   // {note}")
    lines.append("};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--quick", action="store_true", help="fewer classes and repetitions")
    args = ap.parse_args()
    import torch
    dev = torch.cuda.get_device_name(0)

    def log(msg):
        print(msg, flush=True)
    res = tune_resident(args.quick, log)
    blk = tune_block(args.quick, log)
    write_table(args.out, blk, res, dev)
    log(f"wrote {args.out}: {len(blk)} block rows, {len(res)} resident rows")


if __name__ == "__main__":
    main()
