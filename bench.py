"""Benchmark: batched SVD throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--path auto|plain|resident|blocked]

A step is one batched SVD (S, U and V, converged to the FP64 tolerance) of the
whole workload: 10000 FP64 matrices, 5000 of 64 x 64 and 5000 of 128 x 32,
half with a geometric spectrum (kappa = 1e6, Haar factors) and half with
i.i.d. N(0,1) entries, seeded and synthetic.  Inputs are resident in HBM when
the timed region starts.  Prints ONE JSON line with SVDs/s, the plain GPU
Jacobi on the same workload, the roofline of the dominant kernel and the
CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SVDs/sec vs plain GPU Jacobi at equal sigma rel-err; serve p50/p99 latency"
WORKLOAD = ("10000 FP64 SVDs (S,U,V): 5000 x 64x64 + 5000 x 128x32, half geometric "
            "spectrum kappa=1e6 (Haar U,V), half iid N(0,1); tol 30u")
FP64_VALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9      # CUs x SIMDs x lanes x FMA x clock


def measured_traffic(shape: str):
    """HBM bytes of one QR-preconditioned call of this shape (both QRs, the
    Jacobi on R2^T, both applications of Q) from the committed rocprofv3
    summary, or None when a kernel source has changed since the counters were
    taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "precond_mixed_64x64_128x32_traffic.json")
    try:
        rec = json.load(open(prof))
        for src, sha in rec["kernel_source_sha256"].items():
            if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != sha:
                return None
    except (OSError, KeyError, ValueError):
        return None
    call = rec.get("calls", {}).get(shape)
    return call["traffic_bytes"] if call else None


def flops_unblocked(m, n, sweeps):
    """Alg. 2 work for `sweeps` executed sweeps: every sweep forms 3 dots of
    length m per pair (6m flops); every sweep but the last (clean) one also
    rotates both columns of W and V (6(m+n) flops)."""
    pairs = n * (n - 1) / 2
    s = np.asarray(sweeps, dtype=np.float64)
    return float(np.sum(pairs * (6 * m * s + 6 * (m + n) * np.maximum(s - 1, 0))))


def serve_leg(args, dev):
    """Serving workload: requests from 12 shape classes (n in {16..512} x
    {square, m = 2n}), FP64/FP32 alternating, kappa log-uniform in [1, 1e8].
    Saturation = a closed batch of requests submitted at once; then Poisson
    arrivals at `serve_load` x saturation for `serve_seconds`; latency =
    completion - arrival (server clock)."""
    import torch
    from paper_2601_17979_amd import svdb
    from workloads import gen
    pool = gen.serving_pool(per_class=4)
    tdt = {"f64": torch.float64, "f32": torch.float32}
    dev_pool = [svdb.col_major(torch.from_numpy(A)[None].to(tdt[d]).to(dev))[0]
                for A, d in pool]
    torch.cuda.synchronize()
    budget = 8 << 30
    srv = svdb.Server(budget_bytes=budget, max_requests=2048,
                      precondition=args.serve_precondition)

    def drain(n, t_limit):
        lat, t0 = [], time.time()
        while len(lat) < n and time.time() - t0 < t_limit:
            for rid, ts, td, out in srv.poll(timeout_ms=100):
                lat.append(td - ts)
        return lat

    # warm-up and saturation: closed batches of the whole pool
    for x in dev_pool:
        srv.submit(x)
    drain(len(dev_pool), 120)
    reps = 8
    t0 = svdb.Server.clock()
    for _ in range(reps):
        for x in dev_pool:
            srv.submit(x)
    drain(reps * len(dev_pool), 300)
    sat = reps * len(dev_pool) / (svdb.Server.clock() - t0)
    # open loop: Poisson arrivals
    rate = args.serve_load * sat
    rng = np.random.default_rng(17979 + 4000)
    lat, n_sub, cls = [], 0, {}
    by_class = {}

    def collect(items):
        for rid, ts, td, out in items:
            lat.append(td - ts)
            by_class.setdefault(cls.pop(rid), []).append(td - ts)
    t_start = svdb.Server.clock()
    t_next = t_start
    while t_next - t_start < args.serve_seconds:
        now = svdb.Server.clock()
        if now < t_next:
            collect(srv.poll(timeout_ms=0))
            time.sleep(max(0.0, min(t_next - svdb.Server.clock(), 0.002)))
            continue
        k = int(rng.integers(len(dev_pool)))
        rid = srv.submit(dev_pool[k])
        cls[rid] = f"{pool[k][0].shape[0]}x{pool[k][0].shape[1]}"
        n_sub += 1
        t_next += rng.exponential(1.0 / rate)
    t0 = time.time()
    while len(lat) < n_sub and time.time() - t0 < 120:
        collect(srv.poll(timeout_ms=100))
    srv.close()
    lat = np.sort(np.asarray(lat))
    per_class = {c: {"count": len(v), "p50_ms": float(np.percentile(v, 50) * 1e3),
                     "p99_ms": float(np.percentile(v, 99) * 1e3)}
                 for c, v in sorted(by_class.items(), key=lambda kv: int(kv[0].split("x")[1]))}
    return {"workload": "12 shape classes n in {16,...,512} x {square, 2n x n}, FP64/FP32 "
                        "alternating, geometric spectrum kappa log-uniform [1, 1e8]",
            "saturation_svds_per_s": sat, "offered_load": args.serve_load,
            "offered_rate_per_s": rate, "requests": int(n_sub), "completed": int(lat.size),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "per_class": per_class, "budget_bytes": budget,
            "qr_preconditioning": args.serve_precondition != 0}


def host_cpu():
    """The host's CPU model and the cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0))}


def sweep_histogram(sw):
    """Number of matrices per executed sweep count."""
    vals, counts = np.unique(np.asarray(sw), return_counts=True)
    return {str(int(v)): int(c) for v, c in zip(vals, counts)}


def flops_blocked(m, n, nb, sweeps, cf=1):
    """Block method work per executed sweep: cf P nb^2 (14 m + 8 n + 72 nb)
    with P = l (l - 1) / 2 block pairs (Gram 6 nb^2 m, update 8 nb^2 (m + n),
    inner sweep about 72 nb^3 per pair)."""
    l = -(-n // nb)
    l += l & 1
    pairs = l * (l - 1) / 2
    return float(np.sum(np.asarray(sweeps, np.float64)) * cf * pairs * nb * nb *
                 (14 * m + 8 * n + 72 * nb))


def timed_calls(fn, steps, warmup):
    """Runs fn() warmup + steps times; HIP events around each timed call on
    torch's current stream (where the library is launched).  Returns
    (wall seconds per call, event ms per call, last result)."""
    import torch
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record()
        out = fn()
        e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return wall, float(np.mean([a.elapsed_time(b) for a, b in ev])), out


def square256_main(args, dev):
    """4000 FP64 256 x 256 (geometric spectra, kappa 1e2 / 1e8), block
    method, all-FP64 and FP32 sweeps + FP64 refinement."""
    import torch
    from paper_2601_17979_amd import svdb
    from workloads import gen
    batch = args.batch if args.batch != 10000 else 4000
    half = batch // 2
    idx = list(range(half)) + list(range(2000, 2000 + batch - half))
    grp = gen.square256(batch=4000, indices=idx)[0]
    Ag = svdb.col_major(torch.from_numpy(grp.A).to(dev))
    res = {}
    modes = {0: dict(precision=0, precondition=0), 1: dict(precision=1, precondition=0),
             2: dict(precision=0, precondition=1)}
    for mode, kw in modes.items():
        wall, ms, out = timed_calls(lambda: svdb.svd(Ag, path="blocked", nb=16, **kw),
                                    args.steps, args.warmup)
        S, U, V, info, sw = (x.cpu().numpy() for x in out)
        res[mode] = (wall, ms, S, info, sw)
    best = min(res, key=lambda k: res[k][0])
    wall, ms, S, info, sw = res[best]
    # the block Jacobi's work (on A, or on R^T after QR) plus, after QR, the
    # QR and the application of Q
    fl = flops_blocked(256, 256, 16, sw)
    if best == 2:
        fl += len(sw) * (2.0 * 256 ** 2 * (256 - 256 / 3.0) + 2.0 * 256 ** 2 * 256)
    achieved = fl / (ms * 1e-3)
    cpu = None
    sig_err = None
    if args.cpu_sample > 0:
        import oracle
        k = max(2, min(args.cpu_sample // 50, 40))
        pick = np.r_[0:k // 2, half:half + k - k // 2]
        t0 = time.perf_counter()
        Sr, _, _, swr, infor = oracle.gesvj_batch(grp.A[pick])
        t_cpu = time.perf_counter() - t0
        cpu = {"value": len(pick) / t_cpu, "unit": "SVDs/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": f"{len(pick)} matrices (half per kappa), FP64 "
                                           f"row-cyclic one-sided Jacobi, OpenMP over the batch",
               "seconds": t_cpu, **host_cpu()}
        sig_err = {p: float(np.max(np.abs(res[p][2][pick] - Sr) / Sr[:, :1])) for p in res}
    line = {
        "metric": "SVDs/sec, 256 x 256 FP64: all-FP64, FP32 sweeps + FP64 refinement, QR + "
                  "Jacobi on R^T",
        "value": batch / res[best][0], "unit": "SVDs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res[best][0] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{batch} FP64 256x256, geometric spectrum, half kappa 1e2 "
                               f"half 1e8 (Haar factors); block method nb 16",
                   "best_mode": {0: "fp64", 1: "fp32+fp64", 2: "qr+fp64"}[best],
                   **{name: {"svds_per_s": batch / res[k][0],
                             "sweeps_mean": float(np.mean(res[k][4])),
                             "sweeps_hist": sweep_histogram(res[k][4]),
                             "not_converged": int(np.sum(res[k][3] != 0))}
                      for k, name in enumerate(("fp64", "fp32+fp64", "qr+fp64"))},
                   "sigma_rel_err_vs_oracle_sample": sig_err},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                     "frac": achieved / 78.6e12, "traffic": None,
                     "kernel": "best mode's whole call (blk_iter dominant)", "kernel_ms": ms,
                     "flops_per_call": fl},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def uneven_main(args, dev):
    """20000 complex128 matrices, n ~ U{8..256}, m ~ U{n..2n}, complex
    Gaussian entries, in one svdb_svd_batched call."""
    import torch
    from paper_2601_17979_amd import svdb
    from workloads import gen
    batch = args.batch if args.batch != 10000 else 20000
    groups = gen.uneven_complex(batch=batch)
    mats = [svdb.col_major(torch.from_numpy(g.A).to(dev)) for g in groups]
    flat = [x[k] for x in mats for k in range(x.shape[0])]
    call = svdb.BatchedCall(flat)
    wall, ms, out = timed_calls(call, args.steps, args.warmup)
    info, sw = out[3].cpu().numpy(), out[4].cpu().numpy()
    shapes = [(g.m, g.n) for g in groups for _ in range(g.A.shape[0])]
    fl = sum(flops_blocked(m, n, 16, [s], cf=4) for (m, n), s in zip(shapes, sw))
    achieved = fl / (ms * 1e-3)
    cpu = None
    if args.cpu_sample > 0:
        import oracle
        pick = list(range(0, len(flat), max(1, len(flat) // 12)))[:12]
        As = [groups_A for groups_A in (g.A[k] for g in groups for k in range(g.A.shape[0]))]
        t0 = time.perf_counter()
        for k in pick:
            oracle.gesvj(As[k])
        t_cpu = time.perf_counter() - t0
        cpu = {"value": len(pick) / t_cpu, "unit": "SVDs/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(pick)} evenly spaced matrices, one at a time", "seconds": t_cpu,
               **host_cpu()}
    line = {
        "metric": "SVDs/sec, uneven complex128 batch in one call",
        "value": len(flat) / wall, "unit": "SVDs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"{len(flat)} complex128, n ~ U{{8..256}}, m ~ U{{n..2n}}, "
                               f"complex Gaussian entries; {len(groups)} distinct shapes",
                   "not_converged": int(np.sum(info != 0)),
                   "sweeps_mean": float(np.mean(sw)), "sweeps_hist": sweep_histogram(sw)},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                     "frac": achieved / 78.6e12, "traffic": None,
                     "kernel": "vb_iter (whole call)", "kernel_ms": ms, "flops_per_call": fl},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def tallskinny_main(args, dev):
    """The paper's tall-skinny experiment (section "Performance on
    Tall-Skinny Matrices"): batches of 1000 FP64 matrices with 16 columns and
    100 to 2000 rows, uniform [0, 1] entries, with and without the QR
    pre-processing.  The headline value is the m = 1000 point (AUTO)."""
    import torch
    from paper_2601_17979_amd import svdb
    from workloads import gen
    batch = args.batch if args.batch != 10000 else 1000
    points = {}
    for m in (100, 200, 500, 1000, 1500, 2000):
        A = np.stack([gen.uniform01(gen.rng_for(gen.BASE_SEED + 5000 + m, k), m, 16)
                      for k in range(batch)])
        Ag = svdb.col_major(torch.from_numpy(A).to(dev))
        row = {}
        for name, pc in (("auto", -1), ("qr", 1), ("no_qr", 0)):
            try:
                p = svdb.plan(torch.float64, m, 16, precondition=pc)
            except svdb.SvdbError:
                continue
            wall, ms, out = timed_calls(lambda: svdb.svd(Ag, precondition=pc), args.steps,
                                        args.warmup)
            info, sw = out[3].cpu().numpy(), out[4].cpu().numpy()
            row[name] = {"svds_per_s": batch / wall, "ms": wall * 1e3,
                         "sweeps_mean": float(np.mean(sw)), "not_converged": int(np.sum(info != 0)),
                         "path": ["auto", "plain", "resident", "blocked"][p[0]]}
        points[m] = row
    head = points[1000]["auto"]
    line = {
        "metric": "SVDs/sec, 1000 FP64 tall-skinny 1000x16 (uniform [0,1]); rows 100..2000 in config",
        "value": head["svds_per_s"], "unit": "SVDs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{batch} FP64 m x 16, m in 100..2000, uniform [0,1] entries",
                   "points": {str(k): v for k, v in points.items()}},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", default="auto")
    ap.add_argument("--batch", type=int, default=10000)
    ap.add_argument("--streams", type=int, default=1,
                    help="HIP streams the headline's two shape groups are issued on (they are "
                         "independent): 1 = one after the other (default; the roofline is "
                         "then that of the dominant call); 2 = one each, overlapped (the "
                         "roofline is then that of the whole step)")
    ap.add_argument("--cpu-sample", type=int, default=5000,
                    help="matrices per shape for the CPU oracle baseline (default: the whole "
                         "workload, about 20 core-seconds; 0 = skip)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain GPU Jacobi comparator run")
    ap.add_argument("--serve-seconds", type=float, default=8.0,
                    help="length of the Poisson serving run (0 = skip the serving leg)")
    ap.add_argument("--serve-precondition", type=int, default=-1,
                    help="QR preconditioning of the serving leg's real requests: -1 (the "
                         "server default) or 1 on, 0 off")
    ap.add_argument("--serve-load", type=float, default=0.5,
                    help="offered load as a fraction of the measured saturation rate")
    ap.add_argument("--workload", default="mixed", choices=["mixed", "square256", "uneven", "tallskinny"],
                    help="mixed: the headline workload (default); square256: 4000 FP64 "
                         "256 x 256, all-FP64 and mixed precision; uneven: 20000 complex128 "
                         "of random shapes in one svdb_svd_batched call")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run one device-to-device copy of this many bytes (used to "
                         "calibrate the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2601_17979_amd import svdb
    from workloads import gen

    dev = torch.device("cuda:0")
    if args.copy_bytes:
        x = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes}))
        return
    if args.workload == "square256":
        return square256_main(args, dev)
    if args.workload == "tallskinny":
        return tallskinny_main(args, dev)
    if args.workload == "uneven":
        return uneven_main(args, dev)
    groups = gen.mixed_64_128x32(batch=args.batch)
    total = sum(g.A.shape[0] for g in groups)
    stream = torch.cuda.current_stream(dev)

    def prepare(path):
        work = []
        for g in groups:
            Ag = svdb.col_major(torch.from_numpy(g.A).to(dev))
            b = g.A.shape[0]
            out = (torch.empty((b, g.n), dtype=torch.float64, device=dev),
                   svdb.empty_col_major(b, g.m, g.n, torch.float64, dev),
                   svdb.empty_col_major(b, g.n, g.n, torch.float64, dev),
                   torch.empty(b, dtype=torch.int32, device=dev),
                   torch.empty(b, dtype=torch.int32, device=dev))
            work.append((g, Ag, out))
        return work

    # the shape groups are independent: with --streams 2 the first group's
    # call runs on the current stream and every other group's on a side
    # stream of its own, joined back before the step ends
    sides = [torch.cuda.Stream(dev) for _ in groups[1:]] if args.streams > 1 else []

    def issue(calls, events=None):
        for s_ in sides:
            s_.wait_stream(stream)
        for k, call in enumerate(calls):
            st = sides[k - 1] if (k > 0 and sides) else stream
            with torch.cuda.stream(st):
                if events is not None:
                    events[k][0].record(st)
                call()
                if events is not None:
                    events[k][1].record(st)
        for s_ in sides:
            stream.wait_stream(s_)

    def run(work, path, events=None):
        issue([lambda Ag=Ag, out=out: svdb.svd(Ag, path=path, out=out)
               for g, Ag, out in work], events)

    def timed(path, steps, warmup):
        work = prepare(path)
        for _ in range(warmup):
            run(work, path)
        torch.cuda.synchronize()
        ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in work] for _ in range(steps)]
        sev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        t0 = time.perf_counter()
        for s in range(steps):
            sev[s][0].record(stream)
            run(work, path, ev[s])
            sev[s][1].record(stream)   # after the side streams have joined
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_kernel = [np.mean([ev[s][k][0].elapsed_time(ev[s][k][1]) for s in range(steps)])
                      for k in range(len(work))]
        step_ms = float(np.mean([a.elapsed_time(b) for a, b in sev]))
        return work, wall, per_kernel, step_ms

    work, wall, per_kernel, step_ms = timed(args.path, args.steps, args.warmup)
    ms_per_step = wall / args.steps * 1e3
    value = total * args.steps / wall

    results = []
    for g, Ag, out in work:
        S, U, V, info, sw = (x.cpu().numpy() for x in out)
        results.append((g, S, U, V, info, sw))
    bad = int(sum(int(np.sum(r[4] != 0)) for r in results))

    # Work of one call.  With QR preconditioning (the AUTO default for these
    # shapes) a call is the pivoted QR of A (2n^2(m - n/3)), the QR of R1^T
    # (4n^3/3), the Jacobi on R2^T (n x n), U = Q1 [U_x; 0] (2n^2(2m - n))
    # and V = P Q2 J (2n^3); its work is counted as all five.
    def call_flops(g, sw):
        # AUTO preconditions where precondition = 1 is accepted, except FP64
        # with n <= 16 and m < 8 n
        try:
            svdb.plan(torch.float64, g.m, g.n, path="auto", precondition=1)
            pc = args.path == "auto" and not (g.n <= 16 and g.m < 8 * g.n)
        except svdb.SvdbError:
            pc = False
        if not pc:
            return flops_unblocked(g.m, g.n, sw), False
        m_, n_ = g.m, g.n
        return flops_unblocked(n_, n_, sw) + len(sw) * (
            2.0 * n_ * n_ * (m_ - n_ / 3.0) + 4.0 * n_ ** 3 / 3.0 +
            2.0 * n_ * n_ * (2 * m_ - n_) + 2.0 * n_ ** 3), True

    flc = [call_flops(r[0], r[5]) for r in results]
    label = " (pivoted QR, QR of R1^T, Jacobi on R2^T, Q1 and Q2 applied)"
    if sides:
        # the calls overlap on two streams: the unit is one whole step, timed
        # from before the first launch to after the side streams joined
        fl = sum(f for f, _ in flc)
        traffic = [measured_traffic(f"{r[0].m}x{r[0].n}") if pc else None
                   for r, (_, pc) in zip(results, flc)]
        kname = ("one step: " + " and ".join(f"{r[0].m}x{r[0].n}" for r in results) +
                 " calls on two streams" + (label if all(pc for _, pc in flc) else ""))
        kms = step_ms
        tr = sum(traffic) if all(t is not None for t in traffic) else None
    else:
        # the dominant call: the launch sequence with the longest duration
        kdom = int(np.argmax(per_kernel))
        gd = results[kdom][0]
        fl, pc = flc[kdom]
        kname = f"{gd.m}x{gd.n} call" + (label if pc else " (resident Jacobi)")
        kms = per_kernel[kdom]
        tr = measured_traffic(f"{gd.m}x{gd.n}") if pc else None
    achieved = fl / (kms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VALU_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK, "traffic": tr,
                "kernel": kname, "kernel_ms": kms, "flops_per_launch": fl}

    # the same kernels without QR preconditioning (the iteration on A itself)
    noqr = None
    if args.path == "auto" and not args.no_plain:
        def run_noqr():
            issue([lambda Ag=Ag, out=out: svdb.svd(Ag, path="auto", precondition=0, out=out)
                   for g, Ag, out in work])
        wall_n, ms_n, _ = timed_calls(run_noqr, max(1, args.steps // 2), 1)
        noqr = {"value": total / wall_n, "unit": "SVDs/s", "ms_per_step": wall_n * 1e3}

    # the plain GPU Jacobi on the same workload (the comparator of the metric)
    plain = None
    if args.path != "plain" and not args.no_plain:
        _, wall_p, per_p, _ = timed("plain", max(1, args.steps // 2), 1)
        plain = {"value": total * max(1, args.steps // 2) / wall_p, "unit": "SVDs/s",
                 "ms_per_step": wall_p / max(1, args.steps // 2) * 1e3,
                 "kernel_ms": [float(x) for x in per_p]}

    # the serving leg runs before the oracle, whose OpenMP worker threads may
    # keep host cores busy after it returns
    serve = serve_leg(args, dev) if args.serve_seconds > 0 else None

    # accuracy vs the FP64 oracle and the CPU baseline on a bounded sample
    cpu = None
    sig_err = None
    if args.cpu_sample > 0:
        import oracle
        t_cpu, n_cpu, errs, sw_ratio = 0.0, 0, [], []
        for g, S, U, V, info, sw in results:
            b = g.A.shape[0]
            idx = np.linspace(0, b - 1, min(args.cpu_sample, b)).astype(int)
            t0 = time.perf_counter()
            Sr, _, _, swr, infor = oracle.gesvj_batch(g.A[idx])
            t_cpu += time.perf_counter() - t0
            n_cpu += len(idx)
            errs.append(float(np.max(np.abs(S[idx] - Sr) / Sr[:, :1])))
            sw_ratio.append(float(np.sum(swr) / max(np.sum(sw[idx]), 1)))
        cpu = {"value": n_cpu / t_cpu, "unit": "SVDs/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{n_cpu} matrices ({args.cpu_sample} evenly spaced per shape, both "
                         f"spectrum families), FP64 row-cyclic one-sided Jacobi, OpenMP over "
                         f"the batch", "seconds": t_cpu,
               "oracle_sweeps_per_gpu_sweep": sw_ratio, **host_cpu()}
        sig_err = max(errs)


    line = {
        "metric": METRIC, "value": value, "unit": "SVDs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD, "path": args.path, "batch": total,
                   "streams": 2 if sides else 1,
                   "sigma_rel_err_vs_oracle_sample": sig_err, "not_converged": bad,
                   "sweeps_mean": {f"{r[0].m}x{r[0].n}": float(np.mean(r[5])) for r in results},
                   "sweeps_hist": {f"{r[0].m}x{r[0].n}": sweep_histogram(r[5]) for r in results},
                   "kernel_ms": {f"{r[0].m}x{r[0].n}": float(k) for r, k in
                                 zip(results, per_kernel)}},
        "plain_gpu_jacobi": plain,
        "resident_without_qr": noqr,
        "speedup_vs_plain": (value / plain["value"]) if plain else 1.0,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serve": serve,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
