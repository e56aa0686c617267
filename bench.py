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


def serve_setup(args, dev):
    """The serving pool on the device and a server over it; saturation =
    a closed batch of 8 x the pool submitted at once (after one warm-up
    pass), in requests per second."""
    import torch
    from paper_2601_17979_amd import svdb
    from workloads import gen
    pool = gen.serving_pool(per_class=4)
    tdt = {"f64": torch.float64, "f32": torch.float32}
    dev_pool = [svdb.col_major(torch.from_numpy(A)[None].to(tdt[d]).to(dev))[0]
                for A, d in pool]
    names = [f"{A.shape[0]}x{A.shape[1]}" for A, d in pool]
    torch.cuda.synchronize()
    budget = 8 << 30
    srv = svdb.Server(budget_bytes=budget, max_requests=2048,
                      precondition=args.serve_precondition)

    def drain(n, t_limit):
        got, t0 = 0, time.time()
        while got < n and time.time() - t0 < t_limit:
            got += len(srv.poll(timeout_ms=100))
        return got

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
    return srv, dev_pool, names, sat, budget


def poisson_run(srv, dev_pool, names, rate, seconds, max_requests, seed):
    """Poisson arrivals at `rate` for `seconds` or until max_requests were
    submitted; latency = completion - submission on the server's clock."""
    from paper_2601_17979_amd import svdb
    rng = np.random.default_rng(seed)
    lat, n_sub, cls, by_class = [], 0, {}, {}

    def collect(items):
        for rid, ts, td, out in items:
            lat.append(td - ts)
            by_class.setdefault(cls.pop(rid), []).append(td - ts)
    t_start = svdb.Server.clock()
    t_next = t_start
    while t_next - t_start < seconds and n_sub < max_requests:
        now = svdb.Server.clock()
        if now < t_next:
            collect(srv.poll(timeout_ms=0))
            time.sleep(max(0.0, min(t_next - svdb.Server.clock(), 0.002)))
            continue
        k = int(rng.integers(len(dev_pool)))
        rid = srv.submit(dev_pool[k])
        cls[rid] = names[k]
        n_sub += 1
        t_next += rng.exponential(1.0 / rate)
    t_sub_end = svdb.Server.clock()
    t0 = time.time()
    while len(lat) < n_sub and time.time() - t0 < 120:
        collect(srv.poll(timeout_ms=100))
    t_end = svdb.Server.clock()
    lat = np.sort(np.asarray(lat))
    per_class = {c: {"count": len(v), "p50_ms": float(np.percentile(v, 50) * 1e3),
                     "p99_ms": float(np.percentile(v, 99) * 1e3)}
                 for c, v in sorted(by_class.items(), key=lambda kv: int(kv[0].split("x")[1]))}
    return {"offered_rate_per_s": rate, "requests": int(n_sub), "completed": int(lat.size),
            "submit_seconds": t_sub_end - t_start,
            "completed_per_s": lat.size / max(t_end - t_start, 1e-9),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "per_class": per_class}


SERVE_WORKLOAD = ("12 shape classes n in {16,...,512} x {square, 2n x n}, FP64/FP32 "
                  "alternating, geometric spectrum kappa log-uniform [1, 1e8]")


def serve_leg(args, dev):
    """Serving workload: requests from 12 shape classes (n in {16..512} x
    {square, m = 2n}), FP64/FP32 alternating, kappa log-uniform in [1, 1e8].
    Saturation = a closed batch of requests submitted at once; then Poisson
    arrivals at `serve_load` x saturation for `serve_seconds`."""
    srv, dev_pool, names, sat, budget = serve_setup(args, dev)
    r = poisson_run(srv, dev_pool, names, args.serve_load * sat, args.serve_seconds, 10 ** 9,
                    17979 + 4000)
    srv.close()
    return {"workload": SERVE_WORKLOAD, "saturation_svds_per_s": sat,
            "offered_load": args.serve_load, **r, "budget_bytes": budget,
            "qr_preconditioning": args.serve_precondition != 0}


def serve_main(args, dev):
    """The serving rate sweep: Poisson arrivals at 0.25, 0.5, 0.75, 0.9, 1.0
    and 1.2 x the measured saturation, each for 20000 requests or 60 s
    (whichever comes first), p50 / p99 latency per rate."""
    srv, dev_pool, names, sat, budget = serve_setup(args, dev)
    rates = {}
    for i, load in enumerate((0.25, 0.5, 0.75, 0.9, 1.0, 1.2)):
        r = poisson_run(srv, dev_pool, names, load * sat, 60.0, 20000, 17979 + 4100 + i)
        rates[str(load)] = r
        print(json.dumps({"load": load, "rate": r["offered_rate_per_s"],
                          "requests": r["requests"], "p50_ms": r["p50_ms"],
                          "p99_ms": r["p99_ms"]}), file=sys.stderr, flush=True)
    srv.close()
    head = rates["0.5"]
    line = {
        "metric": "serve p50/p99 latency (ms) vs offered load", "value": head["p99_ms"],
        "unit": "ms (p99 at 0.5 x saturation)", "n_gpus": 1, "steps": len(rates), "warmup": 1,
        "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64/f32", "data": "synthetic",
        "config": {"workload": SERVE_WORKLOAD, "saturation_svds_per_s": sat,
                   "budget_bytes": budget, "qr_preconditioning": args.serve_precondition != 0,
                   "rates": rates},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


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


def oracle_each(mats, threads=16):
    """The oracle on a list of matrices of any shapes, one matrix per host
    thread (each a single-threaded row-cyclic Jacobi).  Returns (S list,
    sweeps list, seconds, threads)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda A: oracle.gesvj(A, want_u=False, want_v=False), mats))
    return [r[0] for r in res], [r[3] for r in res], time.perf_counter() - t0, threads


def square256_leg(dev, grp, steps=2, warmup=1, cpu_sample=40):
    """The 256 x 256 workload: 4000 FP64 matrices, geometric spectra, half
    kappa 1e2, half 1e8. Four modes of the same call: all-FP64 block
    sweeps on A, FP32 MFMA sweeps + FP64 refinement, the default (QR
    preconditioning, block sweeps on R2^T), and the QR preconditioning
    with FP32 sweeps + FP64 refinement on R2^T. Each with its sigma error
    against the oracle on a sample."""
    import torch
    from paper_2601_17979_amd import svdb
    batch = grp.A.shape[0]
    half = batch // 2
    Ag = svdb.col_major(torch.from_numpy(grp.A).to(dev))
    modes = {"fp64": dict(path="blocked", nb=16, precision=0, precondition=0),
             "fp32+fp64": dict(path="blocked", nb=16, precision=1, precondition=0),
             "qr+fp64": dict(),
             "qr+fp32+fp64": dict(precision=1)}
    k = max(2, cpu_sample)
    pick = np.r_[0:k // 2, half:half + k - k // 2]
    Sr, swr, t_cpu, thr = oracle_each([grp.A[i] for i in pick])
    Sr = np.stack(Sr)
    res = {}
    for name, kw in modes.items():
        wall, ms, out = timed_calls(lambda: svdb.svd(Ag, **kw), steps, warmup)
        S, info, sw = out[0].cpu().numpy(), out[3].cpu().numpy(), out[4].cpu().numpy()
        res[name] = {"svds_per_s": batch / wall, "ms": wall * 1e3, "event_ms": ms,
                     "sweeps_mean": float(np.mean(sw)), "sweeps_hist": sweep_histogram(sw),
                     "not_converged": int(np.sum(info != 0)),
                     "sigma_rel_err_vs_oracle_sample":
                         float(np.max(np.abs(S[pick] - Sr) / Sr[:, :1])),
                     "_sw": sw}
    best = max(res, key=lambda n_: res[n_]["svds_per_s"])
    # block-method work on the iteration's own matrix (A or R2^T) over the
    # sweeps executed, plus the two QRs and the two applications of Q
    sw = res[best].pop("_sw")
    fl = flops_blocked(256, 256, 16, sw)
    if best in ("qr+fp64", "qr+fp32+fp64"):
        fl += len(sw) * (2 * (4.0 * 256 ** 3 / 3.0) + 2.0 * 256 ** 3 + 2.0 * 256 ** 3)
    for r in res.values():
        r.pop("_sw", None)
    achieved = fl / (res[best]["event_ms"] * 1e-3)
    return {
        "workload": f"{batch} FP64 256x256, geometric spectrum, half kappa 1e2, half 1e8 "
                    f"(Haar factors)",
        "value": res[best]["svds_per_s"], "unit": "SVDs/s", "best_mode": best, "modes": res,
        "mixed_vs_fp64": res["fp32+fp64"]["svds_per_s"] / res["fp64"]["svds_per_s"],
        "qr_mixed_vs_qr_fp64": res["qr+fp32+fp64"]["svds_per_s"] / res["qr+fp64"]["svds_per_s"],
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": 78.6,
                     "unit": "TFLOP/s", "frac": achieved / 78.6e12, "traffic": None,
                     "kernel": f"{best} call (block method dominant)",
                     "kernel_ms": res[best]["event_ms"], "flops_per_call": fl},
        "cpu_baseline": {"value": len(pick) / t_cpu, "unit": "SVDs/s", "cores": thr,
                         "kind": "oracle",
                         "sample": f"{len(pick)} matrices (half per kappa), FP64 row-cyclic "
                                   f"one-sided Jacobi, one matrix per host thread",
                         "seconds": t_cpu, "oracle_sweeps_mean": float(np.mean(swr)),
                         **host_cpu()},
    }


def square256_main(args, dev):
    from workloads import gen
    grp = gen.square256(batch=4000, workers=min(16, os.cpu_count() or 1))[0]
    leg = square256_leg(dev, grp, args.steps, args.warmup, max(2, args.cpu_sample // 125))
    line = {
        "metric": "SVDs/sec, 256 x 256 FP64: all-FP64, FP32 sweeps + FP64 refinement, QR + "
                  "Jacobi on R^T",
        "value": leg["value"], "unit": "SVDs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": leg["modes"][leg["best_mode"]]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {k: v for k, v in leg.items() if k not in ("roofline", "cpu_baseline")},
        "roofline": leg["roofline"], "cpu_baseline": leg["cpu_baseline"],
    }
    print(json.dumps(line), flush=True)


def flops_unblocked_cx(m, n, sweeps, cf):
    """Alg. 2 work (as flops_unblocked) times the flop factor cf (4 for
    complex data)."""
    return cf * flops_unblocked(m, n, sweeps)


def uneven_leg(dev, groups, steps=2, warmup=1, cpu_sample=16):
    """The uneven workload: 20000 complex128 matrices, n ~ U{8..256}, m ~
    U{n..2n}, complex Gaussian entries, in one svdb_svd_batched call (each
    launch of one round-robin iteration covers every shape)."""
    import torch
    from paper_2601_17979_amd import svdb
    mats = [svdb.col_major(torch.from_numpy(g.A).to(dev)) for g in groups]
    flat = [x[k] for x in mats for k in range(x.shape[0])]
    shapes = [(g.m, g.n) for g in groups for _ in range(g.A.shape[0])]
    host = [g.A[k] for g in groups for k in range(g.A.shape[0])]
    call = svdb.BatchedCall(flat)
    wall, ms, out = timed_calls(call, steps, warmup)
    info, sw = out[3].cpu().numpy(), out[4].cpu().numpy()
    pick = np.linspace(0, len(flat) - 1, cpu_sample).astype(int)
    Sr, swr, t_cpu, thr = oracle_each([host[i] for i in pick])
    err = max(float(np.max(np.abs(out[0][i].cpu().numpy() - s) / s[0])) for i, s in zip(pick, Sr))
    # work as in the roofline rule: Alg. 2 on the real shape (complex flops),
    # over the oracle's sweeps; the oracle ran on a sample, so the GPU's
    # sweep counts are scaled by the sample's oracle / GPU sweep ratio
    ratio = float(np.sum(swr) / max(np.sum(sw[pick]), 1))
    fl = sum(flops_unblocked_cx(m, n, [s * ratio], 4) for (m, n), s in zip(shapes, sw))
    achieved = fl / (ms * 1e-3)
    return {
        "workload": f"{len(flat)} complex128, n ~ U{{8..256}}, m ~ U{{n..2n}}, complex Gaussian "
                    f"entries; {len(groups)} distinct shapes, one svdb_svd_batched call",
        "value": len(flat) / wall, "unit": "SVDs/s", "ms": wall * 1e3, "event_ms": ms,
        "not_converged": int(np.sum(info != 0)), "sweeps_mean": float(np.mean(sw)),
        "sweeps_hist": sweep_histogram(sw),
        "sigma_rel_err_vs_oracle_sample": err,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VALU_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK, "traffic": None,
                     "kernel": "whole call (vb_iter dominant); work = Alg. 2 on the real "
                               "shapes over the oracle's sweeps",
                     "kernel_ms": ms, "flops_per_call": fl,
                     "oracle_sweeps_per_gpu_sweep": ratio},
        "cpu_baseline": {"value": len(pick) / t_cpu, "unit": "SVDs/s", "cores": thr,
                         "kind": "oracle",
                         "sample": f"{len(pick)} evenly spaced matrices, complex128 row-cyclic "
                                   f"one-sided Jacobi, one matrix per host thread",
                         "seconds": t_cpu, **host_cpu()},
    }


def uneven_main(args, dev):
    from workloads import gen
    groups = gen.uneven_complex(batch=20000, workers=min(16, os.cpu_count() or 1))
    leg = uneven_leg(dev, groups, args.steps, args.warmup)
    line = {
        "metric": "SVDs/sec, uneven complex128 batch in one call",
        "value": leg["value"], "unit": "SVDs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": leg["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {k: v for k, v in leg.items() if k not in ("roofline", "cpu_baseline")},
        "roofline": leg["roofline"], "cpu_baseline": leg["cpu_baseline"],
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
    ap.add_argument("--workload", default="mixed",
                    choices=["mixed", "square256", "uneven", "tallskinny", "serve"],
                    help="mixed: the headline workload (default); square256: 4000 FP64 "
                         "256 x 256, all-FP64 and mixed precision; uneven: 20000 complex128 "
                         "of random shapes in one svdb_svd_batched call; serve: the "
                         "serving rate sweep (0.25 ... 1.2 x saturation)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run one device-to-device copy of this many bytes (used to "
                         "calibrate the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra keys of the default line: the 256 x 256 precision "
                         "workload and the uneven complex128 workload (each timed with one "
                         "warm-up and two timed calls), and the blocked nb = 8 / 16 runs of "
                         "the headline workload")
    ap.add_argument("--serve-after-oracle", action="store_true",
                    help="run the serving leg after the CPU oracle instead of before it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    from workloads import gen
    # inputs of the default line's extra keys, drawn in worker processes
    # before this process touches the GPU
    workers = min(16, os.cpu_count() or 1)
    extras = None
    if args.workload == "mixed" and not args.no_extras and not args.copy_bytes:
        extras = (gen.square256(batch=4000, workers=workers)[0],
                  gen.uneven_complex(batch=20000, workers=workers))

    import torch
    from paper_2601_17979_amd import svdb

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
    if args.workload == "serve":
        return serve_main(args, dev)
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
    # shapes) a call is the QR of A (2n^2(m - n/3)), the QR of R1^T
    # (4n^3/3), the Jacobi on R2^T (n x n), U = Q1 [U_x; 0] (2n^2(2m - n))
    # and V = P Q2 J (2n^3); its work is counted as all five, the Jacobi with
    # its rotations of V.  For 32 < n <= 64 the library does less than that:
    # the Jacobi leaves V out and V = P R1^-1 U_x S comes from a back
    # substitution (n^3) and a J^T J check (2n^3), Q2 is not applied.
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
    label = (" (QR, QR of R1^T, Jacobi on R2^T, U = Q1 U_x; work counted as"
             " Alg. 2 with V and both applications of Q)")
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
    plain_S = None
    if args.path != "plain" and not args.no_plain:
        work_p, wall_p, per_p, _ = timed("plain", max(1, args.steps // 2), 1)
        plain = {"value": total * max(1, args.steps // 2) / wall_p, "unit": "SVDs/s",
                 "ms_per_step": wall_p / max(1, args.steps // 2) * 1e3,
                 "kernel_ms": [float(x) for x in per_p]}
        plain_S = [out[0].cpu().numpy() for g, Ag, out in work_p]

    # the block method on the same workload with nb = 8 and nb = 16 (no QR)
    blocked = {}
    blocked_S = {}
    if extras is not None:
        for nb_ in (8, 16):
            def run_nb(nb_=nb_):
                return [svdb.svd(Ag, path="blocked", nb=nb_, precondition=0, out=out)
                        for g, Ag, out in work]
            wall_b, ms_b, outs = timed_calls(run_nb, 2, 1)
            blocked[f"nb{nb_}"] = {"value": total / wall_b, "unit": "SVDs/s",
                                   "ms_per_step": wall_b * 1e3,
                                   "not_converged": int(sum(int((o[3] != 0).sum()) for o in outs)),
                                   "sweeps_mean": {f"{g.m}x{g.n}": float(o[4].double().mean())
                                                   for (g, _, _), o in zip(work, outs)}}
            blocked_S[f"nb{nb_}"] = [o[0].cpu().numpy() for o in outs]

    def serve_now():
        return serve_leg(args, dev) if args.serve_seconds > 0 else None
    # by default the serving leg runs before the CPU oracle
    serve = None if args.serve_after_oracle else serve_now()

    # accuracy vs the FP64 oracle and the CPU baseline on a bounded sample
    cpu = None
    sig_err = None
    if args.cpu_sample > 0:
        import oracle
        t_cpu, n_cpu, errs, sw_ratio = 0.0, 0, [], []
        perr = []
        berr = {k: [] for k in blocked_S}
        for gi, (g, S, U, V, info, sw) in enumerate(results):
            b = g.A.shape[0]
            idx = np.linspace(0, b - 1, min(args.cpu_sample, b)).astype(int)
            t0 = time.perf_counter()
            Sr, _, _, swr, infor = oracle.gesvj_batch(g.A[idx])
            t_cpu += time.perf_counter() - t0
            n_cpu += len(idx)
            errs.append(float(np.max(np.abs(S[idx] - Sr) / Sr[:, :1])))
            if plain_S is not None:
                perr.append(float(np.max(np.abs(plain_S[gi][idx] - Sr) / Sr[:, :1])))
            for k in blocked_S:
                berr[k].append(float(np.max(np.abs(blocked_S[k][gi][idx] - Sr) / Sr[:, :1])))
            sw_ratio.append(float(np.sum(swr) / max(np.sum(sw[idx]), 1)))
        if plain is not None and perr:
            plain["sigma_rel_err_vs_oracle_sample"] = max(perr)
        for k in blocked:
            blocked[k]["sigma_rel_err_vs_oracle_sample"] = max(berr[k])
        cpu = {"value": n_cpu / t_cpu, "unit": "SVDs/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{n_cpu} matrices ({args.cpu_sample} evenly spaced per shape, both "
                         f"spectrum families), FP64 row-cyclic one-sided Jacobi, OpenMP over "
                         f"the batch", "seconds": t_cpu,
               "oracle_sweeps_per_gpu_sweep": sw_ratio, **host_cpu()}
        sig_err = max(errs)
    if serve is None:
        serve = serve_now()

    square = uneven = None
    if extras is not None:
        square = square256_leg(dev, extras[0])
        uneven = uneven_leg(dev, extras[1])

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
        "blocked_without_qr": blocked or None,
        "speedup_vs_plain": (value / plain["value"]) if plain else 1.0,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serve": serve,
        "square256": square,
        "uneven_complex128": uneven,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
