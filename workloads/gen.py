"""Seeded synthetic inputs for the batched SVD.

This module holds no arithmetic of the Jacobi method: it only draws random
matrices.  Both the GPU library's users (benchmark, tests) and the oracle's
tests take their inputs from here, so that the two sides see the same data.

Every matrix has its own random stream, derived from (base seed, index) with
numpy's SeedSequence, so a matrix is identical whether it is drawn alone or as
part of any batch.

Singular-value families follow the paper's accuracy table (Table "svd_dist",
section "Numerical Accuracy"): random, arith, cluster0, cluster1, logrand, geo; `logu` is a
log-uniform spectrum on an interval [lo, hi].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 17979


def rng_for(base: int, index: int) -> np.random.Generator:
    """Independent stream for matrix `index` of a workload with seed `base`."""
    return np.random.default_rng(np.random.SeedSequence(entropy=base, spawn_key=(index,)))


def haar(rng: np.random.Generator, n: int, complex_: bool = False) -> np.ndarray:
    """Haar-distributed orthogonal (unitary) n x n matrix: QR of a Gaussian
    matrix with the phases of diag(R) moved into Q."""
    if complex_:
        Z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    else:
        Z = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R)
    ph = d / np.abs(d)
    return Q * ph[None, :]


def spectrum(kind: str, n: int, kappa: float = 1e6, rng: np.random.Generator | None = None,
             lo: float = 1e-3, hi: float = 1.0) -> np.ndarray:
    """Singular values, descending, for the families of the paper's table."""
    i = np.arange(1, n + 1, dtype=np.float64)
    if kind == "arith":
        s = 1.0 - (i - 1) / max(n - 1, 1) * (1.0 - 1.0 / kappa)
    elif kind == "cluster0":
        s = np.full(n, 1.0 / kappa)
        s[0] = 1.0
    elif kind == "cluster1":
        s = np.ones(n)
        s[-1] = 1.0 / kappa
    elif kind == "logrand":
        s = np.exp(rng.uniform(np.log(1.0 / kappa), 0.0, n))
    elif kind == "geo":
        s = kappa ** ((1.0 - i) / max(n - 1, 1))
    elif kind == "logu":
        s = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    else:
        raise ValueError(kind)
    return np.sort(s)[::-1].copy()


def from_spectrum(rng: np.random.Generator, m: int, n: int, s: np.ndarray,
                  complex_: bool = False) -> np.ndarray:
    """A = U[:, :n] diag(s) V^H with Haar U (m x m) and V (n x n), in FP64."""
    U = haar(rng, m, complex_)[:, :n]
    V = haar(rng, n, complex_)
    return (U * s[None, :]) @ V.conj().T


def gaussian(rng: np.random.Generator, m: int, n: int, complex_: bool = False) -> np.ndarray:
    """i.i.d. N(0,1) entries; complex entries are (N + iN)/sqrt(2)."""
    if complex_:
        return (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) / np.sqrt(2.0)
    return rng.standard_normal((m, n))


def uniform01(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """Uniform [0, 1) entries, the paper's `random` family (subsection "Performance of the Baseline
    Implementation")."""
    return rng.uniform(0.0, 1.0, (m, n))


def family(rng, kind: str, m: int, n: int, kappa: float, complex_: bool = False) -> np.ndarray:
    """One matrix of a named family ('random' = uniform entries)."""
    if kind == "random":
        A = uniform01(rng, m, n)
        if complex_:
            A = A + 1j * uniform01(rng, m, n)
        return A
    if kind == "gauss":
        return gaussian(rng, m, n, complex_)
    return from_spectrum(rng, m, n, spectrum(kind, n, kappa, rng), complex_)


# ---------------------------------------------------------------------------
# Workloads.  Each is a list of uniform-shape groups.
# ---------------------------------------------------------------------------

@dataclass
class Group:
    m: int
    n: int
    A: np.ndarray                 # (batch, m, n), FP64 or complex128
    kinds: list = field(default_factory=list)   # per-matrix family tag
    seeds: tuple = ()             # (base, first index)


def _batch(base: int, first: int, count: int, make) -> np.ndarray:
    return np.stack([make(rng_for(base, first + k)) for k in range(count)])


def small16(batch: int = 1000, seed: int = BASE_SEED) -> list:
    """batch x (16 x 16) FP64, A = U diag(s) V^T, Haar U, V, s log-uniform in
    [1e-3, 1]."""
    A = _batch(seed, 0, batch,
               lambda r: from_spectrum(r, 16, 16, spectrum("logu", 16, rng=r, lo=1e-3, hi=1.0)))
    return [Group(16, 16, A, ["logu"] * batch, (seed, 0))]


def mixed_64_128x32(batch: int = 10000, seed: int = BASE_SEED + 1000) -> list:
    """batch FP64 matrices: half 64 x 64, half 128 x 32; within each shape half
    have a geometric spectrum with kappa = 1e6 (Haar factors) and half i.i.d.
    N(0,1) entries."""
    groups = []
    half = batch // 2
    for gi, (m, n) in enumerate(((64, 64), (128, 32))):
        first = gi * half
        nq = half // 2

        def make(r, k, m=m, n=n):
            if k < nq:
                return from_spectrum(r, m, n, spectrum("geo", n, 1e6))
            return gaussian(r, m, n)
        A = np.stack([make(rng_for(seed, first + k), k) for k in range(half)])
        groups.append(Group(m, n, A, ["geo1e6"] * nq + ["gauss"] * (half - nq), (seed, first)))
    return groups


def _pool_map(fn, chunks, workers):
    """fn over chunks, in worker processes when workers > 1 (forked: call this
    before the process uses a GPU).  Every matrix has its own seeded stream,
    so the result does not depend on the split."""
    if not workers or workers <= 1 or len(chunks) <= 1:
        return [fn(c) for c in chunks]
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(fn, chunks))


def _split(ks, workers):
    step = max(1, -(-len(ks) // max(4 * (workers or 1), 1)))
    return [ks[i:i + step] for i in range(0, len(ks), step)]


def _one_thread():
    """Single-threaded BLAS inside a worker process (the pool supplies the
    parallelism)."""
    from threadpoolctl import threadpool_limits
    return threadpool_limits(1)


def _square256_part(arg):
    seed, half, ks = arg
    with _one_thread():
        return np.stack([from_spectrum(rng_for(seed, k), 256, 256,
                                       spectrum("geo", 256, 1e2 if k < half else 1e8))
                         for k in ks])


def square256(batch: int = 4000, seed: int = BASE_SEED + 2000, indices=None,
              workers: int = 0) -> list:
    """batch x (256 x 256) FP64 geometric spectra, half kappa = 1e2, half 1e8.
    `indices` selects a subset of the batch (the same matrices as in the
    full batch); `workers` > 1 draws them in that many processes."""
    half = batch // 2
    ks = list(range(batch)) if indices is None else [int(k) for k in indices]
    parts = _pool_map(_square256_part, [(seed, half, c) for c in _split(ks, workers)], workers)
    A = np.concatenate(parts) if parts else np.zeros((0, 256, 256))
    kinds = ["geo1e2" if k < half else "geo1e8" for k in ks]
    return [Group(256, 256, A, kinds, (seed, ks[0] if ks else 0))]


def uneven_complex(batch: int = 20000, seed: int = BASE_SEED + 3000, nmin: int = 8,
                   nmax: int = 256, workers: int = 0) -> list:
    """complex128 matrices with n ~ U{nmin..nmax}, m ~ U{n..2n}, i.i.d.
    complex Gaussian entries; returned as one group per shape, in order of
    shape.  `workers` > 1 draws them in that many processes."""
    shapes = []
    for k in range(batch):
        r = rng_for(seed, k)
        n = int(r.integers(nmin, nmax + 1))
        m = int(r.integers(n, 2 * n + 1))
        shapes.append((m, n, k))
    by = {}
    for m, n, k in shapes:
        by.setdefault((m, n), []).append(k)
    keys = sorted(by.items())
    offs, total = [], 0
    for (m, n), ks in keys:
        offs.append(total)
        total += m * n * len(ks)
    global _SHARED
    if workers and workers > 1:
        # workers fill one anonymous shared mapping, created before they fork
        import mmap
        _SHARED = mmap.mmap(-1, max(total, 1) * 16)
        tasks = [(seed, [(kk, offs[i]) for i, kk in enumerate(keys)][a:b])
                 for a, b in _ranges(len(keys), 4 * workers)]
        _pool_map(_uneven_fill, tasks, workers)
        flat = np.frombuffer(_SHARED, dtype=np.complex128, count=total).copy()
        _SHARED.close()
        _SHARED = None
    else:
        flat = np.empty(total, np.complex128)
        for ((m, n), ks), o in zip(keys, offs):
            flat[o:o + m * n * len(ks)] = np.stack(
                [gaussian(rng_for(seed + 1, k), m, n, True) for k in ks]).ravel()
    return [Group(m, n, flat[o:o + m * n * len(ks)].reshape(len(ks), m, n), ["cgauss"] * len(ks),
                  (seed, ks[0])) for ((m, n), ks), o in zip(keys, offs)]


_SHARED = None


def _ranges(count, parts):
    step = max(1, -(-count // max(parts, 1)))
    return [(a, min(a + step, count)) for a in range(0, count, step)]


def _uneven_fill(arg):
    seed, items = arg
    buf = np.frombuffer(_SHARED, dtype=np.complex128)
    with _one_thread():
        for ((m, n), ks), o in items:
            buf[o:o + m * n * len(ks)] = np.stack(
                [gaussian(rng_for(seed + 1, k), m, n, True) for k in ks]).ravel()
    return len(items)


SERVE_CLASSES = [(n * r, n) for n in (16, 32, 64, 128, 256, 512) for r in (1, 2)]


def serving_pool(per_class: int = 4, seed: int = BASE_SEED + 4000, max_n: int = 512) -> list:
    """Request pool of the serving workload: shape classes n in {16, ..., 512}
    x {square, m = 2n}, dtype alternating FP64 / FP32, kappa log-uniform in
    [1, 1e8] with a geometric spectrum.  Returns a list of (A, dtype name)
    with A in FP64 (cast on use)."""
    pool = []
    k = 0
    for m, n in SERVE_CLASSES:
        if n > max_n:
            continue
        for j in range(per_class):
            r = rng_for(seed, k)
            kappa = float(np.exp(r.uniform(0.0, np.log(1e8))))
            A = from_spectrum(r, m, n, spectrum("geo", n, kappa))
            pool.append((A, "f64" if k % 2 == 0 else "f32"))
            k += 1
    return pool
