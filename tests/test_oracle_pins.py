"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value is a closed
form, an exact (rational-arithmetic) brute force, a printed number of the
paper, an independent library routine, or an invariant of the method.  A
mutation test at the end plants plausible mistakes in a copy of the oracle
source and checks that these pins catch each of them.
"""
import ctypes
import decimal
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import ref as oref
from workloads import gen
from metrics import U64, orth_err, recon_err, sigma_err

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# helpers: exact references
# ---------------------------------------------------------------------------

def _rat_sym_eigs(M):
    """Eigenvalues of a small symmetric rational matrix by bisection on the
    inertia of M - x I (Sylvester's law), in exact rational arithmetic.
    Returns floats, descending."""
    n = len(M)

    def below(x):
        A = [[M[i][j] - (x if i == j else 0) for j in range(n)] for i in range(n)]
        neg = 0
        for k in range(n):
            p = A[k][k]
            if p == 0:
                return None
            if p < 0:
                neg += 1
            for i in range(k + 1, n):
                f = A[i][k] / p
                if f:
                    for j in range(k + 1, n):
                        A[i][j] -= f * A[k][j]
        return neg

    def count(x):
        c = below(x)
        d = Fraction(1, 2 ** 200)
        while c is None:
            x += d
            d *= 2
            c = below(x)
        return c

    hi = max(sum(abs(v) for v in row) for row in M) + 1
    eigs = []
    for k in range(n):                       # k-th smallest
        lo_, hi_ = Fraction(-1), Fraction(hi)
        for _ in range(90):
            mid = (lo_ + hi_) / 2
            if count(mid) > k:
                hi_ = mid
            else:
                lo_ = mid
        eigs.append(float((lo_ + hi_) / 2))
    return np.array(sorted(eigs, reverse=True))


def _gram_rational(A):
    F = [[Fraction(float(x)) for x in row] for row in np.asarray(A)]
    m, n = len(F), len(F[0])
    return [[sum(F[k][i] * F[k][j] for k in range(m)) for j in range(n)] for i in range(n)]


def _closed_two_column(A):
    """Singular values of an m x 2 matrix from the eigenvalues of its 2 x 2
    Gram matrix, sigma^2 = (a+b)/2 +- sqrt(((a-b)/2)^2 + |g|^2), evaluated
    with exact rationals and 60-digit decimals."""
    A = np.asarray(A)
    decimal.getcontext().prec = 60
    if np.iscomplexobj(A):
        re = [[Fraction(float(x.real)) for x in row] for row in A]
        im = [[Fraction(float(x.imag)) for x in row] for row in A]
        a = sum(re[k][0] ** 2 + im[k][0] ** 2 for k in range(len(re)))
        b = sum(re[k][1] ** 2 + im[k][1] ** 2 for k in range(len(re)))
        gr = sum(re[k][0] * re[k][1] + im[k][0] * im[k][1] for k in range(len(re)))
        gi = sum(re[k][0] * im[k][1] - im[k][0] * re[k][1] for k in range(len(re)))
        g2 = gr * gr + gi * gi
    else:
        G = _gram_rational(A)
        a, b, g2 = G[0][0], G[1][1], G[0][1] ** 2

    def dec(q):
        return decimal.Decimal(q.numerator) / decimal.Decimal(q.denominator)
    mean = dec((a + b) / 2)
    rad = dec(((a - b) / 2) ** 2 + g2).sqrt()
    return np.array([float((mean + rad).sqrt()), float(max(mean - rad, 0).sqrt())])


def _offnorm(W):
    G = W.conj().T @ W
    return float(np.linalg.norm(G - np.diag(np.diag(G))))


def _load_golden(name):
    secs, cur = {}, None
    for line in open(os.path.join(HERE, "golden", name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line[1:-1]
            secs[cur] = []
            continue
        secs[cur].append([float(x) for x in line.split()])
    return {k: np.array(v) for k, v in secs.items()}


# ---------------------------------------------------------------------------
# pins.  Each returns nothing and raises AssertionError on a violation, so the
# mutation test can reuse them.
# ---------------------------------------------------------------------------

def pin_round_robin_valid():
    """Round robin ("Algorithmic Background", "Parallel Ordering"): a sweep is l-1 iterations of l/2 disjoint pairs that
    together cover every pair exactly once."""
    for l in list(range(2, 40, 2)) + [64, 128, 256]:
        rr = oracle.round_robin(l)
        assert rr.shape == (l - 1, l // 2, 2)
        seen = set()
        for it in rr:
            idx = it.reshape(-1)
            assert len(set(idx.tolist())) == l, (l, it)
            for i, j in it:
                assert 0 <= i < j < l
                seen.add((int(i), int(j)))
        assert len(seen) == l * (l - 1) // 2


def pin_round_robin_worked_example():
    """Worked example ("Inexact Hermitian Eigendecomposition", "Motivation"):
    with four block columns the first iteration pairs blocks
    (1,2),(3,4) and the second (1,4),(2,3)."""
    rr = oracle.round_robin(4)
    assert sorted(map(tuple, rr[0].tolist())) == [(0, 1), (2, 3)]
    assert sorted(map(tuple, rr[1].tolist())) == [(0, 3), (1, 2)]


def pin_two_by_two_real():
    """2 x 2 real SVD closed form: with E=(a+d)/2, F=(a-d)/2, G=(c+b)/2,
    H=(c-b)/2, sigma = sqrt(E^2+H^2) +- sqrt(F^2+G^2)."""
    rng = gen.rng_for(11, 0)
    for _ in range(50):
        a, b, c, d = rng.standard_normal(4) * 10.0 ** rng.uniform(-3, 3)
        A = np.array([[a, b], [c, d]])
        E, F, G, H = (a + d) / 2, (a - d) / 2, (c + b) / 2, (c - b) / 2
        Q, R = np.hypot(E, H), np.hypot(F, G)
        ref = np.array([Q + R, abs(Q - R)])
        S, U, V, sw, info = oracle.gesvj(A)
        assert info == 0
        assert sigma_err(S, ref) <= 8 * U64, (A, S, ref)


def pin_sign_zero_convention():
    """Reading R2 (sign(0) = +1 in t_min of eq. sin-cos), on an exact case:
    A = [[3, 4], [4, 3]] has equal column norms (tau = 0), so t = +1 and
    c = s = 1/sqrt(2): the columns become (7, 7)/sqrt(2) and (1, -1)/sqrt(2),
    V = [[1, -1], [1, 1]]/sqrt(2), sigma = (7, 1)."""
    A = np.array([[3.0, 4.0], [4.0, 3.0]])
    S, U, V, sw, info = oracle.gesvj(A)
    r = 1.0 / np.sqrt(2.0)
    assert info == 0
    assert np.allclose(S, [7.0, 1.0], rtol=0, atol=4 * U64 * 7)
    assert np.allclose(U, [[r, r], [r, -r]], rtol=0, atol=4 * U64)
    assert np.allclose(V, [[r, -r], [r, r]], rtol=0, atol=4 * U64)


def pin_two_columns(complex_):
    """m x 2 (real and complex): one rotation diagonalises the 2 x 2 Gram
    matrix, so the singular values equal the closed-form eigenvalues of eq.
    (background-svd-jacobi), computed exactly here."""
    rng = gen.rng_for(12, int(complex_))
    for trial in range(30):
        m = int(rng.integers(2, 9))
        A = gen.gaussian(rng, m, 2, complex_)
        A[:, 1] *= 10.0 ** rng.uniform(-3, 3)
        ref = _closed_two_column(A)
        S, U, V, sw, info = oracle.gesvj(A)
        assert info == 0
        assert sigma_err(S, ref) <= 8 * U64, (trial, S, ref)
        assert np.abs(S[1] - ref[1]) <= 64 * U64 * ref[0]
        assert recon_err(A, S, U, V) <= 16 * U64
        assert orth_err(U) <= 16 * U64 and orth_err(V) <= 16 * U64


def pin_bruteforce_tiny():
    """n <= 4: sigma_i^2 equals the eigenvalues of A^T A found by exact
    rational bisection."""
    rng = gen.rng_for(13, 0)
    for trial in range(12):
        n = int(rng.integers(1, 5))
        m = int(rng.integers(n, n + 3))
        A = gen.gaussian(rng, m, n)
        if trial % 3 == 0:
            A = A * np.logspace(0, -3, n)[None, :]
        lam = _rat_sym_eigs(_gram_rational(A))
        for order in (0, 1):
            S, U, V, sw, info = oracle.gesvj(A, order=order)
            assert info == 0
            assert np.abs(S ** 2 - lam).max() <= 64 * U64 * lam[0], (trial, S ** 2, lam)


def pin_known_sigma(complex_):
    """A = U diag(s) V^H with Haar U, V: the computed singular values match s
    to a normwise error of a modest multiple of n u."""
    for k, (m, n, kind, kappa) in enumerate([(16, 16, "logu", 1e3), (24, 10, "geo", 1e6),
                                             (12, 12, "arith", 1e5), (9, 7, "cluster1", 1e4),
                                             (10, 10, "cluster0", 1e8)]):
        rng = gen.rng_for(14, 10 * k + int(complex_))
        s = gen.spectrum(kind, n, kappa, rng, lo=1e-3, hi=1.0)
        A = gen.from_spectrum(rng, m, n, s, complex_)
        for order in (0, 1):
            S, U, V, sw, info = oracle.gesvj(A, order=order)
            assert info == 0
            assert sigma_err(S, s) <= 4 * n * U64, (kind, sigma_err(S, s))
            assert recon_err(A, S, U, V) <= 8 * n * U64
            assert orth_err(U) <= 8 * n * U64 and orth_err(V) <= 8 * n * U64


def pin_sorted_and_scale_invariant():
    """Alg. 2 sorts sigma descending (T4), and the iteration is invariant under
    scaling by a power of two (the test |g_ij| >= tol sqrt(g_ii) sqrt(g_jj) is
    homogeneous), so the sweep count and the scaled outputs are identical."""
    rng = gen.rng_for(15, 0)
    A = gen.gaussian(rng, 14, 9)
    S, U, V, sw, info = oracle.gesvj(A)
    assert np.all(np.diff(S) <= 0)
    for e in (-60, 40):
        S2, U2, V2, sw2, info2 = oracle.gesvj(A * 2.0 ** e)
        assert sw2 == sw and info2 == info
        assert np.array_equal(S2, S * 2.0 ** e)
        assert np.array_equal(U2, U) and np.array_equal(V2, V)


def pin_offnorm_decreases():
    """Eq. (block-off-norm): each rotation lowers off(W^H W)^2 by 2|g_ij|^2,
    so off(W^H W) decreases sweep by sweep; ||W||_F is preserved and
    W = A V throughout."""
    for complex_ in (False, True):
        rng = gen.rng_for(16, int(complex_))
        A = gen.gaussian(rng, 12, 8, complex_)
        prev = _offnorm(A)
        for k in range(1, 5):
            S, U, V, sw, info = oracle.gesvj(A, max_sweeps=k, order=1)
            W = U * S[None, :]
            off = _offnorm(W)
            assert off < prev, (k, off, prev)
            prev = off
            assert abs(np.linalg.norm(W) - np.linalg.norm(A)) <= 16 * U64 * np.linalg.norm(A)
            assert np.linalg.norm(A @ V - W) <= 64 * 8 * U64 * np.linalg.norm(A)
        assert info == 1 or prev < 1e-10


def pin_numpy_svd(complex_):
    """Cross-check with LAPACK's gesdd (numpy.linalg.svd)."""
    rng = gen.rng_for(17, int(complex_))
    for m, n in [(5, 3), (16, 16), (33, 17), (40, 40), (64, 8)]:
        A = gen.gaussian(rng, m, n, complex_)
        ref = np.linalg.svd(A, compute_uv=False)
        S, U, V, sw, info = oracle.gesvj(A)
        assert info == 0
        assert sigma_err(S, ref) <= 1e-14
        assert recon_err(A, S, U, V) <= 1e-13 * n


def pin_worked_example():
    """Worked example of "Inexact Hermitian Eigendecomposition", subsection
    "Motivation": block size 2 on the printed 8 x 8 matrix.
    With the inner eigensolver run to convergence in round-robin order and the
    eigenvectors left unsorted, the first two round-robin iterations reproduce
    the printed [A_1 A_2] and G_{1,2} (to the four printed decimals, allowing
    for the rounding of the printed input)."""
    g = _load_golden("worked_example_8x8.txt")
    W = np.asfortranarray(g["A"].astype(np.complex128))
    V = np.asfortranarray(np.eye(8, dtype=np.complex128))
    oracle.block_iter(W, V, 4, 2, 0, inner_sweeps=0)
    A1 = W[:, :4].real
    assert np.abs(A1 - g["A1"]).max() <= 2.5e-4
    assert np.abs(A1.T @ A1 - g["G1"]).max() <= 2.5e-4
    oracle.block_iter(W, V, 4, 2, 1, inner_sweeps=0)
    A2 = W[:, :4].real
    assert np.abs(A2 - g["A2"]).max() <= 2.5e-4
    assert np.abs(A2.T @ A2 - g["G2"]).max() <= 2.5e-4
    # V accumulates the same transformations: W = A V
    assert np.abs(g["A"] @ V.real - W.real).max() <= 1e-13


def pin_heevj():
    """Alg. 1: J^H G J is diagonal, J is unitary, and the diagonal holds the
    eigenvalues (exact rational bisection for a real symmetric G)."""
    rng = gen.rng_for(18, 0)
    X = gen.gaussian(rng, 6, 4)
    Gm = X.T @ X
    lam = _rat_sym_eigs([[Fraction(float(v)) for v in row] for row in Gm])
    Go, J, nrot, sw, cv = oracle.heevj(Gm)
    assert cv and nrot > 0
    assert np.abs(Go - np.diag(np.diag(Go))).max() <= 1e-14 * lam[0]
    assert orth_err(J) <= 1e-14
    assert np.abs(np.sort(np.diag(Go).real)[::-1] - lam).max() <= 1e-14 * lam[0]
    assert np.abs(J.conj().T @ Gm @ J - Go).max() <= 1e-13 * lam[0]
    Xc = gen.gaussian(rng, 7, 5, True)
    Gc = Xc.conj().T @ Xc
    Go, J, nrot, sw, cv = oracle.heevj(Gc)
    ref = np.linalg.eigvalsh(Gc)[::-1]
    assert cv and orth_err(J) <= 1e-14
    assert np.abs(np.sort(np.diag(Go).real)[::-1] - ref).max() <= 1e-13 * ref[0]
    assert np.abs(J.conj().T @ Gc @ J - Go).max() <= 1e-13 * ref[0]


def pin_block_matches_definition():
    """The blocked method (one inner sweep, Design 2) converges to the same
    SVD; padding columns never interfere (n not a multiple of nb)."""
    for complex_ in (False, True):
        rng = gen.rng_for(19, int(complex_))
        for m, n, nb in [(12, 12, 2), (20, 11, 3), (16, 16, 4), (30, 13, 8), (9, 5, 1)]:
            A = gen.gaussian(rng, m, n, complex_)
            ref = np.linalg.svd(A, compute_uv=False)
            for inner in (1, 0):
                S, U, V, sw, info = oracle.block_gesvj(A, nb, inner_sweeps=inner)
                assert info == 0
                assert sigma_err(S, ref) <= 1e-14, (m, n, nb, inner)
                assert recon_err(A, S, U, V) <= 1e-13 * n
                assert orth_err(U) <= 1e-13 * n and orth_err(V) <= 1e-13 * n


def pin_block_dynamic_tolerance():
    """The dynamic inner tolerance ("Inexact Hermitian Eigendecomposition",
    first way): with a start at or below tol it is the fixed-threshold block
    solver bit for bit; from a large start it reaches the same SVD, and it
    cannot stop before the threshold has shrunk to tol (a matrix with
    orthogonal columns converges in exactly that sweep)."""
    tol = oracle.default_tol(np.float64)
    t0, rate = 1e-1, 1e-2
    # sweeps until max(tol, t0 rate^s) = tol, plus the sweep at tol
    need = int(np.ceil(np.log(tol / t0) / np.log(rate))) + 1
    for complex_ in (False, True):
        rng = gen.rng_for(23, int(complex_))
        for m, n, nb in [(20, 11, 3), (16, 16, 4), (30, 13, 8), (24, 24, 2)]:
            A = gen.from_spectrum(rng, m, n, gen.spectrum("geo", n, 1e6), complex_)
            fixed = oracle.block_gesvj(A, nb, inner_sweeps=0)
            same = oracle.block_gesvj(A, nb, inner_sweeps=0, tol_start=tol, tol_rate=rate)
            for x, y in zip(fixed[:3], same[:3]):
                assert np.array_equal(x, y)
            S, U, V, sw, info = oracle.block_gesvj(A, nb, inner_sweeps=0, tol_start=t0,
                                                   tol_rate=rate)
            ref = np.linalg.svd(A, compute_uv=False)
            assert info == 0 and sw >= need, (m, n, nb, sw, need)
            assert sigma_err(S, ref) <= 1e-14, (m, n, nb)
            assert recon_err(A, S, U, V) <= 1e-13 * n
            assert orth_err(U) <= 1e-13 * n and orth_err(V) <= 1e-13 * n
        D = np.diag(np.arange(1.0, 9.0))[:, ::-1] * (1 + 1j if complex_ else 1)
        S, U, V, sw, info = oracle.block_gesvj(D, 2, inner_sweeps=0, tol_start=t0,
                                               tol_rate=rate)
        assert info == 0 and sw == need and np.allclose(S, np.abs(np.diag(D[:, ::-1]))[::-1])


def pin_rank_deficient():
    """sigma = 0: U is completed to orthonormal columns; zero matrices and
    exact rank-1 matrices."""
    for complex_ in (False, True):
        rng = gen.rng_for(20, int(complex_))
        Z = np.zeros((6, 4), dtype=np.complex128 if complex_ else np.float64)
        S, U, V, sw, info = oracle.gesvj(Z)
        assert info == 0 and sw == 1 and np.all(S == 0)
        assert orth_err(U) <= 1e-15 and orth_err(V) <= 1e-15
        x = gen.gaussian(rng, 7, 1, complex_)
        y = gen.gaussian(rng, 1, 5, complex_)
        y[0, 2] = 0                      # an exactly zero column as well
        A = x @ y
        S, U, V, sw, info = oracle.gesvj(A)
        assert info == 0
        assert abs(S[0] - np.linalg.norm(x) * np.linalg.norm(y)) <= 1e-14 * S[0]
        assert np.all(S[1:] <= 1e-15 * S[0])
        assert orth_err(U) <= 1e-13 and orth_err(V) <= 1e-13
        assert recon_err(A, S, U, V) <= 1e-14


def pin_info_codes():
    """info = 1 when max_sweeps runs out, 2 on non-finite input."""
    rng = gen.rng_for(21, 0)
    A = gen.gaussian(rng, 16, 16)
    S, U, V, sw, info = oracle.gesvj(A, max_sweeps=1)
    assert info == 1 and sw == 1
    A[3, 4] = np.nan
    S, U, V, sw, info = oracle.gesvj(A)
    assert info == 2
    A[3, 4] = np.inf
    assert oracle.gesvj(A)[4] == 2


def pin_batch_driver():
    """The OpenMP batch driver returns exactly the per-matrix results."""
    groups = gen.small16(batch=6)
    A = groups[0].A
    Sb, Ub, Vb, swb, infob = oracle.gesvj_batch(A, tol=1e-14)
    for b in range(A.shape[0]):
        S, U, V, sw, info = oracle.gesvj(A[b], tol=1e-14)
        assert np.array_equal(S, Sb[b]) and np.array_equal(U, Ub[b]) and np.array_equal(V, Vb[b])
        assert sw == swb[b] and info == infob[b]


def pin_precond():
    """The preconditioned driver (QR with or without column pivoting, second
    QR, Alg. 2 on R2^T) returns an SVD of A itself: sigma as LAPACK's,
    U S V^T = A, orthonormal factors, with columns of A given in scrambled
    scale so that the pivot order is not the identity; on graded matrices it
    needs fewer sweeps than Alg. 2 on A; on a scrambled diagonal matrix R2^T
    is diagonal, so one sweep with no rotation suffices and V is a signed
    permutation."""
    for pivot in (True, False):
        rng = gen.rng_for(22, 0)
        for m, n in [(64, 64), (128, 32), (17, 9), (5, 1)]:
            for kind in ("gauss", "geo"):
                A = gen.family(rng, kind, m, n, 1e10)
                A = A[:, rng.permutation(n)] * (2.0 ** rng.integers(-20, 20, n))
                S, U, V, sw, info = oracle.precond_gesvj(A, pivot=pivot)
                ref = np.linalg.svd(A, compute_uv=False)
                assert info == 0
                assert sigma_err(S, ref) <= 1e-14, (m, n, kind, pivot)
                assert recon_err(A, S, U, V) <= 1e-13 * n
                assert orth_err(U) <= 1e-13 * n and orth_err(V) <= 1e-13 * n
                if kind == "geo" and n >= 32:
                    assert sw < oracle.gesvj(A)[3]
        d = np.array([3.0, -7.0, 0.5, 11.0, 2.0])
        A = np.zeros((7, 5))
        A[:5, :5] = np.diag(d)
        S, U, V, sw, info = oracle.precond_gesvj(A, pivot=pivot)
        assert info == 0 and sw == 1
        assert np.array_equal(S, np.sort(np.abs(d))[::-1])
        assert np.array_equal(np.abs(V), np.abs(V).round()) and np.allclose(np.abs(V).sum(0), 1)
        assert recon_err(A, S, U, V) <= 1e-15
        A[2, 3] = np.nan
        assert oracle.precond_gesvj(A, pivot=pivot)[4] == 2


PINS = {
    "round_robin_valid": pin_round_robin_valid,
    "round_robin_worked_example": pin_round_robin_worked_example,
    "two_by_two_real": pin_two_by_two_real,
    "sign_zero_convention": pin_sign_zero_convention,
    "two_columns_real": lambda: pin_two_columns(False),
    "two_columns_complex": lambda: pin_two_columns(True),
    "bruteforce_tiny": pin_bruteforce_tiny,
    "known_sigma_real": lambda: pin_known_sigma(False),
    "known_sigma_complex": lambda: pin_known_sigma(True),
    "sorted_and_scale_invariant": pin_sorted_and_scale_invariant,
    "offnorm_decreases": pin_offnorm_decreases,
    "numpy_svd_real": lambda: pin_numpy_svd(False),
    "numpy_svd_complex": lambda: pin_numpy_svd(True),
    "worked_example": pin_worked_example,
    "heevj": pin_heevj,
    "block_matches_definition": pin_block_matches_definition,
    "block_dynamic_tolerance": pin_block_dynamic_tolerance,
    "rank_deficient": pin_rank_deficient,
    "info_codes": pin_info_codes,
    "batch_driver": pin_batch_driver,
    "precond": pin_precond,
}


@pytest.mark.parametrize("name", sorted(PINS))
def test_pin(name):
    PINS[name]()


def test_worked_example_needs_converged_inner_solve():
    """The printed example diagonalises G^(1) exactly, i.e. it shows inner
    solves run to convergence; one inner sweep (Design 2) leaves the block
    columns visibly different from the print."""
    g = _load_golden("worked_example_8x8.txt")
    W = np.asfortranarray(g["A"].astype(np.complex128))
    V = np.asfortranarray(np.eye(8, dtype=np.complex128))
    oracle.block_iter(W, V, 4, 2, 0, inner_sweeps=1)
    assert np.abs(W[:, :4].real - g["A1"]).max() > 0.1


# ---------------------------------------------------------------------------
# mutation test: plausible mistakes planted in a copy of the oracle source
# must each break at least one pin.
# ---------------------------------------------------------------------------

MUTATIONS = [
    ("rotation sign (real)", "wj[k] = -e * s * x + c * y;", "wj[k] = e * s * x + c * y;"),
    ("dropped conj (complex update)", "wi[k] = c * x + conj(e) * s * y;\n                wj[k] = -e * s * x + c * y;\n            }\n            zc *vi",
     "wi[k] = c * x + e * s * y;\n                wj[k] = -e * s * x + c * y;\n            }\n            zc *vi"),
    ("transposed Gram entry (complex)", "gij += conj(wi[k]) * wj[k];", "gij += wi[k] * conj(wj[k]);"),
    ("tau sign", "double tau = (gii - gjj) / (2.0 * agij);", "double tau = (gjj - gii) / (2.0 * agij);"),
    ("wrong Gram index", "gjj += wj[k] * wj[k];", "gjj += wi[k] * wj[k];"),
    ("missing V update (real)", "vi[k] = c * x + e * s * y;", "vi[k] = x;"),
    ("threshold not homogeneous", "fabs(gij) < tol * sqrt(gii) * sqrt(gjj)", "fabs(gij) < tol * gii * gjj"),
    ("ascending sort", "sig[perm[j]] < sig[p]) { perm[j + 1] = perm[j]; j--; }\n        perm[j + 1] = p;\n    }\n    for (int r = 0; r < n; r++) {\n        int i = perm[r];\n        if (S) S[r] = sig[i];\n        if (U) for (int k = 0; k < m; k++) U[(size_t)r * ldu + k] = Uw[(size_t)i * m + k];\n        if (V) for (int k = 0; k < n; k++) V[(size_t)r * ldv + k] = Vw[(size_t)i * n + k];\n    }\n    free(sig); free(Uw); free(perm);\n}\n\nstatic void finalize_z",
     "sig[perm[j]] > sig[p]) { perm[j + 1] = perm[j]; j--; }\n        perm[j + 1] = p;\n    }\n    for (int r = 0; r < n; r++) {\n        int i = perm[r];\n        if (S) S[r] = sig[i];\n        if (U) for (int k = 0; k < m; k++) U[(size_t)r * ldu + k] = Uw[(size_t)i * m + k];\n        if (V) for (int k = 0; k < n; k++) V[(size_t)r * ldv + k] = Vw[(size_t)i * n + k];\n    }\n    free(sig); free(Uw); free(perm);\n}\n\nstatic void finalize_z"),
    ("round robin seat shift", "nt[1] = bot[0];", "nt[1] = bot[1];"),
    ("two-sided row update", "G[(size_t)k * n + j] = -conj(e) * s * x + c * y;", "G[(size_t)k * n + j] = -e * s * x + c * y;"),
    ("block update uses J^T", "acc += X[(size_t)col[a] * rows + k] * J[(size_t)b * n2 + a];",
     "acc += X[(size_t)col[a] * rows + k] * J[(size_t)a * n2 + b];"),
    ("sign(0) = -1", "double sg = (tau >= 0.0) ? 1.0 : -1.0;", "double sg = (tau > 0.0) ? 1.0 : -1.0;"),
    ("dynamic tolerance stops above tol", "converged = (nrot == 0 && ts <= tol);",
     "converged = (nrot == 0);"),
    ("dynamic tolerance never shrinks", "ts = ts * tol_rate > tol ? ts * tol_rate : tol;",
     "ts = ts > tol ? ts : tol;"),
]


def _compile_mutant(src, tmpdir, tag):
    path = os.path.join(tmpdir, f"mut_{tag}.c")
    with open(path, "w") as f:
        f.write(src)
    so = os.path.join(tmpdir, f"mut_{tag}.so")
    subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-o", so,
                           path, "-lm"])
    return so


@pytest.mark.parametrize("k", range(len(MUTATIONS)))
def test_pins_catch_planted_mistake(k):
    name, old, new = MUTATIONS[k]
    src = open(oref._SRC).read()
    assert src.count(old) >= 1, f"mutation anchor missing: {name}"
    mutated = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as td:
        so = _compile_mutant(mutated, td, k)
        L = oref.load(so)
        failed = []
        oref.use_library(L)
        try:
            for pname, fn in PINS.items():
                try:
                    fn()
                except (AssertionError, ValueError, FloatingPointError):
                    failed.append(pname)
        finally:
            oref.use_library(None)
    assert failed, f"no pin caught the planted mistake: {name}"
