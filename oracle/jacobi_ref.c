/*
 * jacobi_ref.c -- CPU oracle for the batched one-sided Jacobi SVD.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU library never links, includes or calls anything from here, and this file
 * includes nothing from the GPU library.
 *
 * Paper: A. Abdelfattah and M. Fasi, "An Efficient Batch Solver for the
 * Singular Value Decomposition on GPUs" (arXiv 2601.17979).
 *
 * Everything runs in FP64 (double) or complex128 (double complex), whatever
 * the precision of the caller's data; the caller up-casts FP32 inputs.
 *
 * Functions and the passages they follow:
 *   oracle_round_robin    "Algorithmic Background" (parallel orderings, Brent-Luk round robin,
 *                         Fig. "rr"; pinned by the worked example of "Inexact Hermitian
 *                         Eigendecomposition", subsection "Motivation")
 *   oracle_row_cyclic     "Algorithmic Background" (row-cyclic ordering, Forsythe-Henrici)
 *   oracle_gesvj_d/_z     Alg. 2 (unblocked one-sided Jacobi SVD) with the
 *                         rotation of eq. (sin-cos) in its 2x2 form,
 *                         eq. (background-svd-jacobi)
 *   oracle_heevj_z        Alg. 1 (two-sided Jacobi Hermitian eigensolver)
 *   oracle_block_iter_z   "Algorithmic Background" block method, eqs. (block-gram), (right-sv);
 *                         "Initial Design" steps S1-S5; "Inexact Hermitian Eigendecomposition" inner solve
 *   oracle_block_gesvj_z  the blocked solver built from the above
 *
 * Readings of the paper taken here (each is also listed in the design notes):
 *   R1  complex rotation: the 2x2 form of eq. (background-eigenproblem-jacobi)
 *       with phi = arg(g_ij), g_ij = a_i^H a_j.  Columns update as
 *       a_i <- c a_i + conj(e) s a_j,  a_j <- -e s a_i + c a_j,  e = g_ij/|g_ij|.
 *       (The embedded form eq. (jacobi-rotation) carries a conjugation typo.)
 *   R2  sign(0) = +1 in t_min.
 *   R3  a pair is rotated iff g_ij != 0 and |g_ij| >= tol*sqrt(g_ii)*sqrt(g_jj);
 *       zero (padding) columns never rotate.
 *   R4  tol is the cosine threshold k*u itself.
 *   R5  sigma_i = 0 -> u_i completes U by Gram-Schmidt of e_1, e_2, ...
 *   R6  stable sort by sigma, descending; no sign/phase normalisation.
 *   R7  info: 0 converged, 1 not converged within max_sweeps, 2 non-finite
 *       input (outputs then untouched).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zc;

/* ------------------------------------------------------------------ */
/* Orderings                                                           */
/* ------------------------------------------------------------------ */

/* Brent-Luk round robin on an even number l of indices.  The schedule is a
 * tournament table of two rows, top = [0,2,4,...], bot = [1,3,5,...]; an
 * iteration plays the l/2 games (top[q], bot[q]).  Between iterations every
 * player except top[0] moves one seat around the table: bot[0] goes to
 * top[1], top[q] to top[q+1], the last top seat to the last bottom seat, and
 * bot[q] to bot[q-1].  Writes (l-1) iterations of l/2 pairs (smaller index
 * first) into pairs[2*((l-1)*(l/2))].  Returns 0, or -1 if l is odd or < 2. */
int oracle_round_robin(int l, int *pairs)
{
    if (l < 2 || (l & 1)) return -1;
    int k = l / 2;
    int *top = malloc(sizeof(int) * k), *bot = malloc(sizeof(int) * k);
    int *nt = malloc(sizeof(int) * k), *nbt = malloc(sizeof(int) * k);
    for (int q = 0; q < k; q++) { top[q] = 2 * q; bot[q] = 2 * q + 1; }
    int w = 0;
    for (int it = 0; it < l - 1; it++) {
        for (int q = 0; q < k; q++) {
            int a = top[q], b = bot[q];
            pairs[w++] = a < b ? a : b;
            pairs[w++] = a < b ? b : a;
        }
        if (k == 1) continue;
        nt[0] = top[0];
        nt[1] = bot[0];
        for (int q = 2; q < k; q++) nt[q] = top[q - 1];
        for (int q = 0; q < k - 1; q++) nbt[q] = bot[q + 1];
        nbt[k - 1] = top[k - 1];
        memcpy(top, nt, sizeof(int) * k);
        memcpy(bot, nbt, sizeof(int) * k);
    }
    free(top); free(bot); free(nt); free(nbt);
    return 0;
}

/* Row-cyclic ordering: (0,1),(0,2),...,(0,n-1),(1,2),...  Writes n(n-1)/2
 * pairs. */
void oracle_row_cyclic(int n, int *pairs)
{
    int w = 0;
    for (int i = 0; i < n - 1; i++)
        for (int j = i + 1; j < n; j++) { pairs[w++] = i; pairs[w++] = j; }
}

/* Builds the pair list of one sweep for `order` (0 row-cyclic, 1 round robin).
 * For round robin an odd n is padded with one phantom index n that never
 * rotates.  Returns the number of pairs written (caller frees *out). */
static int sweep_pairs(int n, int order, int **out)
{
    if (order == 1) {
        int l = n + (n & 1);
        int np = (l - 1) * (l / 2);
        int *p = malloc(sizeof(int) * 2 * (np > 0 ? np : 1));
        if (l >= 2) oracle_round_robin(l, p);
        *out = p;
        return l >= 2 ? np : 0;
    }
    int np = n * (n - 1) / 2;
    int *p = malloc(sizeof(int) * 2 * (np > 0 ? np : 1));
    oracle_row_cyclic(n, p);
    *out = p;
    return np;
}

/* ------------------------------------------------------------------ */
/* Rotation (eq. sin-cos), shared by the one- and two-sided solvers    */
/* ------------------------------------------------------------------ */

/* Given the real diagonal entries gii, gjj and |gij| > 0, returns c and s of
 * eq. (sin-cos): tau = (gii - gjj)/(2|gij|), t = sign(tau)/(|tau| +
 * sqrt(1+tau^2)), c = 1/sqrt(1+t^2), s = t c.  hypot keeps 1+tau^2 from
 * overflowing. */
static void jacobi_cs(double gii, double gjj, double agij, double *c, double *s)
{
    double tau = (gii - gjj) / (2.0 * agij);
    double sg = (tau >= 0.0) ? 1.0 : -1.0;          /* R2 */
    double t = sg / (fabs(tau) + hypot(1.0, tau));
    *c = 1.0 / hypot(1.0, t);
    *s = t * (*c);
}

/* 2-norm of a vector with scaling, so that neither overflow nor underflow
 * spoils it. */
static double nrm2_d(int m, const double *x)
{
    double scale = 0.0;
    for (int k = 0; k < m; k++) if (fabs(x[k]) > scale) scale = fabs(x[k]);
    if (scale == 0.0) return 0.0;
    double ss = 0.0;
    for (int k = 0; k < m; k++) { double y = x[k] / scale; ss += y * y; }
    return scale * sqrt(ss);
}

static double nrm2_z(int m, const zc *x)
{
    double scale = 0.0;
    for (int k = 0; k < m; k++) {
        if (fabs(creal(x[k])) > scale) scale = fabs(creal(x[k]));
        if (fabs(cimag(x[k])) > scale) scale = fabs(cimag(x[k]));
    }
    if (scale == 0.0) return 0.0;
    double ss = 0.0;
    for (int k = 0; k < m; k++) {
        double yr = creal(x[k]) / scale, yi = cimag(x[k]) / scale;
        ss += yr * yr + yi * yi;
    }
    return scale * sqrt(ss);
}

/* ------------------------------------------------------------------ */
/* Finalisation (Alg. 2, last two steps)                               */
/* ------------------------------------------------------------------ */

/* sigma_i = ||w_i||, u_i = w_i / sigma_i; sigma_i = 0 -> Gram-Schmidt
 * completion (R5); then a stable descending sort that permutes U and V (R6).
 * W is m x n (ldw = m), Vw is n x n (ldv = n), both column major.  Writes S[n],
 * U (m x n, ldu), V (n x n, ldv) when the pointers are non-NULL. */
static void finalize_d(int m, int n, const double *W, const double *Vw,
                       double *S, double *U, int ldu, double *V, int ldv)
{
    double *sig = malloc(sizeof(double) * (n ? n : 1));
    double *Uw = malloc(sizeof(double) * (size_t)m * (n ? n : 1));
    int *perm = malloc(sizeof(int) * (n ? n : 1));
    for (int i = 0; i < n; i++) {
        sig[i] = nrm2_d(m, W + (size_t)i * m);
        for (int k = 0; k < m; k++)
            Uw[(size_t)i * m + k] = sig[i] > 0.0 ? W[(size_t)i * m + k] / sig[i] : 0.0;
    }
    /* completion of the columns that belong to sigma = 0 */
    int cand = 0;
    for (int i = 0; i < n; i++) {
        if (sig[i] > 0.0) continue;
        double *u = Uw + (size_t)i * m;
        for (; cand < m; cand++) {
            for (int k = 0; k < m; k++) u[k] = (k == cand) ? 1.0 : 0.0;
            for (int pass = 0; pass < 2; pass++)
                for (int j = 0; j < n; j++) {
                    if (j == i || (sig[j] == 0.0 && j > i)) continue;
                    const double *q = Uw + (size_t)j * m;
                    double d = 0.0;
                    for (int k = 0; k < m; k++) d += q[k] * u[k];
                    for (int k = 0; k < m; k++) u[k] -= d * q[k];
                }
            double nu = nrm2_d(m, u);
            if (nu > 0.5) {
                for (int k = 0; k < m; k++) u[k] /= nu;
                cand++;
                break;
            }
        }
    }
    /* stable insertion sort of indices by sigma, descending */
    for (int i = 0; i < n; i++) perm[i] = i;
    for (int i = 1; i < n; i++) {
        int p = perm[i], j = i - 1;
        while (j >= 0 && sig[perm[j]] < sig[p]) { perm[j + 1] = perm[j]; j--; }
        perm[j + 1] = p;
    }
    for (int r = 0; r < n; r++) {
        int i = perm[r];
        if (S) S[r] = sig[i];
        if (U) for (int k = 0; k < m; k++) U[(size_t)r * ldu + k] = Uw[(size_t)i * m + k];
        if (V) for (int k = 0; k < n; k++) V[(size_t)r * ldv + k] = Vw[(size_t)i * n + k];
    }
    free(sig); free(Uw); free(perm);
}

static void finalize_z(int m, int n, const zc *W, const zc *Vw,
                       double *S, zc *U, int ldu, zc *V, int ldv)
{
    double *sig = malloc(sizeof(double) * (n ? n : 1));
    zc *Uw = malloc(sizeof(zc) * (size_t)m * (n ? n : 1));
    int *perm = malloc(sizeof(int) * (n ? n : 1));
    for (int i = 0; i < n; i++) {
        sig[i] = nrm2_z(m, W + (size_t)i * m);
        for (int k = 0; k < m; k++)
            Uw[(size_t)i * m + k] = sig[i] > 0.0 ? W[(size_t)i * m + k] / sig[i] : 0.0;
    }
    int cand = 0;
    for (int i = 0; i < n; i++) {
        if (sig[i] > 0.0) continue;
        zc *u = Uw + (size_t)i * m;
        for (; cand < m; cand++) {
            for (int k = 0; k < m; k++) u[k] = (k == cand) ? 1.0 : 0.0;
            for (int pass = 0; pass < 2; pass++)
                for (int j = 0; j < n; j++) {
                    if (j == i || (sig[j] == 0.0 && j > i)) continue;
                    const zc *q = Uw + (size_t)j * m;
                    zc d = 0.0;
                    for (int k = 0; k < m; k++) d += conj(q[k]) * u[k];
                    for (int k = 0; k < m; k++) u[k] -= d * q[k];
                }
            double nu = nrm2_z(m, u);
            if (nu > 0.5) {
                for (int k = 0; k < m; k++) u[k] /= nu;
                cand++;
                break;
            }
        }
    }
    for (int i = 0; i < n; i++) perm[i] = i;
    for (int i = 1; i < n; i++) {
        int p = perm[i], j = i - 1;
        while (j >= 0 && sig[perm[j]] < sig[p]) { perm[j + 1] = perm[j]; j--; }
        perm[j + 1] = p;
    }
    for (int r = 0; r < n; r++) {
        int i = perm[r];
        if (S) S[r] = sig[i];
        if (U) for (int k = 0; k < m; k++) U[(size_t)r * ldu + k] = Uw[(size_t)i * m + k];
        if (V) for (int k = 0; k < n; k++) V[(size_t)r * ldv + k] = Vw[(size_t)i * n + k];
    }
    free(sig); free(Uw); free(perm);
}

/* ------------------------------------------------------------------ */
/* Alg. 2: unblocked one-sided Jacobi SVD                              */
/* ------------------------------------------------------------------ */

/*
 * Real FP64.  A is m x n column major (lda >= m), m >= n >= 0, read only.
 * tol: rotation threshold (k*u); max_sweeps >= 1; order: 0 row-cyclic,
 * 1 round robin (the order of the paper's parallel solver).
 * Outputs (any may be NULL): S[n] descending, U m x n (ldu), V n x n (ldv),
 * *sweeps_out = sweeps executed.  Returns info (R7).
 */
int oracle_gesvj_d(int m, int n, const double *A, int lda, double tol,
                   int max_sweeps, int order, double *S, double *U, int ldu,
                   double *V, int ldv, int *sweeps_out)
{
    if (sweeps_out) *sweeps_out = 0;
    for (int j = 0; j < n; j++)
        for (int k = 0; k < m; k++)
            if (!isfinite(A[(size_t)j * lda + k])) return 2;
    double *W = malloc(sizeof(double) * (size_t)m * (n ? n : 1));
    double *Vw = calloc((size_t)n * n + 1, sizeof(double));
    for (int j = 0; j < n; j++)
        for (int k = 0; k < m; k++) W[(size_t)j * m + k] = A[(size_t)j * lda + k];
    for (int j = 0; j < n; j++) Vw[(size_t)j * n + j] = 1.0;       /* V <- I */

    int *pairs;
    int np = sweep_pairs(n, order, &pairs);
    int converged = 0, sweeps = 0;
    while (!converged && sweeps < max_sweeps) {
        converged = 1;
        sweeps++;
        for (int p = 0; p < np; p++) {
            int i = pairs[2 * p], j = pairs[2 * p + 1];
            if (j >= n) continue;                      /* phantom index */
            double *wi = W + (size_t)i * m, *wj = W + (size_t)j * m;
            double gii = 0.0, gjj = 0.0, gij = 0.0;     /* Gram entries */
            for (int k = 0; k < m; k++) {
                gii += wi[k] * wi[k];
                gjj += wj[k] * wj[k];
                gij += wi[k] * wj[k];
            }
            if (gij == 0.0 || fabs(gij) < tol * sqrt(gii) * sqrt(gjj)) continue;
            converged = 0;
            double c, s;
            jacobi_cs(gii, gjj, fabs(gij), &c, &s);
            double e = gij > 0.0 ? 1.0 : -1.0;          /* e^{i phi}, real */
            for (int k = 0; k < m; k++) {
                double x = wi[k], y = wj[k];
                wi[k] = c * x + e * s * y;
                wj[k] = -e * s * x + c * y;
            }
            double *vi = Vw + (size_t)i * n, *vj = Vw + (size_t)j * n;
            for (int k = 0; k < n; k++) {
                double x = vi[k], y = vj[k];
                vi[k] = c * x + e * s * y;
                vj[k] = -e * s * x + c * y;
            }
        }
    }
    finalize_d(m, n, W, Vw, S, U, ldu, V, ldv);
    if (sweeps_out) *sweeps_out = sweeps;
    free(pairs); free(W); free(Vw);
    return converged ? 0 : 1;
}

/* Complex128 version of oracle_gesvj_d; A, U, V hold interleaved (re, im)
 * pairs, S is real. */
int oracle_gesvj_z(int m, int n, const zc *A, int lda, double tol,
                   int max_sweeps, int order, double *S, zc *U, int ldu,
                   zc *V, int ldv, int *sweeps_out)
{
    if (sweeps_out) *sweeps_out = 0;
    for (int j = 0; j < n; j++)
        for (int k = 0; k < m; k++) {
            zc a = A[(size_t)j * lda + k];
            if (!isfinite(creal(a)) || !isfinite(cimag(a))) return 2;
        }
    zc *W = malloc(sizeof(zc) * (size_t)m * (n ? n : 1));
    zc *Vw = calloc((size_t)n * n + 1, sizeof(zc));
    for (int j = 0; j < n; j++)
        for (int k = 0; k < m; k++) W[(size_t)j * m + k] = A[(size_t)j * lda + k];
    for (int j = 0; j < n; j++) Vw[(size_t)j * n + j] = 1.0;

    int *pairs;
    int np = sweep_pairs(n, order, &pairs);
    int converged = 0, sweeps = 0;
    while (!converged && sweeps < max_sweeps) {
        converged = 1;
        sweeps++;
        for (int p = 0; p < np; p++) {
            int i = pairs[2 * p], j = pairs[2 * p + 1];
            if (j >= n) continue;
            zc *wi = W + (size_t)i * m, *wj = W + (size_t)j * m;
            double gii = 0.0, gjj = 0.0;
            zc gij = 0.0;                                /* a_i^H a_j */
            for (int k = 0; k < m; k++) {
                gii += creal(conj(wi[k]) * wi[k]);
                gjj += creal(conj(wj[k]) * wj[k]);
                gij += conj(wi[k]) * wj[k];
            }
            double ag = cabs(gij);
            if (ag == 0.0 || ag < tol * sqrt(gii) * sqrt(gjj)) continue;
            converged = 0;
            double c, s;
            jacobi_cs(gii, gjj, ag, &c, &s);
            zc e = gij / ag;                             /* e^{i phi} (R1) */
            for (int k = 0; k < m; k++) {
                zc x = wi[k], y = wj[k];
                wi[k] = c * x + conj(e) * s * y;
                wj[k] = -e * s * x + c * y;
            }
            zc *vi = Vw + (size_t)i * n, *vj = Vw + (size_t)j * n;
            for (int k = 0; k < n; k++) {
                zc x = vi[k], y = vj[k];
                vi[k] = c * x + conj(e) * s * y;
                vj[k] = -e * s * x + c * y;
            }
        }
    }
    finalize_z(m, n, W, Vw, S, U, ldu, V, ldv);
    if (sweeps_out) *sweeps_out = sweeps;
    free(pairs); free(W); free(Vw);
    return converged ? 0 : 1;
}

/* ------------------------------------------------------------------ */
/* Alg. 1: two-sided Jacobi Hermitian eigensolver                      */
/* ------------------------------------------------------------------ */

/*
 * G: n x n Hermitian (column major, ldg = n), overwritten by J^H G J.
 * J: n x n, set to the accumulated product of the rotations.
 * order: 0 row-cyclic, 1 round robin (the order used by the paper's batch
 * eigensolver, "Initial Design", subsection "Hermitian Eigenvalue Problem").  Runs at most
 * max_sweeps sweeps.  Returns the number of rotations applied; *sweeps_out
 * receives the sweeps executed and *conv_out whether the last sweep applied
 * no rotation.
 */
long oracle_heevj_z(int n, zc *G, zc *J, double tol, int max_sweeps, int order,
                    int *sweeps_out, int *conv_out)
{
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) J[(size_t)j * n + i] = (i == j) ? 1.0 : 0.0;
    int *pairs;
    int np = sweep_pairs(n, order, &pairs);
    long nrot = 0;
    int converged = 0, sweeps = 0;
    while (!converged && sweeps < max_sweeps) {
        converged = 1;
        sweeps++;
        for (int p = 0; p < np; p++) {
            int i = pairs[2 * p], j = pairs[2 * p + 1];
            if (j >= n) continue;
            double gii = creal(G[(size_t)i * n + i]), gjj = creal(G[(size_t)j * n + j]);
            zc gij = G[(size_t)j * n + i];               /* entry (i, j) */
            double ag = cabs(gij);
            /* Alg. 1 tests |a_ji| >= k u sqrt(a_ii a_jj); R3 */
            if (ag == 0.0 || ag < tol * sqrt(fabs(gii)) * sqrt(fabs(gjj))) continue;
            converged = 0;
            nrot++;
            double c, s;
            jacobi_cs(gii, gjj, ag, &c, &s);
            zc e = gij / ag;
            /* J2 = [[c, -e s], [conj(e) s, c]];  G <- G J2 (columns i, j) */
            for (int k = 0; k < n; k++) {
                zc x = G[(size_t)i * n + k], y = G[(size_t)j * n + k];
                G[(size_t)i * n + k] = c * x + conj(e) * s * y;
                G[(size_t)j * n + k] = -e * s * x + c * y;
            }
            /* G <- J2^H G (rows i, j) */
            for (int k = 0; k < n; k++) {
                zc x = G[(size_t)k * n + i], y = G[(size_t)k * n + j];
                G[(size_t)k * n + i] = c * x + e * s * y;
                G[(size_t)k * n + j] = -conj(e) * s * x + c * y;
            }
            /* J <- J J2 */
            for (int k = 0; k < n; k++) {
                zc x = J[(size_t)i * n + k], y = J[(size_t)j * n + k];
                J[(size_t)i * n + k] = c * x + conj(e) * s * y;
                J[(size_t)j * n + k] = -e * s * x + c * y;
            }
        }
    }
    free(pairs);
    if (sweeps_out) *sweeps_out = sweeps;
    if (conv_out) *conv_out = converged;
    return nrot;
}

/* ------------------------------------------------------------------ */
/* Block one-sided Jacobi ("Algorithmic Background", "Initial Design";  */
/* inexact inner solve: "Inexact Hermitian Eigendecomposition")          */
/* ------------------------------------------------------------------ */

/*
 * One round-robin iteration `iter` (0 <= iter < l-1) of the block method on
 * W (m x l*nb, ldw = m) and Vw (nv x l*nb, ldv = nv), l = number of block
 * columns (even).  For each block pair (p, q) of the iteration: form
 * G = [W_p W_q]^H [W_p W_q] (eq. block-gram), solve it with Alg. 1 in round
 * robin order for at most inner_sweeps sweeps (the paper's Design 2 uses
 * one; 0 means "to convergence", capped at 100), then post-multiply
 * [W_p W_q] and [V_p V_q] by the accumulated J (eq. right-sv).
 * Returns the number of inner rotations applied.
 */
long oracle_block_iter_z(int m, int nv, int l, int nb, zc *W, zc *Vw, int iter,
                         double tol, int inner_sweeps)
{
    int *pairs = malloc(sizeof(int) * 2 * (l - 1) * (l / 2));
    oracle_round_robin(l, pairs);
    int n2 = 2 * nb;
    zc *G = malloc(sizeof(zc) * n2 * n2), *J = malloc(sizeof(zc) * n2 * n2);
    zc *tmp = malloc(sizeof(zc) * (size_t)(m > nv ? m : nv) * n2);
    long nrot = 0;
    for (int q = 0; q < l / 2; q++) {
        int bp = pairs[2 * (iter * (l / 2) + q)], bq = pairs[2 * (iter * (l / 2) + q) + 1];
        /* column index of local column c in [W_p W_q] */
        int col[256];
        for (int c = 0; c < nb; c++) { col[c] = bp * nb + c; col[nb + c] = bq * nb + c; }
        for (int b = 0; b < n2; b++)
            for (int a = 0; a < n2; a++) {
                zc g = 0.0;
                for (int k = 0; k < m; k++)
                    g += conj(W[(size_t)col[a] * m + k]) * W[(size_t)col[b] * m + k];
                G[(size_t)b * n2 + a] = g;
            }
        nrot += oracle_heevj_z(n2, G, J, tol, inner_sweeps > 0 ? inner_sweeps : 100,
                               1, NULL, NULL);
        /* [W_p W_q] <- [W_p W_q] J and the same for V */
        for (int pass = 0; pass < 2; pass++) {
            zc *X = pass == 0 ? W : Vw;
            int rows = pass == 0 ? m : nv;
            for (int b = 0; b < n2; b++)
                for (int k = 0; k < rows; k++) {
                    zc acc = 0.0;
                    for (int a = 0; a < n2; a++)
                        acc += X[(size_t)col[a] * rows + k] * J[(size_t)b * n2 + a];
                    tmp[(size_t)b * rows + k] = acc;
                }
            for (int b = 0; b < n2; b++)
                for (int k = 0; k < rows; k++)
                    X[(size_t)col[b] * rows + k] = tmp[(size_t)b * rows + k];
        }
    }
    free(pairs); free(G); free(J); free(tmp);
    return nrot;
}

/*
 * Blocked one-sided Jacobi SVD (complex128; real data passes through with a
 * zero imaginary part).  nb is the block width (2*nb <= 256); A is padded
 * with zero columns to l*nb columns, l = ceil(n/nb) rounded up to even.  A
 * sweep is l-1 round-robin iterations; the solver has converged when a sweep
 * applies no inner rotation at all.  Outputs as oracle_gesvj_z.
 */
int oracle_block_gesvj_z(int m, int n, int nb, const zc *A, int lda, double tol,
                         int max_sweeps, int inner_sweeps, double *S, zc *U,
                         int ldu, zc *V, int ldv, int *sweeps_out)
{
    if (sweeps_out) *sweeps_out = 0;
    if (nb < 1 || 2 * nb > 256) return -1;
    for (int j = 0; j < n; j++)
        for (int k = 0; k < m; k++) {
            zc a = A[(size_t)j * lda + k];
            if (!isfinite(creal(a)) || !isfinite(cimag(a))) return 2;
        }
    int l = (n + nb - 1) / nb;
    if (l & 1) l++;
    if (l < 2) l = 2;
    int np = l * nb;                                 /* padded width */
    zc *W = calloc((size_t)m * np + 1, sizeof(zc));
    zc *Vw = calloc((size_t)np * np + 1, sizeof(zc));
    for (int j = 0; j < n; j++)
        for (int k = 0; k < m; k++) W[(size_t)j * m + k] = A[(size_t)j * lda + k];
    for (int j = 0; j < np; j++) Vw[(size_t)j * np + j] = 1.0;
    int converged = 0, sweeps = 0;
    while (!converged && sweeps < max_sweeps) {
        sweeps++;
        long nrot = 0;
        for (int it = 0; it < l - 1; it++)
            nrot += oracle_block_iter_z(m, np, l, nb, W, Vw, it, tol, inner_sweeps);
        converged = (nrot == 0);
    }
    /* the real columns of V: rows/cols 0..n-1 (padding never mixes in, R3) */
    zc *Vn = malloc(sizeof(zc) * (size_t)n * n + 1);
    for (int j = 0; j < n; j++)
        for (int k = 0; k < n; k++) Vn[(size_t)j * n + k] = Vw[(size_t)j * np + k];
    finalize_z(m, n, W, Vn, S, U, ldu, V, ldv);
    if (sweeps_out) *sweeps_out = sweeps;
    free(W); free(Vw); free(Vn);
    return converged ? 0 : 1;
}

/*
 * The block solver with the dynamic tolerance of the inner eigensolver
 * ("Inexact Hermitian Eigendecomposition", subsection "Motivation", first
 * way): outer sweep s (counted from 0) solves every Gram matrix with the
 * threshold t_s = max(tol, tol_start * tol_rate^s), starting large and
 * shrinking at a constant rate until it reaches tol.  A sweep without
 * rotation at a threshold above tol does not mean convergence; the solver
 * has converged when a sweep at t_s = tol applies no rotation.  With
 * tol_start <= tol this is oracle_block_gesvj_z.  Outputs as that.
 */
int oracle_block_gesvj_dyn_z(int m, int n, int nb, const zc *A, int lda, double tol,
                             int max_sweeps, int inner_sweeps, double tol_start,
                             double tol_rate, double *S, zc *U, int ldu, zc *V, int ldv,
                             int *sweeps_out)
{
    if (sweeps_out) *sweeps_out = 0;
    if (nb < 1 || 2 * nb > 256) return -1;
    if (!(tol_rate > 0.0 && tol_rate < 1.0) && tol_start > tol) return -1;
    for (int j = 0; j < n; j++)
        for (int k = 0; k < m; k++) {
            zc a = A[(size_t)j * lda + k];
            if (!isfinite(creal(a)) || !isfinite(cimag(a))) return 2;
        }
    int l = (n + nb - 1) / nb;
    if (l & 1) l++;
    if (l < 2) l = 2;
    int np = l * nb;
    zc *W = calloc((size_t)m * np + 1, sizeof(zc));
    zc *Vw = calloc((size_t)np * np + 1, sizeof(zc));
    for (int j = 0; j < n; j++)
        for (int k = 0; k < m; k++) W[(size_t)j * m + k] = A[(size_t)j * lda + k];
    for (int j = 0; j < np; j++) Vw[(size_t)j * np + j] = 1.0;
    int converged = 0, sweeps = 0;
    double ts = tol_start > tol ? tol_start : tol;
    while (!converged && sweeps < max_sweeps) {
        sweeps++;
        long nrot = 0;
        for (int it = 0; it < l - 1; it++)
            nrot += oracle_block_iter_z(m, np, l, nb, W, Vw, it, ts, inner_sweeps);
        converged = (nrot == 0 && ts <= tol);
        ts = ts * tol_rate > tol ? ts * tol_rate : tol;
    }
    zc *Vn = malloc(sizeof(zc) * (size_t)n * n + 1);
    for (int j = 0; j < n; j++)
        for (int k = 0; k < n; k++) Vn[(size_t)j * n + k] = Vw[(size_t)j * np + k];
    finalize_z(m, n, W, Vn, S, U, ldu, V, ldv);
    if (sweeps_out) *sweeps_out = sweeps;
    free(W); free(Vw); free(Vn);
    return converged ? 0 : 1;
}

/* ------------------------------------------------------------------ */
/* Batch drivers: OpenMP parallel for over the batch (the paper's CPU    */
/* baseline pattern, "Comparison with Existing Batch SVD Solvers"), one matrix per thread at a time.        */
/* ------------------------------------------------------------------ */

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Uniform-shape strided batch, real FP64.  Matrix b starts at A + b*sA etc.;
 * S, U, V, sweeps, info may be NULL (sweeps/info are int[batch]). */
void oracle_gesvj_strided_d(int batch, int m, int n, const double *A, int lda,
                            long sA, double tol, int max_sweeps, int order,
                            double *S, long sS, double *U, int ldu, long sU,
                            double *V, int ldv, long sV, int *sweeps, int *info)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < batch; b++) {
        int sw = 0;
        int inf = oracle_gesvj_d(m, n, A + (size_t)b * sA, lda, tol, max_sweeps, order,
                                 S ? S + (size_t)b * sS : NULL,
                                 U ? U + (size_t)b * sU : NULL, ldu,
                                 V ? V + (size_t)b * sV : NULL, ldv, &sw);
        if (sweeps) sweeps[b] = sw;
        if (info) info[b] = inf;
    }
}

void oracle_gesvj_strided_z(int batch, int m, int n, const zc *A, int lda,
                            long sA, double tol, int max_sweeps, int order,
                            double *S, long sS, zc *U, int ldu, long sU,
                            zc *V, int ldv, long sV, int *sweeps, int *info)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < batch; b++) {
        int sw = 0;
        int inf = oracle_gesvj_z(m, n, A + (size_t)b * sA, lda, tol, max_sweeps, order,
                                 S ? S + (size_t)b * sS : NULL,
                                 U ? U + (size_t)b * sU : NULL, ldu,
                                 V ? V + (size_t)b * sV : NULL, ldv, &sw);
        if (sweeps) sweeps[b] = sw;
        if (info) info[b] = inf;
    }
}
