/*
 * svdb.h -- C ABI of the MI355X batched one-sided Jacobi SVD library.
 *
 * Problem (section "Computing the Singular Value Decomposition", eq. svd): for each m x n matrix A of a batch,
 * compute the reduced SVD A = U diag(S) V^H with k = min(m, n): U is m x k
 * and V is n x k, both with orthonormal columns (V is unitary when m >= n),
 * S is real, non-negative and sorted in descending order (Alg. 2, last step;
 * accuracy check T4 of "Performance of the Baseline Implementation").  A
 * wide matrix (m < n) is solved through its conjugate transpose, A^H =
 * V S U^H (section "Pre-processing the SVD using a QR Factorization").
 * The method is the one-sided (Hestenes) Jacobi iteration of Alg. 2 with the
 * rotation of eq. (sin-cos), the round-robin parallel ordering (Fig. "rr"),
 * and, for wider matrices, the block method (eq. block-gram,
 * eq. right-sv) with a one-sweep inner eigensolver ("Inexact Hermitian
 * Eigendecomposition") and batch masks ("Masked Batch Operations").
 *
 * Conventions for every entry point:
 *  - Matrices are column major (LAPACK style) with a leading dimension.
 *  - All data pointers (A, S, U, V, info, workspace, opts->sweeps) are DEVICE
 *    pointers owned by the caller; the library allocates no device memory in
 *    these calls.  Host-side arrays (m[], n[], lda[], and the pointer arrays
 *    of svdb_svd_batched) are read during the call only.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream);
 *    outputs and info[] are valid after the stream is synchronised.  The
 *    resident and QR-preconditioned resident paths are fully asynchronous.
 *    The block method (BLOCKED path, the mixed-precision mode, the wide and
 *    tall preconditioned paths that end in it, and svdb_svd_batched) runs
 *    one launch per round-robin iteration; how its sweeps end is chosen by
 *    opts->persistent.  With 0 (default) the host waits for the count of
 *    unconverged matrices after every sweep, so the call returns only when
 *    its sweeps are done.  With 1, or when `stream` is being captured, the
 *    launches of all max_sweeps sweeps are queued and the count stays on
 *    the device: the call returns at once, nothing waits on the host, and
 *    svdb_svd_strided_batched can be captured into a HIP graph
 *    (svdb_svd_batched stages its descriptors through pinned host memory
 *    and is not meant for capture).
 *  - Return value: 0 on success; -k when argument k (1-based) is invalid,
 *    detected on the host before anything is launched; SVDB_ERR_UNSUPPORTED
 *    when a valid request is outside what this build implements;
 *    SVDB_ERR_HIP when the HIP runtime reports an error (the launch state of
 *    the batch is then undefined).  svdb_last_error() describes the last
 *    failure of the calling thread.
 *  - Per-matrix status info[b]: 0 converged; 1 not converged within
 *    max_sweeps (outputs hold the last iterate, finalised); 2 non-finite
 *    entry in A (outputs untouched).
 *  - `tol` is the rotation threshold k*u of Alg. 2: the pair (i, j) is
 *    rotated iff g_ij != 0 and |g_ij| >= tol * sqrt(g_ii) * sqrt(g_jj).
 *    tol <= 0 selects 30 u of the working precision (the paper's k = 30,
 *    "Performance of the Baseline Implementation", "Numerical Accuracy").
 */
#ifndef SVDB_H
#define SVDB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element types: the four LAPACK types of the paper (s, d, c, z). */
typedef enum {
    SVDB_R32 = 0,   /* float                       */
    SVDB_R64 = 1,   /* double                      */
    SVDB_C64 = 2,   /* float complex, (re, im)     */
    SVDB_C128 = 3   /* double complex, (re, im)    */
} svdb_dtype_t;

/* Execution paths.  AUTO chooses from the tuned plan table: RESIDENT where
 * an instance covers the shape (SVDB_R64), else BLOCKED.  PLAIN and
 * RESIDENT handle SVDB_R64 only; BLOCKED handles every dtype (complex with
 * nb = 16). */
typedef enum {
    SVDB_PATH_AUTO = 0,
    SVDB_PATH_PLAIN = 1,     /* LDS-resident unblocked kernel, one workgroup
                                per matrix (the plain GPU Jacobi)           */
    SVDB_PATH_RESIDENT = 2,  /* register-resident unblocked kernel (Alg. 2) */
    SVDB_PATH_BLOCKED = 3    /* block method (eq. block-gram) with MFMA Gram and
                                updates                                     */
} svdb_path_t;

#define SVDB_ERR_UNSUPPORTED (-200)
#define SVDB_ERR_HIP (-100)

typedef struct {
    int max_sweeps;   /* cap on sweeps (Alg. 2 max_nsweeps); <= 0 -> 100       */
    int path;         /* svdb_path_t                                          */
    int nb;           /* block width for SVDB_PATH_BLOCKED: 8, 16 or 32 (real), 16
                         (complex); 0 -> tuned                                */
    int masking;      /* blocked path: skip converged matrices ("Masked
                         Batch Operations");
                         < 0 -> default (on)                                   */
    int precision;    /* 0: sweeps in the working precision; 1: FP32 sweeps
                         then FP64 refinement (SVDB_R64, block method; the
                         sweeps count covers both phases)                      */
    int *sweeps;      /* optional DEVICE int[batch]: sweeps executed          */
    int waves;        /* SVDB_PATH_RESIDENT: wavefronts per matrix (1, 2, 4);
                         0 -> tuned                                           */
    int precondition; /* QR pre-processing of real matrices (section
                         "Other Performance Considerations"; FP32 input is
                         widened and runs the FP64 kernels with its own
                         threshold, then the results are narrowed).  n <= 64
                         and m <= 256 (m n <= 8192): A P = Q1 R1, R1^T =
                         Q2 R2, the resident kernel on R2^T, U = Q1 U_x.
                         For 32 < n <= 64 V = P R1^-1 U_x diag(S) by back
                         substitution, kept where the largest row sum of
                         |V^T V - I| is at most 2^-49 n (else the rotations
                         are accumulated), with column pivoting in the
                         first QR (the accuracy of that route needs it);
                         for n <= 32 V = Q2 J and P = I.  n <= 64 and larger
                         m (AUTO: m <= 1024; 1: m <= 4096): A = Q R, the
                         resident kernel on R^T, U = Q J.  n > 64 (m <=
                         1024): A = Q1 R1, R1^T = Q2 R2 (blocked QRs), the
                         block method on R2^T, U = Q1 U_x, V = Q2 J.
                         -1 (default): on for the AUTO path where it
                         applies, except FP64 with n <= 16 and m < 8 n
                         (there the QRs cost more than the sweeps they
                         save); 0: off; 1: on (AUTO, RESIDENT or BLOCKED
                         path; SVDB_ERR_UNSUPPORTED where it does not
                         apply); 2: as 1 with column pivoting in the first
                         QR at every n (Businger-Golub, as LAPACK's xGEQP3;
                         n <= 64 and m n <= 8192 only, SVDB_ERR_UNSUPPORTED
                         elsewhere and for the server).  The sweeps count is
                         that of the iteration on the triangular factor.  */
    int inner_sweeps; /* block method: sweeps of Alg. 1 per block-pair
                         solve ("Inexact Hermitian Eigendecomposition").  0
                         (default, tuned): one (Design 2) when the matrix
                         has more than two block columns; with two (l = 2)
                         two, or for m >= 8 np the converged solve (FP64)
                         or three (FP32); k > 0: at most k, stopping at a
                         sweep that rotates nothing; < 0: to convergence (at
                         most 100).                                          */
    int persistent;   /* block method, sweep control.  0 (default): after
                         every sweep the host waits for the count of
                         unconverged matrices and stops at zero.  Nonzero:
                         the launches of all max_sweeps sweeps are queued on
                         the stream and the count stays on the device; once
                         no matrix is left, every later launch returns at
                         once (a few microseconds each).  Same results, bit
                         for bit; the call returns before the work is done
                         and can be captured into a HIP graph.  Chosen
                         automatically when `stream` is capturing.        */
    double inner_tol_start; /* block method: the dynamic
                         tolerance of the inner eigensolver ("Inexact
                         Hermitian Eigendecomposition", subsection
                         "Motivation", first way).  > tol: outer sweep s
                         (from 0) solves the Gram matrices with threshold
                         max(tol, inner_tol_start * inner_tol_rate^s), and a
                         matrix converges only in a sweep run at tol itself;
                         <= 0 (default): tol in every sweep.               */
    double inner_tol_rate;  /* the shrink factor per outer sweep, in (0, 1)  */
} svdb_opts_t;

/* Fills *o with the defaults (AUTO path, 100 sweeps, masking on,
 * precondition -1, inner_sweeps 0, persistent 0, no dynamic inner
 * tolerance). */
void svdb_opts_default(svdb_opts_t *o);

/*
 * Bytes of device workspace the uniform-shape call needs for this request
 * (0 for the resident paths).  Arguments as svdb_svd_strided_batched; opts
 * may be NULL.  Returns (size_t)-1 on invalid arguments.
 */
size_t svdb_workspace_size(svdb_dtype_t dtype, int batch, int m, int n,
                           const svdb_opts_t *opts);

/*
 * Uniform-shape batch: matrix b of A starts at A + b*strideA elements (of
 * dtype), likewise S (real elements: float for R32/C64, double for
 * R64/C128), U and V.
 *
 *  A       in: batch x (m x n), lda >= max(1, m).  Not modified.
 *  S       out: k = min(m, n) singular values per matrix, descending.
 *  U       out: m x k left singular vectors (ldu >= m), or NULL.
 *  V       out: n x k right singular vectors (ldv >= n), A = U S V^H, or NULL.
 *  For m < n the call first writes A^H into the workspace (its size
 *  includes that copy) and runs the m >= n path on it with U and V
 *  exchanged; the path is the one svdb_plan gives for n x m.
 *  info    out: device int[batch] (see above).  Required.
 *  workspace / ws_bytes: device scratch of at least svdb_workspace_size()
 *          bytes (may be NULL when that is 0).
 *  Arguments, 1-based: dtype 1, batch 2, m 3, n 4, A 5, lda 6, strideA 7,
 *  S 8, strideS 9, U 10, ldu 11, strideU 12, V 13, ldv 14, strideV 15,
 *  tol 16, info 17, workspace 18, ws_bytes 19, opts 20, stream 21.
 */
int svdb_svd_strided_batched(svdb_dtype_t dtype, int batch, int m, int n,
                             const void *A, int lda, long long strideA,
                             void *S, long long strideS,
                             void *U, int ldu, long long strideU,
                             void *V, int ldv, long long strideV,
                             double tol, int *info,
                             void *workspace, size_t ws_bytes,
                             const svdb_opts_t *opts, void *stream);

/*
 * The uniform-shape call without any allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Arguments and results as
 * svdb_svd_strided_batched, without the workspace: the library's own
 * scratch, a static device array of svdb_noalloc_scratch_bytes() (64 MiB)
 * per device, held until the process ends, takes its place.  It neither
 * allocates nor frees anything (device or pinned host memory).
 *  - Only requests that AUTO (or the given path) plans on the resident
 *    kernels qualify: FP64 and FP32 with n <= 64, with or without the QR
 *    pre-processing, and wide matrices whose A^H qualifies (A^H is staged
 *    in the scratch).  A request planned on the block method returns
 *    SVDB_ERR_UNSUPPORTED (its host loop uses pinned memory).
 *  - A batch whose workspace (svdb_workspace_size) exceeds the scratch
 *    returns -2 and launches nothing.
 *  - Every call on a device shares that device's scratch, which keeps the
 *    last call's contents (no part of it needs to start at zero): calls
 *    that overlap on one device (other streams or host threads) race.
 * Arguments, 1-based: as svdb_svd_strided_batched up to info (17), then
 * opts 18, stream 19.
 */
int svdb_svd_strided_batched_noalloc(svdb_dtype_t dtype, int batch, int m, int n,
                                     const void *A, int lda, long long strideA,
                                     void *S, long long strideS,
                                     void *U, int ldu, long long strideU,
                                     void *V, int ldv, long long strideV,
                                     double tol, int *info,
                                     const svdb_opts_t *opts, void *stream);

/* Bytes of the static scratch of svdb_svd_strided_batched_noalloc. */
size_t svdb_noalloc_scratch_bytes(void);

/*
 * Mixed-shape batch (uneven batching): host arrays m[b], n[b], lda[b],
 * ldu[b], ldv[b] and host arrays of device pointers A[b], S[b], U[b], V[b]
 * (U or V may be NULL as a whole).  Any m[b], n[b] >= 0, with outputs as in
 * svdb_svd_strided_batched (k_b = min(m_b, n_b) columns; a wide matrix is
 * read transposed into its working copy); A[b] is not modified.  Every
 * matrix runs the block method (eq. block-gram, nb = 16, any
 * dtype) on its own round-robin schedule over l_b = n_b / 16 (rounded up to
 * even) block columns: one launch per round-robin step covers the block
 * pairs of every unconverged matrix of the batch, and a small matrix
 * completes several sweeps while a large one completes one.  opts->path and
 * opts->nb are ignored; opts->precision must be 0.  The workspace (at least
 * svdb_batched_workspace_size() bytes) holds per-matrix descriptors, the
 * work table and every matrix's working copies of A and V.
 * Arguments, 1-based: dtype 1, batch 2, m 3, n 4, A 5, lda 6, S 7, U 8,
 * ldu 9, V 10, ldv 11, tol 12, info 13, workspace 14, ws_bytes 15, opts 16,
 * stream 17.
 */
int svdb_svd_batched(svdb_dtype_t dtype, int batch, const int *m, const int *n,
                     const void *const *A, const int *lda,
                     void *const *S,
                     void *const *U, const int *ldu,
                     void *const *V, const int *ldv,
                     double tol, int *info,
                     void *workspace, size_t ws_bytes,
                     const svdb_opts_t *opts, void *stream);

/* Bytes of device workspace svdb_svd_batched needs for these shapes
 * (host arrays m[], n[]); (size_t)-1 on invalid arguments. */
size_t svdb_batched_workspace_size(svdb_dtype_t dtype, int batch, const int *m,
                                   const int *n, const svdb_opts_t *opts);

/*
 * The path and launch shape AUTO (or the forced path in opts) would use for
 * one m x n matrix (for m < n: that of the n x m matrix A^H): *path (svdb_path_t), *nb (block width, 0 if unblocked),
 * *threads (threads per matrix).  Returns 0, or SVDB_ERR_UNSUPPORTED if no
 * path handles the shape.
 */
int svdb_plan(svdb_dtype_t dtype, int m, int n, const svdb_opts_t *opts,
              int *path, int *nb, int *threads);

/*
 * Serving runtime: continuous batching of independent requests on one GPU.
 *
 * A server owns a device arena of budget_bytes (allocated at creation, freed
 * at destruction), its own HIP stream (default priority) and a worker
 * thread.  Each request runs the block method (nb = 16, any dtype, n <= 512)
 * on its own schedule; requests are admitted first come, first served while
 * a slot (max_requests per dtype) is free and the arena holds their working
 * copies of A and V ((m np + np^2) elements, np = n rounded up to an even
 * number of 16-column blocks).  A request leaves as soon as it has
 * converged (or reached opts->max_sweeps), so new requests take its place
 * between any two launches: the paper's masks ("Masked Batch Operations")
 * retire converged matrices inside a static batch, the server also refills
 * the batch.
 *
 *  svdb_server_create: opts may be NULL (defaults; precision must be 0).
 *     opts->precondition -1 (default) or 1 runs real requests (m <= 1024)
 *     with QR preconditioning (2, column pivoting, is refused with
 *     SVDB_ERR_UNSUPPORTED): A = Q R, the FP64 Jacobi on R^T, U = Q J
 *     (FP32 requests are solved in FP64 and returned in FP32; requests with
 *     more than 64 columns take the blocked QR, up to eight of one shape
 *     per launch, through about 50 MB of staging memory that the server
 *     allocates beside its arena); 0: off.
 *     Returns 0, -k for invalid argument k, SVDB_ERR_HIP.
 *  svdb_server_submit: device pointers as svdb_svd_batched; A must hold its
 *     values when the call is made (the server reads it on its own stream)
 *     and every buffer must stay valid until the request completes.  The
 *     rotation threshold is 30 u of the dtype (tol is reserved).  Thread
 *     safe.  Any m, n >= 0: outputs as in svdb_svd_strided_batched (a
 *     wide request runs as A^H, read transposed, without preconditioning).
 *     Returns the request id (>= 0), -k for invalid argument k,
 *     SVDB_ERR_UNSUPPORTED when min(m, n) > 512 or the request exceeds the
 *     budget,
 *     SVDB_ERR_HIP after a device failure.
 *  svdb_server_poll: waits up to timeout_ms (< 0: forever, 0: no wait) for
 *     completions and returns up to cap of them: id, submission and
 *     completion times (svdb_server_clock seconds; outputs and *info are
 *     valid at completion).  Returns the count, or SVDB_ERR_HIP.
 *  svdb_server_destroy: finishes every submitted request, then frees all.
 */
typedef struct svdb_server svdb_server_t;

int svdb_server_create(svdb_server_t **srv, size_t budget_bytes, int max_requests,
                       const svdb_opts_t *opts);
long long svdb_server_submit(svdb_server_t *srv, svdb_dtype_t dtype, int m, int n,
                             const void *A, int lda, void *S, void *U, int ldu,
                             void *V, int ldv, double tol, int *info, int *sweeps);
int svdb_server_poll(svdb_server_t *srv, long long *ids, double *t_submit,
                     double *t_done, int cap, int timeout_ms);
/* Counters: submitted, completed, active (admitted, running), queued, and
 * arena bytes in use.  Returns 0 or SVDB_ERR_HIP after a device failure. */
int svdb_server_stats(svdb_server_t *srv, long long *submitted, long long *completed,
                      int *active, int *queued, size_t *bytes_in_use);
/* Text of the server's device failure ("" if none). */
const char *svdb_server_error(svdb_server_t *srv);
int svdb_server_destroy(svdb_server_t *srv);
/* Monotonic clock of the server's timestamps, in seconds. */
double svdb_server_clock(void);

/* Text of the last failure in the calling thread ("" if none). */
const char *svdb_last_error(void);

/* Library version string. */
const char *svdb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SVDB_H */
