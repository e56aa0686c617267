/*
 * svdb.h -- C ABI of the MI355X batched one-sided Jacobi SVD library.
 *
 * Problem (paper Sec. 1, eq. "svd"): for each m x n matrix A of a batch, with
 * m >= n, compute the reduced SVD A = U diag(S) V^H: U is m x n with
 * orthonormal columns, V is n x n unitary, S is real, non-negative and sorted
 * in descending order (Alg. 2, last step; accuracy check T4 in Sec. 4.5).
 * The method is the one-sided (Hestenes) Jacobi iteration of Alg. 2 with the
 * rotation of eq. (sin-cos), the round-robin parallel ordering of Sec. 2/4.1,
 * and, for wider matrices, the block method of Sec. 3 (eq. block-gram,
 * eq. right-sv) with a one-sweep inner eigensolver (Sec. 5) and batch masks
 * (Sec. 7).
 *
 * Conventions for every entry point:
 *  - Matrices are column major (LAPACK style) with a leading dimension.
 *  - All data pointers (A, S, U, V, info, workspace, opts->sweeps) are DEVICE
 *    pointers owned by the caller; the library allocates no device memory in
 *    these calls.  Host-side arrays (m[], n[], lda[], and the pointer arrays
 *    of svdb_svd_batched) are read during the call only.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    is asynchronous: outputs and info[] are valid after the stream is
 *    synchronised.
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
 *    Sec. 4.5 / 8.1).
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

/* Execution paths.  AUTO chooses from the tuned plan table. */
typedef enum {
    SVDB_PATH_AUTO = 0,
    SVDB_PATH_PLAIN = 1,     /* LDS-resident unblocked kernel, one workgroup
                                per matrix (the plain GPU Jacobi)           */
    SVDB_PATH_RESIDENT = 2,  /* register-resident unblocked kernel (Alg. 2) */
    SVDB_PATH_BLOCKED = 3    /* block method (Sec. 3-7) with MFMA Gram and
                                updates                                     */
} svdb_path_t;

#define SVDB_ERR_UNSUPPORTED (-200)
#define SVDB_ERR_HIP (-100)

typedef struct {
    int max_sweeps;   /* cap on sweeps (Alg. 2 max_nsweeps); <= 0 -> 100       */
    int path;         /* svdb_path_t                                          */
    int nb;           /* block width for SVDB_PATH_BLOCKED; 0 -> tuned         */
    int masking;      /* blocked path: skip converged matrices (Sec. 7);
                         < 0 -> default (on)                                   */
    int precision;    /* 0: sweeps in the working precision; 1: FP32 sweeps
                         then FP64 refinement (SVDB_R64 / SVDB_C128 only)      */
    int *sweeps;      /* optional DEVICE int[batch]: sweeps executed          */
    int waves;        /* SVDB_PATH_RESIDENT: wavefronts per matrix (1, 2, 4);
                         0 -> tuned                                           */
} svdb_opts_t;

/* Fills *o with the defaults (AUTO path, 100 sweeps, masking on). */
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
 *  S       out: n singular values per matrix, descending.
 *  U       out: m x n left singular vectors (ldu >= m), or NULL.
 *  V       out: n x n right singular vectors (ldv >= n), A = U S V^H, or NULL.
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
 * Mixed-shape batch (uneven batching): host arrays m[b], n[b], lda[b],
 * ldu[b], ldv[b] and host arrays of device pointers A[b], S[b], U[b], V[b]
 * (U or V may be NULL as a whole).  Requires m[b] >= n[b] >= 0.  Matrices of
 * one shape class are launched together; the whole batch is one call.
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

/* Bytes of device workspace svdb_svd_batched needs for these shapes. */
size_t svdb_batched_workspace_size(svdb_dtype_t dtype, int batch, const int *m,
                                   const int *n, const svdb_opts_t *opts);

/*
 * The path and launch shape AUTO (or the forced path in opts) would use for
 * one m x n matrix: *path (svdb_path_t), *nb (block width, 0 if unblocked),
 * *threads (threads per matrix).  Returns 0, or SVDB_ERR_UNSUPPORTED if no
 * path handles the shape.
 */
int svdb_plan(svdb_dtype_t dtype, int m, int n, const svdb_opts_t *opts,
              int *path, int *nb, int *threads);

/* Text of the last failure in the calling thread ("" if none). */
const char *svdb_last_error(void);

/* Library version string. */
const char *svdb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SVDB_H */
