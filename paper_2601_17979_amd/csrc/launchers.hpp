// launchers.hpp -- host-side launch functions of the kernels (internal to the
// library; the public interface is include/svdb.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace svdb {

// plain.hip: LDS-resident unblocked Jacobi, FP64, one workgroup per matrix.
size_t plain_lds_bytes(int m, int n);
int plain_max_lds_bytes();
hipError_t launch_plain_d(int batch, int m, int n, const double *A, int lda, long long sA,
                          double *S, long long sS, double *U, int ldu, long long sU, double *V,
                          int ldv, long long sV, double tol, int max_sweeps, int *info,
                          int *sweeps, hipStream_t stream);

// resident.hip: register-resident unblocked Jacobi, FP64, n <= 64.
bool resident_config(int m, int n, int ns, int *N, int *R, int *NS);
// nv: iterate on W alone (no V rows; V is not written), for m <= 64 and
// 32 < n <= 64 (resident_nv_supported).  only: NULL or per-matrix flags,
// matrices with flag 0 are skipped.  lower: A is lower triangular (the
// transposed triangular factor of the QR pre-processing); the entries above
// its diagonal are taken as zero without being read.
bool resident_nv_supported(int m, int n);
hipError_t launch_resident_d(int batch, int m, int n, int ns, const double *A, int lda,
                             long long sA, double *S, long long sS, double *U, int ldu,
                             long long sU, double *V, int ldv, long long sV, double tol,
                             int max_sweeps, int *info, int *sweeps, hipStream_t stream,
                             bool nv = false, const int *only = nullptr,
                             bool lower = false);

// qr.hip: QR preconditioning (A P = Q1 R1, R1^T = Q2 R2, the resident Jacobi
// on R2^T; P = I unless pivot).
bool precond_supported(int m, int n);
size_t precond_workspace_bytes(int batch, int m, int n);
hipError_t launch_precond_d(int batch, int m, int n, int ns, const double *A, int lda,
                            long long sA, double *S, long long sS, double *U, int ldu,
                            long long sU, double *V, int ldv, long long sV, double tol,
                            int max_sweeps, int *info, int *sweeps, void *ws, hipStream_t stream,
                            bool pivot = false);
bool precond_tall_supported(int m, int n);
bool precond_tall_auto(int m, int n);   // where AUTO takes it (m <= 1024)
size_t precond_tall_workspace_bytes(int batch, int m, int n);
hipError_t launch_precond_tall_d(int batch, int m, int n, const double *A, int lda, long long sA,
                                 double *S, long long sS, double *U, int ldu, long long sU,
                                 double *V, int ldv, long long sV, double tol, int max_sweeps,
                                 int *info, int *sweeps, void *ws, hipStream_t stream);
bool precond_big_supported(int m, int n);

// QR preconditioning of single requests (serving runtime): one QrJob per
// matrix in device memory; list (device) selects the jobs of a launch.
struct QrJob {
    const void *A;            // input, lda, m x n (m <= 1024, n <= 512)
    int lda, m, n, f32;       // f32: A holds floats
    double *Vq, *X, *tau;     // workspace: reflectors (m x n), X = R^T (n x n), tau (n)
    const double *Y;          // J from the Jacobi on X (n x n, ld n)
    void *U;                  // output U (ldu), or NULL
    int ldu, uf32;            // uf32: U, S and V are floats
    const double *S64, *Vx64; // FP64 staging of S and V (FP32 requests)
    void *Sout, *Vout;        // FP32 outputs S and V (V may be NULL), ldv
    int ldv, pad;
    const int *info;          // the request's status
};
void launch_qr_jobs(const QrJob *jobs, const int *list, int count, hipStream_t stream);
// the blocked QR of a strided batch (m <= 1024, n <= 512): reflectors as
// full columns into H (m n apart), X = R^T, tau; A may equal H.  scratch
// holds qr_blocked_scratch_bytes of any larger or equal batch and shape
size_t qr_blocked_scratch_bytes(int batch, int m, int n);
hipError_t launch_qr_blocked_batch(int batch, int m, int n, const double *A, int lda,
                                   long long sA, double *H, double *X, double *tau,
                                   void *scratch, hipStream_t stream);
void launch_apply_q_jobs(const QrJob *jobs, const int *list, int count, int max_m,
                         hipStream_t stream);
size_t precond_big_workspace_bytes(int batch, int m, int n, int nb, bool mixed = false);
hipError_t launch_precond_big_d(int batch, int m, int n, int nb, const double *A, int lda,
                                long long sA, double *S, long long sS, double *U, int ldu,
                                long long sU, double *V, int ldv, long long sV, double tol,
                                int max_sweeps, int masking, int *info, int *sweeps, void *ws,
                                hipStream_t stream, int inner = 0, int persistent = 0,
                                double tol_start = 0.0, double tol_rate = 0.0,
                                double tol32 = 0.0);

// launch_precond_big_d: tol32 > 0 runs the block Jacobi on R2^T in the mixed
// mode (FP32 sweeps to tol32, then FP64 refinement).
// blocked.hip: block one-sided Jacobi with MFMA Gram/updates (real and
// complex, FP64 and FP32, and FP32 sweeps followed by an FP64 refinement).
// blocked_nb returns the block width for a request (0: not supported).
// `inner` (all block launchers): inner sweeps per block-pair solve; 0 = one,
// or the converged solve for two block columns; k > 0 = at most k; < 0 = to
// convergence.  `persistent`: 1 = all sweeps in one cooperative launch
// (disabled at the public interface: it stalled on the GPU); 0 = one launch
// per round-robin iteration with a host-side loop that waits for the
// pending count after every sweep.  tol_start > tol: the dynamic inner
// tolerance, outer sweep s solving with max(tol, tol_start tol_rate^s).
int blocked_nb(int m, int n, int nb, bool complex_);
int blocked_np(int n, int nb);
size_t blocked_workspace_bytes(int batch, int m, int n, int nb, int elt, bool mixed);
hipError_t launch_blocked_d(int batch, int m, int n, int nb, const double *A, int lda, long long sA,
                            double *S, long long sS, double *U, int ldu, long long sU, double *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream,
                            int inner = 0, int persistent = 0, double tol_start = 0.0,
                            double tol_rate = 0.0);
hipError_t launch_blocked_s(int batch, int m, int n, int nb, const float *A, int lda, long long sA,
                            float *S, long long sS, float *U, int ldu, long long sU, float *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream,
                            int inner = 0, int persistent = 0, double tol_start = 0.0,
                            double tol_rate = 0.0);
hipError_t launch_blocked_z(int batch, int m, int n, int nb, const void *A, int lda, long long sA,
                            double *S, long long sS, void *U, int ldu, long long sU, void *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream,
                            int inner = 0, int persistent = 0, double tol_start = 0.0,
                            double tol_rate = 0.0);
hipError_t launch_blocked_c(int batch, int m, int n, int nb, const void *A, int lda, long long sA,
                            float *S, long long sS, void *U, int ldu, long long sU, void *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream,
                            int inner = 0, int persistent = 0, double tol_start = 0.0,
                            double tol_rate = 0.0);
hipError_t launch_blocked_mixed_d(int batch, int m, int n, int nb, const double *A, int lda,
                                  long long sA, double *S, long long sS, double *U, int ldu,
                                  long long sU, double *V, int ldv, long long sV, double tol,
                                  double tol32, int max_sweeps, int masking, int *info,
                                  int *sweeps, void *ws, hipStream_t stream, int inner = 0,
                                  int persistent = 0, double tol_start = 0.0,
                                  double tol_rate = 0.0);

// tuning.hip: the measured launch table.  tuned_block fills the block
// method's choices for a request of this dtype and shape (false: no row,
// the built-in rules apply); tuned_resident_waves gives the wavefronts per
// matrix of the resident kernel for (N, rows per lane), 0 if none.
struct BlockChoice {
    int nb = 0, inner = 0;
    double tol_start = 0.0, tol_rate = 0.0;
};
bool tuned_block(int dtype, int m, int n, BlockChoice *c);
int tuned_resident_waves(int N, int rw);

// Per-matrix descriptor of the uneven-batch kernels (device memory).
struct VbDesc {
    const void *A;          // input, lda
    void *S, *U, *V;        // outputs (U, V may be NULL), ldu, ldv
    int *info, *sweeps;     // this matrix's status slots (sweeps may be NULL)
    long long woff, voff;   // element offsets of W (m x np) and V (np x np) from the base
    int m, n, np, l, lda, ldu, ldv, it0;   // it0: launch index of its first iteration
    int trans;   // 1: A holds the n x m matrix whose conjugate transpose is this m x n one
    int inner;   // inner sweeps of its block-pair solves when the call leaves them
                 // open (0: the built-in rule)
};

// Launchers of the uneven-batch kernels; dtype as svdb_dtype_t, st points to
// per-matrix state of vb_state_bytes() each; idx (device) selects matrices,
// NULL = 0 .. count-1.
void vb_launch_init(int dtype, const VbDesc *d, const int *idx, int count, void *base, void *st,
                    hipStream_t stream);
// t0, rate: the dynamic inner tolerance (t0 <= tol: tol in every sweep).
// stop: NULL, or a device word; once it is nonzero the launch does nothing.
void vb_launch_iter(int dtype, const VbDesc *d, const int2 *work, int nwork, int itg, void *base,
                    void *st, double tol, hipStream_t stream, int inner = 0, double t0 = 0.0,
                    double rate = 0.0, const int *stop = nullptr);
void vb_launch_sweep_end(int count, const VbDesc *d, int itg, void *st, int max_sweeps,
                         int masking, int *pending, hipStream_t stream, double tol = 0.0,
                         double t0 = 0.0, double rate = 0.0, const int *stop = nullptr);
void vb_launch_collect(int count, const void *st, int *flags, hipStream_t stream);
void vb_launch_mark_empty(int count, void *st, hipStream_t stream);
void vb_launch_finalize(int dtype, const VbDesc *d, const int *idx, int count, int maxn,
                        const void *base, const void *st, hipStream_t stream);
size_t vb_state_bytes();
int vb_nb();

// Uneven batches on the block method (nb = 16): per-matrix pointers and
// shapes; dtype as svdb_dtype_t.  The workspace holds descriptors, the work
// table, per-matrix state and every matrix's W and V.
size_t vbatched_workspace_bytes(int batch, const int *m, const int *n, int elt);
hipError_t launch_vbatched(int dtype, int batch, const int *m, const int *n, const void *const *A,
                           const int *lda, void *const *S, void *const *U, const int *ldu,
                           void *const *V, const int *ldv, double tol, int max_sweeps,
                           int masking, int *info, int *sweeps, void *ws, hipStream_t stream,
                           const int *trans = nullptr, int inner = 0, int persistent = 0,
                           double tol_start = 0.0, double tol_rate = 0.0);

// blocked.hip: batched FP64 GEMM on the matrix cores, column major:
// C = alpha op(A) B + beta D (op(A) = A^T when trans_a; D may be NULL; C may
// equal D but must not overlap A or B).
hipError_t launch_gemm_f64(bool trans_a, int batch, int M, int N, int K, double alpha,
                           const double *A, int lda, long long sA, const double *B, int ldb,
                           long long sB, double beta, const double *D, int ldd, long long sD,
                           double *C, int ldc, long long sC, hipStream_t stream);

// layout.hip: At (n x m, ld n, n m apart) = A^H for a strided batch of m x n
// matrices; dtype as svdb_dtype_t.
hipError_t launch_conj_transpose(int dtype, int batch, int m, int n, const void *A, int lda,
                                 long long sA, void *At, hipStream_t stream);
// FP32 -> FP64 and FP64 -> FP32 copies of strided batches (rows x cols); the
// narrowing skips matrices whose info is 2
hipError_t launch_widen_f32(int batch, int rows, int cols, const float *src, int lds,
                            long long ss, double *dst, int ldd, long long sd, hipStream_t stream);
hipError_t launch_narrow_f64(int batch, int rows, int cols, const double *src, int lds,
                             long long ss, float *dst, int ldd, long long sd, const int *info,
                             hipStream_t stream);

// p[0 .. count) = value, by a small kernel (no hipMemsetAsync, so that a
// caller may capture the call in a HIP graph)
hipError_t launch_fill_int(int *p, int count, int value, hipStream_t stream);

}  // namespace svdb
