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
hipError_t launch_resident_d(int batch, int m, int n, int ns, const double *A, int lda,
                             long long sA, double *S, long long sS, double *U, int ldu,
                             long long sU, double *V, int ldv, long long sV, double tol,
                             int max_sweeps, int *info, int *sweeps, hipStream_t stream);

// blocked.hip: block one-sided Jacobi with MFMA Gram/updates (FP64, FP32,
// and FP32 sweeps followed by an FP64 refinement).
int blocked_nb(int m, int n, int nb);
int blocked_np(int n, int nb);
size_t blocked_workspace_bytes(int batch, int m, int n, int nb, int elt, bool mixed);
hipError_t launch_blocked_d(int batch, int m, int n, int nb, const double *A, int lda, long long sA,
                            double *S, long long sS, double *U, int ldu, long long sU, double *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream);
hipError_t launch_blocked_s(int batch, int m, int n, int nb, const float *A, int lda, long long sA,
                            float *S, long long sS, float *U, int ldu, long long sU, float *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream);
hipError_t launch_blocked_mixed_d(int batch, int m, int n, int nb, const double *A, int lda,
                                  long long sA, double *S, long long sS, double *U, int ldu,
                                  long long sU, double *V, int ldv, long long sV, double tol,
                                  double tol32, int max_sweeps, int masking, int *info,
                                  int *sweeps, void *ws, hipStream_t stream);

}  // namespace svdb
