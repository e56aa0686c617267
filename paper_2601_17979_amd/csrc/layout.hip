// layout.hip -- layout and precision copies of strided batches: the
// conjugate transpose for wide matrices, and FP32 <-> FP64 copies for FP32
// input run on the FP64 preconditioned paths.
//
// For m < n the reduced SVD is taken from the tall matrix A^H (n x m):
// A^H = U' diag(S) V'^H gives A = V' diag(S) U'^H, so U = V' (m x m) and
// V = U' (n x m) (section "Pre-processing the SVD using a QR Factorization":
// the case m < n reduces to A^H).  The kernel writes A^H into the workspace;
// the tall path then runs on it with the two output matrices exchanged.
#include <hip/hip_runtime.h>

#include "launchers.hpp"

namespace svdb {

namespace {

constexpr int kTile = 32;

__device__ __forceinline__ float conj_of(float x) { return x; }
__device__ __forceinline__ double conj_of(double x) { return x; }
__device__ __forceinline__ float2 conj_of(float2 x) { return make_float2(x.x, -x.y); }
__device__ __forceinline__ double2 conj_of(double2 x) { return make_double2(x.x, -x.y); }

// One 32 x 32 tile per workgroup, staged in LDS so that both the reads of A
// (down its columns) and the writes of At (down its columns) are coalesced.
// At is n x m with leading dimension n, matrices n m elements apart.
template <class E>
__global__ __launch_bounds__(256) void conj_transpose(int m, int n, int tm, int tn,
                                                      const E *__restrict__ A, int lda,
                                                      long long sA, E *__restrict__ At)
{
    __shared__ E tile[kTile][kTile + 1];
    const int per = tm * tn;
    const long long blk = blockIdx.x;
    const long long b = blk / per;
    const int t = (int)(blk % per);
    const int r0 = (t % tm) * kTile, c0 = (t / tm) * kTile;
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
    const E *a = A + b * sA;
    E *at = At + b * (long long)n * m;
    for (int k = ty; k < kTile; k += 256 / kTile) {
        const int r = r0 + tx, c = c0 + k;
        if (r < m && c < n) tile[k][tx] = a[(size_t)c * lda + r];
    }
    __syncthreads();
    for (int k = ty; k < kTile; k += 256 / kTile) {
        const int rr = c0 + tx, cc = r0 + k;   // At(rr, cc) = conj(A(cc, rr))
        if (rr < n && cc < m) at[(size_t)cc * n + rr] = conj_of(tile[tx][k]);
    }
}

template <class E>
hipError_t launch_t(int batch, int m, int n, const void *A, int lda, long long sA, void *At,
                    hipStream_t stream)
{
    const int tm = (m + kTile - 1) / kTile, tn = (n + kTile - 1) / kTile;
    const long long blocks = (long long)batch * tm * tn;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((conj_transpose<E>), dim3((unsigned)blocks), dim3(256), 0, stream, m, n,
                       tm, tn, (const E *)A, lda, sA, (E *)At);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_conj_transpose(int dtype, int batch, int m, int n, const void *A, int lda,
                                 long long sA, void *At, hipStream_t stream)
{
    switch (dtype) {
    case 0: return launch_t<float>(batch, m, n, A, lda, sA, At, stream);
    case 1: return launch_t<double>(batch, m, n, A, lda, sA, At, stream);
    case 2: return launch_t<float2>(batch, m, n, A, lda, sA, At, stream);
    case 3: return launch_t<double2>(batch, m, n, A, lda, sA, At, stream);
    default: return hipErrorInvalidValue;
    }
}

namespace {

// dst (rows x cols, ld ldd, matrices sd apart) = src, element by element;
// with info, matrices whose info is 2 (non-finite input) are skipped.
template <class TS, class TD>
__global__ void convert_batch(int batch, int rows, int cols, const TS *__restrict__ src, int lds,
                              long long ss, TD *__restrict__ dst, int ldd, long long sd,
                              const int *info)
{
    const size_t per = (size_t)rows * cols, total = per * batch;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const size_t b = g / per;
        if (info && info[b] == 2) continue;
        const int idx = (int)(g % per), r = idx % rows, c = idx / rows;
        dst[b * sd + (size_t)c * ldd + r] = (TD)src[b * ss + (size_t)c * lds + r];
    }
}

template <class TS, class TD>
hipError_t launch_convert(int batch, int rows, int cols, const TS *src, int lds, long long ss,
                          TD *dst, int ldd, long long sd, const int *info, hipStream_t stream)
{
    const size_t total = (size_t)batch * rows * cols;
    if (total == 0) return hipSuccess;
    size_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL((convert_batch<TS, TD>), dim3((unsigned)g), dim3(256), 0, stream, batch,
                       rows, cols, src, lds, ss, dst, ldd, sd, info);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_widen_f32(int batch, int rows, int cols, const float *src, int lds,
                            long long ss, double *dst, int ldd, long long sd, hipStream_t stream)
{
    return launch_convert<float, double>(batch, rows, cols, src, lds, ss, dst, ldd, sd, nullptr,
                                         stream);
}

hipError_t launch_narrow_f64(int batch, int rows, int cols, const double *src, int lds,
                             long long ss, float *dst, int ldd, long long sd, const int *info,
                             hipStream_t stream)
{
    return launch_convert<double, float>(batch, rows, cols, src, lds, ss, dst, ldd, sd, info,
                                         stream);
}

namespace {

__global__ void fill_int(int *__restrict__ p, int count, int value)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = value;
}

}  // namespace

hipError_t launch_fill_int(int *p, int count, int value, hipStream_t stream)
{
    if (!p || count <= 0) return hipSuccess;
    const int g = (count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024;
    hipLaunchKernelGGL(fill_int, dim3((unsigned)g), dim3(256), 0, stream, p, count, value);
    return hipGetLastError();
}

}  // namespace svdb
