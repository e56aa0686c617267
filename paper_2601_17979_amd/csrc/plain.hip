// plain.hip -- the plain GPU Jacobi: unblocked one-sided Jacobi SVD (Alg. 2)
// with the whole matrix W (m x n) and V (n x n) resident in LDS, one
// 256-thread workgroup per matrix, round-robin pairs ("Algorithmic Background"), FP64.
//
// This kernel is the simple reference point of the library's fast paths: it
// is written for clarity and is not tuned.  Every round-robin iteration
// assigns each of the l/2 disjoint pairs to a group of G lanes (a power of
// two inside one wavefront); the group forms g_ii, g_jj, g_ij over the rows
// (Alg. 2, Gram entries), decides rotate-or-skip (threshold test), computes
// c, s (eq. sin-cos) and rotates both columns of W and V.  One barrier
// separates iterations.  Finalisation (sigma = column norms, U = W / sigma,
// zero-sigma completion, stable descending sort) follows Alg. 2's last steps.
#include "device_common.hpp"
#include "launchers.hpp"

namespace svdb {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void finalize_lds(int m, int n, double *W, double *Vw,
                                             double *sig, int *rank, double scale_back,
                                             double *S, double *U, int ldu, double *V,
                                             int ldv)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int nwaves = kThreads / kWave;
    // sigma_c = ||w_c||_2 with scaling, one wavefront per column
    for (int c = wave; c < n; c += nwaves) {
        const double *w = W + (size_t)c * m;
        double mx = 0.0;
        for (int r = lane; r < m; r += kWave) mx = fmax(mx, fabs(w[r]));
        mx = wave_max(mx);
        double ss = 0.0;
        if (mx > 0.0) {
            const double inv = 1.0 / mx;
            for (int r = lane; r < m; r += kWave) {
                double y = w[r] * inv;
                ss += y * y;
            }
        }
        ss = wave_sum(ss);
        if (lane == 0) sig[c] = mx > 0.0 ? mx * sqrt(ss) : 0.0;
    }
    __syncthreads();
    // u_c = w_c / sigma_c
    for (int c = wave; c < n; c += nwaves) {
        const double sc = sig[c];
        if (sc > 0.0) {
            const double inv = 1.0 / sc;
            for (int r = lane; r < m; r += kWave) W[(size_t)c * m + r] *= inv;
        }
    }
    __syncthreads();
    // sigma = 0: complete U with Gram-Schmidt on e_1, e_2, ... (one wavefront)
    if (wave == 0) {
        int cand = 0;
        for (int i = 0; i < n; i++) {
            if (sig[i] > 0.0) continue;
            double *u = W + (size_t)i * m;
            for (; cand < m; cand++) {
                for (int r = lane; r < m; r += kWave) u[r] = (r == cand) ? 1.0 : 0.0;
                for (int pass = 0; pass < 2; pass++)
                    for (int j = 0; j < n; j++) {
                        if (j == i || (sig[j] == 0.0 && j > i)) continue;
                        const double *qv = W + (size_t)j * m;
                        double d = 0.0;
                        for (int r = lane; r < m; r += kWave) d += qv[r] * u[r];
                        d = wave_sum(d);
                        for (int r = lane; r < m; r += kWave) u[r] -= d * qv[r];
                    }
                double nu = 0.0;
                for (int r = lane; r < m; r += kWave) nu += u[r] * u[r];
                nu = sqrt(wave_sum(nu));
                if (nu > 0.5) {
                    const double inv = 1.0 / nu;
                    for (int r = lane; r < m; r += kWave) u[r] *= inv;
                    cand++;
                    break;
                }
            }
        }
    }
    // stable descending rank of every sigma
    for (int c = tid; c < n; c += kThreads) {
        const double sc = sig[c];
        int rk = 0;
        for (int j = 0; j < n; j++) {
            const double sj = sig[j];
            rk += (sj > sc) || (sj == sc && j < c);
        }
        rank[c] = rk;
    }
    __syncthreads();
    for (int c = wave; c < n; c += nwaves) {
        const int rk = rank[c];
        if (lane == 0) S[rk] = sig[c] * scale_back;
        if (U)
            for (int r = lane; r < m; r += kWave) U[(size_t)rk * ldu + r] = W[(size_t)c * m + r];
        if (V)
            for (int r = lane; r < n; r += kWave) V[(size_t)rk * ldv + r] = Vw[(size_t)c * n + r];
    }
}

__global__ __launch_bounds__(kThreads) void plain_jacobi_d(
    int m, int n, const double *__restrict__ A, int lda, long long sA, double *S, long long sS,
    double *U, int ldu, long long sU, double *V, int ldv, long long sV, double tol,
    int max_sweeps, int *info, int *sweeps_out)
{
    extern __shared__ double smem[];
    __shared__ double s_red[kThreads / kWave];
    __shared__ int s_bad[kThreads / kWave];
    __shared__ int s_rot;

    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    A += (size_t)b * sA;
    S += (size_t)b * sS;
    if (U) U += (size_t)b * sU;
    if (V) V += (size_t)b * sV;

    double *W = smem;                       // m x n, ld m
    double *Vw = W + (size_t)m * n;         // n x n, ld n
    double *sig = Vw + (size_t)n * n;       // n
    int *rank = (int *)(sig + n);           // n

    // ---- load A, check finiteness, find max|a| -----------------------------
    double amax = 0.0;
    int bad = 0;
    for (int c = wave; c < n; c += kThreads / kWave)
        for (int r = lane; r < m; r += kWave) {
            const double a = A[(size_t)c * lda + r];
            bad |= !isfinite(a);
            amax = fmax(amax, fabs(a));
            W[(size_t)c * m + r] = a;
        }
    for (int idx = tid; idx < n * n; idx += kThreads) Vw[idx] = (idx % (n + 1) == 0) ? 1.0 : 0.0;
    amax = wave_max(amax);
    bad = __any(bad);
    if (lane == 0) {
        s_red[wave] = amax;
        s_bad[wave] = bad;
    }
    __syncthreads();
    for (int w = 0; w < kThreads / kWave; w++) bad |= s_bad[w];
    if (bad) {
        if (tid == 0) {
            info[b] = 2;
            if (sweeps_out) sweeps_out[b] = 0;
        }
        return;
    }
    amax = s_red[0];
    for (int w = 1; w < kThreads / kWave; w++) amax = fmax(amax, s_red[w]);
    const double scale = pow2_scale(amax);
    if (scale != 1.0)
        for (int idx = tid; idx < m * n; idx += kThreads) W[idx] *= scale;

    // ---- sweeps -----------------------------------------------------------
    const int l = n + (n & 1);              // odd n: phantom index n never rotates
    const int P = l / 2;
    int G = 1;                              // lanes per pair (power of two, <= 64)
    while (G * 2 * P <= kThreads && G < kWave) G *= 2;
    const int q = tid / G, gl = tid & (G - 1);
    const bool active = q < P;

    int sweeps = 0, converged = 0;
    while (!converged && sweeps < max_sweeps) {
        sweeps++;
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int it = 0; it < l - 1; it++) {
            int i = 0, j = 0;
            double gii = 0.0, gjj = 0.0, gij = 0.0;
            if (active) {
                rr_pair(l, it, q, i, j);
                if (j < n) {
                    const double *wi = W + (size_t)i * m, *wj = W + (size_t)j * m;
                    for (int r = gl; r < m; r += G) {
                        const double x = wi[r], y = wj[r];
                        gii = fma(x, x, gii);
                        gjj = fma(y, y, gjj);
                        gij = fma(x, y, gij);
                    }
                }
            }
            gii = group_sum(gii, G);
            gjj = group_sum(gjj, G);
            gij = group_sum(gij, G);
            if (active && j < n && gij != 0.0 && fabs(gij) >= tol * sqrt(gii) * sqrt(gjj)) {
                double c, s;
                jacobi_cs(gii, gjj, fabs(gij), c, s);
                const double es = gij > 0.0 ? s : -s;      // e^{i phi} s, real
                double *wi = W + (size_t)i * m, *wj = W + (size_t)j * m;
                for (int r = gl; r < m; r += G) {
                    const double x = wi[r], y = wj[r];
                    wi[r] = fma(c, x, es * y);
                    wj[r] = fma(c, y, -es * x);
                }
                double *vi = Vw + (size_t)i * n, *vj = Vw + (size_t)j * n;
                for (int r = gl; r < n; r += G) {
                    const double x = vi[r], y = vj[r];
                    vi[r] = fma(c, x, es * y);
                    vj[r] = fma(c, y, -es * x);
                }
                if (gl == 0) s_rot = 1;
            }
            __syncthreads();
        }
        converged = (s_rot == 0);
        __syncthreads();
    }

    finalize_lds(m, n, W, Vw, sig, rank, 1.0 / scale, S, U, ldu, V, ldv);
    if (tid == 0) {
        info[b] = converged ? 0 : 1;
        if (sweeps_out) sweeps_out[b] = sweeps;
    }
}

}  // namespace

size_t plain_lds_bytes(int m, int n)
{
    return sizeof(double) * ((size_t)m * n + (size_t)n * n + n) + sizeof(int) * n;
}

int plain_max_lds_bytes() { return 160 * 1024 - 1024; }

hipError_t launch_plain_d(int batch, int m, int n, const double *A, int lda, long long sA,
                          double *S, long long sS, double *U, int ldu, long long sU, double *V,
                          int ldv, long long sV, double tol, int max_sweeps, int *info,
                          int *sweeps, hipStream_t stream)
{
    const size_t lds = plain_lds_bytes(m, n);
    hipError_t e = hipFuncSetAttribute((const void *)plain_jacobi_d,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       plain_max_lds_bytes());
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(plain_jacobi_d, dim3(batch), dim3(kThreads), lds, stream, m, n, A, lda,
                       sA, S, sS, U, ldu, sU, V, ldv, sV, tol, max_sweeps, info, sweeps);
    return hipGetLastError();
}

}  // namespace svdb
