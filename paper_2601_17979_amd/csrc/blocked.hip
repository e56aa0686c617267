// blocked.hip -- the block one-sided Jacobi SVD (Sec. 3, eq. block-gram and
// eq. right-sv) with a one-sweep inner eigensolver (Sec. 5, "Design 2"),
// fused vector updates (Sec. 6) and batch masks (Sec. 7), FP64.
//
// Working storage (device workspace, column major): W (m x np) starts as the
// pre-scaled A, V (np x np) as I; np = l nb with l even.  A sweep is l - 1
// round-robin iterations (Sec. 4.1) over block columns; each iteration is one
// launch of blk_iter with one workgroup per (block pair, matrix):
//   1. G = [W_p W_q]^T [W_p W_q] (2nb x 2nb) on the FP64 matrix cores,
//      streaming the pair's rows through LDS in chunks of 64 rows;
//   2. one sweep of the two-sided Jacobi eigensolver (Alg. 1) on G in LDS, in
//      round-robin order over the 2nb indices, accumulating J;
//   3. [W_p W_q] <- [W_p W_q] J and [V_p V_q] <- [V_p V_q] J on the matrix
//      cores, reading every element once and writing it once.
// A matrix whose inner solves applied no rotation during a whole sweep has
// orthogonal columns: it is retired (masked) by blk_sweep_end and skipped by
// every later launch.  blk_finalize forms sigma, U and the sorted outputs.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "launchers.hpp"

namespace svdb {

namespace {

typedef double double4v __attribute__((ext_vector_type(4)));

constexpr int kBT = 256;   // threads per workgroup
constexpr int kCH = 64;    // rows per streamed chunk

// per-matrix state in the workspace
struct BlkState {
    int active;      // 1 while sweeps continue
    int rotated;     // any inner rotation in the current sweep
    int sweeps;
    int bad;         // non-finite input
    double scale;    // power-of-two pre-scaling of A
};

__global__ __launch_bounds__(kBT) void blk_init_d(int m, int n, int np, const double *__restrict__ A,
                                                  int lda, long long sA, double *W, double *Vw,
                                                  BlkState *st)
{
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ double s_max[kBT / 64];
    __shared__ int s_bad[kBT / 64];
    A += (size_t)b * sA;
    W += (size_t)b * m * np;
    Vw += (size_t)b * np * np;
    double amax = 0.0;
    int bad = 0;
    for (int c = wave; c < n; c += kBT / 64)
        for (int r = lane; r < m; r += 64) {
            const double a = A[(size_t)c * lda + r];
            bad |= !isfinite(a);
            amax = fmax(amax, fabs(a));
        }
    amax = wave_max(amax);
    bad = __any(bad);
    if (lane == 0) {
        s_max[wave] = amax;
        s_bad[wave] = bad;
    }
    __syncthreads();
    amax = s_max[0];
    bad = s_bad[0];
    for (int w = 1; w < kBT / 64; w++) {
        amax = fmax(amax, s_max[w]);
        bad |= s_bad[w];
    }
    const double scale = pow2_scale(amax);
    for (int c = wave; c < np; c += kBT / 64)
        for (int r = lane; r < m; r += 64)
            W[(size_t)c * m + r] = (c < n && !bad) ? A[(size_t)c * lda + r] * scale : 0.0;
    for (size_t idx = tid; idx < (size_t)np * np; idx += kBT)
        Vw[idx] = (idx % (np + 1) == 0) ? 1.0 : 0.0;
    if (tid == 0) {
        st[b].active = bad ? 0 : 1;
        st[b].rotated = 0;
        st[b].sweeps = 0;
        st[b].bad = bad;
        st[b].scale = scale;
    }
}

// FP64 MFMA 16x16x4: A operand lane l = (row l%16, k l/16), B operand lane
// l = (k l/16, col l%16); result register v of lane l holds row 4 v + l/16,
// column l%16 (checked on gfx950 with single-entry operands).
__device__ __forceinline__ double4v mfma16x16x4(double a, double b, double4v c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NB>
struct IterShared {
    static constexpr int N2 = 2 * NB;
    double xs[N2][kCH + 1];     // row chunk of [X_p X_q], column major, padded
    double G[N2][N2 + 1];       // Gram matrix, G[row][col]
    double J[N2][N2 + 1];       // accumulated rotation, J[row][col]
    double2 cs[NB];             // (c, e s) of the pairs of an inner iteration
    int rot;
};

// Loads rows [r0, r0 + kCH) of the 2nb columns (col(c) maps local to global
// column) of the rows x np matrix X into s.xs (zero beyond `rows`).
template <int NB>
__device__ __forceinline__ void load_chunk(IterShared<NB> &s, const double *X, int rows, int r0,
                                           int p, int q)
{
    constexpr int N2 = 2 * NB;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < N2 * kCH; idx += kBT) {
        const int c = idx / kCH, r = idx % kCH;
        const int gc = c < NB ? p * NB + c : q * NB + (c - NB);
        const int gr = r0 + r;
        s.xs[c][r] = gr < rows ? X[(size_t)gc * rows + gr] : 0.0;
    }
}

// X_chunk (kCH x 2nb) <- X_chunk J, written back to global rows [r0, r0+kCH).
template <int NB>
__device__ __forceinline__ void update_chunk(IterShared<NB> &s, double *X, int rows, int r0, int p,
                                             int q)
{
    constexpr int N2 = 2 * NB;
    constexpr int TR = kCH / 16, TC = N2 / 16, TILES = TR * TC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    for (int tile = wave; tile < TILES; tile += kBT / 64) {
        const int ti = tile / TC, tj = tile % TC;
        double4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < N2; k0 += 4) {
            const double a = s.xs[k0 + lk][16 * ti + li];      // X[r][k]
            const double bb = s.J[k0 + lk][16 * tj + li];       // J[k][c]
            acc = mfma16x16x4(a, bb, acc);
        }
        const int c = 16 * tj + li;
        const int gc = c < NB ? p * NB + c : q * NB + (c - NB);
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int gr = r0 + 16 * ti + 4 * v + lk;
            if (gr < rows) X[(size_t)gc * rows + gr] = acc[v];
        }
    }
}

template <int NB>
__global__ __launch_bounds__(kBT) void blk_iter_d(int m, int np, int l, int it, double *W,
                                                  double *Vw, BlkState *st, double tol)
{
    constexpr int N2 = 2 * NB;
    constexpr int TC = N2 / 16, GT = TC * TC;   // Gram output tiles
    constexpr int GPW = (GT + 3) / 4;           // tiles per wave
    __shared__ IterShared<NB> s;

    const int b = blockIdx.x / (l / 2), pair = blockIdx.x % (l / 2);
    if (!st[b].active) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    int p, q;
    rr_pair(l, it, pair, p, q);
    W += (size_t)b * m * np;
    Vw += (size_t)b * np * np;

    // ---- 1. Gram matrix on the matrix cores --------------------------------
    double4v acc[GPW];
#pragma unroll
    for (int g = 0; g < GPW; g++) acc[g] = double4v{0.0, 0.0, 0.0, 0.0};
    for (int r0 = 0; r0 < m; r0 += kCH) {
        __syncthreads();
        load_chunk<NB>(s, W, m, r0, p, q);
        __syncthreads();
#pragma unroll
        for (int g = 0; g < GPW; g++) {
            const int tile = wave + 4 * g;
            if (tile < GT) {
                const int ti = tile / TC, tj = tile % TC;
#pragma unroll
                for (int k0 = 0; k0 < kCH; k0 += 4) {
                    const double a = s.xs[16 * ti + li][k0 + lk];   // X^T[i][k] = X[k][i]
                    const double bb = s.xs[16 * tj + li][k0 + lk];  // X[k][j]
                    acc[g] = mfma16x16x4(a, bb, acc[g]);
                }
            }
        }
    }
#pragma unroll
    for (int g = 0; g < GPW; g++) {
        const int tile = wave + 4 * g;
        if (tile < GT) {
            const int ti = tile / TC, tj = tile % TC;
#pragma unroll
            for (int v = 0; v < 4; v++) s.G[16 * ti + 4 * v + lk][16 * tj + li] = acc[g][v];
        }
    }
    for (int idx = tid; idx < N2 * N2; idx += kBT) s.J[idx / N2][idx % N2] = (idx / N2 == idx % N2);
    if (tid == 0) s.rot = 0;
    __syncthreads();

    // ---- 2. one inner sweep of Alg. 1 on G, round-robin over 2nb indices ---
    for (int r = 0; r < N2 - 1; r++) {
        if (tid < NB) {
            int i, j;
            rr_pair(N2, r, tid, i, j);
            const double gii = s.G[i][i], gjj = s.G[j][j], gij = s.G[i][j];
            double c = 1.0, es = 0.0;
            const double ag = fabs(gij);
            if (gij != 0.0 && ag >= tol * sqrt(fabs(gii)) * sqrt(fabs(gjj))) {
                double sn;
                jacobi_cs(gii, gjj, ag, c, sn);
                es = gij > 0.0 ? sn : -sn;
                s.rot = 1;
            }
            s.cs[tid] = make_double2(c, es);
        }
        __syncthreads();
        // G <- J_r^T G J_r on 2x2 blocks {i_a, j_a} x {i_b, j_b}; J <- J J_r
        for (int idx = tid; idx < NB * NB; idx += kBT) {
            const int ka = idx / NB, kb = idx % NB;
            int ia, ja, ib, jb;
            rr_pair(N2, r, ka, ia, ja);
            rr_pair(N2, r, kb, ib, jb);
            const double2 ra = s.cs[ka], rb = s.cs[kb];
            // column i' = c col_i + es col_j, column j' = -es col_i + c col_j
            const double g00 = s.G[ia][ib], g01 = s.G[ia][jb];
            const double g10 = s.G[ja][ib], g11 = s.G[ja][jb];
            // right multiplication by the rotation of pair kb
            const double h00 = rb.x * g00 + rb.y * g01, h01 = -rb.y * g00 + rb.x * g01;
            const double h10 = rb.x * g10 + rb.y * g11, h11 = -rb.y * g10 + rb.x * g11;
            // left multiplication by the transpose of the rotation of pair ka
            s.G[ia][ib] = ra.x * h00 + ra.y * h10;
            s.G[ia][jb] = ra.x * h01 + ra.y * h11;
            s.G[ja][ib] = -ra.y * h00 + ra.x * h10;
            s.G[ja][jb] = -ra.y * h01 + ra.x * h11;
        }
        for (int idx = tid; idx < N2 * NB; idx += kBT) {
            const int row = idx / NB, kb = idx % NB;
            int ib, jb;
            rr_pair(N2, r, kb, ib, jb);
            const double2 rb = s.cs[kb];
            const double x = s.J[row][ib], y = s.J[row][jb];
            s.J[row][ib] = rb.x * x + rb.y * y;
            s.J[row][jb] = -rb.y * x + rb.x * y;
        }
        __syncthreads();
    }

    // ---- 3. fused update of the block columns of W and V --------------------
    const bool any = s.rot != 0;
    if (any) {
        for (int r0 = 0; r0 < m; r0 += kCH) {
            __syncthreads();
            load_chunk<NB>(s, W, m, r0, p, q);
            __syncthreads();
            update_chunk<NB>(s, W, m, r0, p, q);
        }
        for (int r0 = 0; r0 < np; r0 += kCH) {
            __syncthreads();
            load_chunk<NB>(s, Vw, np, r0, p, q);
            __syncthreads();
            update_chunk<NB>(s, Vw, np, r0, p, q);
        }
        if (tid == 0) atomicOr(&st[b].rotated, 1);
    }
}

__global__ void blk_sweep_end(int batch, BlkState *st, int *active_count)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    if (st[b].active) {
        st[b].sweeps += 1;
        if (!st[b].rotated) st[b].active = 0;
        st[b].rotated = 0;
        if (st[b].active) atomicAdd(active_count, 1);
    }
}

__global__ __launch_bounds__(kBT) void blk_finalize_d(int m, int n, int np, const double *W,
                                                      const double *Vw, const BlkState *st,
                                                      double *S, long long sS, double *U, int ldu,
                                                      long long sU, double *V, int ldv,
                                                      long long sV, int *info, int *sweeps_out)
{
    extern __shared__ double dyn[];
    double *sig = dyn;                     // n
    int *rank = (int *)(sig + n);          // n
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const BlkState sb = st[b];
    if (sb.bad) {
        if (tid == 0) {
            info[b] = 2;
            if (sweeps_out) sweeps_out[b] = 0;
        }
        return;
    }
    W += (size_t)b * m * np;
    Vw += (size_t)b * np * np;
    S += (size_t)b * sS;
    if (U) U += (size_t)b * sU;
    if (V) V += (size_t)b * sV;
    for (int c = wave; c < n; c += kBT / 64) {
        const double *w = W + (size_t)c * m;
        double mx = 0.0;
        for (int r = lane; r < m; r += 64) mx = fmax(mx, fabs(w[r]));
        mx = wave_max(mx);
        double ss = 0.0;
        if (mx > 0.0) {
            const double sc = ldexp(1.0, -ilogb(mx));
            for (int r = lane; r < m; r += 64) {
                const double y = w[r] * sc;
                ss += y * y;
            }
        }
        ss = wave_sum(ss);
        if (lane == 0) sig[c] = mx > 0.0 ? ldexp(sqrt(ss), ilogb(mx)) : 0.0;
    }
    __syncthreads();
    for (int c = tid; c < n; c += kBT) {
        const double sc = sig[c];
        int rk = 0;
        for (int j = 0; j < n; j++) {
            const double sj = sig[j];
            rk += (sj > sc) || (sj == sc && j < c);
        }
        rank[c] = rk;
    }
    __syncthreads();
    for (int c = wave; c < n; c += kBT / 64) {
        const int rk = rank[c];
        const double sc = sig[c];
        if (lane == 0) S[rk] = sc / sb.scale;
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        if (U)
            for (int r = lane; r < m; r += 64) U[(size_t)rk * ldu + r] = W[(size_t)c * m + r] * inv;
        if (V)
            for (int r = lane; r < n; r += 64) V[(size_t)rk * ldv + r] = Vw[(size_t)c * np + r];
    }
    // sigma = 0: complete U by Gram-Schmidt on e_1, e_2, ... (wave 0, global U)
    bool any_zero = false;
    for (int c = 0; c < n; c++) any_zero |= !(sig[c] > 0.0);
    if (U && any_zero) {
        __threadfence();
        __syncthreads();
        if (wave == 0) {
            int cand = 0;
            for (int i = 0; i < n; i++) {
                if (sig[i] > 0.0) continue;
                double *u = U + (size_t)rank[i] * ldu;
                for (; cand < m; cand++) {
                    for (int r = lane; r < m; r += 64) u[r] = (r == cand) ? 1.0 : 0.0;
                    __threadfence();
                    for (int pass = 0; pass < 2; pass++)
                        for (int j = 0; j < n; j++) {
                            if (j == i || (sig[j] == 0.0 && j > i)) continue;
                            const double *qv = U + (size_t)rank[j] * ldu;
                            double d = 0.0;
                            for (int r = lane; r < m; r += 64) d += qv[r] * u[r];
                            d = wave_sum(d);
                            for (int r = lane; r < m; r += 64) u[r] -= d * qv[r];
                            __threadfence();
                        }
                    double nu = 0.0;
                    for (int r = lane; r < m; r += 64) nu += u[r] * u[r];
                    nu = sqrt(wave_sum(nu));
                    if (nu > 0.5) {
                        const double inv = 1.0 / nu;
                        for (int r = lane; r < m; r += 64) u[r] *= inv;
                        __threadfence();
                        cand++;
                        break;
                    }
                }
            }
        }
    }
    if (tid == 0) {
        info[b] = sb.active ? 1 : 0;
        if (sweeps_out) sweeps_out[b] = sb.sweeps;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int blocked_nb(int m, int n, int nb)
{
    if (nb == 16 || nb == 32) return nb;
    if (nb != 0) return 0;
    return n <= 96 ? 16 : 32;
}

int blocked_np(int n, int nb)
{
    int l = (n + nb - 1) / nb;
    if (l & 1) l++;
    if (l < 2) l = 2;
    return l * nb;
}

size_t blocked_workspace_bytes(int batch, int m, int n, int nb)
{
    const int np = blocked_np(n, nb);
    return align256((size_t)batch * m * np * sizeof(double)) +
           align256((size_t)batch * np * np * sizeof(double)) +
           align256((size_t)batch * sizeof(BlkState)) + 256;
}

hipError_t launch_blocked_d(int batch, int m, int n, int nb, const double *A, int lda, long long sA,
                            double *S, long long sS, double *U, int ldu, long long sU, double *V,
                            int ldv, long long sV, double tol, int max_sweeps, int *info,
                            int *sweeps, void *ws, hipStream_t stream)
{
    const int np = blocked_np(n, nb);
    const int l = np / nb;
    char *p = (char *)ws;
    double *W = (double *)p;
    p += align256((size_t)batch * m * np * sizeof(double));
    double *Vw = (double *)p;
    p += align256((size_t)batch * np * np * sizeof(double));
    BlkState *st = (BlkState *)p;
    p += align256((size_t)batch * sizeof(BlkState));
    int *count = (int *)p;

    hipLaunchKernelGGL(blk_init_d, dim3(batch), dim3(kBT), 0, stream, m, n, np, A, lda, sA, W, Vw,
                       st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // pinned word for the number of matrices still active after a sweep;
    // allocated once per process and host thread
    static thread_local int *host_count = nullptr;
    if (!host_count) {
        e = hipHostMalloc((void **)&host_count, sizeof(int), hipHostMallocDefault);
        if (e != hipSuccess) return e;
    }
    const unsigned grid = (unsigned)batch * (unsigned)(l / 2);
    for (int sw = 0; sw < max_sweeps; sw++) {
        for (int it = 0; it < l - 1; it++) {
            if (nb == 16)
                hipLaunchKernelGGL(blk_iter_d<16>, dim3(grid), dim3(kBT), 0, stream, m, np, l, it,
                                   W, Vw, st, tol);
            else
                hipLaunchKernelGGL(blk_iter_d<32>, dim3(grid), dim3(kBT), 0, stream, m, np, l, it,
                                   W, Vw, st, tol);
        }
        e = hipMemsetAsync(count, 0, sizeof(int), stream);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(blk_sweep_end, dim3((batch + 255) / 256), dim3(256), 0, stream, batch, st,
                           count);
        e = hipMemcpyAsync(host_count, count, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) break;
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) break;
        if (*host_count == 0) break;
    }
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)n * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL(blk_finalize_d, dim3(batch), dim3(kBT), lds, stream, m, n, np, W, Vw, st, S, sS,
                       U, ldu, sU, V, ldv, sV, info, sweeps);
    return hipGetLastError();
}

}  // namespace svdb
