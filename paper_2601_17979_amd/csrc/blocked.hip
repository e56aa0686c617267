// blocked.hip -- the block one-sided Jacobi SVD (Sec. 3, eq. block-gram and
// eq. right-sv) with a one-sweep inner eigensolver (Sec. 5, "Design 2"),
// fused vector updates (Sec. 6) and batch masks (Sec. 7), in FP64 or FP32
// working precision, plus the mixed mode (FP32 sweeps, FP64 refinement).
//
// Working storage (device workspace, column major): W (m x np) starts as the
// pre-scaled A, V (np x np) as I; np = l nb with l even.  A sweep is l - 1
// round-robin iterations (Sec. 4.1) over block columns; each iteration is one
// launch of blk_iter with one workgroup per (block pair, matrix):
//   1. G = [W_p W_q]^T [W_p W_q] (2nb x 2nb) on the matrix cores (FP64 MFMA,
//      or FP32 MFMA with FP32 accumulation), streaming the pair's rows
//      through LDS in chunks of 64 rows;
//   2. one sweep of the two-sided Jacobi eigensolver (Alg. 1) on G in LDS,
//      always in FP64, in round-robin order over the 2nb indices,
//      accumulating J;
//   3. [W_p W_q] <- [W_p W_q] J and [V_p V_q] <- [V_p V_q] J on the matrix
//      cores, reading every element once and writing it once.
// A matrix whose inner solves applied no rotation during a whole sweep has
// orthogonal columns.  With masking (Sec. 7) it is retired at once and
// skipped by every later launch; without, it keeps being swept until the
// whole batch has converged.  blk_finalize forms sigma (FP64 sums), U and the
// sorted outputs.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "launchers.hpp"

namespace svdb {

namespace {

typedef double double4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kBT = 256;   // threads per workgroup
constexpr int kCH = 64;    // rows per streamed chunk

// The FP32 phase of the mixed mode ends once the largest pair cosine of a
// sweep is below this and no longer halves from sweep to sweep: FP32
// rounding then dominates what is left.
constexpr double kStallCos = 0x1p-10;

// per-matrix state in the workspace
struct BlkState {
    int active;                  // swept by the next launches
    int rotated;                 // an inner rotation happened in this sweep
    int sweeps;                  // sweeps until convergence
    int bad;                     // non-finite input
    int done;                    // converged (or, FP32 phase: stalled)
    int pad;
    double scale;                // power-of-two pre-scaling of A
    unsigned long long maxcos;   // bits of the largest pair cosine this sweep
    double prevcos;              // the previous sweep's
};

// 16x16x4 matrix-core products.  Operands: lane l supplies A[l%16][l/16]
// and B[l/16][l%16].  Result register v of lane l holds row
// Mfma<T>::row(l, v), column l%16; the FP64 and FP32 instructions differ
// here (both checked on gfx950 with single-entry operands).
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
    using acc_t = double4v;
    __device__ static acc_t op(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int l, int v) { return 4 * v + (l >> 4); }
};
template <>
struct Mfma<float> {
    using acc_t = float4v;
    __device__ static acc_t op(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};

__device__ __forceinline__ void state_reset(BlkState &s, int bad)
{
    s.active = bad ? 0 : 1;
    s.rotated = 0;
    s.sweeps = 0;
    s.bad = bad;
    s.done = 0;
    s.maxcos = 0ull;
    s.prevcos = __builtin_inf();
}

// W <- scale * A (zero columns beyond n), V <- I; non-finite input marks the
// matrix bad.  TA: element type of A, T: working type.
template <class TA, class T>
__global__ __launch_bounds__(kBT) void blk_init(int m, int n, int np, const TA *__restrict__ A,
                                                int lda, long long sA, T *W, T *Vw, BlkState *st)
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
            const double a = (double)A[(size_t)c * lda + r];
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
            W[(size_t)c * m + r] =
                (c < n && !bad) ? (T)((double)A[(size_t)c * lda + r] * scale) : T(0);
    for (size_t idx = tid; idx < (size_t)np * np; idx += kBT)
        Vw[idx] = (idx % (np + 1) == 0) ? T(1) : T(0);
    if (tid == 0) {
        state_reset(st[b], bad);
        st[b].scale = scale;
    }
}

template <class T, int NB>
struct IterShared {
    static constexpr int N2 = 2 * NB;
    static constexpr bool kF64 = std::is_same<T, double>::value;
    struct Streaming {                       // live while W or V stream through
        T xs[N2][kCH + 1];                   // row chunk of [X_p X_q], column major
        T Jw[kF64 ? 1 : N2][N2 + 1];         // J rounded to T (FP32 working precision)
    };
    union {
        double G[N2][N2 + 1];                // Gram matrix during the inner solve
        Streaming io;
    } u;
    double J[N2][N2 + 1];                    // accumulated rotation, J[row][col]
    double2 cs[NB];                          // (c, e s) of the pairs of an inner iteration
    int rot;
};

// Per-thread share of one chunk (kCH rows x 2nb columns) held in registers so
// that the next chunk's global loads overlap the current chunk's MFMAs.
template <class T, int NB>
struct ChunkRegs {
    static constexpr int E = 2 * NB * kCH / kBT;
    T v[E];
};

// Loads rows [r0, r0 + kCH) of block columns p, q of the rows x np matrix X
// (zero beyond `rows`).  Element e of thread t is chunk entry
// idx = t + e kBT: column idx / kCH, row idx % kCH (coalesced columns).
template <class T, int NB>
__device__ __forceinline__ void chunk_load(ChunkRegs<T, NB> &R, const T *X, int rows, int r0,
                                           int p, int q)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int e = 0; e < ChunkRegs<T, NB>::E; e++) {
        const int idx = tid + e * kBT;
        const int c = idx / kCH, r = idx % kCH;
        const int gc = c < NB ? p * NB + c : q * NB + (c - NB);
        const int gr = r0 + r;
        R.v[e] = gr < rows ? X[(size_t)gc * rows + gr] : T(0);
    }
}

template <class T, int NB>
__device__ __forceinline__ void chunk_to_lds(IterShared<T, NB> &s, const ChunkRegs<T, NB> &R)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int e = 0; e < ChunkRegs<T, NB>::E; e++) {
        const int idx = tid + e * kBT;
        s.u.io.xs[idx / kCH][idx % kCH] = R.v[e];
    }
}

// Stores the chunk held in s.u.io.xs to rows [r0, r0 + kCH) of X.
template <class T, int NB>
__device__ __forceinline__ void chunk_store(const IterShared<T, NB> &s, T *X, int rows, int r0,
                                            int p, int q)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int e = 0; e < ChunkRegs<T, NB>::E; e++) {
        const int idx = tid + e * kBT;
        const int c = idx / kCH, r = idx % kCH;
        const int gc = c < NB ? p * NB + c : q * NB + (c - NB);
        if (r0 + r < rows) X[(size_t)gc * rows + r0 + r] = s.u.io.xs[c][r];
    }
}

// [X_p X_q] <- [X_p X_q] J for a rows x np matrix X, chunk by chunk: MFMA
// tiles of 16 x 16 from the chunk in LDS and J, results staged back through
// LDS and written with coalesced stores.
template <class T, int NB>
__device__ __forceinline__ void update_block_columns(IterShared<T, NB> &s, T *X, int rows, int p,
                                                     int q)
{
    constexpr int N2 = 2 * NB;
    constexpr int TR = kCH / 16, TC = N2 / 16, TILES = TR * TC, TPW = TILES / 4;
    static_assert(TILES % 4 == 0, "tiles per wave");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    ChunkRegs<T, NB> R;
    chunk_load<T, NB>(R, X, rows, 0, p, q);
    for (int r0 = 0; r0 < rows; r0 += kCH) {
        __syncthreads();                      // xs free (previous chunk stored)
        chunk_to_lds<T, NB>(s, R);
        __syncthreads();
        if (r0 + kCH < rows) chunk_load<T, NB>(R, X, rows, r0 + kCH, p, q);
        typename Mfma<T>::acc_t acc[TPW];
#pragma unroll
        for (int u = 0; u < TPW; u++) {
            const int tile = wave + 4 * u;
            const int ti = tile % TR, tj = tile / TR;
            acc[u] = typename Mfma<T>::acc_t{0, 0, 0, 0};
#pragma unroll
            for (int k0 = 0; k0 < N2; k0 += 4) {
                const T a = s.u.io.xs[k0 + lk][16 * ti + li];   // X[r][k]
                T bb;                                           // J[k][c]
                if constexpr (IterShared<T, NB>::kF64)
                    bb = s.J[k0 + lk][16 * tj + li];
                else
                    bb = s.u.io.Jw[k0 + lk][16 * tj + li];
                acc[u] = Mfma<T>::op(a, bb, acc[u]);
            }
        }
        __syncthreads();                      // every wave has read xs
#pragma unroll
        for (int u = 0; u < TPW; u++) {
            const int tile = wave + 4 * u;
            const int ti = tile % TR, tj = tile / TR;
#pragma unroll
            for (int v = 0; v < 4; v++)
                s.u.io.xs[16 * tj + li][16 * ti + Mfma<T>::row(lane, v)] = acc[u][v];
        }
        __syncthreads();
        chunk_store<T, NB>(s, X, rows, r0, p, q);
    }
}

template <class T, int NB>
__global__ __launch_bounds__(kBT) void blk_iter(int m, int np, int l, int it, T *W, T *Vw,
                                                BlkState *st, double tol)
{
    constexpr int N2 = 2 * NB;
    constexpr int TC = N2 / 16, GT = TC * TC;   // Gram output tiles
    constexpr int GPW = (GT + 3) / 4;           // tiles per wave
    __shared__ IterShared<T, NB> s;

    const int b = blockIdx.x / (l / 2), pair = blockIdx.x % (l / 2);
    if (!st[b].active) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    int p, q;
    rr_pair(l, it, pair, p, q);
    W += (size_t)b * m * np;
    Vw += (size_t)b * np * np;

    // ---- 1. Gram matrix on the matrix cores --------------------------------
    typename Mfma<T>::acc_t acc[GPW];
#pragma unroll
    for (int g = 0; g < GPW; g++) acc[g] = typename Mfma<T>::acc_t{0, 0, 0, 0};
    {
        ChunkRegs<T, NB> R;
        chunk_load<T, NB>(R, W, m, 0, p, q);
        for (int r0 = 0; r0 < m; r0 += kCH) {
            __syncthreads();
            chunk_to_lds<T, NB>(s, R);
            __syncthreads();
            if (r0 + kCH < m) chunk_load<T, NB>(R, W, m, r0 + kCH, p, q);
#pragma unroll
            for (int g = 0; g < GPW; g++) {
                const int tile = wave + 4 * g;
                if (tile < GT) {
                    const int ti = tile / TC, tj = tile % TC;
#pragma unroll
                    for (int k0 = 0; k0 < kCH; k0 += 4) {
                        const T a = s.u.io.xs[16 * ti + li][k0 + lk];    // X^T[i][k]
                        const T bb = s.u.io.xs[16 * tj + li][k0 + lk];   // X[k][j]
                        acc[g] = Mfma<T>::op(a, bb, acc[g]);
                    }
                }
            }
        }
    }
    __syncthreads();                            // xs is dead, G takes its place
#pragma unroll
    for (int g = 0; g < GPW; g++) {
        const int tile = wave + 4 * g;
        if (tile < GT) {
            const int ti = tile / TC, tj = tile % TC;
#pragma unroll
            for (int v = 0; v < 4; v++)
                s.u.G[16 * ti + Mfma<T>::row(lane, v)][16 * tj + li] = (double)acc[g][v];
        }
    }
    for (int idx = tid; idx < N2 * N2; idx += kBT) s.J[idx / N2][idx % N2] = (idx / N2 == idx % N2);
    if (tid == 0) s.rot = 0;
    __syncthreads();

    // ---- 2. one inner sweep of Alg. 1 on G (FP64), round robin -------------
    double mc = 0.0;   // largest pair cosine seen by this thread
    for (int r = 0; r < N2 - 1; r++) {
        if (tid < NB) {
            int i, j;
            rr_pair(N2, r, tid, i, j);
            const double gii = s.u.G[i][i], gjj = s.u.G[j][j], gij = s.u.G[i][j];
            double c = 1.0, es = 0.0;
            const double ag = fabs(gij);
            const double si = sqrt(fabs(gii)), sj = sqrt(fabs(gjj));
            const double den = si * sj;
            mc = fmax(mc, den > 0.0 ? ag / den : (ag != 0.0 ? 1.0 : 0.0));
            if (gij != 0.0 && ag >= tol * si * sj) {
                double sn;
                jacobi_cs(gii, gjj, ag, c, sn);
                es = gij > 0.0 ? sn : -sn;
                s.rot = 1;
            }
            s.cs[tid] = make_double2(c, es);
        }
        __syncthreads();
        // G <- J_r^T G J_r on the 2x2 blocks {i_a, j_a} x {i_b, j_b} with
        // ka <= kb (G stays symmetric: the block (kb, ka) is the transpose);
        // J <- J J_r.  The rotation of a pair maps column i to
        // c col_i + es col_j and column j to -es col_i + c col_j.
        for (int idx = tid; idx < NB * (NB + 1) / 2; idx += kBT) {
            // idx -> (ka, kb), ka <= kb, row-major over the upper triangle
            int ka = 0, rem = idx;
            while (rem >= NB - ka) {
                rem -= NB - ka;
                ka++;
            }
            const int kb = ka + rem;
            int ia, ja, ib, jb;
            rr_pair(N2, r, ka, ia, ja);
            rr_pair(N2, r, kb, ib, jb);
            const double2 ra = s.cs[ka], rb = s.cs[kb];
            const double g00 = s.u.G[ia][ib], g01 = s.u.G[ia][jb];
            const double g10 = s.u.G[ja][ib], g11 = s.u.G[ja][jb];
            const double h00 = rb.x * g00 + rb.y * g01, h01 = -rb.y * g00 + rb.x * g01;
            const double h10 = rb.x * g10 + rb.y * g11, h11 = -rb.y * g10 + rb.x * g11;
            const double n00 = ra.x * h00 + ra.y * h10, n01 = ra.x * h01 + ra.y * h11;
            const double n10 = -ra.y * h00 + ra.x * h10, n11 = -ra.y * h01 + ra.x * h11;
            s.u.G[ia][ib] = n00;
            s.u.G[ia][jb] = n01;
            s.u.G[ja][ib] = n10;
            s.u.G[ja][jb] = n11;
            if (ka != kb) {
                s.u.G[ib][ia] = n00;
                s.u.G[jb][ia] = n01;
                s.u.G[ib][ja] = n10;
                s.u.G[jb][ja] = n11;
            }
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
    if (wave == 0) {
        mc = wave_max(mc);
        if (lane == 0 && mc > 0.0)
            atomicMax(&st[b].maxcos, (unsigned long long)__double_as_longlong(mc));
    }

    // ---- 3. fused update of the block columns of W and V --------------------
    if (s.rot != 0) {
        __syncthreads();                        // G is dead, the chunk buffers take its place
        if constexpr (!IterShared<T, NB>::kF64) {
            for (int idx = tid; idx < N2 * N2; idx += kBT)
                s.u.io.Jw[idx / N2][idx % N2] = (T)s.J[idx / N2][idx % N2];
        }
        update_block_columns<T, NB>(s, W, m, p, q);
        update_block_columns<T, NB>(s, Vw, np, p, q);
        if (tid == 0) atomicOr(&st[b].rotated, 1);
    }
}

// End of a sweep: a matrix with no rotation is converged (done); with
// `stall` (FP32 phase of the mixed mode) one whose largest cosine is small
// and did not halve is done too.  With masking a done matrix is retired;
// without, every matrix stays active until the whole batch is done.
// *pending counts the matrices not done.
__global__ void blk_sweep_end(int batch, BlkState *st, int *pending, int masking, int stall)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    BlkState &s = st[b];
    if (!s.active) return;
    if (!s.done) {
        s.sweeps += 1;
        const double mc = __longlong_as_double((long long)s.maxcos);
        bool fin = !s.rotated;
        if (stall && mc <= kStallCos && mc > 0.5 * s.prevcos) fin = true;
        s.prevcos = mc;
        if (fin) s.done = 1;
    }
    s.rotated = 0;
    s.maxcos = 0ull;
    if (!s.done) atomicAdd(pending, 1);
    if (masking && s.done) s.active = 0;
}

// Mark every matrix with finite input active again (start of the FP64
// refinement); the FP32 phase's sweep count moves to sweeps32.
__global__ void blk_rearm(int batch, BlkState *st, int *sweeps32)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    sweeps32[b] = st[b].sweeps;
    state_reset(st[b], st[b].bad);
}

// sigma_c = ||w_c|| (FP64 sums, power-of-two scaling), stable descending
// rank, U = W diag(sigma)^-1 (sigma = 0: Gram-Schmidt completion), outputs
// permuted.  T: working type, TO: output type.
template <class T, class TO>
__global__ __launch_bounds__(kBT) void blk_finalize(int m, int n, int np, const T *W, const T *Vw,
                                                    const BlkState *st, const int *sweeps_extra,
                                                    TO *S, long long sS, TO *U, int ldu,
                                                    long long sU, TO *V, int ldv, long long sV,
                                                    int *info, int *sweeps_out)
{
    extern __shared__ double dyn[];
    double *sig = dyn;                     // n
    int *rank = (int *)(sig + n);          // n
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const BlkState sb = st[b];
    const int extra = sweeps_extra ? sweeps_extra[b] : 0;
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
        const T *w = W + (size_t)c * m;
        double mx = 0.0;
        for (int r = lane; r < m; r += 64) mx = fmax(mx, fabs((double)w[r]));
        mx = wave_max(mx);
        double ss = 0.0;
        if (mx > 0.0) {
            const double sc = ldexp(1.0, -ilogb(mx));
            for (int r = lane; r < m; r += 64) {
                const double y = (double)w[r] * sc;
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
        if (lane == 0) S[rk] = (TO)(sc / sb.scale);
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        if (U)
            for (int r = lane; r < m; r += 64)
                U[(size_t)rk * ldu + r] = (TO)((double)W[(size_t)c * m + r] * inv);
        if (V)
            for (int r = lane; r < n; r += 64)
                V[(size_t)rk * ldv + r] = (TO)Vw[(size_t)c * np + r];
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
                TO *u = U + (size_t)rank[i] * ldu;
                for (; cand < m; cand++) {
                    for (int r = lane; r < m; r += 64) u[r] = (r == cand) ? TO(1) : TO(0);
                    __threadfence();
                    for (int pass = 0; pass < 2; pass++)
                        for (int j = 0; j < n; j++) {
                            if (j == i || (sig[j] == 0.0 && j > i)) continue;
                            const TO *qv = U + (size_t)rank[j] * ldu;
                            double d = 0.0;
                            for (int r = lane; r < m; r += 64)
                                d += (double)qv[r] * (double)u[r];
                            d = wave_sum(d);
                            for (int r = lane; r < m; r += 64)
                                u[r] = (TO)((double)u[r] - d * (double)qv[r]);
                            __threadfence();
                        }
                    double nu = 0.0;
                    for (int r = lane; r < m; r += 64) nu += (double)u[r] * (double)u[r];
                    nu = sqrt(wave_sum(nu));
                    if (nu > 0.5) {
                        const double inv = 1.0 / nu;
                        for (int r = lane; r < m; r += 64) u[r] = (TO)((double)u[r] * inv);
                        __threadfence();
                        cand++;
                        break;
                    }
                }
            }
        }
    }
    if (tid == 0) {
        info[b] = sb.done ? 0 : 1;
        if (sweeps_out) sweeps_out[b] = sb.sweeps + extra;
    }
}

// ---------------------------------------------------------------------------
// Batched FP64 GEMM on the matrix cores, column major:
//   C = alpha_b op(A) B + beta D,  op(A) = A (M x K) or A^T (A is K x M),
// alpha_b = alpha * st[b].scale when st is given.  One 64 x 64 tile of C per
// workgroup (each wave four 16 x 16 tiles), K staged through LDS 16 at a
// time; workgroup x = b * tiles + tile.  C must not alias A, B or D.
// ---------------------------------------------------------------------------
template <bool TRANS_A>
__global__ __launch_bounds__(kBT) void gemm_f64(int M, int N, int K, double alpha,
                                                const BlkState *st, const double *A, int lda,
                                                long long sA, const double *B, int ldb,
                                                long long sB, double beta, const double *D,
                                                int ldd, long long sD, double *C, int ldc,
                                                long long sC)
{
    __shared__ double as[16][64 + 1];   // as[k][i] = op(A)[i][k]
    __shared__ double bs[16][64 + 1];   // bs[k][j] = B[k][j]
    const int tilesM = (M + 63) / 64, tilesN = (N + 63) / 64;
    const int b = blockIdx.x / (tilesM * tilesN), t = blockIdx.x % (tilesM * tilesN);
    const int bm = t % tilesM, bn = t / tilesM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    A += (size_t)b * sA;
    B += (size_t)b * sB;
    C += (size_t)b * sC;
    if (D) D += (size_t)b * sD;
    const double ab = st ? alpha * st[b].scale : alpha;
    double4v acc[4];
#pragma unroll
    for (int u = 0; u < 4; u++) acc[u] = double4v{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 16) {
        __syncthreads();
        for (int idx = tid; idx < 16 * 64; idx += kBT) {
            // op(A): consecutive threads read consecutive addresses
            int kk, ii;
            if (TRANS_A) {
                ii = idx / 16;
                kk = idx % 16;
            } else {
                kk = idx / 64;
                ii = idx % 64;
            }
            const int gi = 64 * bm + ii, gk = k0 + kk;
            double av = 0.0;
            if (gi < M && gk < K)
                av = TRANS_A ? A[(size_t)gi * lda + gk] : A[(size_t)gk * lda + gi];
            as[kk][ii] = av;
            // B: column j, 16 consecutive k
            const int jj = idx / 16, kb = idx % 16;
            const int gj = 64 * bn + jj, gkb = k0 + kb;
            bs[kb][jj] = (gj < N && gkb < K) ? B[(size_t)gj * ldb + gkb] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int tile = wave * 4 + u;   // 16 tiles of 16 x 16
            const int ti = tile / 4, tj = tile % 4;
#pragma unroll
            for (int kq = 0; kq < 16; kq += 4) {
                const double a = as[kq + lk][16 * ti + li];
                const double bb = bs[kq + lk][16 * tj + li];
                acc[u] = Mfma<double>::op(a, bb, acc[u]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int tile = wave * 4 + u;
        const int ti = tile / 4, tj = tile % 4;
        const int gj = 64 * bn + 16 * tj + li;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int gi = 64 * bm + 16 * ti + Mfma<double>::row(lane, v);
            if (gi < M && gj < N) {
                double y = ab * acc[u][v];
                if (D) y += beta * D[(size_t)gj * ldd + gi];
                C[(size_t)gj * ldc + gi] = y;
            }
        }
    }
}

// Q (n x n, ld n) <- leading n x n block of the FP32 V (np x np).
__global__ void v32_to_q(int batch, int n, int np, const float *V32, double *Q)
{
    const size_t total = (size_t)batch * n * n;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const size_t b = g / ((size_t)n * n);
        const int idx = (int)(g % ((size_t)n * n));
        Q[g] = (double)V32[b * np * np + (size_t)(idx / n) * np + idx % n];
    }
}

// V (np x np) <- [Q 0; 0 I]; columns n.. np-1 of W (m x np) <- 0.
__global__ void q_to_v(int batch, int m, int n, int np, const double *Q, double *Vw, double *W)
{
    const size_t vt = (size_t)np * np, wt = (size_t)m * (np - n);
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < (size_t)batch * vt;
         g += (size_t)gridDim.x * blockDim.x) {
        const size_t b = g / vt;
        const int idx = (int)(g % vt), c = idx / np, r = idx % np;
        Vw[g] = (c < n && r < n) ? Q[b * n * n + (size_t)c * n + r] : (r == c ? 1.0 : 0.0);
    }
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < (size_t)batch * wt;
         g += (size_t)gridDim.x * blockDim.x) {
        const size_t b = g / wt;
        W[b * m * np + (size_t)n * m + g % wt] = 0.0;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// pinned word that receives the number of pending matrices after a sweep;
// one per process and host thread
hipError_t pinned_counter(int **out)
{
    static thread_local int *host_count = nullptr;
    if (!host_count) {
        hipError_t e = hipHostMalloc((void **)&host_count, sizeof(int), hipHostMallocDefault);
        if (e != hipSuccess) return e;
    }
    *out = host_count;
    return hipSuccess;
}

// Sweeps until no matrix is pending or max_sweeps.
template <class T>
hipError_t run_sweeps(int batch, int m, int np, int nb, T *W, T *Vw, BlkState *st, int *pending,
                      double tol, int max_sweeps, int masking, int stall, hipStream_t stream)
{
    const int l = np / nb;
    int *host_count;
    hipError_t e = pinned_counter(&host_count);
    if (e != hipSuccess) return e;
    const unsigned grid = (unsigned)batch * (unsigned)(l / 2);
    for (int sw = 0; sw < max_sweeps; sw++) {
        for (int it = 0; it < l - 1; it++) {
            if (nb == 16)
                hipLaunchKernelGGL((blk_iter<T, 16>), dim3(grid), dim3(kBT), 0, stream, m, np, l,
                                   it, W, Vw, st, tol);
            else
                hipLaunchKernelGGL((blk_iter<T, 32>), dim3(grid), dim3(kBT), 0, stream, m, np, l,
                                   it, W, Vw, st, tol);
        }
        e = hipMemsetAsync(pending, 0, sizeof(int), stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(blk_sweep_end, dim3((batch + 255) / 256), dim3(256), 0, stream, batch,
                           st, pending, masking, stall);
        e = hipMemcpyAsync(host_count, pending, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        if (*host_count == 0) break;
    }
    return hipGetLastError();
}

// Workspace carving; the same order as blocked_workspace_bytes.
struct WsLayout {
    void *W, *Vw, *W32, *V32;
    double *Q, *X;
    BlkState *st;
    int *sw32, *pending;
};

WsLayout carve(void *ws, int batch, int m, int n, int np, size_t elt, bool mixed)
{
    WsLayout L{};
    char *p = (char *)ws;
    L.W = p;
    p += align256((size_t)batch * m * np * elt);
    L.Vw = p;
    p += align256((size_t)batch * np * np * elt);
    if (mixed) {
        L.W32 = p;
        p += align256((size_t)batch * m * np * sizeof(float));
        L.V32 = p;
        p += align256((size_t)batch * np * np * sizeof(float));
        L.Q = (double *)p;
        p += align256((size_t)batch * n * n * sizeof(double));
        L.X = (double *)p;
        p += align256((size_t)batch * n * n * sizeof(double));
    }
    L.st = (BlkState *)p;
    p += align256((size_t)batch * sizeof(BlkState));
    L.sw32 = (int *)p;
    p += align256((size_t)batch * sizeof(int));
    L.pending = (int *)p;
    return L;
}

unsigned elementwise_grid(size_t total)
{
    const size_t g = (total + 255) / 256;
    return (unsigned)(g < 65536 ? (g ? g : 1) : 65536);
}

template <class TA, class T>
hipError_t launch_blocked(int batch, int m, int n, int nb, const TA *A, int lda, long long sA, T *S,
                          long long sS, T *U, int ldu, long long sU, T *V, int ldv, long long sV,
                          double tol, int max_sweeps, int masking, int *info, int *sweeps,
                          void *ws, hipStream_t stream)
{
    const int np = blocked_np(n, nb);
    WsLayout L = carve(ws, batch, m, n, np, sizeof(T), false);
    T *W = (T *)L.W, *Vw = (T *)L.Vw;
    hipLaunchKernelGGL((blk_init<TA, T>), dim3(batch), dim3(kBT), 0, stream, m, n, np, A, lda, sA,
                       W, Vw, L.st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = run_sweeps<T>(batch, m, np, nb, W, Vw, L.st, L.pending, tol, max_sweeps, masking, 0,
                      stream);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)n * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL((blk_finalize<T, T>), dim3(batch), dim3(kBT), lds, stream, m, n, np, W, Vw,
                       L.st, (const int *)nullptr, S, sS, U, ldu, sU, V, ldv, sV, info, sweeps);
    return hipGetLastError();
}

}  // namespace

int blocked_nb(int m, int n, int nb)
{
    (void)m;
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

size_t blocked_workspace_bytes(int batch, int m, int n, int nb, int elt, bool mixed)
{
    const int np = blocked_np(n, nb);
    size_t s = align256((size_t)batch * m * np * elt) + align256((size_t)batch * np * np * elt);
    if (mixed)
        s += align256((size_t)batch * m * np * sizeof(float)) +
             align256((size_t)batch * np * np * sizeof(float)) +
             2 * align256((size_t)batch * n * n * sizeof(double));
    return s + align256((size_t)batch * sizeof(BlkState)) + align256((size_t)batch * sizeof(int)) +
           256;
}

hipError_t launch_blocked_d(int batch, int m, int n, int nb, const double *A, int lda, long long sA,
                            double *S, long long sS, double *U, int ldu, long long sU, double *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream)
{
    return launch_blocked<double, double>(batch, m, n, nb, A, lda, sA, S, sS, U, ldu, sU, V, ldv,
                                          sV, tol, max_sweeps, masking, info, sweeps, ws, stream);
}

hipError_t launch_blocked_s(int batch, int m, int n, int nb, const float *A, int lda, long long sA,
                            float *S, long long sS, float *U, int ldu, long long sU, float *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream)
{
    return launch_blocked<float, float>(batch, m, n, nb, A, lda, sA, S, sS, U, ldu, sU, V, ldv, sV,
                                        tol, max_sweeps, masking, info, sweeps, ws, stream);
}

// Mixed mode: FP32 sweeps (FP32 matrix cores, FP64 inner solves) with
// threshold tol32 until each matrix converges or stalls; then Q = orth(V32)
// in FP64 by two Newton-Schulz steps towards the polar factor,
// Q <- Q (3 I - Q^T Q) / 2; W = scale A Q, V = Q; FP64 sweeps to tol.
hipError_t launch_blocked_mixed_d(int batch, int m, int n, int nb, const double *A, int lda,
                                  long long sA, double *S, long long sS, double *U, int ldu,
                                  long long sU, double *V, int ldv, long long sV, double tol,
                                  double tol32, int max_sweeps, int masking, int *info,
                                  int *sweeps, void *ws, hipStream_t stream)
{
    const int np = blocked_np(n, nb);
    WsLayout L = carve(ws, batch, m, n, np, sizeof(double), true);
    double *W = (double *)L.W, *Vw = (double *)L.Vw;
    float *W32 = (float *)L.W32, *V32 = (float *)L.V32;
    hipLaunchKernelGGL((blk_init<double, float>), dim3(batch), dim3(kBT), 0, stream, m, n, np, A,
                       lda, sA, W32, V32, L.st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = run_sweeps<float>(batch, m, np, nb, W32, V32, L.st, L.pending, tol32, max_sweeps, 1, 1,
                          stream);
    if (e != hipSuccess) return e;

    // Newton-Schulz on Q; Q1 lives in the (not yet used) FP64 V area, ld n
    const long long nn = (long long)n * n, vv = (long long)np * np;
    double *Q0 = L.Q, *X = L.X, *Q1 = Vw;
    hipLaunchKernelGGL(v32_to_q, dim3(elementwise_grid((size_t)batch * nn)), dim3(256), 0, stream,
                       batch, n, np, V32, Q0);
    const int tn = (n + 63) / 64, tm = (m + 63) / 64;
    const dim3 gnn((unsigned)(batch * tn * tn));
    for (int step = 0; step < 2; step++) {
        const double *Qa = step == 0 ? Q0 : Q1;
        double *Qb = step == 0 ? Q1 : Q0;
        const long long sa = step == 0 ? nn : vv, sb = step == 0 ? vv : nn;
        // X = Qa^T Qa
        hipLaunchKernelGGL(gemm_f64<true>, gnn, dim3(kBT), 0, stream, n, n, n, 1.0,
                           (const BlkState *)nullptr, Qa, n, sa, Qa, n, sa, 0.0,
                           (const double *)nullptr, 0, 0LL, X, n, nn);
        // Qb = 1.5 Qa - 0.5 Qa X
        hipLaunchKernelGGL(gemm_f64<false>, gnn, dim3(kBT), 0, stream, n, n, n, -0.5,
                           (const BlkState *)nullptr, Qa, n, sa, (const double *)X, n, nn, 1.5, Qa,
                           n, sa, Qb, n, sb);
    }
    // V = [Q 0; 0 I], W[:, n:] = 0, W[:, :n] = scale A Q
    hipLaunchKernelGGL(q_to_v, dim3(elementwise_grid((size_t)batch * vv)), dim3(256), 0, stream,
                       batch, m, n, np, (const double *)Q0, Vw, W);
    hipLaunchKernelGGL(gemm_f64<false>, dim3((unsigned)(batch * tm * tn)), dim3(kBT), 0, stream, m,
                       n, n, 1.0, (const BlkState *)L.st, A, lda, sA, (const double *)Q0, n, nn,
                       0.0, (const double *)nullptr, 0, 0LL, W, m, (long long)m * np);
    hipLaunchKernelGGL(blk_rearm, dim3((batch + 255) / 256), dim3(256), 0, stream, batch, L.st,
                       L.sw32);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = run_sweeps<double>(batch, m, np, nb, W, Vw, L.st, L.pending, tol, max_sweeps, masking, 0,
                           stream);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)n * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL((blk_finalize<double, double>), dim3(batch), dim3(kBT), lds, stream, m, n,
                       np, (const double *)W, (const double *)Vw, L.st, (const int *)L.sw32, S, sS,
                       U, ldu, sU, V, ldv, sV, info, sweeps);
    return hipGetLastError();
}

}  // namespace svdb
