// blocked.hip -- the block one-sided Jacobi SVD (section "Algorithmic
// Background", eq. block-gram and eq. right-sv) with a one-sweep inner
// eigensolver ("Inexact Hermitian Eigendecomposition", Design 2), fused
// vector updates ("Optimized Vector Updates", Alg. 3) and batch masks
// ("Masked Batch Operations"), for real and
// complex matrices in FP64 or FP32 working precision, plus the mixed mode
// (FP32 sweeps, FP64 refinement) for real FP64 input.
//
// Working storage (device workspace, column major): W (m x np) starts as the
// pre-scaled A, V (np x np) as I; np = l nb with l even.  A sweep is l - 1
// round-robin iterations ("Parallel Ordering") over block columns; each iteration is one
// launch of blk_iter with one workgroup per (block pair, matrix):
//   1. G = [W_p W_q]^H [W_p W_q] (2nb x 2nb) on the matrix cores (FP64 MFMA,
//      or FP32 MFMA with FP32 accumulation), streaming the pair's rows
//      through LDS in chunks of 64 rows.  A complex chunk X = Xr + i Xi is
//      held as the real chunk [Xr Xi]; its real Gram matrix R gives
//      Re G = R_rr + R_ii and Im G = R_ri - R_ir;
//   2. one sweep of the two-sided Jacobi eigensolver (Alg. 1) on G in LDS,
//      always in FP64, in round-robin order over the 2nb indices,
//      accumulating J;
//   3. [W_p W_q] <- [W_p W_q] J and [V_p V_q] <- [V_p V_q] J on the matrix
//      cores (complex: [Xr Xi] [[Jr, Ji], [-Ji, Jr]]), reading every element
//      once and writing it once.
// A matrix whose inner solves applied no rotation during a whole sweep has
// orthogonal columns.  With masking ("Masked Batch Operations") it is retired at once and
// skipped by every later launch; without, it keeps being swept until the
// whole batch has converged.  blk_finalize forms sigma (FP64 sums), U and the
// sorted outputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "device_common.hpp"
#include "launchers.hpp"

namespace svdb {

namespace {

typedef double double4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kBT = 256;   // threads per workgroup
// rows per streamed chunk: 64, or 32 for complex data, whose real form is
// twice as wide (this keeps the workgroup's LDS within a third of a CU's)
template <bool CX>
constexpr int chunk_rows() { return CX ? 32 : 64; }
constexpr int kVbNb = 16;  // block width of uneven batches

// The FP32 phase of the mixed mode hands over to FP64 once the largest pair
// cosine of a sweep is at most kSwitchCos, or once it stalls: from sweep
// kStallSweeps on, a sweep whose largest cosine is more than half the
// previous one's.  FP32 sweeps cannot resolve directions whose singular
// values are below about u32 sigma_1; on such (ill-conditioned) matrices
// the cosine stops falling long before kSwitchCos, and the sweeps past the
// stall would be redone in FP64 anyway.
constexpr double kSwitchCos = 0x1p-7;
constexpr int kStallSweeps = 4;

__host__ __device__ __forceinline__ bool fp32_phase_done(double mc, double prev, int sweeps)
{
    return mc <= kSwitchCos || (sweeps >= kStallSweeps && mc > 0.5 * prev);
}

// A column whose squared norm is below kNegligible (a norm below 2^-480 of
// the pre-scaled matrix, whose largest entry is about 1) is never rotated,
// and a singular value below 2^-480 is taken as zero: rotating such columns
// only pushes rounding noise towards underflow (on exactly rank-deficient
// input the iteration would otherwise not stop).
constexpr double kNegligible = 0x1p-960;

// per-matrix state in the workspace
struct BlkState {
    int active;                  // swept by the next launches
    int rotated;                 // an inner rotation happened in this sweep
    int sweeps;                  // sweeps until convergence
    int bad;                     // non-finite input
    int done;                    // converged (FP32 phase: ready to switch)
    int pad;
    double scale;                // power-of-two pre-scaling of A
    unsigned long long maxcos;   // bits of the largest pair cosine this sweep
    double prevcos;              // the previous sweep's
};

// ---------------------------------------------------------------------------
// Element types: T real scalar of the working precision; E = T (real) or the
// two-component vector (re, im) of T (complex) as stored in HBM.
// ---------------------------------------------------------------------------
template <class T, bool CX>
struct Elem {
    using type = T;
};
template <>
struct Elem<double, true> {
    using type = double2;
};
template <>
struct Elem<float, true> {
    using type = float2;
};

template <class E>
struct EOps {   // real
    static constexpr bool cx = false;
    __device__ static double re(E x) { return (double)x; }
    __device__ static double im(E) { return 0.0; }
    __device__ static E make(double r, double) { return (E)r; }
};
template <>
struct EOps<double2> {
    static constexpr bool cx = true;
    __device__ static double re(double2 x) { return x.x; }
    __device__ static double im(double2 x) { return x.y; }
    __device__ static double2 make(double r, double i) { return make_double2(r, i); }
};
template <>
struct EOps<float2> {
    static constexpr bool cx = true;
    __device__ static double re(float2 x) { return (double)x.x; }
    __device__ static double im(float2 x) { return (double)x.y; }
    __device__ static float2 make(double r, double i) { return make_float2((float)r, (float)i); }
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
// matrix bad.  EA: element type of A, EW: working element type.  One
// workgroup, pointers of this matrix.
template <class EA, class EW>
__device__ __forceinline__ void init_body(int m, int n, int np, const EA *__restrict__ A, int lda,
                                          EW *W, EW *Vw, BlkState *stb, bool trans = false)
{
    // trans: A is the n x m matrix whose conjugate transpose is read, element
    // (r, c) being conj(A(c, r)) (wide inputs of the uneven batch)
    using OA = EOps<EA>;
    using OW = EOps<EW>;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ double s_max[kBT / 64];
    __shared__ int s_bad[kBT / 64];
    double amax = 0.0;
    int bad = 0;
    for (int c = wave; c < n; c += kBT / 64)
        for (int r = lane; r < m; r += 64) {
            const EA a = trans ? A[(size_t)r * lda + c] : A[(size_t)c * lda + r];
            const double ar = OA::re(a), ai = OA::im(a);
            bad |= !isfinite(ar) || !isfinite(ai);
            amax = fmax(amax, fmax(fabs(ar), fabs(ai)));
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
        for (int r = lane; r < m; r += 64) {
            EW w = OW::make(0.0, 0.0);
            if (c < n && !bad) {
                const EA a = trans ? A[(size_t)r * lda + c] : A[(size_t)c * lda + r];
                const double ai = trans ? -OA::im(a) : OA::im(a);
                w = OW::make(OA::re(a) * scale, ai * scale);
            }
            W[(size_t)c * m + r] = w;
        }
    for (size_t idx = tid; idx < (size_t)np * np; idx += kBT)
        Vw[idx] = OW::make((idx % (np + 1) == 0) ? 1.0 : 0.0, 0.0);
    if (tid == 0) {
        state_reset(*stb, bad);
        stb->scale = scale;
    }
}

template <class EA, class EW>
__global__ __launch_bounds__(kBT) void blk_init(int m, int n, int np, const EA *__restrict__ A,
                                                int lda, long long sA, EW *W, EW *Vw, BlkState *st)
{
    const int b = blockIdx.x;
    init_body<EA, EW>(m, n, np, A + (size_t)b * sA, lda, W + (size_t)b * m * np,
                      Vw + (size_t)b * np * np, st + b);
}

// ---------------------------------------------------------------------------
// LDS of one workgroup of blk_iter.  N2 = 2nb complex (or real) columns, NR
// real columns of the streamed chunk.  The chunk and the real Gram matrix
// share storage (never live together); a complex G has its own arrays.
// ---------------------------------------------------------------------------
// Inner sweeps of one block pair's solve: inner > 0 caps them at inner, < 0
// runs the solve to convergence (at most kInnerCap sweeps).  0 (auto), from
// measurements on MI355X: one sweep (Design 2) when the matrix has more than
// two block columns, where more inner sweeps barely lower the outer count;
// with two (l = 2: one pair, the whole matrix, per sweep) two sweeps, and
// for tall matrices (m >= 8 np), whose Gram and update passes dominate, the
// converged solve in FP64 and three sweeps in FP32.
constexpr int kInnerCap = 100;
__host__ __device__ inline int inner_sweeps_of(int inner, int l, int m, int np, bool fp32)
{
    if (inner > 0) return inner;
    if (inner < 0) return kInnerCap;
    if (l > 2) return 1;
    if (m >= 8 * np) return fp32 ? 3 : kInnerCap;
    return 2;
}

template <class T, bool CX, int NB>
struct IterShared {
    static constexpr int N2 = 2 * NB, NR = (CX ? 2 : 1) * N2, CH = chunk_rows<CX>();
    union {
        T xs[NR][CH + 1];             // row chunk [Xr (Xi)], column major
        double R[CX ? 1 : NR][CX ? 1 : NR + 1];   // real: the Gram matrix G itself
    } u;
    double Gr[CX ? N2 : 1][N2 + 1];   // complex G: real and imaginary parts
    double Gi[CX ? N2 : 1][N2 + 1];
    double Jr[N2][N2 + 1];            // accumulated rotation J[row][col]
    double Ji[CX ? N2 : 1][N2 + 1];
    double csc[NB];                   // c of the pairs of an inner iteration
    double cser[NB], csei[NB];        // e s (complex) or sign(g_ij) s
    unsigned char rr[N2 - 1][NB][2];  // inner round robin: pair k of round r
    int rot;
};

// The 2x2 blocks (ka, kb), ka <= kb, of the upper triangle of the NB x NB
// pair grid that thread tid updates in every round of an inner sweep (block
// idx = tid + t kBT, row-major; ka = -1 past the end), decoded once.
template <int NB>
struct InnerBlocks {
    static constexpr int NBLK = NB * (NB + 1) / 2, BPT = (NBLK + kBT - 1) / kBT;
    int ka[BPT], kb[BPT];
    __device__ __forceinline__ InnerBlocks(int tid)
    {
#pragma unroll
        for (int t = 0; t < BPT; t++) {
            const int idx = tid + t * kBT;
            int a = 0, rem = idx;
            while (rem >= NB - a && a < NB) {
                rem -= NB - a;
                a++;
            }
            ka[t] = idx < NBLK ? a : -1;
            kb[t] = a + rem;
        }
    }
};

// Per-thread share of one chunk (CH rows x 2nb columns) held in registers so
// that the next chunk's global loads overlap the current chunk's MFMAs.
template <class E, int NB>
struct ChunkRegs {
    static constexpr int CH = chunk_rows<EOps<E>::cx>();
    static constexpr int K = 2 * NB * CH / kBT;
    E v[K];
};

// Loads rows [r0, r0 + CH) of block columns p, q of the rows x np matrix X
// (zero beyond `rows`).  Element k of thread t is chunk entry
// idx = t + k kBT: column idx / CH, row idx % CH (coalesced columns).
template <class E, int NB>
__device__ __forceinline__ void chunk_load(ChunkRegs<E, NB> &Rg, const E *X, int rows, int r0,
                                           int p, int q)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < ChunkRegs<E, NB>::K; k++) {
        const int idx = tid + k * kBT;
        const int c = idx / ChunkRegs<E, NB>::CH, r = idx % ChunkRegs<E, NB>::CH;
        const int gc = c < NB ? p * NB + c : q * NB + (c - NB);
        const int gr = r0 + r;
        Rg.v[k] = gr < rows ? X[(size_t)gc * rows + gr] : EOps<E>::make(0.0, 0.0);
    }
}

template <class T, bool CX, int NB, class E>
__device__ __forceinline__ void chunk_to_lds(IterShared<T, CX, NB> &s, const ChunkRegs<E, NB> &Rg)
{
    constexpr int N2 = 2 * NB;
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < ChunkRegs<E, NB>::K; k++) {
        const int idx = tid + k * kBT;
        const int c = idx / ChunkRegs<E, NB>::CH, r = idx % ChunkRegs<E, NB>::CH;
        if constexpr (CX) {
            s.u.xs[c][r] = Rg.v[k].x;
            s.u.xs[c + N2][r] = Rg.v[k].y;
        } else {
            s.u.xs[c][r] = Rg.v[k];
        }
    }
}

// Stores the chunk held in s.u.xs to rows [r0, r0 + CH) of X.
template <class T, bool CX, int NB, class E>
__device__ __forceinline__ void chunk_store(const IterShared<T, CX, NB> &s, E *X, int rows, int r0,
                                            int p, int q)
{
    constexpr int N2 = 2 * NB;
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < ChunkRegs<E, NB>::K; k++) {
        const int idx = tid + k * kBT;
        const int c = idx / ChunkRegs<E, NB>::CH, r = idx % ChunkRegs<E, NB>::CH;
        const int gc = c < NB ? p * NB + c : q * NB + (c - NB);
        if (r0 + r < rows) {
            E y;
            if constexpr (CX) {
                y.x = s.u.xs[c][r];
                y.y = s.u.xs[c + N2][r];
            } else {
                y = s.u.xs[c][r];
            }
            X[(size_t)gc * rows + r0 + r] = y;
        }
    }
}

// Entry (k, c) of the real form of J: J itself (real), or
// [[Jr, Ji], [-Ji, Jr]] (complex), rounded to the working precision.
template <class T, bool CX, int NB>
__device__ __forceinline__ T jreal(const IterShared<T, CX, NB> &s, int k, int c)
{
    constexpr int N2 = 2 * NB;
    if constexpr (!CX) {
        return (T)s.Jr[k][c];
    } else {
        const bool top = k < N2, left = c < N2;
        const int kk = top ? k : k - N2, cc = left ? c : c - N2;
        if (top == left) return (T)s.Jr[kk][cc];
        const double v = s.Ji[kk][cc];
        return (T)(top ? v : -v);
    }
}

// [X_p X_q] <- [X_p X_q] J for a rows x np matrix X, chunk by chunk: MFMA
// tiles of 16 x 16 from the real chunk in LDS and the real form of J,
// results staged back through LDS and written with coalesced stores.
template <class T, bool CX, int NB, class E>
__device__ __forceinline__ void update_block_columns(IterShared<T, CX, NB> &s, E *X, int rows,
                                                     int p, int q)
{
    constexpr int NR = IterShared<T, CX, NB>::NR, CH = IterShared<T, CX, NB>::CH;
    constexpr int TR = CH / 16, TC = NR / 16, TILES = TR * TC, TPW = TILES / 4;
    static_assert(TILES % 4 == 0, "tiles per wave");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    ChunkRegs<E, NB> Rg;
    chunk_load<E, NB>(Rg, X, rows, 0, p, q);
    for (int r0 = 0; r0 < rows; r0 += CH) {
        __syncthreads();                      // xs free (previous chunk stored)
        chunk_to_lds<T, CX, NB, E>(s, Rg);
        __syncthreads();
        if (r0 + CH < rows) chunk_load<E, NB>(Rg, X, rows, r0 + CH, p, q);
        typename Mfma<T>::acc_t acc[TPW];
#pragma unroll
        for (int t = 0; t < TPW; t++) {
            const int tile = wave + 4 * t;
            const int ti = tile % TR, tj = tile / TR;
            acc[t] = typename Mfma<T>::acc_t{0, 0, 0, 0};
#pragma unroll
            for (int k0 = 0; k0 < NR; k0 += 4) {
                const T a = s.u.xs[k0 + lk][16 * ti + li];                 // X[r][k]
                const T bb = jreal<T, CX, NB>(s, k0 + lk, 16 * tj + li);    // J[k][c]
                acc[t] = Mfma<T>::op(a, bb, acc[t]);
            }
        }
        __syncthreads();                      // every wave has read xs
#pragma unroll
        for (int t = 0; t < TPW; t++) {
            const int tile = wave + 4 * t;
            const int ti = tile % TR, tj = tile / TR;
#pragma unroll
            for (int v = 0; v < 4; v++)
                s.u.xs[16 * tj + li][16 * ti + Mfma<T>::row(lane, v)] = acc[t][v];
        }
        __syncthreads();
        chunk_store<T, CX, NB, E>(s, X, rows, r0, p, q);
    }
}

// One inner sweep of Alg. 1 on the real symmetric G (in s.u.R), round robin
// over the 2nb indices, accumulating J.  Returns this thread's largest pair
// cosine.
template <class T, int NB>
__device__ __forceinline__ double inner_sweep_real(IterShared<T, false, NB> &s, double tol)
{
    constexpr int N2 = 2 * NB, JPT = (N2 * NB + kBT - 1) / kBT;
    const int tid = threadIdx.x;
    const InnerBlocks<NB> blk(tid);
    double mc = 0.0;
    for (int r = 0; r < N2 - 1; r++) {
        if (tid < NB) {
            const int i = s.rr[r][tid][0], j = s.rr[r][tid][1];
            const double gii = s.u.R[i][i], gjj = s.u.R[j][j], gij = s.u.R[i][j];
            double c = 1.0, es = 0.0;
            const double ag = fabs(gij);
            const double si = sqrt(fabs(gii)), sj = sqrt(fabs(gjj));
            const double den = si * sj;
            mc = fmax(mc, den > 0.0 ? ag / den : (ag != 0.0 ? 1.0 : 0.0));
            if (gij != 0.0 && gii >= kNegligible && gjj >= kNegligible && ag >= tol * si * sj) {
                double sn;
                jacobi_cs(gii, gjj, ag, c, sn);
                es = gij > 0.0 ? sn : -sn;
                s.rot = 1;
            }
            s.csc[tid] = c;
            s.cser[tid] = es;
        }
        __syncthreads();
        // G <- J_r^T G J_r on the 2x2 blocks {i_a, j_a} x {i_b, j_b} with
        // ka <= kb (G stays symmetric: the block (kb, ka) is the transpose);
        // J <- J J_r.  The rotation of a pair maps column i to
        // c col_i + es col_j and column j to -es col_i + c col_j.
#pragma unroll
        for (int t = 0; t < InnerBlocks<NB>::BPT; t++) {
            const int ka = blk.ka[t], kb = blk.kb[t];
            if (ka < 0) continue;
            const int ia = s.rr[r][ka][0], ja = s.rr[r][ka][1];
            const int ib = s.rr[r][kb][0], jb = s.rr[r][kb][1];
            const double ca = s.csc[ka], ea = s.cser[ka], cb = s.csc[kb], eb = s.cser[kb];
            const double g00 = s.u.R[ia][ib], g01 = s.u.R[ia][jb];
            const double g10 = s.u.R[ja][ib], g11 = s.u.R[ja][jb];
            const double h00 = cb * g00 + eb * g01, h01 = -eb * g00 + cb * g01;
            const double h10 = cb * g10 + eb * g11, h11 = -eb * g10 + cb * g11;
            const double n00 = ca * h00 + ea * h10, n01 = ca * h01 + ea * h11;
            const double n10 = -ea * h00 + ca * h10, n11 = -ea * h01 + ca * h11;
            s.u.R[ia][ib] = n00;
            s.u.R[ia][jb] = n01;
            s.u.R[ja][ib] = n10;
            s.u.R[ja][jb] = n11;
            if (ka != kb) {
                s.u.R[ib][ia] = n00;
                s.u.R[jb][ia] = n01;
                s.u.R[ib][ja] = n10;
                s.u.R[jb][ja] = n11;
            }
        }
#pragma unroll
        for (int t = 0; t < JPT; t++) {
            const int idx = tid + t * kBT;
            if (idx >= N2 * NB) break;
            const int row = idx / NB, kb = idx % NB;
            const int ib = s.rr[r][kb][0], jb = s.rr[r][kb][1];
            const double cb = s.csc[kb], eb = s.cser[kb];
            const double x = s.Jr[row][ib], y = s.Jr[row][jb];
            s.Jr[row][ib] = cb * x + eb * y;
            s.Jr[row][jb] = -eb * x + cb * y;
        }
        __syncthreads();
    }
    return mc;
}

// complex helpers (FP64)
struct cd {
    double r, i;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cd cmulc(cd a, cd b)   // a * conj(b)
{
    return {a.r * b.r + a.i * b.i, a.i * b.r - a.r * b.i};
}
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cd cscale(double c, cd a) { return {c * a.r, c * a.i}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.r, -a.i}; }

// One inner sweep of Alg. 1 on the Hermitian G (s.Gr + i s.Gi).  The
// rotation of a pair (R1): with g_ij = |g_ij| e, column i' = c col_i +
// conj(e) s col_j and column j' = -e s col_i + c col_j.
template <class T, int NB>
__device__ __forceinline__ double inner_sweep_cx(IterShared<T, true, NB> &s, double tol)
{
    constexpr int N2 = 2 * NB, JPT = (N2 * NB + kBT - 1) / kBT;
    const int tid = threadIdx.x;
    const InnerBlocks<NB> blk(tid);
    double mc = 0.0;
    for (int r = 0; r < N2 - 1; r++) {
        if (tid < NB) {
            const int i = s.rr[r][tid][0], j = s.rr[r][tid][1];
            const double gii = s.Gr[i][i], gjj = s.Gr[j][j];
            const double gr = s.Gr[i][j], gim = s.Gi[i][j];
            double c = 1.0, er = 0.0, ei = 0.0;
            const double ag = hypot(gr, gim);
            const double si = sqrt(fabs(gii)), sj = sqrt(fabs(gjj));
            const double den = si * sj;
            mc = fmax(mc, den > 0.0 ? ag / den : (ag != 0.0 ? 1.0 : 0.0));
            if (ag != 0.0 && gii >= kNegligible && gjj >= kNegligible && ag >= tol * si * sj) {
                double sn;
                jacobi_cs(gii, gjj, ag, c, sn);
                er = gr / ag * sn;
                ei = gim / ag * sn;
                s.rot = 1;
            }
            s.csc[tid] = c;
            s.cser[tid] = er;
            s.csei[tid] = ei;
        }
        __syncthreads();
        // G <- J_r^H G J_r on the blocks with ka <= kb (the block (kb, ka)
        // is the conjugate transpose); J <- J J_r.
#pragma unroll
        for (int t = 0; t < InnerBlocks<NB>::BPT; t++) {
            const int ka = blk.ka[t], kb = blk.kb[t];
            if (ka < 0) continue;
            const int ia = s.rr[r][ka][0], ja = s.rr[r][ka][1];
            const int ib = s.rr[r][kb][0], jb = s.rr[r][kb][1];
            const double ca = s.csc[ka], cb = s.csc[kb];
            const cd ea = {s.cser[ka], s.csei[ka]}, eb = {s.cser[kb], s.csei[kb]};
            const cd g00 = {s.Gr[ia][ib], s.Gi[ia][ib]}, g01 = {s.Gr[ia][jb], s.Gi[ia][jb]};
            const cd g10 = {s.Gr[ja][ib], s.Gi[ja][ib]}, g11 = {s.Gr[ja][jb], s.Gi[ja][jb]};
            // h = G_block J_b, J_b = [[c, -e s], [conj(e) s, c]]
            const cd h00 = cadd(cscale(cb, g00), cmulc(g01, eb));
            const cd h01 = csub(cscale(cb, g01), cmul(g00, eb));
            const cd h10 = cadd(cscale(cb, g10), cmulc(g11, eb));
            const cd h11 = csub(cscale(cb, g11), cmul(g10, eb));
            // n = J_a^H h, J_a^H = [[c, e s], [-conj(e) s, c]]
            const cd n00 = cadd(cscale(ca, h00), cmul(ea, h10));
            const cd n01 = cadd(cscale(ca, h01), cmul(ea, h11));
            const cd n10 = csub(cscale(ca, h10), cmul(cconj(ea), h00));
            const cd n11 = csub(cscale(ca, h11), cmul(cconj(ea), h01));
            s.Gr[ia][ib] = n00.r;
            s.Gi[ia][ib] = n00.i;
            s.Gr[ia][jb] = n01.r;
            s.Gi[ia][jb] = n01.i;
            s.Gr[ja][ib] = n10.r;
            s.Gi[ja][ib] = n10.i;
            s.Gr[ja][jb] = n11.r;
            s.Gi[ja][jb] = n11.i;
            if (ka != kb) {
                s.Gr[ib][ia] = n00.r;
                s.Gi[ib][ia] = -n00.i;
                s.Gr[jb][ia] = n01.r;
                s.Gi[jb][ia] = -n01.i;
                s.Gr[ib][ja] = n10.r;
                s.Gi[ib][ja] = -n10.i;
                s.Gr[jb][ja] = n11.r;
                s.Gi[jb][ja] = -n11.i;
            }
        }
#pragma unroll
        for (int t = 0; t < JPT; t++) {
            const int idx = tid + t * kBT;
            if (idx >= N2 * NB) break;
            const int row = idx / NB, kb = idx % NB;
            const int ib = s.rr[r][kb][0], jb = s.rr[r][kb][1];
            const double cb = s.csc[kb];
            const cd eb = {s.cser[kb], s.csei[kb]};
            const cd x = {s.Jr[row][ib], s.Ji[row][ib]}, y = {s.Jr[row][jb], s.Ji[row][jb]};
            const cd xn = cadd(cscale(cb, x), cmulc(y, eb));
            const cd yn = csub(cscale(cb, y), cmul(x, eb));
            s.Jr[row][ib] = xn.r;
            s.Ji[row][ib] = xn.i;
            s.Jr[row][jb] = yn.r;
            s.Ji[row][jb] = yn.i;
        }
        __syncthreads();
    }
    return mc;
}

// One block pair (pair `pair` of round-robin iteration `it` over l block
// columns) of one matrix: steps 1-3 above.  W, Vw, stb: this matrix's.
// Real Gram tile (ti TC + tj) that wave `wave` computes as its g-th.  Real:
// tiles wave, wave + 4, ...  Complex (TC = 4, NB = 16): the wave with
// (A, C) = (wave / 2, wave % 2) takes the tiles (A, C), (A + 2, C + 2),
// (A, C + 2), (A + 2, C) of the real form, whose sums and differences are
// block (A, C) of Gr and Gi.
template <bool CX, int TC>
__device__ __forceinline__ int gram_tile(int wave, int g)
{
    if constexpr (CX) {
        const int A = wave >> 1, C = wave & 1;
        const int ti = A + (g == 1 || g == 3 ? 2 : 0), tj = C + (g == 1 || g == 2 ? 2 : 0);
        return ti * TC + tj;
    } else {
        return wave + 4 * g;
    }
}

template <class T, bool CX, int NB>
__device__ __forceinline__ void iter_body(IterShared<T, CX, NB> &s, int m, int np, int l, int it,
                                          int pair, typename Elem<T, CX>::type *W,
                                          typename Elem<T, CX>::type *Vw, BlkState *stb,
                                          double tol, int inner)
{
    using E = typename Elem<T, CX>::type;
    using Sh = IterShared<T, CX, NB>;
    constexpr int N2 = Sh::N2, NR = Sh::NR, CH = Sh::CH;
    constexpr int TC = NR / 16, GT = TC * TC;   // real Gram output tiles
    constexpr int GPW = (GT + 3) / 4;           // tiles per wave
    static_assert(!CX || GPW == 4, "complex: a wave holds the four tiles of one block of G");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    int p, q;
    rr_pair(l, it, pair, p, q);

    // ---- 1. Gram matrix on the matrix cores --------------------------------
    typename Mfma<T>::acc_t acc[GPW];
#pragma unroll
    for (int g = 0; g < GPW; g++) acc[g] = typename Mfma<T>::acc_t{0, 0, 0, 0};
    {
        ChunkRegs<E, NB> Rg;
        chunk_load<E, NB>(Rg, W, m, 0, p, q);
        for (int r0 = 0; r0 < m; r0 += CH) {
            __syncthreads();
            chunk_to_lds<T, CX, NB, E>(s, Rg);
            __syncthreads();
            if (r0 + CH < m) chunk_load<E, NB>(Rg, W, m, r0 + CH, p, q);
#pragma unroll
            for (int g = 0; g < GPW; g++) {
                const int tile = gram_tile<CX, TC>(wave, g);
                if (tile < GT) {
                    const int ti = tile / TC, tj = tile % TC;
#pragma unroll
                    for (int k0 = 0; k0 < CH; k0 += 4) {
                        const T a = s.u.xs[16 * ti + li][k0 + lk];    // X^T[i][k]
                        const T bb = s.u.xs[16 * tj + li][k0 + lk];   // X[k][j]
                        acc[g] = Mfma<T>::op(a, bb, acc[g]);
                    }
                }
            }
        }
    }
    __syncthreads();                            // xs is dead, R takes its place
    if constexpr (CX) {
        // G = X^H X from the real form R = [Xr Xi]^T [Xr Xi]: Gr = R11 + R22,
        // Gi = R12 - R21; this wave holds the four tiles of block (A, C)
        const int A = wave >> 1, C = wave & 1;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int row = 16 * A + Mfma<T>::row(lane, v), col = 16 * C + li;
            s.Gr[row][col] = (double)acc[0][v] + (double)acc[1][v];
            s.Gi[row][col] = (double)acc[2][v] - (double)acc[3][v];
        }
        for (int idx = tid; idx < N2 * N2; idx += kBT) s.Ji[idx / N2][idx % N2] = 0.0;
    } else {
#pragma unroll
        for (int g = 0; g < GPW; g++) {
            const int tile = wave + 4 * g;
            if (tile < GT) {
                const int ti = tile / TC, tj = tile % TC;
#pragma unroll
                for (int v = 0; v < 4; v++)
                    s.u.R[16 * ti + Mfma<T>::row(lane, v)][16 * tj + li] = (double)acc[g][v];
            }
        }
    }
    for (int idx = tid; idx < N2 * N2; idx += kBT) s.Jr[idx / N2][idx % N2] = (idx / N2 == idx % N2);
    // the inner solve's round-robin table (the ordering of Alg. 1's sweep)
    for (int idx = tid; idx < (N2 - 1) * NB; idx += kBT) {
        int i, j;
        rr_pair(N2, idx / NB, idx % NB, i, j);
        s.rr[idx / NB][idx % NB][0] = (unsigned char)i;
        s.rr[idx / NB][idx % NB][1] = (unsigned char)j;
    }
    if (tid == 0) s.rot = 0;
    __syncthreads();

    // ---- 2. inner sweeps of Alg. 1 on G (FP64), round robin -------------
    // Design 2 ("Inexact Hermitian Eigendecomposition") runs one; more, up
    // to the solve's convergence, are the variants of the same section.  A
    // sweep that rotates nothing ends the solve, so "no rotation in the whole
    // outer sweep" still means that every first inner sweep rotated nothing.
    const int nsw = inner_sweeps_of(inner, l, m, np, sizeof(T) == 4);
    bool any = false;
    double mc = 0.0;
    for (int k = 0; k < nsw; k++) {
        double mck;
        if constexpr (CX)
            mck = inner_sweep_cx<T, NB>(s, tol);
        else
            mck = inner_sweep_real<T, NB>(s, tol);
        if (k == 0) mc = mck;   // the switch test of the mixed mode uses the first
        const bool r = s.rot != 0;   // the sweep ended with a barrier
        __syncthreads();             // every thread has read the flag
        if (!r) break;
        any = true;
        if (tid == 0) s.rot = 0;
        __syncthreads();
    }
    if (wave == 0) {
        mc = wave_max(mc);
        if (lane == 0 && mc > 0.0)
            atomicMax(&stb->maxcos, (unsigned long long)__double_as_longlong(mc));
    }

    // ---- 3. fused update of the block columns of W and V --------------------
    if (any) {
        update_block_columns<T, CX, NB, E>(s, W, m, p, q);
        update_block_columns<T, CX, NB, E>(s, Vw, np, p, q);
        if (tid == 0) atomicOr(&stb->rotated, 1);
    }
}

// Resident waves per SIMD the iteration kernels are compiled for.  The
// kernel is bound by the latency of its barrier chain (chunked Gram, inner
// sweep, update), so more resident workgroups pay: measured on 800 256x256
// FP64 matrices, five waves instead of the four that the unconstrained
// register allocation allowed took a call from 184 to 170 ms (22.9 sweeps,
// all-FP64) and 72 to 68.5 ms (7.9 sweeps, QR-preconditioned); FP32 at six
// or eight waves spills and is slower.  nb = 8 fits eight without spills;
// complex data (32-row chunks, no real Gram in LDS: 52 KB) three, nb = 32
// two (its LDS).
template <class T, bool CX, int NB>
constexpr int blk_waves()
{
    return CX ? 3 : (NB == 32 ? 2 : (NB == 8 ? 8 : 5));
}

template <class T, bool CX, int NB>
__global__ __launch_bounds__(kBT, (blk_waves<T, CX, NB>())) void blk_iter(int m, int np, int l, int it,
                                                typename Elem<T, CX>::type *W,
                                                typename Elem<T, CX>::type *Vw, BlkState *st,
                                                double tol, int inner, const int *stop)
{
    __shared__ IterShared<T, CX, NB> s;
    const int b = blockIdx.x / (l / 2), pair = blockIdx.x % (l / 2);
    if ((stop && *stop) || !st[b].active) return;
    iter_body<T, CX, NB>(s, m, np, l, it, pair, W + (size_t)b * m * np, Vw + (size_t)b * np * np,
                         st + b, tol, inner);
}

// Threshold of the inner eigensolver in outer sweep s (counted from 0) with
// the dynamic tolerance of "Inexact Hermitian Eigendecomposition"
// (subsection "Motivation", first way): tol_start shrinks by tol_rate per
// sweep until it reaches tol; tol_start <= tol keeps tol throughout.  The
// products are formed one sweep at a time, as the sequence is defined, so
// host and device obtain the same doubles.
__host__ __device__ __forceinline__ double inner_tol(double tol, double t0, double rate, int s)
{
    if (!(t0 > tol)) return tol;
    double ts = t0;
    for (int k = 0; k < s; k++) ts = ts * rate > tol ? ts * rate : tol;
    return ts;
}

// End of a sweep: a matrix with no rotation is converged (done); with
// `phase32` (FP32 phase of the mixed mode) one whose largest cosine is at
// most kSwitchCos is done too.  With the dynamic inner tolerance (t0 > tol)
// only a sweep run at the final threshold tol can converge a matrix.  With
// masking a done matrix is retired; without, every matrix stays active
// until the whole batch is done.  *pending counts the matrices not done.
__global__ void blk_sweep_end(int batch, BlkState *st, int *pending, int masking, int phase32,
                              double tol, double t0, double rate, const int *stop)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch || (stop && *stop)) return;
    BlkState &s = st[b];
    if (!s.active) return;
    if (!s.done) {
        const bool at_tol = inner_tol(tol, t0, rate, s.sweeps) <= tol;
        s.sweeps += 1;
        const double mc = __longlong_as_double((long long)s.maxcos);
        bool fin = !s.rotated && at_tol;
        if (phase32 && fp32_phase_done(mc, s.prevcos, s.sweeps)) fin = true;
        s.prevcos = mc;
        if (fin) s.done = 1;
    }
    s.rotated = 0;
    s.maxcos = 0ull;
    if (!s.done) atomicAdd(pending, 1);
    if (masking && s.done) s.active = 0;
}

// Sweep control of the queued form: ctl[0] counts the matrices still
// sweeping after a sweep (round), ctl[1] is set once that count is zero, and
// every later launch of the call returns at once.  The count starts from
// zero for the next sweep.
__global__ void sweep_close(int *ctl)
{
    if (threadIdx.x == 0) {
        if (ctl[0] == 0) ctl[1] = 1;
        ctl[0] = 0;
    }
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
// permuted.  EW: working element type, EO: output element type.
template <class EO>
using RealOf = typename std::conditional<std::is_same<EO, float2>::value ||
                                             std::is_same<EO, float>::value,
                                         float, double>::type;

// One matrix per workgroup; pointers of this matrix; dynamic LDS
// n (sizeof(double) + sizeof(int)).  info_b, sweeps_b: this matrix's slots.
template <class EW, class EO>
__device__ __forceinline__ void finalize_body(int m, int n, int np, const EW *W, const EW *Vw,
                                              const BlkState &sb, int extra, RealOf<EO> *S,
                                              EO *U, int ldu, EO *V, int ldv, int *info_b,
                                              int *sweeps_b)
{
    using OW = EOps<EW>;
    using OO = EOps<EO>;
    using SR = RealOf<EO>;
    extern __shared__ double dyn[];
    double *sig = dyn;                     // n
    int *rank = (int *)(sig + n);          // n
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (sb.bad) {
        if (tid == 0) {
            *info_b = 2;
            if (sweeps_b) *sweeps_b = 0;
        }
        return;
    }
    for (int c = wave; c < n; c += kBT / 64) {
        const EW *w = W + (size_t)c * m;
        double mx = 0.0;
        for (int r = lane; r < m; r += 64) mx = fmax(mx, fmax(fabs(OW::re(w[r])), fabs(OW::im(w[r]))));
        mx = wave_max(mx);
        double ss = 0.0;
        if (mx > 0.0) {
            const double sc = ldexp(1.0, -ilogb(mx));
            for (int r = lane; r < m; r += 64) {
                const double yr = OW::re(w[r]) * sc, yi = OW::im(w[r]) * sc;
                ss += yr * yr + yi * yi;
            }
        }
        ss = wave_sum(ss);
        const double sc = mx > 0.0 ? ldexp(sqrt(ss), ilogb(mx)) : 0.0;
        if (lane == 0) sig[c] = sc >= 0x1p-480 ? sc : 0.0;
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
        if (lane == 0) S[rk] = (SR)(sc / sb.scale);
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        if (U)
            for (int r = lane; r < m; r += 64) {
                const EW w = W[(size_t)c * m + r];
                U[(size_t)rk * ldu + r] = OO::make(OW::re(w) * inv, OW::im(w) * inv);
            }
        if (V)
            for (int r = lane; r < n; r += 64) {
                const EW v = Vw[(size_t)c * np + r];
                V[(size_t)rk * ldv + r] = OO::make(OW::re(v), OW::im(v));
            }
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
                EO *u = U + (size_t)rank[i] * ldu;
                for (; cand < m; cand++) {
                    for (int r = lane; r < m; r += 64) u[r] = OO::make(r == cand ? 1.0 : 0.0, 0.0);
                    __threadfence();
                    for (int pass = 0; pass < 2; pass++)
                        for (int j = 0; j < n; j++) {
                            if (j == i || (sig[j] == 0.0 && j > i)) continue;
                            const EO *qv = U + (size_t)rank[j] * ldu;
                            double dr = 0.0, di = 0.0;   // d = q^H u
                            for (int r = lane; r < m; r += 64) {
                                const double qr = OO::re(qv[r]), qi = OO::im(qv[r]);
                                const double ur = OO::re(u[r]), ui = OO::im(u[r]);
                                dr += qr * ur + qi * ui;
                                di += qr * ui - qi * ur;
                            }
                            dr = wave_sum(dr);
                            di = wave_sum(di);
                            for (int r = lane; r < m; r += 64) {
                                const double qr = OO::re(qv[r]), qi = OO::im(qv[r]);
                                u[r] = OO::make(OO::re(u[r]) - (dr * qr - di * qi),
                                                OO::im(u[r]) - (dr * qi + di * qr));
                            }
                            __threadfence();
                        }
                    double nu = 0.0;
                    for (int r = lane; r < m; r += 64)
                        nu += OO::re(u[r]) * OO::re(u[r]) + OO::im(u[r]) * OO::im(u[r]);
                    nu = sqrt(wave_sum(nu));
                    if (nu > 0.5) {
                        const double inv = 1.0 / nu;
                        for (int r = lane; r < m; r += 64)
                            u[r] = OO::make(OO::re(u[r]) * inv, OO::im(u[r]) * inv);
                        __threadfence();
                        cand++;
                        break;
                    }
                }
            }
        }
    }
    if (tid == 0) {
        *info_b = sb.done ? 0 : 1;
        if (sweeps_b) *sweeps_b = sb.sweeps + extra;
    }
}

template <class EW, class EO>
__global__ __launch_bounds__(kBT) void blk_finalize(int m, int n, int np, const EW *W,
                                                    const EW *Vw, const BlkState *st,
                                                    const int *sweeps_extra, RealOf<EO> *S,
                                                    long long sS, EO *U, int ldu, long long sU,
                                                    EO *V, int ldv, long long sV, int *info,
                                                    int *sweeps_out)
{
    const int b = blockIdx.x;
    finalize_body<EW, EO>(m, n, np, W + (size_t)b * m * np, Vw + (size_t)b * np * np, st[b],
                          sweeps_extra ? sweeps_extra[b] : 0, S + (size_t)b * sS,
                          U ? U + (size_t)b * sU : nullptr, ldu, V ? V + (size_t)b * sV : nullptr,
                          ldv, info + b, sweeps_out ? sweeps_out + b : nullptr);
}

// ---------------------------------------------------------------------------
// Batched FP64 GEMM on the matrix cores, column major:
//   C = alpha_b op(A) B + beta D,  op(A) = A (M x K) or A^T (A is K x M),
// alpha_b = alpha * st[b].scale when st is given.  One 64 x 64 tile of C per
// workgroup (each wave four 16 x 16 tiles), K staged through LDS 16 at a
// time; workgroup x = b * tiles + tile.  C must not overlap A or B; it may
// be D itself (each element of D is read by the lane that then writes the
// same element of C).
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

// The queued sweep control is used when asked for, and whenever `stream`
// is being captured into a graph (the host-closed loop cannot wait there).
bool queued_sweeps(int persistent, hipStream_t stream)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;
    return persistent != 0 || cs == hipStreamCaptureStatusActive;
}

template <class T, bool CX>
void launch_iter(int nb, unsigned grid, hipStream_t stream, int m, int np, int l, int it,
                 typename Elem<T, CX>::type *W, typename Elem<T, CX>::type *Vw, BlkState *st,
                 double tol, int inner, const int *stop)
{
    if constexpr (CX) {
        hipLaunchKernelGGL((blk_iter<T, true, 16>), dim3(grid), dim3(kBT), 0, stream, m, np, l,
                           it, W, Vw, st, tol, inner, stop);
        (void)nb;
    } else {
        if (nb == 8)
            hipLaunchKernelGGL((blk_iter<T, false, 8>), dim3(grid), dim3(kBT), 0, stream, m, np,
                               l, it, W, Vw, st, tol, inner, stop);
        else if (nb == 16)
            hipLaunchKernelGGL((blk_iter<T, false, 16>), dim3(grid), dim3(kBT), 0, stream, m, np,
                               l, it, W, Vw, st, tol, inner, stop);
        else
            hipLaunchKernelGGL((blk_iter<T, false, 32>), dim3(grid), dim3(kBT), 0, stream, m, np,
                               l, it, W, Vw, st, tol, inner, stop);
    }
}

// Sweeps of a uniform batch, one launch per round-robin iteration.
// Host-closed form (queued = false): after every sweep the host waits for
// the count of pending matrices and stops once it is zero; the call is
// synchronous.  Queued form (queued = true): the launches of all max_sweeps
// sweeps go onto the stream at once and the count stays on the device
// (sweep_close); after the sweep that leaves no matrix pending, every later
// launch returns at once.  Nothing waits on the host and nothing is copied
// to it, so the call can be captured in a HIP graph; the price is the
// no-op launches after convergence.  Both forms take the same decisions and
// give the same bits.  ctl: two ints of the workspace.
template <class T, bool CX>
hipError_t run_sweeps_host(int batch, int m, int np, int nb, typename Elem<T, CX>::type *W,
                           typename Elem<T, CX>::type *Vw, BlkState *st, int *ctl,
                           double tol, int max_sweeps, int masking, int phase32, int inner,
                           hipStream_t stream, double t0, double rate, bool queued)
{
    const int l = np / nb;
    const unsigned grid = (unsigned)batch * (unsigned)(l / 2);
    const unsigned egrid = (unsigned)((batch + 255) / 256);
    if (queued) {
        hipError_t e = launch_fill_int(ctl, 2, 0, stream);
        if (e != hipSuccess) return e;
        for (int sw = 0; sw < max_sweeps; sw++) {
            const double ts = inner_tol(tol, t0, rate, sw);
            for (int it = 0; it < l - 1; it++)
                launch_iter<T, CX>(nb, grid, stream, m, np, l, it, W, Vw, st, ts, inner, ctl + 1);
            hipLaunchKernelGGL(blk_sweep_end, dim3(egrid), dim3(256), 0, stream, batch, st, ctl,
                               masking, phase32, tol, t0, rate, (const int *)(ctl + 1));
            hipLaunchKernelGGL(sweep_close, dim3(1), dim3(64), 0, stream, ctl);
        }
        return hipGetLastError();
    }
    int *host_count;
    hipError_t e = pinned_counter(&host_count);
    if (e != hipSuccess) return e;
    for (int sw = 0; sw < max_sweeps; sw++) {
        // every matrix still sweeping is in its sweep sw
        const double ts = inner_tol(tol, t0, rate, sw);
        for (int it = 0; it < l - 1; it++)
            launch_iter<T, CX>(nb, grid, stream, m, np, l, it, W, Vw, st, ts, inner, nullptr);
        e = hipMemsetAsync(ctl, 0, sizeof(int), stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(blk_sweep_end, dim3(egrid), dim3(256), 0, stream, batch, st, ctl,
                           masking, phase32, tol, t0, rate, (const int *)nullptr);
        e = hipMemcpyAsync(host_count, ctl, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        if (*host_count == 0) break;
    }
    return hipGetLastError();
}

// Sweep control of the block method: persistent = 0 closes each sweep on
// the host, 1 queues every sweep with the count on the device (see
// run_sweeps_host).  ctl: the control block in the workspace.
template <class T, bool CX>
hipError_t run_sweeps(int batch, int m, int np, int nb, typename Elem<T, CX>::type *W,
                      typename Elem<T, CX>::type *Vw, BlkState *st, int *ctl, double tol,
                      int max_sweeps, int masking, int phase32, int inner, int persistent,
                      hipStream_t stream, double t0 = 0.0, double rate = 0.0)
{
    return run_sweeps_host<T, CX>(batch, m, np, nb, W, Vw, st, ctl, tol, max_sweeps,
                                  masking, phase32, inner, stream, t0, rate,
                                  queued_sweeps(persistent, stream));
}

// Workspace carving; the same order as blocked_workspace_bytes.
struct WsLayout {
    void *W, *Vw, *W32, *V32;
    double *Q, *X;
    BlkState *st;
    int *sw32;
    int *ctl;          // sweep control: the count of pending matrices and the stop word
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
    L.ctl = (int *)p;
    return L;
}

unsigned elementwise_grid(size_t total)
{
    const size_t g = (total + 255) / 256;
    return (unsigned)(g < 65536 ? (g ? g : 1) : 65536);
}

template <class T, bool CX>
hipError_t launch_blocked(int batch, int m, int n, int nb, const typename Elem<T, CX>::type *A,
                          int lda, long long sA, T *S, long long sS,
                          typename Elem<T, CX>::type *U, int ldu, long long sU,
                          typename Elem<T, CX>::type *V, int ldv, long long sV, double tol,
                          int max_sweeps, int masking, int *info, int *sweeps, void *ws,
                          hipStream_t stream, int inner, int persistent, double t0, double rate)
{
    using E = typename Elem<T, CX>::type;
    const int np = blocked_np(n, nb);
    WsLayout L = carve(ws, batch, m, n, np, sizeof(E), false);
    E *W = (E *)L.W, *Vw = (E *)L.Vw;
    hipError_t e;
    hipLaunchKernelGGL((blk_init<E, E>), dim3(batch), dim3(kBT), 0, stream, m, n, np, A, lda, sA,
                       W, Vw, L.st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = run_sweeps<T, CX>(batch, m, np, nb, W, Vw, L.st, L.ctl, tol, max_sweeps, masking, 0,
                          inner, persistent, stream, t0, rate);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)n * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL((blk_finalize<E, E>), dim3(batch), dim3(kBT), lds, stream, m, n, np,
                       (const E *)W, (const E *)Vw, (const BlkState *)L.st, (const int *)nullptr,
                       S, sS, U, ldu, sU, V, ldv, sV, info, sweeps);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Uneven batches (one pointer per matrix, any shape mix) and the serving
// runtime.  Every matrix has its own descriptor (VbDesc) and its own
// round-robin schedule over l_b block columns (nb = 16).  One launch of
// vb_iter covers every block pair of every listed matrix; matrix b runs
// iteration (itg - it0_b) mod (l_b - 1) of its current sweep, so a small
// matrix completes several sweeps while a large one completes one, and a
// matrix admitted later (it0_b > 0) joins the running launches.
// vb_sweep_end closes the sweeps that end at launch itg.
// ---------------------------------------------------------------------------
template <class E>
__global__ __launch_bounds__(kBT) void vb_init(const VbDesc *d, const int *idx, void *base,
                                               BlkState *st)
{
    const int b = idx ? idx[blockIdx.x] : (int)blockIdx.x;
    const VbDesc D = d[b];
    E *Wb = (E *)base;
    init_body<E, E>(D.m, D.n, D.np, (const E *)D.A, D.lda, Wb + D.woff, Wb + D.voff, st + b,
                    D.trans != 0);
}

template <class T, bool CX>
__global__ __launch_bounds__(kBT, (blk_waves<T, CX, kVbNb>())) void vb_iter(const VbDesc *d, const int2 *work, int itg,
                                               void *base, BlkState *st, double tol, int inner,
                                               double t0, double rate, const int *stop)
{
    using E = typename Elem<T, CX>::type;
    __shared__ IterShared<T, CX, kVbNb> s;
    if (stop && *stop) return;
    const int2 w = work[blockIdx.x];
    if (!st[w.x].active) return;
    const VbDesc &D = d[w.x];
    const int m = D.m, np = D.np, l = D.l;
    E *Wb = (E *)base;
    iter_body<T, CX, kVbNb>(s, m, np, l, (itg - D.it0) % (l - 1), w.y, Wb + D.woff, Wb + D.voff,
                            st + w.x, inner_tol(tol, t0, rate, st[w.x].sweeps),
                            inner != 0 ? inner : D.inner);
}

// Closes the sweeps of the matrices whose sweep ends at launch itg; a matrix
// that reaches max_sweeps unconverged stops (info 1).  With `pending`, counts
// the matrices still sweeping.
__global__ void vb_sweep_end(int count, const VbDesc *d, int itg, BlkState *st, int max_sweeps,
                             int masking, int *pending, double tol, double t0, double rate,
                             const int *stop)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count || (stop && *stop)) return;
    BlkState &s = st[b];
    if (s.active && (itg - d[b].it0 + 1) % (d[b].l - 1) == 0) {
        if (!s.done) {
            const bool at_tol = inner_tol(tol, t0, rate, s.sweeps) <= tol;
            s.sweeps += 1;
            if (!s.rotated && at_tol)
                s.done = 1;
            else if (s.sweeps >= max_sweeps)
                s.active = 0;
        }
        s.rotated = 0;
        s.maxcos = 0ull;
        if (masking && s.done) s.active = 0;
    }
    if (pending && s.active && !s.done) atomicAdd(pending, 1);
}

// flags[b] = 1 once matrix b has stopped sweeping (converged or capped).
__global__ void vb_collect(int count, const BlkState *st, int *flags)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < count) flags[b] = st[b].active ? 0 : 1;
}

__global__ void vb_mark_empty(int count, BlkState *st)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < count) {
        state_reset(st[b], 0);
        st[b].active = 0;
        st[b].done = 1;
    }
}

template <class E>
__global__ __launch_bounds__(kBT) void vb_finalize(const VbDesc *d, const int *idx,
                                                   const void *base, const BlkState *st)
{
    const int b = idx ? idx[blockIdx.x] : (int)blockIdx.x;
    const VbDesc D = d[b];
    const E *Wb = (const E *)base;
    finalize_body<E, E>(D.m, D.n, D.np, Wb + D.woff, Wb + D.voff, st[b], 0, (RealOf<E> *)D.S,
                        (E *)D.U, D.ldu, (E *)D.V, D.ldv, D.info, D.sweeps);
}

struct VbLayout {
    VbDesc *desc;
    int2 *work;
    BlkState *st;
    int *pending;
    void *base;   // every matrix's W, then V
    size_t bytes;
};

VbLayout vb_layout(void *ws, int batch, const int *m, const int *n, size_t elt)
{
    size_t nwork = 0, elts = 0;
    for (int b = 0; b < batch; b++) {
        if (n[b] == 0) continue;
        const int np = blocked_np(n[b], kVbNb);
        nwork += np / kVbNb / 2;
        elts += (size_t)m[b] * np + (size_t)np * np;
    }
    size_t off[5], o = 0;
    off[0] = o;
    o += align256((size_t)batch * sizeof(VbDesc));
    off[1] = o;
    o += align256(nwork * sizeof(int2));
    off[2] = o;
    o += align256((size_t)batch * sizeof(BlkState));
    off[3] = o;
    o += 256;
    off[4] = o;
    o += align256(elts * elt);
    VbLayout L{};
    L.bytes = o;
    if (ws) {
        char *p = (char *)ws;
        L.desc = (VbDesc *)(p + off[0]);
        L.work = (int2 *)(p + off[1]);
        L.st = (BlkState *)(p + off[2]);
        L.pending = (int *)(p + off[3]);
        L.base = p + off[4];
    }
    return L;
}

// Host staging of the descriptors and the work table: pinned buffers, each
// reused only once the copy that last read it has executed (an event is
// recorded after the copy), so an asynchronous call never overwrites data
// that a previous call's copy has yet to read.
struct Staging {
    char *buf = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool taken = false;
};

hipError_t vb_staging(size_t bytes, Staging **out)
{
    static std::mutex mu;
    static std::map<int, std::vector<Staging *>> pools;   // per device (its events)
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    std::vector<Staging *> &pool = pools[dev];
    for (Staging *st : pool) {
        if (st->taken || st->cap < bytes) continue;
        const hipError_t q = hipEventQuery(st->ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return q;
        st->taken = true;
        *out = st;
        return hipSuccess;
    }
    Staging *st = new Staging();
    size_t cap = 4096;
    while (cap < bytes) cap *= 2;
    e = hipHostMalloc((void **)&st->buf, cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (st->buf) (void)hipHostFree(st->buf);
        delete st;
        return e;
    }
    st->cap = cap;
    st->taken = true;
    pool.push_back(st);
    *out = st;
    return hipSuccess;
}

// Marks a staging buffer as read by the copies enqueued so far on `stream`.
hipError_t vb_staging_release(Staging *st, hipStream_t stream)
{
    const hipError_t e = hipEventRecord(st->ev, stream);
    st->taken = false;   // the event now guards the buffer
    return e;
}

template <class T, bool CX>
void vb_launch_iter_t(const VbDesc *d, const int2 *work, int nwork, int itg, void *base,
                      BlkState *st, double tol, int inner, double t0, double rate,
                      hipStream_t stream, const int *stop)
{
    hipLaunchKernelGGL((vb_iter<T, CX>), dim3((unsigned)nwork), dim3(kBT), 0, stream, d, work, itg,
                       base, st, tol, inner, t0, rate, stop);
}

template <class E>
void vb_launch_init_t(const VbDesc *d, const int *idx, int count, void *base, BlkState *st,
                      hipStream_t stream)
{
    hipLaunchKernelGGL((vb_init<E>), dim3((unsigned)count), dim3(kBT), 0, stream, d, idx, base,
                       st);
}

template <class E>
void vb_launch_finalize_t(const VbDesc *d, const int *idx, int count, int maxn, const void *base,
                          const BlkState *st, hipStream_t stream)
{
    const size_t lds = (size_t)(maxn > 0 ? maxn : 1) * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL((vb_finalize<E>), dim3((unsigned)count), dim3(kBT), lds, stream, d, idx,
                       base, st);
}

}  // namespace

// dtype-dispatched launchers of the uneven-batch kernels (svdb_dtype_t codes)
void vb_launch_init(int dtype, const VbDesc *d, const int *idx, int count, void *base,
                    void *st, hipStream_t stream)
{
    BlkState *S = (BlkState *)st;
    switch (dtype) {
    case 0: vb_launch_init_t<float>(d, idx, count, base, S, stream); break;
    case 1: vb_launch_init_t<double>(d, idx, count, base, S, stream); break;
    case 2: vb_launch_init_t<float2>(d, idx, count, base, S, stream); break;
    default: vb_launch_init_t<double2>(d, idx, count, base, S, stream); break;
    }
}

void vb_launch_iter(int dtype, const VbDesc *d, const int2 *work, int nwork, int itg, void *base,
                    void *st, double tol, hipStream_t stream, int inner, double t0, double rate,
                    const int *stop)
{
    BlkState *S = (BlkState *)st;
    switch (dtype) {
    case 0:
        vb_launch_iter_t<float, false>(d, work, nwork, itg, base, S, tol, inner, t0, rate, stream,
                                        stop);
        break;
    case 1:
        vb_launch_iter_t<double, false>(d, work, nwork, itg, base, S, tol, inner, t0, rate, stream,
                                        stop);
        break;
    case 2:
        vb_launch_iter_t<float, true>(d, work, nwork, itg, base, S, tol, inner, t0, rate, stream,
                                        stop);
        break;
    default:
        vb_launch_iter_t<double, true>(d, work, nwork, itg, base, S, tol, inner, t0, rate, stream,
                                        stop);
        break;
    }
}

void vb_launch_sweep_end(int count, const VbDesc *d, int itg, void *st, int max_sweeps,
                         int masking, int *pending, hipStream_t stream, double tol, double t0,
                         double rate, const int *stop)
{
    hipLaunchKernelGGL(vb_sweep_end, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       count, d, itg, (BlkState *)st, max_sweeps, masking, pending, tol, t0, rate,
                       stop);
}

void vb_launch_collect(int count, const void *st, int *flags, hipStream_t stream)
{
    hipLaunchKernelGGL(vb_collect, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       count, (const BlkState *)st, flags);
}

void vb_launch_mark_empty(int count, void *st, hipStream_t stream)
{
    hipLaunchKernelGGL(vb_mark_empty, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       count, (BlkState *)st);
}

void vb_launch_finalize(int dtype, const VbDesc *d, const int *idx, int count, int maxn,
                        const void *base, const void *st, hipStream_t stream)
{
    const BlkState *S = (const BlkState *)st;
    switch (dtype) {
    case 0: vb_launch_finalize_t<float>(d, idx, count, maxn, base, S, stream); break;
    case 1: vb_launch_finalize_t<double>(d, idx, count, maxn, base, S, stream); break;
    case 2: vb_launch_finalize_t<float2>(d, idx, count, maxn, base, S, stream); break;
    default: vb_launch_finalize_t<double2>(d, idx, count, maxn, base, S, stream); break;
    }
}

size_t vb_state_bytes() { return sizeof(BlkState); }

int vb_nb() { return kVbNb; }

namespace {

hipError_t launch_vb(int dtype, size_t elt, int batch, const int *m, const int *n,
                     const void *const *A, const int *lda, void *const *S, void *const *U,
                     const int *ldu, void *const *V, const int *ldv, double tol, int max_sweeps,
                     int masking, int *info, int *sweeps, void *ws, hipStream_t stream,
                     const int *trans, int inner, int persistent, double t0, double rate)
{
    VbLayout L = vb_layout(ws, batch, m, n, elt);
    // descriptors, then the work table with the largest matrices first
    std::vector<int> order(batch);
    for (int b = 0; b < batch; b++) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return n[x] > n[y]; });
    const size_t dbytes = (size_t)batch * sizeof(VbDesc);
    size_t nwork = 0;
    for (int b = 0; b < batch; b++)
        if (n[b] > 0) nwork += blocked_np(n[b], kVbNb) / kVbNb / 2;
    Staging *stg;
    hipError_t e = vb_staging(dbytes + nwork * sizeof(int2) + 16, &stg);
    if (e != hipSuccess) return e;
    char *host = stg->buf;
    VbDesc *hd = (VbDesc *)host;
    int2 *hw = (int2 *)(host + dbytes);
    long long off = 0;   // elements
    int lmax = 2, maxn = 0;
    for (int b = 0; b < batch; b++) {
        VbDesc D{};
        D.A = A[b];
        D.S = S[b];
        D.U = U ? U[b] : nullptr;
        D.V = V ? V[b] : nullptr;
        D.info = info + b;
        D.sweeps = sweeps ? sweeps + b : nullptr;
        D.m = m[b];
        D.n = n[b];
        D.lda = lda[b];
        D.ldu = U ? ldu[b] : 1;
        D.ldv = V ? ldv[b] : 1;
        D.np = n[b] > 0 ? blocked_np(n[b], kVbNb) : 0;
        D.l = n[b] > 0 ? D.np / kVbNb : 2;
        D.it0 = 0;
        D.trans = trans ? trans[b] : 0;
        BlockChoice ch;
        D.inner = (inner == 0 && n[b] > 0 && tuned_block(dtype, m[b], n[b], &ch)) ? ch.inner : 0;
        D.woff = off;
        off += (long long)D.m * D.np;
        D.voff = off;
        off += (long long)D.np * D.np;
        hd[b] = D;
        lmax = D.l > lmax ? D.l : lmax;
        maxn = n[b] > maxn ? n[b] : maxn;
    }
    size_t w = 0;
    for (int b : order)
        for (int q = 0; n[b] > 0 && q < hd[b].l / 2; q++) hw[w++] = make_int2(b, q);
    e = hipMemcpyAsync(L.desc, hd, dbytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && nwork)
        e = hipMemcpyAsync(L.work, hw, nwork * sizeof(int2), hipMemcpyHostToDevice, stream);
    const hipError_t er = vb_staging_release(stg, stream);
    if (e != hipSuccess) return e;
    if (er != hipSuccess) return er;
    vb_launch_init(dtype, L.desc, nullptr, batch, L.base, L.st, stream);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // a round is lmax - 1 launches of the iteration (matrices with fewer
    // block columns close sweeps inside it); the matrices still sweeping are
    // counted at its end.  persistent = 0: the host reads the count after
    // every round and stops at zero.  1 (queued): every round goes onto the
    // stream, the count stays on the device and, once it is zero, the later
    // launches return at once (see run_sweeps_host).
    int *ctl = (int *)L.pending;
    int *host_count = nullptr;
    persistent = queued_sweeps(persistent, stream);
    if (persistent) {
        e = launch_fill_int(ctl, 2, 0, stream);
    } else {
        e = pinned_counter(&host_count);
    }
    if (e != hipSuccess) return e;
    const int *stop = persistent ? ctl + 1 : nullptr;
    int itg = 0;
    for (int round = 0; round < max_sweeps; round++) {
        if (!persistent) {
            e = hipMemsetAsync(ctl, 0, sizeof(int), stream);
            if (e != hipSuccess) return e;
        }
        for (int k = 0; k < lmax - 1; k++, itg++) {
            if (nwork)
                vb_launch_iter(dtype, L.desc, L.work, (int)nwork, itg, L.base, L.st, tol, stream,
                               inner, t0, rate, stop);
            vb_launch_sweep_end(batch, L.desc, itg, L.st, max_sweeps, masking,
                                k == lmax - 2 ? ctl : (int *)nullptr, stream, tol, t0, rate,
                                stop);
        }
        if (persistent) {
            hipLaunchKernelGGL(sweep_close, dim3(1), dim3(64), 0, stream, ctl);
            continue;
        }
        e = hipMemcpyAsync(host_count, ctl, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        if (*host_count == 0) break;
    }
    vb_launch_finalize(dtype, L.desc, nullptr, batch, maxn, L.base, L.st, stream);
    return hipGetLastError();
}

}  // namespace

int blocked_nb(int m, int n, int nb, bool complex_)
{
    (void)m;
    if (complex_) return (nb == 0 || nb == 16) ? 16 : 0;
    if (nb == 8 || nb == 16 || nb == 32) return nb;
    if (nb != 0) return 0;
    return 16;   // nb = 32 has half the pairs but a 4x longer inner sweep
                 // and lower occupancy: slower at every measured size
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
                            int *info, int *sweeps, void *ws, hipStream_t stream, int inner,
                            int persistent, double t0, double rate)
{
    return launch_blocked<double, false>(batch, m, n, nb, A, lda, sA, S, sS, U, ldu, sU, V, ldv,
                                         sV, tol, max_sweeps, masking, info, sweeps, ws, stream,
                                         inner, persistent, t0, rate);
}

hipError_t launch_blocked_s(int batch, int m, int n, int nb, const float *A, int lda, long long sA,
                            float *S, long long sS, float *U, int ldu, long long sU, float *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream, int inner,
                            int persistent, double t0, double rate)
{
    return launch_blocked<float, false>(batch, m, n, nb, A, lda, sA, S, sS, U, ldu, sU, V, ldv, sV,
                                        tol, max_sweeps, masking, info, sweeps, ws, stream, inner, persistent, t0, rate);
}

hipError_t launch_blocked_z(int batch, int m, int n, int nb, const void *A, int lda, long long sA,
                            double *S, long long sS, void *U, int ldu, long long sU, void *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream, int inner,
                            int persistent, double t0, double rate)
{
    return launch_blocked<double, true>(batch, m, n, nb, (const double2 *)A, lda, sA, S, sS,
                                        (double2 *)U, ldu, sU, (double2 *)V, ldv, sV, tol,
                                        max_sweeps, masking, info, sweeps, ws, stream, inner, persistent, t0, rate);
}

hipError_t launch_blocked_c(int batch, int m, int n, int nb, const void *A, int lda, long long sA,
                            float *S, long long sS, void *U, int ldu, long long sU, void *V,
                            int ldv, long long sV, double tol, int max_sweeps, int masking,
                            int *info, int *sweeps, void *ws, hipStream_t stream, int inner,
                            int persistent, double t0, double rate)
{
    return launch_blocked<float, true>(batch, m, n, nb, (const float2 *)A, lda, sA, S, sS,
                                       (float2 *)U, ldu, sU, (float2 *)V, ldv, sV, tol, max_sweeps,
                                       masking, info, sweeps, ws, stream, inner, persistent, t0, rate);
}

// Mixed mode: FP32 sweeps (FP32 matrix cores, FP64 inner solves) with
// threshold tol32 until each matrix converges or its largest cosine reaches
// kSwitchCos; then Q = orth(V32) in FP64 by two Newton-Schulz steps towards
// the polar factor, Q <- Q (3 I - Q^T Q) / 2; W = scale A Q, V = Q; FP64
// sweeps to tol.
hipError_t launch_blocked_mixed_d(int batch, int m, int n, int nb, const double *A, int lda,
                                  long long sA, double *S, long long sS, double *U, int ldu,
                                  long long sU, double *V, int ldv, long long sV, double tol,
                                  double tol32, int max_sweeps, int masking, int *info,
                                  int *sweeps, void *ws, hipStream_t stream, int inner,
                                  int persistent, double t0, double rate)
{
    const int np = blocked_np(n, nb);
    WsLayout L = carve(ws, batch, m, n, np, sizeof(double), true);
    double *W = (double *)L.W, *Vw = (double *)L.Vw;
    float *W32 = (float *)L.W32, *V32 = (float *)L.V32;
    hipError_t e;
    hipLaunchKernelGGL((blk_init<double, float>), dim3(batch), dim3(kBT), 0, stream, m, n, np, A,
                       lda, sA, W32, V32, L.st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = run_sweeps<float, false>(batch, m, np, nb, W32, V32, L.st, L.ctl, tol32, max_sweeps,
                                 1, 1, inner, persistent, stream, t0, rate);
    if (e != hipSuccess) return e;

    // Newton-Schulz on Q; Q1 lives in the (not yet used) FP64 V area, ld n
    const long long nn = (long long)n * n, vv = (long long)np * np;
    double *Q0 = L.Q, *X = L.X, *Q1 = Vw;
    hipLaunchKernelGGL(v32_to_q, dim3(elementwise_grid((size_t)batch * nn)), dim3(256), 0, stream,
                       batch, n, np, (const float *)V32, Q0);
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
    e = run_sweeps<double, false>(batch, m, np, nb, W, Vw, L.st, L.ctl, tol, max_sweeps,
                                  masking, 0, inner, persistent, stream, t0, rate);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)n * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL((blk_finalize<double, double>), dim3(batch), dim3(kBT), lds, stream, m, n,
                       np, (const double *)W, (const double *)Vw, (const BlkState *)L.st,
                       (const int *)L.sw32, S, sS, U, ldu, sU, V, ldv, sV, info, sweeps);
    return hipGetLastError();
}

}  // namespace svdb

namespace svdb {

size_t vbatched_workspace_bytes(int batch, const int *m, const int *n, int elt)
{
    return vb_layout(nullptr, batch, m, n, (size_t)elt).bytes + 256;
}

hipError_t launch_vbatched(int dtype, int batch, const int *m, const int *n, const void *const *A,
                           const int *lda, void *const *S, void *const *U, const int *ldu,
                           void *const *V, const int *ldv, double tol, int max_sweeps,
                           int masking, int *info, int *sweeps, void *ws, hipStream_t stream,
                           const int *trans, int inner, int persistent, double t0, double rate)
{
    const size_t elt = dtype == 0 ? 4 : dtype == 3 ? 16 : 8;
    return launch_vb(dtype, elt, batch, m, n, A, lda, S, U, ldu, V, ldv, tol, max_sweeps, masking,
                     info, sweeps, ws, stream, trans, inner, persistent, t0, rate);
}

hipError_t launch_gemm_f64(bool trans_a, int batch, int M, int N, int K, double alpha,
                           const double *A, int lda, long long sA, const double *B, int ldb,
                           long long sB, double beta, const double *D, int ldd, long long sD,
                           double *C, int ldc, long long sC, hipStream_t stream)
{
    if (batch <= 0 || M <= 0 || N <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(batch * ((M + 63) / 64) * ((N + 63) / 64));
    if (trans_a)
        hipLaunchKernelGGL(gemm_f64<true>, dim3(grid), dim3(kBT), 0, stream, M, N, K, alpha,
                           (const BlkState *)nullptr, A, lda, sA, B, ldb, sB, beta, D, ldd, sD, C,
                           ldc, sC);
    else
        hipLaunchKernelGGL(gemm_f64<false>, dim3(grid), dim3(kBT), 0, stream, M, N, K, alpha,
                           (const BlkState *)nullptr, A, lda, sA, B, ldb, sB, beta, D, ldd, sD, C,
                           ldc, sC);
    return hipGetLastError();
}

}  // namespace svdb
