// qr.hip -- QR preconditioning of the one-sided Jacobi method for real FP64
// matrices: the QR pre-processing of the section "Other Performance
// Considerations" (subsection on pre-processing with a QR factorization), in
// the form of Drmac and Veselic that the section "Algorithmic Background"
// cites (paragraph "Efficient implementations"): the iteration runs on the
// transposed triangular factor of a column-pivoted QR, after a second,
// unpivoted QR of that factor.
//
//   A P = Q1 R1                pivoted Householder QR (qr_house_d, PIV)
//   R1^T = Q2 R2               unpivoted Householder QR of R1^T (n x n)
//   R2^T J = U_x diag(S)       one-sided Jacobi on X = R2^T (resident kernel)
//   A = (Q1 [U_x; 0]) diag(S) (P Q2 J)^T
//
// so U = Q1 [U_x; 0] and V = P Q2 J (apply_q_d, the second with the row
// permutation P).  The pivoting makes R1 graded (decreasing row norms); the
// second factorisation moves that grading into the columns of X, where the
// one-sided iteration converges markedly faster: on the mixed 64 x 64 /
// 128 x 32 workload the oracle needs 7.2 / 6.5 sweeps on X against 9.4 / 8.4
// on the unpivoted R^T and 14.7 / 11.7 on A.  For m > n every sweep is also
// cheaper (n x n instead of m x n).
//
// Both kernels run one 256-thread workgroup per matrix (m <= 256, n <= 64,
// m n <= 8192).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "launchers.hpp"

namespace svdb {

namespace {

constexpr int kQT = 256;
constexpr int kQrMaxElems = 8192;   // m n doubles in LDS

// Sum over a row of 16 lanes by DPP rotations 8, 4, 2, 1: every lane of the
// row ends with the same bits.
__device__ __forceinline__ double row_sum16(double v)
{
    v += row_ror16<8>(v);
    v += row_ror16<4>(v);
    v += row_ror16<2>(v);
    v += row_ror16<1>(v);
    return v;
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Value of lane SRC of this lane's row of 16 (ds_swizzle in its bit-mask
// form: lane id & 16 | SRC within each half of the wave).
template <int SRC>
__device__ __forceinline__ double row_bcast16(double v)
{
    constexpr int pat = 0x10 | (SRC << 5);
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), pat);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), pat);
    return __hiloint2double(hi, lo);
}

// Sums of w[0..3] over each row of 16 lanes, all four in every lane of the
// row.  Each level halves the values a lane carries: lanes x and x + 8
// exchange the pair the other keeps (columns 0, 1 below lane 8, 2, 3 above),
// then mirrored lanes of each half-row exchange the other column, and the
// quads sum the one left; quad k then holds the sum of column k, which is
// broadcast from its first lane.  27 VALU instructions and 8 swizzles
// against 48 for four separate row sums.
__device__ __forceinline__ void row_sum16x4(double (&w)[4])
{
    const int x = threadIdx.x & 15;
    const bool hi = (x & 8) != 0, up = (x & 4) != 0;
    const double a0 = (hi ? w[2] : w[0]) + dpp_d<0x128>(hi ? w[0] : w[2]);   // row_ror:8
    const double a1 = (hi ? w[3] : w[1]) + dpp_d<0x128>(hi ? w[1] : w[3]);
    double c = (up ? a1 : a0) + dpp_d<0x141>(up ? a0 : a1);                  // row_half_mirror
    c += dpp_d<0xB1>(c);                                                      // quad lanes ^ 1
    c += dpp_d<0x4E>(c);                                                      // quad lanes ^ 2
    w[0] = row_bcast16<0>(c);
    w[1] = row_bcast16<4>(c);
    w[2] = row_bcast16<8>(c);
    w[3] = row_bcast16<12>(c);
}

// The same for two values: lanes x and x + 8 exchange the column the other
// keeps (column 0 below lane 8, 1 above), then each half-row sums its own.
__device__ __forceinline__ void row_sum16x2(double (&w)[2])
{
    const bool hi = (threadIdx.x & 8) != 0;
    double c = (hi ? w[1] : w[0]) + dpp_d<0x128>(hi ? w[0] : w[1]);   // row_ror:8
    c += dpp_d<0x141>(c);                                              // row_half_mirror
    c += dpp_d<0xB1>(c);                                               // quad lanes ^ 1
    c += dpp_d<0x4E>(c);                                               // quad lanes ^ 2
    w[0] = row_bcast16<0>(c);
    w[1] = row_bcast16<8>(c);
}

// One butterfly step of the pivot search over a row of 16 lanes: keeps the
// larger of (norm, column) and its partner ROR lanes on, ordered by norm and
// then by the lower column.
template <int ROR>
__device__ __forceinline__ void arg_max_step(double &nrm, int &col)
{
    const double on = row_ror16<ROR>(nrm);
    const int oc = row_ror16i<ROR>(col);
    const bool take = on > nrm || (on == nrm && oc < col);
    nrm = take ? on : nrm;
    col = take ? oc : col;
}

// Layout of both kernels: the 256 threads form 16 groups of 16 lanes; group
// g owns columns g, g + 16, ... (CPG of them) and lane x of a group holds
// rows x, x + 16, ... (RPL of them) of its columns in registers, so column
// dot products are 16-lane DPP reductions and up to 16 columns are in
// flight at once.

// Householder QR.  Column j's group forms the reflector (v_j(j) = 1, as in
// LAPACK's xGEQRF) and publishes it in LDS; after one barrier every group
// applies it to its own trailing columns.  A is pre-scaled by a power of two
// (max |a| in [1, 2)) so that no square overflows.  Outputs: X = R^T
// (unscaled, n x n; only its lower triangle is written, every reader takes
// the upper one as zero), and for the application of Q the reflectors as
// columns of V (m x n: ones on the diagonal and the vectors below it; the
// part above the diagonal, zero, is neither written nor read) with tau.
//
// PIV: column pivoting as in LAPACK's xGEQP3 (Businger-Golub), the step-j
// pivot being the open column of largest trailing norm (rows j..m-1; ties
// to the lowest index).  Columns stay in their registers: the step order is
// kept in LDS and a second barrier per step publishes the pivot.  The
// trailing squared norms are downdated, n <- n - R(j, c)^2, and recomputed
// from the column once they fall below sqrt(u) times their last exact value
// (the safeguard of xGEQP3; the norms only steer the pivot order, the
// factorisation is exact for any order).  R, V and tau come out in step
// order; perm_out[k] is the column of A taken at step k, so that A P = Q R
// with P e_k = e_perm[k].  lower: A is lower triangular (the transposed
// factor of a first QR); its upper part is taken as zero without being read.
template <int RPL, int CPG, bool PIV>
__global__ __launch_bounds__(kQT) void qr_house_d(int m, int n, const double *__restrict__ A,
                                                  int lda, long long sA, double *X, double *Vq,
                                                  double *tau_out, int *perm_out, int lower)
{
    __shared__ double vbuf[2][16 * RPL];
    __shared__ double s_tau[64];
    __shared__ double s_max[kQT / 64];
    __shared__ int s_bad[kQT / 64];
    __shared__ double s_cn[16];   // PIV: per group, its largest open trailing norm^2
    __shared__ int s_cc[16];      //      and that column (n if it has none open)
    __shared__ int s_step[64];    // PIV: column -> step that took it
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = tid >> 4, gl = tid & 15;
    A += (size_t)b * sA;
    double h[CPG][RPL];
    double amax = 0.0;
    int bad = 0;
#pragma unroll
    for (int c = 0; c < CPG; c++)
#pragma unroll
        for (int r = 0; r < RPL; r++) {
            const int row = gl + 16 * r, col = grp + 16 * c;
            const double a = (row < m && col < n && (!lower || row >= col))
                                 ? A[(size_t)col * lda + row]
                                 : 0.0;
            bad |= !isfinite(a);
            amax = fmax(amax, fabs(a));
            h[c][r] = a;
        }
    amax = wave_max(amax);
    bad = __any(bad);
    if (lane == 0) {
        s_max[wave] = amax;
        s_bad[wave] = bad;
    }
    __syncthreads();
    amax = fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
    // a non-finite input turns X into NaN, which the Jacobi kernel reports
    // (info 2)
    const bool finite = !(s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]);
    const double scale = finite ? pow2_scale(amax) : 1.0;
    double nrm[CPG];   // PIV: trailing squared norms of this group's columns
    double nref[CPG];  // PIV: their values at the last exact computation
    unsigned done = 0;   // PIV: bit c set once column grp + 16 c is a pivot
#pragma unroll
    for (int c = 0; c < CPG; c++) {
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; r++) {
            h[c][r] *= scale;
            t = fma(h[c][r], h[c][r], t);
        }
        nrm[c] = PIV ? row_sum16(t) : 0.0;
        nref[c] = nrm[c];
    }
    if constexpr (PIV) {
        for (int j = 0; j < n && finite; j++) {
            int p = j;   // the column taken at step j
            if (PIV) {
                double best = -1.0;
                int bc = n;
#pragma unroll
                for (int c = 0; c < CPG; c++) {
                    const int col = grp + 16 * c;
                    if (col < n && !((done >> c) & 1u) && nrm[c] > best) {
                        best = nrm[c];
                        bc = col;
                    }
                }
                if (gl == 0) {
                    s_cn[grp] = best;
                    s_cc[grp] = bc;
                }
                __syncthreads();
                // lane x of every row of 16 takes candidate x; a rotation
                // butterfly leaves the largest (norm first, then lowest column:
                // a total order) in all 16 lanes
                best = s_cn[gl];
                p = s_cc[gl];
                arg_max_step<8>(best, p);
                arg_max_step<4>(best, p);
                arg_max_step<2>(best, p);
                arg_max_step<1>(best, p);
                if (tid == 0) s_step[p] = j;
            }
            double *vb = vbuf[j & 1];
            if (grp == (p & 15)) {
                const int cp = p >> 4;
                double x[RPL];
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    x[r] = h[0][r];
#pragma unroll
                    for (int c = 1; c < CPG; c++) x[r] = c == cp ? h[c][r] : x[r];
                }
                double s = 0.0, a = 0.0;
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    const int row = gl + 16 * r;
                    s = row > j ? fma(x[r], x[r], s) : s;
                    a = row == j ? x[r] : a;
                }
                s = row_sum16(s);
                const double alpha = row_sum16(a);   // one nonzero term: exact
                double beta = alpha, tau = 0.0, scal = 0.0;
                if (s > 0.0) {
                    const double nrmj = sqrt(fma(alpha, alpha, s));
                    beta = alpha >= 0.0 ? -nrmj : nrmj;
                    tau = (beta - alpha) / beta;
                    scal = 1.0 / (alpha - beta);
                }
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    const int row = gl + 16 * r;
                    const double v = row == j ? 1.0 : (row > j ? x[r] * scal : 0.0);
                    vb[row] = v;
                    x[r] = row == j ? beta : (row > j ? v : x[r]);
                }
#pragma unroll
                for (int c = 0; c < CPG; c++)
#pragma unroll
                    for (int r = 0; r < RPL; r++) h[c][r] = c == cp ? x[r] : h[c][r];
                if (PIV) done |= 1u << cp;
                if (gl == 0) s_tau[j] = tau;
            }
            __syncthreads();
            const double tau = s_tau[j];
            double v[RPL];
#pragma unroll
            for (int r = 0; r < RPL; r++) v[r] = vb[gl + 16 * r];
#pragma unroll
            for (int c = 0; c < CPG; c++) {
                const int col = grp + 16 * c;
                const bool open = PIV ? (col < n && !((done >> c) & 1u)) : (col > j && col < n);
                if (open) {   // uniform in the group
                    if (tau != 0.0) {
                        double w = 0.0;
#pragma unroll
                        for (int r = 0; r < RPL; r++) w = fma(v[r], h[c][r], w);
                        w = row_sum16(w) * tau;
#pragma unroll
                        for (int r = 0; r < RPL; r++) h[c][r] = fma(-w, v[r], h[c][r]);
                    }
                    if (PIV) {
                        // R(j, col) sits in lane j mod 16 of the group, slot j / 16
                        double rj = h[c][0];
#pragma unroll
                        for (int r = 1; r < RPL; r++) rj = r == (j >> 4) ? h[c][r] : rj;
                        rj = __shfl(rj, (lane & 48) | (j & 15), 64);
                        double nn = fmax(fma(-rj, rj, nrm[c]), 0.0);
                        if (nn <= 0x1p-26 * nref[c]) {   // uniform in the group
                            double t = 0.0;
#pragma unroll
                            for (int r = 0; r < RPL; r++) {
                                const int row = gl + 16 * r;
                                t = row > j ? fma(h[c][r], h[c][r], t) : t;
                            }
                            nn = row_sum16(t);
                            nref[c] = nn;
                        }
                        nrm[c] = nn;
                    }
                }
            }
        }
        __syncthreads();
        // X = R^T / scale: X(k, row) = R(row, k) for row <= k (the lower
        // triangle of X), where k is the step of the column; the reflectors
        // from the diagonal down, in step order
        X += (size_t)b * n * n;
        const double inv = 1.0 / scale;
        if (Vq) Vq += (size_t)b * m * n;
#pragma unroll
        for (int c = 0; c < CPG; c++) {
            const int col = grp + 16 * c;
            if (col >= n) continue;
            const int k = PIV && finite ? s_step[col] : col;
#pragma unroll
            for (int r = 0; r < RPL; r++) {
                const int row = gl + 16 * r;
                if (row >= m) continue;
                const double x = h[c][r];
                if (row < n && (!finite || row <= k))
                    X[(size_t)row * n + k] = finite ? x * inv : __builtin_nan("");
                if (Vq && row >= k) Vq[(size_t)k * m + row] = row > k ? x : 1.0;
            }
            if (PIV && perm_out && gl == 0) perm_out[(size_t)b * n + k] = col;
        }
    } else {
        // Without pivoting step j takes column j, held in slot j / 16; with
        // the slot loop unrolled the slot is known where the column is read.
        // The column is final at its step (its rows above j were finished by
        // earlier steps), so its owner group writes it out after the barrier
        // (X = R^T, the reflector as a full column) and keeps nothing of it.
        X += (size_t)b * n * n;
        const double inv = 1.0 / scale;
        if (Vq) Vq += (size_t)b * m * n;
        auto step = [&](int j, int cp) __attribute__((always_inline)) {
            double *vb = vbuf[j & 1];
            const bool owner = grp == (j & 15);
            double x[RPL];   // owner: the finished column (R above, beta, v below)
            if (owner) {
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    x[r] = h[0][r];
#pragma unroll
                    for (int c = 1; c < CPG; c++) x[r] = c == cp ? h[c][r] : x[r];
                }
                double s = 0.0, a = 0.0;
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    const int row = gl + 16 * r;
                    s = row > j ? fma(x[r], x[r], s) : s;
                    a = row == j ? x[r] : a;
                }
                s = row_sum16(s);
                const double alpha = row_sum16(a);   // one nonzero term: exact
                double beta = alpha, tau = 0.0, scal = 0.0;
                if (s > 0.0) {
                    const double nrmj = sqrt(fma(alpha, alpha, s));
                    beta = alpha >= 0.0 ? -nrmj : nrmj;
                    tau = (beta - alpha) / beta;
                    scal = 1.0 / (alpha - beta);
                }
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    const int row = gl + 16 * r;
                    const double v = row == j ? 1.0 : (row > j ? x[r] * scal : 0.0);
                    vb[row] = v;
                    x[r] = row == j ? beta : (row > j ? v : x[r]);
                }
                if (gl == 0) s_tau[j] = tau;
            }
            __syncthreads();
            // the owner's stores, off the path to the barrier
            if (owner) {
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    const int row = gl + 16 * r;
                    if (row <= j) X[(size_t)row * n + j] = x[r] * inv;
                    if (Vq && row < m && row >= j) Vq[(size_t)j * m + row] = row > j ? x[r] : 1.0;
                }
            }
            const double tau = s_tau[j];
            double v[RPL];
#pragma unroll
            for (int r = 0; r < RPL; r++) v[r] = vb[gl + 16 * r];
#pragma unroll
            for (int c = 0; c < CPG; c++) {
                const int col = grp + 16 * c;
                if (col > j && col < n) {   // uniform in the group
                    if (tau != 0.0) {
                        double w = 0.0;
#pragma unroll
                        for (int r = 0; r < RPL; r++) w = fma(v[r], h[c][r], w);
                        w = row_sum16(w) * tau;
#pragma unroll
                        for (int r = 0; r < RPL; r++) h[c][r] = fma(-w, v[r], h[c][r]);
                    }
                }
            }
        };
        if (finite) {
#pragma unroll
            for (int cp = 0; cp < CPG; cp++)
                for (int jj = 0; jj < 16; jj++) {
                    const int j = 16 * cp + jj;
                    if (j >= n) break;
                    step(j, cp);
                }
        } else {
            // a non-finite input turns X into NaN, which the Jacobi kernel
            // reports (info 2); nothing else is read
#pragma unroll
            for (int c = 0; c < CPG; c++) {
                const int col = grp + 16 * c;
                if (col >= n) continue;
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    const int row = gl + 16 * r;
                    if (row < n) X[(size_t)row * n + col] = __builtin_nan("");
                }
            }
        }
    }
    if (Vq && tid < n) tau_out[(size_t)b * n + tid] = finite ? s_tau[tid] : 0.0;
}

// ---------------------------------------------------------------------------
// The same factorisation for m <= 64, one wavefront per matrix and one column
// per lane: lane c holds column c in registers, rows in MB blocks of 16
// (a[B][i] = row 16 B + i).  A step then works inside the lanes: the dot
// products of the open columns with the step's column and their update are
// FMA chains in each lane, the step's column reaches every lane as a
// broadcast read of LDS, its norm and entry on the diagonal come from its
// lane by readlane, and the pivot is a maximum over the wave.  Nothing waits
// on another wavefront.
//
// The steps of block B run in a loop over its 16 rows, and the block's 16
// registers form a window that rotates by one register per step: row j is
// always a[B][0], rows j+1 .. 16 B + 15 follow it, and the rows the block has
// finished sit at the window's tail.  The copy of the step's column in LDS
// holds zeros there and in row j, so one dot product over the window and the
// blocks below gives every lane the sum over rows > j, and the update leaves
// the finished rows alone.  After its 16 steps the window is back in order.
//
// Pivot (PIV): the open column of largest downdated trailing norm, ties to
// the lowest column, with the norm compared to 2^-46 relative: the maximum
// over the wave is taken on the bits of the norm (a nonnegative double, so
// its bits order as the values) with the six lowest replaced by 63 - c.
// The downdate and its safeguard are those of qr_house_d.
//
// Outputs as for qr_house_d.  The taken column keeps alpha on its diagonal
// and x below it; beta and 1 / (alpha - beta) are applied when it is written
// out.  The reflectors leave through an LDS tile, 16 rows at a time, so that
// each store covers whole rows of 16 entries.
__device__ __forceinline__ void lane_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Largest signed 64-bit key over the 64 lanes, in every lane (rotations
// inside rows of 16, then the row swaps of v_permlane16_swap and
// v_permlane32_swap: each step pairs two operands the same way in both
// lanes, so every lane ends with the same key).  Integer keys: whatever bits
// an open column's norm holds, its key (sign bit clear) beats the -1 of a
// taken column, so the pivot is always an open column.
__device__ __forceinline__ long long key_of(int lo, int hi)
{
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int ROR>
__device__ __forceinline__ long long row_ror16_key(long long v)
{
    const int lo = __builtin_amdgcn_mov_dpp((int)v, 0x120 + ROR, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), 0x120 + ROR, 0xF, 0xF, false);
    return key_of(lo, hi);
}

__device__ __forceinline__ long long lane_max_key(long long v)
{
    long long o;
    o = row_ror16_key<8>(v);
    v = o > v ? o : v;
    o = row_ror16_key<4>(v);
    v = o > v ? o : v;
    o = row_ror16_key<2>(v);
    v = o > v ? o : v;
    o = row_ror16_key<1>(v);
    v = o > v ? o : v;
    {
        auto lo = __builtin_amdgcn_permlane16_swap((int)v, (int)v, false, false);
        auto hi = __builtin_amdgcn_permlane16_swap((int)(v >> 32), (int)(v >> 32), false, false);
        const long long a = key_of(lo[0], hi[0]), b = key_of(lo[1], hi[1]);
        v = a > b ? a : b;
    }
    {
        auto lo = __builtin_amdgcn_permlane32_swap((int)v, (int)v, false, false);
        auto hi = __builtin_amdgcn_permlane32_swap((int)(v >> 32), (int)(v >> 32), false, false);
        const long long a = key_of(lo[0], hi[0]), b = key_of(lo[1], hi[1]);
        v = a > b ? a : b;
    }
    return v;
}

__device__ __forceinline__ double lane_bcast(double v, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Rows 16 t .. 16 t + 15 of the step's column from LDS (eight 16-byte
// broadcast reads).
__device__ __forceinline__ void lds_chunk(const double *xs, int t, double2 (&x)[8])
{
#pragma unroll
    for (int q = 0; q < 8; q++) x[q] = *reinterpret_cast<const double2 *>(&xs[16 * t + 2 * q]);
}

template <int MB, bool PIV>
__global__ __launch_bounds__(64, 2) void qr_lane_d(int m, int n, const double *__restrict__ A,
                                                   int lda, long long sA, double *X, double *Vq,
                                                   double *tau_out, int *perm_out)
{
    __shared__ __align__(16) double xs_[16 * MB];   // the step's column, rows 16 B ..
    __shared__ double tile[64][17];                 // reflectors on their way out
    const int b = blockIdx.x, c = threadIdx.x;
    // one address register for every access to xs (constant offsets)
    int zero;
    __asm__ volatile("v_mov_b32 %0, 0" : "=v"(zero));
    double *xs = xs_ + zero;
    A += (size_t)b * sA;
    double a[MB][16];
    double amax = 0.0;
    int bad = 0;
#pragma unroll
    for (int B = 0; B < MB; B++)
#pragma unroll
        for (int i = 0; i < 16; i++) {
            const int row = 16 * B + i;
            const double v = (row < m && c < n) ? A[(size_t)c * lda + row] : 0.0;
            bad |= !isfinite(v);
            amax = fmax(amax, fabs(v));
            a[B][i] = v;
        }
    amax = wave_max(amax);
    const bool finite = !__any(bad);
    const double scale = finite ? pow2_scale(amax) : 1.0;
    double nrm = 0.0;
    {
        double t[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int B = 0; B < MB; B++)
#pragma unroll
            for (int i = 0; i < 16; i++) {
                a[B][i] *= scale;
                if (PIV) t[i & 3] = fma(a[B][i], a[B][i], t[i & 3]);
            }
        nrm = (t[0] + t[1]) + (t[2] + t[3]);
    }
    double nref = nrm;
    int step = c < n ? -1 : 64;   // -1 while open
    double beta_l = 0.0, scal_l = 0.0, tau_l = 0.0;
    if (finite) {
#pragma unroll
        for (int B = 0; B < MB; B++) {
            if (16 * B >= n) break;
#pragma unroll 1
            for (int jj = 0; jj < 16; jj++) {
                const int j = 16 * B + jj;
                if (j < n) {   // uniform
                    const bool open = step < 0;
                    int p = j;
                    if constexpr (PIV) {
                        long long key = -1;
                        if (open) {
                            const unsigned long long u = __double_as_longlong(nrm);
                            key = (long long)((u & 0x7fffffffffffffc0ull) | (unsigned)(63 - c));
                        }
                        key = lane_max_key(key);
                        p = __builtin_amdgcn_readfirstlane(63 - (int)(key & 63));
                    }
                    // column p, rows 16 B .. of it, with row j and the
                    // finished rows of the window zeroed
                    if (c == p) {
#pragma unroll
                        for (int k = 0; k < 16; k += 2)
                            *reinterpret_cast<double2 *>(&xs[k]) = make_double2(a[B][k], a[B][k + 1]);
#pragma unroll
                        for (int B2 = B + 1; B2 < MB; B2++)
#pragma unroll
                            for (int i = 0; i < 16; i += 2)
                                *reinterpret_cast<double2 *>(&xs[16 * (B2 - B) + i]) =
                                    make_double2(a[B2][i], a[B2][i + 1]);
                    }
                    if (c < 16 && (c == 0 || c >= 16 - jj)) xs[c] = 0.0;
                    lane_sync_lds();
                    // d = sum over rows > j of x_r a_r (for lane p: ||x below j||^2),
                    // in the lanes that need it: the broadcast reads cost LDS
                    // bandwidth per active lane
                    const bool upd = open && c != p;
                    double dd[4] = {0.0, 0.0, 0.0, 0.0};
                    if (upd || c == p) {
                        // chunk t: rows 16 t .. of xs against a[B + t] (the
                        // window for t = 0, without row j), the next chunk's
                        // reads issued before this chunk's FMAs
                        double2 xb[2][8];
                        lds_chunk(xs, 0, xb[0]);
#pragma unroll
                        for (int t = 0; t < MB - B; t++) {
                            if (t + 1 < MB - B) lds_chunk(xs, t + 1, xb[(t + 1) & 1]);
                            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                            for (int q = 0; q < 8; q++) {
                                const double2 x = xb[t & 1][q];
                                if (t > 0 || q > 0) dd[(2 * q) & 3] = fma(x.x, a[B + t][2 * q], dd[(2 * q) & 3]);
                                dd[(2 * q + 1) & 3] = fma(x.y, a[B + t][2 * q + 1], dd[(2 * q + 1) & 3]);
                            }
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                    const double d = (dd[0] + dd[1]) + (dd[2] + dd[3]);
                    // the reflector of xGEQRF: beta = -sign(alpha) ||x||,
                    // tau = (beta - alpha) / beta, v = x / (alpha - beta), v_j = 1
                    const double s = lane_bcast(d, p), alpha = lane_bcast(a[B][0], p);
                    double beta = alpha, tau = 0.0, scal = 0.0;
                    if (s > 0.0) {
                        const double nrmj = sqrt(fma(alpha, alpha, s));
                        beta = alpha >= 0.0 ? -nrmj : nrmj;
                        tau = (beta - alpha) / beta;
                        scal = 1.0 / (alpha - beta);
                    }
                    if (tau != 0.0 && upd) {
                        // a <- a - tau (v^T a) v on the open columns
                        const double f = tau * fma(scal, d, a[B][0]);
                        const double g = f * scal;
                        a[B][0] -= f;
                        double2 xb[2][8];
                        lds_chunk(xs, 0, xb[0]);
#pragma unroll
                        for (int t = 0; t < MB - B; t++) {
                            if (t + 1 < MB - B) lds_chunk(xs, t + 1, xb[(t + 1) & 1]);
                            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                            for (int q = 0; q < 8; q++) {
                                const double2 x = xb[t & 1][q];
                                if (t > 0 || q > 0) a[B + t][2 * q] = fma(-g, x.x, a[B + t][2 * q]);
                                a[B + t][2 * q + 1] = fma(-g, x.y, a[B + t][2 * q + 1]);
                            }
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                    if (c == p) {
                        step = j;
                        beta_l = beta;
                        scal_l = scal;
                        tau_l = tau;
                    }
                    if constexpr (PIV) {
                        // trailing norm over rows > j: downdate by R(j, c)^2,
                        // recomputed once it has fallen below sqrt(u) of its
                        // last exact value
                        double nn = fmax(fma(-a[B][0], a[B][0], nrm), 0.0);
                        const bool again = upd && nn <= 0x1p-26 * nref;
                        if (__any(again)) {
                            double t = 0.0;
#pragma unroll
                            for (int k = 1; k < 16; k++) t = k <= 15 - jj ? fma(a[B][k], a[B][k], t) : t;
#pragma unroll
                            for (int B2 = B + 1; B2 < MB; B2++)
#pragma unroll
                                for (int i = 0; i < 16; i++) t = fma(a[B2][i], a[B2][i], t);
                            nn = again ? t : nn;
                            nref = again ? t : nref;
                        }
                        nrm = upd ? nn : nrm;
                    }
                    lane_sync_lds();   // the reads of xs before the next step's writes
                }
                // rotate the window: row j + 1 into a[B][0], row j to the tail
                const double r0 = a[B][0];
#pragma unroll
                for (int k = 0; k < 15; k++) a[B][k] = a[B][k + 1];
                a[B][15] = r0;
            }
        }
    }
    // X = R^T / scale: X(k, row) = R(row, k) for row <= k (the lower
    // triangle of X), k the step of the lane's column
    const int k = finite ? step : c;
    const double inv = 1.0 / scale;
    X += (size_t)b * n * n;
    if (c < n) {
#pragma unroll
        for (int B = 0; B < MB; B++)
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const int row = 16 * B + i;
                if (row >= n || (finite && row > k)) continue;
                const double r = row < k ? a[B][i] : beta_l;
                X[(size_t)row * n + k] = finite ? r * inv : __builtin_nan("");
            }
        if (PIV && perm_out) perm_out[(size_t)b * n + k] = c;
        if (Vq) tau_out[(size_t)b * n + k] = tau_l;
    }
    if (Vq && finite) {
        // the reflectors from the diagonal down, in step order
        Vq += (size_t)b * m * n;
#pragma unroll
        for (int B = 0; B < MB; B++) {
            if (c < n) {
#pragma unroll
                for (int i = 0; i < 16; i++) {
                    const int row = 16 * B + i;
                    tile[k][i] = row > k ? a[B][i] * scal_l : (row == k ? 1.0 : 0.0);
                }
            }
            lane_sync_lds();
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int kk = 4 * q + (c >> 4), row = 16 * B + (c & 15);
                if (kk < n && row < m && row >= kk) Vq[(size_t)kk * m + row] = tile[kk][c & 15];
            }
            lane_sync_lds();
        }
    }
}

// U = Q [Y; 0] = H_0 ... H_{n-1} [Y; 0] (Y n x n, ld n), the reflectors (in
// LDS, zero above the diagonal) applied last to first to the register-held
// U; no barrier after the reflectors are loaded.  With perm (m = n), row k of the
// product is stored as row perm[k] of U.  Matrices with info 2 (non-finite
// input) are left untouched.
template <int RPL, int CPG>
__global__ __launch_bounds__(kQT) void apply_q_d(int m, int n, const double *__restrict__ Vq,
                                                 const double *__restrict__ tau,
                                                 const double *__restrict__ Y, double *U, int ldu,
                                                 long long sU, const int *info,
                                                 const int *__restrict__ perm,
                                                 const int *__restrict__ only)
{
    extern __shared__ double Vl[];   // m x n, ld m
    __shared__ double s_tau[64];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int grp = tid >> 4, gl = tid & 15;
    if (info[b] == 2 || (only && !only[b])) return;
    Vq += (size_t)b * m * n;
    Y += (size_t)b * n * n;
    U += (size_t)b * sU;
    // the reflectors are zero above the diagonal: those entries are not read
    {
        int col = tid / m, row = tid - col * m;
        constexpr int kStep = kQT;
        const int dc = kStep / m, dr = kStep - dc * m;
        for (int idx = tid; idx < m * n; idx += kStep) {
            Vl[idx] = row >= col ? Vq[idx] : 0.0;
            row += dr;
            col += dc;
            if (row >= m) {
                row -= m;
                col++;
            }
        }
    }
    if (tid < n) s_tau[tid] = tau[(size_t)b * n + tid];
    double u[CPG][RPL];
#pragma unroll
    for (int c = 0; c < CPG; c++)
#pragma unroll
        for (int r = 0; r < RPL; r++) {
            const int row = gl + 16 * r, col = grp + 16 * c;
            u[c][r] = (row < n && col < n) ? Y[(size_t)col * n + row] : 0.0;
        }
    __syncthreads();
    for (int j = n - 1; j >= 0; j--) {
        const double t = s_tau[j];
        if (t == 0.0) continue;
        double v[RPL];
#pragma unroll
        for (int r = 0; r < RPL; r++) {
            const int row = gl + 16 * r;
            v[r] = row < m ? Vl[(size_t)j * m + row] : 0.0;
        }
        // the transposing row sums where they measured faster (U of 64x64
        // and V of 32x32; not U of 128x32, RPL = 8)
        if constexpr (CPG == 4 || (CPG == 2 && RPL <= 4)) {
            double w[CPG];
#pragma unroll
            for (int c = 0; c < CPG; c++) {
                w[c] = 0.0;
#pragma unroll
                for (int r = 0; r < RPL; r++) w[c] = fma(v[r], u[c][r], w[c]);
            }
            if constexpr (CPG == 4)
                row_sum16x4(w);
            else
                row_sum16x2(w);
#pragma unroll
            for (int c = 0; c < CPG; c++) {
                const double f = w[c] * t;
#pragma unroll
                for (int r = 0; r < RPL; r++) u[c][r] = fma(-f, v[r], u[c][r]);
            }
        } else {
#pragma unroll
            for (int c = 0; c < CPG; c++) {
                double w = 0.0;
#pragma unroll
                for (int r = 0; r < RPL; r++) w = fma(v[r], u[c][r], w);
                w = row_sum16(w) * t;
#pragma unroll
                for (int r = 0; r < RPL; r++) u[c][r] = fma(-w, v[r], u[c][r]);
            }
        }
    }
    if (perm) perm += (size_t)b * n;
#pragma unroll
    for (int r = 0; r < RPL; r++) {
        const int row = gl + 16 * r;
        if (row >= m) continue;
        const int dst = perm ? perm[row] : row;
#pragma unroll
        for (int c = 0; c < CPG; c++) {
            const int col = grp + 16 * c;
            if (col < n) U[(size_t)col * ldu + dst] = u[c][r];
        }
    }
}

// V from the left vectors of the Jacobi on X = R2^T, without its rotations.
// With A P = Q1 R1 and R1^T = Q2 R2 we have X = R1 Q2, so X V_x = U_x S gives
// V = P Q2 V_x = P R1^-1 U_x S: a back substitution with the pivoted QR's
// triangular factor, as in the preconditioned Jacobi SVD of Drmac and
// Veselic (the section "Algorithmic Background", paragraph "Efficient
// implementations", cites it).  Neither the rotations of the Jacobi nor Q2
// are applied.  The product is accurate when U_x S is the one-sided Jacobi's
// (column-wise backward stable) iterate and R1 is well conditioned up to row
// scaling (R1 from the column-pivoted QR, whose rows are graded); it is kept
// only if the largest row sum of |J^T J - I| is at most thr for
// J = R1^-1 U_x S, else flag[b] = 1 asks for the V-accumulating Jacobi on
// this matrix.
//
// One wave per matrix (n <= 64), column c of J in lane c.  R1 = X1^T (X1 n x
// n, ld n, lower triangular) is staged in LDS as a packed upper triangle,
// column k holding rows 0..k (padded to an even length, so that pairs of
// rows are 16-byte reads); every lane reads the same entries.  A system with
// n < 64 is embedded as diag(R1, I).  J^T J is formed on the FP64 matrix
// cores from rows of J passed through LDS eight at a time, ten 16 x 16
// blocks (the upper triangle).  V(perm[k], c) = J(k, c) goes to the output
// directly (perm NULL: the identity, a QR without pivoting).  Matrices with
// info 2 get flag 0 and are left untouched.
__host__ __device__ constexpr int rp_off(int k)
{
    return (k & 1) ? (k + 1) * (k + 1) / 2 : k * (k + 2) / 2;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int N>
__global__ __launch_bounds__(64, 2) void solve_r1_d(int n, const double *__restrict__ X1,
                                                    const double *__restrict__ Ux,
                                                    const double *__restrict__ S, long long sS,
                                                    const int *__restrict__ perm, double *V,
                                                    int ldv, long long sV, int *flag,
                                                    const int *__restrict__ info, double thr)
{
    static_assert(N == 64, "one column of J per lane, four 16-column blocks");
    constexpr int kR = rp_off(N);          // packed triangle
    constexpr int kRow = N + 16;           // row of J in LDS (2-way bank spread)
    constexpr int kChunk = 8;              // rows of J per pass through LDS
    __shared__ __align__(16) double sm[kR > 2 * kChunk * kRow ? kR : 2 * kChunk * kRow];
    __shared__ double s_inv[N], s_sink[N];
    const int b = blockIdx.x, c = threadIdx.x;
    if (info[b] == 2) {
        if (c == 0) flag[b] = 0;
        return;
    }
    const bool act = c < n;
    const int cc = act ? c : n - 1;
    X1 += (size_t)b * n * n;
    Ux += (size_t)b * n * n;
    V += (size_t)b * sV;
    // ---- R1 into LDS: lane c writes its column, rows 0..c -----------------
    // Loads and stores are unconditional (clamped addresses; the entries
    // below the diagonal go to a per-lane sink), so that all the loads of a
    // lane are in flight together.
    {
        double *col = sm + rp_off(c);
        double x[N];
#pragma unroll
        for (int k = 0; k < N; k++) {
            // R1(k, c); lanes below the diagonal (c < k, bound for the sink)
            // read R1(k, k), so that a row's loads touch only its upper part
            const int kk = k < n ? k : n - 1;
            x[k] = X1[(size_t)kk * n + (cc > kk ? cc : kk)];
        }
#pragma unroll
        for (int k = 0; k < N; k++) {
            double *dst = k <= c ? col + k : s_sink + c;
            *dst = act ? x[k] : (k == c ? 1.0 : 0.0);
        }
        s_inv[c] = act ? 1.0 / x[c < N ? c : 0] : 1.0;
    }
    const double sc = act ? S[(size_t)b * sS + c] : 0.0;
    double y[N];
#pragma unroll
    for (int i = 0; i < N; i++) y[i] = Ux[(size_t)cc * n + (i < n ? i : 0)];
#pragma unroll
    for (int i = 0; i < N; i++) y[i] = (act && i < n) ? y[i] * sc : 0.0;
    __syncthreads();
    // ---- back substitution, R1 y = U_x(:, c) s_c ---------------------------
#pragma unroll
    for (int k = N - 1; k >= 0; k--) {
        const double *rk = sm + rp_off(k);
        y[k] *= s_inv[k];
#pragma unroll
        for (int i = 0; i < k; i += 2) {
            const double2 r = *reinterpret_cast<const double2 *>(rk + i);
            y[i] = fma(-r.x, y[k], y[i]);
            if (i + 1 < k) y[i + 1] = fma(-r.y, y[k], y[i + 1]);
        }
    }
    __syncthreads();   // the triangle is no longer read
    // ---- V = P J, through LDS 32 columns at a time ---------------------------
    // lane c puts J(k, c) at row perm[k] of its column (stride N + 1: the 32
    // lanes hit distinct banks), then each column goes out as one coalesced
    // store, lane r writing row r
    {
        constexpr int kLd = N + 1;
        static_assert(32 * kLd <= kR, "32 columns of V fit in the triangle's memory");
        const int pv = perm ? perm[(size_t)b * n + cc] : cc;   // lane k holds perm[k]
#pragma unroll
        for (int h = 0; h < 2; h++) {
            double *col = sm + (c & 31) * kLd;
            const bool mine = (c >> 5) == h && act;
#pragma unroll
            for (int k = 0; k < N; k++) {
                const int pk = __builtin_amdgcn_readlane(pv, k);
                if (mine && k < n) col[pk] = y[k];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 8
            for (int j = 0; j < 32; j++) {
                const int cj = 32 * h + j;
                if (cj < n && act) V[(size_t)cj * ldv + c] = sm[j * kLd + c];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    // ---- J^T J on the matrix cores --------------------------------------------
    // operand of 16-column block P at row step s: lane l supplies
    // J(4 s + l / 16, 16 P + l % 16), as A (transposed) and as B; result
    // register v of lane l is entry (4 v + l / 16, l % 16) of the block
    const int l16 = c & 15, l4 = c >> 4;
    dbl4 acc[10];
#pragma unroll
    for (int t = 0; t < 10; t++) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r0 = 0; r0 < N; r0 += kChunk) {
        double *buf = sm + ((r0 / kChunk) & 1) * kChunk * kRow;
#pragma unroll
        for (int r = 0; r < kChunk; r++) buf[r * kRow + c] = y[r0 + r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int s4 = 0; s4 < kChunk; s4 += 4) {
            double o[4];
#pragma unroll
            for (int P = 0; P < 4; P++) o[P] = buf[(s4 + l4) * kRow + 16 * P + l16];
            int t = 0;
#pragma unroll
            for (int P = 0; P < 4; P++)
#pragma unroll
                for (int Q = P; Q < 4; Q++, t++)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(o[P], o[Q], acc[t], 0, 0, 0);
        }
    }
    // the largest row sum of |J^T J - I| (the 1-norm of this symmetric
    // matrix, the paper's orthogonality measure times n), summed in a fixed
    // order so that the decision is reproducible; FP32 suffices for a test
    // against thr.  NaN or Inf anywhere fails it.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    constexpr int kE = N + 1;
    static_assert(N * kE * sizeof(float) <= kR * sizeof(double), "|E| fits the triangle's memory");
    float *ea = reinterpret_cast<float *>(sm);
    {
        int t = 0;
#pragma unroll
        for (int P = 0; P < 4; P++)
#pragma unroll
            for (int Q = P; Q < 4; Q++, t++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int i = 16 * P + 4 * v + l4, j = 16 * Q + l16;
                    const double e = acc[t][v] - (i == j ? 1.0 : 0.0);
                    const float ae = (i < n && j < n) ? (float)fabs(e) : 0.0f;
                    ea[i * kE + j] = ae;
                    if (P != Q) ea[j * kE + i] = ae;
                }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float rs = 0.0f;
#pragma unroll 8
    for (int k = 0; k < N; k++) rs += ea[c * kE + k];
    const bool bad = !(rs <= (float)thr);
    const bool any_bad = __any(bad);
    if (c == 0) flag[b] = any_bad ? 1 : 0;
}

// rows per lane (power of two) and columns per group for an m x n matrix
bool qr_shape(int m, int n, int *rpl, int *cpg)
{
    const int r = (m + 15) / 16;
    const int rp = r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : r <= 8 ? 8 : r <= 16 ? 16 : 0;
    const int cp = (n + 15) / 16;
    if (!rp || cp < 1 || cp > 4) return false;
    *rpl = rp;
    *cpg = cp;
    return true;
}

// ---------------------------------------------------------------------------
// Wide matrices (n > 64, m <= 1024): the same QR in global memory, for the
// block path.  qr_house_g factors one matrix per workgroup in place in the
// workspace (16-lane groups share out the trailing columns, the reflector of
// the step is staged in LDS, two barriers per column); apply_q_g applies Q to one
// block of 16 columns of U per workgroup, held in registers.
// ---------------------------------------------------------------------------
constexpr int kQrMaxM = 1024;
constexpr int kQrMaxN = 512;
constexpr int kTallMaxM = 4096;   // tall path: m x n with n <= 64

// One matrix per workgroup: A (m x n, lda; FP64 or FP32) -> H (the
// workspace, m x n, ld m): R in the upper triangle, then the reflectors as
// full columns; X = R^T (unscaled, n x n, ld n); tau (n).  vbuf: 2 m
// doubles of LDS (the double-buffered reflector of the step).
template <class TA>
__device__ __forceinline__ void qr_house_body(int m, int n, const TA *__restrict__ A, int lda,
                                              double *H, double *X, double *tau, double *vbuf)
{
    __shared__ double s_tau[2];
    __shared__ double s_max[kQT / 64];
    __shared__ int s_bad[kQT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = tid >> 4, gl = tid & 15;
    double amax = 0.0;
    int bad = 0;
    for (size_t idx = tid; idx < (size_t)m * n; idx += kQT) {
        const double a = (double)A[(idx / m) * lda + idx % m];
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
    amax = fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
    const bool finite = !(s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]);
    const double scale = finite ? pow2_scale(amax) : 1.0;
    for (size_t idx = tid; idx < (size_t)m * n; idx += kQT)
        H[idx] = (double)A[(idx / m) * lda + idx % m] * scale;
    __syncthreads();
    for (int j = 0; j < n && finite; j++) {
        double *vb = vbuf + (j & 1) * m;
        double *hj = H + (size_t)j * m;
        if (grp == (j & 15)) {
            double s = 0.0;
            for (int i = j + 1 + gl; i < m; i += 16) s = fma(hj[i], hj[i], s);
            s = row_sum16(s);
            const double alpha = hj[j];
            double beta = alpha, tau_j = 0.0, scal = 0.0;
            if (s > 0.0) {
                const double nrm = sqrt(fma(alpha, alpha, s));
                beta = alpha >= 0.0 ? -nrm : nrm;
                tau_j = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            for (int i = j + 1 + gl; i < m; i += 16) {
                const double v = hj[i] * scal;
                vb[i] = v;
                hj[i] = v;
            }
            if (gl == 0) {
                vb[j] = 1.0;
                hj[j] = beta;
                s_tau[j & 1] = tau_j;
                tau[j] = tau_j;
            }
        }
        __syncthreads();
        const double t = s_tau[j & 1];
        if (t != 0.0) {
            for (int k = j + 1 + grp; k < n; k += 16) {
                double *hk = H + (size_t)k * m;
                double w = 0.0;
                for (int i = j + gl; i < m; i += 16) w = fma(vb[i], hk[i], w);
                w = row_sum16(w) * t;
                for (int i = j + gl; i < m; i += 16) hk[i] = fma(-w, vb[i], hk[i]);
            }
        }
        __syncthreads();   // the trailing columns are final before the next step reads them
    }
    __syncthreads();
    // X = R^T / scale, then the reflectors as full columns
    const double inv = 1.0 / scale;
    for (size_t idx = tid; idx < (size_t)n * n; idx += kQT) {
        const int r = (int)(idx % n), c = (int)(idx / n);   // X(r, c) = R(c, r)
        X[idx] = !finite ? __builtin_nan("") : (r >= c ? H[(size_t)r * m + c] * inv : 0.0);
    }
    __syncthreads();
    for (size_t idx = tid; idx < (size_t)m * n; idx += kQT) {
        const int row = (int)(idx % m), col = (int)(idx / m);
        if (row <= col) H[idx] = row == col ? 1.0 : 0.0;
    }
    if (!finite)
        for (int j = tid; j < n; j += kQT) tau[j] = 0.0;
}

// reflector buffer: dynamic LDS of 2 m doubles
__global__ __launch_bounds__(kQT) void qr_house_g(int m, int n, const double *__restrict__ A,
                                                  int lda, long long sA, double *Vq, double *X,
                                                  double *tau_out)
{
    extern __shared__ double vdyn[];
    const int b = blockIdx.x;
    qr_house_body<double>(m, n, A + (size_t)b * sA, lda, Vq + (size_t)b * m * n,
                          X + (size_t)b * n * n, tau_out + (size_t)b * n, vdyn);
}

// U = Q [Y; 0] for tall matrices (n <= 64, m <= kTallMaxM): one wave per
// column of U (four per workgroup), lane x holding rows x, x + 64, ...  (RPL
// of them) in registers; the reflector of each step is staged in LDS
// (dynamic, 2 * 64 RPL doubles, double buffered, one barrier per step) and
// every column dot product is a wave reduction.
template <int RPL>
__global__ __launch_bounds__(kQT) void apply_q_tall(int m, int n, const double *__restrict__ Vq,
                                                    const double *__restrict__ tau,
                                                    const double *__restrict__ Y, double *U,
                                                    int ldu, long long sU, const int *info)
{
    extern __shared__ double vdyn[];
    constexpr int L = 64 * RPL;   // staged rows
    const int cpb = kQT / 64, nblk = (n + cpb - 1) / cpb;
    const int b = blockIdx.x / nblk, blk = blockIdx.x % nblk;
    if (info[b] == 2) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int col = cpb * blk + (tid >> 6);
    Vq += (size_t)b * m * n;
    tau += (size_t)b * n;
    Y += (size_t)b * n * n;
    U += (size_t)b * sU;
    double u[RPL];
#pragma unroll
    for (int r = 0; r < RPL; r++) {
        const int row = lane + 64 * r;
        u[r] = (row < n && col < n) ? Y[(size_t)col * n + row] : 0.0;
    }
    for (int i = tid; i < L; i += kQT) vdyn[((n - 1) & 1) * L + i] = i < m ? Vq[(size_t)(n - 1) * m + i] : 0.0;
    for (int j = n - 1; j >= 0; j--) {
        __syncthreads();
        if (j > 0)   // stage the next reflector
            for (int i = tid; i < L; i += kQT)
                vdyn[((j - 1) & 1) * L + i] = i < m ? Vq[(size_t)(j - 1) * m + i] : 0.0;
        const double t = tau[j];
        if (t == 0.0) continue;
        const double *vb = vdyn + (j & 1) * L;
        double w = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; r++) w = fma(vb[lane + 64 * r], u[r], w);
        w = wave_sum(w) * t;
#pragma unroll
        for (int r = 0; r < RPL; r++) u[r] = fma(-w, vb[lane + 64 * r], u[r]);
    }
    if (col < n)
#pragma unroll
        for (int r = 0; r < RPL; r++) {
            const int row = lane + 64 * r;
            if (row < m) U[(size_t)col * ldu + row] = u[r];
        }
}

// U[:, 16 blk .. 16 blk + 15] = Q [Y; 0] for one block of 16 columns: group g
// owns column 16 blk + g, lane x rows x, x + 16, ... (RPL of them).  The
// reflector of each step is staged in LDS (double buffered, one barrier).
// TO: element type of U.
template <int RPL, class TO>
__device__ __forceinline__ void apply_q_body(int m, int n, int blk, const double *__restrict__ Vq,
                                             const double *__restrict__ tau,
                                             const double *__restrict__ Y, TO *U, int ldu)
{
    __shared__ double vbuf[2][16 * RPL];
    const int tid = threadIdx.x, grp = tid >> 4, gl = tid & 15;
    const int col = 16 * blk + grp;
    double u[RPL];
#pragma unroll
    for (int r = 0; r < RPL; r++) {
        const int row = gl + 16 * r;
        u[r] = (row < n && col < n) ? Y[(size_t)col * n + row] : 0.0;
    }
    for (int i = tid; i < 16 * RPL; i += kQT)
        vbuf[(n - 1) & 1][i] = i < m ? Vq[(size_t)(n - 1) * m + i] : 0.0;
    for (int j = n - 1; j >= 0; j--) {
        __syncthreads();
        if (j > 0)   // stage the next reflector
            for (int i = tid; i < 16 * RPL; i += kQT)
                vbuf[(j - 1) & 1][i] = i < m ? Vq[(size_t)(j - 1) * m + i] : 0.0;
        const double t = tau[j];
        if (t == 0.0) continue;
        const double *vb = vbuf[j & 1];
        double w = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; r++) w = fma(vb[gl + 16 * r], u[r], w);
        w = row_sum16(w) * t;
#pragma unroll
        for (int r = 0; r < RPL; r++) u[r] = fma(-w, vb[gl + 16 * r], u[r]);
    }
    if (col < n)
#pragma unroll
        for (int r = 0; r < RPL; r++) {
            const int row = gl + 16 * r;
            if (row < m) U[(size_t)col * ldu + row] = (TO)u[r];
        }
}

template <int RPL>
__global__ __launch_bounds__(kQT) void apply_q_g(int m, int n, const double *__restrict__ Vq,
                                                 const double *__restrict__ tau,
                                                 const double *__restrict__ Y, double *U, int ldu,
                                                 long long sU, const int *info)
{
    const int nblk = (n + 15) / 16;
    const int b = blockIdx.x / nblk, blk = blockIdx.x % nblk;
    if (info[b] == 2) return;
    apply_q_body<RPL, double>(m, n, blk, Vq + (size_t)b * m * n, tau + (size_t)b * n,
                              Y + (size_t)b * n * n, U + (size_t)b * sU, ldu);
}

// ---- blocked Householder QR for the wide path ------------------------------
// A = Q R panel by panel (LAPACK's xGEQRF with xLARFT / xLARFB): a panel of
// kPB columns is factored in registers (one workgroup per matrix), which also
// forms the compact-WY factor T (Q_panel = I - V T V^T); the trailing columns
// then take C <- C - V T^T (V^T C) as three batched GEMMs on the matrix
// cores, where almost all of the QR's flops are.
constexpr int kPB = 16;

// H = s A with the power of two s that brings max |a| into [1, 2) (no
// square overflows); bad[b] flags a non-finite entry (H = A then).
__global__ __launch_bounds__(kQT) void qrb_init(int m, int n, const double *__restrict__ A,
                                                int lda, long long sA, double *H, double *scale,
                                                int *bad)
{
    __shared__ double s_max[kQT / 64];
    __shared__ int s_bad[kQT / 64];
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    A += (size_t)b * sA;
    H += (size_t)b * m * n;
    double amax = 0.0;
    int nf = 0;
    for (size_t idx = tid; idx < (size_t)m * n; idx += kQT) {
        const double a = A[(idx / m) * lda + idx % m];
        nf |= !isfinite(a);
        amax = fmax(amax, fabs(a));
    }
    amax = wave_max(amax);
    nf = __any(nf);
    if (lane == 0) {
        s_max[wave] = amax;
        s_bad[wave] = nf;
    }
    __syncthreads();
    amax = fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
    const bool finite = !(s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]);
    const double sc = finite ? pow2_scale(amax) : 1.0;
    for (size_t idx = tid; idx < (size_t)m * n; idx += kQT)
        H[idx] = A[(idx / m) * lda + idx % m] * sc;
    if (tid == 0) {
        scale[b] = sc;
        bad[b] = !finite;
    }
}

// Factors the panel H[k0:m, k0:k0+pb] in place: group g owns panel column
// k0 + g, lane x rows k0 + x, k0 + x + 16, ... (RPL of them).  At step j the
// owner of column j forms the reflector (as in the register QR above) and
// publishes it in LDS; the later columns of the panel apply it, and the
// earlier ones form v_i . v_j, the entries of V^T V that T needs:
//   T(j, j) = tau_j,  T(0:j-1, j) = -tau_j T(0:j-1, 0:j-1) (V^T v_j)(0:j-1).
// Writes the panel back (R above, reflectors below the diagonal), tau, V
// explicitly (rows k0 .. m-1 of Vp, unit diagonal, zero above it) and T
// (kPB x kPB, upper triangular).
template <int RPL>
__global__ __launch_bounds__(kQT) void qrb_panel(int m, int n, int k0, int pb, double *H,
                                                 double *tau_out, double *Vp, double *T)
{
    __shared__ double vbuf[2][16 * RPL];
    __shared__ double s_tau[kPB];
    __shared__ double s_z[kPB][kPB + 1];   // s_z[i][j] = v_i . v_j, i < j
    __shared__ double s_t[kPB][kPB + 1];
    const int b = blockIdx.x, tid = threadIdx.x, grp = tid >> 4, gl = tid & 15;
    const bool own = grp < pb;
    H += (size_t)b * m * n;
    double *hc = H + (size_t)(k0 + grp) * m;
    double h[RPL];
#pragma unroll
    for (int r = 0; r < RPL; r++) {
        const int row = k0 + gl + 16 * r;
        h[r] = (own && row < m) ? hc[row] : 0.0;
    }
    for (int j = 0; j < pb; j++) {
        double *vb = vbuf[j & 1];
        if (grp == j) {
            double s = 0.0, a = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; r++) {
                const int lr = gl + 16 * r;   // row k0 + lr
                s = lr > j ? fma(h[r], h[r], s) : s;
                a = lr == j ? h[r] : a;
            }
            s = row_sum16(s);
            const double alpha = row_sum16(a);   // one nonzero term: exact
            double beta = alpha, t = 0.0, scal = 0.0;
            if (s > 0.0) {
                const double nrmj = sqrt(fma(alpha, alpha, s));
                beta = alpha >= 0.0 ? -nrmj : nrmj;
                t = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
#pragma unroll
            for (int r = 0; r < RPL; r++) {
                const int lr = gl + 16 * r;
                const double v = lr == j ? 1.0 : (lr > j ? h[r] * scal : 0.0);
                vb[lr] = v;
                h[r] = lr == j ? beta : (lr > j ? v : h[r]);
            }
            if (gl == 0) s_tau[j] = t;
        }
        __syncthreads();
        if (own && grp != j) {   // uniform in the group
            double w = 0.0;
            if (grp > j) {       // apply H_j to a later panel column
#pragma unroll
                for (int r = 0; r < RPL; r++) w = fma(vb[gl + 16 * r], h[r], w);
                w = row_sum16(w) * s_tau[j];
#pragma unroll
                for (int r = 0; r < RPL; r++) h[r] = fma(-w, vb[gl + 16 * r], h[r]);
            } else {             // v_grp . v_j for T
#pragma unroll
                for (int r = 0; r < RPL; r++) {
                    const int lr = gl + 16 * r;
                    const double vi = lr == grp ? 1.0 : (lr > grp ? h[r] : 0.0);
                    w = fma(vb[lr], vi, w);
                }
                w = row_sum16(w);
                if (gl == 0) s_z[grp][j] = w;
            }
        }
    }
    __syncthreads();
    // T row by row: row i depends only on its own earlier entries
    if (tid < pb) {
        const int i = tid;
        for (int j = 0; j < pb; j++) {
            double v = 0.0;
            if (j == i) {
                v = s_tau[j];
            } else if (j > i) {
                double acc = 0.0;
                for (int k = i; k < j; k++) acc = fma(s_t[i][k], s_z[k][j], acc);
                v = -s_tau[j] * acc;
            }
            s_t[i][j] = v;
        }
    }
    __syncthreads();
    double *Tb = T + (size_t)b * kPB * kPB;
    for (int idx = tid; idx < kPB * kPB; idx += kQT) {
        const int i = idx % kPB, j = idx / kPB;
        Tb[(size_t)j * kPB + i] = (i < pb && j < pb) ? s_t[i][j] : 0.0;
    }
    if (tid < pb) tau_out[(size_t)b * n + k0 + tid] = s_tau[tid];
    double *vc = Vp + (size_t)b * m * kPB + (size_t)grp * m;
#pragma unroll
    for (int r = 0; r < RPL; r++) {
        const int lr = gl + 16 * r, row = k0 + lr;
        if (!own || row >= m) continue;
        hc[row] = h[r];
        vc[row] = lr == grp ? 1.0 : (lr > grp ? h[r] : 0.0);
    }
}

// X = R^T / scale (NaN for a non-finite input), then the reflectors as full
// columns in H (ones on the diagonal, zeros above).
__global__ __launch_bounds__(kQT) void qrb_final(int m, int n, double *H, double *X, double *tau,
                                                 const double *scale, const int *bad)
{
    const int b = blockIdx.x, tid = threadIdx.x;
    H += (size_t)b * m * n;
    X += (size_t)b * n * n;
    const bool nf = bad[b] != 0;
    const double inv = 1.0 / scale[b];
    for (size_t idx = tid; idx < (size_t)n * n; idx += kQT) {
        const int r = (int)(idx % n), c = (int)(idx / n);   // X(r, c) = R(c, r)
        X[idx] = nf ? __builtin_nan("") : (r >= c ? H[(size_t)r * m + c] * inv : 0.0);
    }
    __syncthreads();
    for (size_t idx = tid; idx < (size_t)m * n; idx += kQT) {
        const int row = (int)(idx % m), col = (int)(idx / m);
        if (row <= col) H[idx] = row == col ? 1.0 : 0.0;
    }
    if (nf)
        for (int j = tid; j < n; j += kQT) tau[(size_t)b * n + j] = 0.0;
}

// ---- descriptor-driven variants for the serving runtime -------------------
__global__ __launch_bounds__(kQT) void qr_house_job(const QrJob *jobs, const int *list)
{
    __shared__ double vbuf[2 * kQrMaxM];
    const QrJob J = jobs[list[blockIdx.x]];
    if (J.f32)
        qr_house_body<float>(J.m, J.n, (const float *)J.A, J.lda, J.Vq, J.X, J.tau, vbuf);
    else
        qr_house_body<double>(J.m, J.n, (const double *)J.A, J.lda, J.Vq, J.X, J.tau, vbuf);
}

// one workgroup per (job, block of 16 columns); also converts S and V to
// FP32 for FP32 requests (block 0 of the job)
template <int RPL>
__global__ __launch_bounds__(kQT) void apply_q_job(const QrJob *jobs, const int *list)
{
    constexpr int kMaxBlk = kQrMaxN / 16;
    const QrJob J = jobs[list[blockIdx.x / kMaxBlk]];
    const int blk = blockIdx.x % kMaxBlk;
    if (16 * blk >= J.n || *J.info == 2) return;
    if (J.U) {
        if (J.uf32)
            apply_q_body<RPL, float>(J.m, J.n, blk, J.Vq, J.tau, J.Y, (float *)J.U, J.ldu);
        else
            apply_q_body<RPL, double>(J.m, J.n, blk, J.Vq, J.tau, J.Y, (double *)J.U, J.ldu);
    }
    if (J.uf32) {   // S and V from their FP64 staging
        const int tid = threadIdx.x;
        for (int c = 16 * blk; c < 16 * blk + 16 && c < J.n; c++) {
            if (tid == 0) ((float *)J.Sout)[c] = (float)J.S64[c];
            if (J.Vout)
                for (int r = tid; r < J.n; r += kQT)
                    ((float *)J.Vout)[(size_t)c * J.ldv + r] = (float)J.Vx64[(size_t)c * J.n + r];
        }
    }
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

bool precond_supported(int m, int n)
{
    int N, R, NS, rpl, cpg;
    return n >= 1 && m >= n && (size_t)m * n <= (size_t)kQrMaxElems && n <= 64 &&
           qr_shape(m, n, &rpl, &cpg) && resident_config(n, n, 0, &N, &R, &NS);
}

namespace {
// workspace of the small path: X1 = R1^T, X2 = R2^T, J, U_x (n x n each),
// the reflectors of both QRs (m x n, n x n), tau of both, the permutation
struct PrecondWs {
    double *X1, *X2, *J, *Ux, *Vq1, *Vq2, *tau1, *tau2;
    int *perm, *flag;   // flag: the solve for J was rejected
};

size_t precond_carve(int batch, int m, int n, void *ws, PrecondWs *w)
{
    const size_t nn = al256((size_t)batch * n * n * 8), mn = al256((size_t)batch * m * n * 8);
    const size_t tn = al256((size_t)batch * n * 8), pn = al256((size_t)batch * n * 4);
    if (w) {
        char *p = (char *)ws;
        double **nnp[4] = {&w->X1, &w->X2, &w->J, &w->Ux};
        for (double **q : nnp) {
            *q = (double *)p;
            p += nn;
        }
        w->Vq1 = (double *)p;
        p += mn;
        w->Vq2 = (double *)p;
        p += nn;
        w->tau1 = (double *)p;
        p += tn;
        w->tau2 = (double *)p;
        p += tn;
        w->perm = (int *)p;
        p += pn;
        w->flag = (int *)p;
    }
    return 5 * nn + mn + 2 * tn + 2 * pn;
}

// head of the wide path's workspace: X = R^T, reflectors, tau, J, U_x
size_t big_head_bytes(int batch, int m, int n)
{
    return al256((size_t)batch * n * n * 8) + al256((size_t)batch * m * n * 8) +
           al256((size_t)batch * n * 8) + 2 * al256((size_t)batch * n * n * 8);
}

template <bool PIV>
hipError_t launch_qr_d(int batch, int m, int n, const double *A, int lda, long long sA,
                       double *X, double *Vq, double *tau, int *perm, hipStream_t stream,
                       bool lower = false)
{
    // The pivoted QR with m <= 64 runs one wave per matrix, one column per
    // lane; without pivoting the register QR of 16-lane groups, whose steps
    // need one barrier each, is faster (64 x 64: 0.28 against 0.37 ms per
    // 5000 matrices)
    if (PIV && m <= 64 && n <= m) {
        const int mb = (m + 15) / 16;
#define SVDB_QL(MB)                                                                            \
    if (mb == MB)                                                                              \
        hipLaunchKernelGGL((qr_lane_d<MB, PIV>), dim3(batch), dim3(64), 0, stream, m, n, A, lda, \
                           sA, X, Vq, tau, perm);
        SVDB_QL(1)
        SVDB_QL(2)
        SVDB_QL(3)
        SVDB_QL(4)
#undef SVDB_QL
        return hipGetLastError();
    }
    int rpl, cpg;
    if (!qr_shape(m, n, &rpl, &cpg)) return hipErrorInvalidValue;
#define SVDB_QR(RP, CP)                                                                        \
    if (rpl == RP && cpg == CP)                                                                \
        hipLaunchKernelGGL((qr_house_d<RP, CP, PIV>), dim3(batch), dim3(kQT), 0, stream, m, n, \
                           A, lda, sA, X, Vq, tau, perm, lower ? 1 : 0);
#define SVDB_QR_ROW(RP) SVDB_QR(RP, 1) SVDB_QR(RP, 2) SVDB_QR(RP, 3) SVDB_QR(RP, 4)
    SVDB_QR_ROW(1)
    SVDB_QR_ROW(2)
    SVDB_QR_ROW(4)
    SVDB_QR_ROW(8)
    SVDB_QR_ROW(16)
#undef SVDB_QR_ROW
#undef SVDB_QR
    return hipGetLastError();
}

// U = Q [Y; 0], rows permuted by perm when given (m = n); only: NULL, or a
// per-matrix flag, matrices whose flag is 0 are skipped
hipError_t launch_apply_d(int batch, int m, int n, const double *Vq, const double *tau,
                          const double *Y, double *U, int ldu, long long sU, const int *info,
                          const int *perm, hipStream_t stream, const int *only = nullptr)
{
    int rpl, cpg;
    if (!qr_shape(m, n, &rpl, &cpg)) return hipErrorInvalidValue;
    const size_t lds = (size_t)m * n * sizeof(double);
#define SVDB_AQ(RP, CP)                                                                        \
    if (rpl == RP && cpg == CP)                                                                \
        hipLaunchKernelGGL((apply_q_d<RP, CP>), dim3(batch), dim3(kQT), lds, stream, m, n, Vq, \
                           tau, Y, U, ldu, sU, info, perm, only);
#define SVDB_AQ_ROW(RP) SVDB_AQ(RP, 1) SVDB_AQ(RP, 2) SVDB_AQ(RP, 3) SVDB_AQ(RP, 4)
    SVDB_AQ_ROW(1)
    SVDB_AQ_ROW(2)
    SVDB_AQ_ROW(4)
    SVDB_AQ_ROW(8)
    SVDB_AQ_ROW(16)
#undef SVDB_AQ_ROW
#undef SVDB_AQ
    return hipGetLastError();
}
}  // namespace

size_t precond_workspace_bytes(int batch, int m, int n)
{
    return precond_carve(batch, m, n, nullptr, nullptr);
}

hipError_t launch_precond_d(int batch, int m, int n, int ns, const double *A, int lda,
                            long long sA, double *S, long long sS, double *U, int ldu,
                            long long sU, double *V, int ldv, long long sV, double tol,
                            int max_sweeps, int *info, int *sweeps, void *ws, hipStream_t stream,
                            bool pivot)
{
    if (!precond_supported(m, n)) return hipErrorInvalidValue;
    PrecondWs w;
    precond_carve(batch, m, n, ws, &w);
    const long long snn = (long long)n * n;
    // A P = Q1 R1 (reflectors only when U is wanted, P only when V is).  The
    // QR pivots where V comes from the back substitution with R1, whose
    // accuracy needs the row grading that pivoting gives R1, and when asked
    // to; elsewhere P = I, as in the paper's QR step
    const bool nv = resident_nv_supported(n, n);
    pivot = pivot || nv;
    int *perm = pivot && V ? w.perm : nullptr;
    hipError_t e = pivot ? launch_qr_d<true>(batch, m, n, A, lda, sA, w.X1, U ? w.Vq1 : nullptr,
                                             w.tau1, perm, stream)
                         : launch_qr_d<false>(batch, m, n, A, lda, sA, w.X1, U ? w.Vq1 : nullptr,
                                              w.tau1, nullptr, stream);
    if (e != hipSuccess) return e;
    // R1^T = Q2 R2 (reflectors only when V is wanted)
    e = launch_qr_d<false>(batch, n, n, w.X1, n, snn, w.X2, V ? w.Vq2 : nullptr, w.tau2, nullptr,
                           stream, true);
    if (e != hipSuccess) return e;
    // Jacobi on X = R2^T: its left vectors U_x feed U, its rotations J feed V.
    // For 32 < n <= 64 it iterates on W alone and V = P R1^-1 U_x diag(S)
    // comes from a back substitution; matrices whose V fails the
    // orthogonality check run the Jacobi again with J accumulated, and only
    // they get V = P Q2 J.
    if (nv) {
        e = launch_resident_d(batch, n, n, ns, w.X2, n, snn, S, sS, w.Ux, n, snn, nullptr, n, snn,
                              tol, max_sweeps, info, sweeps, stream, true, nullptr, true);
        if (e == hipSuccess && V) {
            hipLaunchKernelGGL(solve_r1_d<64>, dim3(batch), dim3(64), 0, stream, n,
                               (const double *)w.X1, (const double *)w.Ux, (const double *)S, sS,
                               (const int *)perm, V, ldv, sV, w.flag, (const int *)info,
                               0x1p-49 * n);
            e = hipGetLastError();
            if (e == hipSuccess)
                e = launch_resident_d(batch, n, n, ns, w.X2, n, snn, S, sS, w.Ux, n, snn, w.J, n,
                                      snn, tol, max_sweeps, info, sweeps, stream, false, w.flag,
                                      true);
        }
    } else {
        e = launch_resident_d(batch, n, n, ns, w.X2, n, snn, S, sS, U ? w.Ux : nullptr, n, snn,
                              V ? w.J : nullptr, n, snn, tol, max_sweeps, info, sweeps, stream,
                              false, nullptr, true);
    }
    if (e != hipSuccess) return e;
    if (U) {
        e = launch_apply_d(batch, m, n, w.Vq1, w.tau1, w.Ux, U, ldu, sU, info, nullptr, stream);
        if (e != hipSuccess) return e;
    }
    if (V)
        e = launch_apply_d(batch, n, n, w.Vq2, w.tau2, w.J, V, ldv, sV, info, perm, stream,
                           nv ? w.flag : nullptr);
    return e;
}

void launch_qr_jobs(const QrJob *jobs, const int *list, int count, hipStream_t stream)
{
    if (count > 0)
        hipLaunchKernelGGL(qr_house_job, dim3((unsigned)count), dim3(kQT), 0, stream, jobs, list);
}

void launch_apply_q_jobs(const QrJob *jobs, const int *list, int count, int max_m,
                         hipStream_t stream)
{
    if (count <= 0) return;
    const dim3 grid((unsigned)(count * (kQrMaxN / 16)));
    const int rpl = (max_m + 15) / 16;
    if (rpl <= 8)
        hipLaunchKernelGGL(apply_q_job<8>, grid, dim3(kQT), 0, stream, jobs, list);
    else if (rpl <= 16)
        hipLaunchKernelGGL(apply_q_job<16>, grid, dim3(kQT), 0, stream, jobs, list);
    else if (rpl <= 32)
        hipLaunchKernelGGL(apply_q_job<32>, grid, dim3(kQT), 0, stream, jobs, list);
    else
        hipLaunchKernelGGL(apply_q_job<64>, grid, dim3(kQT), 0, stream, jobs, list);
}

namespace {
// scratch of the blocked QR: V of the panel (m x kPB), T, W and T^T W (kPB x
// n), the scale and the non-finite flag of each matrix
struct QrbWs {
    double *Vp, *T, *W, *W2, *scale;
    int *bad;
};

size_t qrb_carve(int batch, int m, int n, void *ws, QrbWs *w)
{
    const size_t vp = al256((size_t)batch * m * kPB * 8), t = al256((size_t)batch * kPB * kPB * 8);
    const size_t wn = al256((size_t)batch * kPB * n * 8), sc = al256((size_t)batch * 8);
    const size_t bd = al256((size_t)batch * 4);
    if (w) {
        char *p = (char *)ws;
        w->Vp = (double *)p;
        p += vp;
        w->T = (double *)p;
        p += t;
        w->W = (double *)p;
        p += wn;
        w->W2 = (double *)p;
        p += wn;
        w->scale = (double *)p;
        p += sc;
        w->bad = (int *)p;
    }
    return vp + t + 2 * wn + sc + bd;
}

// A (m x n, m <= kQrMaxM) = Q R, blocked: H (m x n, ld m) gets the
// reflectors as full columns, X = R^T (unscaled), tau.
hipError_t launch_qr_blocked(int batch, int m, int n, const double *A, int lda, long long sA,
                             double *H, double *X, double *tau, void *scratch, hipStream_t stream)
{
    QrbWs w;
    qrb_carve(batch, m, n, scratch, &w);
    hipLaunchKernelGGL(qrb_init, dim3(batch), dim3(kQT), 0, stream, m, n, A, lda, sA, H, w.scale,
                       w.bad);
    hipError_t e = hipGetLastError();
    const long long smn = (long long)m * n, svp = (long long)m * kPB, swn = (long long)kPB * n;
    for (int k0 = 0; k0 < n && e == hipSuccess; k0 += kPB) {
        const int pb = n - k0 < kPB ? n - k0 : kPB, rows = m - k0;
        const int r = (rows + 15) / 16;
        bool launched = false;
#define SVDB_QRB(RP)                                                                           \
    if (!launched && r <= RP) {                                                                \
        hipLaunchKernelGGL((qrb_panel<RP>), dim3(batch), dim3(kQT), 0, stream, m, n, k0, pb, H, \
                           tau, w.Vp, w.T);                                                    \
        launched = true;                                                                       \
    }
        SVDB_QRB(1)
        SVDB_QRB(2)
        SVDB_QRB(4)
        SVDB_QRB(8)
        SVDB_QRB(16)
        SVDB_QRB(32)
        SVDB_QRB(64)
#undef SVDB_QRB
        if (!launched) return hipErrorInvalidValue;
        e = hipGetLastError();
        const int nt = n - k0 - pb;
        if (e != hipSuccess || nt <= 0) continue;
        double *C = H + (size_t)(k0 + pb) * m + k0;
        const double *V = w.Vp + k0;
        // W = V^T C, W2 = T^T W, C <- C - V W2
        e = launch_gemm_f64(true, batch, pb, nt, rows, 1.0, V, m, svp, C, m, smn, 0.0, nullptr, 0,
                            0, w.W, kPB, swn, stream);
        if (e == hipSuccess)
            e = launch_gemm_f64(true, batch, pb, nt, pb, 1.0, w.T, kPB, (long long)kPB * kPB, w.W,
                                kPB, swn, 0.0, nullptr, 0, 0, w.W2, kPB, swn, stream);
        if (e == hipSuccess)
            e = launch_gemm_f64(false, batch, rows, nt, pb, -1.0, V, m, svp, w.W2, kPB, swn, 1.0, C,
                                m, smn, C, m, smn, stream);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qrb_final, dim3(batch), dim3(kQT), 0, stream, m, n, H, X, tau,
                       (const double *)w.scale, (const int *)w.bad);
    return hipGetLastError();
}
}  // namespace

// The blocked Householder QR of a strided batch, for the serving runtime's
// requests with more than 64 columns (one workgroup per matrix would run the
// whole factorisation serially): H (m x n per matrix, ld m, m n apart) gets
// the reflectors as full columns, X = R^T (n x n apart), tau (n apart).  A
// may equal H (lda = m, sA = m n).
size_t qr_blocked_scratch_bytes(int batch, int m, int n)
{
    return qrb_carve(batch, m, n, nullptr, nullptr);
}

hipError_t launch_qr_blocked_batch(int batch, int m, int n, const double *A, int lda,
                                   long long sA, double *H, double *X, double *tau,
                                   void *scratch, hipStream_t stream)
{
    if (batch < 1 || m < n || n < 1 || m > kQrMaxM || n > kQrMaxN || lda < m)
        return hipErrorInvalidValue;
    return launch_qr_blocked(batch, m, n, A, lda, sA, H, X, tau, scratch, stream);
}

bool precond_big_supported(int m, int n)
{
    return n > 64 && m >= n && m <= kQrMaxM;
}

// second QR of the wide path: X2 = R2^T, its reflectors (n x n) and tau
size_t big_second_bytes(int batch, int n)
{
    return 2 * al256((size_t)batch * n * n * 8) + al256((size_t)batch * n * 8);
}

size_t precond_big_workspace_bytes(int batch, int m, int n, int nb, bool mixed)
{
    return big_head_bytes(batch, m, n) + big_second_bytes(batch, n) +
           qrb_carve(batch, m, n, nullptr, nullptr) +
           blocked_workspace_bytes(batch, n, n, nb, 8, mixed);
}

namespace {
// U = Q [Y; 0] on the global-memory path (m <= 1024), one block of 16
// columns of U per workgroup
hipError_t launch_apply_g(int batch, int m, int n, const double *Vq, const double *tau,
                          const double *Y, double *U, int ldu, long long sU, const int *info,
                          hipStream_t stream)
{
    const int rpl = (m + 15) / 16;
    const dim3 grid((unsigned)(batch * ((n + 15) / 16)));
#define SVDB_AQG(RP)                                                                           \
    if (rpl <= RP) {                                                                           \
        hipLaunchKernelGGL((apply_q_g<RP>), grid, dim3(kQT), 0, stream, m, n, Vq, tau, Y, U,    \
                           ldu, sU, info);                                                     \
        return hipGetLastError();                                                              \
    }
    SVDB_AQG(8)
    SVDB_AQG(16)
    SVDB_AQG(32)
    SVDB_AQG(64)
#undef SVDB_AQG
    return hipErrorInvalidValue;
}
}  // namespace

// Wide FP64 matrices (n > 64, m <= 1024): A = Q1 R1 and R1^T = Q2 R2 by the
// blocked QR, the block Jacobi on X = R2^T (X J = U_x diag(S)), U = Q1 [U_x;
// 0] and V = Q2 J by column blocks.
hipError_t launch_precond_big_d(int batch, int m, int n, int nb, const double *A, int lda,
                                long long sA, double *S, long long sS, double *U, int ldu,
                                long long sU, double *V, int ldv, long long sV, double tol,
                                int max_sweeps, int masking, int *info, int *sweeps, void *ws,
                                hipStream_t stream, int inner, int persistent, double tol_start,
                                double tol_rate, double tol32)
{
    if (!precond_big_supported(m, n)) return hipErrorInvalidValue;
    const long long snn = (long long)n * n;
    char *p = (char *)ws;
    double *X1 = (double *)p;
    p += al256((size_t)batch * n * n * 8);
    double *Vq1 = (double *)p;
    p += al256((size_t)batch * m * n * 8);
    double *tau1 = (double *)p;
    p += al256((size_t)batch * n * 8);
    double *J = (double *)p;
    p += al256((size_t)batch * n * n * 8);
    double *Ux = (double *)p;
    p += al256((size_t)batch * n * n * 8);
    double *X2 = (double *)p;
    p += al256((size_t)batch * n * n * 8);
    double *Vq2 = (double *)p;
    p += al256((size_t)batch * n * n * 8);
    double *tau2 = (double *)p;
    p += al256((size_t)batch * n * 8);
    void *qws = p;
    p += qrb_carve(batch, m, n, nullptr, nullptr);
    void *bws = p;
    hipError_t e = launch_qr_blocked(batch, m, n, A, lda, sA, Vq1, X1, tau1, qws, stream);
    if (e == hipSuccess)
        e = launch_qr_blocked(batch, n, n, X1, n, snn, Vq2, X2, tau2, qws, stream);
    if (e != hipSuccess) return e;
    // the block Jacobi on X = R2^T, all-FP64 or FP32 sweeps + FP64 refinement
    if (tol32 > 0.0)
        e = launch_blocked_mixed_d(batch, n, n, nb, X2, n, snn, S, sS, U ? Ux : nullptr, n, snn,
                                   V ? J : nullptr, n, snn, tol, tol32, max_sweeps, masking,
                                   info, sweeps, bws, stream, inner, persistent, tol_start,
                                   tol_rate);
    else
        e = launch_blocked_d(batch, n, n, nb, X2, n, snn, S, sS, U ? Ux : nullptr, n, snn,
                             V ? J : nullptr, n, snn, tol, max_sweeps, masking, info, sweeps,
                             bws, stream, inner, persistent, tol_start, tol_rate);
    if (e == hipSuccess && U)
        e = launch_apply_g(batch, m, n, Vq1, tau1, Ux, U, ldu, sU, info, stream);
    if (e == hipSuccess && V)
        e = launch_apply_g(batch, n, n, Vq2, tau2, J, V, ldv, sV, info, stream);
    return e;
}

bool precond_tall_supported(int m, int n)
{
    int N, R, NS;
    return n >= 1 && n <= 64 && m >= n && m <= kTallMaxM && !precond_supported(m, n) &&
           resident_config(n, n, 0, &N, &R, &NS);
}

// AUTO takes the tall path up to m = 1024, where its QR is the blocked one
// (a register panel of at most 64 rows per lane): measured on 1000 uniform
// [0, 1] matrices with n = 16 it beats the block method without QR from
// m = 300 (0.36 against 1.18 ms) to m = 1000 (0.67 against 1.55 ms).  Beyond
// 1024 rows only the one-workgroup QR in global memory is left, and it loses
// (m = 2000: 3.14 against 2.28 ms) to the block method, whose converged
// inner solves need about three sweeps there.
bool precond_tall_auto(int m, int n)
{
    return precond_tall_supported(m, n) && m <= kQrMaxM;
}

size_t precond_tall_workspace_bytes(int batch, int m, int n)
{
    return big_head_bytes(batch, m, n) + (m <= kQrMaxM ? qrb_carve(batch, m, n, nullptr, nullptr) : 0);
}

// Tall matrices with few columns (n <= 64, m <= 4096, beyond the register
// QR: m > 256 or m n > 8192): the blocked QR (m <= 1024) or the QR in global
// memory, the resident Jacobi on X = R^T (n x n), U = Q J by one wave
// per column.
hipError_t launch_precond_tall_d(int batch, int m, int n, const double *A, int lda, long long sA,
                                 double *S, long long sS, double *U, int ldu, long long sU,
                                 double *V, int ldv, long long sV, double tol, int max_sweeps,
                                 int *info, int *sweeps, void *ws, hipStream_t stream)
{
    if (!precond_tall_supported(m, n)) return hipErrorInvalidValue;
    char *p = (char *)ws;
    double *X = (double *)p;
    p += al256((size_t)batch * n * n * 8);
    double *Vq = (double *)p;
    p += al256((size_t)batch * m * n * 8);
    double *tau = (double *)p;
    p += al256((size_t)batch * n * 8);
    double *J = (double *)p;
    p += al256((size_t)batch * n * n * 8);
    double *Ux = (double *)p;
    p += al256((size_t)batch * n * n * 8);
    // up to m = 1024 the blocked QR (a register panel, plus GEMMs for n >
    // 16); beyond, the one-workgroup QR in global memory
    hipError_t e;
    if (m <= kQrMaxM) {
        e = launch_qr_blocked(batch, m, n, A, lda, sA, Vq, X, tau, p, stream);
    } else {
        hipLaunchKernelGGL(qr_house_g, dim3(batch), dim3(kQT), (size_t)16 * m, stream, m, n, A,
                           lda, sA, Vq, X, tau);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    // the Jacobi on X = R^T: its left vectors are V, its rotations J feed U
    double *vx = V ? V : Ux;
    const int ldvx = V ? ldv : n;
    const long long svx = V ? sV : (long long)n * n;
    e = launch_resident_d(batch, n, n, 0, X, n, (long long)n * n, S, sS, vx, ldvx, svx,
                          U ? J : nullptr, n, (long long)n * n, tol, max_sweeps, info, sweeps,
                          stream);
    if (e != hipSuccess || !U) return e;
    const int rpl = (m + 63) / 64;
    const dim3 grid((unsigned)(batch * ((n + 3) / 4)));
#define SVDB_AQT(RP)                                                                           \
    if (rpl <= RP) {                                                                           \
        hipLaunchKernelGGL((apply_q_tall<RP>), grid, dim3(kQT), (size_t)2 * 64 * RP * 8, stream, \
                           m, n, (const double *)Vq, (const double *)tau, (const double *)J, U, \
                           ldu, sU, (const int *)info);                                        \
        return hipGetLastError();                                                              \
    }
    SVDB_AQT(8)
    SVDB_AQT(16)
    SVDB_AQT(32)
    SVDB_AQT(64)
#undef SVDB_AQT
    return hipErrorInvalidValue;
}

}  // namespace svdb
