// resident.hip -- register-resident unblocked one-sided Jacobi SVD (Alg. 2),
// FP64, for n <= 64 columns.
//
// Layout.  The matrix is held as the stacked (m + N) x N matrix [W; V] (W
// starts as A, V as I; every rotation acts on whole stacked columns), with one
// stacked row per lane and slot: lane L of wave w, slot t holds stacked row
// 64 (R w + t) + L.  All rows of W live in wave 0, so only wave 0 forms Gram
// entries.  N is n rounded up to 16, 32 or 64 (extra columns are zero and
// never rotate).
//
// Ordering.  The round-robin ordering of Sec. 2 / 4.1 is realised as a
// tournament table of K = N/2 seats per row: seat q of the top row (array T)
// plays seat q of the bottom row (array B).  After an iteration every column
// except the one in top seat 0 moves one ring position, which here is only a
// choice of destination registers for the rotated columns -- no data moves
// between lanes.  After N-1 iterations (one sweep) the table is back in its
// initial state, so sweeps always start from columns (2q, 2q+1) in seat q.
//
// Per iteration (wave 0): g_ij of the K pairs (Alg. 2, Gram entries) as one
// FMA per row, a cross-lane reduction (permlane32/16 swaps, then an LDS
// transpose inside rows of 16 lanes), the rotate-or-skip test and c, s of
// eq. (sin-cos) computed by lanes in parallel, published through LDS; then
// every wave rotates its rows of W and V.  The squared column norms g_ii are
// tracked through the exact identity g_ii' = g_ii + t |g_ij|,
// g_jj' = g_jj - t |g_ij| of a Jacobi rotation, and recomputed from the columns
// at the start of every sweep, so the sweep that finds no pair to rotate --
// the convergence test -- always uses exact norms.
#include "device_common.hpp"
#include "launchers.hpp"

namespace svdb {

namespace {

// ---- cross-lane helpers (gfx950) ------------------------------------------

__device__ __forceinline__ void swap32(double &a, double &b)
{
    // lanes 32..63 of a <-> lanes 0..31 of b
    auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    a = __hiloint2double(hi[0], lo[0]);
    b = __hiloint2double(hi[1], lo[1]);
}

__device__ __forceinline__ void swap16(double &a, double &b)
{
    // odd rows (16 lanes) of a <-> even rows of b
    auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    a = __hiloint2double(hi[0], lo[0]);
    b = __hiloint2double(hi[1], lo[1]);
}

template <int ROR>
__device__ __forceinline__ double row_ror(double v)
{
    // value of lane (x + ROR) mod 16 of the same row of 16 lanes
    constexpr int ctrl = 0x120 + ROR;
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

struct OpSum {
    __device__ static double apply(double a, double b) { return a + b; }
};
struct OpMax {
    __device__ static double apply(double a, double b) { return fmax(a, b); }
};

// Reduces K per-lane values over the 64 lanes of a wave.  On return lane
// L = 16 rho + x holds the reduction of value q = (x mod K/4) + (K/4) rho.
// buf: 64 * K/4 doubles of LDS private to the calling wave.
template <int K, class Op>
__device__ __forceinline__ double reduce_pairs(double (&g)[K], double *buf)
{
    constexpr int H = K / 2, Q = K / 4;
    const int lane = threadIdx.x & 63, rho = lane >> 4, x = lane & 15;
    double h[H];
#pragma unroll
    for (int v = 0; v < H; v++) {
        double a = g[v], b = g[v + H];
        swap32(a, b);
        h[v] = Op::apply(a, b);
    }
    double f[Q];
#pragma unroll
    for (int v = 0; v < Q; v++) {
        double a = h[v], b = h[v + Q];
        swap16(a, b);
        f[v] = Op::apply(a, b);
    }
    // lane (rho, x) now holds, for v < Q, value v + Q rho reduced over the
    // four lanes {x, x+16, x+32, x+48}; finish inside the row of 16 lanes.
#pragma unroll
    for (int v = 0; v < Q; v++) buf[(rho * Q + v) * 16 + x] = f[v];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int v = x % Q, h0 = (x / Q) * Q;
    const double *src = buf + (rho * Q + v) * 16 + h0;
    double s = src[0];
#pragma unroll
    for (int k = 1; k < Q; k++) s = Op::apply(s, src[k]);
    // Rotations by 8, 4, 2, 1 lanes in this order: after each step the values
    // repeat with half the period, so every step adds the same two operands in
    // both lanes of a pair and all lanes of one value end with identical bits
    // (the rotate-or-skip decision below must agree across those lanes).
    s = Op::apply(s, row_ror<8>(s));
    if constexpr (Q < 8) s = Op::apply(s, row_ror<4>(s));
    if constexpr (Q < 4) s = Op::apply(s, row_ror<2>(s));
    if constexpr (Q < 2) s = Op::apply(s, row_ror<1>(s));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return s;
}

// Column ids in the top and bottom seat q at iteration `it` (see rr_pair).
__device__ __forceinline__ void rr_seats(int l, int it, int q, int &ct, int &cb)
{
    const int k = l >> 1, ring = l - 1;
    if (q == 0) {
        ct = 0;
    } else {
        int y = (q - 1) - it;
        y += (y < 0) ? ring : 0;
        ct = rr_initial(y, k);
    }
    int y = (2 * k - 2 - q) - it;
    y += (y < 0) ? ring : 0;
    cb = rr_initial(y, k);
}

template <int N, int R, int NW>
__global__ __launch_bounds__(64 * NW) void resident_jacobi_d(
    int m, int n, const double *__restrict__ A, int lda, long long sA, double *S, long long sS,
    double *U, int ldu, long long sU, double *V, int ldv, long long sV, double tol,
    int max_sweeps, int *info, int *sweeps_out)
{
    constexpr int K = N / 2;
    constexpr int Q = K / 4;
    static_assert(K >= 8 && (K & (K - 1)) == 0, "N must be 16, 32 or 64");

    __shared__ double s_nrm[N];           // squared column norms, by column id
    __shared__ double2 s_cs[2][K];        // (c, signed e s) per pair, double buffered
    __shared__ double s_buf[64 * Q];      // reduction transpose (wave 0)
    __shared__ double s_sig[N];
    __shared__ int s_rank[N];
    __shared__ double s_scale;
    __shared__ int s_bad, s_flag;

    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    A += (size_t)b * sA;

    // stacked row of slot t, and its class
    int srow[R];
#pragma unroll
    for (int t = 0; t < R; t++) srow[t] = 64 * (R * wave + t) + lane;

    double T[K][R], B[K][R];
    // ---- load W = A (zero padded) and V = I ----------------------------------
    double amax = 0.0;
    int bad = 0;
#pragma unroll
    for (int t = 0; t < R; t++) {
        const int s = srow[t];
#pragma unroll
        for (int q = 0; q < K; q++) {
            double xt = 0.0, xb = 0.0;
            const int ct = 2 * q, cb = 2 * q + 1;
            if (s < m) {
                if (ct < n) xt = A[(size_t)ct * lda + s];
                if (cb < n) xb = A[(size_t)cb * lda + s];
            } else if (s < m + N) {
                xt = (s - m == ct) ? 1.0 : 0.0;
                xb = (s - m == cb) ? 1.0 : 0.0;
            }
            if (s < m) {
                bad |= !isfinite(xt) | !isfinite(xb);
                amax = fmax(amax, fmax(fabs(xt), fabs(xb)));
            }
            T[q][t] = xt;
            B[q][t] = xb;
        }
    }
    if (threadIdx.x == 0) {
        s_bad = 0;
        s_flag = 0;
    }
    __syncthreads();
    bad = __any(bad);
    amax = wave_max(amax);
    if (wave == 0 && lane == 0) {
        s_scale = pow2_scale(amax);
        if (bad) s_bad = 1;
    }
    __syncthreads();
    if (s_bad) {
        if (threadIdx.x == 0) {
            info[b] = 2;
            if (sweeps_out) sweeps_out[b] = 0;
        }
        return;
    }
    const double scale = s_scale;
    if (wave == 0 && scale != 1.0) {
#pragma unroll
        for (int t = 0; t < R; t++)
            if (srow[t] < m) {
#pragma unroll
                for (int q = 0; q < K; q++) {
                    T[q][t] *= scale;
                    B[q][t] *= scale;
                }
            }
    }

    // slot classes for the Gram entries (wave-uniform): 2 all rows of W,
    // 1 some rows of W, 0 none
    int wcls[R];
#pragma unroll
    for (int t = 0; t < R; t++) {
        const int base = 64 * (R * wave + t);
        wcls[t] = (base + 63 < m) ? 2 : (base < m ? 1 : 0);
    }

    const int l = N;
    int sweeps = 0, converged = 0;
    int par = 0;
    while (!converged && sweeps < max_sweeps) {
        sweeps++;
        // exact squared norms at the start of the sweep (seat q holds 2q, 2q+1)
        if (wave == 0) {
            double pt[K], pb[K];
#pragma unroll
            for (int q = 0; q < K; q++) {
                pt[q] = 0.0;
                pb[q] = 0.0;
            }
#pragma unroll
            for (int t = 0; t < R; t++) {
                if (wcls[t] == 0) continue;
                const double msk = (srow[t] < m) ? 1.0 : 0.0;
#pragma unroll
                for (int q = 0; q < K; q++) {
                    const double xt = T[q][t] * msk, xb = B[q][t] * msk;
                    pt[q] = fma(xt, xt, pt[q]);
                    pb[q] = fma(xb, xb, pb[q]);
                }
            }
            const double nt = reduce_pairs<K, OpSum>(pt, s_buf);
            const double nb = reduce_pairs<K, OpSum>(pb, s_buf);
            const int x = lane & 15, q = (x % Q) + Q * (lane >> 4);
            if (x < Q) {
                s_nrm[2 * q] = nt;
                s_nrm[2 * q + 1] = nb;
            }
        }
        for (int it = 0; it < l - 1; it++) {
            if (wave == 0) {
                double g[K];
#pragma unroll
                for (int q = 0; q < K; q++) g[q] = 0.0;
#pragma unroll
                for (int t = 0; t < R; t++) {
                    if (wcls[t] == 2) {
#pragma unroll
                        for (int q = 0; q < K; q++) g[q] = fma(T[q][t], B[q][t], g[q]);
                    } else if (wcls[t] == 1) {
                        const double msk = (srow[t] < m) ? 1.0 : 0.0;
#pragma unroll
                        for (int q = 0; q < K; q++) g[q] = fma(T[q][t] * msk, B[q][t], g[q]);
                    }
                }
                const double gq = reduce_pairs<K, OpSum>(g, s_buf);
                const int x = lane & 15, q = (x % Q) + Q * (lane >> 4);
                int ct, cb;
                rr_seats(l, it, q, ct, cb);
                const double at = s_nrm[ct], ab = s_nrm[cb];
                // orientation of the paper: pair (i, j) with i < j
                const bool top_is_i = ct < cb;
                const double gi = top_is_i ? at : ab, gj = top_is_i ? ab : at;
                const double ag = fabs(gq);
                double c = 1.0, es = 0.0;
                const bool rot = (gq != 0.0) && (ag >= tol * sqrt(gi) * sqrt(gj));
                if (rot) {
                    double s;
                    const double tau = (gi - gj) / (2.0 * ag);
                    const double atau = fabs(tau);
                    double tt = (atau > 0x1p500) ? 0.5 / atau : 1.0 / (atau + sqrt(1.0 + atau * atau));
                    tt = (tau >= 0.0) ? tt : -tt;
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                    es = gq > 0.0 ? s : -s;
                    const double ni = fma(tt, ag, gi), nj = fma(-tt, ag, gj);
                    if (x < Q) {
                        s_nrm[top_is_i ? ct : cb] = ni;
                        s_nrm[top_is_i ? cb : ct] = nj;
                    }
                }
                // the top seat's column is a_i when top_is_i; otherwise the
                // roles swap and the sign of e s flips
                if (x < Q) s_cs[par][q] = make_double2(c, top_is_i ? es : -es);
                if (__any(rot && x < Q) && lane == 0) s_flag = 1;
            }
            __syncthreads();
            // ---- rotate every row slot; the destinations realise the seat moves
            double nT[K][R], nB[K][R];
#pragma unroll
            for (int q = K - 1; q >= 0; q--) {
                const double2 cs = s_cs[par][q];
#pragma unroll
                for (int t = 0; t < R; t++) {
                    const double a = T[q][t], bb = B[q][t];
                    const double na = fma(cs.x, a, cs.y * bb);
                    const double nb = fma(cs.x, bb, -cs.y * a);
                    if (q == 0) nT[0][t] = na;
                    else if (q < K - 1) nT[q + 1][t] = na;
                    else nB[K - 1][t] = na;
                    if (q == 0) nT[1][t] = nb;
                    else nB[q - 1][t] = nb;
                }
            }
#pragma unroll
            for (int q = 0; q < K; q++)
#pragma unroll
                for (int t = 0; t < R; t++) {
                    T[q][t] = nT[q][t];
                    B[q][t] = nB[q][t];
                }
            par ^= 1;
        }
        __syncthreads();
        converged = (s_flag == 0);
        __syncthreads();
        if (threadIdx.x == 0) s_flag = 0;
    }

    // ---- finalise: sigma = ||w_c|| (two-pass scaled), stable descending sort
    if (wave == 0) {
        double mt[K], mb[K];
#pragma unroll
        for (int q = 0; q < K; q++) {
            mt[q] = 0.0;
            mb[q] = 0.0;
        }
#pragma unroll
        for (int t = 0; t < R; t++) {
            if (wcls[t] == 0) continue;
            const double msk = (srow[t] < m) ? 1.0 : 0.0;
#pragma unroll
            for (int q = 0; q < K; q++) {
                mt[q] = fmax(mt[q], fabs(T[q][t]) * msk);
                mb[q] = fmax(mb[q], fabs(B[q][t]) * msk);
            }
        }
        const double xt = reduce_pairs<K, OpMax>(mt, s_buf);
        const double xb = reduce_pairs<K, OpMax>(mb, s_buf);
        const int x = lane & 15, q = (x % Q) + Q * (lane >> 4);
        if (x < Q) {
            s_sig[2 * q] = xt;          // column maxima, temporarily
            s_sig[2 * q + 1] = xb;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double pt[K], pb[K];
#pragma unroll
        for (int q2 = 0; q2 < K; q2++) {
            const double it_ = s_sig[2 * q2] > 0.0 ? 1.0 / s_sig[2 * q2] : 0.0;
            const double ib_ = s_sig[2 * q2 + 1] > 0.0 ? 1.0 / s_sig[2 * q2 + 1] : 0.0;
            pt[q2] = 0.0;
            pb[q2] = 0.0;
#pragma unroll
            for (int t = 0; t < R; t++) {
                if (wcls[t] == 0) continue;
                const double msk = (srow[t] < m) ? 1.0 : 0.0;
                const double yt = T[q2][t] * it_ * msk, yb = B[q2][t] * ib_ * msk;
                pt[q2] = fma(yt, yt, pt[q2]);
                pb[q2] = fma(yb, yb, pb[q2]);
            }
        }
        const double st = reduce_pairs<K, OpSum>(pt, s_buf);
        const double sb = reduce_pairs<K, OpSum>(pb, s_buf);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (x < Q) {
            const double mxt = s_sig[2 * q], mxb = s_sig[2 * q + 1];
            s_sig[2 * q] = mxt > 0.0 ? mxt * sqrt(st) : 0.0;
            s_sig[2 * q + 1] = mxb > 0.0 ? mxb * sqrt(sb) : 0.0;
        }
    }
    __syncthreads();
    if (threadIdx.x < N) {
        const int c = threadIdx.x;
        const double sc = s_sig[c];
        int rk = 0;
        for (int j = 0; j < N; j++) {
            const double sj = s_sig[j];
            rk += (sj > sc) || (sj == sc && j < c);
        }
        s_rank[c] = rk;
    }
    __syncthreads();
    S += (size_t)b * sS;
    if (threadIdx.x < n) S[s_rank[threadIdx.x]] = s_sig[threadIdx.x] / scale;
    if (U) U += (size_t)b * sU;
    if (V) V += (size_t)b * sV;
    bool any_zero = false;
#pragma unroll
    for (int q = 0; q < K; q++) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int c = 2 * q + h;
            if (c >= n) continue;
            const int rk = s_rank[c];
            const double sc = s_sig[c];
            const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
            any_zero |= !(sc > 0.0);
#pragma unroll
            for (int t = 0; t < R; t++) {
                const int s = srow[t];
                const double val = h ? B[q][t] : T[q][t];
                if (s < m) {
                    if (U) U[(size_t)rk * ldu + s] = val * inv;
                } else if (s < m + n) {
                    if (V) V[(size_t)rk * ldv + (s - m)] = val;
                }
            }
        }
    }
    // sigma = 0: complete U by Gram-Schmidt on e_1, e_2, ... (rare; wave 0,
    // on the freshly written columns of U in global memory)
    if (U && wave == 0 && any_zero) {
        __threadfence();
        int cand = 0;
        for (int i = 0; i < n; i++) {
            if (s_sig[i] > 0.0) continue;
            double *u = U + (size_t)s_rank[i] * ldu;
            for (; cand < m; cand++) {
                for (int r = lane; r < m; r += 64) u[r] = (r == cand) ? 1.0 : 0.0;
                __threadfence();
                for (int pass = 0; pass < 2; pass++)
                    for (int j = 0; j < n; j++) {
                        if (j == i || (s_sig[j] == 0.0 && j > i)) continue;
                        const double *qv = U + (size_t)s_rank[j] * ldu;
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
    if (threadIdx.x == 0) {
        info[b] = converged ? 0 : 1;
        if (sweeps_out) sweeps_out[b] = sweeps;
    }
}

template <int N, int R, int NW>
hipError_t launch_one(int batch, int m, int n, const double *A, int lda, long long sA, double *S,
                      long long sS, double *U, int ldu, long long sU, double *V, int ldv,
                      long long sV, double tol, int max_sweeps, int *info, int *sweeps,
                      hipStream_t stream)
{
    hipLaunchKernelGGL((resident_jacobi_d<N, R, NW>), dim3(batch), dim3(64 * NW), 0, stream, m,
                       n, A, lda, sA, S, sS, U, ldu, sU, V, ldv, sV, tol, max_sweeps, info,
                       sweeps);
    return hipGetLastError();
}

}  // namespace

// Shape classes of the resident kernel: N = n rounded up to 16/32/64, R rows
// per lane and slot count such that all of W sits in wave 0 (m <= 64 R) and
// [W; V] fits the NW waves (m + N <= 64 R NW).  Returns false when no
// instance covers (m, n).
bool resident_config(int m, int n, int *N, int *R, int *NW)
{
    if (n < 1 || m < n) return false;
    const int nn = n <= 16 ? 16 : (n <= 32 ? 32 : (n <= 64 ? 64 : 0));
    if (!nn) return false;
    int r = (m + 63) / 64;
    const int rmax = nn == 16 ? 4 : (nn == 32 ? 3 : 1);
    if (r > rmax) return false;
    int nw = (m + nn + 64 * r - 1) / (64 * r);
    if (nw > 2) return false;
    // prefer one wave with one more slot when that keeps the register budget
    if (nw == 2 && r + 1 <= rmax && m + nn <= 64 * (r + 1)) {
        r += 1;
        nw = 1;
    }
    *N = nn;
    *R = r;
    *NW = nw;
    return true;
}

hipError_t launch_resident_d(int batch, int m, int n, const double *A, int lda, long long sA,
                             double *S, long long sS, double *U, int ldu, long long sU, double *V,
                             int ldv, long long sV, double tol, int max_sweeps, int *info,
                             int *sweeps, hipStream_t stream)
{
    int N, R, NW;
    if (!resident_config(m, n, &N, &R, &NW)) return hipErrorInvalidValue;
#define SVDB_RES(NN, RR, WW)                                                                   \
    if (N == NN && R == RR && NW == WW)                                                        \
        return launch_one<NN, RR, WW>(batch, m, n, A, lda, sA, S, sS, U, ldu, sU, V, ldv, sV,  \
                                      tol, max_sweeps, info, sweeps, stream);
    SVDB_RES(16, 1, 1)
    SVDB_RES(16, 2, 1)
    SVDB_RES(16, 3, 1)
    SVDB_RES(16, 4, 1)
    SVDB_RES(16, 4, 2)
    SVDB_RES(32, 1, 1)
    SVDB_RES(32, 2, 1)
    SVDB_RES(32, 3, 1)
    SVDB_RES(32, 3, 2)
    SVDB_RES(64, 1, 2)
#undef SVDB_RES
    return hipErrorInvalidValue;
}

}  // namespace svdb
