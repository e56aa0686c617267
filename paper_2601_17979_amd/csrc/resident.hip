// resident.hip -- register-resident unblocked one-sided Jacobi SVD (Alg. 2),
// FP64, for n <= 64 columns.
//
// Layout.  The matrix is held as the stacked matrix [W; V] (W starts as A, V
// as I; a rotation acts on whole stacked columns) in registers: lane L holds
// row 64 t + L of W in slot t < RW and row L of V in slot RW.  N is n rounded
// up to 16, 32 or 64 (extra columns are zero and never rotate).  For m <= 32
// and N <= 32 the packed layout (RW = 0) keeps both in one slot: row L of W
// in lane L < 32 and row L of V in lane 32 + L, so no lane holds only
// padding.
//
// Ordering.  The round-robin ordering (Fig. "rr"; "Parallel Ordering") is a
// tournament table
// of K = N/2 seats per row: top seat q plays bottom seat q.  Between
// iterations every column except the one in top seat 0 moves one position
// around the ring top 1 .. top K-1, bottom K-1 .. bottom 0.  The seats are
// split into NS consecutive groups, one wavefront each; a wave keeps the
// columns of its seats in registers (arrays T, B), so a move inside a group
// is only a choice of destination registers, and the two columns that cross
// each group boundary per iteration go through LDS.  After N-1 iterations
// (one sweep) the table is back in its initial state: sweeps start with
// columns (2q, 2q+1) in seat q.
//
// Per iteration each wave forms g_ij of its pairs (Alg. 2, Gram entries) with
// one FMA per row, reduces them across lanes (permlane32/16 swaps, then an
// LDS transpose inside rows of 16 lanes), takes the rotate-or-skip test and
// the rotation of eq. (sin-cos) with lanes working on different pairs, and
// applies it to its rows of W and V.
//
// Rotations are applied in scaled form: the registers hold w_c / d_c with a
// per-column factor d_c (in LDS).  A Jacobi rotation with cosine c and
// tangent t then costs two FMAs per element, w_i <- w_i + mu_i w_j and
// w_j <- w_j + mu_j w_i, with d_i, d_j <- c d_i, c d_j (the scaled, or
// "fast", plane rotation; LAPACK's xGSVJ0 uses the same device).  Within one
// sweep the stored columns grow by at most (1/c)^(N-1) <= 2^((N-1)/2); the
// factors are folded back into the columns at every sweep start.
//
// The squared column norms g_ii are tracked with the exact identities
// g_ii' = g_ii + t |g_ij|, g_jj' = g_jj - t |g_ij| of a Jacobi rotation and
// recomputed from the columns at every sweep start, so the sweep that finds
// no pair to rotate -- the convergence test -- always uses exact norms.
#include "device_common.hpp"
#include "launchers.hpp"

namespace svdb {

namespace {

// Squared column norm below which a column of the pre-scaled matrix counts
// as zero (see the fold at the sweep start).
constexpr double kNegligible = 0x1p-960;

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
    int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct OpSum {
    __device__ static double apply(double a, double b) { return a + b; }
};
struct OpMax {
    __device__ static double apply(double a, double b) { return fmax(a, b); }
};

// Reduces KG (>= 4, power of two) per-lane values over the 64 lanes of a
// wave.  On return lane L = 16 rho + x holds the reduction of value
// (x mod KG/4) + (KG/4) rho, with identical bits in every lane that holds the
// same value.  buf: 64 * KG/4 doubles of LDS private to the calling wave.
//
// HALF: only lanes 0..31 carry terms (the W rows of the packed layout); the
// values of lanes 32..63 are ignored.
template <int KG, class Op, bool HALF = false>
__device__ __forceinline__ double reduce_pairs(double (&g)[KG], double *buf)
{
    constexpr int H = KG / 2, Q = KG / 4;
    const int lane = threadIdx.x & 63, rho = lane >> 4, x = lane & 15;
    double h[H];
#pragma unroll
    for (int v = 0; v < H; v++) {
        double a = g[v], b = g[v + H];
        swap32(a, b);
        h[v] = HALF ? a : Op::apply(a, b);
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
    wave_sync_lds();
    const int v = x % Q, h0 = (x / Q) * Q;
    const double *src = buf + (rho * Q + v) * 16 + h0;
    double s = src[0];
#pragma unroll
    for (int k = 1; k < Q; k++) s = Op::apply(s, src[k]);
    // Rotations by 8, 4, 2, 1 lanes in this order: after each step the values
    // repeat with half the period, so every step combines the same two
    // operands in both lanes of a pair and all lanes of one value end with
    // identical bits (the rotate-or-skip decision must agree across them).
    s = Op::apply(s, row_ror<8>(s));
    if constexpr (Q < 8) s = Op::apply(s, row_ror<4>(s));
    if constexpr (Q < 4) s = Op::apply(s, row_ror<2>(s));
    if constexpr (Q < 2) s = Op::apply(s, row_ror<1>(s));
    wave_sync_lds();
    return s;
}

// Reciprocal and reciprocal square root: hardware estimate plus two Newton
// steps, r <- r (2 - x r) and y <- y (3 - x y^2) / 2, which take the estimate
// to full double precision for normal positive x.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

__device__ __forceinline__ double rsq_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// Byte offset of a double in an array indexed by column id.
__device__ __forceinline__ double &at_off(double *base, int off)
{
    return *reinterpret_cast<double *>(reinterpret_cast<char *>(base) + off);
}

template <int N, int R, int NS>
struct Shared {
    static constexpr int K = N / 2, KG = K / NS, Q = KG / 4;
    double nrm[N];                    // squared column norms, by column id
    double d[N];                      // column scale factors, by column id
    double2 cs[NS][KG];               // (mu_top, mu_bot) per pair of each wave
    double buf[NS][64 * Q];           // reduction transposes
    double xch[2][NS][2][R][64];      // columns leaving each wave (top, bottom)
    double sig[N];
    int rank[N];
    // 8 x the column id initially at ring position y mod (N - 1), for
    // y < 2 (N - 1) (rr_initial): the top seat q > 0 holds at iteration it
    // the column that started at ring position q - 1 - it (mod N - 1), the
    // bottom seat q the one from N - 2 - q - it, so one table read with a
    // nonnegative index gives either
    int ring[2 * N];
    double amax[NS];
    int bad[NS];
    int flag;
};

// Waves per SIMD the register allocation is asked to allow, from the stored
// doubles per lane d = (RW + 1) N / NS (packed: N / NS): 3 up to d = 32 (168 VGPRs), 2 up to
// d = 64 (256), else 1.  With these bounds the iteration loop stays free of
// spills; what does not fit goes to scratch in the per-sweep fold and the
// finalisation, which run once per sweep, while a second or third resident
// wave per SIMD hides the latency of the loop's reduction and rotation chain.
constexpr int res_waves_per_eu(int N, int RW, int NS, bool NV = false)
{
    return (RW + (NV ? 0 : 1)) * N / NS <= 32 ? 3 : ((RW + (NV ? 0 : 1)) * N / NS <= 64 ? 2 : 1);
}

// W rows live in slots 0..RW-1 (row 64 t + lane), V rows in slot RW (row =
// lane); padding rows are zero, so Gram entries need no masks.  RW = 0 is
// the packed layout: W row L in lane L of slot 0, V row L in lane 32 + L,
// and the reductions over W rows read lanes 0..31 only.
//
// NV: no V rows (unpacked layouts only): the kernel iterates on W alone and
// writes S and U; the caller forms V from W (for the triangular X of the QR
// pre-processing, J = X^-1 W).  only: NULL, or a per-matrix flag; matrices
// whose flag is 0 are skipped (the rerun of the ones a cheaper path left).
// lower: A is lower triangular, its upper part is not read (zeros).
template <int N, int RW, int NS, bool NV = false>
__global__ __launch_bounds__(64 * NS, res_waves_per_eu(N, RW, NS, NV)) void resident_jacobi_d(
    int m, int n, const double *__restrict__ A, int lda, long long sA, double *S, long long sS,
    double *U, int ldu, long long sU, double *V, int ldv, long long sV, double tol,
    int max_sweeps, int *info, int *sweeps_out, const int *only, int lower)
{
    constexpr bool PK = RW == 0;
    static_assert(!(PK && NV), "the packed layout keeps V");
    constexpr int R = PK ? 1 : RW + (NV ? 0 : 1);   // register slots per column
    constexpr int WS = PK ? 1 : RW;      // slots holding W rows
    constexpr int VS = PK ? 0 : RW;      // slot holding V rows
    constexpr int VL = PK ? 32 : 0;      // lane of V row 0
    static_assert(!PK || N <= 32, "packed layout: n <= 32");
    using SH = Shared<N, R, NS>;
    constexpr int K = SH::K, KG = SH::KG, Q = SH::Q;
    static_assert(KG >= 4 && (KG & (KG - 1)) == 0, "4 <= pairs per wave, power of two");
    static_assert(N <= 64, "one V row per lane");
    __shared__ SH sh;

    const int b = blockIdx.x;
    if (only && !only[b]) return;
    const int lane = threadIdx.x & 63;
    // wave index as a scalar, so that per-wave LDS addresses stay in SGPRs
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int x = lane & 15;
    const int qloc = (x % Q) + Q * (lane >> 4);   // pair of this lane after a reduction
    const int q0 = wave * KG;                     // first seat of this wave
    const bool first = (wave == 0), last = (wave == NS - 1);
    A += (size_t)b * sA;

    double T[KG][R], B[KG][R];
    // ---- load W = A (zero padded) and V = I ----------------------------------
    double amax = 0.0;
    int bad = 0;
#pragma unroll
    for (int q = 0; q < KG; q++) {
        const int ct = 2 * (q0 + q), cb = ct + 1;
#pragma unroll
        for (int t = 0; t < WS; t++) {
            const int s = 64 * t + lane;   // packed: m <= 32, lanes >= 32 read nothing
            double xt = 0.0, xb = 0.0;
            if (s < m) {
                if (ct < n && (!lower || s >= ct)) xt = A[(size_t)ct * lda + s];
                if (cb < n && (!lower || s >= cb)) xb = A[(size_t)cb * lda + s];
            }
            bad |= !isfinite(xt) | !isfinite(xb);
            amax = fmax(amax, fmax(fabs(xt), fabs(xb)));
            T[q][t] = xt;
            B[q][t] = xb;
        }
        if constexpr (!NV) {
            T[q][VS] = (lane == VL + ct) ? 1.0 : (PK ? T[q][VS] : 0.0);
            B[q][VS] = (lane == VL + cb) ? 1.0 : (PK ? B[q][VS] : 0.0);
        }
    }
    bad = __any(bad);
    amax = wave_max(amax);
    if (lane == 0) {
        sh.amax[wave] = amax;
        sh.bad[wave] = bad;
    }
    if (threadIdx.x < N) sh.d[threadIdx.x] = 1.0;
    for (int y = threadIdx.x; y < 2 * (N - 1); y += 64 * NS) sh.ring[y] = 8 * rr_initial(y % (N - 1), K);
    if (threadIdx.x == 0) sh.flag = 0;
    __syncthreads();
    for (int w = 0; w < NS; w++) {
        bad |= sh.bad[w];
        amax = fmax(amax, sh.amax[w]);
    }
    if (bad) {
        if (threadIdx.x == 0) {
            info[b] = 2;
            if (sweeps_out) sweeps_out[b] = 0;
        }
        return;
    }
    const double scale = pow2_scale(amax);
    if (scale != 1.0) {
        const double sc = (PK && lane >= 32) ? 1.0 : scale;   // not the V rows
#pragma unroll
        for (int q = 0; q < KG; q++)
#pragma unroll
            for (int t = 0; t < WS; t++) {
                T[q][t] *= sc;
                B[q][t] *= sc;
            }
    }
    const double tol2 = tol * tol;

    double *buf = sh.buf[wave];
    double2 *cs = sh.cs[wave];
    // ring positions of this lane's top and bottom seat at iteration 0, one
    // ring length up (seat 0 of the top row never moves: column 0)
    const int qs = q0 + qloc;
    const int pt = (qs == 0 ? 0 : qs - 1) + (N - 1), pb = (N - 2 - qs) + (N - 1);
    // this wave's columns 2 q0 .. in the factor and norm arrays (one base
    // address, constant offsets)
    double *const dw = sh.d + 2 * q0;
    double *const nw = sh.nrm + 2 * q0;
    int sweeps = 0, converged = 0, par = 0;
    while (true) {
        // ---- fold the scale factors back in; exact squared norms ------------
        {
            // top seats, then bottom seats, KC pairs per reduction, so that
            // few partial sums are live next to the columns
            constexpr int KC = KG >= 8 ? 8 : KG, QC = KC / 4;
            int dead = 0;
#pragma unroll
            for (int side = 0; side < 2; side++)
#pragma unroll
                for (int h0 = 0; h0 < KG; h0 += KC) {
                    double p[KC];
#pragma unroll
                    for (int k = 0; k < KC; k++) {
                        const int q = h0 + k;
                        const double dq = dw[2 * q + side];
                        double(&X)[R] = side ? B[q] : T[q];
                        p[k] = 0.0;
#pragma unroll
                        for (int t = 0; t < R; t++) X[t] *= dq;
#pragma unroll
                        for (int t = 0; t < WS; t++) p[k] = fma(X[t], X[t], p[k]);
                    }
                    // lane (rho, x) holds pair h0 + (x mod QC) + QC rho
                    const double nv = reduce_pairs<KC, OpSum, PK>(p, buf);
                    // a column whose squared norm is below kNegligible (a
                    // norm below 2^-480 of the pre-scaled matrix, whose
                    // largest entry is about 1) is set to zero in W: rotating
                    // it further would only push rounding noise towards
                    // underflow
                    if (x < QC) {
                        const int c = 2 * (q0 + h0 + x + QC * (lane >> 4)) + side;
                        const bool z = nv < kNegligible;
                        dead |= z && nv != 0.0;
                        sh.nrm[c] = z ? 0.0 : nv;
                        sh.d[c] = 1.0;
                    }
                }
            if (__any(dead)) {
                wave_sync_lds();
                const bool wl = !PK || lane < 32;   // lanes of W rows
#pragma unroll
                for (int q = 0; q < KG; q++) {
                    const double2 nn = *reinterpret_cast<const double2 *>(&nw[2 * q]);
#pragma unroll
                    for (int t = 0; t < WS; t++) {
                        T[q][t] = (wl && nn.x == 0.0) ? 0.0 : T[q][t];
                        B[q][t] = (wl && nn.y == 0.0) ? 0.0 : B[q][t];
                    }
                }
            }
            __syncthreads();
        }
        if (converged || sweeps >= max_sweeps) break;
        sweeps++;
#pragma unroll 1
        for (int it = 0; it < N - 1; it++) {
            // columns of this lane's pair (byte offsets), read ahead of the
            // Gram entries that they do not depend on
            const int rt = sh.ring[pt - it], ob = sh.ring[pb - it];
            const int ot = qs == 0 ? 0 : rt;
            // ---- Gram entries of this wave's pairs --------------------------
            double g[KG];
#pragma unroll
            for (int q = 0; q < KG; q++) {
                g[q] = 0.0;
#pragma unroll
                for (int t = 0; t < WS; t++) g[q] = fma(T[q][t], B[q][t], g[q]);
            }
            const double gs = reduce_pairs<KG, OpSum, PK>(g, buf);
            // ---- rotate-or-skip and the rotation, one pair per lane group ---
            const double dt = at_off(sh.d, ot), db = at_off(sh.d, ob);
            const double gam = gs * dt * db;            // true g_ij
            const bool top_is_i = ot < ob;              // pair (i, j), i < j
            const double gt = at_off(sh.nrm, ot), gb = at_off(sh.nrm, ob);
            const double gi = top_is_i ? gt : gb, gj = top_is_i ? gb : gt;
            const double ag = fabs(gam);
            // |g_ij| >= tol sqrt(g_ii) sqrt(g_jj), squared unless the product
            // of the norms would underflow
            const double pij = gi * gj;
            const bool rot = (gam != 0.0) && gi >= kNegligible && gj >= kNegligible &&
                             (pij > 1e-250 ? ag * ag >= tol2 * pij : ag >= tol * sqrt(gi) * sqrt(gj));
            double mut = 0.0, mub = 0.0;
            if (rot) {
                const double tau = (gi - gj) * (0.5 * rcp_nr(ag));
                const double atau = fabs(tau);
                double tt;
                if (atau > 0x1p500) {
                    tt = 0.5 / atau;
                } else {
                    const double q2 = fma(atau, atau, 1.0);
                    tt = rcp_nr(atau + q2 * rsq_nr(q2));
                }
                tt = (tau >= 0.0) ? tt : -tt;           // t of eq. (sin-cos)
                const double c = rsq_nr(fma(tt, tt, 1.0));
                // new columns: a_i' = c (a_i + e t a_j), a_j' = c (a_j - e t a_i)
                const double et = (gam > 0.0) ? tt : -tt;
                const double sg = top_is_i ? et : -et;
                const double r = db * rcp_nr(dt);       // d_bottom / d_top
                mut = sg * r;
                mub = -sg * rcp_nr(r);
                if (x < Q) {
                    at_off(sh.nrm, top_is_i ? ot : ob) = fma(tt, ag, gi);
                    at_off(sh.nrm, top_is_i ? ob : ot) = fma(-tt, ag, gj);
                    at_off(sh.d, ot) = c * dt;
                    at_off(sh.d, ob) = c * db;
                }
            }
            if (x < Q) cs[qloc] = make_double2(mut, mub);
            if (__any(rot && x < Q) && lane == 0) sh.flag = 1;
            wave_sync_lds();
            // ---- apply to W and V and move the seats -------------------------
            // top seat q -> top q+1 and bottom seat q -> bottom q-1 inside the
            // wave; the last top seat leaves for the next wave (the last wave
            // keeps it as its last bottom seat), bottom seat 0 leaves for the
            // previous wave (the first wave moves it to top seat 1), and top
            // seat 0 of the first wave stays.
            // Pairs are processed from the last seat down: the new top column
            // of pair q goes straight into top seat q+1 (consumed one step
            // earlier), the new bottom column waits one step in `prev` until
            // bottom seat q-1 has been read.
            double outT[R], keep0[R], prev[R];
            // (mu_top, mu_bot) are read four pairs at a time, one group ahead,
            // so that at most eight pairs' parameters occupy registers
            constexpr int CH = KG < 4 ? KG : 4;
            double2 mu_nx[CH];
#pragma unroll
            for (int k = 0; k < CH; k++) mu_nx[k] = cs[KG - 1 - k];
#pragma unroll
            for (int c0 = 0; c0 < KG; c0 += CH) {
                double2 mu_cu[CH];
#pragma unroll
                for (int k = 0; k < CH; k++) mu_cu[k] = mu_nx[k];
                if (c0 + CH < KG) {
#pragma unroll
                    for (int k = 0; k < CH; k++) mu_nx[k] = cs[KG - 1 - (c0 + CH + k)];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < CH; k++) {
                    const int q = KG - 1 - (c0 + k);
                    const double2 mu = mu_cu[k];
#pragma unroll
                    for (int t = 0; t < R; t++) {
                        const double a = T[q][t], bb = B[q][t];
                        const double na = fma(mu.x, bb, a);
                        const double nb = fma(mu.y, a, bb);
                        if (q == KG - 1) outT[t] = na;
                        else T[q + 1][t] = na;
                        if (q == 0) keep0[t] = na;
                        if (q < KG - 1) B[q][t] = prev[t];
                        prev[t] = nb;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            double (&outB)[R] = prev;               // new bottom seat 0
            if constexpr (NS > 1) {
#pragma unroll
                for (int t = 0; t < R; t++) {
                    sh.xch[par][wave][0][t][lane] = outT[t];
                    sh.xch[par][wave][1][t][lane] = outB[t];
                }
                __syncthreads();
            }
            const int wprev = first ? 0 : wave - 1, wnext = last ? wave : wave + 1;
#pragma unroll
            for (int t = 0; t < R; t++) {
                // top seat 0: the first wave keeps its own, the others take the
                // last top seat of the previous wave
                T[0][t] = first ? keep0[t] : sh.xch[par][wprev][0][t][lane];
                // bottom seat 0 of the first wave turns into top seat 1
                if (first) T[1][t] = outB[t];
                // last bottom seat: the last wave turns its last top seat, the
                // others take bottom seat 0 of the next wave
                B[KG - 1][t] = last ? outT[t] : sh.xch[par][wnext][1][t][lane];
            }
            par ^= 1;
        }
        __syncthreads();
        converged = (sh.flag == 0);
        __syncthreads();
        if (threadIdx.x == 0) sh.flag = 0;
    }

    // ---- finalise: sigma_c = ||w_c|| from the exact squared norms of the last
    // fold.  A column whose squared norm is below 2^-900 (entries below
    // 2^-450 after the pre-scaling) is first multiplied by 2^600, an exact
    // power of two that keeps every square representable; its factor 2^-600
    // is remembered in d_c and divided out of sigma_c and of its V part.
    {
        const int c = 2 * (q0 + qloc);
        int tiny = 0;
        if (x < Q) {
            const double nt = sh.nrm[c], nb = sh.nrm[c + 1];
            const bool tt = nt < 0x1p-900, tb = nb < 0x1p-900;
            sh.d[c] = tt ? 0x1p-600 : 1.0;
            sh.d[c + 1] = tb ? 0x1p-600 : 1.0;
            tiny = tt || tb;
        }
        tiny = __any(tiny);
        wave_sync_lds();
        if (tiny) {
            double pt[KG], pb[KG];
#pragma unroll
            for (int q = 0; q < KG; q++) {
                const double ft = sh.d[2 * (q0 + q)] < 1.0 ? 0x1p600 : 1.0;
                const double fb = sh.d[2 * (q0 + q) + 1] < 1.0 ? 0x1p600 : 1.0;
                pt[q] = 0.0;
                pb[q] = 0.0;
#pragma unroll
                for (int t = 0; t < R; t++) {
                    T[q][t] *= ft;
                    B[q][t] *= fb;
                }
#pragma unroll
                for (int t = 0; t < WS; t++) {
                    pt[q] = fma(T[q][t], T[q][t], pt[q]);
                    pb[q] = fma(B[q][t], B[q][t], pb[q]);
                }
            }
            const double nt = reduce_pairs<KG, OpSum, PK>(pt, buf);
            const double nb = reduce_pairs<KG, OpSum, PK>(pb, buf);
            if (x < Q) {
                sh.nrm[c] = nt;
                sh.nrm[c + 1] = nb;
            }
        }
        if (x < Q) {
            sh.sig[c] = sqrt(sh.nrm[c]) * sh.d[c];
            sh.sig[c + 1] = sqrt(sh.nrm[c + 1]) * sh.d[c + 1];
        }
    }
    __syncthreads();
    if (threadIdx.x < N) {
        const int c = threadIdx.x;
        const double sc = sh.sig[c];
        int rk = 0;
        for (int j = 0; j < N; j++) {
            const double sj = sh.sig[j];
            rk += (sj > sc) || (sj == sc && j < c);
        }
        sh.rank[c] = rk;
    }
    __syncthreads();
    S += (size_t)b * sS;
    if (threadIdx.x < n) S[sh.rank[threadIdx.x]] = sh.sig[threadIdx.x] / scale;
    if (U) U += (size_t)b * sU;
    if (V) V += (size_t)b * sV;
#pragma unroll
    for (int q = 0; q < KG; q++) {
        if (q % 4 == 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int c = 2 * (q0 + q) + h;
            if (c >= n) continue;
            const int rk = sh.rank[c];
            const double nc = sh.nrm[c];
            const double inv = nc > 0.0 ? rsq_nr(nc) : 0.0;   // 1 / ||stored column||
            const double dv = sh.d[c];
            (void)dv;
#pragma unroll
            for (int t = 0; t < WS; t++) {
                const double val = h ? B[q][t] : T[q][t];
                const int s = 64 * t + lane;
                if (U && s < m) U[(size_t)rk * ldu + s] = val * inv;
            }
            if constexpr (!NV) {
                const int vr = lane - VL;
                if (V && vr >= 0 && vr < n)
                    V[(size_t)rk * ldv + vr] = (h ? B[q][VS] : T[q][VS]) * dv;
            }
        }
    }
    bool any_zero = false;
    for (int c = 0; c < n; c++) any_zero |= !(sh.sig[c] > 0.0);
    // sigma = 0: complete U by Gram-Schmidt on e_1, e_2, ... (rare; wave 0,
    // on the freshly written columns of U in global memory)
    if (U && any_zero) {
        __threadfence();
        __syncthreads();
        if (wave == 0) {
            int cand = 0;
            for (int i = 0; i < n; i++) {
                if (sh.sig[i] > 0.0) continue;
                double *u = U + (size_t)sh.rank[i] * ldu;
                for (; cand < m; cand++) {
                    for (int r = lane; r < m; r += 64) u[r] = (r == cand) ? 1.0 : 0.0;
                    __threadfence();
                    for (int pass = 0; pass < 2; pass++)
                        for (int j = 0; j < n; j++) {
                            if (j == i || (sh.sig[j] == 0.0 && j > i)) continue;
                            const double *qv = U + (size_t)sh.rank[j] * ldu;
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
    if (threadIdx.x == 0) {
        info[b] = converged ? 0 : 1;
        if (sweeps_out) sweeps_out[b] = sweeps;
    }
}

template <int N, int R, int NS, bool NV = false>
hipError_t launch_one(int batch, int m, int n, const double *A, int lda, long long sA, double *S,
                      long long sS, double *U, int ldu, long long sU, double *V, int ldv,
                      long long sV, double tol, int max_sweeps, int *info, int *sweeps,
                      hipStream_t stream, const int *only, bool lower)
{
    hipLaunchKernelGGL((resident_jacobi_d<N, R, NS, NV>), dim3(batch), dim3(64 * NS), 0, stream,
                       m, n, A, lda, sA, S, sS, U, ldu, sU, V, ldv, sV, tol, max_sweeps, info,
                       sweeps, only, lower ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

// Shape classes: N = n rounded up to 16/32/64; RW = ceil(m/64) slots of W
// rows per lane (m <= 256) plus one slot of V rows, or RW = 0 (the packed
// layout, W and V in one slot) for m <= 32 and N <= 32; NS = waves (seat groups)
// per matrix, with at most 96 stored doubles per lane.  `ns` = 0 picks the
// tuned default.  Returns false when no instance covers (m, n, ns).
bool resident_config(int m, int n, int ns, int *N, int *R, int *NS)
{
    if (n < 1 || m < n) return false;
    const int nn = n <= 16 ? 16 : (n <= 32 ? 32 : (n <= 64 ? 64 : 0));
    if (!nn) return false;
    const int rw = (m <= 32 && nn <= 32) ? 0 : (m + 63) / 64;
    if (rw > 4) return false;
    if (ns == 0) {
        // the measured choice for this class if it fits, else the rule
        const int t = tuned_resident_waves(nn, rw);
        ns = ((rw + 1) * nn > 96) ? 2 : 1;
        if ((t == 1 || t == 2 || t == 4) && (nn / 2) / t >= 4 && (rw + 1) * nn / t <= 96) ns = t;
    }
    if (ns != 1 && ns != 2 && ns != 4) return false;
    if ((nn / 2) / ns < 4) return false;
    if ((rw + 1) * nn / ns > 96) return false;
    *N = nn;
    *R = rw;
    *NS = ns;
    return true;
}

bool resident_nv_supported(int m, int n)
{
    return n > 32 && n <= 64 && m >= n && m <= 64;
}

hipError_t launch_resident_d(int batch, int m, int n, int ns, const double *A, int lda,
                             long long sA, double *S, long long sS, double *U, int ldu,
                             long long sU, double *V, int ldv, long long sV, double tol,
                             int max_sweeps, int *info, int *sweeps, hipStream_t stream,
                             bool nv, const int *only, bool lower)
{
    if (nv) {   // W alone: N = 64, one slot of W rows
        if (!resident_nv_supported(m, n)) return hipErrorInvalidValue;
        const int w = ns == 0 ? 2 : ns;
        if (w == 1)
            return launch_one<64, 1, 1, true>(batch, m, n, A, lda, sA, S, sS, U, ldu, sU, nullptr,
                                              ldv, sV, tol, max_sweeps, info, sweeps, stream,
                                              only, lower);
        if (w == 2)
            return launch_one<64, 1, 2, true>(batch, m, n, A, lda, sA, S, sS, U, ldu, sU, nullptr,
                                              ldv, sV, tol, max_sweeps, info, sweeps, stream,
                                              only, lower);
        if (w == 4)
            return launch_one<64, 1, 4, true>(batch, m, n, A, lda, sA, S, sS, U, ldu, sU, nullptr,
                                              ldv, sV, tol, max_sweeps, info, sweeps, stream,
                                              only, lower);
        return hipErrorInvalidValue;
    }
    int N, RW, NS;
    if (!resident_config(m, n, ns, &N, &RW, &NS)) return hipErrorInvalidValue;
#define SVDB_RES(NN, RR, WW)                                                                   \
    if (N == NN && RW == RR && NS == WW)                                                       \
        return launch_one<NN, RR, WW>(batch, m, n, A, lda, sA, S, sS, U, ldu, sU, V, ldv, sV,  \
                                      tol, max_sweeps, info, sweeps, stream, only, lower);
    SVDB_RES(16, 0, 1)
    SVDB_RES(16, 0, 2)
    SVDB_RES(32, 0, 1)
    SVDB_RES(32, 0, 2)
    SVDB_RES(32, 0, 4)
    SVDB_RES(16, 1, 1)
    SVDB_RES(16, 2, 1)
    SVDB_RES(16, 3, 1)
    SVDB_RES(16, 4, 1)
    SVDB_RES(16, 1, 2)
    SVDB_RES(16, 2, 2)
    SVDB_RES(16, 3, 2)
    SVDB_RES(16, 4, 2)
    SVDB_RES(32, 1, 1)
    SVDB_RES(32, 2, 1)
    SVDB_RES(32, 1, 2)
    SVDB_RES(32, 2, 2)
    SVDB_RES(32, 3, 2)
    SVDB_RES(32, 4, 2)
    SVDB_RES(32, 1, 4)
    SVDB_RES(32, 2, 4)
    SVDB_RES(32, 3, 4)
    SVDB_RES(32, 4, 4)
    SVDB_RES(64, 1, 2)
    SVDB_RES(64, 2, 2)
    SVDB_RES(64, 1, 4)
    SVDB_RES(64, 2, 4)
    SVDB_RES(64, 3, 4)
    SVDB_RES(64, 4, 4)
#undef SVDB_RES
    return hipErrorInvalidValue;
}

}  // namespace svdb
