// device_common.hpp -- device helpers shared by the HIP kernels of the
// library: the round-robin pair schedule, the Jacobi rotation of
// eq. (sin-cos), and wavefront reductions.  gfx950 (wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace svdb {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Round-robin parallel ordering ("Algorithmic Background", Fig. "rr"; "Initial
// Design", subsection "Parallel Ordering"; Brent-Luk).
//
// l (even) indices sit at a two-row table; pair q of an iteration is
// (top seat q, bottom seat q).  Top seat 0 never moves; the other 2k-1 seats
// (k = l/2) form a ring -- top seats 1..k-1, then bottom seats k-1..0 -- and
// between iterations every index advances one ring position.  Initially top
// seat t holds 2t and bottom seat b holds 2b+1, so iteration 0 pairs
// (0,1),(2,3),...  The closed form below reads the ring position directly,
// which makes any (iteration, pair) computable in O(1) by any lane.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rr_initial(int x, int k)
{
    // index initially at ring position x
    return x <= k - 2 ? 2 * (x + 1) : 2 * (2 * k - 2 - x) + 1;
}

__device__ __forceinline__ void rr_pair(int l, int it, int q, int &i, int &j)
{
    const int k = l >> 1;
    const int ring = l - 1;                 // it < ring always
    int a, b;
    if (q == 0) {
        a = 0;
    } else {
        int y = (q - 1) - it;
        y += (y < 0) ? ring : 0;
        a = rr_initial(y, k);
    }
    int y = (2 * k - 2 - q) - it;
    y += (y < 0) ? ring : 0;
    b = rr_initial(y, k);
    i = a < b ? a : b;
    j = a < b ? b : a;
}

// ---------------------------------------------------------------------------
// Jacobi rotation of eq. (sin-cos) for a 2x2 Gram block [[gii, gij],
// [conj(gij), gjj]] with |gij| = ag > 0:
//   tau = (gii - gjj) / (2 ag),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1/sqrt(1 + t^2),  s = t c,  sign(0) = +1.
// For |tau| > 2^500 the root is t = 1/(2 tau) to working precision (and
// 1 + tau^2 would overflow).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void jacobi_cs(double gii, double gjj, double ag, double &c,
                                          double &s)
{
    const double tau = (gii - gjj) / (2.0 * ag);
    const double at = fabs(tau);
    double t = (at > 0x1p500) ? 0.5 / at : 1.0 / (at + sqrt(1.0 + at * at));
    t = (tau >= 0.0) ? t : -t;
    c = 1.0 / sqrt(1.0 + t * t);
    s = t * c;
}

// ---------------------------------------------------------------------------
// Wavefront reductions (butterfly through ds_swizzle / DPP chosen by the
// compiler for __shfl_xor).  `width` is a power of two <= 64; lanes are
// reduced within aligned groups of that width.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double group_sum(double v, int width)
{
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double group_max(double v, int width)
{
    for (int off = width >> 1; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum(v, kWave); }
__device__ __forceinline__ double wave_max(double v) { return group_max(v, kWave); }

// Value of lane (x + ROR) mod 16 of the same row of 16 lanes (DPP row_ror).
template <int ROR>
__device__ __forceinline__ double row_ror16(double v)
{
    constexpr int ctrl = 0x120 + ROR;
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int ROR>
__device__ __forceinline__ int row_ror16i(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x120 + ROR, 0xF, 0xF, false);
}

// Power-of-two scale that brings max|a| into [1, 2): multiplying by it is
// exact, so the iteration on the scaled matrix is the iteration on A with
// every quantity scaled by a power of two (no overflow in the Gram sums).
__device__ __forceinline__ double pow2_scale(double amax)
{
    if (!(amax > 0.0) || !isfinite(amax)) return 1.0;
    return ldexp(1.0, -ilogb(amax));
}

}  // namespace svdb
