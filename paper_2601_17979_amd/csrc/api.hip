// api.hip -- host runtime behind include/svdb.h: argument checks, the plan
// (which kernel handles which shape), workspace sizing and launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "launchers.hpp"
#include "svdb.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(SVDB_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

double default_tol(svdb_dtype_t dt)
{
    // k * u with k = 30 and u = 2^-s (s significand bits incl. the implicit one)
    const bool single = (dt == SVDB_R32 || dt == SVDB_C64);
    return 30.0 * (single ? ldexp(1.0, -24) : ldexp(1.0, -53));
}

int elt_bytes(svdb_dtype_t dt)
{
    return dt == SVDB_R32 ? 4 : dt == SVDB_C128 ? 16 : 8;
}

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// bytes of the FP64 copies of A (m x n), S, U (m x n) and V (n x n)
size_t via64_bytes(int batch, int m, int n)
{
    const size_t mn = (size_t)batch * m * n * 8;
    return 2 * al256(mn) + al256((size_t)batch * n * 8) + al256((size_t)batch * n * n * 8);
}

// bytes of the A^H copy of a strided batch of wide matrices
size_t wide_copy_bytes(svdb_dtype_t dtype, int batch, int m, int n)
{
    return ((size_t)batch * m * n * elt_bytes(dtype) + 255) / 256 * 256;
}

struct Plan {
    int path = SVDB_PATH_AUTO;
    int nb = 0;
    int threads = 0;
    int inner = 0;              // block method: inner sweeps (0: the built-in rule)
    double tol_start = 0.0;     // block method: dynamic inner tolerance
    double tol_rate = 0.0;
    bool precond = false;   // QR pre-processing, resident Jacobi on R^T
    bool pivot = false;         // precond: column pivoting in the first QR
    bool precond_big = false;   // QR pre-processing, block Jacobi on R^T
    bool precond_tall = false;  // QR in global memory, resident Jacobi on R^T
    bool via64 = false;         // FP32 input on an FP64 preconditioned path
};

svdb_opts_t resolve_opts(const svdb_opts_t *o)
{
    svdb_opts_t r;
    svdb_opts_default(&r);
    if (o) {
        r = *o;
        if (r.max_sweeps <= 0) r.max_sweeps = 100;
        if (r.masking < 0) r.masking = 1;
        if (r.waves < 0) r.waves = 0;
        if (r.inner_sweeps < -1) r.inner_sweeps = -1;
        r.persistent = r.persistent != 0;
    }
    return r;
}

// Block width and inner solve of the block method for an m x n request of
// this dtype: the caller's choices where given, else the measured table,
// else the built-in rules.  Returns 0 when the width is not supported.
int block_choice(svdb_dtype_t dt, int m, int n, const svdb_opts_t &o, Plan *p)
{
    const bool cx = dt == SVDB_C64 || dt == SVDB_C128;
    svdb::BlockChoice t;
    const bool have = svdb::tuned_block((int)dt, m, n, &t);
    int nb = o.nb;
    if (nb == 0 && have && svdb::blocked_nb(m, n, t.nb, cx) == t.nb) nb = t.nb;
    nb = svdb::blocked_nb(m, n, nb, cx);
    if (!nb) return 0;
    p->nb = nb;
    p->inner = o.inner_sweeps;
    p->tol_start = o.inner_tol_start;
    p->tol_rate = o.inner_tol_rate;
    // the table's inner solve was measured with its own width, on m = n and
    // m = 3 n; two block columns with m >= 8 np (much taller, where the
    // converged solve replaces outer sweeps that each stream all m rows)
    // keep the built-in rule
    const int np = svdb::blocked_np(n, nb);
    const bool very_tall = np == 2 * nb && m >= 8 * np;
    if (o.inner_sweeps == 0 && have && nb == t.nb && !very_tall) {
        p->inner = t.inner;
        if (o.inner_tol_start <= 0.0 && t.tol_start > 0.0) {
            p->tol_start = t.tol_start;
            p->tol_rate = t.tol_rate;
        }
    }
    return nb;
}

bool plain_fits(int m, int n)
{
    return svdb::plain_lds_bytes(m, n) <= (size_t)svdb::plain_max_lds_bytes() && n <= 512;
}

int make_plan(svdb_dtype_t dt, int m, int n, const svdb_opts_t &o, Plan *p)
{
    if (o.precision != 0 && o.precision != 1)
        return fail(SVDB_ERR_UNSUPPORTED, "precision must be 0 or 1");
    if (o.precision == 1 && dt != SVDB_R64)
        return fail(SVDB_ERR_UNSUPPORTED, "precision mode 1 needs SVDB_R64 input");
    if (o.precondition < -1 || o.precondition > 2)
        return fail(SVDB_ERR_UNSUPPORTED, "precondition must be -1, 0, 1 or 2");
    if (o.inner_tol_start > 0.0) {
        if (!(o.inner_tol_rate > 0.0 && o.inner_tol_rate < 1.0) || !isfinite(o.inner_tol_start))
            return fail(SVDB_ERR_UNSUPPORTED, "dynamic inner tolerance: rate must be in (0, 1)");
    }
    int path = o.path;
    int rN = 0, rR = 0, rW = 0;
    // QR preconditioning of real matrices (FP32 input runs it in FP64): AUTO
    // (precondition -1 or 1) and RESIDENT (1)
    const bool real = dt == SVDB_R64 || dt == SVDB_R32;
    p->via64 = dt == SVDB_R32;
    const bool pc_ok = real && o.precision == 0 && svdb::precond_supported(m, n);
    const bool pc_req = (path == SVDB_PATH_AUTO && o.precondition != 0) ||
                        (path == SVDB_PATH_RESIDENT && o.precondition >= 1);
    // FP64 with n <= 16 and m < 8 n: the two QRs and the two applications of
    // Q cost more than the sweeps they save (measured on batches of Gaussian,
    // geometric-spectrum and uniform [0, 1] matrices), so AUTO without an
    // explicit request runs the resident kernel on A itself
    const bool pc_pays = !(dt == SVDB_R64 && n <= 16 && m < 8 * n);
    if (pc_req && pc_ok && (pc_pays || o.precondition >= 1)) {
        if (!svdb::resident_config(n, n, o.waves, &rN, &rR, &rW))
            return fail(SVDB_ERR_UNSUPPORTED,
                        "resident path: no kernel with this many waves per matrix for n");
        p->path = SVDB_PATH_RESIDENT;
        p->nb = 0;
        p->threads = 64 * rW;
        p->precond = true;
        p->pivot = o.precondition == 2;
        return 0;
    }
    if (o.precondition == 2)
        return fail(SVDB_ERR_UNSUPPORTED,
                    "column pivoting (precondition 2) applies to real n <= 64, m n <= 8192");
    // tall matrices with few columns beyond the register QR (m <= 4096): QR
    // in global memory, the resident Jacobi on R^T (AUTO, or RESIDENT with 1)
    const bool pct_ok = real && o.precision == 0 && !pc_ok &&
                        (o.precondition == 1 ? svdb::precond_tall_supported(m, n)
                                             : svdb::precond_tall_auto(m, n));
    if (pc_req && pct_ok) {
        svdb::resident_config(n, n, 0, &rN, &rR, &rW);
        p->path = SVDB_PATH_RESIDENT;
        p->nb = 0;
        p->threads = 64 * rW;
        p->precond_tall = true;
        return 0;
    }
    // wide matrices: the block Jacobi on R^T (AUTO, or BLOCKED with 1)
    // (FP64 input may ask for the mixed mode on R2^T, precision 1)
    const bool pcb_ok = real && (o.precision == 0 || dt == SVDB_R64) && !pc_ok &&
                        svdb::precond_big_supported(m, n);
    const bool pcb_req = (path == SVDB_PATH_AUTO && o.precondition != 0) ||
                         (path == SVDB_PATH_BLOCKED && o.precondition == 1);
    if (pcb_req && pcb_ok) {
        // the block method runs on the n x n FP64 factor R2^T
        const int nb = block_choice(SVDB_R64, n, n, o, p);
        if (!nb) return fail(SVDB_ERR_UNSUPPORTED, "blocked path: nb must be 8, 16 or 32");
        p->path = SVDB_PATH_BLOCKED;
        p->nb = nb;
        p->threads = 256;
        p->precond_big = true;
        return 0;
    }
    p->via64 = false;
    if (o.precondition == 1)
        return fail(SVDB_ERR_UNSUPPORTED, "QR preconditioning does not apply to this request");
    // the unblocked kernels are FP64 only; FP32 and the mixed mode use the block method
    const bool unblocked_ok = dt == SVDB_R64 && o.precision == 0;
    const bool res_ok = unblocked_ok && svdb::resident_config(m, n, o.waves, &rN, &rR, &rW);
    if (path == SVDB_PATH_AUTO) path = res_ok ? SVDB_PATH_RESIDENT : SVDB_PATH_BLOCKED;
    if (path == SVDB_PATH_BLOCKED) {
        const bool cx = dt == SVDB_C64 || dt == SVDB_C128;
        // the mixed mode takes the choices measured for FP64 input
        const int nb = block_choice(o.precision == 1 ? SVDB_R64 : dt, m, n, o, p);
        if (!nb)
            return fail(SVDB_ERR_UNSUPPORTED, cx ? "blocked path: complex needs nb = 16"
                                                 : "blocked path: nb must be 8, 16 or 32");
        if (n < 1) return fail(SVDB_ERR_UNSUPPORTED, "blocked path: n must be >= 1");
        p->path = SVDB_PATH_BLOCKED;
        p->nb = nb;
        p->threads = 256;
        return 0;
    }
    if (!unblocked_ok)
        return fail(SVDB_ERR_UNSUPPORTED, "path %d handles FP64 with precision 0 only", path);
    if (path == SVDB_PATH_RESIDENT) {
        if (!res_ok)
            return fail(SVDB_ERR_UNSUPPORTED, "resident path: no instance for %d x %d", m, n);
        p->path = SVDB_PATH_RESIDENT;
        p->nb = 0;
        p->threads = 64 * rW;
        return 0;
    }
    if (path == SVDB_PATH_PLAIN) {
        if (!plain_fits(m, n))
            return fail(SVDB_ERR_UNSUPPORTED, "plain path: %d x %d does not fit in LDS", m, n);
        p->path = SVDB_PATH_PLAIN;
        p->nb = 0;
        p->threads = 256;
        return 0;
    }
    return fail(SVDB_ERR_UNSUPPORTED, "path %d is not implemented in this build", path);
}

}  // namespace

extern "C" {

void svdb_opts_default(svdb_opts_t *o)
{
    if (!o) return;
    o->max_sweeps = 100;
    o->path = SVDB_PATH_AUTO;
    o->nb = 0;
    o->masking = 1;
    o->precision = 0;
    o->sweeps = nullptr;
    o->waves = 0;
    o->precondition = -1;
    o->inner_sweeps = 0;
    o->persistent = 0;
    o->inner_tol_start = 0.0;
    o->inner_tol_rate = 0.0;
}

const char *svdb_last_error(void) { return g_err.c_str(); }

const char *svdb_version(void) { return "svdb 0.1 (gfx950)"; }

int svdb_plan(svdb_dtype_t dtype, int m, int n, const svdb_opts_t *opts, int *path, int *nb,
              int *threads)
{
    svdb_opts_t o = resolve_opts(opts);
    if (m < 0 || n < 0) return fail(-3, "need m, n >= 0");
    Plan p;
    // a wide matrix runs the plan of its conjugate transpose
    int rc = m >= n ? make_plan(dtype, m, n, o, &p) : make_plan(dtype, n, m, o, &p);
    if (rc) return rc;
    if (path) *path = p.path;
    if (nb) *nb = p.nb;
    if (threads) *threads = p.threads;
    return 0;
}

size_t svdb_workspace_size(svdb_dtype_t dtype, int batch, int m, int n, const svdb_opts_t *opts)
{
    if (batch < 0 || m < 0 || n < 0) return (size_t)-1;
    if (m == 0 || n == 0) return 0;   // nothing to factor
    if (n > m) {   // A^H (n x m) in the workspace, then the tall call's own
        const size_t tall = svdb_workspace_size(dtype, batch, n, m, opts);
        if (tall == (size_t)-1) return tall;
        return wide_copy_bytes(dtype, batch, m, n) + tall;
    }
    svdb_opts_t o = resolve_opts(opts);
    Plan p;
    if (make_plan(dtype, m, n, o, &p)) return (size_t)-1;
    // FP32 on an FP64 path: FP64 copies of A, S, U and V come first
    const size_t w64 = p.via64 ? via64_bytes(batch, m, n) : 0;
    if (p.precond) return w64 + svdb::precond_workspace_bytes(batch, m, n);
    if (p.precond_big)
        return w64 + svdb::precond_big_workspace_bytes(batch, m, n, p.nb, o.precision == 1);
    if (p.precond_tall) return w64 + svdb::precond_tall_workspace_bytes(batch, m, n);
    if (p.path == SVDB_PATH_BLOCKED)
        return svdb::blocked_workspace_bytes(batch, m, n, p.nb, elt_bytes(dtype),
                                             o.precision == 1);
    return 0;
}

namespace {

// The tall (m >= n) call on plan p; outputs as in svdb_svd_strided_batched.
hipError_t run_tall(svdb_dtype_t dtype, const Plan &p, const svdb_opts_t &o, int batch, int m,
                    int n, const void *A, int lda, long long strideA, void *S, long long strideS,
                    void *U, int ldu, long long strideU, void *V, int ldv, long long strideV,
                    double tol, int *info, void *workspace, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (p.via64) {
        // FP32 input on an FP64 preconditioned path: A widened into the
        // workspace, the FP64 results narrowed into the caller's buffers
        // (matrices with info 2 keep their outputs untouched)
        const long long smn = (long long)m * n, snn = (long long)n * n;
        char *q = (char *)workspace;
        double *A64 = (double *)q;
        q += al256((size_t)batch * smn * 8);
        double *U64 = (double *)q;
        q += al256((size_t)batch * smn * 8);
        double *S64 = (double *)q;
        q += al256((size_t)batch * n * 8);
        double *V64 = (double *)q;
        q += al256((size_t)batch * snn * 8);
        Plan p64 = p;
        p64.via64 = false;
        e = svdb::launch_widen_f32(batch, m, n, (const float *)A, lda, strideA, A64, m, smn, s);
        if (e == hipSuccess)
            e = run_tall(SVDB_R64, p64, o, batch, m, n, A64, m, smn, S64, n, U ? U64 : nullptr, m,
                         smn, V ? V64 : nullptr, n, snn, tol, info, q, s);
        if (e == hipSuccess)
            e = svdb::launch_narrow_f64(batch, n, 1, S64, n, n, (float *)S, n, strideS, info, s);
        if (e == hipSuccess && U)
            e = svdb::launch_narrow_f64(batch, m, n, U64, m, smn, (float *)U, ldu, strideU, info, s);
        if (e == hipSuccess && V)
            e = svdb::launch_narrow_f64(batch, n, n, V64, n, snn, (float *)V, ldv, strideV, info, s);
        return e;
    }
    if (p.precond_tall) {
        e = svdb::launch_precond_tall_d(batch, m, n, (const double *)A, lda, strideA, (double *)S,
                                        strideS, (double *)U, ldu, strideU, (double *)V, ldv,
                                        strideV, tol, o.max_sweeps, info, o.sweeps, workspace, s);
    } else if (p.precond_big) {
        e = svdb::launch_precond_big_d(batch, m, n, p.nb, (const double *)A, lda, strideA,
                                       (double *)S, strideS, (double *)U, ldu, strideU,
                                       (double *)V, ldv, strideV, tol, o.max_sweeps, o.masking,
                                       info, o.sweeps, workspace, s, p.inner, o.persistent,
                                       p.tol_start, p.tol_rate,
                                       o.precision == 1 ? fmax(tol, default_tol(SVDB_R32)) : 0.0);
    } else if (p.precond) {
        e = svdb::launch_precond_d(batch, m, n, o.waves, (const double *)A, lda, strideA,
                                   (double *)S, strideS, (double *)U, ldu, strideU, (double *)V,
                                   ldv, strideV, tol, o.max_sweeps, info, o.sweeps, workspace, s,
                                   p.pivot);
    } else if (p.path == SVDB_PATH_RESIDENT) {
        e = svdb::launch_resident_d(batch, m, n, o.waves, (const double *)A, lda, strideA,
                                    (double *)S,
                                    strideS, (double *)U, ldu, strideU, (double *)V, ldv,
                                    strideV, tol, o.max_sweeps, info, o.sweeps, s);
    } else if (p.path == SVDB_PATH_BLOCKED && dtype == SVDB_R32) {
        e = svdb::launch_blocked_s(batch, m, n, p.nb, (const float *)A, lda, strideA, (float *)S,
                                   strideS, (float *)U, ldu, strideU, (float *)V, ldv, strideV,
                                   tol, o.max_sweeps, o.masking, info, o.sweeps, workspace, s,
                                   p.inner, o.persistent,
                                   p.tol_start, p.tol_rate);
    } else if (p.path == SVDB_PATH_BLOCKED && dtype == SVDB_C128) {
        e = svdb::launch_blocked_z(batch, m, n, p.nb, A, lda, strideA, (double *)S, strideS, U,
                                   ldu, strideU, V, ldv, strideV, tol, o.max_sweeps, o.masking,
                                   info, o.sweeps, workspace, s, p.inner, o.persistent,
                                   p.tol_start, p.tol_rate);
    } else if (p.path == SVDB_PATH_BLOCKED && dtype == SVDB_C64) {
        e = svdb::launch_blocked_c(batch, m, n, p.nb, A, lda, strideA, (float *)S, strideS, U,
                                   ldu, strideU, V, ldv, strideV, tol, o.max_sweeps, o.masking,
                                   info, o.sweeps, workspace, s, p.inner, o.persistent,
                                   p.tol_start, p.tol_rate);
    } else if (p.path == SVDB_PATH_BLOCKED && o.precision == 1) {
        const double tol32 = fmax(tol, default_tol(SVDB_R32));
        e = svdb::launch_blocked_mixed_d(batch, m, n, p.nb, (const double *)A, lda, strideA,
                                         (double *)S, strideS, (double *)U, ldu, strideU,
                                         (double *)V, ldv, strideV, tol, tol32, o.max_sweeps,
                                         o.masking, info, o.sweeps, workspace, s,
                                         p.inner, o.persistent,
                                   p.tol_start, p.tol_rate);
    } else if (p.path == SVDB_PATH_BLOCKED) {
        e = svdb::launch_blocked_d(batch, m, n, p.nb, (const double *)A, lda, strideA,
                                   (double *)S, strideS, (double *)U, ldu, strideU, (double *)V,
                                   ldv, strideV, tol, o.max_sweeps, o.masking, info, o.sweeps,
                                   workspace, s, p.inner, o.persistent,
                                   p.tol_start, p.tol_rate);
    } else if (p.path == SVDB_PATH_PLAIN) {
        e = svdb::launch_plain_d(batch, m, n, (const double *)A, lda, strideA, (double *)S,
                                 strideS, (double *)U, ldu, strideU, (double *)V, ldv, strideV,
                                 tol, o.max_sweeps, info, o.sweeps, s);
    }
    return e;
}

}  // namespace

int svdb_svd_strided_batched(svdb_dtype_t dtype, int batch, int m, int n, const void *A, int lda,
                             long long strideA, void *S, long long strideS, void *U, int ldu,
                             long long strideU, void *V, int ldv, long long strideV, double tol,
                             int *info, void *workspace, size_t ws_bytes,
                             const svdb_opts_t *opts, void *stream)
{
    g_err.clear();
    if ((int)dtype < SVDB_R32 || (int)dtype > SVDB_C128) return fail(-1, "invalid dtype");
    if (batch < 0) return fail(-2, "batch < 0");
    if (m < 0) return fail(-3, "m < 0");
    if (n < 0) return fail(-4, "n < 0");
    const int k = m < n ? m : n;   // singular values per matrix
    const bool empty = (batch == 0 || k == 0);
    if (!A && !empty) return fail(-5, "A is NULL");
    if (lda < (m > 1 ? m : 1)) return fail(-6, "lda < max(1, m)");
    if (batch > 1 && !empty && strideA < (long long)lda * n) return fail(-7, "strideA < lda * n");
    if (!S && !empty) return fail(-8, "S is NULL");
    if (batch > 1 && !empty && strideS < k) return fail(-9, "strideS < min(m, n)");
    if (U) {
        if (ldu < (m > 1 ? m : 1)) return fail(-11, "ldu < max(1, m)");
        if (batch > 1 && !empty && strideU < (long long)ldu * k) return fail(-12, "strideU < ldu * min(m, n)");
    }
    if (V) {
        if (ldv < (n > 1 ? n : 1)) return fail(-14, "ldv < max(1, n)");
        if (batch > 1 && !empty && strideV < (long long)ldv * k) return fail(-15, "strideV < ldv * min(m, n)");
    }
    if (!isfinite(tol)) return fail(-16, "tol is not finite");
    if (!info && batch > 0) return fail(-17, "info is NULL");
    svdb_opts_t o = resolve_opts(opts);
    if (empty) {
        // no singular values: every matrix is trivially converged
        if (batch == 0) return 0;
        hipError_t e = svdb::launch_fill_int(info, batch, 0, (hipStream_t)stream);
        if (e == hipSuccess) e = svdb::launch_fill_int(o.sweeps, batch, 0, (hipStream_t)stream);
        return e == hipSuccess ? 0 : hip_fail(e, "launch");
    }
    const bool wide = n > m;
    Plan p;
    int rc = wide ? make_plan(dtype, n, m, o, &p) : make_plan(dtype, m, n, o, &p);
    if (rc) return rc;
    const size_t need = svdb_workspace_size(dtype, batch, m, n, &o);
    if (need > 0 && (!workspace || ws_bytes < need))
        return fail(-19, "workspace too small: need %zu bytes", need);
    if (batch == 0) return 0;
    if (tol <= 0.0) tol = default_tol(dtype);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (!wide) {
        e = run_tall(dtype, p, o, batch, m, n, A, lda, strideA, S, strideS, U, ldu, strideU, V,
                     ldv, strideV, tol, info, workspace, s);
    } else {
        // A^H = U' diag(S) V'^H (n x m, tall): U = V' and V = U'
        void *At = workspace;
        char *rest = (char *)workspace + wide_copy_bytes(dtype, batch, m, n);
        e = k ? svdb::launch_conj_transpose((int)dtype, batch, m, n, A, lda, strideA, At, s)
              : hipSuccess;
        if (e == hipSuccess)
            e = run_tall(dtype, p, o, batch, n, m, At, n, (long long)n * m, S, strideS, V, ldv,
                         strideV, U, ldu, strideU, tol, info, rest, s);
    }
    if (e != hipSuccess) return hip_fail(e, "launch");
    return 0;
}

}  // extern "C"

namespace {

// Scratch of svdb_svd_strided_batched_noalloc: a file-scope device array
// (one copy per device, alive until the process ends).  Its name is a
// host-side stand-in in host code: the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

hipError_t noalloc_scratch(int dev, void **out)
{
    static std::mutex mu;
    static std::map<int, void *> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) {
        const hipError_t r = hipSetDevice(cur);
        if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    addr.emplace(dev, ptr);
    *out = ptr;
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t svdb_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

int svdb_svd_strided_batched_noalloc(svdb_dtype_t dtype, int batch, int m, int n, const void *A,
                                     int lda, long long strideA, void *S, long long strideS,
                                     void *U, int ldu, long long strideU, void *V, int ldv,
                                     long long strideV, double tol, int *info,
                                     const svdb_opts_t *opts, void *stream)
{
    g_err.clear();
    if ((int)dtype < SVDB_R32 || (int)dtype > SVDB_C128) return fail(-1, "invalid dtype");
    if (batch < 0) return fail(-2, "batch < 0");
    if (m < 0) return fail(-3, "m < 0");
    if (n < 0) return fail(-4, "n < 0");
    const int k = m < n ? m : n;
    size_t need = 0;
    if (batch > 0 && k > 0) {
        // the block method waits on the host through pinned memory: only the
        // resident paths (with or without the QR pre-processing) qualify
        svdb_opts_t o = resolve_opts(opts);
        Plan p;
        const int rc = m >= n ? make_plan(dtype, m, n, o, &p) : make_plan(dtype, n, m, o, &p);
        if (rc) return rc;
        if (p.path == SVDB_PATH_BLOCKED)
            return fail(SVDB_ERR_UNSUPPORTED,
                        "noalloc: %d x %d plans the block method, which is not allocation-free",
                        m, n);
        need = svdb_workspace_size(dtype, batch, m, n, &o);
        if (need != (size_t)-1 && need > kNoallocScratchBytes)
            return fail(-2, "noalloc: batch %d of %d x %d needs %zu bytes of scratch, the "
                            "static maximum is %zu", batch, m, n, need, kNoallocScratchBytes);
    }
    void *ws = nullptr;
    if (need > 0 && need != (size_t)-1) {
        int dev = 0;
        hipError_t e = stream ? hipStreamGetDevice((hipStream_t)stream, &dev) : hipGetDevice(&dev);
        if (e == hipSuccess) e = noalloc_scratch(dev, &ws);
        if (e != hipSuccess) return hip_fail(e, "noalloc scratch");
    }
    return svdb_svd_strided_batched(dtype, batch, m, n, A, lda, strideA, S, strideS, U, ldu,
                                    strideU, V, ldv, strideV, tol, info, ws,
                                    ws ? kNoallocScratchBytes : 0, opts, stream);
}

size_t svdb_batched_workspace_size(svdb_dtype_t dtype, int batch, const int *m, const int *n,
                                   const svdb_opts_t *opts)
{
    if ((int)dtype < SVDB_R32 || (int)dtype > SVDB_C128) return (size_t)-1;
    if (batch < 0 || (batch > 0 && (!m || !n))) return (size_t)-1;
    svdb_opts_t o = resolve_opts(opts);
    if (o.precision != 0) return (size_t)-1;
    std::vector<int> mt(batch), nt(batch);   // wide matrices as their (tall) A^H
    for (int b = 0; b < batch; b++) {
        if (m[b] < 0 || n[b] < 0) return (size_t)-1;
        mt[b] = m[b] >= n[b] ? m[b] : n[b];
        nt[b] = m[b] >= n[b] ? n[b] : m[b];
    }
    return svdb::vbatched_workspace_bytes(batch, mt.data(), nt.data(), elt_bytes(dtype));
}

int svdb_svd_batched(svdb_dtype_t dtype, int batch, const int *m, const int *n,
                     const void *const *A, const int *lda, void *const *S, void *const *U,
                     const int *ldu, void *const *V, const int *ldv, double tol, int *info,
                     void *workspace, size_t ws_bytes, const svdb_opts_t *opts, void *stream)
{
    g_err.clear();
    if ((int)dtype < SVDB_R32 || (int)dtype > SVDB_C128) return fail(-1, "invalid dtype");
    if (batch < 0) return fail(-2, "batch < 0");
    if (batch == 0) return 0;
    if (!m) return fail(-3, "m is NULL");
    if (!n) return fail(-4, "n is NULL");
    if (!A) return fail(-5, "A is NULL");
    if (!lda) return fail(-6, "lda is NULL");
    if (!S) return fail(-7, "S is NULL");
    if (U && !ldu) return fail(-9, "ldu is NULL");
    if (V && !ldv) return fail(-11, "ldv is NULL");
    if (!isfinite(tol)) return fail(-12, "tol is not finite");
    if (!info) return fail(-13, "info is NULL");
    for (int b = 0; b < batch; b++) {
        if (m[b] < 0) return fail(-3, "m[%d] < 0", b);
        if (n[b] < 0) return fail(-4, "n[%d] < 0", b);
        const bool empty = n[b] == 0 || m[b] == 0;
        if (!A[b] && !empty) return fail(-5, "A[%d] is NULL", b);
        if (lda[b] < (m[b] > 1 ? m[b] : 1)) return fail(-6, "lda[%d] < max(1, m)", b);
        if (!S[b] && !empty) return fail(-7, "S[%d] is NULL", b);
        if (U && ldu[b] < (m[b] > 1 ? m[b] : 1)) return fail(-9, "ldu[%d] < max(1, m)", b);
        if (V && ldv[b] < (n[b] > 1 ? n[b] : 1)) return fail(-11, "ldv[%d] < max(1, n)", b);
        if (U && !U[b] && !empty) return fail(-8, "U[%d] is NULL", b);
        if (V && !V[b] && !empty) return fail(-10, "V[%d] is NULL", b);
    }
    svdb_opts_t o = resolve_opts(opts);
    if (o.precision != 0)
        return fail(SVDB_ERR_UNSUPPORTED, "uneven batches run in the working precision only");
    if (o.inner_tol_start > 0.0 && !(o.inner_tol_rate > 0.0 && o.inner_tol_rate < 1.0))
        return fail(SVDB_ERR_UNSUPPORTED, "dynamic inner tolerance: rate must be in (0, 1)");
    const size_t need = svdb_batched_workspace_size(dtype, batch, m, n, &o);
    if (!workspace || ws_bytes < need)
        return fail(-14, "workspace too small: need %zu bytes", need);
    if (tol <= 0.0) tol = default_tol(dtype);
    // a wide matrix (m < n) runs as its conjugate transpose, read transposed
    // by the init kernel, with U and V exchanged: A^H = U' S V'^H gives
    // U = V' and V = U'
    std::vector<int> mt(batch), nt(batch), tr(batch), ldut(batch), ldvt(batch);
    std::vector<void *> Ut(batch), Vt(batch);
    for (int b = 0; b < batch; b++) {
        void *ub = U ? U[b] : nullptr, *vb = V ? V[b] : nullptr;
        const int lu = U ? ldu[b] : 1, lv = V ? ldv[b] : 1;
        tr[b] = n[b] > m[b];
        mt[b] = tr[b] ? n[b] : m[b];
        nt[b] = tr[b] ? m[b] : n[b];
        Ut[b] = tr[b] ? vb : ub;
        ldut[b] = tr[b] ? lv : lu;
        Vt[b] = tr[b] ? ub : vb;
        ldvt[b] = tr[b] ? lu : lv;
    }
    hipError_t e = svdb::launch_vbatched((int)dtype, batch, mt.data(), nt.data(), A, lda, S,
                                         Ut.data(), ldut.data(), Vt.data(), ldvt.data(), tol,
                                         o.max_sweeps, o.masking, info, o.sweeps, workspace,
                                         (hipStream_t)stream, tr.data(), o.inner_sweeps,
                                         o.persistent, o.inner_tol_start, o.inner_tol_rate);
    if (e != hipSuccess) return hip_fail(e, "launch");
    return 0;
}

}  // extern "C"
