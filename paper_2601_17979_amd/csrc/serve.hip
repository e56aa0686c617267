// serve.hip -- the serving runtime behind svdb_server_* (include/svdb.h):
// continuous batching of independent SVD requests on one GPU.
//
// Requests arrive one at a time (any thread).  A worker thread owns the GPU
// stream and repeats rounds:
//   1. admit queued requests (first come, first served) while a slot is free
//      and the device arena (the HBM budget) holds the request's working
//      copies W (m x np) and V (np x np); initialise them;
//   2. run a few launches of the uneven-batch block kernels over every
//      admitted request: each request runs its own round-robin schedule from
//      the launch at which it was admitted (VbDesc::it0), so requests join
//      and leave between any two launches;
//   3. collect the requests that stopped sweeping (converged, or capped at
//      max_sweeps), finalise them into the caller's buffers, free their
//      slots and arena ranges, and report completion times.
// The paper's batches are static (its masks, section "Masked Batch
// Operations", retire converged matrices but keep the batch); retiring them
// and admitting new work in their place is what a serving workload needs.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "launchers.hpp"
#include "svdb.h"

namespace {

double now_seconds()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit range allocator over the device arena, with coalescing.
class Arena {
public:
    void reset(size_t bytes)
    {
        free_.clear();
        if (bytes) free_[0] = bytes;
        in_use_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        if (bytes == 0) {
            *off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                in_use_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        if (bytes == 0) return;
        in_use_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t in_use() const { return in_use_; }

private:
    std::map<size_t, size_t> free_;   // offset -> length
    size_t in_use_ = 0;
};

struct Request {
    long long id = 0;
    int dtype = 1, m = 0, n = 0, lda = 1, ldu = 1, ldv = 1;
    int group = 1;   // kernel group (dtype of the working copies)
    int pc = 0;      // QR-preconditioned: FP64 Jacobi on R^T, U = Q J
    int trans = 0;   // wide request run as A^H: m, n, U, V here are those of A^H
    const void *A = nullptr;
    void *S = nullptr, *U = nullptr, *V = nullptr;
    int *info = nullptr, *sweeps = nullptr;
    double tol = 0.0;
    size_t bytes = 0, off = 0;
    double t_submit = 0.0;
};

struct Completion {
    long long id;
    double t_submit, t_done;
};

int elt_of(int dtype) { return dtype == 0 ? 4 : dtype == 3 ? 16 : 8; }

constexpr int kWideChunk = 8;   // requests per blocked-QR launch of the wide QR lane

// Arena layout of a QR-preconditioned request (FP64, byte offsets from its
// range): the Jacobi's W (n x np) and V (np x np), X = R^T, the reflectors
// (m x n), tau, J, and for FP32 requests the FP64 staging of S and V.
struct PcLayout {
    size_t w, v, x, q, tau, j, s64, vx64, bytes;
};

PcLayout pc_layout(int m, int n, int np, bool f32)
{
    PcLayout L{};
    size_t o = 0;
    L.w = o;
    o += al256((size_t)n * np * 8);
    L.v = o;
    o += al256((size_t)np * np * 8);
    L.x = o;
    o += al256((size_t)n * n * 8);
    L.q = o;
    o += al256((size_t)m * n * 8);
    L.tau = o;
    o += al256((size_t)n * 8);
    L.j = o;
    o += al256((size_t)n * n * 8);
    L.s64 = o;
    o += f32 ? al256((size_t)n * 8) : 0;
    L.vx64 = o;
    o += f32 ? al256((size_t)n * n * 8) : 0;
    L.bytes = o;
    return L;
}

// One dtype: the kernels are compiled per element type.
struct Group {
    int dtype = 1;
    int cap = 0;
    svdb::VbDesc *d_desc = nullptr, *h_desc = nullptr;
    void *d_st = nullptr;
    int *d_flags = nullptr, *h_flags = nullptr;
    int2 *d_work = nullptr, *h_work = nullptr;
    // slot lists of the init and the finalize launches: two host buffers, so
    // that a round's init list is never written while the previous round's
    // finalize list may still be in flight to the device
    int *d_idx = nullptr, *h_idx = nullptr, *h_fin = nullptr;
    svdb::QrJob *d_jobs = nullptr, *h_jobs = nullptr;   // QR preconditioning (FP64 group)
    std::vector<Request> slot;
    std::vector<char> used;
    // QR-preconditioned slots: 0 in the launches (or not preconditioned),
    // 1 waiting for or in the QR, 2 waiting for or in the application of Q
    std::vector<char> stage;
    // work on the auxiliary streams: at most one batch in flight per lane, the
    // requests that arrive meanwhile wait and form the next batch, so batches
    // grow with the load
    struct Lane {
        std::vector<int> wait;   // slots waiting for the lane
        std::vector<int> cur;    // the batch in flight
        hipEvent_t ev = nullptr;
        int pos = 0;             // its slot list in the device ring
        bool busy = false;
    };
    Lane lane[3];   // QR of requests with n <= 64, QR of wider ones, application of Q
    int *d_ring = nullptr, *h_ring = nullptr;
    int ring_len = 0, ring_head = 0;
    std::vector<int> fresh;   // slots admitted this round
    int nused = 0, nwork = 0, lmax = 2, maxn = 0;
    bool dirty = false;
    int max_pairs = 0;        // work-table entries per slot
    double tol = 0.0;
};

}  // namespace

struct svdb_server {
    hipStream_t stream = nullptr;
    hipStream_t aux[3] = {};       // the lanes of preconditioned requests
    hipEvent_t ev_fin = nullptr;   // end of the finalisations of a round
    // the worker's waits for its own stream: a blocking-sync event, so that
    // the worker sleeps in the driver instead of spinning on a host core
    hipEvent_t ev_wait = nullptr;
    void *arena = nullptr;
    // the wide QR lane: up to kWideChunk same-shape requests are gathered
    // into H, factored by one blocked-QR launch, and scattered back
    double *qrb_h = nullptr, *qrb_x = nullptr, *qrb_tau = nullptr;
    void *qrb_ws = nullptr;
    size_t budget = 0;
    Arena alloc;
    Group g[4];
    int max_sweeps = 100;
    int max_n = 512;
    int precondition = 1;
    int inner = 0;   // inner sweeps per block-pair solve (svdb_opts_t.inner_sweeps)
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::deque<Completion> done;
    std::thread worker;
    bool stop = false;
    int failed = 0;
    std::string err;
    long long next_id = 0, submitted = 0, completed = 0;
    int itg = 0;
};

namespace {

#define SRV_CHECK(expr)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            std::lock_guard<std::mutex> lk(s->mu);                                       \
            s->failed = 1;                                                               \
            s->err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
            s->cv_done.notify_all();                                                     \
            return;                                                                      \
        }                                                                                \
    } while (0)

void rebuild_work(Group &G)
{
    // largest matrices first; only slots still sweeping
    std::vector<int> order;
    for (int b = 0; b < G.cap; b++)
        if (G.used[b] && G.stage[b] == 0) order.push_back(b);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return G.slot[x].n > G.slot[y].n; });
    int w = 0, lmax = 2, maxn = 0;
    for (int b : order) {
        const svdb::VbDesc &D = G.h_desc[b];
        for (int q = 0; G.slot[b].n > 0 && q < D.l / 2; q++) G.h_work[w++] = make_int2(b, q);
        lmax = D.l > lmax ? D.l : lmax;
        maxn = D.n > maxn ? D.n : maxn;
    }
    G.nwork = w;
    G.lmax = lmax;
    G.maxn = maxn;
}

// Descriptor (and, when preconditioned, QR job) of a request admitted into
// slot b of group G.
void describe(svdb_server *s, Group &G, int b)
{
    const int nb = svdb::vb_nb();
    const size_t elt = (size_t)elt_of(G.dtype);
    char *base = (char *)s->arena;
    const Request &r = G.slot[b];
    svdb::VbDesc D{};
    D.info = r.info;
    D.sweeps = r.sweeps;
    D.n = r.n;
    D.np = r.n > 0 ? svdb::blocked_np(r.n, nb) : 0;
    D.l = r.n > 0 ? D.np / nb : 2;
    D.it0 = s->itg;
    if (r.pc) {
        // the Jacobi runs on X = R^T (n x n); its U is our V, its V is J
        const bool f32 = r.dtype == SVDB_R32;
        const PcLayout P = pc_layout(r.m, r.n, D.np, f32);
        D.A = base + r.off + P.x;
        D.lda = r.n;
        D.m = r.n;
        D.S = f32 ? (void *)(base + r.off + P.s64) : r.S;
        D.U = r.V ? (f32 ? (void *)(base + r.off + P.vx64) : r.V) : nullptr;
        D.ldu = f32 ? r.n : r.ldv;
        D.V = r.U ? (void *)(base + r.off + P.j) : nullptr;
        D.ldv = r.n;
        D.woff = (long long)((r.off + P.w) / 8);
        D.voff = (long long)((r.off + P.v) / 8);
        svdb::QrJob J{};
        J.A = r.A;
        J.lda = r.lda;
        J.m = r.m;
        J.n = r.n;
        J.f32 = f32;
        J.Vq = (double *)(base + r.off + P.q);
        J.X = (double *)(base + r.off + P.x);
        J.tau = (double *)(base + r.off + P.tau);
        J.Y = (const double *)(base + r.off + P.j);
        J.U = r.U;
        J.ldu = r.ldu;
        J.uf32 = f32;
        J.S64 = (const double *)(base + r.off + P.s64);
        J.Vx64 = (const double *)(base + r.off + P.vx64);
        J.Sout = r.S;
        J.Vout = r.V;
        J.ldv = r.ldv;
        J.info = r.info;
        G.h_jobs[b] = J;
    } else {
        D.A = r.A;
        D.trans = r.trans;
        D.S = r.S;
        D.U = r.U;
        D.V = r.V;
        D.m = r.m;
        D.lda = r.lda;
        D.ldu = r.ldu;
        D.ldv = r.ldv;
        D.woff = (long long)(r.off / elt);
        D.voff = D.woff + (long long)D.m * D.np;
    }
    G.h_desc[b] = D;
}

// Copies the lane's waiting slots into the device ring (on `st`) as its
// new batch; first waits for any batch in flight whose list would be
// overwritten.
hipError_t lane_stage(Group &G, Group::Lane &L, hipStream_t st)
{
    const int n = (int)L.wait.size();
    if (G.ring_head + n > G.ring_len) G.ring_head = 0;
    const int lo = G.ring_head, hi = G.ring_head + n;
    for (auto &O : G.lane)
        if (O.busy && O.pos < hi && lo < O.pos + (int)O.cur.size()) {
            const hipError_t e = hipEventSynchronize(O.ev);
            if (e != hipSuccess) return e;
        }
    for (int k = 0; k < n; k++) G.h_ring[lo + k] = L.wait[k];
    G.ring_head = hi;
    L.pos = lo;
    L.cur.swap(L.wait);
    L.wait.clear();
    if (!L.ev) {
        const hipError_t e = hipEventCreateWithFlags(&L.ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    return hipMemcpyAsync(G.d_ring + lo, G.h_ring + lo, (size_t)n * sizeof(int),
                          hipMemcpyHostToDevice, st);
}

// hipSuccess with *done set once the lane's batch has finished
hipError_t lane_done(Group::Lane &L, bool *done)
{
    *done = false;
    if (!L.busy) return hipSuccess;
    const hipError_t q = hipEventQuery(L.ev);
    if (q == hipErrorNotReady) return hipSuccess;
    if (q != hipSuccess) return q;
    L.busy = false;
    *done = true;
    return hipSuccess;
}

// QR of the wide lane's requests: same-shape requests, kWideChunk at a time,
// are gathered (FP32 widened) into the staging H, factored by one launch of
// the blocked QR, and their reflectors, X = R^T and tau copied to the
// request's arena range, where the Jacobi and the application of Q expect
// them.
hipError_t wide_qr(svdb_server *s, Group &G, const std::vector<int> &cur, hipStream_t st)
{
    std::vector<int> todo(cur);
    while (!todo.empty()) {
        const svdb::QrJob &J0 = G.h_jobs[todo[0]];
        const int m = J0.m, n = J0.n;
        std::vector<int> chunk, rest;
        for (int b : todo) {
            const svdb::QrJob &J = G.h_jobs[b];
            if (J.m == m && J.n == n && (int)chunk.size() < kWideChunk)
                chunk.push_back(b);
            else
                rest.push_back(b);
        }
        const size_t mn = (size_t)m * n, nn = (size_t)n * n;
        hipError_t e = hipSuccess;
        for (size_t k = 0; k < chunk.size() && e == hipSuccess; k++) {
            const svdb::QrJob &J = G.h_jobs[chunk[k]];
            double *h = s->qrb_h + k * mn;
            if (J.f32)
                e = svdb::launch_widen_f32(1, m, n, (const float *)J.A, J.lda, 0, h, m, 0, st);
            else
                e = hipMemcpy2DAsync(h, (size_t)m * 8, J.A, (size_t)J.lda * 8, (size_t)m * 8, n,
                                     hipMemcpyDeviceToDevice, st);
        }
        if (e == hipSuccess)
            e = svdb::launch_qr_blocked_batch((int)chunk.size(), m, n, s->qrb_h, m,
                                              (long long)mn, s->qrb_h, s->qrb_x, s->qrb_tau,
                                              s->qrb_ws, st);
        for (size_t k = 0; k < chunk.size() && e == hipSuccess; k++) {
            const svdb::QrJob &J = G.h_jobs[chunk[k]];
            e = hipMemcpyAsync(J.Vq, s->qrb_h + k * mn, mn * 8, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(J.X, s->qrb_x + k * nn, nn * 8, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(J.tau, s->qrb_tau + k * n, (size_t)n * 8,
                                   hipMemcpyDeviceToDevice, st);
        }
        if (e != hipSuccess) return e;
        todo.swap(rest);
    }
    return hipSuccess;
}

// Waits until the worker's stream has finished the work enqueued so far.
hipError_t wait_stream(svdb_server *s)
{
    const hipError_t e = hipEventRecord(s->ev_wait, s->stream);
    return e == hipSuccess ? hipEventSynchronize(s->ev_wait) : e;
}

void worker_main(svdb_server *s)
{
    std::vector<int> init;   // slots to initialise this round
    for (;;) {
        // ---- 1. admission ----------------------------------------------------
        {
            std::unique_lock<std::mutex> lk(s->mu);
            auto active = [&] {
                for (auto &G : s->g)
                    if (G.nused) return true;
                return false;
            };
            s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || active(); });
            if (s->stop && s->queue.empty() && !active()) return;
            while (!s->queue.empty()) {
                Request &r = s->queue.front();
                Group &G = s->g[r.group];
                int b = -1;
                for (int k = 0; k < G.cap; k++)
                    if (!G.used[k]) {
                        b = k;
                        break;
                    }
                size_t off = 0;
                if (b < 0 || !s->alloc.alloc(r.bytes, &off)) break;   // wait for retirements
                r.off = off;
                G.slot[b] = r;
                G.used[b] = 1;
                G.stage[b] = r.pc ? 1 : 0;
                G.nused++;
                G.fresh.push_back(b);
                s->queue.pop_front();
            }
        }
        // ---- preconditioned requests go to a QR lane; the others are
        // initialised below, with those whose QR has finished ------------------
        for (auto &G : s->g) {
            init.clear();
            for (int b : G.fresh) {
                describe(s, G, b);
                if (!G.slot[b].pc) {
                    init.push_back(b);
                    continue;
                }
                const int q = G.slot[b].n <= 64 ? 0 : 1;
                SRV_CHECK(hipMemcpyAsync(G.d_jobs + b, G.h_jobs + b, sizeof(svdb::QrJob),
                                         hipMemcpyHostToDevice, s->aux[q]));
                G.lane[q].wait.push_back(b);
            }
            G.fresh.clear();
            for (int q = 0; q < 2; q++) {
                Group::Lane &L = G.lane[q];
                bool done;
                SRV_CHECK(lane_done(L, &done));
                if (done)
                    for (int b : L.cur) {
                        G.stage[b] = 0;
                        G.h_desc[b].it0 = s->itg;
                        init.push_back(b);
                    }
                if (!L.busy && !L.wait.empty()) {
                    SRV_CHECK(lane_stage(G, L, s->aux[q]));
                    if (q == 0) {   // n <= 64: one workgroup per request
                        svdb::launch_qr_jobs(G.d_jobs, G.d_ring + L.pos, (int)L.cur.size(),
                                             s->aux[q]);
                        SRV_CHECK(hipGetLastError());
                    } else {        // wider: the blocked QR, same shapes batched
                        SRV_CHECK(wide_qr(s, G, L.cur, s->aux[q]));
                    }
                    SRV_CHECK(hipEventRecord(L.ev, s->aux[q]));
                    L.busy = true;
                }
            }
            if (init.empty()) continue;
            int lo = G.cap, hi = -1;
            for (size_t k = 0; k < init.size(); k++) {
                G.h_idx[k] = init[k];
                lo = init[k] < lo ? init[k] : lo;
                hi = init[k] > hi ? init[k] : hi;
            }
            SRV_CHECK(hipMemcpyAsync(G.d_desc + lo, G.h_desc + lo,
                                     (size_t)(hi - lo + 1) * sizeof(svdb::VbDesc),
                                     hipMemcpyHostToDevice, s->stream));
            SRV_CHECK(hipMemcpyAsync(G.d_idx, G.h_idx, init.size() * sizeof(int),
                                     hipMemcpyHostToDevice, s->stream));
            svdb::vb_launch_init(G.dtype, G.d_desc, G.d_idx, (int)init.size(), s->arena, G.d_st,
                                 s->stream);
            SRV_CHECK(hipGetLastError());
            G.dirty = true;
        }
        // ---- 2. a few launches over every request in the launches ----------------
        int K = 0;
        for (auto &G : s->g) {
            if (!G.nused) continue;
            if (G.dirty) {
                rebuild_work(G);
                if (G.nwork)
                    SRV_CHECK(hipMemcpyAsync(G.d_work, G.h_work, (size_t)G.nwork * sizeof(int2),
                                             hipMemcpyHostToDevice, s->stream));
                G.dirty = false;
            }
            if (G.nwork) K = G.lmax - 1 > K ? G.lmax - 1 : K;
        }
        K = K < 8 ? K : 8;
        for (int k = 0; k < K; k++, s->itg++)
            for (auto &G : s->g) {
                if (!G.nused) continue;
                if (G.nwork)
                    svdb::vb_launch_iter(G.dtype, G.d_desc, G.d_work, G.nwork, s->itg, s->arena,
                                         G.d_st, G.tol, s->stream, s->inner);
                svdb::vb_launch_sweep_end(G.cap, G.d_desc, s->itg, G.d_st, s->max_sweeps, 1,
                                          nullptr, s->stream);
            }
        SRV_CHECK(hipGetLastError());
        // ---- 3. retire what stopped ---------------------------------------------------
        for (auto &G : s->g) {
            if (!G.nused) continue;
            svdb::vb_launch_collect(G.cap, G.d_st, G.d_flags, s->stream);
            SRV_CHECK(hipMemcpyAsync(G.h_flags, G.d_flags, (size_t)G.cap * sizeof(int),
                                     hipMemcpyDeviceToHost, s->stream));
        }
        SRV_CHECK(wait_stream(s));
        std::vector<std::pair<int, int>> retired;   // (group, slot) complete now
        bool any_pc = false;
        for (int gi = 0; gi < 4; gi++) {
            Group &G = s->g[gi];
            if (!G.nused) continue;
            int cnt = 0, maxn = 0;
            for (int b = 0; b < G.cap; b++)
                if (G.used[b] && G.stage[b] == 0 && G.h_flags[b]) {
                    G.h_fin[cnt++] = b;
                    maxn = G.slot[b].n > maxn ? G.slot[b].n : maxn;
                    if (G.slot[b].pc)
                        any_pc = true;
                    else
                        retired.push_back({gi, b});
                }
            if (!cnt) continue;
            SRV_CHECK(hipMemcpyAsync(G.d_idx, G.h_fin, (size_t)cnt * sizeof(int),
                                     hipMemcpyHostToDevice, s->stream));
            svdb::vb_launch_finalize(G.dtype, G.d_desc, G.d_idx, cnt, maxn, s->arena, G.d_st,
                                     s->stream);
            SRV_CHECK(hipGetLastError());
        }
        // preconditioned requests: U = Q J (and the FP32 outputs) on the third
        // lane, after the finalisations issued so far
        bool fin_recorded = false;
        for (int gi = 0; gi < 4; gi++) {
            Group &G = s->g[gi];
            Group::Lane &L = G.lane[2];
            if (any_pc)
                for (int b = 0; b < G.cap; b++)
                    if (G.used[b] && G.stage[b] == 0 && G.h_flags[b] && G.slot[b].pc) {
                        G.stage[b] = 2;
                        G.dirty = true;
                        L.wait.push_back(b);
                    }
            bool done;
            SRV_CHECK(lane_done(L, &done));
            if (done)
                for (int b : L.cur) retired.push_back({gi, b});
            if (L.busy || L.wait.empty()) continue;
            if (!fin_recorded) {
                SRV_CHECK(hipEventRecord(s->ev_fin, s->stream));
                SRV_CHECK(hipStreamWaitEvent(s->aux[2], s->ev_fin, 0));
                fin_recorded = true;
            }
            int maxm = 0;
            for (int b : L.wait) maxm = G.slot[b].m > maxm ? G.slot[b].m : maxm;
            SRV_CHECK(lane_stage(G, L, s->aux[2]));
            svdb::launch_apply_q_jobs(G.d_jobs, G.d_ring + L.pos, (int)L.cur.size(), maxm,
                                      s->aux[2]);
            SRV_CHECK(hipGetLastError());
            SRV_CHECK(hipEventRecord(L.ev, s->aux[2]));
            L.busy = true;
        }
        if (!retired.empty()) {
            SRV_CHECK(wait_stream(s));
            const double t = now_seconds();
            {
                std::lock_guard<std::mutex> lk(s->mu);
                for (auto &gb : retired) {
                    Group &G = s->g[gb.first];
                    Request &r = G.slot[gb.second];
                    s->done.push_back({r.id, r.t_submit, t});
                    s->alloc.release(r.off, r.bytes);
                    G.used[gb.second] = 0;
                    G.stage[gb.second] = 0;
                    G.nused--;
                    G.dirty = true;
                    s->completed++;
                }
            }
            s->cv_done.notify_all();
        }
        if (K == 0 && retired.empty()) {
            // every admitted request is in a QR lane: wait briefly, or less
            // when a new request arrives
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait_for(lk, std::chrono::microseconds(200),
                                [&] { return s->stop || !s->queue.empty(); });
        }
    }
}

void destroy_resources(svdb_server *s)
{
    for (auto &G : s->g) {
        if (G.d_desc) (void)hipFree(G.d_desc);
        if (G.d_st) (void)hipFree(G.d_st);
        if (G.d_flags) (void)hipFree(G.d_flags);
        if (G.d_work) (void)hipFree(G.d_work);
        if (G.d_idx) (void)hipFree(G.d_idx);
        if (G.h_desc) (void)hipHostFree(G.h_desc);
        if (G.h_flags) (void)hipHostFree(G.h_flags);
        if (G.h_work) (void)hipHostFree(G.h_work);
        if (G.h_idx) (void)hipHostFree(G.h_idx);
        if (G.h_fin) (void)hipHostFree(G.h_fin);
        if (G.d_jobs) (void)hipFree(G.d_jobs);
        if (G.h_jobs) (void)hipHostFree(G.h_jobs);
        for (auto &L : G.lane)
            if (L.ev) (void)hipEventDestroy(L.ev);
        if (G.d_ring) (void)hipFree(G.d_ring);
        if (G.h_ring) (void)hipHostFree(G.h_ring);
    }
    if (s->arena) (void)hipFree(s->arena);
    for (void *p : {(void *)s->qrb_h, (void *)s->qrb_x, (void *)s->qrb_tau, s->qrb_ws})
        if (p) (void)hipFree(p);
    if (s->ev_fin) (void)hipEventDestroy(s->ev_fin);
    if (s->ev_wait) (void)hipEventDestroy(s->ev_wait);
    for (hipStream_t a : s->aux)
        if (a) (void)hipStreamDestroy(a);
    if (s->stream) (void)hipStreamDestroy(s->stream);
}

}  // namespace

extern "C" {

double svdb_server_clock(void) { return now_seconds(); }

int svdb_server_create(svdb_server_t **out, size_t budget_bytes, int max_requests,
                       const svdb_opts_t *opts)
{
    if (!out) return -1;
    *out = nullptr;
    if (budget_bytes == 0) return -2;
    if (max_requests <= 0) return -3;
    svdb_opts_t o;
    svdb_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision != 0) return SVDB_ERR_UNSUPPORTED;
    if (o.precondition < -1 || o.precondition > 1) return SVDB_ERR_UNSUPPORTED;
    svdb_server *s = new svdb_server();
    s->budget = al256(budget_bytes);
    s->max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 100;
    s->precondition = o.precondition != 0;   // -1 (default) and 1: on
    s->inner = o.inner_sweeps < -1 ? -1 : o.inner_sweeps;
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    for (hipStream_t &a : s->aux)
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_fin, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&s->ev_wait, hipEventDisableTiming | hipEventBlockingSync);
    if (e == hipSuccess) e = hipMalloc(&s->arena, s->budget);
    if (s->precondition) {
        const size_t mn = (size_t)kWideChunk * 1024 * s->max_n,
                     nn = (size_t)kWideChunk * s->max_n * s->max_n;
        if (e == hipSuccess) e = hipMalloc((void **)&s->qrb_h, mn * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void **)&s->qrb_x, nn * sizeof(double));
        if (e == hipSuccess)
            e = hipMalloc((void **)&s->qrb_tau, (size_t)kWideChunk * s->max_n * sizeof(double));
        if (e == hipSuccess)
            e = hipMalloc(&s->qrb_ws, svdb::qr_blocked_scratch_bytes(kWideChunk, 1024, s->max_n));
    }
    const int pairs = s->max_n / svdb::vb_nb() / 2;   // block pairs of the widest request
    for (int gi = 0; gi < 4 && e == hipSuccess; gi++) {
        Group &G = s->g[gi];
        G.dtype = gi;
        G.cap = max_requests;
        G.max_pairs = pairs;
        G.tol = 30.0 * ldexp(1.0, (gi == 0 || gi == 2) ? -24 : -53);
        G.slot.assign(G.cap, Request());
        G.used.assign(G.cap, 0);
        G.stage.assign(G.cap, 0);
        G.ring_len = 4 * G.cap;
        if (e == hipSuccess) e = hipMalloc((void **)&G.d_ring, (size_t)G.ring_len * sizeof(int));
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&G.h_ring, (size_t)G.ring_len * sizeof(int), 0);
        const size_t nc = (size_t)G.cap;
        if (e == hipSuccess) e = hipMalloc((void **)&G.d_desc, nc * sizeof(svdb::VbDesc));
        if (e == hipSuccess) e = hipMalloc(&G.d_st, nc * svdb::vb_state_bytes());
        if (e == hipSuccess) e = hipMalloc((void **)&G.d_flags, nc * sizeof(int));
        if (e == hipSuccess) e = hipMalloc((void **)&G.d_work, nc * pairs * sizeof(int2));
        if (e == hipSuccess) e = hipMalloc((void **)&G.d_idx, nc * sizeof(int));
        if (e == hipSuccess) e = hipHostMalloc((void **)&G.h_desc, nc * sizeof(svdb::VbDesc), 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&G.h_flags, nc * sizeof(int), 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&G.h_work, nc * pairs * sizeof(int2), 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&G.h_idx, nc * sizeof(int), 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&G.h_fin, nc * sizeof(int), 0);
        if (e == hipSuccess) e = hipMalloc((void **)&G.d_jobs, nc * sizeof(svdb::QrJob));
        if (e == hipSuccess) e = hipHostMalloc((void **)&G.h_jobs, nc * sizeof(svdb::QrJob), 0);
        if (e == hipSuccess) svdb::vb_launch_mark_empty(G.cap, G.d_st, s->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        destroy_resources(s);
        delete s;
        return SVDB_ERR_HIP;
    }
    s->alloc.reset(s->budget);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return 0;
}

long long svdb_server_submit(svdb_server_t *s, svdb_dtype_t dtype, int m, int n, const void *A,
                             int lda, void *S, void *U, int ldu, void *V, int ldv, double tol,
                             int *info, int *sweeps)
{
    if (!s) return -1;
    if ((int)dtype < SVDB_R32 || (int)dtype > SVDB_C128) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    const int k = m < n ? m : n;
    if (k > s->max_n) return SVDB_ERR_UNSUPPORTED;
    if (!A && k > 0) return -5;
    if (lda < (m > 1 ? m : 1)) return -6;
    if (!S && k > 0) return -7;
    if (U && ldu < (m > 1 ? m : 1)) return -9;
    if (V && ldv < (n > 1 ? n : 1)) return -11;
    if (!info) return -13;
    Request r;
    r.dtype = (int)dtype;
    r.A = A;
    r.lda = lda;
    r.S = S;
    r.info = info;
    r.sweeps = sweeps;
    // a wide request runs as A^H = V S U^H: read transposed, U and V exchanged
    r.trans = n > m;
    r.m = r.trans ? n : m;
    r.n = k;
    void *u = U, *v = V;
    const int lu = U ? ldu : 1, lv = V ? ldv : 1;
    r.U = r.trans ? v : u;
    r.ldu = r.trans ? lv : lu;
    r.V = r.trans ? u : v;
    r.ldv = r.trans ? lu : lv;
    m = r.m;
    n = r.n;
    const int np = n > 0 ? svdb::blocked_np(n, svdb::vb_nb()) : 0;
    r.pc = s->precondition && !r.trans && (dtype == SVDB_R32 || dtype == SVDB_R64) && n > 0 &&
           m <= 1024;
    r.group = r.pc ? SVDB_R64 : r.dtype;
    r.bytes = r.pc ? pc_layout(m, n, np, dtype == SVDB_R32).bytes
                   : al256(((size_t)m * np + (size_t)np * np) * (size_t)elt_of(r.dtype));
    if (r.bytes > s->budget) return SVDB_ERR_UNSUPPORTED;
    (void)tol;   // per-dtype default threshold (30 u)
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed) return SVDB_ERR_HIP;
    r.id = s->next_id++;
    r.t_submit = now_seconds();
    s->queue.push_back(r);
    s->submitted++;
    s->cv_work.notify_one();
    return r.id;
}

int svdb_server_poll(svdb_server_t *s, long long *ids, double *t_submit, double *t_done, int cap,
                     int timeout_ms)
{
    if (!s || cap < 0) return -1;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_ms != 0 && !s->failed) {
        auto pred = [&] { return !s->done.empty() || s->failed; };
        if (timeout_ms < 0)
            s->cv_done.wait(lk, pred);
        else
            s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
    }
    if (s->failed && s->done.empty()) return SVDB_ERR_HIP;
    int k = 0;
    while (k < cap && !s->done.empty()) {
        const Completion c = s->done.front();
        s->done.pop_front();
        if (ids) ids[k] = c.id;
        if (t_submit) t_submit[k] = c.t_submit;
        if (t_done) t_done[k] = c.t_done;
        k++;
    }
    return k;
}

int svdb_server_stats(svdb_server_t *s, long long *submitted, long long *completed, int *active,
                      int *queued, size_t *bytes_in_use)
{
    if (!s) return -1;
    std::lock_guard<std::mutex> lk(s->mu);
    int a = 0;
    for (auto &G : s->g) a += G.nused;
    if (submitted) *submitted = s->submitted;
    if (completed) *completed = s->completed;
    if (active) *active = a;
    if (queued) *queued = (int)s->queue.size();
    if (bytes_in_use) *bytes_in_use = s->alloc.in_use();
    return s->failed ? SVDB_ERR_HIP : 0;
}

const char *svdb_server_error(svdb_server_t *s)
{
    if (!s) return "";
    std::lock_guard<std::mutex> lk(s->mu);
    return s->err.c_str();
}

int svdb_server_destroy(svdb_server_t *s)
{
    if (!s) return -1;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    for (hipStream_t a : s->aux) (void)hipStreamSynchronize(a);
    destroy_resources(s);
    delete s;
    return 0;
}

}  // extern "C"
