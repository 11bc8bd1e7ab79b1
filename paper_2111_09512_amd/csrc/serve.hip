// Serving runtime: continuous batching of smoother requests on resident
// matrices (the serving form of the scaled-ILU smoother).
//
// Each request is the op sequence of `outer` smoothing steps of eq.
// ILUsplit / Algorithm 2: a residual sweep on A, m_L - 1 sweeps on Ls (the
// last fused with D^{-1}), m_U - 1 sweeps on U~s (the last fused with the
// update of x).  A step admits queued requests in arrival order while their
// workspace fits in the caller's arena, then launches ONE batched kernel that
// advances every active request by one op, whatever op each is at.  A
// request's workspace returns to the arena once the GPU has passed its last
// launch.  Each row is summed by one lane in a fixed order, so a request's
// result does not depend on which requests shared its launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "../../include/scaled_ilu.h"
#include "internal.h"

using namespace silu;

namespace {

constexpr int RING = 4;        // op-table staging slots = steps in flight
constexpr int SERVE_RPB = 256; // rows per workgroup of the batched sweep

struct Matrix {
    silu_csr A;
    silu_factors F;
};

struct Range {
    size_t off, bytes;
};

struct Request {
    int64_t ticket;
    int mid;
    const double *b;
    double *x;
    int outer, mL, mU;
    int op = 0, total = 0;
    Range ws{0, 0};
};

size_t vec_bytes(int64_t n) { return (((size_t)n * 8 + 255) / 256) * 256; }

} // namespace

struct silu_server {
    silu_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int max_active = 0;
    std::vector<Matrix> mats;
    std::deque<Request> queue;
    std::vector<Request> active;
    std::vector<Range> free_list;                      // sorted by offset, coalesced
    std::vector<std::pair<int64_t, Range>> to_release; // (step, range)
    std::map<int64_t, int64_t> finish_step;            // ticket -> step of its last op
    int64_t next_ticket = 0, steps = 0, completed_through = -1;
    hipEvent_t ev[RING] = {};
    SweepArgs *h_ops[RING] = {};
    int32_t *h_first[RING] = {};
    SweepArgs *d_ops = nullptr;
    int32_t *d_first = nullptr;
    int cap = 0; // op-table capacity
    hipError_t last = hipSuccess;
};

namespace {

int fail(silu_server *s, hipError_t e)
{
    s->last = e;
    return SILU_ERR_HIP;
}

void release(silu_server *s, Range r)
{
    auto &fl = s->free_list;
    auto it = std::lower_bound(fl.begin(), fl.end(), r, [](const Range &a, const Range &b) { return a.off < b.off; });
    it = fl.insert(it, r);
    size_t i = (size_t)(it - fl.begin());
    if (i + 1 < fl.size() && fl[i].off + fl[i].bytes == fl[i + 1].off) {
        fl[i].bytes += fl[i + 1].bytes;
        fl.erase(fl.begin() + (long)i + 1);
    }
    if (i > 0 && fl[i - 1].off + fl[i - 1].bytes == fl[i].off) {
        fl[i - 1].bytes += fl[i].bytes;
        fl.erase(fl.begin() + (long)i);
    }
}

bool allocate(silu_server *s, size_t bytes, Range *out)
{
    for (size_t i = 0; i < s->free_list.size(); i++) {
        Range &f = s->free_list[i];
        if (f.bytes >= bytes) {
            *out = {f.off, bytes};
            f.off += bytes;
            f.bytes -= bytes;
            if (f.bytes == 0) s->free_list.erase(s->free_list.begin() + (long)i);
            return true;
        }
    }
    return false;
}

// Steps whose event has completed: reclaim the workspace they held.
void reap(silu_server *s)
{
    for (int64_t k = s->completed_through + 1; k < s->steps; k++) {
        if (hipEventQuery(s->ev[k % RING]) != hipSuccess) break;
        s->completed_through = k;
    }
    auto &tr = s->to_release;
    size_t w = 0;
    for (size_t i = 0; i < tr.size(); i++) {
        if (tr[i].first <= s->completed_through)
            release(s, tr[i].second);
        else
            tr[w++] = tr[i];
    }
    tr.resize(w);
}

// The op request q runs at its current position.
SweepArgs op_of(const silu_server *s, const Request &q)
{
    const Matrix &M = s->mats[(size_t)q.mid];
    const int64_t n = M.A.n_rows;
    const size_t vb = vec_bytes(n);
    char *w = s->arena + q.ws.off;
    double *r = (double *)w, *sv = (double *)(w + vb), *tmp[2] = {(double *)(w + 2 * vb), (double *)(w + 3 * vb)};
    const int per = 1 + (q.mL - 1) + (q.mU - 1);
    const int j = q.op % per;
    SweepArgs a;
    a.n = (int)n;
    a.dinv = M.F.dinv;
    a.x = q.x;
    a.dshift = nullptr;
    a.dcol = M.F.scaled == 2 ? M.F.dc : nullptr; // read by the update epilogues only
    a.out = nullptr;
    if (j == 0) { // residual
        a.rp = M.A.row_ptr;
        a.col = M.A.col_idx;
        a.val = M.A.val;
        a.xin = q.x;
        a.rhs = q.b;
        if (q.mL >= 2) {
            a.epi = EPI_STORE;
            a.out = r;
        } else {
            a.epi = EPI_SCALE;
            a.out = sv;
        }
    } else if (j < q.mL) { // L sweep k = j + 1
        const int k = j + 1;
        a.rp = M.F.Ls.row_ptr;
        a.col = M.F.Ls.col_idx;
        a.val = M.F.Ls.val;
        a.xin = k == 2 ? (const void *)r : (const void *)tmp[(k - 1) & 1];
        a.rhs = r;
        if (k < q.mL) {
            a.epi = EPI_STORE;
            a.out = tmp[k & 1];
        } else if (q.mU >= 2) {
            a.epi = EPI_SCALE;
            a.out = sv;
        } else {
            a.epi = EPI_SCALE_UPDATE;
        }
    } else { // U sweep k
        const int k = j - q.mL + 2;
        a.rp = M.F.Us.row_ptr;
        a.col = M.F.Us.col_idx;
        a.val = M.F.Us.val;
        a.xin = k == 2 ? (const void *)sv : (const void *)tmp[(k - 1) & 1];
        a.rhs = sv;
        if (k < q.mU) {
            a.epi = EPI_STORE;
            a.out = tmp[k & 1];
        } else {
            a.epi = EPI_UPDATE;
        }
    }
    return a;
}

int grow(silu_server *s, int need)
{
    if (need <= s->cap) return SILU_OK;
    // idle the ring before reallocating the staging and device tables
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(s, e);
    int cap = std::max(need, std::max(64, 2 * s->cap));
    for (int i = 0; i < RING; i++) {
        (void)hipHostFree(s->h_ops[i]);
        (void)hipHostFree(s->h_first[i]);
        s->h_ops[i] = nullptr;
        s->h_first[i] = nullptr;
    }
    (void)hipFree(s->d_ops);
    (void)hipFree(s->d_first);
    s->d_ops = nullptr;
    s->d_first = nullptr;
    s->cap = 0;
    for (int i = 0; i < RING; i++) {
        if ((e = hipHostMalloc((void **)&s->h_ops[i], sizeof(SweepArgs) * (size_t)cap)) != hipSuccess) return fail(s, e);
        if ((e = hipHostMalloc((void **)&s->h_first[i], sizeof(int32_t) * (size_t)(cap + 1))) != hipSuccess)
            return fail(s, e);
    }
    if ((e = hipMalloc(&s->d_ops, sizeof(SweepArgs) * (size_t)cap)) != hipSuccess) return fail(s, e);
    if ((e = hipMalloc(&s->d_first, sizeof(int32_t) * (size_t)(cap + 1))) != hipSuccess) return fail(s, e);
    s->cap = cap;
    return SILU_OK;
}

} // namespace

extern "C" {

int silu_server_create(silu_ctx *ctx, void *hip_stream, void *arena, size_t arena_bytes, int max_active,
                       silu_server **out)
{
    if (!ctx || !out || !arena || arena_bytes == 0 || max_active < 1 || ((uintptr_t)arena & 255)) return SILU_ERR_ARG;
    *out = nullptr;
    silu_server *s = new (std::nothrow) silu_server();
    if (!s) return SILU_ERR_NOMEM;
    s->ctx = ctx;
    s->stream = (hipStream_t)hip_stream;
    s->arena = (char *)arena;
    s->arena_bytes = arena_bytes;
    s->max_active = max_active;
    s->free_list.push_back({0, arena_bytes});
    for (int i = 0; i < RING; i++) {
        hipError_t e = hipEventCreateWithFlags(&s->ev[i], hipEventDisableTiming);
        if (e != hipSuccess) {
            silu_server_destroy(s);
            return SILU_ERR_HIP;
        }
    }
    if (grow(s, 64)) {
        silu_server_destroy(s);
        return SILU_ERR_HIP;
    }
    *out = s;
    return SILU_OK;
}

int silu_server_destroy(silu_server *s)
{
    if (!s) return SILU_ERR_ARG;
    (void)hipStreamSynchronize(s->stream);
    for (int i = 0; i < RING; i++) {
        if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
        (void)hipHostFree(s->h_ops[i]);
        (void)hipHostFree(s->h_first[i]);
    }
    (void)hipFree(s->d_ops);
    (void)hipFree(s->d_first);
    delete s;
    return SILU_OK;
}

int silu_server_register(silu_server *s, const silu_csr *A, const silu_factors *F, int *matrix_id)
{
    if (!s || !A || !F || !matrix_id) return SILU_ERR_ARG;
    if (A->n_rows <= 0 || A->n_rows != A->n_cols || F->Ls.n_rows != A->n_rows || F->Us.n_rows != A->n_rows)
        return SILU_ERR_SHAPE;
    if (A->dtype != SILU_F64 || F->Ls.dtype != SILU_F64 || F->Us.dtype != SILU_F64 || !F->dinv || !F->scaled)
        return SILU_ERR_UNSUPPORTED;
    if (F->scaled == 2 && !F->dc) return SILU_ERR_ARG;
    s->mats.push_back({*A, *F});
    *matrix_id = (int)s->mats.size() - 1;
    return SILU_OK;
}

int64_t silu_server_request_bytes(const silu_server *s, int matrix_id)
{
    if (!s || matrix_id < 0 || matrix_id >= (int)s->mats.size()) return -1;
    return (int64_t)(4 * vec_bytes(s->mats[(size_t)matrix_id].A.n_rows));
}

int silu_server_submit(silu_server *s, int matrix_id, const double *b, double *x, int outer, int m_L, int m_U,
                       int64_t *ticket)
{
    if (!s || !b || !x || !ticket || outer < 1 || m_L < 1 || m_U < 1 || (m_L == 1 && m_U == 1)) return SILU_ERR_ARG;
    if (matrix_id < 0 || matrix_id >= (int)s->mats.size()) return SILU_ERR_ARG;
    if ((size_t)silu_server_request_bytes(s, matrix_id) > s->arena_bytes) return SILU_ERR_NOMEM;
    Request q;
    q.ticket = s->next_ticket++;
    q.mid = matrix_id;
    q.b = b;
    q.x = x;
    q.outer = outer;
    q.mL = m_L;
    q.mU = m_U;
    q.total = outer * (1 + (m_L - 1) + (m_U - 1));
    s->queue.push_back(q);
    *ticket = q.ticket;
    return SILU_OK;
}

int silu_server_step(silu_server *s, int *n_active, int *n_queued)
{
    if (!s) return SILU_ERR_ARG;
    reap(s);
    // admission in arrival order while the workspace fits (no overtaking)
    while (!s->queue.empty() && (int)s->active.size() < s->max_active) {
        Request &q = s->queue.front();
        Range r;
        if (!allocate(s, (size_t)silu_server_request_bytes(s, q.mid), &r)) break;
        q.ws = r;
        s->active.push_back(q);
        s->queue.pop_front();
    }
    if (!s->active.empty()) {
        int st = grow(s, (int)s->active.size());
        if (st) return st;
        const int slot = (int)(s->steps % RING);
        if (s->steps >= RING) { // the staging slot was used RING steps ago
            hipError_t e = hipEventSynchronize(s->ev[slot]);
            if (e != hipSuccess) return fail(s, e);
            reap(s);
        }
        SweepArgs *ops = s->h_ops[slot];
        int32_t *first = s->h_first[slot];
        int total = 0;
        const int nops = (int)s->active.size();
        for (int i = 0; i < nops; i++) {
            ops[i] = op_of(s, s->active[(size_t)i]);
            first[i] = total;
            total += (ops[i].n + SERVE_RPB - 1) / SERVE_RPB;
        }
        first[nops] = total;
        hipError_t e = hipMemcpyAsync(s->d_ops, ops, sizeof(SweepArgs) * (size_t)nops, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->d_first, first, sizeof(int32_t) * (size_t)(nops + 1), hipMemcpyHostToDevice,
                               s->stream);
        if (e == hipSuccess) e = launch_sweep_batch(SERVE_RPB, s->d_ops, s->d_first, nops, total, s->stream);
        if (e == hipSuccess) e = hipEventRecord(s->ev[slot], s->stream);
        if (e != hipSuccess) return fail(s, e);
        const int64_t step = s->steps++;
        size_t w = 0;
        for (size_t i = 0; i < s->active.size(); i++) {
            Request &q = s->active[i];
            q.op++;
            if (q.op == q.total) {
                s->finish_step[q.ticket] = step;
                s->to_release.push_back({step, q.ws});
            } else {
                s->active[w++] = q;
            }
        }
        s->active.resize(w);
    }
    if (n_active) *n_active = (int)s->active.size();
    if (n_queued) *n_queued = (int)s->queue.size();
    return SILU_OK;
}

int silu_server_poll(silu_server *s, int64_t ticket, int *state)
{
    if (!s || !state || ticket < 0 || ticket >= s->next_ticket) return SILU_ERR_ARG;
    auto it = s->finish_step.find(ticket);
    if (it == s->finish_step.end()) {
        bool queued = false;
        for (const Request &q : s->queue) queued |= q.ticket == ticket;
        *state = queued ? 0 : 1;
        return SILU_OK;
    }
    reap(s);
    *state = it->second <= s->completed_through ? 3 : 2;
    return SILU_OK;
}

int silu_server_last_hip_error(const silu_server *s) { return s ? (int)s->last : 0; }

} // extern "C"
