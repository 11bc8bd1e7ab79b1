// Serving runtime: continuous batching of smoother and solve requests on
// resident matrices (the serving form of the scaled-ILU smoother).
//
// Each request is the op sequence of `outer` smoothing steps of eq.
// ILUsplit / Algorithm 2: a residual sweep on A, m_L - 1 sweeps on Ls (the
// last fused with D^{-1}), m_U - 1 sweeps on U~s (the last fused with the
// update of x); a solve request adds a final residual and makes every
// residual a convergence check (eq. relres).  A step admits queued requests
// in arrival order while their workspace fits in the caller's arena, then
// launches ONE batched kernel that advances every active request by one op,
// whatever op each is at (with up to 24 active requests the op table goes in
// the kernel arguments, else it is copied to the device first), through the
// server's sliced copies of the matrices; a small second launch closes the
// step's convergence checks.  A request's workspace returns to the arena once
// the GPU has passed its last launch (known from events recorded at the
// steps that need one).  Each row is summed by one lane in a fixed order, so
// a request's result does not depend on which requests shared its launches.
//
// Persistent mode (switched off, see PERSISTENT_AVAILABLE): a step would hand
// the requests it admits, with all of their ops, to one persistent launch
// (k_sweep_persist) on the next of a few server streams, each request's
// sweeps following one another through device-side dependency counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>
#include <new>
#include <vector>

#include "../../include/scaled_ilu.h"
#include "internal.h"
#include "plan.h"

using namespace silu;

namespace {

constexpr int RING = 8;        // events and op-table staging slots
constexpr int SERVE_RPB = SERVE_TILE_ROWS; // rows per workgroup of the batched sweep
constexpr int PSTREAMS = 3;    // persistent mode: streams the launches rotate over
constexpr int DEFAULT_MAX_WG = 1024;
// The persistent mode is switched off: on MI355X its launches did not finish
// (the requests never completed and the process waited for the kernel at
// exit), with the dependency counters at agent scope and again at system
// scope, for a cause not yet shown.  Until it is, set_mode refuses the mode.
constexpr bool PERSISTENT_AVAILABLE = false;
// Stepwise mode: an event at least every MARK_EVERY steps, and at most
// MAX_AHEAD steps enqueued past the last step known complete, so that a newly
// admitted request joins a launch within a few steps.
constexpr int MARK_EVERY = 4;
constexpr int MAX_AHEAD = 8;

struct Matrix {
    silu_csr A;
    silu_factors F;
    // the server's own sliced copies (device views; null where the CSR stream
    // is used) and their owners: A, Ls, Us, then Ls and Us with their FP32
    // values (when the factors carry them: the FP32-inner form)
    const SlicedView *sv[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    void *own[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    SlicedView *d_views = nullptr;
    bool fp32 = false; // the factors carry FP32 values
};

void free_matrix_copies(Matrix &M)
{
    for (int k = 0; k < 5; k++) free_owned_sliced(M.own[k]);
    (void)hipFree(M.d_views);
    M.d_views = nullptr;
    for (int k = 0; k < 5; k++) {
        M.own[k] = nullptr;
        M.sv[k] = nullptr;
    }
}

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
    double tol = 0.0; // > 0: a solve request (outer = its largest number of outer steps)
    int result = -1;  // solve requests: slot of its SolveCtl copy in the pinned result blocks
    int flag = -1;    // solve requests: its word in the pinned stop flags
    bool mixed = false; // the FP32-inner form
};

size_t vec_bytes(int64_t n) { return (((size_t)n * 8 + 255) / 256) * 256; }

// Workspace of a request: r, s and two iterates (n-vectors each), then the
// SolveCtl of a solve request and its per-tile partial sums.
size_t ctl_bytes(int64_t n)
{
    const size_t tiles = (size_t)((n + SERVE_TILE_ROWS - 1) / SERVE_TILE_ROWS);
    return ((sizeof(SolveCtl) + 16 * tiles + 255) / 256) * 256;
}
size_t request_bytes(int64_t n) { return 4 * vec_bytes(n) + ctl_bytes(n); }

// Pinned host copies of finishing solve requests' SolveCtl, in blocks that are
// never moved while the server lives; a slot is read and returned to a free
// list once the step that wrote it is done, so the blocks only cover the solve
// requests finishing at once.
constexpr int RESULTS_PER_BLOCK = 1024;

// What the server remembers of a ticket: kept from submission until
// MAX_RECORDS later tickets have finished (a finished ticket without a
// record is reported done by poll and wait; times and solve_result need its
// record).  The tickets completed() has not handed out yet are bounded the
// same way.
constexpr size_t MAX_RECORDS = (size_t)1 << 16;

struct Record {
    int64_t submitted_ns = 0, done_ns = -1; // steady clock; done_ns once the host saw it finish
    int64_t finish_step = -1;               // the step of its last op, once enqueued
    int result = -1;                        // solve requests: pinned SolveCtl slot until read
    int max_outer = 0;
    bool solve = false;
    int outer_steps = -1; // solve requests, once done
    double relres = 0.0;
};

// One step's launches, planned for the active requests advanced by t ops:
// their ops grouped by precision (one launch per precision present; the ops of
// different requests are independent, so the launch order does not matter).
// Groups of at most BATCH_ARG_OPS ops carry their table in the kernel
// arguments; longer ones are packed into a staging buffer, copied to the
// device before the step's launches.
struct StagedGroup {
    Prec kind;
    size_t ops_off, first_off; // in the staging buffer
    int k, total;
};
struct StepPlan {
    int t = 0;
    std::vector<SweepArgs> ops;
    std::vector<Prec> prec;
    int count[5] = {0, 0, 0, 0, 0};
    StagedGroup sg[5];
    int nsg = 0;
};
const Prec KINDS[5] = {Prec::F64, Prec::MIX_RES, Prec::MIX_L1, Prec::MIX_L, Prec::MIX_U};

int64_t now_ns()
{
    return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

} // namespace

struct silu_server {
    std::vector<SolveCtl *> result_blocks; // pinned, RESULTS_PER_BLOCK each
    int64_t nresults = 0;                  // slots in result_blocks
    std::vector<int> free_results;         // slots not holding a result still to be read
    std::unordered_map<int64_t, Record> recs; // ticket -> record (bounded: MAX_RECORDS finished)
    std::deque<int64_t> retired;               // finished tickets with a record, oldest first
    int32_t *hflags = nullptr;                  // pinned stop flags of solve requests (2 max_active words)
    int32_t *d_hflags = nullptr;                // the same words as the device addresses them
    std::vector<int> free_flags;
    std::map<int64_t, int> ticket_flag;         // ticket -> flag word, until the request is reported done
    bool force_mark = false;                    // the next step must record a mark
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
    std::vector<std::pair<int64_t, int64_t>> to_report; // (step, ticket) not yet known done
    std::deque<int64_t> done_queue;                     // done, not yet returned by completed()
    int64_t next_ticket = 0, steps = 0, completed_through = -1;
    hipEvent_t ev[RING] = {};
    int64_t done_step[RING];   // persistent mode: the step a slot last held, once the GPU has passed it
    // stepwise mode: events are recorded only at steps that need one (a request
    // finishes, the op table was staged through host memory, or MARK_EVERY
    // steps have passed), round-robin over ev[]; marks = (step, slot) recorded
    // and not yet seen complete, in order
    std::deque<std::pair<int64_t, int>> marks;
    int64_t nmarks = 0, last_mark_step = -1;
    // op tables too long for the kernel arguments: each staged group's ops and
    // first-block offsets packed into one pinned buffer per ring slot, copied
    // to d_stage with one copy per step
    char *h_stage[RING] = {};
    char *d_stage = nullptr;
    int cap = 0; // op-table capacity
    StepPlan step_plan;                // reused: the plan of a single step
    std::vector<StepPlan> burst_plans; // and those of a burst
    hipError_t last = hipSuccess;
    // persistent mode
    int mode = 0;
    int max_wg = DEFAULT_MAX_WG;
    int wait_us = PERSIST_WAIT_US;  // bound of one wait inside a persistent launch
    long long clock_khz = 0;        // the device's wall_clock64 rate
    hipStream_t ps[PSTREAMS] = {};
    hipEvent_t ev_in = nullptr;
    char *h_plan[RING] = {};
    char *d_plan[RING] = {};
    size_t plan_cap[RING] = {};
    int32_t *h_ctl[RING] = {}; // ctl words read back after each launch
    int slot_reqs[RING] = {};
    int inflight = 0;            // requests launched whose step the GPU has not passed
    std::vector<int64_t> failed; // steps whose launch gave up a wait
    silu_server()
    {
        for (int i = 0; i < RING; i++) done_step[i] = -1;
    }
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

bool step_done(const silu_server *s, int64_t k) { return k <= s->completed_through || s->done_step[k % RING] == k; }

// Steps whose event has completed (persistent launches may finish out of
// order): reclaim the workspace they held.
void reap(silu_server *s)
{
    while (s->mode == 0 && !s->marks.empty() && hipEventQuery(s->ev[s->marks.front().second]) == hipSuccess) {
        s->completed_through = std::max(s->completed_through, s->marks.front().first);
        s->marks.pop_front();
    }
    for (int64_t k = s->completed_through + 1; s->mode == 1 && k < s->steps; k++) {
        const int slot = (int)(k % RING);
        if (s->done_step[slot] == k) continue;
        if (hipEventQuery(s->ev[slot]) != hipSuccess) {
            if (s->mode == 0) break; // one stream: later steps are not done either
            continue;
        }
        s->done_step[slot] = k;
        if (s->mode == 1) {
            s->inflight -= s->slot_reqs[slot];
            if (s->h_ctl[slot][1] != 0) s->failed.push_back(k);
        }
    }
    while (s->completed_through + 1 < s->steps && step_done(s, s->completed_through + 1)) s->completed_through++;
    auto &tr = s->to_release;
    size_t w = 0;
    for (size_t i = 0; i < tr.size(); i++) {
        if (step_done(s, tr[i].first))
            release(s, tr[i].second);
        else
            tr[w++] = tr[i];
    }
    tr.resize(w);
    auto &rp = s->to_report;
    w = 0;
    for (size_t i = 0; i < rp.size(); i++) {
        if (step_done(s, rp[i].first)) {
            s->done_queue.push_back(rp[i].second);
            if (s->done_queue.size() > MAX_RECORDS) s->done_queue.pop_front();
            Record &rec = s->recs[rp[i].second];
            rec.done_ns = now_ns();
            if (rec.result >= 0) { // the SolveCtl copied when it finished
                const SolveCtl &c = s->result_blocks[(size_t)rec.result / RESULTS_PER_BLOCK]
                                                    [rec.result % RESULTS_PER_BLOCK];
                rec.outer_steps = c.stop ? c.checks - 1 : rec.max_outer + 1;
                rec.relres = std::sqrt(c.rr) / std::sqrt(c.bb);
                s->free_results.push_back(rec.result);
                rec.result = -1;
            }
            s->retired.push_back(rp[i].second);
            while (s->retired.size() > MAX_RECORDS) {
                s->recs.erase(s->retired.front());
                s->retired.pop_front();
            }
            auto fl = s->ticket_flag.find(rp[i].second);
            if (fl != s->ticket_flag.end()) {
                s->free_flags.push_back(fl->second);
                s->ticket_flag.erase(fl);
            }
        } else
            rp[w++] = rp[i];
    }
    rp.resize(w);
}

// The op request q runs at its current position.
SweepArgs op_of(const silu_server *s, const Request &q, Prec *prec = nullptr)
{
    const Matrix &M = s->mats[(size_t)q.mid];
    const int64_t n = M.A.n_rows;
    const size_t vb = vec_bytes(n);
    char *w = s->arena + q.ws.off;
    double *r = (double *)w, *sv = (double *)(w + vb), *tmp[2] = {(double *)(w + 2 * vb), (double *)(w + 3 * vb)};
    const int per = 1 + (q.mL - 1) + (q.mU - 1);
    const int j = q.op % per;
    SweepArgs a;
    Prec p = Prec::F64;
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
        a.sv = M.sv[0];
        a.xin = q.x;
        a.rhs = q.b;
        if (q.mL >= 2) {
            a.epi = EPI_STORE;
            a.out = r;
        } else {
            a.epi = EPI_SCALE;
            a.out = sv;
            p = q.mixed ? Prec::MIX_RES : Prec::F64; // FP32-inner: the residual rounded before D^{-1}
        }
    } else if (j < q.mL) { // L sweep k = j + 1
        const int k = j + 1;
        a.rp = M.F.Ls.row_ptr;
        a.col = M.F.Ls.col_idx;
        a.val = q.mixed ? (const void *)M.F.Ls_val32 : M.F.Ls.val;
        a.sv = M.sv[q.mixed ? 3 : 1];
        if (q.mixed) p = k == 2 ? Prec::MIX_L1 : Prec::MIX_L; // the first gathers r and rounds it
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
        a.val = q.mixed ? (const void *)M.F.Us_val32 : M.F.Us.val;
        a.sv = M.sv[q.mixed ? 4 : 2];
        if (q.mixed) p = Prec::MIX_U;
        a.xin = k == 2 ? (const void *)sv : (const void *)tmp[(k - 1) & 1];
        a.rhs = sv;
        if (k < q.mU) {
            a.epi = EPI_STORE;
            a.out = tmp[k & 1];
        } else {
            a.epi = EPI_UPDATE;
        }
    }
    if (q.tol > 0.0) {
        char *cb = w + 4 * vb;
        a.sctl = (const SolveCtl *)cb;
        if (j == 0) { // the residual at the start of an outer step (or the final one) is a check
            a.spart = (double *)(cb + sizeof(SolveCtl));
            a.scheck = q.op == 0 ? 2 : 1;
        }
    }
    if (prec) *prec = p;
    return a;
}

// Bytes of one staging buffer for cap ops over at most 5 groups: each group's
// ops, then its cap + 1 first-block offsets, the group rounded up to 16 bytes.
size_t stage_bytes(int cap) { return (size_t)cap * (sizeof(SweepArgs) + sizeof(int32_t)) + 5 * 32; }

size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

int grow(silu_server *s, int need)
{
    if (need <= s->cap) return SILU_OK;
    // idle the ring before reallocating the staging buffers and the device table
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(s, e);
    int cap = std::max(need, std::max(64, 2 * s->cap));
    for (int i = 0; i < RING; i++) {
        (void)hipHostFree(s->h_stage[i]);
        s->h_stage[i] = nullptr;
    }
    (void)hipFree(s->d_stage);
    s->d_stage = nullptr;
    s->cap = 0;
    for (int i = 0; i < RING; i++)
        if ((e = hipHostMalloc((void **)&s->h_stage[i], stage_bytes(cap))) != hipSuccess) return fail(s, e);
    if ((e = hipMalloc(&s->d_stage, stage_bytes(cap))) != hipSuccess) return fail(s, e);
    s->cap = cap;
    return SILU_OK;
}

// Stepwise mode: the event slot for the next mark, after the mark that last
// used it (RING marks ago) has completed; its staging buffers are free then too.
int claim_mark(silu_server *s, int *slot_out)
{
    if ((int)s->marks.size() >= RING) {
        const hipError_t e = hipEventSynchronize(s->ev[s->marks.front().second]);
        if (e != hipSuccess) return fail(s, e);
        reap(s);
    }
    *slot_out = (int)(s->nmarks % RING);
    return SILU_OK;
}

int record_mark(silu_server *s, int slot, int64_t step)
{
    const hipError_t e = hipEventRecord(s->ev[slot], s->stream);
    if (e != hipSuccess) return fail(s, e);
    s->marks.push_back({step, slot});
    s->nmarks++;
    s->last_mark_step = step;
    return SILU_OK;
}

// Stepwise mode: hold the host back while more than MAX_AHEAD steps are
// enqueued past the last one known complete.
int throttle(silu_server *s)
{
    reap(s);
    while (s->steps - 1 - s->completed_through > MAX_AHEAD && !s->marks.empty()) {
        const hipError_t e = hipEventSynchronize(s->ev[s->marks.front().second]);
        if (e != hipSuccess) return fail(s, e);
        reap(s);
    }
    return SILU_OK;
}

// Persistent mode: wait for a staging slot's previous launch before reusing it.
int take_slot(silu_server *s, int *slot_out)
{
    const int slot = (int)(s->steps % RING);
    if (s->steps >= RING) {
        hipError_t e = hipEventSynchronize(s->ev[slot]);
        if (e != hipSuccess) return fail(s, e);
        reap(s);
    }
    *slot_out = slot;
    return SILU_OK;
}

size_t align64(size_t v) { return (v + 63) & ~(size_t)63; }

// Persistent mode: one launch runs every op of the admitted batch.  Requests
// go in order of their work (rows x ops), smallest first, each as one chain
// of ops; the plan is [ctl 4 x int32][first nops+1][dep nops][done nops] then
// the op table, copied to the device in one transfer that also zeroes the
// counters.
int launch_persistent(silu_server *s, std::vector<Request> &batch)
{
    std::vector<int64_t> rows(batch.size());
    std::vector<int> nop(batch.size()), order;
    for (size_t r = 0; r < batch.size(); r++) {
        rows[r] = s->mats[(size_t)batch[r].mid].A.n_rows;
        nop[r] = batch[r].total;
    }
    std::vector<int32_t> pfirst, pdep;
    int64_t grid = 0;
    if (!persist_plan(rows, nop, SERVE_RPB, s->max_wg, order, pfirst, pdep, &grid)) return SILU_ERR_UNSUPPORTED;
    const int64_t nops = (int64_t)pdep.size(), tiles = pfirst.back();
    const size_t n_int = 4 + (size_t)(nops + 1) + 2 * (size_t)nops;
    const size_t ops_off = align64(n_int * sizeof(int32_t));
    const size_t bytes = ops_off + (size_t)nops * sizeof(SweepArgs);
    int slot;
    int st = take_slot(s, &slot);
    if (st) return st;
    hipError_t e;
    if (s->plan_cap[slot] < bytes) {
        (void)hipHostFree(s->h_plan[slot]);
        (void)hipFree(s->d_plan[slot]);
        s->h_plan[slot] = nullptr;
        s->d_plan[slot] = nullptr;
        s->plan_cap[slot] = 0;
        const size_t cap = std::max(bytes, (size_t)64 << 10);
        if ((e = hipHostMalloc((void **)&s->h_plan[slot], cap)) != hipSuccess) return fail(s, e);
        if ((e = hipMalloc((void **)&s->d_plan[slot], cap)) != hipSuccess) return fail(s, e);
        s->plan_cap[slot] = cap;
    }
    int32_t *ctl = (int32_t *)s->h_plan[slot];
    int32_t *first = ctl + 4, *dep = first + nops + 1, *done = dep + nops;
    SweepArgs *ops = (SweepArgs *)(s->h_plan[slot] + ops_off);
    ctl[0] = 0;
    ctl[1] = 0;
    ctl[2] = (int32_t)nops;
    ctl[3] = (int32_t)tiles;
    int64_t i = 0;
    for (int r : order) {
        Request q = batch[(size_t)r];
        for (int j = 0; j < q.total; j++, i++) {
            q.op = j;
            ops[i] = op_of(s, q);
            first[i] = pfirst[(size_t)i];
            dep[i] = pdep[(size_t)i];
            done[i] = 0;
        }
    }
    first[nops] = pfirst[(size_t)nops];
    hipStream_t ps = s->ps[s->steps % PSTREAMS];
    char *d = s->d_plan[slot];
    PersistPlan p;
    p.ctl = (int32_t *)d;
    p.first = p.ctl + 4;
    p.dep = p.first + nops + 1;
    p.done = (int32_t *)p.dep + nops;
    p.ops = (const SweepArgs *)(d + ops_off);
    p.nops = (int)nops;
    p.wait_ticks = std::max<long long>(1, (long long)s->wait_us * s->clock_khz / 1000);
    e = hipEventRecord(s->ev_in, s->stream); // b and x are produced on the caller's stream
    if (e == hipSuccess) e = hipStreamWaitEvent(ps, s->ev_in, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(d, s->h_plan[slot], bytes, hipMemcpyHostToDevice, ps);
    if (e == hipSuccess) e = launch_sweep_persist(p, (int)grid, ps);
    if (e == hipSuccess) e = hipMemcpyAsync(s->h_ctl[slot], d, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, ps);
    if (e == hipSuccess) e = hipEventRecord(s->ev[slot], ps);
    if (e != hipSuccess) return fail(s, e);
    s->slot_reqs[slot] = (int)batch.size();
    s->inflight += (int)batch.size();
    const int64_t step = s->steps++;
    for (const Request &q : batch) {
        s->recs[q.ticket].finish_step = step;
        s->to_release.push_back({step, q.ws});
        s->to_report.push_back({step, q.ticket});
    }
    return SILU_OK;
}

int destroy_persistent(silu_server *s)
{
    for (int i = 0; i < PSTREAMS; i++) {
        if (s->ps[i]) {
            (void)hipStreamSynchronize(s->ps[i]);
            (void)hipStreamDestroy(s->ps[i]);
            s->ps[i] = nullptr;
        }
    }
    if (s->ev_in) (void)hipEventDestroy(s->ev_in);
    s->ev_in = nullptr;
    for (int i = 0; i < RING; i++) {
        (void)hipHostFree(s->h_plan[i]);
        (void)hipFree(s->d_plan[i]);
        (void)hipHostFree(s->h_ctl[i]);
        s->h_plan[i] = nullptr;
        s->d_plan[i] = nullptr;
        s->h_ctl[i] = nullptr;
        s->plan_cap[i] = 0;
    }
    return SILU_OK;
}

int create_persistent(silu_server *s)
{
    hipError_t e;
    for (int i = 0; i < PSTREAMS; i++)
        if (!s->ps[i] && (e = hipStreamCreateWithFlags(&s->ps[i], hipStreamNonBlocking)) != hipSuccess)
            return fail(s, e);
    if (!s->ev_in && (e = hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming)) != hipSuccess) return fail(s, e);
    int dev = 0, khz = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return fail(s, e);
    if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess) return fail(s, e);
    if (khz <= 0) return SILU_ERR_UNSUPPORTED;
    s->clock_khz = khz;
    for (int i = 0; i < RING; i++) {
        if (!s->h_ctl[i]) {
            if ((e = hipHostMalloc((void **)&s->h_ctl[i], 4 * sizeof(int32_t))) != hipSuccess) return fail(s, e);
            s->h_ctl[i][1] = 0;
        }
    }
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
    // stop-flag words: one per running solve request, held until it is reported
    // done (twice max_active, so that finished requests not yet reaped leave
    // words for new ones; without a word a request still runs, only not retired
    // early)
    const size_t nflags = 2 * (size_t)max_active;
    if (grow(s, 64) || hipHostMalloc((void **)&s->hflags, sizeof(int32_t) * nflags) != hipSuccess ||
        hipHostGetDevicePointer((void **)&s->d_hflags, s->hflags, 0) != hipSuccess) {
        silu_server_destroy(s);
        return SILU_ERR_HIP;
    }
    for (size_t i = nflags; i-- > 0;) s->free_flags.push_back((int)i);
    *out = s;
    return SILU_OK;
}

int silu_server_destroy(silu_server *s)
{
    if (!s) return SILU_ERR_ARG;
    (void)hipStreamSynchronize(s->stream);
    destroy_persistent(s);
    for (int i = 0; i < RING; i++) {
        if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
        (void)hipHostFree(s->h_stage[i]);
    }
    (void)hipFree(s->d_stage);
    for (Matrix &M : s->mats) free_matrix_copies(M);
    for (SolveCtl *blk : s->result_blocks) (void)hipHostFree(blk);
    (void)hipHostFree(s->hflags);
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
    // the sliced copies the batched sweeps read (built now, owned by the server)
    Matrix M;
    M.A = *A;
    M.F = *F;
    M.fp32 = (F->Ls.nnz == 0 || F->Ls_val32) && (F->Us.nnz == 0 || F->Us_val32);
    const silu_csr *parts[5] = {A, &F->Ls, &F->Us, &F->Ls, &F->Us};
    const void *vals[5] = {A->val, F->Ls.val, F->Us.val, F->Ls_val32, F->Us_val32};
    SlicedView views[5];
    int st = SILU_OK;
    for (int k = 0; k < 5 && st == SILU_OK; k++)
        if (k < 3 || (M.fp32 && vals[k]))
            st = make_owned_sliced(s->ctx, parts[k], vals[k], k < 3 ? 8 : 4, &views[k], &M.own[k]);
    hipError_t e = hipSuccess;
    if (st == SILU_OK) {
        e = hipMalloc((void **)&M.d_views, sizeof(views));
        if (e == hipSuccess) e = hipMemcpy(M.d_views, views, sizeof(views), hipMemcpyHostToDevice);
    }
    if (st != SILU_OK || e != hipSuccess) {
        free_matrix_copies(M);
        return st != SILU_OK ? st : fail(s, e);
    }
    for (int k = 0; k < 5; k++) M.sv[k] = views[k].nslice > 0 ? M.d_views + k : nullptr;
    s->mats.push_back(M);
    *matrix_id = (int)s->mats.size() - 1;
    return SILU_OK;
}

int64_t silu_server_request_bytes(const silu_server *s, int matrix_id)
{
    if (!s || matrix_id < 0 || matrix_id >= (int)s->mats.size()) return -1;
    return (int64_t)request_bytes(s->mats[(size_t)matrix_id].A.n_rows);
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
    s->recs[q.ticket].submitted_ns = now_ns();
    *ticket = q.ticket;
    return SILU_OK;
}

// A finishing solve request: its SolveCtl is copied to the pinned result
// blocks after everything enqueued so far (the mark that ends its step covers
// the copy).
int save_result(silu_server *s, Request &q)
{
    hipError_t e;
    if (s->free_results.empty()) {
        SolveCtl *blk = nullptr;
        if ((e = hipHostMalloc((void **)&blk, sizeof(SolveCtl) * RESULTS_PER_BLOCK)) != hipSuccess) return fail(s, e);
        s->result_blocks.push_back(blk);
        for (int k = RESULTS_PER_BLOCK - 1; k >= 0; k--) s->free_results.push_back((int)s->nresults + k);
        s->nresults += RESULTS_PER_BLOCK;
    }
    q.result = s->free_results.back();
    s->free_results.pop_back();
    SolveCtl *dst = s->result_blocks[(size_t)q.result / RESULTS_PER_BLOCK] + q.result % RESULTS_PER_BLOCK;
    const char *src = s->arena + q.ws.off + 4 * vec_bytes(s->mats[(size_t)q.mid].A.n_rows);
    if ((e = hipMemcpyAsync(dst, src, sizeof(SolveCtl), hipMemcpyDeviceToHost, s->stream)) != hipSuccess)
        return fail(s, e);
    Record &rec = s->recs[q.ticket];
    rec.result = q.result;
    rec.max_outer = q.outer;
    return SILU_OK;
}

int silu_server_submit_flags(silu_server *s, int matrix_id, const double *b, double *x, int outer, int m_L, int m_U,
                             int flags, int64_t *ticket)
{
    if (!s || (flags & ~SILU_MIXED)) return SILU_ERR_ARG;
    const bool mixed = (flags & SILU_MIXED) != 0;
    if (mixed && (s->mode != 0 || matrix_id < 0 || matrix_id >= (int)s->mats.size() ||
                  !s->mats[(size_t)matrix_id].fp32))
        return matrix_id < 0 || matrix_id >= (int)s->mats.size() ? SILU_ERR_ARG : SILU_ERR_UNSUPPORTED;
    const int st = silu_server_submit(s, matrix_id, b, x, outer, m_L, m_U, ticket);
    if (st) return st;
    s->queue.back().mixed = mixed;
    return SILU_OK;
}

int silu_server_submit_solve(silu_server *s, int matrix_id, const double *b, double *x, double tol, int max_outer,
                             int m_L, int m_U, int64_t *ticket)
{
    if (!s || !(tol > 0.0) || max_outer < 0 || max_outer > (1 << 20)) return SILU_ERR_ARG;
    if (s->mode != 0) return SILU_ERR_UNSUPPORTED;
    const int st = silu_server_submit(s, matrix_id, b, x, std::max(max_outer, 1), m_L, m_U, ticket);
    if (st) return st;
    Request &q = s->queue.back();
    q.outer = max_outer;
    q.tol = tol;
    s->recs[q.ticket].solve = true;
    q.total = max_outer * (1 + (m_L - 1) + (m_U - 1)) + 1; // and the check of the last iterate
    return SILU_OK;
}

int silu_server_solve_result(silu_server *s, int64_t ticket, int *outer_steps, double *relres)
{
    if (!s || !outer_steps || !relres) return SILU_ERR_ARG;
    reap(s);
    auto it = s->recs.find(ticket);
    if (it == s->recs.end() || !it->second.solve || it->second.done_ns < 0) return SILU_ERR_ARG;
    *outer_steps = it->second.outer_steps;
    *relres = it->second.relres;
    return SILU_OK;
}

void plan_step(const silu_server *s, int t, StepPlan &p)
{
    const int nops = (int)s->active.size();
    p.t = t;
    p.nsg = 0;
    p.ops.resize((size_t)nops);
    p.prec.resize((size_t)nops);
    for (int i = 0; i < nops; i++) {
        Request q = s->active[(size_t)i];
        q.op += t;
        p.ops[(size_t)i] = op_of(s, q, &p.prec[(size_t)i]);
    }
    for (int g = 0; g < 5; g++) p.count[g] = 0;
    for (int i = 0; i < nops; i++)
        for (int g = 0; g < 5; g++) p.count[g] += p.prec[(size_t)i] == KINDS[g];
}

bool plan_staged(const StepPlan &p)
{
    for (int g = 0; g < 5; g++)
        if (p.count[g] > BATCH_ARG_OPS) return true;
    return false;
}

// The plan's staged groups packed into buf from *used on.
void pack_step(StepPlan &p, char *buf, size_t *used)
{
    const int nops = (int)p.ops.size();
    for (int g = 0; g < 5; g++) {
        if (p.count[g] <= BATCH_ARG_OPS) continue;
        const size_t first_off = *used + sizeof(SweepArgs) * (size_t)p.count[g];
        SweepArgs *h_ops = (SweepArgs *)(buf + *used);
        int32_t *h_first = (int32_t *)(buf + first_off);
        int k = 0, total = 0;
        for (int i = 0; i < nops; i++) {
            if (p.prec[(size_t)i] != KINDS[g]) continue;
            h_ops[k] = p.ops[(size_t)i];
            h_first[k++] = total;
            total += (p.ops[(size_t)i].n + SERVE_RPB - 1) / SERVE_RPB;
        }
        h_first[k] = total;
        p.sg[p.nsg++] = {KINDS[g], *used, first_off, k, total};
        *used = align16(first_off + sizeof(int32_t) * (size_t)(k + 1));
    }
}

// The plan's launches (staged groups reading d_stage, already copied), then
// the closing launch of the convergence checks its ops make.
hipError_t launch_step(silu_server *s, const StepPlan &p, const char *d_stage)
{
    const int nops = (int)p.ops.size();
    hipError_t e = hipSuccess;
    for (int g = 0; g < 5 && e == hipSuccess; g++) {
        if (!p.count[g] || p.count[g] > BATCH_ARG_OPS) continue;
        BatchArgs ba;
        int k = 0, total = 0;
        for (int i = 0; i < nops; i++) {
            if (p.prec[(size_t)i] != KINDS[g]) continue;
            ba.op[k] = p.ops[(size_t)i];
            ba.first[k++] = total;
            total += (p.ops[(size_t)i].n + SERVE_RPB - 1) / SERVE_RPB;
        }
        ba.first[k] = total;
        ba.nops = k;
        e = launch_sweep_batch_args(KINDS[g], ba, s->stream);
    }
    for (int i = 0; i < p.nsg && e == hipSuccess; i++)
        e = launch_sweep_batch(p.sg[i].kind, (const SweepArgs *)(d_stage + p.sg[i].ops_off),
                               (const int32_t *)(d_stage + p.sg[i].first_off), p.sg[i].k, p.sg[i].total, s->stream);
    SolveCheckArgs ca;
    ca.count = 0;
    for (const Request &q0 : s->active) {
        if (e != hipSuccess) break;
        const int op = q0.op + p.t;
        if (q0.tol <= 0.0 || op % (1 + (q0.mL - 1) + (q0.mU - 1)) != 0) continue;
        const int64_t n = s->mats[(size_t)q0.mid].A.n_rows;
        char *cb = s->arena + q0.ws.off + 4 * vec_bytes(n);
        ca.c[ca.count++] = {(SolveCtl *)cb, (const double *)(cb + sizeof(SolveCtl)),
                            (int)((n + SERVE_TILE_ROWS - 1) / SERVE_TILE_ROWS), op == 0 ? 1 : 0, q0.tol,
                            q0.flag >= 0 ? s->d_hflags + q0.flag : nullptr};
        if (ca.count == SOLVE_CHECKS_PER_LAUNCH) {
            e = launch_solve_check(ca, s->stream);
            ca.count = 0;
        }
    }
    if (e == hipSuccess && ca.count) e = launch_solve_check(ca, s->stream);
    return e;
}

// The bookkeeping after the steps up to `last` were enqueued with every
// active request advanced by `adv` ops: requests whose last op ran retire
// (a finishing solve request's state goes to pinned host memory first), and
// the last step records a mark when one is due (slot >= 0: already claimed
// for a staging buffer).
int finish_steps(silu_server *s, int adv, int slot)
{
    const int64_t last = s->steps - 1;
    bool finishing = s->force_mark;
    s->force_mark = false;
    int st;
    for (Request &q : s->active) {
        if (q.op + adv != q.total) continue;
        finishing = true;
        if (q.tol > 0.0 && (st = save_result(s, q))) return st;
    }
    if (slot < 0 && (finishing || last - s->last_mark_step >= MARK_EVERY) && (st = claim_mark(s, &slot)))
        return st;
    if (slot >= 0 && (st = record_mark(s, slot, last))) return st;
    size_t w = 0;
    for (size_t i = 0; i < s->active.size(); i++) {
        Request &q = s->active[i];
        q.op += adv;
        if (q.op == q.total) {
            s->recs[q.ticket].finish_step = last;
            s->to_release.push_back({last, q.ws});
            s->to_report.push_back({last, q.ticket});
        } else {
            s->active[w++] = q;
        }
    }
    s->active.resize(w);
    return SILU_OK;
}

// Several steps enqueued together (silu_server_run): when nothing waits for
// admission, no stop flag is pending and every active request has at least
// k ops left, the next k steps are planned at once, their staged op tables
// copied to the device with one copy, and their launches enqueued back to
// back -- the launches of k single steps, with one copy and at most one mark
// for all of them.  A request the device stops meanwhile skips its sweeps
// there and is retired by the next single step.  *done: the steps enqueued
// (0: none, the caller takes a single step).
int burst(silu_server *s, int k_max, int *done)
{
    *done = 0;
    if (s->mode != 0 || !s->queue.empty() || s->active.empty() || s->force_mark) return SILU_OK;
    int k = std::min(k_max, MAX_AHEAD);
    for (const Request &q : s->active) {
        if (q.flag >= 0 && __atomic_load_n(&s->hflags[q.flag], __ATOMIC_ACQUIRE) != 0) return SILU_OK;
        k = std::min(k, q.total - q.op);
    }
    if (k < 2) return SILU_OK;
    int st;
    if ((st = throttle(s))) return st;
    std::vector<StepPlan> &plans = s->burst_plans;
    if ((int)plans.size() < k) plans.resize((size_t)k);
    bool staged = false;
    for (int t = 0; t < k; t++) {
        plan_step(s, t, plans[(size_t)t]);
        staged |= plan_staged(plans[(size_t)t]);
    }
    int slot = -1;
    if (staged) {
        if ((st = grow(s, k * ((int)s->active.size() + 5)))) return st;
        if ((st = claim_mark(s, &slot))) return st; // its staging buffer is free
    }
    size_t used = 0;
    for (int t = 0; t < k && staged; t++) pack_step(plans[(size_t)t], s->h_stage[slot], &used);
    hipError_t e = hipSuccess;
    if (used) e = hipMemcpyAsync(s->d_stage, s->h_stage[slot], used, hipMemcpyHostToDevice, s->stream);
    for (int t = 0; t < k && e == hipSuccess; t++) e = launch_step(s, plans[(size_t)t], s->d_stage);
    if (e != hipSuccess) return fail(s, e);
    s->steps += k;
    if ((st = finish_steps(s, k, slot))) return st;
    *done = k;
    return SILU_OK;
}

int silu_server_step(silu_server *s, int *n_active, int *n_queued)
{
    if (!s) return SILU_ERR_ARG;
    reap(s);
    if (s->mode == 1) {
        std::vector<Request> batch;
        while (!s->queue.empty() && s->inflight + (int)batch.size() < s->max_active) {
            Request &q = s->queue.front();
            Range r;
            if (!allocate(s, (size_t)silu_server_request_bytes(s, q.mid), &r)) break;
            q.ws = r;
            batch.push_back(q);
            s->queue.pop_front();
        }
        if (!batch.empty()) {
            const int st = launch_persistent(s, batch);
            if (st == SILU_ERR_UNSUPPORTED) { // rejected before anything was enqueued
                for (const Request &q : batch) release(s, q.ws);
                for (auto it = batch.rbegin(); it != batch.rend(); ++it) {
                    Request q = *it;
                    q.ws = {0, 0};
                    s->queue.push_front(q);
                }
            }
            if (st) return st; // a HIP failure leaves the server unusable
        }
        if (n_active) *n_active = s->inflight;
        if (n_queued) *n_queued = (int)s->queue.size();
        return SILU_OK;
    }
    // solve requests the device has stopped: no more sweeps; they finish with
    // the next step, whose mark covers their last (skipped) sweeps and the copy
    // of their state
    {
        size_t w = 0;
        for (size_t i = 0; i < s->active.size(); i++) {
            Request &q = s->active[i];
            if (q.flag >= 0 && __atomic_load_n(&s->hflags[q.flag], __ATOMIC_ACQUIRE) != 0) {
                const int st = save_result(s, q);
                if (st) return st;
                s->recs[q.ticket].finish_step = s->steps;
                s->to_release.push_back({s->steps, q.ws});
                s->to_report.push_back({s->steps, q.ticket});
                s->force_mark = true;
                continue;
            }
            s->active[w++] = s->active[i];
        }
        s->active.resize(w);
    }
    // admission in arrival order while the workspace fits (no overtaking)
    while (!s->queue.empty() && (int)s->active.size() < s->max_active) {
        Request &q = s->queue.front();
        Range r;
        if (!allocate(s, (size_t)silu_server_request_bytes(s, q.mid), &r)) break;
        q.ws = r;
        if (q.tol > 0.0) { // a fresh SolveCtl: not stopped, no checks yet; and a clear host flag
            const size_t vb = vec_bytes(s->mats[(size_t)q.mid].A.n_rows);
            const hipError_t e = launch_fill((int)(sizeof(SolveCtl) / 8), (double *)(s->arena + r.off + 4 * vb),
                                             0.0, nullptr, 0.0, s->stream);
            if (e != hipSuccess) return fail(s, e);
            if (!s->free_flags.empty()) {
                q.flag = s->free_flags.back();
                s->free_flags.pop_back();
                __atomic_store_n(&s->hflags[q.flag], 0, __ATOMIC_RELEASE);
                s->ticket_flag[q.ticket] = q.flag;
            }
        }
        s->active.push_back(q);
        s->queue.pop_front();
    }
    if (!s->active.empty()) {
        StepPlan &p = s->step_plan;
        plan_step(s, 0, p);
        const bool staged = plan_staged(p);
        int st = staged ? grow(s, (int)s->active.size() + 5) : SILU_OK;
        if (st) return st;
        if ((st = throttle(s))) return st;
        int slot = -1;
        if (staged && (st = claim_mark(s, &slot))) return st; // its staging buffer is free
        size_t used = 0;
        if (staged) pack_step(p, s->h_stage[slot], &used);
        hipError_t e = hipSuccess;
        if (used) e = hipMemcpyAsync(s->d_stage, s->h_stage[slot], used, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = launch_step(s, p, s->d_stage);
        if (e != hipSuccess) return fail(s, e);
        s->steps++;
        if ((st = finish_steps(s, 1, slot))) return st;
    } else if (s->force_mark) { // stopped solve requests and nothing to launch: an empty step ends them
        s->force_mark = false;
        const int64_t step = s->steps++;
        int slot;
        int st = claim_mark(s, &slot);
        if (!st) st = record_mark(s, slot, step);
        if (st) return st;
    }
    if (n_active) *n_active = (int)s->active.size();
    if (n_queued) *n_queued = (int)s->queue.size();
    return SILU_OK;
}

int silu_server_run(silu_server *s, int max_steps, int *n_active, int *n_queued)
{
    if (!s || max_steps < 1) return SILU_ERR_ARG;
    int a = 0, q = 0;
    for (int k = 0; k < max_steps;) {
        int done = 0;
        int st = burst(s, max_steps - k, &done);
        if (st) return st;
        if (done) {
            k += done;
            a = (int)s->active.size();
            q = (int)s->queue.size();
        } else {
            if ((st = silu_server_step(s, &a, &q))) return st;
            k++;
        }
        if (a == 0) break;
    }
    if (n_active) *n_active = a;
    if (n_queued) *n_queued = q;
    return SILU_OK;
}

int silu_server_poll(silu_server *s, int64_t ticket, int *state)
{
    if (!s || !state || ticket < 0 || ticket >= s->next_ticket) return SILU_ERR_ARG;
    auto it = s->recs.find(ticket);
    if (it == s->recs.end()) { // finished long ago: its record has been dropped
        *state = 3;
        return SILU_OK;
    }
    const int64_t k = it->second.finish_step;
    if (k < 0) {
        bool queued = false;
        for (const Request &q : s->queue) queued |= q.ticket == ticket;
        *state = queued ? 0 : 1;
        return SILU_OK;
    }
    reap(s);
    *state = step_done(s, k) ? 3 : 2;
    if (*state == 3 && std::find(s->failed.begin(), s->failed.end(), k) != s->failed.end())
        return SILU_ERR_TIMEOUT;
    return SILU_OK;
}

int silu_server_completed(silu_server *s, int64_t *tickets, int capacity, int *count)
{
    if (!s || !count || capacity < 0 || (capacity > 0 && !tickets)) return SILU_ERR_ARG;
    reap(s);
    int k = 0;
    while (k < capacity && !s->done_queue.empty()) {
        tickets[k++] = s->done_queue.front();
        s->done_queue.pop_front();
    }
    *count = k;
    return SILU_OK;
}

int silu_server_times(silu_server *s, int64_t ticket, int64_t *submitted_ns, int64_t *done_ns)
{
    if (!s || !submitted_ns || !done_ns) return SILU_ERR_ARG;
    reap(s);
    auto it = s->recs.find(ticket);
    if (it == s->recs.end()) return SILU_ERR_ARG;
    *submitted_ns = it->second.submitted_ns;
    *done_ns = it->second.done_ns;
    return SILU_OK;
}

int silu_server_footprint(const silu_server *s, int64_t *records, int64_t *result_slots, int64_t *unreported)
{
    if (!s || !records || !result_slots || !unreported) return SILU_ERR_ARG;
    *records = (int64_t)s->recs.size();
    *result_slots = s->nresults;
    *unreported = (int64_t)s->done_queue.size();
    return SILU_OK;
}

int silu_server_wait(silu_server *s, int64_t ticket)
{
    if (!s || ticket < 0 || ticket >= s->next_ticket) return SILU_ERR_ARG;
    for (;;) {
        int state = 0;
        int st = silu_server_poll(s, ticket, &state);
        if (st) return st;
        if (state == 3) return SILU_OK;
        if (state == 2) { // its last launch is enqueued: wait for that step's event
            const int64_t k = s->recs.at(ticket).finish_step;
            hipError_t e = hipSuccess;
            if (s->mode == 1) {
                e = hipEventSynchronize(s->ev[k % RING]);
            } else { // the step that finishes a request always records a mark
                auto m = std::find_if(s->marks.begin(), s->marks.end(),
                                      [k](const std::pair<int64_t, int> &v) { return v.first >= k; });
                e = m != s->marks.end() ? hipEventSynchronize(s->ev[m->second]) : hipStreamSynchronize(s->stream);
                if (e == hipSuccess && m == s->marks.end()) s->completed_through = s->steps - 1;
            }
            if (e != hipSuccess) return fail(s, e);
            continue;
        }
        if ((st = silu_server_step(s, nullptr, nullptr))) return st; // queued or running: advance
    }
}

int silu_server_set_wait_limit(silu_server *s, int microseconds)
{
    if (!s || microseconds < 0) return SILU_ERR_ARG;
    s->wait_us = microseconds ? microseconds : PERSIST_WAIT_US;
    return SILU_OK;
}

int silu_server_set_mode(silu_server *s, int mode, int max_workgroups)
{
    if (!s || (mode != SILU_SERVE_STEPWISE && mode != SILU_SERVE_PERSISTENT) || max_workgroups < 0 ||
        max_workgroups > 65535)
        return SILU_ERR_ARG;
    reap(s);
    if (!s->queue.empty() || !s->active.empty()) return SILU_ERR_ARG;
    if (s->mode == 0) { // steps after the last mark are not tracked: finish them
        const hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return fail(s, e);
        s->completed_through = s->steps - 1;
        reap(s);
    }
    if (s->completed_through + 1 < s->steps) return SILU_ERR_ARG;
    if (mode == SILU_SERVE_PERSISTENT && !PERSISTENT_AVAILABLE) return SILU_ERR_UNSUPPORTED;
    if (mode == SILU_SERVE_PERSISTENT) {
        const int st = create_persistent(s);
        if (st) return st;
    }
    s->mode = mode == SILU_SERVE_PERSISTENT ? 1 : 0;
    s->max_wg = max_workgroups ? max_workgroups : DEFAULT_MAX_WG;
    return SILU_OK;
}

int silu_server_last_hip_error(const silu_server *s) { return s ? (int)s->last : 0; }

} // extern "C"
