// C-ABI of libscaledilu.so: argument checks, context, level analysis,
// per-kernel timing and the launch sequences of the smoother.
//
// One smoothing step (Algorithm 2 with the row scaling of eqs. extractD and
// newD folded into U, eq. ILUsplit) is the launch sequence
//     r = b - A x                          (1 launch; fused D^{-1} when m_L = 1)
//     y_k = r - Ls y_{k-1},  k = 2..m_L     (y_1 = r costs nothing; the last
//                                            launch writes s = D^{-1} y)
//     z_k = s - Us z_{k-1},  k = 2..m_U     (z_1 = s; the last launch does x += z)
// so 1 + (m_L - 1) + (m_U - 1) launches, each streaming one CSR matrix once.
#include <algorithm>
#include <array>
#include <climits>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/scaled_ilu.h"
#include "internal.h"

using namespace silu;

namespace {

struct LevelInfo {
    int32_t *d_perm = nullptr;
    int lanes = 1;                  // lanes per row of the level kernel
    std::vector<int32_t> level_ptr; // [depth + 1], host
    std::vector<int64_t> level_nnz; // off-diagonal entries per level, host
    int depth = 0;
};

using LevelKey = std::tuple<const void *, const void *, int64_t, int64_t, int>;

struct Partition {
    int32_t *d_blk = nullptr; // [nblk + 1] row starts
    int nblk = 0;
};
using PartKey = std::tuple<const void *, int64_t, int64_t, int>;

// 16-bit block-relative column offsets of one matrix for one rows-per-block.
struct Compressed {
    uint16_t *d = nullptr;   // 16-bit offsets (OFF16)
    int shift = 0;
    bool ok = false;
    uint16_t *slot = nullptr; // LDS slot codes (windowed), or null
    int32_t *wo = nullptr;    // windowed: block-relative offset of each slot
    int lw = 0;
    bool win_tried = false;
    int range_hi = 0; // largest block-relative offset (shift is the smallest)
};
using CompKey = std::tuple<const void *, const void *, int64_t, int64_t, int>;

// Sliced-ELL copy of one matrix's values (and its codes), keyed by the
// structure and value pointers, the sizes, the value size and the smallest
// code width allowed.
struct Sliced {
    SlicedView v;
    int32_t *sptr = nullptr, *sk = nullptr, *dtab = nullptr, *ptab = nullptr;
    uint8_t *pid = nullptr;
    uint16_t *ltab = nullptr;
    int32_t *wflag = nullptr;
    void *val = nullptr, *codes = nullptr;
    int64_t masked_rows = 0;
    bool ok = false;
};
using SlicedKey = std::tuple<const void *, const void *, const void *, int64_t, int64_t, int, int>;

// Locality-relabeled copies of A and the factors (SILU_REORDER), keyed by the
// pointers of A, Ls, Us, dinv, the second vector (d or d_c) and the FP32 copies.
struct Reorder {
    int32_t *order = nullptr, *pos = nullptr; // device [n]
    silu_csr A2{}, L2{}, U2{};                // relabeled copies (arrays owned here)
    double *dinv2 = nullptr, *aux2 = nullptr; // dinv, and d (unscaled) or d_c (row/column), relabeled
    float *L32 = nullptr, *U32 = nullptr;     // relabeled FP32 values, when the factors carry them
};
using ReorderKey = std::array<uintptr_t, 13>;

void free_csr_copy(silu_csr &M)
{
    (void)hipFree(M.row_ptr);
    (void)hipFree(M.col_idx);
    (void)hipFree(M.val);
    M = silu_csr();
}

void free_reorder(Reorder &R)
{
    (void)hipFree(R.order);
    (void)hipFree(R.pos);
    free_csr_copy(R.A2);
    free_csr_copy(R.L2);
    free_csr_copy(R.U2);
    (void)hipFree(R.dinv2);
    (void)hipFree(R.aux2);
    (void)hipFree(R.L32);
    (void)hipFree(R.U32);
    R = Reorder();
}

void free_sliced(Sliced &S)
{
    (void)hipFree(S.sptr);
    (void)hipFree(S.sk);
    (void)hipFree(S.dtab);
    (void)hipFree(S.val);
    (void)hipFree(S.codes);
    (void)hipFree(S.ptab);
    (void)hipFree(S.pid);
    (void)hipFree(S.ltab);
    (void)hipFree(S.wflag);
    S = Sliced();
}

void free_compressed(Compressed &C)
{
    (void)hipFree(C.d);
    (void)hipFree(C.slot);
    (void)hipFree(C.wo);
    C.d = C.slot = nullptr;
    C.wo = nullptr;
}

// A captured level sequence: one kernel node per level.
using GraphKey = std::tuple<const void *, const void *, const void *, const void *, const void *, const void *,
                            const void *, const void *, const void *, const void *, int>;

struct Pending {
    int kid;
    hipEvent_t e0, e1;
    double bytes, layout;
};

// A recorded smoother call: the arguments that fix its launch sequence.
using SmoothKey = std::array<uintptr_t, 24>;
struct SmoothGraph {
    hipGraphExec_t ex = nullptr; // null: the sequence could not be recorded
    double bytes = 0.0, layout = 0.0;
};

} // namespace

struct silu_ctx {
    int device = 0;
    void *scratch = nullptr; // this device's copy of the no-allocation scratch array (device address)
    bool no_build = false;   // inside ilu_smooth_noalloc: build no layout, record no timing
    hipStream_t stream = nullptr;
    int64_t bad_row = -1;
    hipError_t last_hip = hipSuccess;
    int32_t *d_flags = nullptr; // [4] device status words
    std::map<LevelKey, LevelInfo> levels;
    std::map<PartKey, Partition> parts;
    std::map<CompKey, Compressed> comp;
    std::map<SlicedKey, Sliced> sliced;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::map<SmoothKey, SmoothGraph> smooth_graphs;
    std::map<ReorderKey, Reorder> reorders;
    hipStream_t capture_stream = nullptr; // private, default priority, for graph capture
    bool recording = false;               // launches go into a capture: add up their bytes
    double rec_bytes = 0.0, rec_layout = 0.0;
    bool timing = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    std::vector<std::string> knames;
    std::vector<int64_t> klaunch;
    std::vector<double> kms, kbytes, klayout;
};

namespace {

int hip_fail(silu_ctx *c, hipError_t e)
{
    c->last_hip = e;
    return SILU_ERR_HIP;
}

#define HIPCHK(ctx, expr)                                                                                           \
    do {                                                                                                            \
        hipError_t _e = (expr);                                                                                     \
        if (_e != hipSuccess) return hip_fail((ctx), _e);                                                           \
    } while (0)

int kernel_id(silu_ctx *c, const char *name)
{
    for (size_t i = 0; i < c->knames.size(); i++)
        if (c->knames[i] == name) return (int)i;
    c->knames.emplace_back(name);
    c->klaunch.push_back(0);
    c->kms.push_back(0.0);
    c->kbytes.push_back(0.0);
    c->klayout.push_back(0.0);
    return (int)c->knames.size() - 1;
}

hipError_t get_event(silu_ctx *c, hipEvent_t *e)
{
    if (!c->free_events.empty()) {
        *e = c->free_events.back();
        c->free_events.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Launch through `fn(const char** name)`, bracketed by timing events when on.
// bytes: the launch's algorithmic bytes; layout: the bytes its data layout
// actually moves (differs from bytes only for compressed sweep layouts).
template <class F>
int timed_launch(silu_ctx *c, double bytes, double layout, F &&fn)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timing = c->timing && !c->no_build;
    if (timing) {
        HIPCHK(c, get_event(c, &e0));
        HIPCHK(c, get_event(c, &e1));
        HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    const char *name = "kernel";
    hipError_t err = fn(&name);
    if (err != hipSuccess) return hip_fail(c, err);
    if (c->recording) {
        c->rec_bytes += bytes;
        c->rec_layout += layout;
    }
    if (timing) {
        HIPCHK(c, hipEventRecord(e1, c->stream));
        c->pending.push_back({kernel_id(c, name), e0, e1, bytes, layout});
    }
    return SILU_OK;
}

template <class F>
int timed_launch(silu_ctx *c, double bytes, F &&fn)
{
    return timed_launch(c, bytes, bytes, fn);
}

bool csr_ok(const silu_csr *M, int dtype)
{
    return M && M->row_ptr && M->n_rows > 0 && M->n_rows < INT32_MAX && M->n_rows == M->n_cols && M->nnz >= 0 &&
           M->nnz < INT32_MAX && (M->nnz == 0 || (M->col_idx && M->val)) && M->dtype == dtype;
}

int check_square(const silu_csr *M, int dtype)
{
    if (!M || !M->row_ptr || (M->nnz > 0 && (!M->col_idx || !M->val))) return SILU_ERR_ARG;
    if (M->n_rows != M->n_cols) return SILU_ERR_SHAPE;
    if (!csr_ok(M, dtype)) return SILU_ERR_ARG;
    return SILU_OK;
}

// Host-side structural check (SILU_VALIDATE).  side: 0 any, -1 strictly
// lower, +1 strictly upper, 2 upper with the diagonal first.
int validate(silu_ctx *c, const silu_csr *M, int side)
{
    const int64_t n = M->n_rows;
    std::vector<int32_t> rp((size_t)n + 1), col((size_t)std::max<int64_t>(M->nnz, 1));
    HIPCHK(c, hipMemcpyAsync(rp.data(), M->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, c->stream));
    if (M->nnz) HIPCHK(c, hipMemcpyAsync(col.data(), M->col_idx, (size_t)M->nnz * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (rp[0] != 0 || rp[(size_t)n] != M->nnz) {
        c->bad_row = 0;
        return SILU_ERR_PATTERN;
    }
    for (int64_t i = 0; i < n; i++) {
        const int32_t a = rp[(size_t)i], b = rp[(size_t)i + 1];
        bool bad = b < a;
        for (int32_t p = a; !bad && p < b; p++) {
            const int32_t j = col[(size_t)p];
            bad = j < 0 || j >= n || (p > a && j <= col[(size_t)p - 1]) || (side == -1 && j >= i) ||
                  (side == 1 && j <= i) || (side == 2 && (p == a ? j != i : j <= i));
        }
        if (side == 2 && b <= a) bad = true;
        if (bad) {
            c->bad_row = i;
            return SILU_ERR_PATTERN;
        }
    }
    return SILU_OK;
}

struct Ws {
    char *base;
    size_t vec; // bytes per vector slot
    void *slot(int k) const { return base + (size_t)k * vec; }
};

size_t ws_vec_bytes(int64_t n) { return (((size_t)n * 8 + 255) / 256) * 256; }

// Bytes of a sweep's epilogue (and of the unscaled variant's diagonal term).
double epi_bytes(Prec p, int64_t n, int epi, bool dshift)
{
    double ob = 8;
    if (p == Prec::MIX_RES || p == Prec::MIX_L || p == Prec::MIX_U || p == Prec::MIX_L1) ob = 4;
    double b = 0.0;
    switch (epi) {
    case EPI_STORE:
    case EPI_SPMV: b = n * ob; break;
    case EPI_STORE_SPLIT: b = n * (ob + 4.0); break;
    case EPI_SCALE: b = n * (8.0 + ob); break;
    case EPI_UPDATE: b = n * 16.0; break;
    default: b = n * 24.0; break;
    }
    if (dshift) b += 8.0 * n;
    return b;
}

// Bytes of a CSR sweep: each entry (value + ib bytes of index) and the row
// pointers read once, the gathered iterate and the rhs once.  With ib = 4
// (the int32 column) these are the sweep's algorithmic bytes.
double sweep_bytes(Prec p, int64_t n, int64_t nnz, int epi, bool dshift, double ib)
{
    double vb = 8, xb = 8, rb = 8;
    if (p == Prec::MIX_L) vb = xb = 4;
    if (p == Prec::MIX_U) vb = xb = rb = 4;
    if (p == Prec::MIX_L1) vb = 4;
    return 4.0 * (double)(n + 1) + (double)nnz * (vb + ib) + (double)n * (xb + rb) + epi_bytes(p, n, epi, dshift);
}

// Row-block partition for the blocked CSR-stream kernel, made on first use
// (the row pointers are copied to the host) and cached per matrix.
int get_partition(silu_ctx *c, const silu_csr *M, int cap, int rmax, Partition **out)
{
    PartKey key{M->row_ptr, M->n_rows, M->nnz, cap * 4096 + rmax};
    auto it = c->parts.find(key);
    if (it != c->parts.end()) {
        *out = &it->second;
        return SILU_OK;
    }
    if (c->no_build) return SILU_ERR_UNSUPPORTED; // the partition is made on the host and allocated
    const int64_t n = M->n_rows;
    std::vector<int32_t> rp((size_t)n + 1);
    HIPCHK(c, hipMemcpyAsync(rp.data(), M->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // (row start, entry start) of every block, then the end sentinel
    std::vector<int32_t> blk{0, rp[0]};
    int64_t r = 0;
    while (r < n) {
        const int64_t start = r;
        if (rp[(size_t)r + 1] - rp[(size_t)r] > cap) {
            r++;
        } else {
            int64_t cnt = 0;
            while (r < n && r - start < rmax && cnt + (rp[(size_t)r + 1] - rp[(size_t)r]) <= cap) {
                cnt += rp[(size_t)r + 1] - rp[(size_t)r];
                r++;
            }
        }
        blk.push_back((int32_t)r);
        blk.push_back(rp[(size_t)r]);
    }
    Partition P;
    P.nblk = (int)blk.size() / 2 - 1;
    HIPCHK(c, hipMalloc(&P.d_blk, blk.size() * 4));
    hipError_t e = hipMemcpy(P.d_blk, blk.data(), blk.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(P.d_blk);
        return hip_fail(c, e);
    }
    auto res = c->parts.emplace(key, P);
    *out = &res.first->second;
    return SILU_OK;
}

// Block-relative 16-bit column offsets, made on first use on the device (one
// synchronous read of the offset range) and cached per matrix; ok = false
// when some offset does not fit 16 bits.
// win_policy: 0 never build the window codes, 1 only when 16-bit offsets do
// not fit, 2 always try.
int get_compressed(silu_ctx *c, const silu_csr *M, int rpb, int win_policy, Compressed **out)
{
    CompKey key{M->row_ptr, M->col_idx, M->n_rows, M->nnz, rpb};
    auto it = c->comp.find(key);
    if (c->no_build) { // what is cached, as it is; else plain 32-bit columns
        static Compressed none;
        *out = it != c->comp.end() ? &it->second : &none;
        return SILU_OK;
    }
    Compressed *C = nullptr;
    int32_t range[2] = {INT32_MAX, INT32_MIN};
    if (it != c->comp.end()) {
        C = &it->second;
        if (win_policy == 0 || (win_policy == 1 && C->ok) || C->win_tried) {
            *out = C;
            return SILU_OK;
        }
        range[0] = C->shift;
        range[1] = C->range_hi;
    } else {
        HIPCHK(c, launch_init_flags(c->d_flags, 1, INT32_MAX, c->stream));
        HIPCHK(c, launch_init_flags(c->d_flags + 1, 1, INT32_MIN, c->stream));
        HIPCHK(c, launch_offset_range((int)M->n_rows, M->row_ptr, M->col_idx, rpb, c->d_flags, c->stream));
        HIPCHK(c, hipMemcpyAsync(range, c->d_flags, sizeof(range), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        Compressed fresh;
        fresh.shift = range[0];
        fresh.range_hi = range[1];
        if (range[0] <= range[1] && (int64_t)range[1] - (int64_t)range[0] <= 65535) {
            HIPCHK(c, hipMalloc(&fresh.d, (size_t)M->nnz * sizeof(uint16_t)));
            hipError_t e = launch_compress16((int)M->n_rows, M->row_ptr, M->col_idx, rpb, fresh.shift, fresh.d,
                                             c->stream);
            if (e != hipSuccess) {
                (void)hipFree(fresh.d);
                return hip_fail(c, e);
            }
            fresh.ok = true;
        }
        C = &c->comp.emplace(key, fresh).first->second;
    }
    *out = C;
    if (win_policy == 0 || (win_policy == 1 && C->ok)) return SILU_OK;
    // windowed codes: number the offsets that occur; worth it only when they are few
    C->win_tried = true;
    const int64_t span = (int64_t)range[1] - (int64_t)range[0] + 1;
    if (range[0] > range[1] || span > (int64_t)1 << 24) return SILU_OK;
    uint8_t *d_used = nullptr;
    const int64_t span8 = (span + 7) / 8; // cleared as doubles (+0.0 is all zero bits) by a fill kernel
    HIPCHK(c, hipMalloc(&d_used, (size_t)span8 * 8));
    hipError_t e = launch_fill((int)span8, (double *)d_used, 0.0, nullptr, 0.0, c->stream);
    if (e == hipSuccess)
        e = launch_mark_offsets((int)M->n_rows, M->row_ptr, M->col_idx, rpb, range[0], d_used, c->stream);
    std::vector<uint8_t> used((size_t)span);
    if (e == hipSuccess) e = hipMemcpyAsync(used.data(), d_used, (size_t)span, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d_used);
    if (e != hipSuccess) return hip_fail(c, e);
    std::vector<int32_t> slot_of((size_t)span, -1), wo;
    for (int64_t t = 0; t < span; t++) {
        if (!used[(size_t)t]) continue;
        if ((int)wo.size() >= WIN_MAX_SLOTS) return SILU_OK; // too many: keep the other modes
        slot_of[(size_t)t] = (int32_t)wo.size();
        wo.push_back((int32_t)(t + range[0]));
    }
    if (wo.empty()) return SILU_OK;
    int32_t *d_slot_of = nullptr;
    HIPCHK(c, hipMalloc(&d_slot_of, (size_t)span * 4));
    e = hipMemcpyAsync(d_slot_of, slot_of.data(), (size_t)span * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMalloc(&C->wo, wo.size() * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(C->wo, wo.data(), wo.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMalloc(&C->slot, (size_t)M->nnz * sizeof(uint16_t));
    if (e == hipSuccess)
        e = launch_encode_slots((int)M->n_rows, M->row_ptr, M->col_idx, rpb, range[0], d_slot_of, C->slot,
                                c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream); // the host tables go out of scope
    (void)hipFree(d_slot_of);
    if (e != hipSuccess) {
        (void)hipFree(C->wo);
        (void)hipFree(C->slot);
        C->wo = nullptr;
        C->slot = nullptr;
        return hip_fail(c, e);
    }
    C->lw = (int)wo.size();
    return SILU_OK;
}

// Row patterns of N: the distinct sequences of offsets col - row (a row's
// pattern includes its length).  Fills pid[r] (rows past n: 0) and the table
// of offsets, kp per pattern, each pattern's last offset repeated into its
// padded slots (an empty row: offset 0).  False when there are more than 256
// patterns or the table would exceed PAT_MAX_ENTRIES offsets.
bool row_patterns(int64_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &col, int kp,
                  std::vector<uint8_t> &pid, std::vector<int32_t> &ptab, int *npat)
{
    std::unordered_map<uint64_t, std::vector<int>> by_hash;
    std::vector<int64_t> first_row; // a row holding each pattern
    pid.assign((size_t)((n + 63) / 64 * 64), 0);
    for (int64_t r = 0; r < n; r++) {
        const int32_t a = rp[(size_t)r], b = rp[(size_t)r + 1];
        uint64_t h = 1469598103934665603ull ^ (uint64_t)(b - a);
        for (int32_t e = a; e < b; e++) h = (h ^ (uint64_t)(uint32_t)(col[(size_t)e] - (int32_t)r)) * 1099511628211ull;
        auto &cands = by_hash[h];
        int found = -1;
        for (int p : cands) {
            const int64_t q = first_row[(size_t)p];
            const int32_t qa = rp[(size_t)q], qb = rp[(size_t)q + 1];
            if (qb - qa != b - a) continue;
            bool same = true;
            for (int32_t k = 0; k < b - a && same; k++)
                same = col[(size_t)(qa + k)] - (int32_t)q == col[(size_t)(a + k)] - (int32_t)r;
            if (same) {
                found = p;
                break;
            }
        }
        if (found < 0) {
            found = (int)first_row.size();
            if (found >= 256 || (int64_t)(found + 1) * kp > PAT_MAX_ENTRIES) return false;
            first_row.push_back(r);
            cands.push_back(found);
        }
        pid[(size_t)r] = (uint8_t)found;
    }
    *npat = (int)first_row.size();
    ptab.assign((size_t)*npat * (size_t)kp, 0);
    for (int p = 0; p < *npat; p++) {
        const int64_t q = first_row[(size_t)p];
        const int32_t qa = rp[(size_t)q], len = rp[(size_t)q + 1] - qa;
        for (int k = 0; k < kp; k++)
            ptab[(size_t)p * kp + k] = len == 0 ? 0 : col[(size_t)(qa + std::min(k, len - 1))] - (int32_t)q;
    }
    return true;
}

// Iterate windows of a pattern table: its distinct offsets in ascending
// order, cut into runs that start at an even offset w and reach at most w +
// 64, so that lane l of a slice starting at row r0 finds every slot of row
// r0 + l in x[r0 + w .. r0 + w + 127] for the run holding the slot's offset.
// A run that fewer than 1/16 of the slices need (a rare fill offset) is
// dropped: every slice would load its window for a few slices' sake, so the
// slices needing it take the gather body instead (wflag[slice] = 0; the
// others 1).  ltab holds each pattern's kp slots as LDS elements in rows of
// kl = kp rounded up to 8 (the padding 0; all 0 for a pattern on a dropped
// run).  False when more than PAT_WIN_MAX runs are kept, or when they span
// more than 2^24 rows (the kernel addresses the span as one buffer of at
// most 2^31 bytes).
bool pattern_windows(const std::vector<int32_t> &ptab, int kp, const std::vector<uint8_t> &pid, int64_t n,
                     std::vector<int32_t> &wst, std::vector<uint16_t> &ltab, std::vector<int32_t> &wflag)
{
    std::vector<int32_t> offs(ptab);
    std::sort(offs.begin(), offs.end());
    offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
    std::vector<int32_t> run_start; // every run, kept or not
    for (int32_t o : offs) {
        if (!run_start.empty() && (int64_t)o - run_start.back() <= 64) continue;
        if (run_start.size() == 64) return false; // one bit per run below
        run_start.push_back((int32_t)((int64_t)o - ((int64_t)o & 1))); // rounded down to even
    }
    const size_t npat = ptab.size() / (size_t)kp, nslice = (size_t)((n + 63) / 64);
    auto run_of = [&](int32_t o) {
        return (int)(std::upper_bound(run_start.begin(), run_start.end(), o) - run_start.begin()) - 1;
    };
    std::vector<uint64_t> pat_runs(npat, 0);
    for (size_t p = 0; p < npat; p++)
        for (size_t k = 0; k < (size_t)kp; k++) pat_runs[p] |= 1ull << run_of(ptab[p * (size_t)kp + k]);
    std::vector<uint64_t> slice_runs(nslice, 0);
    for (int64_t r = 0; r < n; r++) slice_runs[(size_t)(r >> 6)] |= pat_runs[pid[(size_t)r]];
    std::vector<int64_t> need(run_start.size(), 0);
    for (uint64_t m : slice_runs)
        for (size_t c = 0; c < run_start.size(); c++) need[c] += (m >> c) & 1;
    uint64_t kept = 0;
    wst.clear();
    for (size_t c = 0; c < run_start.size(); c++)
        if (need[c] >= (int64_t)(nslice / 16)) {
            kept |= 1ull << c;
            wst.push_back(run_start[c]);
        }
    if (wst.empty() || (int)wst.size() > PAT_WIN_MAX) return false;
    if ((int64_t)wst.back() + 128 - wst.front() > (int64_t)1 << 24) return false;
    const size_t kl = (size_t)(kp + 7) / 8 * 8;
    ltab.assign(npat * kl, 0);
    for (size_t p = 0; p < npat; p++) {
        if (pat_runs[p] & ~kept) continue;
        for (size_t k = 0; k < (size_t)kp; k++) {
            const int32_t o = ptab[p * (size_t)kp + k];
            const int c = (int)(std::upper_bound(wst.begin(), wst.end(), o) - wst.begin()) - 1;
            ltab[p * kl + k] = (uint16_t)(128 * c + (o - wst[(size_t)c])); // in [128 c, 128 c + 64]
        }
    }
    wflag.assign(nslice, 0);
    for (size_t t = 0; t < nslice; t++) wflag[t] = (slice_runs[t] & ~kept) ? 0 : 1;
    return true;
}

// Diagonal slices of N (code 16) when every row lies on at most DIAG_MAX
// diagonals col - row and their slots (one per diagonal for every row, in
// 128-row slices) exceed the entries by at most 1/16: *built is then true.
int build_diag(silu_ctx *c, const silu_csr *N, const void *val, int vbytes, Sliced &S, bool *built)
{
    *built = false;
    const int n = (int)N->n_rows;
    if (n < 2 || N->nnz <= 0) return SILU_OK;
    int32_t range[2];
    HIPCHK(c, launch_init_flags(c->d_flags, 1, INT32_MAX, c->stream));
    HIPCHK(c, launch_init_flags(c->d_flags + 1, 1, INT32_MIN, c->stream));
    HIPCHK(c, launch_offset_range(n, N->row_ptr, N->col_idx, 1, c->d_flags, c->stream));
    HIPCHK(c, hipMemcpyAsync(range, c->d_flags, sizeof(range), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int64_t dlo = range[0], span = (int64_t)range[1] - range[0] + 1;
    if (span < 1 || span > (int64_t)1 << 24) return SILU_OK;
    uint8_t *d_used = nullptr;
    const int64_t span8 = (span + 7) / 8;
    HIPCHK(c, hipMalloc(&d_used, (size_t)span8 * 8));
    hipError_t e = launch_fill((int)span8, (double *)d_used, 0.0, nullptr, 0.0, c->stream);
    if (e == hipSuccess) e = launch_mark_offsets(n, N->row_ptr, N->col_idx, 1, (int)dlo, d_used, c->stream);
    std::vector<uint8_t> used((size_t)span);
    if (e == hipSuccess) e = hipMemcpyAsync(used.data(), d_used, (size_t)span, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d_used);
    if (e != hipSuccess) return hip_fail(c, e);
    std::vector<int32_t> dtab, dmap((size_t)span, 0);
    for (int64_t t = 0; t < span && (int)dtab.size() <= DIAG_MAX; t++) {
        if (!used[(size_t)t]) continue;
        dmap[(size_t)t] = (int32_t)dtab.size();
        dtab.push_back((int32_t)(t + dlo));
    }
    const int u = (int)dtab.size();
    const int nslice = (n + 127) / 128;
    const int64_t slots = (int64_t)nslice * u * 128;
    if (u > DIAG_MAX || slots > N->nnz + N->nnz / 16 + 128 * (int64_t)u || slots > INT32_MAX) return SILU_OK;
    int32_t *d_dmap = nullptr;
    e = hipMalloc(&S.val, (size_t)slots * (size_t)vbytes);
    if (e == hipSuccess) e = hipMalloc(&S.dtab, (size_t)u * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(S.dtab, dtab.data(), (size_t)u * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMalloc(&d_dmap, dmap.size() * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(d_dmap, dmap.data(), dmap.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_fill_diag(n, nslice, u, N->row_ptr, N->col_idx, val, vbytes, d_dmap, (int)dlo, S.val, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream); // the host tables go out of scope
    (void)hipFree(d_dmap);
    if (e != hipSuccess) {
        free_sliced(S);
        return hip_fail(c, e);
    }
    S.v = SlicedView();
    S.v.nslice = nslice;
    S.v.code = 16;
    S.v.val = S.val;
    S.v.dtab = S.dtab;
    S.v.ndiag = u;
    S.v.slots = slots;
    S.ok = true;
    *built = true;
    return SILU_OK;
}

// Build (once) the sliced-ELL copy of N with values `val` of `vbytes` bytes.
// code_min: -1 allows diagonal slices, 0 the row-pattern table,
// 1 the diagonal table, 2 starts at 16-bit offsets, 4 uses columns.  *out->ok
// is false when the matrix has no entries or the copy would not fit 32-bit
// slot indices (the caller then streams the CSR).
int build_sliced(silu_ctx *c, const silu_csr *N, const void *val, int vbytes, int code_min, Sliced &S)
{
    const int n = (int)N->n_rows;
    const int nslice = (n + 63) / 64;
    auto store = [&]() { return SILU_OK; }; // S.ok stays false unless the copy was built
    if (N->nnz <= 0 || n <= 0) return store();
    if (code_min < 0) {
        bool built = false;
        const int st = build_diag(c, N, val, vbytes, S, &built);
        if (st || built) return st;
    }
    // per-slice K and mask bit, then slot offsets
    HIPCHK(c, hipMalloc(&S.sk, (size_t)nslice * 4));
    hipError_t e = launch_slice_meta(n, nslice, N->row_ptr, S.sk, c->stream);
    std::vector<int32_t> sk((size_t)nslice), sptr((size_t)nslice);
    if (e == hipSuccess) e = hipMemcpyAsync(sk.data(), S.sk, (size_t)nslice * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        free_sliced(S);
        return hip_fail(c, e);
    }
    int64_t slots = 0;
    int gmax = 0;
    for (int t = 0; t < nslice; t++) {
        sptr[(size_t)t] = (int32_t)std::min<int64_t>(slots, INT32_MAX);
        slots += (int64_t)(sk[(size_t)t] & 0x7fffffff) * 64;
        gmax = std::max(gmax, (sk[(size_t)t] & 0x7fffffff) >> 2);
        if (sk[(size_t)t] < 0) S.masked_rows += 64;
    }
    // padding beyond 4x the entries (a few very long rows) is not worth the copy
    if (slots + 64 > INT32_MAX || slots > 4 * N->nnz + 64 * (int64_t)nslice) {
        free_sliced(S);
        return store();
    }
    // column codes: none when the rows follow at most 256 patterns (a table
    // of offsets per pattern and one byte per row), else the diagonal table
    // when at most 256 distinct col - row occur, else 16-bit slice-relative
    // offsets when they fit, else columns
    int code = 4, lo = 0;
    std::vector<int32_t> dtab, dmap, ptab;
    std::vector<uint8_t> pid;
    int npat = 0;
    int32_t range[2];
    if (code_min <= 0 && gmax >= 1 && gmax <= 8) { // the pattern kernels take up to 8 groups
        std::vector<int32_t> hrp((size_t)n + 1), hcol((size_t)N->nnz);
        e = hipMemcpyAsync(hrp.data(), N->row_ptr, hrp.size() * 4, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hcol.data(), N->col_idx, hcol.size() * 4, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            free_sliced(S);
            return hip_fail(c, e);
        }
        if (row_patterns(n, hrp, hcol, 4 * gmax, pid, ptab, &npat)) code = 8;
    }
    if (code == 4 && code_min <= 1) {
        HIPCHK(c, launch_init_flags(c->d_flags, 1, INT32_MAX, c->stream));
        HIPCHK(c, launch_init_flags(c->d_flags + 1, 1, INT32_MIN, c->stream));
        HIPCHK(c, launch_offset_range(n, N->row_ptr, N->col_idx, 1, c->d_flags, c->stream));
        HIPCHK(c, hipMemcpyAsync(range, c->d_flags, sizeof(range), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const int64_t dlo = std::min<int64_t>(range[0], 0), dhi = std::max<int64_t>(range[1], 0);
        const int64_t span = dhi - dlo + 1;
        if (span <= (int64_t)1 << 24) {
            uint8_t *d_used = nullptr;
            const int64_t span8 = (span + 7) / 8;
            HIPCHK(c, hipMalloc(&d_used, (size_t)span8 * 8));
            e = launch_fill((int)span8, (double *)d_used, 0.0, nullptr, 0.0, c->stream);
            if (e == hipSuccess) e = launch_mark_offsets(n, N->row_ptr, N->col_idx, 1, (int)dlo, d_used, c->stream);
            std::vector<uint8_t> used((size_t)span);
            if (e == hipSuccess)
                e = hipMemcpyAsync(used.data(), d_used, (size_t)span, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            (void)hipFree(d_used);
            if (e != hipSuccess) {
                free_sliced(S);
                return hip_fail(c, e);
            }
            used[(size_t)(0 - dlo)] = 1; // the empty rows' padding reads diagonal 0
            int64_t cnt = 0;
            for (int64_t t = 0; t < span && cnt <= 256; t++) cnt += used[(size_t)t];
            if (cnt <= 256) {
                dmap.assign((size_t)span, 0);
                for (int64_t t = 0; t < span; t++) {
                    if (!used[(size_t)t]) continue;
                    dmap[(size_t)t] = (int32_t)dtab.size();
                    dtab.push_back((int32_t)(t + dlo));
                }
                code = 1;
                lo = (int)dlo;
            }
        }
    }
    if (code == 4 && code_min <= 2) {
        HIPCHK(c, launch_init_flags(c->d_flags, 1, INT32_MAX, c->stream));
        HIPCHK(c, launch_init_flags(c->d_flags + 1, 1, INT32_MIN, c->stream));
        HIPCHK(c, launch_offset_range(n, N->row_ptr, N->col_idx, 64, c->d_flags, c->stream));
        HIPCHK(c, hipMemcpyAsync(range, c->d_flags, sizeof(range), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const int64_t olo = std::min<int64_t>(range[0], 0), ohi = std::max<int64_t>(range[1], 63);
        if (ohi - olo <= 65535) {
            code = 2;
            lo = (int)olo;
        }
    }
    // a matrix without diagonal or offset structure gathers at random either
    // way; unless 4-byte codes were asked for, the CSR stream (no padding) is
    // used for it instead
    if (code == 4 && code_min < 4) {
        free_sliced(S);
        return store();
    }
    int32_t *d_dmap = nullptr;
    e = hipMalloc(&S.sptr, (size_t)nslice * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(S.sptr, sptr.data(), (size_t)nslice * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMalloc(&S.val, (size_t)slots * (size_t)vbytes);
    if (e == hipSuccess && code != 8) e = hipMalloc(&S.codes, (size_t)slots * (size_t)code);
    std::vector<int32_t> wst, wflag;
    std::vector<uint16_t> ltab;
    if (e == hipSuccess && code == 8) {
        e = hipMalloc(&S.ptab, ptab.size() * 4);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S.ptab, ptab.data(), ptab.size() * 4, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipMalloc(&S.pid, pid.size());
        if (e == hipSuccess) e = hipMemcpyAsync(S.pid, pid.data(), pid.size(), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && pattern_windows(ptab, 4 * gmax, pid, n, wst, ltab, wflag)) {
            e = hipMalloc(&S.ltab, ltab.size() * 2);
            if (e == hipSuccess)
                e = hipMemcpyAsync(S.ltab, ltab.data(), ltab.size() * 2, hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = hipMalloc(&S.wflag, wflag.size() * 4);
            if (e == hipSuccess)
                e = hipMemcpyAsync(S.wflag, wflag.data(), wflag.size() * 4, hipMemcpyHostToDevice, c->stream);
        }
    }
    if (e == hipSuccess && code == 1) {
        e = hipMalloc(&S.dtab, dtab.size() * 4);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S.dtab, dtab.data(), dtab.size() * 4, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipMalloc(&d_dmap, dmap.size() * 4);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_dmap, dmap.data(), dmap.size() * 4, hipMemcpyHostToDevice, c->stream);
    }
    if (e == hipSuccess)
        e = launch_fill_sliced(n, nslice, N->row_ptr, N->col_idx, val, vbytes, S.sptr, S.sk, code, d_dmap, lo, S.val,
                               S.codes, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream); // the host tables go out of scope
    (void)hipFree(d_dmap);
    if (e != hipSuccess) {
        free_sliced(S);
        return hip_fail(c, e);
    }
    S.v.nslice = nslice;
    S.v.code = code;
    S.v.sptr = S.sptr;
    S.v.sk = S.sk;
    S.v.val = S.val;
    S.v.codes = S.codes;
    S.v.dtab = S.dtab;
    S.v.ndiag = (int)dtab.size();
    S.v.shift = lo;
    S.v.slots = slots;
    S.v.gmax = gmax;
    S.v.pid = S.pid;
    S.v.ptab = S.ptab;
    S.v.npat = npat;
    S.v.kp = code == 8 ? 4 * gmax : 0;
    if (S.ltab && S.wflag) {
        S.v.nwin = (int)wst.size();
        S.v.wspan = wst.back() + 128 - wst.front();
        S.v.kl = (4 * gmax + 7) / 8 * 8;
        std::copy(wst.begin(), wst.end(), S.v.wst);
        S.v.ltab = S.ltab;
        S.v.wflag = S.wflag;
    }
    S.ok = true;
    return store();
}

int get_sliced(silu_ctx *c, const silu_csr *N, const void *val, int vbytes, int code_min, Sliced **out)
{
    SlicedKey key{N->row_ptr, N->col_idx, val, N->n_rows, N->nnz, vbytes, code_min};
    auto it = c->sliced.find(key);
    if (it != c->sliced.end()) {
        *out = &it->second;
        return SILU_OK;
    }
    if (c->no_build) { // not cached: the caller streams the CSR arrays instead
        static Sliced none;
        *out = &none;
        return SILU_OK;
    }
    Sliced S;
    const int st = build_sliced(c, N, val, vbytes, code_min, S);
    if (st) {
        free_sliced(S); // whatever a failed build had allocated
        return st;
    }
    *out = &c->sliced.emplace(key, S).first->second;
    return SILU_OK;
}

int sweep(silu_ctx *c, Prec p, SweepGeom g, const silu_csr *N, const void *val, const void *xin,
          const void *rhs, int epi, void *out, const double *dinv, double *x, const double *dshift,
          const double *dcol = nullptr, float *out32 = nullptr)
{
    double sliced_bytes = -1.0;
    bool fell_back = false; // the default sliced layout did not apply
    // diagonal slices add no unscaled-variant diagonal term
    if (g.slice_code_min < 0 && dshift) g.slice_code_min = 0;
    if (g.kind == SweepKernel::SLICED) {
        const int vbytes = (p == Prec::F64 || p == Prec::MIX_RES) ? 8 : 4;
        Sliced *S = nullptr;
        int st = get_sliced(c, N, val, vbytes, g.slice_code_min, &S);
        if (st) return st;
        if (S->ok) {
            g.sl = S->v;
            const double xb = (p == Prec::MIX_L || p == Prec::MIX_U) ? 4.0 : 8.0;
            const double rb = p == Prec::MIX_U ? 4.0 : 8.0;
            // row patterns: one byte per row instead of codes; diagonal slices: neither, no slice table
            const int cb = (S->v.code == 8 || S->v.code == 16) ? 0 : S->v.code;
            sliced_bytes = (double)S->v.slots * (vbytes + cb) + (S->v.code == 16 ? 0.0 : 8.0 * S->v.nslice) +
                           8.0 * (double)S->masked_rows + (double)N->n_rows * (xb + rb) + 4.0 * S->v.ndiag +
                           (S->v.code == 8 ? (double)N->n_rows + 4.0 * S->v.npat * S->v.kp : 0.0);
        } else {
            g.kind = SweepKernel::STREAM; // no entries, too large for the sliced copy, or no structure
            fell_back = true;
        }
    }
    if (g.kind == SweepKernel::STREAM && g.allow16 && N->nnz > 0) {
        Compressed *C = nullptr;
        const int policy = !g.allow_win ? 0 : (g.prefer_win ? 2 : 1);
        int st = get_compressed(c, N, g.rows_per_block, policy, &C);
        if (st) return st;
        if (policy && C->lw > 0 && (g.prefer_win || !C->ok)) {
            g.slot16 = C->slot;
            g.wo = C->wo;
            g.lw = C->lw;
        } else if (C->ok) {
            g.off16 = C->d;
            g.shift = C->shift;
        } else if (fell_back && !c->no_build) {
            // no structure and no narrow column code: 32-bit columns either way; the row-block
            // partition (1,024 entries per workgroup, every load issued at once) streams
            // such matrices faster than CSR-stream (the relabeled random operator: 1.35 ms
            // against 1.41 ms per FP32-inner application)
            g.kind = SweepKernel::BLOCKED;
            g.cap = 1024;
        }
    }
    if (g.kind == SweepKernel::BLOCKED) {
        Partition *P = nullptr;
        int st = get_partition(c, N, g.cap, RB_RMAX, &P);
        if (st) return st;
        g.blk = P->d_blk;
        g.nblk = P->nblk;
    }
    SweepArgs a;
    a.n = (int)N->n_rows;
    a.rp = N->row_ptr;
    a.col = N->col_idx;
    a.val = val;
    a.xin = xin;
    a.rhs = rhs;
    a.epi = epi;
    a.out = out;
    a.dinv = dinv;
    a.x = x;
    a.dshift = dshift;
    if (epi == EPI_STORE_SPLIT) a.out32 = out32; // shares its place with x, which this epilogue does not use
    const bool upd = epi == EPI_UPDATE || epi == EPI_SCALE_UPDATE;
    a.dcol = upd ? dcol : nullptr;
    double bytes = sweep_bytes(p, N->n_rows, N->nnz, epi, dshift != nullptr, 4.0);
    double layout = sweep_bytes(p, N->n_rows, N->nnz, epi, dshift != nullptr, (g.off16 || g.lw) ? 2.0 : 4.0);
    if (sliced_bytes >= 0.0) // the sliced layout's own bytes: padded slots, codes, slice tables
        layout = sliced_bytes + epi_bytes(p, N->n_rows, epi, dshift != nullptr);
    const double adj = (epi == EPI_SPMV ? -(p == Prec::MIX_U ? 4.0 : 8.0) : 0.0) * (double)N->n_rows + // no rhs read
                       (a.dcol ? 8.0 : 0.0) * (double)N->n_rows;
    bytes += adj;
    layout += adj;
    return timed_launch(c, bytes, layout, [&](const char **nm) { return launch_sweep(p, g, a, c->stream, nm); });
}

// ---- locality relabeling (SILU_REORDER) ------------------------------------
// Relabeled copy of one CSR matrix: rows in `order`, entries in their original
// order, columns through pos.  h_rp: the matrix's row pointers on the host.
int relabel_csr(silu_ctx *c, const silu_csr *M, const std::vector<int32_t> &h_rp, const std::vector<int32_t> &h_order,
                const int32_t *order, const int32_t *pos, silu_csr *out, int32_t **rp2_out)
{
    const int64_t n = M->n_rows;
    std::vector<int32_t> rp2((size_t)n + 1, 0);
    for (int64_t k = 0; k < n; k++) {
        const int32_t i = h_order[(size_t)k];
        rp2[(size_t)k + 1] = rp2[(size_t)k] + (h_rp[(size_t)i + 1] - h_rp[(size_t)i]);
    }
    *out = *M;
    out->row_ptr = nullptr;
    out->col_idx = nullptr;
    out->val = nullptr;
    HIPCHK(c, hipMalloc((void **)&out->row_ptr, ((size_t)n + 1) * 4));
    HIPCHK(c, hipMalloc((void **)&out->col_idx, (size_t)std::max<int64_t>(M->nnz, 1) * 4));
    HIPCHK(c, hipMalloc(&out->val, (size_t)std::max<int64_t>(M->nnz, 1) * 8));
    HIPCHK(c, hipMemcpy(out->row_ptr, rp2.data(), ((size_t)n + 1) * 4, hipMemcpyHostToDevice));
    if (M->nnz > 0)
        HIPCHK(c, launch_relabel((int)n, order, pos, M->row_ptr, M->col_idx, M->val, 8, out->row_ptr, out->col_idx,
                                 out->val, c->stream));
    *rp2_out = out->row_ptr;
    return SILU_OK;
}

int get_reorder(silu_ctx *c, const silu_csr *A, const silu_factors *F, Reorder **out)
{
    const double *aux = F->scaled == 0 ? F->d : (F->scaled == 2 ? F->dc : nullptr);
    const ReorderKey key{(uintptr_t)A->row_ptr, (uintptr_t)A->col_idx, (uintptr_t)A->val,
                         (uintptr_t)F->Ls.row_ptr, (uintptr_t)F->Ls.col_idx, (uintptr_t)F->Ls.val,
                         (uintptr_t)F->Us.row_ptr, (uintptr_t)F->Us.col_idx, (uintptr_t)F->Us.val,
                         (uintptr_t)F->dinv, (uintptr_t)aux, (uintptr_t)F->Ls_val32, (uintptr_t)F->Us_val32};
    auto it = c->reorders.find(key);
    if (it != c->reorders.end()) {
        *out = &it->second;
        return SILU_OK;
    }
    const int64_t n = A->n_rows;
    // the order, from A's strong couplings (host)
    std::vector<int32_t> rpA((size_t)n + 1), colA((size_t)std::max<int64_t>(A->nnz, 1));
    std::vector<double> valA((size_t)std::max<int64_t>(A->nnz, 1));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(rpA.data(), A->row_ptr, rpA.size() * 4, hipMemcpyDeviceToHost));
    if (A->nnz > 0) {
        HIPCHK(c, hipMemcpy(colA.data(), A->col_idx, (size_t)A->nnz * 4, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(valA.data(), A->val, (size_t)A->nnz * 8, hipMemcpyDeviceToHost));
    }
    std::vector<int32_t> order((size_t)n), pos((size_t)n);
    int st = rcm_strength_order(n, rpA.data(), colA.data(), valA.data(), REORDER_THETA, order.data());
    if (st) return st;
    for (int64_t k = 0; k < n; k++) pos[(size_t)order[(size_t)k]] = (int32_t)k;
    colA = std::vector<int32_t>();
    valA = std::vector<double>();
    Reorder R;
    auto fail_free = [&](int code) {
        (void)hipStreamSynchronize(c->stream);
        free_reorder(R);
        return code;
    };
    hipError_t e = hipMalloc((void **)&R.order, (size_t)n * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&R.pos, (size_t)n * 4);
    if (e == hipSuccess) e = hipMemcpy(R.order, order.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(R.pos, pos.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_free(hip_fail(c, e));
    int32_t *rp2 = nullptr;
    if ((st = relabel_csr(c, A, rpA, order, R.order, R.pos, &R.A2, &rp2))) return fail_free(st);
    std::vector<int32_t> rp((size_t)n + 1);
    const silu_csr *fac[2] = {&F->Ls, &F->Us};
    silu_csr *dst[2] = {&R.L2, &R.U2};
    const float *f32[2] = {F->Ls_val32, F->Us_val32};
    float **d32[2] = {&R.L32, &R.U32};
    for (int t = 0; t < 2; t++) {
        if (!fac[t]->row_ptr) { // an absent factor (the Gauss-Seidel split has no U): nothing to own
            *dst[t] = silu_csr();
            dst[t]->n_rows = dst[t]->n_cols = fac[t]->n_rows;
            dst[t]->dtype = fac[t]->dtype;
            continue;
        }
        if ((e = hipMemcpy(rp.data(), fac[t]->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost)) != hipSuccess)
            return fail_free(hip_fail(c, e));
        if ((st = relabel_csr(c, fac[t], rp, order, R.order, R.pos, dst[t], &rp2))) return fail_free(st);
        if (f32[t] && fac[t]->nnz > 0) {
            if ((e = hipMalloc((void **)d32[t], (size_t)fac[t]->nnz * 4)) != hipSuccess) return fail_free(hip_fail(c, e));
            if ((e = launch_relabel((int)n, R.order, R.pos, fac[t]->row_ptr, nullptr, f32[t], 4, rp2, nullptr,
                                    *d32[t], c->stream)) != hipSuccess)
                return fail_free(hip_fail(c, e));
        }
    }
    if ((e = hipMalloc((void **)&R.dinv2, (size_t)n * 8)) != hipSuccess) return fail_free(hip_fail(c, e));
    if ((e = launch_gather((int)n, R.order, F->dinv, R.dinv2, c->stream)) != hipSuccess)
        return fail_free(hip_fail(c, e));
    if (aux) {
        if ((e = hipMalloc((void **)&R.aux2, (size_t)n * 8)) != hipSuccess) return fail_free(hip_fail(c, e));
        if ((e = launch_gather((int)n, R.order, aux, R.aux2, c->stream)) != hipSuccess)
            return fail_free(hip_fail(c, e));
    }
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return fail_free(hip_fail(c, e));
    *out = &c->reorders.emplace(key, R).first->second;
    return SILU_OK;
}

// The factors of F with every array replaced by its relabeled copy.
silu_factors relabeled_factors(const silu_factors *F, const Reorder *R)
{
    silu_factors F2 = *F;
    F2.Ls = R->L2;
    F2.Us = R->U2;
    F2.dinv = R->dinv2;
    if (F->scaled == 0) F2.d = R->aux2;
    if (F->scaled == 2) F2.dc = R->aux2;
    F2.Ls_val32 = R->L32;
    F2.Us_val32 = R->U32;
    return F2;
}

// ---- level analysis (Section 4: level-set scheduling) ----------------------
int get_levels(silu_ctx *c, const silu_csr *T, int uplo, LevelInfo **out)
{
    LevelKey key{T->row_ptr, T->col_idx, T->n_rows, T->nnz, uplo};
    auto it = c->levels.find(key);
    if (it != c->levels.end()) {
        *out = &it->second;
        return SILU_OK;
    }
    const int64_t n = T->n_rows;
    std::vector<int32_t> rp((size_t)n + 1), col((size_t)std::max<int64_t>(T->nnz, 1));
    HIPCHK(c, hipMemcpyAsync(rp.data(), T->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, c->stream));
    if (T->nnz) HIPCHK(c, hipMemcpyAsync(col.data(), T->col_idx, (size_t)T->nnz * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<int32_t> lev((size_t)n, 0);
    int32_t depth = 0;
    for (int64_t s = 0; s < n; s++) {
        const int64_t i = uplo == SILU_LOWER ? s : n - 1 - s;
        int32_t l = 0;
        for (int32_t p = rp[(size_t)i]; p < rp[(size_t)i + 1]; p++) {
            const int32_t j = col[(size_t)p];
            if (j == i) continue;
            if (j < 0 || j >= n || (uplo == SILU_LOWER ? j > i : j < i)) {
                c->bad_row = i;
                return SILU_ERR_PATTERN;
            }
            l = std::max(l, lev[(size_t)j] + 1);
        }
        lev[(size_t)i] = l;
        depth = std::max(depth, l + 1);
    }
    LevelInfo info;
    info.depth = depth;
    info.level_ptr.assign((size_t)depth + 1, 0);
    info.level_nnz.assign((size_t)depth, 0);
    for (int64_t i = 0; i < n; i++) {
        info.level_ptr[(size_t)lev[(size_t)i] + 1]++;
        int64_t off = 0;
        for (int32_t p = rp[(size_t)i]; p < rp[(size_t)i + 1]; p++) off += col[(size_t)p] != i;
        info.level_nnz[(size_t)lev[(size_t)i]] += off;
    }
    for (int32_t l = 0; l < depth; l++) info.level_ptr[(size_t)l + 1] += info.level_ptr[(size_t)l];
    {
        int64_t off = 0;
        for (int32_t l = 0; l < depth; l++) off += info.level_nnz[(size_t)l];
        const double mean = n > 0 ? (double)off / (double)n : 0.0;
        info.lanes = mean <= 2.0 ? 1 : (mean <= 6.0 ? 4 : (mean <= 12.0 ? 8 : (mean <= 24.0 ? 16 : 32)));
    }
    std::vector<int32_t> perm((size_t)n), fill(info.level_ptr.begin(), info.level_ptr.end() - 1);
    for (int64_t i = 0; i < n; i++) perm[(size_t)fill[(size_t)lev[(size_t)i]]++] = (int32_t)i;
    HIPCHK(c, hipMalloc(&info.d_perm, (size_t)n * 4));
    hipError_t e = hipMemcpy(info.d_perm, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(info.d_perm);
        return hip_fail(c, e);
    }
    auto res = c->levels.emplace(key, std::move(info));
    *out = &res.first->second;
    return SILU_OK;
}

// Enqueue every level of a level-scheduled substitution on stream s.
hipError_t enqueue_levels(const LevelArgs &a, const LevelInfo *li, int unit, hipStream_t s)
{
    for (int l = 0; l < li->depth; l++) {
        const int start = li->level_ptr[(size_t)l], count = li->level_ptr[(size_t)l + 1] - start;
        hipError_t e = launch_level(a, unit, li->lanes, start, count, s, nullptr);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int run_levels(silu_ctx *c, const silu_csr *T, LevelInfo *li, int unit, const double *rhs, double *out,
               const double *dinv, double *s_out, double *xupd, bool graph, const double *dcol = nullptr)
{
    const double xb = dcol ? 24.0 : 16.0; // bytes per row of the x update
    if (graph && li->depth > 1) {
        LevelArgs a;
        a.perm = li->d_perm;
        a.rp = T->row_ptr;
        a.col = T->col_idx;
        a.val = (const double *)T->val;
        a.rhs = rhs;
        a.out = out;
        a.dinv = dinv;
        a.s_out = s_out;
        a.xupd = xupd;
        a.dcol = dcol;
        GraphKey key{li, T->row_ptr, T->col_idx, T->val, rhs, out, dinv, s_out, xupd, dcol, unit};
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            if (!c->capture_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
            HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_levels(a, li, unit, c->capture_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(c->capture_stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(c, e != hipSuccess ? e : e2);
            }
            hipGraphExec_t ex = nullptr;
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(c, e);
            it = c->graphs.emplace(key, ex).first;
        }
        double bytes = 0.0;
        for (int l = 0; l < li->depth; l++) {
            const int count = li->level_ptr[(size_t)l + 1] - li->level_ptr[(size_t)l];
            bytes += count * (4.0 + 8.0 + 8.0 + 8.0 + 8.0) + 12.0 * (double)li->level_nnz[(size_t)l];
            if (s_out) bytes += count * 16.0;
            if (xupd) bytes += count * xb;
        }
        hipGraphExec_t ex = it->second;
        return timed_launch(c, bytes, [&](const char **nm) {
            *nm = "level_graph";
            return hipGraphLaunch(ex, c->stream);
        });
    }
    LevelArgs a;
    a.perm = li->d_perm;
    a.rp = T->row_ptr;
    a.col = T->col_idx;
    a.val = (const double *)T->val;
    a.rhs = rhs;
    a.out = out;
    a.dinv = dinv;
    a.s_out = s_out;
    a.xupd = xupd;
    a.dcol = dcol;
    for (int l = 0; l < li->depth; l++) {
        const int start = li->level_ptr[(size_t)l], count = li->level_ptr[(size_t)l + 1] - start;
        double bytes = count * (4.0 + 8.0 + 8.0 + 8.0 + 8.0) + 12.0 * (double)li->level_nnz[(size_t)l];
        if (s_out) bytes += count * 16.0;
        if (xupd) bytes += count * xb;
        int st = timed_launch(c, bytes, [&](const char **nm) {
            return launch_level(a, unit, li->lanes, start, count, c->stream, nm);
        });
        if (st) return st;
    }
    return SILU_OK;
}

int check_finite(silu_ctx *c, int64_t n, const double *x)
{
    HIPCHK(c, launch_init_flags(c->d_flags, 4, INT32_MAX, c->stream));
    HIPCHK(c, launch_finite_check((int)n, x, c->d_flags, c->stream));
    int32_t h[4];
    HIPCHK(c, hipMemcpyAsync(h, c->d_flags, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h[2] != INT32_MAX) {
        c->bad_row = h[2];
        return SILU_ERR_NONFINITE;
    }
    return SILU_OK;
}

} // namespace

namespace silu {

int make_owned_sliced(silu_ctx *c, const silu_csr *N, const void *val, int vbytes, SlicedView *view, void **owner)
{
    *view = SlicedView();
    *owner = nullptr;
    if (vbytes != 8 && vbytes != 4) return SILU_ERR_ARG;
    Sliced *S = new (std::nothrow) Sliced();
    if (!S) return SILU_ERR_NOMEM;
    const int st = build_sliced(c, N, val, vbytes, 0, *S);
    if (st || !S->ok) {
        free_sliced(*S);
        delete S;
        return st;
    }
    *view = S->v;
    *owner = S;
    return SILU_OK;
}

void free_owned_sliced(void *owner)
{
    if (!owner) return;
    Sliced *S = (Sliced *)owner;
    free_sliced(*S);
    delete S;
}

} // namespace silu

// Scratch memory of ilu_smooth_noalloc: one array per device, made with the
// code object (nothing is allocated for it at run time) and held until the
// process ends.  Its device address differs per device and is looked up once
// per device, with that device current, when the first context on it is
// created; host code uses only that address, never the array's own name.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};

// The scratch array's address on the current device (resolved once), or null.
void *scratch_address(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[device] = p;
        else (void)hipGetLastError(); // the no-allocation entry point then reports HIP
    }
    return g_scratch[device];
}

} // namespace

extern "C" {

int silu_create(silu_ctx **ctx, void *hip_stream)
{
    if (!ctx) return SILU_ERR_ARG;
    *ctx = nullptr;
    silu_ctx *c = new (std::nothrow) silu_ctx();
    if (!c) return SILU_ERR_NOMEM;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc(&c->d_flags, 4 * sizeof(int32_t));
    if (e != hipSuccess) {
        delete c;
        return SILU_ERR_HIP;
    }
    c->scratch = scratch_address(c->device);
    *ctx = c;
    return SILU_OK;
}

int silu_destroy(silu_ctx *c)
{
    if (!c) return SILU_ERR_ARG;
    (void)hipStreamSynchronize(c->stream);
    for (auto &kv : c->levels) (void)hipFree(kv.second.d_perm);
    for (auto &kv : c->parts) (void)hipFree(kv.second.d_blk);
    for (auto &kv : c->comp) free_compressed(kv.second);
    for (auto &kv : c->sliced) free_sliced(kv.second);
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &kv : c->smooth_graphs)
        if (kv.second.ex) (void)hipGraphExecDestroy(kv.second.ex);
    for (auto &kv : c->reorders) free_reorder(kv.second);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (auto &p : c->pending) {
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
    }
    for (auto e : c->free_events) (void)hipEventDestroy(e);
    (void)hipFree(c->d_flags);
    delete c;
    return SILU_OK;
}

int silu_set_stream(silu_ctx *c, void *hip_stream)
{
    if (!c) return SILU_ERR_ARG;
    c->stream = (hipStream_t)hip_stream;
    return SILU_OK;
}

int64_t silu_bad_row(const silu_ctx *c) { return c ? c->bad_row : -1; }

int silu_last_hip_error(const silu_ctx *c) { return c ? (int)c->last_hip : 0; }

const char *silu_status_string(int s)
{
    switch (s) {
    case SILU_OK: return "ok";
    case SILU_ERR_ARG: return "invalid argument";
    case SILU_ERR_SHAPE: return "dimension mismatch";
    case SILU_ERR_PATTERN: return "CSR pattern violates the required structure";
    case SILU_ERR_ZERO_PIVOT: return "zero or non-finite pivot";
    case SILU_ERR_NONFINITE: return "non-finite value in the result";
    case SILU_ERR_NOMEM: return "workspace too small or out of memory";
    case SILU_ERR_HIP: return "HIP runtime error";
    case SILU_ERR_UNSUPPORTED: return "unsupported combination of arguments";
    case SILU_ERR_TIMEOUT: return "a bounded wait inside a persistent launch expired";
    default: return "unknown status";
    }
}

int silu_workspace_size(silu_ctx *c, int64_t n, int flags, size_t *bytes)
{
    if (!c || !bytes || n < 0) return SILU_ERR_ARG;
    *bytes = ((flags & SILU_REORDER) && !(flags & SILU_RELABELED) ? 6 : 4) * ws_vec_bytes(n);
    return SILU_OK;
}

namespace {

// Shared part of both scalings: argument checks, then k_scale_rows (pattern
// and pivot checks into the device flags, Us pattern, d, dinv and the row-
// scaled or copied values) and the FP32 copy of L.  Asynchronous.
int scale_begin(silu_ctx *c, const silu_csr *L, const silu_csr *U, silu_factors *F, int flags, bool noscale,
                float *us32)
{
    c->bad_row = -1;
    int st = check_square(U, SILU_F64);
    if (st) return st;
    st = check_square(L, SILU_F64);
    if (st) return st;
    const int64_t n = U->n_rows;
    if (L->n_rows != n) return SILU_ERR_SHAPE;
    if (U->nnz < n) return SILU_ERR_PATTERN;
    if (!F->Us.row_ptr || !F->d || !F->dinv || (U->nnz > n && (!F->Us.col_idx || !F->Us.val)))
        return SILU_ERR_ARG;
    if (flags & SILU_VALIDATE) {
        if ((st = validate(c, L, -1))) return st;
        if ((st = validate(c, U, 2))) return st;
    }
    // cached copies of earlier values in these arrays are stale from here on
    if ((st = silu_release(c, F->Us.row_ptr, F->Us.col_idx))) return st;
    if ((st = silu_release(c, L->row_ptr, L->col_idx))) return st;
    F->Ls = *L;
    F->Us.n_rows = F->Us.n_cols = n;
    F->Us.nnz = U->nnz - n;
    F->Us.dtype = SILU_F64;
    HIPCHK(c, launch_init_flags(c->d_flags, 4, INT32_MAX, c->stream));
    HIPCHK(c, launch_scale_rows((int)n, U->row_ptr, U->col_idx, (const double *)U->val, F->Us.row_ptr,
                                F->Us.col_idx, (double *)F->Us.val, F->d, F->dinv, us32, noscale ? 1 : 0,
                                (int32_t)(U->nnz - n), c->d_flags, c->stream));
    if (F->Ls_val32) HIPCHK(c, launch_to_f32(L->nnz, (const double *)L->val, F->Ls_val32, c->stream));
    return SILU_OK;
}

// Wait for the set-up and turn the device flags into a status.
int scale_end(silu_ctx *c)
{
    int32_t h[4];
    HIPCHK(c, hipMemcpyAsync(h, c->d_flags, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h[0] != INT32_MAX) {
        c->bad_row = h[0];
        return SILU_ERR_PATTERN;
    }
    if (h[1] != INT32_MAX) {
        c->bad_row = h[1];
        return SILU_ERR_ZERO_PIVOT;
    }
    return SILU_OK;
}

} // namespace

int ilu_scale_factors(silu_ctx *c, const silu_csr *L, const silu_csr *U, silu_factors *F, int flags)
{
    if (!c || !L || !U || !F) return SILU_ERR_ARG;
    const bool noscale = (flags & SILU_NO_SCALING) != 0;
    int st = scale_begin(c, L, U, F, flags, noscale, F->Us_val32);
    if (st) return st;
    F->scaled = noscale ? 0 : 1;
    return scale_end(c);
}

int ilu_scale_factors_rowcol(silu_ctx *c, const silu_csr *L, const silu_csr *U, int ruiz_iters, silu_factors *F,
                             int flags)
{
    if (!c || !L || !U || !F || !F->dc || ruiz_iters < 0 || ruiz_iters > 100 || (flags & SILU_NO_SCALING))
        return SILU_ERR_ARG;
    int st = scale_begin(c, L, U, F, flags, false, nullptr);
    if (st) return st;
    F->scaled = 2;
    const int n = (int)U->n_rows;
    if (n == 0) return scale_end(c);
    // row maxima [n] doubles, then column maxima [n] as 64-bit patterns
    void *tmp = nullptr;
    HIPCHK(c, hipMalloc(&tmp, (size_t)n * 16));
    double *rmax = (double *)tmp;
    unsigned long long *cmax = (unsigned long long *)((char *)tmp + (size_t)n * 8);
    const int32_t *Urp = U->row_ptr, *Ucol = U->col_idx;
    const double *Uval = (const double *)U->val;
    hipError_t e = launch_fill(n, F->dinv, 1.0, F->dc, 1.0, c->stream);
    for (int it = 0; it < ruiz_iters && e == hipSuccess; it++) {
        e = launch_fill(n, (double *)cmax, 0.0, nullptr, 0.0, c->stream); // +0.0 has the all-zero pattern
        if (e == hipSuccess) e = launch_ruiz_max(n, Urp, Ucol, Uval, F->dinv, F->dc, rmax, cmax, c->d_flags, c->stream);
        if (e == hipSuccess) e = launch_ruiz_scale(n, F->dinv, F->dc, rmax, cmax, c->stream);
    }
    if (e == hipSuccess)
        e = launch_rowcol_finish(n, Urp, Ucol, Uval, F->dc, F->dinv, (double *)F->Us.val, F->Us_val32,
                                 (int32_t)(U->nnz - n), c->stream);
    st = e == hipSuccess ? scale_end(c) : hip_fail(c, e);
    if (e != hipSuccess) (void)hipStreamSynchronize(c->stream); // nothing may still use tmp
    hipError_t ef = hipFree(tmp);
    if (st == SILU_OK && ef != hipSuccess) st = hip_fail(c, ef);
    return st;
}

static int smooth_plain(silu_ctx *c, const silu_csr *A, const silu_factors *F, const double *b, double *x,
                        int outer_sweeps, int m_L, int m_U, int flags, void *ws, size_t ws_bytes)
{
    if (!c || !A || !F || !b || !x || !ws) return SILU_ERR_ARG;
    c->bad_row = -1;
    const bool mixed = (flags & SILU_MIXED) != 0, direct = (flags & SILU_DIRECT) != 0;
    if (outer_sweeps < 1 || (!direct && (m_L < 1 || m_U < 1))) return SILU_ERR_ARG;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    if ((st = check_square(&F->Ls, SILU_F64))) return st;
    if ((st = check_square(&F->Us, SILU_F64))) return st;
    const int64_t n = A->n_rows;
    if (F->Ls.n_rows != n || F->Us.n_rows != n) return SILU_ERR_SHAPE;
    if (!F->dinv || (!F->scaled && !F->d) || (F->scaled == 2 && !F->dc)) return SILU_ERR_ARG;
    if (mixed && ((F->Ls.nnz > 0 && !F->Ls_val32) || (F->Us.nnz > 0 && !F->Us_val32))) return SILU_ERR_UNSUPPORTED;
    if (!F->scaled && (mixed || direct)) return SILU_ERR_UNSUPPORTED;
    if (((uintptr_t)ws & 255) != 0) return SILU_ERR_ARG;
    size_t need = 0;
    silu_workspace_size(c, n, flags, &need);
    if (ws_bytes < need) return SILU_ERR_NOMEM;
    if (flags & SILU_VALIDATE) {
        if ((st = validate(c, A, 0))) return st;
        if ((st = validate(c, &F->Ls, -1))) return st;
        if ((st = validate(c, &F->Us, 1))) return st;
    }
    if ((flags & SILU_RELABELED) && !(flags & SILU_REORDER)) return SILU_ERR_ARG;
    if (flags & SILU_REORDER) {
        // the same steps on the relabeled copies: b and x in, x out
        if (direct) return SILU_ERR_UNSUPPORTED;
        Reorder *R = nullptr;
        if ((st = get_reorder(c, A, F, &R))) return st;
        if (flags & SILU_RELABELED) { // b and x are already in the relabeled order
            const silu_factors F2 = relabeled_factors(F, R);
            const int inner = flags & ~(SILU_REORDER | SILU_RELABELED | SILU_CHECK_FINITE | SILU_VALIDATE);
            if ((st = smooth_plain(c, &R->A2, &F2, b, x, outer_sweeps, m_L, m_U, inner, ws, ws_bytes))) return st;
            return (flags & SILU_CHECK_FINITE) ? check_finite(c, n, x) : SILU_OK;
        }
        Ws w{(char *)ws, ws_vec_bytes(n)};
        double *b2 = (double *)w.slot(4), *x2 = (double *)w.slot(5);
        const double vb = 20.0 * (double)n; // index, read, write
        const bool zero = (flags & SILU_ZERO_GUESS) != 0;
        st = timed_launch(c, vb + (zero ? 0.0 : 16.0 * (double)n), [&](const char **nm) {
            *nm = "reorder_in";
            return launch_permute_in((int)n, R->pos, b, zero ? nullptr : x, b2, x2, c->stream);
        });
        if (!st && zero)
            st = timed_launch(c, 8.0 * (double)n, [&](const char **nm) {
                *nm = "fill";
                return launch_fill((int)n, x2, 0.0, nullptr, 0.0, c->stream);
            });
        if (st) return st;
        const silu_factors F2 = relabeled_factors(F, R);
        const int inner = flags & ~(SILU_REORDER | SILU_CHECK_FINITE | SILU_VALIDATE);
        if ((st = smooth_plain(c, &R->A2, &F2, b2, x2, outer_sweeps, m_L, m_U, inner, ws, ws_bytes))) return st;
        st = timed_launch(c, vb, [&](const char **nm) {
            *nm = "reorder_out";
            return launch_scatter((int)n, R->order, x2, x, c->stream);
        });
        if (st) return st;
        return (flags & SILU_CHECK_FINITE) ? check_finite(c, n, x) : SILU_OK;
    }
    Ws w{(char *)ws, ws_vec_bytes(n)};
    void *r = w.slot(0), *s = w.slot(1), *tmp[2] = {w.slot(2), w.slot(3)};
    const SweepGeom gA = pick_geom(n, A->nnz, flags), gL = pick_geom(n, F->Ls.nnz, flags),
                    gU = pick_geom(n, F->Us.nnz, flags);
    const bool scaled = F->scaled != 0;
    const double *dcol = F->scaled == 2 ? F->dc : nullptr; // row/column scaling: x += d_c * v
    const double *dshift = scaled ? nullptr : F->d;
    const Prec pL = mixed ? Prec::MIX_L : Prec::F64, pU = mixed ? Prec::MIX_U : Prec::F64;
    const void *Lval = mixed ? (const void *)F->Ls_val32 : F->Ls.val;
    const void *Uval = mixed ? (const void *)F->Us_val32 : F->Us.val;
    const int to_s = scaled ? EPI_SCALE : EPI_STORE;
    const int to_x = scaled ? EPI_SCALE_UPDATE : EPI_UPDATE;

    for (int it = 0; it < outer_sweeps; it++) {
        if (direct) {
            LevelInfo *lL = nullptr, *lU = nullptr;
            if ((st = get_levels(c, &F->Ls, SILU_LOWER, &lL))) return st;
            if ((st = get_levels(c, &F->Us, SILU_UPPER, &lU))) return st;
            if ((st = sweep(c, Prec::F64, gA, A, A->val, x, b, EPI_STORE, r, nullptr, nullptr, nullptr))) return st;
            const bool graph = !(flags & SILU_NO_GRAPH);
            if ((st = run_levels(c, &F->Ls, lL, 1, (const double *)r, (double *)tmp[0], F->dinv, (double *)s,
                                 nullptr, graph)))
                return st;
            if ((st = run_levels(c, &F->Us, lU, 1, (const double *)s, (double *)tmp[1], nullptr, nullptr, x, graph,
                                 dcol)))
                return st;
            continue;
        }
        // residual r = b - A x (fused with D^{-1} when m_L = 1); with a zero
        // guess the first one is b itself (b - A 0 = b exactly)
        // the FP32-inner form also stores y_1 = (float) r beside r, for its first L sweep to
        // gather (in tmp[1], which that sweep does not write), where L_s is swept in its sliced
        // copy: its gathers of neighbouring rows' values then take half the bytes.  (The gathers
        // of an unstructured matrix are random, a cache line each whatever their width, and the
        // extra store only costs there: 1.35 against 1.33 ms per application on the relabeled
        // random operator of 16.8M rows.)
        bool split = false;
        if (mixed && m_L >= 2 && gL.kind == SweepKernel::SLICED) {
            Sliced *SL = nullptr;
            if ((st = get_sliced(c, &F->Ls, Lval, 4, gL.slice_code_min, &SL))) return st;
            split = SL->ok;
        }
        const void *rr = r, *y1 = nullptr;
        if (m_L >= 2 && it == 0 && (flags & SILU_ZERO_GUESS)) {
            rr = b;
            st = SILU_OK;
        } else if (split) {
            y1 = tmp[1];
            st = sweep(c, Prec::F64, gA, A, A->val, x, b, EPI_STORE_SPLIT, r, nullptr, nullptr, nullptr, nullptr,
                       (float *)tmp[1]);
        } else if (m_L >= 2) {
            st = sweep(c, Prec::F64, gA, A, A->val, x, b, EPI_STORE, r, nullptr, nullptr, nullptr);
        } else if (scaled) {
            st = sweep(c, mixed ? Prec::MIX_RES : Prec::F64, gA, A, A->val, x, b, EPI_SCALE, s, F->dinv, nullptr,
                       nullptr);
        } else {
            st = sweep(c, Prec::F64, gA, A, A->val, x, b, EPI_STORE, s, nullptr, nullptr, nullptr);
        }
        if (st) return st;
        if (m_L == 1 && m_U == 1) {
            st = timed_launch(c, (dcol ? 32.0 : 24.0) * (double)n, [&](const char **nm) {
                *nm = "axpy";
                return launch_axpy((int)n, s, mixed ? 1 : 0, dcol, x, c->stream);
            });
            if (st) return st;
            continue;
        }
        // L sweeps: y_1 = r, y_k = r - Ls y_{k-1}
        const void *cur = y1 ? y1 : rr;
        for (int k = 2; k <= m_L; k++) {
            const bool last = k == m_L;
            void *out = last ? s : tmp[k & 1];
            int epi = last ? (m_U >= 2 ? to_s : to_x) : EPI_STORE;
            // in the mixed form the first sweep gathers y_1 = (float) r as the residual stored it,
            // or, where no residual was computed (a declared zero guess: r = b), gathers b and
            // rounds it (the same values either way)
            const Prec p = (mixed && k == 2 && !y1) ? Prec::MIX_L1 : pL;
            st = sweep(c, p, gL, &F->Ls, Lval, cur, rr, epi, (epi == EPI_SCALE || epi == EPI_STORE) ? out : nullptr,
                       F->dinv, x, nullptr, dcol);
            if (st) return st;
            cur = out;
        }
        // U sweeps: z_1 = s, z_k = s - Us z_{k-1}; the last adds z to x
        cur = s;
        for (int k = 2; k <= m_U; k++) {
            const bool last = k == m_U;
            void *out = last ? nullptr : tmp[k & 1];
            st = sweep(c, pU, gU, &F->Us, Uval, cur, s, last ? EPI_UPDATE : EPI_STORE, out, F->dinv, x, dshift,
                       dcol);
            if (st) return st;
            cur = out;
        }
    }
    if (flags & SILU_CHECK_FINITE) return check_finite(c, n, x);
    return SILU_OK;
}

// SILU_GRAPH: replay a recorded call, or run it and record it.
int ilu_smooth2(silu_ctx *c, const silu_csr *A, const silu_factors *F, const double *b, double *x,
                int outer_sweeps, int m_L, int m_U, int flags, void *ws, size_t ws_bytes)
{
    if (!(flags & SILU_GRAPH) || (flags & SILU_DIRECT))
        return smooth_plain(c, A, F, b, x, outer_sweeps, m_L, m_U, flags & ~SILU_GRAPH, ws, ws_bytes);
    if (!c || !A || !F || !b || !x || !ws) return SILU_ERR_ARG;
    const int rec_flags = flags & ~(SILU_GRAPH | SILU_CHECK_FINITE | SILU_VALIDATE);
    const SmoothKey key{(uintptr_t)A->row_ptr, (uintptr_t)A->col_idx, (uintptr_t)A->val, (uintptr_t)A->n_rows,
                        (uintptr_t)A->nnz, (uintptr_t)F->Ls.row_ptr, (uintptr_t)F->Ls.col_idx,
                        (uintptr_t)F->Ls.val, (uintptr_t)F->Ls.nnz, (uintptr_t)F->Us.row_ptr,
                        (uintptr_t)F->Us.col_idx, (uintptr_t)F->Us.val, (uintptr_t)F->Us.nnz,
                        (uintptr_t)F->Ls_val32, (uintptr_t)F->Us_val32, (uintptr_t)F->dinv,
                        (uintptr_t)(F->scaled == 0 ? F->d : F->dc) ^ ((uintptr_t)F->scaled << 60), (uintptr_t)b,
                        (uintptr_t)x, (uintptr_t)ws, (uintptr_t)outer_sweeps, (uintptr_t)m_L, (uintptr_t)m_U,
                        (uintptr_t)rec_flags};
    auto it = c->smooth_graphs.find(key);
    if (it != c->smooth_graphs.end() && it->second.ex) {
        int st;
        if (flags & SILU_VALIDATE) {
            if ((st = validate(c, A, 0))) return st;
            if ((st = validate(c, &F->Ls, -1))) return st;
            if ((st = validate(c, &F->Us, 1))) return st;
        }
        const SmoothGraph &g = it->second;
        st = timed_launch(c, g.bytes, g.layout, [&](const char **nm) {
            *nm = "smooth_graph";
            return hipGraphLaunch(g.ex, c->stream);
        });
        if (st) return st;
        return (flags & SILU_CHECK_FINITE) ? check_finite(c, A->n_rows, x) : SILU_OK;
    }
    // the call itself (builds every cached layout the sequence reads)
    int st = smooth_plain(c, A, F, b, x, outer_sweeps, m_L, m_U, flags & ~SILU_GRAPH, ws, ws_bytes);
    if (st || it != c->smooth_graphs.end()) return st; // an unrecordable sequence runs unrecorded
    // record the same sequence: every layout is cached now, so it enqueues kernels only
    SmoothGraph g;
    const hipError_t last = c->last_hip;
    if (!c->capture_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    hipStream_t saved = c->stream;
    const bool timing = c->timing;
    c->stream = c->capture_stream;
    c->timing = false;
    c->recording = true;
    c->rec_bytes = c->rec_layout = 0.0;
    if (hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        const int rst = smooth_plain(c, A, F, b, x, outer_sweeps, m_L, m_U, rec_flags, ws, ws_bytes);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(c->capture_stream, &gr);
        if (rst == SILU_OK && e == hipSuccess && gr &&
            hipGraphInstantiate(&g.ex, gr, nullptr, nullptr, 0) != hipSuccess)
            g.ex = nullptr;
        if (gr) (void)hipGraphDestroy(gr);
    }
    (void)hipGetLastError(); // a failed recording leaves nothing behind
    c->stream = saved;
    c->timing = timing;
    c->recording = false;
    c->last_hip = last;
    g.bytes = c->rec_bytes;
    g.layout = c->rec_layout;
    c->smooth_graphs.emplace(key, g);
    return SILU_OK;
}

int ilu_smooth(silu_ctx *c, const silu_csr *A, const silu_factors *F, const double *b, double *x, int outer_sweeps,
               int inner_iters, int flags, void *ws, size_t ws_bytes)
{
    return ilu_smooth2(c, A, F, b, x, outer_sweeps, inner_iters, inner_iters, flags, ws, ws_bytes);
}

int ilu_smooth_noalloc(silu_ctx *c, const silu_csr *A, const silu_factors *F, const double *b, double *x,
                       int outer_sweeps, int m_L, int m_U, int flags)
{
    constexpr int allowed = SILU_MIXED | SILU_ZERO_GUESS | SILU_CHECK_FINITE | SILU_KERNEL_STREAM |
                            SILU_KERNEL_VECTOR | SILU_INDEX32 | SILU_NO_WINDOW | SILU_CODE16 | SILU_CODE8 |
                            SILU_ROWPAT | SILU_SLICED_LOOP;
    if (!c || !A || (flags & ~allowed)) return SILU_ERR_ARG;
    if (A->n_rows < 0 || A->n_rows >= INT32_MAX) return SILU_ERR_ARG;
    size_t need = 0;
    silu_workspace_size(c, A->n_rows, flags, &need);
    if (need > NOALLOC_SCRATCH_BYTES) return SILU_ERR_NOMEM;
    if (!c->scratch) return SILU_ERR_HIP;
    c->no_build = true;
    const int st = smooth_plain(c, A, F, b, x, outer_sweeps, m_L, m_U, flags, c->scratch, NOALLOC_SCRATCH_BYTES);
    c->no_build = false;
    return st;
}

// ---- polynomial Gauss-Seidel smoother --------------------------------------
namespace {

// Strictly-lower counts of A's rows on the host (copied down), with the
// pattern and pivot checks.
int gs_counts(silu_ctx *c, const silu_csr *A, std::vector<int32_t> &counts)
{
    const int64_t n = A->n_rows;
    counts.assign((size_t)n, 0);
    if (n == 0) return SILU_OK;
    int32_t *d_counts = nullptr;
    HIPCHK(c, hipMalloc(&d_counts, (size_t)n * 4));
    hipError_t e = launch_init_flags(c->d_flags, 4, INT32_MAX, c->stream);
    if (e == hipSuccess)
        e = launch_gs_count((int)n, A->row_ptr, A->col_idx, (const double *)A->val, d_counts, c->d_flags, c->stream);
    int32_t h[4];
    if (e == hipSuccess) e = hipMemcpyAsync(counts.data(), d_counts, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h, c->d_flags, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d_counts);
    if (e != hipSuccess) return hip_fail(c, e);
    if (h[0] != INT32_MAX) {
        c->bad_row = h[0];
        return SILU_ERR_PATTERN;
    }
    if (h[1] != INT32_MAX) {
        c->bad_row = h[1];
        return SILU_ERR_ZERO_PIVOT;
    }
    return SILU_OK;
}

} // namespace

int gs_split_size(silu_ctx *c, const silu_csr *A, int64_t *nnz_lower)
{
    if (!c || !A || !nnz_lower) return SILU_ERR_ARG;
    c->bad_row = -1;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    std::vector<int32_t> counts;
    if ((st = gs_counts(c, A, counts))) return st;
    int64_t t = 0;
    for (int32_t v : counts) t += v;
    *nnz_lower = t;
    return SILU_OK;
}

int gs_scale_split(silu_ctx *c, const silu_csr *A, silu_factors *G, int flags)
{
    if (!c || !A || !G) return SILU_ERR_ARG;
    c->bad_row = -1;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    const int64_t n = A->n_rows;
    if (!G->Ls.row_ptr || !G->d || !G->dinv) return SILU_ERR_ARG;
    if (flags & SILU_VALIDATE) {
        if ((st = validate(c, A, 0))) return st;
    }
    std::vector<int32_t> counts;
    if ((st = gs_counts(c, A, counts))) return st;
    std::vector<int32_t> rp((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; i++) rp[(size_t)i + 1] = rp[(size_t)i] + counts[(size_t)i];
    const int64_t nnz = rp[(size_t)n];
    if (nnz > 0 && (!G->Ls.col_idx || !G->Ls.val)) return SILU_ERR_ARG;
    // cached copies of earlier values in the output arrays are stale from here on
    if ((st = silu_release(c, G->Ls.row_ptr, G->Ls.col_idx))) return st;
    G->Ls.n_rows = G->Ls.n_cols = n;
    G->Ls.nnz = nnz;
    G->Ls.dtype = SILU_F64;
    G->Us.n_rows = G->Us.n_cols = n;
    G->Us.nnz = 0;
    G->Us.dtype = SILU_F64;
    G->scaled = 3;
    HIPCHK(c, hipMemcpyAsync(G->Ls.row_ptr, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_gs_fill((int)n, A->row_ptr, A->col_idx, (const double *)A->val, G->Ls.row_ptr, G->Ls.col_idx,
                             (double *)G->Ls.val, G->d, G->dinv, G->Ls_val32, (int32_t)nnz, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream)); // rp goes out of scope
    return SILU_OK;
}

int gs_smooth(silu_ctx *c, const silu_csr *A, const silu_factors *G, const double *b, double *x, int outer_sweeps,
              int terms, int flags, void *ws, size_t ws_bytes)
{
    if (!c || !A || !G || !b || !x || !ws) return SILU_ERR_ARG;
    c->bad_row = -1;
    const bool mixed = (flags & SILU_MIXED) != 0;
    if (outer_sweeps < 1 || terms < 1 || (flags & SILU_DIRECT)) return SILU_ERR_ARG;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    if ((st = check_square(&G->Ls, SILU_F64))) return st;
    const int64_t n = A->n_rows;
    if (G->Ls.n_rows != n) return SILU_ERR_SHAPE;
    if (G->scaled != 3 || !G->dinv) return SILU_ERR_ARG;
    if (mixed && G->Ls.nnz > 0 && !G->Ls_val32) return SILU_ERR_UNSUPPORTED;
    if (((uintptr_t)ws & 255) != 0) return SILU_ERR_ARG;
    size_t need = 0;
    silu_workspace_size(c, n, flags, &need);
    if (ws_bytes < need) return SILU_ERR_NOMEM;
    if (flags & SILU_VALIDATE) {
        if ((st = validate(c, A, 0))) return st;
        if ((st = validate(c, &G->Ls, -1))) return st;
    }
    if (flags & SILU_REORDER) {
        // the same steps on relabeled copies of A and Gs: b and x in, x out
        Reorder *R = nullptr;
        if ((st = get_reorder(c, A, G, &R))) return st;
        Ws w{(char *)ws, ws_vec_bytes(n)};
        double *b2 = (double *)w.slot(4), *x2 = (double *)w.slot(5);
        st = timed_launch(c, 36.0 * (double)n, [&](const char **nm) {
            *nm = "reorder_in";
            return launch_permute_in((int)n, R->pos, b, x, b2, x2, c->stream);
        });
        if (st) return st;
        const silu_factors G2 = relabeled_factors(G, R);
        const int inner = flags & ~(SILU_REORDER | SILU_CHECK_FINITE | SILU_VALIDATE);
        if ((st = gs_smooth(c, &R->A2, &G2, b2, x2, outer_sweeps, terms, inner, ws, ws_bytes))) return st;
        st = timed_launch(c, 20.0 * (double)n, [&](const char **nm) {
            *nm = "reorder_out";
            return launch_scatter((int)n, R->order, x2, x, c->stream);
        });
        if (st) return st;
        return (flags & SILU_CHECK_FINITE) ? check_finite(c, n, x) : SILU_OK;
    }
    Ws w{(char *)ws, ws_vec_bytes(n)};
    void *s = w.slot(1), *tmp[2] = {w.slot(2), w.slot(3)};
    const SweepGeom gA = pick_geom(n, A->nnz, flags), gG = pick_geom(n, G->Ls.nnz, flags);
    const Prec pG = mixed ? Prec::MIX_U : Prec::F64;
    const void *Gval = mixed ? (const void *)G->Ls_val32 : G->Ls.val;
    for (int it = 0; it < outer_sweeps; it++) {
        // s = D^{-1} (b - A x)  (mixed: the residual rounded to FP32, then scaled, in FP32)
        st = sweep(c, mixed ? Prec::MIX_RES : Prec::F64, gA, A, A->val, x, b, EPI_SCALE, s, G->dinv, nullptr,
                   nullptr);
        if (st) return st;
        if (terms == 1) {
            st = timed_launch(c, 24.0 * (double)n, [&](const char **nm) {
                *nm = "axpy";
                return launch_axpy((int)n, s, mixed ? 1 : 0, nullptr, x, c->stream);
            });
            if (st) return st;
            continue;
        }
        // y_1 = s;  y_k = s - Gs y_{k-1};  the last adds y to x
        const void *cur = s;
        for (int k = 2; k <= terms; k++) {
            const bool last = k == terms;
            void *out = last ? nullptr : tmp[k & 1];
            st = sweep(c, pG, gG, &G->Ls, Gval, cur, s, last ? EPI_UPDATE : EPI_STORE, out, G->dinv, x, nullptr);
            if (st) return st;
            cur = out;
        }
    }
    if (flags & SILU_CHECK_FINITE) return check_finite(c, n, x);
    return SILU_OK;
}

// ---- ILU(0) by fixed-point sweeps on the device ------------------------------
int silu_split_sizes(silu_ctx *c, const silu_csr *A, int64_t *nnz_lower, int64_t *nnz_upper)
{
    if (!c || !A || !nnz_lower || !nnz_upper) return SILU_ERR_ARG;
    int st = gs_split_size(c, A, nnz_lower);
    if (st) return st;
    *nnz_upper = A->nnz - *nnz_lower;
    return SILU_OK;
}

int silu_ilu0_fixed_point_workspace_size(silu_ctx *c, int64_t n, int64_t nnz, size_t *bytes)
{
    if (!c || !bytes || n < 0 || nnz < 0) return SILU_ERR_ARG;
    *bytes = 2 * ws_vec_bytes(nnz) + ws_vec_bytes((nnz + 1) / 2) + ws_vec_bytes((n + 1) / 2);
    return SILU_OK;
}

int silu_ilu0_fixed_point(silu_ctx *c, const silu_csr *A, int sweeps, silu_csr *Ls, silu_csr *U, int *changed,
                          int flags, void *ws, size_t ws_bytes)
{
    if (!c || !A || !Ls || !U || !ws || sweeps < 0) return SILU_ERR_ARG;
    c->bad_row = -1;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    const int64_t n = A->n_rows, nnz = A->nnz;
    if (nnz >= INT32_MAX) return SILU_ERR_SHAPE;
    size_t need = 0;
    silu_ilu0_fixed_point_workspace_size(c, n, nnz, &need);
    if (ws_bytes < need || ((uintptr_t)ws & 255) != 0) return ws_bytes < need ? SILU_ERR_NOMEM : SILU_ERR_ARG;
    if (!Ls->row_ptr || !U->row_ptr) return SILU_ERR_ARG;
    if (flags & SILU_VALIDATE) {
        if ((st = validate(c, A, 0))) return st;
    }
    // row counts of the two parts (with the diagonal and pivot checks)
    std::vector<int32_t> counts;
    if ((st = gs_counts(c, A, counts))) return st;
    std::vector<int32_t> rp((size_t)n + 1), Lrp((size_t)n + 1, 0), Urp((size_t)n + 1, 0);
    HIPCHK(c, hipMemcpyAsync(rp.data(), A->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n; i++) {
        Lrp[(size_t)i + 1] = Lrp[(size_t)i] + counts[(size_t)i];
        Urp[(size_t)i + 1] = Urp[(size_t)i] + (rp[(size_t)i + 1] - rp[(size_t)i] - counts[(size_t)i]);
    }
    const int64_t l_nnz = Lrp[(size_t)n], u_nnz = Urp[(size_t)n];
    if ((l_nnz > 0 && (!Ls->col_idx || !Ls->val)) || (u_nnz > 0 && (!U->col_idx || !U->val))) return SILU_ERR_ARG;
    if ((st = silu_release(c, Ls->row_ptr, Ls->col_idx))) return st;
    if ((st = silu_release(c, U->row_ptr, U->col_idx))) return st;
    char *w = (char *)ws;
    double *LU0 = (double *)w, *LU1 = (double *)(w + ws_vec_bytes(nnz));
    int32_t *row_of = (int32_t *)(w + 2 * ws_vec_bytes(nnz));
    int32_t *dpos = (int32_t *)(w + 2 * ws_vec_bytes(nnz) + ws_vec_bytes((nnz + 1) / 2));
    HIPCHK(c, launch_init_flags(c->d_flags, 4, INT32_MAX, c->stream));
    HIPCHK(c, launch_fp_index((int)n, A->row_ptr, A->col_idx, dpos, row_of, c->d_flags, c->stream));
    HIPCHK(c, launch_fp_init(nnz, A->col_idx, (const double *)A->val, dpos, row_of, LU0, c->stream));
    double *cur = LU0, *nxt = LU1;
    int32_t h[4] = {INT32_MAX, 0, 0, 0};
    for (int sw = 0; sw < sweeps; sw++) {
        HIPCHK(c, launch_init_flags(c->d_flags + 1, 1, 0, c->stream));
        st = timed_launch(c, 8.0 * 3.0 * (double)nnz, [&](const char **nm) {
            *nm = "ilu0_fixed_point_sweep";
            return launch_fp_sweep(nnz, A->row_ptr, A->col_idx, (const double *)A->val, dpos, row_of, cur, nxt,
                                   c->d_flags, c->stream);
        });
        if (st) return st;
        std::swap(cur, nxt);
    }
    HIPCHK(c, hipMemcpyAsync(Ls->row_ptr, Lrp.data(), Lrp.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(U->row_ptr, Urp.data(), Urp.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_fp_split((int)n, A->row_ptr, A->col_idx, cur, Ls->row_ptr, Ls->col_idx, (double *)Ls->val,
                              U->row_ptr, U->col_idx, (double *)U->val, l_nnz, u_nnz, c->stream));
    HIPCHK(c, hipMemcpyAsync(h, c->d_flags, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream)); // host row pointers go out of scope
    Ls->n_rows = Ls->n_cols = U->n_rows = U->n_cols = n;
    Ls->nnz = l_nnz;
    U->nnz = u_nnz;
    Ls->dtype = U->dtype = SILU_F64;
    if (changed) *changed = sweeps > 0 ? h[1] : 1;
    return SILU_OK;
}

// ---- FGMRES with the smoother as right preconditioner -----------------------
namespace {

// Smoother slots: 4 n-vectors, 6 when the smoother runs on relabeled copies.
int smoother_slots(int flags) { return (flags & SILU_REORDER) ? 6 : 4; }

struct KrylovWs {
    size_t vec;     // bytes of one n-vector slot
    char *base;
    int m;
    int ss;         // smoother slots
    double *V(int i) const { return (double *)(base + vec * (size_t)i); }               // i = 0..m
    double *Z(int i) const { return (double *)(base + vec * (size_t)(m + 1 + i)); }     // i = 0..m-1
    double *w() const { return (double *)(base + vec * (size_t)(2 * m + 1)); }
    void *smoother() const { return base + vec * (size_t)(2 * m + 2); }                 // ss slots
    double *part() const { return (double *)(base + vec * (size_t)(2 * m + 2 + ss)); } // DOT_BLOCKS
    double *h() const { return part() + DOT_BLOCKS; }                                    // m + 2 scalars
    double *gram() const { return h() + m + 2; }                                         // m + 2 scalars
};

size_t krylov_ws_bytes(int64_t n, int m, int flags)
{
    const size_t vec = ws_vec_bytes(n);
    return vec * (size_t)(2 * m + 2 + smoother_slots(flags)) +
           ((size_t)DOT_BLOCKS + 2 * ((size_t)m + 2)) * sizeof(double) + 256;
}

} // namespace

int silu_fgmres_workspace_size(silu_ctx *c, int64_t n, int restart, int flags, size_t *bytes)
{
    if (!c || !bytes || n < 0 || restart < 1) return SILU_ERR_ARG;
    *bytes = krylov_ws_bytes(n, restart, flags);
    return SILU_OK;
}

namespace {

// FGMRES(restart) stopped when |g_{j+1}| / (||b|| + norm_a ||x_j||) < tol:
// norm_a = 0 is eq. relres, norm_a = ||A||_2 eq. nbre.
int fgmres_impl(silu_ctx *c, const silu_csr *A, const silu_factors *F, const double *b, double *x, int restart,
                int max_iters, double tol, double norm_a, int outer, int m_L, int m_U, int flags, void *ws,
                size_t ws_bytes, int *iters, double *hist)
{
    if (!c || !A || !F || !b || !x || !ws || !iters) return SILU_ERR_ARG;
    c->bad_row = -1;
    if (restart < 1 || max_iters < 0 || !(tol >= 0.0) || outer < 1 || m_L < 1 || m_U < 1) return SILU_ERR_ARG;
    if (F->scaled != 1 && F->scaled != 2) return SILU_ERR_UNSUPPORTED;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    const int64_t n = A->n_rows;
    if (((uintptr_t)ws & 255) != 0) return SILU_ERR_ARG;
    if (ws_bytes < krylov_ws_bytes(n, restart, flags)) return SILU_ERR_NOMEM;
    if (flags & SILU_VALIDATE) {
        if ((st = validate(c, A, 0))) return st;
    }
    if (flags & SILU_REORDER) {
        // the whole solve on the relabeled copies: b and x in once, x out once,
        // so the products with A and the sweeps gather locally (the two extra
        // smoother slots hold the relabeled b and x)
        Reorder *R = nullptr;
        if ((st = get_reorder(c, A, F, &R))) return st;
        const size_t vec = ws_vec_bytes(n);
        double *b2 = (double *)ws, *x2 = (double *)((char *)ws + vec);
        st = timed_launch(c, 36.0 * (double)n, [&](const char **nm) {
            *nm = "reorder_in";
            return launch_permute_in((int)n, R->pos, b, x, b2, x2, c->stream);
        });
        if (st) return st;
        const silu_factors F2 = relabeled_factors(F, R);
        const int inner = flags & ~(SILU_REORDER | SILU_CHECK_FINITE | SILU_VALIDATE);
        if ((st = fgmres_impl(c, &R->A2, &F2, b2, x2, restart, max_iters, tol, norm_a, outer, m_L, m_U, inner,
                              (char *)ws + 2 * vec, ws_bytes - 2 * vec, iters, hist)))
            return st;
        st = timed_launch(c, 20.0 * (double)n, [&](const char **nm) {
            *nm = "reorder_out";
            return launch_scatter((int)n, R->order, x2, x, c->stream);
        });
        if (st) return st;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return (flags & SILU_CHECK_FINITE) ? check_finite(c, n, x) : SILU_OK;
    }
    const int m = restart;
    KrylovWs K{ws_vec_bytes(n), (char *)ws, m, smoother_slots(flags)};
    const size_t sws_bytes = (size_t)K.ss * K.vec;
    const int pflags = (flags & ~(SILU_CHECK_FINITE | SILU_VALIDATE | SILU_DIRECT | SILU_GRAPH)) | SILU_ZERO_GUESS;
    const SweepGeom gA = pick_geom(n, A->nnz, flags);
    auto dot = [&](const double *a, const double *bb, double *out, bool root) {
        return timed_launch(c, 16.0 * (double)n, [&](const char **nm) {
            *nm = "dot";
            return launch_dot(n, a, bb, K.part(), out, root, c->stream);
        });
    };
    auto fetch = [&](double *host, const double *dev, int count) -> int {
        HIPCHK(c, hipMemcpyAsync(host, dev, sizeof(double) * (size_t)count, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return SILU_OK;
    };
    std::vector<double> H((size_t)(m + 1) * (size_t)m), cs((size_t)m), sn((size_t)m), g((size_t)m + 1),
        y((size_t)m), hcol((size_t)m + 2);
    // eq. nbre: ||x_j||^2 = ||x_0||^2 + 2 y.c + y^T G y with G = Z^T Z, c = Z^T x_0
    const bool nrbe = norm_a > 0.0;
    std::vector<double> G(nrbe ? (size_t)m * (size_t)m : 0), cz(nrbe ? (size_t)m : 0), yt(nrbe ? (size_t)m : 0),
        grow(nrbe ? (size_t)m + 2 : 0);
    double nb = 0.0, beta = 0.0, xx0 = 0.0;
    auto norm_x0 = [&]() -> int { // ||x||^2 of the cycle's start
        int e;
        if (!nrbe) return SILU_OK;
        if ((e = dot(x, x, K.gram(), false))) return e;
        return fetch(&xx0, K.gram(), 1);
    };
    // ||b|| and the first residual
    if ((st = dot(b, b, K.h(), true))) return st;
    if ((st = fetch(&nb, K.h(), 1))) return st;
    if ((st = sweep(c, Prec::F64, gA, A, A->val, x, b, EPI_STORE, K.V(0), nullptr, nullptr, nullptr))) return st;
    if ((st = dot(K.V(0), K.V(0), K.h(), true))) return st;
    if ((st = fetch(&beta, K.h(), 1))) return st;
    if ((st = norm_x0())) return st;
    int k = 0;
    const double est0 = beta / (nb + norm_a * std::sqrt(xx0));
    if (hist) hist[0] = est0;
    if (!(est0 >= tol)) { // converged (or b = 0 and x = 0)
        *iters = 0;
        return SILU_OK;
    }
    while (k < max_iters) {
        HIPCHK(c, launch_div_host(n, K.V(0), beta, K.V(0), c->stream));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        bool done = false;
        for (; j < m && k < max_iters; j++) {
            double *zj = K.Z(j), *w = K.w();
            // z_j = M^{-1} v_j: one smoother call from z = 0
            HIPCHK(c, launch_fill((int)n, zj, 0.0, nullptr, 0.0, c->stream));
            if ((st = ilu_smooth2(c, A, F, K.V(j), zj, outer, m_L, m_U, pflags, K.smoother(), sws_bytes))) return st;
            if (nrbe) { // row j of G and c_j, fetched with the Hessenberg column
                for (int i = 0; i <= j; i++)
                    if ((st = dot(zj, K.Z(i), K.gram() + i, false))) return st;
                if ((st = dot(zj, x, K.gram() + j + 1, false))) return st;
                HIPCHK(c, hipMemcpyAsync(grow.data(), K.gram(), sizeof(double) * (size_t)(j + 2),
                                         hipMemcpyDeviceToHost, c->stream));
            }
            // w = A z_j, then modified Gram-Schmidt against v_0..v_j
            if ((st = sweep(c, Prec::F64, gA, A, A->val, zj, nullptr, EPI_SPMV, w, nullptr, nullptr, nullptr)))
                return st;
            for (int i = 0; i <= j; i++) {
                if ((st = dot(w, K.V(i), K.h() + i, false))) return st;
                st = timed_launch(c, 24.0 * (double)n, [&](const char **nm) {
                    *nm = "mgs_update";
                    return launch_sub_scaled(n, w, K.V(i), K.h() + i, c->stream);
                });
                if (st) return st;
            }
            if ((st = dot(w, w, K.h() + j + 1, true))) return st;
            if ((st = fetch(hcol.data(), K.h(), j + 2))) return st;
            double *h = &H[(size_t)(m + 1) * (size_t)j];
            for (int i = 0; i <= j + 1; i++) h[i] = hcol[(size_t)i];
            if (h[j + 1] != 0.0) HIPCHK(c, launch_div_dev(n, w, K.h() + j + 1, K.V(j + 1), c->stream));
            // Givens rotations on the new column (host; m is small)
            for (int i = 0; i < j; i++) {
                const double a0 = h[i], a1 = h[i + 1];
                h[i] = cs[(size_t)i] * a0 + sn[(size_t)i] * a1;
                h[i + 1] = -sn[(size_t)i] * a0 + cs[(size_t)i] * a1;
            }
            const double den = std::sqrt(h[j] * h[j] + h[j + 1] * h[j + 1]);
            cs[(size_t)j] = h[j] / den;
            sn[(size_t)j] = h[j + 1] / den;
            h[j] = den;
            h[j + 1] = 0.0;
            g[(size_t)j + 1] = -sn[(size_t)j] * g[(size_t)j];
            g[(size_t)j] = cs[(size_t)j] * g[(size_t)j];
            k++;
            double xn = 0.0;
            if (nrbe) {
                for (int i = 0; i <= j; i++) {
                    G[(size_t)j * (size_t)m + (size_t)i] = grow[(size_t)i];
                    G[(size_t)i * (size_t)m + (size_t)j] = grow[(size_t)i];
                }
                cz[(size_t)j] = grow[(size_t)j + 1];
                // y of the first j + 1 steps (back substitution), then the quadratic form
                for (int i = j; i >= 0; i--) {
                    double t = g[(size_t)i];
                    for (int c2 = i + 1; c2 <= j; c2++) t -= H[(size_t)i + (size_t)(m + 1) * (size_t)c2] * yt[(size_t)c2];
                    yt[(size_t)i] = t / H[(size_t)i + (size_t)(m + 1) * (size_t)i];
                }
                double q = xx0;
                for (int i = 0; i <= j; i++) {
                    double gi = 0.0;
                    for (int l = 0; l <= j; l++) gi += G[(size_t)i * (size_t)m + (size_t)l] * yt[(size_t)l];
                    q += yt[(size_t)i] * (2.0 * cz[(size_t)i] + gi);
                }
                xn = std::sqrt(std::max(q, 0.0));
            }
            const double est = std::fabs(g[(size_t)j + 1]) / (nb + norm_a * xn);
            if (hist) hist[k] = est;
            if (est < tol || den == 0.0) {
                done = true;
                j++;
                break;
            }
        }
        // y = H^{-1} g, x = x + sum_i y_i z_i
        for (int i = j - 1; i >= 0; i--) {
            double t = g[(size_t)i];
            for (int c2 = i + 1; c2 < j; c2++) t = t - H[(size_t)i + (size_t)(m + 1) * (size_t)c2] * y[(size_t)c2];
            y[(size_t)i] = t / H[(size_t)i + (size_t)(m + 1) * (size_t)i];
        }
        for (int i = 0; i < j; i++) HIPCHK(c, launch_axpy_host(n, y[(size_t)i], K.Z(i), x, c->stream));
        if (done) break;
        if ((st = sweep(c, Prec::F64, gA, A, A->val, x, b, EPI_STORE, K.V(0), nullptr, nullptr, nullptr))) return st;
        if ((st = dot(K.V(0), K.V(0), K.h(), true))) return st;
        if ((st = fetch(&beta, K.h(), 1))) return st;
        if ((st = norm_x0())) return st;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *iters = k;
    if (flags & SILU_CHECK_FINITE) return check_finite(c, n, x);
    return SILU_OK;
}

} // namespace

int silu_fgmres(silu_ctx *c, const silu_csr *A, const silu_factors *F, const double *b, double *x, int restart,
                int max_iters, double tol, int outer, int m_L, int m_U, int flags, void *ws, size_t ws_bytes,
                int *iters, double *hist)
{
    return fgmres_impl(c, A, F, b, x, restart, max_iters, tol, 0.0, outer, m_L, m_U, flags, ws, ws_bytes, iters,
                       hist);
}

int silu_fgmres_nrbe(silu_ctx *c, const silu_csr *A, const silu_factors *F, const double *b, double *x,
                     int restart, int max_iters, double tol, double norm_a, int outer, int m_L, int m_U, int flags,
                     void *ws, size_t ws_bytes, int *iters, double *hist)
{
    if (!(norm_a >= 0.0) || !std::isfinite(norm_a)) return SILU_ERR_ARG;
    return fgmres_impl(c, A, F, b, x, restart, max_iters, tol, norm_a, outer, m_L, m_U, flags, ws, ws_bytes, iters,
                       hist);
}

int silu_spmv(silu_ctx *c, const silu_csr *A, const double *xin, double *y, int flags)
{
    if (!c || !A || !xin || !y || xin == y) return SILU_ERR_ARG;
    c->bad_row = -1;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    if (flags & SILU_VALIDATE) {
        if ((st = validate(c, A, 0))) return st;
    }
    return sweep(c, Prec::F64, pick_geom(A->n_rows, A->nnz, flags), A, A->val, xin, nullptr, EPI_SPMV, y, nullptr,
                 nullptr, nullptr);
}

int silu_dot(silu_ctx *c, int64_t n, const double *a, const double *b, double *result, void *ws, size_t ws_bytes)
{
    if (!c || !a || !b || !result || !ws || n < 0) return SILU_ERR_ARG;
    if (ws_bytes < (DOT_BLOCKS + 1) * sizeof(double)) return SILU_ERR_NOMEM;
    double *part = (double *)ws, *out = part + DOT_BLOCKS;
    HIPCHK(c, launch_dot(n, a, b, part, out, false, c->stream));
    HIPCHK(c, hipMemcpyAsync(result, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SILU_OK;
}

int silu_aux_workspace_size(int64_t n, size_t *bytes)
{
    if (!bytes || n < 0) return SILU_ERR_ARG;
    *bytes = 2 * ws_vec_bytes(n) + (DOT_BLOCKS + 32) * sizeof(double);
    return SILU_OK;
}

namespace {

struct AuxWs {
    double *v, *w, *part, *s; // two n-vectors, the dot partials, 8 scalars
};

int aux_ws(int64_t n, void *ws, size_t ws_bytes, AuxWs *a)
{
    size_t need = 0;
    silu_aux_workspace_size(n, &need);
    if (((uintptr_t)ws & 255) != 0) return SILU_ERR_ARG;
    if (ws_bytes < need) return SILU_ERR_NOMEM;
    const size_t vec = ws_vec_bytes(n);
    a->v = (double *)ws;
    a->w = (double *)((char *)ws + vec);
    a->part = (double *)((char *)ws + 2 * vec);
    a->s = a->part + DOT_BLOCKS;
    return SILU_OK;
}

} // namespace

int silu_norm2_estimate(silu_ctx *c, const silu_csr *A, const double *v0, int iters, double *result, void *ws,
                        size_t ws_bytes)
{
    if (!c || !A || !v0 || !result || !ws || iters < 1) return SILU_ERR_ARG;
    c->bad_row = -1;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    const int64_t n = A->n_rows;
    AuxWs a;
    if ((st = aux_ws(n, ws, ws_bytes, &a))) return st;
    const SweepGeom gA = pick_geom(n, A->nnz, 0);
    double nv = 0.0, lam = 0.0;
    auto norm = [&](const double *u, double *out) -> int {
        HIPCHK(c, launch_dot(n, u, u, a.part, a.s, true, c->stream));
        HIPCHK(c, hipMemcpyAsync(out, a.s, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return SILU_OK;
    };
    if ((st = norm(v0, &nv))) return st;
    if (!(nv > 0.0) || !std::isfinite(nv)) return SILU_ERR_ARG;
    HIPCHK(c, launch_div_host(n, v0, nv, a.v, c->stream));
    // power iteration: lam = ||A v||, v = A v / lam
    for (int it = 0; it < iters; it++) {
        if ((st = sweep(c, Prec::F64, gA, A, A->val, a.v, nullptr, EPI_SPMV, a.w, nullptr, nullptr, nullptr)))
            return st;
        if ((st = norm(a.w, &lam))) return st;
        if (lam == 0.0) break;
        HIPCHK(c, launch_div_host(n, a.w, lam, a.v, c->stream));
    }
    *result = lam;
    return SILU_OK;
}

int silu_nrbe(silu_ctx *c, const silu_csr *A, const double *b, const double *x, double norm_a, double *result,
              void *ws, size_t ws_bytes)
{
    if (!c || !A || !b || !x || !result || !ws || !(norm_a >= 0.0) || !std::isfinite(norm_a)) return SILU_ERR_ARG;
    c->bad_row = -1;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    const int64_t n = A->n_rows;
    AuxWs a;
    if ((st = aux_ws(n, ws, ws_bytes, &a))) return st;
    if ((st = sweep(c, Prec::F64, pick_geom(n, A->nnz, 0), A, A->val, x, b, EPI_STORE, a.v, nullptr, nullptr,
                    nullptr)))
        return st;
    HIPCHK(c, launch_dot(n, a.v, a.v, a.part, a.s, true, c->stream));
    HIPCHK(c, launch_dot(n, b, b, a.part, a.s + 1, true, c->stream));
    HIPCHK(c, launch_dot(n, x, x, a.part, a.s + 2, true, c->stream));
    double h[3];
    HIPCHK(c, hipMemcpyAsync(h, a.s, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *result = h[0] / (h[1] + norm_a * h[2]);
    return SILU_OK;
}

int trisolve_direct(silu_ctx *c, const silu_csr *T, int uplo, int diag, const double *rhs, double *out, int flags)
{
    if (!c || !T || !rhs || !out || rhs == out) return SILU_ERR_ARG;
    if ((uplo != SILU_LOWER && uplo != SILU_UPPER) || (diag != SILU_UNIT && diag != SILU_NONUNIT)) return SILU_ERR_ARG;
    c->bad_row = -1;
    int st = check_square(T, SILU_F64);
    if (st) return st;
    if (flags & SILU_VALIDATE) {
        if ((st = validate(c, T, 0))) return st;
    }
    LevelInfo *li = nullptr;
    if ((st = get_levels(c, T, uplo, &li))) return st;
    return run_levels(c, T, li, diag == SILU_UNIT ? 1 : 0, rhs, out, nullptr, nullptr, nullptr,
                      !(flags & SILU_NO_GRAPH));
}

int trisolve_iter(silu_ctx *c, const silu_csr *T, const double *dinv, const double *rhs, double *out, int m,
                  int flags, void *ws, size_t ws_bytes)
{
    if (!c || !T || !rhs || !out || !ws || m < 1) return SILU_ERR_ARG;
    c->bad_row = -1;
    int st = check_square(T, SILU_F64);
    if (st) return st;
    const int64_t n = T->n_rows;
    if (((uintptr_t)ws & 255) != 0) return SILU_ERR_ARG;
    size_t need = 0;
    silu_workspace_size(c, n, 0, &need);
    if (ws_bytes < need) return SILU_ERR_NOMEM;
    if (flags & SILU_VALIDATE) {
        if ((st = validate(c, T, 0))) return st;
    }
    Ws w{(char *)ws, ws_vec_bytes(n)};
    double *sv = m == 1 ? out : (double *)w.slot(0);
    void *tmp[2] = {w.slot(1), w.slot(2)};
    st = timed_launch(c, (dinv ? 24.0 : 16.0) * (double)n, [&](const char **nm) {
        *nm = "scale_copy";
        return launch_scale_copy((int)n, rhs, dinv, sv, c->stream);
    });
    if (st) return st;
    const SweepGeom g = pick_geom(n, T->nnz, flags);
    const void *cur = sv;
    for (int k = 2; k <= m; k++) {
        void *o = k == m ? (void *)out : tmp[k & 1];
        if ((st = sweep(c, Prec::F64, g, T, T->val, cur, sv, EPI_STORE, o, nullptr, nullptr, nullptr))) return st;
        cur = o;
    }
    return SILU_OK;
}

int silu_analyze(silu_ctx *c, const silu_csr *T, int uplo, int32_t *depth, int32_t *rows_per_level)
{
    if (!c || !T || !depth || (uplo != SILU_LOWER && uplo != SILU_UPPER)) return SILU_ERR_ARG;
    int st = check_square(T, SILU_F64);
    if (st) return st;
    LevelInfo *li = nullptr;
    if ((st = get_levels(c, T, uplo, &li))) return st;
    *depth = li->depth;
    if (rows_per_level)
        for (int l = 0; l < li->depth; l++) rows_per_level[l] = li->level_ptr[(size_t)l + 1] - li->level_ptr[(size_t)l];
    return SILU_OK;
}

int silu_release(silu_ctx *c, const void *row_ptr, const void *col_idx)
{
    if (!c) return SILU_ERR_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream)); // nothing queued may still use what is dropped
    // recorded smoother calls bake in the cached layouts' addresses: drop them all
    for (auto &kv : c->smooth_graphs)
        if (kv.second.ex) (void)hipGraphExecDestroy(kv.second.ex);
    c->smooth_graphs.clear();
    // relabeled copies made from this matrix, with everything cached for them
    std::vector<Reorder> gone;
    for (auto it = c->reorders.begin(); it != c->reorders.end();) {
        const ReorderKey &k = it->first;
        const uintptr_t r = (uintptr_t)row_ptr, ci = (uintptr_t)col_idx;
        if (k[0] == r || k[3] == r || k[6] == r || (ci && (k[1] == ci || k[4] == ci || k[7] == ci))) {
            gone.push_back(it->second);
            it = c->reorders.erase(it);
        } else {
            ++it;
        }
    }
    for (Reorder &R : gone) {
        const silu_csr *m[3] = {&R.A2, &R.L2, &R.U2};
        for (const silu_csr *M : m)
            if (M->row_ptr) (void)silu_release(c, M->row_ptr, M->col_idx);
        free_reorder(R);
    }
    for (auto it = c->levels.begin(); it != c->levels.end();) {
        if (std::get<0>(it->first) == row_ptr || std::get<1>(it->first) == col_idx) {
            const LevelInfo *li = &it->second;
            for (auto g = c->graphs.begin(); g != c->graphs.end();) {
                if (std::get<0>(g->first) == li) {
                    (void)hipGraphExecDestroy(g->second);
                    g = c->graphs.erase(g);
                } else {
                    ++g;
                }
            }
            (void)hipFree(it->second.d_perm);
            it = c->levels.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = c->parts.begin(); it != c->parts.end();) {
        if (std::get<0>(it->first) == row_ptr) {
            (void)hipFree(it->second.d_blk);
            it = c->parts.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = c->comp.begin(); it != c->comp.end();) {
        if (std::get<0>(it->first) == row_ptr || std::get<1>(it->first) == col_idx) {
            free_compressed(it->second);
            it = c->comp.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = c->sliced.begin(); it != c->sliced.end();) {
        if (std::get<0>(it->first) == row_ptr || std::get<1>(it->first) == col_idx) {
            free_sliced(it->second);
            it = c->sliced.erase(it);
        } else {
            ++it;
        }
    }
    return SILU_OK;
}

int silu_set_timing(silu_ctx *c, int enable)
{
    if (!c) return SILU_ERR_ARG;
    c->timing = enable != 0;
    return SILU_OK;
}

int silu_stats_collect(silu_ctx *c)
{
    if (!c) return SILU_ERR_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, p.e0, p.e1));
        c->klaunch[(size_t)p.kid] += 1;
        c->kms[(size_t)p.kid] += ms;
        c->kbytes[(size_t)p.kid] += p.bytes;
        c->klayout[(size_t)p.kid] += p.layout;
        c->free_events.push_back(p.e0);
        c->free_events.push_back(p.e1);
    }
    c->pending.clear();
    return (int)c->knames.size();
}

int silu_stats_get(silu_ctx *c, int idx, char *name, int name_len, int64_t *launches, double *ms, double *bytes,
                   double *layout_bytes)
{
    if (!c || idx < 0 || idx >= (int)c->knames.size()) return SILU_ERR_ARG;
    if (name && name_len > 0) {
        std::strncpy(name, c->knames[(size_t)idx].c_str(), (size_t)name_len - 1);
        name[name_len - 1] = 0;
    }
    if (launches) *launches = c->klaunch[(size_t)idx];
    if (ms) *ms = c->kms[(size_t)idx];
    if (bytes) *bytes = c->kbytes[(size_t)idx];
    if (layout_bytes) *layout_bytes = c->klayout[(size_t)idx];
    return SILU_OK;
}

int silu_stats_reset(silu_ctx *c)
{
    if (!c) return SILU_ERR_ARG;
    int st = silu_stats_collect(c);
    if (st < 0) return st;
    for (size_t i = 0; i < c->knames.size(); i++) {
        c->klaunch[i] = 0;
        c->kms[i] = 0.0;
        c->kbytes[i] = 0.0;
        c->klayout[i] = 0.0;
    }
    return SILU_OK;
}

int silu_stream_copy(silu_ctx *c, const void *src, void *dst, size_t bytes)
{
    if (!c || !src || !dst || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return SILU_ERR_ARG;
    return timed_launch(c, 2.0 * (double)bytes, [&](const char **nm) {
        *nm = "stream_copy";
        return launch_copy(src, dst, bytes, c->stream);
    });
}

int silu_reorder_vectors(silu_ctx *c, const silu_csr *A, const silu_factors *F, const double *src, double *dst,
                         int to_relabeled)
{
    if (!c || !A || !F || !src || !dst || src == dst || (to_relabeled != 0 && to_relabeled != 1)) return SILU_ERR_ARG;
    int st = check_square(A, SILU_F64);
    if (st) return st;
    if ((st = check_square(&F->Ls, SILU_F64))) return st;
    if ((st = check_square(&F->Us, SILU_F64))) return st;
    const int64_t n = A->n_rows;
    if (F->Ls.n_rows != n || F->Us.n_rows != n) return SILU_ERR_SHAPE;
    if (!F->dinv || (!F->scaled && !F->d) || (F->scaled == 2 && !F->dc)) return SILU_ERR_ARG;
    Reorder *R = nullptr;
    if ((st = get_reorder(c, A, F, &R))) return st;
    return timed_launch(c, 20.0 * (double)n, [&](const char **nm) {
        *nm = to_relabeled ? "reorder_in" : "reorder_out";
        return to_relabeled ? launch_permute_in((int)n, R->pos, src, nullptr, dst, nullptr, c->stream)
                            : launch_scatter((int)n, R->order, src, dst, c->stream);
    });
}

int silu_stream_read(silu_ctx *c, const void *src, size_t bytes, void *out)
{
    if (!c || !src || !out || bytes == 0 || bytes % 49152 || ((uintptr_t)src & 15) || ((uintptr_t)out & 7))
        return SILU_ERR_ARG;
    return timed_launch(c, (double)bytes + (double)(bytes / 24), [&](const char **nm) {
        *nm = "stream_read";
        return launch_read(src, bytes, out, c->stream);
    });
}

} // extern "C"
