// Internal declarations of libscaledilu.so (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/scaled_ilu.h"

namespace silu {

// What a CSR sweep kernel does with t_i = rhs_i - sum_j N_ij xin_j (after
// rounding t to the iterate type IT of its precision):
enum Epi : int {
    EPI_STORE = 0,        // out_i = t_i
    EPI_SCALE = 1,        // out_i = dinv_i * t_i                  (s = D^{-1} y)
    EPI_UPDATE = 2,       // x_i = x_i + c_i * t_i                 (x += z)
    EPI_SCALE_UPDATE = 3, // x_i = x_i + c_i * (OT)(dinv_i * t_i)  (x += D^{-1} y when m_U = 1)
    EPI_SPMV = 4,         // out_i = sum_j N_ij xin_j  (no rhs; the product A z of the Krylov solver)
    EPI_STORE_SPLIT = 5   // out_i = t_i and out32_i = (float) t_i  (r and the FP32-inner form's y_1)
};
// c_i is the column factor d_c,i of the row/column scaling (SweepArgs::dcol),
// or 1 (an exact multiplication) when dcol is null.

// Precision of one sweep launch.
enum class Prec : int {
    F64 = 0,     // FP64 matrix, iterate, rhs, accumulation (residual and FP64 sweeps)
    MIX_RES = 1, // FP64 residual whose result is rounded to FP32 before D^{-1} (mixed, m_L = 1)
    MIX_L = 2,   // FP32 matrix/iterate/accumulation, FP64 rhs r (mixed L sweeps)
    MIX_U = 3,   // FP32 matrix/iterate/accumulation/rhs (mixed U sweeps)
    MIX_L1 = 4   // first mixed L sweep: gathers y_1 = r from the FP64 residual, rounding each value to FP32
};

enum class SweepKernel : int { STREAM = 0, VECTOR = 1, BLOCKED = 2, SLICED = 3 };

// Sliced-ELL copy of a CSR matrix (64-row slices, one wavefront per slice;
// built once per matrix on the device and cached).  code: bytes per column
// code -- 1 (index into the table of distinct diagonals col - row), 2
// (slice-relative offset col - 64 s - shift) or 4 (the column); 8: row
// patterns (below); 16: diagonal slices (below).
// Iterate windows of the row-pattern sweep: at most this many per matrix.
constexpr int PAT_WIN_MAX = 12;

struct SlicedView {
    int nslice = 0;
    int code = 4;
    const int32_t *sptr = nullptr; // [nslice] first slot of each slice
    const int32_t *sk = nullptr;   // [nslice] K rounded up to 4 | bit 31 when rows must be masked
    const void *val = nullptr;     // [slots] values (FP64 or FP32)
    const void *codes = nullptr;   // [slots]
    const int32_t *dtab = nullptr; // code 1: diagonal of each index [ndiag <= 256]
    int ndiag = 0;
    int shift = 0;                 // code 2
    int64_t slots = 0;
    int gmax = 0;                  // most groups of four slots in one slice
    // code 8 (row patterns): no per-slot code; row r's slots gather at
    // r + ptab[pid[r] * kp + k] (the row's offsets col - r in ascending order,
    // the last one repeated into its padded slots)
    const uint8_t *pid = nullptr;  // [nslice * 64] pattern of each row
    const int32_t *ptab = nullptr; // [npat * kp]
    int npat = 0, kp = 0;
    // iterate windows of code 8 (nwin = 0: none): the table's offsets fall
    // in nwin runs, run c covering offsets [wst[c], wst[c] + 64] (wst[c]
    // even, ascending), so the 64 rows of a slice starting at row r0 gather
    // only from x[r0 + wst[c] .. r0 + wst[c] + 127];
    // ltab[pid * kl + k] (k < kp; kl = kp rounded up to 8, for 16-byte
    // loads) is slot k's element in the wave's copy of those windows,
    // 128 c + ptab[pid * kp + k] - wst[c]; runs few slices need are left
    // out, and a slice with a row on one has wflag 0 (gathers)
    int nwin = 0, wspan = 0, kl = 0; // wspan = wst[nwin - 1] + 128 - wst[0]
    int32_t wst[PAT_WIN_MAX] = {};
    const uint16_t *ltab = nullptr;  // [npat * kl]
    const int32_t *wflag = nullptr;  // [nslice] 1: the slice's rows lie on the windows
    // code 16 (diagonal slices, FP64 or FP32 values): every row of the matrix lies
    // on the ndiag <= DIAG_MAX diagonals dtab[] (ascending); nslice slices of
    // 128 rows, slot k of row r holding its entry on diagonal dtab[k] (0 where
    // it has none) at val[diag_slot(r, k, ndiag)]
};
// Diagonal slices: at most this many diagonals, and at most 1/16 more slots
// than entries.
constexpr int DIAG_MAX = 32;
// The value slot of row r (slice r / 128) on the k-th of u diagonals: the
// slice's slots are diagonal-major, each diagonal's 128 rows consecutive.
__host__ __device__ inline int64_t diag_slot(int r, int k, int u)
{
    return ((int64_t)(r >> 7) * u + k) * 128 + (r & 127);
}
// Row-pattern tables are kept to at most this many offsets (16 KB, small
// enough to stay in the caches while a sweep reads it).
constexpr int PAT_MAX_ENTRIES = 4096;

// Row-block partition of the blocked CSR-stream kernel: at most RB_RMAX rows
// and RB_CAP entries per workgroup (a longer row gets a workgroup alone).
constexpr int RB_CAP = 2048;
constexpr int RB_RMAX = 1024;

struct SweepArgs {
    int n;
    const int32_t *rp;
    const int32_t *col;
    const void *val;
    const void *xin;      // iterate gathered through col
    const void *rhs;      // right-hand side of the Richardson step
    int epi;
    void *out;            // EPI_STORE / EPI_SCALE destination
    const double *dinv;   // EPI_SCALE / EPI_SCALE_UPDATE
    union {
        double *x;    // EPI_UPDATE / EPI_SCALE_UPDATE
        float *out32; // EPI_STORE_SPLIT: the FP32 copy of out
    };
    const double *dshift; // unscaled variant: adds (d_i - 1) * xin_i to the row sum (FP64 only)
    const double *dcol = nullptr; // EPI_UPDATE / EPI_SCALE_UPDATE: column factors c_i, or null (c_i = 1)
    const SlicedView *sv = nullptr; // batched sweeps: the op's sliced copy (device), or null: CSR-stream
    // batched sweeps of a solve request (null / 0 otherwise): the op does
    // nothing once sctl->stop is set; a check op (the residual at the start of
    // an outer step) also writes its tile's sums of r_i^2 (and, scheck == 2,
    // of b_i^2) to spart[2 tile], spart[2 tile + 1]
    const struct SolveCtl *sctl = nullptr;
    double *spart = nullptr;
    int scheck = 0;
};

// Device state of a solve request: the convergence test of eq. relres on the
// residual at the start of each outer step (its squared norm rr, that of b, bb,
// from the first check), the number of checks made, and the stop flag.
struct SolveCtl {
    int32_t stop;
    int32_t checks;
    double rr;
    double bb;
    double pad;
};

// One launch that closes the checks of a step: workgroup i sums the tile
// partials of check i in a fixed order and updates its SolveCtl (unless it
// has stopped already): stop when sqrt(rr) / sqrt(bb) < tol.
constexpr int SOLVE_CHECKS_PER_LAUNCH = 32;
struct SolveCheck {
    SolveCtl *ctl;
    const double *part;
    int tiles;
    int first; // the first check: bb comes from this one's partials
    double tol;
    int32_t *hflag; // pinned host word set to 1 with the stop flag (or null)
};
struct SolveCheckArgs {
    SolveCheck c[SOLVE_CHECKS_PER_LAUNCH];
    int count;
};
hipError_t launch_solve_check(const SolveCheckArgs &a, hipStream_t s);

// Kernel geometry for a sweep, picked from the mean row length.
struct SweepGeom {
    SweepKernel kind;
    int rows_per_block;           // STREAM: rows per workgroup
    int lanes;                    // VECTOR: lanes per row
    int cap = RB_CAP;             // BLOCKED: entries per row block
    const int32_t *blk = nullptr; // BLOCKED: device (row start, entry start) pairs [nblk + 1]
    int nblk = 0;
    bool allow16 = false;             // STREAM: may use 16-bit block-relative column offsets
    const uint16_t *off16 = nullptr;  // STREAM: offsets (col = r0 + shift + off16[e]) when available
    int shift = 0;
    bool allow_win = false;           // STREAM: may stage the iterate window in LDS
    bool prefer_win = false;          // STREAM: window even where 16-bit offsets fit
    SlicedView sl;                    // SLICED: the sliced copy (attached by the caller)
    int slice_code_min = 1;           // SLICED: narrowest column code allowed (1, 2 or 4 bytes)
    bool slice_prefetch = true;       // SLICED: a slice's loads all issued up front where it fits
    const uint16_t *slot16 = nullptr; // STREAM, windowed: LDS slot of each entry's iterate value
    const int32_t *wo = nullptr;      // STREAM, windowed: block-relative offset of each slot [lw]
    int lw = 0;
};

// Block-relative 16-bit column offsets for the CSR-stream kernel with `rpb`
// rows per workgroup.  offset_range writes min and max of col - r0(block) over
// all entries into range[0], range[1] (initialised to INT_MAX, INT_MIN);
// compress16 writes off16[e] = col - r0(block) - shift.
hipError_t launch_offset_range(int n, const int32_t *rp, const int32_t *col, int rpb, int32_t *range, hipStream_t s);
hipError_t launch_compress16(int n, const int32_t *rp, const int32_t *col, int rpb, int shift, uint16_t *off16,
                             hipStream_t s);
// Windowed CSR-stream: the block-relative offsets o = col - r0(block) that
// occur anywhere in the matrix, numbered in increasing order, are the LDS
// slots of every workgroup's staged iterate window.  mark_offsets sets
// used[o - lo]; encode_slots writes code[e] = slot_of[o - lo].
hipError_t launch_mark_offsets(int n, const int32_t *rp, const int32_t *col, int rpb, int lo, uint8_t *used,
                               hipStream_t s);
hipError_t launch_encode_slots(int n, const int32_t *rp, const int32_t *col, int rpb, int lo, const int32_t *slot_of,
                               uint16_t *code, hipStream_t s);
// Polynomial Gauss-Seidel set-up: strictly-lower counts (with pattern and
// pivot flags), then Gs = D^{-1} L, d and dinv.
hipError_t launch_gs_count(int n, const int32_t *rp, const int32_t *col, const double *val, int32_t *counts,
                           int32_t *flags, hipStream_t s);
hipError_t launch_gs_fill(int n, const int32_t *rp, const int32_t *col, const double *val, const int32_t *Grp,
                          int32_t *Gcol, double *Gval, double *d, double *dinv, float *G32, int32_t gs_nnz,
                          hipStream_t s);
// Sliced-ELL set-up: per-slice K and mask bit; fill values and codes.
hipError_t launch_slice_meta(int n, int nslice, const int32_t *rp, int32_t *sk, hipStream_t s);
// Diagonal slices (code 16): zero the copy, then place every entry at its
// row's slot on diagonal dmap[col - row - lo].
hipError_t launch_fill_diag(int n, int nslice, int u, const int32_t *rp, const int32_t *col, const void *val,
                            int val_bytes, const int32_t *dmap, int lo, void *sval, hipStream_t s);
hipError_t launch_fill_sliced(int n, int nslice, const int32_t *rp, const int32_t *col, const void *val, int val_bytes,
                              const int32_t *sptr, const int32_t *sk, int code, const int32_t *dmap, int lo,
                              void *sval, void *scode, hipStream_t s);
// Krylov vector kernels (krylov.hip).  launch_dot writes a . b (or its
// square root) to out[0] on the device, reducing in a fixed order through
// part[DOT_BLOCKS]; the others update with a device (h[0]) or host scalar.
constexpr int DOT_BLOCKS = 1024;
hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, double *out, bool take_sqrt,
                      hipStream_t s);
hipError_t launch_sub_scaled(int64_t n, double *w, const double *v, const double *h, hipStream_t s);
hipError_t launch_div_dev(int64_t n, const double *w, const double *h, double *out, hipStream_t s);
hipError_t launch_div_host(int64_t n, const double *w, double d, double *out, hipStream_t s);
hipError_t launch_axpy_host(int64_t n, double alpha, const double *z, double *x, hipStream_t s);
// ILU(0) by fixed-point sweeps (fixedpoint.hip): diagonal positions and the
// row of every entry, the initial guess, one synchronous sweep (flags[1] set
// when a value changed), and the split into Ls and U.
hipError_t launch_fp_index(int n, const int32_t *rp, const int32_t *col, int32_t *dpos, int32_t *row_of,
                           int32_t *flags, hipStream_t s);
hipError_t launch_fp_init(int64_t nnz, const int32_t *col, const double *val, const int32_t *dpos,
                          const int32_t *row_of, double *LU, hipStream_t s);
hipError_t launch_fp_sweep(int64_t nnz, const int32_t *rp, const int32_t *col, const double *val, const int32_t *dpos,
                           const int32_t *row_of, const double *old, double *nw, int32_t *flags, hipStream_t s);
hipError_t launch_fp_split(int n, const int32_t *rp, const int32_t *col, const double *LU, const int32_t *Lrp,
                           int32_t *Lcol, double *Lval, const int32_t *Urp, int32_t *Ucol, double *Uval, int64_t l_nnz,
                           int64_t u_nnz, hipStream_t s);
// Locality relabeling (reorder.hip): order[k] = the row placed at position k,
// pos = its inverse.  relabel writes row k of N' = Q N Q^T (rp2 given, entries
// in the original order, columns through pos; col2 may be null to copy values
// only); gather dst[k] = src[order[k]]; scatter dst[order[k]] = src[k].
hipError_t launch_relabel(int n, const int32_t *order, const int32_t *pos, const int32_t *rp, const int32_t *col,
                          const void *val, int val_bytes, const int32_t *rp2, int32_t *col2, void *val2,
                          hipStream_t s);
hipError_t launch_gather(int n, const int32_t *order, const double *src, double *dst, hipStream_t s);
// b2[pos[i]] = b[i], and x2[pos[i]] = x[i] when x is not null
hipError_t launch_permute_in(int n, const int32_t *pos, const double *b, const double *x, double *b2, double *x2,
                             hipStream_t s);
hipError_t launch_scatter(int n, const int32_t *order, const double *src, double *dst, hipStream_t s);
int rcm_strength_order(int64_t n, const int32_t *rp, const int32_t *col, const double *val, double theta,
                       int32_t *order);
constexpr double REORDER_THETA = 0.25;

// Largest window (LDS slots) the windowed sweep stages per workgroup.
constexpr int WIN_MAX_SLOTS = 3072;

SweepGeom pick_geom(int64_t n, int64_t nnz, int flags);

// A sliced-ELL copy of N with the values `val` (vbytes 8: FP64, 4: FP32)
// owned by the caller (the serving runtime), outside the context's cache, so
// that releasing cached layouts never frees it.  view->nslice stays 0 (and
// *owner null) when N is better streamed as CSR.  free_owned_sliced frees it;
// null is ignored.
int make_owned_sliced(silu_ctx *c, const silu_csr *N, const void *val, int vbytes, SlicedView *view, void **owner);
void free_owned_sliced(void *owner);
hipError_t launch_sweep(Prec p, const SweepGeom &g, const SweepArgs &a, hipStream_t s, const char **name);

// Batched sweeps of one precision (serving): d_ops[i] is one request's sweep,
// d_first[i] its first workgroup (ceil(n_i / SERVE_TILE_ROWS) workgroups
// each), total the sum.  Both arrays live in device memory.  An op whose sv
// points to a sliced copy (device memory) is swept through it, else as a CSR
// stream.
constexpr int SERVE_TILE_ROWS = 256;
hipError_t launch_sweep_batch(Prec p, const SweepArgs *d_ops, const int32_t *d_first, int nops, int total,
                              hipStream_t s);
// The same with the op table passed in the kernel arguments (no copy to the
// device first): at most BATCH_ARG_OPS ops.
constexpr int BATCH_ARG_OPS = 24;
struct BatchArgs {
    SweepArgs op[BATCH_ARG_OPS];
    int32_t first[BATCH_ARG_OPS + 1];
    int nops;
};
hipError_t launch_sweep_batch_args(Prec p, const BatchArgs &b, hipStream_t s);

// Persistent batched FP64 CSR-stream sweeps (serving): one launch runs chains
// of dependent sweeps.  Op i covers tiles [first[i], first[i+1]) of
// PERSIST_RPB rows and may start once done[dep[i]] == first[dep[i]+1] -
// first[dep[i]] (dep[i] < i, or -1).  ctl[0] (next tile) and ctl[1] (0, or
// 1 + the op whose wait expired) and done[] must be zero at launch; all of it
// lives in device memory.  Any grid size >= 1 drains the queue.
constexpr int PERSIST_RPB = 256;
struct PersistPlan {
    int32_t *ctl;
    const int32_t *first; // [nops + 1]
    const int32_t *dep;   // [nops]
    int32_t *done;        // [nops]
    const SweepArgs *ops; // [nops]
    int nops;
    long long wait_ticks; // wall-clock ticks (wall_clock64) a wait may take before it gives up (>= 1)
};
constexpr int PERSIST_WAIT_US = 200000; // default bound of one wait, in microseconds
hipError_t launch_sweep_persist(const PersistPlan &p, int grid, hipStream_t s);

struct LevelArgs {
    const int32_t *perm; // rows ordered by level
    const int32_t *rp;
    const int32_t *col;
    const double *val;
    const double *rhs;
    double *out;
    const double *dinv; // optional: s_out = dinv * out
    double *s_out;
    double *xupd;       // optional: xupd += out (xupd += dcol * out with dcol)
    const double *dcol = nullptr;
};
// lanes: 1 (one lane per row, sequential row sum) or 4/8/16/32 lanes per row.
hipError_t launch_level(const LevelArgs &a, int unit, int lanes, int start, int count, hipStream_t s,
                        const char **name);

hipError_t launch_scale_rows(int n, const int32_t *Urp, const int32_t *Ucol, const double *Uval, int32_t *Usrp,
                             int32_t *Uscol, double *Usval, double *d, double *dinv, float *Us32, int noscale,
                             int32_t us_nnz, int32_t *flags, hipStream_t s);
hipError_t launch_to_f32(int64_t n, const double *src, float *dst, hipStream_t s);
// x_i += s_i, or x_i += dcol_i * s_i with dcol (row/column scaling)
hipError_t launch_axpy(int n, const void *s_vec, int s_is_f32, const double *dcol, double *x, hipStream_t s);
// Row/column scaling set-up (Ruiz steps in the max norm, then the unit
// diagonal): fill, one max pass, one factor update, and the final write of
// d_r and the strictly upper values of D_r U D_c.
hipError_t launch_fill(int n, double *a, double va, double *b, double vb, hipStream_t s);
hipError_t launch_ruiz_max(int n, const int32_t *Urp, const int32_t *Ucol, const double *Uval, const double *dr,
                           const double *dc, double *rmax, unsigned long long *cmax, int32_t *flags, hipStream_t s);
hipError_t launch_ruiz_scale(int n, double *dr, double *dc, const double *rmax, const unsigned long long *cmax,
                             hipStream_t s);
hipError_t launch_rowcol_finish(int n, const int32_t *Urp, const int32_t *Ucol, const double *Uval,
                                const double *dc, double *dr, double *Usval, float *Us32, int32_t us_nnz,
                                hipStream_t s);
hipError_t launch_init_flags(int32_t *flags, int count, int32_t value, hipStream_t s);
hipError_t launch_finite_check(int n, const double *x, int32_t *flags, hipStream_t s);
hipError_t launch_scale_copy(int n, const double *rhs, const double *dinv, double *out, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
// Read-dominant calibration stream: reads `bytes` (a multiple of 49,152), writes bytes / 24 to out.
hipError_t launch_read(const void *src, size_t bytes, void *out, hipStream_t s);

}  // namespace silu
