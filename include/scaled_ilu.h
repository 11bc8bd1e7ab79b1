/*
 * scaled_ilu.h -- C-ABI of libscaledilu.so, the MI355X (gfx950) solve phase of
 * the scaled ILU smoother of Thomas, Carr, Mullowney, Swirydowicz and Day,
 * "Scaled ILU Smoothers for Navier-Stokes Pressure Projection"
 * (arXiv 2111.09512).
 *
 * The smoother step is x <- x + M^{-1} (b - A x) with M = L D U~ (Section 3.1,
 * eq. ILUsplit).  Its two triangular solves are replaced by a few Richardson
 * sweeps on the unit-diagonal factors, the row scaling D^{-1} having been
 * folded into U once (Section 5.1, eqs. extractD and newD; Algorithm 2;
 * Section 5.2, eq. richard).  Each sweep is one CSR pass over a strictly
 * triangular factor.  The level-scheduled direct triangular solve (Section 4)
 * is provided as the comparison solve.
 *
 * Conventions shared by every entry point
 *   - Matrices are CSR with int32 row pointers and column indices, columns
 *     sorted ascending and unique inside each row.  All sizes < 2^31.
 *   - Unless stated otherwise every pointer is a DEVICE pointer on the device
 *     that was current when the context was created.  The caller owns every
 *     buffer it passes (matrices, vectors, workspace) and keeps it alive until
 *     the work queued on the context's stream has passed the call.  The library
 *     never frees caller memory.
 *   - Calls marked "asynchronous" only enqueue work on the context's stream and
 *     return; calls marked "synchronous" wait for their own work to finish.
 *   - Every entry point returns an int status: SILU_OK (0) or a negative code
 *     below.  Nothing throws and nothing exits across the ABI.  After
 *     SILU_ERR_HIP, silu_last_hip_error() gives the HIP error code.
 */
#ifndef SCALED_ILU_H
#define SCALED_ILU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SILU_OK 0
#define SILU_ERR_ARG (-1)         /* null pointer, negative size, bad flag or count */
#define SILU_ERR_SHAPE (-2)       /* dimension mismatch or non-square matrix */
#define SILU_ERR_PATTERN (-3)     /* CSR structure violates the stated pattern */
#define SILU_ERR_ZERO_PIVOT (-4)  /* u_ii == 0 or not finite; see silu_bad_row() */
#define SILU_ERR_NONFINITE (-5)   /* SILU_CHECK_FINITE found a NaN/Inf in x */
#define SILU_ERR_NOMEM (-6)       /* caller workspace smaller than silu_workspace_size() */
#define SILU_ERR_HIP (-7)         /* a HIP runtime call failed */
#define SILU_ERR_UNSUPPORTED (-8) /* valid request this library version does not implement */
#define SILU_ERR_TIMEOUT (-9)     /* a persistent serving launch gave up a bounded wait */

/* ---- value types of silu_csr.val ------------------------------------- */
#define SILU_F64 0
#define SILU_F32 1

/* ---- flags ------------------------------------------------------------- */
#define SILU_ITER 0x0         /* ilu_smooth: Richardson sweeps (default)                  */
#define SILU_DIRECT 0x1       /* ilu_smooth: level-scheduled substitution instead          */
#define SILU_MIXED 0x2        /* ilu_smooth: FP32 factor values, iterates, accumulation    */
#define SILU_CHECK_FINITE 0x4 /* ilu_smooth: after the step, scan x (synchronous)          */
#define SILU_VALIDATE 0x8     /* check CSR structure first (synchronous; copies to host)   */
#define SILU_NO_SCALING 0x10  /* ilu_scale_factors: keep U's values (the unscaled variant) */
#define SILU_KERNEL_STREAM 0x100  /* CSR-stream sweep kernel (instead of the sliced default)   */
#define SILU_KERNEL_VECTOR 0x200  /* vector-CSR (lanes-per-row) sweep kernel                */
#define SILU_KERNEL_BLOCKED 0x400 /* CSR-stream over a row-block partition                  */
#define SILU_NO_GRAPH 0x800       /* level-scheduled solves: plain launches, no hipGraph     */
#define SILU_INDEX32 0x1000       /* sweeps read the 32-bit col_idx, never 16-bit codes      */
#define SILU_NO_WINDOW 0x2000     /* sweeps never stage the iterate window in LDS            */
#define SILU_WINDOW 0x4000        /* sweeps stage the window wherever it fits                */
#define SILU_CODE16 0x8000        /* sliced sweeps: no diagonal table (16-bit codes or wider) */
#define SILU_ZERO_GUESS 0x10000   /* ilu_smooth: x is zero on entry, so the first residual   */
                                  /* is b itself (skips one pass over A when m_L >= 2)       */
#define SILU_GRAPH 0x20000        /* ilu_smooth: replay the call's sweeps from a hipGraph    */
#define SILU_REORDER 0x40000      /* ilu_smooth: sweep locality-relabeled copies             */
#define SILU_SLICED_LOOP 0x80000  /* sliced sweeps: two groups of slots in flight at a time   */
#define SILU_CODE8 0x100000       /* sliced sweeps: a 1-byte diagonal code per slot instead of */
                                  /* the per-row pattern table                                */
#define SILU_RELABELED 0x200000   /* ilu_smooth with SILU_REORDER: b and x are already in the  */
                                  /* relabeled order (silu_reorder_vectors); no permutations  */
#define SILU_ROWPAT 0x400000      /* sliced sweeps: the per-row pattern table even where every  */
                                  /* row lies on a few diagonals (no diagonal slices)          */

#define SILU_LOWER 0
#define SILU_UPPER 1
#define SILU_UNIT 0
#define SILU_NONUNIT 1

/* Square sparse matrix (n_rows == n_cols) in CSR form. */
typedef struct {
    int64_t n_rows;
    int64_t n_cols;
    int64_t nnz;
    int32_t *row_ptr; /* [n_rows + 1] */
    int32_t *col_idx; /* [nnz]        */
    void *val;        /* [nnz] of dtype */
    int32_t dtype;    /* SILU_F64 or SILU_F32 */
} silu_csr;

/*
 * The factors the smoother reads, all on the device.
 *   Ls       strictly lower part of L = I + Ls (the unit diagonal is implied),
 *            FP64 values.  ilu_scale_factors copies the caller's L here.
 *   Us       strictly upper part of U~ = D^{-1} U (eq. newD), FP64; written by
 *            ilu_scale_factors into caller-allocated arrays: row_ptr [n+1],
 *            col_idx and val [nnz(U) - n].  With SILU_NO_SCALING, Us holds
 *            the strictly upper part of U itself.
 *            After ilu_scale_factors_rowcol, Us holds the strictly upper part
 *            of U^ = D_r U D_c (eq. rowcolScale) instead.
 *   d        diag(U) [n] (eq. extractD)
 *   dinv     the row factor applied to y before the U solve [n]:
 *            1 / diag(U) after row scaling, d_r after row/column scaling
 *   Ls_val32 optional FP32 copy of Ls.val (round to nearest even), or NULL
 *   Us_val32 optional FP32 copy of Us.val, or NULL
 *   scaled   1 after row scaling, 0 with SILU_NO_SCALING, 2 after
 *            row/column scaling, 3 for the Gauss-Seidel split (gs_scale_split)
 *   dc       column factors d_c [n] (scaled == 2: the smoother adds d_c * v
 *            to x, v the U^ iterate), else ignored (may be NULL)
 */
typedef struct {
    silu_csr Ls;
    silu_csr Us;
    double *d;
    double *dinv;
    float *Ls_val32;
    float *Us_val32;
    int32_t scaled;
    double *dc;
} silu_factors;

typedef struct silu_ctx silu_ctx;

/* ---- context ----------------------------------------------------------- */

/* Create a context on the current device that enqueues on `hip_stream` (a
 * hipStream_t; NULL = the null stream).  The stream is borrowed, not owned.
 * The context owns its level analyses, graphs, events and a few bytes of
 * device flags, all freed by silu_destroy.  Synchronous. */
int silu_create(silu_ctx **ctx, void *hip_stream);
int silu_destroy(silu_ctx *ctx);
/* Change the stream later calls enqueue on (borrowed). */
int silu_set_stream(silu_ctx *ctx, void *hip_stream);

/* Row of the last ZERO_PIVOT / PATTERN error, or -1. */
int64_t silu_bad_row(const silu_ctx *ctx);
/* HIP error code behind the last SILU_ERR_HIP on this context (0 if none). */
int silu_last_hip_error(const silu_ctx *ctx);
/* Static description of a status code. */
const char *silu_status_string(int status);

/* Workspace bytes ilu_smooth / trisolve_iter need for n rows under `flags`.
 * The caller allocates the workspace (at least 256-byte aligned) and passes
 * it in, so every byte the library touches is visible to the caller. */
int silu_workspace_size(silu_ctx *ctx, int64_t n, int flags, size_t *bytes);

/* ---- setup: row scaling (Section 5.1, eqs. extractD and newD) ----------- */

/*
 * L: strictly lower CSR (unit diagonal implied), FP64.  U: upper CSR, FP64,
 * whose FIRST entry in every row is the diagonal.  Writes, in F:
 *   F->Ls = *L;  F->d[i] = u_ii;  F->dinv[i] = 1/u_ii;
 *   F->Us (row_ptr, col_idx, val) = strictly upper part of U with every value
 *   divided by its row's diagonal (one IEEE division per entry), or copied
 *   unchanged with SILU_NO_SCALING;
 *   F->Ls_val32 / F->Us_val32 if non-NULL: FP32 copies of the values.
 * The caller allocates F->Us.row_ptr [n+1], F->Us.col_idx and F->Us.val
 * [nnz(U)-n] (FP64), F->d and F->dinv [n], and the optional FP32 arrays.
 * Synchronous.  Errors: ARG, SHAPE, PATTERN (a row of U does not start with
 * its diagonal), ZERO_PIVOT (u_ii == 0 or not finite; silu_bad_row gives the
 * first such row).
 */
int ilu_scale_factors(silu_ctx *ctx, const silu_csr *L, const silu_csr *U, silu_factors *F, int flags);

/* ---- setup: row/column scaling (Section 5.1, eq. rowcolScale) ------------ */

/*
 * The paper's second scaling: the Richardson loop on U runs on
 * U^ = D_r U D_c, which has a unit diagonal, and U z = y is solved as
 * U^ v = D_r y, z = D_c v.  The paper names Ruiz scaling (Table 2) without
 * further detail; this library's reading:
 *   d_r = d_c = 1; then `ruiz_iters` times, with a_ij = (|u_ij| d_r,i) d_c,j,
 *     d_r,i *= 1/sqrt(max_j a_ij),  d_c,j *= 1/sqrt(max_i a_ij)
 *   (both maxima of a step from the same a); finally the unit diagonal fixes
 *   the row factor, d_r,i = 1/(u_ii d_c,i), and u^_ij = (u_ij d_r,i) d_c,j.
 * So U^ = D_c^{-1} (D^{-1} U) D_c: a diagonal similarity of the row-scaled
 * factor, with the same truncated Neumann sums in exact arithmetic and a
 * different departure from normality (eq. depB).
 * Same arguments and ownership as ilu_scale_factors, plus F->dc [n] (caller
 * allocated); writes F->Us (values of U^), F->d = diag(U), F->dinv = d_r,
 * F->dc = d_c, F->scaled = 2, and the optional FP32 copies.
 * ruiz_iters in [0, 100] (0: d_c = 1, which is the row scaling up to
 * rounding).  Allocates 16 n bytes of temporary device memory for the call.
 * Synchronous.  Errors: as ilu_scale_factors, and ARG for ruiz_iters out of
 * range or F->dc == NULL; PATTERN also for a column index outside [0, n).
 */
int ilu_scale_factors_rowcol(silu_ctx *ctx, const silu_csr *L, const silu_csr *U, int ruiz_iters, silu_factors *F,
                             int flags);

/* ---- the smoother (eq. ILUsplit, Algorithm 2, eq. richard) -------------- */

/*
 * Layout the sweeps read.  By default the first sweep over a matrix (A, Ls,
 * Us, and the FP32 value arrays in the mixed form) builds on the device a
 * sliced copy of it and caches it in the context: 64-row slices (one
 * wavefront each), entry k of every row of a slice stored contiguously,
 * short rows padded to the slice's longest with value 0 at the row's last
 * column, and a column code per slot -- 1 byte (an index into the table of
 * the matrix's distinct diagonals col - row, when there are at most 256: a
 * stencil operator and its ILU factors), else 2 bytes (slice-relative offset,
 * when it fits); a matrix with neither structure (random columns) is swept
 * in CSR-stream instead (SILU_INDEX32 forces a sliced copy with 4-byte
 * columns).  Each row's products are still added
 * in ascending column order, so finite results are bit-identical to the
 * row-by-row definition; a padded slot adds +0.0.  The first use synchronizes
 * a few times.  The copy holds the VALUES as they were at that first sweep:
 * a caller that changes a matrix's values in place afterwards must call
 * silu_release(ctx, row_ptr, col_idx) first (ilu_scale_factors does this for
 * the factors it writes; the Python binding does it whenever a tensor's
 * version changes).  SILU_CODE16 skips the diagonal table; SILU_INDEX32 keeps
 * 4-byte columns.
 *
 * With SILU_KERNEL_STREAM the sweeps read the CSR arrays themselves
 * (CSR-stream), with a 16-bit code per entry when the matrix allows it, also
 * built on the first sweep and cached (2 bytes per entry, structure only):
 *  - offsets (preferred): when every block-relative offset col - r0 (r0 =
 *    the first row of the entry's row block) lies within a span of 65,536,
 *    the code is the offset;
 *  - windowed: else when the distinct offsets that occur number at most
 *    3072 (a wide stencil operator), each workgroup stages the iterate
 *    values at those offsets into LDS and the code is the LDS slot;
 *    SILU_WINDOW prefers this mode wherever it fits;
 *  - else (a randomly permuted matrix) col_idx itself.
 * SILU_NO_WINDOW keeps to offsets; SILU_INDEX32 always reads col_idx.
 *
 * `outer_sweeps` smoothing steps on x (in/out; x = 0 for a pure
 * preconditioner application):
 *   r = b - A x;  y = m_L Richardson steps on L y = r from y = 0;
 *   s = D^{-1} y;  z = m_U Richardson steps on U~ z = s from z = 0;  x += z.
 * With row/column-scaled factors (F->scaled == 2): s = d_r * y, v = m_U
 * steps on U^ v = s, x += d_c * v (and with SILU_MIXED, x += d_c * (double)v).
 * A: n x n FP64 CSR.  F: from ilu_scale_factors.  b, x: FP64 [n].
 * flags: SILU_DIRECT replaces both Richardson loops by level-scheduled
 * substitution (m_L, m_U ignored); SILU_MIXED runs the two Richardson loops on
 * F->Ls_val32 / F->Us_val32 with FP32 iterates and accumulation (r, the
 * scaling s = (float)(dinv * y) and x += z stay FP64); SILU_CHECK_FINITE adds
 * a synchronous scan of x (returns NONFINITE); SILU_VALIDATE checks the CSR
 * structures first.  With F->scaled == 0 (SILU_NO_SCALING) the U loop is the
 * unscaled Richardson iteration z <- y - (U - I) z (FP64 only).
 * SILU_GRAPH (iterative form; ignored with SILU_DIRECT, whose level sweeps
 * are captured anyway): the first call with a given set of arguments (the
 * matrices' and vectors' pointers, sizes, counts and flags) runs as usual and
 * then records its whole launch sequence into a hipGraph kept in the context;
 * later calls with the same arguments replay it with one launch, on the same
 * data layouts, with the same results bit for bit.  The graph bakes in the
 * pointers: the caller keeps b, x and ws at those addresses, and any
 * silu_release on the context drops every recorded graph (the cached layouts
 * they read may be rebuilt).  If the sequence cannot be recorded the call
 * still succeeds and later calls run unrecorded.
 * SILU_REORDER (iterative form; UNSUPPORTED with SILU_DIRECT): the sweeps run
 * on copies of A and the factors whose rows and columns are relabeled so that
 * strongly coupled rows sit next to each other (silu_reorder_rcm, theta 0.25,
 * from A's values), each row keeping its entries in their original order;
 * b and x are permuted in and x back out by the call.  A Richardson sweep
 * updates all rows from the previous iterate, so the relabeling changes
 * nothing in the arithmetic: results are bit-identical to the call without
 * the flag.  It pays where the given order scatters the gathers (a randomly
 * permuted matrix).  The copies are built on the first call (synchronous: A
 * is read back to order it on the host) and cached like the sliced copies;
 * silu_release of A or a factor drops them.  The workspace grows to six
 * n-vectors (silu_workspace_size with the flag).
 * ws: workspace of at least silu_workspace_size(ctx, n, flags) bytes.
 * Asynchronous on the context stream (unless CHECK_FINITE / VALIDATE).
 * Errors: ARG (null, outer_sweeps < 1, m_L < 1 or m_U < 1 in ITER mode,
 * F->scaled == 2 without F->dc), SHAPE, NOMEM (ws_bytes too small), UNSUPPORTED (MIXED without FP32 copies,
 * MIXED or DIRECT with unscaled factors), PATTERN (with VALIDATE), NONFINITE,
 * HIP.
 */
int ilu_smooth(silu_ctx *ctx, const silu_csr *A, const silu_factors *F, const double *b, double *x,
               int outer_sweeps, int inner_iters, int flags, void *ws, size_t ws_bytes);
/* Same with separate inner iteration counts for the L and the U factor. */
int ilu_smooth2(silu_ctx *ctx, const silu_csr *A, const silu_factors *F, const double *b, double *x,
                int outer_sweeps, int m_L, int m_U, int flags, void *ws, size_t ws_bytes);

/* Moves a vector into the order of the SILU_REORDER copies of (A, F)
 * (to_relabeled = 1: dst[k] = src[order[k]]) or back (0: dst[order[k]] =
 * src[k]); the copies are built first if they are not cached (synchronous
 * then, as for ilu_smooth with SILU_REORDER).  A caller that smooths the same
 * vectors many times moves b and x in once, calls ilu_smooth with SILU_REORDER
 * | SILU_RELABELED (which then permutes nothing and needs only the four-vector
 * workspace of the plain call), and moves x back once; the result is the
 * plain call's bit for bit.  src, dst: device FP64 [n], distinct.
 * Asynchronous.  Errors: ARG, SHAPE, HIP. */
int silu_reorder_vectors(silu_ctx *ctx, const silu_csr *A, const silu_factors *F, const double *src, double *dst,
                         int to_relabeled);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * iterative ilu_smooth2 with its four work vectors in a scratch array the
 * library holds on each device (64 MiB, made with the code object and kept
 * until the process ends), so no workspace argument and no allocation: no
 * hipMalloc, no layout built.  Sweeps read the sliced or 16-bit layouts an
 * earlier ilu_smooth call with the same matrices and flags cached in the
 * context, else the caller's CSR arrays directly (same results bit for bit);
 * per-kernel timing is not recorded.  n at most 2,097,152 rows (four FP64
 * n-vectors, 256-byte rounded, in 64 MiB), else SILU_ERR_NOMEM.  flags: only
 * SILU_MIXED, SILU_ZERO_GUESS, SILU_CHECK_FINITE and the kernel-choice flags
 * (SILU_KERNEL_STREAM, SILU_KERNEL_VECTOR, SILU_INDEX32, SILU_NO_WINDOW,
 * SILU_CODE16, SILU_CODE8, SILU_ROWPAT, SILU_SLICED_LOOP), else SILU_ERR_ARG.  Every call
 * on one device shares that device's scratch array, which keeps the last
 * call's contents: calls that overlap on one GPU (other streams, other
 * contexts, other threads) race and must be ordered by the caller.
 * Asynchronous.  Errors: as ilu_smooth2, and HIP if the scratch array's
 * address could not be found when the context was created.
 */
int ilu_smooth_noalloc(silu_ctx *ctx, const silu_csr *A, const silu_factors *F, const double *b, double *x,
                       int outer_sweeps, int m_L, int m_U, int flags);

/* The relabeling of SILU_REORDER, on HOST arrays: reverse Cuthill-McKee on
 * the graph of strong couplings, row i coupled to j != i when |a_ij| >= theta
 * * max_{k != i} |a_ik| (the strength of connection of algebraic multigrid,
 * Section 3).  Each component starts from its unvisited row of least strong
 * degree; a row's unvisited strong neighbours are queued by increasing degree
 * (ties: lower index); the visit order is reversed.  order[k] receives the
 * row placed at position k (a permutation of 0..n-1).  row_ptr [n+1], col_idx
 * and val [nnz] (FP64) are read only; order [n] is written.  Synchronous, no
 * GPU needed.  Errors: ARG (null, n < 0, theta < 0 or NaN), PATTERN (row
 * pointers decreasing, a column outside 0..n-1). */
int silu_reorder_rcm(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val, double theta,
                     int32_t *order);

/* ---- polynomial Gauss-Seidel smoother (Section 2) ------------------------ */

/*
 * The polynomial smoother the paper compares the ILU smoother with:
 * Gauss-Seidel's (D + L)^{-1} (D = diag(A), L = strictly lower part of A)
 * written as (I + D^{-1}L)^{-1} D^{-1}, the inverse replaced by a truncated
 * Neumann series of `terms` terms (terms = p + 1 for the paper's sum over
 * j = 0..p):
 *   x <- x + sum_{j<terms} (-D^{-1}L)^j D^{-1} (b - A x).
 *
 * gs_split_size: the number of strictly lower entries of A (synchronous).
 * gs_scale_split: writes G->Ls = D^{-1} L (row_ptr [n+1], col_idx and val
 * [that count], caller-allocated; g_ij = a_ij / a_ii, one IEEE division
 * each), G->d = diag(A), G->dinv = 1 / diag(A), G->Ls_val32 if non-NULL (FP32
 * copy), G->Us = an empty n x n matrix, G->scaled = 3.  Synchronous.
 * Errors (both): ARG, SHAPE, PATTERN (a row of A without its diagonal),
 * ZERO_PIVOT (a_ii == 0 or not finite; silu_bad_row gives the first row).
 */
int gs_split_size(silu_ctx *ctx, const silu_csr *A, int64_t *nnz_lower);
int gs_scale_split(silu_ctx *ctx, const silu_csr *A, silu_factors *G, int flags);

/*
 * `outer_sweeps` steps of the smoother on x (in/out), each
 *   s = D^{-1}(b - A x);  y = `terms` Richardson steps on (I + D^{-1}L) y = s
 *   from y = 0 (the first is free);  x += y.
 * G from gs_scale_split.  flags: SILU_MIXED runs the Richardson loop on
 * G->Ls_val32 with FP32 iterates and accumulation (the residual is computed
 * in FP64 and rounded to FP32 before the scaling; x += y in FP64);
 * SILU_CHECK_FINITE, SILU_VALIDATE, SILU_REORDER and the layout flags as for
 * ilu_smooth (G->Us may be empty).  Workspace as for ilu_smooth.
 * Asynchronous.  Errors: ARG (nulls,
 * outer_sweeps or terms < 1, SILU_DIRECT, G not from gs_scale_split), SHAPE,
 * NOMEM, UNSUPPORTED (MIXED without the FP32 copy), PATTERN, NONFINITE, HIP.
 */
int gs_smooth(silu_ctx *ctx, const silu_csr *A, const silu_factors *G, const double *b, double *x, int outer_sweeps,
              int terms, int flags, void *ws, size_t ws_bytes);

/* ---- ILU(0) on the device by fixed-point sweeps (Section 7) -------------- */

/*
 * The factorization the paper plans to move to the GPU with the fixed-point
 * ILU of Chow and Patel.  The entries of L (unit lower) and U on the pattern
 * S of A satisfy, for every (i,j) in S,
 *   u_ij = a_ij - sum_{k<i} l_ik u_kj,   l_ij = (a_ij - sum_{k<j} l_ik u_kj) / u_jj
 * (k over the pairs (i,k), (k,j) in S).  Starting from u_ij = a_ij,
 * l_ij = a_ij / a_jj, each of `sweeps` synchronous sweeps evaluates every
 * equation from the previous sweep's values, subtracting the products from
 * a_ij in ascending k; swept to a standstill the result is the row-wise
 * ILU(0) bit for bit, and a few sweeps give an approximate factorization.
 *
 * silu_split_sizes: entries strictly below the diagonal and on or above it
 * (synchronous).  silu_ilu0_fixed_point writes Ls (strictly lower, unit
 * diagonal implied) and U (upper, diagonal first in every row), in the
 * format ilu_scale_factors takes: caller-allocated row_ptr [n+1], col_idx and
 * val of the two sizes.  *changed (may be NULL): 1 if the last sweep still
 * changed a value.  ws: silu_ilu0_fixed_point_workspace_size bytes (two value
 * arrays and two index arrays), 256-byte aligned.  Synchronous.  Errors: ARG,
 * SHAPE, NOMEM, PATTERN (a row of A without its diagonal), ZERO_PIVOT (a zero
 * or non-finite diagonal of A), HIP.
 */
int silu_split_sizes(silu_ctx *ctx, const silu_csr *A, int64_t *nnz_lower, int64_t *nnz_upper);
int silu_ilu0_fixed_point_workspace_size(silu_ctx *ctx, int64_t n, int64_t nnz, size_t *bytes);
int silu_ilu0_fixed_point(silu_ctx *ctx, const silu_csr *A, int sweeps, silu_csr *Ls, silu_csr *U, int *changed,
                          int flags, void *ws, size_t ws_bytes);

/* ---- Krylov solver around the smoother (Section 6) ---------------------- */

/*
 * FGMRES(restart) with the ILU smoother as right preconditioner: the paper
 * runs flexible GMRES [Saad03] stopped on the relative residual (eq.
 * relres).  Each step applies M^{-1} as one smoother call from z = 0
 * (`outer` steps with m_L, m_U; SILU_MIXED gives the FP32-inner form, whose
 * rounding makes M^{-1} slightly non-linear, which the flexible variant
 * allows), one product with A, modified Gram-Schmidt against the basis and a
 * Givens rotation; it stops when the residual estimate |g_{j+1}| / ||b|| falls
 * below tol (or at max_iters steps, or on breakdown), and restarts from the
 * current x every `restart` steps.  x: initial guess in, solution out.
 * F: row- or row/column-scaled factors.  *iters: steps taken.  hist: NULL or
 * a host array of max_iters + 1 doubles receiving the relative residual
 * estimates (hist[0] for the initial x).  Dot products reduce in a fixed order
 * (reproducible; not the sequential order).  flags: SILU_MIXED, SILU_REORDER
 * (the whole solve runs on the relabeled copies of A and the factors: b and x
 * are permuted in once and x out once, so the products with A gather locally
 * too; the iterates equal those of the given order up to rounding, since the
 * dot products then sum in the relabeled order), the kernel choices,
 * SILU_VALIDATE; SILU_GRAPH is ignored.  ws: at least
 * silu_fgmres_workspace_size(ctx, n, restart, flags) bytes (2 restart + 6
 * n-vectors, 2 more with SILU_REORDER, and a few KB), 256-byte aligned.  Synchronous (the small
 * least-squares problem is solved on the host every step).  Errors: ARG,
 * SHAPE, NOMEM, UNSUPPORTED (factors neither row- nor row/column-scaled),
 * and those of ilu_smooth.
 */
int silu_fgmres_workspace_size(silu_ctx *ctx, int64_t n, int restart, int flags, size_t *bytes);
int silu_fgmres(silu_ctx *ctx, const silu_csr *A, const silu_factors *F, const double *b, double *x, int restart,
                int max_iters, double tol, int outer, int m_L, int m_U, int flags, void *ws, size_t ws_bytes,
                int *iters, double *hist);

/*
 * silu_fgmres stopped on the norm-wise relative backward error instead (eq.
 * nbre, the alternative that the numerical results of Section 6 set beside
 * eq. relres): it stops when |g_{j+1}| / (||b|| + norm_a ||x_j||) falls below
 * tol, x_j being the iterate that the first j steps define, and hist receives
 * these estimates.  norm_a: ||A||_2 or an estimate of it (silu_norm2_estimate),
 * >= 0 and finite; 0 gives exactly silu_fgmres.  ||x_j|| comes from the Gram
 * matrix of the preconditioned directions, kept up to date with j + 2 more dot
 * products per step: ||x_j||^2 = ||x_0||^2 + 2 y.(Z^T x_0) + y^T (Z^T Z) y
 * (taken as 0 should rounding make it negative, which only delays the stop).
 * Same arguments, workspace and errors as silu_fgmres, and ARG for a bad norm_a.
 */
int silu_fgmres_nrbe(silu_ctx *ctx, const silu_csr *A, const silu_factors *F, const double *b, double *x,
                     int restart, int max_iters, double tol, double norm_a, int outer, int m_L, int m_U, int flags,
                     void *ws, size_t ws_bytes, int *iters, double *hist);

/* y = A x (FP64, the sweep kernels' layout and row order).  Asynchronous. */
int silu_spmv(silu_ctx *ctx, const silu_csr *A, const double *x, double *y, int flags);
/* *result = a . b over n entries, reduced in the fixed order of the Krylov
 * solver; ws: device scratch of at least 8200 bytes.  Synchronous. */
int silu_dot(silu_ctx *ctx, int64_t n, const double *a, const double *b, double *result, void *ws, size_t ws_bytes);

/* Device scratch for silu_norm2_estimate and silu_nrbe: two n-vectors (8 n
 * bytes each, rounded up to 256) and 8448 bytes for the dot products. */
int silu_aux_workspace_size(int64_t n, size_t *bytes);
/*
 * Power-iteration estimate of ||A||_2 for the NRBE of eq. nbre: v = v0 /
 * ||v0||, then `iters` times lam = ||A v||, v = A v / lam (stopping early if
 * lam = 0).  *result = the last lam: ||A||_2 for a symmetric A as the iteration
 * converges, a lower bound in general.  v0: device FP64 [n], nonzero (the
 * caller's random start; not modified).  ws: device scratch of at least
 * silu_aux_workspace_size(n) bytes, 256-byte aligned.  Synchronous.  Errors:
 * ARG (null pointer, iters < 1, v0 zero or not finite), SHAPE, NOMEM.
 */
int silu_norm2_estimate(silu_ctx *ctx, const silu_csr *A, const double *v0, int iters, double *result, void *ws,
                        size_t ws_bytes);
/*
 * Norm-wise relative backward error (eq. nbre) of x as a solution of A x = b:
 * *result = ||b - A x|| / (||b|| + norm_a ||x||), the residual formed by the
 * sweep kernel and the norms by the fixed-order dot product.  b, x: device
 * FP64 [n].  norm_a >= 0, finite.  ws: as for silu_norm2_estimate.
 * Synchronous.  Errors: ARG, SHAPE, NOMEM.
 */
int silu_nrbe(silu_ctx *ctx, const silu_csr *A, const double *b, const double *x, double norm_a, double *result,
              void *ws, size_t ws_bytes);

/* ---- triangular solves ------------------------------------------------- */

/*
 * Direct solve T out = rhs by level-set scheduling (Section 4): rows are
 * grouped by the level of the elimination DAG and each level is one kernel
 * launch, rows inside a level in parallel.  The launch sequence is captured
 * once into a hipGraph (cached in the context, keyed by the pointers of T,
 * rhs and out) and replayed; SILU_NO_GRAPH launches the levels one by one.  T: FP64 CSR, lower (uplo =
 * SILU_LOWER) or upper triangular.  diag = SILU_UNIT: the diagonal is taken
 * as 1 and stored diagonal entries are not read; SILU_NONUNIT: every row must
 * store its diagonal, and the row is divided by it.  rhs, out: FP64 [n],
 * distinct.  The level analysis of T is made on first use (synchronous: the
 * pattern is copied to the host) and cached in the context, keyed by T's
 * pointers and sizes; the solve itself is asynchronous.
 * Errors: ARG, SHAPE, PATTERN (an entry on the wrong side), HIP.
 */
int trisolve_direct(silu_ctx *ctx, const silu_csr *T, int uplo, int diag, const double *rhs, double *out,
                    int flags);

/*
 * Iterative counterpart (Section 4; eq. richard): m Richardson steps
 * out_k = s - T out_{k-1} from out_0 = 0 for the unit triangular system
 * (I + T) out = s, where T is STRICTLY triangular (no stored diagonal; lower
 * or upper) and s = rhs, or s = dinv * rhs when dinv is non-NULL.  m >= the
 * number of levels of T gives the exact solution (T is nilpotent).  FP64;
 * rhs and out distinct.  ws: silu_workspace_size(ctx, n, 0) bytes.
 * Asynchronous.  Errors: ARG (m < 1), SHAPE, NOMEM, PATTERN (with
 * SILU_VALIDATE), HIP.
 */
int trisolve_iter(silu_ctx *ctx, const silu_csr *T, const double *dinv, const double *rhs, double *out, int m,
                  int flags, void *ws, size_t ws_bytes);

/* Level analysis of T (made now if not cached): number of levels in
 * *depth and, if rows_per_level is non-NULL, the row count of every level
 * (host array of at least *depth entries; call once with NULL to size it).
 * Synchronous. */
int silu_analyze(silu_ctx *ctx, const silu_csr *T, int uplo, int32_t *depth, int32_t *rows_per_level);

/* Drop everything the context cached for the matrix whose row_ptr or
 * col_idx is given (level sets and their graphs, row-block partitions,
 * 16-bit codes, sliced copies).  The caches are keyed by pointers and sizes,
 * so call this before freeing a matrix, or changing its pattern or (for the
 * sliced copies) its values in place.  Synchronizes the context stream. */
int silu_release(silu_ctx *ctx, const void *row_ptr, const void *col_idx);

/* ---- measurement ------------------------------------------------------- */

/*
 * Per-kernel timing.  With timing on, every kernel launch the context makes
 * is bracketed by a pair of HIP events recorded on the context stream, and the
 * launch is credited with two byte counts.  Algorithmic bytes: the CSR form of
 * the step -- every entry of the matrix read once as its value plus a 4-byte
 * column index, 4 bytes of row pointer per row, every dense vector read or
 * written once.  Layout bytes: what the layout the kernel actually streams
 * occupies (a sliced copy's padded slots, 1- or 2-byte column codes and slice
 * tables; 16-bit offsets), never more than the algorithmic bytes by more than
 * the padding.  silu_stats_collect synchronizes the stream and folds the
 * recorded events into per-kernel totals; it returns the number of kernel
 * kinds seen.  silu_stats_get reads entry idx: kernel name (NUL-terminated,
 * truncated to name_len), launch count, summed duration in milliseconds,
 * summed algorithmic bytes and summed layout bytes (either pointer may be
 * NULL).  silu_stats_reset clears them.
 */
int silu_set_timing(silu_ctx *ctx, int enable);
int silu_stats_collect(silu_ctx *ctx);
int silu_stats_get(silu_ctx *ctx, int idx, char *name, int name_len, int64_t *launches, double *ms,
                   double *bytes, double *layout_bytes);
int silu_stats_reset(silu_ctx *ctx);

/* Plain device copy dst[0..bytes) = src[0..bytes) with a streaming kernel
 * (16-byte vector loads and stores), used to measure achievable HBM
 * bandwidth and to calibrate traffic counters.  bytes must be a multiple of
 * 16 and both pointers 16-byte aligned.  Asynchronous. */
int silu_stream_copy(silu_ctx *ctx, const void *src, void *dst, size_t bytes);

/* Read-dominant calibration stream shaped like a sweep's traffic (8 bytes
 * written per 192 read, about 96 % reads): reads src[0..bytes) with 16-byte
 * non-temporal loads and writes bytes / 24 bytes of check words to out.  The
 * achievable bandwidth for the sweeps' mix of traffic.  bytes a positive
 * multiple of 49,152; src 16-byte and out 8-byte aligned.  Asynchronous.
 * Errors: ARG. */
int silu_stream_read(silu_ctx *ctx, const void *src, size_t bytes, void *out);

/* ---- serving: continuous batching on resident matrices ---------------- */

/*
 * A server keeps registered matrices (A and their factors) resident and runs
 * smoother requests on them (each request: `outer` steps of ilu_smooth's
 * iteration, FP64).  silu_server_step() first admits queued requests in
 * arrival order while their workspace (silu_server_request_bytes: four
 * n-vectors and 16 bytes per 256 rows) fits in the caller's arena and fewer than max_active are
 * running, then enqueues ONE batched launch that advances every active
 * request by one sweep (residual, an L sweep or a U sweep), whatever sweep
 * each is at; requests that arrive later join at the next step.  A request's
 * workspace returns to the arena once the GPU has passed its last launch.
 * Each row is summed in a fixed order by one lane, so a request's result is
 * bit-identical to ilu_smooth on its own.  silu_server_register copies A, Ls
 * and Us into the sliced layout the sweeps read (synchronous; device memory
 * about that of the CSR arrays, held until silu_server_destroy): values
 * changed afterwards take effect only for a matrix registered again.  A
 * matrix without diagonal or offset structure is streamed from its CSR
 * arrays instead.  The host keeps at most 8 steps enqueued beyond the last
 * one known to be complete.
 *
 * arena: device memory owned by the caller, 256-byte aligned, alive until
 * silu_server_destroy.  b and x of a request: device FP64 [n], alive until
 * poll reports it done; x is the initial guess and receives the result.
 * m_L, m_U >= 1 but not both 1.  Row-scaled and row/column-scaled factors
 * are both served.  Errors: ARG, SHAPE, UNSUPPORTED (unscaled or non-FP64
 * factors), NOMEM (one request alone exceeds the arena), HIP
 * (silu_server_last_hip_error).  A server is used by one host thread.
 * Per-ticket state is bounded: a ticket's record (its times, and a solve
 * request's result) is kept until 65,536 later tickets have finished; after
 * that poll and wait report it done and times / solve_result return ARG.
 */
typedef struct silu_server silu_server;
int silu_server_create(silu_ctx *ctx, void *hip_stream, void *arena, size_t arena_bytes, int max_active,
                       silu_server **server);
int silu_server_destroy(silu_server *server);
int silu_server_register(silu_server *server, const silu_csr *A, const silu_factors *F, int *matrix_id);
int64_t silu_server_request_bytes(const silu_server *server, int matrix_id);
int silu_server_submit(silu_server *server, int matrix_id, const double *b, double *x, int outer, int m_L, int m_U,
                       int64_t *ticket);
/* The same with flags: 0, or SILU_MIXED for the FP32-inner form of
 * ilu_smooth (the L and U~ sweeps on FP32 copies of the factor values, the
 * residual and the update of x in FP64), bit-identical to that call.  The
 * matrix must have been registered with factors that carry FP32 values
 * (register then also builds their sliced copies); UNSUPPORTED otherwise, or
 * outside the stepwise mode.  Each step launches one batch per precision
 * present. */
int silu_server_submit_flags(silu_server *server, int matrix_id, const double *b, double *x, int outer, int m_L,
                             int m_U, int flags, int64_t *ticket);
/*
 * A solve request: the smoother iterated until the relative residual of eq.
 * relres, ||b - A x|| / ||b||, falls below tol, checked for the initial x and
 * after each outer step, at most max_outer steps.  It is scheduled like a
 * smoother request of max_outer steps plus one final residual; the residual
 * at the start of each outer step is the check: its tile sums of r_i^2 are
 * closed by one small launch per step, which sets the request's stop flag on
 * the device, and every later sweep of a stopped request does nothing, so x
 * keeps the first iterate that passed.  The same launch sets a pinned host
 * word, which the next steps read: a stopped request gets no more sweeps and
 * is reported done with the step after that (otherwise after its scheduled
 * sweeps).  Each sweep is the one ilu_smooth makes, so
 * x equals that many ilu_smooth outer steps bit for bit; the norms are summed
 * in a fixed order (not the sequential one).  tol > 0, 0 <= max_outer <=
 * 2^20; stepwise mode only (UNSUPPORTED otherwise).
 * silu_server_solve_result, once the request is done: *outer_steps = the
 * number of outer steps after which the test first passed (0: x0 already
 * did), or max_outer + 1 if it never did; *relres = the relative residual of
 * the last check made.  ARG for an unknown ticket, one that is not a solve
 * request, or one not yet done.
 */
int silu_server_submit_solve(silu_server *server, int matrix_id, const double *b, double *x, double tol,
                             int max_outer, int m_L, int m_U, int64_t *ticket);
int silu_server_solve_result(silu_server *server, int64_t ticket, int *outer_steps, double *relres);
/* One scheduling step (asynchronous; blocks only when 8 steps are in flight). */
int silu_server_step(silu_server *server, int *n_active, int *n_queued);
/* Up to max_steps steps in one call (each one admits and launches as above),
 * stopping early when no request is active: a host loop that calls this
 * keeps the GPU fed with fewer round trips.  While no request waits for
 * admission, no stop flag is pending and every active request has k or more
 * ops left, up to 8 steps are enqueued together (their op tables copied to
 * the device at once): the same launches, so the same results, with less host
 * work per step; a solve request the device stops meanwhile skips its sweeps
 * and is retired by the next single step. */
int silu_server_run(silu_server *server, int max_steps, int *n_active, int *n_queued);
/* state: 0 queued, 1 running, 2 last sweep enqueued, 3 done (result in x).
 * Returns SILU_ERR_TIMEOUT (state 3) for a request whose persistent launch
 * gave up a wait: its x is not a valid result. */
int silu_server_poll(silu_server *server, int64_t ticket, int *state);
/* The tickets of requests found done (state 3) since the last call, each
 * returned once, oldest first, at most `capacity` of them in tickets[] (host
 * array); *count receives how many.  One call replaces a poll per pending
 * request.  Done tickets are kept until returned here (8 bytes each), at
 * most the 65,536 most recent: older ones are dropped unreported. */
int silu_server_completed(silu_server *server, int64_t *tickets, int capacity, int *count);
/* Block until the ticket's request is done (state 3), stepping the server
 * while it is queued or running, then waiting for its last launch.  The
 * server's other requests advance with it. */
int silu_server_wait(silu_server *server, int64_t ticket);
/* Host steady-clock times in ns: when the ticket was submitted and when the
 * server first found it done (-1 while it is not).  ARG for unknown tickets
 * and for those whose record has been dropped (see above). */
int silu_server_times(silu_server *server, int64_t ticket, int64_t *submitted_ns, int64_t *done_ns);
/* What the server holds per ticket now: ticket records, pinned result slots
 * for solve requests (allocated 1,024 at a time, reused once read), and done
 * tickets not yet returned by silu_server_completed. */
int silu_server_footprint(const silu_server *server, int64_t *records, int64_t *result_slots, int64_t *unreported);
int silu_server_last_hip_error(const silu_server *server);

/*
 * Scheduling mode of a server (the serving form; Algorithm 2 per request).
 *   SILU_SERVE_STEPWISE (default): as above, one batched launch per step, one
 *     sweep per active request.
 *   SILU_SERVE_PERSISTENT: NOT AVAILABLE in this version -- set_mode returns
 *     SILU_ERR_UNSUPPORTED (its launches did not finish on MI355X, for a
 *     cause not yet found).  As designed: a step hands the requests it admits, with all of
 *     their sweeps, to ONE persistent launch on the next of three streams the
 *     server creates (default priority) after the caller's stream has passed
 *     the point of the step.  Inside the launch each request's sweeps follow
 *     one another through device-side counters, with no kernel boundary; the
 *     launches of different steps run concurrently, so a request that arrives
 *     while others run starts at once.  Results are bit-identical to the
 *     stepwise mode and to ilu_smooth.  max_workgroups caps the workgroups of
 *     one launch (0: 1024; at most 65535); a launch needs no more than twice
 *     the row tiles (256 rows) of its requests' matrices.  max_active counts
 *     requests whose launch the GPU has not passed.  A wait inside the launch
 *     is bounded; one that expires makes poll return SILU_ERR_TIMEOUT for the
 *     requests of that launch.  x is written on the server's streams: use it
 *     after poll reports state 3.
 * The mode may change only while no request is queued, active or in flight
 * (else SILU_ERR_ARG).  Synchronous.
 */
#define SILU_SERVE_STEPWISE 0
#define SILU_SERVE_PERSISTENT 1
int silu_server_set_mode(silu_server *server, int mode, int max_workgroups);
/* Wall-clock time in microseconds a persistent launch's bounded wait may
 * take before it gives up (measured on the device's constant-rate clock, so
 * the bound holds however long each poll takes; 0 restores the default
 * 200,000).  For tests of the failure path: a limit of 1 makes most waits
 * expire, and the launch still drains and reports SILU_ERR_TIMEOUT through
 * poll. */
int silu_server_set_wait_limit(silu_server *server, int microseconds);

#ifdef __cplusplus
}
#endif

#endif /* SCALED_ILU_H */
