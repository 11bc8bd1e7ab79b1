// Fused Richardson-sweep kernels for gfx950 (CDNA4, wave64).
//
// One launch computes, for every row i of a CSR matrix N,
//     t_i = rhs_i - sum_j N_ij xin_j
// and applies an epilogue (store t, store D^{-1} t, x += t, x += D^{-1} t;
// the updates optionally scaled by the column factors of a row/column scaling).
// With N = A and rhs = b this is the residual r = b - A x (eq. ILUsplit);
// with N = the strictly triangular part of a unit factor it is one Richardson
// step y_k = rhs - N y_{k-1} (eq. richard; Algorithm 2).  The diagonal scaling
// and the update of x are fused into the last sweep, so each step reads its
// matrix exactly once.  The work is bandwidth-bound (about 0.1 flop per byte),
// so there is no MFMA: the kernels are shaped for coalesced HBM streaming.
//
// Shapes:
//  * CSR-stream (default): a workgroup owns RPB consecutive rows, streams
//    their contiguous val/col range with unit-stride, non-temporal loads
//    (the factor is read once per sweep and must not evict the gathered
//    iterate from L2), writes the products val*xin[col] to LDS, then one lane
//    per row adds its products in ascending column order -- the oracle's
//    order, so FP64 results are bit-identical to it.
//  * CSR-stream over a row-block partition (entries per workgroup capped,
//    computed once per matrix on the host).
//  * vector-CSR: K lanes per row, partial sums combined with cross-lane
//    shuffles (different summation order; within rounding of the oracle).
// Workgroups are remapped so that each XCD (the hardware deals workgroups
// round-robin over the 8 XCDs) walks one contiguous slab of rows, keeping the
// gathered iterate window resident in that XCD's L2.
#include <cstdio>
#include <cstdlib>

#include "internal.h"

#pragma clang fp contract(off)

namespace silu {
namespace {

// precision bundles: value, gathered-iterate, rhs, accumulate, iterate-rounding, output types
struct TF64 {
    using VT = double;
    using XT = double;
    using RT = double;
    using AT = double;
    using IT = double;
    using OT = double;
};
struct TMixRes {
    using VT = double;
    using XT = double;
    using RT = double;
    using AT = double;
    using IT = float;
    using OT = float;
};
struct TMixL {
    using VT = float;
    using XT = float;
    using RT = double;
    using AT = float;
    using IT = float;
    using OT = float;
};
struct TMixL1 {
    using VT = float;
    using XT = double;
    using RT = double;
    using AT = float;
    using IT = float;
    using OT = float;
};
struct TMixU {
    using VT = float;
    using XT = float;
    using RT = float;
    using AT = float;
    using IT = float;
    using OT = float;
};

// Workgroups are dealt round-robin over the 8 XCDs; this remap gives each XCD
// one contiguous slab of the grid's blocks, so neighbouring blocks share an
// L2.  Kept where it measured faster (the row-block kernel on the relabeled
// random operator: 1.54 against 1.63 ms per application, and the coded sliced
// and vector kernels, not re-measured); the row-pattern, diagonal-slice,
// CSR-stream and batched kernels take blocks in launch order, which measured
// 2-10 % faster for them.
__device__ __forceinline__ int xcd_slab_block(int b, int G)
{
    const int q = G >> 3, r = G & 7, xcd = b & 7, k = b >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

template <class T>
__device__ __forceinline__ void epilogue(const SweepArgs &a, int row, typename T::AT t)
{
    using IT = typename T::IT;
    using OT = typename T::OT;
    const IT v = (IT)t;
    const double c = a.dcol ? a.dcol[row] : 1.0; // column factor; 1.0 * v is exact
    switch (a.epi) {
    case EPI_STORE:
    case EPI_SPMV:
        ((OT *)a.out)[row] = (OT)v;
        break;
    case EPI_STORE_SPLIT:
        ((OT *)a.out)[row] = (OT)v;
        a.out32[row] = (float)v;
        break;
    case EPI_SCALE:
        ((OT *)a.out)[row] = (OT)(a.dinv[row] * (double)v);
        break;
    case EPI_UPDATE:
        a.x[row] = a.x[row] + c * (double)v;
        break;
    default: // EPI_SCALE_UPDATE
        a.x[row] = a.x[row] + c * (double)(OT)(a.dinv[row] * (double)v);
        break;
    }
}

// Epilogue with its operands loaded up front: aux = x_i (UPDATE) or dinv_i
// (SCALE, SCALE_UPDATE); aux2 = x_i (SCALE_UPDATE); c = the column factor
// (UPDATE, SCALE_UPDATE; 1.0 without one).
template <class T>
__device__ __forceinline__ void epilogue_pre(const SweepArgs &a, int row, typename T::AT t, double aux, double aux2,
                                             double c)
{
    using IT = typename T::IT;
    using OT = typename T::OT;
    const IT v = (IT)t;
    switch (a.epi) {
    case EPI_STORE:
    case EPI_SPMV:
        ((OT *)a.out)[row] = (OT)v;
        break;
    case EPI_STORE_SPLIT:
        ((OT *)a.out)[row] = (OT)v;
        a.out32[row] = (float)v;
        break;
    case EPI_SCALE:
        ((OT *)a.out)[row] = (OT)(aux * (double)v);
        break;
    case EPI_UPDATE:
        a.x[row] = aux + c * (double)v;
        break;
    default: // EPI_SCALE_UPDATE
        a.x[row] = aux2 + c * (double)(OT)(aux * (double)v);
        break;
    }
}

// ---------------------------------------------------------------------------
// CSR-stream: RPB rows per workgroup of BLOCK lanes (RPB <= BLOCK); products
// staged in LDS in chunks of CAP entries.  The lane of each row loads the
// row's rhs and epilogue operands together with the row pointers, so those
// loads overlap the block's stream instead of following it.
// ---------------------------------------------------------------------------
// Index modes of an entry's iterate value:
//   IDX32:  xin[col[e]]                                   (4 bytes of index)
//   OFF16:  xin[r0 + shift + off16[e]], block-relative 16-bit offsets (2 bytes)
//   WIN:    xs[code[e]], the block's iterate window staged in LDS (2 bytes)
// WIN: the block-relative offsets o = col - r0 that occur anywhere in the
// matrix are numbered 0..lw-1 (wo[t] = the offset of slot t); every workgroup
// first copies xin[r0 + wo[t]] into LDS slot t with unit-stride loads, so the
// entry stream's gathers hit LDS instead of going through the vector memory
// pipeline one 8-byte word at a time.  Banded factors use a few hundred slots.
enum IdxMode : int { IDX32 = 0, OFF16 = 1, WIN = 2 };

// Returns the lane's row value t (0 for a lane without a row).
template <class T, int BLOCK, int RPB, int CAP, int MODE>
__device__ __forceinline__ double stream_rows(const SweepArgs &a, int blk, const uint16_t *__restrict__ code,
                                              int shift, const int32_t *__restrict__ wo, int lw)
{
    using VT = typename T::VT;
    using XT = typename T::XT;
    using RT = typename T::RT;
    using AT = typename T::AT;
    static_assert(RPB <= BLOCK && CAP % BLOCK == 0, "geometry");
    __shared__ AT prod[CAP];
    __shared__ int32_t srp[RPB + 1];
    extern __shared__ double lds_window[]; // WIN: XT xs[lw] (dynamic size)

    const int r0 = blk * RPB;
    const int nr = min(RPB, a.n - r0);
    const int tid = (int)threadIdx.x;
    const XT *__restrict__ xin = (const XT *)a.xin;
    XT *xs = (XT *)lds_window;
    RT rhs_v = (RT)0;
    double aux = 0.0, aux2 = 0.0, dsh = 1.0, cf = 1.0;
    if (tid < nr) {
        const int row = r0 + tid;
        if (a.epi != EPI_SPMV) rhs_v = ((const RT *)a.rhs)[row];
        if (a.epi == EPI_UPDATE) aux = a.x[row];
        if (a.epi == EPI_SCALE || a.epi == EPI_SCALE_UPDATE) aux = a.dinv[row];
        if (a.epi == EPI_SCALE_UPDATE) aux2 = a.x[row];
        if (a.dcol && (a.epi == EPI_UPDATE || a.epi == EPI_SCALE_UPDATE)) cf = a.dcol[row];
        if (a.dshift) dsh = a.dshift[row];
    }
    for (int t = tid; t <= nr; t += BLOCK) srp[t] = a.rp[r0 + t];
    if (MODE == WIN) {
        for (int t = tid; t < lw; t += BLOCK) {
            const int j = r0 + wo[t];
            xs[t] = (unsigned)j < (unsigned)a.n ? xin[j] : (XT)0;
        }
    }
    __syncthreads();

    const VT *__restrict__ val = (const VT *)a.val;
    const int32_t *__restrict__ col = a.col;
    const int e0 = srp[0], e1 = srp[nr];

    AT sum = (AT)0;
    int mylo = 0, myhi = 0;
    if (tid < nr) {
        mylo = srp[tid];
        myhi = srp[tid + 1];
        if (a.dshift) sum = (AT)((dsh - 1.0) * (double)xin[r0 + tid]);
    }
    for (int c0 = e0; c0 < e1; c0 += CAP) {
        const int c1 = min(c0 + CAP, e1);
#pragma unroll 4
        for (int e = c0 + tid; e < c1; e += BLOCK) {
            XT xv;
            if (MODE == WIN)
                xv = xs[__builtin_nontemporal_load(&code[e])];
            else if (MODE == OFF16)
                xv = xin[r0 + shift + (int)__builtin_nontemporal_load(&code[e])];
            else
                xv = xin[__builtin_nontemporal_load(&col[e])];
            prod[e - c0] = (AT)__builtin_nontemporal_load(&val[e]) * (AT)xv;
        }
        __syncthreads();
        const int lo = max(mylo, c0), hi = min(myhi, c1);
        for (int k = lo; k < hi; ++k) sum = sum + prod[k - c0];
        __syncthreads();
    }
    const AT t = a.epi == EPI_SPMV ? sum : (AT)rhs_v - sum;
    if (tid < nr) epilogue_pre<T>(a, r0 + tid, t, aux, aux2, cf);
    return tid < nr ? (double)t : 0.0;
}

template <class T, int BLOCK, int RPB, int CAP>
__global__ void __launch_bounds__(BLOCK) k_sweep_stream(SweepArgs a)
{
    stream_rows<T, BLOCK, RPB, CAP, IDX32>(a, (int)blockIdx.x, nullptr, 0, nullptr, 0);
}

template <class T, int BLOCK, int RPB, int CAP>
__global__ void __launch_bounds__(BLOCK) k_sweep_stream16(SweepArgs a, const uint16_t *__restrict__ off16, int shift)
{
    stream_rows<T, BLOCK, RPB, CAP, OFF16>(a, (int)blockIdx.x, off16, shift, nullptr, 0);
}

template <class T, int BLOCK, int RPB, int CAP>
__global__ void __launch_bounds__(BLOCK) k_sweep_win(SweepArgs a, const uint16_t *__restrict__ code,
                                                     const int32_t *__restrict__ wo, int lw)
{
    stream_rows<T, BLOCK, RPB, CAP, WIN>(a, (int)blockIdx.x, code, 0, wo, lw);
}

// ---------------------------------------------------------------------------
// Sliced-ELL: one wavefront per 64-row slice, lane = row.  The slots of a
// slice come in groups of four entries per row (see the set-up kernels), so a
// lane fetches a group with one 16-byte (FP64: two) value load and one code
// load of 4, 8 or 16 bytes, all unit-stride across the wave; neighbouring
// rows gather neighbouring iterate values.  Each lane adds its row's products
// in ascending column order (the oracle's order) in registers: no LDS staging
// of products and no barrier.  Slices whose rows all have entries run without
// per-row lengths: a padded slot holds value 0 at the row's last column, which
// adds +0.0 to the sum (a sum started at +0.0 is never -0.0), so finite
// results are unchanged and a non-finite value there already makes the row's
// sum non-finite.  Slices with an empty row, or rows past the end, mask by
// the row lengths.
// ---------------------------------------------------------------------------
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// One wavefront's slice (wave = slice index); dtab: the diagonal table in LDS
// (code 1).  Returns the lane's row value t (0 for a lane without a row).
template <class T, int CODE, int UNR>
__device__ __forceinline__ double sliced_wave(const SweepArgs &a, const SlicedView &s, int wave,
                                              const int32_t *dtab)
{
    using VT = typename T::VT;
    using XT = typename T::XT;
    using RT = typename T::RT;
    using AT = typename T::AT;
    if (wave >= s.nslice) return 0.0;
    const int lane = (int)threadIdx.x & 63;
    const int row = wave * 64 + lane;
    const bool live = row < a.n;
    const XT *__restrict__ xin = (const XT *)a.xin;

    RT rhs_v = (RT)0;
    double aux = 0.0, aux2 = 0.0, dsh = 1.0, cf = 1.0;
    if (live) {
        if (a.epi != EPI_SPMV) rhs_v = ((const RT *)a.rhs)[row];
        if (a.epi == EPI_UPDATE) aux = a.x[row];
        if (a.epi == EPI_SCALE || a.epi == EPI_SCALE_UPDATE) aux = a.dinv[row];
        if (a.epi == EPI_SCALE_UPDATE) aux2 = a.x[row];
        if (a.dcol && (a.epi == EPI_UPDATE || a.epi == EPI_SCALE_UPDATE)) cf = a.dcol[row];
        if (a.dshift) dsh = a.dshift[row];
    }
    const int kf = s.sk[wave];
    const int G = (kf & 0x7fffffff) >> 2; // groups of four entries
    const int p0 = s.sptr[wave];          // a multiple of 256
    const int base = wave * 64 + s.shift;
    AT sum = (AT)0;
    if (live && a.dshift) sum = (AT)((dsh - 1.0) * (double)xin[row]);
    const int len = kf >= 0 ? 4 * G : (live ? a.rp[row + 1] - a.rp[row] : 0);
    const int safe = min(row, a.n - 1);

    // the four entries of group q: values v[0..3], columns j[0..3]
    auto group = [&](int q, VT *v, int *j) {
        if (sizeof(VT) == 8) {
            const f64x2 *pv = (const f64x2 *)s.val + (p0 >> 1) + 128 * q + lane;
            const f64x2 lo2 = __builtin_nontemporal_load(pv), hi2 = __builtin_nontemporal_load(pv + 64);
            v[0] = (VT)lo2.x;
            v[1] = (VT)lo2.y;
            v[2] = (VT)hi2.x;
            v[3] = (VT)hi2.y;
        } else {
            const f32x4 v4 = __builtin_nontemporal_load((const f32x4 *)s.val + (p0 >> 2) + 64 * q + lane);
            v[0] = (VT)v4.x;
            v[1] = (VT)v4.y;
            v[2] = (VT)v4.z;
            v[3] = (VT)v4.w;
        }
        const int pc = (p0 >> 2) + 64 * q + lane;
        if (CODE == 1) {
            const unsigned c = __builtin_nontemporal_load((const unsigned *)s.codes + pc);
            j[0] = row + dtab[c & 0xffu];
            j[1] = row + dtab[(c >> 8) & 0xffu];
            j[2] = row + dtab[(c >> 16) & 0xffu];
            j[3] = row + dtab[c >> 24];
        } else if (CODE == 2) {
            const u32x2 c = __builtin_nontemporal_load((const u32x2 *)s.codes + pc);
            j[0] = base + (int)(c.x & 0xffffu);
            j[1] = base + (int)(c.x >> 16);
            j[2] = base + (int)(c.y & 0xffffu);
            j[3] = base + (int)(c.y >> 16);
        } else {
            const i32x4 c = __builtin_nontemporal_load((const i32x4 *)s.codes + pc);
            j[0] = c.x;
            j[1] = c.y;
            j[2] = c.z;
            j[3] = c.w;
        }
    };
    if (kf >= 0) {
#pragma unroll UNR
        for (int q = 0; q < G; ++q) {
            VT v[4];
            int j[4];
            group(q, v, j);
#pragma unroll
            for (int r = 0; r < 4; ++r) sum = sum + (AT)v[r] * (AT)xin[j[r]];
        }
    } else {
#pragma unroll UNR
        for (int q = 0; q < G; ++q) {
            VT v[4];
            int j[4];
            group(q, v, j);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool on = 4 * q + r < len;
                const AT t = sum + (AT)v[r] * (AT)xin[on ? j[r] : safe];
                sum = on ? t : sum;
            }
        }
    }
    const AT t = a.epi == EPI_SPMV ? sum : (AT)rhs_v - sum;
    if (live) epilogue_pre<T>(a, row, t, aux, aux2, cf);
    return live ? (double)t : 0.0;
}

// The same slice with every load of the slice in flight at once (diagonal-
// table codes, slices of at most GM groups without masked rows): the values
// and codes of all groups, then all gathers, then the row sum in ascending
// column order as above.  The loop form above keeps two groups in flight and
// waits for a group's codes before its gathers, so each wave makes several
// dependent round trips to memory per slice; here it makes two.  The body is
// specialised on the slice's exact group count so that it has no branches
// between the loads (the waits for each group's codes and gathers are then
// counted exactly instead of draining every load in flight).  The slice
// header (a wave-uniform index) is read through the scalar cache.
template <class T, int GG>
__device__ __forceinline__ typename T::AT slice_sum_pf(const SlicedView &s, int p0, int lane, int row,
                                                       const typename T::XT *__restrict__ xin, const int32_t *dtab,
                                                       typename T::AT sum)
{
    using VT = typename T::VT;
    using XT = typename T::XT;
    using AT = typename T::AT;
    VT v[GG][4];
    unsigned c[GG];
#pragma unroll
    for (int q = 0; q < GG; ++q) {
        if (sizeof(VT) == 8) {
            const f64x2 *pv = (const f64x2 *)s.val + (p0 >> 1) + 128 * q + lane;
            const f64x2 lo2 = __builtin_nontemporal_load(pv), hi2 = __builtin_nontemporal_load(pv + 64);
            v[q][0] = (VT)lo2.x;
            v[q][1] = (VT)lo2.y;
            v[q][2] = (VT)hi2.x;
            v[q][3] = (VT)hi2.y;
        } else {
            const f32x4 v4 = __builtin_nontemporal_load((const f32x4 *)s.val + (p0 >> 2) + 64 * q + lane);
            v[q][0] = (VT)v4.x;
            v[q][1] = (VT)v4.y;
            v[q][2] = (VT)v4.z;
            v[q][3] = (VT)v4.w;
        }
        c[q] = __builtin_nontemporal_load((const unsigned *)s.codes + (p0 >> 2) + 64 * q + lane);
    }
    XT xv[GG][4];
#pragma unroll
    for (int q = 0; q < GG; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) xv[q][r] = xin[row + dtab[(c[q] >> (8 * r)) & 0xffu]];
    }
#pragma unroll
    for (int q = 0; q < GG; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) sum = sum + (AT)v[q][r] * (AT)xv[q][r];
    }
    return sum;
}

template <class T, int GG>
__device__ __forceinline__ typename T::AT slice_sum_pf_g(int G, const SlicedView &s, int p0, int lane, int row,
                                                         const typename T::XT *__restrict__ xin, const int32_t *dtab,
                                                         typename T::AT sum)
{
    if (G == GG) return slice_sum_pf<T, GG>(s, p0, lane, row, xin, dtab, sum);
    if constexpr (GG > 1) return slice_sum_pf_g<T, GG - 1>(G, s, p0, lane, row, xin, dtab, sum);
    return sum;
}

template <class T, int GM>
__device__ __forceinline__ double sliced_wave_pf(const SweepArgs &a, const SlicedView &s, int wave,
                                                 const int32_t *dtab)
{
    using XT = typename T::XT;
    using RT = typename T::RT;
    using AT = typename T::AT;
    wave = __builtin_amdgcn_readfirstlane(wave);
    if (wave >= s.nslice) return 0.0;
    const int kf = s.sk[wave];
    const int G = kf >> 2;
    if (kf < 0 || G > GM || G < 1) return sliced_wave<T, 1, 2>(a, s, wave, dtab);
    // an unmasked slice: all 64 rows exist and hold entries
    const int lane = (int)threadIdx.x & 63;
    const int row = wave * 64 + lane;
    const int p0 = s.sptr[wave];
    const XT *__restrict__ xin = (const XT *)a.xin;
    RT rhs_v = (RT)0;
    double aux = 0.0, aux2 = 0.0, dsh = 1.0, cf = 1.0;
    if (a.epi != EPI_SPMV) rhs_v = ((const RT *)a.rhs)[row];
    if (a.epi == EPI_UPDATE) aux = a.x[row];
    if (a.epi == EPI_SCALE || a.epi == EPI_SCALE_UPDATE) aux = a.dinv[row];
    if (a.epi == EPI_SCALE_UPDATE) aux2 = a.x[row];
    if (a.dcol && (a.epi == EPI_UPDATE || a.epi == EPI_SCALE_UPDATE)) cf = a.dcol[row];
    if (a.dshift) dsh = a.dshift[row];
    AT sum = (AT)0;
    if (a.dshift) sum = (AT)((dsh - 1.0) * (double)xin[row]);
    sum = slice_sum_pf_g<T, GM>(G, s, p0, lane, row, xin, dtab, sum);
    const AT t = a.epi == EPI_SPMV ? sum : (AT)rhs_v - sum;
    epilogue_pre<T>(a, row, t, aux, aux2, cf);
    return (double)t;
}

template <class T, int WPB, int GM>
__global__ void __launch_bounds__(64 * WPB) k_sweep_sliced_pf(SweepArgs a, SlicedView s)
{
    __shared__ int32_t dtab[256];
    for (int t = (int)threadIdx.x; t < s.ndiag; t += 64 * WPB) dtab[t] = s.dtab[t];
    __syncthreads();
    const int wave = xcd_slab_block((int)blockIdx.x, (int)gridDim.x) * WPB + ((int)threadIdx.x >> 6);
    sliced_wave_pf<T, GM>(a, s, wave, dtab);
}

// Row-pattern slices (code 8): no per-slot code at all.  Row r's slot k gathers
// at r + pt[k], pt being the row's pattern in the matrix's pattern table (the
// row's offsets col - r in ascending order, its last offset repeated into the
// padded slots), found through one byte per row.  A group's four offsets are
// one 16-byte read of the table.  Unmasked slices of at most GM groups
// take the prefetched body (every value load in flight, then every gather);
// masked slices (an empty row, rows past the end) the loop below with per-row
// lengths.  The sums and padding are those of the coded layouts, so results
// are the same bit for bit.
template <class T, int GG>
__device__ __forceinline__ typename T::AT slice_sum_pat(const SlicedView &s, int p0, int lane, int row,
                                                        const typename T::XT *__restrict__ xin, const int32_t *pt,
                                                        typename T::AT sum)
{
    using VT = typename T::VT;
    using XT = typename T::XT;
    using AT = typename T::AT;
    VT v[GG][4];
#pragma unroll
    for (int q = 0; q < GG; ++q) {
        if (sizeof(VT) == 8) {
            const f64x2 *pv = (const f64x2 *)s.val + (p0 >> 1) + 128 * q + lane;
            const f64x2 lo2 = __builtin_nontemporal_load(pv), hi2 = __builtin_nontemporal_load(pv + 64);
            v[q][0] = (VT)lo2.x;
            v[q][1] = (VT)lo2.y;
            v[q][2] = (VT)hi2.x;
            v[q][3] = (VT)hi2.y;
        } else {
            const f32x4 v4 = __builtin_nontemporal_load((const f32x4 *)s.val + (p0 >> 2) + 64 * q + lane);
            v[q][0] = (VT)v4.x;
            v[q][1] = (VT)v4.y;
            v[q][2] = (VT)v4.z;
            v[q][3] = (VT)v4.w;
        }
    }
    XT xv[GG][4];
#pragma unroll
    for (int q = 0; q < GG; ++q) {
        const i32x4 o = *(const i32x4 *)(pt + 4 * q);
        xv[q][0] = xin[row + o.x];
        xv[q][1] = xin[row + o.y];
        xv[q][2] = xin[row + o.z];
        xv[q][3] = xin[row + o.w];
    }
#pragma unroll
    for (int q = 0; q < GG; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) sum = sum + (AT)v[q][r] * (AT)xv[q][r];
    }
    return sum;
}

template <class T, int GG>
__device__ __forceinline__ typename T::AT slice_sum_pat_g(int G, const SlicedView &s, int p0, int lane, int row,
                                                          const typename T::XT *__restrict__ xin, const int32_t *pt,
                                                          typename T::AT sum)
{
    if (G == GG) return slice_sum_pat<T, GG>(s, p0, lane, row, xin, pt, sum);
    if constexpr (GG > 1) return slice_sum_pat_g<T, GG - 1>(G, s, p0, lane, row, xin, pt, sum);
    return sum;
}

template <class T, int GM>
__device__ __forceinline__ double sliced_wave_pat(const SweepArgs &a, const SlicedView &s, int wave, int kf,
                                                  int p0, const int32_t *pt)
{
    using VT = typename T::VT;
    using XT = typename T::XT;
    using RT = typename T::RT;
    using AT = typename T::AT;
    const int G = (kf & 0x7fffffff) >> 2;
    const int lane = (int)threadIdx.x & 63;
    const int row = wave * 64 + lane;
    const bool live = row < a.n;
    const XT *__restrict__ xin = (const XT *)a.xin;
    RT rhs_v = (RT)0;
    double aux = 0.0, aux2 = 0.0, dsh = 1.0, cf = 1.0;
    if (live) {
        if (a.epi != EPI_SPMV) rhs_v = ((const RT *)a.rhs)[row];
        if (a.epi == EPI_UPDATE) aux = a.x[row];
        if (a.epi == EPI_SCALE || a.epi == EPI_SCALE_UPDATE) aux = a.dinv[row];
        if (a.epi == EPI_SCALE_UPDATE) aux2 = a.x[row];
        if (a.dcol && (a.epi == EPI_UPDATE || a.epi == EPI_SCALE_UPDATE)) cf = a.dcol[row];
        if (a.dshift) dsh = a.dshift[row];
    }
    AT sum = (AT)0;
    if (live && a.dshift) sum = (AT)((dsh - 1.0) * (double)xin[row]);
    if (kf >= 0 && G <= GM && G >= 1) {
        sum = slice_sum_pat_g<T, GM>(G, s, p0, lane, row, xin, pt, sum);
    } else {
        const int len = kf >= 0 ? 4 * G : (live ? a.rp[row + 1] - a.rp[row] : 0);
        const int safe = min(row, a.n - 1);
        for (int q = 0; q < G; ++q) {
            VT v[4];
            if (sizeof(VT) == 8) {
                const f64x2 *pv = (const f64x2 *)s.val + (p0 >> 1) + 128 * q + lane;
                const f64x2 lo2 = __builtin_nontemporal_load(pv), hi2 = __builtin_nontemporal_load(pv + 64);
                v[0] = (VT)lo2.x;
                v[1] = (VT)lo2.y;
                v[2] = (VT)hi2.x;
                v[3] = (VT)hi2.y;
            } else {
                const f32x4 v4 = __builtin_nontemporal_load((const f32x4 *)s.val + (p0 >> 2) + 64 * q + lane);
                v[0] = (VT)v4.x;
                v[1] = (VT)v4.y;
                v[2] = (VT)v4.z;
                v[3] = (VT)v4.w;
            }
            const i32x4 o = *(const i32x4 *)(pt + 4 * q);
            const int j[4] = {row + o.x, row + o.y, row + o.z, row + o.w};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool on = 4 * q + r < len;
                const AT t = sum + (AT)v[r] * (AT)xin[on ? j[r] : safe];
                sum = on ? t : sum;
            }
        }
    }
    const AT t = a.epi == EPI_SPMV ? sum : (AT)rhs_v - sum;
    if (live) epilogue_pre<T>(a, row, t, aux, aux2, cf);
    return live ? (double)t : 0.0;
}

// One slice per wave, slices in launch order (the XCD slab remap measured 3 %
// slower here).  The pattern table is small (at most PAT_MAX_ENTRIES offsets)
// and stays in the caches, so each lane reads its row's offsets from it
// directly, one 16-byte load per group of four slots: no copy to LDS and no
// barrier ahead of the value loads.  (Measured on the n = 8M 27-point factors:
// 295 us per sweep against 300 us with the table staged in LDS for four
// rounds of slices per workgroup, and 34.8 against 35.6 us at n = 2M.)
template <class T, int WPB, int GM>
__global__ void __launch_bounds__(64 * WPB) k_sweep_sliced_pat(SweepArgs a, SlicedView s)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WPB + ((int)threadIdx.x >> 6));
    if (wave >= s.nslice) return;
    const int lane = (int)threadIdx.x & 63;
    sliced_wave_pat<T, GM>(a, s, wave, s.sk[wave], s.sptr[wave], s.ptab + (int)s.pid[wave * 64 + lane] * s.kp);
}

// Launch of the row-pattern sweep, the body specialised on the matrix's
// largest group count.
template <class T, int WPB>
hipError_t go_pat(const SweepGeom &g, const SweepArgs &a, hipStream_t s)
{
    const dim3 pgrid((g.sl.nslice + WPB - 1) / WPB), block(64 * WPB);
    switch (g.sl.gmax) {
    case 1: hipLaunchKernelGGL((k_sweep_sliced_pat<T, WPB, 1>), pgrid, block, 0, s, a, g.sl); break;
    case 2: hipLaunchKernelGGL((k_sweep_sliced_pat<T, WPB, 2>), pgrid, block, 0, s, a, g.sl); break;
    case 3: hipLaunchKernelGGL((k_sweep_sliced_pat<T, WPB, 3>), pgrid, block, 0, s, a, g.sl); break;
    case 4: hipLaunchKernelGGL((k_sweep_sliced_pat<T, WPB, 4>), pgrid, block, 0, s, a, g.sl); break;
    case 5: hipLaunchKernelGGL((k_sweep_sliced_pat<T, WPB, 5>), pgrid, block, 0, s, a, g.sl); break;
    case 6: hipLaunchKernelGGL((k_sweep_sliced_pat<T, WPB, 6>), pgrid, block, 0, s, a, g.sl); break;
    case 7: hipLaunchKernelGGL((k_sweep_sliced_pat<T, WPB, 7>), pgrid, block, 0, s, a, g.sl); break;
    default: hipLaunchKernelGGL((k_sweep_sliced_pat<T, WPB, 8>), pgrid, block, 0, s, a, g.sl); break;
    }
    return hipGetLastError();
}

// Diagonal slices (code 16): every row lies on the same few diagonals (a
// stencil operator and its ILU(0)/ILU(1) factors), so slot k of every row
// holds its entry on diagonal d_k (0 where the row has none) and the rows of
// a slice share their slots' column offsets: no per-slot code, no per-row
// pattern, and neighbouring rows gather neighbouring iterate values.  Each
// lane owns two consecutive rows of a 128-row slice: one load (16 bytes in
// FP64, 8 in FP32) brings both rows' values of a slot, one load both rows'
// iterate values on that slot's diagonal -- half the iterate loads of one row
// per lane, whose count (not their bytes) bounds the row-pattern sweeps.
// Every value and iterate load of the slice is issued before the first is
// waited for (the FP64 kernel is compiled for two waves per SIMD where the U
// slots need the registers), the rhs after them; so are the other epilogue
// operands, except above 24 slots, where their registers would not fit
// beside the slots' and they are loaded once the sums are done.  Each row's
// products are summed in ascending diagonal (= column) order in the
// precision's accumulator (no unscaled-variant diagonal term: such sweeps
// take the row-pattern copy); a slot the row lacks adds 0 * x = +-0 to a sum
// that started at +0 and so is never -0, which leaves it unchanged: finite
// results are the row sums of the oracle (and of its FP32-inner emulation)
// bit for bit.  In the slices at either end of the matrix the iterate pair
// is loaded at the column clamped into [0, n - 2]: a column outside the
// matrix only occurs on a slot whose value is 0, and the clamped pair still
// gives the other row of the lane its own value.
// A row's epilogue operands (those of epilogue_pre), for rows that exist.
__device__ __forceinline__ void diag_operands(const SweepArgs &a, int row, double &aux, double &aux2, double &cf)
{
    if (row >= a.n) return;
    if (a.epi == EPI_UPDATE) aux = a.x[row];
    if (a.epi == EPI_SCALE || a.epi == EPI_SCALE_UPDATE) aux = a.dinv[row];
    if (a.epi == EPI_SCALE_UPDATE) aux2 = a.x[row];
    if (a.dcol && (a.epi == EPI_UPDATE || a.epi == EPI_SCALE_UPDATE)) cf = a.dcol[row];
}

// Two consecutive elements (the lane's two rows) as one vector, and their
// load from a buffer resource: 16 bytes for FP64, 8 for FP32.
template <class E>
struct Pair2 {
    using type = f64x2;
};
template <>
struct Pair2<float> {
    using type = f32x2;
};
// AUX: the load's cache policy bits (2: non-temporal).
template <class E, int AUX>
__device__ __forceinline__ typename Pair2<E>::type buf_pair(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    if constexpr (sizeof(E) == 8)
        return __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
    else
        return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
}

template <class T, int U>
__device__ __forceinline__ void diag_slice(const SweepArgs &a, const SlicedView &s, int wave)
{
    using VT = typename T::VT;
    using XT = typename T::XT;
    using RT = typename T::RT;
    using AT = typename T::AT;
    using IT = typename T::IT;
    using OT = typename T::OT;
    using VP = typename Pair2<VT>::type;
    using XP = typename Pair2<XT>::type;
    constexpr int vb = (int)sizeof(VT), xb = (int)sizeof(XT);
    const int n = a.n;
    const int lane = (int)threadIdx.x & 63;
    const int ra = wave * 128 + 2 * lane;
    const XT *__restrict__ xin = (const XT *)a.xin;
    int d[U];
#pragma unroll
    for (int k = 0; k < U; ++k) d[k] = __builtin_amdgcn_readfirstlane(s.dtab[k]);
    VP v[U];
    XP xv[U];
    const int r0 = wave * 128;
    if (r0 + d[0] >= 0 && r0 + 127 + d[U - 1] <= n - 1) { // every column inside the matrix
        // buffer loads: the slice's values and its iterate window as two
        // resources, the slot's offset in a scalar register, the lane's in one
        // vector register shared by every load (no address registers per load)
        const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((const VT *)s.val + (int64_t)wave * U * 128), (short)0, U * 128 * vb, 0x00020000);
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(xin + (r0 + d[0])), (short)0, (128 + d[U - 1] - d[0]) * xb, 0x00020000);
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = buf_pair<VT, 2>(rv, lane * 2 * vb, k * 128 * vb);
#pragma unroll
        for (int k = 0; k < U; ++k) xv[k] = buf_pair<XT, 0>(rx, lane * 2 * xb, (d[k] - d[0]) * xb);
    } else { // a slice at either end of the matrix
        const VP *pv = (const VP *)((const VT *)s.val + (int64_t)wave * U * 128) + lane;
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = __builtin_nontemporal_load(pv + 64 * k);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int raw = ra + d[k];
            const int idx = min(max(raw, 0), n - 2);
            XP t;
            __builtin_memcpy(&t, xin + idx, 2 * xb);
            xv[k].x = raw > n - 2 ? t.y : t.x;
            xv[k].y = raw < 0 ? t.x : t.y;
        }
    }
    RT rh0 = (RT)0, rh1 = (RT)0;
    if (a.epi != EPI_SPMV) { // the lane's two rows with one load
        if (ra + 1 < n) {
            RT t2[2];
            __builtin_memcpy(t2, (const RT *)a.rhs + ra, 2 * sizeof(RT));
            rh0 = t2[0];
            rh1 = t2[1];
        } else if (ra < n) {
            rh0 = ((const RT *)a.rhs)[ra];
        }
    }
    double aux0 = 0.0, aux1 = 0.0, aux20 = 0.0, aux21 = 0.0, cf0 = 1.0, cf1 = 1.0;
    if constexpr (U <= 24) {
        diag_operands(a, ra, aux0, aux20, cf0);
        diag_operands(a, ra + 1, aux1, aux21, cf1);
    }
    AT sa = (AT)0, sb = (AT)0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
        sa = sa + (AT)v[k].x * (AT)xv[k].x;
        sb = sb + (AT)v[k].y * (AT)xv[k].y;
    }
    if constexpr (U > 24) {
        diag_operands(a, ra, aux0, aux20, cf0);
        diag_operands(a, ra + 1, aux1, aux21, cf1);
    }
    const AT ta = a.epi == EPI_SPMV ? sa : (AT)rh0 - sa, tb = a.epi == EPI_SPMV ? sb : (AT)rh1 - sb;
    if (ra + 1 < n && (a.epi == EPI_STORE || a.epi == EPI_SPMV || a.epi == EPI_STORE_SPLIT)) {
        // the stores of epilogue_pre for both rows, each one store
        const OT o2[2] = {(OT)(IT)ta, (OT)(IT)tb};
        __builtin_memcpy((OT *)a.out + ra, o2, 2 * sizeof(OT));
        if (a.epi == EPI_STORE_SPLIT) {
            const float f2[2] = {(float)(IT)ta, (float)(IT)tb};
            __builtin_memcpy(a.out32 + ra, f2, 8);
        }
    } else {
        if (ra < n) epilogue_pre<T>(a, ra, ta, aux0, aux20, cf0);
        if (ra + 1 < n) epilogue_pre<T>(a, ra + 1, tb, aux1, aux21, cf1);
    }
}

// Slices in launch order (the XCD slab remap of the other sweeps measured 2 %
// slower for this kernel).
template <class T, int U>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_sweep_diag_wide(SweepArgs a,
                                                                                                      SlicedView s)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + ((int)threadIdx.x >> 6));
    if (wave < s.nslice) diag_slice<T, U>(a, s, wave);
}

template <class T, int U>
__global__ void __launch_bounds__(256) k_sweep_diag(SweepArgs a, SlicedView s)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + ((int)threadIdx.x >> 6));
    if (wave < s.nslice) diag_slice<T, U>(a, s, wave);
}

// Launch of the diagonal-slice sweep, specialised on the number of diagonals
// (13 to 28 take the two-waves-per-SIMD build, which keeps all the loads of a
// slice in flight without spilling; with fewer the registers allow that at
// any occupancy, with more only at one wave per SIMD).
template <class T, int U>
hipError_t go_diag_u(const SweepGeom &g, const SweepArgs &a, hipStream_t s)
{
    const dim3 grid((g.sl.nslice + 3) / 4), block(256);
    if constexpr (sizeof(typename T::VT) + sizeof(typename T::XT) == 16 && U > 12 && U <= 28)
        hipLaunchKernelGGL((k_sweep_diag_wide<T, U>), grid, block, 0, s, a, g.sl);
    else
        hipLaunchKernelGGL((k_sweep_diag<T, U>), grid, block, 0, s, a, g.sl);
    return hipGetLastError();
}

template <class T, int U = DIAG_MAX>
hipError_t go_diag(const SweepGeom &g, const SweepArgs &a, hipStream_t s)
{
    if (g.sl.ndiag == U) return go_diag_u<T, U>(g, a, s);
    if constexpr (U > 1) return go_diag<T, U - 1>(g, a, s);
    return hipErrorInvalidValue;
}

// Row-pattern slices with iterate windows (s.nwin > 0).  A slice's 64 rows
// gather from nwin windows of 128 consecutive iterate entries (the runs of the
// pattern table's offsets, each run within 64 of its even start): the wave
// loads each window with one load of two entries per lane into its own LDS
// region (FP64: a 16-byte buffer load straight into LDS; FP32: through
// registers, there being no 8-byte form) and takes every slot's x from
// there, at lane + ltab[...], instead of one gather per slot from the caches
// -- nwin loads in place of 4G gathers (aniso 27-point ILUT factors: 7
// windows against 20 gathers per row).  The windows, the value loads and the
// slots' LDS indices are all issued before the first is waited for.  Each wave writes and reads only its own region,
// and LDS operations of one wave complete in order, so no barrier is needed.
// The x read for a slot is x[row + offset] as in the gather body, and the
// sums keep the same order: results are the same bit for bit.  Masked slices,
// slices above GM groups, those whose windows would reach outside the matrix
// and those with a row on an offset run left without a window take the
// gather body.  On the n = 8M 27-point ILUT factors: about 241 us per FP64
// sweep (252 us with the windows staged through registers) against 269 us
// with gathers; the FP32-inner sweeps gain
// 1-1.5 % (137 against 139 us), and only when held to six waves per SIMD
// (70-72 registers; at the unconstrained 85 registers and five waves they
// were 4-5 % slower than their 4-byte gathers, at eight waves they spill;
// above six groups six waves spill too, so those bodies get five).
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

template <class T, int NW>
__device__ __forceinline__ void load_windows(const SlicedView &s, const typename T::XT *__restrict__ xin, int r0,
                                             int lane, typename T::XT *lw)
{
    using XT = typename T::XT;
    using XP = typename Pair2<XT>::type;
    constexpr int xb = (int)sizeof(XT);
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc((void *)(xin + (r0 + s.wst[0])), (short)0, s.wspan * xb, 0x00020000);
    if constexpr (xb == 8) {
        // straight into LDS, lane l's 16 bytes at window + 16 l: no registers
        // and no LDS writes; the caller waits for them before reading
#pragma unroll
        for (int c = 0; c < NW; ++c)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (__attribute__((address_space(3))) void *)(lw + 128 * c), 16,
                                                     lane * 16, (s.wst[c] - s.wst[0]) * 8, 0, 0);
    } else { // no 8-byte form of those loads: through registers
        XP w[NW];
#pragma unroll
        for (int c = 0; c < NW; ++c) w[c] = buf_pair<XT, 0>(rx, lane * 2 * xb, (s.wst[c] - s.wst[0]) * xb);
#pragma unroll
        for (int c = 0; c < NW; ++c) *(XP *)(lw + 128 * c + 2 * lane) = w[c];
    }
}

// All of the slice's windows, one case per window count.
template <class T>
__device__ __forceinline__ void stage_windows(const SlicedView &s, const typename T::XT *__restrict__ xin, int r0,
                                              int lane, typename T::XT *lw)
{
    switch (s.nwin) {
    case 1: load_windows<T, 1>(s, xin, r0, lane, lw); break;
    case 2: load_windows<T, 2>(s, xin, r0, lane, lw); break;
    case 3: load_windows<T, 3>(s, xin, r0, lane, lw); break;
    case 4: load_windows<T, 4>(s, xin, r0, lane, lw); break;
    case 5: load_windows<T, 5>(s, xin, r0, lane, lw); break;
    case 6: load_windows<T, 6>(s, xin, r0, lane, lw); break;
    case 7: load_windows<T, 7>(s, xin, r0, lane, lw); break;
    case 8: load_windows<T, 8>(s, xin, r0, lane, lw); break;
    case 9: load_windows<T, 9>(s, xin, r0, lane, lw); break;
    case 10: load_windows<T, 10>(s, xin, r0, lane, lw); break;
    case 11: load_windows<T, 11>(s, xin, r0, lane, lw); break;
    default: load_windows<T, 12>(s, xin, r0, lane, lw); break;
    }
    static_assert(PAT_WIN_MAX == 12, "one case per window count");
}

template <class T, int GG>
__device__ __forceinline__ typename T::AT slice_sum_win(const SlicedView &s, int p0, int lane, int r0,
                                                        const typename T::XT *__restrict__ xin, typename T::XT *lw,
                                                        const uint16_t *lt, typename T::AT sum)
{
    using VT = typename T::VT;
    using XT = typename T::XT;
    using AT = typename T::AT;
    VT v[GG][4];
#pragma unroll
    for (int q = 0; q < GG; ++q) {
        if (sizeof(VT) == 8) {
            const f64x2 *pv = (const f64x2 *)s.val + (p0 >> 1) + 128 * q + lane;
            const f64x2 lo2 = __builtin_nontemporal_load(pv), hi2 = __builtin_nontemporal_load(pv + 64);
            v[q][0] = (VT)lo2.x;
            v[q][1] = (VT)lo2.y;
            v[q][2] = (VT)hi2.x;
            v[q][3] = (VT)hi2.y;
        } else {
            const f32x4 v4 = __builtin_nontemporal_load((const f32x4 *)s.val + (p0 >> 2) + 64 * q + lane);
            v[q][0] = (VT)v4.x;
            v[q][1] = (VT)v4.y;
            v[q][2] = (VT)v4.z;
            v[q][3] = (VT)v4.w;
        }
    }
    u16x4 o[GG]; // two groups' elements per 16-byte load
#pragma unroll
    for (int q = 0; q < GG; q += 2) {
        const u16x8 t = *(const u16x8 *)(lt + 4 * q);
        o[q] = t.lo;
        if (q + 1 < GG) o[q + 1] = t.hi;
    }
    if constexpr (sizeof(XT) == 8)
        __builtin_amdgcn_s_waitcnt(0x0F70); // vmcnt(0): the windows, loaded straight into LDS, have landed
    else
        stage_windows<T>(s, xin, r0, lane, lw);
    __builtin_amdgcn_wave_barrier();
    XT xv[GG][4];
#pragma unroll
    for (int q = 0; q < GG; ++q) {
        xv[q][0] = lw[lane + o[q].x];
        xv[q][1] = lw[lane + o[q].y];
        xv[q][2] = lw[lane + o[q].z];
        xv[q][3] = lw[lane + o[q].w];
    }
#pragma unroll
    for (int q = 0; q < GG; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) sum = sum + (AT)v[q][r] * (AT)xv[q][r];
    }
    return sum;
}

template <class T, int GG>
__device__ __forceinline__ typename T::AT slice_sum_win_g(int G, const SlicedView &s, int p0, int lane, int r0,
                                                          const typename T::XT *__restrict__ xin,
                                                          typename T::XT *lw, const uint16_t *lt,
                                                          typename T::AT sum)
{
    if (G == GG) return slice_sum_win<T, GG>(s, p0, lane, r0, xin, lw, lt, sum);
    if constexpr (GG > 1) return slice_sum_win_g<T, GG - 1>(G, s, p0, lane, r0, xin, lw, lt, sum);
    return sum;
}

template <class T, int WPB, int GM>
__global__ void __launch_bounds__(64 * WPB)
    __attribute__((amdgpu_waves_per_eu(sizeof(typename T::XT) == 4 ? (GM <= 6 ? 6 : 5) : 1)))
    k_sweep_pat_win(SweepArgs a, SlicedView s)
{
    using XT = typename T::XT;
    using RT = typename T::RT;
    using AT = typename T::AT;
    extern __shared__ f64x2 win_lds[];
    const int wave = __builtin_amdgcn_readfirstlane((int)blockIdx.x * WPB + ((int)threadIdx.x >> 6));
    if (wave >= s.nslice) return;
    const int lane = (int)threadIdx.x & 63;
    const int kf = s.sk[wave], p0 = s.sptr[wave];
    const int pidl = (int)s.pid[wave * 64 + lane];
    const int G = (kf & 0x7fffffff) >> 2;
    const int r0 = wave * 64;
    if (kf < 0 || G > GM || G < 1 || !s.wflag[wave] || r0 + s.wst[0] < 0 || (int64_t)r0 + s.wst[0] + s.wspan > a.n) {
        sliced_wave_pat<T, GM>(a, s, wave, kf, p0, s.ptab + pidl * s.kp);
        return;
    }
    // an unmasked slice inside the matrix: all 64 rows exist and hold entries
    XT *lw = (XT *)win_lds + ((int)threadIdx.x >> 6) * s.nwin * 128;
    const int row = r0 + lane;
    const XT *__restrict__ xin = (const XT *)a.xin;
    RT rhs_v = (RT)0;
    double aux = 0.0, aux2 = 0.0, dsh = 1.0, cf = 1.0;
    if (a.epi != EPI_SPMV) rhs_v = ((const RT *)a.rhs)[row];
    if (a.epi == EPI_UPDATE) aux = a.x[row];
    if (a.epi == EPI_SCALE || a.epi == EPI_SCALE_UPDATE) aux = a.dinv[row];
    if (a.epi == EPI_SCALE_UPDATE) aux2 = a.x[row];
    if (a.dcol && (a.epi == EPI_UPDATE || a.epi == EPI_SCALE_UPDATE)) cf = a.dcol[row];
    if (a.dshift) dsh = a.dshift[row];
    AT sum = (AT)0;
    if (a.dshift) sum = (AT)((dsh - 1.0) * (double)xin[row]);
    // FP64 windows go straight to LDS and are issued here, once, ahead of the
    // group dispatch: issued inside each group count's body, the compiler
    // merged the bodies' copies and waited for every load in flight before
    // each window, not telling the windows' LDS targets apart
    if constexpr (sizeof(XT) == 8) stage_windows<T>(s, xin, r0, lane, lw);
    sum = slice_sum_win_g<T, GM>(G, s, p0, lane, r0, xin, lw, s.ltab + pidl * s.kl, sum);
    const AT t = a.epi == EPI_SPMV ? sum : (AT)rhs_v - sum;
    epilogue_pre<T>(a, row, t, aux, aux2, cf);
}

// Launch of the windowed row-pattern sweep, the body specialised on the
// matrix's largest group count; the LDS holds each wave's windows.
template <class T, int WPB>
hipError_t go_pat_win(const SweepGeom &g, const SweepArgs &a, hipStream_t s)
{
    const dim3 pgrid((g.sl.nslice + WPB - 1) / WPB), block(64 * WPB);
    const size_t lds = (size_t)WPB * g.sl.nwin * 128 * sizeof(typename T::XT);
    switch (g.sl.gmax) {
    case 1: hipLaunchKernelGGL((k_sweep_pat_win<T, WPB, 1>), pgrid, block, lds, s, a, g.sl); break;
    case 2: hipLaunchKernelGGL((k_sweep_pat_win<T, WPB, 2>), pgrid, block, lds, s, a, g.sl); break;
    case 3: hipLaunchKernelGGL((k_sweep_pat_win<T, WPB, 3>), pgrid, block, lds, s, a, g.sl); break;
    case 4: hipLaunchKernelGGL((k_sweep_pat_win<T, WPB, 4>), pgrid, block, lds, s, a, g.sl); break;
    case 5: hipLaunchKernelGGL((k_sweep_pat_win<T, WPB, 5>), pgrid, block, lds, s, a, g.sl); break;
    case 6: hipLaunchKernelGGL((k_sweep_pat_win<T, WPB, 6>), pgrid, block, lds, s, a, g.sl); break;
    case 7: hipLaunchKernelGGL((k_sweep_pat_win<T, WPB, 7>), pgrid, block, lds, s, a, g.sl); break;
    default: hipLaunchKernelGGL((k_sweep_pat_win<T, WPB, 8>), pgrid, block, lds, s, a, g.sl); break;
    }
    return hipGetLastError();
}

template <class T, int CODE, int WPB, int UNR>
__global__ void __launch_bounds__(64 * WPB) k_sweep_sliced(SweepArgs a, SlicedView s)
{
    __shared__ int32_t dtab[256];
    if (CODE == 1) {
        for (int t = (int)threadIdx.x; t < s.ndiag; t += 64 * WPB) dtab[t] = s.dtab[t];
        __syncthreads();
    }
    const int wave = xcd_slab_block((int)blockIdx.x, (int)gridDim.x) * WPB + ((int)threadIdx.x >> 6);
    sliced_wave<T, CODE, UNR>(a, s, wave, dtab);
}

// One 256-row tile of a batched op, run by a workgroup of 256 lanes: as four
// 64-row slices of the op's sliced copy when it has one (a.sv), else as the
// CSR stream.  Row-pattern and diagonal-table slices of at most two groups
// take the prefetched bodies, larger ones their loops: with a bound of two
// the kernel keeps the loop form's 76 registers, where bounds of four and
// eight (122 and 132 registers) cost 20 and 32 % of the batched saturation
// rate on 7-point matrices.  Either way each row is summed in ascending column order, so
// the result is the single-request one bit for bit.
// A solve request's op is skipped once its request has stopped (the flag was
// set by an earlier launch); a check op then reduces r_i^2 (and b_i^2 on the
// first check) over its tile in a fixed order (lane i holds row 256 tile + i
// in both paths) and writes the two sums for the step's check launch.
template <class T>
__device__ __forceinline__ void batch_tile(const SweepArgs &a, int tile)
{
    static_assert(SERVE_TILE_ROWS == 256, "four slices per workgroup");
    if (a.sctl && *(const volatile int32_t *)&a.sctl->stop) return;
    double t;
    if (!a.sv) {
        t = stream_rows<T, 256, 256, 1024, IDX32>(a, tile, nullptr, 0, nullptr, 0);
    } else {
        __shared__ int32_t dtab[256];
        const SlicedView s = *a.sv;
        const int wave = tile * 4 + ((int)threadIdx.x >> 6);
        if (s.code == 8) {
            const int wc = min(__builtin_amdgcn_readfirstlane(wave), s.nslice - 1);
            const int lane = (int)threadIdx.x & 63;
            t = wave < s.nslice ? sliced_wave_pat<T, 2>(a, s, wc, s.sk[wc], s.sptr[wc],
                                                         s.ptab + (int)s.pid[wc * 64 + lane] * s.kp)
                                : 0.0;
        } else if (s.code == 1) {
            for (int k = (int)threadIdx.x; k < s.ndiag; k += 256) dtab[k] = s.dtab[k];
            __syncthreads();
            t = sliced_wave_pf<T, 2>(a, s, wave, dtab);
        } else if (s.code == 2) {
            t = sliced_wave<T, 2, 2>(a, s, wave, dtab);
        } else {
            t = sliced_wave<T, 4, 2>(a, s, wave, dtab);
        }
    }
    if (!a.scheck) return;
    // butterfly sums within each wave (every lane ends with the same bits:
    // both operands of each addition are the same on all lanes), then the
    // four wave sums in order
    __shared__ double wsum[2][4];
    const int tid = (int)threadIdx.x, row = tile * 256 + tid;
    double bv = 0.0;
    if (a.scheck == 2 && row < a.n) bv = ((const double *)a.rhs)[row];
    double r2 = t * t, b2 = bv * bv;
    for (int off = 32; off > 0; off >>= 1) {
        r2 = r2 + __shfl_xor(r2, off, 64);
        b2 = b2 + __shfl_xor(b2, off, 64);
    }
    if ((tid & 63) == 0) {
        wsum[0][tid >> 6] = r2;
        wsum[1][tid >> 6] = b2;
    }
    __syncthreads();
    if (tid == 0) {
        a.spart[2 * tile] = ((wsum[0][0] + wsum[0][1]) + wsum[0][2]) + wsum[0][3];
        a.spart[2 * tile + 1] = ((wsum[1][0] + wsum[1][1]) + wsum[1][2]) + wsum[1][3];
    }
}

// Closes the checks of one step (one workgroup per check): the tile partials
// summed in a fixed order, then the test of eq. relres.
__global__ void __launch_bounds__(256) k_solve_check(SolveCheckArgs ca)
{
    const SolveCheck c = ca.c[blockIdx.x];
    if (*(const volatile int32_t *)&c.ctl->stop) return; // its check op did nothing
    __shared__ double red[2][256];
    const int tid = (int)threadIdx.x;
    double rr = 0.0, bb = 0.0;
    for (int k = tid; k < c.tiles; k += 256) {
        rr = rr + c.part[2 * k];
        bb = bb + c.part[2 * k + 1];
    }
    red[0][tid] = rr;
    red[1][tid] = bb;
    for (int off = 128; off > 0; off >>= 1) {
        __syncthreads();
        if (tid < off) {
            red[0][tid] = red[0][tid] + red[0][tid + off];
            red[1][tid] = red[1][tid] + red[1][tid + off];
        }
    }
    if (tid == 0) {
        SolveCtl *ctl = c.ctl;
        const double b2 = c.first ? red[1][0] : ctl->bb;
        ctl->rr = red[0][0];
        ctl->bb = b2;
        ctl->checks = ctl->checks + 1;
        if (sqrt(red[0][0]) / sqrt(b2) < c.tol) {
            ctl->stop = 1;
            if (c.hflag) { // tells the host, which then schedules no more sweeps for the request
                __threadfence_system();
                *(volatile int32_t *)c.hflag = 1;
            }
        }
    }
}

// Batched sweeps: one launch runs one sweep of one precision for each of
// `nops` independent requests (different matrices, sizes and epilogues).  Op
// i owns workgroups [first[i], first[i+1]); each workgroup finds its op
// (find_op) and runs exactly the single-request body for its tile
// (batch_tile), so a request's result does not depend on what else shares
// the launch.
// The op owning workgroup b: the largest i < nops with first[i] <= b (first
// increases strictly from first[0] = 0).  Up to 64 ops each lane of the wave
// tests one entry and a ballot counts those at or below b, so the wave issues
// one load instead of a chain of dependent ones; beyond that, bisection.
__device__ __forceinline__ int find_op(const int32_t *first, int nops, int b)
{
    if (nops <= 64) {
        const int lane = (int)threadIdx.x & 63;
        bool le = false;
        if (lane < nops) le = first[lane] <= b; // lanes past the table load nothing
        return __popcll(__ballot(le)) - 1;
    }
    int lo = 0, hi = nops - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class T>
__global__ void __launch_bounds__(256) k_sweep_batch(const SweepArgs *__restrict__ ops,
                                                     const int32_t *__restrict__ first, int nops)
{
    const int b = (int)blockIdx.x;
    const int i = find_op(first, nops, b);
    batch_tile<T>(ops[i], b - first[i]);
}

// The same with the op table in the kernel arguments, sized for at most CAP
// ops (the argument block is copied at every launch, so small batches use a
// small one).
template <int CAP>
struct BatchArgsN {
    SweepArgs op[CAP];
    int32_t first[CAP + 1];
    int nops;
};

template <class T, int CAP>
__global__ void __launch_bounds__(256) k_sweep_batch_args(BatchArgsN<CAP> ba)
{
    const int b = (int)blockIdx.x;
    const int i = find_op(ba.first, ba.nops, b);
    batch_tile<T>(ba.op[i], b - ba.first[i]);
}

template <class T, int CAP>
hipError_t go_batch_args(const BatchArgs &b, hipStream_t s)
{
    BatchArgsN<CAP> n;
    for (int i = 0; i < b.nops; i++) {
        n.op[i] = b.op[i];
        n.first[i] = b.first[i];
    }
    n.first[b.nops] = b.first[b.nops];
    n.nops = b.nops;
    hipLaunchKernelGGL((k_sweep_batch_args<T, CAP>), dim3(b.first[b.nops]), dim3(256), 0, s, n);
    return hipGetLastError();
}

template <class T>
hipError_t go_batch_args_sized(const BatchArgs &b, hipStream_t s)
{
    if (b.nops <= 2) return go_batch_args<T, 2>(b, s);
    if (b.nops <= 8) return go_batch_args<T, 8>(b, s);
    return go_batch_args<T, BATCH_ARG_OPS>(b, s);
}

// Persistent batched CSR-stream: one launch runs whole chains of sweeps (all
// the ops of several requests).  The tiles of every op (RPB rows each) form
// one queue, numbered in the plan's op order, in which each op comes after
// the op it depends on (the previous sweep of its request).  A workgroup
// takes the next tile number from ctl[0]; before running a tile of an op
// with a dependency it waits until done[dep] counts every tile of that op.
// The wait cannot deadlock: the tiles it waits for have smaller numbers, so
// workgroups that are already running took them, and the smallest unfinished
// tile never waits.  Each wait is bounded in wall-clock time (p.wait_ticks of
// the constant-rate clock wall_clock64 reads, however long each poll takes):
// on expiry the op's index + 1 goes to ctl[1], the tile is skipped and still
// counted, so every workgroup drains in bounded time and the host reports the
// failure.
// Memory order: every XCD has its own L2; the counters are updated and
// polled at system scope so that their coherence does not rest on any one
// L2.  A finished tile's stores reach memory through each thread's fence (L2
// write-back) before the barrier and the count; the waiting thread fences (L2
// invalidate) after observing the count, before the barrier that releases its
// workgroup.  (The serving runtime does not launch this kernel: on MI355X its
// launches did not finish, at agent and at system scope, for a cause not yet
// found.)
template <class T, int BLOCK, int RPB, int CAP>
__global__ void __launch_bounds__(BLOCK) k_sweep_persist(PersistPlan p)
{
    __shared__ int s_tile, s_op, s_skip;
    const int total = p.first[p.nops];
    for (;;) {
        if (threadIdx.x == 0) {
            const int t = __hip_atomic_fetch_add(&p.ctl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            int op = 0, skip = 0;
            if (t < total) {
                int lo = 0, hi = p.nops - 1; // largest op with first[op] <= t
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (p.first[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                op = lo;
                const int d = p.dep[op];
                if (d >= 0) {
                    const int need = p.first[d + 1] - p.first[d];
                    const long long t0 = wall_clock64();
                    while (__hip_atomic_load(&p.done[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) < need) {
                        __builtin_amdgcn_s_sleep(4);
                        if (wall_clock64() - t0 >= p.wait_ticks) {
                            int zero = 0;
                            __hip_atomic_compare_exchange_strong(&p.ctl[1], &zero, op + 1, __ATOMIC_RELAXED,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                            skip = 1;
                            break;
                        }
                    }
                    __threadfence();
                }
            }
            s_tile = t;
            s_op = op;
            s_skip = skip;
        }
        __syncthreads();
        const int t = s_tile, op = s_op, skip = s_skip;
        __syncthreads();
        if (t >= total) return;
        if (!skip) stream_rows<T, BLOCK, RPB, CAP, IDX32>(p.ops[op], t - p.first[op], nullptr, 0, nullptr, 0);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(&p.done[op], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// ---------------------------------------------------------------------------
// CSR-stream over a row-block partition: workgroup b owns rows
// [blk[b].row, blk[b+1].row) whose entries are [blk[b].ent, blk[b+1].ent): at
// most RMAX rows and CAP entries (a single longer row gets a workgroup alone
// and is streamed in chunks).  The partition carries the entry offsets, so
// every lane issues its CAP/BLOCK val and col loads at once, with no wait on
// the row pointers, and with non-temporal hints: the factor is streamed once
// per sweep and must not evict the gathered iterate window from L2.  The
// products go to LDS and each row is then summed by one lane in ascending
// column order.
// ---------------------------------------------------------------------------
template <class T, int BLOCK, int CAP, int RMAX>
__global__ void __launch_bounds__(BLOCK) k_sweep_rb(SweepArgs a, const int2 *__restrict__ blk)
{
    using VT = typename T::VT;
    using XT = typename T::XT;
    using RT = typename T::RT;
    using AT = typename T::AT;
    constexpr int U = CAP / BLOCK;
    static_assert(CAP % BLOCK == 0 && RMAX % BLOCK == 0, "geometry");
    __shared__ AT prod[CAP];
    __shared__ int32_t srp[RMAX + 1];

    const int b = xcd_slab_block((int)blockIdx.x, (int)gridDim.x);
    const int2 lo = blk[b], hi = blk[b + 1];
    const int r0 = lo.x, nr = hi.x - lo.x, e0 = lo.y, e1 = hi.y;
    const int tid = (int)threadIdx.x;

    const VT *__restrict__ val = (const VT *)a.val;
    const int32_t *__restrict__ col = a.col;
    const XT *__restrict__ xin = (const XT *)a.xin;
    const RT *__restrict__ rhs = (const RT *)a.rhs;

    if (e1 - e0 <= CAP) {
        const int cn = e1 - e0;
        VT v[U];
        int32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = u * BLOCK + tid;
            if (k < cn) {
                v[u] = __builtin_nontemporal_load(&val[e0 + k]);
                c[u] = __builtin_nontemporal_load(&col[e0 + k]);
            }
        }
        for (int t = tid; t <= nr; t += BLOCK) srp[t] = a.rp[r0 + t];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = u * BLOCK + tid;
            if (k < cn) prod[k] = (AT)v[u] * (AT)xin[c[u]];
        }
        __syncthreads();
        for (int t = tid; t < nr; t += BLOCK) {
            const int row = r0 + t;
            AT sum = (AT)0;
            if (a.dshift) sum = (AT)((a.dshift[row] - 1.0) * (double)xin[row]);
            const int klo = srp[t] - e0, khi = srp[t + 1] - e0;
            for (int k = klo; k < khi; ++k) sum = sum + prod[k];
            epilogue<T>(a, row, a.epi == EPI_SPMV ? sum : (AT)rhs[row] - sum);
        }
        return;
    }
    // one long row, streamed through LDS in chunks of CAP entries
    const int row = r0;
    AT sum = (AT)0;
    if (a.dshift) sum = (AT)((a.dshift[row] - 1.0) * (double)xin[row]);
    for (int c0 = e0; c0 < e1; c0 += CAP) {
        const int cn = min(CAP, e1 - c0);
        for (int k = tid; k < cn; k += BLOCK) prod[k] = (AT)val[c0 + k] * (AT)xin[col[c0 + k]];
        __syncthreads();
        if (tid == 0)
            for (int k = 0; k < cn; ++k) sum = sum + prod[k];
        __syncthreads();
    }
    if (tid == 0) epilogue<T>(a, row, a.epi == EPI_SPMV ? sum : (AT)rhs[row] - sum);
}

// ---------------------------------------------------------------------------
// vector-CSR: K lanes per row (K divides 64).
// ---------------------------------------------------------------------------
template <class T, int BLOCK, int K>
__global__ void __launch_bounds__(BLOCK) k_sweep_vector(SweepArgs a)
{
    using VT = typename T::VT;
    using XT = typename T::XT;
    using RT = typename T::RT;
    using AT = typename T::AT;
    static_assert(64 % K == 0 && BLOCK % 64 == 0, "geometry");
    const int blk = xcd_slab_block((int)blockIdx.x, (int)gridDim.x);
    const int lane = (int)threadIdx.x & (K - 1);
    const int row = (blk * BLOCK + (int)threadIdx.x) / K;
    const bool live = row < a.n;
    const VT *__restrict__ val = (const VT *)a.val;
    const int32_t *__restrict__ col = a.col;
    const XT *__restrict__ xin = (const XT *)a.xin;
    AT sum = (AT)0;
    if (live) {
        const int rs = a.rp[row], re = a.rp[row + 1];
        for (int e = rs + lane; e < re; e += K) sum = sum + (AT)val[e] * (AT)xin[col[e]];
    }
#pragma unroll
    for (int off = K / 2; off > 0; off >>= 1) sum = sum + __shfl_xor(sum, off, K);
    if (live && lane == 0) {
        if (a.dshift) sum = sum + (AT)((a.dshift[row] - 1.0) * (double)xin[row]);
        const AT t = a.epi == EPI_SPMV ? sum : (AT)((const RT *)a.rhs)[row] - sum;
        epilogue<T>(a, row, t);
    }
}

template <class T, int BLOCK, int RPB, int CAP>
hipError_t go_stream(const SweepGeom &g, const SweepArgs &a, hipStream_t s)
{
    const int grid = (a.n + RPB - 1) / RPB;
    if (g.slot16 && g.lw > 0 && g.lw <= WIN_MAX_SLOTS)
        hipLaunchKernelGGL((k_sweep_win<T, BLOCK, RPB, CAP>), dim3(grid), dim3(BLOCK),
                           (size_t)g.lw * sizeof(typename T::XT), s, a, g.slot16, g.wo, g.lw);
    else if (g.off16)
        hipLaunchKernelGGL((k_sweep_stream16<T, BLOCK, RPB, CAP>), dim3(grid), dim3(BLOCK), 0, s, a, g.off16, g.shift);
    else
        hipLaunchKernelGGL((k_sweep_stream<T, BLOCK, RPB, CAP>), dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <class T, int K>
hipError_t go_vector(const SweepArgs &a, hipStream_t s)
{
    constexpr int BLOCK = 256;
    const long long rows_per_block = BLOCK / K;
    const int grid = (int)((a.n + rows_per_block - 1) / rows_per_block);
    hipLaunchKernelGGL((k_sweep_vector<T, BLOCK, K>), dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <class T>
hipError_t dispatch(const SweepGeom &g, const SweepArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    if (g.kind == SweepKernel::BLOCKED) {
        if (g.nblk <= 0 || !g.blk) return hipErrorInvalidValue;
        const int2 *blk = (const int2 *)g.blk;
        switch (g.cap) {
        case 1024: hipLaunchKernelGGL((k_sweep_rb<T, 256, 1024, RB_RMAX>), dim3(g.nblk), dim3(256), 0, s, a, blk); break;
        case 2048: hipLaunchKernelGGL((k_sweep_rb<T, 256, 2048, RB_RMAX>), dim3(g.nblk), dim3(256), 0, s, a, blk); break;
        case 4096: hipLaunchKernelGGL((k_sweep_rb<T, 256, 4096, RB_RMAX>), dim3(g.nblk), dim3(256), 0, s, a, blk); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (g.kind == SweepKernel::SLICED) {
        constexpr int WPB = 4, UNR = 2;
        if (g.sl.nslice <= 0) return hipErrorInvalidValue;
        const dim3 grid((g.sl.nslice + WPB - 1) / WPB), block(64 * WPB);
        if (g.sl.code == 16) {
            if (g.sl.ndiag < 1 || g.sl.ndiag > DIAG_MAX || a.n < 2 || (int64_t)g.sl.nslice * 128 < a.n || a.dshift)
                return hipErrorInvalidValue;
            return go_diag<T>(g, a, s);
        }
        if (g.sl.code == 8) {
            if (g.sl.npat < 1 || g.sl.kp < 4 || (g.sl.kp & 3) || g.sl.npat * g.sl.kp > PAT_MAX_ENTRIES ||
                g.sl.gmax > 8 || g.sl.kp != 4 * g.sl.gmax)
                return hipErrorInvalidValue;
            // windows load two iterate entries per lane at even offsets: with
            // an iterate aligned to that width (the library's own vectors
            // are; a caller's may not be) every load is aligned to its size
            if (g.sl.nwin > 0 && ((uintptr_t)a.xin & (2 * sizeof(typename T::XT) - 1)) == 0) {
                if (g.sl.nwin > PAT_WIN_MAX || !g.sl.ltab || !g.sl.wflag || g.sl.wspan < 128 || (g.sl.wst[0] & 1) ||
                    g.sl.kl < g.sl.kp || (g.sl.kl & 7))
                    return hipErrorInvalidValue;
                // eight waves per workgroup (1 % faster) while two such
                // workgroups' FP64 windows fit in a CU's 160 KB of LDS
                return g.sl.nwin <= 9 ? go_pat_win<T, 8>(g, a, s) : go_pat_win<T, WPB>(g, a, s);
            }
            return go_pat<T, WPB>(g, a, s);
        }
        if (g.slice_prefetch && g.sl.code == 1 && g.sl.gmax >= 1 && g.sl.gmax <= 8) {
            switch (g.sl.gmax) {
            case 1: hipLaunchKernelGGL((k_sweep_sliced_pf<T, WPB, 1>), grid, block, 0, s, a, g.sl); break;
            case 2: hipLaunchKernelGGL((k_sweep_sliced_pf<T, WPB, 2>), grid, block, 0, s, a, g.sl); break;
            case 3: hipLaunchKernelGGL((k_sweep_sliced_pf<T, WPB, 3>), grid, block, 0, s, a, g.sl); break;
            case 4: hipLaunchKernelGGL((k_sweep_sliced_pf<T, WPB, 4>), grid, block, 0, s, a, g.sl); break;
            case 5: hipLaunchKernelGGL((k_sweep_sliced_pf<T, WPB, 5>), grid, block, 0, s, a, g.sl); break;
            case 6: hipLaunchKernelGGL((k_sweep_sliced_pf<T, WPB, 6>), grid, block, 0, s, a, g.sl); break;
            case 7: hipLaunchKernelGGL((k_sweep_sliced_pf<T, WPB, 7>), grid, block, 0, s, a, g.sl); break;
            default: hipLaunchKernelGGL((k_sweep_sliced_pf<T, WPB, 8>), grid, block, 0, s, a, g.sl); break;
            }
            return hipGetLastError();
        }
        switch (g.sl.code) {
        case 1: hipLaunchKernelGGL((k_sweep_sliced<T, 1, WPB, UNR>), grid, block, 0, s, a, g.sl); break;
        case 2: hipLaunchKernelGGL((k_sweep_sliced<T, 2, WPB, UNR>), grid, block, 0, s, a, g.sl); break;
        case 4: hipLaunchKernelGGL((k_sweep_sliced<T, 4, WPB, UNR>), grid, block, 0, s, a, g.sl); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (g.kind == SweepKernel::STREAM) {
        switch (g.rows_per_block) {
        case 256: return go_stream<T, 256, 256, 1024>(g, a, s);
        case 128: return go_stream<T, 256, 128, 1024>(g, a, s);
        case 64: return go_stream<T, 256, 64, 2048>(g, a, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (g.lanes) {
    case 4: return go_vector<T, 4>(a, s);
    case 8: return go_vector<T, 8>(a, s);
    case 16: return go_vector<T, 16>(a, s);
    case 32: return go_vector<T, 32>(a, s);
    case 64: return go_vector<T, 64>(a, s);
    default: return hipErrorInvalidValue;
    }
}

const char *kname16(Prec p)
{
    static const char *names[5] = {"sweep_stream16_f64", "sweep_stream16_mixres", "sweep_stream16_mixL",
                                   "sweep_stream16_mixU", "sweep_stream16_mixL1"};
    return names[(int)p];
}

const char *kname_win(Prec p)
{
    static const char *names[5] = {"sweep_win_f64", "sweep_win_mixres", "sweep_win_mixL", "sweep_win_mixU",
                                   "sweep_win_mixL1"};
    return names[(int)p];
}

const char *kname(Prec p, SweepKernel k)
{
    static const char *names[4][5] = {
        {"sweep_stream_f64", "sweep_stream_mixres", "sweep_stream_mixL", "sweep_stream_mixU", "sweep_stream_mixL1"},
        {"sweep_vector_f64", "sweep_vector_mixres", "sweep_vector_mixL", "sweep_vector_mixU", "sweep_vector_mixL1"},
        {"sweep_rb_f64", "sweep_rb_mixres", "sweep_rb_mixL", "sweep_rb_mixU", "sweep_rb_mixL1"},
        {"sweep_sliced_f64", "sweep_sliced_mixres", "sweep_sliced_mixL", "sweep_sliced_mixU", "sweep_sliced_mixL1"}};
    return names[(int)k][(int)p];
}

} // namespace

// SILU_SWEEP_GEOM (tuning override, read per call): "blocked:CAP",
// "stream:RPB", "stream16:RPB", "win:RPB", "sliced:CODE" or "vector:LANES".
static bool geom_override(SweepGeom &g)
{
    const char *e = getenv("SILU_SWEEP_GEOM");
    if (!e || !*e) return false;
    int v = 0;
    if (sscanf(e, "blocked:%d", &v) == 1 && (v == 1024 || v == 2048 || v == 4096)) {
        g.kind = SweepKernel::BLOCKED;
        g.cap = v;
        return true;
    }
    if (sscanf(e, "stream16:%d", &v) == 1 && (v == 64 || v == 128 || v == 256)) {
        g.kind = SweepKernel::STREAM;
        g.rows_per_block = v;
        g.allow16 = true;
        return true;
    }
    if (sscanf(e, "win:%d", &v) == 1 && (v == 64 || v == 128 || v == 256)) {
        g.kind = SweepKernel::STREAM;
        g.rows_per_block = v;
        g.allow16 = true;
        g.allow_win = true;
        g.prefer_win = true;
        return true;
    }
    if (sscanf(e, "stream:%d", &v) == 1 && (v == 64 || v == 128 || v == 256)) {
        g.kind = SweepKernel::STREAM;
        g.rows_per_block = v;
        return true;
    }
    if (sscanf(e, "sliced:%d", &v) == 1 && (v == 1 || v == 2 || v == 4)) {
        g.kind = SweepKernel::SLICED;
        g.rows_per_block = 64;
        g.slice_code_min = v;
        return true;
    }
    if (sscanf(e, "vector:%d", &v) == 1 && v >= 4 && v <= 64 && (v & (v - 1)) == 0) {
        g.kind = SweepKernel::VECTOR;
        g.lanes = v;
        return true;
    }
    return false;
}

SweepGeom pick_geom(int64_t n, int64_t nnz, int flags)
{
    const double mean = n > 0 ? (double)nnz / (double)n : 0.0;
    SweepGeom g;
    g.rows_per_block = 0;
    g.lanes = 1;
    g.cap = RB_CAP;
    if (geom_override(g)) return g;
    if (flags & 0x400) { // SILU_KERNEL_BLOCKED
        g.kind = SweepKernel::BLOCKED;
        return g; // the caller attaches the row-block partition
    }
    if (flags & 0x200) { // SILU_KERNEL_VECTOR
        g.kind = SweepKernel::VECTOR;
        g.lanes = mean <= 6.0 ? 4 : (mean <= 12.0 ? 8 : (mean <= 24.0 ? 16 : (mean <= 48.0 ? 32 : 64)));
        return g;
    }
    if (!(flags & 0x100)) { // default: sliced-ELL (the caller attaches the sliced copy, else falls back)
        g.kind = SweepKernel::SLICED;
        g.rows_per_block = (mean <= 8.0 || mean > 24.0 || (flags & 0x2)) ? 256 : (mean <= 16.0 ? 128 : 64);
        g.allow16 = !(flags & 0x1000);
        g.allow_win = !(flags & 0x1000) && !(flags & 0x2000);
        g.prefer_win = false;
        // SILU_INDEX32, SILU_CODE16, SILU_CODE8, SILU_ROWPAT; by default diagonal slices, else the
        // row-pattern table where it fits
        g.slice_code_min = (flags & 0x1000) ? 4
                                            : ((flags & 0x8000) ? 2 : ((flags & 0x100000) ? 1 : ((flags & 0x400000) ? 0 : -1)));
        g.slice_prefetch = !(flags & 0x80000);                                // SILU_SLICED_LOOP
        return g;
    }
    // SILU_KERNEL_STREAM: CSR-stream; short rows fill a
    // workgroup with 256 of them, long rows take 64 so one LDS chunk holds them
    // FP64 factor rows of 9-24 entries stream best 64-128 rows at a time;
    // short rows, long rows and the FP32-value sweeps (SILU_MIXED) with 256
    g.kind = SweepKernel::STREAM;
    g.rows_per_block = (mean <= 8.0 || mean > 24.0 || (flags & 0x2)) ? 256 : (mean <= 16.0 ? 128 : 64);
    g.allow16 = !(flags & 0x1000); // SILU_INDEX32 keeps 32-bit column indices
    // the LDS window where 16-bit offsets do not fit (wide stencils), or when
    // asked for (SILU_WINDOW); SILU_NO_WINDOW: 16-bit offsets at most
    g.allow_win = !(flags & 0x1000) && !(flags & 0x2000);
    g.prefer_win = g.allow_win && (flags & 0x4000);
    return g;
}

hipError_t launch_sweep_batch(Prec p, const SweepArgs *d_ops, const int32_t *d_first, int nops, int total,
                              hipStream_t s)
{
    if (nops <= 0 || total <= 0) return hipSuccess;
    switch (p) {
    case Prec::F64: hipLaunchKernelGGL((k_sweep_batch<TF64>), dim3(total), dim3(256), 0, s, d_ops, d_first, nops); break;
    case Prec::MIX_RES:
        hipLaunchKernelGGL((k_sweep_batch<TMixRes>), dim3(total), dim3(256), 0, s, d_ops, d_first, nops);
        break;
    case Prec::MIX_L1:
        hipLaunchKernelGGL((k_sweep_batch<TMixL1>), dim3(total), dim3(256), 0, s, d_ops, d_first, nops);
        break;
    case Prec::MIX_L: hipLaunchKernelGGL((k_sweep_batch<TMixL>), dim3(total), dim3(256), 0, s, d_ops, d_first, nops); break;
    case Prec::MIX_U: hipLaunchKernelGGL((k_sweep_batch<TMixU>), dim3(total), dim3(256), 0, s, d_ops, d_first, nops); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep_batch_args(Prec p, const BatchArgs &b, hipStream_t s)
{
    if (b.nops <= 0 || b.nops > BATCH_ARG_OPS || b.first[b.nops] <= 0) return hipSuccess;
    switch (p) {
    case Prec::F64: return go_batch_args_sized<TF64>(b, s);
    case Prec::MIX_RES: return go_batch_args_sized<TMixRes>(b, s);
    case Prec::MIX_L1: return go_batch_args_sized<TMixL1>(b, s);
    case Prec::MIX_L: return go_batch_args_sized<TMixL>(b, s);
    case Prec::MIX_U: return go_batch_args_sized<TMixU>(b, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve_check(const SolveCheckArgs &a, hipStream_t s)
{
    if (a.count <= 0 || a.count > SOLVE_CHECKS_PER_LAUNCH) return a.count == 0 ? hipSuccess : hipErrorInvalidValue;
    hipLaunchKernelGGL(k_solve_check, dim3(a.count), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sweep_persist(const PersistPlan &p, int grid, hipStream_t s)
{
    if (p.nops <= 0 || grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_sweep_persist<TF64, 256, PERSIST_RPB, 1024>), dim3(grid), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_sweep(Prec p, const SweepGeom &g, const SweepArgs &a, hipStream_t s, const char **name)
{
    if (name) {
        if (g.kind == SweepKernel::STREAM && g.slot16 && g.lw > 0)
            *name = kname_win(p);
        else
            *name = (g.kind == SweepKernel::STREAM && g.off16) ? kname16(p) : kname(p, g.kind);
    }
    switch (p) {
    case Prec::F64: return dispatch<TF64>(g, a, s);
    case Prec::MIX_RES: return dispatch<TMixRes>(g, a, s);
    case Prec::MIX_L: return dispatch<TMixL>(g, a, s);
    case Prec::MIX_U: return dispatch<TMixU>(g, a, s);
    case Prec::MIX_L1: return dispatch<TMixL1>(g, a, s);
    }
    return hipErrorInvalidValue;
}

} // namespace silu
