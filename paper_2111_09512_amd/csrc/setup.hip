// Set-up and auxiliary kernels: row scaling of the U factor, FP32 copies,
// the level-scheduled substitution step, small vector kernels and a
// streaming copy for bandwidth calibration.
#include "internal.h"

#pragma clang fp contract(off)

namespace silu {
namespace {

// flags[0]: first row whose U row does not start with its diagonal (or has
//           an entry left of it); flags[1]: first row with a zero or
//           non-finite pivot.  Both start at INT32_MAX.
__global__ void __launch_bounds__(256) k_scale_rows(int n, const int32_t *__restrict__ Urp,
                                                    const int32_t *__restrict__ Ucol,
                                                    const double *__restrict__ Uval, int32_t *__restrict__ Usrp,
                                                    int32_t *__restrict__ Uscol, double *__restrict__ Usval,
                                                    double *__restrict__ d, double *__restrict__ dinv,
                                                    float *__restrict__ Us32, int noscale, int32_t us_nnz,
                                                    int32_t *flags)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int p0 = Urp[i], p1 = Urp[i + 1];
    if (i == n - 1) Usrp[n] = p1 - n;
    Usrp[i] = p0 - i;
    if (p1 <= p0 || Ucol[p0] != i) {
        atomicMin(&flags[0], i);
        return;
    }
    const double u = Uval[p0];
    if (!(u != 0.0) || !isfinite(u)) atomicMin(&flags[1], i);
    d[i] = u;
    dinv[i] = 1.0 / u;
    // rows before i each lost exactly their diagonal; a malformed U (flagged
    // above by the row that lacks it) could shift o, so every store is bounded
    int o = p0 - i;
    for (int p = p0 + 1; p < p1; ++p, ++o) {
        const int j = Ucol[p];
        if (j <= i) atomicMin(&flags[0], i);
        if (o < 0 || o >= us_nnz) {
            atomicMin(&flags[0], i);
            continue;
        }
        const double v = noscale ? Uval[p] : Uval[p] / u;
        Uscol[o] = j;
        Usval[o] = v;
        if (Us32) Us32[o] = (float)v;
    }
}

__global__ void __launch_bounds__(256) k_to_f32(int64_t n, const double *__restrict__ src, float *__restrict__ dst)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = (float)src[i];
}

template <typename ST>
__global__ void __launch_bounds__(256) k_axpy(int n, const ST *__restrict__ s, const double *__restrict__ dcol,
                                              double *__restrict__ x)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) x[i] = x[i] + (dcol ? dcol[i] : 1.0) * (double)s[i];
}

// ---- row/column scaling of U (Section 5.1, eq. rowcolScale) ---------------
// Ruiz steps in the max norm: with a_ij = (|u_ij| d_r,i) d_c,j, the row maxima
// and column maxima of one step are taken from the same a, then
// d_r,i *= 1/sqrt(row max), d_c,j *= 1/sqrt(column max).  Maxima are exact,
// so the order in which rows meet a column does not change the result.
__global__ void __launch_bounds__(256) k_fill2(int n, double *__restrict__ a, double va, double *__restrict__ b,
                                               double vb)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    a[i] = va;
    if (b) b[i] = vb;
}

// One lane per row; the column maxima are combined with 64-bit atomic max on
// the bit patterns, which order like the values for non-negative doubles.  A
// NaN never raises a maximum (like a strict > comparison), and a column index
// outside [0, n) flags the row and is skipped.
__global__ void __launch_bounds__(256) k_ruiz_max(int n, const int32_t *__restrict__ Urp,
                                                  const int32_t *__restrict__ Ucol, const double *__restrict__ Uval,
                                                  const double *__restrict__ dr, const double *__restrict__ dc,
                                                  double *__restrict__ rmax, unsigned long long *cmax, int32_t *flags)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const double ri = dr[i];
    double rm = 0.0;
    for (int p = Urp[i]; p < Urp[i + 1]; ++p) {
        const int j = Ucol[p];
        if ((unsigned)j >= (unsigned)n) {
            atomicMin(&flags[0], i);
            continue;
        }
        const double v = (fabs(Uval[p]) * ri) * dc[j];
        if (v > rm) rm = v;
        if (v > 0.0) atomicMax(&cmax[j], (unsigned long long)__double_as_longlong(v));
    }
    rmax[i] = rm;
}

__global__ void __launch_bounds__(256) k_ruiz_scale(int n, double *__restrict__ dr, double *__restrict__ dc,
                                                    const double *__restrict__ rmax,
                                                    const unsigned long long *__restrict__ cmax)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    dr[i] = dr[i] * (1.0 / sqrt(rmax[i]));
    dc[i] = dc[i] * (1.0 / sqrt(__longlong_as_double((long long)cmax[i])));
}

// The unit diagonal fixes the row factor, d_r,i = 1/(u_ii d_c,i); the strictly
// upper values are u^_ij = (u_ij d_r,i) d_c,j.  Us row pointers and columns
// were written by k_scale_rows; stores are bounded like there.
__global__ void __launch_bounds__(256) k_rowcol_finish(int n, const int32_t *__restrict__ Urp,
                                                       const int32_t *__restrict__ Ucol,
                                                       const double *__restrict__ Uval, const double *__restrict__ dc,
                                                       double *__restrict__ dr, double *__restrict__ Usval,
                                                       float *__restrict__ Us32, int32_t us_nnz)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int p0 = Urp[i], p1 = Urp[i + 1];
    if (p1 <= p0) return;
    const double di = 1.0 / (Uval[p0] * dc[i]);
    dr[i] = di;
    int o = p0 - i;
    for (int p = p0 + 1; p < p1; ++p, ++o) {
        const int j = Ucol[p];
        if (o < 0 || o >= us_nnz || (unsigned)j >= (unsigned)n) continue;
        const double v = (Uval[p] * di) * dc[j];
        Usval[o] = v;
        if (Us32) Us32[o] = (float)v;
    }
}

__global__ void k_init_flags(int32_t *flags, int count, int32_t value)
{
    const int i = (int)threadIdx.x;
    if (i < count) flags[i] = value;
}

__global__ void __launch_bounds__(256) k_finite_check(int n, const double *__restrict__ x, int32_t *flags)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n && !isfinite(x[i])) atomicMin(&flags[2], i);
}

// One level of a level-scheduled substitution with K lanes per row: every
// row of the level depends only on rows of earlier levels.  Lanes take the
// row's entries round-robin, so the loads of a row are in flight together;
// the partial sums are combined with cross-lane shuffles (the stored
// diagonal, held by one lane, is combined exactly as a sum with zeros).
template <int UNIT, int K>
__global__ void __launch_bounds__(256) k_level_vec(LevelArgs a, int start, int count)
{
    const int slot = (int)((blockIdx.x * blockDim.x + threadIdx.x) / K);
    const int lane = (int)threadIdx.x & (K - 1);
    const bool live = slot < count;
    int i = 0;
    double sum = 0.0, dii = 0.0;
    if (live) {
        i = a.perm[start + slot];
        const int p1 = a.rp[i + 1];
#pragma unroll 2
        for (int p = a.rp[i] + lane; p < p1; p += K) {
            const int j = a.col[p];
            const double v = a.val[p];
            if (j == i)
                dii = v;
            else
                sum = sum + v * a.out[j];
        }
    }
#pragma unroll
    for (int off = K / 2; off > 0; off >>= 1) {
        sum = sum + __shfl_xor(sum, off, K);
        if (!UNIT) dii = dii + __shfl_xor(dii, off, K);
    }
    if (live && lane == 0) {
        double v = a.rhs[i] - sum;
        if (!UNIT) v = v / dii;
        a.out[i] = v;
        if (a.s_out) a.s_out[i] = a.dinv[i] * v;
        if (a.xupd) a.xupd[i] = a.xupd[i] + (a.dcol ? a.dcol[i] : 1.0) * v;
    }
}

// One level, one lane per row, the row summed in ascending column order like
// a sequential substitution (bit-identical to it; used for short rows).
template <int UNIT>
__global__ void __launch_bounds__(256) k_level(LevelArgs a, int start, int count)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= count) return;
    const int i = a.perm[start + t];
    const int p0 = a.rp[i], p1 = a.rp[i + 1];
    double sum = 0.0, dii = 1.0;
    for (int p = p0; p < p1; ++p) {
        const int j = a.col[p];
        const double v = a.val[p];
        if (j == i) {
            dii = v;
            continue;
        }
        sum = sum + v * a.out[j];
    }
    double v = a.rhs[i] - sum;
    if (!UNIT) v = v / dii;
    a.out[i] = v;
    if (a.s_out) a.s_out[i] = a.dinv[i] * v;
    if (a.xupd) a.xupd[i] = a.xupd[i] + (a.dcol ? a.dcol[i] : 1.0) * v;
}

__global__ void __launch_bounds__(256) k_scale_copy(int n, const double *__restrict__ rhs,
                                                    const double *__restrict__ dinv, double *__restrict__ out)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) out[i] = dinv ? dinv[i] * rhs[i] : rhs[i];
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Streaming copy: each lane moves four 16-byte vectors per iteration, all four
// loads issued before the stores; non-temporal hints keep the stream out of
// the caches.
__global__ void __launch_bounds__(256) k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, size_t n16)
{
    const size_t bd = blockDim.x;
    const size_t stride = (size_t)gridDim.x * bd * 4;
    size_t i = (size_t)blockIdx.x * bd * 4 + threadIdx.x;
    for (; i + 3 * bd < n16; i += stride) {
        const u32x4 a = __builtin_nontemporal_load(&src[i]);
        const u32x4 b = __builtin_nontemporal_load(&src[i + bd]);
        const u32x4 c = __builtin_nontemporal_load(&src[i + 2 * bd]);
        const u32x4 d = __builtin_nontemporal_load(&src[i + 3 * bd]);
        __builtin_nontemporal_store(a, &dst[i]);
        __builtin_nontemporal_store(b, &dst[i + bd]);
        __builtin_nontemporal_store(c, &dst[i + 2 * bd]);
        __builtin_nontemporal_store(d, &dst[i + 3 * bd]);
    }
    for (; i < n16; i += bd) dst[i] = src[i];
}

__global__ void __launch_bounds__(256) k_offset_range(int n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col, int rpb, int32_t *range)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int lo = INT32_MAX, hi = INT32_MIN;
    if (i < n) {
        const int r0 = (i / rpb) * rpb;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int o = col[p] - r0;
            lo = min(lo, o);
            hi = max(hi, o);
        }
    }
    // one atomic pair per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off));
        hi = max(hi, __shfl_xor(hi, off));
    }
    if ((threadIdx.x & 63) == 0 && lo <= hi) {
        atomicMin(&range[0], lo);
        atomicMax(&range[1], hi);
    }
}

// used[col - r0(block) - lo] = 1 for every entry (all writers store the same
// byte, so the races are benign).
__global__ void __launch_bounds__(256) k_mark_offsets(int n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col, int rpb, int lo,
                                                      uint8_t *__restrict__ used)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int base = (i / rpb) * rpb + lo;
    for (int p = rp[i]; p < rp[i + 1]; ++p) used[col[p] - base] = 1;
}

// code[e] = slot_of[col - r0(block) - lo]: the LDS slot that holds the entry's
// iterate value in the windowed sweep.
__global__ void __launch_bounds__(256) k_encode_slots(int n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col, int rpb, int lo,
                                                      const int32_t *__restrict__ slot_of, uint16_t *__restrict__ code)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int base = (i / rpb) * rpb + lo;
    for (int p = rp[i]; p < rp[i + 1]; ++p) code[p] = (uint16_t)slot_of[col[p] - base];
}

__global__ void __launch_bounds__(256) k_compress16(int n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col, int rpb, int shift,
                                                    uint16_t *__restrict__ off16)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int base = (i / rpb) * rpb + shift;
    for (int p = rp[i]; p < rp[i + 1]; ++p) off16[p] = (uint16_t)(col[p] - base);
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

// ---- polynomial Gauss-Seidel split: Gs = D^{-1} L, dinv = 1/diag(A) ---------
// counts[i] = entries of row i left of the diagonal; flags[0] <- the first
// row without a stored diagonal, flags[1] <- the first zero or non-finite one.
__global__ void __launch_bounds__(256) k_gs_count(int n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                                  int32_t *__restrict__ counts, int32_t *flags)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    int c = 0;
    bool has = false;
    double aii = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = col[p];
        if (j < i) ++c;
        if (j == i) {
            has = true;
            aii = val[p];
        }
    }
    counts[i] = c;
    if (!has) atomicMin(&flags[0], i);
    else if (!(aii != 0.0) || !isfinite(aii)) atomicMin(&flags[1], i);
}

// Row i of Gs: g_ij = a_ij / a_ii for j < i (one IEEE division each), at
// Gs_rp[i]..; stores bounded by gs_nnz.
__global__ void __launch_bounds__(256) k_gs_fill(int n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                                 const int32_t *__restrict__ Grp, int32_t *__restrict__ Gcol,
                                                 double *__restrict__ Gval, double *__restrict__ d,
                                                 double *__restrict__ dinv, float *__restrict__ G32, int32_t gs_nnz)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    double aii = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (col[p] == i) aii = val[p];
    d[i] = aii;
    dinv[i] = 1.0 / aii;
    int o = Grp[i];
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = col[p];
        if (j >= i) continue;
        if (o >= 0 && o < gs_nnz) {
            const double g = val[p] / aii;
            Gcol[o] = j;
            Gval[o] = g;
            if (G32) G32[o] = (float)g;
        }
        ++o;
    }
}

// ---- sliced-ELL copies (64-row slices, one wavefront per slice) ------------
// Slice s holds rows [64 s, 64 s + 64) and K4 = (its longest row rounded up
// to a multiple of 4) slots per row, in groups of four entries so that a lane
// fetches a group with wide loads: within group q (entries 4q..4q+3 of every
// row of the slice, 256 slots starting at sptr[s] + 256 q),
//   FP64 values of entries 4q + 2h + {0,1} of lane l at 128 h + 2 l + {0,1}
//   FP32 values and all codes of entry 4q + r of lane l at 4 l + r.
// sk[s] = K4, with bit 31 set when some row of the slice is empty or past the
// end (those slices run with per-row lengths).
__global__ void __launch_bounds__(256) k_slice_meta(int n, int nslice, const int32_t *__restrict__ rp,
                                                    int32_t *__restrict__ sk)
{
    const int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= nslice) return;
    int K = 0;
    bool masked = false;
    for (int r = s * 64; r < s * 64 + 64; ++r) {
        if (r >= n) {
            masked = true;
            break;
        }
        const int len = rp[r + 1] - rp[r];
        K = max(K, len);
        if (len == 0) masked = true;
    }
    sk[s] = ((K + 3) & ~3) | (masked ? (int32_t)0x80000000 : 0);
}

__device__ __forceinline__ int64_t value_slot(int64_t base, int k, int lane, int vbytes)
{
    const int q = k >> 2, r = k & 3;
    if (vbytes == 8) return base + 256 * q + 128 * (r >> 1) + 2 * lane + (r & 1);
    return base + 256 * q + 4 * lane + r;
}

// One lane per row (rows past n fill the last slice's padding).  A padded slot
// repeats the row's last column with value 0 (an empty row: its own column),
// so an unmasked sweep reads only columns the row reads anyway.  Codes: 1 =
// u8 index into the diagonal table (dmap[col - row - dlo]), 2 = u16 offset
// col - 64 s - shift, 4 = the int32 column, 8 = none (the row's pattern
// table entry gives its columns).
template <typename VT, int CODE>
__global__ void __launch_bounds__(256) k_fill_sliced(int n, int nslice, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col, const VT *__restrict__ val,
                                                     const int32_t *__restrict__ sptr, const int32_t *__restrict__ sk,
                                                     const int32_t *__restrict__ dmap, int lo, VT *__restrict__ sval,
                                                     void *__restrict__ scode)
{
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= nslice * 64) return;
    const int s = r >> 6, lane = r & 63;
    const int K4 = sk[s] & 0x7fffffff;
    const int p0 = r < n ? rp[r] : 0, len = r < n ? rp[r + 1] - p0 : 0;
    const int last = len > 0 ? col[p0 + len - 1] : min(r, n - 1);
    const int64_t base = sptr[s];
    for (int k = 0; k < K4; ++k) {
        const int c = k < len ? col[p0 + k] : last;
        sval[value_slot(base, k, lane, (int)sizeof(VT))] = k < len ? val[p0 + k] : (VT)0;
        const int64_t pc = base + 256 * (k >> 2) + 4 * lane + (k & 3);
        if (CODE == 8) continue; // row patterns: no per-slot code
        if (CODE == 1) ((uint8_t *)scode)[pc] = (uint8_t)dmap[c - min(r, n - 1) - lo];
        else if (CODE == 2) ((uint16_t *)scode)[pc] = (uint16_t)(c - s * 64 - lo);
        else ((int32_t *)scode)[pc] = c;
    }
}

// Diagonal slices: one thread per row places the row's entries (the copy
// was zeroed first, so slots of diagonals the row lacks hold 0).
template <typename VT>
__global__ void __launch_bounds__(256) k_fill_diag(int n, int u, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col, const VT *__restrict__ val,
                                                   const int32_t *__restrict__ dmap, int lo, VT *__restrict__ sval)
{
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= n) return;
    for (int e = rp[r]; e < rp[r + 1]; ++e) sval[diag_slot(r, dmap[col[e] - r - lo], u)] = val[e];
}

} // namespace

hipError_t launch_scale_rows(int n, const int32_t *Urp, const int32_t *Ucol, const double *Uval, int32_t *Usrp,
                             int32_t *Uscol, double *Usval, double *d, double *dinv, float *Us32, int noscale,
                             int32_t us_nnz, int32_t *flags, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_rows, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, Urp, Ucol, Uval, Usrp, Uscol,
                       Usval, d, dinv, Us32, noscale, us_nnz, flags);
    return hipGetLastError();
}

hipError_t launch_to_f32(int64_t n, const double *src, float *dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(blocks_for(n, 256), 65536);
    hipLaunchKernelGGL(k_to_f32, dim3(grid), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_axpy(int n, const void *s_vec, int s_is_f32, const double *dcol, double *x, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (s_is_f32)
        hipLaunchKernelGGL(k_axpy<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, (const float *)s_vec, dcol,
                           x);
    else
        hipLaunchKernelGGL(k_axpy<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, (const double *)s_vec, dcol,
                           x);
    return hipGetLastError();
}

hipError_t launch_fill(int n, double *a, double va, double *b, double vb, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill2, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, a, va, b, vb);
    return hipGetLastError();
}

hipError_t launch_ruiz_max(int n, const int32_t *Urp, const int32_t *Ucol, const double *Uval, const double *dr,
                           const double *dc, double *rmax, unsigned long long *cmax, int32_t *flags, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ruiz_max, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, Urp, Ucol, Uval, dr, dc, rmax, cmax,
                       flags);
    return hipGetLastError();
}

hipError_t launch_ruiz_scale(int n, double *dr, double *dc, const double *rmax, const unsigned long long *cmax,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ruiz_scale, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, dr, dc, rmax, cmax);
    return hipGetLastError();
}

hipError_t launch_rowcol_finish(int n, const int32_t *Urp, const int32_t *Ucol, const double *Uval,
                                const double *dc, double *dr, double *Usval, float *Us32, int32_t us_nnz,
                                hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rowcol_finish, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, Urp, Ucol, Uval, dc, dr, Usval,
                       Us32, us_nnz);
    return hipGetLastError();
}

hipError_t launch_init_flags(int32_t *flags, int count, int32_t value, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_flags, dim3(1), dim3(64), 0, s, flags, count, value);
    return hipGetLastError();
}

hipError_t launch_finite_check(int n, const double *x, int32_t *flags, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finite_check, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, flags);
    return hipGetLastError();
}

template <int UNIT, int K>
void go_level(const LevelArgs &a, int start, int count, hipStream_t s)
{
    hipLaunchKernelGGL((k_level_vec<UNIT, K>), dim3(blocks_for((int64_t)count * K, 256)), dim3(256), 0, s, a, start,
                       count);
}

hipError_t launch_level(const LevelArgs &a, int unit, int lanes, int start, int count, hipStream_t s,
                        const char **name)
{
    if (name) *name = "level_f64";
    if (count <= 0) return hipSuccess;
    switch (lanes * 2 + (unit ? 1 : 0)) {
    case 1 * 2 + 1: hipLaunchKernelGGL(k_level<1>, dim3(blocks_for(count, 256)), dim3(256), 0, s, a, start, count); break;
    case 1 * 2: hipLaunchKernelGGL(k_level<0>, dim3(blocks_for(count, 256)), dim3(256), 0, s, a, start, count); break;
    case 4 * 2 + 1: go_level<1, 4>(a, start, count, s); break;
    case 4 * 2: go_level<0, 4>(a, start, count, s); break;
    case 8 * 2 + 1: go_level<1, 8>(a, start, count, s); break;
    case 8 * 2: go_level<0, 8>(a, start, count, s); break;
    case 16 * 2 + 1: go_level<1, 16>(a, start, count, s); break;
    case 16 * 2: go_level<0, 16>(a, start, count, s); break;
    case 32 * 2 + 1: go_level<1, 32>(a, start, count, s); break;
    case 32 * 2: go_level<0, 32>(a, start, count, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_scale_copy(int n, const double *rhs, const double *dinv, double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_copy, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rhs, dinv, out);
    return hipGetLastError();
}

hipError_t launch_offset_range(int n, const int32_t *rp, const int32_t *col, int rpb, int32_t *range, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_offset_range, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, col, rpb, range);
    return hipGetLastError();
}

hipError_t launch_mark_offsets(int n, const int32_t *rp, const int32_t *col, int rpb, int lo, uint8_t *used,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark_offsets, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, col, rpb, lo, used);
    return hipGetLastError();
}

hipError_t launch_encode_slots(int n, const int32_t *rp, const int32_t *col, int rpb, int lo, const int32_t *slot_of,
                               uint16_t *code, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_encode_slots, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, col, rpb, lo, slot_of, code);
    return hipGetLastError();
}

hipError_t launch_compress16(int n, const int32_t *rp, const int32_t *col, int rpb, int shift, uint16_t *off16,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compress16, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, col, rpb, shift, off16);
    return hipGetLastError();
}

// Read-dominant stream, shaped like a sweep's traffic (about 96 % reads): each
// tile of 256 lanes reads READ_VECS 16-byte vectors per lane (all loads issued
// before they are combined, non-temporal) and writes one 8-byte word per lane,
// 8 bytes written per 192 read.  The writes matter: the same loads with no
// writes stream about 7.1 TB/s on MI355X, with these 4 % of writes about
// 6.3 TB/s (the bus turns around between reads and writes).
constexpr int READ_VECS = 12;
__global__ void __launch_bounds__(256) k_read16(const u32x4 *__restrict__ src, unsigned long long *__restrict__ out,
                                                size_t ntiles)
{
    for (size_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const size_t base = t * 256 * READ_VECS + threadIdx.x;
        u32x4 v[READ_VECS];
#pragma unroll
        for (int k = 0; k < READ_VECS; ++k) v[k] = __builtin_nontemporal_load(&src[base + (size_t)k * 256]);
        u32x4 acc = v[0];
#pragma unroll
        for (int k = 1; k < READ_VECS; ++k) acc ^= v[k];
        const unsigned long long w = ((unsigned long long)(acc.x ^ acc.z) << 32) | (acc.y ^ acc.w);
        __builtin_nontemporal_store(w, &out[t * 256 + threadIdx.x]);
    }
}

hipError_t launch_read(const void *src, size_t bytes, void *out, hipStream_t s)
{
    const size_t ntiles = bytes / (256 * READ_VECS * 16);
    if (ntiles == 0) return hipSuccess;
    // one tile per workgroup: measured faster than fewer workgroups looping over tiles
    const int grid = (int)std::min<size_t>(ntiles, (size_t)1 << 30);
    hipLaunchKernelGGL(k_read16, dim3(grid), dim3(256), 0, s, (const u32x4 *)src, (unsigned long long *)out, ntiles);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const int grid = (int)std::min<size_t>((n16 + 1023) / 1024, 256 * 16);
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, s, (const u32x4 *)src, (u32x4 *)dst, n16);
    return hipGetLastError();
}


hipError_t launch_slice_meta(int n, int nslice, const int32_t *rp, int32_t *sk, hipStream_t s)
{
    if (nslice <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slice_meta, dim3(blocks_for(nslice, 256)), dim3(256), 0, s, n, nslice, rp, sk);
    return hipGetLastError();
}

hipError_t launch_fill_diag(int n, int nslice, int u, const int32_t *rp, const int32_t *col, const void *val,
                            int val_bytes, const int32_t *dmap, int lo, void *sval, hipStream_t s)
{
    if (nslice <= 0 || u <= 0) return hipSuccess;
    const int64_t slots = (int64_t)nslice * u * 128;
    if (slots > INT32_MAX) return hipErrorInvalidValue; // the caller keeps copies below 2^31 slots
    // zeroed as doubles: slots is a multiple of 128, so FP32 copies are whole doubles too
    const hipError_t e = launch_fill((int)(slots * val_bytes / 8), (double *)sval, 0.0, nullptr, 0.0, s);
    if (e != hipSuccess) return e;
    if (val_bytes == 8)
        hipLaunchKernelGGL(k_fill_diag<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, u, rp, col,
                           (const double *)val, dmap, lo, (double *)sval);
    else
        hipLaunchKernelGGL(k_fill_diag<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, u, rp, col,
                           (const float *)val, dmap, lo, (float *)sval);
    return hipGetLastError();
}

hipError_t launch_fill_sliced(int n, int nslice, const int32_t *rp, const int32_t *col, const void *val, int val_bytes,
                              const int32_t *sptr, const int32_t *sk, int code, const int32_t *dmap, int lo,
                              void *sval, void *scode, hipStream_t s)
{
    if (nslice <= 0) return hipSuccess;
    const dim3 g(blocks_for((int64_t)nslice * 64, 256)), b(256);
#define SILU_FILL(VT, C)                                                                                              \
    hipLaunchKernelGGL((k_fill_sliced<VT, C>), g, b, 0, s, n, nslice, rp, col, (const VT *)val, sptr, sk, dmap, lo,     \
                       (VT *)sval, scode)
    if (val_bytes == 8) {
        if (code == 8) SILU_FILL(double, 8);
        else if (code == 1) SILU_FILL(double, 1);
        else if (code == 2) SILU_FILL(double, 2);
        else SILU_FILL(double, 4);
    } else {
        if (code == 8) SILU_FILL(float, 8);
        else if (code == 1) SILU_FILL(float, 1);
        else if (code == 2) SILU_FILL(float, 2);
        else SILU_FILL(float, 4);
    }
#undef SILU_FILL
    return hipGetLastError();
}


hipError_t launch_gs_count(int n, const int32_t *rp, const int32_t *col, const double *val, int32_t *counts,
                           int32_t *flags, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gs_count, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, col, val, counts, flags);
    return hipGetLastError();
}

hipError_t launch_gs_fill(int n, const int32_t *rp, const int32_t *col, const double *val, const int32_t *Grp,
                          int32_t *Gcol, double *Gval, double *d, double *dinv, float *G32, int32_t gs_nnz,
                          hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gs_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, col, val, Grp, Gcol, Gval, d, dinv,
                       G32, gs_nnz);
    return hipGetLastError();
}

} // namespace silu
