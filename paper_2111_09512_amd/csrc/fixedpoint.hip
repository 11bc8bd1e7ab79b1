// ILU(0) on the device by synchronous fixed-point sweeps (the fixed-point ILU
// of Chow and Patel, which Section 7 names for computing the factorization on
// GPUs).  For every (i,j) in the pattern S of A:
//   u_ij = a_ij - sum_{k < i} l_ik u_kj            (j >= i)
//   l_ij = (a_ij - sum_{k < j} l_ik u_kj) / u_jj    (j <  i)
// A sweep evaluates every equation from the previous sweep's values, one lane
// per entry; the products are subtracted from a_ij in ascending k (the order
// of row-wise elimination), so a sweep's values do not depend on the launch
// shape and the standstill is the row-wise ILU(0) bit for bit.  L and U live
// in one value array aligned with A's entries until they are split.
#include "internal.h"

#pragma clang fp contract(off)

namespace silu {
namespace {

__device__ __forceinline__ int find_col(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int row, int c)
{
    int lo = rp[row], hi = rp[row + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = col[mid];
        if (v == c) return mid;
        if (v < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// dpos[i] = the entry of a_ii; row_of[p] = the row of entry p.  A row without
// its diagonal lowers flags[0] to its index.
__global__ void __launch_bounds__(256) k_fp_index(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                  int32_t *__restrict__ dpos, int32_t *__restrict__ row_of,
                                                  int32_t *flags)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int d = find_col(rp, col, i, i);
    dpos[i] = d;
    if (d < 0) atomicMin(&flags[0], i);
    for (int p = rp[i]; p < rp[i + 1]; ++p) row_of[p] = i;
}

// The initial guess u_ij = a_ij, l_ij = a_ij / a_jj.
__global__ void __launch_bounds__(256) k_fp_init(int64_t nnz, const int32_t *__restrict__ col,
                                                 const double *__restrict__ val, const int32_t *__restrict__ dpos,
                                                 const int32_t *__restrict__ row_of, double *__restrict__ LU)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int i = row_of[p], j = col[p];
    LU[p] = j < i ? val[p] / val[dpos[j]] : val[p];
}

// One synchronous sweep: nw from old.  flags[1] is set to 1 when any value
// changed.
__global__ void __launch_bounds__(256) k_fp_sweep(int64_t nnz, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                                  const int32_t *__restrict__ dpos, const int32_t *__restrict__ row_of,
                                                  const double *__restrict__ old, double *__restrict__ nw,
                                                  int32_t *flags)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int i = row_of[p], j = col[p];
    const int kmax = j < i ? j : i;
    double s = val[p];
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
        const int k = col[q];
        if (k >= kmax) break;
        const int pk = find_col(rp, col, k, j);
        if (pk >= 0) s = s - old[q] * old[pk];
    }
    const double v = j < i ? s / old[dpos[j]] : s;
    nw[p] = v;
    if (v != old[p]) atomicOr(&flags[1], 1);
}

// Split the combined values into Ls (strict lower) and U (upper, diagonal
// first): row i's lower entries go to Lrp[i].., its upper ones to Urp[i]...
__global__ void __launch_bounds__(256) k_fp_split(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                  const double *__restrict__ LU, const int32_t *__restrict__ Lrp,
                                                  int32_t *__restrict__ Lcol, double *__restrict__ Lval,
                                                  const int32_t *__restrict__ Urp, int32_t *__restrict__ Ucol,
                                                  double *__restrict__ Uval, int64_t l_nnz, int64_t u_nnz)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    int64_t ol = Lrp[i], ou = Urp[i];
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = col[p];
        if (j < i) {
            if (ol < l_nnz) {
                Lcol[ol] = j;
                Lval[ol] = LU[p];
            }
            ++ol;
        } else {
            if (ou < u_nnz) {
                Ucol[ou] = j;
                Uval[ou] = LU[p];
            }
            ++ou;
        }
    }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

} // namespace

hipError_t launch_fp_index(int n, const int32_t *rp, const int32_t *col, int32_t *dpos, int32_t *row_of,
                           int32_t *flags, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fp_index, dim3(blocks(n)), dim3(256), 0, s, n, rp, col, dpos, row_of, flags);
    return hipGetLastError();
}

hipError_t launch_fp_init(int64_t nnz, const int32_t *col, const double *val, const int32_t *dpos,
                          const int32_t *row_of, double *LU, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fp_init, dim3(blocks(nnz)), dim3(256), 0, s, nnz, col, val, dpos, row_of, LU);
    return hipGetLastError();
}

hipError_t launch_fp_sweep(int64_t nnz, const int32_t *rp, const int32_t *col, const double *val, const int32_t *dpos,
                           const int32_t *row_of, const double *old, double *nw, int32_t *flags, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fp_sweep, dim3(blocks(nnz)), dim3(256), 0, s, nnz, rp, col, val, dpos, row_of, old, nw,
                       flags);
    return hipGetLastError();
}

hipError_t launch_fp_split(int n, const int32_t *rp, const int32_t *col, const double *LU, const int32_t *Lrp,
                           int32_t *Lcol, double *Lval, const int32_t *Urp, int32_t *Ucol, double *Uval, int64_t l_nnz,
                           int64_t u_nnz, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fp_split, dim3(blocks(n)), dim3(256), 0, s, n, rp, col, LU, Lrp, Lcol, Lval, Urp, Ucol, Uval,
                       l_nnz, u_nnz);
    return hipGetLastError();
}

} // namespace silu
