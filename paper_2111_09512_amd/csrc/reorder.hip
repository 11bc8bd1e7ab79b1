// Locality relabeling for the sweeps (SILU_REORDER).
//
// A Richardson sweep y_k = rhs - N y_{k-1} updates every row from the
// previous iterate at once, so the rows and columns of N, A and the vectors
// may be relabeled by any permutation Q (N' = Q N Q^T) without changing what
// is computed; keeping every row's entries in their original storage order
// keeps each row's sum bit for bit.  The relabeling places strongly coupled
// rows next to each other, so the iterate gathers of neighbouring rows share
// cache lines and stay in L2.  Order: reverse Cuthill-McKee on the graph of
// strong couplings (|a_ij| >= theta * max_{k != i} |a_ik|, the strength of
// connection of algebraic multigrid, Section 3), which ignores weak
// long-range couplings that would otherwise collapse the BFS levels; the
// order is computed on the host (order.cpp).
#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/scaled_ilu.h"
#include "internal.h"

namespace silu {
namespace {

template <class VT>
__global__ void __launch_bounds__(256) k_relabel(int n, const int32_t *__restrict__ order,
                                                 const int32_t *__restrict__ pos, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col, const VT *__restrict__ val,
                                                 const int32_t *__restrict__ rp2, int32_t *__restrict__ col2,
                                                 VT *__restrict__ val2)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const int i = order[k];
    const int e0 = rp[i], len = rp[i + 1] - e0, d0 = rp2[k];
    for (int t = 0; t < len; ++t) {
        if (col2) col2[d0 + t] = pos[col[e0 + t]];
        val2[d0 + t] = val[e0 + t];
    }
}

__global__ void __launch_bounds__(256) k_gather(int n, const int32_t *__restrict__ order,
                                                const double *__restrict__ src, double *__restrict__ dst)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < n) dst[k] = src[order[k]];
}

// Vectors into the relabeled order: b2[pos[i]] = b[i] and, when x is given,
// x2[pos[i]] = x[i] (unit-stride reads, scattered writes, one pass for both).
__global__ void __launch_bounds__(256) k_permute_in(int n, const int32_t *__restrict__ pos,
                                                    const double *__restrict__ b, const double *__restrict__ x,
                                                    double *__restrict__ b2, double *__restrict__ x2)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int k = pos[i];
    b2[k] = b[i];
    if (x) x2[k] = x[i];
}

__global__ void __launch_bounds__(256) k_scatter(int n, const int32_t *__restrict__ order,
                                                 const double *__restrict__ src, double *__restrict__ dst)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < n) dst[order[k]] = src[k];
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

} // namespace

hipError_t launch_relabel(int n, const int32_t *order, const int32_t *pos, const int32_t *rp, const int32_t *col,
                          const void *val, int val_bytes, const int32_t *rp2, int32_t *col2, void *val2,
                          hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (val_bytes == 8)
        hipLaunchKernelGGL(k_relabel<double>, dim3(blocks(n)), dim3(256), 0, s, n, order, pos, rp, col,
                           (const double *)val, rp2, col2, (double *)val2);
    else
        hipLaunchKernelGGL(k_relabel<float>, dim3(blocks(n)), dim3(256), 0, s, n, order, pos, rp, col,
                           (const float *)val, rp2, col2, (float *)val2);
    return hipGetLastError();
}

hipError_t launch_gather(int n, const int32_t *order, const double *src, double *dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(blocks(n)), dim3(256), 0, s, n, order, src, dst);
    return hipGetLastError();
}

hipError_t launch_permute_in(int n, const int32_t *pos, const double *b, const double *x, double *b2, double *x2,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_in, dim3(blocks(n)), dim3(256), 0, s, n, pos, b, x, b2, x2);
    return hipGetLastError();
}

hipError_t launch_scatter(int n, const int32_t *order, const double *src, double *dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(blocks(n)), dim3(256), 0, s, n, order, src, dst);
    return hipGetLastError();
}

} // namespace silu
