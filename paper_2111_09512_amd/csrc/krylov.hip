// Vector kernels of the Krylov solver around the smoother (FGMRES with
// modified Gram-Schmidt): deterministic dot products, and the updates of the
// Arnoldi step whose scalars stay on the device.
//
// Dot products are two-stage and always reduce in the same order: stage one
// gives each of DOT_BLOCKS workgroups a fixed contiguous chunk, each lane adds
// its strided elements in index order and the workgroup combines its lanes by
// a fixed tree; stage two adds the partial sums the same way.  The result is
// reproducible run to run (it is not the sequential sum of the definition;
// the difference is rounding).
#include "internal.h"

#pragma clang fp contract(off)

namespace silu {
namespace {

constexpr int DOT_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double *lds)
{
    const int t = (int)threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int s = DOT_THREADS / 2; s > 0; s >>= 1) {
        if (t < s) lds[t] = lds[t] + lds[t + s];
        __syncthreads();
    }
    return lds[0];
}

__global__ void __launch_bounds__(DOT_THREADS) k_dot_partial(int64_t n, const double *__restrict__ a,
                                                             const double *__restrict__ b, double *__restrict__ part)
{
    __shared__ double lds[DOT_THREADS];
    const int64_t chunk = (n + DOT_BLOCKS - 1) / DOT_BLOCKS;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += DOT_THREADS) s = s + a[i] * b[i];
    const double tot = block_sum(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// out[0] = the sum of the partials (sqrt of it with take_sqrt)
__global__ void __launch_bounds__(DOT_THREADS) k_dot_final(const double *__restrict__ part, double *__restrict__ out,
                                                           int take_sqrt)
{
    __shared__ double lds[DOT_THREADS];
    double s = 0.0;
    for (int i = (int)threadIdx.x; i < DOT_BLOCKS; i += DOT_THREADS) s = s + part[i];
    const double tot = block_sum(s, lds);
    if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(tot) : tot;
}

// w = w - h[0] * v  (h on the device: one Gram-Schmidt projection)
__global__ void __launch_bounds__(256) k_sub_scaled(int64_t n, double *__restrict__ w, const double *__restrict__ v,
                                                    const double *__restrict__ h)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = w[i] - h[0] * v[i];
}

// out = w / h[0]  (the next Arnoldi vector)
__global__ void __launch_bounds__(256) k_div_dev(int64_t n, const double *__restrict__ w, const double *__restrict__ h,
                                                 double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = w[i] / h[0];
}

// out = w / s  (host scalar)
__global__ void __launch_bounds__(256) k_div_host(int64_t n, const double *__restrict__ w, double s,
                                                  double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = w[i] / s;
}

// x = x + alpha * z  (host scalar)
__global__ void __launch_bounds__(256) k_axpy_host(int64_t n, double alpha, const double *__restrict__ z,
                                                   double *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = x[i] + alpha * z[i];
}

inline unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

} // namespace

hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, double *out, bool take_sqrt,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial, dim3(DOT_BLOCKS), dim3(DOT_THREADS), 0, s, n, a, b, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(DOT_THREADS), 0, s, part, out, take_sqrt ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_sub_scaled(int64_t n, double *w, const double *v, const double *h, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sub_scaled, dim3(blocks256(n)), dim3(256), 0, s, n, w, v, h);
    return hipGetLastError();
}

hipError_t launch_div_dev(int64_t n, const double *w, const double *h, double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_div_dev, dim3(blocks256(n)), dim3(256), 0, s, n, w, h, out);
    return hipGetLastError();
}

hipError_t launch_div_host(int64_t n, const double *w, double d, double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_div_host, dim3(blocks256(n)), dim3(256), 0, s, n, w, d, out);
    return hipGetLastError();
}

hipError_t launch_axpy_host(int64_t n, double alpha, const double *z, double *x, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy_host, dim3(blocks256(n)), dim3(256), 0, s, n, alpha, z, x);
    return hipGetLastError();
}

} // namespace silu
