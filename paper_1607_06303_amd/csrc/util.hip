// Output helpers: zero the strict lower triangle, write +-I.
#include "common.h"

namespace sgt {

namespace {

// Column j = blockIdx.y (+ multiples of gridDim.y); rows j+1 .. n-1.
template <typename S>
__global__ __launch_bounds__(256) void k_zero_lower(S *__restrict__ U, int64_t ldu, int64_t n)
{
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = j + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x)
            U[i + j * ldu] = scalar_traits<S>::zero();
}

template <typename S>
__global__ __launch_bounds__(256) void k_fill_pm_identity(S *__restrict__ U, int64_t ldu, int64_t n,
                                                          double s)
{
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x)
            U[i + j * ldu] = (i == j) ? scalar_traits<S>::from_real(s) : scalar_traits<S>::zero();
}

dim3 column_grid(int64_t n)
{
    int64_t gx = (n + 255) / 256;
    if (gx > 64) gx = 64;
    int64_t gy = n < 65535 ? n : 65535;
    return dim3((unsigned)(gx < 1 ? 1 : gx), (unsigned)(gy < 1 ? 1 : gy));
}

}  // namespace

hipError_t launch_zero_lower(void *U, int64_t ldu, int64_t n, bool cplx, hipStream_t st)
{
    if (n <= 1) return hipSuccess;
    if (cplx)
        hipLaunchKernelGGL(k_zero_lower<cd>, column_grid(n), dim3(256), 0, st, (cd *)U, ldu, n);
    else
        hipLaunchKernelGGL(k_zero_lower<double>, column_grid(n), dim3(256), 0, st, (double *)U,
                           ldu, n);
    return hipGetLastError();
}

hipError_t launch_fill_pm_identity(void *U, int64_t ldu, int64_t n, bool cplx, double s,
                                   hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (cplx)
        hipLaunchKernelGGL(k_fill_pm_identity<cd>, column_grid(n), dim3(256), 0, st, (cd *)U,
                           ldu, n, s);
    else
        hipLaunchKernelGGL(k_fill_pm_identity<double>, column_grid(n), dim3(256), 0, st,
                           (double *)U, ldu, n, s);
    return hipGetLastError();
}

}  // namespace sgt
