// Output helpers: zero the strict lower triangle, write +-I or diag(s I, -s I),
// and transpose (row-major arguments).
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

__global__ __launch_bounds__(256) void k_fill_split_identity(double *__restrict__ U, int64_t ldu,
                                                             int64_t n, int64_t p, double s)
{
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x)
            U[i + j * ldu] = (i == j) ? (i < p ? s : -s) : 0.0;
}

// dst(i, j) = src(j, i) for an n x n matrix, through a 32 x 33 LDS tile so that
// both the reads and the writes run along columns.
template <typename S>
__global__ __launch_bounds__(256) void k_transpose(const S *__restrict__ src, int64_t lds,
                                                   S *__restrict__ dst, int64_t ldd, int64_t n)
{
    __shared__ S tile[32][33];
    const int64_t bi = (int64_t)blockIdx.x * 32, bj = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bi + tx, j = bj + r;  // src(i, j)
        if (i < n && j < n) tile[r][tx] = src[i + j * lds];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bj + tx, j = bi + r;  // dst(i, j) = src(j, i)
        if (i < n && j < n) dst[i + j * ldd] = tile[tx][r];
    }
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

hipError_t launch_fill_split_identity(double *U, int64_t ldu, int64_t n, int64_t p, double s,
                                      hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_split_identity, column_grid(n), dim3(256), 0, st, U, ldu, n, p, s);
    return hipGetLastError();
}

hipError_t launch_transpose(const void *src, int64_t lds, void *dst, int64_t ldd, int64_t n,
                            bool cplx, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t nt = (n + 31) / 32;
    if (nt > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nt, (unsigned)nt);
    if (cplx)
        hipLaunchKernelGGL(k_transpose<cd>, grid, dim3(256), 0, st, (const cd *)src, lds, (cd *)dst,
                           ldd, n);
    else
        hipLaunchKernelGGL(k_transpose<double>, grid, dim3(256), 0, st, (const double *)src, lds,
                           (double *)dst, ldd, n);
    return hipGetLastError();
}

}  // namespace sgt
