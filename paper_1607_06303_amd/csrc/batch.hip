// Table-driven kernels that let one launch serve a whole set of real matrices
// (the batched entry point, and the single-matrix one as a set of one): the
// diagonal scan, the output preparation, and the diagonal blocks.
#include "common.h"

namespace sgt {

namespace {

constexpr int TB = kFlowTile;

// One workgroup per matrix: sign(Re t_ii) as +1/-1 (Section 1), the first
// index whose sign is undefined (zero or non-finite), the number of positive
// signs, and the diagonal itself (the divisors t_ii - t_jj).
__global__ __launch_bounds__(1024) void k_scan_b(const ScanMat *__restrict__ mats)
{
    const ScanMat d = mats[blockIdx.x];
    __shared__ unsigned long long bad;
    __shared__ unsigned long long npos;
    if (threadIdx.x == 0) {
        bad = (unsigned long long)d.n;
        npos = 0;
    }
    __syncthreads();
    unsigned long long my_pos = 0;
    for (int64_t i = threadIdx.x; i < d.n; i += blockDim.x) {
        double re, im = 0.0;
        if (d.cplx) {
            re = d.T[2 * (i + i * d.ldt)];
            im = d.T[2 * (i + i * d.ldt) + 1];
            d.dg[2 * i] = re;
            d.dg[2 * i + 1] = im;
        } else {
            re = d.T[i + i * d.ldt];
            d.dg[i] = re;
        }
        int s = 0;
        if (isfinite(re) && isfinite(im)) s = re > 0.0 ? 1 : (re < 0.0 ? -1 : 0);
        d.sgn[i] = (int8_t)s;
        if (s == 0) atomicMin(&bad, (unsigned long long)i);
        my_pos += (s > 0);
    }
    atomicAdd(&npos, my_pos);
    __syncthreads();
    if (threadIdx.x == 0) {
        d.res->bad_index = (int64_t)bad;
        d.res->n_pos = (int64_t)npos;
    }
}

// Output preparation of matrix blockIdx.z: kind 0 zeroes the strict lower
// triangle (the sweep writes the rest), kind 1 writes diag(s I_p, -s I_{n-p})
// (Parlett-Sylvester: the sweep writes X), kind 2 writes s I (one sign).
// P = 2: complex entries (interleaved re, im).
template <int P> __global__ __launch_bounds__(256) void k_prepare_b(const PrepMat *__restrict__ mats)
{
    const PrepMat d = mats[blockIdx.z];
    for (int64_t j = blockIdx.y; j < d.n; j += gridDim.y) {
        const int64_t i0 = d.kind == 0 ? j + 1 : 0;
        for (int64_t i = i0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.n;
             i += (int64_t)gridDim.x * blockDim.x) {
            double v = 0.0;
            if (i == j && d.kind != 0) v = (d.kind == 2 || i < d.p) ? d.s : -d.s;
            d.U[P * (i + j * d.ldu)] = v;
            if (P == 2) d.U[P * (i + j * d.ldu) + 1] = 0.0;
        }
    }
}

// Diagonal 32 x 32 blocks (Algorithm 3 per block, superdiagonal by
// superdiagonal), one per workgroup: task (matrix, block row).  Eight lanes
// share each entry's inner product.  P = 2: complex entries, kept in LDS as
// real and imaginary planes.
template <int P>
__global__ __launch_bounds__(256) void k_diag_b(const PrepMat *__restrict__ mats,
                                                const int2 *__restrict__ tasks)
{
    constexpr int LD = TB + 1, LPE = 256 / TB, PL = TB * LD;
    __shared__ double sT[P * PL], sU[P * PL];
    __shared__ int8_t ss[TB];
    const int2 tk = tasks[blockIdx.x];
    const PrepMat d = mats[uniform(tk.x)];
    const int64_t r0 = (int64_t)uniform(tk.y) * TB;
    const int bt = uniform((int)min((int64_t)TB, d.n - r0));
    for (int e = threadIdx.x; e < TB * TB; e += 256) {
        const int i = e % TB, j = e / TB;
        const bool in = i < bt && j < bt;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            sT[q * PL + i + j * LD] =
                (in && i <= j) ? d.T[P * ((r0 + i) + (r0 + j) * d.ldt) + q] : 0.0;
            double u = 0.0;
            if (in && i == j) {
                if (d.fd) u = d.fd[P * (r0 + i) + q];
                else if (q == 0) u = (double)d.sgn[r0 + i];
            }
            sU[q * PL + i + j * LD] = u;
        }
    }
    // (a general function: every pair by Eq. (1)'s form, the element Parlett
    // equation of Algorithm 1: distinct classes for the two ends of every pair)
    if (threadIdx.x < TB) ss[threadIdx.x] = threadIdx.x < bt ? (d.fd ? 1 : d.sgn[r0 + threadIdx.x]) : 1;
    const bool gen = d.fd != nullptr;
    __syncthreads();
    const int i = threadIdx.x / LPE, q = threadIdx.x % LPE;
    for (int dd = 1; dd < bt; ++dd) {
        const int j = i + dd;
        if (j < bt) {
            const int si = ss[i], sj = ss[j];
            const bool opp = gen || si != sj;
            double sr = 0.0, sim = 0.0;
            if (opp) {
                for (int k = i + 1 + q; k < j; k += LPE) {
                    const int ik = i + k * LD, kj = k + j * LD;
                    sr += sU[ik] * sT[kj] - sT[ik] * sU[kj];
                    if (P == 2) {
                        sr += -sU[PL + ik] * sT[PL + kj] + sT[PL + ik] * sU[PL + kj];
                        sim += sU[ik] * sT[PL + kj] + sU[PL + ik] * sT[kj] - sT[ik] * sU[PL + kj] -
                               sT[PL + ik] * sU[kj];
                    }
                }
            } else {
                for (int k = i + 1 + q; k < j; k += LPE) {
                    const int ik = i + k * LD, kj = k + j * LD;
                    sr += sU[ik] * sU[kj];
                    if (P == 2) {
                        sr -= sU[PL + ik] * sU[PL + kj];
                        sim += sU[ik] * sU[PL + kj] + sU[PL + ik] * sU[kj];
                    }
                }
            }
            sr = group_sum<LPE>(sr);
            if (P == 2) sim = group_sum<LPE>(sim);
            if (q == 0) {
                double ur, ui = 0.0;
                if (opp) {
                    // Eq. (1): t_ij (u_ii - u_jj) = 2 s_i t_ij for the sign; for a general
                    // function t_ij (f_ii - f_jj)
                    double cr = 2.0 * si, ci = 0.0;
                    if (gen) {
                        cr = sU[i + i * LD] - sU[j + j * LD];
                        if (P == 2) ci = sU[PL + i + i * LD] - sU[PL + j + j * LD];
                    }
                    const double tr = sT[i + j * LD], ti = P == 2 ? sT[PL + i + j * LD] : 0.0;
                    const double nr = (cr * tr - ci * ti) + sr;
                    const double dr = sT[i + i * LD] - sT[j + j * LD];
                    if (P == 2) {
                        const double ni = (cr * ti + ci * tr) + sim;
                        const double di = sT[PL + i + i * LD] - sT[PL + j + j * LD];
                        // (nr + i ni) / (dr + i di), scaled against overflow
                        const double s = fmax(fabs(dr), fabs(di));
                        const double xr = dr / s, xi = di / s;
                        const double den = s * (xr * xr + xi * xi);
                        ur = (nr * xr + ni * xi) / den;
                        ui = (ni * xr - nr * xi) / den;
                    } else {
                        ur = nr / dr;
                    }
                } else {
                    // Eq. (2): -sum / (u_ii + u_jj) = -(s_i / 2) sum, an exact scaling
                    ur = -0.5 * si * sr;
                    ui = -0.5 * si * sim;
                }
                sU[i + j * LD] = ur;
                if (P == 2) sU[PL + i + j * LD] = ui;
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TB * TB; e += 256) {
        const int ii = e % TB, jj = e / TB;
        if (ii < bt && jj < bt && ii <= jj)
#pragma unroll
            for (int p2 = 0; p2 < P; ++p2)
                d.U[P * ((r0 + ii) + (r0 + jj) * d.ldu) + p2] = sU[p2 * PL + ii + jj * LD];
    }
}

}  // namespace

hipError_t launch_scan_b(const ScanMat *mats, int nmat, hipStream_t st)
{
    if (nmat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_b, dim3(nmat), dim3(1024), 0, st, mats);
    return hipGetLastError();
}

hipError_t launch_prepare_b(const PrepMat *mats, int nmat, int64_t nmax, bool cplx, hipStream_t st)
{
    if (nmat <= 0 || nmax <= 0) return hipSuccess;
    const int64_t gx = std::min<int64_t>((nmax + 255) / 256, 8);
    const int64_t gy = std::min<int64_t>(nmax, nmat > 1 ? 64 : 1024);
    const dim3 g((unsigned)gx, (unsigned)gy, (unsigned)nmat);
    if (cplx)
        hipLaunchKernelGGL(k_prepare_b<2>, g, dim3(256), 0, st, mats);
    else
        hipLaunchKernelGGL(k_prepare_b<1>, g, dim3(256), 0, st, mats);
    return hipGetLastError();
}

hipError_t launch_diag_b(const PrepMat *mats, const int2 *tasks, int ntasks, bool cplx,
                         hipStream_t st)
{
    if (ntasks <= 0) return hipSuccess;
    if (cplx)
        hipLaunchKernelGGL(k_diag_b<2>, dim3(ntasks), dim3(256), 0, st, mats, tasks);
    else
        hipLaunchKernelGGL(k_diag_b<1>, dim3(ntasks), dim3(256), 0, st, mats, tasks);
    return hipGetLastError();
}

}  // namespace sgt
