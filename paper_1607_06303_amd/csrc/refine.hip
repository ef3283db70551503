// Kernels of the mixed-precision path with iterative refinement (real).
//
// A U0 computed with FP32 products is improved by Newton's method on the two
// matrix equations that define U = sign(T) entry by entry in the substitution
// (Eq. (2): U^2 = I where sign(t_ii) == sign(t_jj); Eq. (1): TU = UT where they
// differ).  One step:
//   1. residual in FP64, per block (I, J) off the block diagonal,
//        R_ij = (U^2 - I)_ij = sum_{k=i..j} u_ik u_kj          (equal signs)
//        R_ij = (U T - T U)_ij = sum_{k=i..j} (u_ik t_kj - t_ik u_kj)  (opposite)
//      as MFMA products over K = I .. J (k_resid); its per-block Frobenius
//      norms decide convergence;
//   2. the correction E from the linearised equations, U0 E + E U0 = -R and
//      T E - E T = R (the CORR sweep of flow.hip, FP32);
//   3. U <- U + E in FP64 (k_add_correction).
// The diagonal blocks are computed in FP64 from the start and are not refined.
#include <algorithm>

#include "common.h"

namespace sgt {

namespace {

constexpr int TB = kFlowTile;
constexpr int NT = 256;
constexpr int APITCH = TB + 16;
constexpr int BSLAB = 4 * TB + 4;

__device__ inline void atomic_max_nonneg(unsigned long long *p, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

__device__ inline double block_max(double v, double *red)
{
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    return r;
}

#define REF_MAT(a) (a.mats ? a.mats[blockIdx.z] : a.m0)

// FP32 copies for the reduced-precision sweeps: the upper triangle of T, and
// the (FP64-computed) diagonal blocks of U; max |t_ij| on the side.  Matrix
// blockIdx.z of the table; columns strided over blockIdx.y.
__global__ __launch_bounds__(NT) void k_to_f32(RefArgs a)
{
    __shared__ double red[NT / 64];
    const RefMat d = REF_MAT(a);
    double m = 0.0;
    for (int64_t j = blockIdx.y; j < d.n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i <= j;
             i += (int64_t)gridDim.x * NT) {
            const double t = d.T[i + j * d.ldt];
            d.T32[i + j * d.ld32] = (float)t;
            m = fmax(m, fabs(t));
            if (d.split == 0 && i / TB == j / TB) d.U32[i + j * d.ld32] = (float)d.U[i + j * d.ldu];
        }
    m = block_max(m, red);
    if (threadIdx.x == 0) atomic_max_nonneg(&d.maxes[0], m);
}

// Rows of column j that the reduced-precision sweep computed: above the
// diagonal block of column j (split == 0), or the rows of X (split > 0).
__device__ inline int64_t region_rows(int64_t j, int64_t split)
{
    if (split > 0) return j >= split ? split : 0;
    return (j / TB) * TB;
}

// U(i, j) = U32(i, j) in FP64 for the entries of the computed region.
__global__ __launch_bounds__(NT) void k_widen(RefArgs a)
{
    __shared__ double red[NT / 64];
    const RefMat d = REF_MAT(a);
    double m = 0.0;
    for (int64_t j = blockIdx.y; j < d.n; j += gridDim.y) {
        const int64_t iend = region_rows(j, d.split);
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < iend;
             i += (int64_t)gridDim.x * NT) {
            const double u = (double)d.U32[i + j * d.ld32];
            d.U[i + j * d.ldu] = u;
            m = fmax(m, fabs(u));
        }
    }
    m = block_max(m, red);
    if (threadIdx.x == 0) atomic_max_nonneg(&d.maxes[1], m);
}

// U += E on the entries of the computed region; max |E| on the side.
__global__ __launch_bounds__(NT) void k_add_correction(RefArgs a)
{
    __shared__ double red[NT / 64];
    const RefMat d = REF_MAT(a);
    double m = 0.0;
    for (int64_t j = blockIdx.y; j < d.n; j += gridDim.y) {
        const int64_t iend = region_rows(j, d.split);
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < iend;
             i += (int64_t)gridDim.x * NT) {
            const double e = (double)d.E32[i + j * d.ld32];
            d.U[i + j * d.ldu] += e;
            m = fmax(m, fabs(e));
        }
    }
    m = block_max(m, red);
    if (threadIdx.x == 0) atomic_max_nonneg(&d.maxes[2], m);
}

__global__ void k_clear_correction_max(RefArgs a)
{
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z < a.nmat) (a.mats ? a.mats[z] : a.m0).maxes[2] = 0;
}

// FP64 residual of one off-diagonal block per workgroup (tasks in reverse
// order: the longest products first).  Output: R as FP32 (the right-hand side
// of the correction sweep, into E32) and the block's squared Frobenius norm.
__global__ __launch_bounds__(NT) void k_resid(RefArgs a, const int2 *__restrict__ tasks,
                                              int ntasks, double *__restrict__ norm2)
{
    __shared__ double sAU[TB * APITCH], sAT[TB * APITCH];
    __shared__ double sBU[(TB / 4) * BSLAB], sBT[(TB / 4) * BSLAB];
    __shared__ int8_t rs[TB], cs[TB];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pr = wave >> 1, pc = wave & 1;
    const int lc = tid >> 3, lr = (tid & 7) * 4;
    const int2 tk = tasks[ntasks - 1 - (int)blockIdx.x];
    const RefMat d = a.mats ? a.mats[uniform(tk.x)] : a.m0;
    const int I = uniform(tk.y >> 16), J = uniform(tk.y & 0xffff);
    const int64_t n = uniform(d.n);
    const double *T = d.T, *U = d.U;
    const int64_t ldt = d.ldt, ldu = d.ldu;
    const int64_t r0 = (int64_t)I * TB, c0 = (int64_t)J * TB;
    const int bj = (int)min((int64_t)TB, n - c0);
    if (tid < TB) {
        rs[tid] = d.sgn[r0 + tid];
        cs[tid] = tid < bj ? d.sgn[c0 + tid] : 0;
    }
    __syncthreads();
    bool needY = false, needX = false;
    {
        bool rp = false, rn = false, cp = false, cn = false;
        for (int u = 0; u < 16; ++u) {
            const int vr = rs[16 * pr + u], vc = cs[16 * pc + u];
            rp |= vr > 0;
            rn |= vr < 0;
            cp |= vc > 0;
            cn |= vc < 0;
        }
        needY = (rp && cp) || (rn && cn);
        needX = (rp && cn) || (rn && cp);
    }
    const bool any_x = __syncthreads_or(needX);

    dx4 accY, accX;
    for (int r = 0; r < 4; ++r) accY[r] = accX[r] = 0.0;

    double gaU[4], gaT[4], gbU[4], gbT[4];
    auto load = [&](int K) {
        const int64_t k0 = (int64_t)K * TB;
        const bool dA = K == I, dB = K == J;
        const int64_t ca = k0 + lc;  // column of the A tiles
        const int64_t cb = c0 + lc;  // column of the B tiles
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t ra = r0 + lr + e, rb = k0 + lr + e;
            const bool okA = ca < n && !(dA && ra > ca);
            const bool okB = rb < n && cb < n && !(dB && rb > cb);
            gaU[e] = okA ? U[ra + ca * ldu] : 0.0;
            gaT[e] = (okA && any_x) ? T[ra + ca * ldt] : 0.0;
            gbU[e] = okB ? U[rb + cb * ldu] : 0.0;
            gbT[e] = (okB && any_x) ? T[rb + cb * ldt] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            sAU[lc * APITCH + lr + e] = gaU[e];
            sAT[lc * APITCH + lr + e] = -gaT[e];
            sBU[(lr >> 2) * BSLAB + lc * 4 + e] = gbU[e];
            sBT[(lr >> 2) * BSLAB + lc * 4 + e] = gbT[e];
        }
    };
    const int g = lane >> 4, tl = lane & 15;
    load(I);
    store();
    __syncthreads();
    for (int K = I; K <= J; ++K) {
        const bool more = K < J;
        if (more) load(K + 1);
#pragma unroll
        for (int k4 = 0; k4 < TB / 4; ++k4) {
            const int ao = (k4 * 4 + g) * APITCH + 16 * pr + tl;
            const int bo = k4 * BSLAB + (16 * pc + tl) * 4 + g;
            const double aU = sAU[ao], aT = sAT[ao], bU = sBU[bo], bT = sBT[bo];
            if (needY) accY = mfma_f64(aU, bU, accY);
            if (needX) {
                accX = mfma_f64(aU, bT, accX);
                accX = mfma_f64(aT, bU, accX);
            }
        }
        __syncthreads();
        if (more) {
            store();
            __syncthreads();
        }
    }
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = 16 * pr + mfma64_row(lane, r);
        const int j = 16 * pc + tl;
        const double v = rs[i] == cs[j] ? accY[r] : accX[r];
        if (j < bj) {
            d.E32[(r0 + i) + (c0 + j) * d.ld32] = (float)v;
            ss += v * v;
        }
    }
    for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m, 64);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) norm2[d.f0 + (int64_t)I * d.nbc + J] = red[0] + red[1] + red[2] + red[3];
}

// FP64 residual of the Sylvester equation T11 X - X T22 = 2 s T12 for one
// block of X per workgroup: R = 2 s T12 - T11 X + X T22, with X = U(0:p, p:n).
// K steps: blocks K >= I of T11's rows (K = I keeps its upper triangle), then
// blocks K <= J of T22's columns (K = J likewise).
__global__ __launch_bounds__(NT) void k_resid_syl(RefArgs a, const int2 *__restrict__ tasks,
                                                  int ntasks, double *__restrict__ norm2)
{
    __shared__ double sA[TB * APITCH];
    __shared__ double sB[(TB / 4) * BSLAB];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pr = wave >> 1, pc = wave & 1;
    const int lc = tid >> 3, lr = (tid & 7) * 4;
    const int2 tk = tasks[ntasks - 1 - (int)blockIdx.x];
    const RefMat d = a.mats ? a.mats[uniform(tk.x)] : a.m0;
    const int I = uniform(tk.y >> 16), J = uniform(tk.y & 0xffff);
    const int64_t n = uniform(d.n), p = uniform(d.split);
    const double *T = d.T, *U = d.U;
    const int64_t ldt = d.ldt, ldu = d.ldu;
    const int64_t r0 = (int64_t)I * TB, c0 = p + (int64_t)J * TB;

    dx4 acc;
    for (int r = 0; r < 4; ++r) acc[r] = 0.0;
    const int na = uniform(d.nbr) - I, nsteps = uniform(na + J + 1);
    double ga[4], gb[4];
    auto load = [&](int s) {
        int64_t ar, ac, aend_r, aend_c, br, bc, bend_r, bend_c;
        bool adiag, bdiag;
        const double *pa, *pb;
        int64_t lda, ldb;
        double sa;
        if (s < na) {  // -T11(I, K) * X(K, J)
            const int K = I + s;
            pa = T; lda = ldt; ar = r0; ac = (int64_t)K * TB; aend_r = p; aend_c = p;
            adiag = K == I; sa = -1.0;
            pb = U; ldb = ldu; br = (int64_t)K * TB; bc = c0; bend_r = p; bend_c = n;
            bdiag = false;
        } else {       // X(I, K) * T22(K, J)
            const int K = s - na;
            pa = U; lda = ldu; ar = r0; ac = p + (int64_t)K * TB; aend_r = p; aend_c = n;
            adiag = false; sa = 1.0;
            pb = T; ldb = ldt; br = p + (int64_t)K * TB; bc = c0; bend_r = n; bend_c = n;
            bdiag = K == J;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t ra = ar + lr + e, ca = ac + lc;
            const int64_t rb = br + lr + e, cb = bc + lc;
            const bool okA = ra < aend_r && ca < aend_c && !(adiag && ra > ca);
            const bool okB = rb < bend_r && cb < bend_c && !(bdiag && rb > cb);
            ga[e] = okA ? sa * pa[ra + ca * lda] : 0.0;
            gb[e] = okB ? pb[rb + cb * ldb] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            sA[lc * APITCH + lr + e] = ga[e];
            sB[(lr >> 2) * BSLAB + lc * 4 + e] = gb[e];
        }
    };
    const int g = lane >> 4, tl = lane & 15;
    load(0);
    store();
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const bool more = s + 1 < nsteps;
        if (more) load(s + 1);
#pragma unroll
        for (int k4 = 0; k4 < TB / 4; ++k4) {
            const double av = sA[(k4 * 4 + g) * APITCH + 16 * pr + tl];
            const double bv = sB[k4 * BSLAB + (16 * pc + tl) * 4 + g];
            acc = mfma_f64(av, bv, acc);
        }
        __syncthreads();
        if (more) {
            store();
            __syncthreads();
        }
    }
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = r0 + 16 * pr + mfma64_row(lane, r);
        const int64_t j = c0 + 16 * pc + tl;
        if (i < p && j < n) {
            const double v = d.two_s * T[i + j * ldt] + acc[r];
            d.E32[i + j * d.ld32] = (float)v;
            ss += v * v;
        }
    }
    for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m, 64);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) norm2[d.f0 + (int64_t)I * d.nbc + J] = red[0] + red[1] + red[2] + red[3];
}

// Grid of the column-wise elementwise kernels: a few thousand workgroups per
// matrix, each over a strided set of columns, so that each publishes its
// maximum with one atomic (one atomic per column made the maxima cost more
// than the copies).  nmax: the largest order in the table.
dim3 col_grid(int64_t nmax, int nmat)
{
    const int64_t bx = std::min<int64_t>((nmax + NT - 1) / NT, 8);
    const int64_t by = std::max<int64_t>(std::min<int64_t>(nmax, nmat > 1 ? 64 : 512), 1);
    return dim3((unsigned)std::max<int64_t>(bx, 1), (unsigned)by, (unsigned)nmat);
}

}  // namespace

hipError_t launch_to_f32(const RefArgs &a, int64_t nmax, hipStream_t st)
{
    if (nmax <= 0 || a.nmat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, col_grid(nmax, a.nmat), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_widen(const RefArgs &a, int64_t nmax, hipStream_t st)
{
    if (nmax <= 0 || a.nmat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_widen, col_grid(nmax, a.nmat), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_add_correction(const RefArgs &a, int64_t nmax, hipStream_t st)
{
    if (nmax <= 0 || a.nmat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_correction_max, dim3((a.nmat + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_add_correction, col_grid(nmax, a.nmat), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_resid(const RefArgs &a, bool syl, const int2 *tasks, int ntasks, double *norm2,
                        hipStream_t st)
{
    if (ntasks <= 0) return hipSuccess;
    if (syl)
        hipLaunchKernelGGL(k_resid_syl, dim3(ntasks), dim3(NT), 0, st, a, tasks, ntasks, norm2);
    else
        hipLaunchKernelGGL(k_resid, dim3(ntasks), dim3(NT), 0, st, a, tasks, ntasks, norm2);
    return hipGetLastError();
}

}  // namespace sgt
