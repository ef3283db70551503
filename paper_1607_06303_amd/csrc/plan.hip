// Diagonal scan and the Section 3 work model (Arithmetic Efficiency).
#include <algorithm>
#include <cmath>

#include "common.h"

namespace sgt {

// One workgroup reads the diagonal, records sign(Re t_ii) as +1/-1 (Section 1),
// the first index whose sign is undefined (zero or non-finite entry), and the
// number of positive signs; optionally the diagonal itself.
__global__ __launch_bounds__(1024) void k_scan(const double *__restrict__ T, int64_t ldt,
                                               int64_t n, int cplx, int8_t *__restrict__ sgn,
                                               double *__restrict__ dg,
                                               ScanResult *__restrict__ res)
{
    __shared__ unsigned long long bad;
    __shared__ unsigned long long npos;
    __shared__ unsigned long long amin, amax;
    if (threadIdx.x == 0) {
        bad = (unsigned long long)n;
        npos = 0;
        amin = ~0ull;
        amax = 0;
    }
    __syncthreads();
    unsigned long long my_pos = 0, my_min = ~0ull, my_max = 0;
    // The diagonal entries lie a column apart (a separate line, often a separate
    // page, each): every thread issues the loads of eight of them before using
    // any, so that their latencies overlap.
    constexpr int BATCH = 8;
    const int64_t stride = blockDim.x;
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += BATCH * stride) {
        double vre[BATCH], vim[BATCH];
#pragma unroll
        for (int k = 0; k < BATCH; ++k) {
            const int64_t i = i0 + k * stride;
            vre[k] = 0.0;
            vim[k] = 0.0;
            if (i < n) {
                if (cplx) {
                    const double *p = T + 2 * (i + i * ldt);
                    vre[k] = p[0];
                    vim[k] = p[1];
                } else {
                    vre[k] = T[i + i * ldt];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < BATCH; ++k) {
            const int64_t i = i0 + k * stride;
            if (i >= n) break;
            const double re = vre[k], im = vim[k];
            int s = 0;
            if (isfinite(re) && isfinite(im)) s = re > 0.0 ? 1 : (re < 0.0 ? -1 : 0);
            sgn[i] = (int8_t)s;
            // the divisors t_ii - t_jj of the sweeps, in FP64 (complex: re, im pairs)
            if (dg && cplx) {
                dg[2 * i] = re;
                dg[2 * i + 1] = im;
            } else if (dg) {
                dg[i] = re;
            }
            if (s == 0) atomicMin(&bad, (unsigned long long)i);
            my_pos += (s > 0);
            if (s != 0) {
                const unsigned long long a = (unsigned long long)__double_as_longlong(fabs(re));
                my_min = a < my_min ? a : my_min;
                my_max = a > my_max ? a : my_max;
            }
        }
    }
    atomicAdd(&npos, my_pos);
    atomicMin(&amin, my_min);
    atomicMax(&amax, my_max);
    __syncthreads();
    if (threadIdx.x == 0) {
        res->bad_index = (int64_t)bad;
        res->n_pos = (int64_t)npos;
        res->absmin = amin;
        res->absmax = amax;
    }
}

hipError_t launch_scan(const void *T, int64_t ldt, int64_t n, bool cplx, int8_t *sgn, double *dg,
                       ScanResult *res, hipStream_t st)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, (const double *)T, ldt, n,
                       cplx ? 1 : 0, sgn, dg, res);
    return hipGetLastError();
}

// Work model of Section 3, in O(n) with running counts.
//   W_PH = c * sum_{i<j} (j-i-1) * (2 if s_i == s_j else 4), c = 4 for complex.
//   k    = adjacent swaps to group by sign (inversions), the fewer of the two orders.
//   W_PS = c * (12 n k + n_- n_+ (n_- + n_+) + 12 n k): reorder with the Schur
//          vectors, the Sylvester equation, and the same rotations applied again
//          to bring the sign back (nothing when k = 0).
HostPlan plan_from_signs(const int8_t *s, int64_t n, bool is_complex)
{
    HostPlan p;
    const double c = is_complex ? 4.0 : 1.0;
    int64_t cnt[2] = {0, 0};   // [0]: negatives seen, [1]: positives seen
    double sumidx[2] = {0, 0};
    double opp_terms = 0.0;    // sum over opposite-sign pairs of (j - i - 1)
    for (int64_t j = 0; j < n; ++j) {
        int cls = s[j] > 0 ? 1 : 0;
        int opp = 1 - cls;
        opp_terms += (double)cnt[opp] * (double)(j - 1) - sumidx[opp];
        if (cls == 1) p.swaps_pos_first += cnt[0];  // a negative before this positive
        else p.swaps_neg_first += cnt[1];
        cnt[cls] += 1;
        sumidx[cls] += (double)j;
    }
    p.n_pos = cnt[1];
    p.n_neg = cnt[0];
    double nd = (double)n;
    double c3 = nd * (nd - 1.0) * (nd - 2.0) / 6.0;
    if (n < 3) c3 = 0.0;
    p.w_ph = c * (2.0 * c3 + 2.0 * opp_terms);
    int64_t k = std::min(p.swaps_pos_first, p.swaps_neg_first);
    double npn = (double)p.n_pos, nng = (double)p.n_neg;
    p.w_ps = c * (24.0 * nd * (double)k + nng * npn * (nng + npn));
    p.model_pick = (p.w_ps < p.w_ph) ? SIGNTRI_PATH_PS : SIGNTRI_PATH_PH;
    if (p.n_pos == 0 || p.n_neg == 0) {
        p.auto_path = SIGNTRI_PATH_TRIVIAL;
        p.model_pick = SIGNTRI_PATH_TRIVIAL;
        p.w_ps = 0.0;
        return p;
    }
    if (p.swaps_pos_first == 0) {
        p.ps_sign = 1;
        p.split = p.n_pos;
    } else if (p.swaps_neg_first == 0) {
        p.ps_sign = -1;
        p.split = p.n_neg;
    }
    // PS runs as such only on an already grouped diagonal.
    double w_ps_grouped = c * nng * npn * nd;
    p.auto_path = (p.ps_sign != 0 && w_ps_grouped < p.w_ph) ? SIGNTRI_PATH_PS : SIGNTRI_PATH_PH;
    // Otherwise the same result through the minority class's spectral projector:
    // two substitutions of about n^2 m / 2 multiply-adds each and the n^2 m / 2
    // multiply-adds of the rank-m product, 3 n^2 m flops in all (real T; complex
    // multiply-adds count four times as much, as in W_PH).
    p.n_min = std::min(p.n_pos, p.n_neg);
    p.min_sign = p.n_neg <= p.n_pos ? -1 : 1;
    // Complex T: the complex projector kernels (per-block launches, plain FMA
    // products) reach about an eighth of complex Parlett-Higham's rate (n = 4096:
    // 1.05 against 9.1 TFLOP/s), so their estimate is weighted by 8 against W_PH.
    const double w_proj = (is_complex ? 8.0 * c : 1.0) * 3.0 * nd * nd * (double)p.n_min;
    p.proj_pick = p.auto_path == SIGNTRI_PATH_PH && p.n_min >= 1 &&
                  p.n_min <= (is_complex ? kProjMaxMinority : kProjMaxMinorityReal) &&
                  w_proj < p.w_ph;
    return p;
}

}  // namespace sgt
