// sign(A) for a general square A of small order (Section 1): a complex Schur
// decomposition A = Q T Q* (the first step of Algorithm 3), U = sign(T) by the
// element substitution of Algorithm 3 (Eq. (1) where the signs of Re t_ii and
// Re t_jj differ, Eq. (2) where they agree), and sign(A) = Q U Q*.
//
// One workgroup of one wave per matrix; the matrix, reduced in place, stays in
// LDS (64 x 65 complex entries, 67 KB, for orders 33 to 64: two workgroups per
// compute unit; 32 x 33 for orders up to 32), Q in a global workspace.
//   1. Hessenberg form by Householder reflections P = I - 2 w w* / (w* w)
//      (Hermitian and unitary), H <- P H P and Q <- Q P, one column at a time;
//      lane j updates column j from the left, lane i row i from the right.
//   2. The shifted QR iteration on the Hessenberg matrix, one implicit single
//      shift per sweep (the eigenvalue of the trailing 2 x 2 block nearer its
//      last diagonal entry; an exceptional shift after 10 and 20 sweeps
//      without deflation), the bulge chased by plane rotations
//      G = [c s; -conj(s) c] applied to the whole rows and columns (the full
//      Schur form, not only the eigenvalues) and, after each sweep, to Q.  A subdiagonal entry is
//      set to zero when it is at most the unit roundoff times the two diagonal
//      entries beside it (or below the smallest normal number scaled by n / u).
//      At most 30 max(10, n) sweeps, else the matrix is reported as not
//      converged.
//   3. U = sign(T), superdiagonal by superdiagonal (lane i: entry (i, i + d)),
//      kept in the strict lower triangle of the same LDS array (U_ij at
//      position (j, i)), which the Schur form leaves free.
//   4. sign(A) = (Q U) Q*, a row at a time: row i of Q U into an LDS row, then
//      lane j forms entry (i, j) against row j of Q.  A real A gets the real
//      part (sign of a real matrix is real; its imaginary part is rounding).
// A is first scaled by a power of two (exactly; the sign is unchanged) so that
// its largest entry lies in [1, 2).  An eigenvalue on the imaginary axis leaves
// S untouched and reports SIGNM_EDOMAIN.  The computed Schur form moves
// eigenvalues by rounding, so "on the axis" means |Re t_ii| <= n u ||A||_F (u
// the unit roundoff), where the sign of Re t_ii is not determined by A; a
// non-finite t_ii counts too.
#include <cfloat>

#include "common.h"
#include "signm.h"

namespace sgt {

namespace {

constexpr int NT = 64;  // one wave

__device__ inline cd cconj(cd a) { return {a.re, -a.im}; }
__device__ inline double cabs2(cd a) { return a.re * a.re + a.im * a.im; }
__device__ inline double cabsv(cd a) { return hypot(a.re, a.im); }
__device__ inline double cabs1(cd a) { return fabs(a.re) + fabs(a.im); }

// principal square root
__device__ inline cd csqrt_p(cd z)
{
    const double r = hypot(z.re, z.im);
    if (r == 0.0) return {0.0, 0.0};
    const double t = sqrt(0.5 * (r + fabs(z.re)));
    if (z.re >= 0.0) return {t, z.im / (2.0 * t)};
    return {fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// 1 / sqrt(a) for a > 0: the hardware estimate and two Newton steps (each
// squares the relative error; the estimate's is below 2^-22)
__device__ inline double rsqrt_nr(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// The plane rotation G = [c s; -conj(s) c] (c real) with G [x; y] = [r; 0]:
// c = |x| / nu, s = (x / |x|) conj(y) / nu, r = (x / |x|) nu, nu = |(x, y)|
// (x = 0: c = 0, s = 1, r = y).  The operands are scaled by a power of two so
// that their squares neither overflow nor underflow.
__device__ inline void givens(cd x, cd y, double &c, cd &s, cd &r)
{
    const double mx = fmax(fmax(fabs(x.re), fabs(x.im)), fmax(fabs(y.re), fabs(y.im)));
    if (!(mx > 0.0)) {
        c = 1.0;
        s = {0.0, 0.0};
        r = x;
        return;
    }
    const int e = ilogb(mx);
    const double sc = ldexp(1.0, -e);
    const cd xs = {x.re * sc, x.im * sc}, ys = {y.re * sc, y.im * sc};
    const double ax2 = xs.re * xs.re + xs.im * xs.im;
    const double nu2 = ax2 + (ys.re * ys.re + ys.im * ys.im);
    if (ax2 == 0.0) {
        c = 0.0;
        s = {1.0, 0.0};
        r = y;
        return;
    }
    const double iax = rsqrt_nr(ax2), inu = rsqrt_nr(nu2);
    const cd px = {xs.re * iax, xs.im * iax};  // x / |x|
    c = ax2 * iax * inu;
    s = px * cd{ys.re * inu, -ys.im * inu};
    const double nu = ldexp(nu2 * inu, e);
    r = {px.re * nu, px.im * nu};
}

// Lane src's complex value, held by every lane
__device__ inline double readlane_d(double v, int src)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, src);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ inline cd readlane_c(cd v, int src) { return {readlane_d(v.re, src), readlane_d(v.im, src)}; }

// sum over the wave
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Q lives in global memory (M.Q, row-major, pitch n), so that LDS holds only
// the matrix (two workgroups of the larger instance fit on a compute unit);
// the rotations of a QR sweep are logged in LDS and applied to Q after the
// sweep, each lane running its row through them with the next entries loaded
// ahead.
template <int NM, bool CPLX>
__global__ __launch_bounds__(NT) void k_signm(const SignmMat *__restrict__ mats,
                                              int32_t *__restrict__ status, int max_sweeps)
{
    constexpr int P = NM + 1;  // LDS pitch in complex entries
    __shared__ cd H[NM * P];   // row-major: H[r * P + c]
    __shared__ cd w[NM];       // Householder vector; then a row of Q U
    __shared__ cd qr[NM];      // a row of Q
    __shared__ double rc[NM];  // the sweep's rotations
    __shared__ cd rs[NM];
    const int lane = threadIdx.x;
    const SignmMat M = mats[blockIdx.x];
    const int n = uniform(M.n);
    auto h = [&](int r, int c) -> cd & { return H[r * P + c]; };
    cd *const Qg = M.Q;
    auto qget = [&](int r, int c) -> cd {
        const double *d = (const double *)(Qg + (int64_t)r * n + c);
        return {gload(d), gload(d + 1)};
    };
    auto qset = [&](int r, int c, cd v) {
        double *d = (double *)(Qg + (int64_t)r * n + c);
        gstore(d, v.re);
        gstore(d + 1, v.im);
    };

    // sign(c A) = sign(A) for c > 0: A is scaled by the power of two that brings its
    // largest entry to [1, 2), exactly, so that no square in the reduction or the
    // rotations overflows or underflows, whatever A's magnitude
    double amax = 0.0;
    for (int e = lane; e < n * n; e += NT) {
        const int r = e % n, c = e / n;
        const int64_t off = r + (int64_t)c * M.lda;
        cd v;
        if (CPLX) v = {gload(M.A + 2 * off), gload(M.A + 2 * off + 1)};
        else v = {gload(M.A + off), 0.0};
        h(r, c) = v;
        amax = fmax(amax, fmax(fabs(v.re), fabs(v.im)));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
    const double ascale = (amax > 0.0 && isfinite(amax)) ? ldexp(1.0, -ilogb(amax)) : 1.0;
    __syncthreads();
    double fro2 = 0.0;
    for (int e = lane; e < n * n; e += NT) {
        const int r = e % n, c = e / n;
        const cd v = h(r, c) * ascale;
        h(r, c) = v;
        fro2 += cabs2(v);
    }
    for (int e = lane; e < n * n; e += NT) {
        const int r = e / n, c = e % n;
        qset(r, c, cd{r == c ? 1.0 : 0.0, 0.0});
    }
    // an eigenvalue whose real part is within rounding of zero has no defined sign
    const double axis_tol = (double)n * DBL_EPSILON * sqrt(wave_sum(fro2));
    __syncthreads();

    // ---- 1. Hessenberg form
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;  // rows k+1 .. n-1 of column k
        const cd xl = lane < m ? h(k + 1 + lane, k) : cd{0.0, 0.0};
        const double below = wave_sum(lane >= 1 && lane < m ? cabs2(xl) : 0.0);
        if (uniform(below > 0.0 ? 1 : 0) == 0) continue;  // column already reduced
        const cd x0 = h(k + 1, k);
        const double a0 = cabsv(x0);
        const cd ph = a0 > 0.0 ? x0 * (1.0 / a0) : cd{1.0, 0.0};
        const double alpha = sqrt(a0 * a0 + below);
        // w = x + ph alpha e1: P x = -ph alpha e1
        if (lane < m) w[lane] = lane == 0 ? x0 + ph * alpha : xl;
        const double wn2 = (a0 + alpha) * (a0 + alpha) + below;
        const double beta = 2.0 / wn2;
        __syncthreads();
        // from the left, columns k+1 .. n-1 (column k is set below)
        if (lane > k && lane < n) {
            const int j = lane;
            cd s = {0.0, 0.0};
            for (int i = 0; i < m; ++i) s = s + cconj(w[i]) * h(k + 1 + i, j);
            s = s * beta;
            for (int i = 0; i < m; ++i) h(k + 1 + i, j) = h(k + 1 + i, j) - w[i] * s;
        }
        __syncthreads();
        // from the right, every row; and Q <- Q P
        if (lane < n) {
            const int i = lane;
            cd t = {0.0, 0.0}, u = {0.0, 0.0};
            for (int l = 0; l < m; ++l) {
                t = t + h(i, k + 1 + l) * w[l];
                u = u + qget(i, k + 1 + l) * w[l];
            }
            t = t * beta;
            u = u * beta;
            for (int l = 0; l < m; ++l) {
                h(i, k + 1 + l) = h(i, k + 1 + l) - t * cconj(w[l]);
                qset(i, k + 1 + l, qget(i, k + 1 + l) - u * cconj(w[l]));
            }
        }
        __syncthreads();
        if (lane < m) h(k + 1 + lane, k) = lane == 0 ? -(ph * alpha) : cd{0.0, 0.0};
        __syncthreads();
    }

    // ---- 2. shifted QR iteration to the Schur form
    const double ulp = DBL_EPSILON;
    const double smlnum = DBL_MIN * ((double)n / ulp);
    const int itmax = max_sweeps > 0 ? max_sweeps : 30 * max(10, n);
    int ihi = n - 1, its = 0, total = 0;
    bool fail = false;
    while (ihi >= 1) {
        // the lowest l such that H[l, l-1] is negligible (0: none)
        int l = 0;
        for (int k = ihi; k >= 1; --k) {
            const double a = cabs1(h(k, k - 1));
            double tst = cabs1(h(k - 1, k - 1)) + cabs1(h(k, k));
            if (tst == 0.0) {
                if (k - 2 >= 0) tst += fabs(h(k - 1, k - 2).re);
                if (k + 1 <= ihi) tst += fabs(h(k + 1, k).re);
            }
            if (a <= smlnum || a <= ulp * tst) {
                l = k;
                break;
            }
        }
        l = uniform(l);
        __syncthreads();
        if (l > 0) {
            if (lane == 0) h(l, l - 1) = cd{0.0, 0.0};
            __syncthreads();
        }
        if (l == ihi) {
            // a 1 x 1 block has converged
            ihi = uniform(ihi - 1);
            its = 0;
            continue;
        }
        if (uniform(++total > itmax ? 1 : 0)) {
            fail = true;
            break;
        }
        ++its;
        cd mu;
        if (its == 10) {
            mu = h(l, l) + cd{0.75 * fabs(h(l + 1, l).re), 0.0};
        } else if (its == 20) {
            mu = h(ihi, ihi) + cd{0.75 * fabs(h(ihi, ihi - 1).re), 0.0};
        } else {
            // the eigenvalue of the trailing 2 x 2 block nearer its last diagonal entry
            const cd a = h(ihi - 1, ihi - 1), b = h(ihi - 1, ihi), c = h(ihi, ihi - 1),
                     d = h(ihi, ihi);
            const cd hm = (a - d) * 0.5;
            const cd disc = csqrt_p(hm * hm + b * c);
            const cd mid = (a + d) * 0.5;
            const cd e1 = mid + disc, e2 = mid - disc;
            mu = cabs2(e1 - d) <= cabs2(e2 - d) ? e1 : e2;
        }
        // The entries that define rotation k (k > l) are those the column update of
        // rotation k - 1 has just formed in lanes k and k + 1: taken from there
        // by readlane rather than through LDS.
        cd x = h(l, l) - mu, y = h(l + 1, l);
        for (int k = l; k < ihi; ++k) {
            double c;
            cd s, r;
            givens(x, y, c, s, r);
            // rows k, k+1 from column jlo on
            const int jlo = k == l ? l : k;
            if (lane >= jlo && lane < n) {
                const int j = lane;
                const cd h1 = h(k, j), h2 = h(k + 1, j);
                h(k, j) = h1 * c + s * h2;
                h(k + 1, j) = h2 * c - cconj(s) * h1;
            }
            if (k > l && lane == 0) {
                h(k, k - 1) = r;
                h(k + 1, k - 1) = cd{0.0, 0.0};
            }
            __syncthreads();
            // columns k, k+1 of rows 0 .. min(k + 2, ihi) (Q: after the sweep)
            const int ilast = min(k + 2, ihi);
            cd nk = {0.0, 0.0};
            if (lane < n) {
                const int i = lane;
                if (i <= ilast) {
                    const cd h1 = h(i, k), h2 = h(i, k + 1);
                    nk = h1 * c + h2 * cconj(s);
                    h(i, k) = nk;
                    h(i, k + 1) = h2 * c - h1 * s;
                }
            }
            if (lane == 0) {
                rc[k - l] = c;
                rs[k - l] = s;
            }
            if (k + 1 < ihi) {
                x = readlane_c(nk, k + 1);
                y = readlane_c(nk, k + 2);
            }
            __syncthreads();
        }
        {
            // the sweep's rotations, in order, on columns l .. ihi of every row of Q
            if (lane < n) {
                const int i = lane;
                cd carry = qget(i, l);
                for (int k0 = l; k0 < ihi; k0 += 8) {
                    cd nx[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (k0 + u < ihi) nx[u] = qget(i, k0 + u + 1);
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (k0 + u < ihi) {
                            const double c = rc[k0 + u - l];
                            const cd s = rs[k0 + u - l];
                            qset(i, k0 + u, carry * c + nx[u] * cconj(s));
                            carry = nx[u] * c - carry * s;
                        }
                }
                qset(i, ihi, carry);
            }
            __syncthreads();
        }
    }
    if (fail) {
        if (lane == 0) status[M.index] = SIGNM_ENOCONV;
        return;
    }

    // ---- 3. U = sign(T)
    bool bad = false;
    if (lane < n) {
        const cd t = h(lane, lane);
        bad = !(fabs(t.re) > axis_tol) || !isfinite(t.re) || !isfinite(t.im);
    }
    if (__builtin_amdgcn_ballot_w64(bad) != 0) {
        if (lane == 0) status[M.index] = SIGNM_EDOMAIN;
        return;
    }
    auto sgn = [&](int i) -> double { return h(i, i).re > 0.0 ? 1.0 : -1.0; };
    for (int d = 1; d < n; ++d) {
        if (lane + d < n) {
            const int i = lane, j = lane + d;
            const double si = sgn(i), sj = sgn(j);
            cd sum = {0.0, 0.0};
            cd u;
            if (si != sj) {
                // Eq. (1): u_ii - u_jj = 2 si
                for (int k = i + 1; k < j; ++k) sum = sum + h(k, i) * h(k, j) - h(i, k) * h(j, k);
                u = (h(i, j) * (2.0 * si) + sum) / (h(i, i) - h(j, j));
            } else {
                // Eq. (2): u_ii + u_jj = 2 si
                for (int k = i + 1; k < j; ++k) sum = sum + h(k, i) * h(j, k);
                u = sum * (-0.5 * si);
            }
            h(j, i) = u;
        }
        __syncthreads();
    }

    // ---- 4. S = (Q U) Q*, row by row
    // (every lane's stores of Q reach the other lanes' loads below)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    for (int i = 0; i < n; ++i) {
        if (lane < n) qr[lane] = qget(i, lane);
        __syncthreads();
        if (lane < n) {
            const int j = lane;
            cd acc = qr[j] * sgn(j);
            for (int k = 0; k < j; ++k) acc = acc + qr[k] * h(j, k);
            w[j] = acc;
        }
        __syncthreads();
        if (lane < n) {
            const int j = lane;
            cd acc = {0.0, 0.0};
#pragma unroll 8
            for (int k = 0; k < n; ++k) acc = acc + w[k] * cconj(qget(j, k));
            const int64_t off = i + (int64_t)j * M.lds;
            if (CPLX) {
                gstore(M.S + 2 * off, acc.re);
                gstore(M.S + 2 * off + 1, acc.im);
            } else {
                gstore(M.S + off, acc.re);
            }
        }
        __syncthreads();
    }
    if (lane == 0) status[M.index] = SIGNM_OK;
}

template <bool CPLX>
hipError_t launch_signm_t(const SignmMat *mats, int count, int n32, int32_t *status,
                          int max_sweeps, hipStream_t st)
{
    if (n32 > 0)
        hipLaunchKernelGGL((k_signm<32, CPLX>), dim3(n32), dim3(NT), 0, st, mats, status,
                           max_sweeps);
    if (count > n32)
        hipLaunchKernelGGL((k_signm<kSignmMaxOrder, CPLX>), dim3(count - n32), dim3(NT), 0, st,
                           mats + n32, status, max_sweeps);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_signm(const SignmMat *mats, int count, int n32, bool cplx, int32_t *status,
                        int max_sweeps, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    return cplx ? launch_signm_t<true>(mats, count, n32, status, max_sweeps, st)
                : launch_signm_t<false>(mats, count, n32, status, max_sweeps, st);
}

}  // namespace sgt
