// Blocked Parlett-Higham sweep in FP64 (real: 64 x 64 blocks, complex: 32 x 32).
//
// With U and T cut into square blocks, block (I, J), I < J, satisfies (Section 5,
// the block equations behind Algorithms 4-6), entry by entry:
//   where sign(t_ii) == sign(t_jj) (from U^2 = I, Eq. (2) in block form):
//     (u_ii + u_jj) u_ij + sum_{k in I, k > i} u_ik u_kj + sum_{k in J, k < j} u_ik u_kj
//         = - Y_ij,            Y_IJ = sum_{I < K < J} U_IK U_KJ
//   where they differ (from TU = UT, Eq. (1) in block form):
//     (t_ii - t_jj) u_ij + sum_{k in I, k > i} t_ik u_kj - sum_{k in J, k < j} u_ik t_kj
//         = X_ij + (U_II T_IJ - T_IJ U_JJ)_ij,
//                              X_IJ = sum_{I < K < J} (U_IK T_KJ - T_IK U_KJ)
// The left-hand sides involve only the block being solved and the diagonal
// blocks; the right-hand sides are block products of finished blocks.
//
// Blocks are finished in order of their block superdiagonal D = J - I (every
// block of diagonal D depends only on diagonals < D).  One sweep step is
//   1. k_gemm_*:  the right-hand side of every block on diagonal D, as MFMA
//                 products, only the X or Y entries each 16 x 16 piece needs
//                 (the arithmetic saving of the single-accumulator variant of
//                 Section 5.3, kept at matrix-core granularity), split over K
//                 into partial sums when the diagonal has few blocks;
//   2. k_solve_*: each block's own equations, entry by entry along
//                 anti-diagonals from its bottom-left corner.
// Diagonal blocks come first, all at once (k_diag_tiles): a diagonal block of
// sign(T) is the sign of the diagonal block of T (Algorithm 5 computes both
// halves before the off-diagonal part), by Algorithm 3 along superdiagonals.
#include <algorithm>

#include "common.h"

namespace sgt {

namespace {

constexpr int kThreads = 256;

template <typename S> __device__ inline S ldg_or_zero(const S *p, bool ok)
{
    return ok ? *p : scalar_traits<S>::zero();
}

// ---------------------------------------------------------------------------
// Diagonal blocks: Algorithm 3 on one TB x TB block, superdiagonal by
// superdiagonal; LPE lanes share each entry's inner product.
// ---------------------------------------------------------------------------
template <typename S, int TB>
__global__ __launch_bounds__(kThreads) void k_diag_tiles(const S *__restrict__ T, int64_t ldt,
                                                         S *__restrict__ U, int64_t ldu,
                                                         int64_t n, const int8_t *__restrict__ sgn)
{
    using tr = scalar_traits<S>;
    constexpr int LD = TB + 1;
    constexpr int LPE = kThreads / TB;
    __shared__ S sT[TB * LD];
    __shared__ S sU[TB * LD];
    __shared__ int8_t ss[TB];
    const int64_t r0 = (int64_t)blockIdx.x * TB;
    const int bt = (int)min((int64_t)TB, n - r0);
    for (int e = threadIdx.x; e < TB * TB; e += kThreads) {
        int i = e % TB, j = e / TB;
        bool in = (i < bt && j < bt);
        sT[i + j * LD] = ldg_or_zero(T + (r0 + i) + (r0 + j) * ldt, in && i <= j);
        sU[i + j * LD] = (in && i == j) ? tr::from_real((double)sgn[r0 + i]) : tr::zero();
    }
    if (threadIdx.x < TB) ss[threadIdx.x] = threadIdx.x < bt ? sgn[r0 + threadIdx.x] : 1;
    __syncthreads();
    const int i = threadIdx.x / LPE, q = threadIdx.x % LPE;
    for (int d = 1; d < bt; ++d) {
        const int j = i + d;
        if (j < bt) {
            const int si = ss[i], sj = ss[j];
            S sum = tr::zero();
            if (si + sj == 0) {
                for (int k = i + 1 + q; k < j; k += LPE)
                    sum = sum + (sU[i + k * LD] * sT[k + j * LD] - sT[i + k * LD] * sU[k + j * LD]);
            } else {
                for (int k = i + 1 + q; k < j; k += LPE) sum = sum + sU[i + k * LD] * sU[k + j * LD];
            }
#pragma unroll
            for (int m = 1; m < LPE; m <<= 1) sum = sum + tr::shfl_xor(sum, m);
            if (q == 0) {
                S u;
                if (si + sj == 0) {
                    // Eq. (1)
                    S den = sT[i + i * LD] - sT[j + j * LD];
                    u = sT[i + j * LD] * (double)(si - sj) / den + sum / den;
                } else {
                    // Eq. (2); -1/(u_ii + u_jj) = -+1/2 is exact
                    u = sum * (-1.0 / (double)(si + sj));
                }
                sU[i + j * LD] = u;
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TB * TB; e += kThreads) {
        int ii = e % TB, jj = e / TB;
        if (ii < bt && jj < bt) U[(r0 + ii) + (r0 + jj) * ldu] = sU[ii + jj * LD];
    }
}

// Sign summaries of the 16-wide row and column groups of block (I, J).
struct GroupSigns {
    bool pos, neg;
};

__device__ inline GroupSigns group_signs(const int8_t *s, int g0, int lim)
{
    GroupSigns r{false, false};
    for (int t = 0; t < 16; ++t) {
        if (g0 + t >= lim) break;
        int v = s[g0 + t];
        r.pos |= v > 0;
        r.neg |= v < 0;
    }
    return r;
}

enum KKind { K_MID = 0, K_SPEC_I = 1, K_SPEC_J = 2 };

// ---------------------------------------------------------------------------
// Right-hand sides of diagonal D, real FP64, 64 x 64 blocks.  Wave w owns the
// 32 x 32 quarter (w / 2, w % 2) as 2 x 2 MFMA pieces of 16 x 16.
// Block (I, J) = (I0 + blockIdx.x, I + D); blockIdx.y is the K split.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_gemm_r64(const double *__restrict__ T, int64_t ldt,
                                                       const double *__restrict__ U, int64_t ldu,
                                                       int64_t n, const int8_t *__restrict__ sgn,
                                                       int D, int I0, int nsplit,
                                                       double *__restrict__ Z)
{
    constexpr int TB = 64, KC = 16, LDB = TB + 1;
    __shared__ double sAU[KC][TB];
    __shared__ double sAT[KC][TB];
    __shared__ double sBU[KC][LDB];
    __shared__ double sBT[KC][LDB];
    __shared__ int8_t rs[TB], cs[TB];
    __shared__ int tile_any_x;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int I = I0 + blockIdx.x, J = I + D, split = blockIdx.y;
    const int64_t r0 = (int64_t)I * TB, c0 = (int64_t)J * TB;
    const int bj = (int)min((int64_t)TB, n - c0);
    if (tid < TB) {
        rs[tid] = sgn[r0 + tid];
        cs[tid] = tid < bj ? sgn[c0 + tid] : 0;
    }
    if (tid == 0) tile_any_x = 0;
    __syncthreads();

    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    bool needY[2][2], needX[2][2];
    bool wave_x = false;
    {
        GroupSigns rg[2], cg[2];
        for (int b = 0; b < 2; ++b) {
            rg[b] = group_signs(rs, wr + 16 * b, TB);
            cg[b] = group_signs(cs, wc + 16 * b, bj);
        }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                needY[a][b] = (rg[a].pos && cg[b].pos) || (rg[a].neg && cg[b].neg);
                needX[a][b] = (rg[a].pos && cg[b].neg) || (rg[a].neg && cg[b].pos);
                wave_x |= needX[a][b];
            }
    }
    if (wave_x && lane == 0) atomicOr(&tile_any_x, 1);
    __syncthreads();
    const bool any_x = tile_any_x != 0;

    dx4 accY[2][2], accX[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            accY[a][b] = dx4{0, 0, 0, 0};
            accX[a][b] = dx4{0, 0, 0, 0};
        }

    const int nmid = D - 1;
    const int chunk = (nmid + nsplit - 1) / nsplit;
    const int kb = I + 1 + split * chunk;
    const int ke = min(J, kb + chunk);
    const bool specials = any_x && (split == nsplit - 1);

    // Thread roles for the global -> LDS copies.
    const int am = tid & 63, akq = tid >> 6;   // A: row am, k = akq + 4t
    const int bkk = tid & 15, bjq = tid >> 4;  // B: k = bkk, col = bjq + 16t

    auto run = [&](int kind, int K) {
        // A operand columns / B operand rows in global index space.
        int64_t acol = 0, brow = 0;
        int klim = TB;
        if (kind == K_MID) {
            acol = (int64_t)K * TB;
            brow = (int64_t)K * TB;
        } else if (kind == K_SPEC_I) {
            acol = r0;  // U_II
            brow = r0;  // T_IJ
        } else {
            acol = c0;  // T_IJ
            brow = c0;  // U_JJ
            klim = bj;
        }
        for (int k0 = 0; k0 < klim; k0 += KC) {
            // A tiles
            for (int kk = akq; kk < KC; kk += 4) {
                bool ok = (k0 + kk) < klim;
                int64_t col = acol + k0 + kk;
                if (kind != K_SPEC_J) sAU[kk][am] = ldg_or_zero(U + (r0 + am) + col * ldu, ok);
                if ((kind == K_MID && any_x) || kind == K_SPEC_J)
                    sAT[kk][am] = ldg_or_zero(T + (r0 + am) + col * ldt, ok);
            }
            // B tiles
            for (int j = bjq; j < TB; j += 16) {
                bool ok = (j < bj) && (k0 + bkk) < klim;
                int64_t row = brow + k0 + bkk;
                if (kind != K_SPEC_I) sBU[bkk][j] = ldg_or_zero(U + row + (c0 + j) * ldu, ok);
                if ((kind == K_MID && any_x) || kind == K_SPEC_I)
                    sBT[bkk][j] = ldg_or_zero(T + row + (c0 + j) * ldt, ok);
            }
            __syncthreads();
#pragma unroll
            for (int k4 = 0; k4 < KC / 4; ++k4) {
                const int kr = k4 * 4 + (lane >> 4);
                double aU[2], aT[2], bU[2], bT[2];
                for (int a = 0; a < 2; ++a) {
                    aU[a] = sAU[kr][wr + 16 * a + (lane & 15)];
                    aT[a] = -sAT[kr][wr + 16 * a + (lane & 15)];
                    bU[a] = sBU[kr][wc + 16 * a + (lane & 15)];
                    bT[a] = sBT[kr][wc + 16 * a + (lane & 15)];
                }
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        if (kind == K_MID) {
                            if (needY[a][b]) accY[a][b] = mfma_f64(aU[a], bU[b], accY[a][b]);
                            if (needX[a][b]) {
                                accX[a][b] = mfma_f64(aU[a], bT[b], accX[a][b]);
                                accX[a][b] = mfma_f64(aT[a], bU[b], accX[a][b]);
                            }
                        } else if (kind == K_SPEC_I) {
                            if (needX[a][b]) accX[a][b] = mfma_f64(aU[a], bT[b], accX[a][b]);
                        } else {
                            if (needX[a][b]) accX[a][b] = mfma_f64(aT[a], bU[b], accX[a][b]);
                        }
                    }
            }
            __syncthreads();
        }
    };

    for (int K = kb; K < ke; ++K) run(K_MID, K);
    if (specials) {
        run(K_SPEC_I, I);
        run(K_SPEC_J, J);
    }

    double *Zt = Z + ((int64_t)blockIdx.x * nsplit + split) * TB * TB;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 4; ++r) {
                int i = wr + 16 * a + mfma64_row(lane, r);
                int j = wc + 16 * b + (lane & 15);
                Zt[i * TB + j] = (rs[i] == cs[j]) ? accY[a][b][r] : accX[a][b][r];
            }
}

// ---------------------------------------------------------------------------
// Right-hand sides of diagonal D, complex128, 32 x 32 blocks: wave w owns the
// 16 x 16 piece (w / 2, w % 2); each complex product is four real MFMAs.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_gemm_c128(const cd *__restrict__ T, int64_t ldt,
                                                        const cd *__restrict__ U, int64_t ldu,
                                                        int64_t n, const int8_t *__restrict__ sgn,
                                                        int D, int I0, int nsplit,
                                                        cd *__restrict__ Z)
{
    constexpr int TB = 32, KC = 16, LDB = TB + 1;
    __shared__ double sAUr[KC][TB], sAUi[KC][TB], sATr[KC][TB], sATi[KC][TB];
    __shared__ double sBUr[KC][LDB], sBUi[KC][LDB], sBTr[KC][LDB], sBTi[KC][LDB];
    __shared__ int8_t rs[TB], cs[TB];
    __shared__ int tile_any_x;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int I = I0 + blockIdx.x, J = I + D, split = blockIdx.y;
    const int64_t r0 = (int64_t)I * TB, c0 = (int64_t)J * TB;
    const int bj = (int)min((int64_t)TB, n - c0);
    if (tid < TB) {
        rs[tid] = sgn[r0 + tid];
        cs[tid] = tid < bj ? sgn[c0 + tid] : 0;
    }
    if (tid == 0) tile_any_x = 0;
    __syncthreads();
    const int wr = (wave >> 1) * 16, wc = (wave & 1) * 16;
    GroupSigns rg = group_signs(rs, wr, TB), cg = group_signs(cs, wc, bj);
    const bool needY = (rg.pos && cg.pos) || (rg.neg && cg.neg);
    const bool needX = (rg.pos && cg.neg) || (rg.neg && cg.pos);
    if (needX && lane == 0) atomicOr(&tile_any_x, 1);
    __syncthreads();
    const bool any_x = tile_any_x != 0;

    dx4 yR = {0, 0, 0, 0}, yI = {0, 0, 0, 0}, xR = {0, 0, 0, 0}, xI = {0, 0, 0, 0};
    const int nmid = D - 1;
    const int chunk = (nmid + nsplit - 1) / nsplit;
    const int kb = I + 1 + split * chunk;
    const int ke = min(J, kb + chunk);
    const bool specials = any_x && (split == nsplit - 1);
    const int am = tid & 31, akq = tid >> 5;   // A: row am, k = akq + 8t
    const int bkk = tid & 15, bjq = tid >> 4;  // B: k = bkk, col = bjq + 16t

    auto run = [&](int kind, int K) {
        int64_t acol = 0, brow = 0;
        int klim = TB;
        if (kind == K_MID) {
            acol = (int64_t)K * TB;
            brow = (int64_t)K * TB;
        } else if (kind == K_SPEC_I) {
            acol = r0;
            brow = r0;
        } else {
            acol = c0;
            brow = c0;
            klim = bj;
        }
        for (int k0 = 0; k0 < klim; k0 += KC) {
            for (int kk = akq; kk < KC; kk += 8) {
                bool ok = (k0 + kk) < klim;
                int64_t col = acol + k0 + kk;
                if (kind != K_SPEC_J) {
                    cd v = ldg_or_zero(U + (r0 + am) + col * ldu, ok);
                    sAUr[kk][am] = v.re;
                    sAUi[kk][am] = v.im;
                }
                if ((kind == K_MID && any_x) || kind == K_SPEC_J) {
                    cd v = ldg_or_zero(T + (r0 + am) + col * ldt, ok);
                    sATr[kk][am] = v.re;
                    sATi[kk][am] = v.im;
                }
            }
            for (int j = bjq; j < TB; j += 16) {
                bool ok = (j < bj) && (k0 + bkk) < klim;
                int64_t row = brow + k0 + bkk;
                if (kind != K_SPEC_I) {
                    cd v = ldg_or_zero(U + row + (c0 + j) * ldu, ok);
                    sBUr[bkk][j] = v.re;
                    sBUi[bkk][j] = v.im;
                }
                if ((kind == K_MID && any_x) || kind == K_SPEC_I) {
                    cd v = ldg_or_zero(T + row + (c0 + j) * ldt, ok);
                    sBTr[bkk][j] = v.re;
                    sBTi[bkk][j] = v.im;
                }
            }
            __syncthreads();
#pragma unroll
            for (int k4 = 0; k4 < KC / 4; ++k4) {
                const int kr = k4 * 4 + (lane >> 4);
                const int ai = wr + (lane & 15), bi = wc + (lane & 15);
                double aUr = sAUr[kr][ai], aUi = sAUi[kr][ai];
                double aTr = -sATr[kr][ai], aTi = -sATi[kr][ai];
                double bUr = sBUr[kr][bi], bUi = sBUi[kr][bi];
                double bTr = sBTr[kr][bi], bTi = sBTi[kr][bi];
                if (kind == K_MID && needY) {
                    yR = mfma_f64(aUr, bUr, yR);
                    yR = mfma_f64(-aUi, bUi, yR);
                    yI = mfma_f64(aUr, bUi, yI);
                    yI = mfma_f64(aUi, bUr, yI);
                }
                if (needX && (kind == K_MID || kind == K_SPEC_I)) {
                    xR = mfma_f64(aUr, bTr, xR);
                    xR = mfma_f64(-aUi, bTi, xR);
                    xI = mfma_f64(aUr, bTi, xI);
                    xI = mfma_f64(aUi, bTr, xI);
                }
                if (needX && (kind == K_MID || kind == K_SPEC_J)) {
                    xR = mfma_f64(aTr, bUr, xR);
                    xR = mfma_f64(-aTi, bUi, xR);
                    xI = mfma_f64(aTr, bUi, xI);
                    xI = mfma_f64(aTi, bUr, xI);
                }
            }
            __syncthreads();
        }
    };

    for (int K = kb; K < ke; ++K) run(K_MID, K);
    if (specials) {
        run(K_SPEC_I, I);
        run(K_SPEC_J, J);
    }
    cd *Zt = Z + ((int64_t)blockIdx.x * nsplit + split) * TB * TB;
    for (int r = 0; r < 4; ++r) {
        int i = wr + mfma64_row(lane, r);
        int j = wc + (lane & 15);
        bool same = rs[i] == cs[j];
        Zt[i * TB + j] = same ? cd{yR[r], yI[r]} : cd{xR[r], xI[r]};
    }
}

// ---------------------------------------------------------------------------
// Block solve for diagonal D: each block's own equations (see top of file),
// entry by entry along anti-diagonals from the bottom-left corner.  Row i of
// the block is handled by LPR lanes; at step a it owns entry (i, a - (TB-1-i)).
// Diagonal blocks are kept packed: U_II, T_II row-wise (rows read), U_JJ, T_JJ
// column-wise (columns read).
// ---------------------------------------------------------------------------
template <typename S, int TB>
__global__ __launch_bounds__(kThreads) void k_solve(const S *__restrict__ T, int64_t ldt,
                                                    S *__restrict__ U, int64_t ldu, int64_t n,
                                                    const int8_t *__restrict__ sgn, int D, int I0,
                                                    int nsplit, const S *__restrict__ Z)
{
    using tr = scalar_traits<S>;
    constexpr int LD = TB + 1;
    constexpr int LPR = kThreads / TB;
    constexpr int P = TB * (TB + 1) / 2;
    __shared__ S Lu[P], Lt[P], Ru[P], Rt[P];
    __shared__ S X[TB * LD];
    __shared__ S dI[TB], dJ[TB];
    __shared__ int8_t rs[TB], cs[TB];

    const int tid = threadIdx.x;
    const int I = I0 + blockIdx.x, J = I + D;
    const int64_t r0 = (int64_t)I * TB, c0 = (int64_t)J * TB;
    const int bj = (int)min((int64_t)TB, n - c0);
    // packed row-major upper: row i starts at i*TB - i*(i-1)/2, entry (i,k) at +k-i
    // packed column-major upper: column j starts at j*(j+1)/2, entry (k,j) at +k
    for (int e = tid; e < TB * TB; e += kThreads) {
        int i = e % TB, j = e / TB;
        if (i <= j) {
            int pr = i * TB - (i * (i - 1)) / 2 + (j - i);
            Lu[pr] = U[(r0 + i) + (r0 + j) * ldu];
            Lt[pr] = T[(r0 + i) + (r0 + j) * ldt];
            bool in = j < bj;
            int pc = (j * (j + 1)) / 2 + i;
            Ru[pc] = ldg_or_zero(U + (c0 + i) + (c0 + j) * ldu, in);
            Rt[pc] = ldg_or_zero(T + (c0 + i) + (c0 + j) * ldt, in);
        }
    }
    if (tid < TB) {
        rs[tid] = sgn[r0 + tid];
        cs[tid] = tid < bj ? sgn[c0 + tid] : 1;
        dI[tid] = T[(r0 + tid) + (r0 + tid) * ldt];
        dJ[tid] = ldg_or_zero(T + (c0 + tid) + (c0 + tid) * ldt, tid < bj);
    }
    __syncthreads();

    const int i = tid / LPR, q = tid % LPR;
    const int rowstart = i * TB - (i * (i - 1)) / 2 - i;  // + k gives (i, k)
    const S *Zt = Z + (int64_t)blockIdx.x * nsplit * TB * TB + i * TB;
    const int steps = (TB - 1) + bj;
    for (int a = 0; a < steps; ++a) {
        const int j = a - (TB - 1 - i);
        if (j >= 0 && j < bj) {
            S rhs = tr::zero();
            if (q == 0)
                for (int s = 0; s < nsplit; ++s) rhs = rhs + Zt[(int64_t)s * TB * TB + j];
            const bool same = rs[i] == cs[j];
            const S *L = same ? Lu : Lt;
            const S *R = same ? Ru : Rt;
            const int colstart = (j * (j + 1)) / 2;
            S col = tr::zero(), row = tr::zero();
            for (int k = i + 1 + q; k < TB; k += LPR) col = col + L[rowstart + k] * X[k + j * LD];
            for (int k = q; k < j; k += LPR) row = row + X[i + k * LD] * R[colstart + k];
#pragma unroll
            for (int m = 1; m < LPR; m <<= 1) {
                col = col + tr::shfl_xor(col, m);
                row = row + tr::shfl_xor(row, m);
            }
            if (q == 0) {
                S u;
                if (same) u = (rhs + col + row) * (-0.5 * (double)rs[i]);
                else u = (rhs - col + row) / (dI[i] - dJ[j]);
                X[i + j * LD] = u;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < TB * TB; e += kThreads) {
        int ii = e % TB, jj = e / TB;
        if (jj < bj) U[(r0 + ii) + (c0 + jj) * ldu] = X[ii + jj * LD];
    }
}

constexpr int kTargetWorkgroups = 512;

int choose_splits(int D, int ntiles, int max_splits, int64_t zslots)
{
    int s = (kTargetWorkgroups + ntiles - 1) / ntiles;
    s = std::min(s, std::max(1, (D - 1) / 2));
    if (max_splits > 0) s = std::min(s, max_splits);
    s = std::max(s, 1);
    while ((int64_t)s * ntiles > zslots && s > 1) --s;
    return s;
}

// Algorithmic flops (Section 3 counting) of each launch family, from the host
// signs: a pair (i, j) with i < j costs 2 (equal signs) or 4 (opposite) real
// flops per k strictly between them; its k are split into those inside blocks
// I and J (solve kernels) and those in blocks strictly between (products).
struct FlopCounter {
    const int8_t *s;
    int64_t n;
    int tb;
    double c;  // 1 real, 4 complex

    void counts(int64_t i0, int len, int64_t &pos, int64_t &neg) const
    {
        pos = neg = 0;
        for (int t = 0; t < len; ++t) (s[i0 + t] > 0 ? pos : neg)++;
    }
    double gemm(int D) const
    {
        const int64_t nb = (n + tb - 1) / tb;
        double f = 0.0;
        for (int64_t I = 0; I + D < nb; ++I) {
            int64_t J = I + D;
            int bj = (int)std::min<int64_t>(tb, n - J * tb);
            int64_t rp, rn, cp, cn;
            counts(I * tb, tb, rp, rn);
            counts(J * tb, bj, cp, cn);
            double same = (double)(rp * cp + rn * cn), opp = (double)(rp * cn + rn * cp);
            f += (2.0 * same + 4.0 * opp) * (double)tb * (double)(D - 1);
        }
        return c * f;
    }
    double solve(int D) const
    {
        const int64_t nb = (n + tb - 1) / tb;
        double f = 0.0;
        for (int64_t I = 0; I + D < nb; ++I) {
            int64_t J = I + D;
            int bj = (int)std::min<int64_t>(tb, n - J * tb);
            for (int i = 0; i < tb; ++i)
                for (int j = 0; j < bj; ++j) {
                    double w = (double)((tb - 1 - i) + j);
                    f += (s[I * tb + i] == s[J * tb + j] ? 2.0 : 4.0) * w;
                }
        }
        return c * f;
    }
    double diag() const
    {
        double f = 0.0;
        for (int64_t r0 = 0; r0 < n; r0 += tb) {
            int bt = (int)std::min<int64_t>(tb, n - r0);
            for (int j = 0; j < bt; ++j)
                for (int i = 0; i < j; ++i)
                    f += (s[r0 + i] == s[r0 + j] ? 2.0 : 4.0) * (double)(j - i - 1);
        }
        return c * f;
    }
};

}  // namespace

int ph_tile_size(bool cplx) { return cplx ? 32 : 64; }

int64_t ph_zslots(int64_t n, bool cplx)
{
    int tb = ph_tile_size(cplx);
    int64_t nb = (n + tb - 1) / tb;
    return nb + kTargetWorkgroups + 64;
}

hipError_t run_ph_fp64(const PhArgs &a, bool cplx, hipStream_t st)
{
    const int tb = ph_tile_size(cplx);
    const int64_t nb = (a.n + tb - 1) / tb;
    const bool prof = prof_on() && a.hsgn;
    const FlopCounter fc{a.hsgn, a.n, tb, cplx ? 4.0 : 1.0};
    prof_begin(st);
    hipError_t e = launch_zero_lower(a.U, a.ldu, a.n, cplx, st);
    if (e != hipSuccess) return e;
    prof_end(st, PK_AUX, 0.0);
    prof_begin(st);
    if (cplx) {
        hipLaunchKernelGGL((k_diag_tiles<cd, 32>), dim3(nb), dim3(kThreads), 0, st,
                           (const cd *)a.T, a.ldt, (cd *)a.U, a.ldu, a.n, a.sgn);
    } else {
        hipLaunchKernelGGL((k_diag_tiles<double, 64>), dim3(nb), dim3(kThreads), 0, st,
                           (const double *)a.T, a.ldt, (double *)a.U, a.ldu, a.n, a.sgn);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_end(st, PK_DIAG, prof ? fc.diag() : 0.0);
    for (int D = 1; D < nb; ++D) {
        const int ntiles = (int)(nb - D);
        const int ns = (D == 1) ? 1 : choose_splits(D, ntiles, a.max_splits, a.zslots);
        prof_begin(st);
        if (cplx)
            hipLaunchKernelGGL(k_gemm_c128, dim3(ntiles, ns), dim3(kThreads), 0, st,
                               (const cd *)a.T, a.ldt, (const cd *)a.U, a.ldu, a.n, a.sgn, D, 0,
                               ns, (cd *)a.zbuf);
        else
            hipLaunchKernelGGL(k_gemm_r64, dim3(ntiles, ns), dim3(kThreads), 0, st,
                               (const double *)a.T, a.ldt, (const double *)a.U, a.ldu, a.n,
                               a.sgn, D, 0, ns, (double *)a.zbuf);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        prof_end(st, PK_GEMM, prof ? fc.gemm(D) : 0.0);
        prof_begin(st);
        if (cplx)
            hipLaunchKernelGGL((k_solve<cd, 32>), dim3(ntiles), dim3(kThreads), 0, st,
                               (const cd *)a.T, a.ldt, (cd *)a.U, a.ldu, a.n, a.sgn, D, 0, ns,
                               (const cd *)a.zbuf);
        else
            hipLaunchKernelGGL((k_solve<double, 64>), dim3(ntiles), dim3(kThreads), 0, st,
                               (const double *)a.T, a.ldt, (double *)a.U, a.ldu, a.n, a.sgn, D,
                               0, ns, (const double *)a.zbuf);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        prof_end(st, PK_SOLVE, prof ? fc.solve(D) : 0.0);
    }
    return hipSuccess;
}

}  // namespace sgt
