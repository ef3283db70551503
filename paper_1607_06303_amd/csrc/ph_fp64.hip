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

    // The products run over a sequence of 16-deep chunks: two per middle block K
    // in [kb, ke), then (the last split of a tile with X entries) two of each
    // diagonal-block term.  Chunk c + 1 is loaded into registers while chunk c is
    // multiplied from LDS.
    const int nmc = uniform(2 * max(0, ke - kb));
    const int nch = uniform(nmc + (specials ? 4 : 0));
    struct Chunk {
        int kind, klim, k0;
        int64_t acol, brow;
    };
    auto chunk_at = [&](int c) {
        Chunk d;
        if (c < nmc) {
            d.kind = K_MID;
            d.acol = d.brow = (int64_t)(kb + (c >> 1)) * TB;
            d.klim = TB;
        } else {
            const int sp = c - nmc;
            d.kind = sp < 2 ? K_SPEC_I : K_SPEC_J;
            d.acol = d.brow = d.kind == K_SPEC_I ? r0 : c0;
            d.klim = d.kind == K_SPEC_I ? TB : bj;
        }
        d.k0 = (c & 1) * KC;
        return d;
    };
    struct Regs {
        cd au[KC / 8], at[KC / 8], bu[TB / 16], bt[TB / 16];
    };
    auto load = [&](const Chunk &d, Regs &R) {
#pragma unroll
        for (int t = 0; t < KC / 8; ++t) {
            const int kk = akq + 8 * t;
            const bool ok = (d.k0 + kk) < d.klim;
            const int64_t col = d.acol + d.k0 + kk;
            R.au[t] = d.kind != K_SPEC_J ? ldg_or_zero(U + (r0 + am) + col * ldu, ok) : cd{0.0, 0.0};
            R.at[t] = ((d.kind == K_MID && any_x) || d.kind == K_SPEC_J)
                          ? ldg_or_zero(T + (r0 + am) + col * ldt, ok) : cd{0.0, 0.0};
        }
#pragma unroll
        for (int t = 0; t < TB / 16; ++t) {
            const int jj = bjq + 16 * t;
            const bool ok = (jj < bj) && (d.k0 + bkk) < d.klim;
            const int64_t row = d.brow + d.k0 + bkk;
            R.bu[t] = d.kind != K_SPEC_I ? ldg_or_zero(U + row + (c0 + jj) * ldu, ok) : cd{0.0, 0.0};
            R.bt[t] = ((d.kind == K_MID && any_x) || d.kind == K_SPEC_I)
                          ? ldg_or_zero(T + row + (c0 + jj) * ldt, ok) : cd{0.0, 0.0};
        }
    };
    auto store = [&](const Regs &R) {
#pragma unroll
        for (int t = 0; t < KC / 8; ++t) {
            const int kk = akq + 8 * t;
            sAUr[kk][am] = R.au[t].re;
            sAUi[kk][am] = R.au[t].im;
            sATr[kk][am] = R.at[t].re;
            sATi[kk][am] = R.at[t].im;
        }
#pragma unroll
        for (int t = 0; t < TB / 16; ++t) {
            const int jj = bjq + 16 * t;
            sBUr[bkk][jj] = R.bu[t].re;
            sBUi[bkk][jj] = R.bu[t].im;
            sBTr[bkk][jj] = R.bt[t].re;
            sBTi[bkk][jj] = R.bt[t].im;
        }
    };
    auto compute = [&](int kind) {
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
    };
    Regs cur, nxt;
    if (nch > 0) load(chunk_at(0), cur);
    for (int c = 0; c < nch; ++c) {
        __syncthreads();  // the previous chunk's products are done with LDS
        store(cur);
        __syncthreads();
        const int kind = chunk_at(c).kind;
        if (c + 1 < nch) load(chunk_at(c + 1), nxt);
        compute(kind);
        cur = nxt;
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
// The right-hand side (the sum of the K-split partial products) is staged in
// the block's LDS tile and each entry is overwritten by its solution.
// Diagonal blocks are kept packed: U_II, T_II row-wise (rows are read),
// U_JJ, T_JJ column-wise (columns are read); index 0 = U, 1 = T.
// ---------------------------------------------------------------------------
constexpr int kSolveThreads = 512;

template <typename S, int TB>
__global__ __launch_bounds__(kSolveThreads) void k_solve(const S *__restrict__ T, int64_t ldt,
                                                         S *__restrict__ U, int64_t ldu, int64_t n,
                                                         const int8_t *__restrict__ sgn, int D,
                                                         int I0, int nsplit,
                                                         const S *__restrict__ Z)
{
    using tr = scalar_traits<S>;
    constexpr int NT = kSolveThreads;
    constexpr int LD = TB + 1;
    constexpr int LPR = NT / TB;
    constexpr int P = TB * (TB + 1) / 2;
    __shared__ S sL[2 * P], sR[2 * P];
    __shared__ S X[TB * LD];
    __shared__ S dI[TB], dJ[TB];
    __shared__ int8_t rs[TB], cs[TB];

    const int tid = threadIdx.x;
    const int I = I0 + blockIdx.x, J = I + D;
    const int64_t r0 = (int64_t)I * TB, c0 = (int64_t)J * TB;
    const int bj = (int)min((int64_t)TB, n - c0);
    // packed row-major upper: row i starts at i*TB - i*(i-1)/2, entry (i,k) at +k-i
    // packed column-major upper: column j starts at j*(j+1)/2, entry (k,j) at +k
    for (int e = tid; e < TB * TB; e += NT) {
        int i = e % TB, j = e / TB;
        if (i <= j) {
            int pr = i * TB - (i * (i - 1)) / 2 + (j - i);
            sL[pr] = U[(r0 + i) + (r0 + j) * ldu];
            sL[P + pr] = T[(r0 + i) + (r0 + j) * ldt];
            bool in = j < bj;
            int pc = (j * (j + 1)) / 2 + i;
            sR[pc] = ldg_or_zero(U + (c0 + i) + (c0 + j) * ldu, in);
            sR[P + pc] = ldg_or_zero(T + (c0 + i) + (c0 + j) * ldt, in);
        }
    }
    // right-hand sides: partial products summed in split order
    const S *Zb = Z + (int64_t)blockIdx.x * nsplit * TB * TB;
    for (int e = tid; e < TB * TB; e += NT) {
        int i = e / TB, j = e % TB;
        S z = tr::zero();
        for (int s = 0; s < nsplit; ++s) z = z + Zb[(int64_t)s * TB * TB + e];
        X[i + j * LD] = z;
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
    const int steps = (TB - 1) + bj;
    for (int a = 0; a < steps; ++a) {
        const int j = a - (TB - 1 - i);
        if (j >= 0 && j < bj) {
            const bool same = rs[i] == cs[j];
            const int sel = same ? 0 : P;
            // Y: u = -(rhs + col + row) * s_i / 2;  X: u = (rhs - col + row) / (t_ii - t_jj)
            const S scale = same ? tr::from_real(-0.5 * (double)rs[i])
                                 : tr::from_real(1.0) / (dI[i] - dJ[j]);
            const double csign = same ? 1.0 : -1.0;
            const int colstart = (j * (j + 1)) / 2;
            // fixed trip counts with predication, so that all LDS loads of a
            // step are issued back to back
            S col = tr::zero(), row = tr::zero();
            S lv[TB / LPR], xv[TB / LPR];
#pragma unroll
            for (int t = 0; t < TB / LPR; ++t) {
                const int k = i + 1 + q + t * LPR;
                const int kk = k < TB ? k : TB - 1;
                lv[t] = k < TB ? sL[sel + rowstart + kk] : tr::zero();
                xv[t] = X[kk + j * LD];
            }
#pragma unroll
            for (int t = 0; t < TB / LPR; ++t) col = col + lv[t] * xv[t];
#pragma unroll
            for (int t = 0; t < TB / LPR; ++t) {
                const int k = q + t * LPR;
                const int kk = k < j ? k : 0;
                xv[t] = k < j ? X[i + kk * LD] : tr::zero();
                lv[t] = sR[sel + colstart + kk];
            }
#pragma unroll
            for (int t = 0; t < TB / LPR; ++t) row = row + xv[t] * lv[t];
            S tot = col * csign + row;
#pragma unroll
            for (int m = 1; m < LPR; m <<= 1) tot = tot + tr::shfl_xor(tot, m);
            if (q == 0) X[i + j * LD] = (X[i + j * LD] + tot) * scale;
        }
        __syncthreads();
    }
    for (int e = tid; e < TB * TB; e += NT) {
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

}  // namespace

int ph_tile_size(bool cplx, int requested)
{
    if (cplx) return 32;
    return requested == 64 ? 64 : 32;
}

int64_t ph_zslots(int64_t n, int tb)
{
    int64_t nb = (n + tb - 1) / tb;
    return 2 * nb + kTargetWorkgroups + 128;
}

hipError_t launch_diag_blocks(const double *T, int64_t ldt, double *U, int64_t ldu, int64_t n,
                              const int8_t *sgn, hipStream_t st)
{
    const int64_t nb = (n + 31) / 32;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_diag_tiles<double, 32>), dim3(nb), dim3(kThreads), 0, st, T, ldt, U, ldu,
                       n, sgn);
    return hipGetLastError();
}

hipError_t run_ph_fp64(const PhArgs &a, bool cplx, hipStream_t st)
{
    const int tb = a.tile;
    if (tb != 32 && tb != 64) return hipErrorInvalidValue;
    if (cplx && tb != 32) return hipErrorInvalidValue;
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
    } else if (tb == 64) {
        hipLaunchKernelGGL((k_diag_tiles<double, 64>), dim3(nb), dim3(kThreads), 0, st,
                           (const double *)a.T, a.ldt, (double *)a.U, a.ldu, a.n, a.sgn);
    } else {
        hipLaunchKernelGGL((k_diag_tiles<double, 32>), dim3(nb), dim3(kThreads), 0, st,
                           (const double *)a.T, a.ldt, (double *)a.U, a.ldu, a.n, a.sgn);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_end(st, PK_DIAG, prof ? fc.diag() : 0.0);
    if (!cplx) {
        RealSweep w;
        w.T = (const double *)a.T;
        w.ldt = a.ldt;
        w.U = (double *)a.U;
        w.ldu = a.ldu;
        w.n = a.n;
        w.sgn = a.sgn;
        w.zbuf[0] = (double *)a.zbuf;
        for (int b = 1; b < kLookahead; ++b) w.zbuf[b] = (double *)a.zbufs[b - 1];
        w.ebuf = (double *)a.ebuf;
        w.zslots = a.zslots;
        w.max_splits = a.max_splits;
        w.tile = tb;
        w.flops = prof ? &fc : nullptr;
        w.bulk_nm.assign(nb + 2, 0);
        return run_ph_real(w, st);
    }
    for (int D = 1; D < nb; ++D) {
        const int ntiles = (int)(nb - D);
        // ns K slices, the diagonal-block terms in the last one
        const int ns = (D == 1) ? 1 : choose_splits(D, ntiles, a.max_splits, a.zslots);
        prof_begin(st);
        hipLaunchKernelGGL(k_gemm_c128, dim3(ntiles, ns), dim3(kThreads), 0, st, (const cd *)a.T,
                           a.ldt, (const cd *)a.U, a.ldu, a.n, a.sgn, D, 0, ns, (cd *)a.zbuf);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        prof_end(st, PK_GEMM, prof ? fc.per_k_block(D) * (D - 1) : 0.0);
        prof_begin(st);
        hipLaunchKernelGGL((k_solve<cd, 32>), dim3(ntiles), dim3(kSolveThreads), 0, st,
                           (const cd *)a.T, a.ldt, (cd *)a.U, a.ldu, a.n, a.sgn, D, 0, ns,
                           (const cd *)a.zbuf);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        prof_end(st, PK_SOLVE, prof ? fc.solve(D) : 0.0);
    }
    return hipSuccess;
}

}  // namespace sgt
