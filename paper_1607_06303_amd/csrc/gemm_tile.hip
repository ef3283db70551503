// Right-hand sides of the off-diagonal block equations as MFMA products
// (real FP64 or FP32), for every block (I, I + D) of one block superdiagonal.
//
// For block (I, J) and K strictly between them (Section 5: the accumulators
// X and Y of the block equations, filled by the products of Algorithm 6):
//   Y_IJ = sum_K U_IK U_KJ                      (entries with equal signs)
//   X_IJ = sum_K (U_IK T_KJ - T_IK U_KJ)        (entries with opposite signs)
// and, for the X entries, the terms of the equation that involve only the
// finished diagonal blocks, U_II T_IJ - T_IJ U_JJ.  Only the X or Y entries a
// 16 x 16 matrix-core piece contains are computed (the saving of the
// single-accumulator variant of Section 5.3, at MFMA granularity).
//
// The K blocks of block (I, J) on superdiagonal D are split by availability,
// with a lookahead L >= 2:
//   bulk:  K = I+L .. J-L, which only need superdiagonals <= D-L, so they are
//          computed L-1 superdiagonals ahead, beside the solves in between;
//   edge:  the other K (I < K < I+L or J-L < K < J), which need up to D-1.
// Grid: x = block of the superdiagonal, y = slice.  Bulk launches use slices
// 0 .. nmid-1 for the bulk K range and slice nmid for the diagonal-block terms
// (zeros when the block has no X entry); edge launches use one slice per edge
// K block, in increasing K.  Partial results go to
// Z[(x * nslices + y) * TB * TB + i * TB + j].
//
// Workgroup = one TB x TB output block (TB = 64 or 32); four waves each own a
// (TB/2) x (TB/2) quarter as 16 x 16 MFMA pieces.  K advances in stages of 32:
// the next stage's global loads go to registers before the current stage's
// MFMAs and to LDS after them.  LDS layouts: A as [k][m] with a padded row
// (conflict-free stores, two-way reads); B as [k/4][n][k%4] slabs with a
// padded slab pitch, so the 4 x 16 operand of one MFMA is 64 consecutive
// elements.
#include <algorithm>

#include "common.h"

namespace sgt {

namespace {

constexpr int KC = 32;               // K stage depth
constexpr int NTHR = 256;

template <typename F> struct mf;
template <> struct mf<double> {
    typedef dx4 acc;
    __device__ static acc mma(double a, double b, acc c) { return mfma_f64(a, b, c); }
    __device__ static int row(int lane, int r) { return mfma64_row(lane, r); }
};
template <> struct mf<float> {
    typedef fx4 acc;
    __device__ static acc mma(float a, float b, acc c) { return mfma_f32(a, b, c); }
    __device__ static int row(int lane, int r) { return mfma32_row(lane, r); }
};

enum { K_MID = 0, K_SPEC_I = 1, K_SPEC_J = 2 };

// Number of edge K blocks of superdiagonal D with lookahead L, and the s-th
// of them (increasing K) for block (I, J).
__host__ __device__ inline int wave_gemm_edge_slices_d(int D, int L)
{
    return D <= 1 ? 0 : (D - 1 < 2 * (L - 1) ? D - 1 : 2 * (L - 1));
}
__device__ inline int edge_block(int I, int J, int L, int s)
{
    const int lo = (L - 1 < J - I - 1) ? L - 1 : J - I - 1;
    if (s < lo) return I + 1 + s;
    const int hi0 = (J - L + 1 > I + L) ? J - L + 1 : I + L;
    return hi0 + (s - lo);
}

template <typename F, int TB>
__global__ __launch_bounds__(NTHR) void k_wave_gemm(const F *__restrict__ T, int64_t ldt,
                                                    const F *__restrict__ U, int64_t ldu,
                                                    int64_t n, const int8_t *__restrict__ sgn,
                                                    int D, int edge, int nmid_split, int L,
                                                    F *__restrict__ Z)
{
    typedef typename mf<F>::acc acc_t;
    constexpr int APITCH = TB + 16;          // A row pitch (elements)
    constexpr int BSLAB = 4 * TB + 4;        // B slab pitch (elements)
    constexpr int NA = TB * KC / NTHR;       // A elements per thread per stage
    constexpr int NB = KC * TB / NTHR;       // B elements per thread per stage
    constexpr int WQ = TB / 2;               // wave quarter edge
    constexpr int NBW = WQ / 16;             // MFMA pieces per quarter edge
    constexpr int AROWS = NTHR / TB;         // A: k rows covered per pass
    constexpr int BCOLS = NTHR / KC;         // B: columns covered per pass
    __shared__ F sAU[KC * APITCH], sAT[KC * APITCH];
    __shared__ F sBU[(KC / 4) * BSLAB], sBT[(KC / 4) * BSLAB];
    __shared__ int8_t rs[TB], cs[TB];
    __shared__ int tile_any_x;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int I = blockIdx.x, J = I + D, split = blockIdx.y;
    const int64_t r0 = (int64_t)I * TB, c0 = (int64_t)J * TB;
    const int bj = (int)min((int64_t)TB, n - c0);
    if (tid < TB) {
        rs[tid] = sgn[r0 + tid];
        cs[tid] = tid < bj ? sgn[c0 + tid] : 0;
    }
    if (tid == 0) tile_any_x = 0;
    __syncthreads();

    // which products each 16 x 16 piece needs: bit (NBW a + b)
    const int wr = (wave >> 1) * WQ, wc = (wave & 1) * WQ;
    int needY = 0, needX = 0;
    {
        bool rp[NBW], rn[NBW], cp[NBW], cn[NBW];
        for (int b = 0; b < NBW; ++b) {
            rp[b] = rn[b] = cp[b] = cn[b] = false;
            for (int t = 0; t < 16; ++t) {
                int vr = rs[wr + 16 * b + t];
                rp[b] |= vr > 0;
                rn[b] |= vr < 0;
                int vc = cs[wc + 16 * b + t];
                cp[b] |= vc > 0;
                cn[b] |= vc < 0;
            }
        }
        for (int a = 0; a < NBW; ++a)
            for (int b = 0; b < NBW; ++b) {
                if ((rp[a] && cp[b]) || (rn[a] && cn[b])) needY |= 1 << (NBW * a + b);
                if ((rp[a] && cn[b]) || (rn[a] && cp[b])) needX |= 1 << (NBW * a + b);
            }
    }
    if (needX && lane == 0) atomicOr(&tile_any_x, 1);
    __syncthreads();
    const bool any_x = tile_any_x != 0;

    acc_t accY[NBW][NBW], accX[NBW][NBW];
#pragma unroll
    for (int a = 0; a < NBW; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                accY[a][b][r] = 0;
                accX[a][b][r] = 0;
            }

    // stage list of this slice
    const bool special = !edge && split == nmid_split;
    const int nslices = edge ? wave_gemm_edge_slices_d(D, L) : nmid_split + 1;
    int kb = 0, ke = 0;
    if (edge) {
        kb = edge_block(I, J, L, split);
        ke = kb + 1;
    } else if (!special) {
        const int nmid = D - 2 * L + 1;  // K = I+L .. J-L
        const int chunk = (nmid + nmid_split - 1) / nmid_split;
        kb = I + L + split * chunk;
        ke = min(J - L + 1, kb + chunk);
    }
    constexpr int SPB = TB / KC;  // stages per K block
    const int n_mid_stages = ke > kb ? SPB * (ke - kb) : 0;
    const int n_spj = (bj + KC - 1) / KC;
    const int nstages = special ? (any_x ? SPB + n_spj : 0) : n_mid_stages;

    const int am = tid % TB, akq = tid / TB;   // A loads: row am, k = akq + AROWS p
    const int bkk = tid % KC, bjq = tid / KC;  // B loads: k = bkk, col = bjq + BCOLS p

    auto describe = [&](int s, int &kind, int64_t &kofs, int &klim) {
        if (!special) {
            kind = K_MID;
            kofs = (int64_t)(kb + s / SPB) * TB + (s % SPB) * KC;
            klim = KC;
        } else if (s < SPB) {
            kind = K_SPEC_I;  // A = U_II (columns of I), B = T_IJ (rows of I)
            kofs = r0 + s * KC;
            klim = KC;
        } else {
            kind = K_SPEC_J;  // A = T_IJ (columns of J), B = U_JJ (rows of J)
            const int kk0 = (s - SPB) * KC;
            kofs = c0 + kk0;
            klim = min(KC, bj - kk0);
        }
    };

    F gaU[NA], gaT[NA], gbU[NB], gbT[NB];

    auto load = [&](int s) {
        int kind, klim;
        int64_t kofs;
        describe(s, kind, kofs, klim);
        const bool wantAU = kind != K_SPEC_J;
        const bool wantAT = (kind == K_MID && any_x) || kind == K_SPEC_J;
        const bool wantBU = kind != K_SPEC_I;
        const bool wantBT = (kind == K_MID && any_x) || kind == K_SPEC_I;
#pragma unroll
        for (int p = 0; p < NA; ++p) {
            const int k = akq + AROWS * p;
            const bool ok = k < klim;
            const int64_t col = kofs + k;
            gaU[p] = (wantAU && ok) ? U[(r0 + am) + col * ldu] : (F)0;
            gaT[p] = (wantAT && ok) ? T[(r0 + am) + col * ldt] : (F)0;
        }
#pragma unroll
        for (int p = 0; p < NB; ++p) {
            const int j = bjq + BCOLS * p;
            const bool ok = (j < bj) && (bkk < klim);
            const int64_t row = kofs + bkk;
            gbU[p] = (wantBU && ok) ? U[row + (c0 + j) * ldu] : (F)0;
            gbT[p] = (wantBT && ok) ? T[row + (c0 + j) * ldt] : (F)0;
        }
    };

    auto store = [&]() {
#pragma unroll
        for (int p = 0; p < NA; ++p) {
            const int k = akq + AROWS * p;
            sAU[k * APITCH + am] = gaU[p];
            if (any_x) sAT[k * APITCH + am] = -gaT[p];  // stored negated: -T_IK U_KJ
        }
#pragma unroll
        for (int p = 0; p < NB; ++p) {
            const int j = bjq + BCOLS * p;
            const int off = (bkk >> 2) * BSLAB + j * 4 + (bkk & 3);
            sBU[off] = gbU[p];
            if (any_x) sBT[off] = gbT[p];
        }
    };

    auto compute = [&](int s) {
        int kind, klim;
        int64_t kofs;
        describe(s, kind, kofs, klim);
        const int g = lane >> 4, t = lane & 15;
#pragma unroll
        for (int k4 = 0; k4 < KC / 4; ++k4) {
            F aU[NBW], aT[NBW], bU[NBW], bT[NBW];
#pragma unroll
            for (int a = 0; a < NBW; ++a) {
                aU[a] = sAU[(k4 * 4 + g) * APITCH + wr + 16 * a + t];
                bU[a] = sBU[k4 * BSLAB + (wc + 16 * a + t) * 4 + g];
                if (any_x) {
                    aT[a] = sAT[(k4 * 4 + g) * APITCH + wr + 16 * a + t];
                    bT[a] = sBT[k4 * BSLAB + (wc + 16 * a + t) * 4 + g];
                } else {
                    aT[a] = 0;
                    bT[a] = 0;
                }
            }
#pragma unroll
            for (int a = 0; a < NBW; ++a)
#pragma unroll
                for (int b = 0; b < NBW; ++b) {
                    const int bit = 1 << (NBW * a + b);
                    if (kind == K_MID) {
                        if (needY & bit) accY[a][b] = mf<F>::mma(aU[a], bU[b], accY[a][b]);
                        if (needX & bit) {
                            accX[a][b] = mf<F>::mma(aU[a], bT[b], accX[a][b]);
                            accX[a][b] = mf<F>::mma(aT[a], bU[b], accX[a][b]);
                        }
                    } else if (kind == K_SPEC_I) {
                        if (needX & bit) accX[a][b] = mf<F>::mma(aU[a], bT[b], accX[a][b]);
                    } else {
                        if (needX & bit) accX[a][b] = mf<F>::mma(aT[a], bU[b], accX[a][b]);
                    }
                }
        }
    };

    if (nstages > 0) {
        load(0);
        store();
        __syncthreads();
        for (int s = 0; s < nstages; ++s) {
            const bool more = s + 1 < nstages;
            if (more) load(s + 1);
            compute(s);
            __syncthreads();
            if (more) {
                store();
                __syncthreads();
            }
        }
    }

    F *Zt = Z + ((int64_t)blockIdx.x * nslices + split) * TB * TB;
#pragma unroll
    for (int a = 0; a < NBW; ++a)
#pragma unroll
        for (int b = 0; b < NBW; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = wr + 16 * a + mf<F>::row(lane, r);
                const int j = wc + 16 * b + (lane & 15);
                Zt[i * TB + j] = (rs[i] == cs[j]) ? accY[a][b][r] : accX[a][b][r];
            }
}

}  // namespace

int wave_gemm_mid_splits(int D, int L, int ntiles, int max_splits, int64_t zslots)
{
    const int nmid = D - 2 * L + 1;  // bulk K blocks I+L .. J-L
    if (nmid <= 0) return 0;
    int s = (512 + ntiles - 1) / ntiles;
    s = std::min(s, nmid);
    s = std::min(s, max_splits > 0 ? max_splits : 16);
    s = std::max(s, 1);
    while ((int64_t)(s + 1) * ntiles > zslots && s > 1) --s;
    return s;
}

int wave_gemm_edge_slices(int D, int L) { return wave_gemm_edge_slices_d(D, L); }

template <typename F>
hipError_t launch_wave_gemm(int tb, const F *T, int64_t ldt, const F *U, int64_t ldu, int64_t n,
                            const int8_t *sgn, int D, int ntiles, int edge, int nmid_split, int L,
                            F *Z, hipStream_t st)
{
    const int ny = edge ? wave_gemm_edge_slices_d(D, L) : nmid_split + 1;
    if (ny <= 0 || ntiles <= 0) return hipSuccess;
    if (tb == 64)
        hipLaunchKernelGGL((k_wave_gemm<F, 64>), dim3(ntiles, ny), dim3(NTHR), 0, st, T, ldt, U,
                           ldu, n, sgn, D, edge, nmid_split, L, Z);
    else if (tb == 32)
        hipLaunchKernelGGL((k_wave_gemm<F, 32>), dim3(ntiles, ny), dim3(NTHR), 0, st, T, ldt, U,
                           ldu, n, sgn, D, edge, nmid_split, L, Z);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template hipError_t launch_wave_gemm<double>(int, const double *, int64_t, const double *, int64_t,
                                             int64_t, const int8_t *, int, int, int, int, int,
                                             double *, hipStream_t);
template hipError_t launch_wave_gemm<float>(int, const float *, int64_t, const float *, int64_t,
                                            int64_t, const int8_t *, int, int, int, int, int,
                                            float *, hipStream_t);

}  // namespace sgt
