// Kernels of the mixed-precision path with iterative refinement, for real
// entries (P = 1) and complex entries (P = 2: interleaved re, im).
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

// |z| of entry e (P planes at p[P * e + q]).
template <int P, typename S> __device__ inline double mag(const S *p, int64_t e)
{
    if constexpr (P == 1) {
        return fabs((double)p[e]);
    } else {
        return hypot((double)p[2 * e], (double)p[2 * e + 1]);
    }
}

#define REF_MAT(a) (a.mats ? gload(a.mats + blockIdx.z) : a.m0)

// A kernel of a refinement step the device decided against: nothing to do.
__device__ inline bool gated_off(const RefArgs &a) { return a.live && uniform(*a.live) == 0; }

// FP32 copies for the reduced-precision sweeps: the upper triangle of T, and
// the (FP64-computed) diagonal blocks of U; max |t_ij| on the side.  Matrix
// blockIdx.z of the table; columns strided over blockIdx.y.
template <int P> __global__ __launch_bounds__(NT) void k_to_f32(RefArgs a)
{
    __shared__ double red[NT / 64];
    const RefMat d = REF_MAT(a);
    double m = 0.0;
    for (int64_t j = blockIdx.y; j < d.n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i <= j;
             i += (int64_t)gridDim.x * NT) {
            const int64_t et = i + j * d.ldt, e32 = i + j * d.ld32, eu = i + j * d.ldu;
#pragma unroll
            for (int q = 0; q < P; ++q) gstore(d.T32 + P * e32 + q, (float)gload(d.T + P * et + q));
            m = fmax(m, mag<P>(d.T, et));
            if (d.split == 0 && i / TB == j / TB)
#pragma unroll
                for (int q = 0; q < P; ++q) gstore(d.U32 + P * e32 + q, (float)gload(d.U + P * eu + q));
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
template <int P> __global__ __launch_bounds__(NT) void k_widen(RefArgs a)
{
    __shared__ double red[NT / 64];
    const RefMat d = REF_MAT(a);
    double m = 0.0;
    for (int64_t j = blockIdx.y; j < d.n; j += gridDim.y) {
        const int64_t iend = region_rows(j, d.split);
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < iend;
             i += (int64_t)gridDim.x * NT) {
            const int64_t e32 = i + j * d.ld32, eu = i + j * d.ldu;
#pragma unroll
            for (int q = 0; q < P; ++q) gstore(d.U + P * eu + q, (double)gload(d.U32 + P * e32 + q));
            m = fmax(m, mag<P>(d.U32, e32));
        }
    }
    m = block_max(m, red);
    if (threadIdx.x == 0) atomic_max_nonneg(&d.maxes[1], m);
}

// U += E on the entries of the computed region; max |E| on the side.
template <int P> __global__ __launch_bounds__(NT) void k_add_correction(RefArgs a)
{
    __shared__ double red[NT / 64];
    if (gated_off(a)) return;
    const RefMat d = REF_MAT(a);
    double m = 0.0;
    for (int64_t j = blockIdx.y; j < d.n; j += gridDim.y) {
        const int64_t iend = region_rows(j, d.split);
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < iend;
             i += (int64_t)gridDim.x * NT) {
            const int64_t e32 = i + j * d.ld32, eu = i + j * d.ldu;
#pragma unroll
            for (int q = 0; q < P; ++q) d.U[P * eu + q] += (double)gload(d.E32 + P * e32 + q);
            m = fmax(m, mag<P>(d.E32, e32));
        }
    }
    m = block_max(m, red);
    if (threadIdx.x == 0) atomic_max_nonneg(&d.maxes[2], m);
}

__global__ void k_clear_correction_max(RefArgs a)
{
    if (gated_off(a)) return;
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z < a.nmat) (a.mats ? gload(a.mats + z) : a.m0).maxes[2] = 0;
}

// acc (P planes) += a * b for one MFMA operand pair (complex: four products)
template <int P>
__device__ inline void mac64(const double *a, const double *b, int ao, int bo, int as, int bs,
                             dx4 (&acc)[P])
{
    if constexpr (P == 1) {
        acc[0] = mfma_f64(a[ao], b[bo], acc[0]);
    } else {
        const double ar = a[ao], ai = a[as + ao], br = b[bo], bi = b[bs + bo];
        acc[0] = mfma_f64(ar, br, acc[0]);
        acc[0] = mfma_f64(-ai, bi, acc[0]);
        acc[1] = mfma_f64(ar, bi, acc[1]);
        acc[1] = mfma_f64(ai, br, acc[1]);
    }
}

// FP64 residual of one off-diagonal block per workgroup (tasks in reverse
// order: the longest products first).  Output: R as FP32 (the right-hand side
// of the correction sweep, into E32) and the block's squared Frobenius norm.
template <int P>
__global__ __launch_bounds__(NT) void k_resid(RefArgs a, const int2 *__restrict__ tasks,
                                              int ntasks, double *__restrict__ norm2)
{
    constexpr int AS = TB * APITCH, BS = (TB / 4) * BSLAB;  // plane strides
    __shared__ double sAU[P * AS], sAT[P * AS];
    __shared__ double sBU[P * BS], sBT[P * BS];
    __shared__ int8_t rs[TB], cs[TB];
    __shared__ double red[NT / 64];

    if (gated_off(a)) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pr = wave >> 1, pc = wave & 1;
    const int lc = tid >> 3, lr = (tid & 7) * 4;
    const int2 tk = gload(tasks + ntasks - 1 - (int)blockIdx.x);
    const RefMat d = a.mats ? gload(a.mats + uniform(tk.x)) : a.m0;
    const int I = uniform(tk.y >> 16), J = uniform(tk.y & 0xffff);
    const int64_t n = uniform(d.n);
    const double *T = d.T, *U = d.U;
    const int64_t ldt = d.ldt, ldu = d.ldu;
    const int64_t r0 = (int64_t)I * TB, c0 = (int64_t)J * TB;
    const int bj = (int)min((int64_t)TB, n - c0);
    if (tid < TB) {
        rs[tid] = gload(d.sgn + r0 + tid);
        cs[tid] = tid < bj ? gload(d.sgn + c0 + tid) : 0;
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

    dx4 accY[P], accX[P];
#pragma unroll
    for (int q = 0; q < P; ++q)
        for (int r = 0; r < 4; ++r) accY[q][r] = accX[q][r] = 0.0;

    double gaU[P][4], gaT[P][4], gbU[P][4], gbT[P][4];
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
#pragma unroll
            for (int q = 0; q < P; ++q) {
                gaU[q][e] = okA ? gload(U + P * (ra + ca * ldu) + q) : 0.0;
                gaT[q][e] = (okA && any_x) ? gload(T + P * (ra + ca * ldt) + q) : 0.0;
                gbU[q][e] = okB ? gload(U + P * (rb + cb * ldu) + q) : 0.0;
                gbT[q][e] = (okB && any_x) ? gload(T + P * (rb + cb * ldt) + q) : 0.0;
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sAU[q * AS + lc * APITCH + lr + e] = gaU[q][e];
                sAT[q * AS + lc * APITCH + lr + e] = -gaT[q][e];
                sBU[q * BS + (lr >> 2) * BSLAB + lc * 4 + e] = gbU[q][e];
                sBT[q * BS + (lr >> 2) * BSLAB + lc * 4 + e] = gbT[q][e];
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
            if (needY) mac64<P>(sAU, sBU, ao, bo, AS, BS, accY);
            if (needX) {
                mac64<P>(sAU, sBT, ao, bo, AS, BS, accX);
                mac64<P>(sAT, sBU, ao, bo, AS, BS, accX);
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
        const bool same = rs[i] == cs[j];
        if (j < bj) {
            const int64_t e = (r0 + i) + (c0 + j) * d.ld32;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const double v = same ? accY[q][r] : accX[q][r];
                gstore(d.E32 + P * e + q, (float)v);
                ss += v * v;
            }
        }
    }
    for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m, 64);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) norm2[d.f0 + (int64_t)I * d.nbc + J] = red[0] + red[1] + red[2] + red[3];
}

// FP64 residual of the real substitution form on 128 x 128 tiles: tile (a, b)
// covers blocks 4a .. 4a+3 x 4b .. 4b+3.  Eight waves; wave w owns the 32 x 64
// region at rows 32 (w >> 1), columns 64 (w & 1): two 32 x 32 blocks, 2 x 4
// MFMA pieces, each piece's products chosen by the signs of its rows and
// columns (U U for equal signs, U T - T U for opposite ones).  K runs over
// [128 a, 128 b + 128) in 16-deep stages with every operand masked to its upper
// triangle (row <= column), which zeroes the terms outside a block's own range
// I .. J and T's strict lower triangle; a piece skips the stages in which its
// operands are all zero.  Two LDS buffers: the next stage's operands are loaded
// into registers while the current one is multiplied, then stored into the
// other buffer, one barrier per stage.  Blocks outside the strict upper block
// triangle are skipped.  Output as k_resid: R in FP32 into E32, squared
// Frobenius norm per block.  Tiles in reverse task order (longest first).
constexpr int RT = 4 * TB;          // tile rows and columns
constexpr int RK = 16;              // K per stage
constexpr int RAP = RT + 16;        // LDS: A as [k][row], padded
constexpr int RBS = 4 * RT + 4;     // LDS: B as [k / 4][column][k % 4], padded
constexpr int NT8 = 512;

// YO: the entries of equal signs only (U^2 - I); the others come from
// k_resid_strip, which runs after this kernel (norm2 is assigned here and added
// to there).  T is then neither staged nor multiplied.
template <bool YO>
__global__ __launch_bounds__(NT8) void k_resid128(RefArgs a, const int2 *__restrict__ tiles,
                                                  int ntiles, double *__restrict__ norm2)
{
    constexpr int TS = YO ? 1 : 2;  // T's LDS stages
    __shared__ double sAU[2][RK * RAP], sAT[TS][YO ? 1 : RK * RAP];
    __shared__ double sBU[2][(RK / 4) * RBS], sBT[TS][YO ? 1 : (RK / 4) * RBS];
    __shared__ int8_t rs[RT], cs[RT];

    if (gated_off(a)) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    const int mg = lane >> 4, mt = lane & 15;
    const int2 tk = gload(tiles + ntiles - 1 - (int)blockIdx.x);
    const RefMat d = a.mats ? gload(a.mats + uniform(tk.x)) : a.m0;
    const int ta = uniform(tk.y >> 16), tb = uniform(tk.y & 0xffff);
    const int64_t n = uniform(d.n);
    const int nb = uniform(d.nbc);
    const double *T = d.T, *U = d.U;
    const int64_t ldt = d.ldt, ldu = d.ldu;
    const int64_t r0 = (int64_t)ta * RT, c0 = (int64_t)tb * RT;
    const int I = 4 * ta + wr, J0 = 4 * tb + 2 * wc;
    const bool mine[2] = {I < J0 && J0 < nb, I < J0 + 1 && J0 + 1 < nb};
    if (tid < RT) {
        rs[tid] = r0 + tid < n ? gload(d.sgn + r0 + tid) : 0;
        cs[tid] = c0 + tid < n ? gload(d.sgn + c0 + tid) : 0;
    }
    __syncthreads();
    // which products each 16 x 16 piece needs, as wave-uniform bit masks (bit
    // 4 ra + cb), so that the tests around the MFMAs are scalar branches
    int ym = 0, xm = 0;
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            bool rp = false, rn = false, cp = false, cn = false;
            for (int u = 0; u < 16; ++u) {
                const int vr = rs[32 * wr + 16 * ra + u], vc = cs[64 * wc + 16 * cb + u];
                rp |= vr > 0;
                rn |= vr < 0;
                cp |= vc > 0;
                cn |= vc < 0;
            }
            const bool m = mine[cb >> 1];
            if (m && ((rp && cp) || (rn && cn))) ym |= 1 << (4 * ra + cb);
            if (!YO && m && ((rp && cn) || (rn && cp))) xm |= 1 << (4 * ra + cb);
        }
    ym = uniform(ym);
    xm = YO ? 0 : uniform(xm);
    const bool any_x = YO ? false : __syncthreads_or(xm != 0);

    dx4 accY[2][4], accX[2][4];
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
            for (int r = 0; r < 4; ++r) accY[ra][cb][r] = accX[ra][cb][r] = 0.0;

    // staging of one stage: A 128 x 16 (U, T), B 16 x 128 (U, T); thread t loads
    // A rows t & 127 at k = 4 (t >> 7) .. + 3 and B column t >> 2 at k = 4 (t & 3) .. + 3
    const int arow = tid & (RT - 1), akh = tid >> 7;
    const int bcol = tid >> 2, bkq = tid & 3;
    double gaU[4], gaT[4], gbU[4], gbT[4];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t ra = r0 + arow, ka = k0 + 4 * akh + e;
            const int64_t kb = k0 + 4 * bkq + e, cb = c0 + bcol;
            const bool okA = ra < n && ka < n && ra <= ka;
            const bool okB = kb < n && cb < n && kb <= cb;
            gaU[e] = okA ? gload(U + ra + ka * ldu) : 0.0;
            gaT[e] = (okA && any_x) ? gload(T + ra + ka * ldt) : 0.0;
            gbU[e] = okB ? gload(U + kb + cb * ldu) : 0.0;
            gbT[e] = (okB && any_x) ? gload(T + kb + cb * ldt) : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            sAU[buf][(4 * akh + e) * RAP + arow] = gaU[e];
            sBU[buf][bkq * RBS + bcol * 4 + e] = gbU[e];
            if constexpr (!YO) {
                sAT[buf][(4 * akh + e) * RAP + arow] = -gaT[e];
                sBT[buf][bkq * RBS + bcol * 4 + e] = gbT[e];
            }
        }
    };
    const int64_t kbeg = r0, kend = min(n, c0 + RT);
    const int nst = uniform((int)((kend - kbeg + RK - 1) / RK));
    load(kbeg);
    store(0);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        const int64_t k0 = kbeg + (int64_t)s * RK;
        const bool more = s + 1 < nst;
        if (more) load(k0 + RK);
        // pieces with a nonzero term in this stage: A[i][k] needs i <= k, B[k][j] k <= j
        bool live[2][4];
#pragma unroll
        for (int ra = 0; ra < 2; ++ra)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                live[ra][cb] = r0 + 32 * wr + 16 * ra <= k0 + RK - 1 &&
                               c0 + 64 * wc + 16 * cb + 15 >= k0;
#pragma unroll
        for (int k4 = 0; k4 < RK / 4; ++k4) {
            double aU[2], aT[2], bU[4], bT[4];
#pragma unroll
            for (int ra = 0; ra < 2; ++ra) {
                const int ao = (4 * k4 + mg) * RAP + 32 * wr + 16 * ra + mt;
                aU[ra] = sAU[buf][ao];
                aT[ra] = YO ? 0.0 : sAT[YO ? 0 : buf][YO ? 0 : ao];
            }
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int bo = k4 * RBS + (64 * wc + 16 * cb + mt) * 4 + mg;
                bU[cb] = sBU[buf][bo];
                bT[cb] = YO ? 0.0 : sBT[YO ? 0 : buf][YO ? 0 : bo];
            }
#pragma unroll
            for (int ra = 0; ra < 2; ++ra)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    if (!live[ra][cb]) continue;
                    if (ym >> (4 * ra + cb) & 1) accY[ra][cb] = mfma_f64(aU[ra], bU[cb], accY[ra][cb]);
                    if (xm >> (4 * ra + cb) & 1) {
                        accX[ra][cb] = mfma_f64(aU[ra], bT[cb], accX[ra][cb]);
                        accX[ra][cb] = mfma_f64(aT[ra], bU[cb], accX[ra][cb]);
                    }
                }
        }
        if (more) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
        if (!mine[hb]) continue;  // uniform
        double ss = 0.0;
#pragma unroll
        for (int ra = 0; ra < 2; ++ra)
#pragma unroll
            for (int cbb = 0; cbb < 2; ++cbb) {
                const int cb = 2 * hb + cbb;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 32 * wr + 16 * ra + mfma64_row(lane, r);
                    const int j = 64 * wc + 16 * cb + mt;
                    if (c0 + j < n && (!YO || rs[i] == cs[j])) {
                        const double v = rs[i] == cs[j] ? accY[ra][cb][r] : accX[ra][cb][r];
                        gstore(d.E32 + (r0 + i) + (c0 + j) * d.ld32, (float)v);
                        ss += v * v;
                    }
                }
            }
        for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m, 64);
        if (lane == 0) norm2[d.f0 + (int64_t)I * d.nbc + J0 + hb] = ss;
    }
}

// FP64 residual (UT - TU)_ij of the entries whose signs differ, for a matrix
// with a small minority sign class, on its minority rows and columns.  A task
// (matrix, kind, group, tile start) takes 16 minority indices (minl[group ..
// group + 15], ascending, -1 past the class's end) and a 16-wide range of the
// other index:
//   kind 0: rows i of the range against the group's columns c (i majority);
//   kind 1: the group's rows r against columns j of the range (j majority).
// Each entry is a sum over k from its row to its column, formed as FP64 MFMA
// products (A = U or T on the piece's rows, B = T or U on its columns); the
// four waves take every fourth batch of K steps and add their pieces in LDS.
// Only entries in blocks above the diagonal are written (E32, and their squares
// added to norm2 of their 32 x 32 block).
constexpr int SKB = 8;  // K steps of 4 per batch of loads

// The minority rows and columns of a group (16 indices of minl), copied k-major
// so that the strips read them coalesced: for k < n and slot s (index x_s),
//   G[0][k][s] = U[x_s, k], G[1][k][s] = T[x_s, k]   (rows)
//   G[2][k][s] = T[k, x_s], G[3][k][s] = U[k, x_s]   (columns)
// (zero for a padding slot).  groups[g] = (matrix, unused, offset of G in
// doubles: low, high word); one workgroup per (group, 64 consecutive k).
__global__ __launch_bounds__(256) void k_resid_gather(RefArgs a, const int4 *__restrict__ groups,
                                                     const int *__restrict__ minl,
                                                     double *__restrict__ gbuf)
{
    if (gated_off(a)) return;
    const int4 gq = gload(groups + blockIdx.x);
    const RefMat d = a.mats ? gload(a.mats + uniform(gq.x)) : a.m0;
    const int64_t n = uniform(d.n);
    const int64_t k0 = (int64_t)blockIdx.y * 64;
    if (k0 >= n) return;
    double *G = gbuf + (((int64_t)(unsigned)gq.w << 32) | (unsigned)gq.z);
    const int s = threadIdx.x & 15;
    const int x = gload(minl + 16 * (int64_t)blockIdx.x + s);
    for (int e = threadIdx.x >> 4; e < 64; e += 16) {
        const int64_t k = k0 + e;
        if (k >= n) break;
        const bool ok = x >= 0;
        const double ru = ok ? gload(d.U + x + k * d.ldu) : 0.0;
        const double rt = ok ? gload(d.T + x + k * d.ldt) : 0.0;
        const double ct = ok ? gload(d.T + k + (int64_t)x * d.ldt) : 0.0;
        const double cu = ok ? gload(d.U + k + (int64_t)x * d.ldu) : 0.0;
        gstore(G + (0 * n + k) * 16 + s, ru);
        gstore(G + (1 * n + k) * 16 + s, rt);
        gstore(G + (2 * n + k) * 16 + s, ct);
        gstore(G + (3 * n + k) * 16 + s, cu);
    }
}

__global__ __launch_bounds__(256) void k_resid_strip(RefArgs a, const int4 *__restrict__ tasks,
                                                    int ntasks, const int *__restrict__ minl,
                                                    const int4 *__restrict__ groups,
                                                    const double *__restrict__ gbuf,
                                                    double *__restrict__ norm2)
{
    __shared__ double part[3][4][64];
    if (gated_off(a)) return;
    const int lane = threadIdx.x & 63, wave = uniform(threadIdx.x >> 6);
    const int mg = lane >> 4, mt = lane & 15;
    const int4 tk = gload(tasks + blockIdx.x);
    const RefMat d = a.mats ? gload(a.mats + uniform(tk.x)) : a.m0;
    const int kind = uniform(tk.y), gi = uniform(tk.z), t0 = uniform(tk.w);
    const int grp = 16 * gi;  // the group's first entry in minl
    const int4 gq = gload(groups + gi);
    const double *G = gbuf + (((int64_t)(unsigned)gq.w << 32) | (unsigned)gq.z);
    const int64_t n = uniform(d.n);
    const double *T = d.T, *U = d.U;
    const int64_t ldt = d.ldt, ldu = d.ldu;
    // the group's indices (ascending; -1 past the end): its first and last
    int gmin = gload(minl + grp), gmax = gmin;
    for (int u = 1; u < 16; ++u) {
        const int v = gload(minl + grp + u);
        if (v >= 0) gmax = v;
    }
    gmin = uniform(gmin);
    gmax = uniform(gmax);
    const int gl = gload(minl + grp + mt);  // this lane's column (kind 0) or row (kind 1)
    // K range, inclusive: from the piece's lowest row to its highest column
    const int64_t kbeg = kind == 0 ? t0 : gmin;
    const int64_t kend = kind == 0 ? gmax : min<int64_t>(n - 1, (int64_t)t0 + 15);
    const int nk4 = kend >= kbeg ? uniform((int)((kend - kbeg) / 4 + 1)) : 0;
    // this lane's A row and B column
    const int64_t ar = kind == 0 ? (int64_t)t0 + mt : (int64_t)gl;
    const int64_t bc = kind == 0 ? (int64_t)gl : (int64_t)t0 + mt;
    const bool arok = ar >= 0 && ar < n, bcok = bc >= 0 && bc < n;
    dx4 acc = dx4{0.0, 0.0, 0.0, 0.0};
    for (int s0 = SKB * wave; s0 < nk4; s0 += 4 * SKB) {
        double au[SKB], at[SKB], bt[SKB], bu[SKB];
#pragma unroll
        for (int q = 0; q < SKB; ++q) {
            const int64_t k = kbeg + 4 * (int64_t)(s0 + q) + mg;
            const bool in = s0 + q < nk4 && k <= kend;
            const bool oka = in && arok && k >= ar, okb = in && bcok && k <= bc;
            // (the group's rows or columns from G, the other side from U and T)
            if (kind == 0) {
                au[q] = oka ? gload(U + ar + k * ldu) : 0.0;
                at[q] = oka ? -gload(T + ar + k * ldt) : 0.0;
                bt[q] = okb ? gload(G + (2 * n + k) * 16 + mt) : 0.0;
                bu[q] = okb ? gload(G + (3 * n + k) * 16 + mt) : 0.0;
            } else {
                au[q] = oka ? gload(G + (0 * n + k) * 16 + mt) : 0.0;
                at[q] = oka ? -gload(G + (1 * n + k) * 16 + mt) : 0.0;
                bt[q] = okb ? gload(T + k + bc * ldt) : 0.0;
                bu[q] = okb ? gload(U + k + bc * ldu) : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < SKB; ++q) {
            acc = mfma_f64(au[q], bt[q], acc);
            acc = mfma_f64(at[q], bu[q], acc);
        }
    }
    // the four waves' pieces summed in a fixed order
    if (wave > 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) part[wave - 1][r][lane] = acc[r];
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = ((acc[r] + part[0][r][lane]) + part[1][r][lane]) + part[2][r][lane];
    // entry (row slot mg + 4 r, column slot mt)
    double colsum = 0.0;  // kind 0: this lane's column (one block column)
    double rowsum[4];     // kind 1: per row slot (one block row each)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rs = mg + 4 * r;
        const int64_t i = kind == 0 ? (int64_t)t0 + rs : (int64_t)gload(minl + grp + rs);
        const int64_t j = kind == 0 ? (int64_t)gl : (int64_t)t0 + mt;
        bool ok = i >= 0 && j >= 0 && i < n && j < n && (i >> 5) < (j >> 5);
        if (ok) ok = gload(d.sgn + i) != gload(d.sgn + j);
        const double v = acc[r];
        rowsum[r] = 0.0;
        if (ok) {
            gstore(d.E32 + i + j * d.ld32, (float)v);
            if (kind == 0) colsum += v * v;
            else rowsum[r] = v * v;
        }
    }
    if (kind == 0) {
        // lanes mt, mt + 16, mt + 32, mt + 48: the 16 rows (one block row) of column slot mt
        colsum += __shfl_xor(colsum, 16, 64);
        colsum += __shfl_xor(colsum, 32, 64);
        const int64_t i0 = t0, j = gl;
        if (mg == 0 && j >= 0 && i0 < n && (i0 >> 5) < (j >> 5) && colsum != 0.0)
            atomicAdd(norm2 + d.f0 + (i0 >> 5) * d.nbc + (j >> 5), colsum);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // the 16 columns (one block column) of row slot mg + 4 r
            const double v = group_sum<16>(rowsum[r]);
            const int64_t i = gload(minl + grp + mg + 4 * r), j0 = t0;
            if (mt == 0 && i >= 0 && j0 < n && v != 0.0)
                atomicAdd(norm2 + d.f0 + (i >> 5) * d.nbc + (j0 >> 5), v);
        }
    }
}

// FP64 residual of the Sylvester equation T11 X - X T22 = 2 s T12 for one
// block of X per workgroup: R = 2 s T12 - T11 X + X T22, with X = U(0:p, p:n).
// K steps: blocks K >= I of T11's rows (K = I keeps its upper triangle), then
// blocks K <= J of T22's columns (K = J likewise).
template <int P>
__global__ __launch_bounds__(NT) void k_resid_syl(RefArgs a, const int2 *__restrict__ tasks,
                                                  int ntasks, double *__restrict__ norm2)
{
    constexpr int AS = TB * APITCH, BS = (TB / 4) * BSLAB;
    __shared__ double sA[P * AS];
    __shared__ double sB[P * BS];
    __shared__ double red[NT / 64];

    if (gated_off(a)) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pr = wave >> 1, pc = wave & 1;
    const int lc = tid >> 3, lr = (tid & 7) * 4;
    const int2 tk = gload(tasks + ntasks - 1 - (int)blockIdx.x);
    const RefMat d = a.mats ? gload(a.mats + uniform(tk.x)) : a.m0;
    const int I = uniform(tk.y >> 16), J = uniform(tk.y & 0xffff);
    const int64_t n = uniform(d.n), p = uniform(d.split);
    const double *T = d.T, *U = d.U;
    const int64_t ldt = d.ldt, ldu = d.ldu;
    const int64_t r0 = (int64_t)I * TB, c0 = p + (int64_t)J * TB;

    dx4 acc[P];
#pragma unroll
    for (int q = 0; q < P; ++q)
        for (int r = 0; r < 4; ++r) acc[q][r] = 0.0;
    const int na = uniform(d.nbr) - I, nsteps = uniform(na + J + 1);
    double ga[P][4], gb[P][4];
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
#pragma unroll
            for (int q = 0; q < P; ++q) {
                ga[q][e] = okA ? sa * gload(pa + P * (ra + ca * lda) + q) : 0.0;
                gb[q][e] = okB ? gload(pb + P * (rb + cb * ldb) + q) : 0.0;
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sA[q * AS + lc * APITCH + lr + e] = ga[q][e];
                sB[q * BS + (lr >> 2) * BSLAB + lc * 4 + e] = gb[q][e];
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
            const int ao = (k4 * 4 + g) * APITCH + 16 * pr + tl;
            const int bo = k4 * BSLAB + (16 * pc + tl) * 4 + g;
            mac64<P>(sA, sB, ao, bo, AS, BS, acc);
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
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const double v = d.two_s * gload(T + P * (i + j * ldt) + q) + acc[q][r];
                gstore(d.E32 + P * (i + j * d.ld32) + q, (float)v);
                ss += v * v;
            }
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

// ---------------------------------------------------------------------------
// The refinement's decisions, on the device.
// ---------------------------------------------------------------------------

// One thread per block of the task list: converged, stalled, and whether another
// step is needed (as the host loop of the refinement would decide).
__global__ __launch_bounds__(256) void k_refine_decide(DecideArgs d)
{
    if (uniform(*d.live_in) == 0) return;  // this step did not run: nothing changes
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= d.ntasks) return;
    const int2 tk = d.tasks[t];
    const RefMat &m = d.mats[tk.x];
    const int I = tk.y >> 16, J = tk.y & 0xffff;
    const int64_t lf = (int64_t)I * m.nbc + J, f = m.f0 + lf;
    const double aprev = sqrt(d.prev[f]), a = sqrt(d.cur[f]);
    if (d.step == 1) d.rinit[f] = aprev;
    const double r0 = d.rinit[f];
    const double tmax = __longlong_as_double((long long)m.maxes[0]);
    const double umax = __longlong_as_double((long long)m.maxes[1]);
    // K blocks in each entry's residual products
    const bool syl = m.split > 0;
    const int kb = syl ? (m.nbr - I) + (J + 1) : (J - I + 1);
    // the rounding level of an FP64 residual block: kb * TB products per entry of
    // size up to umax * max(umax, tmax)
    const double floor_ = 0x1p-52 * (double)kb * TB * TB * umax * fmax(umax, tmax);
    const bool forced = d.force == -1 || (d.nmat == 1 && d.force > 0 && d.force - 1 == lf);
    const bool good = !forced && a <= fmax(floor_, d.conv * r0);
    d.ok[f] = good ? 1 : 0;
    const bool hop = d.hopeless[f] != 0 || (!good && (forced || a > d.stall * aprev));
    d.hopeless[f] = hop ? 1 : 0;
    if (!good && !hop) __hip_atomic_store(d.live_out, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// rowmin[fr0 + I] = min J over the blocks of row I that did not converge
// (initially INT_MAX), one thread per block.
__global__ __launch_bounds__(256) void k_refine_rowmin(ConeArgs c)
{
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= c.nph + c.nps) return;
    const int2 tk = c.tasks[t];
    const RefMat &m = c.mats[tk.x];
    const int I = tk.y >> 16, J = tk.y & 0xffff;
    if (!c.ok[m.f0 + (int64_t)I * m.nbc + J]) atomicMin(&c.rowmin[m.fr0 + I], J);
}

// Over the rows below, per matrix (one thread each): rowmin[I] = min over I' >= I.
// Block (I, J) is then recomputed iff J >= rowmin[I]: some block (I', J') with
// I' >= I and J' <= J did not converge, and (I, J) reads it, directly or through
// the blocks between.
__global__ __launch_bounds__(256) void k_refine_rowsuffix(ConeArgs c, int nmat)
{
    const int z = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (z >= nmat) return;
    const RefMat &m = c.mats[z];
    int *r = c.rowmin + m.fr0;
    for (int I = m.nbr - 2; I >= 0; --I) r[I] = min(r[I], r[I + 1]);
}

// The recomputation's task lists in the task lists' order (one workgroup of 1024
// threads, 1024 tasks at a time: ballot counts per wave, then the waves' counts
// in order), their lengths, and the blocks per matrix.
__global__ __launch_bounds__(1024) void k_refine_compact(ConeArgs c)
{
    __shared__ int wcnt[2][16];
    __shared__ int base[2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < 2) base[tid] = 0;
    __syncthreads();
    const int total = c.nph + c.nps;
    for (int start = 0; start < total; start += 1024) {
        const int t = start + tid;
        int keep = 0, part = 0;
        int2 tk = make_int2(0, 0);
        if (t < total) {
            tk = c.tasks[t];
            const RefMat &m = c.mats[tk.x];
            const int I = tk.y >> 16, J = tk.y & 0xffff;
            keep = J >= c.rowmin[m.fr0 + I];
            part = t < c.nph ? 0 : 1;
        }
        const uint64_t b0 = __builtin_amdgcn_ballot_w64(keep && part == 0);
        const uint64_t b1 = __builtin_amdgcn_ballot_w64(keep && part == 1);
        const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
        if (lane == 0) {
            wcnt[0][wv] = __popcll(b0);
            wcnt[1][wv] = __popcll(b1);
        }
        __syncthreads();
        if (keep) {
            int off = base[part];
            for (int w = 0; w < wv; ++w) off += wcnt[part][w];
            off += __popcll((part ? b1 : b0) & below);
            (part ? c.out_ps : c.out_ph)[off] = tk;
            atomicAdd((unsigned long long *)&c.nfb[tk.x], 1ull);
        }
        __syncthreads();
        if (tid < 2) {
            int sum = 0;
            for (int w = 0; w < 16; ++w) sum += wcnt[tid][w];
            base[tid] += sum;
        }
        __syncthreads();
    }
    if (tid < 2) c.cnt[tid] = base[tid];
}

}  // namespace

hipError_t launch_to_f32(const RefArgs &a, int64_t nmax, bool cplx, hipStream_t st)
{
    if (nmax <= 0 || a.nmat <= 0) return hipSuccess;
    if (cplx)
        hipLaunchKernelGGL(k_to_f32<2>, col_grid(nmax, a.nmat), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL(k_to_f32<1>, col_grid(nmax, a.nmat), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_widen(const RefArgs &a, int64_t nmax, bool cplx, hipStream_t st)
{
    if (nmax <= 0 || a.nmat <= 0) return hipSuccess;
    if (cplx)
        hipLaunchKernelGGL(k_widen<2>, col_grid(nmax, a.nmat), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL(k_widen<1>, col_grid(nmax, a.nmat), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_add_correction(const RefArgs &a, int64_t nmax, bool cplx, hipStream_t st)
{
    if (nmax <= 0 || a.nmat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_correction_max, dim3((a.nmat + 255) / 256), dim3(256), 0, st, a);
    if (cplx)
        hipLaunchKernelGGL(k_add_correction<2>, col_grid(nmax, a.nmat), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL(k_add_correction<1>, col_grid(nmax, a.nmat), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_resid128(const RefArgs &a, const int2 *tiles, int ntiles, double *norm2,
                           hipStream_t st, bool yonly)
{
    if (ntiles <= 0) return hipSuccess;
    if (yonly)
        hipLaunchKernelGGL(k_resid128<true>, dim3(ntiles), dim3(NT8), 0, st, a, tiles, ntiles, norm2);
    else
        hipLaunchKernelGGL(k_resid128<false>, dim3(ntiles), dim3(NT8), 0, st, a, tiles, ntiles, norm2);
    return hipGetLastError();
}

hipError_t launch_resid_strips(const RefArgs &a, const int4 *tasks, int ntasks, const int *minl,
                               const int4 *groups, int ngroups, int64_t nmax, double *gbuf,
                               double *norm2, hipStream_t st)
{
    if (ntasks <= 0 || ngroups <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_resid_gather, dim3(ngroups, (unsigned)((nmax + 63) / 64)), dim3(256), 0, st,
                       a, groups, minl, gbuf);
    hipLaunchKernelGGL(k_resid_strip, dim3(ntasks), dim3(256), 0, st, a, tasks, ntasks, minl, groups,
                       gbuf, norm2);
    return hipGetLastError();
}

hipError_t launch_resid(const RefArgs &a, bool syl, bool cplx, const int2 *tasks, int ntasks,
                        double *norm2, hipStream_t st)
{
    if (ntasks <= 0) return hipSuccess;
    const dim3 g(ntasks), b(NT);
    if (syl && cplx)
        hipLaunchKernelGGL(k_resid_syl<2>, g, b, 0, st, a, tasks, ntasks, norm2);
    else if (syl)
        hipLaunchKernelGGL(k_resid_syl<1>, g, b, 0, st, a, tasks, ntasks, norm2);
    else if (cplx)
        hipLaunchKernelGGL(k_resid<2>, g, b, 0, st, a, tasks, ntasks, norm2);
    else
        hipLaunchKernelGGL(k_resid<1>, g, b, 0, st, a, tasks, ntasks, norm2);
    return hipGetLastError();
}

hipError_t launch_refine_decide(const DecideArgs &d, hipStream_t st)
{
    if (d.ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine_decide, dim3((unsigned)((d.ntasks + 255) / 256)), dim3(256), 0, st,
                       d);
    return hipGetLastError();
}

hipError_t launch_refine_cone(const ConeArgs &c, int nmat, int64_t nrows, hipStream_t st)
{
    hipError_t r = launch_fill_int(c.rowmin, nrows, 0x7fffffff, st);
    if (r == hipSuccess) r = launch_fill_int(c.cnt, 2, 0, st);
    if (r == hipSuccess) r = launch_fill_int((int *)c.nfb, 2 * (int64_t)nmat, 0, st);
    if (r != hipSuccess) return r;
    const int total = c.nph + c.nps;
    if (total > 0)
        hipLaunchKernelGGL(k_refine_rowmin, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                           c);
    if (nmat > 0)
        hipLaunchKernelGGL(k_refine_rowsuffix, dim3((unsigned)((nmat + 255) / 256)), dim3(256), 0,
                           st, c, nmat);
    hipLaunchKernelGGL(k_refine_compact, dim3(1), dim3(1024), 0, st, c);
    return hipGetLastError();
}

}  // namespace sgt
