// The Sylvester form for a diagonal whose signs are not grouped, without a
// Schur reordering.
//
// Section 3 makes the Parlett-Sylvester form apply to any inertia by reordering
// T (adjacent swaps by plane rotations) until the signs are grouped, solving the
// Sylvester equation T11 X - X T22 = 2 s T12 of the sign-split case (Algorithm 2
// with diagonal blocks +-I) and transforming back.  The swaps form a long serial
// chain of small rotations, so the same result is reached here through the
// invariant subspaces that the reordering exposes.  With m entries in the
// minority sign class, at rows b_0 < ... < b_{m-1}:
//
//   right basis Z (n x m):  T Z = Z L,   Z[b_l, :] = e_l,  Z[i, l] = 0 for i > b_l
//   left basis  W (n x m):  W^T T = L' W^T,  W[b_l, :] = e_l,  W[i, l] = 0 for i < b_l
//
// L and L' are upper triangular with the minority eigenvalues on the diagonal.
// The spectral projector of the minority eigenvalues is P = Z (W^T Z)^-1 W^T,
// W^T Z is unit upper triangular, and sign(T) = s (I - 2 P) with s the majority
// sign.  When the signs are already grouped, Z = [X; I] with X the solution of
// the sign-split Sylvester equation above, W = [0; I], and this is the
// Parlett-Sylvester form itself.
//
// Z is found by substitution from the bottom row up.  Row i of T Z = Z L reads
//   t_ii z_il + sum_{j>i} t_ij z_jl = sum_{l'} z_il' L[l', l],
// so at a minority row i = b_l0 it defines row l0 of L (z_i = e_l0), and at any
// other row it gives z_il from the columns l' < l of the same row (the L
// coupling) and the rows below:
//   z_il = (sum_{l'<l} z_il' L[l', l] - sum_{j>i} t_ij z_jl) / (t_ii - L[l, l]).
// The divisions are by differences of eigenvalues of opposite sign, the same
// divisions as Eq. (1).  W is Z of the flipped matrix J T^T J (J the reversal),
// which is upper triangular with the same diagonal in reverse order; it is
// read from T through the reversal, not copied.
//
// Kernels (real T):
//   k_proj_prep    minority rows and row types of both bases, from the signs;
//   k_proj_run     one persistent launch for both bases: a workgroup per
//                  basis runs the substitution above block by block (64 rows,
//                  bottom up) as a wavefront over waves of eight columns (wave w
//                  at row r1 - 1 - s + (w - wmin) at step s, wmin the wave of the
//                  first column not still zero in the block; the coupling among a
//                  wave's own columns solved in order within the wave; block
//                  operands in LDS), while the other workgroups keep acc, the
//                  sums over the rows below each block, up to date with FP64 MFMA
//                  products as the blocks are published (per-block flags);
//   k_proj_gram    partial sums of W^T Z over 64-row chunks (MFMA);
//   k_proj_gsum    W^T Z, the partials summed;
//   k_proj_minv    its inverse (unit upper triangular, m x m);
//   k_proj_a       A = Z (W^T Z)^-1;
//   k_proj_u       U = s (I - 2 A W^T) on the upper triangle, zeros below
//                  (FP64 MFMA, 64 x 64 output tiles).
// Complex T runs simpler kernels of the same structure (k_projc_*, below).
#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"

namespace sgt {

namespace {

constexpr int PM = kProjMaxMinority;  // minority columns: one lane each
constexpr int PB = 64;                // rows per front block
constexpr int AP = PM + 1;            // LDS pitch of the accumulated sums

struct ProjBasis {
    const double *T;      // T (column-major); the left basis reads it as J T^T J
    int64_t ldt;
    int flip;             // 1: entry (i, j) of this basis's matrix is T[n-1-j, n-1-i]
    double *Z;            // n x PM, leading dimension n
    double *acc;          // n x PM: sum over the rows below the current block
    const int *rowtype;   // n: minority column of row i, or -1
    const int *pos;       // PM: row of minority column l, or -1 (l >= m)
};

struct ProjArgs {
    ProjBasis b[2];
    int64_t n;
    int m;
};

// Lane src's double, as a value every lane holds.
__device__ inline double readlane_f64(double v, int src)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, src);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Offset of entry (i, j) of a basis's matrix in T: T itself, or J T^T J.
__device__ inline int64_t toff(const ProjBasis &B, int64_t n, int64_t i, int64_t j)
{
    return B.flip ? (n - 1 - j) + (n - 1 - i) * B.ldt : i + j * B.ldt;
}

// ---------------------------------------------------------------------------
// Minority rows of both bases from the signs (one workgroup).
// Basis 0 (T):      pos[l] = b_l,              rowtype[b_l] = l
// Basis 1 (J T^T J): pos[l] = n-1-b_{m-1-l},   rowtype[n-1-b_l] = m-1-l
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_proj_prep(const int8_t *__restrict__ sgn, int64_t n,
                                                    int minority, int m, int *__restrict__ rt0,
                                                    int *__restrict__ pos0, int *__restrict__ rt1,
                                                    int *__restrict__ pos1)
{
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t lo = std::min<int64_t>(n, t * per), hi = std::min<int64_t>(n, lo + per);
    int c = 0;
    for (int64_t i = lo; i < hi; ++i) c += sgn[i] == minority;
    part[t] = c;
    __syncthreads();
    // exclusive scan (Hillis-Steele over 1024 entries)
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int l = part[t] - c;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t f = n - 1 - i;
        if (sgn[i] == minority) {
            rt0[i] = l;
            pos0[l] = (int)i;
            rt1[f] = m - 1 - l;
            pos1[m - 1 - l] = (int)f;
            ++l;
        } else {
            rt0[i] = -1;
            rt1[f] = -1;
        }
    }
    for (int q = m + t; q < PM; q += 1024) {
        pos0[q] = -1;
        pos1[q] = -1;
    }
}

// ---------------------------------------------------------------------------
// 64 x 64 x 64 FP64 MFMA product of two LDS operands, 4 waves in a 2 x 2
// arrangement of 32 x 32 quarters: d[i][j] += sum_k A[k][i] B[k][j] with A
// and B stored k-major (pitches PA and PBB).
// ---------------------------------------------------------------------------
constexpr int OP = 65;

template <int PA, int PBB>
__device__ inline void mm64_acc(const double *As, const double *Bs, dx4 (&d)[2][2])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
    const int kr = lane >> 4, cc = lane & 15;
    for (int k = 0; k < 64; k += 4) {
        double av[2], bv[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) av[x] = As[(k + kr) * PA + rb + 16 * x + cc];
#pragma unroll
        for (int y = 0; y < 2; ++y) bv[y] = Bs[(k + kr) * PBB + cb + 16 * y + cc];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) d[x][y] = mfma_f64(av[x], bv[y], d[x][y]);
    }
}

__device__ inline void mm64_acc_zero(dx4 (&d)[2][2])
{
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) d[x][y] = dx4{0.0, 0.0, 0.0, 0.0};
}

__device__ inline void mm64(const double *As, const double *Bs, dx4 (&d)[2][2])
{
    mm64_acc_zero(d);
    mm64_acc<OP, OP>(As, Bs, d);
}

// ---------------------------------------------------------------------------
// The substitutions of both bases in one persistent launch.
//
// Rows are taken in blocks of PB = 64 from the bottom up: block b holds rows
// [r0(b), r1(b)) with r1(b) = n - 64 b (the top block may be short).  Row i of
// T Z = Z L needs the sums acc[i, l] = sum_{j > i} t_ij z_jl over the rows below
// it; for the rows of block b these split into the rows of block b itself
// (solved in order within the block), of block b - 1 (the block just below),
// and of the blocks further down.
//
// Workgroups 0 and 1 ("fronts") run the two bases, block after block: each
// adds block b - 1's part of its sums itself (one 64 x 64 x 64 FP64 MFMA
// product, with block b - 1's Z still in LDS), solves block b row by row as a
// wavefront over waves of eight columns, and publishes block b's rows of Z.
// The other workgroups ("owners") each own row blocks i >= 2 of one basis and
// keep the far part of their sums, sum over the blocks j <= i - 2, in MFMA
// accumulators: as each block j is published they add T[block i, block j]
// Z[block j], and after the last one (j = i - 2) they publish acc of block i.
// A front therefore waits only for work that finished a whole block earlier,
// and its operands for the next block (T's diagonal block and the panel
// against the block below) are fetched while the current block is solved.
//
// Hand-offs go through flags in device memory.  The data behind a flag is
// written with device-coherent stores that complete before the flag's store,
// and read with device-coherent loads issued after the flag was seen, so no L2
// is written back or invalidated (the eight L2s of the chip are not coherent
// with each other).  Every wait is bounded: past the limit it sets the error
// word, which the host reports, and goes on, so the grid always drains.  All
// workgroups of the launch are resident at once (the host sizes the grid to
// the compute units), and a front never waits for an owner that waits for it.
// ---------------------------------------------------------------------------
constexpr int NQ = 8;          // lanes per column, each taking every NQ-th term
constexpr int NU = PB / NQ;    // terms per lane
constexpr int NTS = 64 * NQ;   // threads of a workgroup (one column per NQ lanes)
constexpr int NWS = NTS / 64;  // its waves
constexpr int FP = PB + NQ;    // LDS pitch of the staged T block and of the Z block: one
                               // 16-lane pass of a read falls in distinct banks
constexpr int KMAX = 2;        // row blocks per owner at most

struct ProjSync {
    int *zdone;     // [basis * nb + b]: block b's rows of Z published
    int *accready;  // [basis * nb + b]: acc of block b's rows holds the blocks j <= b - 2
    int *err;       // error word: a wait gave up
    int spin_limit; // polls before a wait gives up (negative: at once; a testing hook)
    int nb;         // row blocks
    int nown;       // owner workgroups per basis
    int kper;       // row blocks per owner (<= KMAX)
    int rcp_guard;  // some |t_ii| outside [2^-1020, 2^1019]: reciprocals checked for range
};

__device__ inline int flag_load(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double coherent_load(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void coherent_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish: every wave's stores complete, then one flag store.
__device__ inline void publish_flag(int *flag)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (thread 0 polls, the workgroup meets at a barrier after it) until *flag
// is set, at most spin_limit polls.
__device__ inline void wait_flag(const int *flag, const ProjSync &S)
{
    if (threadIdx.x == 0) {
        bool ok = S.spin_limit >= 0;
        for (int it = 0; ok && flag_load(flag) == 0; ++it)
            if (it >= S.spin_limit || flag_load(S.err) != 0) {
                ok = false;
            } else {
                __builtin_amdgcn_s_sleep(1);
            }
        if (!ok) atomicOr(S.err, 1);
    }
    __syncthreads();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no load moves above the poll
}

__device__ inline int64_t blk_r1(int64_t n, int b) { return n - (int64_t)PB * b; }
__device__ inline int64_t blk_r0(int64_t n, int b)
{
    const int64_t r = n - (int64_t)PB * (b + 1);
    return r > 0 ? r : 0;
}

// Owner: row blocks i = 2 + w + k nown (k < kper) of basis `beta`; block i's sum
// over the blocks j <= i - 2 in MFMA accumulators (eight waves, each two 16 x 16
// pieces of the 64 x 64 block: rows 16 (wave / 2), columns 32 (wave % 2)).
__device__ void proj_owner(const ProjArgs &a, const ProjSync &S, double *As, double *Bs)
{
    const int o = (int)blockIdx.x - 2;
    const int beta = o & 1, w = o >> 1;
    const ProjBasis &B = a.b[beta];
    const int64_t n = a.n;
    const int m = a.m;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int rb = 16 * (wv >> 1), cb = 32 * (wv & 1);
    const int kr = lane >> 4, cc = lane & 15;
    int ilast = -1;
    for (int k = 0; k < S.kper; ++k)
        if (2 + w + k * S.nown < S.nb) ilast = 2 + w + k * S.nown;
    ilast = uniform(ilast);
    dx4 d[KMAX][2];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) d[k][0] = d[k][1] = dx4{0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j + 2 <= ilast; ++j) {
        const int64_t k0 = blk_r0(n, j), k1 = blk_r1(n, j);
        wait_flag(S.zdone + beta * S.nb + j, S);
        // Bs[kk * OP + c] = Z[k0 + kk, c]: published in this launch, coherent loads
        for (int c = wv; c < 64; c += NWS)
            Bs[lane * OP + c] = (c < m && k0 + lane < k1) ? coherent_load(B.Z + (k0 + lane) + (int64_t)c * n) : 0.0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int i = 2 + w + k * S.nown;
            if (k >= S.kper || i > ilast || i < j + 2) continue;  // uniform
            const int64_t r0 = blk_r0(n, i), r1 = blk_r1(n, i);
            // As[kk * OP + r] = entry (r0 + r, k0 + kk) of the basis's matrix (its
            // upper triangle: block i lies above block j)
            for (int x = wv; x < 64; x += NWS) {
                if (B.flip) {
                    // entry (r0 + x, k0 + lane) is T[n-1-k0-lane, n-1-r0-x]: lane along T's column
                    As[lane * OP + x] = (r0 + x < r1 && k0 + lane < k1)
                                            ? B.T[(n - 1 - k0 - lane) + (n - 1 - r0 - x) * B.ldt] : 0.0;
                } else {
                    As[x * OP + lane] = (r0 + lane < r1 && k0 + x < k1)
                                            ? B.T[(r0 + lane) + (k0 + x) * B.ldt] : 0.0;
                }
            }
            __syncthreads();
            for (int kk = 0; kk < 64; kk += 4) {
                const double av = As[(kk + kr) * OP + rb + cc];
                const double b0 = Bs[(kk + kr) * OP + cb + cc];
                const double b1 = Bs[(kk + kr) * OP + cb + 16 + cc];
                d[k][0] = mfma_f64(av, b0, d[k][0]);
                d[k][1] = mfma_f64(av, b1, d[k][1]);
            }
            __syncthreads();
            if (i == j + 2) {
                // the last block below: publish acc of block i
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t row = r0 + rb + mfma64_row(lane, e);
                        const int c = cb + 16 * y + cc;
                        if (row < r1 && c < m) coherent_store(B.acc + row + (int64_t)c * n, d[k][y][e]);
                    }
                publish_flag(S.accready + beta * S.nb + i);
            }
        }
    }
}

// Front of one basis (blockIdx.x): every block, bottom up.
__global__ __launch_bounds__(NTS) void k_proj_run(ProjArgs a, ProjSync S)
{
    // one arena, so that a step's row of T and row of Z sit within the reach of
    // one base address and the loads' immediate offsets
    __shared__ double arena[PB * FP + PB * FP + PM * FP + PB * AP];
    double *const Tt = arena;         // Tt[r * FP + c] = T[r0 + r, r0 + c], zero below the diagonal
    double *const Zr = Tt + PB * FP;  // Zr[r * FP + l] = Z[r0 + r, l] (zero until computed)
    double *const Zc = Zr + PB * FP;  // Zc[l * FP + r] = Z[r0 + r, l], the same values by column;
                                      // at a block's start, the panel against the block below
    double *const Ab = Zc + PM * FP;  // Ab[r * AP + l] = acc[r0 + r, l]

    if (blockIdx.x >= 2) {
        proj_owner(a, S, Tt, Zr);
        return;
    }

    const ProjBasis B = a.b[blockIdx.x];
    const int beta = blockIdx.x;
    const int64_t n = a.n;
    const int m = a.m;
    constexpr int CW = 64 / NQ;  // columns per wave
    constexpr int NK = 64 / NWS;
    const int wv = uniform(threadIdx.x >> 6);
    // The thread's index, opaque to the compiler where it is read: what derives
    // from it is computed again per block instead of being held in registers
    // across the block loop (which would not leave enough for the wavefront).
    auto tid = [] {
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        return t;
    };
    // Per column, across blocks: the coefficients L[NQ u + q][l], and L[CW wv + k'][l]
    // for the rows of this wave's columns (k' < kw), in every lane of the column;
    // L[l][l] (t at row b_l, set at that row); all zero until the rows that define
    // them are reached.  The column's minority row, and lane x's minority row x.
    double lreg[NU], lw[CW], lamll = 0.0;
#pragma unroll
    for (int u = 0; u < NU; ++u) lreg[u] = 0.0;
#pragma unroll
    for (int kp = 0; kp < CW; ++kp) lw[kp] = 0.0;
    const int pl = B.pos[(threadIdx.x >> 6) * CW + (threadIdx.x & 63) / NQ];  // (-1 from m on)
    const int posl = B.pos[threadIdx.x & 63];
    const bool fl = B.flip != 0;

    // operands of a block fetched ahead: its diagonal block of T and its panel
    // against the block below (T[r0 + i, r1 + k]); lane = block row, wave =
    // column offset (in J T^T J the lane runs along the block's columns, which
    // are T's rows)
    double tv[NK], pv[NK];
    auto fetch = [&](int b) {
        const int t = tid(), row = t & 63, c0 = t >> 6;
        const int64_t r1 = blk_r1(n, b), r0 = blk_r0(n, b);
        const int nr = (int)(r1 - r0);
        const int nk = b > 0 ? (int)(blk_r1(n, b - 1) - r1) : 0;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int c = c0 + NWS * k;
            const int tr = fl ? c : row, tc = fl ? row : c;  // block row and column
            tv[k] = (tr < nr && tc < nr && tr <= tc) ? B.T[toff(B, n, r0 + tr, r0 + tc)] : 0.0;
            pv[k] = (tr < nr && tc < nk) ? B.T[toff(B, n, r0 + tr, r1 + tc)] : 0.0;
        }
    };
    fetch(0);

    for (int b = 0; b < S.nb; ++b) {
        const int t = tid();
        const int col = (t >> 6) * CW + ((t & 63) / NQ);
        const int q = t % NQ;
        const int row = t & 63, c0 = t >> 6;       // staging: lane = row, wave = column offset
        const int64_t r1 = blk_r1(n, b), r0 = blk_r0(n, b);
        const int nr = (int)(r1 - r0);
        const bool below = b > 0;
        // the block's sums over the blocks j <= b - 2, from its owner
        double av[NK];
        if (b >= 2) wait_flag(S.accready + beta * S.nb + b, S);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int c = c0 + NWS * k;
            av[k] = (b >= 2 && row < nr && c < m) ? coherent_load(B.acc + (r0 + row) + (int64_t)c * n) : 0.0;
        }
        // the block's row types, lane i holding row i's (every wave)
        const int rtl = (t & 63) < nr ? B.rowtype[r0 + (t & 63)] : -1;
        __syncthreads();  // the previous block's wavefront and stores of Z are done
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int c = c0 + NWS * k;
            const int tr = fl ? c : row, tc = fl ? row : c;
            Tt[tr * FP + tc] = tv[k];
            Zc[tc * FP + tr] = pv[k];  // k-major: Zc[k * FP + r] = T[r0 + r, r1 + k]
            Ab[row * AP + c] = av[k];
        }
        __syncthreads();
        if (below) {
            // block b - 1's part of the sums: Zr still holds its rows of Z (k-major)
            if (t < 256) {  // the product runs on four waves
                dx4 d[2][2];
                mm64_acc_zero(d);
                mm64_acc<FP, FP>(Zc, Zr, d);
                const int lane = t & 63, w = t >> 6;
                const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int r = rb + 16 * x + mfma64_row(lane, e);
                            const int c = cb + 16 * y + (lane & 15);
                            Ab[r * AP + c] += d[x][y][e];
                        }
            }
            __syncthreads();
        }
        for (int e = t; e < PB * FP; e += NTS) {
            Zr[e] = 0.0;
            Zc[e] = 0.0;
        }
        // block b - 1's rows of Z, stored at the end of its wavefront, are complete:
        // flag them for the owners
        if (below) {
            publish_flag(S.zdone + beta * S.nb + (b - 1));
        }
        __syncthreads();
        // the next block's operands, fetched during this block's wavefront
        if (b + 1 < S.nb) fetch(b + 1);

        // ---- wavefront by waves: at step s the columns of wave w all handle block
        // row r = nr - 1 - s + (w - wmin), wmin the wave of the first active column.
        // A column's sums read its own column (earlier steps) and row r of the
        // columns of the waves before it (written at step s - 1 and earlier); the
        // coupling among the wave's own columns, whose entries of row r are still
        // zero in those sums, is solved after the reduction, column by column within
        // the wave.  At a minority row that coupling is zero (the row of Z is e_typ
        // and L's row typ is not set yet), so only majority rows take that chain.
        // lmin: the minority columns whose row lies above the block (b_l < r0) stay
        // zero throughout it, and the wavefront starts at the first column after them.
        const int lmin = __builtin_popcountll(
            __builtin_amdgcn_ballot_w64((t & 63) < m && posl >= 0 && posl < r0));
        const int wmin = lmin / CW, wlast = (m - 1) / CW;
        const int steps = uniform(m > lmin ? nr + (wlast - wmin) : 0);
        // the column's minority row within the block (-1: above it, PB: below it)
        const int plr = pl < r0 ? -1 : (int)(pl - r0 < PB ? pl - r0 : PB);
        const int rhi = col < m ? (plr < nr - 1 ? plr : nr - 1) : -1;  // last row it computes
        const double *const zcol = Zc + col * FP + q;
        // The coupling terms of wave w come from the columns of the waves before it
        // (chunks u < w); the others are still zero when read.  The step loop is
        // instantiated per wave with that chunk count, so no step tests it.
        auto front = [&](auto wtag) {
        constexpr int NCU = decltype(wtag)::value;  // coupling chunks of this wave
        for (int s = 0; s < steps; ++s) {
            const int r = nr - 1 - s + (wv - wmin);  // the wave's row (uniform)
            const bool act = r >= 0 && r <= rhi;
            // the wave's active columns: a contiguous range (b_l grows with l)
            const uint64_t am = __builtin_amdgcn_ballot_w64(act);
            if (am != 0) {  // then 0 <= r < nr
                // chain steps: the active columns but the last, as a bit mask
                const int klo = __builtin_ctzll(am) / NQ, khi = (64 - __builtin_clzll(am)) / NQ;
                const int chain = uniform(((1 << (khi - 1)) - 1) & ~((1 << klo) - 1));
                int ro = r * FP;
                // opaque to loop strength reduction: one base address for the step's
                // reads of both rows, with immediate offsets
                asm volatile("" : "+v"(ro));
                const double *trow = Tt + ro;
                const double *zrow = Zr + ro;
                // Full sums: every term outside the ranges that count is zero (the
                // lower triangle of the staged block, entries of Z not computed yet).
                // all operands first (paired LDS reads), then the multiply-adds
                double tv_[NU], zv[NU], rv[NCU > 0 ? NCU : 1];
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    tv_[u] = trow[NQ * u + q];
                    zv[u] = zcol[NQ * u];
                    if (u < NCU) rv[u] = zrow[NQ * u + q];
                }
                const double tii = Tt[r * FP + r];
                // (the block's sum read by all the column's lanes, one address: a broadcast,
                // no branch)
                const double ab = Ab[r * AP + col];
                // 1 / (t_ii - L[l, l]): the hardware estimate (relative error below 5e-8)
                // and one Newton step, which squares it (below 2.3e-15).  The signs of
                // t_ii and L[l, l] differ, so |dx| >= min |t_kk| and |dx| <= 2 max |t_kk|;
                // only when the diagonal leaves [2^-1020, 2^1019] (a uniform test) can
                // |dx| leave [2^-1020, 2^1020], where the estimate or its reciprocal would
                // not be normal: then the IEEE division for those entries
                const double dx = tii - lamll;
                double rcp = __builtin_amdgcn_rcp(dx);
                rcp = fma(rcp, fma(-dx, rcp, 1.0), rcp);
                if (__builtin_expect(S.rcp_guard != 0, 0)) {
                    const double adx = fabs(dx);
                    if (adx > 0x1p1020 || adx < 0x1p-1020) rcp = 1.0 / dx;
                }
                double v0 = q == 0 ? ab : 0.0, v1 = 0.0, cp0 = 0.0, cp1 = 0.0;
#pragma unroll
                for (int u = 0; u < NU; u += 2) {
                    v0 += tv_[u] * zv[u];
                    v1 += tv_[u + 1] * zv[u + 1];
                }
#pragma unroll
                for (int u = 0; u < NCU; u += 2) {
                    cp0 += rv[u] * lreg[u];
                    if (u + 1 < NCU) cp1 += rv[u + 1] * lreg[u + 1];
                }
                // d = coupling (waves before this one) - sum
                const double d = group_sum<NQ>((cp0 + cp1) - (v0 + v1));
                const int typ = __builtin_amdgcn_readlane(rtl, r);
                double z = 0.0;
                if (typ >= 0) {
                    // (the active columns only: an inactive one's column of L stays as is)
                    if (act && r == plr) {
                        z = 1.0;
                        lamll = tii;
#pragma unroll
                        for (int u = 0; u < NU; ++u)
                            if (NQ * u + q == col) lreg[u] = tii;
                    } else if (act) {
                        // minority row b_typ (typ < l): row typ of L
#pragma unroll
                        for (int u = 0; u < NU; ++u)
                            if (NQ * u + q == typ) lreg[u] = -d;
#pragma unroll
                        for (int kp = 0; kp < CW; ++kp)
                            if (CW * wv + kp == typ) lw[kp] = -d;
                    }
                } else {
                    // z_l = (d_l + sum_{k' < k} z_k' L[k', l]) / (t_ii - L[l, l]) over the
                    // wave's active columns in order, with the reciprocal folded into
                    // the coefficients (one multiply-add per link); lw is zero from the
                    // diagonal on, so the later terms add nothing to a column solved
                    double lwr[CW - 1];
#pragma unroll
                    for (int kp = 0; kp < CW - 1; ++kp) lwr[kp] = lw[kp] * rcp;
                    z = d * rcp;
#pragma unroll
                    for (int kp = 0; kp < CW - 1; ++kp)
                        if (chain & (1 << kp)) z = fma(readlane_f64(z, kp * NQ), lwr[kp], z);
                }
                if (q == 0 && act) {
                    Zr[r * FP + col] = z;
                    Zc[col * FP + r] = z;
                }
            }
            __syncthreads();
        }
        };
        static_assert(NWS == 8, "one instance per wave");
        switch (wv) {
            case 0: front(std::integral_constant<int, 0>{}); break;
            case 1: front(std::integral_constant<int, 1>{}); break;
            case 2: front(std::integral_constant<int, 2>{}); break;
            case 3: front(std::integral_constant<int, 3>{}); break;
            case 4: front(std::integral_constant<int, 4>{}); break;
            case 5: front(std::integral_constant<int, 5>{}); break;
            case 6: front(std::integral_constant<int, 6>{}); break;
            default: front(std::integral_constant<int, 7>{}); break;
        }
        __syncthreads();

        // ---- the block's rows of Z, for the owners and the output stage (flagged
        // at the next block's start, by when the stores have long completed); the
        // columns from m on are stored too (zeros), so that Z is fully defined
        for (int c = t >> 6; c < PM; c += NWS)
            if (row < nr) coherent_store(B.Z + (r0 + row) + (int64_t)c * n, Zr[row * FP + c]);
    }
    if (S.nb > 0) publish_flag(S.zdone + beta * S.nb + (S.nb - 1));
}

// Partial W^T Z over rows [64 g, 64 g + 64): part[g][l * PM + l'] (row-major l).
// W[j, l] = Zf[n-1-j, m-1-l] with Zf the basis of the flipped matrix.
__global__ __launch_bounds__(256) void k_proj_gram(const double *__restrict__ Z,
                                                   const double *__restrict__ Zf, int64_t n, int m,
                                                   double *__restrict__ part)
{
    __shared__ double As[64 * OP];  // As[k * OP + l]  = W[j0 + k, l]
    __shared__ double Bs[64 * OP];  // Bs[k * OP + l'] = Z[j0 + k, l']
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int t = threadIdx.x, lr = t & 63, q = t >> 6;
    for (int k = q; k < 64; k += 4) {
        const int64_t j = j0 + k;
        const bool ok = j < n && lr < m;
        As[k * OP + lr] = ok ? Zf[(n - 1 - j) + (int64_t)(m - 1 - lr) * n] : 0.0;
        Bs[k * OP + lr] = ok ? Z[j + (int64_t)lr * n] : 0.0;
    }
    __syncthreads();
    dx4 d[2][2];
    mm64(As, Bs, d);
    const int lane = t & 63, w = t >> 6;
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
    double *out = part + (int64_t)blockIdx.x * PM * PM;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = rb + 16 * x + mfma64_row(lane, e);
                const int c = cb + 16 * y + (lane & 15);
                out[r * PM + c] = d[x][y][e];
            }
}

// M = sum of the partials (one entry per thread, coalesced over the partials).
__global__ __launch_bounds__(64) void k_proj_gsum(const double *__restrict__ part, int nparts,
                                                  int m, double *__restrict__ M)
{
    const int e = blockIdx.x * 64 + threadIdx.x;
    const int r = e / PM, c = e % PM;
    double s = 0.0;
    if (r < m && c < m) {
        // eight independent partial sums, so that the loads are issued ahead
        double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int g = 0;
        for (; g + 8 <= nparts; g += 8)
#pragma unroll
            for (int k = 0; k < 8; ++k) p[k] += part[(int64_t)(g + k) * PM * PM + e];
        for (; g < nparts; ++g) p[0] += part[(int64_t)g * PM * PM + e];
        s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    } else {
        s = r == c ? 1.0 : 0.0;
    }
    M[e] = s;
}

// Minv = M^-1 for the upper triangular M (unit diagonal on the leading m x m
// block, identity beyond; zero below the diagonal), by elimination from the last
// row up: row k of the inverse is row k of the running right-hand side R
// (initially I) divided by M[k][k], and then every row i of R loses M[i][k]
// times it (no change for i > k, where M[i][k] = 0; row k itself is not read
// again).  Thread (l, q) keeps R[4 j + q][l] for j < 16 in registers; a
// finished row goes through LDS (two buffers, so one barrier per row).  Mg and
// minv may be the same array: M is read whole before the first row is written.
__global__ __launch_bounds__(256) void k_proj_minv(const double *Mg, double *minv)
{
    __shared__ double M[PM * PM];
    __shared__ double dinv[PM];
    __shared__ double xr[2][PM];
    const int t = threadIdx.x, l = t & 63, q = uniform(t >> 6);
    for (int e = t; e < PM * PM; e += 256) M[e] = Mg[e];
    if (t < PM) dinv[t] = 1.0 / Mg[t * PM + t];
    double R[PM / 4];
#pragma unroll
    for (int j = 0; j < PM / 4; ++j) R[j] = 4 * j + q == l ? 1.0 : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = PM - 1; k >= 0; --k) {
        // column k of M for this thread's rows, read ahead of the barrier
        double mv[PM / 4];
#pragma unroll
        for (int j = 0; j < PM / 4; ++j) mv[j] = M[(4 * j + q) * PM + k];
        if (q == (k & 3)) {
            const double x = R[k >> 2] * dinv[k];
            xr[k & 1][l] = x;
            minv[k * PM + l] = x;
        }
        __syncthreads();
        const double x = xr[k & 1][l];
#pragma unroll
        for (int j = 0; j < PM / 4; ++j) R[j] -= mv[j] * x;
        // applied now: otherwise the compiler defers each row's updates to the
        // row's last step and keeps every earlier row of the inverse live
#pragma unroll
        for (int j = 0; j < PM / 4; ++j) asm volatile("" : "+v"(R[j]));
    }
}

// A = Z Minv over the rows [64 g, 64 g + 64): A[i, l] = sum_k Z[i, k] Minv[k][l]
// (Minv is the identity beyond m, where Z's columns are zero).  Computed as the
// transposed product C[l][i] = sum_k Minv[k][l] Z[i, k] (FP64 MFMA), so that the
// accumulator's lanes run down A's columns.
__global__ __launch_bounds__(256) void k_proj_a(const double *__restrict__ Z,
                                                const double *__restrict__ minv, int64_t n,
                                                double *__restrict__ A)
{
    __shared__ double Ms[PM * OP];  // Ms[k * OP + l]  = Minv[k][l]
    __shared__ double Zs[PM * OP];  // Zs[k * OP + ii] = Z[i0 + ii, k]
    const int t = threadIdx.x, lr = t & 63, q = t >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    for (int k = q; k < PM; k += 4) {
        const int64_t i = i0 + lr;
        Ms[k * OP + lr] = minv[k * PM + lr];
        Zs[k * OP + lr] = i < n ? Z[i + (int64_t)k * n] : 0.0;
    }
    __syncthreads();
    dx4 d[2][2];
    mm64(Ms, Zs, d);
    const int lane = t & 63, w = t >> 6;
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int l = rb + 16 * x + mfma64_row(lane, e);
                const int64_t i = i0 + cb + 16 * y + (lane & 15);
                if (i < n) A[i + (int64_t)l * n] = d[x][y][e];
            }
}

// U[i, j] = s (delta_ij - 2 sum_l A[i, l] W[j, l]) for i <= j, 0 for i > j.
// Computed as the transpose product C[j][i] = sum_l W[j, l] A[i, l], so that
// the accumulator's lane index runs down a column of U.  A[i, l] is zero for
// i > b_l and W[j, l] for j < b_l, and the columns are ordered by b_l: a tile
// with rows [i0, i0 + 64) and columns [j0, j0 + 64) takes only the columns l
// with i0 <= b_l < j0 + 64, in chunks of 16.
constexpr int UK = 16;

__global__ __launch_bounds__(256) void k_proj_u(const double *__restrict__ A,
                                                const double *__restrict__ Zf,
                                                const int *__restrict__ pos, int64_t n, int m,
                                                double smaj, double *__restrict__ U, int64_t ldu)
{
    __shared__ double Ws[UK * OP];  // Ws[k * OP + jj] = W[j0 + jj, l0 + k]
    __shared__ double As[UK * OP];  // As[k * OP + ii] = A[i0 + ii, l0 + k]
    const int64_t ti = blockIdx.x, tj = blockIdx.y;
    const int64_t i0 = ti * 64, j0 = tj * 64;
    const int t = threadIdx.x, lr = t & 63, q = t >> 6;
    if (ti > tj) {
        for (int c = q; c < 64; c += 4) {
            const int64_t i = i0 + lr, j = j0 + c;
            if (i < n && j < n) U[i + j * ldu] = 0.0;
        }
        return;
    }
    // the contributing columns [lo, hi)
    int lo = 0, hi = 0;
    for (int l = 0; l < m; ++l) {
        const int64_t b = pos[l];
        lo += b < i0;
        hi += b < j0 + 64;
    }
    lo = uniform(lo);
    hi = uniform(hi);
    dx4 d[2][2];
    mm64_acc_zero(d);
    const int lane = t & 63, w = t >> 6;
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
    const int kr = lane >> 4, cc = lane & 15;
    for (int l0 = lo; l0 < hi; l0 += UK) {
        for (int k = q; k < UK; k += 4) {
            const int l = l0 + k;
            const int64_t j = j0 + lr, i = i0 + lr;
            Ws[k * OP + lr] = (j < n && l < hi) ? Zf[(n - 1 - j) + (int64_t)(m - 1 - l) * n] : 0.0;
            As[k * OP + lr] = (i < n && l < hi) ? A[i + (int64_t)l * n] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < UK; k += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) av[x] = Ws[(k + kr) * OP + rb + 16 * x + cc];
#pragma unroll
            for (int y = 0; y < 2; ++y) bv[y] = As[(k + kr) * OP + cb + 16 * y + cc];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) d[x][y] = mfma_f64(av[x], bv[y], d[x][y]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t j = j0 + rb + 16 * x + mfma64_row(lane, e);
                const int64_t i = i0 + cb + 16 * y + (lane & 15);
                if (i < n && j < n) {
                    double v = 0.0;
                    if (i <= j) v = smaj * ((i == j ? 1.0 : 0.0) - 2.0 * d[x][y][e]);
                    U[i + j * ldu] = v;
                }
            }
}

inline size_t al(size_t x) { return (x + 255) / 256 * 256; }


// ===========================================================================
// Complex T.  The same form with transposes (not conjugate transposes): the
// left basis solves W^T T = L' W^T, i.e. it is the right basis of J T^T J, and
// P = Z (W^T Z)^-1 W^T.  Simpler kernels than the real ones: 32-row blocks (the
// complex operands of a block fit in LDS), four lanes per column, a separate
// update launch per block, and plain FMA products.
// ===========================================================================
constexpr int PBC = 32;          // rows per block
constexpr int TPC = PBC + 1;     // LDS pitch of the staged block and the column copy
constexpr int ZPC = PM + 1;      // LDS pitch of the Z rows and the running sums

struct CBasis {
    const cd *T;
    int64_t ldt;
    int flip;             // 1: entry (i, j) of this basis's matrix is T[n-1-j, n-1-i]
    cd *Z;                // n x PM, leading dimension n
    cd *acc;              // n x PM: sum over the rows below the current block
    cd *lam;              // PM x PM, lam[lp * PM + l] = L[lp][l]
    const int *rowtype;
    const int *pos;
};

struct CArgs {
    CBasis b[2];
    int64_t n;
    int m;
};

__device__ inline int64_t ctoff(const CBasis &B, int64_t n, int64_t i, int64_t j)
{
    return B.flip ? (n - 1 - j) + (n - 1 - i) * B.ldt : i + j * B.ldt;
}

__device__ inline cd cfma(cd a, cd b, cd c)
{
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}

// Front of one 32-row block [r0, r1) for both bases (blockIdx.x = basis): column
// l handles block row r1 - 1 - s + (l - lmin) at step s, four lanes per column
// each taking every fourth term of the block-row sum (32 terms) and of the L
// coupling (64 terms).
__global__ __launch_bounds__(256) void k_projc_front(CArgs a, int64_t r0, int64_t r1, int lmin0,
                                                     int lmin1)
{
    __shared__ cd Tt[PBC * TPC];  // Tt[r * TPC + c] = T[r0 + r, r0 + c], zero below the diagonal
    __shared__ cd Zr[PBC * ZPC];  // Zr[r * ZPC + l] = Z[r0 + r, l] (zero until computed)
    __shared__ cd Zc[PM * TPC];   // Zc[l * TPC + r]: the same values by column
    __shared__ cd Ab[PBC * ZPC];  // Ab[r * ZPC + l] = acc[r0 + r, l]
    __shared__ int rt[PBC];
    const CBasis B = a.b[blockIdx.x];
    const int64_t n = a.n;
    const int m = a.m;
    const int t = threadIdx.x;
    const int nr = (int)(r1 - r0);
    const cd zero = {0.0, 0.0};
    for (int e = t; e < PBC * PBC; e += 256) {
        const int r = e % PBC, c = e / PBC;
        Tt[r * TPC + c] = (r < nr && c < nr && r <= c) ? B.T[ctoff(B, n, r0 + r, r0 + c)] : zero;
    }
    for (int e = t; e < PBC * PM; e += 256) {
        const int r = e % PBC, c = e / PBC;
        Ab[r * ZPC + c] = (r < nr && c < m) ? B.acc[(r0 + r) + (int64_t)c * n] : zero;
        Zr[r * ZPC + c] = zero;
    }
    for (int e = t; e < PM * TPC; e += 256) Zc[e] = zero;
    if (t < PBC) rt[t] = t < nr ? B.rowtype[r0 + t] : -1;
    const int col = t >> 2, q = t & 3;
    cd lreg[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) lreg[u] = B.lam[(4 * u + q) * PM + col];
    cd lamll = B.lam[col * PM + col];
    const int pl = col < m ? B.pos[col] : -1;
    __syncthreads();

    const int lmin = uniform(blockIdx.x == 0 ? lmin0 : lmin1);
    const int steps = uniform(m > lmin ? nr + (m - lmin) - 1 : 0);
    for (int s = 0; s < steps; ++s) {
        const int r = nr - 1 - s + (col - lmin);
        const int64_t i = r0 + r;
        if (col < m && r >= 0 && r < nr && i <= pl) {
            cd v = q == 0 ? Ab[r * ZPC + col] : zero, cp = zero;
#pragma unroll
            for (int u = 0; u < PBC / 4; ++u) {
                const int c = 4 * u + q;
                v = cfma(Tt[r * TPC + c], Zc[col * TPC + c], v);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) cp = cfma(Zr[r * ZPC + 4 * u + q], lreg[u], cp);
            // coupling minus sum; at a minority row the coupling is zero (see the real kernel)
            cd d = {cp.re - v.re, cp.im - v.im};
            d.re = group_sum<4>(d.re);
            d.im = group_sum<4>(d.im);
            const cd tii = Tt[r * TPC + r];
            const int typ = rt[r];
            cd z;
            if (i == pl) {
                z = {1.0, 0.0};
                lamll = tii;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (4 * u + q == col) lreg[u] = tii;
            } else if (typ >= 0) {
                z = zero;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (4 * u + q == typ) lreg[u] = {-d.re, -d.im};
            } else {
                z = d / (tii - lamll);
            }
            if (q == 0) {
                Zr[r * ZPC + col] = z;
                Zc[col * TPC + r] = z;
            }
        }
        __syncthreads();
    }
    for (int e = t; e < PBC * m; e += 256) {
        const int r = e % PBC, c = e / PBC;
        if (r < nr) B.Z[(r0 + r) + (int64_t)c * n] = Zr[r * ZPC + c];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) B.lam[(4 * u + q) * PM + col] = lreg[u];
}

// acc[0:r0, :] += T[0:r0, r0:r1] Z[r0:r1, :] (64-row tiles, blockIdx.y = basis)
__global__ __launch_bounds__(256) void k_projc_update(CArgs a, int64_t r0, int64_t r1)
{
    __shared__ cd As[64 * (PBC + 1)];  // As[r * (PBC + 1) + k] = T[row0 + r, r0 + k]
    __shared__ cd Bs[PBC * ZPC];       // Bs[k * ZPC + l] = Z[r0 + k, l]
    const CBasis B = a.b[blockIdx.y];
    const int64_t n = a.n;
    const int m = a.m;
    const int64_t row0 = (int64_t)blockIdx.x * 64;
    const int nk = (int)(r1 - r0);
    const int t = threadIdx.x;
    const cd zero = {0.0, 0.0};
    for (int e = t; e < 64 * PBC; e += 256) {
        const int r = e % 64, k = e / 64;
        As[r * (PBC + 1) + k] = (row0 + r < r0 && k < nk) ? B.T[ctoff(B, n, row0 + r, r0 + k)] : zero;
    }
    for (int e = t; e < PBC * PM; e += 256) {
        const int k = e % PBC, l = e / PBC;
        Bs[k * ZPC + l] = (k < nk && l < m) ? B.Z[(r0 + k) + (int64_t)l * n] : zero;
    }
    __syncthreads();
    const int l = t & 63, rg = t >> 6;
    if (l >= m) return;
    for (int rr = 0; rr < 16; ++rr) {
        const int r = rg * 16 + rr;
        const int64_t row = row0 + r;
        if (row >= r0) break;
        cd sum = zero;
        for (int k = 0; k < PBC; ++k) sum = cfma(As[r * (PBC + 1) + k], Bs[k * ZPC + l], sum);
        cd &o = B.acc[row + (int64_t)l * n];
        o = {o.re + sum.re, o.im + sum.im};
    }
}

// Partial W^T Z over rows [64 g, 64 g + 64): part[g][l * PM + l'].
__global__ __launch_bounds__(256) void k_projc_gram(const cd *__restrict__ Z,
                                                    const cd *__restrict__ Zf, int64_t n, int m,
                                                    cd *__restrict__ part)
{
    __shared__ cd Ws[64 * ZPC];  // Ws[k * ZPC + l] = W[j0 + k, l]
    __shared__ cd Zs[64 * ZPC];  // Zs[k * ZPC + l] = Z[j0 + k, l]
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int t = threadIdx.x;
    const cd zero = {0.0, 0.0};
    for (int e = t; e < 64 * PM; e += 256) {
        const int k = e % 64, l = e / 64;
        const int64_t j = j0 + k;
        const bool ok = j < n && l < m;
        Ws[k * ZPC + l] = ok ? Zf[(n - 1 - j) + (int64_t)(m - 1 - l) * n] : zero;
        Zs[k * ZPC + l] = ok ? Z[j + (int64_t)l * n] : zero;
    }
    __syncthreads();
    const int l = t & 63, g = t >> 6;
    cd *out = part + (int64_t)blockIdx.x * PM * PM;
    for (int c = 0; c < 16; ++c) {
        const int lp = g * 16 + c;
        cd sum = zero;
        for (int k = 0; k < 64; ++k) sum = cfma(Ws[k * ZPC + l], Zs[k * ZPC + lp], sum);
        out[l * PM + lp] = sum;
    }
}

// M = sum of the partials (identity beyond the leading m x m block), then
// Minv = M^-1 by back substitution, one column per thread.
__global__ __launch_bounds__(64) void k_projc_minv(const cd *__restrict__ part, int nparts, int m,
                                                   cd *__restrict__ minv)
{
    __shared__ cd M[PM * PM];
    __shared__ cd X[PM * ZPC];
    const int l = threadIdx.x;
    for (int e = l; e < PM * PM; e += 64) {
        const int r = e / PM, c = e % PM;
        cd s = {0.0, 0.0};
        if (r < m && c < m)
            for (int g = 0; g < nparts; ++g) {
                const cd v = part[(int64_t)g * PM * PM + e];
                s = {s.re + v.re, s.im + v.im};
            }
        else
            s = {r == c ? 1.0 : 0.0, 0.0};
        M[e] = s;
    }
    __syncthreads();
    for (int k = PM - 1; k >= 0; --k) {
        cd v = {k == l ? 1.0 : 0.0, 0.0};
        if (k < l)
            for (int kk = k + 1; kk <= l; ++kk) {
                const cd p = M[k * PM + kk] * X[kk * ZPC + l];
                v = {v.re - p.re, v.im - p.im};
            }
        X[k * ZPC + l] = k <= l ? v / M[k * PM + k] : cd{0.0, 0.0};
    }
    __syncthreads();
    for (int e = l; e < PM * PM; e += 64) minv[e] = X[(e / PM) * ZPC + e % PM];
}

// A = Z Minv, 4 rows per workgroup.
__global__ __launch_bounds__(256) void k_projc_a(const cd *__restrict__ Z,
                                                 const cd *__restrict__ minv, int64_t n, int m,
                                                 cd *__restrict__ A)
{
    __shared__ cd X[PM * PM];
    const int t = threadIdx.x;
    for (int e = t; e < PM * PM; e += 256) X[e] = minv[e];
    __syncthreads();
    const int l = t & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (t >> 6);
    if (i >= n) return;
    cd s = {0.0, 0.0};
    if (l < m)
        for (int lp = 0; lp <= l; ++lp) s = cfma(Z[i + (int64_t)lp * n], X[lp * PM + l], s);
    A[i + (int64_t)l * n] = s;
}

// U[i, j] = s (delta_ij - 2 sum_l A[i, l] W[j, l]) on the upper triangle, zeros
// below; a tile takes the columns l with i0 <= b_l < j0 + 64, 16 at a time.
__global__ __launch_bounds__(256) void k_projc_u(const cd *__restrict__ A,
                                                 const cd *__restrict__ Zf,
                                                 const int *__restrict__ pos, int64_t n, int m,
                                                 double smaj, cd *__restrict__ U, int64_t ldu)
{
    __shared__ cd As[64 * 17];  // As[ii * 17 + k] = A[i0 + ii, l0 + k]
    __shared__ cd Ws[64 * 17];  // Ws[jj * 17 + k] = W[j0 + jj, l0 + k]
    const int64_t ti = blockIdx.x, tj = blockIdx.y;
    const int64_t i0 = ti * 64, j0 = tj * 64;
    const int t = threadIdx.x, ii = t & 63, jg = t >> 6;
    const cd zero = {0.0, 0.0};
    if (ti > tj) {
        for (int c = jg; c < 64; c += 4) {
            const int64_t i = i0 + ii, j = j0 + c;
            if (i < n && j < n) U[i + j * ldu] = zero;
        }
        return;
    }
    int lo = 0, hi = 0;
    for (int l = 0; l < m; ++l) {
        const int64_t b = pos[l];
        lo += b < i0;
        hi += b < j0 + 64;
    }
    lo = uniform(lo);
    hi = uniform(hi);
    cd acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = zero;
    for (int l0 = lo; l0 < hi; l0 += 16) {
        for (int e = t; e < 64 * 16; e += 256) {
            const int r = e % 64, k = e / 64, l = l0 + k;
            const int64_t i = i0 + r, j = j0 + r;
            As[r * 17 + k] = (i < n && l < hi) ? A[i + (int64_t)l * n] : zero;
            Ws[r * 17 + k] = (j < n && l < hi) ? Zf[(n - 1 - j) + (int64_t)(m - 1 - l) * n] : zero;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int jj = jg * 16 + c;
            for (int k = 0; k < 16; ++k) acc[c] = cfma(As[ii * 17 + k], Ws[jj * 17 + k], acc[c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int64_t i = i0 + ii, j = j0 + jg * 16 + c;
        if (i < n && j < n) {
            cd v = zero;
            if (i <= j) v = {smaj * ((i == j ? 1.0 : 0.0) - 2.0 * acc[c].re), -2.0 * smaj * acc[c].im};
            U[i + j * ldu] = v;
        }
    }
}

}  // namespace

// flags of the persistent run: two per block and basis, and the error word
size_t proj_sync_bytes(int64_t n) { return (size_t)(4 * ((n + PB - 1) / PB) + 1) * sizeof(int); }

size_t proj_workspace_bytes(int64_t n, bool cplx)
{
    const size_t nn = (size_t)n, es = cplx ? 16 : 8;
    const size_t nparts = (nn + 63) / 64;
    return 4 * al(nn * PM * es)             // Z and acc, two bases
           + 2 * al(PM * PM * es)           // L, two bases
           + 2 * al(nn * 4) + 2 * al(PM * 4)  // row types and minority rows
           + al(nparts * PM * PM * es)      // partial Gram matrices
           + al(PM * PM * es)               // Minv
           + al(nn * PM * es)               // A
           + al(proj_sync_bytes(n));        // flags (real T)
}

int run_proj_c(const void *Tv, int64_t ldt, void *Uv, int64_t ldu, int64_t n, const int8_t *sgn,
               const int8_t *hsgn, int minority, int m, double flops, void *ws, hipStream_t st)
{
    if (m < 1 || m > PM || n < 2) return SIGNTRI_ENOTSUP;
    const cd *T = (const cd *)Tv;
    cd *U = (cd *)Uv;
    std::vector<int64_t> mrow;
    mrow.reserve(m);
    for (int64_t i = 0; i < n; ++i)
        if (hsgn[i] == minority) mrow.push_back(i);
    if ((int)mrow.size() != m) return SIGNTRI_ENOTSUP;
    const size_t nn = (size_t)n;
    const int64_t nparts = (n + 63) / 64;
    char *p = (char *)ws;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += al(bytes);
        return (void *)q;
    };
    cd *Z0 = (cd *)take(nn * PM * 16), *Z1 = (cd *)take(nn * PM * 16);
    cd *C0 = (cd *)take(nn * PM * 16), *C1 = (cd *)take(nn * PM * 16);
    cd *L0 = (cd *)take(PM * PM * 16), *L1 = (cd *)take(PM * PM * 16);
    int *rt0 = (int *)take(nn * 4), *rt1 = (int *)take(nn * 4);
    int *ps0 = (int *)take(PM * 4), *ps1 = (int *)take(PM * 4);
    cd *part = (cd *)take((size_t)nparts * PM * PM * 16);
    cd *minv = (cd *)take(PM * PM * 16);
    cd *A = (cd *)take(nn * PM * 16);
    if (hipMemsetAsync(Z0, 0, (char *)rt0 - (char *)Z0, st) != hipSuccess) return SIGNTRI_EHIP;
    prof_begin(st);
    hipLaunchKernelGGL(k_proj_prep, dim3(1), dim3(1024), 0, st, sgn, n, minority, m, rt0, ps0, rt1,
                       ps1);
    prof_end(st, PK_AUX, 0.0, 1);
    CArgs a;
    a.n = n;
    a.m = m;
    a.b[0] = CBasis{T, ldt, 0, Z0, C0, L0, rt0, ps0};
    a.b[1] = CBasis{T, ldt, 1, Z1, C1, L1, rt1, ps1};
    const double nd = (double)n, md = (double)m;
    prof_begin(st);
    int launches = 0;
    for (int64_t r1 = n; r1 > 0;) {
        const int64_t r0 = std::max<int64_t>(0, r1 - PBC);
        const int lmin0 = (int)(std::lower_bound(mrow.begin(), mrow.end(), r0) - mrow.begin());
        const int lmin1 =
            (int)(mrow.end() - std::upper_bound(mrow.begin(), mrow.end(), n - 1 - r0));
        hipLaunchKernelGGL(k_projc_front, dim3(2), dim3(256), 0, st, a, r0, r1, lmin0, lmin1);
        ++launches;
        if (r0 > 0) {
            hipLaunchKernelGGL(k_projc_update, dim3((r0 + 63) / 64, 2), dim3(256), 0, st, a, r0, r1);
            ++launches;
        }
        r1 = r0;
    }
    prof_end(st, PK_PROJ, flops, launches);
    prof_begin(st);
    hipLaunchKernelGGL(k_projc_gram, dim3(nparts), dim3(256), 0, st, Z0, Z1, n, m, part);
    hipLaunchKernelGGL(k_projc_minv, dim3(1), dim3(64), 0, st, part, (int)nparts, m, minv);
    hipLaunchKernelGGL(k_projc_a, dim3((n + 3) / 4), dim3(256), 0, st, Z0, minv, n, m, A);
    const int64_t nu = (n + 63) / 64;
    hipLaunchKernelGGL(k_projc_u, dim3(nu, nu), dim3(256), 0, st, A, Z1, ps0, n, m,
                       minority > 0 ? -1.0 : 1.0, U, ldu);
    // complex multiply-adds count 8 flops
    prof_end(st, PK_PROJ_OUT, 4.0 * (nd * nd * md + 3.0 * nd * md * md), 4);
    return hipGetLastError() == hipSuccess ? SIGNTRI_OK : SIGNTRI_EHIP;
}

// Compute units of the current device (cached per device), for the size of the
// persistent grid.
int device_cus()
{
    static std::vector<int> cache;
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> g(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cache[dev] = v;
    }
    return cache[dev];
}

// Owners per basis and row blocks per owner for a persistent run over nb blocks:
// every workgroup must be resident at once (one per compute unit: the front's
// LDS arena leaves room for no second one).  False when nb is too large.
bool proj_grid(int64_t nb, int cus, int *nown, int *kper)
{
    const int64_t tiles = nb > 2 ? nb - 2 : 0;
    if (tiles == 0) {
        *nown = 0;
        *kper = 0;
        return true;
    }
    const int64_t slots = (int64_t)(cus - 2) / 2;
    if (slots < 1) return false;
    const int64_t no = std::min<int64_t>(tiles, slots);
    const int64_t kp = (tiles + no - 1) / no;
    if (kp > KMAX) return false;
    // as few owners as keep kp: fewer workgroups polling
    *nown = (int)((tiles + kp - 1) / kp);
    *kper = (int)kp;
    return true;
}

bool proj_fits(int64_t n)
{
    int nown = 0, kper = 0;
    return n >= 2 && proj_grid((n + PB - 1) / PB, device_cus(), &nown, &kper);
}

int run_proj(const double *T, int64_t ldt, double *U, int64_t ldu, int64_t n, const int8_t *sgn,
             const int8_t *hsgn, int minority, int m, double flops, void *ws, hipStream_t st,
             int *herr, bool rcp_guard)
{
    if (m < 1 || m > PM || n < 2) return SIGNTRI_ENOTSUP;
    int nown = 0, kper = 0;
    const int64_t nb = (n + PB - 1) / PB;
    if (!proj_grid(nb, device_cus(), &nown, &kper)) return SIGNTRI_ENOTSUP;
    int cnt = 0;
    for (int64_t i = 0; i < n; ++i) cnt += hsgn[i] == minority;
    if (cnt != m) return SIGNTRI_ENOTSUP;
    const size_t nn = (size_t)n;
    const int64_t nparts = (n + 63) / 64;
    char *p = (char *)ws;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += al(bytes);
        return (void *)q;
    };
    double *Z0 = (double *)take(nn * PM * 8), *Z1 = (double *)take(nn * PM * 8);
    double *C0 = (double *)take(nn * PM * 8), *C1 = (double *)take(nn * PM * 8);
    take(PM * PM * 8);  // (L of both bases: only the complex kernels keep it in memory)
    take(PM * PM * 8);
    int *rt0 = (int *)take(nn * 4), *rt1 = (int *)take(nn * 4);
    int *ps0 = (int *)take(PM * 4), *ps1 = (int *)take(PM * 4);
    double *part = (double *)take((size_t)nparts * PM * PM * 8);
    double *minv = (double *)take(PM * PM * 8);
    double *A = (double *)take(nn * PM * 8);
    int *sync = (int *)take(proj_sync_bytes(n));

    // flags and error word: a fill kernel (no memset node, should the call be captured)
    prof_begin(st);
    hipLaunchKernelGGL(k_proj_prep, dim3(1), dim3(1024), 0, st, sgn, n, minority, m, rt0, ps0, rt1,
                       ps1);
    if (launch_fill_int(sync, (int64_t)(4 * nb + 1), 0, st) != hipSuccess) return SIGNTRI_EHIP;
    prof_end(st, PK_AUX, 0.0, 2);

    ProjArgs a;
    a.n = n;
    a.m = m;
    a.b[0] = ProjBasis{T, ldt, 0, Z0, C0, rt0, ps0};
    a.b[1] = ProjBasis{T, ldt, 1, Z1, C1, rt1, ps1};
    ProjSync S;
    S.zdone = sync;
    S.accready = sync + 2 * nb;
    S.err = sync + 4 * nb;
    S.spin_limit = flow_spin_limit();
    S.nb = (int)nb;
    S.nown = nown;
    S.kper = kper;
    S.rcp_guard = rcp_guard ? 1 : 0;
    const double nd = (double)n, md = (double)m;
    prof_begin(st);
    hipLaunchKernelGGL(k_proj_run, dim3(2 + 2 * nown), dim3(NTS), 0, st, a, S);
    prof_end(st, PK_PROJ, flops, 1);
    prof_begin(st);
    // four launches: W^T Z partials, their sum, its inverse, A; then the product
    hipLaunchKernelGGL(k_proj_gram, dim3(nparts), dim3(256), 0, st, Z0, Z1, n, m, part);
    hipLaunchKernelGGL(k_proj_gsum, dim3(PM * PM / 64), dim3(64), 0, st, part, (int)nparts, m,
                       minv);
    hipLaunchKernelGGL(k_proj_minv, dim3(1), dim3(256), 0, st, minv, minv);
    hipLaunchKernelGGL(k_proj_a, dim3((n + 63) / 64), dim3(256), 0, st, Z0, minv, n, A);
    const int64_t nu = (n + 63) / 64;
    hipLaunchKernelGGL(k_proj_u, dim3(nu, nu), dim3(256), 0, st, A, Z1, ps0, n, m,
                       minority > 0 ? -1.0 : 1.0, U, ldu);
    // W^T Z and A = Z Minv (3 n m^2), the rank-m product on the upper triangle (n^2 m)
    prof_end(st, PK_PROJ_OUT, nd * nd * md + 3.0 * nd * md * md, 5);
    if (hipGetLastError() != hipSuccess) return SIGNTRI_EHIP;
    if (herr) {
        // wait, and report a wait of the substitutions that gave up
        if (hipMemcpyAsync(herr, S.err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SIGNTRI_EHIP;
        if (*herr) return SIGNTRI_EHIP;
    }
    return SIGNTRI_OK;
}

}  // namespace sgt
