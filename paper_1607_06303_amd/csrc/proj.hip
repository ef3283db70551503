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
    double *Z;            // n x mp (m rounded up to 64), leading dimension n
    double *acc;          // n x mp: sum over the rows below the current block
    const int *rowtype;   // n: minority column of row i, or -1
    const int *pos;       // mp: row of minority column l, or -1 (l >= m)
};

struct ProjArgs {
    ProjBasis b[2];
    int64_t n;
    int m;
};

// The double of lane Q of each group of eight lanes, held by the whole group
// (a swizzle in bitmask mode: source lane = (lane & 0x18) | Q within each half
// of the wave).
template <int Q> __device__ inline double bcast8_f64(double v)
{
    constexpr int pat = 0x18 | (Q << 5);
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)b, pat);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(b >> 32), pat);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

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
// pos is padded with -1 to mp entries.  kx (if not null): for each basis and
// 64-row block b counted from the bottom (rows [r0(b), r1(b)), r0(b) =
// max(0, n - 64 (b + 1))), kx[basis * (nb + 2) + b + 2] = K(b), the number of
// minority rows above the block (pos[l] < r0(b)), for b = -2 .. nb - 1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_proj_prep(const int8_t *__restrict__ sgn, int64_t n,
                                                    int minority, int m, int mp, int nb,
                                                    int *__restrict__ rt0, int *__restrict__ pos0,
                                                    int *__restrict__ rt1, int *__restrict__ pos1,
                                                    int *__restrict__ kx)
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
    for (int q = m + t; q < mp; q += 1024) {
        pos0[q] = -1;
        pos1[q] = -1;
    }
    if (kx) {
        // the minority rows above each block, by bisection of the finished pos
        __threadfence_block();
        __syncthreads();
        for (int e = t; e < 2 * (nb + 2); e += 1024) {
            const int *pos = e < nb + 2 ? pos0 : pos1;
            const int b = e % (nb + 2) - 2;
            const int64_t r0 = n - (int64_t)PB * (b + 1);
            int lo2 = 0, hi2 = m;  // the first l with pos[l] >= r0
            while (lo2 < hi2) {
                const int mid = (lo2 + hi2) / 2;
                if (pos[mid] < r0) lo2 = mid + 1;
                else hi2 = mid;
            }
            kx[e] = lo2;
        }
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
// The minority columns are split into groups of GC = 8 consecutive columns.
// Column l is zero below its minority row b_l and couples only with the
// columns l' < l (through L[l', l]), so group g needs, besides its own rows,
// only the finished values of the groups before it, which start higher up (their
// minority rows lie above g's) and so run ahead of it.  Each group of each
// basis has its own workgroup ("front"): wave 0 solves the group's columns row
// by row (eight lanes per column, one row per step, no barrier inside a block;
// the coupling among the group's own columns solved in order by lane
// broadcasts), from the block of the group's lowest minority row to the top;
// waves 1..3 meanwhile publish the previous block's rows of the group and fetch
// the next block's operands.  The coupling with the earlier columns l' < c0 on
// block b's rows, sum_{l'} z_il' L[l', l], is split by where b_l' lies (L[l', l]
// is set at row b_l', so it is known once that row is solved):
//   * in block b: at most 64 columns, taken term by term in the steps;
//   * in block b - 1: one 64 x 64 x 8 FP64 MFMA product between the blocks,
//     together with the block just below's part of the sums (the group's rows
//     of block b - 1 still in LDS);
//   * further down: a 64 x (up to 504) x 8 product that waves 1..3 form while
//     block b - 1 is solved.
// The bottom group, which covers nearly every row, is the critical path; a row
// costs it one single-wave step.
//
// The other workgroups ("owners") each take tasks (row block i >= 2, chunk of
// eight groups) of one basis in turn and keep the far part of the task's sums,
// sum over the blocks j <= i - 2, in MFMA accumulators: as block j is published
// by a group of the chunk, they add T[block i, block j] Z[block j, its
// columns], and after the last one (j = i - 2) they publish acc of block i for
// that group.
//
// Hand-offs go through flags in device memory.  The data behind a flag is
// written with device-coherent stores that complete before the flag's store,
// and read with device-coherent loads issued after the flag was seen, so no L2
// is written back or invalidated (the eight L2s of the chip are not coherent
// with each other).  Every wait is bounded: past the limit it sets the error
// word, which the host reports, and goes on, so the grid always drains.  All
// workgroups of the launch are resident at once (the host sizes the grid to
// the compute units).  A front's waits point to earlier groups at the same
// block and to owners; an owner's, to fronts at blocks at least two below the
// task's block and to its own earlier tasks, whose blocks are not higher: no
// cycle.
// ---------------------------------------------------------------------------
constexpr int NQ = 8;             // lanes per column, each taking every NQ-th term
constexpr int GC = 64 / NQ;       // columns per group (one wave)
constexpr int NU = PB / NQ;       // block-row terms per lane
constexpr int MPM = kProjMaxMinorityReal;  // minority columns at most (real T)
constexpr int MAXG = MPM / GC;    // groups at most
constexpr int OC = 32;            // columns of an owner task (a chunk)
constexpr int CG = OC / GC;       // groups per chunk
constexpr int NPO = OC / 16;      // 16-column MFMA pieces of a chunk
constexpr int NT = 256;           // threads of a workgroup (four waves)
constexpr int TP = PB + 1;        // LDS pitch of the T block, the window values and the panel
constexpr int ZCP = PB + NQ;      // LDS pitch of a group column (conflict-free column reads)
constexpr int ABP = GC + 1;       // LDS pitch of the group's sums
constexpr int LFP = GC;           // LDS pitch of the coupling coefficients
constexpr int NH = NT - 64;       // helper lanes (waves 1..3)
constexpr int HK = (PB * PB + NH - 1) / NH;  // a 64 x 64 operand: entries per helper lane
constexpr int HW = 8;             // a window's values fetched ahead per helper lane
constexpr int HWC = HW * NH / PB; // columns of a window fetched ahead
constexpr int HA = (PB * GC + NH - 1) / NH;  // the group's sums of a block
static_assert(HW * NH % PB == 0, "whole window columns per fetch");

struct ProjSync {
    int *zdone;     // [(basis * G + g) * nb + b]: group g's rows of block b published
    int *accready;  // same index: group g's far sums of block b published
    int *err;       // error word: a wait gave up
    const int *kx;  // [basis * (nb + 2) + b + 2] = K(b): the minority columns whose row lies
                    // above block b (b_l < r0(b)), for b = -2 .. nb - 1 (K(-1) = K(-2) = m)
    int spin_limit; // polls before a wait gives up (negative: at once; a testing hook)
    int nb;         // row blocks
    int G;          // column groups
    int nown;       // owner workgroups per basis
    int rcp_guard;  // some |t_ii| outside [2^-1020, 2^1019]: reciprocals checked for range
    int bstart[2 * MAXG];  // [basis * G + g]: the block of the group's lowest minority row
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
__device__ inline void set_flag(int *p)
{
    __hip_atomic_store(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-level wait (lane 0 polls, the wave goes on together after it) until *flag
// is set, at most spin_limit polls; on giving up it sets the error word and
// returns.
__device__ inline void wave_wait(const int *flag, const ProjSync &S)
{
    int ok = 1;
    if ((threadIdx.x & 63) == 0) {
        ok = S.spin_limit >= 0;
        for (int it = 0; ok && flag_load(flag) == 0; ++it)
            if (it >= S.spin_limit || flag_load(S.err) != 0) {
                ok = 0;
            } else {
                __builtin_amdgcn_s_sleep(1);
            }
        if (!ok) atomicOr(S.err, 1);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no load moves above the poll
}

__device__ inline int64_t blk_r1(int64_t n, int b) { return n - (int64_t)PB * b; }
__device__ inline int64_t blk_r0(int64_t n, int b)
{
    const int64_t r = n - (int64_t)PB * (b + 1);
    return r > 0 ? r : 0;
}

// Entry (e) of a 64 x 64 operand staged by a helper lane: (row, col) chosen so
// that consecutive lanes read consecutive addresses of T (its columns for T
// itself; for J T^T J the operand's rows run along T's columns).
__device__ inline void op_entry(bool flip, int e, int &row, int &col)
{
    if (flip) {
        row = e >> 6;
        col = e & 63;
    } else {
        col = e >> 6;
        row = e & 63;
    }
}

// A range of earlier columns [lo, lo + cnt) (cnt <= 0: none).
struct Win {
    int lo, cnt;
};

// Owner: tasks (row block i, chunk c of CG groups) of basis `beta`, in the order
// of i, then c, every nown-th one; one task at a time.  A task keeps block i's
// sums over the blocks j <= i - 2 for the chunk's OC columns in MFMA
// accumulators (four waves, each 16 rows x OC columns: 16 x 16 pieces, a
// group's eight columns in half a piece).  Chunks of four groups: at the top of
// the matrix every group publishes a block per block time, and a task serving
// more groups than that would fall behind (the groups then wait for their sums).  The groups run at their own pace and
// each is followed on its own: thread 0 takes the lowest block j that some group
// of the chunk has published and the task has not yet added, with every group
// that has published it, and the workgroup adds T[block i, block j] Z[block j,
// those groups' columns] (the 16-column pieces without such a group skipped).
// All of a step's loads are issued before any is used.
__device__ void proj_owner(const ProjArgs &a, const ProjSync &S, double *As, double *Bs)
{
    const int o = (int)blockIdx.x - 2 * S.G;
    const int beta = o & 1, w = o >> 1;
    const ProjBasis &B = a.b[beta];
    const int64_t n = a.n;
    const int m = a.m;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int rb = 16 * wv;
    const int kr = lane >> 4, cc = lane & 15;
    const int *bst = S.bstart + beta * S.G;
    const int nch = (S.G + CG - 1) / CG;
    __shared__ int s_next[CG];  // per group of the chunk: its next block (> i - 2: done)
    __shared__ int s_j, s_mask;
    int idle = 0;
    for (int task = w;; task += S.nown) {
        const int i = uniform(2 + task / nch), c = uniform(task % nch);
        if (i >= S.nb) break;
        const int g0 = c * CG, gn = min(CG, S.G - g0);
        __syncthreads();  // the previous task's last reads of s_next are done
        if (t < CG) s_next[t] = (t < gn && bst[g0 + t] <= i - 2) ? bst[g0 + t] : i - 1;
        const int64_t r0 = blk_r0(n, i), r1 = blk_r1(n, i);
        dx4 d[NPO];
#pragma unroll
        for (int y = 0; y < NPO; ++y) d[y] = dx4{0.0, 0.0, 0.0, 0.0};
        for (;;) {
            __syncthreads();
            if (t == 0) {
                // the lowest published block not yet added, and the groups that have it
                // (j = -1: none published yet; -2: the task is done)
                int jmin = 1 << 30, mask = 0, first = -1, jfirst = 1 << 30;
                for (int gg = 0; gg < gn; ++gg) {
                    const int j = s_next[gg];
                    if (j > i - 2) continue;
                    if (j < jfirst) {
                        jfirst = j;
                        first = gg;
                    }
                    if (flag_load(S.zdone + (beta * S.G + g0 + gg) * S.nb + j) == 0) continue;
                    if (j < jmin) {
                        jmin = j;
                        mask = 0;
                    }
                    if (j == jmin) mask |= 1 << gg;
                }
                int jp = mask ? jmin : (first < 0 ? -2 : -1);
                if (jp == -1) {
                    // bounded: past the limit (or after another wait gave up) take the
                    // lowest unfinished group anyway, so that the grid drains
                    if (S.spin_limit < 0 || ++idle > S.spin_limit || flag_load(S.err) != 0) {
                        atomicOr(S.err, 1);
                        jp = jfirst;
                        for (int gg = 0; gg < gn; ++gg)
                            if (s_next[gg] == jfirst) mask |= 1 << gg;
                    } else {
                        __builtin_amdgcn_s_sleep(1);
                    }
                } else {
                    idle = 0;
                }
                s_j = jp;
                s_mask = mask;
            }
            __syncthreads();
            const int j = uniform(s_j), mask = uniform(s_mask);
            if (j == -2) break;
            if (j < 0) continue;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no load moves above the flags
            const int64_t k0 = blk_r0(n, j), k1 = blk_r1(n, j);
            // the step's loads: block j's rows of the groups in the mask (coherent: they
            // were published in this launch), and T's tile [block i, block j]
            double zb[OC / 4], ta[16];
#pragma unroll
            for (int x = 0; x < OC / 4; ++x) {
                const int cl = wv + 4 * x;  // column within the chunk
                const int col = OC * c + cl;
                const bool live = col < m && ((mask >> (cl / GC)) & 1) && k0 + lane < k1;
                zb[x] = live ? coherent_load(B.Z + (k0 + lane) + (int64_t)col * n) : 0.0;
            }
#pragma unroll
            for (int x = 0; x < 16; ++x) {
                const int y = wv + 4 * x;
                if (B.flip) {
                    // entry (r0 + y, k0 + lane) is T[n-1-k0-lane, n-1-r0-y]: lane along T's column
                    ta[x] = (r0 + y < r1 && k0 + lane < k1)
                                ? B.T[(n - 1 - k0 - lane) + (n - 1 - r0 - y) * B.ldt] : 0.0;
                } else {
                    ta[x] = (r0 + lane < r1 && k0 + y < k1) ? B.T[(r0 + lane) + (k0 + y) * B.ldt]
                                                            : 0.0;
                }
            }
            // Bs[kk * OP + cl] = Z[k0 + kk, OC c + cl]; As[kk * OP + r] = entry (r0 + r, k0 + kk)
#pragma unroll
            for (int x = 0; x < OC / 4; ++x) Bs[lane * OP + wv + 4 * x] = zb[x];
#pragma unroll
            for (int x = 0; x < 16; ++x) {
                const int y = wv + 4 * x;
                if (B.flip) As[lane * OP + y] = ta[x];
                else As[y * OP + lane] = ta[x];
            }
            __syncthreads();
#pragma unroll
            for (int y = 0; y < NPO; ++y) {
                if (!((mask >> (2 * y)) & 3)) continue;  // no group of this piece (uniform)
                for (int kk = 0; kk < 64; kk += 4)
                    d[y] = mfma_f64(As[(kk + kr) * OP + rb + cc], Bs[(kk + kr) * OP + 16 * y + cc],
                                    d[y]);
            }
            if (i == j + 2) {
                // block j is the last below block i: publish the mask's groups' sums
                // of block i
#pragma unroll
                for (int y = 0; y < NPO; ++y)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t row = r0 + rb + mfma64_row(lane, e);
                        const int cl = 16 * y + cc, col = OC * c + cl;
                        if (row < r1 && col < m && ((mask >> (cl / GC)) & 1))
                            coherent_store(B.acc + row + (int64_t)col * n, d[y][e]);
                    }
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (t < gn && ((mask >> t) & 1))
                    set_flag(S.accready + (beta * S.G + g0 + t) * S.nb + i);
            }
            __syncthreads();
            if (t < CG && ((mask >> t) & 1)) s_next[t] = j + 1;
        }
    }
}

__global__ __launch_bounds__(NT) void k_proj_run(ProjArgs a, ProjSync S)
{
    __shared__ double arena[3 * PB * TP + GC * ZCP + 3 * PB * ABP + MPM * LFP + 2 * GC * GC];
    __shared__ int yok;  // the eigenvector form is taken from block by on
    if ((int)blockIdx.x >= 2 * S.G) {
        proj_owner(a, S, arena, arena + PB * OP);
        return;
    }
    double *const Tt = arena;              // Tt[r * TP + c] = T[r0 + r, r0 + c], zero below the diagonal
    double *const Zr = Tt + PB * TP;       // the earlier columns' values on the block's rows: between
                                           // blocks, the window of block b - 1's minority rows,
                                           // Zr[k * TP + r] = Z[r0 + r, lo + k]; in the steps, that
                                           // of block b's own, Zr[r * TP + k] = Z[r0 + r, lo + k]
    double *const Pn = Zr + PB * TP;       // Pn[k * TP + r] = T[r0 + r, r1 + k], the panel below
    double *const Zc = Pn + PB * TP;       // Zc[k * ZCP + r] = Z[r0 + r, c0 + k], the group's columns
    double *const Ab = Zc + GC * ZCP;      // Ab[r * ABP + k]: the group's sums minus the coupling
                                           // with the columns of the blocks below
    double *const Cf = Ab + PB * ABP;      // Cf[r * ABP + k]: the coupling with the far columns
    double *const Lf = Cf + PB * ABP;      // Lf[l * LFP + k] = L[l, c0 + k], earlier columns l < c0
    double *const AbY = Lf + MPM * LFP;    // AbY[r * ABP + k] = (Ab V)[r, k] (eigenvector form)
    double *const Vg = AbY + PB * ABP;     // Vg[k * GC + l] = V[k, l]: L_gg V = V diag(L_gg)
    double *const Wg = Vg + GC * GC;       // Wg = V^-1

    const int beta = (int)blockIdx.x & 1, g = uniform((int)blockIdx.x >> 1);
    const ProjBasis B = a.b[beta];
    const int64_t n = a.n;
    const int m = a.m;
    const int c0 = g * GC;                 // the group's first column
    const int cw = uniform(min(GC, m - c0));  // its columns
    const int bs = uniform(S.bstart[beta * S.G + g]);
    const int *bst = S.bstart + beta * S.G;
    const int *const kx = S.kx + beta * (S.nb + 2);
    const int t = threadIdx.x, wv = uniform(t >> 6);
    const bool fl = B.flip != 0;
    int *const zdone = S.zdone + (beta * S.G + g) * S.nb;
    // The eigenvector form.  Above the group's topmost minority row (b_c0, in
    // block by - 1) the group's block L_gg of L is final; with L_gg V = V Lambda
    // (V unit upper triangular, Lambda its diagonal, the group's minority
    // eigenvalues), Y = Z_g V satisfies row by row
    //   (t_ii - lambda_l) y_il = (d V)_l,
    // d the coupling with the other columns minus the sums over the rows below:
    // the columns no longer couple to one another, so the chain of the row step
    // drops out.  In those blocks the group's sums Ab enter as Ab V, the walk
    // keeps Y in Zc and the near window's coefficients as L[l', g] V, and both go
    // back with V^-1 after the block.  Taken only when V is well conditioned
    // (max |V| max |V^-1| <= 1e3; distinct minority eigenvalues), else the
    // substitution keeps its chain to the top.
    const int by = uniform(B.pos[c0] >= 0 ? (int)((n - 1 - B.pos[c0]) / PB) + 1 : S.nb);
    if (t == 0) yok = 0;
    // Ab V into AbY (all waves, between the boundary's third and fourth barriers)
    auto ab_to_y = [&]() {
        for (int e = t; e < PB * GC; e += NT) {
            const int r = e >> 3, l = e & 7;
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < GC; ++k) v = fma(Ab[r * ABP + k], Vg[k * GC + l], v);
            AbY[r * ABP + l] = v;
        }
    };

    // The earlier columns by where their minority row lies: in block b (near), in
    // block b - 1 (prev), further down (far).  Columns are ordered by their row,
    // so each is a range.
    auto K = [&](int b) { return uniform(kx[b + 2]); };
    auto near = [&](int b) {
        const int lo = K(b);
        return Win{lo, min(K(b - 1), c0) - lo};
    };
    auto prev = [&](int b) {
        const int lo = K(b - 1);
        return Win{lo, min(K(b - 2), c0) - lo};
    };
    auto far = [&](int b) {
        const int lo = K(b - 2);
        return Win{lo, c0 - lo};
    };

    // Between blocks (all four waves): Ab += Pn^T Zc - Zr^T L[prev, group] - Cf,
    // with Zc still holding the group's rows of block b - 1 and Zr the prev
    // window's values on block b's rows; each wave 16 rows, the columns padded to 16.
    auto below_product = [&](int b) {
        const int lane = t & 63, kr = lane >> 4, cc = lane & 15, rb = 16 * wv;
        dx4 dd = dx4{0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < PB; k += 4) {
            const double av = Pn[(k + kr) * TP + rb + cc];
            const double bv = cc < GC ? Zc[cc * ZCP + k + kr] : 0.0;
            dd = mfma_f64(av, bv, dd);
        }
        const Win pw = prev(b);
        for (int k = 0; k < pw.cnt; k += 4) {
            const int kk = k + kr;
            const double bv = (cc < GC && kk < pw.cnt) ? -Lf[(pw.lo + kk) * LFP + cc] : 0.0;
            dd = mfma_f64(Zr[kk * TP + rb + cc], bv, dd);
        }
        const bool hf = far(b).cnt > 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = rb + mfma64_row(lane, e);
            if (cc < GC) Ab[r * ABP + cc] += hf ? dd[e] - Cf[r * ABP + cc] : dd[e];
        }
    };
    // The two roles run separate loops with the same barriers per block (four),
    // so that neither holds the other's registers.

    if (wv > 0) {
        // ==== waves 1..3: the next block's operands.  T's diagonal block and the
        // panel (inputs) are fetched into registers while the current block is
        // solved; so are the earlier groups' values on the next block's rows (the
        // near and prev windows, up to HWC columns each), with the far product, and
        // the group's far sums, when their flags are already set, and otherwise
        // after the boundary's first barrier.  (Only the inputs are fetched ahead
        // unconditionally: a wait before that barrier could close a cycle with the
        // owners, which wait for every group's earlier blocks.)
        double hT[HK], hP[HK], hN[HW], hV[HW], hA[HA];
        const int h = t - 64, hw = wv - 1;  // helper lane, helper wave
        auto fetch_inputs = [&](int b) {
            const int64_t r1 = blk_r1(n, b), r0 = blk_r0(n, b);
            const int nr = (int)(r1 - r0);
            const int nk = b > 0 ? (int)(blk_r1(n, b - 1) - r1) : 0;
#pragma unroll
            for (int k = 0; k < HK; ++k) {
                const int e = h + NH * k;
                int row, col;
                op_entry(fl, e, row, col);
                const bool in = e < PB * PB;
                hT[k] = (in && row < nr && col < nr && row <= col) ? B.T[toff(B, n, r0 + row, r0 + col)]
                                                                   : 0.0;
                hP[k] = (in && row < nr && col < nk) ? B.T[toff(B, n, r0 + row, r1 + col)] : 0.0;
            }
        };
        // the earlier groups' values on block b's rows: their flags (uniform test)
        auto coupling_ready = [&](int b) {
            int ok = 1;
            for (int gp = 0; gp < g; ++gp)
                if (bst[gp] <= b) ok &= flag_load(S.zdone + (beta * S.G + gp) * S.nb + b) != 0;
            return uniform(ok) != 0;
        };
        // a window's first HWC columns on block b's rows, into registers
        auto fetch_win = [&](int b, Win wn, double(&hv)[HW]) {
            const int64_t r1 = blk_r1(n, b), r0 = blk_r0(n, b);
            const int nr = (int)(r1 - r0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no load moves above the flags
#pragma unroll
            for (int k = 0; k < HW; ++k) {
                const int e = h + NH * k, col = e >> 6, row = e & 63;
                hv[k] = (col < wn.cnt && row < nr)
                            ? coherent_load(B.Z + (r0 + row) + (int64_t)(wn.lo + col) * n) : 0.0;
            }
        };
        // a window into Zr (k-major for the product between blocks, else row-major
        // for the steps), zeros up to the padding its reader takes; the columns past
        // HWC, or all of them when not fetched ahead, loaded now
        auto put_win = [&](int b, Win wn, const double(&hv)[HW], bool have, bool kmaj) {
            const int64_t r1 = blk_r1(n, b), r0 = blk_r0(n, b);
            const int nr = (int)(r1 - r0);
            const int cpad = kmaj ? (wn.cnt + 3) & ~3 : (wn.cnt + NQ - 1) / NQ * NQ;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
            for (int k = 0; k < HW; ++k) {
                const int e = h + NH * k, col = e >> 6, row = e & 63;
                if (col < cpad) {
                    double v = 0.0;
                    if (col < wn.cnt && row < nr)
                        v = have ? hv[k] : coherent_load(B.Z + (r0 + row) + (int64_t)(wn.lo + col) * n);
                    if (kmaj) Zr[col * TP + row] = v;
                    else Zr[row * TP + col] = v;
                }
            }
            for (int e = h + HW * NH; e < cpad * PB; e += NH) {
                const int col = e >> 6, row = e & 63;
                const double v = (col < wn.cnt && row < nr)
                                     ? coherent_load(B.Z + (r0 + row) + (int64_t)(wn.lo + col) * n) : 0.0;
                if (kmaj) Zr[col * TP + row] = v;
                else Zr[row * TP + col] = v;
            }
        };
        // Cf = Z[block b, far] L[far, group] (FP64 MFMA, operands straight from
        // memory and from Lf; helper wave 0 takes the 16-row pieces 0 and 3, waves 1
        // and 2 the pieces 1 and 2).  Lf holds the far columns' coefficients: their
        // rows were solved at least a block ago.
        auto far_product = [&](int b) {
            const Win fw = far(b);
            if (fw.cnt <= 0) return;
            const int64_t r1 = blk_r1(n, b), r0 = blk_r0(n, b);
            const int nr = (int)(r1 - r0);
            const int lane = t & 63, kr = lane >> 4, cc = lane & 15;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            for (int p = hw; p < 4; p += 3) {
                const int rr = 16 * p + cc;
                const double *zp = B.Z + (r0 + rr) + (int64_t)fw.lo * n;
                dx4 dd = dx4{0.0, 0.0, 0.0, 0.0};
                for (int k0 = 0; k0 < fw.cnt; k0 += 32) {
                    double av[8], bv[8];
#pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        const int kk = k0 + 4 * s + kr;
                        const bool in = kk < fw.cnt;
                        av[s] = (in && rr < nr) ? coherent_load(zp + (int64_t)kk * n) : 0.0;
                        bv[s] = (in && cc < GC) ? Lf[(fw.lo + kk) * LFP + cc] : 0.0;
                    }
#pragma unroll
                    for (int s = 0; s < 8; ++s) dd = mfma_f64(av[s], bv[s], dd);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (cc < GC) Cf[(16 * p + mfma64_row(lane, e)) * ABP + cc] = dd[e];
            }
        };
        // the group's sums over the blocks j <= b - 2, from their owner
        auto acc_ready = [&](int b) {
            return uniform(flag_load(S.accready + (beta * S.G + g) * S.nb + b) != 0) != 0;
        };
        auto fetch_acc = [&](int b) {
            const int64_t r1 = blk_r1(n, b), r0 = blk_r0(n, b);
            const int nr = (int)(r1 - r0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
            for (int k = 0; k < HA; ++k) {
                const int e = h + NH * k, c = e >> 6, row = e & 63;
                hA[k] = (c < cw && row < nr) ? coherent_load(B.acc + (r0 + row) + (int64_t)(c0 + c) * n)
                                             : 0.0;
            }
        };
        bool have_c = false, have_a = false;
        fetch_inputs(bs);
        for (int b = bs; b < S.nb; ++b) {
            __syncthreads();  // (1) wave 0 has solved block b - 1 (and set Lf for its rows)
#pragma unroll
            for (int k = 0; k < HK; ++k) {
                const int e = h + NH * k;
                int row, col;
                op_entry(fl, e, row, col);
                if (e < PB * PB) {
                    Tt[row * TP + col] = hT[k];
                    Pn[col * TP + row] = hP[k];  // k-major
                }
            }
            if (!have_c) {
                for (int gp = 0; gp < g; ++gp)
                    if (bst[gp] <= b) wave_wait(S.zdone + (beta * S.G + gp) * S.nb + b, S);
                far_product(b);
            }
            if (b > bs) put_win(b, prev(b), hV, have_c, true);
            const bool farsum = b - 2 >= bs;
            if (farsum && !have_a) {
                wave_wait(S.accready + (beta * S.G + g) * S.nb + b, S);
                fetch_acc(b);
            }
#pragma unroll
            for (int k = 0; k < HA; ++k) {
                const int e = h + NH * k, c = e >> 6, row = e & 63;
                if (c < GC) Ab[row * ABP + c] = farsum ? hA[k] : 0.0;
            }
            __syncthreads();  // (2)
            if (b > bs) below_product(b);
            __syncthreads();  // (3)
            for (int e = t; e < GC * ZCP; e += NT) Zc[e] = 0.0;
            put_win(b, near(b), hN, have_c, false);
            if (b >= by && uniform(yok) != 0) ab_to_y();
            __syncthreads();  // (4)
            have_c = have_a = false;
            if (b + 1 < S.nb) {
                fetch_inputs(b + 1);
                if (coupling_ready(b + 1)) {
                    fetch_win(b + 1, near(b + 1), hN);
                    fetch_win(b + 1, prev(b + 1), hV);
                    far_product(b + 1);
                    have_c = true;
                }
                if (b + 1 - 2 >= bs && acc_ready(b + 1)) {
                    fetch_acc(b + 1);
                    have_a = true;
                }
            }
        }
        __syncthreads();  // wave 0 has solved the top block
        return;
    }

    // ==== wave 0: the group's columns, block after block.  Per column: the
    // coefficients L[lo + NQ u + q][l] of the near window's columns (lreg; zero at
    // the block's start, set at their rows, stored to Lf after the block) and
    // L[c0 + k'][l] of the group's own earlier columns (k' < kw), in every lane
    // of the column; L[l][l] (t at row b_l, set at that row).
    const int kw = (t & 63) / NQ, q = t % NQ;
    double lreg[NU], lw[GC], lamll = 0.0;
#pragma unroll
    for (int kp = 0; kp < GC; ++kp) lw[kp] = 0.0;
    const int pl = kw < cw ? B.pos[c0 + kw] : -1;
    const double *const zcol = Zc + kw * ZCP + q;

    // the group's rows of block b, stored at the end of its wavefront; their flag
    // is set after the next barrier, once the stores have completed
    auto store_rows = [&](int b) {
        const int64_t p0 = blk_r0(n, b), p1 = blk_r1(n, b);
#pragma unroll
        for (int k = 0; k < GC; ++k)
            if (k < cw && p0 + (t & 63) < p1)
                coherent_store(B.Z + (p0 + (t & 63)) + (int64_t)(c0 + k) * n, Zc[k * ZCP + (t & 63)]);
    };
    auto flag_rows = [&](int b) {
        __builtin_amdgcn_s_waitcnt(0);
        if (t == 0) set_flag(S.zdone + (beta * S.G + g) * S.nb + b);
    };
    for (int b = bs; b < S.nb; ++b) {
        const int64_t r1 = blk_r1(n, b), r0 = blk_r0(n, b);
        const int nr = (int)(r1 - r0);
        const Win nw = near(b);
        // the block's row types, lane i holding row i's (loaded ahead of its use)
        const int rtl = (t & 63) < nr ? B.rowtype[r0 + (t & 63)] : -1;
        __syncthreads();  // (1)
        if (b > bs) flag_rows(b - 1);
        __syncthreads();  // (2) the helpers have staged block b's operands
        if (b > bs) below_product(b);
        __syncthreads();  // (3)
        for (int e = t; e < GC * ZCP; e += NT) Zc[e] = 0.0;
        const bool yf = b >= by && uniform(yok) != 0;  // the eigenvector form (uniform)
        if (yf) ab_to_y();
        __syncthreads();  // (4)
#pragma unroll
        for (int u = 0; u < NU; ++u) lreg[u] = 0.0;

        // Row by row from the bottom; every column of the group takes the same row.
        // A column's sum for row r takes the rows below it within the block (its
        // own column) and the near window's values on row r (chunks u < NCU); the
        // coupling among the group's own columns, still zero in that sum, is solved
        // after the reduction, column by column.  At a minority row that coupling is
        // zero (the row of Z is e_typ and L's row typ is not set yet), so only
        // majority rows take that chain.  A column is active on the rows at and above
        // its minority row.
        //
        // Pipelined: while row r is solved, the sum of row r - 1 is formed (its LDS
        // reads, the multiply-adds and the reduction) from what is known before row
        // r: every term but the one of row r itself, -t[r-1][r] z_r, which is added
        // once z_r is known (one multiply-add on the chain from row to row).  A
        // minority row changes L (and so row r - 1's coupling terms, coefficients or
        // divisor): after one, row r - 1's sum is formed again, with z_r included.
        // One wave: the LDS reads see the earlier stores in program order, with no
        // barrier.
        const int plr = pl < r0 ? -1 : (int)(pl - r0 < PB ? pl - r0 : PB);
        const int rhi = kw < cw ? (plr < nr - 1 ? plr : nr - 1) : -1;  // last row it computes
        auto front = [&](auto gtag, auto guardtag, auto ytag) {
        constexpr int NCU = decltype(gtag)::value;  // coupling chunks: the near window's
        constexpr bool GUARD = decltype(guardtag)::value;  // reciprocals checked for range
        constexpr bool YF = decltype(ytag)::value;  // the eigenvector form: no chain
        // Row r's prepared state: dpart = coupling - sum without row r + 1's term,
        // tnext = t[r][r+1] (that term's coefficient; 0 when already included or
        // outside the block), t_rr and 1 / (t_rr - L[l, l]).
        struct Prep {
            double dpart, tnext, tii, rcp;
        };
        auto prep = [&](int r, bool included) {
            Prep P;
            int ro = r * TP;
            // opaque to loop strength reduction: one base address for the step's
            // reads of both rows, with immediate offsets
            asm volatile("" : "+v"(ro));
            const double *trow = Tt + ro;
            const double *zrow = Zr + ro;
            double tv[NU], zv[NU], rv[NCU > 0 ? NCU : 1];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                tv[u] = trow[NQ * u + q];
                zv[u] = zcol[NQ * u];
                if (u < NCU) rv[u] = zrow[NQ * u + q];
            }
            P.tii = trow[r];
            // (read from an address inside the row in every case, then chosen)
            const double tn = trow[r + 1 < PB ? r + 1 : r];
            P.tnext = (!included && r + 1 < nr) ? tn : 0.0;
            // (the group's sum of the row, read by all the column's lanes: a broadcast)
            const double ab = (YF ? AbY : Ab)[r * ABP + kw];
            // 1 / (t_ii - L[l, l]): the hardware estimate (relative error below 5e-8)
            // and one Newton step, which squares it (below 2.3e-15).  The signs of
            // t_ii and L[l, l] differ, so |dx| >= min |t_kk| and |dx| <= 2 max |t_kk|;
            // only when the diagonal leaves [2^-1020, 2^1019] (the GUARD instances) can
            // |dx| leave [2^-1020, 2^1020], where the estimate or its reciprocal would
            // not be normal: then the IEEE division for those entries
            const double dx = P.tii - lamll;
            double rcp = __builtin_amdgcn_rcp(dx);
            rcp = fma(rcp, fma(-dx, rcp, 1.0), rcp);
            if constexpr (GUARD) {
                const double adx = fabs(dx);
                if (adx > 0x1p1020 || adx < 0x1p-1020) rcp = 1.0 / dx;
            }
            P.rcp = rcp;
            double v0 = q == 0 ? ab : 0.0, v1 = 0.0, cp0 = 0.0, cp1 = 0.0;
#pragma unroll
            for (int u = 0; u < NU; u += 2) {
                v0 += tv[u] * zv[u];
                v1 += tv[u + 1] * zv[u + 1];
            }
#pragma unroll
            for (int u = 0; u < NCU; u += 2) {
                cp0 += rv[u] * lreg[u];
                if (u + 1 < NCU) cp1 += rv[u + 1] * lreg[u + 1];
            }
            // coupling (near window) - sum
            P.dpart = group_sum<NQ>((cp0 + cp1) - (v0 + v1));
            return P;
        };
        // One row: solve row r with its prepared state Pc while row r - 1's is
        // prepared into Pnx.  The loop below takes two rows per iteration with the
        // two states in fixed roles, so that no state is copied from row to row.
        double zprev = 0.0;  // z of the row below, in every lane of its column
        auto step = [&](int r, const Prep &Pc, Prep &Pnx) {
            // The common case, a majority row, in one straight run of code (the next
            // row's sum, formed from what is known before this row is solved, and
            // this row's coupling chain, independent of each other), so that the
            // compiler can interleave the two; a minority row replaces the result
            // afterwards.  (Row 0 prepares row 0 again: unused.)
            Pnx = prep(r > 0 ? r - 1 : 0, false);
            const bool act = r <= rhi;
            // d = coupling - sum, with row r + 1's term
            const double d = fma(-Pc.tnext, zprev, Pc.dpart);
            // z_l = (d_l + sum_{k' < k} z_k' L[k', l]) / (t_ii - L[l, l]) over the
            // group's columns in order, with the reciprocal folded into the
            // coefficients (one multiply-add per link).  Every link runs: an inactive
            // column's z is zero, and lw is zero from the diagonal on and for the
            // coefficients not set yet, so those links add exact zeros.
            // (the chain's coefficients with the reciprocal folded in, formed off the
            // chain)
            double lwr[GC - 1];
#pragma unroll
            for (int kp = 0; kp < GC - 1; ++kp) lwr[kp] = lw[kp] * Pc.rcp;
            double z = act ? d * Pc.rcp : 0.0;
            if constexpr (!YF) {
#pragma unroll
                for (int kp = 0; kp < GC - 1; ++kp) z = fma(readlane_f64(z, kp * NQ), lwr[kp], z);
            }
            const int typ = __builtin_amdgcn_readlane(rtl, r);
            const bool minority = typ >= 0;  // (uniform)
            if (minority) {
                // At minority row b_typ the row of Z is e_typ: z is 1 in column typ's
                // own lanes and 0 elsewhere, and the row defines row typ of L (for
                // the active columns only: an inactive one's column of L stays as is).
                const bool own = act && r == plr;
                z = own ? 1.0 : 0.0;
                if (own) {
                    lamll = Pc.tii;
                } else if (act) {
                    if (typ < c0) {
                        // an earlier column of the near window
                        const int idx = typ - nw.lo;
#pragma unroll
                        for (int u = 0; u < NU; ++u)
                            if (NQ * u + q == idx) lreg[u] = -d;
                    } else {
#pragma unroll
                        for (int kp = 0; kp < GC; ++kp)
                            if (c0 + kp == typ) lw[kp] = -d;
                    }
                }
            }
            if (q == 0 && act) Zc[kw * ZCP + r] = z;
            // The column's other lanes read this value from LDS in later steps, with
            // no barrier: the hardware keeps one wave's LDS operations in order, and
            // this fence (wavefront scope: no instruction) keeps the compiler from
            // moving those reads above the store.
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            // after a minority row, row r - 1's sum again, with the state L has now
            // and z_r included
            if (minority && r > 0) Pnx = prep(r - 1, true);
            zprev = z;
        };
        Prep P0 = prep(nr - 1, false), P1;
        int s2 = 0;
        for (; s2 + 1 < nr; s2 += 2) {
            step(nr - 1 - s2, P0, P1);
            step(nr - 2 - s2, P1, P0);
        }
        if (s2 < nr) step(nr - 1 - s2, P0, P1);
        };
        // The eigenvector form, column-oriented: the group's columns are
        // independent triangular systems (T_bb - lambda_l I) y_l = -AbY_l + (the
        // coupling with the near window's columns) over the block's rows.  Lane
        // (kw, q) keeps the running sums s_i = AbY[i] + sum_{j > i} t_ij y_j -
        // sum_c Zr[i][c] L[c] of its rows i = q + 8u in registers; row r's owner
        // (q = r mod 8) forms y_r = -s_r / (t_rr - lambda_l), the column's lanes
        // receive it by a swizzle and add t_ir y_r to the rows above.  Only the
        // owner's multiply, the swizzle and the next row's multiply-add are on the
        // chain from row to row (no reduction).  A minority row of a near-window
        // column c instead sets that column's coefficient L[c] = s_r (the group's
        // y_r is zero there) and subtracts Zr[i][c] L[c] from the rows above.
        auto walk_y = [&](auto mintag) {
            constexpr bool MIN = decltype(mintag)::value;  // the block holds minority rows
            const bool on = kw < cw;
            double sv[NU], rv[NU];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int i = NQ * u + q;
                sv[u] = (on && i < nr) ? AbY[i * ABP + kw] : 0.0;
                rv[u] = (on && i < nr) ? 1.0 / (Tt[i * TP + i] - lamll) : 0.0;
            }
            // T's diagonal now lives in the reciprocals: zero it, so that row r's
            // update may run over every slot of every lane (t_ir = 0 for i >= r; the
            // owner's own slot keeps s_r, from which y_r is formed again at the end)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if (kw == 0)
#pragma unroll
                for (int u = 0; u < NU; ++u) Tt[(NQ * u + q) * (TP + 1)] = 0.0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            // T's column of the next row, loaded one row ahead (two register sets
            // in turn, chosen by the row's parity)
            double ta[NU], tb[NU];
#pragma unroll
            for (int u = 0; u < NU; ++u) ta[u] = Tt[(NQ * u + q) * TP + (PB - 1)];
            auto row = [&](auto ut, auto qt) {
                constexpr int u = decltype(ut)::value, qq = decltype(qt)::value;
                constexpr int r = NQ * u + qq;
                double(&tc)[NU] = (qq & 1) ? ta : tb;  // row r's column (row 63: ta)
                double(&tn)[NU] = (qq & 1) ? tb : ta;
                auto prefetch = [&] {
                    if constexpr (r > 0) {
#pragma unroll
                        for (int v = 0; v < NU; ++v) tn[v] = Tt[(NQ * v + q) * TP + (r - 1)];
                    }
                };
                if (r >= nr) {  // (uniform: the top block may be short)
                    prefetch();
                    return;
                }
                if constexpr (MIN) {
                    const int typ = __builtin_amdgcn_readlane(rtl, r);
                    if (typ >= 0) {
                        // a near-window column's minority row (uniform branch); that
                        // column's z is zero below the row and one at it, where the
                        // owner's slot is then reset (the group's y_r is zero)
                        prefetch();
                        const int cn = typ - nw.lo;
                        const double lc = bcast8_f64<qq>(sv[u]);
                        if (on)
#pragma unroll
                            for (int w = 0; w < NU; ++w)
                                if (NQ * w + q == cn) lreg[w] = lc;
#pragma unroll
                        for (int v = 0; v <= u; ++v)
                            sv[v] = fma(-Zr[(NQ * v + q) * TP + cn], lc, sv[v]);
                        if (q == qq) sv[u] = 0.0;
                        return;
                    }
                }
                // the broadcast ahead of the next column's loads (LDS returns in
                // order), and first the update of row r - 1's own slot, which the next
                // row's broadcast waits for
                const double y = bcast8_f64<qq>(-sv[u] * rv[u]);
                prefetch();
                constexpr int vn = qq > 0 ? u : u - 1;
                if constexpr (vn >= 0) sv[vn] = fma(tc[vn], y, sv[vn]);
#pragma unroll
                for (int v = 0; v <= u; ++v)
                    if (v != vn) sv[v] = fma(tc[v], y, sv[v]);
            };
            auto rows8 = [&](auto ut) {
                row(ut, std::integral_constant<int, 7>{});
                row(ut, std::integral_constant<int, 6>{});
                row(ut, std::integral_constant<int, 5>{});
                row(ut, std::integral_constant<int, 4>{});
                row(ut, std::integral_constant<int, 3>{});
                row(ut, std::integral_constant<int, 2>{});
                row(ut, std::integral_constant<int, 1>{});
                row(ut, std::integral_constant<int, 0>{});
            };
            rows8(std::integral_constant<int, 7>{});
            rows8(std::integral_constant<int, 6>{});
            rows8(std::integral_constant<int, 5>{});
            rows8(std::integral_constant<int, 4>{});
            rows8(std::integral_constant<int, 3>{});
            rows8(std::integral_constant<int, 2>{});
            rows8(std::integral_constant<int, 1>{});
            rows8(std::integral_constant<int, 0>{});
            // y of each lane's rows from their final sums (the value the row's
            // broadcast carried; +0 at a minority row, whose sum was reset)
            if (on)
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    const int i = NQ * u + q;
                    if (i < nr) Zc[kw * ZCP + i] = fma(-sv[u], rv[u], 0.0);
                }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        };
        static_assert(NU == 8, "one instance per chunk count");
        // (one instance per chunk count, reciprocal check and form)
        auto front2 = [&](auto gtag) {
            if (S.rcp_guard) {
                if (yf) front(gtag, std::true_type{}, std::true_type{});
                else front(gtag, std::true_type{}, std::false_type{});
            } else {
                if (yf) front(gtag, std::false_type{}, std::true_type{});
                else front(gtag, std::false_type{}, std::false_type{});
            }
        };
        if (yf) {
            if (uniform(nw.cnt) > 0) walk_y(std::true_type{});
            else walk_y(std::false_type{});
        } else switch (uniform(nw.cnt > 0 ? (nw.cnt + NQ - 1) / NQ : 0)) {
            case 0: front2(std::integral_constant<int, 0>{}); break;
            case 1: front2(std::integral_constant<int, 1>{}); break;
            case 2: front2(std::integral_constant<int, 2>{}); break;
            case 3: front2(std::integral_constant<int, 3>{}); break;
            case 4: front2(std::integral_constant<int, 4>{}); break;
            case 5: front2(std::integral_constant<int, 5>{}); break;
            case 6: front2(std::integral_constant<int, 6>{}); break;
            case 7: front2(std::integral_constant<int, 7>{}); break;
            default: front2(std::integral_constant<int, 8>{}); break;
        }
        const int lane = t & 63;
        if (yf) {
            // the block's rows back from Y to Z = Y V^-1 (lane i: row i; V^-1 unit upper)
            double yv[GC];
#pragma unroll
            for (int k = 0; k < GC; ++k) yv[k] = Zc[k * ZCP + lane];
#pragma unroll
            for (int l = 0; l < GC; ++l) {
                double v = yv[l];
#pragma unroll
                for (int k = 0; k < l; ++k) v = fma(yv[k], Wg[k * GC + l], v);
                Zc[l * ZCP + lane] = v;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        store_rows(b);
        // the near window's coefficients, for the products of the blocks above
        // (read after the next barrier)
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int c = NQ * u + q;
            if (c < nw.cnt) Lf[(nw.lo + c) * LFP + kw] = lreg[u];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (yf && lane < nw.cnt) {
            // L[l', g] V back to L[l', g] (lane c: window column lo + c)
            double lv[GC];
#pragma unroll
            for (int k = 0; k < GC; ++k) lv[k] = Lf[(nw.lo + lane) * LFP + k];
#pragma unroll
            for (int l = 0; l < GC; ++l) {
                double v = lv[l];
#pragma unroll
                for (int k = 0; k < l; ++k) v = fma(lv[k], Wg[k * GC + l], v);
                Lf[(nw.lo + lane) * LFP + l] = v;
            }
        }
        if (b == by - 1 && by < S.nb) {
            // L_gg is final: V (L_gg V = V Lambda, unit upper), V^-1, and whether
            // the form is well conditioned.  L_gg goes through Wg; column kw of V and
            // of V^-1 in the registers of column kw's lanes.
            if (q == 0)
#pragma unroll
                for (int kp = 0; kp < GC; ++kp)
                    Wg[kp * GC + kw] = kp < kw ? lw[kp] : (kp == kw ? lamll : 0.0);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const bool on = kw < cw;
            double vc[GC], wc[GC];
#pragma unroll
            for (int k = 0; k < GC; ++k) vc[k] = k == kw ? 1.0 : 0.0;
            const double lam = Wg[kw * GC + kw];
#pragma unroll
            for (int k = GC - 2; k >= 0; --k) {
                double sum = 0.0;
#pragma unroll
                for (int j = k + 1; j < GC; ++j) sum = fma(Wg[k * GC + j], vc[j], sum);
                if (on && k < kw) vc[k] = sum / (lam - Wg[k * GC + k]);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if (q == 0)
#pragma unroll
                for (int k = 0; k < GC; ++k) Vg[k * GC + kw] = vc[k];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int k = 0; k < GC; ++k) wc[k] = k == kw ? 1.0 : 0.0;
#pragma unroll
            for (int k = GC - 2; k >= 0; --k) {
                double sum = 0.0;
#pragma unroll
                for (int j = k + 1; j < GC; ++j) sum = fma(Vg[k * GC + j], wc[j], sum);
                if (on && k < kw) wc[k] = -sum;
            }
            double vmax = 0.0, wmax = 0.0;
#pragma unroll
            for (int k = 0; k < GC; ++k) {
                vmax = fmax(vmax, fabs(vc[k]));  // (fmax drops a NaN: tested below)
                wmax = fmax(wmax, fabs(wc[k]));
            }
            bool fin = true;
#pragma unroll
            for (int k = 0; k < GC; ++k) fin = fin && isfinite(vc[k]) && isfinite(wc[k]);
            const bool good = __builtin_amdgcn_ballot_w64(!(fin && vmax * wmax <= 1e3)) == 0;
            double vm = vmax, wm = wmax;
#pragma unroll
            for (int kp = 0; kp < GC; ++kp) {
                vm = fmax(vm, readlane_f64(vmax, kp * NQ));
                wm = fmax(wm, readlane_f64(wmax, kp * NQ));
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if (q == 0)
#pragma unroll
                for (int k = 0; k < GC; ++k) Wg[k * GC + kw] = wc[k];
            if (t == 0) yok = (good && vm * wm <= 1e3) ? 1 : 0;
        }
    }
    __syncthreads();
    flag_rows(S.nb - 1);
}

// The upper block triangle of an mp x mp matrix in 64 x 64 tiles (mp = 64 nc),
// numbered row by row: tile (a, c), a <= c, is number a nc - a (a - 1) / 2 + c - a.
__host__ __device__ inline int utile_index(int a, int c, int nc) { return a * nc - a * (a - 1) / 2 + (c - a); }
__device__ inline void utile_of(int idx, int nc, int &a, int &c)
{
    a = 0;
    while (idx >= nc - a) {
        idx -= nc - a;
        ++a;
    }
    c = a + idx;
}

// Partial W^T Z: part[(p * ntiles + tile) * 4096 + r * 64 + c] = sum over the rows
// j of part p (rows [p rpp, p rpp + rpp), rpp a multiple of 64) of W[j, 64 a + r]
// Z[j, 64 c + c'] for tile (a, c) (blockIdx.y).  W[j, l] = Zf[n-1-j, m-1-l] with
// Zf the basis of the flipped matrix.  W^T Z is upper triangular (W[j, l] = 0
// for j < b_l, Z[j, l'] = 0 for j > b_l'), so only tiles a <= c are formed.
__global__ __launch_bounds__(256) void k_proj_gram(const double *__restrict__ Z,
                                                   const double *__restrict__ Zf, int64_t n, int m,
                                                   int nc, int64_t rpp, double *__restrict__ part)
{
    __shared__ double As[64 * OP];  // As[k * OP + l]  = W[j0 + k, 64 a + l]
    __shared__ double Bs[64 * OP];  // Bs[k * OP + l'] = Z[j0 + k, 64 c + l']
    int ta = 0, tc = 0;
    utile_of((int)blockIdx.y, nc, ta, tc);
    ta = uniform(ta);
    tc = uniform(tc);
    const int t = threadIdx.x, lr = t & 63, q = t >> 6;
    const int la = 64 * ta + lr, lc = 64 * tc + lr;
    dx4 d[2][2];
    mm64_acc_zero(d);
    const int64_t jb = (int64_t)blockIdx.x * rpp, je = std::min<int64_t>(n, jb + rpp);
    for (int64_t j0 = jb; j0 < je; j0 += 64) {
        for (int k = q; k < 64; k += 4) {
            const int64_t j = j0 + k;
            As[k * OP + lr] = (j < n && la < m) ? Zf[(n - 1 - j) + (int64_t)(m - 1 - la) * n] : 0.0;
            Bs[k * OP + lr] = (j < n && lc < m) ? Z[j + (int64_t)lc * n] : 0.0;
        }
        __syncthreads();
        mm64_acc<OP, OP>(As, Bs, d);
        __syncthreads();
    }
    const int lane = t & 63, w = t >> 6;
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
    double *out = part + ((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * 4096;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = rb + 16 * x + mfma64_row(lane, e);
                const int c = cb + 16 * y + (lane & 15);
                out[r * 64 + c] = d[x][y][e];
            }
}

// M = sum of the partials, row-major with pitch mp (one entry per thread,
// coalesced over the partials); zero below the block diagonal, the identity
// beyond the leading m x m block.
__global__ __launch_bounds__(64) void k_proj_gsum(const double *__restrict__ part, int nparts,
                                                  int m, int mp, double *__restrict__ M)
{
    const int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int r = (int)(e / mp), c = (int)(e % mp);
    const int nc = mp / 64, ntiles = nc * (nc + 1) / 2;
    double s = 0.0;
    if (r < m && c < m) {
        if (r / 64 <= c / 64) {
            const int64_t off = (int64_t)utile_index(r / 64, c / 64, nc) * 4096 + (r % 64) * 64 + c % 64;
            const int64_t stride = (int64_t)ntiles * 4096;
            // eight independent partial sums, so that the loads are issued ahead
            double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int g = 0;
            for (; g + 8 <= nparts; g += 8)
#pragma unroll
                for (int k = 0; k < 8; ++k) p[k] += part[(int64_t)(g + k) * stride + off];
            for (; g < nparts; ++g) p[0] += part[(int64_t)g * stride + off];
            s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
        }
    } else {
        s = r == c ? 1.0 : 0.0;
    }
    M[e] = s;
}

// Minv = M^-1 for the upper triangular M of order 64 (unit diagonal on the leading
// m x m block, identity beyond; zero below the diagonal), by elimination from the
// last row up: row k of the inverse is row k of the running right-hand side R
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

// Minv = M^-1 for the same kind of M of order mp > 64 (pitch mp): one wave per
// column c, by substitution from row c up: x_c = 1 / M[c][c] and
// x_k = -(sum_{k < j <= c} M[k][j] x_j) / M[k][k] for k = c - 1 down to 0.  Lane
// i keeps x_{i + 64 p}; the x not yet computed (and those beyond c) are zero, so
// each row's sum runs over all of them.  The sum is reduced in a fixed order.
__global__ __launch_bounds__(256) void k_proj_minv_col(const double *__restrict__ M, int mp,
                                                       double *__restrict__ minv)
{
    constexpr int NPX = MPM / 64;
    const int lane = threadIdx.x & 63;
    const int c = uniform((int)blockIdx.x * 4 + ((int)threadIdx.x >> 6));
    if (c >= mp) return;
    double x[NPX];
#pragma unroll
    for (int p = 0; p < NPX; ++p) x[p] = 0.0;
    const double xc = 1.0 / M[(int64_t)c * mp + c];
#pragma unroll
    for (int p = 0; p < NPX; ++p)
        if (lane + 64 * p == c) x[p] = xc;
    for (int k = c - 1; k >= 0; --k) {
        const double *row = M + (int64_t)k * mp;
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < NPX; ++p)
            if (64 * p < mp) s = fma(row[lane + 64 * p], x[p], s);
        s = group_sum<16>(s);
        s = (readlane_f64(s, 0) + readlane_f64(s, 16)) + (readlane_f64(s, 32) + readlane_f64(s, 48));
        const double xk = -s / row[k];
#pragma unroll
        for (int p = 0; p < NPX; ++p)
            if (lane + 64 * p == k) x[p] = xk;
    }
#pragma unroll
    for (int p = 0; p < NPX; ++p)
        if (lane + 64 * p < mp) minv[(int64_t)(lane + 64 * p) * mp + c] = x[p];
}

// A = Z Minv over the rows [64 g, 64 g + 64) and the columns [64 lb, 64 lb + 64)
// (blockIdx.y = lb): A[i, l] = sum_k Z[i, k] Minv[k][l], over k < 64 lb + 64
// (Minv is upper triangular; the identity beyond m, where Z's columns are zero).
// Computed as the transposed product C[l][i] = sum_k Minv[k][l] Z[i, k] (FP64
// MFMA), so that the accumulator's lanes run down A's columns.
__global__ __launch_bounds__(256) void k_proj_a(const double *__restrict__ Z,
                                                const double *__restrict__ minv, int64_t n, int mp,
                                                double *__restrict__ A)
{
    __shared__ double Ms[64 * OP];  // Ms[k * OP + l]  = Minv[64 kb + k][64 lb + l]
    __shared__ double Zs[64 * OP];  // Zs[k * OP + ii] = Z[i0 + ii, 64 kb + k]
    const int t = threadIdx.x, lr = t & 63, q = t >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int lb = (int)blockIdx.y;
    dx4 d[2][2];
    mm64_acc_zero(d);
    for (int kb = 0; kb <= lb; ++kb) {
        for (int k = q; k < 64; k += 4) {
            const int64_t i = i0 + lr;
            Ms[k * OP + lr] = minv[(int64_t)(64 * kb + k) * mp + 64 * lb + lr];
            Zs[k * OP + lr] = i < n ? Z[i + (int64_t)(64 * kb + k) * n] : 0.0;
        }
        __syncthreads();
        mm64_acc<OP, OP>(Ms, Zs, d);
        __syncthreads();
    }
    const int lane = t & 63, w = t >> 6;
    const int rb = (w >> 1) * 32, cb = (w & 1) * 32;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int l = 64 * lb + rb + 16 * x + mfma64_row(lane, e);
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

// flags of the persistent run: two per block, group and basis, and the error word
size_t proj_sync_bytes(int64_t n, int m)
{
    const int64_t G = (std::max(1, m) + GC - 1) / GC;
    return (size_t)(4 * G * ((n + PB - 1) / PB) + 1) * sizeof(int);
}

namespace {

// The complex form's workspace (at most PM minority columns).
size_t projc_workspace_bytes(int64_t n)
{
    const size_t nn = (size_t)n, es = 16;
    const size_t nparts = (nn + 63) / 64;
    return 4 * al(nn * PM * es)             // Z and acc, two bases
           + 2 * al(PM * PM * es)           // L, two bases
           + 2 * al(nn * 4) + 2 * al(PM * 4)  // row types and minority rows
           + al(nparts * PM * PM * es)      // partial Gram matrices
           + al(PM * PM * es)               // Minv
           + al(nn * PM * es);              // A
}

}  // namespace

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
    hipLaunchKernelGGL(k_proj_prep, dim3(1), dim3(1024), 0, st, sgn, n, minority, m, PM, 0, rt0, ps0,
                       rt1, ps1, (int *)nullptr);
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

// Owners per basis for a persistent run over nb blocks with G column groups (2 G
// fronts): every workgroup must be resident at once (one per compute unit: the
// front's LDS arena leaves room for no second one).  False when the fronts and
// at least one owner per basis do not fit.
bool proj_grid(int64_t nb, int cus, int G, int *nown)
{
    const int fronts = 2 * G;
    if (fronts > cus) return false;
    const int64_t tasks = (nb > 2 ? nb - 2 : 0) * ((G + CG - 1) / CG);
    if (tasks == 0) {
        *nown = 0;
        return true;
    }
    const int64_t slots = (int64_t)(cus - fronts) / 2;
    if (slots < 1) return false;
    *nown = (int)std::min<int64_t>(slots, tasks);
    return true;
}

bool proj_fits(int64_t n, int m)
{
    int nown = 0;
    return n >= 2 && m >= 1 && m <= MPM &&
           proj_grid((n + PB - 1) / PB, device_cus(), (m + GC - 1) / GC, &nown);
}

namespace {

// The real form's workspace, in the order run_proj takes it.
struct ProjLayout {
    int mp, nc, ntiles, nparts;
    int64_t nb, rpp;
    size_t bytes;
};

ProjLayout proj_layout(int64_t n, int m)
{
    ProjLayout L;
    L.mp = (std::max(1, std::min(m, MPM)) + 63) / 64 * 64;
    L.nc = L.mp / 64;
    L.ntiles = L.nc * (L.nc + 1) / 2;
    L.nb = (n + PB - 1) / PB;
    // partial sums of W^T Z over row ranges: about 256 workgroups in all
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>(L.nb, 256 / L.ntiles));
    L.rpp = (L.nb + want - 1) / want * PB;
    L.nparts = (int)((n + L.rpp - 1) / L.rpp);
    const size_t nn = (size_t)n, mp = (size_t)L.mp;
    L.bytes = 4 * al(nn * mp * 8)                       // Z and acc, two bases
              + 2 * al(nn * 4) + 2 * al(mp * 4)         // row types and minority rows
              + al((size_t)2 * (L.nb + 2) * 4)          // K(b) of both bases
              + al((size_t)L.nparts * L.ntiles * 4096 * 8)  // partial Gram matrices
              + 2 * al(mp * mp * 8)                     // W^T Z and its inverse
              + al(nn * mp * 8)                         // A
              + al(proj_sync_bytes(n, m));              // flags
    return L;
}

}  // namespace

int run_proj(const double *T, int64_t ldt, double *U, int64_t ldu, int64_t n, const int8_t *sgn,
             const int8_t *hsgn, int minority, int m, double flops, void *ws, hipStream_t st,
             int *herr, bool rcp_guard)
{
    if (m < 1 || m > MPM || n < 2) return SIGNTRI_ENOTSUP;
    const int G = (m + GC - 1) / GC;
    int nown = 0;
    const ProjLayout PL = proj_layout(n, m);
    const int64_t nb = PL.nb;
    if (!proj_grid(nb, device_cus(), G, &nown)) return SIGNTRI_ENOTSUP;
    // the minority rows of both bases, ascending (basis 1: rows of J T^T J), and
    // each group's first block (that of its lowest minority row)
    int bsh[2 * MAXG];
    {
        std::vector<int64_t> rows0, rows1((size_t)m);
        rows0.reserve((size_t)m);
        for (int64_t i = 0; i < n; ++i)
            if (hsgn[i] == minority) {
                if ((int)rows0.size() >= m) return SIGNTRI_ENOTSUP;
                rows0.push_back(i);
            }
        if ((int)rows0.size() != m) return SIGNTRI_ENOTSUP;
        for (int l = 0; l < m; ++l) rows1[l] = n - 1 - rows0[m - 1 - l];
        for (int g = 0; g < G; ++g) {
            const int last = std::min(m, (g + 1) * GC) - 1;
            bsh[g] = (int)((n - 1 - rows0[last]) / PB);
            bsh[G + g] = (int)((n - 1 - rows1[last]) / PB);
        }
    }
    const size_t nn = (size_t)n, mp = (size_t)PL.mp;
    char *p = (char *)ws;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += al(bytes);
        return (void *)q;
    };
    double *Z0 = (double *)take(nn * mp * 8), *Z1 = (double *)take(nn * mp * 8);
    double *C0 = (double *)take(nn * mp * 8), *C1 = (double *)take(nn * mp * 8);
    int *rt0 = (int *)take(nn * 4), *rt1 = (int *)take(nn * 4);
    int *ps0 = (int *)take(mp * 4), *ps1 = (int *)take(mp * 4);
    int *kx = (int *)take((size_t)2 * (nb + 2) * 4);
    double *part = (double *)take((size_t)PL.nparts * PL.ntiles * 4096 * 8);
    double *Mg = (double *)take(mp * mp * 8);
    double *minv = (double *)take(mp * mp * 8);
    double *A = (double *)take(nn * mp * 8);
    int *sync = (int *)take(proj_sync_bytes(n, m));

    // Z of both bases (contiguous) cleared: a group writes only the blocks it
    // reaches; flags and error word cleared.  Fill kernels, no memset node
    // (should the call be captured).
    prof_begin(st);
    hipLaunchKernelGGL(k_proj_prep, dim3(1), dim3(1024), 0, st, sgn, n, minority, m, (int)mp,
                       (int)nb, rt0, ps0, rt1, ps1, kx);
    if (launch_fill_int((int *)Z0, (int64_t)(((char *)C0 - (char *)Z0) / 4), 0, st) != hipSuccess ||
        launch_fill_int(sync, (int64_t)(4 * G * nb + 1), 0, st) != hipSuccess)
        return SIGNTRI_EHIP;
    prof_end(st, PK_AUX, 0.0, 3);

    ProjArgs a;
    a.n = n;
    a.m = m;
    a.b[0] = ProjBasis{T, ldt, 0, Z0, C0, rt0, ps0};
    a.b[1] = ProjBasis{T, ldt, 1, Z1, C1, rt1, ps1};
    ProjSync S;
    S.zdone = sync;
    S.accready = sync + 2 * G * nb;
    S.err = sync + 4 * G * nb;
    S.kx = kx;
    for (int x = 0; x < 2 * G; ++x) S.bstart[x] = bsh[x];
    S.spin_limit = flow_spin_limit();
    S.nb = (int)nb;
    S.G = G;
    S.nown = nown;
    S.rcp_guard = rcp_guard ? 1 : 0;
    const double nd = (double)n, md = (double)m;
    prof_begin(st);
    hipLaunchKernelGGL(k_proj_run, dim3(2 * G + 2 * nown), dim3(NT), 0, st, a, S);
    prof_end(st, PK_PROJ, flops, 1);
    prof_begin(st);
    // W^T Z (partials, their sum), its inverse, A; then the product
    hipLaunchKernelGGL(k_proj_gram, dim3(PL.nparts, PL.ntiles), dim3(256), 0, st, Z0, Z1, n, m,
                       PL.nc, PL.rpp, part);
    hipLaunchKernelGGL(k_proj_gsum, dim3((unsigned)(mp * mp / 64)), dim3(64), 0, st, part,
                       PL.nparts, m, (int)mp, Mg);
    if (mp == 64)
        hipLaunchKernelGGL(k_proj_minv, dim3(1), dim3(256), 0, st, Mg, minv);
    else
        hipLaunchKernelGGL(k_proj_minv_col, dim3((unsigned)(mp / 4)), dim3(256), 0, st, Mg, (int)mp,
                           minv);
    hipLaunchKernelGGL(k_proj_a, dim3((unsigned)((n + 63) / 64), PL.nc), dim3(256), 0, st, Z0, minv,
                       n, (int)mp, A);
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

size_t proj_workspace_bytes(int64_t n, int m, bool cplx)
{
    return cplx ? projc_workspace_bytes(n) : proj_layout(n, m).bytes;
}

}  // namespace sgt
