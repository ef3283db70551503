// Persistent dataflow sweep over the off-diagonal blocks of real triangular
// systems (FP64 or FP32), one workgroup per block at a time.
//
// Three kinds of sweep share the kernel; every one solves, block by block,
// equations whose left-hand side couples a 32 x 32 block only with diagonal
// blocks and whose right-hand side is a sum of products of finished blocks:
//
//   MAIN  the block equations of the substitution (Section 5; Eq. (1) and
//         Eq. (2) in block form, accumulators X and Y of Algorithms 4-6):
//           equal signs:     (u_ii + u_jj) u_ij + sum_{k in I,k>i} u_ik u_kj
//                            + sum_{k in J,k<j} u_ik u_kj = -Y_ij
//           opposite signs:  (t_ii - t_jj) u_ij + sum_{k in I,k>i} t_ik u_kj
//                            - sum_{k in J,k<j} u_ik t_kj
//                            = X_ij + (U_II T_IJ - T_IJ U_JJ)_ij
//         with Y_IJ = sum_{I<K<J} U_IK U_KJ, X_IJ = sum_{I<K<J} (U_IK T_KJ - T_IK U_KJ).
//   CORR  the same equations linearised about a computed U0 (refinement of a
//         reduced-precision U0): the unknown is the correction E, U0 supplies
//         the coefficients, and the right-hand side starts from the residual
//         R_ij = (U0^2 - I)_ij (equal signs) or (U0 T - T U0)_ij (opposite):
//           Y_IJ = R_IJ + sum_{I<K<J} (U0_IK E_KJ + E_IK U0_KJ),
//           X_IJ = R_IJ + sum_{I<K<J} (E_IK T_KJ - T_IK E_KJ).
//         The residual is read from the output array and overwritten by E.
//   SYL   the Sylvester equation T11 X - X T22 = 2 s T12 of the Parlett-
//         Sylvester form (Algorithm 2 with F11 = s I, F22 = -s I) for a diagonal
//         grouped by sign, T11 = T(0:p, 0:p), T22 = T(p:n, p:n):
//           (a_ii - b_jj) x_ij + sum_{k in I,k>i} a_ik x_kj - sum_{k in J,k<j} x_ik b_kj
//             = 2 s t_ij - sum_{K>I} A_IK X_KJ + sum_{K<J} X_IK B_KJ,
//         the opposite-sign equation of MAIN with the products by the identity
//         blocks of U dropped.
//
// Scheduling.  A task is one block (I, J).  Tasks are handed out in a
// dependency-respecting order by an atomic ticket; a block's completion is
// published through a per-block flag (release), and a task waits (acquire)
// for the flags of the blocks its products read, in three groups by how
// recently those blocks can have finished (lag >= 3, lag 2, lag 1, where the
// lag of a product is how many block diagonals -- MAIN/CORR -- or
// anti-diagonals -- SYL -- earlier its later operand lies).  The lag-1 group is
// the critical path; everything else overlaps the solves of other blocks.  The
// lag >= 3 steps are ordered by readiness and multiplied prefix by prefix as
// their flags appear, so that a long block does most of its products while the
// few blocks it still waits for are being solved.
// Every task only waits for tasks with smaller tickets, which are held by
// running workgroups, so the schedule cannot deadlock; every wait is also
// bounded and, when the bound is hit, sets an error word and gives up, so the
// grid always drains.
//
// Products.  Four waves each own a 16 x 16 piece of the block and run FP64 or
// FP32 16x16x4 MFMAs over K steps of 32, only for the products their piece
// needs (the X entries and Y entries of a piece are known from the signs: the
// saving of the single-accumulator variant of Section 5.3 at MFMA
// granularity).  Operands are staged through LDS: the next K step is loaded
// into registers while the current one is multiplied.
//
// Solve.  The right-hand side is assembled in LDS and the block's entries are
// solved along anti-diagonals from the bottom-left corner, each entry's two
// inner products (column part with row i of the left diagonal block, row part
// with column j of the right one) shared by 8 lanes and reduced with DPP; the
// divisions use reciprocals 1/(t_ii - t_jj) tabulated in FP64 before the sweep.
#include <algorithm>

#include "common.h"

namespace sgt {

namespace {

constexpr int TB = kFlowTile;    // block edge
constexpr int NT = 256;          // threads per workgroup (4 waves)
constexpr int LPR = NT / TB;     // lanes per block row in the solve
constexpr int CPL = TB / LPR;    // row entries per lane
constexpr int LDX = TB + 4;      // LDS pitch of the block being solved
constexpr int APITCH = TB + 16;  // LDS: A operand as [k][m], padded row
constexpr int BSLAB = 4 * TB + 4;  // LDS: B operand as [k/4][n][k%4] slabs

template <typename F> struct mm;
template <> struct mm<double> {
    typedef dx4 acc;
    __device__ static acc mma(double a, double b, acc c) { return mfma_f64(a, b, c); }
    __device__ static int row(int lane, int r) { return mfma64_row(lane, r); }
};
template <> struct mm<float> {
    typedef fx4 acc;
    __device__ static acc mma(float a, float b, acc c) { return mfma_f32(a, b, c); }
    __device__ static int row(int lane, int r) { return mfma32_row(lane, r); }
};

// Kinds of K step.
enum { ST_MID = 0, ST_SYLA = 1, ST_SYLB = 2, ST_SPI = 3, ST_SPJ = 4 };

// One operand tile: rows r0 .. r0+31 and columns c0 .. c0+31 of a column-major
// array, valid below row rend and left of column cend; `diag` keeps only the
// upper triangle.
struct TileRef {
    int64_t r0, c0;
    int64_t rend, cend;
    bool diag;
};

// Blocks written by the running sweep are read and written with device-coherent
// accesses (the flag and the data both go through the point of coherence of the
// eight L2 caches), so a consumer never needs to invalidate its L2 and a
// producer never needs to write its L2 back: the producer's stores complete
// (s_waitcnt) before its flag store is issued, and the consumer issues its loads
// only after it has read the flag.  Inputs and blocks written before the launch
// use ordinary cached loads.
__device__ inline int flag_load(const int *p) { return gload_coherent(p); }
template <typename F> __device__ inline F coherent_load(const F *p) { return gload_coherent(p); }
template <typename F> __device__ inline void coherent_store(F *p, F v) { gstore_coherent(p, v); }

// Global-to-LDS staging of one K step: each thread carries 4 consecutive rows
// of one column of every operand tile the step needs (A side: unknown, -T, U0;
// B side: unknown, T, U0), one plane per component (P = 2 for complex
// entries: real and imaginary parts), and a mask of the slots it loaded.
template <typename F, int NS, int P> struct Stage {
    F ga[NS][P][4], gb[NS][P][4];
    unsigned live;
};

// Complex multiply-accumulate of 16 x 16 MFMA pieces kept as real and
// imaginary planes: (ar + i ai)(br + i bi) = (ar br - ai bi) + i (ar bi + ai br).
template <typename F, typename A>
__device__ inline void cmma(F ar, F ai, F br, F bi, A &cr, A &ci)
{
    cr = mm<F>::mma(ar, br, cr);
    cr = mm<F>::mma(-ai, bi, cr);
    ci = mm<F>::mma(ar, bi, ci);
    ci = mm<F>::mma(ai, br, ci);
}

// C selects complex entries: every array then holds interleaved (re, im)
// pairs and every leading dimension counts complex elements.
// Two builds of the real kernels: as the compiler allocates registers (two
// workgroups per compute unit for FP64, three for FP32), and within the
// registers of one more workgroup (WPE waves per SIMD; the LDS allows it, the
// few values spilled for it are read once per block, outside the K and solve
// loops).  The launch takes the second when the grid asks for that many.
template <typename F, bool C> struct FlowWaves { static constexpr int value = 0; };
template <> struct FlowWaves<double, false> { static constexpr int value = 3; };
template <> struct FlowWaves<float, false> { static constexpr int value = 4; };

template <typename F, int KIND, bool C, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void k_flow(FlowArgs<F> a)
{
    typedef typename mm<F>::acc acc_t;
    constexpr bool CORR = KIND == FLOW_CORR;
    constexpr bool syl = KIND == FLOW_SYL;
    constexpr int NS = CORR ? 3 : 2;  // operand slots per side
    constexpr int P = C ? 2 : 1;      // planes per entry
    constexpr int SV = 0, ST = 1, SC = 2;  // slot roles: unknown, T, U0
    // Operand staging of the products; during the solve the same memory holds
    // the block (column-major X and a row-major copy XT, pitch LDX) and the
    // column coefficients of block J (RU, RT: column-major, zero for k >= j),
    // each as P planes.
    __shared__ __align__(16) F sA[NS][P][TB * APITCH];
    __shared__ __align__(16) F sB[NS][P][(TB / 4) * BSLAB];
    __shared__ double rcp[P][TB * TB];  // 1/(d_i - d_j) for opposite-sign entries, row-major
    static_assert(2 * P * TB * LDX <= NS * P * TB * APITCH, "X and XT fit in the A staging");
    static_assert(2 * P * TB * TB <= NS * P * (TB / 4) * BSLAB, "RU and RT fit in the B staging");
    F *const X = &sA[0][0][0];     // plane q at X + q * TB * LDX
    F *const XT = X + P * TB * LDX;
    F *const RU = &sB[0][0][0];    // plane q at RU + q * TB * TB
    F *const RT = RU + P * TB * TB;
    __shared__ int8_t rs[TB], cs[TB];
    __shared__ int s_task, s_first;
    typedef F f4 __attribute__((ext_vector_type(4)));

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pr = wave >> 1, pc = wave & 1;   // MFMA piece of this wave
    const int mg = lane >> 4, mt = lane & 15;  // MFMA lane group and index
    const int lc = tid >> 3, lr = (tid & 7) * 4;  // operand loads: column, first row
    const int li = tid / LPR, lq = tid % LPR;  // solve: row, lane within the row
    const int kq = CPL * lq;                     // solve: this lane's k = kq .. kq + 3

    // Every value that decides whether a barrier is reached is provably uniform
    // (an SGPR), and the single-lane work (publishing a flag, taking a ticket)
    // sits in one branch between two barriers inside the loop body: with a loop
    // condition the compiler sees as divergent, or single-lane branches on both
    // sides of the back edge, the loop gets restructured so that lane 0 and the
    // other lanes pass the barriers in different iterations.
    // a sweep of a refinement step the device decided against: nothing to do
    if (a.live && uniform(*a.live) == 0) return;
    const int ntasks = a.ntasks_dev ? uniform(min(*a.ntasks_dev, a.ntasks)) : a.ntasks;
    if (tid == 0) s_task = atomicAdd(&a.ctrl[0], 1);
    __syncthreads();
    int t = uniform(s_task);
    while (t < ntasks) {
        const int2 tk = gload(a.tasks + t);
        const int mat = uniform(tk.x), ij = uniform(tk.y);
        const FlowMat<F> M = a.mats ? gload(a.mats + mat) : a.m0;
        const int I = ij >> 16, J = ij & 0xffff;
        // row and column spaces of the unknown
        const int64_t ro = 0, co = syl ? M.split : 0;
        const int64_t rend = syl ? M.split : M.n, cend = M.n;
        const int64_t gr0 = ro + (int64_t)I * TB, gc0 = co + (int64_t)J * TB;
        const int bi = uniform((int)min((int64_t)TB, rend - gr0));
        const int bj = uniform((int)min((int64_t)TB, cend - gc0));
        // entry (r, c), plane q of a column-major array with leading dimension ld
        auto at = [&](int64_t r, int64_t c, int64_t ld, int q) -> int64_t {
            return P * (r + c * ld) + q;
        };

        if (tid < TB) {
            // (the Sylvester form and a general function: every entry by the
            // opposite-class equations)
            if (syl || M.general) {
                rs[tid] = tid < bi ? 1 : 0;
                cs[tid] = tid < bj ? -1 : 0;
            } else {
                rs[tid] = tid < bi ? gload(M.sgn + gr0 + tid) : 0;
                cs[tid] = tid < bj ? gload(M.sgn + gc0 + tid) : 0;
            }
        }
        __syncthreads();

        // which products this wave's piece needs, and the whole block
        bool pneedY = false, pneedX = false;
        {
            bool rp = false, rn = false, cp = false, cn = false;
            for (int u = 0; u < 16; ++u) {
                const int vr = rs[16 * pr + u], vc = cs[16 * pc + u];
                rp |= vr > 0;
                rn |= vr < 0;
                cp |= vc > 0;
                cn |= vc < 0;
            }
            pneedY = uniform((rp && cp) || (rn && cn));  // the same in every lane of a wave
            pneedX = uniform((rp && cn) || (rn && cp));
            if (M.dense && !syl && !M.general) pneedY = pneedX = true;
        }
        const bool any_x = uniform(__syncthreads_or(pneedX));

        acc_t accY[P], accX[P];
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                accY[q][r] = 0;
                accX[q][r] = 0;
            }
        const int D = J - I;
        const int na = syl ? uniform(M.nbr) - 1 - I : 0;  // SYL: K blocks of T11 below I
        const int nb_ = syl ? J : 0;             // SYL: K blocks of T22 left of J

        // K step s of group g (0: diagonal-block terms, 1: lag >= 3, 2: lag 2, 3: lag 1)
        auto group_count_raw = [&](int g) -> int {
            if (KIND == FLOW_MAIN && g == 0) return any_x ? 2 : 0;
            if (g == 0) return 0;
            if (!syl) {
                if (g == 1) return max(0, D - 5);
                if (g == 2) return D >= 5 ? 2 : (D == 4 ? 1 : 0);
                return D >= 3 ? 2 : (D == 2 ? 1 : 0);
            }
            if (g == 1) return max(0, na - 2) + max(0, nb_ - 2);
            if (g == 2) return (na >= 2) + (nb_ >= 2);
            return (na >= 1) + (nb_ >= 1);
        };
        auto group_count = [&](int g) -> int { return uniform(group_count_raw(g)); };
        auto step_of = [&](int g, int s, int &kind, int &K) {
            if (g == 0) {
                kind = s == 0 ? ST_SPI : ST_SPJ;
                K = 0;
                return;
            }
            if (!syl) {
                kind = ST_MID;
                if (g == 1) {
                    // middle out: K's operands (I, K) and (K, J) are both finished once
                    // superdiagonal max(K - I, J - K) is, so the steps come in order of
                    // readiness
                    const int off = (s & 1) ? ((s + 1) >> 1) : -(s >> 1);
                    K = I + (D >> 1) + off;
                } else if (g == 2) {
                    K = s == 0 ? I + 2 : J - 2;
                } else {
                    K = s == 0 ? I + 1 : J - 1;
                }
                return;
            }
            if (g == 1) {
                // A steps (K, J) with lag K - I and B steps (I, K) with lag J - K,
                // merged by decreasing lag (in order of readiness)
                const int L1 = max(na, nb_), L2 = min(na, nb_);
                const int f = max(0, L1 - max(L2, 2));
                bool isA;
                int lag;
                if (s < f) {
                    lag = L1 - s;
                    isA = na >= nb_;
                } else {
                    const int q = s - f;
                    lag = L2 - (q >> 1);
                    isA = (q & 1) == 0;
                }
                kind = isA ? ST_SYLA : ST_SYLB;
                K = isA ? I + lag : J - lag;
                return;
            }
            const int lagA = g == 2 ? (na >= 2) : (na >= 1);
            if (s < lagA) {
                kind = ST_SYLA;
                K = g == 2 ? I + 2 : I + 1;
            } else {
                kind = ST_SYLB;
                K = g == 2 ? J - 2 : J - 1;
            }
        };
        auto dep_flag = [&](int kind, int K, int d) -> const int * {
            int64_t idx;
            if (kind == ST_MID) idx = d == 0 ? (int64_t)I * M.nbc + K : (int64_t)K * M.nbc + J;
            else if (kind == ST_SYLA) idx = (int64_t)K * M.nbc + J;
            else idx = (int64_t)I * M.nbc + K;
            return a.flags + M.flag0 + idx;
        };
        // wait until the flags of every K step of group g are set
        auto wait_group = [&](int g, int cnt) {
            if (g == 0 || cnt == 0) return;
            const int per = syl ? 1 : 2;  // flags per K step
            const int total = per * cnt;
            // (a negative limit, a testing hook, gives up at once)
            bool timed_out = a.spin_limit < 0;
            for (int it = 0; !timed_out; ++it) {
                bool ok = true;
                for (int e = tid; e < total; e += NT) {
                    int kind, K;
                    step_of(g, e / per, kind, K);
                    ok &= flag_load(dep_flag(kind, K, e % per)) != 0;
                }
                if (uniform(__syncthreads_and(ok))) break;
                const bool err = uniform(__syncthreads_or(tid == 0 && flag_load(a.ctrl + 1) != 0));
                if (err || it >= a.spin_limit) {
                    timed_out = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (timed_out && tid == 0) atomicOr(a.ctrl + 1, 1);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no load moves above the poll
        };

        // First step in [from, cnt) of group g whose operand flags are not all set
        // (cnt when every one is).
        auto ready_prefix = [&](int g, int from, int cnt) -> int {
            const int per = syl ? 1 : 2;
            if (tid == 0) s_first = cnt;
            __syncthreads();
            const int total = per * (cnt - from);
            for (int e = tid; e < total; e += NT) {
                int kind, K;
                const int st = from + e / per;
                step_of(g, st, kind, K);
                if (flag_load(dep_flag(kind, K, e % per)) == 0) atomicMin(&s_first, st);
            }
            __syncthreads();
            const int pfx = uniform(s_first);
            __syncthreads();  // s_first is reused
            __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no operand load moves above the poll
            return pfx;
        };

        // operand tiles of a K step for a slot (false: the step does not use it)
        const bool any_y = uniform(__syncthreads_or(pneedY));
        auto slotA = [&](int kind, int K, int role, const F *&p, int64_t &ld, TileRef &tr,
                         bool &coh) -> bool {
            const int64_t kc = (int64_t)K * TB;
            coh = false;
            switch (kind) {
            case ST_MID:
                tr = {gr0, kc, M.n, M.n, false};
                if (role == SV) { p = M.V; ld = M.ldv; coh = true; return true; }
                if (role == ST) { p = M.T; ld = M.ldt; return any_x; }
                p = M.C; ld = M.ldc; return any_y;
            case ST_SYLA:
                tr = {gr0, ro + kc, rend, rend, false};
                if (role == ST) { p = M.T; ld = M.ldt; return true; }
                return false;
            case ST_SYLB:
                tr = {gr0, co + kc, rend, cend, false};
                if (role == SV) { p = M.V; ld = M.ldv; coh = true; return true; }
                return false;
            case ST_SPI:
                tr = {gr0, gr0, M.n, M.n, true};
                if (role == SV) { p = M.V; ld = M.ldv; return true; }
                return false;
            default:  // ST_SPJ
                tr = {gr0, gc0, M.n, M.n, false};
                if (role == ST) { p = M.T; ld = M.ldt; return true; }
                return false;
            }
        };
        auto slotB = [&](int kind, int K, int role, const F *&p, int64_t &ld, TileRef &tr,
                         bool &coh) -> bool {
            const int64_t kr = (int64_t)K * TB;
            coh = false;
            switch (kind) {
            case ST_MID:
                tr = {kr, gc0, M.n, M.n, false};
                if (role == SV) { p = M.V; ld = M.ldv; coh = true; return true; }
                if (role == ST) { p = M.T; ld = M.ldt; return any_x; }
                p = M.C; ld = M.ldc; return any_y;
            case ST_SYLA:
                tr = {ro + kr, gc0, rend, cend, false};
                if (role == SV) { p = M.V; ld = M.ldv; coh = true; return true; }
                return false;
            case ST_SYLB:
                tr = {co + kr, gc0, cend, cend, false};
                if (role == ST) { p = M.T; ld = M.ldt; return true; }
                return false;
            case ST_SPI:
                tr = {gr0, gc0, M.n, M.n, false};
                if (role == ST) { p = M.T; ld = M.ldt; return true; }
                return false;
            default:  // ST_SPJ
                tr = {gc0, gc0, M.n, M.n, true};
                if (role == SV) { p = M.V; ld = M.ldv; return true; }
                return false;
            }
        };
        typedef Stage<F, NS, P> stage_t;
        auto load_tile = [&](const F *p, int64_t ld, const TileRef &tr, bool coh, F (&dst)[P][4]) {
            const int64_t c = tr.c0 + lc;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t r = tr.r0 + lr + e;
                const bool ok = r < tr.rend && c < tr.cend && !(tr.diag && r > c);
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    F v = 0;
                    if (ok) v = coh ? coherent_load(p + at(r, c, ld, q)) : gload(p + at(r, c, ld, q));
                    dst[q][e] = v;
                }
            }
        };
        auto load_step = [&](int kind, int K, stage_t &g) {
            g.live = 0;
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const F *p = nullptr;
                int64_t ld = 0;
                TileRef tr;
                bool coh;
                if (slotA(kind, K, q, p, ld, tr, coh)) {
                    load_tile(p, ld, tr, coh, g.ga[q]);
                    g.live |= 1u << q;
                }
                if (slotB(kind, K, q, p, ld, tr, coh)) {
                    load_tile(p, ld, tr, coh, g.gb[q]);
                    g.live |= 1u << (8 + q);
                }
            }
        };
        // Slots not loaded for a step are not read by its products either.
        auto store_step = [&](const stage_t &g) {
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const F sg = q == ST ? (F)-1 : (F)1;  // T is stored negated on the A side
#pragma unroll
                for (int pl = 0; pl < P; ++pl) {
                    if (g.live & (1u << q))
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            sA[q][pl][lc * APITCH + lr + e] = sg * g.ga[q][pl][e];
                    if (g.live & (1u << (8 + q)))
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            sB[q][pl][(lr >> 2) * BSLAB + lc * 4 + e] = g.gb[q][pl][e];
                }
            }
        };
        // acc += a * b for one slot pair at LDS offsets ao, bo
        auto mac = [&](int qa, int qb, int ao, int bo, acc_t (&acc)[P]) {
            if constexpr (C) {
                cmma<F>(sA[qa][0][ao], sA[qa][1][ao], sB[qb][0][bo], sB[qb][1][bo], acc[0], acc[1]);
            } else {
                acc[0] = mm<F>::mma(sA[qa][0][ao], sB[qb][0][bo], acc[0]);
            }
        };
        auto compute_step = [&](int kind) {
            const bool mid = kind == ST_MID;
            const bool xv_t = pneedX && (mid || kind == ST_SYLB || kind == ST_SPI);  // V * T
            const bool xt_v = pneedX && (mid || kind == ST_SYLA || kind == ST_SPJ);  // -T * V
            const bool yy = pneedY && mid;
#pragma unroll
            for (int k4 = 0; k4 < TB / 4; ++k4) {
                const int ao = (k4 * 4 + mg) * APITCH + 16 * pr + mt;
                const int bo = k4 * BSLAB + (16 * pc + mt) * 4 + mg;
                if (yy) {
                    if constexpr (CORR) {
                        mac(SC, SV, ao, bo, accY);
                        mac(SV, SC, ao, bo, accY);
                    } else {
                        mac(SV, SV, ao, bo, accY);
                    }
                }
                if (xv_t) mac(SV, ST, ao, bo, accX);
                if (xt_v) mac(ST, SV, ao, bo, accX);
            }
        };
        // Steps s0 .. s1-1 of a group: step s is multiplied from LDS while steps
        // s+1 and s+2 are in flight from global memory into two register stages.
        auto run_group = [&](int g, int s0, int s1) {
            const int cnt = s1 - s0;
            if (cnt <= 0) return;
            auto step_at = [&](int s, int &kind, int &K) { step_of(g, s0 + s, kind, K); };
            stage_t r0, r1;
            int kd[3], kk[3];
            step_at(0, kd[0], kk[0]);
            load_step(kd[0], kk[0], r0);
            if (cnt > 1) {
                step_at(1, kd[1], kk[1]);
                load_step(kd[1], kk[1], r1);
            }
            __syncthreads();  // earlier users of the staging memory are done
            store_step(r0);
            __syncthreads();
            for (int s = 0; s < cnt; s += 2) {
                // step s in LDS, s + 1 in r1
                if (s + 2 < cnt) {
                    step_at(s + 2, kd[2], kk[2]);
                    load_step(kd[2], kk[2], r0);
                }
                compute_step(kd[0]);
                __syncthreads();
                if (s + 1 >= cnt) break;
                store_step(r1);
                __syncthreads();
                // step s + 1 in LDS, s + 2 in r0
                if (s + 3 < cnt) {
                    step_at(s + 3, kd[0], kk[0]);
                    load_step(kd[0], kk[0], r1);
                }
                compute_step(kd[1]);
                __syncthreads();
                if (s + 2 >= cnt) break;
                store_step(r0);
                __syncthreads();
                // rotate the step descriptors: s + 2 -> slot 0, s + 3 -> slot 1
                const int nk0 = kd[2], nK0 = kk[2];
                kd[1] = kd[0];
                kk[1] = kk[0];
                kd[0] = nk0;
                kk[0] = nK0;
            }
        };

        run_group(0, 0, group_count(0));
        // lag >= 3: multiply each ready prefix of the steps as soon as it is
        // ready, so a long block's products proceed while the blocks it still
        // needs are being solved
        {
            const int cnt = group_count(1);
            int s = 0, idle = 0;
            while (s < cnt) {
                const int pfx = ready_prefix(1, s, cnt);
                if (pfx > s) {
                    run_group(1, s, pfx);
                    s = pfx;
                    idle = 0;
                    continue;
                }
                const bool err = uniform(__syncthreads_or(tid == 0 && flag_load(a.ctrl + 1) != 0));
                if (err || ++idle >= a.spin_limit) {
                    if (tid == 0) atomicOr(a.ctrl + 1, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        {
            const int cnt = group_count(2);
            wait_group(2, cnt);
            run_group(2, 0, cnt);
        }

        // ---- solve prologue, loaded before the lag-1 wait: row li of the left
        // diagonal block (k = kq .. kq+3 > li), this thread's share of the right
        // diagonal block's columns and the initial right-hand side in registers
        // (the staging memory they go to is busy until the last product), the
        // reciprocals 1/(d_i - d_j) in their own LDS table.
        F cu[P][CPL], ct[P][CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            const int k = kq + u;
            const bool up = k > li && k < bi;
            const int64_t gi = gr0 + li, gk = gr0 + k;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                cu[q][u] = (up && !syl) ? (CORR ? gload(M.C + at(gi, gk, M.ldc, q)) : gload(M.V + at(gi, gk, M.ldv, q)))
                                        : (F)0;
                ct[q][u] = up ? gload(M.T + at(gi, gk, M.ldt, q)) : (F)0;
            }
        }
        constexpr int RPT = TB * TB / NT;  // entries per thread of a 32 x 32 table
        F ru[P][RPT], rt[P][RPT], r0v[P][RPT];
#pragma unroll
        for (int w = 0; w < RPT; ++w) {
            const int e = tid + NT * w, k = e % TB, c = e / TB;
            const bool in = k < c && c < bj;
            const int64_t gi = gc0 + k, gk = gc0 + c;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                rt[q][w] = in ? gload(M.T + at(gi, gk, M.ldt, q)) : (F)0;
                ru[q][w] = (in && !syl) ? (CORR ? gload(M.C + at(gi, gk, M.ldc, q)) : gload(M.V + at(gi, gk, M.ldv, q)))
                                        : (F)0;
                F v = 0;
                if (k < bi && c < bj) {
                    if (CORR) v = gload(M.V + at(gr0 + k, gc0 + c, M.ldv, q));
                    if (syl) v = (F)M.rhs_scale * gload(M.Rh + at(gr0 + k, gc0 + c, M.ldrh, q));
                }
                r0v[q][w] = v;
            }
        }
        for (int e = tid; e < TB * TB; e += NT) {
            const int r = e / TB, c = e % TB;
            const bool opp = r < bi && c < bj && rs[r] != cs[c];
            if constexpr (C) {
                double zr = 0.0, zi = 0.0;
                if (opp) {
                    // 1 / (d_i - d_j) for a complex difference z: conj(z) / |z|^2
                    const double dr = gload(M.dg + 2 * (gr0 + r)) - gload(M.dg + 2 * (gc0 + c));
                    const double di = gload(M.dg + 2 * (gr0 + r) + 1) - gload(M.dg + 2 * (gc0 + c) + 1);
                    const double s = fmax(fabs(dr), fabs(di));
                    const double xr = dr / s, xi = di / s;
                    const double den = s * (xr * xr + xi * xi);
                    zr = xr / den;
                    zi = -xi / den;
                }
                rcp[0][e] = zr;
                rcp[1][e] = zi;
            } else {
                rcp[0][e] = opp ? 1.0 / (gload(M.dg + gr0 + r) - gload(M.dg + gc0 + c)) : 0.0;
            }
        }

        // ---- lag-1 products: the critical path
        {
            const int cnt = group_count(3);
            wait_group(3, cnt);
            run_group(3, 0, cnt);
        }
        __syncthreads();  // the staging memory becomes the solve's

        // ---- right-hand side: initial part + products (X or Y by the entry's signs)
#pragma unroll
        for (int w = 0; w < RPT; ++w) {
            const int e = tid + NT * w;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                X[q * TB * LDX + (e % TB) + (e / TB) * LDX] = r0v[q][w];
                RU[q * TB * TB + e] = ru[q][w];
                RT[q * TB * TB + e] = rt[q][w];
            }
        }
        for (int e = tid; e < P * TB * LDX; e += NT) XT[e] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * pr + mm<F>::row(lane, r);
            const int j = 16 * pc + mt;
            const bool same = rs[i] == cs[j];
#pragma unroll
            for (int q = 0; q < P; ++q) X[q * TB * LDX + i + j * LDX] += same ? accY[q][r] : accX[q][r];
        }
        const int si = rs[li];
        unsigned long long cpos = 0;
        for (int c = 0; c < bj; ++c) cpos |= (unsigned long long)(cs[c] > 0) << c;
        __syncthreads();

        // ---- block solve along anti-diagonals from the bottom-left corner.  Every
        // lane of row li reads and multiplies unconditionally (the coefficients
        // are zero where a term must not contribute); lane 0 of the row writes.
        const int steps = uniform((bi - 1) + bj);
        for (int st = 0; st < steps; ++st) {
            const int j = st - (bi - 1 - li);
            const int jj = min(max(j, 0), TB - 1);
            const bool same = !syl && ((((cpos >> jj) & 1ull) != 0) == (si > 0));
            const F *rsrc = same ? RU : RT;
            F tot[P], rhs[P];
            double rsc = 0.0;  // real entries: the entry's scale, read before the reduction
            if constexpr (C) {
                const f4 xcr = *(const f4 *)&X[kq + jj * LDX];
                const f4 xci = *(const f4 *)&X[TB * LDX + kq + jj * LDX];
                const f4 xrr = *(const f4 *)&XT[kq + li * LDX];
                const f4 xri = *(const f4 *)&XT[TB * LDX + kq + li * LDX];
                const f4 rrr = *(const f4 *)&rsrc[kq + jj * TB];
                const f4 rri = *(const f4 *)&rsrc[TB * TB + kq + jj * TB];
                rhs[0] = X[li + jj * LDX];
                rhs[1] = X[TB * LDX + li + jj * LDX];
                F cur = 0, cui = 0, ctr = 0, cti = 0, rwr = 0, rwi = 0;
#pragma unroll
                for (int u = 0; u < CPL; ++u) {
                    cur += cu[0][u] * xcr[u] - cu[1][u] * xci[u];
                    cui += cu[0][u] * xci[u] + cu[1][u] * xcr[u];
                    ctr += ct[0][u] * xcr[u] - ct[1][u] * xci[u];
                    cti += ct[0][u] * xci[u] + ct[1][u] * xcr[u];
                    rwr += xrr[u] * rrr[u] - xri[u] * rri[u];
                    rwi += xrr[u] * rri[u] + xri[u] * rrr[u];
                }
                tot[0] = same ? cur + rwr : rwr - ctr;
                tot[1] = same ? cui + rwi : rwi - cti;
            } else {
                // one column coefficient set per entry, selected without a branch:
                // U's row where the signs agree, -T's row where they differ
                const f4 xc = *(const f4 *)&X[kq + jj * LDX];
                const f4 xr = *(const f4 *)&XT[kq + li * LDX];
                const f4 rr = *(const f4 *)&rsrc[kq + jj * TB];
                rhs[0] = X[li + jj * LDX];
                F cc[CPL];
#pragma unroll
                for (int u = 0; u < CPL; ++u) cc[u] = same ? cu[0][u] : -ct[0][u];
                const F col = (cc[0] * xc[0] + cc[1] * xc[1]) + (cc[2] * xc[2] + cc[3] * xc[3]);
                const F row = (xr[0] * rr[0] + xr[1] * rr[1]) + (xr[2] * rr[2] + xr[3] * rr[3]);
                tot[0] = col + row;
                rsc = same ? -0.5 * (double)si : rcp[0][li * TB + jj];
            }
#pragma unroll
            for (int q = 0; q < P; ++q) tot[q] = group_sum<LPR>(tot[q]);
            if (li < bi && j >= 0 && j < bj && lq == 0) {
                if constexpr (C) {
                    const double vr = (double)rhs[0] + (double)tot[0];
                    const double vi = (double)rhs[1] + (double)tot[1];
                    double xr, xi;
                    if (same) {
                        const double h = -0.5 * (double)si;
                        xr = vr * h;
                        xi = vi * h;
                    } else {
                        const double zr = rcp[0][li * TB + jj], zi = rcp[1][li * TB + jj];
                        xr = vr * zr - vi * zi;
                        xi = vr * zi + vi * zr;
                    }
                    X[li + jj * LDX] = (F)xr;
                    X[TB * LDX + li + jj * LDX] = (F)xi;
                    XT[jj + li * LDX] = (F)xr;
                    XT[TB * LDX + jj + li * LDX] = (F)xi;
                } else {
                    const F x = (F)(((double)rhs[0] + (double)tot[0]) * rsc);
                    X[li + jj * LDX] = x;
                    XT[jj + li * LDX] = x;
                }
            }
            __syncthreads();
        }

        // ---- publish the block: coherent stores, all complete before the flag
        for (int e = tid; e < TB * TB; e += NT) {
            const int r = e % TB, c = e / TB;
            if (r < bi && c < bj)
#pragma unroll
                for (int q = 0; q < P; ++q)
                    coherent_store(M.V + at(gr0 + r, gc0 + c, M.ldv, q), X[q * TB * LDX + r + c * LDX]);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_store(a.flags + M.flag0 + (int64_t)I * M.nbc + J, 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            s_task = atomicAdd(&a.ctrl[0], 1);
        }
        __syncthreads();
        t = uniform(s_task);
    }
}

// Task lists in dependency order.  MAIN/CORR: blocks (I, I + D) by increasing
// D, then I.  SYL: blocks by increasing anti-diagonal (nbr - 1 - I) + J.
__global__ void k_tasks_tri(int nb, int mat, int2 *out, int64_t count)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    int64_t rem = t;
    int D = 1;
    while (rem >= nb - D) {
        rem -= nb - D;
        ++D;
    }
    const int I = (int)rem, J = I + D;
    out[t] = make_int2(mat, (I << 16) | J);
}

__global__ void k_tasks_rect(int nbr, int nbc, int mat, int2 *out, int64_t count)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    int64_t rem = t;
    for (int d = 0; d < nbr + nbc - 1; ++d) {
        // blocks with (nbr - 1 - I) + J = d: J = d - (nbr - 1 - I), 0 <= J < nbc
        const int ilo = max(0, nbr - 1 - d), ihi = min(nbr - 1, nbr - 1 - d + nbc - 1);
        const int cnt = ihi - ilo + 1;
        if (rem < cnt) {
            const int I = ihi - (int)rem;
            const int J = d - (nbr - 1 - I);
            out[t] = make_int2(mat, (I << 16) | J);
            return;
        }
        rem -= cnt;
    }
}

__global__ void k_fill_int(int *p, int64_t n, int v)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// Mark the blocks of a task list as not finished (flag 0).
__global__ void k_clear_task_flags(const int2 *tasks, int64_t ntasks, const int *ntasks_dev,
                                   const FlowMat<double> *mats, int *flags)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntasks || (ntasks_dev && t >= *ntasks_dev)) return;
    const int2 tk = tasks[t];
    const int I = tk.y >> 16, J = tk.y & 0xffff;
    flags[mats[tk.x].flag0 + (int64_t)I * mats[tk.x].nbc + J] = 0;
}

}  // namespace

hipError_t launch_fill_int(int *p, int64_t n, int v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_tasks_tri(int nb, int mat, int2 *out, hipStream_t st)
{
    const int64_t cnt = (int64_t)nb * (nb - 1) / 2;
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tasks_tri, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, nb, mat,
                       out, cnt);
    return hipGetLastError();
}

hipError_t launch_tasks_rect(int nbr, int nbc, int mat, int2 *out, hipStream_t st)
{
    const int64_t cnt = (int64_t)nbr * nbc;
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tasks_rect, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, nbr,
                       nbc, mat, out, cnt);
    return hipGetLastError();
}

hipError_t launch_clear_task_flags(const int2 *tasks, int64_t ntasks, const int *ntasks_dev,
                                   const FlowMat<double> *mats, int *flags, hipStream_t st)
{
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_task_flags, dim3((unsigned)((ntasks + 255) / 256)), dim3(256), 0,
                       st, tasks, ntasks, ntasks_dev, mats, flags);
    return hipGetLastError();
}

// Workgroups of a persistent sweep: as many as fit on the device at once
// (more would only queue behind the first wave of them).
struct FlowFit {
    int cus = 0, per = 0;
};

// Compute units of the current device and resident workgroups of this kernel per unit.
template <typename F, int KIND, bool C, int WPE> static FlowFit flow_fit()
{
    FlowFit f;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&f.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        f.cus <= 0)
        f.cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&f.per, k_flow<F, KIND, C, WPE>, NT, 0) !=
            hipSuccess ||
        f.per <= 0)
        f.per = 1;
    return f;
}

template <typename F, int KIND, bool C, int WPE> static const FlowFit &flow_fit_cached()
{
    static const FlowFit f = flow_fit<F, KIND, C, WPE>();
    return f;
}

// Resident workgroups per compute unit: of the build as allocated (lo) and the
// most of any build (hi).
template <typename F, int KIND, bool C> static int flow_per(bool hi)
{
    const int lo = flow_fit_cached<F, KIND, C, 0>().per;
    if constexpr (FlowWaves<F, C>::value > 0) {
        if (hi) return std::max(lo, flow_fit_cached<F, KIND, C, FlowWaves<F, C>::value>().per);
    }
    return lo;
}

// The persistent grid: wgs_per_cu workgroups on every compute unit (0: as many
// as the first build fits; more than any build fits: as many as fit), never
// more than there are tasks.  Tasks are taken by ticket in dependency order, so
// any grid size is deadlock-free.
template <typename F, int KIND, bool C>
hipError_t launch_flow(const FlowArgs<F> &a, int wgs_per_cu, hipStream_t st)
{
    if (a.ntasks <= 0) return hipSuccess;
    const int cus = flow_fit_cached<F, KIND, C, 0>().cus;
    const int lo = flow_per<F, KIND, C>(false), hi = flow_per<F, KIND, C>(true);
    const int per = wgs_per_cu <= 0 ? lo : std::min(wgs_per_cu, hi);
    const int g = std::min(cus * per, a.ntasks);
    if constexpr (FlowWaves<F, C>::value > 0) {
        if (per > lo) {
            hipLaunchKernelGGL((k_flow<F, KIND, C, FlowWaves<F, C>::value>), dim3(g), dim3(NT), 0,
                               st, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_flow<F, KIND, C, 0>), dim3(g), dim3(NT), 0, st, a);
    return hipGetLastError();
}

// Workgroups per compute unit: the most any build of a mode's sweeps fits (hi,
// the autotuner's range and the batched form's default), or the most the first
// build fits (the default of a single call, whose large blocks gain nothing
// from the second build's extra workgroup).
static int flow_wgs_per_cu(bool fp32, bool cplx, bool hi)
{
    if (cplx) {
        if (fp32)
            return std::min({flow_per<float, FLOW_MAIN, true>(hi),
                             flow_per<float, FLOW_CORR, true>(hi),
                             flow_per<float, FLOW_SYL, true>(hi)});
        return std::min(flow_per<double, FLOW_MAIN, true>(hi),
                        flow_per<double, FLOW_SYL, true>(hi));
    }
    if (fp32)
        return std::min({flow_per<float, FLOW_MAIN, false>(hi),
                         flow_per<float, FLOW_CORR, false>(hi),
                         flow_per<float, FLOW_SYL, false>(hi)});
    return std::min(flow_per<double, FLOW_MAIN, false>(hi),
                    flow_per<double, FLOW_SYL, false>(hi));
}

int flow_max_wgs_per_cu(bool fp32, bool cplx) { return flow_wgs_per_cu(fp32, cplx, true); }

int flow_default_wgs_per_cu(bool fp32, bool cplx) { return flow_wgs_per_cu(fp32, cplx, false); }

#define SGT_FLOW(F, K, C) \
    template hipError_t launch_flow<F, K, C>(const FlowArgs<F> &, int, hipStream_t);
SGT_FLOW(double, FLOW_MAIN, false)
SGT_FLOW(double, FLOW_SYL, false)
SGT_FLOW(float, FLOW_MAIN, false)
SGT_FLOW(float, FLOW_CORR, false)
SGT_FLOW(float, FLOW_SYL, false)
SGT_FLOW(double, FLOW_MAIN, true)
SGT_FLOW(double, FLOW_SYL, true)
SGT_FLOW(float, FLOW_MAIN, true)
SGT_FLOW(float, FLOW_CORR, true)
SGT_FLOW(float, FLOW_SYL, true)
#undef SGT_FLOW

}  // namespace sgt
