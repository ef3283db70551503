// Real blocked Parlett-Higham sweep (64 x 64 or 32 x 32 blocks) on two streams.
//
// The block equations (Section 5; see ph_fp64.hip for their form) are solved
// superdiagonal by superdiagonal.  For block (I, J) on superdiagonal D the
// right-hand side is split by when its inputs exist (gemm_tile.hip):
//   bulk(D): K = I+2 .. J-2 and the diagonal-block terms -- needs D-2;
//   edge(D): K = I+1 and K = J-1                          -- needs D-1.
// The main stream runs edge(D) then solve(D) for D = 1, 2, ...; a side stream
// runs bulk(D+2) as soon as solve(D) has finished, so the bulk products of
// later superdiagonals overlap the solves of the current one.  Bulk partial
// sums alternate between two buffers by the parity of D.
//
// solve(D): one workgroup per block.  The right-hand side (bulk and edge
// partials) is summed into the block's LDS tile; then the entries are solved
// along anti-diagonals from the bottom-left corner, row i by LPR lanes.  The
// lanes of row i keep row i of U_II and T_II in registers (it is used at every
// step of that row); U_JJ and T_JJ are packed column-wise in LDS, and the
// reciprocals 1/(t_ii - t_jj) of the opposite-sign entries are tabulated
// before the sweep so no division sits on its critical path.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.h"

namespace sgt {

namespace {

template <typename F, int TB, int NT>
__global__ __launch_bounds__(NT) void k_solve_r(const F *__restrict__ T, int64_t ldt,
                                                F *__restrict__ U, int64_t ldu, int64_t n,
                                                const int8_t *__restrict__ sgn, int D, int nbulk,
                                                const F *__restrict__ Zb, int nedge,
                                                const F *__restrict__ Ze)
{
    constexpr int LPR = NT / TB;     // lanes per row
    constexpr int CPL = TB / LPR;    // row entries per lane
    constexpr int LDX = TB + 4;      // LDS pitch of the block being solved
    constexpr int P = TB * (TB + 1) / 2;
    __shared__ F sR[2 * P];          // packed column-major U_JJ (0) and T_JJ (P)
    __shared__ F X[TB * LDX];
    __shared__ double rcp[TB * TB];  // 1/(t_ii - t_jj), row-major
    __shared__ int8_t rs[TB], cs[TB];

    const int tid = threadIdx.x;
    const int I = blockIdx.x, J = I + D;
    const int64_t r0 = (int64_t)I * TB, c0 = (int64_t)J * TB;
    const int bj = (int)min((int64_t)TB, n - c0);
    const int i = tid / LPR, q = tid % LPR;

    // row i of U_II and T_II (upper part, k > i) in registers: entry k = q + LPR t
    F cu[CPL], ct[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
        const int k = q + LPR * t;
        const bool up = k > i;
        cu[t] = up ? U[(r0 + i) + (r0 + k) * ldu] : (F)0;
        ct[t] = up ? T[(r0 + i) + (r0 + k) * ldt] : (F)0;
    }
    for (int e = tid; e < TB * TB; e += NT) {
        const int r = e % TB, c = e / TB;
        if (r <= c) {
            const bool in = c < bj;
            const int pc = (c * (c + 1)) / 2 + r;
            sR[pc] = in ? U[(c0 + r) + (c0 + c) * ldu] : (F)0;
            sR[P + pc] = in ? T[(c0 + r) + (c0 + c) * ldt] : (F)0;
        }
    }
    // right-hand sides: bulk then edge partials, in slice order
    const F *zb = Zb + (int64_t)blockIdx.x * nbulk * TB * TB;
    const F *ze = Ze + (int64_t)blockIdx.x * nedge * TB * TB;
    for (int e = tid; e < TB * TB; e += NT) {
        const int r = e / TB, c = e % TB;
        F z = 0;
        for (int s = 0; s < nbulk; ++s) z += zb[(int64_t)s * TB * TB + e];
        for (int s = 0; s < nedge; ++s) z += ze[(int64_t)s * TB * TB + e];
        X[r + c * LDX] = z;
    }
    if (tid < TB) {
        rs[tid] = sgn[r0 + tid];
        cs[tid] = tid < bj ? sgn[c0 + tid] : sgn[r0 + tid];
    }
    __syncthreads();
    for (int e = tid; e < TB * TB; e += NT) {
        const int r = e / TB, c = e % TB;
        double v = 0.0;
        if (c < bj && rs[r] != cs[c])
            v = 1.0 / ((double)T[(r0 + r) + (r0 + r) * ldt] - (double)T[(c0 + c) + (c0 + c) * ldt]);
        rcp[e] = v;
    }
    // per-thread constants: sign of row i, bit mask of positive column signs
    const int si = rs[i];
    unsigned long long cpos = 0;
    for (int c = 0; c < bj; ++c) cpos |= (unsigned long long)(cs[c] > 0) << c;
    __syncthreads();

    const int steps = (TB - 1) + bj;
    for (int a = 0; a < steps; ++a) {
        const int j = a - (TB - 1 - i);
        if (j >= 0 && j < bj) {
            // equal signs: u = -(rhs + sum U_II u + sum u U_JJ) * s_i / 2        (U^2 = I)
            // opposite:    u = (rhs - sum T_II u + sum u T_JJ) / (t_ii - t_jj)   (TU = UT)
            const bool same = (((cpos >> j) & 1ull) != 0) == (si > 0);
            const int sel = same ? 0 : P;
            const int colstart = (j * (j + 1)) / 2;
            // every LDS load of the step is issued before any is used; the
            // register rows cu, ct are only indexed by compile-time constants
            F xc[CPL], xr[CPL], rr[CPL];
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const int k = q + LPR * t;
                xc[t] = k > i ? X[k + j * LDX] : (F)0;
                xr[t] = k < j ? X[i + k * LDX] : (F)0;
                rr[t] = k < j ? sR[sel + colstart + k] : (F)0;
            }
            const F rhs = X[i + j * LDX];
            const double rc = rcp[i * TB + j];
            F colu0 = 0, colu1 = 0, colt0 = 0, colt1 = 0, row0 = 0, row1 = 0;
#pragma unroll
            for (int t = 0; t < CPL; t += 2) {
                colu0 += cu[t] * xc[t];
                colt0 += ct[t] * xc[t];
                row0 += xr[t] * rr[t];
                if (t + 1 < CPL) {
                    colu1 += cu[t + 1] * xc[t + 1];
                    colt1 += ct[t + 1] * xc[t + 1];
                    row1 += xr[t + 1] * rr[t + 1];
                }
            }
            const double scale = same ? -0.5 * (double)si : rc;
            F tot = same ? (colu0 + colu1) + (row0 + row1) : (row0 + row1) - (colt0 + colt1);
            tot = group_sum<LPR>(tot);
            if (q == 0) X[i + j * LDX] = (F)(((double)rhs + (double)tot) * scale);
        }
        __syncthreads();
    }
    for (int e = tid; e < TB * TB; e += NT) {
        const int r = e % TB, c = e / TB;
        if (c < bj) U[(r0 + r) + (c0 + c) * ldu] = X[r + c * LDX];
    }
}

// Library-owned side stream and event pool, one per device.
struct Side {
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> events;
};
std::mutex side_mu;
std::vector<Side> sides;

hipError_t get_side(int nev, Side **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(side_mu);
    if ((int)sides.size() <= dev) sides.resize(dev + 1);
    Side &s = sides[dev];
    if (!s.stream) {
        e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    while ((int)s.events.size() < nev) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        s.events.push_back(ev);
    }
    *out = &s;
    return hipSuccess;
}

}  // namespace

int64_t ph_real_edge_slots(int64_t n, int tb)
{
    return 2 * (kLookahead - 1) * ((n + tb - 1) / tb);
}

template <typename F>
hipError_t launch_solve_r(int tb, const F *T, int64_t ldt, F *U, int64_t ldu, int64_t n,
                          const int8_t *sgn, int D, int ntiles, int nbulk, const F *Zb, int nedge,
                          const F *Ze, hipStream_t st)
{
    if (tb == 64)
        hipLaunchKernelGGL((k_solve_r<F, 64, 512>), dim3(ntiles), dim3(512), 0, st, T, ldt, U,
                           ldu, n, sgn, D, nbulk, Zb, nedge, Ze);
    else if (tb == 32)
        hipLaunchKernelGGL((k_solve_r<F, 32, 256>), dim3(ntiles), dim3(256), 0, st, T, ldt, U,
                           ldu, n, sgn, D, nbulk, Zb, nedge, Ze);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
template hipError_t launch_solve_r<double>(int, const double *, int64_t, double *, int64_t, int64_t,
                                           const int8_t *, int, int, int, const double *, int,
                                           const double *, hipStream_t);

// The block sweep of one triangular system, bulk products on the side stream.
hipError_t run_ph_real(RealSweep &w, hipStream_t st)
{
    const int tb = w.tile;
    const int64_t nb = (w.n + tb - 1) / tb;
    if (nb <= 1) return hipSuccess;
    Side *side = nullptr;
    hipError_t e = get_side((int)(2 * nb + 4), &side);
    if (e != hipSuccess) return e;
    hipStream_t ss = side->stream;
    hipEvent_t *ev = side->events.data();
    hipEvent_t ev_start = ev[0], ev_end = ev[1];
    auto ev_bulk = [&](int D) { return ev[2 + 2 * (D - 1)]; };
    auto ev_solve = [&](int D) { return ev[3 + 2 * (D - 1)]; };

    if ((e = hipEventRecord(ev_start, st)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(ss, ev_start, 0)) != hipSuccess) return e;

    constexpr int L = kLookahead;
    auto bulk = [&](int D) -> hipError_t {
        const int ntiles = (int)(nb - D);
        const int nm = wave_gemm_mid_splits(D, L, ntiles, w.max_splits, w.zslots);
        w.bulk_nm[D] = nm;
        prof_begin(ss);
        hipError_t r = launch_wave_gemm<double>(tb, w.T, w.ldt, w.U, w.ldu, w.n, w.sgn, D, ntiles,
                                                0, nm, L, w.zbuf[D % L], ss);
        prof_end(ss, PK_GEMM, w.flops ? w.flops->gemm_bulk(D, L) : 0.0);
        if (r != hipSuccess) return r;
        return hipEventRecord(ev_bulk(D), ss);
    };

    // bulk(D) needs superdiagonals <= D - L: the first L need only the diagonal blocks
    for (int D = 1; D <= L && D < nb; ++D)
        if ((e = bulk(D)) != hipSuccess) return e;
    for (int D = 1; D < nb; ++D) {
        const int ntiles = (int)(nb - D);
        if ((e = hipStreamWaitEvent(st, ev_bulk(D), 0)) != hipSuccess) return e;
        const int ne = wave_gemm_edge_slices(D, L);
        if (ne > 0) {
            prof_begin(st);
            e = launch_wave_gemm<double>(tb, w.T, w.ldt, w.U, w.ldu, w.n, w.sgn, D, ntiles, 1, 0,
                                         L, w.ebuf, st);
            prof_end(st, PK_GEMM, w.flops ? w.flops->gemm_edge(D, L) : 0.0);
            if (e != hipSuccess) return e;
        }
        prof_begin(st);
        e = launch_solve_r<double>(tb, w.T, w.ldt, w.U, w.ldu, w.n, w.sgn, D, ntiles,
                                   w.bulk_nm[D] + 1, w.zbuf[D % L], ne, w.ebuf, st);
        prof_end(st, PK_SOLVE, w.flops ? w.flops->solve(D) : 0.0);
        if (e != hipSuccess) return e;
        if ((e = hipEventRecord(ev_solve(D), st)) != hipSuccess) return e;
        // bulk(D + L) reuses the buffer solve(D) has just consumed
        if (D + L < nb) {
            if ((e = hipStreamWaitEvent(ss, ev_solve(D), 0)) != hipSuccess) return e;
            if ((e = bulk(D + L)) != hipSuccess) return e;
        }
    }
    if ((e = hipEventRecord(ev_end, ss)) != hipSuccess) return e;
    return hipStreamWaitEvent(st, ev_end, 0);
}

}  // namespace sgt
