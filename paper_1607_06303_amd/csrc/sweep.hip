// Host orchestration of the real dataflow sweeps (flow.hip) for the three
// precision modes, the Parlett-Higham and Parlett-Sylvester forms, and the
// refinement loop with its FP64 fallback (refine.hip).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace sgt {

namespace {

constexpr int TB = kFlowTile;
constexpr int kSpinLimit = 1 << 22;  // polls before a dependency wait gives up

int64_t nblocks(int64_t m) { return (m + TB - 1) / TB; }

// Zero the flags of every block and the control words, then run one sweep.
template <typename F, int KIND>
hipError_t run_sweep(const FlowMat<F> &m, const FlowWs &w, int64_t ntasks, int64_t nflags,
                     bool fresh_flags, int pk, double flops, hipStream_t st)
{
    hipError_t e;
    prof_begin(st);
    if (fresh_flags && (e = launch_fill_int(w.flags, nflags, 0, st)) != hipSuccess) return e;
    if ((e = launch_fill_int(w.ctrl, 2, 0, st)) != hipSuccess) return e;
    prof_end(st, PK_AUX, 0.0);
    FlowArgs<F> a;
    a.m0 = m;
    a.mats = nullptr;
    a.tasks = w.tasks;
    a.ntasks = (int)ntasks;
    a.ctrl = w.ctrl;
    a.flags = w.flags;
    a.spin_limit = kSpinLimit;
    prof_begin(st);
    e = launch_flow<F, KIND>(a, 0, st);
    prof_end(st, pk, flops);
    return e;
}

// Run a launch between the timer marks of its family.
template <typename Fn> hipError_t timed(hipStream_t st, int pk, double flops, Fn fn)
{
    prof_begin(st);
    hipError_t e = fn();
    prof_end(st, pk, flops);
    return e;
}

template <typename F>
FlowMat<F> ph_mat(const F *T, int64_t ldt, const F *C, int64_t ldc, F *V, int64_t ldv,
                  const double *dg, const int8_t *sgn, int64_t n)
{
    FlowMat<F> m;
    std::memset(&m, 0, sizeof(m));
    m.T = T;
    m.ldt = ldt;
    m.C = C;
    m.ldc = ldc;
    m.V = V;
    m.ldv = ldv;
    m.dg = dg;
    m.sgn = sgn;
    m.n = (int)n;
    m.nbr = m.nbc = (int)nblocks(n);
    return m;
}

template <typename F>
FlowMat<F> syl_mat(const F *T, int64_t ldt, F *V, int64_t ldv, const F *Rh, int64_t ldrh,
                   double scale, const double *dg, int64_t n, int64_t p)
{
    FlowMat<F> m;
    std::memset(&m, 0, sizeof(m));
    m.T = T;
    m.ldt = ldt;
    m.V = V;
    m.ldv = ldv;
    m.Rh = Rh;
    m.ldrh = ldrh;
    m.dg = dg;
    m.n = (int)n;
    m.split = (int)p;
    m.nbr = (int)nblocks(p);
    m.nbc = (int)nblocks(n - p);
    m.rhs_scale = scale;
    return m;
}

double ulp_floor(int D, double umax, double tmax)
{
    // rounding level of an FP64 residual block: (D + 1) * TB products per entry
    // of size up to umax * max(umax, tmax), TB x TB entries
    const double eps = std::ldexp(1.0, -52);
    return eps * (double)(D + 1) * TB * TB * umax * std::max(umax, tmax);
}

}  // namespace

FlowWs flow_ws_layout(char *base, int64_t n, bool mixed, size_t *total)
{
    const int64_t nb = std::max<int64_t>(nblocks(n), 1);
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    size_t off = 0;
    FlowWs w;
    std::memset(&w, 0, sizeof(w));
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += al(bytes);
        return p;
    };
    w.ctrl = (int *)take(64 * sizeof(int));
    // ctrl: [0] ticket, [1] error word, [8..13] three maxima, [16..18] flag-reset tables
    w.maxes = (unsigned long long *)(w.ctrl + 8);
    w.flags = (int *)take((size_t)nb * nb * sizeof(int));
    w.tasks = (int2 *)take((size_t)nb * nb * sizeof(int2));
    if (mixed) {
        w.ftasks = (int2 *)take((size_t)nb * nb * sizeof(int2));
        w.norms[0] = (double *)take((size_t)nb * nb * sizeof(double));
        w.norms[1] = (double *)take((size_t)nb * nb * sizeof(double));
        w.ld32 = std::max<int64_t>(n, 1);
        const size_t mat = (size_t)w.ld32 * std::max<int64_t>(n, 1) * sizeof(float);
        w.T32 = (float *)take(mat);
        w.U32 = (float *)take(mat);
        w.E32 = (float *)take(mat);
    }
    if (total) *total = off;
    return w;
}

size_t flow_host_bytes(int64_t n)
{
    const int64_t nb = std::max<int64_t>(nblocks(n), 1);
    return (size_t)nb * nb * (2 * sizeof(double) + sizeof(int2)) + 256;  // + small words
}

// FP64 Parlett-Higham: diagonal blocks, then the dataflow sweep.
hipError_t sweep_ph_fp64(const double *T, int64_t ldt, double *U, int64_t ldu, int64_t n,
                         const int8_t *sgn, const double *dg, const FlowWs &w,
                         const SweepFlops &fl, hipStream_t st)
{
    hipError_t e;
    const int64_t nb = nblocks(n), ntasks = nb * (nb - 1) / 2;
    e = timed(st, PK_AUX, 0.0, [&] {
        hipError_t r = launch_fill_int(w.ctrl, 16, 0, st);  // control words and maxima
        if (r == hipSuccess) r = launch_zero_lower(U, ldu, n, false, st);
        if (r == hipSuccess && ntasks > 0) r = launch_tasks_tri((int)nb, 0, w.tasks, st);
        return r;
    });
    if (e != hipSuccess) return e;
    e = timed(st, PK_DIAG, fl.diag, [&] { return launch_diag_blocks(T, ldt, U, ldu, n, sgn, st); });
    if (e != hipSuccess || ntasks == 0) return e;
    return run_sweep<double, FLOW_MAIN>(ph_mat<double>(T, ldt, nullptr, 0, U, ldu, dg, sgn, n), w,
                                        ntasks, nb * nb, true, PK_FLOW, fl.flow, st);
}

// FP64 Parlett-Sylvester for a diagonal grouped by sign: the first p entries
// have sign s, the rest -s; U = [[s I, X], [0, -s I]].
hipError_t sweep_ps_fp64(const double *T, int64_t ldt, double *U, int64_t ldu, int64_t n,
                         int64_t p, int s, const double *dg, const FlowWs &w,
                         const SweepFlops &fl, hipStream_t st)
{
    const int64_t nbr = nblocks(p), nbc = nblocks(n - p), ntasks = nbr * nbc;
    hipError_t e = timed(st, PK_AUX, 0.0, [&] {
        hipError_t r = launch_fill_int(w.ctrl, 16, 0, st);  // control words and maxima
        if (r == hipSuccess) r = launch_fill_split_identity(U, ldu, n, p, (double)s, st);
        if (r == hipSuccess) r = launch_tasks_rect((int)nbr, (int)nbc, 0, w.tasks, st);
        return r;
    });
    if (e != hipSuccess) return e;
    return run_sweep<double, FLOW_SYL>(syl_mat<double>(T, ldt, U, ldu, T, ldt, 2.0 * s, dg, n, p),
                                       w, ntasks, nbr * nbc, true, PK_SYL, fl.syl, st);
}

// Reduced-precision sweep, then (mode MIXED_REFINED) refinement steps with FP64
// residuals, and FP64 recomputation of the blocks that do not converge.
// p == 0: Parlett-Higham; p > 0: Parlett-Sylvester with leading sign s.
int sweep_mixed(const double *T, int64_t ldt, double *U, int64_t ldu, int64_t n,
                const int8_t *sgn, const double *dg, int64_t p, int s, bool refine,
                const signtri_options *opts, const FlowWs &w, void *host,
                const SweepFlops &fl, hipStream_t st, signtri_info *info)
{
    const bool syl = p > 0;
    const int64_t ld = w.ld32;
    hipError_t e;
#define HIPCHK(x)                                \
    do {                                         \
        if ((e = (x)) != hipSuccess) return SIGNTRI_EHIP; \
    } while (0)
    const int64_t nbr = syl ? nblocks(p) : nblocks(n), nbc = syl ? nblocks(n - p) : nbr;
    const int64_t ntasks = syl ? nbr * nbc : nbr * (nbr - 1) / 2, nflags = nbr * nbc;
    HIPCHK(timed(st, PK_AUX, 0.0, [&] {
        hipError_t r = launch_fill_int(w.ctrl, 16, 0, st);  // control words and maxima
        if (r == hipSuccess)
            r = syl ? launch_fill_split_identity(U, ldu, n, p, (double)s, st)
                    : launch_zero_lower(U, ldu, n, false, st);
        if (r == hipSuccess && ntasks > 0)
            r = syl ? launch_tasks_rect((int)nbr, (int)nbc, 0, w.tasks, st)
                    : launch_tasks_tri((int)nbr, 0, w.tasks, st);
        return r;
    }));
    if (!syl)
        HIPCHK(timed(st, PK_DIAG, fl.diag,
                     [&] { return launch_diag_blocks(T, ldt, U, ldu, n, sgn, st); }));
    HIPCHK(timed(st, PK_CONVERT, 0.0, [&] {
        return launch_to_f32(T, ldt, w.T32, U, ldu, w.U32, ld, n, &w.maxes[0], st);
    }));
    if (ntasks == 0) return SIGNTRI_OK;

    // U0 in FP32
    if (syl)
        HIPCHK((run_sweep<float, FLOW_SYL>(
            syl_mat<float>(w.T32, ld, w.U32, ld, w.T32, ld, 2.0 * s, dg, n, p), w, ntasks, nflags,
            true, PK_SYL, fl.syl, st)));
    else
        HIPCHK((run_sweep<float, FLOW_MAIN>(
            ph_mat<float>(w.T32, ld, nullptr, 0, w.U32, ld, dg, sgn, n), w, ntasks, nflags, true,
            PK_FLOW, fl.flow, st)));
    HIPCHK(timed(st, PK_CONVERT, 0.0,
                 [&] { return launch_widen(w.U32, ld, U, ldu, n, p, &w.maxes[1], st); }));
    if (!refine) return SIGNTRI_OK;

    auto resid = [&](double *norm2) -> hipError_t {
        return timed(st, PK_RESID, fl.resid, [&] {
            if (syl)
                return launch_resid_syl(T, ldt, U, ldu, n, p, 2.0 * s, w.tasks, (int)ntasks,
                                        (int)nbr, (int)nbc, w.E32, ld, norm2, st);
            return launch_resid(T, ldt, U, ldu, sgn, n, w.tasks, (int)ntasks, w.E32, ld, norm2,
                                st);
        });
    };
    HIPCHK(resid(w.norms[0]));

    const int max_steps = (opts && opts->max_refine_steps > 0) ? opts->max_refine_steps : 2;
    const double stall = (opts && opts->stall_ratio > 0) ? opts->stall_ratio : 0.5;
    const double conv = 1e-5;  // residual reduction that counts as converged
    const int64_t force = opts ? opts->force_stall : 0;

    char *hb = (char *)host;
    double *h0 = (double *)hb, *h1 = h0 + nflags;
    int2 *hf = (int2 *)(h1 + nflags);
    unsigned long long *hm = (unsigned long long *)(hf + nflags);  // 3 maxima
    int *herr = (int *)(hm + 3);                                   // 2 control words
    int64_t *hflag0 = (int64_t *)(herr + 2);
    int *hnbc = (int *)(hflag0 + 1);
    // per block: residual norm before the first step, converged, hopeless (stalled)
    std::vector<double> rinit((size_t)nflags, 0.0);
    std::vector<char> ok((size_t)nflags, 0), hopeless((size_t)nflags, 0);
    int steps = 0;
    int cur = 0;
    double emax_all = 0.0;
    for (int step = 1; step <= max_steps; ++step) {
        // correction E (FP32): residual in E32 on entry, E on exit
        if (syl)
            HIPCHK((run_sweep<float, FLOW_SYL>(
                syl_mat<float>(w.T32, ld, w.E32, ld, w.E32, ld, 1.0, dg, n, p), w, ntasks, nflags,
                true, PK_CORR, fl.syl, st)));
        else
            HIPCHK((run_sweep<float, FLOW_CORR>(
                ph_mat<float>(w.T32, ld, w.U32, ld, w.E32, ld, dg, sgn, n), w, ntasks, nflags,
                true, PK_CORR, fl.corr, st)));
        HIPCHK(timed(st, PK_CONVERT, 0.0, [&] {
            hipError_t r = launch_fill_int((int *)&w.maxes[2], 2, 0, st);
            if (r == hipSuccess) r = launch_add_correction(w.E32, ld, U, ldu, n, p, &w.maxes[2], st);
            return r;
        }));
        HIPCHK(resid(w.norms[cur ^ 1]));
        steps = step;
        // convergence decision on the host
        HIPCHK(hipMemcpyAsync(h0, w.norms[cur], nflags * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h1, w.norms[cur ^ 1], nflags * sizeof(double), hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipMemcpyAsync(hm, w.maxes, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipMemcpyAsync(herr, w.ctrl, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (herr[1]) return SIGNTRI_EHIP;
        double tmax, umax, emax;
        std::memcpy(&tmax, &hm[0], 8);
        std::memcpy(&umax, &hm[1], 8);
        std::memcpy(&emax, &hm[2], 8);
        emax_all = umax > 0 ? emax / umax : emax;
        bool pending = false;
        for (int64_t I = 0; I < nbr; ++I)
            for (int64_t J = syl ? 0 : I + 1; J < nbc; ++J) {
                const int64_t f = I * nbc + J;
                const double aprev = std::sqrt(h0[f]), a = std::sqrt(h1[f]);
                if (step == 1) rinit[f] = aprev;
                // K blocks in each entry's residual products
                const int kb = syl ? (int)((nbr - I) + (J + 1)) : (int)(J - I + 1);
                const bool forced = force == -1 || (force > 0 && force - 1 == f);
                const bool good = !forced && a <= std::max(ulp_floor(kb - 1, umax, tmax),
                                                           conv * rinit[f]);
                ok[f] = good;
                if (!good && (forced || a > stall * aprev)) hopeless[f] = 1;
                if (!good && !hopeless[f]) pending = true;
            }
        cur ^= 1;
        if (!pending) break;
    }
    std::vector<char> bad((size_t)nflags, 0);
    bool any_bad = false;
    for (int64_t I = 0; I < nbr; ++I)
        for (int64_t J = syl ? 0 : I + 1; J < nbc; ++J) {
            bad[I * nbc + J] = !ok[I * nbc + J];
            any_bad |= bad[I * nbc + J] != 0;
        }
    if (info) {
        info->refine_steps = steps;
        info->correction_rel = emax_all;
    }
    if (!any_bad) return SIGNTRI_OK;
    if (opts && opts->no_fallback) return SIGNTRI_ENOCONV;

    // FP64 recomputation of the blocks that did not converge and of every block
    // whose products read them.  In both forms block (I, J) is read by the
    // blocks (I', J') with I' <= I and J' >= J (MAIN: U_IK U_KJ with K = I or J;
    // SYL: A_I'K X_KJ with K = I, X_IK B_KJ' with K = J), so the cone is grown
    // from below and from the left.
    std::vector<char> mk(bad);
    for (int64_t I = nbr - 1; I >= 0; --I)
        for (int64_t J = syl ? 0 : I + 1; J < nbc; ++J) {
            char m = mk[I * nbc + J];
            if (I + 1 < nbr && (syl || I + 1 < J)) m |= mk[(I + 1) * nbc + J];
            if (J - 1 >= (syl ? 0 : I + 1)) m |= mk[I * nbc + J - 1];
            mk[I * nbc + J] = m;
        }
    int64_t nfb = 0;
    if (syl) {
        for (int64_t d = 0; d < nbr + nbc - 1; ++d)
            for (int64_t I = nbr - 1; I >= 0; --I) {
                const int64_t J = d - (nbr - 1 - I);
                if (J >= 0 && J < nbc && mk[I * nbc + J]) hf[nfb++] = make_int2(0, (int)((I << 16) | J));
            }
    } else {
        for (int64_t D = 1; D < nbr; ++D)
            for (int64_t I = 0; I + D < nbr; ++I)
                if (mk[I * nbc + I + D]) hf[nfb++] = make_int2(0, (int)((I << 16) | (I + D)));
    }
    if (info) info->fallback_tiles = nfb;
    if (nfb == 0) return SIGNTRI_OK;
    HIPCHK(hipMemcpyAsync(w.ftasks, hf, nfb * sizeof(int2), hipMemcpyHostToDevice, st));
    HIPCHK(launch_fill_int(w.flags, nflags, 1, st));
    int64_t *flag0 = (int64_t *)(w.ctrl + 16);  // one-matrix tables for the flag reset
    int *nbcd = w.ctrl + 18;
    *hflag0 = 0;
    *hnbc = (int)nbc;
    HIPCHK(hipMemcpyAsync(flag0, hflag0, sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(nbcd, hnbc, sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(launch_clear_task_flags(w.ftasks, nfb, flag0, nbcd, w.flags, st));
    FlowWs wf = w;
    wf.tasks = w.ftasks;
    if (syl)
        HIPCHK((run_sweep<double, FLOW_SYL>(syl_mat<double>(T, ldt, U, ldu, T, ldt, 2.0 * s, dg, n, p),
                                            wf, nfb, nflags, false, PK_SYL, 0.0, st)));
    else
        HIPCHK((run_sweep<double, FLOW_MAIN>(ph_mat<double>(T, ldt, nullptr, 0, U, ldu, dg, sgn, n),
                                             wf, nfb, nflags, false, PK_FLOW, 0.0, st)));
    HIPCHK(hipMemcpyAsync(herr, w.ctrl, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr[1]) return SIGNTRI_EHIP;
#undef HIPCHK
    return SIGNTRI_OK;
}

}  // namespace sgt
