// Host orchestration of the real sweeps (flow.hip) for a set of matrices --
// one for signtri(), many for signtri_batched() -- in the three precision
// modes, with the Parlett-Higham and Parlett-Sylvester forms side by side and
// the refinement loop with its FP64 fallback (refine.hip).  Every phase is one
// launch over all matrices: the dataflow kernel takes one task list spanning
// them (dependency order within each matrix, interleaved across matrices), and
// the other kernels take per-matrix tables.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"

namespace sgt {

namespace {

constexpr int TB = kFlowTile;
constexpr int kSpinLimit = 1 << 22;  // polls before a dependency wait gives up


int64_t nblocks(int64_t m) { return (m + TB - 1) / TB; }
size_t al(size_t x) { return (x + 255) / 256 * 256; }

template <typename Fn> hipError_t timed(hipStream_t st, int pk, double flops, Fn fn)
{
    prof_begin(st);
    hipError_t e = fn();
    prof_end(st, pk, flops);
    return e;
}

// One dataflow sweep over a task list (after zeroing the control words).
template <typename F, int KIND, bool C>
hipError_t run_flow(const FlowMat<F> *mats, const int2 *tasks, int64_t nt, int *ctrl, int *flags,
                    int pk, double flops, int wgs, hipStream_t st, const int *live,
                    const int *ntasks_dev)
{
    if (nt == 0) return hipSuccess;
    // the ticket counter only: the error word (ctrl[1]) is cleared once per run,
    // so that a wait that gave up in an earlier sweep of the run is still reported
    hipError_t r = launch_fill_int(ctrl, 1, 0, st);
    if (r != hipSuccess) return r;
    FlowArgs<F> a;
    std::memset(&a, 0, sizeof(a));
    a.mats = mats;
    a.tasks = tasks;
    a.ntasks = (int)nt;
    a.ctrl = ctrl;
    a.flags = flags;
    a.spin_limit = flow_spin_limit();
    a.live = live;
    a.ntasks_dev = ntasks_dev;
    prof_begin(st);
    r = launch_flow<F, KIND, C>(a, wgs, st);
    prof_end(st, pk, flops);
    return r;
}

// live: the sweep runs only if *live != 0 (a refinement step); ntasks_dev: the
// task count, read on the device (a task list built there); both optional.
template <typename F, int KIND>
hipError_t run_flow_any(bool cplx, const FlowMat<F> *mats, const int2 *tasks, int64_t nt, int *ctrl,
                        int *flags, int pk, double flops, int wgs, hipStream_t st,
                        const int *live = nullptr, const int *ntasks_dev = nullptr)
{
    return cplx ? run_flow<F, KIND, true>(mats, tasks, nt, ctrl, flags, pk, flops, wgs, st, live,
                                          ntasks_dev)
                : run_flow<F, KIND, false>(mats, tasks, nt, ctrl, flags, pk, flops, wgs, st, live,
                                           ntasks_dev);
}

template <typename F>
FlowMat<F> ph_mat(const F *T, int64_t ldt, const F *C, int64_t ldc, F *V, int64_t ldv,
                  const double *dg, const int8_t *sgn, int64_t n, int64_t flag0)
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
    m.flag0 = flag0;
    return m;
}

template <typename F>
FlowMat<F> syl_mat(const F *T, int64_t ldt, F *V, int64_t ldv, const F *Rh, int64_t ldrh,
                   double scale, const double *dg, int64_t n, int64_t p, int64_t flag0)
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
    m.flag0 = flag0;
    return m;
}

// The refinement's summary, read back once at the end: live[0 .. kMaxRefineSteps]
// (live[k - 1]: step k ran), the recomputation's task counts (two), and the
// blocks recomputed per matrix.
constexpr int kSumInts = kMaxRefineSteps + 1 + 2;
size_t sum_bytes(int nm) { return al(kSumInts * sizeof(int)) + (size_t)nm * sizeof(int64_t); }

// Byte layout of a run.  The tables and task lists are built in pinned host
// memory at the same offsets they take in device memory (one copy uploads
// them); the rest of each buffer is its own.  Sizes are upper bounds valid for
// any diagonal: a matrix has at most nb^2 blocks in either form.
struct Lay {
    size_t fm64, fm32, fmc, rm, pm, dtasks, tasks, rtiles, minl, stasks, sgroups, shared;  // shared
    size_t ctrl, flags, ftasks, norms0, norms1, maxes, rinit, okf, hop, rowmin, sum, f32, gbuf, dev;
    size_t h_err, h_sum, h_maxes, host;
    int64_t nflags_max, ntasks_max, ndiag_max, nrows, nminl_max, nstasks_max, ngroups_max, ngbuf_max;
    std::vector<int64_t> off32;  // per matrix, in floats, of its three FP32 n x n arrays
                                 // (complex: interleaved pairs, twice the floats)
};

Lay make_lay(const int64_t *ns, int nm, bool mixed, bool cplx)
{
    Lay L;
    int64_t sq = 0, sq4 = 0, nbsum = 0, f32 = 0, nminl = 0, nstasks = 0, ngroups = 0, ngbuf = 0;
    L.off32.resize(nm);
    for (int m = 0; m < nm; ++m) {
        const int64_t nb = nblocks(ns[m]), nb4 = (nb + 3) / 4;
        sq += nb * nb;
        sq4 += nb4 * nb4;
        nbsum += nb;
        // the residual's strips (a minority class of at most n / kStripDiv entries)
        const int64_t groups = (ns[m] / kStripDiv + 15) / 16;
        nminl += 16 * groups;
        nstasks += 2 * groups * ((ns[m] + 15) / 16);
        ngroups += groups;
        ngbuf += groups * 64 * ns[m];  // four k-major copies of 16 rows or columns
        L.off32[m] = f32;
        if (mixed) f32 += (cplx ? 6 : 3) * ns[m] * ns[m];
    }
    L.nflags_max = L.ntasks_max = std::max<int64_t>(sq, 1);
    L.ndiag_max = std::max<int64_t>(nbsum, 1);
    L.nrows = nbsum + nm;  // block rows, one more per matrix
    size_t o = 0;
    L.fm64 = o; o += al(nm * sizeof(FlowMat<double>));
    L.fm32 = o; o += al(mixed ? nm * sizeof(FlowMat<float>) : 0);
    L.fmc = o; o += al(mixed ? nm * sizeof(FlowMat<float>) : 0);
    L.rm = o; o += al(mixed ? nm * sizeof(RefMat) : 0);
    L.pm = o; o += al(nm * sizeof(PrepMat));
    L.dtasks = o; o += al(L.ndiag_max * sizeof(int2));
    L.tasks = o; o += al(L.ntasks_max * sizeof(int2));
    L.rtiles = o; o += al((mixed ? std::max<int64_t>(sq4, 1) : 0) * sizeof(int2));
    L.nminl_max = mixed && !cplx ? nminl : 0;
    L.nstasks_max = mixed && !cplx ? nstasks : 0;
    L.ngroups_max = mixed && !cplx ? ngroups : 0;
    L.ngbuf_max = mixed && !cplx ? ngbuf : 0;
    L.minl = o; o += al((size_t)L.nminl_max * sizeof(int));
    L.stasks = o; o += al((size_t)L.nstasks_max * sizeof(int4));
    L.sgroups = o; o += al((size_t)L.ngroups_max * sizeof(int4));
    L.shared = o;
    size_t d = o;
    L.ctrl = d; d += al(64 * sizeof(int));
    L.flags = d; d += al(L.nflags_max * sizeof(int));
    L.ftasks = d; d += al(mixed ? L.ntasks_max * sizeof(int2) : 0);
    L.norms0 = d; d += al(mixed ? L.nflags_max * sizeof(double) : 0);
    L.norms1 = d; d += al(mixed ? L.nflags_max * sizeof(double) : 0);
    L.maxes = d; d += al(mixed ? 3 * nm * sizeof(unsigned long long) : 0);
    L.rinit = d; d += al(mixed ? L.nflags_max * sizeof(double) : 0);
    L.okf = d; d += al(mixed ? (size_t)L.nflags_max : 0);
    L.hop = d; d += al(mixed ? (size_t)L.nflags_max : 0);
    L.rowmin = d; d += al(mixed ? L.nrows * sizeof(int) : 0);
    L.sum = d; d += al(mixed ? sum_bytes(nm) : 0);
    L.f32 = d; d += al((size_t)f32 * sizeof(float));
    L.gbuf = d; d += al((size_t)L.ngbuf_max * sizeof(double));
    L.dev = d;
    size_t h = o;
    L.h_err = h; h += al(64);
    L.h_sum = h; h += al(mixed ? sum_bytes(nm) : 0);
    L.h_maxes = h; h += al(mixed ? 3 * nm * sizeof(unsigned long long) : 0);
    L.host = h;
    return L;
}

// Refinement steps at most: 0 = the default of two; a negative value takes none
// (every block then counts as not converged: the FP64 recomputation, or
// SIGNTRI_ENOCONV).
int refine_step_count(const signtri_options *opts)
{
    if (!opts || opts->max_refine_steps == 0) return 2;
    return std::min(std::max(0, opts->max_refine_steps), kMaxRefineSteps);
}

// Algorithmic flops (Section 3 counting, real) of one matrix's launches.
SweepFlops item_flops(const int8_t *s, const RealItem &it)
{
    SweepFlops f;
    const int64_t n = it.n;
    if (it.path == SIGNTRI_PATH_TRIVIAL || !s) return f;
    const HostPlan p = plan_from_signs(s, n, false);
    const double dn = (double)n, np = (double)p.n_pos, nn = (double)p.n_neg;
    if (it.path == SIGNTRI_PATH_PS) {
        // (p - 1 - i) + (j - p) multiply-adds per entry of X
        f.syl = np * nn * (dn - 2.0);
        f.resid = f.syl + 4.0 * np * nn;
        return f;
    }
    const FlopCounter fc{s, n, TB, 1.0};
    f.diag = fc.diag();
    f.flow = p.w_ph - f.diag;
    double cdiag = 0.0;
    for (int64_t r0 = 0; r0 < n; r0 += TB) {
        const double b = (double)std::min<int64_t>(TB, n - r0);
        cdiag += b * (b - 1) * (b - 2) / 6.0;
    }
    // correction: two products per k strictly between i and j, off the diagonal blocks
    f.corr = 4.0 * (dn * (dn - 1) * (dn - 2) / 6.0 - cdiag);
    // residual: k = i .. j, two more terms per entry than the sweep
    f.resid = f.flow + 2.0 * (2.0 * dn * (dn - 1) / 2.0 + 2.0 * np * nn);
    return f;
}

}  // namespace

int flow_spin_limit()
{
    const char *v = getenv("SIGNTRI_DEBUG_SPIN_LIMIT");
    if (v && *v) return atoi(v);
    return kSpinLimit;
}

void run_sizes(const int64_t *ns, int nmat, bool mixed, bool cplx, size_t *dev_bytes,
               size_t *host_bytes)
{
    const Lay L = make_lay(ns, nmat, mixed, cplx);
    if (dev_bytes) *dev_bytes = L.dev;
    if (host_bytes) *host_bytes = L.host;
}

int sweep_error(void *dev_ws, const int64_t *ns, int nmat, bool mixed, bool cplx, void *host_ws,
                hipStream_t st, int *err)
{
    const Lay L = make_lay(ns, nmat, mixed, cplx);
    int *herr = (int *)((char *)host_ws + L.h_err);
    if (hipMemcpyAsync(herr, (char *)dev_ws + L.ctrl, 2 * sizeof(int), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return SIGNTRI_EHIP;
    if (err) *err = herr[1];
    return herr[1] ? SIGNTRI_EHIP : SIGNTRI_OK;
}

int run_real(std::vector<RealItem> &items, signtri_mode mode, const signtri_options *opts,
             void *dev_ws, void *host_ws, bool prof, const int8_t *const *host_signs,
             hipStream_t st, bool finish)
{
    const int nm = (int)items.size();
    if (nm == 0) return SIGNTRI_OK;
    const bool mixed = mode != SIGNTRI_FP64, refine = mode == SIGNTRI_MIXED_REFINED;
    const bool cplx = items[0].cplx;  // every item of a run has the same entry type
    const int P = cplx ? 2 : 1;
    const int wgs = opts ? opts->wgs_per_cu : 0;
    std::vector<int64_t> ns(nm);
    int64_t nmax = 0;
    for (int m = 0; m < nm; ++m) {
        ns[m] = items[m].n;
        nmax = std::max(nmax, ns[m]);
    }
    const Lay L = make_lay(ns.data(), nm, mixed, cplx);
    char *D = (char *)dev_ws, *H = (char *)host_ws;
    FlowMat<double> *hf64 = (FlowMat<double> *)(H + L.fm64);
    FlowMat<float> *hf32 = (FlowMat<float> *)(H + L.fm32);
    FlowMat<float> *hfc = (FlowMat<float> *)(H + L.fmc);
    RefMat *hrm = (RefMat *)(H + L.rm);
    PrepMat *hpm = (PrepMat *)(H + L.pm);
    int2 *hdt = (int2 *)(H + L.dtasks);
    int2 *htk = (int2 *)(H + L.tasks);
    int *ctrl = (int *)(D + L.ctrl);
    int *flags = (int *)(D + L.flags);
    unsigned long long *maxes = (unsigned long long *)(D + L.maxes);
    float *f32 = (float *)(D + L.f32);

    // ---- per-matrix geometry and tables
    std::vector<int64_t> f0(nm, 0);
    std::vector<int> nbr(nm, 0), nbc(nm, 0);
    int64_t nflags = 0, ndiag = 0, fr0 = 0;
    SweepFlops fl;
    for (int m = 0; m < nm; ++m) {
        const RealItem &it = items[m];
        const int64_t n = it.n;
        const bool ps = it.path == SIGNTRI_PATH_PS, triv = it.path == SIGNTRI_PATH_TRIVIAL;
        nbr[m] = triv ? 0 : (int)(ps ? nblocks(it.p) : nblocks(n));
        nbc[m] = triv ? 0 : (int)(ps ? nblocks(n - it.p) : nblocks(n));
        f0[m] = nflags;
        nflags += (int64_t)nbr[m] * nbc[m];
        hpm[m] = PrepMat{it.T, it.ldt, it.U, it.ldu, n, it.sgn, triv ? 2 : (ps ? 1 : 0), it.p,
                         (double)it.s, it.fd};
        if (ps)
            hf64[m] = syl_mat<double>(it.T, it.ldt, it.U, it.ldu, it.T, it.ldt, 2.0 * it.s, it.dg,
                                      n, it.p, f0[m]);
        else
            hf64[m] = ph_mat<double>(it.T, it.ldt, nullptr, 0, it.U, it.ldu, it.dg, it.sgn, n,
                                     f0[m]);
        hf64[m].general = it.fd != nullptr;
        const int dense = opts && opts->products == SIGNTRI_PRODUCTS_DENSE;
        hf64[m].dense = dense;
        if (!triv && !ps)
            for (int64_t I = 0; I < nblocks(n); ++I) hdt[ndiag++] = make_int2(m, (int)I);
        if (mixed) {
            float *T32 = f32 + L.off32[m], *U32 = T32 + P * n * n, *E32 = U32 + P * n * n;
            const int64_t ld = std::max<int64_t>(n, 1);
            if (ps) {
                hf32[m] = syl_mat<float>(T32, ld, U32, ld, T32, ld, 2.0 * it.s, it.dg, n, it.p,
                                         f0[m]);
                hfc[m] = syl_mat<float>(T32, ld, E32, ld, E32, ld, 1.0, it.dg, n, it.p, f0[m]);
            } else {
                hf32[m] = ph_mat<float>(T32, ld, nullptr, 0, U32, ld, it.dg, it.sgn, n, f0[m]);
                hfc[m] = ph_mat<float>(T32, ld, U32, ld, E32, ld, it.dg, it.sgn, n, f0[m]);
                hf32[m].dense = hfc[m].dense = dense;
            }
            RefMat &r = hrm[m];
            std::memset(&r, 0, sizeof(r));
            r.T = it.T;
            r.ldt = it.ldt;
            r.U = it.U;
            r.ldu = it.ldu;
            r.T32 = T32;
            r.U32 = U32;
            r.E32 = E32;
            r.ld32 = ld;
            r.sgn = it.sgn;
            r.n = triv ? 0 : (int)n;
            r.split = ps ? (int)it.p : 0;
            r.nbr = nbr[m];
            r.nbc = nbc[m];
            r.two_s = 2.0 * it.s;
            r.f0 = f0[m];
            r.fr0 = fr0;
            r.maxes = maxes + 3 * m;
        }
        fr0 += nbr[m] + 1;
        if (prof && host_signs) {
            const SweepFlops g = item_flops(host_signs[m], it);
            fl.diag += g.diag;
            fl.flow += g.flow;
            fl.corr += g.corr;
            fl.resid += g.resid;
            fl.syl += g.syl;
        }
    }
    // ---- task lists: Parlett-Higham blocks by superdiagonal D across the
    // matrices (largest first), then Sylvester blocks by anti-diagonal
    std::vector<int> order(nm);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ns[a] > ns[b]; });
    int64_t nph = 0, nps = 0;
    const int nbmax = (int)nblocks(nmax);
    for (int Dd = 1; Dd < nbmax; ++Dd)
        for (int m : order)
            if (items[m].path == SIGNTRI_PATH_PH)
                for (int I = 0; I + Dd < nbr[m]; ++I)
                    htk[nph++] = make_int2(m, (I << 16) | (I + Dd));
    for (int d = 0; d < 2 * nbmax; ++d)
        for (int m : order)
            if (items[m].path == SIGNTRI_PATH_PS)
                for (int I = nbr[m] - 1; I >= 0; --I) {
                    const int J = d - (nbr[m] - 1 - I);
                    if (J >= 0 && J < nbc[m]) htk[nph + nps++] = make_int2(m, (I << 16) | J);
                }
    // 128 x 128 tiles (four blocks a side) of the real substitution form's
    // residual, shortest first (the kernel takes them in reverse); a diagonal
    // tile only if it holds a block above the diagonal.  A matrix whose minority
    // sign class has at most n / kStripDiv entries (known from the host's copy of
    // the signs) takes its entries of equal signs from the tiles (its tiles
    // after the others', for the tile kernel's equal-signs form) and those of
    // differing signs from strips over the minority rows and columns.
    int64_t nrt = 0, nrty = 0, nstr = 0, ngr = 0;
    if (mixed && !cplx) {
        std::vector<char> strips(nm, 0);
        int *hminl = (int *)(H + L.minl);
        int4 *hst = (int4 *)(H + L.stasks);
        int4 *hgr = (int4 *)(H + L.sgroups);
        int64_t nminl = 0, goff = 0;
        for (int m = 0; m < nm && host_signs; ++m) {
            const RealItem &it = items[m];
            if (it.path != SIGNTRI_PATH_PH || it.fd || it.n < 2 * kFlowTile) continue;
            const int8_t *hs = host_signs[m];
            int64_t npos = 0;
            for (int64_t i = 0; i < it.n; ++i) npos += hs[i] > 0;
            const int64_t nneg = it.n - npos, mc = std::min(npos, nneg);
            if (mc == 0 || mc > it.n / kStripDiv) continue;
            const int8_t ms = nneg <= npos ? -1 : 1;  // the minority sign (ties: negative)
            const int64_t o0 = nminl;
            for (int64_t i = 0; i < it.n; ++i)
                if (hs[i] == ms) hminl[nminl++] = (int)i;
            while ((nminl - o0) % 16) hminl[nminl++] = -1;
            for (int64_t go = o0; go < nminl; go += 16, ++ngr) {
                const int gmin = hminl[go];
                int gmax = gmin;
                for (int u = 1; u < 16; ++u)
                    if (hminl[go + u] >= 0) gmax = hminl[go + u];
                hgr[ngr] = make_int4(m, 0, (int)(uint32_t)goff, (int)(uint32_t)(goff >> 32));
                goff += 64 * it.n;
                // rows of blocks above the group's last column's block, nearest the top
                // (longest) first; columns of blocks past its first row's block, farthest first
                for (int t0 = 0; t0 < (gmax >> 5) << 5; t0 += 16) hst[nstr++] = make_int4(m, 0, (int)ngr, t0);
                for (int64_t t0 = (it.n - 1) / 16 * 16; t0 >= (int64_t)((gmin >> 5) + 1) << 5; t0 -= 16)
                    hst[nstr++] = make_int4(m, 1, (int)ngr, (int)t0);
            }
            strips[m] = 1;
        }
        // longest K range first (the strips are taken in launch order)
        auto klen = [&](const int4 &t) {
            const int *g = hminl + 16 * (int64_t)t.z;
            int gmax = g[0];
            for (int u = 1; u < 16; ++u)
                if (g[u] >= 0) gmax = g[u];
            return t.y == 0 ? (int64_t)gmax - t.w
                            : std::min<int64_t>(items[t.x].n - 1, (int64_t)t.w + 15) - g[0];
        };
        std::stable_sort(hst, hst + nstr, [&](const int4 &a, const int4 &b) { return klen(a) > klen(b); });
        int2 *hrt = (int2 *)(H + L.rtiles);
        const int nb4max = (int)((nblocks(nmax) + 3) / 4);
        int64_t k = 0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int dd = 0; dd < nb4max; ++dd)
                for (auto it = order.rbegin(); it != order.rend(); ++it) {
                    const int m = *it;
                    if (items[m].path != SIGNTRI_PATH_PH || strips[m] != pass) continue;
                    const int nb4 = (nbc[m] + 3) / 4;
                    for (int ta = 0; ta + dd < nb4; ++ta)
                        if (dd > 0 || 4 * ta + 1 < nbc[m]) hrt[k++] = make_int2(m, (ta << 16) | (ta + dd));
                }
            if (pass == 0) nrt = k;
        }
        nrty = k - nrt;
    }
    const int2 *drt = (const int2 *)(D + L.rtiles);
    const int *dminl = (const int *)(D + L.minl);
    const int4 *dst = (const int4 *)(D + L.stasks);
    const int4 *dgr = (const int4 *)(D + L.sgroups);
    double *dgbuf = (double *)(D + L.gbuf);
    const int2 *dtk = (const int2 *)(D + L.tasks);
    const int2 *dtk_ps = dtk + nph;
    const int2 *ddt = (const int2 *)(D + L.dtasks);

    hipError_t e;
#define HIPCHK(x)                                          \
    do {                                                   \
        if ((e = (x)) != hipSuccess) return SIGNTRI_EHIP;  \
    } while (0)
    HIPCHK(hipMemcpyAsync(D, H, L.shared, hipMemcpyHostToDevice, st));
    const FlowMat<double> *df64 = (const FlowMat<double> *)(D + L.fm64);
    const FlowMat<float> *df32 = (const FlowMat<float> *)(D + L.fm32);
    const FlowMat<float> *dfc = (const FlowMat<float> *)(D + L.fmc);
    const RefMat *drm = (const RefMat *)(D + L.rm);
    const PrepMat *dpm = (const PrepMat *)(D + L.pm);
    auto clear_flags = [&](int v) {
        return timed(st, PK_AUX, 0.0, [&] { return launch_fill_int(flags, nflags, v, st); });
    };

    // ---- outputs, diagonal blocks (FP64 in every mode)
    HIPCHK(timed(st, PK_AUX, 0.0, [&] {
        hipError_t r = launch_fill_int(ctrl, 16, 0, st);
        if (r == hipSuccess) r = launch_prepare_b(dpm, nm, nmax, cplx, st);
        // the refinement's summary and maxima start at zero (also when nothing is refined)
        if (r == hipSuccess && refine) r = launch_fill_int((int *)(D + L.sum), (int64_t)(sum_bytes(nm) / 4), 0, st);
        if (r == hipSuccess && refine) r = launch_fill_int((int *)maxes, 6 * nm, 0, st);
        return r;
    }));
    HIPCHK(timed(st, PK_DIAG, fl.diag, [&] { return launch_diag_b(dpm, ddt, (int)ndiag, cplx, st); }));
    if (nph + nps == 0)
        return refine && finish ? refine_finish(items, opts, dev_ws, host_ws, st) : SIGNTRI_OK;

    if (!mixed) {
        HIPCHK(clear_flags(0));
        HIPCHK((run_flow_any<double, FLOW_MAIN>(cplx, df64, dtk, nph, ctrl, flags, PK_FLOW, fl.flow, wgs, st)));
        HIPCHK((run_flow_any<double, FLOW_SYL>(cplx, df64, dtk_ps, nps, ctrl, flags, PK_SYL, fl.syl, wgs, st)));
        return SIGNTRI_OK;
    }

    // ---- reduced precision: FP32 copies, U0 by the FP32 sweeps, widened into U
    RefArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.mats = drm;
    ra.nmat = nm;
    HIPCHK(timed(st, PK_AUX, 0.0, [&] { return launch_fill_int((int *)maxes, 6 * nm, 0, st); }));
    HIPCHK(timed(st, PK_CONVERT, 0.0, [&] { return launch_to_f32(ra, nmax, cplx, st); }));
    HIPCHK(clear_flags(0));
    HIPCHK((run_flow_any<float, FLOW_MAIN>(cplx, df32, dtk, nph, ctrl, flags, PK_FLOW, fl.flow, wgs, st)));
    HIPCHK((run_flow_any<float, FLOW_SYL>(cplx, df32, dtk_ps, nps, ctrl, flags, PK_SYL, fl.syl, wgs, st)));
    HIPCHK(timed(st, PK_CONVERT, 0.0, [&] { return launch_widen(ra, nmax, cplx, st); }));
    if (!refine) return SIGNTRI_OK;

    double *norms[2] = {(double *)(D + L.norms0), (double *)(D + L.norms1)};
    auto resid = [&](const RefArgs &rg, double *norm2) -> hipError_t {
        return timed(st, PK_RESID, fl.resid, [&] {
            hipError_t r = cplx ? launch_resid(rg, false, cplx, dtk, (int)nph, norm2, st)
                                : launch_resid128(rg, drt, (int)nrt, norm2, st);
            // equal signs on the tiles, then the strips add the differing ones
            if (r == hipSuccess) r = launch_resid128(rg, drt + nrt, (int)nrty, norm2, st, true);
            if (r == hipSuccess)
                r = launch_resid_strips(rg, dst, (int)nstr, dminl, dgr, (int)ngr, nmax, dgbuf, norm2, st);
            if (r == hipSuccess) r = launch_resid(rg, true, cplx, dtk_ps, (int)nps, norm2, st);
            return r;
        });
    };

    // ---- refinement steps, every decision taken on the device: nothing below waits
    // for the host, so the batched form captures the whole of it in its graph.
    // live[k - 1] != 0: step k runs (live[0] = 1; step k sets live[k] when some
    // block is neither converged nor stalled); the kernels of a step that is not
    // needed return at once.
    const int max_steps = refine_step_count(opts);
    const double stall = (opts && opts->stall_ratio > 0) ? opts->stall_ratio : 0.5;
    const double conv = 1e-5;  // residual reduction that counts as converged
    const int64_t force = opts ? opts->force_stall : 0;
    double *rinit = (double *)(D + L.rinit);
    int8_t *okf = (int8_t *)(D + L.okf), *hop = (int8_t *)(D + L.hop);
    int *sum = (int *)(D + L.sum);
    int *live = sum, *cnt = sum + kMaxRefineSteps + 1;
    int64_t *nfb = (int64_t *)((char *)sum + al(kSumInts * sizeof(int)));
    HIPCHK(timed(st, PK_AUX, 0.0, [&] {
        hipError_t r = launch_fill_int(live, kMaxRefineSteps + 1, 0, st);
        if (r == hipSuccess) r = launch_fill_int(live, 1, 1, st);
        // converged and stalled flags (bytes), cleared as whole words
        if (r == hipSuccess) r = launch_fill_int((int *)okf, (int64_t)((L.rowmin - L.okf) / 4), 0, st);
        return r;
    }));
    HIPCHK(resid(ra, norms[0]));
    int cur = 0;
    for (int step = 1; step <= max_steps; ++step) {
        RefArgs rs = ra;
        rs.live = live + step - 1;
        // correction E (FP32): the residual in E32 on entry, E on exit
        HIPCHK(clear_flags(0));
        HIPCHK((run_flow_any<float, FLOW_CORR>(cplx, dfc, dtk, nph, ctrl, flags, PK_CORR, fl.corr, wgs,
                                               st, rs.live)));
        HIPCHK((run_flow_any<float, FLOW_SYL>(cplx, dfc, dtk_ps, nps, ctrl, flags, PK_CORR, fl.syl, wgs,
                                              st, rs.live)));
        HIPCHK(timed(st, PK_CONVERT, 0.0, [&] { return launch_add_correction(rs, nmax, cplx, st); }));
        HIPCHK(resid(rs, norms[cur ^ 1]));
        DecideArgs da;
        da.mats = drm;
        da.tasks = dtk;
        da.ntasks = (int)(nph + nps);
        da.prev = norms[cur];
        da.cur = norms[cur ^ 1];
        da.rinit = rinit;
        da.ok = okf;
        da.hopeless = hop;
        da.live_in = live + step - 1;
        da.live_out = live + step;
        da.step = step;
        da.nmat = nm;
        da.stall = stall;
        da.conv = conv;
        da.force = force;
        HIPCHK(timed(st, PK_AUX, 0.0, [&] { return launch_refine_decide(da, st); }));
        cur ^= 1;
    }

    // ---- FP64 recomputation of the blocks that did not converge and of every
    // block whose products read them.  In both forms block (I, J) is read by the
    // blocks (I', J') with I' <= I and J' >= J (Parlett-Higham: U_IK U_KJ with
    // K = I or J; Sylvester: A_I'K X_KJ with K = I, X_IK B_KJ' with K = J), so a
    // block is recomputed iff some block (I', J') with I' >= I and J' <= J did not
    // converge.  The task lists are built on the device, in dependency order.
    int2 *dft = (int2 *)(D + L.ftasks);
    ConeArgs ca;
    ca.mats = drm;
    ca.tasks = dtk;
    ca.nph = (int)nph;
    ca.nps = (int)nps;
    ca.ok = okf;
    ca.rowmin = (int *)(D + L.rowmin);
    ca.out_ph = dft;
    ca.out_ps = dft + nph;
    ca.cnt = cnt;
    ca.nfb = nfb;
    HIPCHK(timed(st, PK_AUX, 0.0, [&] { return launch_refine_cone(ca, nm, L.nrows, st); }));
    if (!(opts && opts->no_fallback)) {
        HIPCHK(clear_flags(1));
        HIPCHK(timed(st, PK_AUX, 0.0, [&] {
            hipError_t r = launch_clear_task_flags(dft, nph, cnt, df64, flags, st);
            if (r == hipSuccess) r = launch_clear_task_flags(dft + nph, nps, cnt + 1, df64, flags, st);
            return r;
        }));
        HIPCHK((run_flow_any<double, FLOW_MAIN>(cplx, df64, dft, nph, ctrl, flags, PK_FLOW, 0.0, wgs, st,
                                                nullptr, cnt)));
        HIPCHK((run_flow_any<double, FLOW_SYL>(cplx, df64, dft + nph, nps, ctrl, flags, PK_SYL, 0.0,
                                               wgs, st, nullptr, cnt + 1)));
    }
#undef HIPCHK
    return finish ? refine_finish(items, opts, dev_ws, host_ws, st) : SIGNTRI_OK;
}

int refine_finish(std::vector<RealItem> &items, const signtri_options *opts, void *dev_ws,
                  void *host_ws, hipStream_t st)
{
    const int nm = (int)items.size();
    if (nm == 0) return SIGNTRI_OK;
    const bool cplx = items[0].cplx;
    std::vector<int64_t> ns(nm);
    for (int m = 0; m < nm; ++m) ns[m] = items[m].n;
    const Lay L = make_lay(ns.data(), nm, true, cplx);
    char *D = (char *)dev_ws, *H = (char *)host_ws;
    int *herr = (int *)(H + L.h_err);
    int *hsum = (int *)(H + L.h_sum);
    unsigned long long *hm = (unsigned long long *)(H + L.h_maxes);
    if (hipMemcpyAsync(herr, D + L.ctrl, 2 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(hsum, D + L.sum, sum_bytes(nm), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(hm, D + L.maxes, 3 * nm * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                       st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return SIGNTRI_EHIP;
    // steps run: live[k - 1] != 0 for k = 1 .. steps
    const int max_steps = refine_step_count(opts);
    int steps = 0;
    while (steps < max_steps && hsum[steps] != 0) ++steps;
    const int *hcnt = hsum + kMaxRefineSteps + 1;
    const int64_t *hnfb = (const int64_t *)((char *)hsum + al(kSumInts * sizeof(int)));
    for (int m = 0; m < nm; ++m) {
        if (!items[m].info) continue;
        double umax, emax;
        std::memcpy(&umax, &hm[3 * m + 1], 8);
        std::memcpy(&emax, &hm[3 * m + 2], 8);
        const bool triv = items[m].path == SIGNTRI_PATH_TRIVIAL;
        items[m].info->refine_steps = triv ? 0 : steps;
        items[m].info->correction_rel = triv ? 0.0 : (umax > 0 ? emax / umax : emax);
        items[m].info->fallback_tiles = hnfb[m];
    }
    if (herr[1]) return SIGNTRI_EHIP;
    if (opts && opts->no_fallback && hcnt[0] + hcnt[1] > 0) return SIGNTRI_ENOCONV;
    return SIGNTRI_OK;
}

}  // namespace sgt
