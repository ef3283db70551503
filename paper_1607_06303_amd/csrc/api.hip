// C-ABI entry points: argument checks, workspace, planning and dispatch.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

using namespace sgt;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t scan = 0, sgn = 0, dg = 0, flow = 0, tcopy = 0, ucopy = 0;
    size_t zbuf = 0, zbufs[2] = {0, 0}, ebuf = 0, total = 0;
    int64_t zslots = 0;
    bool flow_path = false;  // real, 32 x 32 blocks: the dataflow sweeps
};

// Real matrices run the dataflow sweeps (32 x 32 blocks) unless the two-stream
// 64 x 64 sweep is requested; complex matrices run the superdiagonal sweep.
bool uses_flow(signtri_dtype dtype, int tb) { return dtype == SIGNTRI_R64 && tb == 32; }

Layout layout_for(int64_t n, signtri_dtype dtype, signtri_layout layout, signtri_mode mode,
                  signtri_algo algo, int tb)
{
    (void)algo;
    const bool cplx = dtype == SIGNTRI_C128;
    const size_t es = cplx ? 16 : 8;
    Layout L;
    size_t off = 0;
    L.scan = off;
    off += align_up(sizeof(ScanResult));
    L.sgn = off;
    off += align_up((size_t)std::max<int64_t>(n, 1));
    L.dg = off;
    off += align_up((size_t)std::max<int64_t>(n, 1) * sizeof(double));
    L.flow_path = uses_flow(dtype, tb);
    if (L.flow_path) {
        size_t fb = 0;
        (void)flow_ws_layout(nullptr, n, mode != SIGNTRI_FP64, &fb);
        L.flow = off;
        off += align_up(fb);
    } else {
        L.zslots = ph_zslots(n, tb);
        L.zbuf = off;
        off += align_up((size_t)L.zslots * tb * tb * es);
        if (!cplx) {
            static_assert(kLookahead - 1 <= 2, "bulk buffer count");
            for (int b = 0; b < kLookahead - 1; ++b) {
                L.zbufs[b] = off;
                off += align_up((size_t)L.zslots * tb * tb * es);
            }
            L.ebuf = off;
            off += align_up((size_t)ph_real_edge_slots(n, tb) * tb * tb * es);
        }
    }
    if (layout == SIGNTRI_ROW_MAJOR) {
        // column-major copies of T and U (leading dimension n)
        const size_t mat = (size_t)std::max<int64_t>(n, 1) * std::max<int64_t>(n, 1) * es;
        L.tcopy = off;
        off += align_up(mat);
        L.ucopy = off;
        off += align_up(mat);
    }
    L.total = off;
    return L;
}

// Workspace valid for every block size the call may choose.
size_t max_total(int64_t n, signtri_dtype dtype, signtri_layout layout, signtri_mode mode,
                 signtri_algo algo)
{
    size_t m = layout_for(n, dtype, layout, mode, algo, 32).total;
    if (dtype == SIGNTRI_R64 && mode == SIGNTRI_FP64)
        m = std::max(m, layout_for(n, dtype, layout, mode, algo, 64).total);
    return m;
}

// Library-owned device workspace and pinned host staging, grown on demand.
struct Owned {
    std::mutex mu;
    std::vector<std::pair<void *, size_t>> dev;  // per device id
    void *host = nullptr;
    size_t host_bytes = 0;
};
Owned &owned()
{
    static Owned o;
    return o;
}

int owned_workspace(size_t bytes, void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SIGNTRI_EHIP;
    Owned &o = owned();
    std::lock_guard<std::mutex> g(o.mu);
    if ((int)o.dev.size() <= dev) o.dev.resize(dev + 1, {nullptr, 0});
    auto &slot = o.dev[dev];
    if (slot.second < bytes) {
        if (slot.first) {
            if (hipDeviceSynchronize() != hipSuccess) return SIGNTRI_EHIP;
            (void)hipFree(slot.first);
            slot = {nullptr, 0};
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return SIGNTRI_ENOMEM;
        slot = {p, bytes};
    }
    *out = slot.first;
    return SIGNTRI_OK;
}

int owned_host(size_t bytes, void **out)
{
    Owned &o = owned();
    std::lock_guard<std::mutex> g(o.mu);
    if (o.host_bytes < bytes) {
        if (o.host) (void)hipHostFree(o.host);
        o.host = nullptr;
        o.host_bytes = 0;
        void *p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return SIGNTRI_ENOMEM;
        o.host = p;
        o.host_bytes = bytes;
    }
    *out = o.host;
    return SIGNTRI_OK;
}

bool ranges_overlap(const void *a, size_t an, const void *b, size_t bn)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + bn && pb < pa + an;
}

size_t extent_bytes(int64_t n, int64_t ld, size_t es)
{
    if (n <= 0) return 0;
    return ((size_t)(n - 1) * (size_t)ld + (size_t)n) * es;
}

// Captured launch sequences of the blocked sweep.  Every launch shape depends
// only on the arguments in the key (the kernels read the signs from device
// memory), so one graph serves every T of that shape.  Capture runs on a
// library-owned stream; the graph is then launched on the caller's stream.
struct GraphKey {
    const void *T;
    int64_t ldt;
    void *U;
    int64_t ldu;
    int64_t n;
    int dtype, tile, max_splits, device;
    void *ws;
    bool operator==(const GraphKey &o) const
    {
        return T == o.T && ldt == o.ldt && U == o.U && ldu == o.ldu && n == o.n &&
               dtype == o.dtype && tile == o.tile && max_splits == o.max_splits &&
               device == o.device && ws == o.ws;
    }
};
struct GraphCache {
    std::mutex mu;
    std::vector<std::pair<GraphKey, hipGraphExec_t>> entries;  // most recent last
    std::vector<hipStream_t> capture_streams;                 // per device
};
GraphCache &graphs()
{
    static GraphCache g;
    return g;
}
constexpr size_t kGraphCacheSize = 8;

bool graphs_enabled()
{
    const char *v = getenv("SIGNTRI_NO_GRAPH");
    return !(v && *v && *v != '0');
}

// Launch the sweep described by `a` on `st`, through a cached graph when possible.
hipError_t launch_ph(const PhArgs &a, bool cplx, hipStream_t st, int device)
{
    if (!graphs_enabled() || prof_on()) return run_ph_fp64(a, cplx, st);
    GraphKey key{a.T, a.ldt, a.U, a.ldu, a.n, cplx ? 1 : 0, a.tile, a.max_splits, device,
                 a.zbuf};
    GraphCache &g = graphs();
    std::lock_guard<std::mutex> lk(g.mu);
    for (size_t k = 0; k < g.entries.size(); ++k)
        if (g.entries[k].first == key) {
            auto hit = g.entries[k];
            g.entries.erase(g.entries.begin() + k);
            g.entries.push_back(hit);
            return hipGraphLaunch(hit.second, st);
        }
    if ((int)g.capture_streams.size() <= device) g.capture_streams.resize(device + 1, nullptr);
    hipStream_t &cs = g.capture_streams[device];
    hipError_t e;
    if (!cs && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
    hipError_t run = run_ph_fp64(a, cplx, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (run != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return run;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    if (g.entries.size() >= kGraphCacheSize) {
        (void)hipGraphExecDestroy(g.entries.front().second);
        g.entries.erase(g.entries.begin());
    }
    g.entries.push_back({key, exec});
    return hipGraphLaunch(exec, st);
}

// Algorithmic flops of the dataflow launches (Section 3 counting, real).
SweepFlops sweep_flops(const int8_t *s, int64_t n, const HostPlan &p)
{
    SweepFlops f;
    const FlopCounter fc{s, n, kFlowTile, 1.0};
    f.diag = fc.diag();
    f.flow = p.w_ph - f.diag;
    const double dn = (double)n, np = (double)p.n_pos, nn = (double)p.n_neg;
    // correction sweep: two products (4 flops) per k strictly between i and j,
    // off the diagonal blocks
    double cdiag = 0.0;
    for (int64_t r0 = 0; r0 < n; r0 += kFlowTile) {
        const double b = (double)std::min<int64_t>(kFlowTile, n - r0);
        cdiag += b * (b - 1) * (b - 2) / 6.0;
    }
    f.corr = 4.0 * (dn * (dn - 1) * (dn - 2) / 6.0 - cdiag);
    // residual: k = i .. j, i.e. two more terms per entry than the sweep
    f.resid = f.flow + 2.0 * (2.0 * dn * (dn - 1) / 2.0 + 2.0 * np * nn);
    // Sylvester: (p - 1 - i) + (j - p) multiply-adds per entry of X
    f.syl = np * nn * (dn - 2.0);
    return f;
}

void fill_info(signtri_info *info, const HostPlan &p)
{
    if (!info) return;
    info->model_pick = p.model_pick;
    info->n_pos = p.n_pos;
    info->n_neg = p.n_neg;
    info->swaps = std::min(p.swaps_pos_first, p.swaps_neg_first);
    info->w_ph = p.w_ph;
    info->w_ps = p.w_ps;
}

}  // namespace

extern "C" {

const char *signtri_strerror(int code)
{
    switch (code) {
    case SIGNTRI_OK: return "success";
    case SIGNTRI_EDOMAIN:
        return "sign(T) is undefined: a diagonal entry has a zero real part or is not finite";
    case SIGNTRI_EHIP: return "a HIP runtime call failed";
    case SIGNTRI_EWORKSPACE: return "workspace smaller than signtri_workspace_size()";
    case SIGNTRI_ENOCONV: return "iterative refinement did not converge and fallback is disabled";
    case SIGNTRI_ENOTSUP: return "this combination of arguments is not implemented";
    case SIGNTRI_ENOMEM: return "the library could not allocate its workspace";
    default: break;
    }
    if (code < 0) return "invalid argument";
    return "unknown error code";
}

size_t signtri_workspace_size(int64_t n, signtri_dtype dtype, signtri_layout layout,
                              signtri_mode mode, signtri_algo algo)
{
    if (n < 0) return 0;
    if (dtype != SIGNTRI_R64 && dtype != SIGNTRI_C128) return 0;
    if (layout != SIGNTRI_COL_MAJOR && layout != SIGNTRI_ROW_MAJOR) return 0;
    if (mode < SIGNTRI_FP64 || mode > SIGNTRI_FP32) return 0;
    if (algo < SIGNTRI_AUTO || algo > SIGNTRI_PS) return 0;
    return max_total(n, dtype, layout, mode, algo);
}

int signtri_plan_host(const int8_t *s, int64_t n, signtri_dtype dtype, signtri_info *info)
{
    if (n < 0 || (n > 0 && !s) || !info) return -1;
    if (dtype != SIGNTRI_R64 && dtype != SIGNTRI_C128) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (s[i] != 1 && s[i] != -1) return -1;
    std::memset(info, 0, sizeof(*info));
    HostPlan p = plan_from_signs(s, n, dtype == SIGNTRI_C128);
    fill_info(info, p);
    info->path = n == 0 ? SIGNTRI_PATH_TRIVIAL : p.auto_path;
    return 0;
}

int signtri(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n, signtri_dtype dtype,
            signtri_layout layout, signtri_mode mode, signtri_algo algo, void *workspace,
            size_t ws_bytes, void *stream, const signtri_options *opts, signtri_info *info)
{
    if (info) std::memset(info, 0, sizeof(*info));
    // argument checks, in argument order (LAPACK style -p)
    if (n > 0 && !T) return -1;
    if (ldt < std::max<int64_t>(1, n)) return -2;
    if (n > 0 && !U) return -3;
    if (ldu < std::max<int64_t>(1, n)) return -4;
    if (n < 0) return -5;
    if (dtype != SIGNTRI_R64 && dtype != SIGNTRI_C128) return -6;
    if (layout != SIGNTRI_COL_MAJOR && layout != SIGNTRI_ROW_MAJOR) return -7;
    if (mode < SIGNTRI_FP64 || mode > SIGNTRI_FP32) return -8;
    if (algo < SIGNTRI_AUTO || algo > SIGNTRI_PS) return -9;
    if (workspace && ws_bytes == 0) return -11;
    const bool cplx = dtype == SIGNTRI_C128;
    const size_t es = cplx ? 16 : 8;
    if (n > 0 && ranges_overlap(T, extent_bytes(n, ldt, es), U, extent_bytes(n, ldu, es))) return -3;
    if (opts && opts->tile != 0 && opts->tile != 32 && opts->tile != 64) return -13;
    if (n == 0) return SIGNTRI_OK;
    if (cplx && mode != SIGNTRI_FP64) return SIGNTRI_ENOTSUP;

    int tb = ph_tile_size(cplx, opts ? opts->tile : 0);
    if (mode != SIGNTRI_FP64) tb = 32;  // reduced precision runs on the dataflow sweeps
    const Layout L = layout_for(n, dtype, layout, mode, algo, tb);
    const size_t need = max_total(n, dtype, layout, mode, algo);
    if (workspace) {
        if (ws_bytes < need) return SIGNTRI_EWORKSPACE;
    } else {
        int rc = owned_workspace(need, &workspace);
        if (rc != SIGNTRI_OK) return rc;
    }
    void *hostbuf = nullptr;
    const size_t host_bytes = align_up(sizeof(ScanResult)) + align_up((size_t)n) +
                              (L.flow_path ? flow_host_bytes(n) : 0);
    if (int rc = owned_host(host_bytes, &hostbuf)) return rc;
    char *hb = (char *)hostbuf;
    void *hflow = hb + align_up(sizeof(ScanResult)) + align_up((size_t)n);

    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    ScanResult *scan = (ScanResult *)(ws + L.scan);
    int8_t *sgn = (int8_t *)(ws + L.sgn);
    double *dg = (double *)(ws + L.dg);

    // row-major arguments run on column-major copies
    const void *Tc = T;
    void *Uc = U;
    int64_t ldtc = ldt, lduc = ldu;
    if (layout == SIGNTRI_ROW_MAJOR) {
        Tc = ws + L.tcopy;
        Uc = ws + L.ucopy;
        ldtc = lduc = n;
        if (launch_transpose(T, ldt, (void *)Tc, n, n, cplx, st) != hipSuccess) return SIGNTRI_EHIP;
    }

    if (launch_scan(Tc, ldtc, n, cplx, sgn, cplx ? nullptr : dg, scan, st) != hipSuccess)
        return SIGNTRI_EHIP;
    // scan result and signs are adjacent in the workspace: one copy
    if (hipMemcpyAsync(hb, ws + L.scan, L.sgn - L.scan + (size_t)n, hipMemcpyDeviceToHost, st) !=
        hipSuccess)
        return SIGNTRI_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SIGNTRI_EHIP;
    ScanResult sr;
    std::memcpy(&sr, hb, sizeof(sr));
    const int8_t *hs = (const int8_t *)(hb + (L.sgn - L.scan));
    if (sr.bad_index < n) {
        if (info) info->bad_index = sr.bad_index + 1;
        return SIGNTRI_EDOMAIN;
    }
    HostPlan p = plan_from_signs(hs, n, cplx);
    fill_info(info, p);

    int path = p.auto_path;
    if (algo == SIGNTRI_PH && path != SIGNTRI_PATH_TRIVIAL) path = SIGNTRI_PATH_PH;
    if (algo == SIGNTRI_PS && path != SIGNTRI_PATH_TRIVIAL) {
        if (p.ps_sign == 0) return SIGNTRI_ENOTSUP;
        path = SIGNTRI_PATH_PS;
    }
    if (path == SIGNTRI_PATH_PS && !L.flow_path) {
        if (algo == SIGNTRI_PS) return SIGNTRI_ENOTSUP;
        path = SIGNTRI_PATH_PH;  // the Sylvester form runs on the real dataflow sweeps
    }

    int rc = SIGNTRI_OK;
    hipError_t e = hipSuccess;
    bool waited = false;
    FlowWs fw{};
    if (L.flow_path) fw = flow_ws_layout(ws + L.flow, n, mode != SIGNTRI_FP64, nullptr);
    if (path == SIGNTRI_PATH_TRIVIAL) {
        e = launch_fill_pm_identity(Uc, lduc, n, cplx, p.n_pos > 0 ? 1.0 : -1.0, st);
    } else if (L.flow_path) {
        const double *Td = (const double *)Tc;
        double *Ud = (double *)Uc;
        const int64_t split = path == SIGNTRI_PATH_PS ? p.split : 0;
        const SweepFlops fl = prof_on() ? sweep_flops(hs, n, p) : SweepFlops();
        if (mode == SIGNTRI_FP64) {
            if (path == SIGNTRI_PATH_PS)
                e = sweep_ps_fp64(Td, ldtc, Ud, lduc, n, split, p.ps_sign, dg, fw, fl, st);
            else
                e = sweep_ph_fp64(Td, ldtc, Ud, lduc, n, sgn, dg, fw, fl, st);
        } else {
            rc = sweep_mixed(Td, ldtc, Ud, lduc, n, sgn, dg, split, p.ps_sign,
                             mode == SIGNTRI_MIXED_REFINED, opts, fw, hflow, fl, st, info);
            waited = mode == SIGNTRI_MIXED_REFINED;
        }
    } else {
        PhArgs a;
        a.T = Tc;
        a.ldt = ldtc;
        a.U = Uc;
        a.ldu = lduc;
        a.n = n;
        a.sgn = sgn;
        a.zbuf = ws + L.zbuf;
        a.zbufs[0] = ws + L.zbufs[0];
        a.zbufs[1] = ws + L.zbufs[1];
        a.ebuf = ws + L.ebuf;
        a.zslots = L.zslots;
        a.hsgn = hs;
        a.max_splits = opts ? opts->max_splits : 0;
        a.tile = tb;
        int device = 0;
        if (hipGetDevice(&device) != hipSuccess) return SIGNTRI_EHIP;
        e = launch_ph(a, cplx, st, device);
    }
    if (e != hipSuccess) return SIGNTRI_EHIP;
    if (rc != SIGNTRI_OK) return rc;
    if (layout == SIGNTRI_ROW_MAJOR && launch_transpose(Uc, lduc, U, ldu, n, cplx, st) != hipSuccess)
        return SIGNTRI_EHIP;
    // with info requested, wait and report a dependency-wait timeout of the sweep
    if (info && L.flow_path && path != SIGNTRI_PATH_TRIVIAL && !waited) {
        int *herr = (int *)hflow;
        if (hipMemcpyAsync(herr, fw.ctrl, 2 * sizeof(int), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SIGNTRI_EHIP;
        if (herr[1]) return SIGNTRI_EHIP;
    }
    if (info) {
        info->path = path;
        info->tile = path == SIGNTRI_PATH_TRIVIAL ? 0 : tb;
    }
    return SIGNTRI_OK;
}

int sign_tri(const void *T, int64_t n, int64_t ld, signtri_dtype dtype, void *U)
{
    int rc = signtri(T, ld, U, ld, n, dtype, SIGNTRI_COL_MAJOR, SIGNTRI_FP64, SIGNTRI_AUTO, nullptr,
                     0, nullptr, nullptr, nullptr);
    if (rc != SIGNTRI_OK) return rc;
    return hipStreamSynchronize(nullptr) == hipSuccess ? SIGNTRI_OK : SIGNTRI_EHIP;
}

size_t signtri_batched_workspace_size(const int64_t *n, int64_t batch, signtri_dtype dtype,
                                      signtri_mode mode)
{
    if (batch < 0 || (batch > 0 && !n)) return 0;
    size_t m = 0;
    for (int64_t b = 0; b < batch; ++b) {
        if (n[b] < 0) return 0;
        m = std::max(m, signtri_workspace_size(n[b], dtype, SIGNTRI_COL_MAJOR, mode, SIGNTRI_AUTO));
    }
    return m;
}

int signtri_batched(const void *const *T, const int64_t *ldt, void *const *U, const int64_t *ldu,
                    const int64_t *n, int64_t batch, signtri_dtype dtype, signtri_layout layout,
                    signtri_mode mode, void *workspace, size_t ws_bytes, void *stream,
                    const signtri_options *opts, signtri_info *infos)
{
    if (batch > 0 && !T) return -1;
    if (batch > 0 && !ldt) return -2;
    if (batch > 0 && !U) return -3;
    if (batch > 0 && !ldu) return -4;
    if (batch > 0 && !n) return -5;
    if (batch < 0) return -6;
    for (int64_t b = 0; b < batch; ++b) {
        int rc = signtri(T[b], ldt[b], U[b], ldu[b], n[b], dtype, layout, mode, SIGNTRI_AUTO,
                         workspace, ws_bytes, stream, opts, infos ? infos + b : nullptr);
        if (rc != SIGNTRI_OK) return rc;
    }
    return SIGNTRI_OK;
}

void signtri_release(void)
{
    Owned &o = owned();
    std::lock_guard<std::mutex> g(o.mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (size_t d = 0; d < o.dev.size(); ++d) {
        if (o.dev[d].first) {
            (void)hipSetDevice((int)d);
            (void)hipDeviceSynchronize();
            (void)hipFree(o.dev[d].first);
        }
        o.dev[d] = {nullptr, 0};
    }
    (void)hipSetDevice(cur);
    if (o.host) (void)hipHostFree(o.host);
    o.host = nullptr;
    o.host_bytes = 0;
    GraphCache &gc = graphs();
    std::lock_guard<std::mutex> lk(gc.mu);
    for (auto &kv : gc.entries) (void)hipGraphExecDestroy(kv.second);
    gc.entries.clear();
}

}  // extern "C"
