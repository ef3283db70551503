// C-ABI entry points: argument checks, workspace, planning and dispatch.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"
#include "signm.h"

using namespace sgt;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t scan = 0, sgn = 0, dg = 0, flow = 0, tcopy = 0, ucopy = 0, prefix = 0;
    size_t zbuf = 0, zbufs[2] = {0, 0}, ebuf = 0, total = 0;
    int64_t zslots = 0;
    bool flow_path = false;  // the dataflow sweeps (32 x 32 blocks)
};

// Workspace layout of one call.  The prefix (scan result, signs, diagonal, the
// column-major copies of row-major arguments) does not depend on the sweep, so
// it can be used before the sweep is chosen.
Layout layout_for(int64_t n, signtri_dtype dtype, signtri_layout layout, signtri_mode mode,
                  int tb, bool flow)
{
    const bool cplx = dtype == SIGNTRI_C128;
    const size_t es = cplx ? 16 : 8;
    Layout L;
    size_t off = 0;
    L.scan = off;
    off += align_up(sizeof(ScanResult));
    L.sgn = off;
    off += align_up((size_t)std::max<int64_t>(n, 1));
    L.dg = off;
    off += align_up((size_t)std::max<int64_t>(n, 1) * sizeof(double) * (cplx ? 2 : 1));
    if (layout == SIGNTRI_ROW_MAJOR) {
        // column-major copies of T and U (leading dimension n)
        const size_t mat = (size_t)std::max<int64_t>(n, 1) * std::max<int64_t>(n, 1) * es;
        L.tcopy = off;
        off += align_up(mat);
        L.ucopy = off;
        off += align_up(mat);
    }
    L.prefix = off;
    L.flow_path = flow;
    if (flow) {
        size_t fb = 0;
        run_sizes(&n, 1, mode != SIGNTRI_FP64, cplx, &fb, nullptr);
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
    L.total = off;
    return L;
}

// Workspace valid for every sweep and block size the call may choose.
size_t max_total(int64_t n, signtri_dtype dtype, signtri_layout layout, signtri_mode mode,
                 signtri_algo algo)
{
    size_t m = layout_for(n, dtype, layout, mode, 32, true).total;
    if (mode == SIGNTRI_FP64) {
        m = std::max(m, layout_for(n, dtype, layout, mode, 32, false).total);
        if (dtype == SIGNTRI_R64) m = std::max(m, layout_for(n, dtype, layout, mode, 64, false).total);
    }
    if (algo == SIGNTRI_AUTO || algo == SIGNTRI_PROJ) {
        // the projector form for any minority count it takes (at most n / 2)
        const int mub = (int)std::min<int64_t>(n / 2, kProjMaxMinorityReal);
        m = std::max(m, layout_for(n, dtype, layout, mode, 32, true).prefix +
                            align_up(proj_workspace_bytes(n, mub, dtype == SIGNTRI_C128)));
    }
    return m;
}

// Option checks that do not depend on T: -13 for values out of range,
// SIGNTRI_ENOTSUP for combinations no sweep implements.
int check_options(const signtri_options *o, signtri_dtype dtype, signtri_mode mode)
{
    if (!o) return SIGNTRI_OK;
    if (o->tile != 0 && o->tile != 32 && o->tile != 64) return -13;
    if (o->sweep < SIGNTRI_SWEEP_AUTO || o->sweep > SIGNTRI_SWEEP_SUPERDIAG) return -13;
    if (o->wgs_per_cu < 0) return -13;
    if (o->max_refine_steps > kMaxRefineSteps) return -13;
    if (o->products != SIGNTRI_PRODUCTS_MASKED && o->products != SIGNTRI_PRODUCTS_DENSE) return -13;
    const bool cplx = dtype == SIGNTRI_C128;
    if (cplx && o->tile == 64) return SIGNTRI_ENOTSUP;
    if (mode != SIGNTRI_FP64 && (o->sweep == SIGNTRI_SWEEP_SUPERDIAG || o->tile == 64))
        return SIGNTRI_ENOTSUP;
    if (o->sweep == SIGNTRI_SWEEP_DATAFLOW && o->tile == 64) return SIGNTRI_ENOTSUP;
    return SIGNTRI_OK;
}

// Fill the options left at 0 from the tuning table, then from the defaults.
signtri_options resolve_options(const signtri_options *opts, signtri_dtype dtype,
                                signtri_mode mode, int path, int64_t n)
{
    signtri_options o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    signtri_tune_entry te;
    if ((o.sweep == 0 || o.wgs_per_cu == 0) && path != SIGNTRI_PATH_TRIVIAL &&
        tune_find(dtype, mode, path, n, &te)) {
        // a recorded block size belongs to its sweep: take both or neither
        if (o.sweep == 0 && (o.tile == 0 || o.tile == te.tile)) {
            o.sweep = te.sweep;
            o.tile = te.tile;
        }
        if (o.wgs_per_cu == 0 && o.sweep == SIGNTRI_SWEEP_DATAFLOW) o.wgs_per_cu = te.wgs_per_cu;
    }
    if (o.sweep == 0) o.sweep = o.tile == 64 ? SIGNTRI_SWEEP_SUPERDIAG : SIGNTRI_SWEEP_DATAFLOW;
    if (o.tile == 0) o.tile = 32;
    if (o.sweep == SIGNTRI_SWEEP_DATAFLOW) {
        const bool f32 = mode != SIGNTRI_FP64, cx = dtype == SIGNTRI_C128;
        const int mx = flow_max_wgs_per_cu(f32, cx);
        if (o.wgs_per_cu <= 0) o.wgs_per_cu = flow_default_wgs_per_cu(f32, cx);
        if (o.wgs_per_cu > mx) o.wgs_per_cu = mx;
    } else {
        o.wgs_per_cu = 0;
    }
    return o;
}

// Bumped whenever the library-owned workspace moves; part of every graph key.
std::atomic<uint64_t> &ws_generation()
{
    static std::atomic<uint64_t> g{0};
    return g;
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
        // testing hook: SIGNTRI_DEBUG_FAIL_ALLOC=1 makes every allocation of the
        // library-owned workspace fail, as hipMalloc does when memory runs out
        const char *fail = getenv("SIGNTRI_DEBUG_FAIL_ALLOC");
        if (fail && *fail && *fail != '0') return SIGNTRI_ENOMEM;
        if (slot.first) {
            if (hipDeviceSynchronize() != hipSuccess) return SIGNTRI_EHIP;
            (void)hipFree(slot.first);
            slot = {nullptr, 0};
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return SIGNTRI_ENOMEM;
        slot = {p, bytes};
        ws_generation().fetch_add(1);  // graphs captured on the old buffer are stale
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
    uint64_t gen;
    bool operator==(const GraphKey &o) const
    {
        return T == o.T && ldt == o.ldt && U == o.U && ldu == o.ldu && n == o.n &&
               dtype == o.dtype && tile == o.tile && max_splits == o.max_splits &&
               device == o.device && ws == o.ws && gen == o.gen;
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
    GraphKey key{a.T,    a.ldt,        a.U,    a.ldu,  a.n,
                 cplx ? 1 : 0, a.tile, a.max_splits, device, a.zbuf,
                 ws_generation().load()};
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

// Workspace of a batched call: scan table and results, per-matrix signs and
// diagonals, then the run's own region.  The host staging mirrors the scan
// part at the same offsets, then holds the run's host part.
struct BatchLayout {
    size_t scan_tab = 0, res = 0, sgn_end = 0, run = 0, dev = 0, run_host = 0, host = 0;
    std::vector<size_t> sgn, dg;
};

BatchLayout batch_layout(const int64_t *n, int64_t batch, signtri_mode mode, bool cplx)
{
    BatchLayout B;
    const int nm = (int)batch;
    size_t o = 0;
    B.scan_tab = o;
    o += align_up(nm * sizeof(ScanMat));
    B.res = o;
    o += align_up(nm * sizeof(ScanResult));
    B.sgn.resize(nm);
    B.dg.resize(nm);
    for (int m = 0; m < nm; ++m) {
        B.sgn[m] = o;
        o += (size_t)(n[m] + 7) / 8 * 8;
    }
    B.sgn_end = o;
    o = align_up(o);
    for (int m = 0; m < nm; ++m) {
        B.dg[m] = o;
        o += (size_t)n[m] * sizeof(double) * (cplx ? 2 : 1);
    }
    o = align_up(o);
    std::vector<int64_t> ns;
    for (int m = 0; m < nm; ++m)
        if (n[m] > 0) ns.push_back(n[m]);
    size_t rd = 0, rh = 0;
    run_sizes(ns.data(), (int)ns.size(), mode != SIGNTRI_FP64, cplx, &rd, &rh);
    B.run = o;
    B.dev = o + rd;
    B.run_host = align_up(B.sgn_end);
    B.host = B.run_host + rh;
    return B;
}

// Captured launch sequences of batched runs (FP64 and unrefined FP32: no host
// decision inside).  Each graph owns the pinned copy of the tables and task
// lists its upload node reads, so later calls cannot change what it replays.
struct BatchGraph {
    std::vector<int64_t> key;
    hipGraphExec_t exec = nullptr;
    void *host = nullptr;
};
std::mutex batch_graph_mu;
std::vector<BatchGraph> batch_graphs;  // most recent last
constexpr size_t kBatchGraphs = 4;
std::vector<hipStream_t> batch_capture_streams;

void drop_batch_graph(BatchGraph &g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.host) (void)hipHostFree(g.host);
    g.exec = nullptr;
    g.host = nullptr;
}

int launch_batch_graph(std::vector<RealItem> &items, signtri_mode mode,
                       const signtri_options *opts, char *run_dev, hipStream_t st, int device)
{
    const bool cplx = !items.empty() && items[0].cplx;
    std::vector<int64_t> key{(int64_t)mode, (int64_t)device, (int64_t)(intptr_t)run_dev,
                             (int64_t)ws_generation().load(), (int64_t)items.size(),
                             (int64_t)(opts ? opts->wgs_per_cu : 0), (int64_t)cplx,
                             (int64_t)flow_spin_limit(), (int64_t)(opts ? opts->products : 0)};
    if (mode == SIGNTRI_MIXED_REFINED) {
        // the refinement's options are part of what was captured
        int64_t stall_bits = 0;
        const double stall = opts ? opts->stall_ratio : 0.0;
        std::memcpy(&stall_bits, &stall, sizeof(stall_bits));
        key.insert(key.end(), {(int64_t)(opts ? opts->max_refine_steps : 0), stall_bits,
                               (int64_t)(opts ? opts->no_fallback : 0),
                               (int64_t)(opts ? opts->force_stall : 0)});
    }
    std::vector<int64_t> ns;
    for (const RealItem &it : items) {
        key.insert(key.end(), {(int64_t)(intptr_t)it.T, it.ldt, (int64_t)(intptr_t)it.U, it.ldu,
                               it.n, it.path, it.p, it.s});
        ns.push_back(it.n);
    }
    std::lock_guard<std::mutex> lk(batch_graph_mu);
    for (size_t k = 0; k < batch_graphs.size(); ++k)
        if (batch_graphs[k].key == key) {
            BatchGraph hit = batch_graphs[k];
            batch_graphs.erase(batch_graphs.begin() + k);
            batch_graphs.push_back(hit);
            return hipGraphLaunch(hit.exec, st) == hipSuccess ? SIGNTRI_OK : SIGNTRI_EHIP;
        }
    size_t host_bytes = 0;
    run_sizes(ns.data(), (int)ns.size(), mode != SIGNTRI_FP64, cplx, nullptr, &host_bytes);
    BatchGraph g;
    g.key = key;
    if (hipHostMalloc(&g.host, std::max<size_t>(host_bytes, 256), hipHostMallocDefault) !=
        hipSuccess)
        return SIGNTRI_ENOMEM;
    if ((int)batch_capture_streams.size() <= device) batch_capture_streams.resize(device + 1, nullptr);
    hipStream_t &cs = batch_capture_streams[device];
    if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        drop_batch_graph(g);
        return SIGNTRI_EHIP;
    }
    // capture on a library stream (nothing runs there); the graph then runs on st
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
        drop_batch_graph(g);
        return SIGNTRI_EHIP;
    }
    const int rc = run_real(items, mode, opts, run_dev, g.host, false, nullptr, cs, false);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (rc != SIGNTRI_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        drop_batch_graph(g);
        return rc != SIGNTRI_OK ? rc : SIGNTRI_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        drop_batch_graph(g);
        return SIGNTRI_EHIP;
    }
    if (batch_graphs.size() >= kBatchGraphs) {
        drop_batch_graph(batch_graphs.front());
        batch_graphs.erase(batch_graphs.begin());
    }
    batch_graphs.push_back(g);
    return hipGraphLaunch(g.exec, st) == hipSuccess ? SIGNTRI_OK : SIGNTRI_EHIP;
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
    case SIGNTRI_ETOOBIG:
        return "the order exceeds what the no-allocation entry point's fixed scratch holds";
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
    if (algo < SIGNTRI_AUTO || algo > SIGNTRI_PROJ) return 0;
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
    info->path = n == 0 ? SIGNTRI_PATH_TRIVIAL : (p.proj_pick ? SIGNTRI_PATH_PROJ : p.auto_path);
    return 0;
}

int signtri(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n, signtri_dtype dtype,
            signtri_layout layout, signtri_mode mode, signtri_algo algo, void *workspace,
            size_t ws_bytes, void *stream, const signtri_options *opts, signtri_info *info)
{
    return sgt::signtri_run(T, ldt, U, ldu, n, dtype, layout, mode, algo, workspace, ws_bytes,
                            stream, opts, info, nullptr);
}

}  // extern "C"

namespace sgt {

size_t noalloc_device_bytes(int64_t n, signtri_dtype dtype)
{
    const Layout F = layout_for(n, dtype, SIGNTRI_COL_MAJOR, SIGNTRI_FP64, 32, true);
    // the projector form only up to kProjMaxMinority minority entries here
    return std::max(F.total, F.prefix + align_up(proj_workspace_bytes(n, kProjMaxMinority,
                                                                      dtype == SIGNTRI_C128)));
}

size_t noalloc_host_bytes(int64_t n, signtri_dtype dtype)
{
    size_t run_host = 0;
    run_sizes(&n, 1, false, dtype == SIGNTRI_C128, nullptr, &run_host);
    return align_up(sizeof(ScanResult)) + align_up((size_t)n) + run_host;
}

int signtri_run(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n, signtri_dtype dtype,
                signtri_layout layout, signtri_mode mode, signtri_algo algo, void *workspace,
                size_t ws_bytes, void *stream, const signtri_options *opts, signtri_info *info,
                const NoAllocBuffers *na)
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
    if (algo < SIGNTRI_AUTO || algo > SIGNTRI_PROJ) return -9;
    if (workspace && ws_bytes == 0) return -11;
    const bool cplx = dtype == SIGNTRI_C128;
    const size_t es = cplx ? 16 : 8;
    if (n > 0 && ranges_overlap(T, extent_bytes(n, ldt, es), U, extent_bytes(n, ldu, es))) return -3;
    if (int rc = check_options(opts, dtype, mode)) return rc;
    if (n == 0) return SIGNTRI_OK;

    const Layout L0 = layout_for(n, dtype, layout, mode, 32, false);  // the common prefix
    void *hostbuf = nullptr;
    size_t run_host = 0;
    run_sizes(&n, 1, mode != SIGNTRI_FP64, cplx, nullptr, &run_host);
    const size_t host_bytes = align_up(sizeof(ScanResult)) + align_up((size_t)n) + run_host;
    if (na) {
        // the caller's fixed buffers: FP64, column-major, dataflow sweeps or the projector
        // form only (no captured graph, which would allocate)
        if (mode != SIGNTRI_FP64 || layout != SIGNTRI_COL_MAJOR || algo != SIGNTRI_AUTO || opts)
            return SIGNTRI_ENOTSUP;
        if (na->dev_bytes < noalloc_device_bytes(n, dtype) || na->host_bytes < host_bytes)
            return SIGNTRI_ETOOBIG;
        workspace = na->dev;
        hostbuf = na->host;
    } else {
        const size_t need = max_total(n, dtype, layout, mode, algo);
        if (workspace) {
            if (ws_bytes < need) return SIGNTRI_EWORKSPACE;
        } else {
            int rc = owned_workspace(need, &workspace);
            if (rc != SIGNTRI_OK) return rc;
        }
        if (int rc = owned_host(host_bytes, &hostbuf)) return rc;
    }
    char *hb = (char *)hostbuf;
    void *hflow = hb + align_up(sizeof(ScanResult)) + align_up((size_t)n);

    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    ScanResult *scan = (ScanResult *)(ws + L0.scan);
    int8_t *sgn = (int8_t *)(ws + L0.sgn);
    double *dg = (double *)(ws + L0.dg);

    // row-major arguments run on column-major copies
    const void *Tc = T;
    void *Uc = U;
    int64_t ldtc = ldt, lduc = ldu;
    if (layout == SIGNTRI_ROW_MAJOR) {
        Tc = ws + L0.tcopy;
        Uc = ws + L0.ucopy;
        ldtc = lduc = n;
        if (launch_transpose(T, ldt, (void *)Tc, n, n, cplx, st) != hipSuccess) return SIGNTRI_EHIP;
    }

    if (launch_scan(Tc, ldtc, n, cplx, sgn, dg, scan, st) != hipSuccess)
        return SIGNTRI_EHIP;
    // scan result and signs are adjacent in the workspace: one copy
    if (hipMemcpyAsync(hb, ws + L0.scan, L0.sgn - L0.scan + (size_t)n, hipMemcpyDeviceToHost, st) !=
        hipSuccess)
        return SIGNTRI_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SIGNTRI_EHIP;
    ScanResult sr;
    std::memcpy(&sr, hb, sizeof(sr));
    const int8_t *hs = (const int8_t *)(hb + (L0.sgn - L0.scan));
    if (sr.bad_index < n) {
        if (info) info->bad_index = sr.bad_index + 1;
        return SIGNTRI_EDOMAIN;
    }
    HostPlan p = plan_from_signs(hs, n, cplx);
    fill_info(info, p);
    double dmin = 0.0, dmax = 0.0;
    std::memcpy(&dmin, &sr.absmin, sizeof(double));
    std::memcpy(&dmax, &sr.absmax, sizeof(double));
    const bool rcp_guard = !(dmin >= 0x1p-1020 && dmax <= 0x1p1019);

    int path = p.auto_path;
    // AUTO takes the projector form in FP64 mode when no sweep or block size is pinned
    const bool pinned_sweep = opts && (opts->sweep != 0 || opts->tile != 0);
    // (with the caller's fixed buffers, up to kProjMaxMinority minority entries)
    const int mmax = cplx || na ? kProjMaxMinority : kProjMaxMinorityReal;
    if (algo == SIGNTRI_AUTO && p.proj_pick && mode == SIGNTRI_FP64 && !pinned_sweep &&
        p.n_min <= mmax && (cplx || proj_fits(n, (int)p.n_min)))
        path = SIGNTRI_PATH_PROJ;
    if (algo == SIGNTRI_PH && path != SIGNTRI_PATH_TRIVIAL) path = SIGNTRI_PATH_PH;
    if (algo == SIGNTRI_PS && path != SIGNTRI_PATH_TRIVIAL) {
        if (p.ps_sign == 0) return SIGNTRI_ENOTSUP;
        path = SIGNTRI_PATH_PS;
    }
    if (algo == SIGNTRI_PROJ && path != SIGNTRI_PATH_TRIVIAL) {
        if (p.n_min < 1 || p.n_min > mmax) return SIGNTRI_ENOTSUP;
        if (!cplx && !proj_fits(n, (int)p.n_min)) return SIGNTRI_ENOTSUP;
        path = SIGNTRI_PATH_PROJ;
    }
    if (path == SIGNTRI_PATH_PROJ) {
        // every mode: FP64 substitutions and products, no sweep options apply
        // algorithmic flops of the substitutions: column l of Z takes the rows above
        // its minority row b_l, about b_l^2 / 2 multiply-adds, and of W the rows below;
        // the L coupling adds about m^2 n / 2 per basis
        double flops = 2.0 * (double)p.n_min * (double)p.n_min * (double)n;
        for (int64_t i = 0; i < n; ++i)
            if (hs[i] == p.min_sign) {
                const double b = (double)i, f = (double)(n - 1 - i);
                flops += b * b + f * f;
            }
        const int prc = cplx ? run_proj_c(Tc, ldtc, Uc, lduc, n, sgn, hs, p.min_sign,
                                          (int)p.n_min, 4.0 * flops, ws + L0.prefix, st)
                             : run_proj((const double *)Tc, ldtc, (double *)Uc, lduc, n, sgn, hs,
                                        p.min_sign, (int)p.n_min, flops, ws + L0.prefix, st,
                                        info ? (int *)hflow : nullptr, rcp_guard);
        if (prc != SIGNTRI_OK) return prc == SIGNTRI_ENOTSUP ? SIGNTRI_ENOTSUP : SIGNTRI_EHIP;
        if (layout == SIGNTRI_ROW_MAJOR && launch_transpose(Uc, lduc, U, ldu, n, cplx, st) != hipSuccess)
            return SIGNTRI_EHIP;
        if (info) {
            info->path = path;
            info->tile = 0;
            info->sweep = 0;
            info->wgs_per_cu = 0;
        }
        return SIGNTRI_OK;
    }
    signtri_options eo = resolve_options(opts, dtype, mode, path, n);
    if (na) {
        // no captured graph: the dataflow sweep, whatever the tuning table recorded
        eo.sweep = SIGNTRI_SWEEP_DATAFLOW;
        eo.tile = 32;
        eo.wgs_per_cu = flow_default_wgs_per_cu(false, cplx);
    }
    if (path == SIGNTRI_PATH_PS && eo.sweep != SIGNTRI_SWEEP_DATAFLOW) {
        // the Sylvester form runs on the dataflow sweeps only
        const bool pinned = opts && (opts->sweep == SIGNTRI_SWEEP_SUPERDIAG || opts->tile == 64);
        if (algo == SIGNTRI_PS && pinned) return SIGNTRI_ENOTSUP;
        if (pinned) {
            path = SIGNTRI_PATH_PH;
        } else {
            eo.sweep = SIGNTRI_SWEEP_DATAFLOW;
            eo.tile = 32;
            eo.wgs_per_cu = flow_default_wgs_per_cu(mode != SIGNTRI_FP64, cplx);
        }
    }
    const bool flow = eo.sweep == SIGNTRI_SWEEP_DATAFLOW;
    const int tb = eo.tile;
    const Layout L = layout_for(n, dtype, layout, mode, tb, flow);

    int rc = SIGNTRI_OK;
    hipError_t e = hipSuccess;
    if (path == SIGNTRI_PATH_TRIVIAL) {
        e = launch_fill_pm_identity(Uc, lduc, n, cplx, p.n_pos > 0 ? 1.0 : -1.0, st);
    } else if (flow) {
        std::vector<RealItem> items(1);
        RealItem &it = items[0];
        it.T = (const double *)Tc;
        it.ldt = ldtc;
        it.U = (double *)Uc;
        it.ldu = lduc;
        it.n = n;
        it.path = path;
        it.p = path == SIGNTRI_PATH_PS ? p.split : 0;
        it.s = p.ps_sign;
        it.sgn = sgn;
        it.dg = dg;
        it.cplx = cplx;
        it.info = info;
        const int8_t *hsv[1] = {hs};
        rc = run_real(items, mode, &eo, ws + L.flow, hflow, prof_on(), hsv, st);
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
        a.max_splits = eo.max_splits;
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
    if (info && flow && path != SIGNTRI_PATH_TRIVIAL && mode != SIGNTRI_MIXED_REFINED) {
        int herr = 0;
        if ((rc = sweep_error(ws + L.flow, &n, 1, mode != SIGNTRI_FP64, cplx, hflow, st, &herr)) !=
            0)
            return rc;
    }
    if (info) {
        const bool triv = path == SIGNTRI_PATH_TRIVIAL;
        info->path = path;
        info->tile = triv ? 0 : tb;
        info->sweep = triv ? 0 : eo.sweep;
        info->wgs_per_cu = triv ? 0 : eo.wgs_per_cu;
    }
    return SIGNTRI_OK;
}

// F = phi(T) for a general function phi given on the diagonal (Algorithm 1):
// the FP64 dataflow sweep of the substitution with every pair of entries by the
// element Parlett equation, diagonal blocks by the same equation element by
// element.
int signtri_fun_run(const void *T, int64_t ldt, const void *fdiag, void *F, int64_t ldf,
                    int64_t n, signtri_dtype dtype, void *stream, signtri_info *info)
{
    if (info) std::memset(info, 0, sizeof(*info));
    if (n > 0 && !T) return -1;
    if (ldt < std::max<int64_t>(1, n)) return -2;
    if (n > 0 && !fdiag) return -3;
    if (n > 0 && !F) return -4;
    if (ldf < std::max<int64_t>(1, n)) return -5;
    if (n < 0) return -6;
    if (dtype != SIGNTRI_R64 && dtype != SIGNTRI_C128) return -7;
    const bool cplx = dtype == SIGNTRI_C128;
    const size_t es = cplx ? 16 : 8;
    if (n > 0 && ranges_overlap(T, extent_bytes(n, ldt, es), F, extent_bytes(n, ldf, es))) return -4;
    if (n > 0 && ranges_overlap(fdiag, (size_t)n * es, F, extent_bytes(n, ldf, es))) return -4;
    if (n == 0) return SIGNTRI_OK;
    const Layout L = layout_for(n, dtype, SIGNTRI_COL_MAJOR, SIGNTRI_FP64, 32, true);
    void *ws = nullptr, *hostbuf = nullptr;
    size_t run_host = 0;
    run_sizes(&n, 1, false, cplx, nullptr, &run_host);
    if (int rc = owned_workspace(L.total, &ws)) return rc;
    if (int rc = owned_host(align_up(sizeof(ScanResult)) + align_up((size_t)n) + run_host, &hostbuf))
        return rc;
    char *w = (char *)ws;
    void *hflow = (char *)hostbuf + align_up(sizeof(ScanResult)) + align_up((size_t)n);
    hipStream_t st = (hipStream_t)stream;
    int8_t *sgn = (int8_t *)(w + L.sgn);
    double *dg = (double *)(w + L.dg);
    // the diagonal (the divisors t_ii - t_jj); its signs are not used
    if (launch_scan(T, ldt, n, cplx, sgn, dg, (ScanResult *)(w + L.scan), st) != hipSuccess)
        return SIGNTRI_EHIP;
    signtri_options eo;
    std::memset(&eo, 0, sizeof(eo));
    eo.sweep = SIGNTRI_SWEEP_DATAFLOW;
    eo.tile = 32;
    eo.wgs_per_cu = flow_default_wgs_per_cu(false, cplx);
    std::vector<RealItem> items(1);
    RealItem &it = items[0];
    it.T = (const double *)T;
    it.ldt = ldt;
    it.U = (double *)F;
    it.ldu = ldf;
    it.n = n;
    it.path = SIGNTRI_PATH_PH;
    it.p = 0;
    it.s = 0;
    it.sgn = sgn;
    it.dg = dg;
    it.cplx = cplx;
    it.info = info;
    it.fd = (const double *)fdiag;
    int rc = run_real(items, SIGNTRI_FP64, &eo, w + L.flow, hflow, prof_on(), nullptr, st);
    if (rc != SIGNTRI_OK) return rc;
    if (info) {
        int herr = 0;
        if ((rc = sweep_error(w + L.flow, &n, 1, false, cplx, hflow, st, &herr)) != 0) return rc;
        info->path = SIGNTRI_PATH_PH;
        info->tile = 32;
        info->sweep = SIGNTRI_SWEEP_DATAFLOW;
        info->wgs_per_cu = eo.wgs_per_cu;
    }
    return SIGNTRI_OK;
}

}  // namespace sgt

extern "C" {

int sign_tri(const void *T, int64_t n, int64_t ld, signtri_dtype dtype, void *U)
{
    // with an info, signtri() waits for the sweep and reports a dependency wait
    // that gave up; this form waits anyway
    signtri_info info;
    int rc = signtri(T, ld, U, ld, n, dtype, SIGNTRI_COL_MAJOR, SIGNTRI_FP64, SIGNTRI_AUTO, nullptr,
                     0, nullptr, nullptr, &info);
    if (rc != SIGNTRI_OK) return rc;
    return hipStreamSynchronize(nullptr) == hipSuccess ? SIGNTRI_OK : SIGNTRI_EHIP;
}

int signtri_fun(const void *T, int64_t ldt, const void *fdiag, void *F, int64_t ldf, int64_t n,
                signtri_dtype dtype, void *stream, signtri_info *info)
{
    return sgt::signtri_fun_run(T, ldt, fdiag, F, ldf, n, dtype, stream, info);
}

size_t signtri_batched_workspace_size(const int64_t *n, int64_t batch, signtri_dtype dtype,
                                      signtri_mode mode)
{
    if (batch < 0 || (batch > 0 && !n)) return 0;
    if (dtype != SIGNTRI_R64 && dtype != SIGNTRI_C128) return 0;
    if (mode < SIGNTRI_FP64 || mode > SIGNTRI_FP32) return 0;
    for (int64_t b = 0; b < batch; ++b)
        if (n[b] < 0) return 0;
    return batch_layout(n, batch, mode, dtype == SIGNTRI_C128).dev;
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
    if (batch < 0 || batch > (1 << 24)) return -6;
    if (dtype != SIGNTRI_R64 && dtype != SIGNTRI_C128) return -7;
    if (layout != SIGNTRI_COL_MAJOR && layout != SIGNTRI_ROW_MAJOR) return -8;
    if (mode < SIGNTRI_FP64 || mode > SIGNTRI_FP32) return -9;
    if (workspace && ws_bytes == 0) return -11;
    for (int64_t b = 0; b < batch; ++b) {
        if (infos) std::memset(&infos[b], 0, sizeof(signtri_info));
        if (n[b] < 0 || n[b] > 65535 * (int64_t)kFlowTile) return -5;
        if (n[b] > 0 && (!T[b] || !U[b])) return T[b] ? -3 : -1;
        if (ldt[b] < std::max<int64_t>(1, n[b])) return -2;
        if (ldu[b] < std::max<int64_t>(1, n[b])) return -4;
        const size_t es = dtype == SIGNTRI_C128 ? 16 : 8;
        if (n[b] > 0 && ranges_overlap(T[b], extent_bytes(n[b], ldt[b], es), U[b],
                                       extent_bytes(n[b], ldu[b], es)))
            return -3;
    }
    if (batch == 0) return SIGNTRI_OK;
    if (layout != SIGNTRI_COL_MAJOR) return SIGNTRI_ENOTSUP;
    const bool cplx = dtype == SIGNTRI_C128;
    if (int rc = check_options(opts, dtype, mode)) return rc;
    if (opts && (opts->sweep == SIGNTRI_SWEEP_SUPERDIAG || opts->tile == 64)) return SIGNTRI_ENOTSUP;
    // the batched form runs on the dataflow sweeps; only the grid is a choice
    signtri_options eo;
    std::memset(&eo, 0, sizeof(eo));
    if (opts) eo = *opts;
    eo.sweep = SIGNTRI_SWEEP_DATAFLOW;
    eo.tile = kFlowTile;
    {
        // the grid: the caller's, else the autotuner's for this size class of the
        // batch's largest order, else as many workgroups as fit
        const int mx = flow_max_wgs_per_cu(mode != SIGNTRI_FP64, cplx);
        if (eo.wgs_per_cu <= 0) {
            int64_t nmax = 0;
            for (int64_t b = 0; b < batch; ++b) nmax = std::max(nmax, n[b]);
            signtri_tune_entry te;
            if (nmax > 0 && tune_find(dtype, mode, SIGNTRI_TUNE_BATCHED, nmax, &te))
                eo.wgs_per_cu = te.wgs_per_cu;
        }
        if (eo.wgs_per_cu <= 0 || eo.wgs_per_cu > mx) eo.wgs_per_cu = mx;
    }

    const BatchLayout BL = batch_layout(n, batch, mode, cplx);
    if (workspace) {
        if (ws_bytes < BL.dev) return SIGNTRI_EWORKSPACE;
    } else if (int rc = owned_workspace(BL.dev, &workspace)) {
        return rc;
    }
    void *hostbuf = nullptr;
    if (int rc = owned_host(BL.host, &hostbuf)) return rc;
    char *ws = (char *)workspace, *hb = (char *)hostbuf;
    hipStream_t st = (hipStream_t)stream;
    const int nm = (int)batch;

    // diagonal scan of every matrix, one workgroup each
    ScanMat *hsm = (ScanMat *)(hb + BL.scan_tab);
    for (int m = 0; m < nm; ++m)
        hsm[m] = ScanMat{(const double *)T[m], ldt[m], n[m], (int8_t *)(ws + BL.sgn[m]),
                         (double *)(ws + BL.dg[m]), (ScanResult *)(ws + BL.res) + m, cplx ? 1 : 0};
    if (hipMemcpyAsync(ws + BL.scan_tab, hsm, nm * sizeof(ScanMat), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return SIGNTRI_EHIP;
    if (launch_scan_b((const ScanMat *)(ws + BL.scan_tab), nm, st) != hipSuccess) return SIGNTRI_EHIP;
    // results and signs are adjacent: one copy back
    if (hipMemcpyAsync(hb + BL.res, ws + BL.res, BL.sgn_end - BL.res, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return SIGNTRI_EHIP;
    const ScanResult *hres = (const ScanResult *)(hb + BL.res);
    for (int m = 0; m < nm; ++m)
        if (n[m] > 0 && hres[m].bad_index < n[m]) {
            if (infos) infos[m].bad_index = hres[m].bad_index + 1;
            return SIGNTRI_EDOMAIN;
        }

    // plan every matrix (Section 3 choice, as signtri() with SIGNTRI_AUTO)
    std::vector<RealItem> items;
    std::vector<const int8_t *> hsigns;
    items.reserve(nm);
    for (int m = 0; m < nm; ++m) {
        if (n[m] == 0) continue;
        const int8_t *hs = (const int8_t *)(hb + BL.sgn[m]);
        const HostPlan p = plan_from_signs(hs, n[m], cplx);
        signtri_info *inf = infos ? &infos[m] : nullptr;
        fill_info(inf, p);
        RealItem it;
        it.T = (const double *)T[m];
        it.ldt = ldt[m];
        it.U = (double *)U[m];
        it.ldu = ldu[m];
        it.n = n[m];
        it.path = p.auto_path;
        it.p = p.auto_path == SIGNTRI_PATH_PS ? p.split : 0;
        it.s = it.path == SIGNTRI_PATH_TRIVIAL ? (p.n_pos > 0 ? 1 : -1) : p.ps_sign;
        it.sgn = (const int8_t *)(ws + BL.sgn[m]);
        it.dg = (const double *)(ws + BL.dg[m]);
        it.cplx = cplx;
        it.info = inf;
        if (inf) {
            const bool triv = it.path == SIGNTRI_PATH_TRIVIAL;
            inf->path = it.path;
            inf->tile = triv ? 0 : kFlowTile;
            inf->sweep = triv ? 0 : SIGNTRI_SWEEP_DATAFLOW;
            inf->wgs_per_cu = triv ? 0 : eo.wgs_per_cu;
        }
        items.push_back(it);
        hsigns.push_back(hs);
    }
    std::vector<int64_t> ns(items.size());
    for (size_t m = 0; m < items.size(); ++m) ns[m] = items[m].n;
    char *run_dev = ws + BL.run, *run_host = hb + BL.run_host;
    // every mode as one graph (captured at the first call with these arguments,
    // replayed after): the refinement decides on the device, so nothing in it
    // waits for the host
    int rc;
    const bool graph = graphs_enabled() && !prof_on();
    if (graph) {
        int device = 0;
        if (hipGetDevice(&device) != hipSuccess) return SIGNTRI_EHIP;
        rc = launch_batch_graph(items, mode, &eo, run_dev, st, device);
    } else {
        rc = run_real(items, mode, &eo, run_dev, run_host, prof_on(), hsigns.data(), st, false);
    }
    if (rc != SIGNTRI_OK) return rc;
    // wait; report a dependency wait of the sweep that gave up (and the refinement's
    // outcome in the infos)
    if (mode == SIGNTRI_MIXED_REFINED) return refine_finish(items, &eo, run_dev, run_host, st);
    return sweep_error(run_dev, ns.data(), (int)ns.size(), mode != SIGNTRI_FP64, cplx, run_host, st,
                       nullptr);
}

int signtri_signm_batched(const void *const *A, const int64_t *lda, void *const *S,
                          const int64_t *lds, const int64_t *n, int64_t batch,
                          signtri_dtype dtype, void *stream, int32_t *status)
{
    if (batch > 0 && !A) return -1;
    if (batch > 0 && !lda) return -2;
    if (batch > 0 && !S) return -3;
    if (batch > 0 && !lds) return -4;
    if (batch > 0 && !n) return -5;
    if (batch < 0 || batch > (1 << 24)) return -6;
    if (dtype != SIGNTRI_R64 && dtype != SIGNTRI_C128) return -7;
    const size_t es = dtype == SIGNTRI_C128 ? 16 : 8;
    for (int64_t b = 0; b < batch; ++b) {
        if (status) status[b] = SIGNTRI_OK;
        if (n[b] < 0) return -5;
        if (n[b] > 0 && (!A[b] || !S[b])) return A[b] ? -3 : -1;
        if (lda[b] < std::max<int64_t>(1, n[b])) return -2;
        if (lds[b] < std::max<int64_t>(1, n[b])) return -4;
        if (n[b] > 0 && ranges_overlap(A[b], extent_bytes(n[b], lda[b], es), S[b],
                                       extent_bytes(n[b], lds[b], es)))
            return -3;
    }
    for (int64_t b = 0; b < batch; ++b)
        if (n[b] > sgt::kSignmMaxOrder) return SIGNTRI_ENOTSUP;
    // the table: orders up to 32 first (the smaller kernel), then the rest
    std::vector<sgt::SignmMat> tab;
    tab.reserve((size_t)batch);
    for (int pass = 0; pass < 2; ++pass)
        for (int64_t b = 0; b < batch; ++b) {
            if (n[b] == 0 || (pass == 0) != (n[b] <= 32)) continue;
            tab.push_back(sgt::SignmMat{(const double *)A[b], (double *)S[b], lda[b], lds[b],
                                        (int32_t)n[b], (int32_t)b, nullptr});
        }
    if (tab.empty()) return SIGNTRI_OK;
    int n32 = 0;
    while (n32 < (int)tab.size() && tab[n32].n <= 32) ++n32;
    const size_t tb = align_up(tab.size() * sizeof(sgt::SignmMat));
    const size_t sb = align_up((size_t)batch * sizeof(int32_t));
    // every matrix keeps Q (n x n complex) in the workspace
    size_t qb = 0;
    for (const sgt::SignmMat &m : tab) qb += (size_t)m.n * m.n * 16;
    void *dev = nullptr, *host = nullptr;
    if (int rc = owned_workspace(tb + sb + align_up(qb), &dev)) return rc;
    if (int rc = owned_host(tb + sb, &host)) return rc;
    {
        char *qp = (char *)dev + tb + sb;
        for (sgt::SignmMat &m : tab) {
            m.Q = (sgt::cd *)qp;
            qp += (size_t)m.n * m.n * 16;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    // testing hook: SIGNTRI_DEBUG_SIGNM_SWEEPS=k limits the QR iteration to k sweeps
    // per matrix, so that its not-converged report can be exercised
    int max_sweeps = 0;
    if (const char *e = getenv("SIGNTRI_DEBUG_SIGNM_SWEEPS")) max_sweeps = std::max(0, atoi(e));
    std::memcpy(host, tab.data(), tab.size() * sizeof(sgt::SignmMat));
    int32_t *dstatus = (int32_t *)((char *)dev + tb), *hstatus = (int32_t *)((char *)host + tb);
    if (hipMemcpyAsync(dev, host, tab.size() * sizeof(sgt::SignmMat), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        sgt::launch_signm((const sgt::SignmMat *)dev, (int)tab.size(), n32,
                          dtype == SIGNTRI_C128, dstatus, max_sweeps, st) != hipSuccess ||
        hipMemcpyAsync(hstatus, dstatus, (size_t)batch * sizeof(int32_t), hipMemcpyDeviceToHost,
                       st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return SIGNTRI_EHIP;
    int rc = SIGNTRI_OK;
    for (const sgt::SignmMat &m : tab) {
        const int v = hstatus[m.index];
        const int code = v == sgt::SIGNM_EDOMAIN ? SIGNTRI_EDOMAIN
                         : v == sgt::SIGNM_ENOCONV ? SIGNTRI_ENOCONV
                                                   : SIGNTRI_OK;
        if (status) status[m.index] = code;
    }
    for (int64_t b = 0; b < batch && rc == SIGNTRI_OK; ++b)
        if (n[b] > 0) {
            const int v = hstatus[b];
            rc = v == sgt::SIGNM_EDOMAIN ? SIGNTRI_EDOMAIN
                 : v == sgt::SIGNM_ENOCONV ? SIGNTRI_ENOCONV
                                           : SIGNTRI_OK;
        }
    return rc;
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
    std::lock_guard<std::mutex> lb(batch_graph_mu);
    for (auto &g : batch_graphs) drop_batch_graph(g);
    batch_graphs.clear();
}

}  // extern "C"
