// Autotuner: which sweep variant, block size and persistent grid run fastest
// for a given (dtype, mode, path, size class) is measured on the device, kept
// in a process-wide table, and consulted by signtri() for options left at 0.
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

namespace sgt {

namespace {

struct TuneTable {
    std::mutex mu;
    std::vector<signtri_tune_entry> entries;
    bool env_loaded = false;
};

TuneTable &table()
{
    static TuneTable t;
    return t;
}

int32_t size_class(int64_t n)
{
    int32_t c = 0;
    while (c < 62 && ((int64_t)1 << c) < n) ++c;
    return c;
}

bool same_key(const signtri_tune_entry &a, const signtri_tune_entry &b)
{
    return a.dtype == b.dtype && a.mode == b.mode && a.path == b.path && a.log2n == b.log2n;
}

bool valid_entry(const signtri_tune_entry &e)
{
    const bool key = (e.dtype == SIGNTRI_R64 || e.dtype == SIGNTRI_C128) &&
                     e.mode >= SIGNTRI_FP64 && e.mode <= SIGNTRI_FP32 &&
                     (e.path == SIGNTRI_PATH_PH || e.path == SIGNTRI_PATH_PS ||
                      e.path == SIGNTRI_TUNE_BATCHED) &&
                     e.log2n >= 0 && e.log2n <= 62;
    // the batched form runs the dataflow sweep on 32 x 32 blocks only
    if (e.path == SIGNTRI_TUNE_BATCHED && (e.sweep != SIGNTRI_SWEEP_DATAFLOW || e.tile != 32))
        return false;
    const bool choice = (e.sweep == SIGNTRI_SWEEP_DATAFLOW || e.sweep == SIGNTRI_SWEEP_SUPERDIAG) &&
                        (e.tile == 32 || e.tile == 64) && e.wgs_per_cu >= 0 && e.wgs_per_cu <= 64;
    return key && choice && std::isfinite(e.ms) && e.ms >= 0.0;
}

// Insert or replace (caller holds the lock).
void put(TuneTable &t, const signtri_tune_entry &e)
{
    for (signtri_tune_entry &x : t.entries)
        if (same_key(x, e)) {
            x = e;
            return;
        }
    t.entries.push_back(e);
}

// Parse a table file written by save(): "dtype mode path log2n sweep tile wgs ms" per line,
// '#' starts a comment line.
int read_file(const char *path, std::vector<signtri_tune_entry> &out)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return -1;
    char line[512];
    int rc = 0;
    while (std::fgets(line, sizeof(line), f)) {
        const char *p = line;
        while (*p == ' ' || *p == '\t') ++p;
        if (*p == '#' || *p == '\n' || *p == '\0') continue;
        signtri_tune_entry e;
        std::memset(&e, 0, sizeof(e));
        char tail[8];
        const int k = std::sscanf(p, "%d %d %d %d %d %d %d %lf %7s", &e.dtype, &e.mode, &e.path,
                                  &e.log2n, &e.sweep, &e.tile, &e.wgs_per_cu, &e.ms, tail);
        if (k != 8 || !valid_entry(e)) {
            rc = -1;
            break;
        }
        out.push_back(e);
    }
    std::fclose(f);
    return rc;
}

void load_env_once(TuneTable &t)
{
    if (t.env_loaded) return;
    t.env_loaded = true;
    const char *path = std::getenv("SIGNTRI_TUNE_FILE");
    if (!path || !*path) return;
    std::vector<signtri_tune_entry> es;
    if (read_file(path, es) == 0)
        for (const signtri_tune_entry &e : es) put(t, e);
}

struct Candidate {
    int sweep, tile, wgs;
};

}  // namespace

bool tune_find(signtri_dtype dtype, signtri_mode mode, int path, int64_t n, signtri_tune_entry *out)
{
    TuneTable &t = table();
    std::lock_guard<std::mutex> g(t.mu);
    load_env_once(t);
    signtri_tune_entry k;
    std::memset(&k, 0, sizeof(k));
    k.dtype = dtype;
    k.mode = mode;
    k.path = path;
    k.log2n = size_class(n);
    for (const signtri_tune_entry &e : t.entries)
        if (same_key(e, k)) {
            if (out) *out = e;
            return true;
        }
    return false;
}

}  // namespace sgt

using namespace sgt;

extern "C" {

int signtri_tune_lookup(signtri_dtype dtype, signtri_mode mode, int32_t path, int64_t n,
                        signtri_tune_entry *out)
{
    return tune_find(dtype, mode, path, n, out) ? 1 : 0;
}

int signtri_tune_save(const char *path)
{
    if (!path) return -1;
    TuneTable &t = table();
    std::lock_guard<std::mutex> g(t.mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return -1;
    std::fprintf(f, "# signtri tuning table: dtype mode path log2n sweep tile wgs_per_cu ms\n");
    for (const signtri_tune_entry &e : t.entries)
        std::fprintf(f, "%d %d %d %d %d %d %d %.6f\n", e.dtype, e.mode, e.path, e.log2n, e.sweep,
                     e.tile, e.wgs_per_cu, e.ms);
    return std::fclose(f) == 0 ? 0 : -1;
}

int signtri_tune_load(const char *path)
{
    if (!path) return -1;
    std::vector<signtri_tune_entry> es;
    if (read_file(path, es) != 0) return -1;
    TuneTable &t = table();
    std::lock_guard<std::mutex> g(t.mu);
    for (const signtri_tune_entry &e : es) put(t, e);
    return 0;
}

void signtri_tune_clear(void)
{
    TuneTable &t = table();
    std::lock_guard<std::mutex> g(t.mu);
    t.entries.clear();
    t.env_loaded = true;  // a cleared table stays empty
}

int signtri_autotune(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n,
                     signtri_dtype dtype, signtri_mode mode, signtri_algo algo, void *stream,
                     int32_t reps, signtri_tune_entry *best)
{
    if (n > 0 && !T) return -1;
    if (ldt < std::max<int64_t>(1, n)) return -2;
    if (n > 0 && !U) return -3;
    if (ldu < std::max<int64_t>(1, n)) return -4;
    if (n < 0) return -5;
    if (dtype != SIGNTRI_R64 && dtype != SIGNTRI_C128) return -6;
    if (mode < SIGNTRI_FP64 || mode > SIGNTRI_FP32) return -7;
    if (algo < SIGNTRI_AUTO || algo > SIGNTRI_PS) return -8;
    if (reps < 1 || reps > 1000) return -10;
    if (!best) return -11;
    std::memset(best, 0, sizeof(*best));
    if (n == 0) return SIGNTRI_OK;
    hipStream_t st = (hipStream_t)stream;

    // the path this T takes, from a default call
    signtri_info info;
    int rc = signtri(T, ldt, U, ldu, n, dtype, SIGNTRI_COL_MAJOR, mode, algo, nullptr, 0, stream,
                     nullptr, &info);
    if (rc != SIGNTRI_OK) return rc;
    best->dtype = dtype;
    best->mode = mode;
    best->path = info.path;
    best->log2n = size_class(n);
    // nothing to choose on the trivial path and the projector form
    if (info.path == SIGNTRI_PATH_TRIVIAL || info.path == SIGNTRI_PATH_PROJ)
        return hipStreamSynchronize(st) == hipSuccess ? SIGNTRI_OK : SIGNTRI_EHIP;

    std::vector<Candidate> cands;
    const bool cplx = dtype == SIGNTRI_C128;
    const int mx = flow_max_wgs_per_cu(mode != SIGNTRI_FP64, cplx);
    for (int w = 1; w <= mx; ++w) cands.push_back({SIGNTRI_SWEEP_DATAFLOW, 32, w});
    if (mode == SIGNTRI_FP64 && info.path == SIGNTRI_PATH_PH) {
        cands.push_back({SIGNTRI_SWEEP_SUPERDIAG, 32, 0});
        if (!cplx) cands.push_back({SIGNTRI_SWEEP_SUPERDIAG, 64, 0});
    }

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return SIGNTRI_EHIP;
    }
    double best_ms = -1.0;
    rc = SIGNTRI_OK;
    for (const Candidate &c : cands) {
        signtri_options o;
        std::memset(&o, 0, sizeof(o));
        o.sweep = c.sweep;
        o.tile = c.tile;
        o.wgs_per_cu = c.wgs;
        // one untimed call (with info: it waits and reports a failed sweep)
        signtri_info ci;
        rc = signtri(T, ldt, U, ldu, n, dtype, SIGNTRI_COL_MAJOR, mode, algo, nullptr, 0, stream,
                     &o, &ci);
        if (rc != SIGNTRI_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) {
            rc = SIGNTRI_EHIP;
            break;
        }
        for (int r = 0; r < reps && rc == SIGNTRI_OK; ++r)
            rc = signtri(T, ldt, U, ldu, n, dtype, SIGNTRI_COL_MAJOR, mode, algo, nullptr, 0,
                         stream, &o, nullptr);
        if (rc != SIGNTRI_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = SIGNTRI_EHIP;
            break;
        }
        const double per = (double)ms / reps;
        if (best_ms < 0.0 || per < best_ms) {
            best_ms = per;
            best->sweep = c.sweep;
            best->tile = c.tile;
            best->wgs_per_cu = ci.wgs_per_cu;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SIGNTRI_OK) return rc;
    best->ms = best_ms;
    TuneTable &t = table();
    std::lock_guard<std::mutex> g(t.mu);
    load_env_once(t);
    put(t, *best);
    return SIGNTRI_OK;
}

int signtri_autotune_batched(const void *const *T, const int64_t *ldt, void *const *U,
                             const int64_t *ldu, const int64_t *n, int64_t batch,
                             signtri_dtype dtype, signtri_mode mode, void *stream, int32_t reps,
                             signtri_tune_entry *best)
{
    if (reps < 1 || reps > 1000) return -12;
    if (!best) return -13;
    std::memset(best, 0, sizeof(*best));
    // argument checks and the first (untimed) run: the default grid
    int rc = signtri_batched(T, ldt, U, ldu, n, batch, dtype, SIGNTRI_COL_MAJOR, mode, nullptr, 0,
                             stream, nullptr, nullptr);
    if (rc != SIGNTRI_OK) return rc;
    int64_t nmax = 0;
    for (int64_t b = 0; b < batch; ++b) nmax = std::max(nmax, n[b]);
    best->dtype = dtype;
    best->mode = mode;
    best->path = SIGNTRI_TUNE_BATCHED;
    best->log2n = size_class(nmax);
    best->sweep = SIGNTRI_SWEEP_DATAFLOW;
    best->tile = 32;
    if (nmax == 0) return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? SIGNTRI_OK
                                                                                : SIGNTRI_EHIP;
    hipStream_t st = (hipStream_t)stream;
    const int mx = flow_max_wgs_per_cu(mode != SIGNTRI_FP64, dtype == SIGNTRI_C128);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return SIGNTRI_EHIP;
    }
    double best_ms = -1.0;
    for (int w = 1; w <= mx && rc == SIGNTRI_OK; ++w) {
        signtri_options o;
        std::memset(&o, 0, sizeof(o));
        o.sweep = SIGNTRI_SWEEP_DATAFLOW;
        o.tile = 32;
        o.wgs_per_cu = w;
        // one untimed call (it also captures this grid's graph)
        rc = signtri_batched(T, ldt, U, ldu, n, batch, dtype, SIGNTRI_COL_MAJOR, mode, nullptr, 0,
                             stream, &o, nullptr);
        if (rc != SIGNTRI_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) {
            rc = SIGNTRI_EHIP;
            break;
        }
        for (int r = 0; r < reps && rc == SIGNTRI_OK; ++r)
            rc = signtri_batched(T, ldt, U, ldu, n, batch, dtype, SIGNTRI_COL_MAJOR, mode, nullptr,
                                 0, stream, &o, nullptr);
        if (rc != SIGNTRI_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = SIGNTRI_EHIP;
            break;
        }
        const double per = (double)ms / reps;
        if (best_ms < 0.0 || per < best_ms) {
            best_ms = per;
            best->wgs_per_cu = w;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SIGNTRI_OK) return rc;
    best->ms = best_ms;
    TuneTable &t = table();
    std::lock_guard<std::mutex> g(t.mu);
    load_env_once(t);
    put(t, *best);
    return SIGNTRI_OK;
}

}  // extern "C"
