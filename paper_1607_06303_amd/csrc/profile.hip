// Opt-in per-family kernel timers (HIP events on the launching stream).
#include <mutex>
#include <vector>

#include "common.h"

namespace sgt {

namespace {

struct Rec {
    hipEvent_t a, b;
    int kind;
    double flops;
    int launches;
};

struct Prof {
    std::mutex mu;
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t pending = nullptr;
};

Prof &prof()
{
    static Prof p;
    return p;
}

hipEvent_t take_event(Prof &p)
{
    if (!p.pool.empty()) {
        hipEvent_t e = p.pool.back();
        p.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

bool prof_on() { return prof().on; }

void prof_begin(hipStream_t st)
{
    Prof &p = prof();
    if (!p.on) return;
    std::lock_guard<std::mutex> g(p.mu);
    p.pending = take_event(p);
    if (p.pending) (void)hipEventRecord(p.pending, st);
}

void prof_end(hipStream_t st, int kind, double flops, int launches)
{
    Prof &p = prof();
    if (!p.on) return;
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.pending) return;
    hipEvent_t e = take_event(p);
    if (!e) return;
    (void)hipEventRecord(e, st);
    p.recs.push_back({p.pending, e, kind, flops, launches});
    p.pending = nullptr;
}

}  // namespace sgt

using namespace sgt;

extern "C" {

void signtri_profile_enable(int on)
{
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    for (auto &r : p.recs) {
        p.pool.push_back(r.a);
        p.pool.push_back(r.b);
    }
    p.recs.clear();
    p.on = on != 0;
}

int signtri_profile_read(int kind, double *ms, int64_t *launches, double *flops)
{
    if (kind < 0 || kind >= PK_COUNT) return -1;
    Prof &p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    double t = 0.0, f = 0.0;
    int64_t c = 0;
    for (auto &r : p.recs) {
        if (r.kind != kind) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return SIGNTRI_EHIP;
        float x = 0.0f;
        if (hipEventElapsedTime(&x, r.a, r.b) != hipSuccess) return SIGNTRI_EHIP;
        t += x;
        f += r.flops;
        c += r.launches;
    }
    if (ms) *ms = t;
    if (launches) *launches = c;
    if (flops) *flops = f;
    return 0;
}

}  // extern "C"
