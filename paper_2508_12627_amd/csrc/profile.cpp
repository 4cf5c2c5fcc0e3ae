#include "profile.hpp"

namespace ustat {

namespace {
Profiler g_prof;
bool g_on = false;
bool g_suspended = false;
}  // namespace

Profiler *Profiler::active() { return (g_on && !g_suspended) ? &g_prof : nullptr; }
void Profiler::enable(bool on) { g_on = on; }
bool Profiler::enabled() { return g_on; }
void Profiler::suspend(bool s) { g_suspended = s; }

hipEvent_t Profiler::get() {
    if (!pool_.empty()) {
        hipEvent_t e = pool_.back();
        pool_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void Profiler::begin(int kind, hipStream_t s, double fl, double by) {
    Rec r;
    r.kind = kind;
    r.a = get();
    r.b = get();
    r.flops = fl;
    r.bytes = by;
    (void)hipEventRecord(r.a, s);
    pending_.push_back(r);
}

void Profiler::end(int kind, hipStream_t s) {
    for (auto it = pending_.rbegin(); it != pending_.rend(); ++it)
        if (it->kind == kind) {
            (void)hipEventRecord(it->b, s);
            return;
        }
}

void Profiler::collect() {
    for (Rec &r : pending_) {
        float t = 0;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            ms[r.kind] += t;
            launches[r.kind] += 1;
            flops[r.kind] += r.flops;
            bytes[r.kind] += r.bytes;
        }
        pool_.push_back(r.a);
        pool_.push_back(r.b);
    }
    pending_.clear();
}

void Profiler::reset() {
    for (int k = 0; k < KIND_COUNT; ++k) {
        ms[k] = 0;
        launches[k] = 0;
        flops[k] = 0;
        bytes[k] = 0;
    }
}

}  // namespace ustat
