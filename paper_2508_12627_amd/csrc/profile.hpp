// Optional per-kernel-kind timing with HIP events recorded on the launch
// stream.  Disabled by default; enabled through the C ABI.  Never active
// while a launch sequence is being captured into a graph.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace ustat {

enum ProfKind { KIND_PREP = 0, KIND_GEMM = 1, KIND_ELIM1 = 2, KIND_REDUCE = 3, KIND_RBF = 4,
                KIND_LR_STEP = 5, KIND_LR_REDUCE = 6, KIND_LR_KR = 7, KIND_COUNT = 8 };

class Profiler {
public:
    static Profiler *active();
    static void enable(bool on);
    static bool enabled();
    static void suspend(bool s);
    void begin(int kind, hipStream_t s, double flops, double bytes = 0);
    void end(int kind, hipStream_t s);
    void collect();  // after the stream has been synchronised
    void reset();
    double ms[KIND_COUNT] = {0};
    int64_t launches[KIND_COUNT] = {0};
    double flops[KIND_COUNT] = {0};
    double bytes[KIND_COUNT] = {0};

private:
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double flops, bytes;
    };
    std::vector<Rec> pending_;
    std::vector<hipEvent_t> pool_;
    hipEvent_t get();
};

struct ProfScope {
    Profiler *p;
    int kind;
    hipStream_t s;
    ProfScope(Profiler *p_, int k, hipStream_t s_, double flops, double bytes = 0)
        : p(p_), kind(k), s(s_) {
        if (p) p->begin(kind, s, flops, bytes);
    }
    ~ProfScope() {
        if (p) p->end(kind, s);
    }
};

}  // namespace ustat
