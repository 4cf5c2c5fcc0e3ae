// Failure-injection countdowns (see inject.hpp).
#include "inject.hpp"

#include <atomic>

namespace ustat {

namespace {
std::atomic<int64_t> g_countdown[INJ_KINDS] = {{-1}, {-1}, {-1}};
}  // namespace

void inject_arm(int kind, int64_t countdown) {
    if (kind >= 0 && kind < INJ_KINDS) g_countdown[kind].store(countdown);
}

bool inject_fire(int kind) {
    std::atomic<int64_t> &c = g_countdown[kind];
    int64_t v = c.load(std::memory_order_relaxed);
    while (v >= 0) {
        if (c.compare_exchange_weak(v, v - 1)) return v == 0;
    }
    return false;
}

}  // namespace ustat
