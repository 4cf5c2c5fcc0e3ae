// Host-only exercise of the engine's planner, dry schedules and argument
// checks through the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (no device call is made).
// Exit status 0 when every call returned the expected status.
#include <cstdio>
#include <cstring>
#include <vector>

#include "ustat.h"

static int failures = 0;
#define EXPECT(cond)                                                         \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

static std::vector<int32_t> flat(const std::vector<std::pair<int, int>> &e) {
    std::vector<int32_t> v;
    for (auto &p : e) {
        v.push_back(p.first);
        v.push_back(p.second);
    }
    return v;
}

static void exercise(int m, const std::vector<std::pair<int, int>> &edges) {
    const std::vector<int32_t> E = flat(edges);
    for (int prec = 0; prec < 4; ++prec)
        for (int order = 0; order < 2; ++order)
            for (int sp = 0; sp < 2; ++sp)
                for (int flags = 0; flags < 4; ++flags) {
                    ustat_plan_opts o;
                    EXPECT(ustat_plan_opts_default(&o) == USTAT_OK);
                    o.precision = prec;
                    o.order = order;
                    o.sparsify = sp;
                    o.flags = flags;
                    ustat_plan p = nullptr;
                    ustat_status st = ustat_plan_create(m, (int)edges.size(), E.data(), &o, &p);
                    EXPECT(st == USTAT_OK);
                    if (st != USTAT_OK) continue;
                    int32_t nv = 0, M = 0, w = 0;
                    std::vector<int64_t> Nl(m + 1);
                    EXPECT(ustat_plan_info(p, &nv, &M, Nl.data(), &w) == USTAT_OK);
                    for (int i = 0; i < nv; ++i) {
                        std::vector<int32_t> blk(m), ord(m);
                        int64_t mu = 0;
                        int32_t tw = 0, wd = 0, len = 0, sv = 0;
                        EXPECT(ustat_plan_partition(p, i, blk.data(), &mu, &tw, &wd) == USTAT_OK);
                        EXPECT(ustat_plan_order(p, i, ord.data(), &len, &sv) == USTAT_OK);
                        if (sv < 0 && w <= 2) {
                            std::vector<float> f(USTAT_NUM_FEATURES);
                            EXPECT(ustat_order_features(p, blk.data(), ord.data(), len, sv, 1000, f.data()) ==
                                   USTAT_OK);
                        }
                    }
                    EXPECT(ustat_plan_partition(p, nv, nullptr, nullptr, nullptr, nullptr) == USTAT_E_INVALID);
                    for (int64_t n : {(int64_t)m, (int64_t)37, (int64_t)300, (int64_t)4096}) {
                        double fl = 0, by = 0;
                        uint64_t ws = 0;
                        ustat_status c = ustat_plan_cost(p, n, &fl, &by, &ws);
                        EXPECT(c == USTAT_OK || c == USTAT_E_OVERFLOW);
                        std::vector<int64_t> ns = {n, n / 2 + m, 129};
                        uint64_t b = 0;
                        ustat_status c2 = ustat_plan_workspace(p, 3, ns.data(), 1, &b);
                        EXPECT(c2 == USTAT_OK || c2 == USTAT_E_UNSUPPORTED);
                    }
                    int64_t gb = 0, cb = 0;
                    EXPECT(ustat_plan_tuning(p, &gb, &cb) == USTAT_OK);
                    EXPECT(ustat_plan_set_tuning(p, 0, 0) == USTAT_E_INVALID);
                    EXPECT(ustat_plan_set_tuning(p, gb, cb) == USTAT_OK);
                    EXPECT(ustat_eval(p, m - 1, nullptr, nullptr, nullptr) == USTAT_E_INVALID);
                    if (flags == 0 && sp == 0 && order == 0) {
                        // low-rank schedules: all panels distinct, then all one panel
                        ustat_lowrank_stats ls;
                        const ustat_status want = prec == 3 ? USTAT_E_UNSUPPORTED : USTAT_OK;
                        EXPECT(ustat_lowrank_info(p, 1000, 3, nullptr, &ls) == want);
                        std::vector<int32_t> same(2 * edges.size(), 0);
                        EXPECT(ustat_lowrank_info(p, 77, 1, same.data(), &ls) == want);
                        EXPECT(ustat_lowrank_info(p, 77, 0, nullptr, &ls) == USTAT_E_INVALID);
                        EXPECT(ustat_eval_lowrank(p, 77, 2, nullptr, nullptr, nullptr, nullptr) ==
                               (prec == 3 ? USTAT_E_UNSUPPORTED : USTAT_E_INVALID));
                    }
                    EXPECT(ustat_plan_destroy(p) == USTAT_OK);
                }
}

int main() {
    exercise(3, {{0, 1}, {1, 2}, {2, 0}});
    exercise(4, {{0, 1}, {1, 2}, {2, 3}, {3, 0}});
    exercise(5, {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 0}, {0, 2}});
    exercise(4, {{0, 1}, {1, 0}, {1, 2}, {2, 3}, {3, 1}});
    exercise(4, {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}});
    exercise(2, {{0, 1}});
    // invalid graphs and options
    ustat_plan p = nullptr;
    const int32_t self[] = {0, 0, 0, 1};
    EXPECT(ustat_plan_create(2, 2, self, nullptr, &p) == USTAT_E_INVALID);
    const int32_t gap[] = {0, 2};
    EXPECT(ustat_plan_create(3, 1, gap, nullptr, &p) == USTAT_E_INVALID);
    EXPECT(ustat_plan_create(3, 1, nullptr, nullptr, &p) == USTAT_E_INVALID);
    // host allocation failures at every injection point of a plan creation
    const std::vector<int32_t> E = flat({{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 0}, {0, 2}});
    int nomem = 0;
    for (int64_t k = 0; k < 400; ++k) {
        EXPECT(ustat_debug_inject(0, k) == USTAT_OK);
        ustat_plan q = nullptr;
        ustat_status st = ustat_plan_create(5, 6, E.data(), nullptr, &q);
        EXPECT(st == USTAT_OK || st == USTAT_E_NOMEM);
        if (st == USTAT_E_NOMEM) {
            ++nomem;
            EXPECT(q == nullptr);
        }
        if (q) {
            uint64_t ws = 0;
            ustat_status c = ustat_plan_cost(q, 500, nullptr, nullptr, &ws);
            EXPECT(c == USTAT_OK || c == USTAT_E_NOMEM);
            ustat_plan_destroy(q);
        }
    }
    EXPECT(ustat_debug_inject(0, -1) == USTAT_OK);
    EXPECT(nomem > 0);
    EXPECT(ustat_debug_inject(7, 0) == USTAT_E_INVALID);
    std::printf("sanitized planner run: %d failures, %d injected allocation failures\n", failures, nomem);
    return failures ? 1 : 0;
}
