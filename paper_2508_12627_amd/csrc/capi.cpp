// C ABI of libustat (declared in include/ustat.h).  Argument checking,
// plan handles, error strings; the work is done by plan.cpp (host) and
// exec.cpp / kernels.hip (device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ustat.h"
#include "costmodel.hpp"
#include "guard.hpp"
#include "inject.hpp"
#include "exec.hpp"
#include "kernels.hpp"
#include "lowrank.hpp"
#include "plan.hpp"
#include "profile.hpp"

using namespace ustat;

struct ustat_plan_s {
    Plan plan;
    Runtime rt;
    std::unique_ptr<CostModel> model;
    std::vector<const VProgram *> all;
    // device buffer holding factor matrices built from samples
    char *factors = nullptr;
    size_t factors_bytes = 0;
    // motif plans (ustat_plan_create_motifs): one kernel per motif, and the
    // automorphism count that turns its U-statistic into the motif count
    std::vector<Plan> motifs;
    std::vector<int64_t> motif_aut;
    int motif_size = 0;
    // low-rank schedules by sample size, rank and panel identity
    std::map<std::string, std::unique_ptr<LrSchedule>> lowrank;
    ~ustat_plan_s() {
        if (factors) (void)hipFree(factors);
    }
};

namespace {

thread_local std::string g_err;

}  // namespace

void ustat::set_last_error(const std::string &msg) { g_err = msg; }

namespace {

ustat_status fail(ustat_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

ustat_status ok() {
    g_err.clear();
    return USTAT_OK;
}

ustat_status from_exec(int st, const std::string &msg) {
    if (st == 0 && msg.empty()) return ok();
    switch (st) {
        case 2: return fail(USTAT_E_UNSUPPORTED, msg);
        case 3: return fail(USTAT_E_NOMEM, msg);
        case 5: return fail(USTAT_E_OVERFLOW, msg);
        case 6: return fail(USTAT_E_INFEASIBLE, msg);
        case 1: return fail(USTAT_E_INVALID, msg);
        default: return fail(USTAT_E_HIP, msg);
    }
}

bool canonical_rgs(const int32_t *block_of, int m, std::vector<int> &out) {
    out.assign(m, 0);
    std::vector<int> map;
    std::vector<int> seen;
    for (int i = 0; i < m; ++i) {
        int b = block_of[i];
        int j = -1;
        for (size_t q = 0; q < seen.size(); ++q)
            if (seen[q] == b) j = (int)q;
        if (j < 0) {
            j = (int)seen.size();
            seen.push_back(b);
        }
        out[i] = j;
    }
    return true;
}

hipError_t grow(char **p, size_t *have, size_t need, Runtime *rt = nullptr) {
    if (inject_fire(INJ_DEVICE_ALLOC)) return hipErrorOutOfMemory;
    if (*p && *have >= need) return hipSuccess;
    if (rt) rt->drop_graphs();  // captured graphs reference the old buffer
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    hipError_t e = hipMalloc(p, std::max<size_t>(need, 256));
    if (e == hipSuccess) *have = need;
    return e;
}

void fill_result(ustat_result *out, const DatasetResult &r, const Plan &p, int64_t n, int nv) {
    std::memset(out, 0, sizeof *out);
    out->value = r.value;
    out->exact_hi = r.exact_hi;
    out->exact_lo = r.exact_lo;
    out->err_scale = r.scale;
    out->err_est = r.err_est;
    out->num_vstats = nv;
}

}  // namespace

extern "C" {

ustat_status ustat_plan_opts_default(ustat_plan_opts *opts) {
    USTAT_GUARD_BEGIN
    if (!opts) return fail(USTAT_E_INVALID, "opts is NULL");
    std::memset(opts, 0, sizeof *opts);
    opts->precision = USTAT_F64;
    opts->order = USTAT_ORDER_MINFILL;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_plan_create(int32_t m, int32_t num_edges, const int32_t *edges,
                               const ustat_plan_opts *opts, ustat_plan *out) {
    USTAT_GUARD_BEGIN
    if (!out) return fail(USTAT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!edges || num_edges < 1) return fail(USTAT_E_INVALID, "need at least one edge");
    if (num_edges > 64) return fail(USTAT_E_INVALID, "at most 64 edges");
    ustat_plan_opts o;
    ustat_plan_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision < 0 || o.precision > 3) return fail(USTAT_E_INVALID, "unknown precision");
    if (o.order < 0 || o.order > 2) return fail(USTAT_E_INVALID, "unknown order policy");
    if (o.sparsify != 0 && o.sparsify != 1) return fail(USTAT_E_INVALID, "sparsify must be 0 or 1");
    if (o.flags & ~(USTAT_FLAG_NO_CSE | USTAT_FLAG_SYMMETRIC | USTAT_FLAG_NO_SYM_GEMM |
                    USTAT_FLAG_OVERLAP_LEVELS))
        return fail(USTAT_E_INVALID, "unknown flag bits");
    try {
        std::unique_ptr<ustat_plan_s> p(new ustat_plan_s());
        std::vector<Edge> E;
        for (int k = 0; k < num_edges; ++k) E.push_back({edges[2 * k], edges[2 * k + 1]});
        PlanOptions po;
        po.precision = o.precision;
        po.order = o.order;
        po.sparsify = o.sparsify;
        po.workspace_limit = o.workspace_limit;
        if (o.n_hint < 0 || o.n_hint > (1ll << 20)) return fail(USTAT_E_INVALID, "n_hint out of range");
        if (o.n_hint > 0) po.n_hint = (double)o.n_hint;
        po.cse = !(o.flags & USTAT_FLAG_NO_CSE);
        po.symmetric = (o.flags & USTAT_FLAG_SYMMETRIC) != 0;
        po.sym_gemm = !(o.flags & USTAT_FLAG_NO_SYM_GEMM);
        po.overlap = (o.flags & USTAT_FLAG_OVERLAP_LEVELS) != 0;
        if (o.cost_model_path) po.cost_model_path = o.cost_model_path;
        const OrderScorer *scorer = nullptr;
        if (o.order == USTAT_ORDER_LEARNED) {
            if (!o.cost_model_path)
                return fail(USTAT_E_INVALID, "the learned order policy needs cost_model_path");
            p->model.reset(new CostModel());
            std::string err = p->model->load(o.cost_model_path);
            if (!err.empty()) return fail(USTAT_E_INVALID, "cost model: " + err);
            scorer = p->model.get();
        }
        std::string err = make_plan(m, E, po, scorer, p->plan);
        if (!err.empty()) return fail(USTAT_E_INVALID, err);
        for (auto &pr : p->plan.progs) p->all.push_back(&pr);
        *out = p.release();
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(USTAT_E_NOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        return fail(USTAT_E_INVALID, ex.what());
    }
    USTAT_GUARD_END
}

ustat_status ustat_plan_destroy(ustat_plan plan) {
    USTAT_GUARD_BEGIN
    delete plan;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_plan_info(ustat_plan plan, int32_t *num_vstats, int32_t *M, int64_t *N_l,
                             int32_t *max_width) {
    USTAT_GUARD_BEGIN
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (num_vstats) *num_vstats = (int32_t)plan->plan.progs.size();
    if (M) *M = plan->plan.M;
    if (N_l)
        for (int l = 0; l <= plan->plan.m; ++l) N_l[l] = plan->plan.N_l[l];
    if (max_width) *max_width = plan->plan.max_width;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_plan_cost(ustat_plan plan, int64_t n, double *flops, double *bytes,
                             uint64_t *workspace) {
    USTAT_GUARD_BEGIN
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (n < 1) return fail(USTAT_E_INVALID, "n must be positive");
    double f = 0, b = 0;
    double es = plan->plan.opts.precision == USTAT_F64 ? 8 : plan->plan.opts.precision == USTAT_I8 ? 1 : 4;
    for (auto &pr : plan->plan.progs) {
        double pf, pb;
        program_cost(pr, (double)n, es, &pf, &pb);
        f += pf;
        b += pb;
    }
    if (flops) *flops = f;
    if (bytes) *bytes = b;
    if (workspace) {
        if (!plan->plan.executable) {
            *workspace = 0;
        } else {
            int st = 0;
            const size_t w = workspace_bytes(plan->plan, plan->all, {n}, false, &st);
            if (st == 5)
                return fail(USTAT_E_OVERFLOW,
                            "an exact intermediate may overflow for inputs of magnitude up to 127");
            if (st == 2) return fail(USTAT_E_UNSUPPORTED, "this size is outside what the engine runs");
            *workspace = w;
        }
    }
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_plan_workspace(ustat_plan plan, int32_t batch, const int64_t *n,
                                  int32_t shared_factor, uint64_t *bytes) {
    USTAT_GUARD_BEGIN
    if (!plan || batch < 1 || !n || !bytes) return fail(USTAT_E_INVALID, "bad arguments");
    if (!plan->plan.executable) return fail(USTAT_E_UNSUPPORTED, plan->plan.lower_error);
    for (int b = 0; b < batch; ++b)
        if (n[b] < plan->plan.m) return fail(USTAT_E_INVALID, "n must be at least m");
    std::vector<int64_t> ns(n, n + batch);
    *bytes = workspace_bytes(plan->plan, plan->all, ns, shared_factor != 0);
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_plan_partition(ustat_plan plan, int32_t idx, int32_t *block_of, int64_t *mu,
                                  int32_t *tw, int32_t *width) {
    USTAT_GUARD_BEGIN
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (idx < 0 || idx >= (int32_t)plan->plan.progs.size())
        return fail(USTAT_E_INVALID, "partition index out of range");
    const VProgram &p = plan->plan.progs[idx];
    if (block_of)
        for (int i = 0; i < plan->plan.m; ++i) block_of[i] = p.block_of[i];
    if (mu) *mu = p.mu;
    if (tw) *tw = p.tw;
    if (width) *width = p.width;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_plan_order(ustat_plan plan, int32_t idx, int32_t *order, int32_t *len,
                              int32_t *slice_var) {
    USTAT_GUARD_BEGIN
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (idx < 0 || idx >= (int32_t)plan->plan.progs.size())
        return fail(USTAT_E_INVALID, "partition index out of range");
    const VProgram &p = plan->plan.progs[idx];
    if (order)
        for (size_t i = 0; i < p.order.size(); ++i) order[i] = p.order[i];
    if (len) *len = (int32_t)p.order.size();
    if (slice_var) *slice_var = p.slice_var;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_graph_treewidth(int32_t m, int32_t num_edges, const int32_t *edges,
                                   int32_t *tw) {
    USTAT_GUARD_BEGIN
    if (m < 1 || m > 16) return fail(USTAT_E_INVALID, "m must be in 1..16");
    if (num_edges < 0 || (num_edges > 0 && !edges) || !tw)
        return fail(USTAT_E_INVALID, "bad arguments");
    std::vector<uint32_t> adj(m, 0);
    for (int k = 0; k < num_edges; ++k) {
        int u = edges[2 * k], v = edges[2 * k + 1];
        if (u < 0 || u >= m || v < 0 || v >= m) return fail(USTAT_E_INVALID, "endpoint out of range");
        if (u != v) {
            adj[u] |= 1u << v;
            adj[v] |= 1u << u;
        }
    }
    *tw = exact_treewidth(m, adj);
    return ok();
    USTAT_GUARD_END
}

}  // extern "C"

namespace {

int log2_bucket(int64_t x) {
    int b = 0;
    while ((int64_t(1) << b) < x && b < 62) ++b;
    return b;
}

// Cache key of an autotuning result: the device (architecture and compute
// units), the plan (graph, precision, order policy, options) and the shape.
std::string tune_key(ustat_plan plan, const std::string &shape) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::string devs = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        devs = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
    const PlanOptions &o = plan->plan.opts;
    std::string k = devs + "|m" + std::to_string(plan->plan.m) + "|e";
    for (const Edge &e : plan->plan.edges) k += std::to_string(e.u) + "-" + std::to_string(e.v) + ",";
    k += "|p" + std::to_string(o.precision) + "|o" + std::to_string(o.order) + "|s" +
         std::to_string(o.sparsify) + "|y" + std::to_string((int)o.symmetric) + "|c" +
         std::to_string((int)o.cse) + "|" + shape;
    for (char &ch : k)
        if (ch == ' ' || ch == '\n') ch = '_';
    return k;
}

// The per-device tuning cache: a text file named by USTAT_TUNE_CACHE, one
// line "key gemm_big_min colred_blocks ms" per tuned shape.
bool tune_cache_lookup(ustat_plan plan, const std::string &key, double *ms) {
    const char *path = std::getenv("USTAT_TUNE_CACHE");
    if (!path || !*path) return false;
    std::FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[4096];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[3900];
        long long gb = 0, cb = 0;
        double t = 0;
        if (std::sscanf(line, "%3899s %lld %lld %lf", k, &gb, &cb, &t) == 4 && key == k && cb >= 1 &&
            cb <= (1 << 20) && gb >= 0) {
            plan->plan.tuning.gemm_big_min = gb;
            plan->plan.tuning.colred_blocks = cb;
            if (ms) *ms = t;
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    if (found) plan->rt.drop_graphs();
    return found;
}

void tune_cache_store(ustat_plan plan, const std::string &key, double ms) {
    const char *path = std::getenv("USTAT_TUNE_CACHE");
    if (!path || !*path || key.size() >= 3900) return;
    std::FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %lld %lld %.6f\n", key.c_str(), (long long)plan->plan.tuning.gemm_big_min,
                 (long long)plan->plan.tuning.colred_blocks, ms);
    std::fclose(f);
}

// Every candidate tuning (gemm_big_min in {256, 0, never} for fp32 and
// split-bf16, colred_blocks in {256, 1024, 4096}): one warm-up evaluation
// (which captures the graph), then the best of reps timed evaluations; the
// fastest candidate is kept, the previous tuning restored on error.
ustat_status tune_loop(ustat_plan plan, int32_t reps, const std::function<ustat_status()> &eval,
                       double *best_ms) {
    const int prec = plan->plan.opts.precision;
    std::vector<int64_t> gbs = {256};
    if (prec == USTAT_F32 || prec == USTAT_BF16X3) gbs = {256, 0, int64_t(1) << 62};
    const int64_t cbs[3] = {256, 1024, 4096};
    const Tuning keep = plan->plan.tuning;
    Tuning best = keep;
    double best_s = std::numeric_limits<double>::infinity();
    ustat_status st = USTAT_OK;
    for (int64_t gb : gbs) {
        for (int64_t cb : cbs) {
            plan->plan.tuning.gemm_big_min = gb;
            plan->plan.tuning.colred_blocks = cb;
            plan->rt.drop_graphs();
            st = eval();
            if (st != USTAT_OK) break;
            double t = std::numeric_limits<double>::infinity();
            for (int r = 0; r < reps && st == USTAT_OK; ++r) {
                auto t0 = std::chrono::steady_clock::now();
                st = eval();
                t = std::min(t, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
            }
            if (st != USTAT_OK) break;
            if (t < best_s) {
                best_s = t;
                best = plan->plan.tuning;
            }
        }
        if (st != USTAT_OK) break;
    }
    plan->plan.tuning = st == USTAT_OK ? best : keep;
    plan->rt.drop_graphs();
    if (best_ms) *best_ms = best_s * 1e3;
    return st;
}

}  // namespace

extern "C" {

static ustat_status run(ustat_plan plan, const std::vector<const VProgram *> &progs,
                        std::vector<Dataset> &data, hipStream_t s, std::vector<DatasetResult> &res,
                        std::vector<double> *vout, const std::function<hipError_t(hipStream_t)> &pre,
                        const std::string &key, const ExtMem *ext = nullptr) {
    int st = 0;
    // Launch sequences are captured into a HIP graph and replayed when the
    // stream is not the null stream; profiled runs launch kernel by kernel so
    // that every launch can be timed with events.
    bool capture = (s != nullptr) && !key.empty() && !Profiler::enabled() && !ext;
    std::string err;
    try {
        if (capture) Profiler::suspend(true);
        err = execute_all(plan->plan, progs, data, s, plan->rt, res, vout, &st, capture, key, pre, ext);
        if (capture) Profiler::suspend(false);
    } catch (const std::bad_alloc &) {
        Profiler::suspend(false);
        return fail(USTAT_E_NOMEM, "host allocation failed");
    }
    return from_exec(st, err);
}

static ustat_status check_eval(ustat_plan plan, int64_t n) {
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (n < plan->plan.m) return fail(USTAT_E_INVALID, "n must be at least m");
    if (n > (1ll << 20)) return fail(USTAT_E_INVALID, "n above 2^20 is not supported");
    if (!plan->plan.executable)
        return fail(USTAT_E_UNSUPPORTED, "plan needs a step kind the engine lacks: " +
                                             plan->plan.lower_error);
    return USTAT_OK;
}

ustat_status ustat_plan_tuning(ustat_plan plan, int64_t *gemm_big_min, int64_t *colred_blocks) {
    USTAT_GUARD_BEGIN
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (gemm_big_min) *gemm_big_min = plan->plan.tuning.gemm_big_min;
    if (colred_blocks) *colred_blocks = plan->plan.tuning.colred_blocks;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_plan_set_tuning(ustat_plan plan, int64_t gemm_big_min, int64_t colred_blocks) {
    USTAT_GUARD_BEGIN
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (colred_blocks < 1 || colred_blocks > (1 << 20))
        return fail(USTAT_E_INVALID, "colred_blocks must be in 1..2^20");
    plan->plan.tuning.gemm_big_min = gemm_big_min < 0 ? 0 : gemm_big_min;
    plan->plan.tuning.colred_blocks = colred_blocks;
    plan->rt.drop_graphs();
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_plan_autotune(ustat_plan plan, int64_t n, const void *const *factors,
                                 ustat_stream stream, int32_t reps, double *ms) {
    USTAT_GUARD_BEGIN
    ustat_status c = check_eval(plan, n);
    if (c != USTAT_OK) return c;
    if (!factors) return fail(USTAT_E_INVALID, "factors is NULL");
    if (reps < 1 || reps > 100) return fail(USTAT_E_INVALID, "reps must be in 1..100");
    std::vector<Dataset> data(1);
    data[0].n = n;
    data[0].symmetric = plan->plan.opts.symmetric;
    for (size_t k = 0; k < plan->plan.edges.size(); ++k) {
        if (!factors[k]) return fail(USTAT_E_INVALID, "a factor pointer is NULL");
        data[0].factors.push_back(factors[k]);
    }
    const std::string key = tune_key(plan, "single:n" + std::to_string(log2_bucket(n)));
    if (tune_cache_lookup(plan, key, ms)) return ok();
    hipStream_t s = (hipStream_t)stream;
    bool own = false;
    if (!s) {
        if (hipStreamCreate(&s) != hipSuccess) return fail(USTAT_E_HIP, "stream creation failed");
        own = true;
    }
    std::string gkey = "tune:" + std::to_string(n);
    for (auto f : data[0].factors) gkey += ":" + std::to_string((uintptr_t)f);
    double best_ms = 0;
    ustat_status st = tune_loop(plan, reps, [&]() {
        std::vector<DatasetResult> res;
        return run(plan, plan->all, data, s, res, nullptr, nullptr, gkey);
    }, &best_ms);
    if (own) (void)hipStreamDestroy(s);
    if (st != USTAT_OK) return st;
    tune_cache_store(plan, key, best_ms);
    if (ms) *ms = best_ms;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_plan_autotune_batched(ustat_plan plan, int32_t batch, const int64_t *n, int32_t d,
                                         const double *const *X, double rbf_divisor,
                                         ustat_stream stream, int32_t reps, double *ms) {
    USTAT_GUARD_BEGIN
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (batch < 1 || !n || !X || d < 1 || d > 256) return fail(USTAT_E_INVALID, "bad arguments");
    if (reps < 1 || reps > 100) return fail(USTAT_E_INVALID, "reps must be in 1..100");
    int64_t nmax = 0, ntot = 0;
    for (int b = 0; b < batch; ++b) {
        nmax = std::max(nmax, n[b]);
        ntot += n[b];
    }
    const std::string key = tune_key(plan, "batched:b" + std::to_string(batch) + ":n" +
                                               std::to_string(log2_bucket(nmax)) + ":t" +
                                               std::to_string(log2_bucket(ntot)) + ":d" + std::to_string(d));
    if (tune_cache_lookup(plan, key, ms)) return ok();
    std::vector<ustat_result> out(batch);
    double best_ms = 0;
    ustat_status st = tune_loop(plan, reps, [&]() {
        return ustat_eval_batched(plan, batch, n, d, X, rbf_divisor, stream, out.data());
    }, &best_ms);
    if (st != USTAT_OK) return st;
    tune_cache_store(plan, key, best_ms);
    if (ms) *ms = best_ms;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_eval(ustat_plan plan, int64_t n, const void *const *factors, ustat_stream stream,
                        ustat_result *out) {
    USTAT_GUARD_BEGIN
    ustat_status c = check_eval(plan, n);
    if (c != USTAT_OK) return c;
    if (!factors || !out) return fail(USTAT_E_INVALID, "factors and out must be non-NULL");
    std::vector<Dataset> data(1);
    data[0].n = n;
    data[0].symmetric = plan->plan.opts.symmetric;
    for (size_t k = 0; k < plan->plan.edges.size(); ++k) {
        if (!factors[k]) return fail(USTAT_E_INVALID, "a factor pointer is NULL");
        data[0].factors.push_back(factors[k]);
    }
    std::string key = "eval:" + std::to_string(n);
    for (auto f : data[0].factors) key += ":" + std::to_string((uintptr_t)f);
    std::vector<DatasetResult> res;
    ustat_status st = run(plan, plan->all, data, (hipStream_t)stream, res, nullptr, nullptr, key);
    if (st != USTAT_OK) return st;
    fill_result(out, res[0], plan->plan, n, (int)plan->all.size());
    return ok();
    USTAT_GUARD_END
}

}  // extern "C"

namespace {

// Table slot (1-based) of every panel F_0, G_0, F_1, G_1, ...: equal
// pointers (or equal caller ids) share a slot.
template <typename T>
std::vector<int> panel_slots(const std::vector<T> &ids) {
    std::vector<int> slot(ids.size());
    std::vector<T> seen;
    for (size_t k = 0; k < ids.size(); ++k) {
        auto it = std::find(seen.begin(), seen.end(), ids[k]);
        if (it == seen.end()) {
            seen.push_back(ids[k]);
            slot[k] = (int)seen.size();
        } else {
            slot[k] = (int)(it - seen.begin()) + 1;
        }
    }
    return slot;
}

ustat_status check_lowrank(ustat_plan plan, int64_t n, int32_t r) {
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (!plan->motifs.empty()) return fail(USTAT_E_INVALID, "motif plans take adjacency matrices");
    if (n < plan->plan.m) return fail(USTAT_E_INVALID, "n must be at least m");
    if (n > (1ll << 31)) return fail(USTAT_E_INVALID, "n above 2^31 is not supported");
    if (r < 1 || r > 4096) return fail(USTAT_E_INVALID, "r must be in 1..4096");
    if (plan->plan.opts.precision == USTAT_I8)
        return fail(USTAT_E_UNSUPPORTED, "the low-rank path is floating point (fp64)");
    return USTAT_OK;
}

// The schedule for (n, r, panel identity), built and uploaded on first use.
ustat_status lowrank_schedule(ustat_plan plan, int64_t n, int32_t r, const std::vector<int> &slots,
                              bool upload, LrSchedule **out) {
    std::string key = std::to_string(n) + ":" + std::to_string(r);
    for (int s : slots) key += ":" + std::to_string(s);
    auto it = plan->lowrank.find(key);
    if (it == plan->lowrank.end()) {
        std::unique_ptr<LrSchedule> s(new LrSchedule());
        std::string err = build_lowrank(plan->plan, n, r, slots, *s);
        if (!err.empty()) return fail(USTAT_E_UNSUPPORTED, err);
        it = plan->lowrank.emplace(key, std::move(s)).first;
    }
    LrSchedule &s = *it->second;
    const uint64_t lim = plan->plan.opts.workspace_limit;
    if (lim && (uint64_t)s.ws_elems * 8 > lim)
        return fail(USTAT_E_INFEASIBLE, "low-rank workspace of " + std::to_string(s.ws_elems * 8) +
                                            " bytes exceeds the workspace limit");
    if (upload) {
        hipError_t e = upload_lowrank(s);
        if (e == hipErrorOutOfMemory) return fail(USTAT_E_NOMEM, "low-rank descriptors: out of memory");
        if (e != hipSuccess) return fail(USTAT_E_HIP, std::string("low-rank descriptors: ") + hipGetErrorString(e));
    }
    *out = &s;
    return USTAT_OK;
}

}  // namespace

extern "C" {

ustat_status ustat_eval_lowrank(ustat_plan plan, int64_t n, int32_t r, const double *const *F,
                                const double *const *G, ustat_stream stream, ustat_result *out) {
    USTAT_GUARD_BEGIN
    ustat_status c = check_lowrank(plan, n, r);
    if (c != USTAT_OK) return c;
    if (!F || !G || !out) return fail(USTAT_E_INVALID, "F, G and out must be non-NULL");
    const size_t E = plan->plan.edges.size();
    std::vector<const double *> ptrs;
    for (size_t k = 0; k < E; ++k) {
        if (!F[k] || !G[k]) return fail(USTAT_E_INVALID, "a panel pointer is NULL");
        ptrs.push_back(F[k]);
        ptrs.push_back(G[k]);
    }
    const std::vector<int> slots = panel_slots(ptrs);
    LrSchedule *s = nullptr;
    c = lowrank_schedule(plan, n, r, slots, true, &s);
    if (c != USTAT_OK) return c;
    if (plan->rt.reserve_arena((size_t)s->ws_elems * 8 + 256) != hipSuccess ||
        plan->rt.reserve_hres(64) != hipSuccess)
        return fail(USTAT_E_NOMEM, "low-rank workspace: out of memory");
    std::vector<const double *> tab(s->nslots - 1, nullptr);
    for (size_t k = 0; k < ptrs.size(); ++k) tab[slots[k] - 1] = ptrs[k];
    double *hres = (double *)plan->rt.hres;
    hipError_t e = run_lowrank(*s, tab.data(), (double *)plan->rt.arena, (hipStream_t)stream, hres);
    if (e != hipSuccess) return fail(USTAT_E_HIP, std::string("low-rank evaluation: ") + hipGetErrorString(e));
    std::memset(out, 0, sizeof *out);
    out->value = hres[0];
    out->err_scale = hres[1];
    out->err_est = error_estimate(0, n, s->depth, false);
    out->num_vstats = s->nparts;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_lowrank_info(ustat_plan plan, int64_t n, int32_t r, const int32_t *panel_ids,
                                ustat_lowrank_stats *out) {
    USTAT_GUARD_BEGIN
    ustat_status c = check_lowrank(plan, n, r);
    if (c != USTAT_OK) return c;
    if (!out) return fail(USTAT_E_INVALID, "out is NULL");
    const size_t E2 = 2 * plan->plan.edges.size();
    std::vector<int32_t> ids(E2);
    for (size_t k = 0; k < E2; ++k) ids[k] = panel_ids ? panel_ids[k] : (int32_t)k;
    LrSchedule *s = nullptr;
    c = lowrank_schedule(plan, n, r, panel_slots(ids), false, &s);
    if (c != USTAT_OK && c != USTAT_E_INFEASIBLE) return c;
    if (!s) {
        // over the workspace limit: still report the schedule
        std::string key = std::to_string(n) + ":" + std::to_string(r);
        for (int q : panel_slots(ids)) key += ":" + std::to_string(q);
        s = plan->lowrank.at(key).get();
    }
    std::memset(out, 0, sizeof *out);
    out->madds = s->flops;
    out->madds_unmerged = s->flops_unmerged;
    out->workspace_bytes = s->ws_elems * 8;
    out->num_partitions = s->nparts;
    out->num_steps = (int32_t)(s->steps.size() + s->krs.size());
    out->depth = s->depth;
    out->num_exact_orders = s->ndp;
    out->num_greedy_orders = s->ngreedy;
    out->num_gemm_steps = (int32_t)s->krs.size();
    return ok();
    USTAT_GUARD_END
}

}  // extern "C"

// Fixed device buffer of ustat_eval_noalloc: every evaluation through that
// entry point takes its workspace, descriptors and accumulators from here.
// Each device the library runs on holds its own copy from the moment the
// code object is loaded there until the process ends.
static __device__ __align__(256) char scratch[USTAT_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.  Host code
// never uses the array's own name (a host-side stand-in): the address is
// looked up once per device, with that device current, and kept.
hipError_t scratch_address(char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

ustat_status ustat_eval_noalloc(ustat_plan plan, int64_t n, const void *const *factors,
                                ustat_stream stream, ustat_result *out) {
    USTAT_GUARD_BEGIN
    ustat_status c = check_eval(plan, n);
    if (c != USTAT_OK) return c;
    if (!factors || !out) return fail(USTAT_E_INVALID, "factors and out must be non-NULL");
    try {
        std::vector<Dataset> data(1);
        data[0].n = n;
        data[0].symmetric = plan->plan.opts.symmetric;
        for (size_t k = 0; k < plan->plan.edges.size(); ++k) {
            if (!factors[k]) return fail(USTAT_E_INVALID, "a factor pointer is NULL");
            data[0].factors.push_back(factors[k]);
        }
        ExtMem ext;
        hipError_t e = scratch_address(&ext.base);
        if (e != hipSuccess)
            return fail(USTAT_E_HIP, std::string("fixed device buffer: ") + hipGetErrorString(e));
        ext.bytes = USTAT_NOALLOC_MAX_BYTES;
        std::vector<DatasetResult> res;
        ustat_status st = run(plan, plan->all, data, (hipStream_t)stream, res, nullptr, nullptr, "", &ext);
        if (st != USTAT_OK) return st;
        fill_result(out, res[0], plan->plan, n, (int)plan->all.size());
        return ok();
    } catch (const std::bad_alloc &) {
        return fail(USTAT_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(USTAT_E_INVALID, "unexpected host exception");
    }
    USTAT_GUARD_END
}

ustat_status ustat_build_rbf(int64_t n, int32_t d, const double *X, double rbf_divisor,
                             int32_t precision, void *out, ustat_stream stream) {
    USTAT_GUARD_BEGIN
    if (n < 1 || d < 1 || d > 256 || !X || !out) return fail(USTAT_E_INVALID, "bad arguments");
    if (!(rbf_divisor > 0) || !std::isfinite(rbf_divisor))
        return fail(USTAT_E_INVALID, "rbf_divisor must be positive");
    if (precision != USTAT_F64 && precision != USTAT_F32)
        return fail(USTAT_E_INVALID, "precision must be USTAT_F64 or USTAT_F32");
    hipError_t e = launch_rbf(X, n, d, rbf_divisor, out, precision == USTAT_F64 ? DT_F64 : DT_F32,
                              (hipStream_t)stream);
    if (e != hipSuccess) return fail(USTAT_E_HIP, hipGetErrorString(e));
    return ok();
    USTAT_GUARD_END
}

}  // extern "C"

namespace {

// Times one launch of a peak microbenchmark with HIP events on `s` (after
// one untimed launch), returning seconds.
template <class L>
hipError_t time_launch(hipStream_t s, L &&launch, double *sec) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(a, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    *sec = ms * 1e-3;
    return e;
}

hipError_t compute_units(int *cu) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(cu, hipDeviceAttributeMultiprocessorCount, dev);
    return e;
}

}  // namespace

extern "C" {

ustat_status ustat_peak_mfma(int32_t kind, int64_t iters, void *sink, ustat_stream stream,
                             double *rate) {
    USTAT_GUARD_BEGIN
    if (kind < 0 || kind > 3 || iters < 1 || iters > (int64_t)1 << 32 || !sink || !rate)
        return fail(USTAT_E_INVALID, "bad arguments");
    int cu = 0;
    hipError_t e = compute_units(&cu);
    if (e != hipSuccess) return fail(USTAT_E_HIP, hipGetErrorString(e));
    double flops = 0, sec = 0;
    e = time_launch((hipStream_t)stream, [&] {
        return launch_peak_mfma(kind, 2 * cu, iters, static_cast<char *>(sink), (hipStream_t)stream, &flops);
    }, &sec);
    if (e != hipSuccess) return fail(USTAT_E_HIP, hipGetErrorString(e));
    *rate = sec > 0 ? flops / sec : 0.0;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_peak_copy(const void *src, void *dst, int64_t bytes, ustat_stream stream,
                             double *rate) {
    USTAT_GUARD_BEGIN
    if (!src || !dst || !rate || bytes < 16 || bytes % 16 != 0)
        return fail(USTAT_E_INVALID, "bad arguments");
    int cu = 0;
    hipError_t e = compute_units(&cu);
    if (e != hipSuccess) return fail(USTAT_E_HIP, hipGetErrorString(e));
    double sec = 0;
    e = time_launch((hipStream_t)stream, [&] {
        return launch_peak_copy(src, dst, bytes, 8 * cu, (hipStream_t)stream);
    }, &sec);
    if (e != hipSuccess) return fail(USTAT_E_HIP, hipGetErrorString(e));
    *rate = sec > 0 ? 2.0 * (double)bytes / sec : 0.0;
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_eval_samples(ustat_plan plan, int64_t n, int32_t d, const double *X,
                                double rbf_divisor, ustat_stream stream, ustat_result *out) {
    USTAT_GUARD_BEGIN
    ustat_status c = check_eval(plan, n);
    if (c != USTAT_OK) return c;
    if (d < 1 || d > 256 || !X || !out) return fail(USTAT_E_INVALID, "bad arguments");
    if (!(rbf_divisor > 0) || !std::isfinite(rbf_divisor))
        return fail(USTAT_E_INVALID, "rbf_divisor must be positive");
    if (plan->plan.opts.precision == USTAT_I8)
        return fail(USTAT_E_INVALID, "samples with an RBF kernel need a floating-point precision");
    const int dt = plan->plan.opts.precision == USTAT_F64 ? DT_F64 : DT_F32;
    const size_t es = dt == DT_F64 ? 8 : 4;
    // the factor and, when a GEMM reads it alone, its operand form behind it
    const int opf = factor_operand_format(plan->plan, n, true);
    const size_t kb = ((size_t)n * n * es + 255) / 256 * 256;
    hipError_t e = grow(&plan->factors, &plan->factors_bytes, kb + factor_operand_bytes(opf, n), &plan->rt);
    if (e != hipSuccess) return fail(USTAT_E_NOMEM, hipGetErrorString(e));
    std::vector<Dataset> data(1);
    data[0].n = n;
    data[0].symmetric = true;  // the RBF factor is symmetric bit for bit
    data[0].nonneg = true;     // and positive
    for (size_t k = 0; k < plan->plan.edges.size(); ++k) data[0].factors.push_back(plan->factors);
    char *fb = plan->factors;
    char *ob = opf >= 0 ? plan->factors + kb : nullptr;
    data[0].operand = ob;
    data[0].operand_format = opf;
    auto pre = [=](hipStream_t s) -> hipError_t {
        ProfScope ps(Profiler::active(), KIND_RBF, s, 0);
        return launch_rbf(X, n, d, rbf_divisor, fb, dt, s, ob, opf);
    };
    std::string key = "samples:" + std::to_string(n) + ":" + std::to_string(d) + ":" +
                      std::to_string((uintptr_t)X) + ":" + std::to_string(rbf_divisor) + ":" +
                      std::to_string((uintptr_t)fb);
    std::vector<DatasetResult> res;
    ustat_status st = run(plan, plan->all, data, (hipStream_t)stream, res, nullptr, pre, key);
    if (st != USTAT_OK) return st;
    fill_result(out, res[0], plan->plan, n, (int)plan->all.size());
    return ok();
    USTAT_GUARD_END
}

ustat_status vstat_eval(ustat_plan plan, const int32_t *block_of, int64_t n,
                        const void *const *factors, ustat_stream stream, ustat_result *out) {
    USTAT_GUARD_BEGIN
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (!block_of || !factors || !out) return fail(USTAT_E_INVALID, "NULL argument");
    if (n < 1 || n > (1ll << 20)) return fail(USTAT_E_INVALID, "n out of range");
    for (size_t k = 0; k < plan->plan.edges.size(); ++k)
        if (!factors[k]) return fail(USTAT_E_INVALID, "a factor pointer is NULL");
    std::vector<int> rgs;
    canonical_rgs(block_of, plan->plan.m, rgs);
    VProgram prog;
    std::string err;
    try {
        err = build_program(plan->plan.edges, plan->plan.m, rgs, plan->plan.opts,
                            plan->model.get(), prog);
    } catch (const std::bad_alloc &) {
        return fail(USTAT_E_NOMEM, "host allocation failed");
    }
    if (!err.empty()) return fail(USTAT_E_INVALID, err);
    if (!prog.executable) return fail(USTAT_E_UNSUPPORTED, prog.lower_error);
    prog.mu = 1;  // the combination then returns V_pi itself
    Plan sub = plan->plan;
    sub.opts.sparsify = plan->plan.opts.sparsify;
    std::vector<Dataset> data(1);
    data[0].n = n;
    data[0].symmetric = plan->plan.opts.symmetric;
    for (size_t k = 0; k < plan->plan.edges.size(); ++k) data[0].factors.push_back(factors[k]);
    std::vector<DatasetResult> res;
    std::vector<const VProgram *> progs = {&prog};
    ustat_status st = run(plan, progs, data, (hipStream_t)stream, res, nullptr, nullptr, "");
    if (st != USTAT_OK) return st;
    fill_result(out, res[0], plan->plan, n, 1);
    out->err_scale = std::fabs(res[0].value);
    return ok();
    USTAT_GUARD_END
}

static ustat_status lower_given(ustat_plan plan, const int32_t *block_of, const int32_t *order,
                                int32_t len, int32_t slice_var, VProgram &prog) {
    if (!plan || !block_of || (!order && len > 0)) return fail(USTAT_E_INVALID, "NULL argument");
    std::vector<int> rgs;
    canonical_rgs(block_of, plan->plan.m, rgs);
    int J = 0;
    for (int b : rgs) J = std::max(J, b + 1);
    if (slice_var < -1 || slice_var >= J) return fail(USTAT_E_INVALID, "slice_var out of range");
    const int want = slice_var >= 0 ? J - 1 : J;
    if (len != want)
        return fail(USTAT_E_INVALID, "order must list every block (but the conditioned one)");
    std::vector<int> ord(order, order + len), chk = ord;
    if (slice_var >= 0) chk.push_back(slice_var);
    std::sort(chk.begin(), chk.end());
    for (int i = 0; i < J; ++i)
        if (chk[i] != i) return fail(USTAT_E_INVALID, "order is not a permutation of the blocks");
    prog.block_of = rgs;
    prog.J = J;
    prog.mu = mobius_mu(rgs);
    std::string err = lower_order(plan->plan.edges, rgs, J, ord, prog, slice_var);
    if (!err.empty()) return fail(USTAT_E_UNSUPPORTED, err);
    return USTAT_OK;
}

ustat_status ustat_order_features(ustat_plan plan, const int32_t *block_of, const int32_t *order,
                                  int32_t len, int32_t slice_var, int64_t n, float *feat) {
    USTAT_GUARD_BEGIN
    if (!feat || n < 1) return fail(USTAT_E_INVALID, "bad arguments");
    VProgram prog;
    ustat_status st = lower_given(plan, block_of, order, len, slice_var, prog);
    if (st != USTAT_OK) return st;
    std::vector<float> f = program_features(prog, (double)n);
    if ((int)f.size() != USTAT_NUM_FEATURES) return fail(USTAT_E_INVALID, "feature size mismatch");
    std::copy(f.begin(), f.end(), feat);
    return ok();
    USTAT_GUARD_END
}

ustat_status vstat_eval_ordered(ustat_plan plan, const int32_t *block_of, const int32_t *order,
                                int32_t len, int32_t slice_var, int64_t n,
                                const void *const *factors, ustat_stream stream,
                                ustat_result *out) {
    USTAT_GUARD_BEGIN
    if (!factors || !out) return fail(USTAT_E_INVALID, "NULL argument");
    if (n < 1 || n > (1ll << 20)) return fail(USTAT_E_INVALID, "n out of range");
    VProgram prog;
    ustat_status st = lower_given(plan, block_of, order, len, slice_var, prog);
    if (st != USTAT_OK) return st;
    for (size_t k = 0; k < plan->plan.edges.size(); ++k)
        if (!factors[k]) return fail(USTAT_E_INVALID, "a factor pointer is NULL");
    prog.mu = 1;
    std::vector<Dataset> data(1);
    data[0].n = n;
    data[0].symmetric = plan->plan.opts.symmetric;
    for (size_t k = 0; k < plan->plan.edges.size(); ++k) data[0].factors.push_back(factors[k]);
    std::vector<DatasetResult> res;
    std::vector<const VProgram *> progs = {&prog};
    st = run(plan, progs, data, (hipStream_t)stream, res, nullptr, nullptr, "");
    if (st != USTAT_OK) return st;
    fill_result(out, res[0], plan->plan, n, 1);
    out->err_scale = std::fabs(res[0].value);
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_eval_batched(ustat_plan plan, int32_t batch, const int64_t *n, int32_t d,
                                const double *const *X, double rbf_divisor, ustat_stream stream,
                                ustat_result *out) {
    USTAT_GUARD_BEGIN
    if (!plan) return fail(USTAT_E_INVALID, "plan is NULL");
    if (batch < 1 || !n || !X || !out || d < 1 || d > 256)
        return fail(USTAT_E_INVALID, "bad arguments");
    if (!(rbf_divisor > 0) || !std::isfinite(rbf_divisor))
        return fail(USTAT_E_INVALID, "rbf_divisor must be positive");
    if (plan->plan.opts.precision == USTAT_I8)
        return fail(USTAT_E_INVALID, "samples with an RBF kernel need a floating-point precision");
    for (int b = 0; b < batch; ++b) {
        ustat_status c = check_eval(plan, n[b]);
        if (c != USTAT_OK) return c;
        if (!X[b]) return fail(USTAT_E_INVALID, "a sample pointer is NULL");
    }
    const int dt = plan->plan.opts.precision == USTAT_F64 ? DT_F64 : DT_F32;
    const size_t es = dt == DT_F64 ? 8 : 4;
    // per dataset: the factor and, when a GEMM reads it alone, its operand
    // form behind it
    auto kbytes = [&](int64_t nn) { return ((size_t)nn * nn * es + 255) / 256 * 256; };
    auto opfmt = [&](int64_t nn) { return factor_operand_format(plan->plan, nn, true); };
    auto fbytes = [&](int64_t nn) {
        return kbytes(nn) + (factor_operand_bytes(opfmt(nn), nn) + 255) / 256 * 256;
    };
    // Split the batch into chunks whose factor matrices and workspace fit
    // the budget: opts.workspace_limit, else half of the free device memory
    // (counting the buffers this plan already holds as free).
    size_t budget = plan->plan.opts.workspace_limit;
    if (!budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(USTAT_E_HIP, "hipMemGetInfo failed");
        budget = (fr + plan->rt.arena_bytes + plan->factors_bytes) / 2;
    }
    std::map<int64_t, size_t> ws_one;
    auto per_dataset = [&](int64_t nn) {
        auto it = ws_one.find(nn);
        if (it != ws_one.end()) return it->second;
        size_t w = workspace_bytes(plan->plan, plan->all, {nn}, true) + fbytes(nn);
        ws_one[nn] = w;
        return w;
    };
    std::vector<std::pair<int, int>> chunks;  // [begin, end)
    {
        int b0 = 0;
        size_t acc = 0;
        for (int b = 0; b < batch; ++b) {
            size_t w = per_dataset(n[b]);
            if (b > b0 && acc + w > budget) {
                chunks.push_back({b0, b});
                b0 = b;
                acc = 0;
            }
            acc += w;
        }
        chunks.push_back({b0, batch});
    }
    // Sizes of every chunk, so that all buffers are reserved once and the
    // graphs captured for the chunks stay valid across calls.
    size_t max_f = 0, max_arena = 0, max_blob = 0, max_res = 0;
    std::vector<std::vector<Dataset>> cdata(chunks.size());
    std::vector<std::vector<size_t>> coff(chunks.size());
    for (size_t c = 0; c < chunks.size(); ++c) {
        size_t tot = 0;
        for (int b = chunks[c].first; b < chunks[c].second; ++b) {
            coff[c].push_back(tot);
            tot += fbytes(n[b]);
        }
        max_f = std::max(max_f, tot);
    }
    hipError_t e = grow(&plan->factors, &plan->factors_bytes, max_f, &plan->rt);
    if (e != hipSuccess) return fail(USTAT_E_NOMEM, hipGetErrorString(e));
    for (size_t c = 0; c < chunks.size(); ++c) {
        for (int b = chunks[c].first, i = 0; b < chunks[c].second; ++b, ++i) {
            Dataset ds;
            ds.n = n[b];
            ds.symmetric = true;  // RBF factors: symmetric and positive
            ds.nonneg = true;
            for (size_t k = 0; k < plan->plan.edges.size(); ++k)
                ds.factors.push_back(plan->factors + coff[c][i]);
            ds.operand_format = opfmt(n[b]);
            ds.operand = ds.operand_format >= 0 ? plan->factors + coff[c][i] + kbytes(n[b]) : nullptr;
            cdata[c].push_back(ds);
        }
        ScheduleSizes z = schedule_sizes(plan->plan, plan->all, cdata[c]);
        max_arena = std::max(max_arena, z.arena);
        max_blob = std::max(max_blob, z.blob);
        max_res = std::max(max_res, z.results);
    }
    if ((e = plan->rt.reserve_arena(max_arena)) != hipSuccess)
        return fail(USTAT_E_NOMEM, std::string("device workspace allocation failed: ") + hipGetErrorString(e));
    if ((e = plan->rt.reserve_desc(max_blob + 1024)) != hipSuccess) return fail(USTAT_E_NOMEM, hipGetErrorString(e));
    if ((e = plan->rt.reserve_hres(max_res + 64)) != hipSuccess) return fail(USTAT_E_NOMEM, hipGetErrorString(e));
    for (size_t c = 0; c < chunks.size(); ++c) {
        const int b0 = chunks[c].first, b1 = chunks[c].second;
        std::string key = "batch:" + std::to_string(d) + ":" + std::to_string(rbf_divisor) + ":" +
                          std::to_string((uintptr_t)plan->factors);
        for (int b = b0; b < b1; ++b)
            key += ":" + std::to_string(n[b]) + "@" + std::to_string((uintptr_t)X[b]);
        std::vector<const double *> xs(X + b0, X + b1);
        std::vector<int64_t> ns(n + b0, n + b1);
        std::vector<char *> fps;
        std::vector<void *> ops;
        std::vector<int> opfs;
        for (size_t i = 0; i < ns.size(); ++i) {
            fps.push_back(plan->factors + coff[c][i]);
            ops.push_back(const_cast<void *>(cdata[c][i].operand));
            opfs.push_back(cdata[c][i].operand_format);
        }
        auto pre = [=](hipStream_t s) -> hipError_t {
            for (size_t i = 0; i < xs.size(); ++i) {
                hipError_t e2 = launch_rbf(xs[i], ns[i], d, rbf_divisor, fps[i], dt, s, ops[i], opfs[i]);
                if (e2 != hipSuccess) return e2;
            }
            return hipSuccess;
        };
        std::vector<DatasetResult> res;
        ustat_status st = run(plan, plan->all, cdata[c], (hipStream_t)stream, res, nullptr, pre, key);
        if (st != USTAT_OK) return st;
        for (int b = b0; b < b1; ++b)
            fill_result(&out[b], res[b - b0], plan->plan, n[b], (int)plan->all.size());
    }
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_profile_enable(int32_t on) {
    USTAT_GUARD_BEGIN
    Profiler::enable(on != 0);
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_profile_reset(void) {
    USTAT_GUARD_BEGIN
    Profiler::enable(true);
    if (Profiler::active()) Profiler::active()->reset();
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_profile_read(int32_t kind, double *ms, int64_t *launches, double *flops,
                                double *bytes) {
    USTAT_GUARD_BEGIN
    if (kind < 0 || kind >= KIND_COUNT) return fail(USTAT_E_INVALID, "unknown kind");
    Profiler *p = Profiler::active();
    if (!p) return fail(USTAT_E_INVALID, "profiling is not enabled");
    if (ms) *ms = p->ms[kind];
    if (launches) *launches = p->launches[kind];
    if (flops) *flops = p->flops[kind];
    if (bytes) *bytes = p->bytes[kind];
    return ok();
    USTAT_GUARD_END
}

}  // extern "C"

namespace {

// The motif kernels of the motif application: the complete graph on 3 or 4
// vertices, with factor A (an edge of the motif) or B = 1 - A (a non-edge)
// on every vertex pair, and the motif's automorphism count.  Order: V-shape,
// triangle; 3-star, path, tailed triangle, square, diamond, K4.
struct MotifKernel {
    std::vector<int> on_a;  // per pair: 1 reads A, 0 reads B
    int64_t aut;
};

const std::vector<Edge> &motif_pairs(int size) {
    static const std::vector<Edge> p3 = {{0, 1}, {1, 2}, {2, 0}};
    static const std::vector<Edge> p4 = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    return size == 3 ? p3 : p4;
}

const std::vector<MotifKernel> &motif_kernels(int size) {
    static const std::vector<MotifKernel> m3 = {{{1, 1, 0}, 2}, {{1, 1, 1}, 6}};
    static const std::vector<MotifKernel> m4 = {{{1, 1, 1, 0, 0, 0}, 6}, {{1, 0, 0, 1, 0, 1}, 2},
                                                {{1, 1, 0, 1, 0, 1}, 2}, {{1, 0, 1, 1, 0, 1}, 8},
                                                {{1, 1, 1, 1, 1, 0}, 4}, {{1, 1, 1, 1, 1, 1}, 24}};
    return size == 3 ? m3 : m4;
}

}  // namespace

extern "C" {

ustat_status ustat_plan_create_motifs(int32_t size, const ustat_plan_opts *opts, ustat_plan *out) {
    USTAT_GUARD_BEGIN
    if (!out) return fail(USTAT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (size != 3 && size != 4) return fail(USTAT_E_INVALID, "motif size must be 3 or 4");
    ustat_plan_opts o;
    ustat_plan_opts_default(&o);
    if (opts) o = *opts;
    if (o.order < 0 || o.order > 1) return fail(USTAT_E_INVALID, "order policy must be min-fill or exhaustive");
    if (o.flags & ~(USTAT_FLAG_NO_CSE | USTAT_FLAG_SYMMETRIC | USTAT_FLAG_NO_SYM_GEMM |
                    USTAT_FLAG_OVERLAP_LEVELS))
        return fail(USTAT_E_INVALID, "unknown flag bits");
    std::unique_ptr<ustat_plan_s> p(new ustat_plan_s());
    PlanOptions po;
    po.precision = USTAT_I8;  // exact counts
    po.order = o.order;
    po.sparsify = 1;          // Lemma 3: only the finest partition of a complete graph survives
    po.workspace_limit = o.workspace_limit;
    if (o.n_hint < 0 || o.n_hint > (1ll << 20)) return fail(USTAT_E_INVALID, "n_hint out of range");
    if (o.n_hint > 0) po.n_hint = (double)o.n_hint;
    po.cse = !(o.flags & USTAT_FLAG_NO_CSE);
    po.symmetric = true;      // A and B are symmetric
    po.sym_gemm = !(o.flags & USTAT_FLAG_NO_SYM_GEMM);
    po.overlap = (o.flags & USTAT_FLAG_OVERLAP_LEVELS) != 0;
    for (const MotifKernel &mo : motif_kernels(size)) {
        Plan pl;
        std::string err = make_plan(size, motif_pairs(size), po, nullptr, pl);
        if (!err.empty()) return fail(USTAT_E_INVALID, err);
        p->motifs.push_back(std::move(pl));
        p->motif_aut.push_back(mo.aut);
    }
    p->motif_size = size;
    p->plan = p->motifs[0];
    for (auto &pr : p->plan.progs) p->all.push_back(&pr);
    *out = p.release();
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_motif_counts(ustat_plan plan, int64_t n, const int8_t *A, ustat_stream stream,
                                int64_t *counts) {
    USTAT_GUARD_BEGIN
    if (!plan || !plan->motif_size) return fail(USTAT_E_INVALID, "not a motif plan");
    if (!A || !counts) return fail(USTAT_E_INVALID, "A and counts must be non-NULL");
    if (n < plan->motif_size || n > (1ll << 20)) return fail(USTAT_E_INVALID, "n out of range");
    const int size = plan->motif_size;
    hipStream_t s = (hipStream_t)stream;
    // B = 1 - A off the diagonal (0 on it), and a check that A is a
    // symmetric 0/1 matrix with a zero diagonal
    hipError_t e = grow(&plan->factors, &plan->factors_bytes, (size_t)n * n + 256, &plan->rt);
    if (e != hipSuccess) return fail(USTAT_E_NOMEM, hipGetErrorString(e));
    int8_t *B = reinterpret_cast<int8_t *>(plan->factors);
    unsigned int bad = 0;
    e = launch_motif_complement(A, B, n, reinterpret_cast<unsigned int *>(plan->factors + (size_t)n * n), &bad, s);
    if (e != hipSuccess) return fail(USTAT_E_HIP, hipGetErrorString(e));
    if (bad) return fail(USTAT_E_INVALID, "A is not a symmetric 0/1 adjacency with a zero diagonal");
    // one dataset per motif, all reading A and B: equal steps of different
    // motifs are computed once
    const std::vector<MotifKernel> &kern = motif_kernels(size);
    std::vector<Dataset> data(plan->motifs.size());
    std::vector<std::vector<const VProgram *>> progs(plan->motifs.size());
    for (size_t r = 0; r < plan->motifs.size(); ++r) {
        data[r].n = n;
        data[r].symmetric = true;
        data[r].nonneg = true;
        for (int a : kern[r].on_a) data[r].factors.push_back(a ? (const void *)A : (const void *)B);
        for (auto &pr : plan->motifs[r].progs) data[r].progs.push_back(&pr);
    }
    std::vector<DatasetResult> res;
    ustat_status st = run(plan, plan->all, data, s, res, nullptr, nullptr, "");
    if (st != USTAT_OK) return st;
    for (size_t r = 0; r < res.size(); ++r) {
        const __int128 u = ((__int128)res[r].exact_hi << 64) | (__int128)res[r].exact_lo;
        const int64_t aut = plan->motif_aut[r];
        if (u < 0 || u % aut != 0) return fail(USTAT_E_HIP, "motif sum not divisible by its automorphisms");
        counts[r] = (int64_t)(u / aut);
    }
    return ok();
    USTAT_GUARD_END
}

ustat_status ustat_debug_inject(int32_t kind, int64_t countdown) {
    if (kind < 0 || kind >= INJ_KINDS) return fail(USTAT_E_INVALID, "unknown failure kind");
    inject_arm(kind, countdown);
    return ok();
}

const char *ustat_status_string(ustat_status s) {
    switch (s) {
        case USTAT_OK: return "ok";
        case USTAT_E_INVALID: return "invalid argument";
        case USTAT_E_UNSUPPORTED: return "unsupported";
        case USTAT_E_NOMEM: return "out of memory";
        case USTAT_E_HIP: return "HIP runtime error";
        case USTAT_E_OVERFLOW: return "exact integer overflow";
        case USTAT_E_INFEASIBLE: return "workspace above limit";
    }
    return "unknown status";
}

const char *ustat_last_error(void) { return g_err.c_str(); }

}  // extern "C"
