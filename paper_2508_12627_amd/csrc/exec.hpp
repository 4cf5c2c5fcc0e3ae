// Executor: lowers the programs of a plan, for one or many datasets, to
// grouped kernel launches ordered by dependency level.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "plan.hpp"

namespace ustat {

struct Dataset {
    int64_t n = 0;
    std::vector<const void *> factors;  // one device pointer per edge
    bool symmetric = false;             // every factor matrix is symmetric
    // every factor entry is known to be >= 0 (the RBF factors the engine
    // builds); otherwise split-bf16 plans scan the factors for signs
    bool nonneg = false;
    // the GEMM-operand form of factors[0] (every edge's factor, in the
    // sample entry points) in prep format operand_format, written with the
    // factor; GEMM operands that are that factor alone then need no prep
    const void *operand = nullptr;
    int operand_format = -1;
    // programs of this dataset when non-empty (their input values index
    // `factors`), otherwise the programs the evaluation is called with;
    // datasets with their own programs let one evaluation serve several
    // kernels on shared inputs, with equal steps merged across them
    std::vector<const VProgram *> progs;
};

// The programs dataset d evaluates.
inline const std::vector<const VProgram *> &progs_of(const std::vector<const VProgram *> &progs,
                                                      const Dataset &d) {
    return d.progs.empty() ? progs : d.progs;
}

// Prep format in which a GEMM of the plan reads the shared factor of a
// dataset of size n on its own (no vectors, no other matrices), or -1 when
// none does; the sample entry points then write that form with the factor.
int factor_operand_format(const Plan &plan, int64_t n, bool nonneg);
// Bytes of that operand form at size n.
size_t factor_operand_bytes(int format, int64_t n);

struct DatasetResult {
    double value = 0, scale = 0;
    int64_t exact_hi = 0;
    uint64_t exact_lo = 0;
    double err_est = 0;  // estimate of |value - exact| / scale (0 when exact)
};

// Estimate of |U - U_exact| / S for an evaluation at size n whose deepest
// program has `depth` dependency levels, under the probabilistic model of
// rounding errors (independent with mean zero): see exec.cpp.
double error_estimate(int precision, int64_t n, int depth, bool two_plane);

// Device and pinned-host memory owned by a plan, grown on demand and reused
// across evaluations.
struct Runtime {
    int device = -1;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    char *ddesc = nullptr;  // device copy of the descriptor blob
    size_t ddesc_bytes = 0;
    char *hdesc = nullptr;  // pinned host descriptor blob
    size_t hdesc_bytes = 0;
    char *hres = nullptr;   // pinned host result buffer
    size_t hres_bytes = 0;
    char *vacc = nullptr;   // device accumulators of V_pi across slice chunks
    size_t vacc_bytes = 0;
    // Captured graphs by key, each with its own pinned descriptor blob and
    // result layout.  Any reallocation of the buffers they reference drops
    // them all.
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        char *blob = nullptr;   // device descriptor blob read by the graph
        size_t blob_bytes = 0;
        int nd = 0, nprog = 0;
        std::vector<double> err_est;  // per dataset
        // exact path: the input maxima the graph copies from the pinned
        // staging buffer at this offset (rewritten there before a replay)
        std::vector<unsigned long long> inmx;
        size_t inmx_off = 0;
    };
    std::map<std::string, GraphEntry> graphs;
    // Second stream (default priority, not blocking on the null stream) for
    // the reductions that run beside a level's GEMMs, and a fork and a join
    // event per level; created on first use on the runtime's device.
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> level_events;
    hipError_t reserve_side(size_t levels);
    void drop_graphs();
    ~Runtime();
    hipError_t reserve_arena(size_t bytes);
    hipError_t reserve_desc(size_t bytes);
    hipError_t reserve_hres(size_t bytes);
    hipError_t reserve_vacc(size_t bytes);
};

// Optional per-launch timing, filled when non-null (milliseconds per step
// kind, measured with HIP events on the launch stream).
struct LaunchStats {
    double ms_prep = 0, ms_gemm = 0, ms_elim1 = 0, ms_reduce = 0, ms_other = 0;
    int n_launch = 0;
    double gemm_flops = 0;  // algorithmic (2 n^3 per GEMM)
};

// Evaluate programs `progs` (indices into plan.progs, or the explicit
// programs in `extra` when non-empty) on every dataset.  The factor
// matrices of each dataset must be ready on `stream`.  Results per dataset
// and, when vout is non-null, every V_pi (dataset-major).
// Returns "" or an error message; *status receives a ustat_status code.
// One pass over slices [slice_lo, slice_hi) of the programs conditioned on
// a vertex (and over the unconditioned programs when include_unsliced);
// `first` starts the V accumulators, `last` forms U and S.
struct SliceRange {
    int64_t lo = 0, hi = INT64_MAX;
    bool include_unsliced = true, first = true, last = true;
};

// Device memory an evaluation may use instead of the runtime's own buffers
// (the entry point that allocates nothing).  With it, the workspace, the
// descriptor blob and the per-program accumulators are carved out of
// [base, base + bytes): the accumulators at the end (they persist across
// slice chunks), the rest from the start; nothing is captured as a graph and
// results come back through ordinary host memory.  An evaluation that does
// not fit fails with status 6 before any launch.
struct ExtMem {
    char *base = nullptr;
    size_t bytes = 0;
};

std::string execute(const Plan &plan, const std::vector<const VProgram *> &progs,
                    const std::vector<Dataset> &data, hipStream_t stream, Runtime &rt,
                    std::vector<DatasetResult> &out, std::vector<double> *vout, int *status,
                    bool capture = false, const std::string &capture_key = "",
                    const std::function<hipError_t(hipStream_t)> &pre = nullptr,
                    const SliceRange &range = SliceRange(), const ExtMem *ext = nullptr);

// Whole evaluation: programs conditioned on a vertex run in slice chunks
// sized to the workspace budget (no graph capture); otherwise one pass.
std::string execute_all(const Plan &plan, const std::vector<const VProgram *> &progs,
                        const std::vector<Dataset> &data, hipStream_t stream, Runtime &rt,
                        std::vector<DatasetResult> &out, std::vector<double> *vout, int *status,
                        bool capture, const std::string &capture_key,
                        const std::function<hipError_t(hipStream_t)> &pre,
                        const ExtMem *ext = nullptr);

// Sizes an evaluation of `data` needs: arena, descriptor blob, pinned
// result bytes (a dry schedule; pointers only fix the sharing pattern).
struct ScheduleSizes {
    size_t arena = 0, blob = 0, results = 0;
};
ScheduleSizes schedule_sizes(const Plan &plan, const std::vector<const VProgram *> &progs,
                             const std::vector<Dataset> &data, const SliceRange &range = SliceRange());

// Upper bound of the workspace bytes an evaluation at size n needs.
// *status (may be null) receives the dry schedule's ustat_status code: 0,
// or e.g. 5 when an exact intermediate's a-priori bound (from inputs of
// magnitude up to 127) may overflow; the bytes are 0 then.
size_t workspace_bytes(const Plan &plan, const std::vector<const VProgram *> &progs,
                       const std::vector<int64_t> &ns, bool shared_factor, int *status = nullptr);

}  // namespace ustat
