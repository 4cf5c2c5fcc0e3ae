// Host-side planner: partitions, Moebius coefficients, quotient multigraphs,
// elimination orders and their lowering to kernel steps.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ustat {

constexpr int kMaxM = 10;

struct Edge {
    int u, v;
};

// A value flowing through one restricted V-statistic's elimination.
enum class ValKind : uint8_t {
    InputMat,   // factor matrix `src` of the kernel, rows indexed by var r
    InputDiag,  // diagonal of factor matrix `src` (a self-loop of the quotient)
    Vec,        // n-vector over quotient var `r`, produced by step `src`
    Mat,        // n x n matrix, rows var r, columns var c, produced by step `src`
    Scalar,     // produced by step `src`
    SliceVec    // slice i of factor matrix `src` as a vector over var r: row i
                // (c == 0, factor stored (slice var, r)) or column i (c == 1);
                // scaled by the diagonals of the factors in `scale` at i
};

struct Value {
    ValKind kind;
    int src;  // input factor index or producing step index
    int r, c; // variables (Mat/InputMat: row, col; Vec/InputDiag: r)
    std::vector<int> scale;  // SliceVec: factors whose diagonal scales slice i
};

// A matrix operand of an elimination step.  `trans` says how the stored
// matrix is oriented relative to the step's canonical (first, second) order.
struct MatOp {
    int val;
    bool trans;
};

enum class StepKind : uint8_t {
    Elim0,   // s = sum_v prod sv(v)
    Elim1,   // y(w) = sum_v prod_A M(v,w) prod sv(v)
    Final1,  // s = sum_w aw(w) sum_v prod_A M(v,w) prod sv(v)
    Elim2,   // R(w,x) = sum_v prod_A M(v,w) prod sv(v) prod_B M(v,x)
    Final2   // s = sum_{w,x} R(w,x) prod_Z Z(w,x) prod aw(w) prod bx(x)
};

// One elimination step.  For A and B the canonical orientation is
// (v, w) / (v, x): trans == false means the operand is stored with rows over
// the eliminated variable v.  For Z the canonical orientation is (w, x).
struct Step {
    StepKind kind;
    int v = -1, w = -1, x = -1;
    std::vector<MatOp> A, B, Z;
    std::vector<int> sv, aw, bx;
    int out = -1;   // value produced
    int level = 0;  // dependency depth (inputs are level 0)
};

struct VProgram {
    std::vector<int> block_of;  // restricted-growth labels, size m
    int J = 0;                  // number of blocks
    int64_t mu = 0;             // Moebius coefficient (Lemma 2)
    int tw = 0;                 // exact treewidth of the quotient graph
    int width = 0;              // largest elimination degree of `order`
    std::vector<int> order;     // elimination order over quotient vars
    std::vector<Value> vals;
    std::vector<Step> steps;
    std::vector<int> scalars;   // value ids whose product is V_pi
    int depth = 0;              // max step level
    bool executable = true;     // false when lowering needs a step kind the
    std::string lower_error;    // engine lacks (reason in lower_error)
    // Conditioning: V_pi = sum_i (V of the quotient with var slice_var fixed
    // to sample i); -1 when the quotient is eliminated directly.
    int slice_var = -1;
};

struct PlanOptions {
    int precision = 0;
    int order = 0;
    int sparsify = 0;
    bool cse = true;  // merge equal steps across partitions at evaluation
    bool symmetric = false;  // caller's factor matrices are symmetric
    bool sym_gemm = true;    // products P P^T on the tiles on and above the diagonal
    bool overlap = false;    // a level's reductions on a second stream beside its GEMMs
    uint64_t workspace_limit = 0;
    std::string cost_model_path;
    double n_hint = 4096.0;  // sample size orders are ranked for
};

// Candidate-order scorer used by the learned ordering policy.
struct OrderScorer {
    virtual ~OrderScorer() = default;
    // Lower is better.  `feat` describes one complete candidate program.
    virtual double score(const std::vector<float> &feat) const = 0;
};

// Launch-shape choices of the executor, set by the autotuner or the caller.
struct Tuning {
    // a GEMM level uses 256-wide tiles for its eligible problems once they
    // give at least this many such tiles (2^62: never)
    int64_t gemm_big_min = 256;
    // column-reduction strips are cut so that a level has at least this
    // many blocks (strips of 512 down to 32 rows)
    int64_t colred_blocks = 1024;
};

struct Plan {
    int m = 0;
    std::vector<Edge> edges;
    PlanOptions opts;
    Tuning tuning;
    std::vector<VProgram> progs;
    int M = 0;
    int max_width = 0;
    std::vector<int64_t> N_l;  // size m+1
    bool executable = true;    // every program lowered
    std::string lower_error;
};

// Set partitions of {0..m-1} as restricted-growth strings, in lexicographic
// order of the string.
std::vector<std::vector<int>> enumerate_rgs(int m);

int64_t mobius_mu(const std::vector<int> &block_of);

// Lemma 3 filter: true when no block holds both endpoints of an edge.
bool survives_sparsification(const std::vector<int> &block_of, const std::vector<Edge> &edges);

// Exact treewidth by dynamic programming over vertex subsets (adjacency as
// bitmasks, J <= 16).
int exact_treewidth(int J, const std::vector<uint32_t> &adj);

// Build the program of one partition.  `order` may be empty (then chosen by
// the policy in opts).  Returns an empty string on success, else a message.
std::string build_program(const std::vector<Edge> &edges, int m, const std::vector<int> &block_of,
                          const PlanOptions &opts, const OrderScorer *scorer, VProgram &out);

// Lower a given elimination order to steps (used by build_program and by
// the ordering search).
std::string lower_order(const std::vector<Edge> &edges, const std::vector<int> &block_of, int J,
                        const std::vector<int> &order, VProgram &out, int slice_var = -1);

// Cost of a program at size n: multiply-add count of contraction steps
// and minimum bytes touched (elements, scaled by `elem_bytes`).
void program_cost(const VProgram &p, double n, double elem_bytes, double *flops, double *bytes);

// Features of a lowered program, for the learned cost model.
// Features of a lowered program at sample size n for the order cost model
// (kOrderFeatures of them).
constexpr int kOrderFeatures = 18;
std::vector<float> program_features(const VProgram &p, double n);

// Per step: does it depend on the conditioned (sliced) vertex?  All false
// for a program that is not conditioned.
std::vector<char> slice_dependent_steps(const VProgram &p);

std::string make_plan(int m, const std::vector<Edge> &edges, const PlanOptions &opts,
                      const OrderScorer *scorer, Plan &out);

}  // namespace ustat
