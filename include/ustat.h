/*
 * ustat.h -- C ABI of libustat, an MI355X (gfx950) engine for exact
 * higher-order U-statistics whose kernel factorises over the edges of a
 * small graph.
 *
 * Method (Chen, Liu & Zhang, arXiv 2508.12627):
 *   - U(h, X) is the unnormalised sum of h over ordered m-tuples of distinct
 *     sample indices (Definition 1).
 *   - The kernel is multiplicative-decomposable with one bivariate factor per
 *     edge (u, v) of a graph on m vertices (Definition "Multiplicative
 *     Decomposition"); factor k is tensorised to the n x n matrix
 *     T_k(i, j) = h_k(X_i, X_j) (Algorithm 1).
 *   - Lemma 2 rewrites U as sum over set partitions pi of [m] of
 *     mu_pi * V_pi, mu_pi = (-1)^(m-|pi|) prod_{C in pi} (|C|-1)!, where V_pi
 *     is the restricted V-statistic (Definition "Restricted V-Statistic").
 *   - V_pi is the Einsum of the induced notation A_pi (Algorithm 3, identity
 *     "restricted identity"), evaluated by eliminating one index at a time
 *     (Proposition 1 and its proof in Appendix "complexity_einsum").
 *   - Optional sparsification (Lemma 3): factor diagonals are treated as
 *     zero and only partitions in Pi_m^A are evaluated (Algorithm 4).
 *
 * Conventions for every call:
 *   - Every function returns a ustat_status; nothing throws or aborts across
 *     the ABI.  On error no output is written and ustat_last_error() holds a
 *     thread-local message.
 *   - The caller owns every input and output buffer.  "device" pointers are
 *     HIP device memory on the current device; "host" pointers are ordinary
 *     host memory.
 *   - Matrices are n x n, row-major, leading dimension n, element (i, j) at
 *     offset i*n + j.  Factor k belongs to edge k = (u_k, v_k) and is read as
 *     T_k(i_{u_k}, i_{v_k}).  The same pointer may be passed for several
 *     edges.
 *   - Factor element type follows the plan's precision: USTAT_F64 -> double,
 *     USTAT_F32 and USTAT_BF16X3 -> float, USTAT_I8 -> int8_t.
 *   - Work is enqueued on the given HIP stream (0 = default stream); results
 *     are copied to the host after the call synchronises that stream.
 *   - A plan is immutable after creation except for its device workspace and
 *     launch cache; calls that share one plan must not overlap in time.
 */
#ifndef USTAT_H
#define USTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ustat_plan_s *ustat_plan;
typedef void *ustat_stream; /* a hipStream_t */

typedef enum {
    USTAT_OK = 0,
    USTAT_E_INVALID = 1,     /* bad graph, sizes, pointers or options       */
    USTAT_E_UNSUPPORTED = 2, /* valid request this engine cannot run        */
    USTAT_E_NOMEM = 3,       /* device or host allocation failed            */
    USTAT_E_HIP = 4,         /* a HIP runtime call failed                   */
    USTAT_E_OVERFLOW = 5,    /* exact integer result may not fit 127 bits   */
    USTAT_E_INFEASIBLE = 6   /* workspace above opts.workspace_limit        */
} ustat_status;

typedef enum {
    USTAT_F64 = 0,    /* fp64 MFMA contractions, fp64 everywhere            */
    USTAT_F32 = 1,    /* fp32 MFMA contractions, fp64 reductions/combine    */
    USTAT_BF16X3 = 2, /* split-bf16 MFMA (hi*hi + hi*lo + lo*hi, or six
                         products of a three-plane split, see below), fp32
                         accumulation, fp64 reductions/combine              */
    USTAT_I8 = 3      /* exact: int8 MFMA on 7-bit limbs, int32 tiles,
                         int64 matrices, 128-bit totals                     */
} ustat_precision;

typedef enum {
    USTAT_ORDER_MINFILL = 0,    /* greedy min-fill, ties by degree then id  */
    USTAT_ORDER_EXHAUSTIVE = 1, /* cheapest of all elimination orders       */
    USTAT_ORDER_LEARNED = 2     /* candidates ranked by the MLP cost model  */
} ustat_order;

/*
 * Evaluation merges steps that compute the same value in several restricted
 * V-statistics (equal operation on the same factor matrices or upstream
 * values, up to transposition): each is computed once.  Results are
 * unchanged bit for bit (every kernel is deterministic).  USTAT_FLAG_NO_CSE
 * turns the merging off, so every partition's steps run separately.
 */
#define USTAT_FLAG_NO_CSE 1
/*
 * USTAT_FLAG_SYMMETRIC: every factor matrix given to ustat_eval, vstat_eval
 * and vstat_eval_ordered is symmetric (T(i,j) == T(j,i)), so the engine
 * reads it in whichever orientation a step streams: no transposed copies,
 * and steps that differ only by the orientation of an input are merged.
 * Values change at most by rounding (exact results not at all).  The RBF
 * factors that ustat_eval_samples and ustat_eval_batched build are
 * symmetric by construction and always read this way.
 */
#define USTAT_FLAG_SYMMETRIC 2
/*
 * USTAT_FLAG_NO_SYM_GEMM: a product P P^T of one prepared operand with
 * itself (R = K K for a symmetric factor K) is by default computed on the
 * tiles on and above the diagonal only, their K steps spread evenly over
 * the compute units, each tile mirrored below (split-bf16 with 256-wide
 * tiles).  This flag computes every tile instead, for comparisons; results
 * agree up to the order of fp32 additions.
 */
#define USTAT_FLAG_NO_SYM_GEMM 4
/*
 * USTAT_FLAG_OVERLAP_LEVELS: the reductions of a dependency level (the
 * one-index eliminations and the dot products) read only results of earlier
 * levels, as do the level's GEMMs.  With this flag they run on a second
 * stream of the plan (default priority) beside the GEMMs, joined by an
 * event before the level's partial sums; by default every launch runs on
 * the caller's stream.  Results are identical bit for bit.  The entry point
 * that allocates nothing always runs serially.
 */
#define USTAT_FLAG_OVERLAP_LEVELS 8

typedef struct {
    int32_t precision;          /* ustat_precision                          */
    int32_t order;              /* ustat_order                              */
    int32_t sparsify;           /* 0: every partition (Lemma 2); 1: Lemma 3 */
    int32_t flags;              /* USTAT_FLAG_* bits, 0 by default          */
    uint64_t workspace_limit;   /* bytes of device workspace, 0 = no limit  */
    const char *cost_model_path;/* weights file for USTAT_ORDER_LEARNED     */
    int64_t n_hint;             /* sample size the exhaustive and learned
                                   order policies rank for, 0 = 4096        */
} ustat_plan_opts;

typedef struct {
    double value;       /* U (or V_pi for vstat_eval), as a double          */
    int64_t exact_hi;   /* USTAT_I8: exact value = exact_hi*2^64 + exact_lo */
    uint64_t exact_lo;
    double err_scale;   /* S = sum_pi |mu_pi V_pi| (|V_pi| for vstat_eval)  */
    double err_est;     /* estimate of |value - exact| / S, see below       */
    int32_t num_vstats; /* restricted V-statistics evaluated                */
    int32_t reserved;
} ustat_result;
/*
 * err_est is an estimate, not a worst-case bound: the typical relative
 * error (about two standard deviations) under the probabilistic model of
 * rounding errors (independent, mean zero), from the unit roundoff and
 * inner length of the contraction instructions, the sample size n and the
 * number of dependency levels of the evaluation; 0 for USTAT_I8.  It does
 * not credit the averaging of independent element errors in the final
 * sums, so at large n it usually overstates the error; inputs built to
 * align rounding errors can exceed it.
 *
 * USTAT_BF16X3 contracts operands split into bf16 planes: two planes
 * (hi + lo, three products per pair) when every contracted value is known
 * to be non-negative and n >= 1024, otherwise three planes (hi + mid + lo,
 * six products, every term down to 2^-18), which keeps fp32-level accuracy
 * when signs cancel.  ustat_eval, vstat_eval and their variants scan the
 * factor matrices for negative entries on the device first (one read of
 * each matrix and one small read-back per call); the RBF factors that the
 * sample entry points build are known to be positive.
 */

/* Fill *opts with defaults: USTAT_F64, min-fill, no sparsification. */
ustat_status ustat_plan_opts_default(ustat_plan_opts *opts);

/*
 * Plan the evaluation of U for the kernel graph with m vertices (1..10) and
 * num_edges ordered edges (host int32 array [num_edges][2], labels 0..m-1,
 * u != v, every vertex used; parallel edges allowed).  Enumerates the set
 * partitions of [m] with mu_pi (Lemma 2), filters them by Lemma 3 when
 * opts->sparsify, forms each quotient graph G/pi (Definition "Quotient
 * Graph") with self-loops as diagonal vectors and parallel edges as
 * Hadamard groups, chooses an elimination order per quotient and lowers it
 * to kernel steps.  Host only; touches no device.
 * Errors: USTAT_E_INVALID (graph/opts), USTAT_E_NOMEM.
 */
ustat_status ustat_plan_create(int32_t m, int32_t num_edges, const int32_t *edges,
                               const ustat_plan_opts *opts, ustat_plan *out);

/* Free the plan, its device workspace and cached launches. NULL is a no-op. */
ustat_status ustat_plan_destroy(ustat_plan plan);

/*
 * Plan summary.  num_vstats: partitions evaluated; M: largest quotient
 * treewidth (Corollary 2); N_l (host int64 array of m+1 entries, may be
 * NULL): number of evaluated quotients of exact treewidth l = 0..m;
 * max_width: largest elimination degree of the chosen orders.
 */
ustat_status ustat_plan_info(ustat_plan plan, int32_t *num_vstats, int32_t *M,
                             int64_t *N_l, int32_t *max_width);

/*
 * Cost of one evaluation at sample size n under the chosen orders:
 * flops counts 2 per multiply-add of every contraction step (fp64-equivalent
 * products; a split-bf16 step executes three times as many MFMA flops), and
 * bytes the minimum HBM traffic of the steps.  workspace: device bytes the
 * evaluation needs.  Errors: USTAT_E_OVERFLOW (workspace requested, exact
 * plan) when an intermediate may overflow for factors of magnitude up to
 * 127 (evaluation bounds with the factors' true maxima instead).
 */
ustat_status ustat_plan_cost(ustat_plan plan, int64_t n, double *flops, double *bytes,
                             uint64_t *workspace);

/*
 * Device workspace (bytes) of one evaluation of `batch` datasets with sizes
 * n (host int64 array), as ustat_eval_batched would allocate it.
 * shared_factor = 1 models every edge reading one factor matrix per dataset
 * (the sample entry points); 0 models independent factors per edge.
 */
ustat_status ustat_plan_workspace(ustat_plan plan, int32_t batch, const int64_t *n,
                                  int32_t shared_factor, uint64_t *bytes);

/*
 * Launch-shape tuning of a plan (how the engine cuts work into launches;
 * results change at most by rounding, exact results not at all).
 *   gemm_big_min:  a GEMM level takes 256 x 256 tiles for its fp32 and
 *                  split-bf16 problems whose padded size is a multiple of
 *                  256 once they give at least this many such tiles
 *                  (default 256, one per compute unit; 0: whenever
 *                  eligible; 2^62: never);
 *   colred_blocks: column-reduction strips are cut so that a level has at
 *                  least this many blocks (default 1024; 1..2^20).
 * Setting a tuning drops the plan's cached graphs.
 */
ustat_status ustat_plan_tuning(ustat_plan plan, int64_t *gemm_big_min, int64_t *colred_blocks);
ustat_status ustat_plan_set_tuning(ustat_plan plan, int64_t gemm_big_min, int64_t colred_blocks);

/*
 * Autotune the plan's launch shapes for sample size n on the given device
 * factors (as for ustat_eval): every candidate tuning (gemm_big_min in
 * {256, 0, never} for fp32 and split-bf16, colred_blocks in {256, 1024,
 * 4096}) evaluates U once to warm up and then reps times (1..100) on
 * stream (a temporary stream when NULL); the candidate with the least
 * time per evaluation is kept.  *ms (may be NULL) receives that time.
 * On error the previous tuning is restored.
 */
ustat_status ustat_plan_autotune(ustat_plan plan, int64_t n, const void *const *factors,
                                 ustat_stream stream, int32_t reps, double *ms);

/*
 * The same search for a batch of sample sets (arguments as
 * ustat_eval_batched): every candidate times whole batched evaluations, so
 * the choice accounts for how the datasets' steps share launches.
 *
 * Both autotuning calls keep a per-device cache when the environment
 * variable USTAT_TUNE_CACHE names a writable file: a result is stored under
 * a key of the device (architecture and compute-unit count), the plan
 * (graph, precision, order policy, options) and the shape (log2 buckets of
 * n, or of the batch's largest and total n, the batch size and d); a later
 * call with the same key applies the stored tuning and returns its time
 * without measuring.
 */
ustat_status ustat_plan_autotune_batched(ustat_plan plan, int32_t batch, const int64_t *n, int32_t d,
                                         const double *const *X, double rbf_divisor,
                                         ustat_stream stream, int32_t reps, double *ms);

/*
 * Partition idx (0 <= idx < num_vstats) in restricted-growth form:
 * block_of (host int32 [m]) gives each vertex's block, blocks numbered in
 * order of first appearance; *mu its Moebius coefficient; *tw the exact
 * treewidth of its quotient graph; *width the largest elimination degree of
 * its chosen order.  Any output pointer may be NULL.
 */
ustat_status ustat_plan_partition(ustat_plan plan, int32_t idx, int32_t *block_of, int64_t *mu,
                                  int32_t *tw, int32_t *width);

/*
 * Elimination order chosen for partition idx: order (host int32 array of
 * at least m entries) receives the quotient vertices in elimination order;
 * *len their number.  *slice_var is -1, or the quotient vertex the program
 * conditions on when no order stays within degree 2 (its n values are
 * summed outside the elimination, which then lists the other vertices).
 * Any output pointer may be NULL.
 */
ustat_status ustat_plan_order(ustat_plan plan, int32_t idx, int32_t *order, int32_t *len,
                              int32_t *slice_var);

/* Exact treewidth of the simple graph underlying an edge list (m <= 16);
 * self-loops and repeated edges are ignored (Definition "Treewidth"). */
ustat_status ustat_graph_treewidth(int32_t m, int32_t num_edges, const int32_t *edges,
                                   int32_t *tw);

/*
 * U(h, X) from the factor matrices: factors is a host array of num_edges
 * device pointers to n x n matrices (element type per precision).  n >= m.
 * Errors: USTAT_E_INVALID, USTAT_E_NOMEM, USTAT_E_HIP, USTAT_E_OVERFLOW,
 * USTAT_E_INFEASIBLE.
 */
ustat_status ustat_eval(ustat_plan plan, int64_t n, const void *const *factors,
                        ustat_stream stream, ustat_result *out);

/*
 * U(h, X) for the RBF kernel on every edge, k(x, y) = exp(-||x-y||^2 /
 * rbf_divisor): X is a device fp64 n x d row-major sample (d <= 256); the
 * factor matrix is built on the device (Algorithm 1) in the plan's
 * precision, then evaluated as in ustat_eval.  Not valid for USTAT_I8.
 */
ustat_status ustat_eval_samples(ustat_plan plan, int64_t n, int32_t d, const double *X,
                                double rbf_divisor, ustat_stream stream, ustat_result *out);

/*
 * One restricted V-statistic V_pi (Definition "Restricted V-Statistic"):
 * block_of (host int32 [m]) is any labelling of a partition of [m] by block
 * (it is canonicalised); the partition need not be among the plan's
 * evaluated ones.  out->value = V_pi, out->err_scale = |V_pi|.
 */
ustat_status vstat_eval(ustat_plan plan, const int32_t *block_of, int64_t n,
                        const void *const *factors, ustat_stream stream, ustat_result *out);

/*
 * Many independent datasets at once: dataset b has n[b] samples (host
 * int64 array) at X[b] (host array of device fp64 n[b] x d pointers); the
 * RBF kernel as in ustat_eval_samples.  Every (dataset, partition) pair is
 * evaluated in one replay of a captured HIP graph of grouped launches.
 * out: host array of batch results.
 */
ustat_status ustat_eval_batched(ustat_plan plan, int32_t batch, const int64_t *n, int32_t d,
                                const double *const *X, double rbf_divisor, ustat_stream stream,
                                ustat_result *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture elsewhere in the program, tight serving loops, harnesses that
 * forbid hipMalloc): ustat_eval with every device buffer it needs (the
 * workspace of intermediates, the launch descriptors and the per-program
 * accumulators) taken from a fixed array of USTAT_NOALLOC_MAX_BYTES bytes
 * that the library holds on each device it runs on, from the first kernel
 * launch there until the process ends.  Arguments, results and errors are
 * those of ustat_eval, plus USTAT_E_INFEASIBLE when the evaluation needs
 * more than the array (ustat_plan_cost's workspace tells ahead; programs
 * conditioned on a vertex run in slice chunks that fit).  The call makes no
 * device or pinned-host allocation and captures no graph; results come back
 * through ordinary host memory after a synchronisation of the stream.
 * All calls on one device share its array, which keeps the last call's
 * contents: calls that overlap in time on one device (from several host
 * threads or streams) race and must be serialised by the caller.
 */
#define USTAT_NOALLOC_MAX_BYTES ((uint64_t)128 << 20)
ustat_status ustat_eval_noalloc(ustat_plan plan, int64_t n, const void *const *factors,
                                ustat_stream stream, ustat_result *out);

/*
 * U(h, X) from low-rank factors, without forming any n x n matrix: factor e
 * is T_e = F_e G_e^T with F[e], G[e] device pointers to row-major fp64
 * n x r panels (host arrays of num_edges pointers; the same pointer may
 * appear several times, as in the chains of the higher-order influence
 * function estimators of Section 4.1, where g = (A phi)(A phi)^T and
 * f = (A phi)(Y phi)^T).  Writing T_e(i, j) = sum_a F_e(i, a) G_e(j, a)
 * adds one rank index per edge to the Einsum of every restricted
 * V-statistic (Definition "Restricted V-Statistic", Algorithm 3); the engine
 * sums out sample and rank indices one at a time (the proof of Proposition
 * 1), in the order of least multiply-adds among those that never give a
 * value two sample indices, merges equal steps across partitions and forms
 * the Moebius combination of Lemma 2 over every partition of [m] (the
 * plan's sparsification is ignored: Lemma 3 needs zero-diagonal factors).
 * fp64 throughout, whatever the plan's floating-point precision; err_scale
 * and err_est as for USTAT_F64, num_vstats = Bell(m).  The plan's
 * workspace limit applies.  n in [m, 2^31], r in 1..4096.
 * Errors: USTAT_E_INVALID (sizes, NULL pointers, motif plan),
 * USTAT_E_UNSUPPORTED (USTAT_I8 plan; a step with more than 8 operands or
 * a value with more than 8 indices; a network of more than 32 indices),
 * USTAT_E_INFEASIBLE, USTAT_E_NOMEM, USTAT_E_HIP.
 */
ustat_status ustat_eval_lowrank(ustat_plan plan, int64_t n, int32_t r, const double *const *F,
                                const double *const *G, ustat_stream stream, ustat_result *out);

/*
 * The low-rank schedule of ustat_eval_lowrank, host only (no device call):
 * panel_ids (host int32 [2 num_edges], the ids of F_0, G_0, F_1, G_1, ...;
 * equal ids mean the same panel; NULL = all distinct) stand for the
 * pointers.  madds counts the multiply-adds of the merged steps (the size
 * of the summed index times the size of the value produced), madds_unmerged
 * the same over every partition's own steps; workspace_bytes is the device
 * workspace; num_exact_orders / num_greedy_orders count the partitions
 * whose order came from the exact search (networks of at most 16 indices)
 * or from the greedy rule; num_gemm_steps counts the steps over a sample
 * index that run as fp64 MFMA GEMMs (their operands split into two groups
 * with disjoint indices, each side of the output at least 32 long; the
 * others run on the vector units).  Errors as ustat_eval_lowrank, without
 * USTAT_E_INFEASIBLE, USTAT_E_NOMEM and USTAT_E_HIP.
 */
typedef struct {
    double madds;
    double madds_unmerged;
    int64_t workspace_bytes;
    int32_t num_partitions;
    int32_t num_steps;
    int32_t depth;
    int32_t num_exact_orders;
    int32_t num_greedy_orders;
    int32_t num_gemm_steps;
} ustat_lowrank_stats;
ustat_status ustat_lowrank_info(ustat_plan plan, int64_t n, int32_t r, const int32_t *panel_ids,
                                ustat_lowrank_stats *out);

/*
 * Build the RBF factor matrix alone (Algorithm 1 for the RBF kernel):
 * out (device, n x n) receives exp(-||X_i - X_j||^2 / rbf_divisor) with the
 * squared distance formed in fp64 as ||X_i||^2 + ||X_j||^2 - 2 X_i.X_j (the
 * Gram term on fp64 MFMA, the result clamped at 0), the diagonal exactly 1
 * and the matrix exactly symmetric; precision USTAT_F64 writes double,
 * USTAT_F32 writes float (rounded once).
 */
ustat_status ustat_build_rbf(int64_t n, int32_t d, const double *X, double rbf_divisor,
                             int32_t precision, void *out, ustat_stream stream);

/*
 * Peak microbenchmarks: the rates the kernels' rooflines are compared with,
 * measured on the current device (HIP events around one launch, after one
 * untimed launch, on `stream`; both calls synchronise with it).
 *
 * ustat_peak_mfma: two blocks of four waves per compute unit, each wave
 * issuing `iters` (1 .. 2^32) rounds of eight independent MFMA instructions
 * of one kind on register operands: kind 0 bf16 16x16x32 (fp32
 * accumulation), 1 fp64 16x16x4, 2 int8 16x16x64 (int32 accumulation),
 * 3 fp32 16x16x4.  *rate receives operations per second (2 per
 * multiply-add).  sink: device memory of at least 4096 x 32 bytes, owned by
 * the caller, overwritten with the waves' sums (keeps the work live).
 *
 * ustat_peak_copy: a streaming copy of `bytes` (a positive multiple of 16)
 * from src to dst (device buffers owned by the caller, not overlapping),
 * eight blocks of 256 threads per compute unit; *rate receives bytes read
 * plus bytes written per second.
 *
 * Errors: USTAT_E_INVALID for bad arguments, USTAT_E_HIP for a failed
 * launch or event.
 */
ustat_status ustat_peak_mfma(int32_t kind, int64_t iters, void *sink, ustat_stream stream,
                             double *rate);
ustat_status ustat_peak_copy(const void *src, void *dst, int64_t bytes, ustat_stream stream,
                             double *rate);

/*
 * Kernel timing (HIP events recorded around every grouped launch on the
 * launch stream; off by default, never active inside graph capture).
 * kind: 0 operand prep, 1 GEMM, 2 column reduction, 3 partial reduction,
 * 4 factor build, 5 low-rank summation steps, 6 low-rank chunk sums,
 * 7 low-rank outer-product (GEMM) steps.  ustat_profile_read returns
 * totals since the last reset: milliseconds, number of launches,
 * algorithmic flops (2 n^3 per GEMM step, symmetric products P P^T
 * included, 2 M N n per low-rank GEMM step) and
 * algorithmic bytes (every operand element read once plus the outputs
 * written, for the column reduction and operand prep kernels).  Any output
 * pointer may be NULL.
 */
ustat_status ustat_profile_enable(int32_t on);
ustat_status ustat_profile_reset(void);
ustat_status ustat_profile_read(int32_t kind, double *ms, int64_t *launches, double *flops,
                                double *bytes);

/*
 * Features of partition block_of (any labelling) eliminated in the given
 * order (quotient vertices, labels as in ustat_plan_order) at sample size
 * n.  slice_var is -1 (order lists all len = J quotient vertices) or a
 * vertex to condition on (order lists the other len = J - 1 vertices).
 * feat (host float array of at least USTAT_NUM_FEATURES entries) receives
 * step-kind counts, operand and transposition counts, dependency depth,
 * width (conditioning counts one), log-size terms, the log of the
 * program's algorithmic flops and bytes at n, and the number of GEMM steps
 * repeated per slice of a conditioned program.  USTAT_E_UNSUPPORTED
 * if the order needs a step of degree above 2.
 */
#define USTAT_NUM_FEATURES 18
ustat_status ustat_order_features(ustat_plan plan, const int32_t *block_of, const int32_t *order,
                                  int32_t len, int32_t slice_var, int64_t n, float *feat);

/* vstat_eval with an explicit elimination order (arguments as above). */
ustat_status vstat_eval_ordered(ustat_plan plan, const int32_t *block_of, const int32_t *order,
                                int32_t len, int32_t slice_var, int64_t n,
                                const void *const *factors, ustat_stream stream,
                                ustat_result *out);

/*
 * Cost-model MLP, F -> H1 -> H2 -> 1 with ReLU hidden layers, on the GPU
 * (its own forward, backward and Adam kernels).  params is one host fp32
 * array of ustat_mlp_num_params(F, H1, H2) entries:
 *   mean[F] inv_std[F] W1[H1*F] b1[H1] W2[H2*H1] b2[H2] W3[H2] b3[1]
 * (inputs are standardised with mean/inv_std, which are not trained).
 * X is host fp32 N x F row-major, y host fp32 [N].  The loss is the mean
 * squared error.  Reductions over samples use a fixed order, so results
 * are reproducible.
 */
size_t ustat_mlp_num_params(int32_t F, int32_t H1, int32_t H2);
/* out[i] = network output for row i of X. */
ustat_status ustat_mlp_predict(int32_t F, int32_t H1, int32_t H2, const float *params,
                               const float *X, int64_t N, float *out);
/* *loss = mean squared error; grad (host, num_params entries) = its gradient
 * with respect to every parameter (zero for mean and inv_std). */
ustat_status ustat_mlp_loss_grad(int32_t F, int32_t H1, int32_t H2, const float *params,
                                 const float *X, const float *y, int64_t N, double *loss,
                                 float *grad);
/* steps full-batch Adam steps (learning rate lr) updating params in place;
 * losses (host, may be NULL) receives the loss before each step. */
ustat_status ustat_mlp_train(int32_t F, int32_t H1, int32_t H2, float *params, const float *X,
                             const float *y, int64_t N, int32_t steps, float lr, double *losses);
/* Write params as a cost-model file readable through opts.cost_model_path. */
ustat_status ustat_mlp_save(const char *path, int32_t F, int32_t H1, int32_t H2,
                            const float *params);

/*
 * Induced motif counts of a simple graph (the motif application of Section
 * 4.2 and its appendix): for each connected motif r on `size` vertices,
 * the number of vertex subsets inducing r equals U(h_r) / |Aut(r)|, where
 * h_r is the kernel over the complete graph on `size` vertices with factor
 * A on the motif's edges and B = 1 - A on its non-edges.  Every pair is an
 * edge of that kernel graph, so with Lemma 3 only the finest partition
 * remains; its quotient for size 4 (K4) has treewidth 3 and is evaluated
 * by conditioning on one vertex.
 *
 * ustat_plan_create_motifs plans the motifs of size 3 (V-shape, triangle)
 * or 4 (3-star, path, tailed triangle, square, diamond, K4) on the exact
 * path (the precision and sparsify options are ignored: USTAT_I8, Lemma
 * 3); the plan queries (ustat_plan_info, ...) describe the first motif.
 * ustat_motif_counts evaluates every motif of the plan in one pass, steps
 * equal across motifs (products of A and B) computed once: A is a device
 * int8 n x n symmetric 0/1 adjacency with a zero diagonal (else
 * USTAT_E_INVALID, checked on the device), counts a host int64 array of 2
 * (size 3) or 6 (size 4) entries, in the order above.
 */
ustat_status ustat_plan_create_motifs(int32_t size, const ustat_plan_opts *opts, ustat_plan *out);
ustat_status ustat_motif_counts(ustat_plan plan, int64_t n, const int8_t *A, ustat_stream stream,
                                int64_t *counts);

/*
 * For tests of the error paths (not for production callers): arm a
 * one-shot failure.  kind 0: the (countdown + 1)-th host allocation point
 * of the planner or executor fails (the call returns USTAT_E_NOMEM);
 * kind 1: the (countdown + 1)-th device or pinned-host allocation reports
 * out of memory (USTAT_E_NOMEM); kind 2: the (countdown + 1)-th evaluation
 * fails at its first launch, after any graph capture has begun
 * (USTAT_E_HIP; the capture is ended and the stream left usable).
 * countdown < 0 disarms the kind.  Process-wide, not thread-safe with
 * concurrent calls.  Errors: USTAT_E_INVALID for an unknown kind.
 */
ustat_status ustat_debug_inject(int32_t kind, int64_t countdown);

const char *ustat_status_string(ustat_status s);
const char *ustat_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* USTAT_H */
