// Evaluation from low-rank factors.  Every factor is given as two n x r
// panels, T_e = F_e G_e^T, and no n x n matrix is ever formed.
//
// Writing T_e(i, j) = sum_a F_e(i, a) G_e(j, a) adds one rank index a_e per
// edge to the Einsum of a restricted V-statistic (Definition "Restricted
// V-Statistic", Algorithm 3): the quotient's sample indices (size n) and the
// rank indices (size r) form one network in which every input is an n x r
// panel.  The proof of Proposition 1 sums indices out one at a time; here an
// index of either kind may be summed out, subject to one rule: no value may
// carry two sample indices (that would be an n x n matrix).  Each restricted
// V-statistic gets the order of least multiply-add count under that rule
// (exact dynamic programme over the eliminated set, greedy for large
// networks), equal steps are merged across partitions, and the U-statistic
// is the Moebius combination of Lemma 2 over every partition (Lemma 3 does
// not apply: it needs factors with a zero diagonal, and F G^T has none).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "plan.hpp"

namespace ustat {

constexpr int kLrMaxIn = 8;    // operands of one step
constexpr int kLrMaxDim = 8;   // indices of one value
constexpr int kLrThreads = 256;

// One summation step: out[o] = sum_{x < nx} prod_t in_t[off_t(o) + x sx_t],
// off_t(o) = base_t + sum_d digit_d(o) so_t[d], digits of o in the mixed
// radix dim[] (dim[nd-1] fastest).  Inputs are addressed as (pointer-table
// slot, element offset): slot 0 is the workspace, slots 1.. the caller's
// panels.  mode 0 ("short" index, a rank index): one thread per output.
// mode 1 ("long" index, a sample index): the x range is cut into nchunk
// chunks of xchunk, each block sums one chunk for `otile` outputs with
// `xlanes` threads per output and writes partials [nchunk][nout] at `out`.
struct LrStepDesc {
    int32_t nin, nd, mode, nchunk;
    int32_t otile, xlanes, pad0, pad1;
    int32_t slot[kLrMaxIn];
    int64_t base[kLrMaxIn];
    int64_t sx[kLrMaxIn];
    int64_t so[kLrMaxIn][kLrMaxDim];
    int64_t dim[kLrMaxDim];
    int64_t nout, nx, xchunk;
    int64_t out;     // workspace element offset of the output / partials
    int64_t block0;  // first block of this step in its launch
};

// A long step whose operands split into two groups with disjoint indices,
// out[l, r] = sum_x A(x, l) B(x, r) with A(x, l) the product of the left
// operands and B(x, r) that of the right ones (a sum of outer products of
// Khatri-Rao rows): an fp64 MFMA GEMM with inner dimension x whose operand
// values are formed in registers.  Up to kLrKrSide operands a side:
// operands 0..nl-1 are the left ones, kLrKrSide..kLrKrSide+nr-1 the right
// ones.  Operand u is read at slot base[u] + x sx[u] +
// sum_d digit_d st[u][d] over the digits of l (left, radix dl) or of r
// (right, radix dr); the output element (l, r) is at out + c nout +
// sum_d digit_d(l) ol[d] + sum_d digit_d(r) orr[d] (c the chunk of x;
// partials when nchunk > 1).  Offsets within a value fit 31 bits.
// small = 1 marks a step whose left side has at most 16 indices and right
// side at most 64: it runs as one "tile" per chunk on a register-only path.
constexpr int kLrKrTile = 64;
constexpr int kLrKrSmall = 16, kLrKrSmallWide = 64;
constexpr int kLrKrSide = 4;
struct LrKrDesc {
    int32_t ndl, ndr, nl, nr;  // side indices, side operands (1..kLrKrSide)
    int32_t slot[2 * kLrKrSide];
    int64_t base[2 * kLrKrSide];
    int32_t sx[2 * kLrKrSide];
    int32_t st[2 * kLrKrSide][kLrMaxDim];
    int32_t dl[kLrMaxDim], dr[kLrMaxDim];
    int32_t ol[kLrMaxDim], orr[kLrMaxDim];
    int32_t M, N, nx, xchunk, nchunk, tiles_n, tiles, nout;
    int32_t small, pad;
    int64_t out, block0;
};

// Sum of the nchunk partials of a long step: a block covers `otile`
// outputs with `clanes` threads each; lane l sums chunks l, l + clanes, ...
// and the lanes' sums are added in lane order.
struct LrReduceDesc {
    int64_t part, out, nout, block0;
    int32_t nchunk, otile, clanes, pad;
};

struct LrLevel {
    int64_t steps_off = 0, nsteps = 0, blocks = 0;    // into the step array
    int64_t red_off = 0, nred = 0, rblocks = 0;        // into the reduce array
    int64_t kr_off = 0, nkr = 0, krblocks = 0;         // into the outer-product array
    double kr_flops = 0, kr_bytes = 0;
    // algorithmic work of the level's steps: nin flops per term (nin - 1
    // products and one addition), bytes of every operand read once and of
    // every value written once (fp64)
    double flops = 0, bytes = 0, red_bytes = 0;
};

struct LrSchedule {
    int64_t n = 0;
    int r = 0;
    std::vector<int> slot_of;  // 2E entries: table slot of F_e, G_e
    int nslots = 0;            // 1 + distinct panels
    std::vector<LrStepDesc> steps;
    std::vector<LrReduceDesc> reds;
    std::vector<LrKrDesc> krs;
    std::vector<LrLevel> levels;
    // Moebius combination: partition p has coefficient mu[p], a constant
    // factor cst[p] (n per block without edges) and the product of the
    // scalar values at workspace offsets sc[sc_first[p] .. sc_first[p+1]).
    std::vector<double> mu, cst;
    std::vector<int32_t> sc_first;
    std::vector<int64_t> sc;
    int64_t ws_elems = 0;     // values, then partials
    int64_t part_elems = 0;   // largest partial buffer of one level
    double flops = 0;         // multiply-adds of the steps after merging
    double flops_unmerged = 0;
    int nvalues = 0, depth = 0, nparts = 0, ndp = 0, ngreedy = 0;
    // device copies: steps, reduces, combine arrays (one blob)
    char *blob = nullptr;
    size_t blob_bytes = 0;
    size_t off_steps = 0, off_reds = 0, off_krs = 0, off_mu = 0, off_cst = 0, off_first = 0, off_sc = 0,
           off_tab = 0, off_res = 0;
    int device = -1;
    ~LrSchedule();
};

// Build the schedule of every partition of the plan's kernel graph for
// sample size n and rank r.  slot_of gives, for F_0, G_0, F_1, G_1, ..., the
// pointer-table slot (1-based) of that panel: equal slots mean the same
// panel, which lets equal steps merge.  Host only; "" on success.
std::string build_lowrank(const Plan &plan, int64_t n, int r, const std::vector<int> &slot_of,
                          LrSchedule &out);

// Upload the schedule's descriptors to the current device (once).
hipError_t upload_lowrank(LrSchedule &s);

// Run a schedule: panels[k] is the device pointer of table slot k+1,
// ws a device workspace of s.ws_elems doubles.  Writes {U, S} to the pinned
// host buffer hres and synchronises the stream.
hipError_t run_lowrank(LrSchedule &s, const double *const *panels, double *ws, hipStream_t stream,
                       double *hres);

// Launchers (k_lowrank.hip).
void launch_lr_steps(const LrStepDesc *d, int64_t nsteps, int64_t blocks,
                     const double *const *tab, hipStream_t s);
void launch_lr_kr(const LrKrDesc *d, int64_t nkr, int64_t blocks, const double *const *tab,
                  hipStream_t s);
void launch_lr_reduce(const LrReduceDesc *d, int64_t nred, int64_t blocks, double *ws,
                      hipStream_t s);
void launch_lr_combine(const double *mu, const double *cst, const int32_t *first,
                       const int64_t *sc, int nparts, const double *ws, double *res,
                       hipStream_t s);

}  // namespace ustat
