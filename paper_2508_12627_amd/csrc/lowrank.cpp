// Host side of the low-rank evaluation: the network of sample and rank
// indices of each restricted V-statistic, its elimination order, the merged
// step list, and the launches (kernels in k_lowrank.hip).
#include "lowrank.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>

#include "inject.hpp"
#include "profile.hpp"

namespace ustat {

LrSchedule::~LrSchedule() {
    if (blob) (void)hipFree(blob);
}

namespace {

// Exact order search up to this many active network nodes, greedy above.
constexpr int kLrDpMaxNodes = 16;

struct Net {
    int N = 0;                    // active nodes
    std::vector<uint32_t> adj;    // adjacency bitmasks over active nodes
    std::vector<double> size;     // index extent
    uint32_t sample_mask = 0;     // active nodes that are sample indices
};

// Nodes outside S u {v} reachable from v through eliminated nodes (S): the
// indices of the value that eliminating v produces.
uint32_t frontier(const Net &g, uint32_t S, int v) {
    uint32_t seen = 1u << v, res = 0, stack = 1u << v;
    while (stack) {
        int x = __builtin_ctz(stack);
        stack &= stack - 1;
        uint32_t nb = g.adj[x] & ~seen;
        seen |= nb;
        res |= nb & ~S;
        stack |= nb & S;
    }
    return res;
}

double step_cost(const Net &g, int v, uint32_t nb) {
    double c = g.size[v];
    for (uint32_t m = nb; m; m &= m - 1) c *= g.size[__builtin_ctz(m)];
    return c;
}

bool allowed(const Net &g, uint32_t nb) { return __builtin_popcount(nb & g.sample_mask) <= 1; }

// Least total multiply-adds over all orders that never form a value with two
// sample indices: dynamic programme over the set of eliminated nodes (the
// value produced by eliminating v depends only on that set).
std::vector<int> order_dp(const Net &g) {
    const uint32_t full = g.N == 32 ? 0xffffffffu : ((1u << g.N) - 1);
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<double> best((size_t)full + 1, inf);
    std::vector<int8_t> last((size_t)full + 1, -1);
    best[0] = 0;
    uint32_t cmask[32], cnb[32];
    for (uint32_t S = 0; S < full; ++S) {
        if (best[S] == inf) continue;
        // connected components of the eliminated set and their frontiers
        int nc = 0;
        for (uint32_t left = S; left;) {
            uint32_t comp = left & (~left + 1), grow = comp;
            while (grow) {
                const int x = __builtin_ctz(grow);
                grow &= grow - 1;
                const uint32_t add = g.adj[x] & S & ~comp;
                comp |= add;
                grow |= add;
            }
            uint32_t nb = 0;
            for (uint32_t q = comp; q; q &= q - 1) nb |= g.adj[__builtin_ctz(q)];
            cmask[nc] = comp;
            cnb[nc++] = nb & ~S;
            left &= ~comp;
        }
        for (int v = 0; v < g.N; ++v) {
            if (S >> v & 1) continue;
            uint32_t nb = g.adj[v] & ~S;
            for (int c = 0; c < nc; ++c)
                if (g.adj[v] & cmask[c]) nb |= cnb[c];
            nb &= ~(1u << v);
            if (!allowed(g, nb)) continue;
            double c = best[S] + step_cost(g, v, nb);
            uint32_t T = S | (1u << v);
            if (c < best[T]) {
                best[T] = c;
                last[T] = (int8_t)v;
            }
        }
    }
    std::vector<int> order;
    for (uint32_t S = full; S; S &= ~(1u << last[S])) order.push_back(last[S]);
    std::reverse(order.begin(), order.end());
    return order;
}

// Greedy: the cheapest allowed elimination next (lowest node on ties).
std::vector<int> order_greedy(const Net &g) {
    std::vector<int> order;
    uint32_t S = 0;
    for (int k = 0; k < g.N; ++k) {
        int bv = -1;
        double bc = 0;
        for (int v = 0; v < g.N; ++v) {
            if (S >> v & 1) continue;
            uint32_t nb = frontier(g, S, v);
            if (!allowed(g, nb)) continue;
            double c = step_cost(g, v, nb);
            if (bv < 0 || c < bc) bv = v, bc = c;
        }
        order.push_back(bv);  // a sample index with only rank neighbours is always allowed
        S |= 1u << bv;
    }
    return order;
}

// A value: a panel (kind 0) or the output of a step (kind 1).  `samp` says
// which of its indices is a sample index (at most one, always the first).
struct LrValue {
    int kind = 0;
    int slot = 0;                  // panel: table slot
    bool samp_first = false;       // first index is a sample index
    int nd = 0;
    int64_t dims[kLrMaxDim] = {};
    int64_t size = 1;
    int level = 0;
    int64_t off = 0;               // workspace offset (steps)
    // step
    bool long_x = false;
    int64_t nx = 0;
    std::vector<int> ins;
    std::vector<std::vector<int>> maps;  // per input index: output position or -1 (= x)
};

struct Tensor {
    int vid;
    std::vector<int> nodes;  // network node of each index
};

// Row-major element strides of a value's indices.
void value_strides(const LrValue &v, int64_t *st) {
    int64_t s = 1;
    for (int q = v.nd - 1; q >= 0; --q) {
        st[q] = s;
        s *= v.dims[q];
    }
}

// Split of a long step's operands into a left and a right group whose
// output indices are disjoint (operands without output indices go left),
// with the largest min(M, N) of the two index-space sizes; 0 when no split
// gives both sides at least kLrKrMin (the generic kernel is used then: a
// GEMM of a side shorter than 8 wastes most of each 16-wide MFMA block).
constexpr int64_t kLrKrMin = 8;
uint32_t kr_split(const LrValue &v, const std::vector<LrValue> &vals) {
    const int nin = (int)v.ins.size();
    const int64_t lim = (int64_t)1 << 31;
    if (v.nx >= lim || v.size >= lim) return 0;
    for (int t : v.ins)
        if (vals[t].size >= lim) return 0;
    std::vector<uint32_t> dm(nin, 0);
    for (int t = 0; t < nin; ++t)
        for (int p : v.maps[t])
            if (p >= 0) dm[t] |= 1u << p;
    uint32_t best = 0;
    int64_t best_min = kLrKrMin - 1;
    for (uint32_t mask = 1; mask + 1 < (1u << nin); ++mask) {
        if (__builtin_popcount(mask) > kLrKrSide || nin - __builtin_popcount(mask) > kLrKrSide) continue;
        uint32_t dl = 0, dr = 0;
        for (int t = 0; t < nin; ++t) (mask >> t & 1 ? dl : dr) |= dm[t];
        if (dl & dr) continue;
        bool empty_right = false;
        for (int t = 0; t < nin; ++t) empty_right |= !(mask >> t & 1) && dm[t] == 0;
        if (empty_right) continue;
        int64_t M = 1, N = 1;
        for (int q = 0; q < v.nd; ++q) (dl >> q & 1 ? M : N) *= v.dims[q];
        if (std::min(M, N) > best_min) {
            best_min = std::min(M, N);
            best = mask;
        }
    }
    return best;
}

}  // namespace

std::string build_lowrank(const Plan &plan, int64_t n, int r, const std::vector<int> &slot_of,
                          LrSchedule &out) {
    inject_host_alloc();
    const int m = plan.m;
    const int E = (int)plan.edges.size();
    if (n < 1 || r < 1) return "n and r must be positive";
    if ((int)slot_of.size() != 2 * E) return "one table slot per panel expected";
    out.n = n;
    out.r = r;
    out.slot_of = slot_of;
    out.nslots = 1 + *std::max_element(slot_of.begin(), slot_of.end());

    std::vector<LrValue> vals;
    std::map<std::vector<int64_t>, int> memo;
    std::vector<int> panel_vid(out.nslots, -1);
    for (int s : slot_of) {
        if (panel_vid[s] >= 0) continue;
        LrValue v;
        v.kind = 0;
        v.slot = s;
        v.samp_first = true;
        v.nd = 2;
        v.dims[0] = n;
        v.dims[1] = r;
        v.size = n * (int64_t)r;
        panel_vid[s] = (int)vals.size();
        vals.push_back(v);
    }

    out.mu.clear();
    out.cst.clear();
    out.sc_first.assign(1, 0);
    out.sc.clear();
    for (const auto &blk : enumerate_rgs(m)) {
        int J = 0;
        for (int b : blk) J = std::max(J, b + 1);
        // network nodes: sample index of each block with an edge, then one
        // rank index per edge
        std::vector<int> node_of_block(J, -1);
        std::vector<char> has(J, 0);
        for (const Edge &e : plan.edges) has[blk[e.u]] = has[blk[e.v]] = 1;
        Net g;
        int isolated = 0;
        for (int b = 0; b < J; ++b) {
            if (!has[b]) {
                ++isolated;
                continue;
            }
            node_of_block[b] = g.N++;
            g.size.push_back((double)n);
        }
        const int first_rank = g.N;
        g.N += E;
        if (g.N > 32) return "low-rank network has more than 32 indices";
        for (int e = 0; e < E; ++e) g.size.push_back((double)r);
        g.adj.assign(g.N, 0);
        g.sample_mask = first_rank >= 32 ? 0xffffffffu : ((1u << first_rank) - 1);
        std::vector<Tensor> tens;
        for (int e = 0; e < E; ++e) {
            const int a = first_rank + e;
            const int su = node_of_block[blk[plan.edges[e].u]];
            const int sv = node_of_block[blk[plan.edges[e].v]];
            g.adj[a] |= (1u << su) | (1u << sv);
            g.adj[su] |= 1u << a;
            g.adj[sv] |= 1u << a;
            tens.push_back({panel_vid[slot_of[2 * e]], {su, a}});
            tens.push_back({panel_vid[slot_of[2 * e + 1]], {sv, a}});
        }
        std::vector<int> order;
        if (g.N <= kLrDpMaxNodes) {
            order = order_dp(g);
            ++out.ndp;
        } else {
            order = order_greedy(g);
            ++out.ngreedy;
        }
        // A value from `ins`: summed over node x (x >= 0), or, with x < 0,
        // their elementwise product over the union of their indices (used to
        // cut a step with more than kLrMaxIn operands).
        std::string err;
        auto make_value = [&](const std::vector<Tensor> &ins, int x) -> Tensor {
            std::vector<int> onodes;
            for (auto &t : ins)
                for (int q : t.nodes)
                    if (q != x && std::find(onodes.begin(), onodes.end(), q) == onodes.end())
                        onodes.push_back(q);
            std::sort(onodes.begin(), onodes.end());  // the sample index (if any) first
            if ((int)onodes.size() > kLrMaxDim) err = "a low-rank value has more than 8 indices";
            int nsamp = 0;
            for (int q : onodes) nsamp += q < first_rank;
            if (nsamp > 1) err = "internal: low-rank order formed an n x n value";
            if (!err.empty()) return Tensor{-1, {}};
            // canonical key: (kind, sorted (input value, index map))
            std::vector<std::pair<int, std::vector<int>>> parts;
            for (auto &t : ins) {
                std::vector<int> mp;
                for (int q : t.nodes)
                    mp.push_back(q == x ? -1
                                        : (int)(std::find(onodes.begin(), onodes.end(), q) -
                                                onodes.begin()));
                parts.push_back({t.vid, mp});
            }
            std::sort(parts.begin(), parts.end());
            const bool long_x = x >= 0 && x < first_rank;
            std::vector<int64_t> key{x < 0 ? 2 : long_x ? 1 : 0, (int64_t)onodes.size()};
            for (auto &p : parts) {
                key.push_back(p.first);
                key.push_back((int64_t)p.second.size());
                for (int q : p.second) key.push_back(q);
            }
            double cost = x < 0 ? 1.0 : g.size[x];
            for (int q : onodes) cost *= g.size[q];
            if (cost > 1e15) err = "a low-rank value or step is too large";
            if (!err.empty()) return Tensor{-1, {}};
            out.flops_unmerged += cost;
            auto it = memo.find(key);
            if (it != memo.end()) return Tensor{it->second, onodes};
            LrValue v;
            v.kind = 1;
            v.long_x = long_x;
            v.nx = x < 0 ? 1 : long_x ? n : r;
            v.samp_first = !onodes.empty() && onodes[0] < first_rank;
            v.nd = (int)onodes.size();
            for (int d = 0; d < v.nd; ++d) {
                v.dims[d] = onodes[d] < first_rank ? n : r;
                v.size *= v.dims[d];
            }
            int lev = 0;
            for (auto &p : parts) {
                v.ins.push_back(p.first);
                v.maps.push_back(p.second);
                lev = std::max(lev, vals[p.first].level);
            }
            v.level = lev + 1;
            out.flops += cost;
            const int vid = (int)vals.size();
            vals.push_back(v);
            memo.emplace(key, vid);
            return Tensor{vid, onodes};
        };
        for (int x : order) {
            std::vector<Tensor> ins, rest;
            for (auto &t : tens)
                (std::find(t.nodes.begin(), t.nodes.end(), x) != t.nodes.end() ? ins : rest).push_back(t);
            while ((int)ins.size() > kLrMaxIn) {
                std::vector<Tensor> head(ins.begin(), ins.begin() + kLrMaxIn);
                Tensor t = make_value(head, -1);
                if (!err.empty()) return err;
                ins.erase(ins.begin(), ins.begin() + kLrMaxIn);
                ins.insert(ins.begin(), t);
            }
            Tensor t = make_value(ins, x);
            if (!err.empty()) return err;
            rest.push_back(t);
            tens.swap(rest);
        }
        std::vector<int> scal;
        for (auto &t : tens) {
            if (!t.nodes.empty()) return "internal: low-rank elimination left an index";
            scal.push_back(t.vid);
        }
        out.mu.push_back((double)mobius_mu(blk));
        out.cst.push_back(std::pow((double)n, (double)isolated));
        for (int s : scal) out.sc.push_back(s);  // value ids for now, offsets below
        out.sc_first.push_back((int32_t)out.sc.size());
    }
    out.nparts = (int)out.mu.size();

    // workspace: every step value, then one level's partial sums
    int64_t off = 0;
    int depth = 0;
    for (auto &v : vals) {
        if (v.kind != 1) continue;
        v.off = off;
        off += (v.size + 31) & ~int64_t(31);  // 256-byte aligned values
        depth = std::max(depth, v.level);
    }
    const int64_t values_end = off;
    out.depth = depth;
    out.nvalues = 0;
    for (auto &v : vals) out.nvalues += v.kind == 1;
    for (auto &s : out.sc) s = vals[s].off;

    // descriptors, level by level
    out.steps.clear();
    out.reds.clear();
    out.krs.clear();
    out.levels.assign(depth, LrLevel());
    int64_t part_max = 0;
    for (int L = 1; L <= depth; ++L) {
        LrLevel &lv = out.levels[L - 1];
        lv.steps_off = (int64_t)out.steps.size();
        lv.red_off = (int64_t)out.reds.size();
        lv.kr_off = (int64_t)out.krs.size();
        int64_t part_off = values_end, blocks = 0, rblocks = 0, krblocks = 0;
        // partial sums of a long step cut into nch chunks: the output goes
        // to a partial buffer and a reduce descriptor sums it into the value
        auto partials = [&](const LrValue &v, int64_t nch) -> int64_t {
            if (nch == 1) return v.off;
            LrReduceDesc rd;
            std::memset(&rd, 0, sizeof rd);
            rd.part = part_off;
            rd.out = v.off;
            rd.nout = v.size;
            rd.nchunk = (int32_t)nch;
            int64_t ot = 1;
            while (ot < v.size && ot < kLrThreads) ot <<= 1;
            while (ot > 16 && kLrThreads / ot * 8 < nch) ot >>= 1;  // at most ~8 chunks a lane
            rd.otile = (int32_t)ot;
            rd.clanes = (int32_t)(kLrThreads / ot);
            rd.block0 = rblocks;
            rblocks += (v.size + ot - 1) / ot;
            lv.red_bytes += 8.0 * (double)v.size * (double)(nch + 1);
            out.reds.push_back(rd);
            const int64_t at = part_off;
            part_off += (nch * v.size + 31) & ~int64_t(31);
            return at;
        };
        for (auto &v : vals) {
            if (v.kind != 1 || v.level != L) continue;
            const uint32_t split = v.long_x ? kr_split(v, vals) : 0;
            if (split) {
                LrKrDesc k;
                std::memset(&k, 0, sizeof k);
                int64_t ost[kLrMaxDim];
                value_strides(v, ost);
                uint32_t dlm = 0;
                for (size_t t = 0; t < v.ins.size(); ++t)
                    if (split >> t & 1)
                        for (int p : v.maps[t])
                            if (p >= 0) dlm |= 1u << p;
                int posl[kLrMaxDim], posr[kLrMaxDim];
                k.M = k.N = 1;
                for (int q = 0; q < v.nd; ++q) {
                    if (dlm >> q & 1) {
                        posl[k.ndl] = q;
                        k.dl[k.ndl] = (int32_t)v.dims[q];
                        k.ol[k.ndl++] = (int32_t)ost[q];
                        k.M *= (int32_t)v.dims[q];
                    } else {
                        posr[k.ndr] = q;
                        k.dr[k.ndr] = (int32_t)v.dims[q];
                        k.orr[k.ndr++] = (int32_t)ost[q];
                        k.N *= (int32_t)v.dims[q];
                    }
                }
                int cnt[2] = {0, 0};
                for (int side = 0; side < 2; ++side)
                    for (size_t t = 0; t < v.ins.size(); ++t) {
                        if ((split >> t & 1) != (side == 0 ? 1u : 0u)) continue;
                        const int u = side * kLrKrSide + cnt[side]++;
                        const LrValue &in = vals[v.ins[t]];
                        k.slot[u] = in.kind == 0 ? in.slot : 0;
                        k.base[u] = in.kind == 0 ? 0 : in.off;
                        int64_t ist[kLrMaxDim];
                        value_strides(in, ist);
                        const int nds = side == 0 ? k.ndl : k.ndr;
                        const int *pos = side == 0 ? posl : posr;
                        for (int q = 0; q < in.nd; ++q) {
                            const int p = v.maps[t][q];
                            if (p < 0) {
                                k.sx[u] += (int32_t)ist[q];
                                continue;
                            }
                            for (int d = 0; d < nds; ++d)
                                if (pos[d] == p) k.st[u][d] += (int32_t)ist[q];
                        }
                    }
                k.nl = cnt[0];
                k.nr = cnt[1];
                k.nx = (int32_t)v.nx;
                k.nout = (int32_t)v.size;
                if (k.M <= kLrKrSmall && k.N <= kLrKrSmallWide) k.small = 1;
                k.tiles_n = k.small ? 1 : (k.N + kLrKrTile - 1) / kLrKrTile;
                k.tiles = k.small ? 1 : ((k.M + kLrKrTile - 1) / kLrKrTile) * k.tiles_n;
                int64_t nch = std::min<int64_t>(32, std::max<int64_t>(1, (2048 + k.tiles - 1) / k.tiles));
                nch = std::min<int64_t>(nch, std::max<int64_t>(1, k.nx / 256));
                nch = std::min<int64_t>(nch, std::max<int64_t>(1, (((int64_t)1 << 31) - 1) / v.size));
                k.xchunk = (int32_t)(((k.nx + nch - 1) / nch + 15) / 16 * 16);
                nch = (k.nx + k.xchunk - 1) / k.xchunk;
                k.nchunk = (int32_t)nch;
                k.out = partials(v, nch);
                k.block0 = krblocks;
                krblocks += nch * k.tiles;
                lv.kr_flops += 2.0 * (double)k.M * (double)k.N * (double)k.nx;
                lv.kr_bytes += 8.0 * (double)v.size;
                for (int t : v.ins) lv.kr_bytes += 8.0 * (double)vals[t].size;
                out.krs.push_back(k);
                continue;
            }
            LrStepDesc d;
            std::memset(&d, 0, sizeof d);
            d.nin = (int32_t)v.ins.size();
            d.nd = v.nd;
            d.nx = v.nx;
            d.nout = v.size;
            for (int q = 0; q < v.nd; ++q) d.dim[q] = v.dims[q];
            for (int t = 0; t < d.nin; ++t) {
                const LrValue &in = vals[v.ins[t]];
                d.slot[t] = in.kind == 0 ? in.slot : 0;
                d.base[t] = in.kind == 0 ? 0 : in.off;
                int64_t stride = 1;
                for (int q = in.nd - 1; q >= 0; --q) {
                    const int p = v.maps[t][q];
                    if (p < 0) d.sx[t] += stride;
                    else d.so[t][p] += stride;
                    stride *= in.dims[q];
                }
            }
            d.block0 = blocks;
            lv.flops += (double)d.nout * (double)d.nx * d.nin;
            lv.bytes += 8.0 * (double)d.nout;
            for (int t = 0; t < d.nin; ++t) lv.bytes += 8.0 * (double)vals[v.ins[t]].size;
            if (!v.long_x) {
                d.mode = 0;
                d.nchunk = 1;
                d.xchunk = d.nx;
                d.otile = kLrThreads;
                d.xlanes = 1;
                d.out = v.off;
                blocks += (d.nout + kLrThreads - 1) / kLrThreads;
            } else {
                d.mode = 1;
                int64_t ot = 1;
                while (ot < d.nout && ot < kLrThreads) ot <<= 1;
                d.otile = (int32_t)ot;
                d.xlanes = (int32_t)(kLrThreads / ot);
                const int64_t ntile = (d.nout + ot - 1) / ot;
                // about 16 values of x per thread for small outputs (short
                // dependent chains; such steps are latency-bound), 64 for
                // larger ones (fewer partials); at most 4096 blocks per step
                const int64_t per = d.nout <= 256 ? 16 : 64;
                int64_t nch = (d.nx + d.xlanes * per - 1) / (d.xlanes * per);
                nch = std::max<int64_t>(1, std::min(nch, 4096 / ntile));
                d.xchunk = (d.nx + nch - 1) / nch;
                nch = (d.nx + d.xchunk - 1) / d.xchunk;
                d.nchunk = (int32_t)nch;
                d.out = partials(v, nch);
                blocks += ntile * nch;
            }
            out.steps.push_back(d);
        }
        lv.nsteps = (int64_t)out.steps.size() - lv.steps_off;
        lv.nred = (int64_t)out.reds.size() - lv.red_off;
        lv.nkr = (int64_t)out.krs.size() - lv.kr_off;
        lv.blocks = blocks;
        lv.rblocks = rblocks;
        lv.krblocks = krblocks;
        part_max = std::max(part_max, part_off - values_end);
    }
    out.part_elems = part_max;
    out.ws_elems = values_end + part_max;
    return "";
}

hipError_t upload_lowrank(LrSchedule &s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (s.blob && s.device == dev) return hipSuccess;
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 0;
    s.off_steps = off;
    off = align(off + s.steps.size() * sizeof(LrStepDesc));
    s.off_reds = off;
    off = align(off + s.reds.size() * sizeof(LrReduceDesc));
    s.off_krs = off;
    off = align(off + s.krs.size() * sizeof(LrKrDesc));
    s.off_mu = off;
    off = align(off + s.mu.size() * 8);
    s.off_cst = off;
    off = align(off + s.cst.size() * 8);
    s.off_first = off;
    off = align(off + s.sc_first.size() * 4);
    s.off_sc = off;
    off = align(off + s.sc.size() * 8);
    s.off_tab = off;
    off = align(off + (size_t)s.nslots * 8);
    s.off_res = off;
    off = align(off + 16);
    if (s.blob) (void)hipFree(s.blob);
    s.blob = nullptr;
    if (inject_fire(INJ_DEVICE_ALLOC)) return hipErrorOutOfMemory;
    e = hipMalloc(&s.blob, off);
    if (e != hipSuccess) return e;
    s.blob_bytes = off;
    s.device = dev;
    std::vector<char> h(off, 0);
    std::memcpy(h.data() + s.off_steps, s.steps.data(), s.steps.size() * sizeof(LrStepDesc));
    std::memcpy(h.data() + s.off_reds, s.reds.data(), s.reds.size() * sizeof(LrReduceDesc));
    std::memcpy(h.data() + s.off_krs, s.krs.data(), s.krs.size() * sizeof(LrKrDesc));
    std::memcpy(h.data() + s.off_mu, s.mu.data(), s.mu.size() * 8);
    std::memcpy(h.data() + s.off_cst, s.cst.data(), s.cst.size() * 8);
    std::memcpy(h.data() + s.off_first, s.sc_first.data(), s.sc_first.size() * 4);
    std::memcpy(h.data() + s.off_sc, s.sc.data(), s.sc.size() * 8);
    return hipMemcpy(s.blob, h.data(), off, hipMemcpyHostToDevice);
}

hipError_t run_lowrank(LrSchedule &s, const double *const *panels, double *ws, hipStream_t stream,
                       double *hres) {
    if (inject_fire(INJ_HIP)) return hipErrorLaunchFailure;
    std::vector<const double *> tab(s.nslots);
    tab[0] = ws;
    for (int k = 1; k < s.nslots; ++k) tab[k] = panels[k - 1];
    hipError_t e = hipMemcpyAsync(s.blob + s.off_tab, tab.data(), tab.size() * 8,
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    const auto *dtab = (const double *const *)(s.blob + s.off_tab);
    const auto *dsteps = (const LrStepDesc *)(s.blob + s.off_steps);
    const auto *dreds = (const LrReduceDesc *)(s.blob + s.off_reds);
    const auto *dkrs = (const LrKrDesc *)(s.blob + s.off_krs);
    Profiler *prof = Profiler::active();
    for (const LrLevel &lv : s.levels) {
        if (lv.nsteps) {
            ProfScope ps(prof, KIND_LR_STEP, stream, lv.flops, lv.bytes);
            launch_lr_steps(dsteps + lv.steps_off, lv.nsteps, lv.blocks, dtab, stream);
        }
        if (lv.nkr) {
            ProfScope ps(prof, KIND_LR_KR, stream, lv.kr_flops, lv.kr_bytes);
            launch_lr_kr(dkrs + lv.kr_off, lv.nkr, lv.krblocks, dtab, stream);
        }
        if (lv.nred) {
            ProfScope ps(prof, KIND_LR_REDUCE, stream, 0.0, lv.red_bytes);
            launch_lr_reduce(dreds + lv.red_off, lv.nred, lv.rblocks, ws, stream);
        }
    }
    double *dres = (double *)(s.blob + s.off_res);
    launch_lr_combine((const double *)(s.blob + s.off_mu), (const double *)(s.blob + s.off_cst),
                      (const int32_t *)(s.blob + s.off_first), (const int64_t *)(s.blob + s.off_sc),
                      s.nparts, ws, dres, stream);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(hres, dres, 16, hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(stream);
    if (e == hipSuccess && prof) prof->collect();
    return e;
}

}  // namespace ustat
