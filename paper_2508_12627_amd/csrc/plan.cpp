// Host-side planner.  Lemma 2 supplies the partitions and their Moebius
// coefficients, Algorithm 3 the induced notation (here: the quotient
// multigraph), Lemma 3 the optional sparsification filter, and the proof of
// Proposition 1 (one index summed out at a time) the lowering of an
// elimination order to kernel steps.
#include "plan.hpp"

#include "inject.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <limits>
#include <numeric>
#include <string>

namespace ustat {

std::vector<std::vector<int>> enumerate_rgs(int m) {
    std::vector<std::vector<int>> out;
    std::vector<int> a(m, 0);
    std::function<void(int, int)> rec = [&](int i, int mx) {
        if (i == m) {
            out.push_back(a);
            return;
        }
        for (int b = 0; b <= mx + 1; ++b) {
            a[i] = b;
            rec(i + 1, std::max(mx, b));
        }
    };
    if (m >= 1) {
        a[0] = 0;
        rec(1, 0);
    }
    return out;
}

int64_t mobius_mu(const std::vector<int> &block_of) {
    int m = (int)block_of.size();
    int J = 0;
    for (int b : block_of) J = std::max(J, b + 1);
    std::vector<int> size(J, 0);
    for (int b : block_of) size[b]++;
    int64_t p = 1;
    for (int s : size)
        for (int t = 2; t < s; ++t) p *= t;
    return ((m - J) % 2) ? -p : p;
}

bool survives_sparsification(const std::vector<int> &block_of, const std::vector<Edge> &edges) {
    for (const Edge &e : edges)
        if (block_of[e.u] == block_of[e.v]) return false;
    return true;
}

// Treewidth by the subset recurrence TW(S) = min_{v in S} max(TW(S\v),
// |Q(S\v, v)|), where Q(S, v) is the set of vertices outside S + v reachable
// from v through S; TW(V) is the treewidth (eliminating S first costs the
// largest such |Q|).
int exact_treewidth(int J, const std::vector<uint32_t> &adj) {
    if (J <= 1) return 0;
    const uint32_t full = (J >= 32) ? 0xffffffffu : ((1u << J) - 1);
    std::vector<int8_t> TW((size_t)full + 1, 0);
    auto Q = [&](uint32_t S, int v) {
        uint32_t seen = 1u << v, frontier = 1u << v, out = 0;
        while (frontier) {
            int x = __builtin_ctz(frontier);
            frontier &= frontier - 1;
            uint32_t nb = adj[x] & ~seen;
            seen |= nb;
            out |= nb & ~S;
            frontier |= nb & S;
        }
        return __builtin_popcount(out);
    };
    TW[0] = -1;
    for (uint32_t S = 1; S <= full; ++S) {
        int best = 127;
        for (uint32_t rest = S; rest; rest &= rest - 1) {
            int v = __builtin_ctz(rest);
            uint32_t Sv = S & ~(1u << v);
            int val = std::max<int>(TW[Sv], Q(Sv, v));
            best = std::min(best, val);
        }
        TW[S] = (int8_t)best;
        if (S == full) break;
    }
    return std::max<int>(0, TW[full]);
}

namespace {

struct LiveFactor {
    int val;
    int nv;    // 1 (vector) or 2 (matrix)
    int a, b;  // vars; for matrices (row, col) of the stored value
};

std::vector<uint32_t> quotient_adjacency(const std::vector<Edge> &edges,
                                         const std::vector<int> &block_of, int J) {
    std::vector<uint32_t> adj(J, 0);
    for (const Edge &e : edges) {
        int a = block_of[e.u], b = block_of[e.v];
        if (a != b) {
            adj[a] |= 1u << b;
            adj[b] |= 1u << a;
        }
    }
    return adj;
}

// Greedy min-fill.  Ties are broken by degree, then by how many of the
// vertex's factors are intermediates (results of earlier eliminations), then
// by whether it carries a vector (a self-loop diagonal or a degree-1
// result), then by id.  The last two keys favour contractions of input
// factors without diagonal scaling, which different partitions share.
std::vector<int> minfill_order(int J, std::vector<uint32_t> adj, std::vector<char> hasvec) {
    std::vector<int> order;
    std::vector<uint32_t> interm(J, 0);
    uint32_t alive = (J >= 32) ? 0xffffffffu : ((1u << J) - 1);
    while (alive) {
        int best = -1;
        long best_key = std::numeric_limits<long>::max();
        for (uint32_t r = alive; r; r &= r - 1) {
            int v = __builtin_ctz(r);
            uint32_t nb = adj[v] & alive;
            int fill = 0;
            for (uint32_t p = nb; p; p &= p - 1) {
                int x = __builtin_ctz(p);
                fill += __builtin_popcount(nb & ~adj[x] & ~(1u << x));
            }
            fill /= 2;
            long key = ((long)fill << 40) | ((long)__builtin_popcount(nb) << 32) |
                       ((long)__builtin_popcount(interm[v] & alive) << 24) |
                       ((long)(hasvec[v] ? 1 : 0) << 16) | v;
            if (key < best_key) {
                best_key = key;
                best = v;
            }
        }
        uint32_t nb = adj[best] & alive & ~(1u << best);
        for (uint32_t p = nb; p; p &= p - 1) {
            int x = __builtin_ctz(p);
            adj[x] |= nb & ~(1u << x);
            interm[x] |= nb & ~(1u << x);
        }
        if (__builtin_popcount(nb) == 1) hasvec[__builtin_ctz(nb)] = 1;
        alive &= ~(1u << best);
        order.push_back(best);
    }
    return order;
}

}  // namespace

std::string lower_order(const std::vector<Edge> &edges, const std::vector<int> &block_of, int J,
                        const std::vector<int> &order, VProgram &out, int slice_var) {
    out.vals.clear();
    out.steps.clear();
    out.scalars.clear();
    out.order = order;
    out.width = 0;
    out.slice_var = slice_var;
    std::vector<LiveFactor> live;
    // Conditioning on slice_var: its self-loop diagonals scale one slice
    // vector (every edge at slice_var becomes a slice vector).
    std::vector<int> slice_diag;
    int first_slice = -1;
    if (slice_var >= 0)
        for (size_t k = 0; k < edges.size(); ++k) {
            int a = block_of[edges[k].u], b = block_of[edges[k].v];
            if (a == slice_var && b == slice_var) slice_diag.push_back((int)k);
            else if ((a == slice_var || b == slice_var) && first_slice < 0) first_slice = (int)k;
        }
    if (slice_var >= 0 && first_slice < 0) return "conditioning on a vertex without edges";
    for (size_t k = 0; k < edges.size(); ++k) {
        int a = block_of[edges[k].u], b = block_of[edges[k].v];
        Value val;
        val.src = (int)k;
        if (slice_var >= 0 && (a == slice_var || b == slice_var)) {
            if (a == b) continue;  // folded into the first slice vector
            val.kind = ValKind::SliceVec;
            val.r = (a == slice_var) ? b : a;
            val.c = (a == slice_var) ? 0 : 1;
            if ((int)k == first_slice) val.scale = slice_diag;
            live.push_back({(int)out.vals.size(), 1, val.r, -1});
            out.vals.push_back(val);
            continue;
        }
        if (a == b) {
            val.kind = ValKind::InputDiag;
            val.r = a;
            val.c = -1;
            live.push_back({(int)out.vals.size(), 1, a, -1});
        } else {
            val.kind = ValKind::InputMat;
            val.r = a;
            val.c = b;
            live.push_back({(int)out.vals.size(), 2, a, b});
        }
        out.vals.push_back(val);
    }
    std::vector<char> gone(J, 0);
    if (slice_var >= 0) gone[slice_var] = 1;
    std::vector<int> val_level;  // level of each value
    auto level_of = [&](int val) {
        const Value &v = out.vals[val];
        if (v.kind == ValKind::InputMat || v.kind == ValKind::InputDiag ||
            v.kind == ValKind::SliceVec)
            return 0;
        return out.steps[v.src].level;
    };
    for (int v : order) {
        if (v < 0 || v >= J) return "order names a vertex outside the quotient";
        if (v == slice_var) continue;
        if (gone[v]) continue;
        std::vector<LiveFactor> touch, keep;
        for (const LiveFactor &f : live) {
            bool hit = (f.a == v) || (f.nv == 2 && f.b == v);
            (hit ? touch : keep).push_back(f);
        }
        live.swap(keep);
        std::vector<int> nbrs;
        for (const LiveFactor &f : touch)
            if (f.nv == 2) {
                int o = (f.a == v) ? f.b : f.a;
                if (std::find(nbrs.begin(), nbrs.end(), o) == nbrs.end()) nbrs.push_back(o);
            }
        std::sort(nbrs.begin(), nbrs.end());
        gone[v] = 1;
        std::vector<int> remaining;
        for (int q = 0; q < J; ++q)
            if (!gone[q]) remaining.push_back(q);
        int deg = (int)nbrs.size();
        out.width = std::max(out.width, deg);
        Step st;
        st.v = v;
        for (const LiveFactor &f : touch)
            if (f.nv == 1) st.sv.push_back(f.val);
        auto take_vecs = [&](int var, std::vector<int> &dst) {
            std::vector<LiveFactor> k2;
            for (const LiveFactor &f : live) {
                if (f.nv == 1 && f.a == var) dst.push_back(f.val);
                else k2.push_back(f);
            }
            live.swap(k2);
        };
        Value res;
        res.src = (int)out.steps.size();
        res.r = res.c = -1;
        if (deg == 0) {
            st.kind = StepKind::Elim0;
            res.kind = ValKind::Scalar;
        } else if (deg == 1) {
            int w = nbrs[0];
            st.w = w;
            for (const LiveFactor &f : touch)
                if (f.nv == 2) st.A.push_back({f.val, f.a != v});
            if (remaining.size() == 1 && remaining[0] == w) {
                st.kind = StepKind::Final1;
                take_vecs(w, st.aw);
                gone[w] = 1;
                res.kind = ValKind::Scalar;
            } else {
                st.kind = StepKind::Elim1;
                res.kind = ValKind::Vec;
                res.r = w;
            }
        } else if (deg == 2) {
            int w = nbrs[0], x = nbrs[1];
            st.w = w;
            st.x = x;
            for (const LiveFactor &f : touch)
                if (f.nv == 2) {
                    int o = (f.a == v) ? f.b : f.a;
                    (o == w ? st.A : st.B).push_back({f.val, f.a != v});
                }
            if (remaining.size() == 2 && remaining[0] == w && remaining[1] == x) {
                st.kind = StepKind::Final2;
                std::vector<LiveFactor> k2;
                for (const LiveFactor &f : live) {
                    if (f.nv == 2) st.Z.push_back({f.val, f.a != w});
                    else k2.push_back(f);
                }
                live.swap(k2);
                take_vecs(w, st.aw);
                take_vecs(x, st.bx);
                gone[w] = gone[x] = 1;
                res.kind = ValKind::Scalar;
            } else {
                st.kind = StepKind::Elim2;
                res.kind = ValKind::Mat;
                res.r = w;
                res.c = x;
            }
        } else {
            return "elimination degree " + std::to_string(deg) + " is not supported";
        }
        int lvl = 0;
        auto bump = [&](int val) { lvl = std::max(lvl, level_of(val)); };
        for (auto &o : st.A) bump(o.val);
        for (auto &o : st.B) bump(o.val);
        for (auto &o : st.Z) bump(o.val);
        for (int q : st.sv) bump(q);
        for (int q : st.aw) bump(q);
        for (int q : st.bx) bump(q);
        st.level = lvl + 1;
        st.out = (int)out.vals.size();
        out.vals.push_back(res);
        out.steps.push_back(st);
        if (res.kind == ValKind::Scalar) {
            out.scalars.push_back(st.out);
        } else if (res.kind == ValKind::Vec) {
            live.push_back({st.out, 1, res.r, -1});
        } else {
            live.push_back({st.out, 2, res.r, res.c});
        }
    }
    if (!live.empty()) return "elimination order left factors unconsumed";
    out.depth = 0;
    for (const Step &s : out.steps) out.depth = std::max(out.depth, s.level);
    if (slice_var >= 0) out.width += 1;  // the summed-over conditioned vertex
    (void)val_level;
    return "";
}

std::vector<char> slice_dependent_steps(const VProgram &p) {
    std::vector<char> vdep(p.vals.size(), 0), sdep(p.steps.size(), 0);
    if (p.slice_var < 0) return sdep;
    for (size_t v = 0; v < p.vals.size(); ++v) vdep[v] = p.vals[v].kind == ValKind::SliceVec;
    for (size_t i = 0; i < p.steps.size(); ++i) {
        const Step &s = p.steps[i];
        bool d = false;
        for (auto *g : {&s.A, &s.B, &s.Z})
            for (auto &o : *g) d = d || vdep[o.val];
        for (auto *g : {&s.sv, &s.aw, &s.bx})
            for (int q : *g) d = d || vdep[q];
        sdep[i] = d;
        if (s.out >= 0) vdep[s.out] = d;
    }
    return sdep;
}

// Algorithmic work of one evaluation at size n.  In a conditioned program
// the steps that depend on the conditioned vertex run once per slice (n
// times); the others run once, since the executor shares them across slices.
void program_cost(const VProgram &p, double n, double elem_bytes, double *flops, double *bytes) {
    double f = 0, b = 0;
    const std::vector<char> dep = slice_dependent_steps(p);
    for (size_t i = 0; i < p.steps.size(); ++i) {
        const Step &s = p.steps[i];
        const double rep = dep[i] ? n : 1.0;
        switch (s.kind) {
            case StepKind::Elim0:
                f += rep * 2 * n * std::max<size_t>(1, s.sv.size());
                b += rep * 8 * n * s.sv.size();
                break;
            case StepKind::Elim1:
            case StepKind::Final1:
                f += rep * 2 * n * n * s.A.size();
                b += rep * elem_bytes * n * n * s.A.size();
                break;
            case StepKind::Elim2:
            case StepKind::Final2:
                f += rep * 2 * n * n * n;
                b += rep * elem_bytes * n * n *
                     (s.A.size() + s.B.size() + s.Z.size() + (s.kind == StepKind::Elim2 ? 1 : 0));
                break;
        }
    }
    if (flops) *flops = f;
    if (bytes) *bytes = b;
}

std::vector<float> program_features(const VProgram &p, double n) {
    // Counts per step kind, operand counts, transposition counts, depth,
    // and log-size terms; the learned model maps them to a log-time.
    float c[5] = {0, 0, 0, 0, 0};
    float nA = 0, nTransA = 0, nZ = 0, nVec = 0, nPrep = 0;
    for (const Step &s : p.steps) {
        c[(int)s.kind] += 1;
        nA += (float)(s.A.size() + s.B.size());
        for (auto &o : s.A) nTransA += o.trans ? 0.f : 1.f;
        for (auto &o : s.B) nTransA += o.trans ? 0.f : 1.f;
        nZ += (float)s.Z.size();
        nVec += (float)(s.sv.size() + s.aw.size() + s.bx.size());
        if (s.kind == StepKind::Elim2 || s.kind == StepKind::Final2) {
            bool directA = s.A.size() == 1 && s.A[0].trans && s.sv.empty();
            bool directB = s.B.size() == 1 && s.B[0].trans;
            nPrep += (directA ? 0.f : 1.f) + (directB ? 0.f : 1.f);
        }
    }
    float ln = (float)std::log(n);
    // the work model behind the exhaustive policy, as log flops and bytes,
    // and the GEMM steps repeated per slice of a conditioned program
    double fl, by;
    program_cost(p, n, 4.0, &fl, &by);
    const std::vector<char> dep = slice_dependent_steps(p);
    float dep_gemm = 0;
    for (size_t i = 0; i < p.steps.size(); ++i)
        if (dep[i] && (p.steps[i].kind == StepKind::Elim2 || p.steps[i].kind == StepKind::Final2))
            dep_gemm += 1;
    std::vector<float> f = {c[0], c[1], c[2], c[3], c[4], nA, nTransA, nZ, nVec, nPrep,
                            (float)p.depth, (float)p.width, ln, ln * (c[3] + c[4]),
                            ln * (c[1] + c[2]), (float)std::log(std::max(fl, 1.0)),
                            (float)std::log(std::max(by, 1.0)), dep_gemm};
    return f;
}

// Count of GEMM steps with a diagonal scaling plus GEMM operand groups that
// contain an intermediate value.
static int sharing_penalty(const VProgram &p) {
    int pen = 0;
    for (const Step &s : p.steps) {
        if (s.kind != StepKind::Elim2 && s.kind != StepKind::Final2) continue;
        if (!s.sv.empty()) ++pen;
        auto interm = [&](const std::vector<MatOp> &g) {
            for (auto &o : g)
                if (p.vals[o.val].kind == ValKind::Mat) return true;
            return false;
        };
        pen += interm(s.A) + interm(s.B);
    }
    return pen;
}

std::string build_program(const std::vector<Edge> &edges, int m, const std::vector<int> &block_of,
                          const PlanOptions &opts, const OrderScorer *scorer, VProgram &out) {
    inject_host_alloc();
    int J = 0;
    for (int b : block_of) J = std::max(J, b + 1);
    out.block_of = block_of;
    out.J = J;
    out.mu = mobius_mu(block_of);
    auto adj = quotient_adjacency(edges, block_of, J);
    out.tw = exact_treewidth(J, adj);
    (void)m;
    std::vector<char> hasvec(J, 0);
    for (const Edge &e : edges)
        if (block_of[e.u] == block_of[e.v]) hasvec[block_of[e.u]] = 1;
    const double nref = opts.n_hint;
    // Time proxy of a lowered program: MFMA work plus memory traffic plus a
    // per-level launch latency, in seconds at nominal rates; among equal
    // proxies, contractions of input factors without diagonal scaling are
    // preferred, since they can be shared across partitions.
    auto proxy_key = [&](const VProgram &p) {
        double f, b;
        program_cost(p, nref, 4.0, &f, &b);
        return f / 100e12 + b / 5e12 + p.depth * 8e-6 + 1e-9 * sharing_penalty(p);
    };
    auto keep_program = [&](VProgram &p) {
        p.block_of = out.block_of;
        p.J = out.J;
        p.mu = out.mu;
        p.tw = out.tw;
        p.executable = true;
        p.lower_error.clear();
        out = std::move(p);
    };
    std::vector<int> mf = minfill_order(J, adj, hasvec);
    std::string first_err;
    // Candidate programs: every plain order (J <= 8), or, when none stays
    // within degree 2, every (conditioned vertex c, order of the others).
    auto plain_candidates = [&](auto &&cb) {
        std::vector<int> cur(J);
        std::iota(cur.begin(), cur.end(), 0);
        do {
            VProgram tmp;
            std::string err = lower_order(edges, block_of, J, cur, tmp);
            if (!err.empty()) {
                if (first_err.empty()) first_err = err;
                continue;
            }
            cb(tmp);
        } while (std::next_permutation(cur.begin(), cur.end()));
    };
    auto conditioned_candidates = [&](auto &&cb) {
        for (int c = 0; c < J; ++c) {
            std::vector<int> rest;
            for (int q = 0; q < J; ++q)
                if (q != c) rest.push_back(q);
            do {
                VProgram cand;
                if (lower_order(edges, block_of, J, rest, cand, c).empty()) cb(cand);
            } while (std::next_permutation(rest.begin(), rest.end()));
        }
    };
    // Search policies rank only among the candidates of smallest width (the
    // width sets the power of n in the work).  Exhaustive keeps the smallest
    // proxy.  Learned lets the model choose among the candidates whose
    // modelled work is close to the least and that share steps across
    // partitions at least as well (the model, trained on partitions timed
    // alone, sees neither sharing nor work gaps outside its training range):
    // the smallest predicted log-time wins, predictions within kLearnedTie of
    // it (about the model's error) count as ties, and the proxy breaks ties.
    const bool learned = opts.order == 2 && scorer;
    constexpr double kLearnedTie = 0.1, kLearnedGate = 0.25;
    auto search_select = [&](auto &&candidates) {
        int wmin = std::numeric_limits<int>::max(), share_at_min = 0;
        double kmin = std::numeric_limits<double>::infinity();
        candidates([&](VProgram &c) {
            if (c.width < wmin) {
                wmin = c.width;
                kmin = std::numeric_limits<double>::infinity();
            }
            if (c.width == wmin) {
                const double k = proxy_key(c);
                if (k < kmin) {
                    kmin = k;
                    share_at_min = sharing_penalty(c);
                }
            }
        });
        if (wmin == std::numeric_limits<int>::max()) return false;
        // learned: the model chooses among the candidates whose modelled
        // work is within kLearnedGate of the least and that are at least as
        // shareable as the proxy's choice (which always qualifies)
        auto gated = [&](const VProgram &c) {
            if (c.width != wmin) return false;
            if (!learned) return true;
            return proxy_key(c) <= kmin * (1.0 + kLearnedGate) && sharing_penalty(c) <= share_at_min;
        };
        double pmin = std::numeric_limits<double>::infinity();
        if (learned)
            candidates([&](VProgram &c) {
                if (gated(c)) pmin = std::min(pmin, scorer->score(program_features(c, nref)));
            });
        VProgram best_p;
        double best = std::numeric_limits<double>::infinity();
        candidates([&](VProgram &c) {
            if (!gated(c)) return;
            if (learned && scorer->score(program_features(c, nref)) > pmin + kLearnedTie) return;
            const double k = proxy_key(c);
            if (k < best - 1e-15) {
                best = k;
                best_p = std::move(c);
            }
        });
        keep_program(best_p);
        return true;
    };
    const bool search = opts.order != 0 && J > 1 && J <= 8;
    if (search) {
        if (search_select(plain_candidates)) return "";
        if (search_select(conditioned_candidates)) return "";
    } else {
        // Min-fill: its own order; failing that, for every conditioned
        // vertex c the min-fill order of the graph without c, keeping the
        // smallest work.
        VProgram tmp;
        std::string err = lower_order(edges, block_of, J, mf, tmp);
        if (err.empty()) {
            keep_program(tmp);
            return "";
        }
        first_err = err;
        VProgram best_p;
        double best = std::numeric_limits<double>::infinity();
        for (int c = 0; c < J; ++c) {
            std::vector<uint32_t> a2 = adj;
            for (int q = 0; q < J; ++q) a2[q] &= ~(1u << c);
            a2[c] = 0;
            std::vector<char> hv = hasvec;
            for (int q = 0; q < J; ++q)
                if (adj[c] & (1u << q)) hv[q] = 1;
            std::vector<int> rest;
            for (int v : minfill_order(J, a2, hv))
                if (v != c) rest.push_back(v);
            VProgram cand;
            if (!lower_order(edges, block_of, J, rest, cand, c).empty()) continue;
            double f, b;
            program_cost(cand, nref, 4.0, &f, &b);
            if (f < best) {
                best = f;
                best_p = std::move(cand);
            }
        }
        if (std::isfinite(best)) {
            keep_program(best_p);
            return "";
        }
    }
    out.executable = false;
    out.lower_error = first_err;
    out.order = mf;
    return "";
}

std::string make_plan(int m, const std::vector<Edge> &edges, const PlanOptions &opts,
                      const OrderScorer *scorer, Plan &out) {
    inject_host_alloc();
    if (m < 1 || m > kMaxM) return "m must be in 1..10";
    if (edges.empty()) return "the kernel graph needs at least one edge";
    std::vector<char> used(m, 0);
    for (const Edge &e : edges) {
        if (e.u < 0 || e.u >= m || e.v < 0 || e.v >= m) return "edge endpoint out of range";
        if (e.u == e.v) return "self-loop edges are not allowed";
        used[e.u] = used[e.v] = 1;
    }
    for (int i = 0; i < m; ++i)
        if (!used[i]) return "every vertex must appear in some edge";
    out.m = m;
    out.edges = edges;
    out.opts = opts;
    out.progs.clear();
    out.N_l.assign(m + 1, 0);
    out.M = 0;
    out.max_width = 0;
    for (const auto &rgs : enumerate_rgs(m)) {
        if (opts.sparsify && !survives_sparsification(rgs, edges)) continue;
        VProgram p;
        std::string err = build_program(edges, m, rgs, opts, scorer, p);
        if (!err.empty()) return err;
        out.N_l[p.tw]++;
        out.M = std::max(out.M, p.tw);
        if (!p.executable && out.executable) {
            out.executable = false;
            out.lower_error = p.lower_error;
        }
        out.max_width = std::max(out.max_width, p.width);
        out.progs.push_back(std::move(p));
    }
    return "";
}

}  // namespace ustat
