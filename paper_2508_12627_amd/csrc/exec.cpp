// Executor.  All steps of all restricted V-statistics (and of all datasets
// of a batch) are grouped by dependency level; each level issues at most one
// launch per step kind: operand prep, GEMM, column reduction, deg-0
// reduction, then the fixed-order partial reductions.  A final launch forms
// V_pi as the product of its scalars and the Moebius combination
// U = sum mu_pi V_pi (Lemma 2) with S = sum |mu_pi V_pi|.
#include "exec.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <unordered_map>

#include "inject.hpp"
#include "kernels.hpp"
#include "profile.hpp"

namespace ustat {

void Runtime::drop_graphs() {
    for (auto &kv : graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.blob) (void)hipFree(kv.second.blob);
    }
    graphs.clear();
}

hipError_t Runtime::reserve_side(size_t levels) {
    if (!side) {
        hipError_t e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
        if (e != hipSuccess) {
            side = nullptr;
            return e;
        }
    }
    while (level_events.size() < 2 * levels) {
        hipEvent_t ev;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        level_events.push_back(ev);
    }
    return hipSuccess;
}

Runtime::~Runtime() {
    drop_graphs();
    for (hipEvent_t ev : level_events) (void)hipEventDestroy(ev);
    if (side) (void)hipStreamDestroy(side);
    if (arena) (void)hipFree(arena);
    if (ddesc) (void)hipFree(ddesc);
    if (hdesc) (void)hipHostFree(hdesc);
    if (hres) (void)hipHostFree(hres);
    if (vacc) (void)hipFree(vacc);
}

hipError_t Runtime::reserve_arena(size_t bytes) {
    if (inject_fire(INJ_DEVICE_ALLOC)) return hipErrorOutOfMemory;
    if (bytes <= arena_bytes && arena) return hipSuccess;
    drop_graphs();
    if (arena) (void)hipFree(arena);
    arena = nullptr;
    arena_bytes = 0;
    hipError_t e = hipMalloc(&arena, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) arena_bytes = bytes;
    return e;
}

hipError_t Runtime::reserve_desc(size_t bytes) {
    if (inject_fire(INJ_DEVICE_ALLOC)) return hipErrorOutOfMemory;
    if (bytes <= ddesc_bytes && ddesc) return hipSuccess;
    drop_graphs();
    if (ddesc) (void)hipFree(ddesc);
    if (hdesc) (void)hipHostFree(hdesc);
    ddesc = hdesc = nullptr;
    ddesc_bytes = hdesc_bytes = 0;
    size_t b = std::max<size_t>(bytes * 3 / 2, 1 << 16);
    hipError_t e = hipMalloc(&ddesc, b);
    if (e != hipSuccess) return e;
    e = hipHostMalloc((void **)&hdesc, b, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    ddesc_bytes = hdesc_bytes = b;
    return hipSuccess;
}

hipError_t Runtime::reserve_vacc(size_t bytes) {
    if (inject_fire(INJ_DEVICE_ALLOC)) return hipErrorOutOfMemory;
    if (bytes <= vacc_bytes && vacc) return hipSuccess;
    drop_graphs();
    if (vacc) (void)hipFree(vacc);
    vacc = nullptr;
    vacc_bytes = 0;
    hipError_t e = hipMalloc(&vacc, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) vacc_bytes = bytes;
    return e;
}

hipError_t Runtime::reserve_hres(size_t bytes) {
    if (inject_fire(INJ_DEVICE_ALLOC)) return hipErrorOutOfMemory;
    if (bytes <= hres_bytes && hres) return hipSuccess;
    drop_graphs();
    if (hres) (void)hipHostFree(hres);
    hres = nullptr;
    size_t b = std::max<size_t>(bytes * 3 / 2, 4096);
    hipError_t e = hipHostMalloc((void **)&hres, b, hipHostMallocDefault);
    if (e == hipSuccess) hres_bytes = b;
    return e;
}

namespace {

constexpr size_t kAlign = 256;
inline size_t up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t up64(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// First-fit offset allocator with coalescing (host-side bookkeeping of the
// device arena; offsets only).
struct Arena {
    std::map<size_t, size_t> free_;
    size_t top = 0;
    size_t alloc(size_t bytes) {
        bytes = up(std::max<size_t>(bytes, 1), kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                size_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > bytes) free_[off + bytes] = sz - bytes;
                return off;
            }
        }
        size_t off = top;
        top += bytes;
        return off;
    }
    void release(size_t off, size_t bytes) {
        bytes = up(std::max<size_t>(bytes, 1), kAlign);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Append-only blob of descriptor arrays (copied to the device in one go).
struct Blob {
    std::vector<char> h;
    template <class T>
    size_t put(const std::vector<T> &v) {
        size_t off = up(h.size(), 64);
        h.resize(off + sizeof(T) * v.size());
        if (!v.empty()) std::memcpy(h.data() + off, v.data(), sizeof(T) * v.size());
        return off;
    }
};

struct LevelWork {
    std::vector<PrepDesc> prep;
    int64_t prep_tiles = 0;
    std::vector<GemmDesc> gemm;
    int64_t gemm_tiles = 0;
    double gemm_flops = 0;
    // problems of the level on 256-wide tiles, in a launch of their own
    std::vector<GemmDesc> gemm_big;
    int64_t gemm_big_tiles = 0;
    double gemm_big_flops = 0;
    bool big = false;  // the level's eligible GEMMs take 256-wide tiles
    size_t off_gemm_big = 0;
    // symmetric products P P^T on 256-wide tiles (stream-K over the tiles on
    // and above the diagonal, then the fix-up of split tiles)
    std::vector<GemmDesc> gemm_sym;
    int64_t gemm_sym_units = 0, gemm_sym_nk = 0, gemm_sym_tiles = 0;
    double gemm_sym_flops = 0;
    int sym_blocks = 0;
    float *sym_part = nullptr;
    size_t off_gemm_sym = 0;
    // split-bf16 problems on three-plane operands (six products per pair)
    std::vector<GemmDesc> gemm6;
    int64_t gemm6_tiles = 0;
    double gemm6_flops = 0;
    size_t off_gemm6 = 0;
    std::vector<Elim1Desc> e1;  // column reductions over more than kColMat matrices
    int64_t e1_tiles = 0;
    // grouped column reductions, one launch per slot: slot nm - 1 in column
    // mode, kColMat + nm - 1 in row mode (nm distinct matrices)
    static constexpr int kColSlots = 2 * kColMat;
    std::vector<ColDesc> col[kColSlots];
    int64_t col_tiles[kColSlots] = {0, 0, 0, 0, 0, 0};
    double col_bytes[kColSlots] = {0, 0, 0, 0, 0, 0};  // algorithmic HBM bytes per launch
    int col_maxout[kColSlots] = {0, 0, 0, 0, 0, 0};     // largest output count of a group
    // DType of every matrix, -1 if mixed, -2 none yet
    int col_dtype[kColSlots] = {-2, -2, -2, -2, -2, -2};
    size_t off_col[kColSlots] = {0, 0, 0, 0, 0, 0};
    double e1_bytes = 0, prep_bytes = 0, tr_bytes = 0;  // algorithmic HBM bytes
    std::vector<TransDesc> tr;
    int64_t tr_tiles = 0;
    size_t off_tr = 0;
    std::vector<SliceDesc> sl;
    int64_t sl_tiles = 0;
    size_t off_sl = 0;
    std::vector<Elim0Desc> e0;
    std::vector<ReduceDesc> red;
    int64_t red_maxlen = 1;
    size_t off_prep = 0, off_gemm = 0, off_e1 = 0, off_e0 = 0, off_red = 0;
};

int limbs_for(double bound, int cap) {
    int L = 1;
    double X = bound;
    while (X > 127.0 && L < cap) {
        X = std::floor((X + 64.0) / 128.0);
        ++L;
    }
    return L;
}

struct Schedule {
    // arena layout
    size_t arena_bytes = 0;
    // fixed regions (offsets in arena)
    size_t off_scal = 0, off_v = 0, off_mx = 0, off_limbs = 0,
           off_inmx = 0;
    size_t n_scal = 0, n_mx = 0, n_limbs = 0, n_inmx = 0;
    std::vector<DiagDesc> diag;
    int64_t diag_maxn = 1;
    std::vector<LevelWork> levels;
    std::vector<CombineDesc> comb;
    std::vector<int32_t> term_off, term_cnt, scal_off, scal_cnt, scal_idx;
    std::vector<int64_t> mu;
    size_t off_diag = 0, off_comb = 0, off_toff = 0, off_tcnt = 0, off_soff = 0, off_scnt = 0,
           off_sidx = 0, off_mu = 0;
    size_t blob_bytes = 0;
    Blob blob;
    int nprog_total = 0;
    size_t n_nodes = 0;
    int depth = 0;                 // dependency levels of the DAG
    std::vector<char> two_plane;   // per dataset: a GEMM took two-plane split-bf16
};

struct Cfg {
    int in_es;     // input element size (set in make_cfg)
    int prec;      // ustat_precision
    int domain;    // DOM_FP / DOM_INT
    int in_dt;     // input factor dtype
    int mat_dt;    // intermediate matrix dtype
    int mat_es;    // its element size
    int pformat;   // prep format
    int wide_es;   // scalar element size
};

Cfg make_cfg(int prec) {
    Cfg c;
    switch (prec) {
        case 0: c = {8, 0, DOM_FP, DT_F64, DT_F64, 8, PF_F64, 8}; break;
        case 1: c = {4, 1, DOM_FP, DT_F32, DT_F32, 4, PF_F32, 8}; break;
        case 2: c = {4, 2, DOM_FP, DT_F32, DT_F32, 4, PF_BF16X2, 8}; break;
        default: c = {1, 3, DOM_INT, DT_I8, DT_I64, 8, PF_I8LIMBS, 16}; break;
    }
    return c;
}

size_t prep_bytes(int pformat, int64_t npad, int limbs) {
    size_t plane = (size_t)npad * (size_t)npad;
    switch (pformat) {
        case PF_F64: return plane * 8;
        case PF_F32: return plane * 4;
        case PF_BF16X2: return plane * 4;
        case PF_BF16X3: return plane * 6;
        default: return plane * (size_t)limbs;
    }
}

// Split-bf16 GEMMs below this size always take the three-plane scheme: the
// two-plane scheme's per-product residual (up to about 3 * 2^-18 relative)
// is only averaged down to fp32 level by long sums of same-sign terms.
constexpr int64_t kSplit6Below = 1024;

// ---------------------------------------------------------------------------
// Node DAG.  Every step of every (dataset, V-statistic) program becomes a
// node keyed by a canonical signature of its operation and operands (input
// factor pointers or upstream nodes, with orientation).  Equal signatures
// denote the same values, so repeated work across partitions (and across
// datasets that share inputs) is computed once.  All kernels are
// deterministic, so this does not change any result bit.
// ---------------------------------------------------------------------------

enum class NK : uint8_t { E0, E1, Dot, GemmStore, GemmFinal, Transpose, SliceSrc };

struct MOp {        // matrix operand
    int node;       // producing node, or -1 for an input factor
    const void *p;  // input factor pointer when node < 0
    bool trans;     // relative to the consuming step's canonical orientation
};
struct VOp {        // vector operand
    int node;       // producing node, or -1 for the diagonal of input factor p
    const void *p;
    int64_t off = 0;  // element offset into the node's buffer (slice rows)
};

struct Node {
    NK kind;
    int d = 0;
    int64_t n = 0;
    std::vector<MOp> A, B, Z;
    std::vector<VOp> sv, aw, bx;
    int level = 0, last_use = 0;
    // a stored matrix equal to its transpose: a product sum_v A(w,v) s(v)
    // A(x,v) whose two operand groups are the same
    bool sym = false;
    // storage
    size_t off = 0, bytes = 0;
    int scal = -1, mx = -1;
    double bound = 0;
    bool neg = false;  // may hold negative entries (split-bf16 scheme choice)
    // Transpose: source (node or input pointer) in A[0]
};

struct Ref {  // a program value resolved to a node or an input
    int node = -1;
    const void *p = nullptr;
    bool flip = false;  // stored transposed relative to the program value
    int64_t off = 0;    // slice row offset (slice vectors)
};

// Fixed-width binary key fragments (keys are only compared and hashed):
// every fragment starts with a tag byte that never equals a separator, so
// concatenations stay unambiguous.
std::string ptr_id(const void *p) { return std::string(reinterpret_cast<const char *>(&p), sizeof p); }
std::string int_id(int64_t v) { return std::string(reinterpret_cast<const char *>(&v), sizeof v); }

struct Dag {
    std::vector<Node> nodes;
    std::unordered_map<std::string, int> by_key;
    // per (dataset, program), dataset-major: terms, each a list of scalar
    // nodes whose product is the term (one term, or one per slice)
    std::vector<std::vector<std::vector<int>>> prog_terms;
    // distinct input diagonals (dataset, factor pointer)
    std::map<std::pair<int, const void *>, int> diag_index;
    int max_level = 0;
};

std::string mop_sig(const MOp &m) {
    return (m.node < 0 ? "I" + ptr_id(m.p) : "N" + int_id(m.node)) + (m.trans ? "t" : "n");
}
std::string vop_sig(const VOp &v) {
    std::string s = v.node < 0 ? "D" + ptr_id(v.p) : "N" + int_id(v.node);
    if (v.off) s += "+" + int_id(v.off);
    return s;
}
template <class T, class F>
std::string group_sig(const std::vector<T> &v, F f) {
    std::vector<std::string> s;
    for (auto &x : v) s.push_back(f(x));
    std::sort(s.begin(), s.end());
    std::string out;
    for (auto &x : s) out += x + ",";
    return out;
}

int node_level(const Dag &G, const Node &nd) {
    int l = 0;
    auto m = [&](int id) {
        if (id >= 0) l = std::max(l, G.nodes[id].level);
    };
    for (auto &o : nd.A) m(o.node);
    for (auto &o : nd.B) m(o.node);
    for (auto &o : nd.Z) m(o.node);
    for (auto &o : nd.sv) m(o.node);
    for (auto &o : nd.aw) m(o.node);
    for (auto &o : nd.bx) m(o.node);
    return l + 1;
}

int add_node(Dag &G, Node nd, const std::string &key, bool cse);

// An operand read in the orientation the consuming kernel streams:
// want_trans == false for column reductions (stored (v, w)), true for GEMM
// operand prep (stored (w, v)).  Otherwise the matrix is replaced by its
// materialised transpose (one per matrix, shared by all consumers).
MOp direct(Dag &G, const MOp &o, bool want_trans, int d, int64_t n, bool cse, bool sym) {
    if (o.trans == want_trans) return o;
    if (sym && o.node < 0) return MOp{o.node, o.p, want_trans};  // symmetric input
    if (o.node >= 0 && G.nodes[o.node].sym) return MOp{o.node, o.p, want_trans};
    Node t;
    t.kind = NK::Transpose;
    t.d = d;
    t.n = n;
    t.A.push_back(MOp{o.node, o.p, false});
    std::string key = "T|" + std::to_string(n) + "|" + (o.node < 0 ? "I" + ptr_id(o.p) : "N" + int_id(o.node));
    int id = add_node(G, t, key, cse);
    return MOp{id, nullptr, want_trans};
}

int add_node(Dag &G, Node nd, const std::string &key, bool cse) {
    if (cse) {
        auto it = G.by_key.find(key);
        if (it != G.by_key.end()) return it->second;
    }
    nd.level = node_level(G, nd);
    G.max_level = std::max(G.max_level, nd.level);
    int id = (int)G.nodes.size();
    G.nodes.push_back(nd);
    if (cse) G.by_key.emplace(key, id);
    return id;
}

// GEMM part of an Elim2/Final2 step, canonicalised so that the operand
// group with the smaller signature comes first; *swapped reports that the
// node computes the transpose of the step's R(w, x).
std::string gemm_key(int64_t n, const std::vector<MOp> &A, const std::vector<VOp> &sv,
                     const std::vector<MOp> &B, bool *swapped) {
    std::string sa = group_sig(A, mop_sig), sb = group_sig(B, mop_sig);
    std::string ss = group_sig(sv, vop_sig);
    *swapped = sb < sa;
    if (*swapped) std::swap(sa, sb);
    return "G" + std::to_string(n) + "|" + sa + "|" + ss + "|" + sb;
}

// Replicates the first slice of every conditioned program over the other
// slices of the range.  A node depends on the slice when it reads a slice
// source vector or a node that does; slice-independent nodes stay shared.
// Each clone reads the clones of its slice-dependent inputs and the slice
// source at the next row offset, so slice s + k is the first slice's
// computation with the conditioned index advanced by k.
template <class Inst>
void clone_slices(Dag &G, const std::vector<Inst> &insts) {
    const int T = (int)G.nodes.size();
    auto slice_vop = [&](const VOp &v) { return v.node >= 0 && G.nodes[v.node].kind == NK::SliceSrc; };
    std::vector<char> dep(T, 0);
    for (int i = 0; i < T; ++i) {
        const Node &x = G.nodes[i];
        bool dd = false;
        auto m = [&](int id) { dd = dd || (id >= 0 && dep[id]); };
        for (auto *g : {&x.A, &x.B, &x.Z})
            for (auto &o : *g) m(o.node);
        for (auto *g : {&x.sv, &x.aw, &x.bx})
            for (auto &o : *g) {
                m(o.node);
                dd = dd || slice_vop(o);
            }
        dep[i] = dd;
    }
    // per dataset: its slice-dependent nodes (reachable from the first
    // slice's terms) in creation order, which is topological
    std::map<int, std::vector<int>> tmpl;
    std::map<int, int64_t> extra;
    {
        std::map<int, std::vector<char>> seen;
        for (const Inst &si : insts) {
            extra[si.d] = std::max(extra[si.d], si.extra);
            std::vector<char> &sn = seen[si.d];
            sn.resize(T, 0);
            std::vector<int> stack;
            for (int id : G.prog_terms[si.dp][0])
                if (dep[id]) stack.push_back(id);
            while (!stack.empty()) {
                int id = stack.back();
                stack.pop_back();
                if (sn[id]) continue;
                sn[id] = 1;
                const Node &x = G.nodes[id];
                auto push = [&](int u) {
                    if (u >= 0 && dep[u] && !sn[u]) stack.push_back(u);
                };
                for (auto *g : {&x.A, &x.B, &x.Z})
                    for (auto &o : *g) push(o.node);
                for (auto *g : {&x.sv, &x.aw, &x.bx})
                    for (auto &o : *g) push(o.node);
            }
        }
        for (auto &kv : seen)
            for (int i = 0; i < T; ++i)
                if (kv.second[i]) tmpl[kv.first].push_back(i);
    }
    int64_t max_extra = 0;
    for (auto &kv : extra) max_extra = std::max(max_extra, kv.second);
    std::vector<int> cmap(T, -1);
    for (int64_t k = 1; k <= max_extra; ++k) {
        std::fill(cmap.begin(), cmap.end(), -1);
        for (auto &kv : tmpl) {
            if (k > extra[kv.first]) continue;
            for (int t : kv.second) {
                if (cmap[t] >= 0) continue;
                Node c = G.nodes[t];
                auto rm = [&](int &id) {
                    if (id >= 0 && id < T && dep[id]) id = cmap[id];
                };
                for (auto *g : {&c.A, &c.B, &c.Z})
                    for (auto &o : *g) rm(o.node);
                for (auto *g : {&c.sv, &c.aw, &c.bx})
                    for (auto &o : *g) {
                        if (slice_vop(o)) o.off += k * c.n;
                        rm(o.node);
                    }
                c.level = node_level(G, c);
                c.last_use = 0;
                cmap[t] = (int)G.nodes.size();
                G.nodes.push_back(std::move(c));
            }
        }
        for (const Inst &si : insts) {
            if (k > si.extra) continue;
            std::vector<int> term = G.prog_terms[si.dp][0];
            for (int &id : term)
                if (dep[id]) id = cmap[id];
            G.prog_terms[si.dp].push_back(std::move(term));
        }
    }
}

std::string build_dag(const Plan &plan, const std::vector<const VProgram *> &progs,
                      const std::vector<Dataset> &data, bool cse, const SliceRange &range, Dag &G,
                      const std::vector<char> &in_binary = std::vector<char>()) {
    const int nd = (int)data.size();
    // programs of dataset d are numbered poff[d] .. poff[d + 1] - 1
    std::vector<int> poff(nd + 1, 0);
    for (int d = 0; d < nd; ++d) poff[d + 1] = poff[d] + (int)progs_of(progs, data[d]).size();
    G.prog_terms.assign((size_t)poff[nd], {});
    struct Pending {
        int dp, term, pos;
        int64_t n;
        int d;
        std::vector<MOp> A, B, Z;
        std::vector<VOp> sv, aw, bx;
        std::string gkey;
        bool swapped;
    };
    std::vector<Pending> pending;
    std::unordered_map<std::string, int> gkey_count;
    // Conditioned programs: only the first slice of the range is built with
    // CSE keys; the other slices are clones of its slice-dependent nodes.
    struct SlicedInst {
        int dp, d;
        int64_t extra;  // slices after the first one in the range
    };
    std::vector<SlicedInst> sliced_insts;
    auto use_diag = [&](int d, const void *ptr) {
        auto key = std::make_pair(d, ptr);
        if (!G.diag_index.count(key)) {
            int idx = (int)G.diag_index.size();
            G.diag_index[key] = idx;
        }
    };
    for (int d = 0; d < nd; ++d) {
        inject_host_alloc();
        const int64_t n = data[d].n;
        const bool sym = data[d].symmetric;
        const std::vector<const VProgram *> &dprogs = progs_of(progs, data[d]);
        const int np = (int)dprogs.size();
        for (int p = 0; p < np; ++p) {
          const VProgram &pr = *dprogs[p];
          const bool sliced = pr.slice_var >= 0;
          if (!sliced && !range.include_unsliced) continue;
          const int64_t s_lo = sliced ? std::max<int64_t>(0, range.lo) : -1;
          const int64_t s_hi = sliced ? std::min<int64_t>(n, range.hi) : 0;
          if (sliced && s_hi - s_lo > 1) sliced_insts.push_back({poff[d] + p, d, s_hi - s_lo - 1});
          for (int64_t slice = s_lo; slice < std::min(s_hi, s_lo + 1); ++slice) {
            std::vector<Ref> ref(pr.vals.size());
            for (size_t v = 0; v < pr.vals.size(); ++v) {
                const Value &val = pr.vals[v];
                if (val.kind == ValKind::InputMat || val.kind == ValKind::InputDiag) {
                    ref[v].p = data[d].factors[val.src];
                    if (val.kind == ValKind::InputDiag) use_diag(d, ref[v].p);
                } else if (val.kind == ValKind::SliceVec) {
                    Node sn;
                    sn.kind = NK::SliceSrc;
                    sn.d = d;
                    sn.n = n;
                    const void *mp = data[d].factors[val.src];
                    const int col = sym ? 0 : val.c;  // rows and columns agree
                    sn.A.push_back(MOp{-1, mp, col == 1});
                    std::string key = "S|" + std::to_string(n) + "|" + ptr_id(mp) + "|" + std::to_string(col);
                    for (int k : val.scale) {
                        const void *dp_ = data[d].factors[k];
                        use_diag(d, dp_);
                        sn.sv.push_back(VOp{-1, dp_});
                    }
                    key += "|" + group_sig(sn.sv, vop_sig);
                    ref[v].node = add_node(G, sn, key, cse);
                    ref[v].off = slice * n;
                }
            }
            // a symmetric input is keyed in one orientation, so that steps
            // differing only by its orientation merge
            auto mop = [&](const MatOp &o) {
                const Ref &r = ref[o.val];
                if (sym && r.node < 0) return MOp{r.node, r.p, false};
                if (r.node >= 0 && G.nodes[r.node].sym) return MOp{r.node, r.p, false};
                return MOp{r.node, r.p, (bool)(o.trans ^ r.flip)};
            };
            auto vop = [&](int v) { return VOp{ref[v].node, ref[v].p, ref[v].off}; };
            // A Hadamard group that repeats a 0/1 input (in the same
            // orientation) keeps one copy: M o M = M entry by entry.
            auto binary_input = [&](const void *ptr) {
                if (in_binary.empty()) return false;
                const int ne_ = (int)data[d].factors.size();
                for (int k = 0; k < ne_; ++k)
                    if (data[d].factors[k] == ptr) return in_binary[(size_t)d * ne_ + k] != 0;
                return false;
            };
            auto dedupe = [&](std::vector<MOp> &L) {
                std::vector<MOp> keep;
                for (const MOp &o : L) {
                    bool dup = false;
                    if (o.node < 0 && binary_input(o.p))
                        for (const MOp &q : keep) dup = dup || (q.node < 0 && q.p == o.p && q.trans == o.trans);
                    if (!dup) keep.push_back(o);
                }
                L.swap(keep);
            };
            const int dp = poff[d] + p;
            std::vector<int> term;
            for (const Step &st : pr.steps) {
                std::vector<MOp> A, B, Z;
                std::vector<VOp> sv, aw, bx;
                for (auto &o : st.A) A.push_back(mop(o));
                for (auto &o : st.B) B.push_back(mop(o));
                for (auto &o : st.Z) Z.push_back(mop(o));
                dedupe(A);
                dedupe(B);
                dedupe(Z);
                for (int q : st.sv) sv.push_back(vop(q));
                for (int q : st.aw) aw.push_back(vop(q));
                for (int q : st.bx) bx.push_back(vop(q));
                Node nd_;
                nd_.d = d;
                nd_.n = n;
                switch (st.kind) {
                    case StepKind::Elim0: {
                        nd_.kind = NK::E0;
                        nd_.sv = sv;
                        int id = add_node(G, nd_, "E0|" + std::to_string(n) + "|" + group_sig(sv, vop_sig), cse);
                        ref[st.out].node = id;
                        term.push_back(id);
                        break;
                    }
                    case StepKind::Elim1:
                    case StepKind::Final1: {
                        nd_.kind = NK::E1;
                        for (auto &o : A) nd_.A.push_back(direct(G, o, false, d, n, cse, sym));
                        nd_.sv = sv;
                        std::string k1 = "E1|" + std::to_string(n) + "|" + group_sig(nd_.A, mop_sig) + "|" +
                                         group_sig(sv, vop_sig);
                        int id = add_node(G, nd_, k1, cse);
                        if (st.kind == StepKind::Elim1) {
                            ref[st.out].node = id;
                        } else {
                            Node dot;
                            dot.kind = NK::Dot;
                            dot.d = d;
                            dot.n = n;
                            dot.sv.push_back(VOp{id, nullptr});
                            for (auto &v : aw) dot.sv.push_back(v);
                            int did = add_node(G, dot, "DOT|" + std::to_string(n) + "|" + group_sig(dot.sv, vop_sig), cse);
                            ref[st.out].node = did;
                            term.push_back(did);
                        }
                        break;
                    }
                    case StepKind::Elim2: {
                        for (auto &o : A) o = direct(G, o, true, d, n, cse, sym);
                        for (auto &o : B) o = direct(G, o, true, d, n, cse, sym);
                        bool sw;
                        std::string k = gemm_key(n, A, sv, B, &sw);
                        nd_.kind = NK::GemmStore;
                        nd_.A = sw ? B : A;
                        nd_.B = sw ? A : B;
                        nd_.sv = sv;
                        nd_.sym = group_sig(A, mop_sig) == group_sig(B, mop_sig);
                        int id = add_node(G, nd_, k, cse);
                        ref[st.out].node = id;
                        ref[st.out].flip = sw;
                        gkey_count[k] += 2;  // a stored product is always reusable
                        break;
                    }
                    case StepKind::Final2: {
                        for (auto &o : A) o = direct(G, o, true, d, n, cse, sym);
                        for (auto &o : B) o = direct(G, o, true, d, n, cse, sym);
                        Pending pd;
                        pd.dp = dp;
                        pd.term = (int)G.prog_terms[dp].size();
                        pd.pos = (int)term.size();
                        pd.n = n;
                        pd.d = d;
                        pd.A = A;
                        pd.B = B;
                        pd.Z = Z;
                        pd.sv = sv;
                        pd.aw = aw;
                        pd.bx = bx;
                        pd.gkey = gemm_key(n, A, sv, B, &pd.swapped);
                        gkey_count[pd.gkey] += 1;
                        term.push_back(-1);  // patched below
                        pending.push_back(pd);
                        break;
                    }
                }
            }
            G.prog_terms[dp].push_back(term);
          }
        }
    }
    // Final2 steps: fused GEMM + consumer unless their product is shared.
    for (size_t i = 0; i < pending.size(); ++i) {
        Pending &pd = pending[i];
        // node orientation (w', x'): swapped -> w' = x, x' = w
        std::vector<MOp> A = pd.swapped ? pd.B : pd.A, B = pd.swapped ? pd.A : pd.B, Z = pd.Z;
        std::vector<VOp> aw = pd.swapped ? pd.bx : pd.aw, bx = pd.swapped ? pd.aw : pd.bx;
        if (pd.swapped)
            for (auto &z : Z) z.trans = !z.trans;
        int sid;
        if (cse && gkey_count[pd.gkey] >= 2) {
            Node g;
            g.kind = NK::GemmStore;
            g.d = pd.d;
            g.n = pd.n;
            g.A = A;
            g.B = B;
            g.sv = pd.sv;
            g.sym = group_sig(A, mop_sig) == group_sig(B, mop_sig);
            int gid = add_node(G, g, pd.gkey, cse);
            // consumer: y(x') = sum_w' R(w',x') prod Z(w',x') prod aw(w'), an
            // Elim1 over v := w' (R is stored with rows over w'), then a dot
            // with bx.
            Node e;
            e.kind = NK::E1;
            e.d = pd.d;
            e.n = pd.n;
            e.A.push_back(MOp{gid, nullptr, false});
            for (auto &z : Z) e.A.push_back(direct(G, z, false, pd.d, pd.n, cse, data[pd.d].symmetric));
            e.sv = aw;
            int eid = add_node(G, e, "E1|" + std::to_string(pd.n) + "|" + group_sig(e.A, mop_sig) + "|" +
                                         group_sig(e.sv, vop_sig), cse);
            Node dot;
            dot.kind = NK::Dot;
            dot.d = pd.d;
            dot.n = pd.n;
            dot.sv.push_back(VOp{eid, nullptr});
            for (auto &v : bx) dot.sv.push_back(v);
            sid = add_node(G, dot, "DOT|" + std::to_string(pd.n) + "|" + group_sig(dot.sv, vop_sig), cse);
        } else {
            Node f;
            f.kind = NK::GemmFinal;
            f.d = pd.d;
            f.n = pd.n;
            f.A = A;
            f.B = B;
            f.Z = Z;
            f.sv = pd.sv;
            f.aw = aw;
            f.bx = bx;
            std::string k = "F" + pd.gkey + "|" + group_sig(Z, mop_sig) + "|" + group_sig(aw, vop_sig) +
                            "|" + group_sig(bx, vop_sig);
            sid = add_node(G, f, k, cse);
        }
        G.prog_terms[pd.dp][pd.term][pd.pos] = sid;
    }
    if (!sliced_insts.empty()) clone_slices(G, sliced_insts);
    // last uses
    for (auto &nd : G.nodes) {
        auto use = [&](int id) {
            if (id >= 0) G.nodes[id].last_use = std::max(G.nodes[id].last_use, nd.level);
        };
        for (auto &o : nd.A) use(o.node);
        for (auto &o : nd.B) use(o.node);
        for (auto &o : nd.Z) use(o.node);
        for (auto &o : nd.sv) use(o.node);
        for (auto &o : nd.aw) use(o.node);
        for (auto &o : nd.bx) use(o.node);
    }
    (void)plan;
    return "";
}

bool same_matrix(const MatRef &a, const MatRef &b) {
    return a.p == b.p && a.ld == b.ld && a.dtype == b.dtype && a.trans == b.trans &&
           a.zdiag == b.zdiag;
}

size_t dtype_bytes(int32_t dt) {
    return dt == DT_F64 || dt == DT_I64 ? 8 : dt == DT_F32 ? 4 : 1;
}

// A column reduction of one level before its blocks are laid out: the
// descriptor (operands and vectors), where its result goes, and the
// running-maximum slot of the exact path.
struct ColPending {
    Elim1Desc e;
    void *out;
    unsigned long long *mx;
    bool rows = false;  // every matrix symmetric: reduce along rows
};

// Lays out a level's symmetric products for the stream-K launch: the block
// count (at most one per compute unit, and few enough that every block
// covers at least half a tile's K steps, so a tile is split over at most
// three blocks) and the partial buffer (two slots per block).
template <class Alloc>
void layout_symmetric(LevelWork &W, Alloc &&alloc_part) {
    const int64_t U = W.gemm_sym_units;
    const int64_t half = std::max<int64_t>(1, (W.gemm_sym_nk + 1) / 2);
    const int64_t G = std::max<int64_t>(1, std::min<int64_t>(kSymBlocks, U / half));
    W.sym_blocks = (int)G;
    W.sym_part = alloc_part((size_t)G * 2 * kSymSlot * sizeof(float));
}

// Lays out a level's column reductions.  Those reading few distinct
// matrices are grouped greedily, in node order: a reduction joins the first
// group of its size n whose matrices together with its own stay within
// kColMat and that has an output slot left; the rest keep one launch entry
// each.  The strip height is then chosen for the whole level: the largest
// of 512, 256, ..., 32 rows that still gives at least min_blocks blocks, so
// that a lone problem fills the chip while batched levels keep few partial
// rows.
// alloc_part(bytes) returns a scratch partial buffer of the level; each
// output gets a fixed-order reduction of its partials into its result.
template <class Alloc>
void layout_column_reductions(const std::vector<ColPending> &recs, LevelWork &W, int64_t min_blocks,
                              Alloc &&alloc_part) {
    struct Out {
        ColOut o;
        int rec;
    };
    struct Grp {
        int64_t n;
        bool rows;
        std::vector<MatRef> M;
        std::vector<Out> outs;
    };
    std::vector<Grp> groups;
    std::vector<int> single;  // records keeping their own launch entry
    for (int ri = 0; ri < (int)recs.size(); ++ri) {
        const Elim1Desc &e = recs[ri].e;
        std::vector<MatRef> dm;
        std::vector<int> cnt;
        for (int q = 0; q < e.nA; ++q) {
            int k = 0;
            while (k < (int)dm.size() && !same_matrix(dm[k], e.A[q])) ++k;
            if (k == (int)dm.size()) {
                dm.push_back(e.A[q]);
                cnt.push_back(0);
            }
            ++cnt[k];
        }
        if ((int)dm.size() > kColMat) {
            single.push_back(ri);
            continue;
        }
        Grp *home = nullptr;
        for (Grp &g : groups) {
            if (g.n != e.n || g.rows != recs[ri].rows || (int)g.outs.size() >= kColOut) continue;
            std::vector<MatRef> un = g.M;
            for (const MatRef &m : dm) {
                bool have = false;
                for (const MatRef &u : un) have = have || same_matrix(u, m);
                if (!have) un.push_back(m);
            }
            if ((int)un.size() > kColMat) continue;
            g.M = un;
            home = &g;
            break;
        }
        if (!home) {
            groups.push_back(Grp{e.n, recs[ri].rows, dm, {}});
            home = &groups.back();
        }
        Out o;
        std::memset(&o.o, 0, sizeof o.o);
        o.rec = ri;
        for (size_t k = 0; k < dm.size(); ++k)
            for (size_t u = 0; u < home->M.size(); ++u)
                if (same_matrix(home->M[u], dm[k])) {
                    o.o.e[u] = (int8_t)cnt[k];
                    o.o.zd[u] = (int8_t)dm[k].zdiag;
                }
        o.o.nS = e.nS;
        for (int q = 0; q < e.nS; ++q) o.o.s[q] = e.s[q];
        home->outs.push_back(o);
    }
    auto wstrips = [](int64_t n) { return (n + 255) / 256; };
    auto row_blocks = [](int64_t n) { return (n + kRowBlock - 1) / kRowBlock; };
    auto blocks = [&](int S) {
        int64_t b = 0;
        for (const Grp &g : groups)
            b += g.rows ? row_blocks(g.n) * ((g.n + row_segment(g.n) - 1) / row_segment(g.n))
                        : ((g.n + S - 1) / S) * wstrips(g.n);
        for (int ri : single) b += ((recs[ri].e.n + S - 1) / S) * wstrips(recs[ri].e.n);
        return b;
    };
    int S = kElimStrip;
    while (S > 32 && blocks(S) < min_blocks) S /= 2;
    // partials of one output and the reduction that consumes them
    auto partials = [&](const ColPending &r, int64_t strips) {
        const int64_t n = r.e.n;
        void *part = alloc_part((size_t)strips * n * 8);
        ReduceDesc rd;
        std::memset(&rd, 0, sizeof rd);
        rd.part = part;
        rd.T = strips;
        rd.len = n;
        rd.stride = n;
        rd.out = r.out;
        rd.mx_out = r.mx;
        W.red.push_back(rd);
        W.red_maxlen = std::max<int64_t>(W.red_maxlen, n);
        return part;
    };
    for (int ri : single) {
        Elim1Desc f = recs[ri].e;
        f.strip = S;
        f.tiles_v = (int)((f.n + S - 1) / S);
        f.tiles_w = (int)wstrips(f.n);
        f.part = partials(recs[ri], f.tiles_v);
        f.tile_start = W.e1_tiles;
        W.e1_tiles += (int64_t)f.tiles_v * f.tiles_w;
        W.e1.push_back(f);
        for (int q = 0; q < f.nA; ++q) W.e1_bytes += (double)f.n * f.n * dtype_bytes(f.A[q].dtype);
        W.e1_bytes += (double)f.n * 8 * (f.nS + f.tiles_v);
    }
    for (const Grp &g : groups) {
        ColDesc c;
        std::memset(&c, 0, sizeof c);
        c.n = g.n;
        c.nm = (int)g.M.size();
        c.nout = (int)g.outs.size();
        for (int k = 0; k < c.nm; ++k) {
            c.M[k] = g.M[k];
            c.M[k].zdiag = 0;  // applied per output
        }
        c.rows = g.rows ? 1 : 0;
        c.strip = g.rows ? row_segment(g.n) : S;
        c.tiles_v = (int)((g.n + c.strip - 1) / c.strip);
        c.tiles_w = g.rows ? (int)row_blocks(g.n) : (int)wstrips(g.n);
        for (int o = 0; o < c.nout; ++o) {
            c.o[o] = g.outs[o].o;
            c.o[o].part = partials(recs[g.outs[o].rec], c.tiles_v);
        }
        const int b = (g.rows ? kColMat : 0) + c.nm - 1;
        W.col_maxout[b] = std::max(W.col_maxout[b], c.nout);
        for (int k = 0; k < c.nm; ++k) {
            int &cd = W.col_dtype[b];
            cd = cd == -2 ? c.M[k].dtype : (cd == c.M[k].dtype ? cd : -1);
        }
        c.tile_start = W.col_tiles[b];
        W.col_tiles[b] += (int64_t)c.tiles_v * c.tiles_w;
        W.col[b].push_back(c);
        double bytes = 0;
        for (int k = 0; k < c.nm; ++k) bytes += (double)g.n * g.n * dtype_bytes(g.M[k].dtype);
        for (const Out &o : g.outs) bytes += (double)g.n * 8 * (o.o.nS + c.tiles_v);
        W.col_bytes[b] += bytes;
    }
}

// Builds the schedule.  With base == nullptr only sizes are computed; a
// second call with the real arena base fills every pointer (the layout is
// deterministic, so offsets agree).
std::string build_schedule(const Plan &plan, const std::vector<const VProgram *> &progs,
                           const std::vector<Dataset> &data, const Cfg &cfg,
                           const std::vector<double> &in_bound,  // per dataset*edge (INT)
                           const std::vector<char> &in_signed,   // per dataset*edge, empty: none
                           char *base, Schedule &S, int *status,
                           const SliceRange &range = SliceRange(),
                           const std::vector<char> &in_binary = std::vector<char>()) {
    S = Schedule();
    Arena A;
    const int nd = (int)data.size();
    // Symmetric products are not used in evaluations that hold a program
    // conditioned on a vertex.  One run of such evaluations (split-bf16,
    // symmetric factors, levels of thousands of products of slice operands)
    // stopped on an illegal memory access whose cause has not been found;
    // those evaluations take the full product.
    bool conditioned_eval = false;
    for (const VProgram *p : progs) conditioned_eval = conditioned_eval || p->slice_var >= 0;
    for (const Dataset &d : data)
        for (const VProgram *p : d.progs) conditioned_eval = conditioned_eval || p->slice_var >= 0;
    const int ne = nd ? (int)data[0].factors.size() : 0;  // factors per dataset (equal for all)
    std::vector<int> poff(nd + 1, 0);
    for (int d = 0; d < nd; ++d) poff[d + 1] = poff[d] + (int)progs_of(progs, data[d]).size();
    S.nprog_total = poff[nd];
    auto P = [&](size_t off) -> void * { return base ? (void *)(base + off) : nullptr; };
    Dag G;
    std::string err = build_dag(plan, progs, data, plan.opts.cse, range, G, in_binary);
    if (!err.empty()) {
        *status = 1;
        return err;
    }
    S.n_nodes = G.nodes.size();
    S.depth = G.max_level;
    S.two_plane.assign(nd, 0);
    const bool is_int = cfg.domain == DOM_INT;
    if ((base || getenv("USTAT_DEBUG_DAG_DRY")) && getenv("USTAT_DEBUG_DAG")) {
        int cnt[6] = {0, 0, 0, 0, 0, 0};
        for (auto &x : G.nodes) cnt[(int)x.kind]++;
        fprintf(stderr, "dag: nodes=%zu E0=%d E1=%d Dot=%d GemmStore=%d GemmFinal=%d Transpose=%d levels=%d\n",
                G.nodes.size(), cnt[0], cnt[1], cnt[2], cnt[3], cnt[4], cnt[5], G.max_level);
        for (size_t i = 0; i < G.nodes.size(); ++i) {
            auto &x = G.nodes[i];
            if (x.kind != NK::E1 && x.kind != NK::GemmStore && x.kind != NK::GemmFinal) continue;
            fprintf(stderr, "  node %zu kind=%d level=%d nA=%zu nB=%zu nZ=%zu nsv=%zu\n", i,
                    (int)x.kind, x.level, x.A.size(), x.B.size(), x.Z.size(), x.sv.size());
        }
    }
    // scalar and running-max slots
    size_t nscal = 0, nmx = 0;
    for (auto &nd_ : G.nodes) {
        if (nd_.kind == NK::E0 || nd_.kind == NK::Dot || nd_.kind == NK::GemmFinal) nd_.scal = (int)nscal++;
        if (is_int && (nd_.kind == NK::E1 || nd_.kind == NK::GemmStore || nd_.kind == NK::SliceSrc))
            nd_.mx = (int)nmx++;
    }
    std::vector<int> diag_mx(G.diag_index.size(), -1);
    if (is_int)
        for (auto &kv : G.diag_index) diag_mx[kv.second] = (int)nmx++;
    S.n_scal = nscal;
    S.n_mx = nmx;
    S.off_scal = A.alloc(nscal * cfg.wide_es + 16);
    S.off_mx = A.alloc(nmx * 8 + 16);
    // input maxima: one slot per (dataset, edge)
    std::map<std::pair<int, const void *>, int> inmx_of;
    if (is_int)
        for (int d = 0; d < nd; ++d)
            for (int k = 0; k < ne; ++k) {
                auto key = std::make_pair(d, data[d].factors[k]);
                if (!inmx_of.count(key)) inmx_of[key] = d * ne + k;
            }
    S.n_inmx = is_int ? (size_t)nd * ne : 0;
    S.off_inmx = A.alloc(S.n_inmx * 8 + 16);
    unsigned long long *mxbase =
        base ? reinterpret_cast<unsigned long long *>(base + S.off_mx) : nullptr;
    unsigned long long *inmxbase =
        base ? reinterpret_cast<unsigned long long *>(base + S.off_inmx) : nullptr;
    auto in_b = [&](int d, const void *ptr) {
        if (in_bound.empty()) return 127.0;
        return in_bound[inmx_of[std::make_pair(d, ptr)]];
    };
    // inputs that may hold negative entries: one flag per (dataset, edge),
    // looked up by pointer (the first edge carrying it)
    std::map<std::pair<int, const void *>, int> in_index;
    for (int d = 0; d < nd; ++d)
        for (int k = 0; k < ne; ++k) in_index.emplace(std::make_pair(d, data[d].factors[k]), d * ne + k);
    auto in_neg = [&](int d, const void *ptr) -> bool {
        if (in_signed.empty()) return false;
        return in_signed[in_index[std::make_pair(d, ptr)]] != 0;
    };
    // diagonals (prologue)
    std::vector<size_t> diag_off(G.diag_index.size());
    for (auto &kv : G.diag_index) {
        const int d = kv.first.first;
        const size_t off = A.alloc((size_t)data[d].n * 8);
        diag_off[kv.second] = off;
        DiagDesc dd;
        dd.src = {kv.first.second, data[d].n, cfg.in_dt, 0, 0, 0};
        dd.dst = P(off);
        dd.n = data[d].n;
        dd.mx_out = (is_int && mxbase) ? mxbase + diag_mx[kv.second] : nullptr;
        S.diag.push_back(dd);
        S.diag_maxn = std::max(S.diag_maxn, dd.n);
    }
    const bool sparsify = plan.opts.sparsify != 0;
    auto vptr = [&](int d, const VOp &v) -> const void * {
        if (v.node >= 0) return base ? (const void *)(base + G.nodes[v.node].off + v.off * 8) : nullptr;
        return P(diag_off[G.diag_index[std::make_pair(d, v.p)]]);
    };
    auto vbound = [&](int d, const VOp &v) {
        if (v.node >= 0) return G.nodes[v.node].bound;
        return in_b(d, v.p);
    };
    auto vmx = [&](int d, const VOp &v) -> const unsigned long long * {
        if (!mxbase) return nullptr;
        if (v.node >= 0) return mxbase + G.nodes[v.node].mx;
        return mxbase + diag_mx[G.diag_index[std::make_pair(d, v.p)]];
    };
    // A transpose node stands for its source matrix read the other way:
    // same element type, bound, running maximum and diagonal handling.
    auto src_of = [&](MOp o) {
        while (o.node >= 0 && G.nodes[o.node].kind == NK::Transpose) o = G.nodes[o.node].A[0];
        return o;
    };
    auto mref = [&](int d, const MOp &o) -> MatRef {
        MatRef m;
        const MOp s0 = src_of(o);
        const bool input = s0.node < 0;
        m.p = o.node < 0 ? o.p : P(G.nodes[o.node].off);
        m.ld = data[d].n;
        m.dtype = input ? cfg.in_dt : cfg.mat_dt;
        m.trans = o.trans ? 1 : 0;
        m.zdiag = (input && sparsify) ? 1 : 0;
        m.pad = 0;
        return m;
    };
    auto mbound = [&](int d, const MOp &o) {
        const MOp s0 = src_of(o);
        return s0.node >= 0 ? G.nodes[s0.node].bound : in_b(d, s0.p);
    };
    auto mneg = [&](int d, const MOp &o) {
        const MOp s0 = src_of(o);
        return s0.node >= 0 ? G.nodes[s0.node].neg : in_neg(d, s0.p);
    };
    auto vneg = [&](int d, const VOp &v) { return v.node >= 0 ? G.nodes[v.node].neg : in_neg(d, v.p); };
    auto mmx = [&](int d, const MOp &o) -> const unsigned long long * {
        if (!inmxbase) return nullptr;
        const MOp s0 = src_of(o);
        if (s0.node >= 0) return mxbase + G.nodes[s0.node].mx;
        return inmxbase + inmx_of[std::make_pair(d, s0.p)];
    };
    auto scal_ptr = [&](const Node &nd_) -> void * {
        return P(S.off_scal + (size_t)nd_.scal * cfg.wide_es);
    };
    const double kOverflow = 4.0e18;  // < 2^62
    const double kOverflowWide = 8.0e37;

    struct PrepRec {
        size_t off, bytes;
        int limbs, limb_slot;
    };
    std::map<std::string, PrepRec> persistent;
    size_t nlimb = 0;
    for (auto &nd_ : G.nodes)
        if (nd_.kind == NK::GemmStore || nd_.kind == NK::GemmFinal) nlimb += 2;
    S.n_limbs = nlimb;
    S.off_limbs = A.alloc(nlimb * 4 + 16);
    size_t limb_next = 0;
    auto limb_ptr = [&](size_t slot) -> int32_t * {
        return base ? reinterpret_cast<int32_t *>(base + S.off_limbs) + slot : nullptr;
    };

    // last GEMM level of every operand prep built only from inputs, so that
    // it can be released after that level
    auto prep_key = [&](int d, int64_t n, const std::vector<MOp> &ops, const std::vector<VOp> &sv,
                        int format) {
        std::string key = std::to_string(d) + "|" + std::to_string(n) + "|" + std::to_string(format) + "|";
        bool pers = true;
        for (auto &o : ops) {
            pers = pers && (o.node < 0);
            key += mop_sig(o);
        }
        key += "|";
        for (auto &v : sv) {
            pers = pers && (v.node < 0);
            key += vop_sig(v);
        }
        return std::make_pair(key, pers);
    };
    // Sign of every node (nodes come in topological order): a value may be
    // negative only when one of its operands may be.
    for (auto &nd_ : G.nodes) {
        bool ng = false;
        const int d = nd_.d;
        if (nd_.kind == NK::SliceSrc || nd_.kind == NK::Transpose) {
            ng = mneg(d, nd_.A[0]);
        } else {
            for (auto *g : {&nd_.A, &nd_.B, &nd_.Z})
                for (auto &o : *g) ng = ng || mneg(d, o);
        }
        for (auto *g : {&nd_.sv, &nd_.aw, &nd_.bx})
            for (auto &v : *g) ng = ng || vneg(d, v);
        nd_.neg = ng;
    }
    // operand format of a GEMM node: split-bf16 takes three planes when a
    // contracted operand may be negative or the size is small
    auto gemm_format = [&](const Node &q) {
        if (cfg.pformat != PF_BF16X2) return cfg.pformat;
        bool ng = q.n < kSplit6Below;
        for (auto &o : q.A) ng = ng || mneg(q.d, o);
        for (auto &o : q.B) ng = ng || mneg(q.d, o);
        for (auto &v : q.sv) ng = ng || vneg(q.d, v);
        return ng ? (int)PF_BF16X3 : (int)PF_BF16X2;
    };
    std::map<std::string, int> prep_last;
    for (auto &nd_ : G.nodes)
        if (nd_.kind == NK::GemmStore || nd_.kind == NK::GemmFinal) {
            const int fm = gemm_format(nd_);
            auto ka = prep_key(nd_.d, nd_.n, nd_.A, nd_.sv, fm);
            auto kb = prep_key(nd_.d, nd_.n, nd_.B, {}, fm);
            prep_last[ka.first] = std::max(prep_last[ka.first], nd_.level);
            prep_last[kb.first] = std::max(prep_last[kb.first], nd_.level);
        }

    // nodes by level
    std::vector<std::vector<int>> by_level(G.max_level + 1);
    for (size_t i = 0; i < G.nodes.size(); ++i) by_level[G.nodes[i].level].push_back((int)i);
    S.levels.assign(G.max_level + 1, LevelWork());
    for (int L = 1; L <= G.max_level; ++L) {
        inject_host_alloc();
        LevelWork &W = S.levels[L];
        // 256-wide tiles (fp32 and split-bf16 only) for the level's GEMMs
        // whose padded size is a multiple of 256, in a launch of their own,
        // when together they give at least one tile per compute unit; the
        // other GEMMs of the level keep 128-wide tiles
        {
            int64_t t256 = 0;
            for (int id : by_level[L]) {
                const Node &q = G.nodes[id];
                if (q.kind != NK::GemmStore && q.kind != NK::GemmFinal) continue;
                if (gemm_format(q) == PF_BF16X3) continue;
                const int64_t np_ = gemm_npad(q.n, gemm_format(q));
                if (np_ % 256 == 0) t256 += (np_ / 256) * (np_ / 256);
            }
            W.big = (cfg.prec == 1 || cfg.prec == 2) && t256 > 0 && t256 >= plan.tuning.gemm_big_min;
        }
        std::vector<std::pair<size_t, size_t>> scratch;
        std::vector<ColPending> e1recs;  // this level's column reductions
        std::map<std::string, PrepRec> local;
        for (int id : by_level[L]) {
            Node &nd_ = G.nodes[id];
            const int d = nd_.d;
            const int64_t n = nd_.n;
            const bool is_gemm = nd_.kind == NK::GemmStore || nd_.kind == NK::GemmFinal;
            const int64_t npad = is_gemm ? gemm_npad(n, gemm_format(nd_)) : up64(n, 128);
            const int tiles64 = (int)((n + 63) / 64);
            if ((int)nd_.A.size() > kMaxMat || (int)nd_.B.size() > kMaxMat ||
                (int)nd_.Z.size() > kMaxMat || (int)nd_.sv.size() > kMaxVec ||
                (int)nd_.aw.size() > kMaxVec || (int)nd_.bx.size() > kMaxVec) {
                *status = 2;
                return "a step has more parallel factors than the engine supports";
            }
            double pA = 1, pB = 1, pZ = 1, pS = 1, paw = 1, pbx = 1;
            for (auto &o : nd_.A) pA *= mbound(d, o);
            for (auto &o : nd_.B) pB *= mbound(d, o);
            for (auto &o : nd_.Z) pZ *= mbound(d, o);
            for (auto &o : nd_.sv) pS *= vbound(d, o);
            for (auto &o : nd_.aw) paw *= vbound(d, o);
            for (auto &o : nd_.bx) pbx *= vbound(d, o);
            switch (nd_.kind) {
                case NK::E0: {
                    Elim0Desc e;
                    e.n = n;
                    e.nS = (int)nd_.sv.size();
                    for (int q = 0; q < e.nS; ++q) e.s[q] = vptr(d, nd_.sv[q]);
                    e.out = scal_ptr(nd_);
                    W.e0.push_back(e);
                    nd_.bound = n * pS;
                    break;
                }
                case NK::Dot: {
                    // sv[0] is the vector being summed, the rest multiply it
                    ReduceDesc r;
                    std::memset(&r, 0, sizeof r);
                    r.part = vptr(d, nd_.sv[0]);
                    r.T = 1;
                    r.len = n;
                    r.stride = n;
                    r.out = scal_ptr(nd_);
                    r.dot = 1;
                    r.nmul = (int)nd_.sv.size() - 1;
                    for (int q = 1; q < (int)nd_.sv.size(); ++q) r.mul[q - 1] = vptr(d, nd_.sv[q]);
                    W.red.push_back(r);
                    W.red_maxlen = std::max<int64_t>(W.red_maxlen, n);
                    nd_.bound = n * pS;
                    break;
                }
                case NK::E1: {
                    ColPending cp;
                    Elim1Desc &e = cp.e;
                    std::memset(&e, 0, sizeof e);
                    e.n = n;
                    e.nA = (int)nd_.A.size();
                    e.nS = (int)nd_.sv.size();
                    for (int q = 0; q < e.nA; ++q) e.A[q] = mref(d, nd_.A[q]);
                    for (int q = 0; q < e.nS; ++q) e.s[q] = vptr(d, nd_.sv[q]);
                    nd_.bytes = (size_t)n * 8;
                    nd_.off = A.alloc(nd_.bytes);
                    nd_.bound = n * pA * pS;
                    if (is_int && nd_.bound > kOverflow) {
                        *status = 5;
                        return "an intermediate vector may exceed int64";
                    }
                    cp.out = P(nd_.off);
                    cp.mx = (is_int && mxbase) ? mxbase + nd_.mx : nullptr;
                    cp.rows = true;
                    for (auto &o : nd_.A)
                        cp.rows = cp.rows && (o.node < 0 ? data[d].symmetric : G.nodes[o.node].sym);
                    e1recs.push_back(cp);
                    break;
                }
                case NK::SliceSrc: {
                    SliceDesc sd;
                    std::memset(&sd, 0, sizeof sd);
                    sd.src = {nd_.A[0].p, n, cfg.in_dt, nd_.A[0].trans ? 1 : 0, 0, 0};
                    sd.nscale = (int)nd_.sv.size();
                    for (int q = 0; q < sd.nscale; ++q) sd.scale[q] = vptr(d, nd_.sv[q]);
                    sd.tiles = tiles64;
                    sd.n = n;
                    nd_.bytes = (size_t)n * n * 8;
                    nd_.off = A.alloc(nd_.bytes);
                    sd.out = P(nd_.off);
                    sd.tile_start = W.sl_tiles;
                    W.sl_tiles += (int64_t)tiles64 * tiles64;
                    sd.mx_out = (is_int && mxbase) ? mxbase + nd_.mx : nullptr;
                    W.sl.push_back(sd);
                    nd_.bound = in_b(d, nd_.A[0].p) * pS;
                    break;
                }
                case NK::Transpose: {
                    const MOp s0 = src_of(nd_.A[0]);
                    const int es = s0.node < 0 ? cfg.in_es : cfg.mat_es;
                    TransDesc td;
                    td.src = nd_.A[0].node < 0 ? nd_.A[0].p : P(G.nodes[nd_.A[0].node].off);
                    td.n = n;
                    td.ld = n;
                    td.dtype = s0.node < 0 ? cfg.in_dt : cfg.mat_dt;
                    td.tiles = tiles64;
                    nd_.bytes = (size_t)n * n * es;
                    nd_.off = A.alloc(nd_.bytes);
                    td.dst = P(nd_.off);
                    td.tile_start = W.tr_tiles;
                    W.tr_tiles += (int64_t)tiles64 * tiles64;
                    W.tr.push_back(td);
                    W.tr_bytes += 2.0 * (double)n * n * es;
                    nd_.bound = mbound(d, nd_.A[0]);
                    break;
                }
                case NK::GemmStore:
                case NK::GemmFinal: {
                    const int fmt = gemm_format(nd_);
                    auto make_prep = [&](const std::vector<MOp> &ops, const std::vector<VOp> &sv,
                                         double bound, const int32_t **limbs_p, int *max_limbs) {
                        // the factor's operand form, written with the factor
                        if (data[d].operand && fmt == data[d].operand_format && !sparsify &&
                            data[d].symmetric && ops.size() == 1 && sv.empty() && ops[0].node < 0 &&
                            ops[0].p == data[d].factors[0]) {
                            *limbs_p = nullptr;
                            *max_limbs = 1;
                            return data[d].operand;
                        }
                        auto kp = prep_key(d, n, ops, sv, fmt);
                        const std::string &key = kp.first;
                        const bool pers = kp.second;
                        int cap = cfg.pformat == PF_I8LIMBS ? limbs_for(bound, 9) : 1;
                        auto &tab = pers ? persistent : local;
                        auto it = tab.find(key);
                        if (it == tab.end()) {
                            PrepRec rec;
                            rec.limbs = cap;
                            rec.bytes = prep_bytes(fmt, npad, cap);
                            rec.off = A.alloc(rec.bytes);
                            rec.limb_slot = (int)limb_next++;
                            if (!pers) scratch.push_back({rec.off, rec.bytes});
                            PrepDesc pd;
                            std::memset(&pd, 0, sizeof pd);
                            pd.n = n;
                            pd.npad = npad;
                            pd.ldo = npad;
                            pd.plane = npad * npad;
                            pd.nA = (int)ops.size();
                            pd.nS = (int)sv.size();
                            for (int q = 0; q < pd.nA; ++q) pd.A[q] = mref(d, ops[q]);
                            for (int q = 0; q < pd.nS; ++q) pd.s[q] = vptr(d, sv[q]);
                            pd.out = P(rec.off);
                            pd.format = fmt;
                            pd.limbs = cap;
                            pd.tiles = (int)(npad / 64);
                            pd.tile_start = W.prep_tiles;
                            W.prep_tiles += (int64_t)(npad / 64) * (npad / 128);
                            pd.nmx = 0;
                            if (is_int) {
                                for (auto &o : ops) pd.mx[pd.nmx++] = mmx(d, o);
                                for (auto &v : sv) pd.mx[pd.nmx++] = vmx(d, v);
                            }
                            pd.limbs_out = limb_ptr(rec.limb_slot);
                            W.prep.push_back(pd);
                            for (auto &o : ops)
                                W.prep_bytes += (double)n * n * (src_of(o).node < 0 ? cfg.in_es : cfg.mat_es);
                            W.prep_bytes += (double)rec.bytes;
                            it = tab.emplace(key, rec).first;
                        }
                        *limbs_p = limb_ptr(it->second.limb_slot);
                        *max_limbs = it->second.limbs;
                        return (const void *)P(it->second.off);
                    };
                    GemmDesc g;
                    std::memset(&g, 0, sizeof g);
                    const int32_t *lap = nullptr, *lbp = nullptr;
                    int cla = 1, clb = 1;
                    g.A = make_prep(nd_.A, nd_.sv, pA * pS, &lap, &cla);
                    g.B = make_prep(nd_.B, {}, pB, &lbp, &clb);
                    // the GEMM addresses its operands with 32-bit offsets
                    if ((double)prep_bytes(fmt, npad, std::max(cla, clb)) >= 4294967296.0) {
                        *status = 2;
                        return "a GEMM operand of this size exceeds the 4 GiB the kernels address";
                    }
                    g.n = n;
                    g.npad = npad;
                    g.ld = npad;
                    g.plane = npad * npad;
                    g.la = cla;
                    g.lb = clb;
                    g.la_p = is_int ? lap : nullptr;
                    g.lb_p = is_int ? lbp : nullptr;
                    const bool six = fmt == PF_BF16X3;
                    if (fmt == PF_BF16X2) S.two_plane[d] = 1;
                    const bool big = W.big && npad % 256 == 0 && !six;
                    g.tiles = (int)(npad / (big ? 256 : 128));
                    // one prepared operand on both sides: C = P P^T is symmetric
                    // (not in evaluations with programs conditioned on a
                    // vertex: that combination is switched off, see below)
                    const bool sym = big && plan.opts.sym_gemm && !conditioned_eval &&
                                     fmt == PF_BF16X2 && nd_.kind == NK::GemmStore &&
                                     g.A == g.B && cfg.mat_dt == DT_F32;
                    if (sym) {
                        const int64_t t = g.tiles, nk = npad / 32;
                        g.tile_start = W.gemm_sym_units;  // first unit (tile K step)
                        g.sym_tile0 = W.gemm_sym_tiles;
                        W.gemm_sym_tiles += t * (t + 1) / 2;
                        W.gemm_sym_units += t * (t + 1) / 2 * nk;
                        W.gemm_sym_nk = std::max(W.gemm_sym_nk, nk);
                        // the step's algorithmic work, 2 n^3 as for any product,
                        // although only the tiles on and above the diagonal run
                        W.gemm_sym_flops += 2.0 * (double)n * n * n;
                    } else {
                        int64_t &tcount = six ? W.gemm6_tiles : big ? W.gemm_big_tiles : W.gemm_tiles;
                        g.tile_start = tcount;
                        tcount += (int64_t)g.tiles * g.tiles;
                        (six ? W.gemm6_flops : big ? W.gemm_big_flops : W.gemm_flops) +=
                            2.0 * (double)n * n * n;
                    }
                    const double cb = n * pA * pS * pB;
                    if (is_int) {
                        if (cb > kOverflow) {
                            *status = 5;
                            return "an intermediate matrix may exceed int64";
                        }
                        if (n >= 131072) {
                            *status = 2;
                            return "the exact path needs n < 131072 (int32 limb accumulation)";
                        }
                    }
                    if (nd_.kind == NK::GemmStore) {
                        nd_.bytes = (size_t)n * n * cfg.mat_es;
                        nd_.off = A.alloc(nd_.bytes);
                        nd_.bound = cb;
                        g.final_ = 0;
                        g.dtype_c = cfg.mat_dt;
                        g.C = P(nd_.off);
                        g.ldc = n;
                        g.mx_out = (is_int && mxbase) ? mxbase + nd_.mx : nullptr;
                    } else {
                        g.final_ = 1;
                        g.nZ = (int)nd_.Z.size();
                        g.naw = (int)nd_.aw.size();
                        g.nbx = (int)nd_.bx.size();
                        for (int q = 0; q < g.nZ; ++q) g.Z[q] = mref(d, nd_.Z[q]);
                        for (int q = 0; q < g.naw; ++q) g.aw[q] = vptr(d, nd_.aw[q]);
                        for (int q = 0; q < g.nbx; ++q) g.bx[q] = vptr(d, nd_.bx[q]);
                        size_t pb = (size_t)g.tiles * g.tiles * 16;
                        size_t poff = A.alloc(pb);
                        scratch.push_back({poff, pb});
                        g.part = P(poff);
                        ReduceDesc r;
                        std::memset(&r, 0, sizeof r);
                        r.part = P(poff);
                        r.T = (int64_t)g.tiles * g.tiles;
                        r.len = 1;
                        r.stride = 1;
                        r.out = scal_ptr(nd_);
                        r.dot = 1;
                        W.red.push_back(r);
                        nd_.bound = (double)n * n * cb * pZ * paw * pbx;
                    }
                    (sym ? W.gemm_sym : six ? W.gemm6 : big ? W.gemm_big : W.gemm).push_back(g);
                    break;
                }
            }
            if (is_int && nd_.scal >= 0 && nd_.bound > kOverflowWide) {
                *status = 5;
                return "a V-statistic may exceed the 127-bit range";
            }
        }
        if (!W.gemm_sym.empty())
            layout_symmetric(W, [&](size_t bytes) {
                const size_t off = A.alloc(bytes);
                scratch.push_back({off, bytes});
                return reinterpret_cast<float *>(P(off));
            });
        layout_column_reductions(e1recs, W, plan.tuning.colred_blocks, [&](size_t bytes) {
            const size_t off = A.alloc(bytes);
            scratch.push_back({off, bytes});
            return P(off);
        });
        for (auto &sc : scratch) A.release(sc.first, sc.second);
        for (auto it = persistent.begin(); it != persistent.end();) {
            if (prep_last[it->first] <= L) {
                A.release(it->second.off, it->second.bytes);
                it = persistent.erase(it);
            } else {
                ++it;
            }
        }
        for (auto &nd_ : G.nodes)
            if (nd_.bytes && nd_.last_use == L) {
                A.release(nd_.off, nd_.bytes);
                nd_.bytes = 0;
            }
        // nodes never consumed (possible only for vectors of unused results)
        for (int id : by_level[L]) {
            Node &nd_ = G.nodes[id];
            if (nd_.bytes && nd_.last_use == 0) {
                // keep until the end; released implicitly
            }
        }
    }
    // combine tables: programs -> terms -> scalar slots
    for (int d = 0; d < nd; ++d) {
        CombineDesc c;
        const std::vector<const VProgram *> &dprogs = progs_of(progs, data[d]);
        const int np = (int)dprogs.size();
        c.p_begin = poff[d];
        c.p_end = poff[d + 1];
        S.comb.push_back(c);
        for (int p = 0; p < np; ++p) {
            const auto &terms = G.prog_terms[poff[d] + p];
            S.term_off.push_back((int32_t)S.scal_off.size());
            S.term_cnt.push_back((int32_t)terms.size());
            double bsum = 0;
            for (const auto &sc : terms) {
                S.scal_off.push_back((int32_t)S.scal_idx.size());
                S.scal_cnt.push_back((int32_t)sc.size());
                double b = 1;
                for (int id : sc) {
                    S.scal_idx.push_back(G.nodes[id].scal);
                    b *= G.nodes[id].bound;
                }
                bsum += b;
            }
            if (dprogs[p]->slice_var >= 0 && !terms.empty())
                bsum *= (double)data[d].n / (double)terms.size();  // all slices, every chunk
            S.mu.push_back(dprogs[p]->mu);
            if (is_int && bsum * std::fabs((double)dprogs[p]->mu) * np > kOverflowWide) {
                *status = 5;
                return "the combined U-statistic may exceed the 127-bit range";
            }
        }
    }
    S.arena_bytes = A.top;
    S.off_diag = S.blob.put(S.diag);
    for (auto &W : S.levels) {
        W.off_sl = S.blob.put(W.sl);
        W.off_tr = S.blob.put(W.tr);
        W.off_prep = S.blob.put(W.prep);
        W.off_gemm = S.blob.put(W.gemm);
        W.off_gemm_big = S.blob.put(W.gemm_big);
        W.off_gemm_sym = S.blob.put(W.gemm_sym);
        W.off_gemm6 = S.blob.put(W.gemm6);
        W.off_e1 = S.blob.put(W.e1);
        for (int k = 0; k < LevelWork::kColSlots; ++k) W.off_col[k] = S.blob.put(W.col[k]);
        W.off_e0 = S.blob.put(W.e0);
        W.off_red = S.blob.put(W.red);
    }
    S.off_comb = S.blob.put(S.comb);
    S.off_toff = S.blob.put(S.term_off);
    S.off_tcnt = S.blob.put(S.term_cnt);
    S.off_soff = S.blob.put(S.scal_off);
    S.off_scnt = S.blob.put(S.scal_cnt);
    S.off_sidx = S.blob.put(S.scal_idx);
    S.off_mu = S.blob.put(S.mu);
    S.blob_bytes = S.blob.h.size();
    return "";
}

}  // namespace

// The estimate follows the probabilistic model of rounding errors of Higham
// and Mary (2019): errors independent with mean zero, so that a sequential
// sum of k terms of unit roundoff u carries a relative error of order
// sqrt(k) u rather than k u.  Every dependency level (plus the diagonal
// prologue and the combination) is a stage; stages add in quadrature.  A
// stage's contraction accumulates n / k_c MFMA results in sequence (k_c the
// instruction's inner length: 4 for fp64 and fp32, 32 for bf16) in unit
// roundoff u_c, and its fp64 reductions and the combination add up to n
// terms in sequence.  The two-plane split-bf16 scheme leaves a residual of
// up to about 3 * 2^-18 per product, of random sign, averaged over the n
// products of a contraction.  The factor 2 covers about two standard
// deviations.  This is an estimate of the typical error, not a worst-case
// bound: it does not credit the further averaging of independent element
// errors in the final sums (so it usually overstates the error at large n),
// and data built to align the errors can exceed it.
double error_estimate(int precision, int64_t n, int depth, bool two_plane) {
    double uc, kc;
    switch (precision) {
        case 0: uc = std::ldexp(1.0, -53); kc = 4; break;
        case 1: uc = std::ldexp(1.0, -24); kc = 4; break;
        case 2: uc = std::ldexp(1.0, -24); kc = 32; break;
        default: return 0.0;  // exact
    }
    const double D = depth + 2.0, nn = (double)std::max<int64_t>(n, 1);
    const double ur = std::ldexp(1.0, -53);
    double e = 2.0 * std::sqrt(D) * (uc * std::sqrt(std::max(1.0, nn / kc)) + ur * std::sqrt(nn));
    if (two_plane) e += 2.0 * std::sqrt(D) * 3.0 * std::ldexp(1.0, -18) / std::sqrt(nn);
    return e;
}

namespace {

__global__ void k_fill_zero(unsigned long long *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Sign flags for sizing a schedule before the inputs are scanned: every
// input not known to be non-negative may be negative (three-plane operands
// are the larger ones).
std::vector<char> worst_signs(const Cfg &cfg, const std::vector<Dataset> &data) {
    std::vector<char> f;
    if (cfg.pformat != PF_BF16X2 || data.empty()) return f;
    const size_t ne = data[0].factors.size();
    for (const Dataset &d : data)
        for (size_t k = 0; k < ne; ++k) f.push_back(d.nonneg ? 0 : 1);
    return f;
}

}  // namespace

int factor_operand_format(const Plan &plan, int64_t n, bool nonneg) {
    const Cfg cfg = make_cfg(plan.opts.precision);
    if (cfg.domain != DOM_FP || plan.opts.sparsify) return -1;
    int fmt = cfg.pformat;
    if (fmt == PF_BF16X2 && (!nonneg || n < kSplit6Below)) fmt = PF_BF16X3;
    if (fmt == PF_BF16X3) return -1;  // the three-plane form is not written with the factor
    for (const VProgram &p : plan.progs)
        for (const Step &st : p.steps) {
            if (st.kind != StepKind::Elim2 && st.kind != StepKind::Final2) continue;
            const bool a = st.A.size() == 1 && st.sv.empty() && p.vals[st.A[0].val].kind == ValKind::InputMat;
            const bool b = st.B.size() == 1 && p.vals[st.B[0].val].kind == ValKind::InputMat;
            if (a || b) return fmt;
        }
    return -1;
}

size_t factor_operand_bytes(int format, int64_t n) {
    if (format < 0) return 0;
    return prep_bytes(format, gemm_npad(n, format), 1);
}

ScheduleSizes schedule_sizes(const Plan &plan, const std::vector<const VProgram *> &progs,
                             const std::vector<Dataset> &data, const SliceRange &range) {
    Schedule S;
    int st = 0;
    const Cfg cfg = make_cfg(plan.opts.precision);
    ScheduleSizes z;
    std::string err = build_schedule(plan, progs, data, cfg, {}, worst_signs(cfg, data), nullptr, S, &st, range);
    if (!err.empty()) return z;
    z.arena = S.arena_bytes;
    z.blob = S.blob_bytes;
    z.results = (size_t)S.nprog_total * cfg.wide_es + data.size() * (cfg.wide_es + 8);
    return z;
}

size_t workspace_bytes(const Plan &plan, const std::vector<const VProgram *> &progs,
                       const std::vector<int64_t> &ns, bool shared_factor, int *status) {
    std::vector<Dataset> data;
    static char fake[1 << 16];
    size_t slot = 0;
    for (int64_t n : ns) {
        Dataset d;
        d.n = n;
        d.symmetric = plan.opts.symmetric;
        d.nonneg = shared_factor;  // the sample entry points' RBF factors
        // distinct placeholder pointers per dataset (and per edge unless shared)
        for (size_t k = 0; k < plan.edges.size(); ++k) {
            d.factors.push_back(&fake[slot % sizeof fake]);
            if (!shared_factor) ++slot;
        }
        if (shared_factor) ++slot;
        data.push_back(d);
    }
    // Conditioned programs run in slice chunks; report the one-slice chunk.
    SliceRange rg;
    for (const VProgram *p : progs)
        if (p->slice_var >= 0) rg.hi = 1;
    Schedule S;
    int st = 0;
    const Cfg cfg = make_cfg(plan.opts.precision);
    std::string err = build_schedule(plan, progs, data, cfg, {}, worst_signs(cfg, data), nullptr, S,
                                     &st, rg);
    if (status) *status = st;
    if (!err.empty()) {
        if (getenv("USTAT_DEBUG_DAG")) fprintf(stderr, "workspace: %s\n", err.c_str());
        return 0;
    }
    return S.arena_bytes;
}

// a device or pinned-host allocation: failure is USTAT_E_NOMEM
#define ALLOCCHK(x)                                                            \
    do {                                                                       \
        hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) {                                                \
            *status = 3;                                                       \
            return std::string(#x) + ": " + hipGetErrorString(e_);             \
        }                                                                      \
    } while (0)

#define HIPCHK(x)                                                              \
    do {                                                                       \
        hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) {                                                \
            *status = 4;                                                       \
            return std::string(#x) + ": " + hipGetErrorString(e_);             \
        }                                                                      \
    } while (0)

std::string execute(const Plan &plan, const std::vector<const VProgram *> &progs,
                    const std::vector<Dataset> &data, hipStream_t stream, Runtime &rt,
                    std::vector<DatasetResult> &out, std::vector<double> *vout, int *status,
                    bool capture, const std::string &capture_key,
                    const std::function<hipError_t(hipStream_t)> &pre, const SliceRange &range,
                    const ExtMem *ext) {
    *status = 0;
    const Cfg cfg = make_cfg(plan.opts.precision);
    if (ext) capture = false;
    // host staging of the external-memory mode (ordinary host memory; every
    // copy through it completes before this function returns)
    std::vector<char> hstage_ext, hres_ext;
    const int ne = data.empty() ? 0 : (int)data[0].factors.size();
    // Split-bf16: which inputs may hold negative entries (one device scan of
    // the factors not known to be non-negative, read back once); the choice
    // of contraction scheme depends on it, so it is part of the graph key.
    std::vector<char> in_signed;
    std::string key = capture_key;
    if (cfg.pformat == PF_BF16X2) {
        std::vector<const void *> srcs;
        std::vector<int64_t> ns;
        std::vector<int> slot;
        in_signed.assign((size_t)data.size() * ne, 0);
        for (size_t d = 0; d < data.size(); ++d) {
            if (data[d].nonneg) continue;
            for (int k = 0; k < ne; ++k) {
                int dup = -1;
                for (int q = 0; q < k; ++q)
                    if (data[d].factors[q] == data[d].factors[k]) dup = q;
                if (dup >= 0) continue;
                srcs.push_back(data[d].factors[k]);
                ns.push_back(data[d].n);
                slot.push_back((int)(d * ne + k));
            }
        }
        if (!srcs.empty()) {
            const size_t cnt = srcs.size();
            char *dpre, *hpre;
            if (ext) {
                if (cnt * 20 + 256 > ext->bytes) {
                    *status = 6;
                    return "the sign scan needs more than the external workspace";
                }
                hstage_ext.assign(cnt * 20 + 64, 0);
                dpre = ext->base;
                hpre = hstage_ext.data();
            } else {
                ALLOCCHK(rt.reserve_desc(cnt * 20 + 1024));
                dpre = rt.ddesc;
                hpre = rt.hdesc;
            }
            std::memcpy(hpre, srcs.data(), cnt * 8);
            std::memcpy(hpre + cnt * 8, ns.data(), cnt * 8);
            HIPCHK(hipMemcpyAsync(dpre, hpre, cnt * 16, hipMemcpyHostToDevice, stream));
            unsigned int *dfl = reinterpret_cast<unsigned int *>(dpre + cnt * 16);
            HIPCHK(hipMemsetAsync(dfl, 0, cnt * 4, stream));
            HIPCHK(launch_signscan(reinterpret_cast<const void *const *>(dpre),
                                   reinterpret_cast<const int64_t *>(dpre + cnt * 8), (int)cnt,
                                   cfg.in_dt == DT_F32, dfl, stream));
            std::vector<unsigned int> fl(cnt);
            HIPCHK(hipMemcpyAsync(fl.data(), dfl, cnt * 4, hipMemcpyDeviceToHost, stream));
            HIPCHK(hipStreamSynchronize(stream));
            for (size_t i = 0; i < cnt; ++i) in_signed[slot[i]] = fl[i] ? 1 : 0;
            // repeated pointers share their first edge's flag
            for (size_t d = 0; d < data.size(); ++d)
                for (int k = 0; k < ne; ++k)
                    for (int q = 0; q < k; ++q)
                        if (data[d].factors[q] == data[d].factors[k]) {
                            in_signed[d * ne + k] = in_signed[d * ne + q];
                            break;
                        }
            key += "|sign:";
            for (char c : in_signed) key += c ? '1' : '0';
        }
    }
    std::vector<double> in_bound;
    std::vector<char> in_binary;  // per dataset*edge (INT): all entries 0 or 1
    Profiler *prof = Profiler::active();
    if (cfg.domain == DOM_INT) {
        // Exact path: the a-priori bounds start from the inputs' true
        // maxima (one small device-to-host copy).
        // one scan per distinct matrix; slot_of maps (dataset, edge) to it
        std::vector<const int8_t *> srcs;
        std::vector<int64_t> ns;
        std::vector<size_t> slot_of;
        for (auto &d : data)
            for (int k = 0; k < ne; ++k) {
                const int8_t *ptr = static_cast<const int8_t *>(d.factors[k]);
                size_t j = 0;
                while (j < srcs.size() && !(srcs[j] == ptr && ns[j] == d.n)) ++j;
                if (j == srcs.size()) {
                    srcs.push_back(ptr);
                    ns.push_back(d.n);
                }
                slot_of.push_back(j);
            }
        size_t cnt = srcs.size();
        size_t bytes = cnt * (8 + 8 + 16);
        char *dpre, *hpre, *hmx;
        if (ext) {
            // the start of the external region; done with before the
            // evaluation's own layout is written there
            if (bytes + 256 > ext->bytes) {
                *status = 6;
                return "the input maxima pass needs more than the external workspace";
            }
            hstage_ext.assign(cnt * 32, 0);
            dpre = ext->base;
            hpre = hstage_ext.data();
            hmx = hstage_ext.data() + cnt * 16;
        } else {
            ALLOCCHK(rt.reserve_desc(bytes + 1024));
            ALLOCCHK(rt.reserve_hres(cnt * 16 + 64));
            dpre = rt.ddesc;
            hpre = rt.hdesc;
            hmx = rt.hres;
        }
        std::memcpy(hpre, srcs.data(), cnt * 8);
        std::memcpy(hpre + cnt * 8, ns.data(), cnt * 8);
        HIPCHK(hipMemcpyAsync(dpre, hpre, cnt * 16, hipMemcpyHostToDevice, stream));
        unsigned long long *dmx = reinterpret_cast<unsigned long long *>(dpre + cnt * 16);
        hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(256), 0, stream, dmx, 2 * cnt);
        HIPCHK(hipGetLastError());
        HIPCHK(launch_absmax_i8(reinterpret_cast<const int8_t *const *>(dpre),
                                reinterpret_cast<const int64_t *>(dpre + cnt * 8), (int)cnt,
                                dmx, stream));
        HIPCHK(hipMemcpyAsync(hmx, dmx, cnt * 16, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        const size_t nin = slot_of.size();
        in_bound.resize(nin);
        in_binary.assign(nin, 0);
        const unsigned long long *hm = reinterpret_cast<const unsigned long long *>(hmx);
        for (size_t i = 0; i < nin; ++i) {
            const size_t j = slot_of[i];
            in_bound[i] = (double)hm[j];
            in_binary[i] = hm[j] <= 1 && hm[cnt + j] == 0;  // every entry 0 or 1
        }
    }
    if (cfg.domain == DOM_INT) {
        // the schedule depends on which inputs are 0/1 and on their maxima
        key += "|int:";
        for (char c : in_binary) key += c ? '1' : '0';
        for (double b : in_bound) key += "," + std::to_string((unsigned long long)b);
    }
    if (capture) {
        auto git = rt.graphs.find(key);
        if (git != rt.graphs.end() && git->second.nd == (int)data.size()) {
            // Replay: the graph reads its own device descriptor blob and
            // recomputes everything in the workspace from the inputs (the
            // exact path's input maxima are staged again where it copies
            // them from).
            const Runtime::GraphEntry &ge = git->second;
            if (!ge.inmx.empty())
                std::memcpy(rt.hdesc + ge.inmx_off, ge.inmx.data(), ge.inmx.size() * 8);
            HIPCHK(hipGraphLaunch(ge.exec, stream));
            HIPCHK(hipStreamSynchronize(stream));
            const int nd = ge.nd, nprog = ge.nprog;
            out.assign(nd, DatasetResult());
            size_t vbytes = (size_t)nprog * cfg.wide_es, ubytes = (size_t)nd * cfg.wide_es;
            const char *h = rt.hres;
            if (vout) {
                vout->assign(nprog, 0.0);
                for (int i = 0; i < nprog; ++i)
                    (*vout)[i] = cfg.domain == DOM_FP ? reinterpret_cast<const double *>(h)[i]
                                                      : (double)reinterpret_cast<const __int128 *>(h)[i];
            }
            for (int d = 0; d < nd; ++d) {
                if (cfg.domain == DOM_FP) {
                    out[d].value = reinterpret_cast<const double *>(h + vbytes)[d];
                } else {
                    const __int128 u = reinterpret_cast<const __int128 *>(h + vbytes)[d];
                    out[d].value = (double)u;
                    out[d].exact_hi = (int64_t)(u >> 64);
                    out[d].exact_lo = (uint64_t)u;
                }
                out[d].scale = reinterpret_cast<const double *>(h + vbytes + ubytes)[d];
                out[d].err_est = ge.err_est[d];
            }
            return "";
        }
    }
    // The layout is deterministic: build once against the arena already
    // held and keep the result when it fits; otherwise size it, grow the
    // arena and build again with the new base.
    Schedule S;
    std::string err;
    bool built = false;
    // the arena, blob and accumulators used below
    char *arena = rt.arena, *vacc = rt.vacc, *hres = rt.hres, *hdesc = rt.hdesc;
    const int nd = (int)data.size();
    if (ext) {
        err = build_schedule(plan, progs, data, cfg, in_bound, in_signed, ext->base, S, status, range,
                             in_binary);
        if (!err.empty()) return err;
        const size_t nres_ext = (size_t)S.nprog_total * cfg.wide_es + (size_t)nd * cfg.wide_es + (size_t)nd * 8;
        const size_t need = up(S.arena_bytes, kAlign) + up(S.blob_bytes, kAlign) + S.n_inmx * 8 +
                            up(nres_ext + 64, kAlign);
        if (need > ext->bytes) {
            *status = 6;
            return "the evaluation needs " + std::to_string(need) + " bytes of workspace, above the " +
                   std::to_string(ext->bytes) + " bytes of the fixed device buffer";
        }
        arena = ext->base;
        vacc = ext->base + ext->bytes - up(nres_ext + 64, kAlign);
        hres_ext.assign(nres_ext + 64, 0);
        hres = hres_ext.data();
        hstage_ext.assign(up(S.blob_bytes, 64) + S.n_inmx * 8 + 64, 0);
        hdesc = hstage_ext.data();
        built = true;
    } else if (rt.arena) {
        err = build_schedule(plan, progs, data, cfg, in_bound, in_signed, rt.arena, S, status, range,
                             in_binary);
        if (!err.empty()) return err;
        built = S.arena_bytes <= rt.arena_bytes;
    } else {
        err = build_schedule(plan, progs, data, cfg, in_bound, in_signed, nullptr, S, status, range,
                             in_binary);
        if (!err.empty()) return err;
    }
    if (plan.opts.workspace_limit && S.arena_bytes > plan.opts.workspace_limit) {
        *status = 6;
        return "workspace of " + std::to_string(S.arena_bytes) + " bytes exceeds the limit";
    }
    if (!built) {
        hipError_t e = rt.reserve_arena(S.arena_bytes);
        if (e != hipSuccess) {
            *status = 3;
            return std::string("device workspace allocation failed: ") + hipGetErrorString(e);
        }
        err = build_schedule(plan, progs, data, cfg, in_bound, in_signed, rt.arena, S, status, range,
                             in_binary);
        if (!err.empty()) return err;
        arena = rt.arena;
    }
    // results buffer [V per program | U per dataset | S per dataset], read
    // back with one copy
    const size_t vbytes0 = (size_t)S.nprog_total * cfg.wide_es, ubytes0 = (size_t)nd * cfg.wide_es;
    const size_t nres = vbytes0 + ubytes0 + (size_t)nd * 8;
    if (!ext) {
        // room for the blob and, behind it, the staged input maxima (reserved
        // before any asynchronous copy reads the pinned buffer)
        ALLOCCHK(rt.reserve_desc(up(S.blob_bytes, 64) + S.n_inmx * 8 + 1024));
        ALLOCCHK(rt.reserve_hres(nres + 64));
        if (range.first) ALLOCCHK(rt.reserve_vacc(nres + 64));
        vacc = rt.vacc;
        hres = rt.hres;
        hdesc = rt.hdesc;
    }

    {
        char *hblob = hdesc;
        Runtime::GraphEntry entry;
        if (capture) {
            auto old = rt.graphs.find(key);
            if (old != rt.graphs.end()) {
                if (old->second.exec) (void)hipGraphExecDestroy(old->second.exec);
                if (old->second.blob) (void)hipFree(old->second.blob);
                rt.graphs.erase(old);
            }
            if (rt.graphs.size() >= 64) rt.drop_graphs();
            // the graph's own descriptors, uploaded once before capture
            ALLOCCHK(hipMalloc((void **)&entry.blob, S.blob_bytes + 64));
            entry.blob_bytes = S.blob_bytes + 64;
        }
        std::memcpy(hblob, S.blob.h.data(), S.blob_bytes);
        char *dd = capture ? entry.blob : ext ? arena + up(S.arena_bytes, kAlign) : rt.ddesc;
        {
            hipError_t ue = hipMemcpyAsync(dd, hblob, S.blob_bytes, hipMemcpyHostToDevice, stream);
            if (ue != hipSuccess) {
                if (entry.blob) (void)hipFree(entry.blob);
                *status = 4;
                return std::string("descriptor upload: ") + hipGetErrorString(ue);
            }
        }
        hipGraph_t g = nullptr;
        // Ends a capture left open when a host exception unwinds through the
        // launch sequence (the error paths below end it themselves).
        struct CaptureGuard {
            hipStream_t s;
            char **blob;
            bool active = false;
            ~CaptureGuard() {
                if (!active) return;
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(s, &junk);
                if (junk) (void)hipGraphDestroy(junk);
                (void)hipStreamSynchronize(s);
                if (*blob) (void)hipFree(*blob);
                *blob = nullptr;
            }
        } cguard{stream, &entry.blob};
        // a level's reductions run on a second stream beside its GEMMs
        // (created before any capture begins; never for external memory)
        const bool overlap = plan.opts.overlap && !ext;
        if (overlap) HIPCHK(rt.reserve_side(S.levels.size()));
        if (capture) {
            HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            cguard.active = true;
        }
        auto fail = [&](hipError_t e, const char *what) -> std::string {
            cguard.active = false;
            if (capture) {
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(stream, &junk);
                if (junk) (void)hipGraphDestroy(junk);
                (void)hipStreamSynchronize(stream);
                if (entry.blob) (void)hipFree(entry.blob);
                entry.blob = nullptr;
            }
            *status = 4;
            return std::string(what) + ": " + hipGetErrorString(e);
        };
        hipError_t e = hipSuccess;
        if (inject_fire(INJ_HIP)) return fail(hipErrorLaunchFailure, "injected launch failure");
        if (pre) {
            e = pre(stream);
            if (e != hipSuccess) return fail(e, "factor build");
        }
        // zero running maxima (a fill kernel, safe under graph capture)
        if (cfg.domain == DOM_INT && S.n_mx) {
            hipLaunchKernelGGL(k_fill_zero, dim3(64), dim3(256), 0, stream,
                               reinterpret_cast<unsigned long long *>(arena + S.off_mx), S.n_mx);
            if ((e = hipGetLastError()) != hipSuccess) return fail(e, "fill");
        }
        if (cfg.domain == DOM_INT) {
            // input maxima, from the host copy taken above
            std::vector<unsigned long long> im(S.n_inmx);
            for (size_t i = 0; i < S.n_inmx; ++i) im[i] = (unsigned long long)in_bound[i];
            // stage behind the blob in the pinned buffer
            size_t off = up(S.blob_bytes, 64);
            std::memcpy(hdesc + off, im.data(), im.size() * 8);
            e = hipMemcpyAsync(arena + S.off_inmx, hdesc + off, im.size() * 8,
                               hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return fail(e, "input maxima upload");
            if (capture) {
                entry.inmx = im;
                entry.inmx_off = off;
            }
        }
        if (!S.diag.empty()) {
            e = launch_diag(reinterpret_cast<DiagDesc *>(dd + S.off_diag), (int)S.diag.size(),
                            S.diag_maxn, cfg.domain, stream);
            if (e != hipSuccess) return fail(e, "diag");
        }
        for (size_t L = 0; L < S.levels.size(); ++L) {
            auto &W = S.levels[L];
            if (!W.sl.empty()) {
                e = launch_slicesrc(reinterpret_cast<SliceDesc *>(dd + W.off_sl), (int)W.sl.size(),
                                    W.sl_tiles, cfg.domain, stream);
                if (e != hipSuccess) return fail(e, "slice sources");
            }
            if (!W.tr.empty()) {
                ProfScope ps(prof, KIND_PREP, stream, 0, W.tr_bytes);
                e = launch_transpose(reinterpret_cast<TransDesc *>(dd + W.off_tr), (int)W.tr.size(),
                                     W.tr_tiles, stream);
                if (e != hipSuccess) return fail(e, "transpose");
            }
            // The level's reductions read only earlier levels' results, as do
            // its GEMMs: with both present they run on the second stream,
            // forked here and joined before the level's partial sums.
            bool any_red = !W.e1.empty() || !W.e0.empty();
            for (int k = 0; k < LevelWork::kColSlots; ++k) any_red = any_red || !W.col[k].empty();
            const bool fork = overlap && any_red &&
                              (!W.gemm_big.empty() || !W.gemm_sym.empty() || !W.gemm6.empty() ||
                               !W.gemm.empty());
            hipStream_t rs = stream;
            if (fork) {
                if ((e = hipEventRecord(rt.level_events[2 * L], stream)) != hipSuccess ||
                    (e = hipStreamWaitEvent(rt.side, rt.level_events[2 * L], 0)) != hipSuccess)
                    return fail(e, "fork to the second stream");
                rs = rt.side;
            }
            if (!W.prep.empty()) {
                ProfScope ps(prof, KIND_PREP, stream, 0, W.prep_bytes);
                e = launch_prep(reinterpret_cast<PrepDesc *>(dd + W.off_prep), (int)W.prep.size(),
                                W.prep_tiles, cfg.domain, stream);
                if (e != hipSuccess) return fail(e, "prep");
            }
            if (!W.gemm_big.empty()) {
                ProfScope ps(prof, KIND_GEMM, stream, W.gemm_big_flops);
                e = launch_gemm(reinterpret_cast<GemmDesc *>(dd + W.off_gemm_big),
                                (int)W.gemm_big.size(), W.gemm_big_tiles, cfg.prec, 256, stream);
                if (e != hipSuccess) return fail(e, "gemm");
            }
            if (!W.gemm_sym.empty()) {
                // the product and its fix-up, timed together
                ProfScope ps(prof, KIND_GEMM, stream, W.gemm_sym_flops);
                e = launch_gemm_sym(reinterpret_cast<GemmDesc *>(dd + W.off_gemm_sym),
                                    (int)W.gemm_sym.size(), W.gemm_sym_units, W.sym_blocks,
                                    W.gemm_sym_tiles, W.sym_part, stream);
                if (e != hipSuccess) return fail(e, "symmetric gemm");
            }
            if (!W.gemm6.empty()) {
                ProfScope ps(prof, KIND_GEMM, stream, W.gemm6_flops);
                e = launch_gemm(reinterpret_cast<GemmDesc *>(dd + W.off_gemm6), (int)W.gemm6.size(),
                                W.gemm6_tiles, kGemmBf16x6, 128, stream);
                if (e != hipSuccess) return fail(e, "gemm");
            }
            if (!W.gemm.empty()) {
                ProfScope ps(prof, KIND_GEMM, stream, W.gemm_flops);
                e = launch_gemm(reinterpret_cast<GemmDesc *>(dd + W.off_gemm), (int)W.gemm.size(),
                                W.gemm_tiles, cfg.prec, 128, stream);
                if (e != hipSuccess) return fail(e, "gemm");
            }
            for (int k = 0; k < LevelWork::kColSlots; ++k) {
                if (W.col[k].empty()) continue;
                ProfScope ps(prof, KIND_ELIM1, rs, 0, W.col_bytes[k]);
                e = launch_colred(reinterpret_cast<ColDesc *>(dd + W.off_col[k]), (int)W.col[k].size(),
                                  W.col_tiles[k], k % kColMat + 1, W.col_maxout[k], W.col_dtype[k],
                                  cfg.domain, k >= kColMat, rs);
                if (e != hipSuccess) return fail(e, "column reduction");
            }
            if (!W.e1.empty()) {
                ProfScope ps(prof, KIND_ELIM1, rs, 0, W.e1_bytes);
                e = launch_elim1(reinterpret_cast<Elim1Desc *>(dd + W.off_e1), (int)W.e1.size(),
                                 W.e1_tiles, cfg.domain, rs);
                if (e != hipSuccess) return fail(e, "elim1");
            }
            if (!W.e0.empty()) {
                e = launch_elim0(reinterpret_cast<Elim0Desc *>(dd + W.off_e0), (int)W.e0.size(),
                                 cfg.domain, rs);
                if (e != hipSuccess) return fail(e, "elim0");
            }
            if (fork) {
                if ((e = hipEventRecord(rt.level_events[2 * L + 1], rt.side)) != hipSuccess ||
                    (e = hipStreamWaitEvent(stream, rt.level_events[2 * L + 1], 0)) != hipSuccess)
                    return fail(e, "join of the second stream");
            }
            if (!W.red.empty()) {
                ProfScope ps(prof, KIND_REDUCE, stream, 0);
                e = launch_reduce(reinterpret_cast<ReduceDesc *>(dd + W.off_red), (int)W.red.size(),
                                  W.red_maxlen, cfg.domain, stream);
                if (e != hipSuccess) return fail(e, "reduce");
            }
        }
        e = launch_combine(reinterpret_cast<CombineDesc *>(dd + S.off_comb), nd,
                           reinterpret_cast<int32_t *>(dd + S.off_toff),
                           reinterpret_cast<int32_t *>(dd + S.off_tcnt),
                           reinterpret_cast<int32_t *>(dd + S.off_soff),
                           reinterpret_cast<int32_t *>(dd + S.off_scnt),
                           reinterpret_cast<int32_t *>(dd + S.off_sidx),
                           reinterpret_cast<int64_t *>(dd + S.off_mu), arena + S.off_scal,
                           vacc, range.first ? 1 : 0, range.last ? 1 : 0, vacc + vbytes0,
                           reinterpret_cast<double *>(vacc + vbytes0 + ubytes0), cfg.domain,
                           stream);
        if (e != hipSuccess) return fail(e, "combine");
        // results: V (all), U (per dataset), S (per dataset) in one copy
        e = hipMemcpyAsync(hres, vacc, nres, hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return fail(e, "result copy");
        if (capture) {
            e = hipStreamEndCapture(stream, &g);
            cguard.active = false;
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(stream);
                (void)hipFree(entry.blob);
                *status = 4;
                return std::string("end capture: ") + hipGetErrorString(e);
            }
            hipError_t ie = hipGraphInstantiate(&entry.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                (void)hipStreamSynchronize(stream);
                (void)hipFree(entry.blob);
                *status = 4;
                return std::string("graph instantiate: ") + hipGetErrorString(ie);
            }
            entry.nd = nd;
            entry.nprog = S.nprog_total;
            for (int d = 0; d < nd; ++d)
                entry.err_est.push_back(error_estimate(cfg.prec, data[d].n, S.depth, S.two_plane[d] != 0));
            rt.graphs[key] = entry;
            HIPCHK(hipGraphLaunch(entry.exec, stream));
        }
    }
    HIPCHK(hipStreamSynchronize(stream));
    if (prof) prof->collect();
    // unpack
    out.assign(nd, DatasetResult());
    size_t vbytes = (size_t)S.nprog_total * cfg.wide_es, ubytes = (size_t)nd * cfg.wide_es;
    const char *h = hres;
    if (vout) vout->assign(S.nprog_total, 0.0);
    for (int i = 0; i < S.nprog_total && vout; ++i) {
        if (cfg.domain == DOM_FP) (*vout)[i] = reinterpret_cast<const double *>(h)[i];
        else (*vout)[i] = (double)reinterpret_cast<const __int128 *>(h)[i];
    }
    for (int d = 0; d < nd; ++d) {
        if (cfg.domain == DOM_FP) {
            out[d].value = reinterpret_cast<const double *>(h + vbytes)[d];
        } else {
            __int128 u = reinterpret_cast<const __int128 *>(h + vbytes)[d];
            out[d].value = (double)u;
            out[d].exact_hi = (int64_t)(u >> 64);
            out[d].exact_lo = (uint64_t)u;
        }
        out[d].scale = reinterpret_cast<const double *>(h + vbytes + ubytes)[d];
        out[d].err_est = error_estimate(cfg.prec, data[d].n, S.depth, S.two_plane[d] != 0);
    }
    return "";
}

std::string execute_all(const Plan &plan, const std::vector<const VProgram *> &progs,
                        const std::vector<Dataset> &data, hipStream_t stream, Runtime &rt,
                        std::vector<DatasetResult> &out, std::vector<double> *vout, int *status,
                        bool capture, const std::string &capture_key,
                        const std::function<hipError_t(hipStream_t)> &pre, const ExtMem *ext) {
    bool sliced = false;
    for (const VProgram *p : progs) sliced = sliced || p->slice_var >= 0;
    for (const Dataset &d : data)
        for (const VProgram *p : d.progs) sliced = sliced || p->slice_var >= 0;
    if (!sliced)
        return execute(plan, progs, data, stream, rt, out, vout, status, capture, capture_key, pre,
                       SliceRange(), ext);
    // Slice chunks sized to the budget: opts.workspace_limit, else half of
    // the free device memory (plus what this runtime already holds), or the
    // external buffer less its accumulators and descriptors.
    int64_t nmax = 0;
    for (auto &d : data) nmax = std::max(nmax, d.n);
    size_t budget = plan.opts.workspace_limit;
    if (ext) {
        const size_t keep = ext->bytes / 8;
        budget = budget ? std::min(budget, ext->bytes - keep) : ext->bytes - keep;
    } else if (!budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            *status = 4;
            return "hipMemGetInfo failed";
        }
        budget = (fr + rt.arena_bytes) / 2;
    }
    SliceRange r1, r2;
    r1.hi = 1;
    r2.hi = 2;
    const size_t a1 = schedule_sizes(plan, progs, data, r1).arena;
    const size_t a2 = schedule_sizes(plan, progs, data, r2).arena;
    const size_t per = a2 > a1 ? a2 - a1 : 1;
    int64_t chunk = a1 >= budget ? 1 : (int64_t)((budget - a1) / per) + 1;
    chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, nmax));
    std::vector<double> est;  // largest estimate over the chunks, per dataset
    for (int64_t lo = 0; lo < nmax; lo += chunk) {
        SliceRange rg;
        rg.lo = lo;
        rg.hi = std::min(nmax, lo + chunk);
        rg.include_unsliced = lo == 0;
        rg.first = lo == 0;
        rg.last = rg.hi >= nmax;
        std::string err = execute(plan, progs, data, stream, rt, out, vout, status, false, "",
                                  lo == 0 ? pre : nullptr, rg, ext);
        if (!err.empty()) return err;
        est.resize(out.size(), 0.0);
        for (size_t d = 0; d < out.size(); ++d) est[d] = std::max(est[d], out[d].err_est);
    }
    for (size_t d = 0; d < out.size(); ++d) out[d].err_est = est[d];
    return "";
}

}  // namespace ustat
