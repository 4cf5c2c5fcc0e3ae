// Executor.  All steps of all restricted V-statistics (and of all datasets
// of a batch) are grouped by dependency level; each level issues at most one
// launch per step kind: operand prep, GEMM, column reduction, deg-0
// reduction, then the fixed-order partial reductions.  A final launch forms
// V_pi as the product of its scalars and the Moebius combination
// U = sum mu_pi V_pi (Lemma 2) with S = sum |mu_pi V_pi|.
#include "exec.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "kernels.hpp"
#include "profile.hpp"

namespace ustat {

Runtime::~Runtime() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (arena) (void)hipFree(arena);
    if (ddesc) (void)hipFree(ddesc);
    if (hdesc) (void)hipHostFree(hdesc);
    if (hres) (void)hipHostFree(hres);
    if (gblob) (void)hipHostFree(gblob);
}

hipError_t Runtime::reserve_arena(size_t bytes) {
    if (bytes <= arena_bytes && arena) return hipSuccess;
    if (graph) {
        (void)hipGraphExecDestroy(graph);
        graph = nullptr;
        graph_key.clear();
    }
    if (arena) (void)hipFree(arena);
    arena = nullptr;
    arena_bytes = 0;
    hipError_t e = hipMalloc(&arena, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) arena_bytes = bytes;
    return e;
}

hipError_t Runtime::reserve_desc(size_t bytes) {
    if (bytes <= ddesc_bytes && ddesc) return hipSuccess;
    if (graph) {
        (void)hipGraphExecDestroy(graph);
        graph = nullptr;
        graph_key.clear();
    }
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

hipError_t Runtime::reserve_hres(size_t bytes) {
    if (bytes <= hres_bytes && hres) return hipSuccess;
    if (graph) {
        (void)hipGraphExecDestroy(graph);
        graph = nullptr;
        graph_key.clear();
    }
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
    std::vector<Elim1Desc> e1;
    int64_t e1_tiles = 0;
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
    size_t off_scal = 0, off_v = 0, off_u = 0, off_s = 0, off_mx = 0, off_limbs = 0,
           off_inmx = 0;
    size_t n_scal = 0, n_mx = 0, n_limbs = 0, n_inmx = 0;
    std::vector<DiagDesc> diag;
    int64_t diag_maxn = 1;
    std::vector<LevelWork> levels;
    std::vector<CombineDesc> comb;
    std::vector<int32_t> scal_off, scal_cnt, scal_idx;
    std::vector<int64_t> mu;
    size_t off_diag = 0, off_comb = 0, off_soff = 0, off_scnt = 0, off_sidx = 0, off_mu = 0;
    size_t blob_bytes = 0;
    Blob blob;
    int nprog_total = 0;
};

struct Cfg {
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
    c.prec = prec;
    switch (prec) {
        case 0: c = {0, DOM_FP, DT_F64, DT_F64, 8, PF_F64, 8}; break;
        case 1: c = {1, DOM_FP, DT_F32, DT_F32, 4, PF_F32, 8}; break;
        case 2: c = {2, DOM_FP, DT_F32, DT_F32, 4, PF_BF16X2, 8}; break;
        default: c = {3, DOM_INT, DT_I8, DT_I64, 8, PF_I8LIMBS, 16}; break;
    }
    return c;
}

size_t prep_bytes(const Cfg &c, int64_t npad, int limbs) {
    size_t plane = (size_t)npad * (size_t)npad;
    switch (c.pformat) {
        case PF_F64: return plane * 8;
        case PF_F32: return plane * 4;
        case PF_BF16X2: return plane * 4;
        default: return plane * (size_t)limbs;
    }
}

// Builds the schedule.  With base == nullptr only sizes are computed; a
// second call with the real arena base fills every pointer (the layout is
// deterministic, so offsets agree).
std::string build_schedule(const Plan &plan, const std::vector<const VProgram *> &progs,
                           const std::vector<Dataset> &data, const Cfg &cfg,
                           const std::vector<double> &in_bound,  // per dataset*edge (INT)
                           char *base, Schedule &S, int *status) {
    S = Schedule();
    Arena A;
    const int ne = (int)plan.edges.size();
    const int nd = (int)data.size();
    const int np = (int)progs.size();
    S.nprog_total = nd * np;
    auto P = [&](size_t off) -> void * { return base ? (void *)(base + off) : nullptr; };

    // ---- scalar slots and value bookkeeping
    struct VInfo {
        size_t off = 0, bytes = 0;
        int last_use = 0;
        int scal = -1;     // scalar slot
        int mx = -1;       // INT max slot
        double bound = 0;  // INT a-priori bound
        bool persistent = false;
    };
    std::vector<std::vector<VInfo>> vinfo(nd * np);
    int max_depth = 0;
    size_t nscal = 0, nmx = 0;
    for (int d = 0; d < nd; ++d)
        for (int p = 0; p < np; ++p) {
            const VProgram &pr = *progs[p];
            auto &vi = vinfo[d * np + p];
            vi.assign(pr.vals.size(), VInfo());
            max_depth = std::max(max_depth, pr.depth);
            for (const Step &st : pr.steps) {
                auto use = [&](int v) { vi[v].last_use = std::max(vi[v].last_use, st.level); };
                for (auto &o : st.A) use(o.val);
                for (auto &o : st.B) use(o.val);
                for (auto &o : st.Z) use(o.val);
                for (int q : st.sv) use(q);
                for (int q : st.aw) use(q);
                for (int q : st.bx) use(q);
            }
            for (size_t v = 0; v < pr.vals.size(); ++v) {
                if (pr.vals[v].kind == ValKind::Scalar) vi[v].scal = (int)nscal++;
                if (cfg.domain == DOM_INT && (pr.vals[v].kind == ValKind::Vec ||
                                              pr.vals[v].kind == ValKind::Mat))
                    vi[v].mx = (int)nmx++;
            }
        }
    S.n_scal = nscal;
    // input diag vectors, deduped per (dataset, factor pointer)
    std::map<std::pair<int, const void *>, std::pair<size_t, int>> diag_of;  // -> (offset, mx slot)
    for (int d = 0; d < nd; ++d)
        for (int p = 0; p < np; ++p)
            for (const Value &v : progs[p]->vals)
                if (v.kind == ValKind::InputDiag) {
                    auto key = std::make_pair(d, data[d].factors[v.src]);
                    if (!diag_of.count(key)) {
                        int slot = cfg.domain == DOM_INT ? (int)nmx++ : -1;
                        diag_of[key] = {0, slot};
                    }
                }
    S.n_mx = nmx;
    // fixed regions
    S.off_scal = A.alloc(nscal * cfg.wide_es + 16);
    S.off_v = A.alloc((size_t)S.nprog_total * cfg.wide_es + 16);
    S.off_u = A.alloc((size_t)nd * cfg.wide_es + 16);
    S.off_s = A.alloc((size_t)nd * 8 + 16);
    S.off_mx = A.alloc(nmx * 8 + 16);
    for (auto &kv : diag_of) {
        kv.second.first = A.alloc((size_t)data[kv.first.first].n * 8);
        const void *src = kv.first.second;
        DiagDesc dd;
        dd.src = {src, data[kv.first.first].n, cfg.in_dt, 0, 0, 0};
        dd.dst = P(kv.second.first);
        dd.n = data[kv.first.first].n;
        dd.mx_out = (cfg.domain == DOM_INT && base)
                        ? reinterpret_cast<unsigned long long *>(base + S.off_mx) + kv.second.second
                        : nullptr;
        S.diag.push_back(dd);
        S.diag_maxn = std::max(S.diag_maxn, dd.n);
    }

    // a-priori bounds (INT)
    auto in_b = [&](int d, int k) { return in_bound.empty() ? 127.0 : in_bound[d * ne + k]; };

    // helpers to resolve operands
    auto vptr = [&](int d, int p, int val) -> const void * {
        const VProgram &pr = *progs[p];
        const Value &v = pr.vals[val];
        if (v.kind == ValKind::InputMat) return data[d].factors[v.src];
        if (v.kind == ValKind::InputDiag)
            return P(diag_of[std::make_pair(d, data[d].factors[v.src])].first);
        return P(vinfo[d * np + p][val].off);
    };
    auto mxptr = [&](int d, int p, int val) -> unsigned long long * {
        if (!base || cfg.domain != DOM_INT) return nullptr;
        const VProgram &pr = *progs[p];
        const Value &v = pr.vals[val];
        unsigned long long *mx = reinterpret_cast<unsigned long long *>(base + S.off_mx);
        if (v.kind == ValKind::InputDiag)
            return mx + diag_of[std::make_pair(d, data[d].factors[v.src])].second;
        if (v.kind == ValKind::InputMat) return nullptr;  // filled via in_mx below
        return mx + vinfo[d * np + p][val].mx;
    };
    // input matrices' maxima live in their own region
    std::map<std::pair<int, int>, int> inmx_slot;  // (d, k) -> slot
    if (cfg.domain == DOM_INT)
        for (int d = 0; d < nd; ++d)
            for (int k = 0; k < ne; ++k) inmx_slot[{d, k}] = (int)S.n_inmx++;
    S.off_inmx = A.alloc(S.n_inmx * 8 + 16);
    auto inmx = [&](int d, int k) -> unsigned long long * {
        if (!base) return nullptr;
        return reinterpret_cast<unsigned long long *>(base + S.off_inmx) + inmx_slot[{d, k}];
    };
    auto mx_any = [&](int d, int p, int val) -> const unsigned long long * {
        const Value &v = progs[p]->vals[val];
        if (v.kind == ValKind::InputMat) return inmx(d, v.src);
        return mxptr(d, p, val);
    };
    auto bound_of = [&](int d, int p, int val) -> double {
        const Value &v = progs[p]->vals[val];
        if (v.kind == ValKind::InputMat || v.kind == ValKind::InputDiag) return in_b(d, v.src);
        return vinfo[d * np + p][val].bound;
    };
    const bool sparsify = plan.opts.sparsify != 0;
    auto matref = [&](int d, int p, const MatOp &o) -> MatRef {
        const Value &v = progs[p]->vals[o.val];
        MatRef m;
        m.p = vptr(d, p, o.val);
        m.ld = data[d].n;
        bool input = v.kind == ValKind::InputMat;
        m.dtype = input ? cfg.in_dt : cfg.mat_dt;
        m.trans = o.trans ? 1 : 0;
        m.zdiag = (input && sparsify) ? 1 : 0;
        m.pad = 0;
        return m;
    };
    auto level0 = [&](int p, int val) {
        ValKind k = progs[p]->vals[val].kind;
        return k == ValKind::InputMat || k == ValKind::InputDiag;
    };

    // persistent preps (operands built only from inputs), deduped per eval
    struct PrepRec {
        size_t off, bytes;
        int limbs;
        int limb_slot;
    };
    std::map<std::string, PrepRec> persistent;
    std::vector<int> limb_slots_used;
    size_t nlimb = 0;
    const double kOverflow = 4.0e18;  // < 2^62
    const double kOverflowWide = 8.0e37;

    // Pass 1 over levels: allocate, build descriptors.
    S.levels.assign(max_depth + 1, LevelWork());
    std::vector<std::pair<size_t, size_t>> level_free;  // scratch per level
    // limb-count slots are allocated lazily; they need a region sized after
    // the walk, so count first with a dry walk of the steps.
    for (int d = 0; d < nd; ++d)
        for (int p = 0; p < np; ++p)
            for (const Step &st : progs[p]->steps)
                if (st.kind == StepKind::Elim2 || st.kind == StepKind::Final2) nlimb += 2;
    S.n_limbs = nlimb;
    S.off_limbs = A.alloc(nlimb * 4 + 16);
    size_t limb_next = 0;
    auto limb_ptr = [&](size_t slot) -> int32_t * {
        return base ? reinterpret_cast<int32_t *>(base + S.off_limbs) + slot : nullptr;
    };

    for (int L = 1; L <= max_depth; ++L) {
        LevelWork &W = S.levels[L];
        std::vector<std::pair<size_t, size_t>> scratch;  // freed after level
        std::map<std::string, PrepRec> local;
        for (int d = 0; d < nd; ++d) {
            const int64_t n = data[d].n;
            const int64_t npad = up64(n, 128);
            const int tiles64 = (int)((n + 63) / 64);
            for (int p = 0; p < np; ++p) {
                const VProgram &pr = *progs[p];
                auto &vi = vinfo[d * np + p];
                for (size_t si = 0; si < pr.steps.size(); ++si) {
                    const Step &st = pr.steps[si];
                    if (st.level != L) continue;
                    VInfo &out = vi[st.out];
                    const void *scal_ptr =
                        (out.scal >= 0) ? P(S.off_scal + (size_t)out.scal * cfg.wide_es) : nullptr;
                    double prodA = 1, prodS = 1, prodB = 1, prodZ = 1, prodaw = 1, prodbx = 1;
                    for (auto &o : st.A) prodA *= bound_of(d, p, o.val);
                    for (auto &o : st.B) prodB *= bound_of(d, p, o.val);
                    for (auto &o : st.Z) prodZ *= bound_of(d, p, o.val);
                    for (int q : st.sv) prodS *= bound_of(d, p, q);
                    for (int q : st.aw) prodaw *= bound_of(d, p, q);
                    for (int q : st.bx) prodbx *= bound_of(d, p, q);
                    if ((int)st.A.size() > kMaxMat || (int)st.B.size() > kMaxMat ||
                        (int)st.Z.size() > kMaxMat || (int)st.sv.size() > kMaxVec ||
                        (int)st.aw.size() > kMaxVec || (int)st.bx.size() > kMaxVec) {
                        *status = 2;
                        return "a step has more parallel factors than the engine supports";
                    }
                    if (st.kind == StepKind::Elim0) {
                        Elim0Desc e;
                        e.n = n;
                        e.nS = (int)st.sv.size();
                        for (int q = 0; q < e.nS; ++q) e.s[q] = vptr(d, p, st.sv[q]);
                        e.out = (void *)scal_ptr;
                        W.e0.push_back(e);
                        out.bound = n * prodS;
                    } else if (st.kind == StepKind::Elim1 || st.kind == StepKind::Final1) {
                        Elim1Desc e;
                        e.n = n;
                        e.nA = (int)st.A.size();
                        e.nS = (int)st.sv.size();
                        for (int q = 0; q < e.nA; ++q) e.A[q] = matref(d, p, st.A[q]);
                        for (int q = 0; q < e.nS; ++q) e.s[q] = vptr(d, p, st.sv[q]);
                        size_t pbytes = (size_t)tiles64 * n * 8;
                        size_t poff = A.alloc(pbytes);
                        scratch.push_back({poff, pbytes});
                        e.part = P(poff);
                        e.tiles_v = tiles64;
                        e.tiles_w = tiles64;
                        e.tile_start = W.e1_tiles;
                        W.e1_tiles += (int64_t)tiles64 * tiles64;
                        W.e1.push_back(e);
                        ReduceDesc r;
                        r.part = P(poff);
                        r.T = tiles64;
                        r.len = n;
                        r.stride = n;
                        r.mx_out = nullptr;
                        double vb = n * prodA * prodS;
                        if (st.kind == StepKind::Elim1) {
                            out.bytes = (size_t)n * 8;
                            out.off = A.alloc(out.bytes);
                            out.bound = vb;
                            r.out = P(out.off);
                            r.nmul = 0;
                            r.dot = 0;
                            r.mx_out = mxptr(d, p, st.out);
                            if (cfg.domain == DOM_INT && vb > kOverflow) {
                                *status = 5;
                                return "an intermediate vector may exceed int64";
                            }
                        } else {
                            r.out = (void *)scal_ptr;
                            r.nmul = (int)st.aw.size();
                            for (int q = 0; q < r.nmul; ++q) r.mul[q] = vptr(d, p, st.aw[q]);
                            r.dot = 1;
                            out.bound = n * vb * prodaw;
                            if (cfg.domain == DOM_INT && vb > kOverflow) {
                                *status = 5;
                                return "an intermediate vector may exceed int64";
                            }
                        }
                        W.red.push_back(r);
                        W.red_maxlen = std::max<int64_t>(W.red_maxlen, n);
                    } else {
                        // GEMM step: operand preps (deduped), then the GEMM.
                        auto make_prep = [&](const std::vector<MatOp> &ops,
                                             const std::vector<int> &sv, double bound,
                                             const int32_t **limbs_p, int *max_limbs) -> const void * {
                            bool pers = true;
                            std::string key = std::to_string(d) + "|";
                            for (auto &o : ops) {
                                pers = pers && level0(p, o.val);
                                MatRef m = matref(d, p, o);
                                char buf[96];
                                const Value &v = progs[p]->vals[o.val];
                                // identity: input factor index or value pointer
                                if (v.kind == ValKind::InputMat)
                                    snprintf(buf, sizeof buf, "I%p:%d:%d;",
                                             data[d].factors[v.src], m.trans, m.zdiag);
                                else
                                    snprintf(buf, sizeof buf, "V%d.%d.%d:%d;", d, p, o.val, m.trans);
                                key += buf;
                            }
                            key += "|";
                            for (int q : sv) {
                                pers = pers && level0(p, q);
                                char buf[96];
                                const Value &v = progs[p]->vals[q];
                                if (v.kind == ValKind::InputDiag)
                                    snprintf(buf, sizeof buf, "D%p;", data[d].factors[v.src]);
                                else
                                    snprintf(buf, sizeof buf, "V%d.%d.%d;", d, p, q);
                                key += buf;
                            }
                            int cap = cfg.pformat == PF_I8LIMBS ? limbs_for(bound, 9) : 1;
                            auto &tab = pers ? persistent : local;
                            auto it = tab.find(key);
                            if (it == tab.end()) {
                                PrepRec rec;
                                rec.limbs = cap;
                                rec.bytes = prep_bytes(cfg, npad, cap);
                                rec.off = A.alloc(rec.bytes);
                                rec.limb_slot = (int)limb_next++;
                                if (!pers) scratch.push_back({rec.off, rec.bytes});
                                PrepDesc pd;
                                pd.n = n;
                                pd.npad = npad;
                                pd.ldo = npad;
                                pd.plane = npad * npad;
                                pd.nA = (int)ops.size();
                                pd.nS = (int)sv.size();
                                for (int q = 0; q < pd.nA; ++q) pd.A[q] = matref(d, p, ops[q]);
                                for (int q = 0; q < pd.nS; ++q) pd.s[q] = vptr(d, p, sv[q]);
                                pd.out = P(rec.off);
                                pd.format = cfg.pformat;
                                pd.limbs = cap;
                                pd.tiles = (int)(npad / 64);
                                pd.tile_start = W.prep_tiles;
                                W.prep_tiles += (int64_t)pd.tiles * pd.tiles;
                                pd.nmx = 0;
                                if (cfg.domain == DOM_INT) {
                                    for (auto &o : ops) pd.mx[pd.nmx++] = mx_any(d, p, o.val);
                                    for (int q : sv) pd.mx[pd.nmx++] = mx_any(d, p, q);
                                }
                                pd.limbs_out = limb_ptr(rec.limb_slot);
                                W.prep.push_back(pd);
                                it = tab.emplace(key, rec).first;
                            }
                            *limbs_p = limb_ptr(it->second.limb_slot);
                            *max_limbs = it->second.limbs;
                            return P(it->second.off);
                        };
                        GemmDesc g;
                        std::memset(&g, 0, sizeof g);
                        const int32_t *lap = nullptr, *lbp = nullptr;
                        int cla = 1, clb = 1;
                        g.A = make_prep(st.A, st.sv, prodA * prodS, &lap, &cla);
                        g.B = make_prep(st.B, {}, prodB, &lbp, &clb);
                        g.n = n;
                        g.npad = npad;
                        g.ld = npad;
                        g.plane = npad * npad;
                        g.la = cla;
                        g.lb = clb;
                        g.la_p = cfg.domain == DOM_INT ? lap : nullptr;
                        g.lb_p = cfg.domain == DOM_INT ? lbp : nullptr;
                        g.tiles = (int)(npad / 128);
                        g.tile_start = W.gemm_tiles;
                        W.gemm_tiles += (int64_t)g.tiles * g.tiles;
                        W.gemm_flops += 2.0 * (double)n * n * n;
                        double cb = n * prodA * prodS * prodB;
                        if (cfg.domain == DOM_INT) {
                            if (cb > kOverflow) {
                                *status = 5;
                                return "an intermediate matrix may exceed int64";
                            }
                            if (n >= 131072) {
                                *status = 2;
                                return "the exact path needs n < 131072 (int32 limb accumulation)";
                            }
                        }
                        if (st.kind == StepKind::Elim2) {
                            out.bytes = (size_t)n * n * cfg.mat_es;
                            out.off = A.alloc(out.bytes);
                            out.bound = cb;
                            g.final_ = 0;
                            g.dtype_c = cfg.mat_dt;
                            g.C = P(out.off);
                            g.ldc = n;
                            g.mx_out = mxptr(d, p, st.out);
                        } else {
                            g.final_ = 1;
                            g.nZ = (int)st.Z.size();
                            g.naw = (int)st.aw.size();
                            g.nbx = (int)st.bx.size();
                            for (int q = 0; q < g.nZ; ++q) g.Z[q] = matref(d, p, st.Z[q]);
                            for (int q = 0; q < g.naw; ++q) g.aw[q] = vptr(d, p, st.aw[q]);
                            for (int q = 0; q < g.nbx; ++q) g.bx[q] = vptr(d, p, st.bx[q]);
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
                            r.out = (void *)scal_ptr;
                            r.dot = 1;
                            W.red.push_back(r);
                            out.bound = (double)n * n * cb * prodZ * prodaw * prodbx;
                        }
                        W.gemm.push_back(g);
                    }
                    if (cfg.domain == DOM_INT && out.scal >= 0 && out.bound > kOverflowWide) {
                        *status = 5;
                        return "a V-statistic may exceed the 127-bit range";
                    }
                }
            }
        }
        // free scratch and values whose last use is this level
        for (auto &sc : scratch) A.release(sc.first, sc.second);
        for (int d = 0; d < nd; ++d)
            for (int p = 0; p < np; ++p) {
                auto &vi = vinfo[d * np + p];
                const VProgram &pr = *progs[p];
                for (size_t v = 0; v < pr.vals.size(); ++v)
                    if ((pr.vals[v].kind == ValKind::Vec || pr.vals[v].kind == ValKind::Mat) &&
                        vi[v].bytes && vi[v].last_use == L) {
                        A.release(vi[v].off, vi[v].bytes);
                        vi[v].bytes = 0;
                    }
            }
    }
    (void)limb_slots_used;
    (void)level_free;
    // combine tables
    for (int d = 0; d < nd; ++d) {
        CombineDesc c;
        c.p_begin = d * np;
        c.p_end = (d + 1) * np;
        S.comb.push_back(c);
        for (int p = 0; p < np; ++p) {
            const VProgram &pr = *progs[p];
            S.scal_off.push_back((int32_t)S.scal_idx.size());
            S.scal_cnt.push_back((int32_t)pr.scalars.size());
            for (int v : pr.scalars) S.scal_idx.push_back(vinfo[d * np + p][v].scal);
            S.mu.push_back(pr.mu);
            if (cfg.domain == DOM_INT) {
                double b = 1;
                for (int v : pr.scalars) b *= vinfo[d * np + p][v].bound;
                if (b * std::fabs((double)pr.mu) * np > kOverflowWide) {
                    *status = 5;
                    return "the combined U-statistic may exceed the 127-bit range";
                }
            }
        }
    }
    S.arena_bytes = A.top;
    // descriptor blob
    S.off_diag = S.blob.put(S.diag);
    for (auto &W : S.levels) {
        W.off_prep = S.blob.put(W.prep);
        W.off_gemm = S.blob.put(W.gemm);
        W.off_e1 = S.blob.put(W.e1);
        W.off_e0 = S.blob.put(W.e0);
        W.off_red = S.blob.put(W.red);
    }
    S.off_comb = S.blob.put(S.comb);
    S.off_soff = S.blob.put(S.scal_off);
    S.off_scnt = S.blob.put(S.scal_cnt);
    S.off_sidx = S.blob.put(S.scal_idx);
    S.off_mu = S.blob.put(S.mu);
    S.blob_bytes = S.blob.h.size();
    return "";
}

__global__ void k_fill_zero(unsigned long long *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

size_t workspace_bytes(const Plan &plan, const std::vector<const VProgram *> &progs,
                       const std::vector<int64_t> &ns) {
    std::vector<Dataset> data;
    static char fake;
    for (int64_t n : ns) {
        Dataset d;
        d.n = n;
        // distinct placeholder pointers per edge
        for (size_t k = 0; k < plan.edges.size(); ++k) d.factors.push_back(&fake + k);
        data.push_back(d);
    }
    Schedule S;
    int st = 0;
    std::string err = build_schedule(plan, progs, data, make_cfg(plan.opts.precision), {}, nullptr, S, &st);
    if (!err.empty()) return 0;
    return S.arena_bytes;
}

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
                    const std::function<hipError_t(hipStream_t)> &pre) {
    *status = 0;
    const Cfg cfg = make_cfg(plan.opts.precision);
    if (capture && rt.graph && rt.graph_key == capture_key && rt.g_nd == (int)data.size()) {
        // Replay: the graph uploads its own descriptor blob and recomputes
        // everything in the workspace from the inputs.
        HIPCHK(hipGraphLaunch(rt.graph, stream));
        HIPCHK(hipStreamSynchronize(stream));
        const int nd = rt.g_nd, nprog = rt.g_nprog;
        out.assign(nd, DatasetResult());
        size_t vbytes = (size_t)nprog * cfg.wide_es, ubytes = (size_t)nd * cfg.wide_es;
        const char *h = rt.hres;
        if (vout) {
            vout->assign(nprog, 0.0);
            for (int i = 0; i < nprog; ++i) (*vout)[i] = reinterpret_cast<const double *>(h)[i];
        }
        for (int d = 0; d < nd; ++d) {
            out[d].value = reinterpret_cast<const double *>(h + vbytes)[d];
            out[d].scale = reinterpret_cast<const double *>(h + vbytes + ubytes)[d];
        }
        return "";
    }
    const int ne = (int)plan.edges.size();
    std::vector<double> in_bound;
    Profiler *prof = Profiler::active();
    if (cfg.domain == DOM_INT) {
        // Exact path: the a-priori bounds start from the inputs' true
        // maxima (one small device-to-host copy).
        std::vector<const int8_t *> srcs;
        std::vector<int64_t> ns;
        for (auto &d : data)
            for (int k = 0; k < ne; ++k) {
                srcs.push_back(static_cast<const int8_t *>(d.factors[k]));
                ns.push_back(d.n);
            }
        size_t cnt = srcs.size();
        size_t bytes = cnt * (8 + 8 + 8);
        HIPCHK(rt.reserve_desc(bytes + 1024));
        HIPCHK(rt.reserve_hres(cnt * 8 + 64));
        std::memcpy(rt.hdesc, srcs.data(), cnt * 8);
        std::memcpy(rt.hdesc + cnt * 8, ns.data(), cnt * 8);
        HIPCHK(hipMemcpyAsync(rt.ddesc, rt.hdesc, cnt * 16, hipMemcpyHostToDevice, stream));
        unsigned long long *dmx = reinterpret_cast<unsigned long long *>(rt.ddesc + cnt * 16);
        hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(256), 0, stream, dmx, cnt);
        HIPCHK(hipGetLastError());
        HIPCHK(launch_absmax_i8(reinterpret_cast<const int8_t *const *>(rt.ddesc),
                                reinterpret_cast<const int64_t *>(rt.ddesc + cnt * 8), (int)cnt,
                                dmx, stream));
        HIPCHK(hipMemcpyAsync(rt.hres, dmx, cnt * 8, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        in_bound.resize(cnt);
        for (size_t i = 0; i < cnt; ++i)
            in_bound[i] = (double)reinterpret_cast<unsigned long long *>(rt.hres)[i];
    }
    Schedule S;
    std::string err = build_schedule(plan, progs, data, cfg, in_bound, nullptr, S, status);
    if (!err.empty()) return err;
    if (plan.opts.workspace_limit && S.arena_bytes > plan.opts.workspace_limit) {
        *status = 6;
        return "workspace of " + std::to_string(S.arena_bytes) + " bytes exceeds the limit";
    }
    {
        hipError_t e = rt.reserve_arena(S.arena_bytes);
        if (e != hipSuccess) {
            *status = 3;
            return std::string("device workspace allocation failed: ") + hipGetErrorString(e);
        }
    }
    err = build_schedule(plan, progs, data, cfg, in_bound, rt.arena, S, status);
    if (!err.empty()) return err;
    // room for the blob and, behind it, the staged input maxima (reserved
    // before any asynchronous copy reads the pinned buffer)
    HIPCHK(rt.reserve_desc(up(S.blob_bytes, 64) + S.n_inmx * 8 + 1024));
    const int nd = (int)data.size();
    const size_t nres = (size_t)S.nprog_total * cfg.wide_es + (size_t)nd * cfg.wide_es + nd * 8;
    HIPCHK(rt.reserve_hres(nres + 64));

    {
        char *hblob = rt.hdesc;
        if (capture) {
            if (rt.graph) {
                (void)hipGraphExecDestroy(rt.graph);
                rt.graph = nullptr;
                rt.graph_key.clear();
            }
            if (rt.gblob_bytes < S.blob_bytes + 64) {
                if (rt.gblob) (void)hipHostFree(rt.gblob);
                rt.gblob = nullptr;
                rt.gblob_bytes = 0;
                HIPCHK(hipHostMalloc((void **)&rt.gblob, S.blob_bytes * 3 / 2 + 64, hipHostMallocDefault));
                rt.gblob_bytes = S.blob_bytes * 3 / 2 + 64;
            }
            hblob = rt.gblob;
        }
        std::memcpy(hblob, S.blob.h.data(), S.blob_bytes);
        hipGraph_t g = nullptr;
        if (capture) HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        char *dd = rt.ddesc;
        auto fail = [&](hipError_t e, const char *what) -> std::string {
            if (capture) {
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(stream, &junk);
                if (junk) (void)hipGraphDestroy(junk);
            }
            *status = 4;
            return std::string(what) + ": " + hipGetErrorString(e);
        };
        hipError_t e = hipSuccess;
        if (pre) {
            e = pre(stream);
            if (e != hipSuccess) return fail(e, "factor build");
        }
        e = hipMemcpyAsync(dd, hblob, S.blob_bytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return fail(e, "descriptor upload");
        // zero running maxima (a fill kernel, safe under graph capture)
        if (cfg.domain == DOM_INT && S.n_mx) {
            hipLaunchKernelGGL(k_fill_zero, dim3(64), dim3(256), 0, stream,
                               reinterpret_cast<unsigned long long *>(rt.arena + S.off_mx), S.n_mx);
            if ((e = hipGetLastError()) != hipSuccess) return fail(e, "fill");
        }
        if (cfg.domain == DOM_INT) {
            // input maxima, from the host copy taken above
            std::vector<unsigned long long> im(S.n_inmx);
            for (size_t i = 0; i < S.n_inmx; ++i) im[i] = (unsigned long long)in_bound[i];
            // stage behind the blob in the pinned buffer
            size_t off = up(S.blob_bytes, 64);
            std::memcpy(rt.hdesc + off, im.data(), im.size() * 8);
            e = hipMemcpyAsync(rt.arena + S.off_inmx, rt.hdesc + off, im.size() * 8,
                               hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return fail(e, "input maxima upload");
        }
        if (!S.diag.empty()) {
            e = launch_diag(reinterpret_cast<DiagDesc *>(dd + S.off_diag), (int)S.diag.size(),
                            S.diag_maxn, cfg.domain, stream);
            if (e != hipSuccess) return fail(e, "diag");
        }
        for (auto &W : S.levels) {
            if (!W.prep.empty()) {
                ProfScope ps(prof, KIND_PREP, stream, 0);
                e = launch_prep(reinterpret_cast<PrepDesc *>(dd + W.off_prep), (int)W.prep.size(),
                                W.prep_tiles, cfg.domain, stream);
                if (e != hipSuccess) return fail(e, "prep");
            }
            if (!W.gemm.empty()) {
                ProfScope ps(prof, KIND_GEMM, stream, W.gemm_flops);
                e = launch_gemm(reinterpret_cast<GemmDesc *>(dd + W.off_gemm), (int)W.gemm.size(),
                                W.gemm_tiles, cfg.prec, stream);
                if (e != hipSuccess) return fail(e, "gemm");
            }
            if (!W.e1.empty()) {
                ProfScope ps(prof, KIND_ELIM1, stream, 0);
                e = launch_elim1(reinterpret_cast<Elim1Desc *>(dd + W.off_e1), (int)W.e1.size(),
                                 W.e1_tiles, cfg.domain, stream);
                if (e != hipSuccess) return fail(e, "elim1");
            }
            if (!W.e0.empty()) {
                e = launch_elim0(reinterpret_cast<Elim0Desc *>(dd + W.off_e0), (int)W.e0.size(),
                                 cfg.domain, stream);
                if (e != hipSuccess) return fail(e, "elim0");
            }
            if (!W.red.empty()) {
                ProfScope ps(prof, KIND_REDUCE, stream, 0);
                e = launch_reduce(reinterpret_cast<ReduceDesc *>(dd + W.off_red), (int)W.red.size(),
                                  W.red_maxlen, cfg.domain, stream);
                if (e != hipSuccess) return fail(e, "reduce");
            }
        }
        e = launch_combine(reinterpret_cast<CombineDesc *>(dd + S.off_comb), nd,
                           reinterpret_cast<int32_t *>(dd + S.off_soff),
                           reinterpret_cast<int32_t *>(dd + S.off_scnt),
                           reinterpret_cast<int32_t *>(dd + S.off_sidx),
                           reinterpret_cast<int64_t *>(dd + S.off_mu), rt.arena + S.off_scal,
                           rt.arena + S.off_v, rt.arena + S.off_u,
                           reinterpret_cast<double *>(rt.arena + S.off_s), cfg.domain, stream);
        if (e != hipSuccess) return fail(e, "combine");
        // results: V (all), U (per dataset), S (per dataset)
        size_t vbytes = (size_t)S.nprog_total * cfg.wide_es, ubytes = (size_t)nd * cfg.wide_es;
        e = hipMemcpyAsync(rt.hres, rt.arena + S.off_v, vbytes, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rt.hres + vbytes, rt.arena + S.off_u, ubytes, hipMemcpyDeviceToHost,
                               stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rt.hres + vbytes + ubytes, rt.arena + S.off_s, (size_t)nd * 8,
                               hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return fail(e, "result copy");
        if (capture) {
            HIPCHK(hipStreamEndCapture(stream, &g));
            if (rt.graph) (void)hipGraphExecDestroy(rt.graph);
            rt.graph = nullptr;
            hipError_t ie = hipGraphInstantiate(&rt.graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                rt.graph = nullptr;
                *status = 4;
                return std::string("graph instantiate: ") + hipGetErrorString(ie);
            }
            rt.graph_key = capture_key;
            rt.g_nd = nd;
            rt.g_nprog = S.nprog_total;
            HIPCHK(hipGraphLaunch(rt.graph, stream));
        }
    }
    HIPCHK(hipStreamSynchronize(stream));
    if (prof) prof->collect();
    // unpack
    out.assign(nd, DatasetResult());
    size_t vbytes = (size_t)S.nprog_total * cfg.wide_es, ubytes = (size_t)nd * cfg.wide_es;
    const char *h = rt.hres;
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
    }
    return "";
}

}  // namespace ustat
