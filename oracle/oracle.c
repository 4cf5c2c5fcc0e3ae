/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously correct reference computations for exact
 * higher-order U-statistics with edge-factorised kernels.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library.  It shares no code, header or table with the HIP engine.
 *
 * What is computed here, and where the paper defines it:
 *   - oracle_sum_tuples: the U-statistic of Definition 1 (sum over ordered
 *     tuples of distinct indices) and the V-statistic of Definition 2 (sum
 *     over all tuples), for a kernel that is a product of one n x n factor
 *     per edge (Definition "Multiplicative Decomposition", tensorised as in
 *     Algorithm 1).  A restricted V-statistic (Definition "Restricted
 *     V-Statistic") is the V-statistic of the edge list relabelled by block,
 *     which the Python wrapper builds.
 *   - oracle_sum_tuples_i64: the same sums in exact integer arithmetic.
 *   - oracle_lowrank_dp: the U-statistic of Definition 1 for factors of low
 *     rank, T_k = F_k G_k^T, by a subset dynamic programme over the samples.
 *     It never forms a V-statistic, so it is independent of the paper's
 *     decomposition and works at any n.
 *   - oracle_cycle_walks: closed-walk quantities of a 0/1 graph used by the
 *     textbook 5-cycle trace formula (Harary & Manvel), exact in int64.
 *
 * Floating point: every sum is in fp64 with Neumaier compensation; partial
 * sums over the outermost index are combined in a fixed order, so results
 * are bitwise reproducible for any thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORACLE_MAX_M 10
#define ORACLE_MAX_E 64

typedef struct { double s, c; } ksum;

static inline void ks_add(ksum *a, double x) {
    /* Neumaier's improved Kahan summation. */
    double t = a->s + x;
    if (__builtin_fabs(a->s) >= __builtin_fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double ks_val(const ksum *a) { return a->s + a->c; }

/* Per-depth edge schedule: after index d is chosen, multiply every factor
 * whose later endpoint is d.  Vertices are visited in the order 0..m-1. */
typedef struct {
    int m, ne, distinct;
    long n;
    const double *const *T;
    const int64_t *const *Ti;
    int cnt[ORACLE_MAX_M];
    int list[ORACLE_MAX_M][ORACLE_MAX_E];
    const int *eu, *ev;
} sched_t;

static int build_sched(sched_t *s, int m, int ne, const int *eu, const int *ev) {
    if (m < 1 || m > ORACLE_MAX_M || ne < 0 || ne > ORACLE_MAX_E) return -1;
    s->m = m; s->ne = ne; s->eu = eu; s->ev = ev;
    memset(s->cnt, 0, sizeof(s->cnt));
    for (int k = 0; k < ne; ++k) {
        if (eu[k] < 0 || eu[k] >= m || ev[k] < 0 || ev[k] >= m) return -1;
        int d = eu[k] > ev[k] ? eu[k] : ev[k];
        s->list[d][s->cnt[d]++] = k;
    }
    return 0;
}

static void rec_f64(const sched_t *s, int d, long *idx, double prod, ksum *acc) {
    const long n = s->n;
    for (long i = 0; i < n; ++i) {
        if (s->distinct) {
            int clash = 0;
            for (int j = 0; j < d; ++j) if (idx[j] == i) { clash = 1; break; }
            if (clash) continue;
        }
        idx[d] = i;
        double p = prod;
        for (int t = 0; t < s->cnt[d]; ++t) {
            int k = s->list[d][t];
            p *= s->T[k][idx[s->eu[k]] * n + idx[s->ev[k]]];
        }
        if (d + 1 == s->m) ks_add(acc, p);
        else rec_f64(s, d + 1, idx, p, acc);
    }
}

/*
 * Sum over tuples (i_0..i_{m-1}) in [n]^m -- restricted to pairwise distinct
 * indices when `distinct` is nonzero -- of
 *     prod_k T_k[i_{eu[k]}, i_{ev[k]}]
 * (factors row-major n x n, fp64).  eu[k] == ev[k] is allowed and reads the
 * diagonal.  Only prefixes numbered item_lo <= item < item_hi are summed,
 * where item = i_0 * n + i_1 for m >= 2 and item = i_0 for m == 1 (the full
 * sum is items [0, n^2) or [0, n)); a sub-range is a bounded sample of the
 * sum.  Returns 0, or -1 on bad arguments.
 */
int oracle_sum_tuples(int m, int ne, const int *eu, const int *ev,
                      const double *const *T, long n, int distinct,
                      long item_lo, long item_hi, double *out) {
    sched_t s;
    if (build_sched(&s, m, ne, eu, ev)) return -1;
    long inner = (m >= 2) ? n : 1;
    if (n < 1 || item_lo < 0 || item_hi > n * inner || item_lo > item_hi || !out) return -1;
    s.n = n; s.T = T; s.Ti = NULL; s.distinct = distinct;
    /* Parallel work items are (i_0, i_1) pairs so that even a one-value
     * range of i_0 keeps every core busy. */
    long items = item_hi - item_lo;
    ksum *part = (ksum *)calloc(items > 0 ? items : 1, sizeof(ksum));
    if (!part) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long tt = 0; tt < items; ++tt) {
        long t = item_lo + tt;
        long idx[ORACLE_MAX_M];
        idx[0] = t / inner;
        double p = 1.0;
        for (int q = 0; q < s.cnt[0]; ++q) {
            int k = s.list[0][q];
            p *= T[k][idx[0] * n + idx[0]];
        }
        ksum acc = {0.0, 0.0};
        if (m == 1) {
            ks_add(&acc, p);
        } else {
            idx[1] = t % inner;
            if (!(distinct && idx[1] == idx[0])) {
                for (int q = 0; q < s.cnt[1]; ++q) {
                    int k = s.list[1][q];
                    p *= T[k][idx[eu[k]] * n + idx[ev[k]]];
                }
                if (m == 2) ks_add(&acc, p);
                else rec_f64(&s, 2, idx, p, &acc);
            }
        }
        part[tt] = acc;
    }
    ksum tot = {0.0, 0.0};
    for (long t = 0; t < items; ++t) { ks_add(&tot, part[t].s); ks_add(&tot, part[t].c); }
    free(part);
    *out = ks_val(&tot);
    return 0;
}

static void rec_i64(const sched_t *s, int d, long *idx, __int128 prod, __int128 *acc) {
    const long n = s->n;
    for (long i = 0; i < n; ++i) {
        if (s->distinct) {
            int clash = 0;
            for (int j = 0; j < d; ++j) if (idx[j] == i) { clash = 1; break; }
            if (clash) continue;
        }
        idx[d] = i;
        __int128 p = prod;
        for (int t = 0; t < s->cnt[d]; ++t) {
            int k = s->list[d][t];
            p *= (__int128)s->Ti[k][idx[s->eu[k]] * n + idx[s->ev[k]]];
        }
        if (d + 1 == s->m) *acc += p;
        else rec_i64(s, d + 1, idx, p, acc);
    }
}

/* Exact integer version of oracle_sum_tuples (int64 factors, 128-bit sum).
 * The result is returned as (hi, lo) with value = hi * 2^64 + (uint64)lo. */
int oracle_sum_tuples_i64(int m, int ne, const int *eu, const int *ev,
                          const int64_t *const *T, long n, int distinct,
                          long lo, long hi, int64_t *out_hi, uint64_t *out_lo) {
    sched_t s;
    if (build_sched(&s, m, ne, eu, ev)) return -1;
    if (n < 1 || lo < 0 || hi > n || lo > hi || !out_hi || !out_lo) return -1;
    s.n = n; s.T = NULL; s.Ti = T; s.distinct = distinct;
    long cnt = hi - lo;
    __int128 *part = (__int128 *)calloc(cnt > 0 ? cnt : 1, sizeof(__int128));
    if (!part) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < cnt; ++t) {
        long idx[ORACLE_MAX_M];
        idx[0] = lo + t;
        __int128 p = 1;
        for (int q = 0; q < s.cnt[0]; ++q) {
            int k = s.list[0][q];
            p *= (__int128)T[k][idx[0] * n + idx[0]];
        }
        __int128 acc = 0;
        if (m == 1) acc = p;
        else rec_i64(&s, 1, idx, p, &acc);
        part[t] = acc;
    }
    __int128 tot = 0;
    for (long t = 0; t < cnt; ++t) tot += part[t];
    free(part);
    *out_hi = (int64_t)(tot >> 64);
    *out_lo = (uint64_t)tot;
    return 0;
}

/*
 * U-statistic (ordered distinct tuples) for rank-r factors
 *     T_k(i, j) = sum_c F_k[i*r + c] * G_k[j*r + c],
 * F and G given as arrays of ne pointers to n x r row-major fp64 blocks.
 * Expanding every factor over its rank index c_k turns the kernel into a
 * product of per-vertex weights phi_u(i); the sum of prod_u phi_u(i_u) over
 * distinct tuples is then a 0/1-knapsack style dynamic programme over the
 * samples: D[S] = weight of assigning the vertex set S to distinct samples
 * seen so far.  Cost r^ne * n * 2^m * m.
 */
int oracle_lowrank_dp(int m, int ne, const int *eu, const int *ev, long n, int r,
                      const double *const *F, const double *const *G, double *out) {
    if (m < 1 || m > ORACLE_MAX_M || ne < 1 || ne > 24 || r < 1 || n < 1 || !out) return -1;
    for (int k = 0; k < ne; ++k)
        if (eu[k] < 0 || eu[k] >= m || ev[k] < 0 || ev[k] >= m) return -1;
    long ncol = 1;
    for (int k = 0; k < ne; ++k) { ncol *= r; if (ncol > (1L << 24)) return -1; }
    const int full = (1 << m) - 1;
    ksum *part = (ksum *)calloc(ncol, sizeof(ksum));
    if (!part) return -1;
#pragma omp parallel
    {
        double *D = (double *)malloc(sizeof(double) * (full + 1));
        double *phi = (double *)malloc(sizeof(double) * m);
        int col[ORACLE_MAX_E];
#pragma omp for schedule(dynamic, 1)
        for (long c = 0; c < ncol; ++c) {
            long cc = c;
            for (int k = 0; k < ne; ++k) { col[k] = (int)(cc % r); cc /= r; }
            for (int S = 0; S <= full; ++S) D[S] = 0.0;
            D[0] = 1.0;
            for (long i = 0; i < n; ++i) {
                for (int u = 0; u < m; ++u) phi[u] = 1.0;
                for (int k = 0; k < ne; ++k) {
                    phi[eu[k]] *= F[k][i * r + col[k]];
                    phi[ev[k]] *= G[k][i * r + col[k]];
                }
                /* descending masks: D[S] is read before any update of this pass */
                for (int S = full; S >= 0; --S) {
                    double ds = D[S];
                    if (ds == 0.0) continue;
                    for (int u = 0; u < m; ++u)
                        if (!(S & (1 << u))) D[S | (1 << u)] += ds * phi[u];
                }
            }
            part[c].s = D[full];
            part[c].c = 0.0;
        }
        free(D); free(phi);
    }
    ksum tot = {0.0, 0.0};
    for (long c = 0; c < ncol; ++c) ks_add(&tot, part[c].s);
    free(part);
    *out = ks_val(&tot);
    return 0;
}

/*
 * Closed-walk counts of a simple undirected 0/1 graph given in CSR form
 * (both directions stored, no self-loops):
 *   out[0] = tr(A^3), out[1] = tr(A^5), out[2] = sum_i deg_i * (A^3)_ii,
 *   out[3] = tr(A^4), out[4] = sum_i deg_i^2, out[5] = number of directed
 *   edges (= 2|E|).
 * A^2 is formed densely by walking paths of length two; tr(A^5) is
 * sum over directed edges (j,k) of <row_j(A^2), row_k(A^2)>.
 */
int oracle_cycle_walks(long n, const int64_t *rowptr, const int32_t *col, int64_t *out) {
    if (n < 1 || !rowptr || !col || !out) return -1;
    int32_t *B = (int32_t *)calloc((size_t)n * (size_t)n, sizeof(int32_t));
    if (!B) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < n; ++i) {
        int32_t *Bi = B + (size_t)i * n;
        for (int64_t a = rowptr[i]; a < rowptr[i + 1]; ++a) {
            long j = col[a];
            for (int64_t b = rowptr[j]; b < rowptr[j + 1]; ++b) Bi[col[b]] += 1;
        }
    }
    int64_t trA3 = 0, trA5 = 0, degA3 = 0, trA4 = 0, deg2 = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : trA3, trA5, degA3, trA4, deg2)
    for (long i = 0; i < n; ++i) {
        const int32_t *Bi = B + (size_t)i * n;
        int64_t deg = rowptr[i + 1] - rowptr[i];
        int64_t a3 = 0;
        for (int64_t a = rowptr[i]; a < rowptr[i + 1]; ++a) {
            long k = col[a];
            a3 += Bi[k];
            const int32_t *Bk = B + (size_t)k * n;
            int64_t dot = 0;
            for (long t = 0; t < n; ++t) dot += (int64_t)Bi[t] * Bk[t];
            trA5 += dot;
        }
        int64_t sq = 0;
        for (long t = 0; t < n; ++t) sq += (int64_t)Bi[t] * Bi[t];
        trA4 += sq;
        trA3 += a3;
        degA3 += deg * a3;
        deg2 += deg * deg;
    }
    free(B);
    out[0] = trA3; out[1] = trA5; out[2] = degA3; out[3] = trA4; out[4] = deg2;
    out[5] = rowptr[n];
    return 0;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }

/* Threads used by later calls (timing the oracle on one core). */
void oracle_set_num_threads(int t) {
    if (t >= 1) omp_set_num_threads(t);
}

/* ------------------------------------------------------------------------
 * Induced motif counts of a simple graph (the motif application): for
 * every connected graph on k = 3 or 4 vertices, the number of vertex
 * subsets of size k whose induced subgraph is isomorphic to it.  Classes
 * are told apart by edge count and degree sequence:
 *   k = 3: out[0] two edges (V-shape), out[1] three (triangle);
 *   k = 4: out[0] three edges, one vertex of degree 3 (3-star);
 *          out[1] three edges, a path (degrees 2,2,1,1);
 *          out[2] four edges, a triangle with a tail (a vertex of degree 3);
 *          out[3] four edges, a 4-cycle (all degrees 2);
 *          out[4] five edges (diamond); out[5] six edges (K4).
 * ------------------------------------------------------------------------ */

static int motif_class(int k, const int *deg, int edges) {
    if (k == 3) return edges == 2 ? 0 : edges == 3 ? 1 : -1;
    int has3 = 0;
    for (int a = 0; a < 4; ++a) has3 |= deg[a] == 3;
    switch (edges) {
        case 3: return has3 ? 0 : 1;  /* connected with 3 edges: star or path */
        case 4: return has3 ? 2 : 3;
        case 5: return 4;
        case 6: return 5;
        default: return -1;
    }
}

static int connected_small(int k, const int8_t *A, long n, const long *v) {
    int seen = 1, changed = 1;
    while (changed) {
        changed = 0;
        for (int a = 0; a < k; ++a)
            if (seen >> a & 1)
                for (int b = 0; b < k; ++b)
                    if (!(seen >> b & 1) && A[v[a] * n + v[b]]) {
                        seen |= 1 << b;
                        changed = 1;
                    }
    }
    return seen == (1 << k) - 1;
}

/* Class of the induced subgraph on the k vertices v (or -1 when it is not
 * connected). */
static int induced_class(int k, const int8_t *A, long n, const long *v) {
    int deg[4] = {0, 0, 0, 0}, e = 0;
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if (A[v[a] * n + v[b]]) {
                ++deg[a];
                ++deg[b];
                ++e;
            }
    if (!connected_small(k, A, n, v)) return -1;
    return motif_class(k, deg, e);
}

/* Brute force over all k-subsets i < j < l (< q); O(n^k / k!). */
int oracle_motifs_bruteforce(long n, const int8_t *A, int k, int64_t *out) {
    if (n < 1 || !A || !out || (k != 3 && k != 4)) return -1;
    const int ncls = k == 3 ? 2 : 6;
    int64_t tot[6] = {0, 0, 0, 0, 0, 0};
#pragma omp parallel
    {
        int64_t loc[6] = {0, 0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (long i = 0; i < n; ++i)
            for (long j = i + 1; j < n; ++j)
                for (long l = j + 1; l < n; ++l) {
                    if (k == 3) {
                        const long v[4] = {i, j, l, 0};
                        int c = induced_class(3, A, n, v);
                        if (c >= 0) ++loc[c];
                        continue;
                    }
                    for (long q = l + 1; q < n; ++q) {
                        const long v[4] = {i, j, l, q};
                        int c = induced_class(4, A, n, v);
                        if (c >= 0) ++loc[c];
                    }
                }
#pragma omp critical
        for (int c = 0; c < 6; ++c) tot[c] += loc[c];
    }
    for (int c = 0; c < ncls; ++c) out[c] = tot[c];
    return 0;
}

/* Enumeration of the connected induced k-subgraphs of a sparse graph (CSR),
 * each exactly once, by the extension rule of Wernicke's ESU algorithm:
 * grow a set from its smallest vertex v, adding candidates that are larger
 * than v and adjacent to the set, where a vertex becomes a candidate only
 * through the first set member it is adjacent to (its exclusive
 * neighbourhood). */
typedef struct {
    long n;
    const int64_t *rp;
    const int32_t *col;
    int k;
    int64_t cnt[6];
} esu_t;

static int adj_csr(const esu_t *g, long a, long b) {
    long lo = g->rp[a], hi = g->rp[a + 1];
    while (lo < hi) { /* columns are sorted */
        long mid = (lo + hi) / 2;
        if (g->col[mid] < b) lo = mid + 1;
        else hi = mid;
    }
    return lo < g->rp[a + 1] && g->col[lo] == b;
}

static void esu_extend(esu_t *g, long *sub, int ns, long *ext, int ne, long v) {
    if (ns == g->k) {
        int deg[4] = {0, 0, 0, 0}, e = 0;
        for (int a = 0; a < ns; ++a)
            for (int b = a + 1; b < ns; ++b)
                if (adj_csr(g, sub[a], sub[b])) {
                    ++deg[a];
                    ++deg[b];
                    ++e;
                }
        int c = motif_class(g->k, deg, e);
        if (c >= 0) ++g->cnt[c];
        return;
    }
    /* candidates are consumed one at a time, as the rule prescribes */
    long *cand = malloc(sizeof(long) * (size_t)(ne + 1));
    int nc = ne;
    for (int i = 0; i < ne; ++i) cand[i] = ext[i];
    while (nc > 0) {
        long w = cand[--nc];
        /* new extension: the remaining candidates plus w's exclusive
         * neighbours larger than v */
        long cap = nc + (g->rp[w + 1] - g->rp[w]);
        long *next = malloc(sizeof(long) * (size_t)(cap + 1));
        int nn = 0;
        for (int i = 0; i < nc; ++i) next[nn++] = cand[i];
        for (long p = g->rp[w]; p < g->rp[w + 1]; ++p) {
            long u = g->col[p];
            if (u <= v) continue;
            int bad = 0;
            for (int a = 0; a < ns && !bad; ++a) bad = u == sub[a] || adj_csr(g, u, sub[a]);
            for (int i = 0; i < nc && !bad; ++i) bad = u == cand[i];
            if (!bad) next[nn++] = u;
        }
        sub[ns] = w;
        esu_extend(g, sub, ns + 1, next, nn, v);
        free(next);
    }
    free(cand);
}

int oracle_motifs_esu(long n, const int64_t *rowptr, const int32_t *col, int k, int64_t *out) {
    if (n < 1 || !rowptr || !col || !out || (k != 3 && k != 4)) return -1;
    int64_t tot[6] = {0, 0, 0, 0, 0, 0};
#pragma omp parallel
    {
        esu_t g = {n, rowptr, col, k, {0, 0, 0, 0, 0, 0}};
#pragma omp for schedule(dynamic, 16)
        for (long v = 0; v < n; ++v) {
            long sub[4] = {v, 0, 0, 0};
            long deg = rowptr[v + 1] - rowptr[v];
            long *ext = malloc(sizeof(long) * (size_t)(deg + 1));
            int ne = 0;
            for (long p = rowptr[v]; p < rowptr[v + 1]; ++p)
                if (col[p] > v) ext[ne++] = col[p];
            esu_extend(&g, sub, 1, ext, ne, v);
            free(ext);
        }
#pragma omp critical
        for (int c = 0; c < 6; ++c) tot[c] += g.cnt[c];
    }
    for (int c = 0; c < (k == 3 ? 2 : 6); ++c) out[c] = tot[c];
    return 0;
}
