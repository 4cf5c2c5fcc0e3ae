"""CPU ORACLE -- test infrastructure only.

Plain, slow, obviously correct reference computations for exact higher-order
U-statistics whose kernel is a product of one n x n factor per edge of a small
graph.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the HIP engine and never
imports it; inputs come from the seeded generators or from the caller.

Section references are to Chen, Liu & Zhang, "On computing and the complexity
of computing higher-order U-statistics, exactly" (arXiv 2508.12627).

Pins (each checked in ``tests/test_oracle.py`` against something other than
the function itself): tuple counts of all-ones kernels, subgraph counts of
named graphs, the tournament cyclic-triangle formula, Lemma 2 in exact
integers, the V-to-U decomposition of Appendix A, matrix-product forms of
finest-partition V-statistics, Bell numbers, and the falling-factorial
identity of the Moebius coefficients.  Every function below is pinned.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
from typing import List, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

Edges = Sequence[Tuple[int, int]]


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        c_int, c_long, c_dbl = ctypes.c_int, ctypes.c_long, ctypes.c_double
        pint, pdbl = ctypes.POINTER(c_int), ctypes.POINTER(c_dbl)
        ppdbl = ctypes.POINTER(pdbl)
        pi64 = ctypes.POINTER(ctypes.c_int64)
        ppi64 = ctypes.POINTER(pi64)
        lib.oracle_sum_tuples.argtypes = [c_int, c_int, pint, pint, ppdbl, c_long, c_int,
                                          c_long, c_long, pdbl]
        lib.oracle_sum_tuples_i64.argtypes = [c_int, c_int, pint, pint, ppi64, c_long, c_int,
                                              c_long, c_long, pi64,
                                              ctypes.POINTER(ctypes.c_uint64)]
        lib.oracle_lowrank_dp.argtypes = [c_int, c_int, pint, pint, c_long, c_int, ppdbl, ppdbl,
                                          pdbl]
        lib.oracle_cycle_walks.argtypes = [c_long, pi64, ctypes.POINTER(ctypes.c_int32), pi64]
        lib.oracle_num_threads.restype = c_int
        _LIB = lib
    return _LIB


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


def set_num_threads(t: int) -> None:
    """Threads the C routines use from now on."""
    _lib().oracle_set_num_threads(int(t))


def _edge_arrays(edges: Edges):
    ne = len(edges)
    eu = (ctypes.c_int * ne)(*[int(u) for u, _ in edges])
    ev = (ctypes.c_int * ne)(*[int(v) for _, v in edges])
    return ne, eu, ev


def _num_vertices(edges: Edges) -> int:
    return 1 + max(max(u, v) for u, v in edges)


# --------------------------------------------------------------------------
# Definitions 1 and 2: brute-force U- and V-statistics.
# --------------------------------------------------------------------------

def _sum_tuples(m: int, edges: Edges, mats, distinct: bool, lo=0, hi=None,
                items=None) -> float:
    mats = [np.ascontiguousarray(M, dtype=np.float64) for M in mats]
    n = mats[0].shape[0]
    for M in mats:
        assert M.shape == (n, n)
    inner = n if m >= 2 else 1
    if items is None:
        hi = n if hi is None else hi
        items = (lo * inner, hi * inner)
    lo, hi = items
    ne, eu, ev = _edge_arrays(edges)
    ptrs = (ctypes.POINTER(ctypes.c_double) * ne)(
        *[M.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for M in mats])
    out = ctypes.c_double()
    rc = _lib().oracle_sum_tuples(m, ne, eu, ev, ptrs, n, 1 if distinct else 0, lo, hi,
                                  ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_sum_tuples: bad arguments")
    return float(out.value)


def _sum_tuples_int(m: int, edges: Edges, mats, distinct: bool) -> int:
    mats = [np.ascontiguousarray(M, dtype=np.int64) for M in mats]
    n = mats[0].shape[0]
    ne, eu, ev = _edge_arrays(edges)
    ptrs = (ctypes.POINTER(ctypes.c_int64) * ne)(
        *[M.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) for M in mats])
    hi, lo = ctypes.c_int64(), ctypes.c_uint64()
    rc = _lib().oracle_sum_tuples_i64(m, ne, eu, ev, ptrs, n, 1 if distinct else 0, 0, n,
                                      ctypes.byref(hi), ctypes.byref(lo))
    if rc != 0:
        raise ValueError("oracle_sum_tuples_i64: bad arguments")
    return (int(hi.value) << 64) + int(lo.value)


def ustat_bruteforce(edges: Edges, mats, lo: int = 0, hi=None, items=None) -> float:
    """U(h, X) of Definition 1 (unnormalised sum over ordered distinct
    m-tuples) for the kernel prod_k T_k(x_{u_k}, x_{v_k}), fp64 with
    compensated sums.  ``lo``/``hi`` restrict the first index; ``items``
    restricts the (i_0, i_1) prefixes, numbered i_0 * n + i_1 (a bounded
    sample of the sum, used to time the oracle)."""
    return _sum_tuples(_num_vertices(edges), edges, mats, True, lo, hi, items)


def ustat_bruteforce_int(edges: Edges, mats) -> int:
    """Exact-integer U(h, X) of Definition 1 for integer factors."""
    return _sum_tuples_int(_num_vertices(edges), edges, mats, True)


def quotient_edges(edges: Edges, block_of: Sequence[int]):
    """Algorithm 3 (induced notation): relabel every index by its block."""
    return [(int(block_of[u]), int(block_of[v])) for u, v in edges]


def vstat_bruteforce(edges: Edges, mats, block_of: Sequence[int]) -> float:
    """Restricted V-statistic V_pi (Definition "Restricted V-Statistic"):
    the sum over [n]^{|pi|} of the kernel with indices tied within blocks."""
    J = 1 + max(block_of)
    return _sum_tuples(J, quotient_edges(edges, block_of), mats, False)


def vstat_bruteforce_int(edges: Edges, mats, block_of: Sequence[int]) -> int:
    J = 1 + max(block_of)
    return _sum_tuples_int(J, quotient_edges(edges, block_of), mats, False)


# --------------------------------------------------------------------------
# Set partitions and the Moebius coefficients of Lemma 2.
# --------------------------------------------------------------------------

def partitions(m: int) -> List[List[List[int]]]:
    """All set partitions of {0..m-1}, by inserting element i into each
    existing block or into a new block (recursive block insertion)."""
    out: List[List[List[int]]] = []

    def rec(i, blocks):
        if i == m:
            out.append([list(b) for b in blocks])
            return
        for b in blocks:
            b.append(i)
            rec(i + 1, blocks)
            b.pop()
        blocks.append([i])
        rec(i + 1, blocks)
        blocks.pop()

    rec(0, [])
    return out


def block_labels(blocks: List[List[int]], m: int) -> List[int]:
    """Label blocks 0..J-1 in order of their smallest element."""
    lab = [0] * m
    for j, b in enumerate(sorted(blocks, key=min)):
        for i in b:
            lab[i] = j
    return lab


def mobius_mu(blocks: List[List[int]]) -> int:
    """mu_pi = (-1)^(m - |pi|) prod_{C in pi} (|C| - 1)!   (Lemma 2)."""
    m = sum(len(b) for b in blocks)
    s = -1 if (m - len(blocks)) % 2 else 1
    p = 1
    for b in blocks:
        p *= math.factorial(len(b) - 1)
    return s * p


def ustat_mobius_bruteforce_int(edges: Edges, mats) -> int:
    """Lemma 2 evaluated literally: sum over all partitions of mu_pi times
    the brute-force restricted V-statistic.  Exact integers."""
    m = _num_vertices(edges)
    tot = 0
    for blocks in partitions(m):
        tot += mobius_mu(blocks) * vstat_bruteforce_int(edges, mats, block_labels(blocks, m))
    return tot


# --------------------------------------------------------------------------
# Einsum form of a restricted V-statistic (Definition "Einsum Operation" with
# the induced notation of Algorithm 3), via numpy.einsum in fp64.
# --------------------------------------------------------------------------

def vstat_einsum(edges: Edges, mats, block_of: Sequence[int]) -> float:
    letters = "abcdefghijklmnopqrstuvwxyz"
    qe = quotient_edges(edges, block_of)
    subs = ",".join(letters[a] + letters[b] for a, b in qe)
    ops = [np.asarray(M, dtype=np.float64) for M in mats]
    return float(np.einsum(subs + "->", *ops, optimize="greedy"))


def ustat_and_scale_einsum(edges: Edges, mats):
    """Lemma 2 with einsum V-statistics: returns (U, S, {labels: V_pi}) where
    S = sum_pi |mu_pi V_pi| is the magnitude scale of the signed sum."""
    m = _num_vertices(edges)
    U, S, vs = 0.0, 0.0, {}
    for blocks in partitions(m):
        lab = block_labels(blocks, m)
        v = vstat_einsum(edges, mats, lab)
        mu = mobius_mu(blocks)
        vs[tuple(lab)] = v
        U += mu * v
        S += abs(mu * v)
    return U, S, vs


# --------------------------------------------------------------------------
# Low-rank factors at any n (independent of the decomposition).
# --------------------------------------------------------------------------

def ustat_lowrank(edges: Edges, F, G) -> float:
    """Definition 1 for T_k = F_k G_k^T (F_k, G_k of shape n x r), by a
    subset dynamic programme over the samples."""
    m = _num_vertices(edges)
    F = [np.ascontiguousarray(f, dtype=np.float64) for f in F]
    G = [np.ascontiguousarray(g, dtype=np.float64) for g in G]
    n, r = F[0].shape
    ne, eu, ev = _edge_arrays(edges)
    PD = ctypes.POINTER(ctypes.c_double)
    pf = (PD * ne)(*[f.ctypes.data_as(PD) for f in F])
    pg = (PD * ne)(*[g.ctypes.data_as(PD) for g in G])
    out = ctypes.c_double()
    rc = _lib().oracle_lowrank_dp(m, ne, eu, ev, n, r, pf, pg, ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_lowrank_dp: bad arguments")
    return float(out.value)


# --------------------------------------------------------------------------
# RBF factor (the kernel of the cycle workloads), fp64 by direct differences.
# --------------------------------------------------------------------------

def rbf_matrix(X, divisor: float, block: int = 512) -> np.ndarray:
    """K_ij = exp(-||x_i - x_j||^2 / divisor) in fp64, from direct
    differences (so K_ii = 1 exactly)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    K = np.empty((n, n), dtype=np.float64)
    for s in range(0, n, block):
        D = X[s:s + block, None, :] - X[None, :, :]
        K[s:s + block] = np.exp(-np.einsum("ijk,ijk->ij", D, D) / divisor)
    return K


# --------------------------------------------------------------------------
# Closed forms.
# --------------------------------------------------------------------------

def triangle_closed_form(K) -> float:
    """Triangle kernel with one symmetric factor of unit diagonal:
    U = tr K^3 - 3 sum_ij K_ij^2 + 2 n."""
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    K2 = K @ K
    return float(np.sum(K2 * K) - 3.0 * np.sum(K * K) + 2.0 * n)


def cycle4_closed_form(K) -> float:
    """4-cycle kernel with one symmetric factor K; with Kt = K - diag(K):
    U = tr Kt^4 - 2 sum_i (sum_j Kt_ij^2)^2 + sum_ij Kt_ij^4."""
    Kt = np.array(K, dtype=np.float64, copy=True)
    np.fill_diagonal(Kt, 0.0)
    K2 = Kt @ Kt
    r = np.sum(Kt * Kt, axis=1)
    return float(np.sum(K2 * K2) - 2.0 * np.sum(r * r) + np.sum(Kt ** 4))


def _csr(adj):
    A = np.asarray(adj)
    n = A.shape[0]
    rows, cols = np.nonzero(A)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int64)
    return n, rowptr, cols.astype(np.int32)


def cycle_walks(adj) -> dict:
    """Closed-walk counts of a simple 0/1 graph (exact int64)."""
    n, rowptr, col = _csr(adj)
    out = (ctypes.c_int64 * 6)()
    rc = _lib().oracle_cycle_walks(n, rowptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), out)
    if rc != 0:
        raise ValueError("oracle_cycle_walks failed")
    keys = ["trA3", "trA5", "deg_A3", "trA4", "deg2", "two_e"]
    return {k: int(out[i]) for i, k in enumerate(keys)}


def count_5cycles(adj) -> int:
    """Number of 5-cycles of a simple graph by the trace formula
    10 C5 = tr A^5 - 5 tr A^3 - 5 sum_i (deg_i - 2) (A^3)_ii."""
    w = cycle_walks(adj)
    deg_minus2 = w["deg_A3"] - 2 * w["trA3"]
    ten = w["trA5"] - 5 * w["trA3"] - 5 * deg_minus2
    assert ten % 10 == 0
    return ten // 10


def count_4cycles(adj) -> int:
    """8 C4 = tr A^4 - 2 sum_i deg_i^2 + 2 |E|."""
    w = cycle_walks(adj)
    eight = w["trA4"] - 2 * w["deg2"] + w["two_e"]
    assert eight % 8 == 0
    return eight // 8


def count_triangles(adj) -> int:
    w = cycle_walks(adj)
    assert w["trA3"] % 6 == 0
    return w["trA3"] // 6


def tournament_cyclic_triangles(A) -> int:
    """Cyclic (3-cycle) triangles of a tournament: C(n,3) - sum_v C(out_v, 2)."""
    A = np.asarray(A)
    n = A.shape[0]
    out = A.sum(axis=1).astype(np.int64)
    return math.comb(n, 3) - int(sum(math.comb(int(o), 2) for o in out))


def tuple_pattern_sums(edges: Edges, mats) -> dict:
    """Pure-Python enumeration of [n]^m (tiny n only): the kernel summed over
    tuples grouped by their exact equality pattern, i.e. the restricted
    U-statistics U_rho of Appendix A.  Keys are block-label tuples."""
    m = _num_vertices(edges)
    mats = [np.asarray(M) for M in mats]
    n = mats[0].shape[0]
    out: dict = {}
    for tup in itertools.product(range(n), repeat=m):
        first = {}
        lab = []
        for x in tup:
            if x not in first:
                first[x] = len(first)
            lab.append(first[x])
        val = 1
        for k, (u, v) in enumerate(edges):
            val = val * mats[k][tup[u], tup[v]]
        out[tuple(lab)] = out.get(tuple(lab), 0) + val
    return out


# --------------------------------------------------------------------------
# Induced motif counts (the motif application), independent of the
# U-statistic decomposition: brute force over vertex subsets, and an
# enumeration of connected induced subgraphs for sparse graphs.
# --------------------------------------------------------------------------

MOTIFS3 = ["v-shape", "triangle"]
MOTIFS4 = ["3-star", "path", "tailed-triangle", "square", "diamond", "k4"]


def motifs_bruteforce(A, k: int) -> list:
    """Induced counts of the connected k-vertex motifs (k = 3: V-shape,
    triangle; k = 4: 3-star, path, tailed triangle, square, diamond, K4)
    by testing every k-subset of vertices."""
    A = np.ascontiguousarray(np.asarray(A) != 0, dtype=np.int8)
    n = A.shape[0]
    out = (ctypes.c_int64 * 6)()
    lib = _lib()
    lib.oracle_motifs_bruteforce.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int64)]
    rc = lib.oracle_motifs_bruteforce(n, A.ctypes.data, int(k), out)
    if rc != 0:
        raise ValueError("oracle_motifs_bruteforce: bad arguments")
    return [int(x) for x in list(out)[: (2 if k == 3 else 6)]]


def motifs_esu(A, k: int) -> list:
    """The same counts by enumerating each connected induced k-subgraph
    once (suited to large sparse graphs)."""
    n, rowptr, col = _csr(A)
    out = (ctypes.c_int64 * 6)()
    lib = _lib()
    lib.oracle_motifs_esu.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int64)]
    rc = lib.oracle_motifs_esu(n, rowptr.ctypes.data, col.ctypes.data, int(k), out)
    if rc != 0:
        raise ValueError("oracle_motifs_esu: bad arguments")
    return [int(x) for x in list(out)[: (2 if k == 3 else 6)]]


def motifs3_closed_form(A) -> list:
    """Induced 3-vertex motif counts from degrees and the trace formula:
    triangles T = tr(A^3) / 6, and V-shapes = sum_i C(deg_i, 2) - 3 T (every
    path of length two is an induced V-shape unless its ends are adjacent,
    which happens three times per triangle)."""
    A = np.asarray(A)
    deg = np.count_nonzero(A, axis=1).astype(np.int64)
    T = count_triangles(A)
    return [int(np.sum(deg * (deg - 1) // 2)) - 3 * T, T]
