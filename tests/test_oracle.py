"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Every oracle function is checked here against something other than itself:
closed-form tuple counts, subgraph counts of named graphs, a textbook
tournament formula, Lemma 2 in exact integers, the V-to-U decomposition of
Appendix A, matrix-product forms of finest-partition V-statistics, and the
values printed in the paper's tables (``tests/golden/paper_tables.json``).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2508_12627_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))

GRAPHS = {
    "triangle": W.TRIANGLE,
    "path4": W.PATH4,
    "cycle4": W.CYCLE4,
    "cycle5": W.CYCLE5,
    "c5chord": W.CYCLE5_CHORD,
    "k4": [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
    "star": [(0, 1), (0, 2), (0, 3)],
}


def falling(n, m):
    return math.perm(n, m)


def petersen():
    A = np.zeros((10, 10), dtype=np.int64)
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    for u, v in outer + spokes + inner:
        A[u, v] = A[v, u] = 1
    return A


def complete(n):
    A = np.ones((n, n), dtype=np.int64)
    np.fill_diagonal(A, 0)
    return A


def cycle_graph(k):
    A = np.zeros((k, k), dtype=np.int64)
    for i in range(k):
        A[i, (i + 1) % k] = A[(i + 1) % k, i] = 1
    return A


# ---------------------------------------------------------------- Definition 1
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_all_ones_counts_ordered_distinct_tuples(name):
    """With h = 1 the U-statistic counts ordered distinct m-tuples: n!/(n-m)!;
    the V-statistic counts all of [n]^m."""
    edges = GRAPHS[name]
    m = 1 + max(max(e) for e in edges)
    n = 7
    ones = [np.ones((n, n))] * len(edges)
    assert oracle.ustat_bruteforce(edges, ones) == falling(n, m)
    assert oracle.ustat_bruteforce_int(edges, [np.ones((n, n), np.int64)] * len(edges)) == falling(n, m)
    assert oracle.vstat_bruteforce(edges, ones, list(range(m))) == n ** m


def test_named_graph_subgraph_counts():
    """U of a cycle kernel on a 0/1 adjacency is |Aut(C_k)| = 2k times the
    number of k-cycles (motif counting, Section 4 / Appendix on motifs)."""
    P = petersen()
    # Petersen graph: girth 5, twelve 5-cycles, no triangles or 4-cycles.
    assert oracle.ustat_bruteforce_int(W.TRIANGLE, [P] * 3) == 0
    assert oracle.ustat_bruteforce_int(W.CYCLE4, [P] * 4) == 0
    assert oracle.ustat_bruteforce_int(W.CYCLE5, [P] * 5) == 10 * 12
    K5 = complete(5)
    assert oracle.ustat_bruteforce_int(W.TRIANGLE, [K5] * 3) == 6 * math.comb(5, 3)
    # K_{3,3} has nine 4-cycles.
    B = np.zeros((6, 6), dtype=np.int64)
    B[:3, 3:] = 1
    B[3:, :3] = 1
    assert oracle.ustat_bruteforce_int(W.CYCLE4, [B] * 4) == 8 * 9
    # K_n has n!/((n-k)! 2k) k-cycles.
    for n in (5, 6, 7):
        Kn = complete(n)
        assert oracle.ustat_bruteforce_int(W.CYCLE5, [Kn] * 5) == falling(n, 5)


def test_orientation_via_tournament_formula():
    """Directed 3-cycles: U = 3 * (C(n,3) - sum_v C(out_v, 2)); a transposed
    factor would count transitive triangles instead."""
    for seed in range(3):
        A = W.random_tournament(9, seed)
        cyc = oracle.tournament_cyclic_triangles(A)
        assert oracle.ustat_bruteforce_int(W.TRIANGLE, [A] * 3) == 3 * cyc
        assert oracle.ustat_bruteforce(W.TRIANGLE, [A.astype(float)] * 3) == 3 * cyc
        # Reorienting two factors, A(i0,i1) A(i2,i1) A(i2,i0), matches each
        # transitive triple once (i2 source, i0 middle, i1 sink) and no
        # cyclic triple.
        trans = math.comb(9, 3) - cyc
        assert oracle.ustat_bruteforce_int([(0, 1), (2, 1), (2, 0)], [A] * 3) == trans


# ---------------------------------------------------------------- Lemma 2
@pytest.mark.parametrize("name", ["triangle", "path4", "cycle4", "c5chord", "star"])
def test_lemma2_exact_integers(name):
    """U = sum_pi mu_pi V_pi, exactly, for independent asymmetric integer
    factors (one per edge)."""
    edges = GRAPHS[name]
    n = 6
    mats = W.random_int_matrices(len(edges), n, seed=11, lo=-3, hi=4)
    assert oracle.ustat_bruteforce_int(edges, mats) == oracle.ustat_mobius_bruteforce_int(edges, mats)


def test_v_to_u_decomposition_appendix():
    """Appendix A: V_pi = sum_{rho >= pi} U_rho, where U_rho sums over tuples
    whose equality pattern is exactly rho.  Checked for the finest pi (V is
    the sum over every pattern) and against the brute-force U (the finest
    pattern)."""
    edges = W.PATH4
    n = 4
    mats = W.random_int_matrices(3, n, seed=5, lo=-2, hi=3)
    pats = oracle.tuple_pattern_sums(edges, mats)
    assert sum(pats.values()) == oracle.vstat_bruteforce_int(edges, mats, [0, 1, 2, 3])
    assert pats[(0, 1, 2, 3)] == oracle.ustat_bruteforce_int(edges, mats)
    # V for pi = {1,3}{2}{4} collects every pattern that ties positions 1 and 3.
    tied = sum(v for k, v in pats.items() if k[0] == k[2])
    assert tied == oracle.vstat_bruteforce_int(edges, mats, [0, 1, 0, 2])


def test_finest_vstat_matches_matrix_products():
    """Finest-partition V-statistics of a path and of a cycle are
    1^T T1 T2 T3 1 and tr(T1 T2 T3 T4) (library matmul)."""
    n = 9
    T = W.random_matrices(4, n, seed=3)
    v_path = oracle.vstat_bruteforce(W.PATH4, T[:3], [0, 1, 2, 3])
    ref = float(np.ones(n) @ T[0] @ T[1] @ T[2] @ np.ones(n))
    assert v_path == pytest.approx(ref, rel=1e-12, abs=1e-12)
    v_cyc = oracle.vstat_bruteforce(W.CYCLE4, T, [0, 1, 2, 3])
    assert v_cyc == pytest.approx(float(np.trace(T[0] @ T[1] @ T[2] @ T[3])), rel=1e-12, abs=1e-12)
    # A self-loop block reads the diagonal: pi = {1,2}{3}{4} on the path.
    v = oracle.vstat_bruteforce(W.PATH4, T[:3], [0, 0, 1, 2])
    ref = float(np.diag(T[0]) @ T[1] @ T[2] @ np.ones(n))
    assert v == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_partitions_bell_numbers():
    """Number of partitions = Bell(m) (Table 'tab:HOIF')."""
    g = GOLDEN["bell_terms"]
    for m, b in zip(g["m"], g["values"]):
        if m <= 8:
            assert len(oracle.partitions(m)) == b


def test_mu_falling_factorial_identity():
    """With h = 1, Lemma 2 reads n!/(n-m)! = sum_pi mu_pi n^|pi| for every n:
    a closed-form pin of the Moebius coefficients (signs and factorials)."""
    for m in range(1, 8):
        parts = oracle.partitions(m)
        for n in range(m, m + 5):
            assert sum(oracle.mobius_mu(p) * n ** len(p) for p in parts) == falling(n, m)


def test_mu_values_of_worked_example():
    g = GOLDEN["path4_mu_signs"]
    for blocks, mu in zip(g["partitions"], g["mu"]):
        assert oracle.mobius_mu([[i - 1 for i in b] for b in blocks]) == mu


# ---------------------------------------------------------------- einsum form
@pytest.mark.parametrize("name", ["triangle", "cycle4", "c5chord"])
def test_vstat_einsum_equals_bruteforce(name):
    edges = GRAPHS[name]
    m = 1 + max(max(e) for e in edges)
    n = 5
    mats = W.random_matrices(len(edges), n, seed=21)
    for blocks in oracle.partitions(m):
        lab = oracle.block_labels(blocks, m)
        assert oracle.vstat_einsum(edges, mats, lab) == pytest.approx(
            oracle.vstat_bruteforce(edges, mats, lab), rel=1e-11, abs=1e-11)
    U, S, _ = oracle.ustat_and_scale_einsum(edges, mats)
    assert U == pytest.approx(oracle.ustat_bruteforce(edges, mats), abs=1e-10 * S)


# ---------------------------------------------------------------- low rank DP
def test_lowrank_dp_special_cases():
    n = 8
    # all-ones rank 1: n!/(n-m)!
    for name in ("triangle", "cycle5", "c5chord", "star"):
        edges = GRAPHS[name]
        m = 1 + max(max(e) for e in edges)
        F = [np.ones((n, 1))] * len(edges)
        assert oracle.ustat_lowrank(edges, F, F) == pytest.approx(falling(n, m), rel=1e-14)
    # one edge: sum_{i != j} f_i g_j = (sum f)(sum g) - sum f_i g_i
    rng = np.random.default_rng(0)
    f, g = rng.random((n, 1)), rng.random((n, 1))
    ref = f.sum() * g.sum() - float(f[:, 0] @ g[:, 0])
    assert oracle.ustat_lowrank([(0, 1)], [f], [g]) == pytest.approx(ref, rel=1e-14)


@pytest.mark.parametrize("name", ["triangle", "cycle4", "c5chord"])
def test_lowrank_dp_equals_bruteforce(name):
    edges = GRAPHS[name]
    n = 9
    fg = W.lowrank_factors(len(edges), n, 2, seed=8, lo=-1.0, hi=1.0)
    mats = [F @ G.T for F, G in fg]
    bf = oracle.ustat_bruteforce(edges, mats)
    dp = oracle.ustat_lowrank(edges, [F for F, _ in fg], [G for _, G in fg])
    scale = oracle.ustat_and_scale_einsum(edges, mats)[1]
    assert dp == pytest.approx(bf, abs=1e-12 * scale)


# ---------------------------------------------------------------- closed forms
def test_rbf_matrix_definition():
    d = 4
    X = np.zeros((3, d))
    X[1, 0] = math.sqrt(2 * d)          # squared distance 2d -> exp(-1)
    X[2, :] = 1.0                       # squared distance d from X[0]
    K = oracle.rbf_matrix(X, 2.0 * d)
    assert np.all(np.diag(K) == 1.0)
    assert K[0, 1] == pytest.approx(math.exp(-1.0), rel=1e-15)
    assert K[0, 2] == pytest.approx(math.exp(-0.5), rel=1e-15)
    assert np.array_equal(K, K.T)


def test_triangle_and_cycle4_closed_forms():
    X = W.gaussian_samples(10, 3, seed=4)
    K = oracle.rbf_matrix(X, 6.0)
    assert oracle.triangle_closed_form(K) == pytest.approx(
        oracle.ustat_bruteforce(W.TRIANGLE, [K] * 3), rel=1e-12)
    assert oracle.cycle4_closed_form(K) == pytest.approx(
        oracle.ustat_bruteforce(W.CYCLE4, [K] * 4), rel=1e-12)


def test_cycle_count_formulas():
    assert oracle.count_5cycles(petersen()) == 12
    assert oracle.count_5cycles(cycle_graph(5)) == 1
    assert oracle.count_5cycles(complete(7)) == falling(7, 5) // 10
    assert oracle.count_4cycles(complete(6)) == falling(6, 4) // 8
    assert oracle.count_triangles(complete(6)) == math.comb(6, 3)
    for seed in range(4):
        A = W.erdos_renyi(11, 0.5, seed).astype(np.int64)
        assert 10 * oracle.count_5cycles(A) == oracle.ustat_bruteforce_int(W.CYCLE5, [A] * 5)
        assert 8 * oracle.count_4cycles(A) == oracle.ustat_bruteforce_int(W.CYCLE4, [A] * 4)
        assert 6 * oracle.count_triangles(A) == oracle.ustat_bruteforce_int(W.TRIANGLE, [A] * 3)


def test_bounded_sample_partitions_the_sum():
    """Sums over disjoint ranges of the first index add up to the full sum."""
    n = 12
    mats = W.random_matrices(4, n, seed=9)
    full = oracle.ustat_bruteforce(W.CYCLE4, mats)
    parts = sum(oracle.ustat_bruteforce(W.CYCLE4, mats, lo, lo + 3) for lo in range(0, n, 3))
    assert parts == pytest.approx(full, rel=1e-12, abs=1e-12)


def test_bounded_sample_by_prefix_items():
    """Prefix-item ranges (i_0 * n + i_1) also partition the sum."""
    n = 10
    mats = W.random_matrices(3, n, seed=19)
    full = oracle.ustat_bruteforce(W.TRIANGLE, mats)
    cuts = [0, 7, 33, 34, 90, 100]
    parts = sum(oracle.ustat_bruteforce(W.TRIANGLE, mats, items=(a, b))
                for a, b in zip(cuts[:-1], cuts[1:]))
    assert parts == pytest.approx(full, rel=1e-12, abs=1e-12)
