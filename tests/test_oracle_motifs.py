"""Pins of the oracle's induced motif counts (the motif application):
named graphs with counts known in closed form, and the two independent
routines (brute force over vertex subsets; enumeration of connected
induced subgraphs) agreeing on random graphs."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2508_12627_amd import workloads as W


def adj(n, edges):
    A = np.zeros((n, n), dtype=np.int8)
    for a, b in edges:
        A[a, b] = A[b, a] = 1
    return A


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return adj(10, outer + spokes + inner)


@pytest.mark.parametrize("fn", [oracle.motifs_bruteforce, oracle.motifs_esu])
def test_complete_graph(fn):
    n = 9
    K = np.ones((n, n), dtype=np.int8) - np.eye(n, dtype=np.int8)
    assert fn(K, 3) == [0, math.comb(n, 3)]
    assert fn(K, 4) == [0, 0, 0, 0, 0, math.comb(n, 4)]


@pytest.mark.parametrize("fn", [oracle.motifs_bruteforce, oracle.motifs_esu])
def test_star_and_cycle(fn):
    n = 11
    S = adj(n, [(0, i) for i in range(1, n)])
    assert fn(S, 3) == [math.comb(n - 1, 2), 0]
    assert fn(S, 4) == [math.comb(n - 1, 3), 0, 0, 0, 0, 0]
    C = adj(n, [(i, (i + 1) % n) for i in range(n)])
    # every vertex centres one V-shape; every 3-edge stretch is an induced path
    assert fn(C, 3) == [n, 0]
    assert fn(C, 4) == [0, n, 0, 0, 0, 0]
    C4 = adj(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    assert fn(C4, 4) == [0, 0, 0, 1, 0, 0]


@pytest.mark.parametrize("fn", [oracle.motifs_bruteforce, oracle.motifs_esu])
def test_petersen(fn):
    """Girth 5 and 3-regular: 30 V-shapes, no triangles; each vertex with its
    three (pairwise non-adjacent) neighbours is an induced 3-star; each of
    the 15 edges extends to 2 x 2 induced paths on 4 vertices."""
    P = petersen()
    assert fn(P, 3) == [30, 0]
    assert fn(P, 4) == [10, 60, 0, 0, 0, 0]


def test_small_named_motifs():
    """Each 4-vertex motif on exactly 4 vertices is counted once, in its
    own class."""
    shapes = {0: [(0, 1), (0, 2), (0, 3)], 1: [(0, 1), (1, 2), (2, 3)],
              2: [(0, 1), (0, 2), (1, 2), (2, 3)], 3: [(0, 1), (1, 2), (2, 3), (3, 0)],
              4: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3)], 5: list(itertools.combinations(range(4), 2))}
    for c, e in shapes.items():
        want = [0] * 6
        want[c] = 1
        assert oracle.motifs_bruteforce(adj(4, e), 4) == want
        assert oracle.motifs_esu(adj(4, e), 4) == want


@pytest.mark.parametrize("n,p,seed", [(40, 0.3, 1), (90, 0.08, 2), (150, 0.03, 3)])
def test_bruteforce_and_enumeration_agree(n, p, seed):
    A = W.erdos_renyi(n, p, seed=seed)
    for k in (3, 4):
        assert oracle.motifs_bruteforce(A, k) == oracle.motifs_esu(A, k)


def test_triangles_match_trace_formula():
    A = W.erdos_renyi(200, 0.1, seed=5)
    assert oracle.motifs_bruteforce(A, 3)[1] == oracle.count_triangles(A.astype(np.int64))


@pytest.mark.parametrize("n,p,seed", [(60, 0.2, 7), (150, 0.05, 8)])
def test_closed_form_3_motifs(n, p, seed):
    A = W.erdos_renyi(n, p, seed=seed)
    assert oracle.motifs3_closed_form(A) == oracle.motifs_bruteforce(A, 3)
