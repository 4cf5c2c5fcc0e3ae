"""Seeded synthetic input generators shared by the tests, the benchmark and
the oracle's callers.

This module holds no arithmetic of the method: it only draws samples, graphs
and random matrices from numpy's PCG64 generator.  Factor matrices of the
workloads (RBF kernels, adjacency casts) are built separately by the engine
on the GPU and by the oracle on the CPU.
"""
from __future__ import annotations

import numpy as np

# Kernel graphs used by the workloads (0-based vertex labels, ordered edges).
TRIANGLE = [(0, 1), (1, 2), (2, 0)]
CYCLE4 = [(0, 1), (1, 2), (2, 3), (3, 0)]
CYCLE5 = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]
CYCLE5_CHORD = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (0, 2)]
PATH4 = [(0, 1), (1, 2), (2, 3)]


def path(m: int):
    return [(i, i + 1) for i in range(m - 1)]


def gaussian_samples(n: int, d: int, seed: int) -> np.ndarray:
    """n iid N(0, I_d) samples, fp64, row-major n x d."""
    return np.random.default_rng(seed).standard_normal((n, d))


def student_t_samples(n: int, d: int, seed: int, dof: float = 5.0) -> np.ndarray:
    """n samples whose coordinates are iid standard Student-t(dof)."""
    return np.random.default_rng(seed).standard_t(dof, size=(n, d))


def erdos_renyi(n: int, p: float, seed: int) -> np.ndarray:
    """Symmetric 0/1 int8 adjacency of G(n, p): Bernoulli(p) upper triangle
    mirrored, zero diagonal."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=np.int8)
    for i in range(n - 1):
        row = (rng.random(n - 1 - i) < p).astype(np.int8)
        A[i, i + 1:] = row
    A = A | A.T
    return A


def ragged_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """count sizes drawn uniformly from {lo..hi}."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=count)


def random_kernel_graphs(count: int, m: int, e_lo: int, e_hi: int, seed: int):
    """Random simple graphs on m vertices with e ~ U{e_lo..e_hi} edges drawn
    uniformly without replacement from all vertex pairs; draws with an
    isolated vertex are rejected (every index must appear in some factor)."""
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(m) for j in range(i + 1, m)]
    out = []
    while len(out) < count:
        e = int(rng.integers(e_lo, e_hi + 1))
        sel = rng.choice(len(pairs), size=e, replace=False)
        edges = [pairs[s] for s in sorted(sel)]
        used = set(v for ed in edges for v in ed)
        if len(used) < m:
            continue
        out.append(edges)
    return out


def random_matrices(count: int, n: int, seed: int, lo=-1.0, hi=1.0) -> list:
    """count independent asymmetric fp64 n x n matrices, entries U[lo, hi)."""
    rng = np.random.default_rng(seed)
    return [rng.uniform(lo, hi, size=(n, n)) for _ in range(count)]


def random_int_matrices(count: int, n: int, seed: int, lo: int, hi: int) -> list:
    """count independent asymmetric integer n x n matrices, entries in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return [rng.integers(lo, hi + 1, size=(n, n)).astype(np.int64) for _ in range(count)]


def random_tournament(n: int, seed: int) -> np.ndarray:
    """0/1 adjacency of a random tournament: exactly one of (i,j), (j,i)."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < 0.5:
                A[i, j] = 1
            else:
                A[j, i] = 1
    return A


def lowrank_factors(count: int, n: int, r: int, seed: int, lo=0.1, hi=1.0):
    """count pairs (F, G) of n x r fp64 matrices with entries U[lo, hi)."""
    rng = np.random.default_rng(seed)
    return [(rng.uniform(lo, hi, size=(n, r)), rng.uniform(lo, hi, size=(n, r)))
            for _ in range(count)]


def hoif_chain(order: int):
    """Kernel graph of the order-j chain (Section 4.1): factors g on edges
    (0,1) .. (j-3, j-2), f on the last edge (j-2, j-1)."""
    return path(order)


def hoif_panels(n: int, k: int, seed: int, d: int = 4):
    """Panels of the two factors of the influence-function chains of Section
    4.1, g(X1, X2) = A1 phi(Z1)^T A2 phi(Z2) and f(X1, X2) = A1 phi(Z1)^T
    phi(Z2) Y2, i.e. g = P P^T and f = P Q^T with P = A phi(Z), Q = Y phi(Z)
    (n x k each, fp64).  The paper leaves the data-generating process open;
    this one draws Z iid uniform on [0, 1]^d, treatment A ~ Bernoulli(expit(
    Z_1 + Z_2 - 1)), outcome Y = A + sum(Z) + N(0, 1), and a cosine
    dictionary that is orthonormal under the uniform law, phi_l(z) =
    sqrt(2) cos(pi (1 + l // d) z_{l mod d}) for l < k.  Building the panels
    is the kernel evaluation step, not part of the method."""
    rng = np.random.default_rng(seed)
    Z = rng.uniform(0.0, 1.0, size=(n, d))
    A = (rng.uniform(size=n) < 1.0 / (1.0 + np.exp(-(Z[:, 0] + Z[:, 1 % d] - 1.0)))).astype(np.float64)
    Y = A + Z.sum(axis=1) + rng.standard_normal(n)
    lidx = np.arange(k)
    phi = np.sqrt(2.0) * np.cos(np.pi * (1 + lidx // d)[None, :] * Z[:, lidx % d])
    P = A[:, None] * phi
    Q = Y[:, None] * phi
    return np.ascontiguousarray(P), np.ascontiguousarray(Q)


def hoif_factor_panels(order: int, P, Q):
    """(F, G) panel lists of the order-j chain: g = P P^T on the first j-2
    edges, f = P Q^T on the last."""
    e = order - 1
    return [P] * e, [P] * (e - 1) + [Q]
