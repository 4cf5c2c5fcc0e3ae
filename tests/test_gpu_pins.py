"""GPU parity at full size and at the edges of the input space, through the
C ABI, against the CPU oracle:

- programs conditioned on a vertex (quotients of treewidth 3) at n = 2048
  against the oracle's subset DP on rank-2 factors, with and without a
  workspace limit that forces slice chunks;
- row-mode reductions over several column segments (n = 1500, 16-byte
  loads; n = 1027, element loads and a ragged tail) against the same DP;
- m = 2, n = m, and kernel graphs with parallel edges (same and opposite
  orientation) against brute force;
- the per-result error estimate (err_est) against the measured error.

Floating-point results are held to |U - U_ref| <= tol * S (tol 1e-12 for
fp64, 1e-6 for fp32 and split-bf16; S the engine's sum_pi |mu_pi V_pi|,
pinned against the oracle's S elsewhere); exact results bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2508_12627_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "bf16x3": 1e-6}
K4 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def U():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_12627_amd import ustat
    ustat.load_library()
    return ustat


def dev(a, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def nverts(edges):
    return 1 + max(max(e) for e in edges)


def as_device_sees(mats, prec):
    """The factors as the engine receives them: fp32 for the fp32 and
    split-bf16 paths (the oracle then measures the engine's own error)."""
    if prec in ("f32", "bf16x3"):
        return [np.asarray(M, dtype=np.float32).astype(np.float64) for M in mats]
    return mats


def check(tag, r, ref, S, prec):
    err = abs(r.value - ref) / S
    say(f"ERRSTAT {tag} {prec} err={err:.3e} est={r.err_est:.3e}")
    assert err <= TOL[prec], (err, TOL[prec])
    assert err <= r.err_est, (err, r.err_est)


def m3_graphs(count):
    """The first `count` random m = 6 workload graphs (seed 5) whose worst
    quotient has treewidth 3."""
    from paper_2508_12627_amd import ustat
    out = []
    for g in W.random_kernel_graphs(16, 6, 6, 10, seed=5):
        if ustat.Plan(6, g).info()["M"] == 3:
            out.append(g)
        if len(out) == count:
            break
    return out


# ------------------------------------------------------------------ conditioning at size
@pytest.mark.parametrize("limit", [False, True])
def test_conditioned_k4_full_size(U, limit):
    """K4 (its finest quotient has treewidth 3) at n = 2048 in fp64, rank-2
    positive symmetric factors, against the subset DP."""
    n = 2048
    (F, _), = W.lowrank_factors(1, n, 2, seed=61, lo=0.1, hi=1.0)
    K = F @ F.T
    ref = oracle.ustat_lowrank(K4, [F] * 6, [F] * 6)
    kw = {}
    if limit:
        ws1 = U.Plan(4, K4, precision="f64", symmetric=True).workspace([n], shared_factor=False)
        kw["workspace_limit"] = 40 * ws1  # a few dozen slices per chunk, ragged last chunk
    P = U.Plan(4, K4, precision="f64", symmetric=True, **kw)
    assert P.info()["M"] == 3
    say(f"conditioned K4 n={n} f64 limit={limit}")
    r = P.eval([dev(K, P.factor_dtype)] * 6)
    check(f"cond-k4-{limit}", r, ref, r.err_scale, "f64")


@pytest.mark.parametrize("gi", [0, 1])
def test_conditioned_workload_graphs_full_size(U, gi):
    """Two treewidth-3 workload graphs (m = 6, 203 partitions) at n = 2048 in
    split-bf16 on rank-2 positive factors against the subset DP; the second
    under a workspace limit that forces slice chunks."""
    n = 2048
    g = m3_graphs(2)[gi]
    (F, G), = W.lowrank_factors(1, n, 2, seed=62 + gi, lo=0.1, hi=1.0)
    K = F @ G.T
    ref = oracle.ustat_lowrank(g, [F] * len(g), [G] * len(g))
    kw = {}
    if gi == 1:
        ws1 = U.Plan(6, g, precision="bf16x3").workspace([n], shared_factor=False)
        kw["workspace_limit"] = 24 * ws1
    P = U.Plan(6, g, precision="bf16x3", **kw)
    say(f"conditioned m=6 graph {g} n={n} bf16x3 {kw}")
    r = P.eval([dev(K, P.factor_dtype)] * len(g))
    check(f"cond-m6-{gi}", r, ref, r.err_scale, "bf16x3")


# ------------------------------------------------------------------ row reductions at size
@pytest.mark.parametrize("name,edges", [("cycle4", W.CYCLE4), ("c5chord", W.CYCLE5_CHORD),
                                        ("bowtie", [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 2)])])
def test_row_reductions_against_oracle(U, name, edges):
    """Symmetric rank-2 factors at n = 1500 and 1027: the row-mode reduction
    plan in fp64 against the subset DP."""
    m = nverts(edges)
    for n in (1500, 1027):
        (F, _), = W.lowrank_factors(1, n, 2, seed=70 + n, lo=0.1, hi=1.0)
        ref = oracle.ustat_lowrank(edges, [F] * len(edges), [F] * len(edges))
        P = U.Plan(m, edges, precision="f64", symmetric=True)
        say(f"row reductions {name} n={n} vs oracle")
        r = P.eval([dev(F @ F.T, P.factor_dtype)] * len(edges))
        check(f"rows-{name}-{n}", r, ref, r.err_scale, "f64")


# ------------------------------------------------------------------ edge cases
EDGE_GRAPHS = {
    "m2": [(0, 1)],
    "m2-antiparallel": [(0, 1), (1, 0)],
    "parallel-same": [(0, 1), (0, 1), (1, 2), (2, 0)],
    "parallel-opposite": [(0, 1), (1, 0), (1, 2), (2, 3), (3, 1)],
    "triple": [(0, 1), (1, 0), (0, 1), (1, 2)],
}


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("sign", ["signed", "nonneg"])
@pytest.mark.parametrize("name", sorted(EDGE_GRAPHS))
def test_small_graphs_and_parallel_edges(U, name, prec, sign):
    """m = 2 and kernel graphs with repeated edges (Hadamard groups of the
    same or opposite orientation) at a ragged n, against brute force."""
    edges = EDGE_GRAPHS[name]
    m = nverts(edges)
    n = {2: 301, 3: 130, 4: 61}[m]
    lo = -1.0 if sign == "signed" else 0.0
    mats = as_device_sees(W.random_matrices(len(edges), n, seed=200 + m, lo=lo, hi=1.0), prec)
    ref = oracle.ustat_bruteforce(edges, mats)
    _, S, _ = oracle.ustat_and_scale_einsum(edges, mats)
    P = U.Plan(m, edges, precision=prec)
    say(f"edge case {name} n={n} {prec} {sign}")
    r = P.eval([dev(M, P.factor_dtype) for M in mats])
    check(f"edge-{name}-{sign}", r, ref, S, prec)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "i8"])
@pytest.mark.parametrize("name,edges", [("m2", [(0, 1)]), ("triangle", W.TRIANGLE),
                                        ("cycle4", W.CYCLE4), ("c5chord", W.CYCLE5_CHORD)])
def test_n_equals_m(U, name, edges, prec):
    """The smallest sample, n = m: a single tuple up to order."""
    import torch
    m = nverts(edges)
    n = m
    if prec == "i8":
        mats = W.random_int_matrices(len(edges), n, seed=300 + m, lo=-128, hi=127)
        ref = oracle.ustat_bruteforce_int(edges, mats)
        say(f"n=m {name} i8")
        r = U.Plan(m, edges, precision="i8").eval([dev(M, torch.int8) for M in mats])
        assert r.exact == ref
        return
    mats = as_device_sees(W.random_matrices(len(edges), n, seed=300 + m, lo=-1.0, hi=1.0), prec)
    ref = oracle.ustat_bruteforce(edges, mats)
    _, S, _ = oracle.ustat_and_scale_einsum(edges, mats)
    P = U.Plan(m, edges, precision=prec)
    say(f"n=m {name} {prec}")
    r = P.eval([dev(M, P.factor_dtype) for M in mats])
    check(f"n=m-{name}", r, ref, S, prec)


@pytest.mark.parametrize("name,edges", [("m2", [(0, 1)]), ("parallel", [(0, 1), (1, 0), (1, 2)])])
def test_edge_graphs_exact(U, name, edges):
    """The same graphs on the exact path with full-range int8 factors."""
    import torch
    m = nverts(edges)
    n = 97
    mats = W.random_int_matrices(len(edges), n, seed=400 + m, lo=-128, hi=127)
    ref = oracle.ustat_bruteforce_int(edges, mats)
    say(f"exact {name} n={n}")
    r = U.Plan(m, edges, precision="i8").eval([dev(M, torch.int8) for M in mats])
    assert r.exact == ref


# ------------------------------------------------------------------ factor operand form
@pytest.mark.parametrize("prec,n", [("bf16x3", 1500), ("bf16x3", 700), ("f32", 1100), ("f64", 530)])
def test_factor_operand_form_matches_prep(U, prec, n):
    """The sample entry point writes the GEMM-operand form of the RBF factor
    together with the factor (no separate operand preparation); evaluating
    the same factor through ustat_eval, whose GEMMs prepare it, gives the
    same U bit for bit (n = 700 in split-bf16 takes three-plane operands,
    which are still prepared)."""
    import torch
    d = 16
    X = dev(W.gaussian_samples(n, d, seed=800 + n), torch.float64)
    for name, edges in (("cycle4", W.CYCLE4), ("c5chord", W.CYCLE5_CHORD)):
        m = nverts(edges)
        P = U.Plan(m, edges, precision=prec)
        Q = U.Plan(m, edges, precision=prec, symmetric=True)
        say(f"operand form {name} {prec} n={n}")
        a = P.eval_samples(X, 2.0 * d)
        K = U.ustat_build_rbf(X, 2.0 * d, "f64" if prec == "f64" else "f32")
        b = Q.eval([K] * len(edges))
        assert a.value == b.value and a.err_scale == b.err_scale
