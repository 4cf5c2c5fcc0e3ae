"""The entry point that allocates nothing (ustat_eval_noalloc) against
ustat_eval on the same inputs, through the C ABI.

Both run the same kernels in the same order on the same descriptors, so the
results must agree bit for bit (floating point and exact integers alike).
Each case calls the pair twice in a row, the second time with a smaller n,
so that the fixed device buffer is reused with the first call's contents
still in it.  The floating-point cases are also held to the oracle at the
tolerance of their precision.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2508_12627_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "bf16x3": 1e-6}


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


def same(a, b):
    return (a.value == b.value and a.err_scale == b.err_scale and a.exact_hi == b.exact_hi
            and a.exact_lo == b.exact_lo and a.num_vstats == b.num_vstats)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("name,edges", [("cycle4", W.CYCLE4), ("c5chord", W.CYCLE5_CHORD)])
def test_noalloc_matches_eval_fp(U, prec, name, edges):
    m = 1 + max(max(e) for e in edges)
    P = U.Plan(m, edges, precision=prec)
    sizes = (300, 97) if m == 4 else (160, 31)
    for n in sizes:
        mats = W.random_matrices(len(edges), n, seed=40 + n, lo=0.0, hi=1.0)
        fs = [dev(M, P.factor_dtype) for M in mats]
        say(f"noalloc {name} {prec} n={n}")
        a = P.eval(fs)
        b = P.eval_noalloc(fs)
        say(f"  eval={a.value!r} noalloc={b.value!r}")
        assert same(a, b)
    # the second (smaller) call also against the oracle's brute force
    ref = oracle.ustat_bruteforce(edges, mats)
    _, S, _ = oracle.ustat_and_scale_einsum(edges, mats)
    assert abs(b.value - ref) <= TOL[prec] * S


def test_noalloc_matches_eval_exact(U):
    """Exact 5-cycle counts of two random graphs, the second smaller."""
    import torch
    P = U.Plan(5, W.CYCLE5, precision="i8")
    for n, p in ((400, 0.05), (150, 0.1)):
        A = W.erdos_renyi(n, p, seed=3 + n)
        fs = [dev(A, torch.int8)] * 5
        say(f"noalloc exact n={n}")
        a = P.eval(fs)
        b = P.eval_noalloc(fs)
        assert same(a, b)
        assert b.exact == 10 * oracle.count_5cycles(A)


def test_noalloc_conditioned_program(U):
    """A kernel graph whose quotients include treewidth 3 (programs
    conditioned on a vertex, run in slice chunks inside the fixed buffer)."""
    import torch
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (3, 4), (4, 5), (5, 0)]
    P = U.Plan(6, edges, precision="f64")
    for n in (40, 23):
        mats = W.random_matrices(len(edges), n, seed=90 + n, lo=-1.0, hi=1.0)
        fs = [dev(M, torch.float64) for M in mats]
        say(f"noalloc conditioned n={n}")
        a = P.eval(fs)
        b = P.eval_noalloc(fs)
        assert same(a, b)
    ref = oracle.ustat_bruteforce(edges, mats)
    assert abs(b.value - ref) <= 1e-10 * b.err_scale


def test_noalloc_rejects_oversize(U):
    """A workspace above the fixed buffer is refused before any launch."""
    import torch
    P = U.Plan(5, W.CYCLE5_CHORD, precision="f64")
    n = 2048
    ws = P.cost(n)["workspace"]
    assert ws > (128 << 20)
    K = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(U.UstatError) as ei:
        P.eval_noalloc([K] * len(W.CYCLE5_CHORD))
    assert ei.value.status == "infeasible"
    # the buffer still serves a fitting call afterwards
    mats = W.random_matrices(6, 50, seed=5, lo=0.0, hi=1.0)
    fs = [dev(M, torch.float64) for M in mats]
    assert same(P.eval(fs), P.eval_noalloc(fs))
