"""Induced motif counts through ustat_plan_create_motifs / ustat_motif_counts
(the motif application: complete-graph kernels with factors A and
B = 1 - A, all motifs of a size in one evaluation) against the oracle's
independent counts, bit for bit."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2508_12627_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def dev(A):
    import torch
    return torch.tensor(np.ascontiguousarray(A), dtype=torch.int8, device="cuda")


@pytest.mark.parametrize("k", [3, 4])
@pytest.mark.parametrize("n,p,seed", [(40, 0.3, 1), (73, 0.12, 2), (130, 0.05, 3)])
def test_motifs_small_bruteforce(U, k, n, p, seed):
    A = W.erdos_renyi(n, p, seed=seed)
    say(f"motifs k={k} n={n} p={p}")
    got = U.MotifPlan(k).counts(dev(A))
    assert got == oracle.motifs_bruteforce(A, k)


@pytest.mark.parametrize("k", [3, 4])
def test_named_graphs(U, k):
    n = 12
    K = np.ones((n, n), dtype=np.int8) - np.eye(n, dtype=np.int8)
    want = [0] * (2 if k == 3 else 6)
    want[-1] = math.comb(n, k)
    assert U.MotifPlan(k).counts(dev(K)) == want
    S = np.zeros((n, n), dtype=np.int8)
    S[0, 1:] = S[1:, 0] = 1
    want = [math.comb(n - 1, k - 1)] + [0] * (1 if k == 3 else 5)
    assert U.MotifPlan(k).counts(dev(S)) == want


@pytest.mark.parametrize("k,n,p", [(3, 4096, 0.01), (4, 1500, 0.01), (4, 2048, 0.004)])
def test_motifs_at_size_enumeration(U, k, n, p):
    """Larger sparse graphs (several 128-wide GEMM tiles, ragged n, and for
    size 4 programs conditioned on one vertex in slice chunks) against the
    oracle's enumeration of connected induced subgraphs; triangles also
    against the trace formula."""
    A = W.erdos_renyi(n, p, seed=n)
    say(f"motifs at size k={k} n={n} p={p}: oracle...")
    ref = oracle.motifs_esu(A, k)
    say(f"  oracle {ref}; gpu")
    got = U.MotifPlan(k).counts(dev(A))
    assert got == ref
    if k == 3:
        assert got[1] == oracle.count_triangles(A.astype(np.int64))


def test_cse_across_motifs_changes_nothing(U):
    A = W.erdos_renyi(200, 0.08, seed=9)
    a = U.MotifPlan(4).counts(dev(A))
    b = U.MotifPlan(4, cse=False).counts(dev(A))
    assert a == b


def test_rejects_non_adjacency(U):
    A = W.erdos_renyi(50, 0.2, seed=4)
    bad = A.copy()
    bad[3, 7] = 1 - bad[3, 7]  # asymmetric
    with pytest.raises(U.UstatError) as ei:
        U.MotifPlan(3).counts(dev(bad))
    assert ei.value.status == "invalid"
    two = A.copy()
    two[5, 6] = two[6, 5] = 2
    with pytest.raises(U.UstatError):
        U.MotifPlan(4).counts(dev(two))
    assert U.MotifPlan(3).counts(dev(A)) == oracle.motifs_bruteforce(A, 3)
