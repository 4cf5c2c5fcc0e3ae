"""The autotuner (a search over the executor's launch shapes: GEMM tile width
and column-strip target) on single and batched evaluations, and its
per-device cache (USTAT_TUNE_CACHE).  Tuned results are checked against the
oracle; a second tuning with the same key comes from the cache, unmeasured."""
import sys

import numpy as np
import pytest

import oracle
from paper_2508_12627_amd import workloads as W

pytestmark = pytest.mark.gpu

GEMM_BIG = {256, 0, 1 << 62}
COLRED = {256, 1024, 4096}


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


def dev(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


def test_batched_autotune_oracle_and_cache(U, tmp_path, monkeypatch):
    ns = [60, 97, 130, 200]
    d, div = 8, 16.0
    Xh = [W.student_t_samples(n, d, seed=70 + i) for i, n in enumerate(ns)]
    Xs = [dev(x) for x in Xh]
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("USTAT_TUNE_CACHE", str(cache))
    P = U.Plan(5, W.CYCLE5_CHORD, precision="bf16x3")
    say("batched autotune")
    ms = P.autotune_batched(Xs, div, reps=1)
    t = P.tuning()
    assert t["gemm_big_min"] in GEMM_BIG and t["colred_blocks"] in COLRED and ms > 0
    assert len(cache.read_text().splitlines()) == 1
    res = P.eval_batched(Xs, div)
    for X, r in zip(Xh, res):
        K = oracle.rbf_matrix(X, div)
        ref, S, _ = oracle.ustat_and_scale_einsum(W.CYCLE5_CHORD, [K] * 6)
        say(f"  n={X.shape[0]} err/S={abs(r.value - ref) / S:.2e}")
        assert abs(r.value - ref) <= 1e-6 * S
    # same key: applied from the cache, nothing measured or appended
    Q = U.Plan(5, W.CYCLE5_CHORD, precision="bf16x3")
    ms2 = Q.autotune_batched(Xs, div, reps=1)
    assert Q.tuning() == t and ms2 == pytest.approx(ms, rel=1e-5)
    assert len(cache.read_text().splitlines()) == 1


def test_single_autotune_cache_per_size_bucket(U, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("USTAT_TUNE_CACHE", str(cache))
    for n in (300, 700):
        X = W.gaussian_samples(n, 8, seed=80 + n)
        K = oracle.rbf_matrix(X, 16.0)
        P = U.Plan(4, W.CYCLE4, precision="f32", symmetric=True)
        say(f"single autotune n={n}")
        P.autotune([dev(K, __import__("torch").float32)] * 4, reps=1)
        r = P.eval([dev(K, __import__("torch").float32)] * 4)
        ref, S, _ = oracle.ustat_and_scale_einsum(W.CYCLE4, [np.float32(K).astype(np.float64)] * 4)
        assert abs(r.value - ref) <= 1e-6 * S
    # two size buckets: two entries; a repeat of the first adds none
    assert len(cache.read_text().splitlines()) == 2
    P = U.Plan(4, W.CYCLE4, precision="f32", symmetric=True)
    X = W.gaussian_samples(300, 8, seed=380)
    P.autotune([dev(oracle.rbf_matrix(X, 16.0), __import__("torch").float32)] * 4, reps=1)
    assert len(cache.read_text().splitlines()) == 2
