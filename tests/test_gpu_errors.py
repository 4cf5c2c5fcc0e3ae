"""Error paths of evaluations on the GPU, forced from the host with the
failure-injection hook: a device allocation failure (USTAT_E_NOMEM), a
launch failure after a graph capture has begun (USTAT_E_HIP; the capture
is ended and the stream stays usable) and a host allocation failure
inside the scheduler (USTAT_E_NOMEM).  After each, the same evaluation
succeeds and gives the reference value bit for bit."""
import sys

import numpy as np
import pytest

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
    yield ustat
    for k in (0, 1, 2):
        ustat.ustat_debug_inject(k, -1)


def factors(n, seed):
    import torch
    mats = W.random_matrices(4, n, seed=seed, lo=0.0, hi=1.0)
    return [torch.tensor(M, dtype=torch.float32, device="cuda") for M in mats]


@pytest.mark.parametrize("kind,expect", [(1, "nomem"), (2, "hip"), (0, "nomem")])
def test_injected_failure_then_recovery(U, kind, expect):
    import torch
    fs = factors(300, 11)
    ref = U.Plan(4, W.CYCLE4, precision="bf16x3").eval(fs).value
    s = torch.cuda.Stream()
    P = U.Plan(4, W.CYCLE4, precision="bf16x3")
    say(f"inject kind={kind}")
    U.ustat_debug_inject(kind, 0)
    with torch.cuda.stream(s):
        with pytest.raises(U.UstatError) as ei:
            P.eval(fs, stream=s)
        U.ustat_debug_inject(kind, -1)
        assert ei.value.status == expect
        # the stream is usable and the plan recovers
        x = torch.ones(1000, device="cuda")
        assert float((x * 2).sum().item()) == 2000.0
        a = P.eval(fs, stream=s)
        b = P.eval(fs, stream=s)  # graph replay
    torch.cuda.synchronize()
    assert a.value == ref and b.value == ref
