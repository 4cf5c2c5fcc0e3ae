"""Every ustat_status the C ABI defines, forced from the host (CPU, no
device work): argument checks (USTAT_E_INVALID), a plan needing a step
kind the engine lacks (USTAT_E_UNSUPPORTED), injected host allocation
failures at every point of plan creation and of a dry schedule
(USTAT_E_NOMEM), a HIP call that fails without a device (USTAT_E_HIP), an
exact plan whose a-priori bound overflows (USTAT_E_OVERFLOW).  The
workspace limit (USTAT_E_INFEASIBLE) needs an evaluation and is covered by
the GPU tests.  After every failure the library keeps working."""
import ctypes

import pytest

from paper_2508_12627_amd import workloads as W


@pytest.fixture(scope="module")
def U():
    from paper_2508_12627_amd import ustat
    ustat.load_library()
    yield ustat
    ustat.ustat_debug_inject(ustat.INJECT_HOST_ALLOC, -1)


def status_of(fn, *a):
    from paper_2508_12627_amd import ustat
    try:
        fn(*a)
    except ustat.UstatError as e:
        return e.status
    return "ok"


def test_status_strings(U):
    L = U.load_library()
    names = {L.ustat_status_string(c).decode() for c in range(7)}
    assert len(names) == 7 and "ok" in names


def test_invalid_and_unsupported(U):
    assert status_of(U.Plan, 3, [(0, 0), (1, 2)]) == "invalid"
    K5 = [(a, b) for a in range(5) for b in range(a + 1, 5)]
    P = U.Plan(5, K5)  # the finest quotient has treewidth 4
    L = U.load_library()
    ptrs = (ctypes.c_void_p * len(K5))(*[ctypes.c_void_p(4096)] * len(K5))
    r = U.Result()
    assert L.ustat_eval(P.h, 64, ptrs, None, ctypes.byref(r)) == 2  # unsupported, before device work


def test_peak_arguments(U):
    """The peak microbenchmarks check their arguments before any device
    call."""
    L = U.load_library()
    rate = ctypes.c_double()
    fake = ctypes.c_void_p(4096)
    assert L.ustat_peak_mfma(4, 10, fake, None, ctypes.byref(rate)) == 1  # unknown kind
    assert L.ustat_peak_mfma(0, 0, fake, None, ctypes.byref(rate)) == 1   # no rounds
    assert L.ustat_peak_mfma(0, 10, None, None, ctypes.byref(rate)) == 1  # no sink
    assert L.ustat_peak_copy(fake, fake, 24, None, ctypes.byref(rate)) == 1  # not a multiple of 16
    assert L.ustat_peak_copy(fake, None, 32, None, ctypes.byref(rate)) == 1


def test_hip_failure_without_device(U):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    L = U.load_library()
    P = U.Plan(4, W.CYCLE4, precision="f32")
    ptrs = (ctypes.c_void_p * 4)(*[ctypes.c_void_p(4096)] * 4)
    r = U.Result()
    assert L.ustat_eval_noalloc(P.h, 100, ptrs, None, ctypes.byref(r)) == 4
    assert b"device" in L.ustat_last_error()


def test_overflow_reported_by_cost(U):
    """The exact 5-cycle plan: its a-priori bound (factors of magnitude up
    to 127) fits at n = 100 and may overflow at n = 1000; n = 2^20 is past
    the exact path's int32 limb accumulation."""
    P = U.Plan(5, W.CYCLE5, precision="i8")
    assert P.cost(100)["workspace"] > 0
    assert status_of(P.cost, 1000) == "overflow"
    assert status_of(P.cost, 1 << 20) == "unsupported"


@pytest.mark.parametrize("edges,m", [(W.CYCLE5_CHORD, 5), ([(0, 1), (1, 0), (1, 2)], 3),
                                     (W.random_kernel_graphs(1, 6, 6, 10, seed=5)[0], 6)])
def test_injected_host_allocation_failures(U, edges, m):
    """A host allocation failure at each injection point of plan creation
    and of the dry schedule behind ustat_plan_cost: the call reports
    USTAT_E_NOMEM (never crashes, never returns a half-built plan), and the
    same calls succeed once the injection is disarmed."""
    ref = U.Plan(m, edges, precision="bf16x3").cost(300)
    seen = set()
    for k in range(0, 300, 3):
        U.ustat_debug_inject(U.INJECT_HOST_ALLOC, k)
        st = status_of(lambda: U.Plan(m, edges, precision="bf16x3").cost(300))
        seen.add(st)
        assert st in ("ok", "nomem")
    U.ustat_debug_inject(U.INJECT_HOST_ALLOC, -1)
    assert "nomem" in seen
    assert U.Plan(m, edges, precision="bf16x3").cost(300) == ref


def test_inject_rejects_unknown_kind(U):
    assert status_of(U.ustat_debug_inject, 9, 0) == "invalid"
