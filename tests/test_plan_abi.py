"""Host-side tests of the planner and of the C ABI (no GPU needed).

The planner's partitions, Moebius coefficients, sparsification filter and
treewidths are pinned to values printed in the paper
(``tests/golden/paper_tables.json``) and to the CPU oracle's independent
partition enumerator.  Error paths of the ABI are forced from the host.
"""
import itertools
import json
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2508_12627_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))
LIB = os.path.join(ROOT, "paper_2508_12627_amd", "libustat.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libustat.so not built")


@pytest.fixture(scope="module")
def U():
    from paper_2508_12627_amd import ustat
    ustat.load_library()
    return ustat


def header_functions():
    src = open(os.path.join(ROOT, "include", "ustat.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(?:ustat_status|const char \*)\s*\**\s*(\w+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert "ustat_plan_create" in names and "vstat_eval" in names and "ustat_eval_batched" in names
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(U):
    for n in header_functions():
        assert n in U.EXPORTS, n


def test_bell_and_mu_match_oracle_enumeration(U):
    for m in range(1, 8):
        edges = W.path(m) if m > 1 else None
        if edges is None:
            continue
        P = U.Plan(m, edges)
        parts = P.partitions()
        assert len(parts) == len(oracle.partitions(m))
        ref = {}
        for blocks in oracle.partitions(m):
            ref[tuple(oracle.block_labels(blocks, m))] = oracle.mobius_mu(blocks)
        got = {tuple(p["block_of"]): p["mu"] for p in parts}
        assert got == ref


def test_bell_terms_table(U):
    g = GOLDEN["bell_terms"]
    for m, b in zip(g["m"], g["values"]):
        if m <= 7:
            assert U.Plan(m, W.path(m)).info()["num_vstats"] == b


def test_sparsified_path_terms_and_M(U):
    """Table 'tab:HOIF': sparsified term counts and M(m) for the m-path."""
    gs, gm = GOLDEN["sparsified_path_terms"], GOLDEN["M_path"]
    for m, cnt, M in zip(gs["m"], gs["values"], gm["values"]):
        if m > 10:
            continue
        info = U.Plan(m, W.path(m), sparsify=True).info()
        assert info["num_vstats"] == cnt, m
        assert info["M"] == M, m


def test_dp_Nl_counts(U):
    """Table 'tab:HOIF_Nl', dp rows: exact treewidth counts N_l."""
    g = GOLDEN["dp_Nl_path"]
    for m, row in zip(g["m"], g["values"]):
        info = U.Plan(m, W.path(m), sparsify=True).info()
        assert info["N_l"][1:5] == row, m
        assert info["N_l"][0] == 0


def test_t_of_e_over_all_graphs_on_six_vertices(U):
    """Observation on t(e): the largest treewidth of a graph with e edges,
    e = 1..8 (attained on six vertices), via the exact treewidth routine."""
    g = GOLDEN["t_of_e"]
    pairs = list(itertools.combinations(range(6), 2))
    best = {}
    for e in g["e"]:
        mx = 0
        for sel in itertools.combinations(pairs, e):
            mx = max(mx, U.ustat_graph_treewidth(6, list(sel)))
        best[e] = mx
    assert [best[e] for e in g["e"]] == g["values"]
    assert U.ustat_graph_treewidth(4, W.CYCLE4) == GOLDEN["cycle4_treewidth"]["value"]
    assert U.ustat_graph_treewidth(6, pairs) == 5


def test_worked_example_path4(U):
    """Sub-examples on the 4-path: the five surviving partitions, their
    treewidths, M = 2, N_1 = 4, N_2 = 1; the induced partition {1,3}{2,4}."""
    g = GOLDEN["path4_surviving_partitions"]
    P = U.Plan(4, W.PATH4, sparsify=True)
    parts = P.partitions()
    want = {}
    for blocks, tw in zip(g["partitions"], g["treewidths"]):
        lab = oracle.block_labels([[i - 1 for i in b] for b in blocks], 4)
        want[tuple(lab)] = tw
    assert {tuple(p["block_of"]): p["tw"] for p in parts} == want
    info = P.info()
    assert info["M"] == g["M"] and info["N_l"][1] == g["N1"] and info["N_l"][2] == g["N2"]
    # Example 'eg:quotient': quotient types of all 15 partitions by treewidth
    # (path/edge: 1, triangle: 2, vertex: 0).
    full = U.Plan(4, W.PATH4).info()
    q = GOLDEN["path4_quotient_types"]["counts"]
    assert full["N_l"][0] == q["vertex"]
    assert full["N_l"][1] == q["P4"] + q["P3"] + q["edge"]
    assert full["N_l"][2] == q["triangle"]


def test_mu_worked_example(U):
    g = GOLDEN["path4_mu_signs"]
    P = U.Plan(4, W.PATH4)
    got = {tuple(p["block_of"]): p["mu"] for p in P.partitions()}
    for blocks, mu in zip(g["partitions"], g["mu"]):
        lab = tuple(oracle.block_labels([[i - 1 for i in b] for b in blocks], 4))
        assert got[lab] == mu


def test_orders_are_permutations_and_widths_bounded(U):
    for edges in (W.CYCLE4, W.CYCLE5, W.CYCLE5_CHORD):
        m = 1 + max(max(e) for e in edges)
        for order in ("minfill", "exhaustive"):
            P = U.Plan(m, edges, order=order)
            for i, p in enumerate(P.partitions()):
                J = 1 + max(p["block_of"])
                o = P.order(i)
                assert sorted(o) == list(range(J))
                assert p["width"] >= p["tw"]
                # min-fill reaches the exact treewidth on these graphs
                assert p["width"] == p["tw"]
                assert P.slice_var(i) == -1


def test_m6_graphs_condition_treewidth3_quotients(U):
    """Random 6-vertex kernel graphs (6-10 edges, the learned-order
    workload's generator): every partition whose quotient has treewidth at
    most 3 gets an executable program; treewidth-3 quotients are conditioned
    on one vertex (order lists the other J-1 vertices) and keep width equal to
    the treewidth, under every order policy."""
    graphs = W.random_kernel_graphs(12, 6, 6, 10, seed=5)
    for edges in graphs:
        for order in ("minfill", "exhaustive"):
            P = U.Plan(6, edges, order=order)
            info = P.info()
            if info["M"] > 3:
                continue
            assert info["num_vstats"] == 203
            for i, p in enumerate(P.partitions()):
                J = 1 + max(p["block_of"])
                o, sv = U.ustat_plan_order(P.h, i, 6)
                assert p["width"] == p["tw"]
                if p["tw"] <= 2:
                    assert sv == -1 and sorted(o) == list(range(J))
                else:
                    assert 0 <= sv < J and sorted(o + [sv]) == list(range(J))


def test_config_step_counts(U):
    """Step structure of the workloads: largest width and quotient treewidth
    distribution (4-cycle: {0:1, 1:9, 2:5}; 5-cycle: {0:1, 1:25, 2:26};
    5-cycle with chord: {0:1, 1:22, 2:29})."""
    for edges, nl in ((W.CYCLE4, [1, 9, 5]), (W.CYCLE5, [1, 25, 26]), (W.CYCLE5_CHORD, [1, 22, 29])):
        m = 1 + max(max(e) for e in edges)
        info = U.Plan(m, edges).info()
        assert info["N_l"][:3] == nl
        assert info["max_width"] == 2


def test_cost_model_flops(U):
    """4-cycle, full decomposition: six n^3 contractions (2 n^3 flops each)."""
    P = U.Plan(4, W.CYCLE4, precision="f32")
    n = 4096
    c = P.cost(n)
    assert c["flops"] >= 12 * n ** 3
    assert c["flops"] < 12 * n ** 3 * 1.01
    assert c["workspace"] > 0


@pytest.mark.parametrize("m,edges,msg", [
    (3, [(0, 0), (1, 2)], "self-loop"),
    (4, [(0, 1), (1, 2)], "every vertex"),
    (3, [(0, 5)], "out of range"),
    (11, [(i, i + 1) for i in range(10)], "m must be"),
])
def test_invalid_graphs(U, m, edges, msg):
    with pytest.raises(U.UstatError) as ei:
        U.Plan(m, edges)
    assert ei.value.status == "invalid"
    assert msg in str(ei.value)


def test_invalid_options(U):
    with pytest.raises(U.UstatError):
        U.Plan(3, W.TRIANGLE, precision=7)
    with pytest.raises(U.UstatError):
        U.Plan(3, W.TRIANGLE, order=9)
    # the C ABI needs a weights file for the learned policy (the binding
    # passes the shipped one by default)
    import ctypes
    L = U.load_library()
    o = U.PlanOpts()
    L.ustat_plan_opts_default(ctypes.byref(o))
    o.order = U.ORDER_LEARNED
    h = ctypes.c_void_p()
    rc = L.ustat_plan_create(3, 3, U._edges_array(W.TRIANGLE), ctypes.byref(o), ctypes.byref(h))
    assert rc == 1 and "cost_model_path" in L.ustat_last_error().decode()
    assert h.value is None
    with pytest.raises(U.UstatError) as ei:
        U.Plan(3, W.TRIANGLE, n_hint=-5)
    assert "n_hint" in str(ei.value)
    with pytest.raises(U.UstatError) as ei:
        U.Plan(3, W.TRIANGLE, order="learned", cost_model_path="/nonexistent/model.txt")
    assert "cost model" in str(ei.value)


def test_eval_argument_errors_before_any_device_work(U):
    import ctypes
    P = U.Plan(3, W.TRIANGLE)
    L = U.load_library()
    r = U.Result()
    # n < m
    ptrs = (ctypes.c_void_p * 3)(1, 1, 1)
    assert L.ustat_eval(P.h, 2, ptrs, None, ctypes.byref(r)) == 1
    assert "at least m" in L.ustat_last_error().decode()
    # NULL factor pointer
    ptrs = (ctypes.c_void_p * 3)(1, None, 1)
    assert L.ustat_eval(P.h, 10, ptrs, None, ctypes.byref(r)) == 1
    # NULL plan
    assert L.ustat_eval(None, 10, ptrs, None, ctypes.byref(r)) == 1
    # samples with the exact path
    Pi = U.Plan(3, W.TRIANGLE, precision="i8")
    assert L.ustat_eval_samples(Pi.h, 10, 4, ctypes.c_void_p(1), 8.0, None, ctypes.byref(r)) == 1
    # bad divisor
    assert L.ustat_eval_samples(P.h, 10, 4, ctypes.c_void_p(1), -1.0, None, ctypes.byref(r)) == 1
    assert L.ustat_build_rbf(10, 0, ctypes.c_void_p(1), 8.0, 0, ctypes.c_void_p(1), None) == 1
    assert U.load_library().ustat_status_string(5).decode() == "exact integer overflow"


def test_unsupported_width_reported(U):
    """K5 minus nothing: the finest quotient has treewidth 4; the plan is
    created (planning is host-only) but evaluation reports unsupported."""
    import ctypes
    k5 = list(itertools.combinations(range(5), 2))
    P = U.Plan(5, k5)
    assert P.info()["M"] == 4
    r = U.Result()
    ptrs = (ctypes.c_void_p * len(k5))(*([1] * len(k5)))
    rc = U.load_library().ustat_eval(P.h, 16, ptrs, None, ctypes.byref(r))
    assert rc == 2


def test_shipped_cost_model_ranks_orders(U):
    """The shipped MI355X weights load, learned plans are complete, and
    their predicted log-times are finite and ordered sensibly in n."""
    import os
    assert os.path.exists(U.DEFAULT_COST_MODEL)
    for edges in W.random_kernel_graphs(4, 6, 6, 10, seed=5):
        P = U.Plan(6, edges, order="learned", n_hint=2048)
        info = P.info()
        if info["M"] > 3:
            continue
        assert info["num_vstats"] == 203
        for i, p in enumerate(P.partitions()):
            assert p["width"] == p["tw"]
    with open(U.DEFAULT_COST_MODEL) as f:
        assert f.readline().split() == ["ustat-mlp", "1"]
        F, H1, H2 = (int(x) for x in f.readline().split())
    assert F == U.NUM_FEATURES
    # the same plain order at growing n is predicted to take longer
    P = U.Plan(4, W.CYCLE4)
    i = max(range(15), key=lambda k: max(P.partition(k)["block_of"]))
    blk, order = P.partition(i)["block_of"], P.order(i)
    X = np.stack([U.ustat_order_features(P.h, blk, order, n) for n in (512, 1024, 2048, 4096)])
    params = np.array(open(U.DEFAULT_COST_MODEL).read().split()[5:], dtype=np.float64)
    assert params.size == U.ustat_mlp_num_params(F, H1, H2)
    from oracle import mlp_ref
    pred, _ = mlp_ref.forward(params, F, H1, H2, X.astype(np.float64))
    assert np.all(np.isfinite(pred)) and np.all(np.diff(pred) > 0)


def test_tuning_defaults_and_validation(U):
    """Launch-shape tuning: defaults, setting, and rejected values (host only)."""
    P = U.Plan(4, W.CYCLE4, precision="bf16x3")
    assert P.tuning() == {"gemm_big_min": 256, "colred_blocks": 1024}
    P.set_tuning(0, 256)
    assert P.tuning() == {"gemm_big_min": 0, "colred_blocks": 256}
    P.set_tuning(-7, 4096)
    assert P.tuning()["gemm_big_min"] == 0
    for bad in (0, -1, (1 << 20) + 1):
        with pytest.raises(U.UstatError):
            P.set_tuning(256, bad)

