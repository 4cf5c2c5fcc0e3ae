"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Floating-point results must satisfy |U_gpu - U_ref| <= tol * S with
S = sum_pi |mu_pi V_pi| computed by the oracle (or a lower bound of S, which
only tightens the test); tol is 1e-12 for the fp64 path and 1e-6 for the
fp32 and split-bf16 paths.  Integer results must match exactly.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2508_12627_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "bf16x3": 1e-6}


def as_device_sees(mats, prec):
    """The factors as the engine receives them: fp32 for the fp32 and
    split-bf16 paths (the oracle then measures the engine's own error)."""
    if prec in ("f32", "bf16x3"):
        return [np.asarray(M, dtype=np.float32).astype(np.float64) for M in mats]
    return mats


def check_est(tag, r, err, prec):
    """The result's own error estimate covers the measured error."""
    say(f"ERRSTAT {tag} {prec} err={err:.3e} est={r.err_est:.3e}")
    assert err <= r.err_est, (err, r.err_est)


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


GRAPHS = {
    "triangle": W.TRIANGLE,
    "path4": W.PATH4,
    "cycle4": W.CYCLE4,
    "cycle5": W.CYCLE5,
    "c5chord": W.CYCLE5_CHORD,
    "star": [(0, 1), (0, 2), (0, 3)],
    "bowtie": [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 2)],
    "reversed": [(1, 0), (2, 1), (0, 2), (3, 2)],
}


def nverts(edges):
    return 1 + max(max(e) for e in edges)


# ------------------------------------------------------------------ H1
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("d", [12, 40])
def test_rbf_factor_build(U, prec, d):
    """The device factor against the oracle's direct-difference RBF, at a
    ragged n spanning several 64-row tiles (and d above one 32-wide chunk):
    symmetric bit for bit, unit diagonal."""
    import torch
    n, div = 301, 2.0 * d
    say(f"rbf n={n} d={d} {prec}")
    X = W.gaussian_samples(n, d, seed=7)
    K = U.ustat_build_rbf(dev(X, torch.float64), div, prec)
    torch.cuda.synchronize()
    ref = oracle.rbf_matrix(X, div)
    got = K.double().cpu().numpy()
    assert np.all(np.diag(got) == 1.0)
    assert np.array_equal(got, got.T)
    # The device forms |x_i - x_j|^2 as |x_i|^2 + |x_j|^2 - 2 x_i.x_j (Gram
    # on fp64 MFMA, sums of d terms): its rounding error is at most about
    # (d + 3) u (|x_i|^2 + |x_j|^2 + 2 |x_i| |x_j|); the oracle's direct
    # differences carry a (d + 2) u relative in a = |x_i - x_j|^2 / div;
    # exp adds an ulp on each side.
    u = 2.0 ** -53
    a = -np.log(ref)
    nr = np.sqrt(np.sum(X * X, axis=1))
    scale = (nr[:, None] + nr[None, :]) ** 2
    bound = ((d + 3) * scale / div + a * (d + 3) + 6) * u * ref
    if prec == "f64":
        assert np.all(np.abs(got - ref) <= bound)
    else:
        assert np.all(np.abs(got - ref) <= 2.0 ** -24 * ref + bound)


# ------------------------------------------------------------------ small n, every path
@pytest.mark.parametrize("sign", ["signed", "nonneg"])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_small_asymmetric_factors(U, name, prec, sign):
    """Independent asymmetric factors per edge at a ragged n spanning several
    tiles, against the brute-force oracle, every precision held to tol * S
    (signed factors make the split-bf16 path contract three-plane operands,
    whose products keep every term down to 2^-18)."""
    import torch
    edges = GRAPHS[name]
    m = nverts(edges)
    n = {3: 150, 4: 70, 5: 29}[m]
    lo = -1.0 if sign == "signed" else 0.0
    mats = as_device_sees(W.random_matrices(len(edges), n, seed=100 + m, lo=lo, hi=1.0), prec)
    ref = oracle.ustat_bruteforce(edges, mats)
    _, S, _ = oracle.ustat_and_scale_einsum(edges, mats)
    P = U.Plan(m, edges, precision=prec)
    say(f"small {name} n={n} {prec} {sign}")
    r = P.eval([dev(M, P.factor_dtype) for M in mats])
    err = abs(r.value - ref) / S
    say(f"  U={r.value:.10e} ref={ref:.10e} S={S:.3e} err/S={err:.2e} gpuS={r.err_scale:.3e}")
    assert err <= TOL[prec]
    check_est(f"small-{name}-{sign}-n{n}", r, err, prec)
    assert r.err_scale == pytest.approx(S, rel=1e-3 if prec != "f64" else 1e-9)


@pytest.mark.parametrize("name", ["triangle", "cycle4", "c5chord", "bowtie"])
def test_vstat_every_partition(U, name):
    import torch
    edges = GRAPHS[name]
    m = nverts(edges)
    n = {3: 90, 4: 45, 5: 21}[m]
    mats = W.random_matrices(len(edges), n, seed=5, lo=-1.0, hi=1.0)
    P = U.Plan(m, edges, precision="f64")
    fs = [dev(M, torch.float64) for M in mats]
    say(f"vstat {name} n={n}")
    for blocks in oracle.partitions(m):
        lab = oracle.block_labels(blocks, m)
        ref = oracle.vstat_einsum(edges, mats, lab)
        # a non-canonical labelling of the same partition
        perm = [7 * b + 3 for b in lab]
        r = P.vstat(perm, fs)
        assert r.value == pytest.approx(ref, rel=1e-11, abs=1e-11 * max(1.0, abs(ref)))


@pytest.mark.parametrize("name", ["cycle4", "c5chord", "path4"])
def test_sparsified_and_orders_agree(U, name):
    """Lemma 3 and every order policy give the same U."""
    import torch
    edges = GRAPHS[name]
    m = nverts(edges)
    n = 133
    mats = W.random_matrices(len(edges), n, seed=9, lo=0.0, hi=1.0)
    fs = [dev(M, torch.float64) for M in mats]
    _, S, _ = oracle.ustat_and_scale_einsum(edges, mats)
    vals = []
    for kw in (dict(), dict(sparsify=True), dict(order="exhaustive"),
               dict(order="exhaustive", sparsify=True)):
        say(f"variants {name} {kw}")
        vals.append(U.Plan(m, edges, precision="f64", **kw).eval(fs).value)
    for v in vals[1:]:
        assert abs(v - vals[0]) <= 1e-12 * S


def test_sparsified_plan_counts(U):
    P = U.Plan(4, W.CYCLE4, sparsify=True)
    assert P.info()["num_vstats"] == 4


# ------------------------------------------------------------------ exact integers
@pytest.mark.parametrize("name", ["triangle", "cycle4", "cycle5", "c5chord", "bowtie", "reversed"])
def test_int8_signed_factors_exact(U, name):
    """Signed int8 factors over the full range exercise multi-limb operands."""
    import torch
    edges = GRAPHS[name]
    m = nverts(edges)
    n = {3: 70, 4: 30, 5: 14}[m]
    mats = W.random_int_matrices(len(edges), n, seed=31, lo=-128, hi=127)
    ref = oracle.ustat_bruteforce_int(edges, mats)
    P = U.Plan(m, edges, precision="i8")
    say(f"int8 {name} n={n}")
    r = P.eval([dev(M, torch.int8) for M in mats])
    assert r.exact == ref


@pytest.mark.parametrize("name,n", [("triangle", 300), ("cycle4", 160)])
def test_int8_signed_multilimb_k_steps(U, name, n):
    """Multi-limb products over several 128-wide K steps and a ragged tail:
    full-range signed factors need two limbs each (four limb passes), and the
    4-cycle's stored product feeds a second GEMM with more limbs."""
    import torch
    edges = GRAPHS[name]
    m = nverts(edges)
    mats = W.random_int_matrices(len(edges), n, seed=37, lo=-128, hi=127)
    ref = oracle.ustat_bruteforce_int(edges, mats)
    say(f"int8 multi-limb {name} n={n}")
    r = U.Plan(m, edges, precision="i8").eval([dev(M, torch.int8) for M in mats])
    assert r.exact == ref


def test_int8_graph_capture_and_replay(U):
    """Exact plans on a side stream are captured as a graph and replayed:
    the same 0/1 input twice (capture, then replay), new 0/1 data in the same
    buffer (replay: the graph reads the inputs again) and entries up to 3 in
    that buffer (other input maxima: a new schedule and capture), each
    exact against the oracle's cycle counts or brute force."""
    import torch
    n = 120
    A1 = W.erdos_renyi(n, 0.1, seed=5)
    A2 = W.erdos_renyi(n, 0.1, seed=6)
    s = torch.cuda.Stream()
    P = U.Plan(5, W.CYCLE5, precision="i8")
    with torch.cuda.stream(s):
        Ad = dev(A1, torch.int8)
        for rep in range(2):
            say(f"int8 capture rep {rep}")
            r = P.eval([Ad] * 5, stream=s)
            assert r.exact == 10 * oracle.count_5cycles(A1.astype(np.int64))
        Ad.copy_(dev(A2, torch.int8))
        s.synchronize()
        r = P.eval([Ad] * 5, stream=s)
        assert r.exact == 10 * oracle.count_5cycles(A2.astype(np.int64))
        rng = np.random.default_rng(7)
        A3 = (A2 * rng.integers(1, 4, size=(n, n))).astype(np.int8)
        Ad.copy_(dev(A3, torch.int8))
        s.synchronize()
        ref = oracle.ustat_bruteforce_int(W.CYCLE5, [A3[:40, :40]] * 5)
        Ad3 = dev(np.ascontiguousarray(A3[:40, :40]), torch.int8)
        P3 = U.Plan(5, W.CYCLE5, precision="i8")
        for rep in range(2):
            r = P3.eval([Ad3] * 5, stream=s)
            assert r.exact == ref
        r = P.eval([Ad] * 5, stream=s)
        r2 = P.eval([Ad] * 5, stream=s)
        assert r2.exact == r.exact
    full = U.Plan(5, W.CYCLE5, precision="i8").eval([dev(A3, torch.int8)] * 5)
    assert r.exact == full.exact


def test_int8_er_cycle_counts(U):
    import torch
    n, p = 300, 0.08
    A = W.erdos_renyi(n, p, seed=3)
    Ad = dev(A, torch.int8)
    for edges, fn, aut in ((W.TRIANGLE, oracle.count_triangles, 6),
                           (W.CYCLE4, oracle.count_4cycles, 8),
                           (W.CYCLE5, oracle.count_5cycles, 10)):
        m = nverts(edges)
        say(f"int8 ER n={n} m={m}")
        r = U.Plan(m, edges, precision="i8").eval([Ad] * len(edges))
        assert r.exact == aut * fn(A.astype(np.int64))
        rs = U.Plan(m, edges, precision="i8", sparsify=True).eval([Ad] * len(edges))
        assert rs.exact == r.exact


# ------------------------------------------------------------------ workload sizes
def test_triangle_workload_n256(U):
    """Triangle kernel, n = 256 samples in R^8, divisor 16, fp64 path."""
    import torch
    n, d, div = 256, 8, 16.0
    X = W.gaussian_samples(n, d, seed=1)
    K = oracle.rbf_matrix(X, div)
    ref = oracle.ustat_bruteforce(W.TRIANGLE, [K] * 3)
    _, S, _ = oracle.ustat_and_scale_einsum(W.TRIANGLE, [K] * 3)
    assert oracle.triangle_closed_form(K) == pytest.approx(ref, rel=1e-12)
    say("triangle workload n=256")
    r = U.Plan(3, W.TRIANGLE, precision="f64").eval_samples(dev(X, torch.float64), div)
    assert abs(r.value - ref) <= 1e-12 * S
    check_est("triangle-n256", r, abs(r.value - ref) / S, "f64")
    assert r.num_vstats == 5


@pytest.fixture(scope="module")
def c2_data():
    n, d = 4096, 16
    X = W.gaussian_samples(n, d, seed=2)
    K = oracle.rbf_matrix(X, 2.0 * d)
    ref = oracle.cycle4_closed_form(K)
    K2 = K @ K
    vfin = float(np.sum(K2 * K2))  # V of the finest partition, a lower bound of S
    return X, ref, vfin


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_cycle4_workload_full_size(U, c2_data, prec):
    """4-cycle RBF kernel at n = 4096, d = 16 (the benchmark workload) against
    the oracle's closed form."""
    import torch
    X, ref, vfin = c2_data
    say(f"cycle4 n=4096 {prec}")
    P = U.Plan(4, W.CYCLE4, precision=prec)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Xd = dev(X, torch.float64)
        r1 = P.eval_samples(Xd, 32.0, stream=s)
        r2 = P.eval_samples(Xd, 32.0, stream=s)  # graph replay
    err = abs(r1.value - ref) / vfin
    say(f"  U={r1.value:.12e} ref={ref:.12e} err/Vfin={err:.2e}")
    assert err <= TOL[prec]
    check_est("cycle4-n4096", r1, abs(r1.value - ref) / r1.err_scale, prec)
    assert r2.value == r1.value  # replays are bitwise identical
    assert r2.err_est == r1.err_est


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_large_tiles_ragged(U, prec):
    """n = 4000 pads to 4096, so the GEMM level takes 256-wide tiles whose
    last row and column of tiles are partly outside the matrix: the 4-cycle
    U against the oracle's closed form (stored product consumed by column
    reductions) and rank-2 factors on the 5-cycle-with-chord kernel against
    the subset DP (fused final GEMMs)."""
    import torch
    n, d = 4000, 16
    X = W.gaussian_samples(n, d, seed=21)
    K = oracle.rbf_matrix(X, 2.0 * d)
    ref = oracle.cycle4_closed_form(K)
    K2 = K @ K
    vfin = float(np.sum(K2 * K2))
    say(f"large tiles cycle4 n={n} {prec}")
    r = U.Plan(4, W.CYCLE4, precision=prec).eval_samples(dev(X, torch.float64), 32.0)
    assert abs(r.value - ref) / vfin <= TOL[prec]
    check_est("large-tiles-cycle4", r, abs(r.value - ref) / r.err_scale, prec)
    (F, G), = W.lowrank_factors(1, n, 2, seed=22, lo=0.1, hi=1.0)
    ref = oracle.ustat_lowrank(W.CYCLE5_CHORD, [F] * 6, [G] * 6)
    say(f"large tiles lowrank c5chord n={n} {prec}")
    P = U.Plan(5, W.CYCLE5_CHORD, precision=prec)
    res = P.eval([dev(F @ G.T, P.factor_dtype)] * 6)
    assert abs(res.value - ref) <= TOL[prec] * abs(ref)
    check_est("large-tiles-lowrank", res, abs(res.value - ref) / res.err_scale, prec)


@pytest.mark.parametrize("n", [1280, 2498, 4096])
def test_symmetric_products_stream_k(U, n):
    """R = K K computed on the tiles on and above the diagonal only, their K
    steps spread evenly over the blocks (tiles split between two or three
    blocks and summed by the fix-up) and each tile mirrored: the 4-cycle U
    against the oracle's closed form, with and without the symmetric path
    (256-wide tiles forced).  The path is seen in the dry schedule: its
    workspace holds two fp32 partial tiles per block.  Two evaluations in a
    row give the same bits.  n = 1280 gives 15 tiles split over 30 blocks;
    n = 2498 is not a multiple of 4 (element-wise mirror stores) and leaves
    the last row and column of tiles partly outside the matrix.  (Below
    n = 1024 the operands take three planes and 128-wide tiles, outside this
    path.)"""
    import torch
    X = W.gaussian_samples(n, 16, seed=23)
    K = oracle.rbf_matrix(X, 32.0)
    ref = oracle.cycle4_closed_form(K)
    K2 = K @ K
    vfin = float(np.sum(K2 * K2))
    vals, ws = {}, {}
    for sym in (True, False):
        say(f"symmetric products n={n} sym={sym}")
        Q = U.Plan(4, W.CYCLE4, precision="bf16x3", sym_gemm=sym, symmetric=True)
        Q.set_tuning(0, 1024)
        ws[sym] = Q.workspace([n])
        P = U.Plan(4, W.CYCLE4, precision="bf16x3", sym_gemm=sym)
        P.set_tuning(0, 1024)
        r = P.eval_samples(dev(X, torch.float64), 32.0)
        r2 = P.eval_samples(dev(X, torch.float64), 32.0)
        assert r2.value == r.value
        err = abs(r.value - ref) / vfin
        say(f"  U={r.value:.12e} ref={ref:.12e} err/Vfin={err:.2e}")
        assert err <= TOL["bf16x3"]
        vals[sym] = r.value
    assert ws[True] > ws[False]
    # the two paths differ only in the order of fp32 additions
    assert abs(vals[True] - vals[False]) <= 1e-7 * vfin


def test_large_tiles_batched_level(U):
    """Four n = 2048 datasets put 4 x 64 tiles of 256 in each GEMM level, so
    their GEMMs run in a 256-wide launch, while the two sizes whose padding
    is not a multiple of 256 (1900, 333) share the level in a 128-wide one,
    and a single dataset (64 such tiles) takes 128-wide tiles: all agree to
    rounding, match the f64 path and, dataset by dataset, the oracle."""
    import torch
    ns = [2048] * 4 + [1900, 333]
    Xh = [W.gaussian_samples(n, 16, seed=80 + i) for i, n in enumerate(ns)]
    Xs = [dev(X, torch.float64) for X in Xh]
    P = U.Plan(4, W.CYCLE4, precision="bf16x3")
    say("large tiles batched 4 x 2048 bf16x3")
    rb = P.eval_batched(Xs, 32.0)
    r64 = U.Plan(4, W.CYCLE4, precision="f64").eval_batched(Xs, 32.0)
    for i, X in enumerate(Xs):
        single = P.eval_samples(X, 32.0)
        assert abs(rb[i].value - single.value) <= 1e-6 * single.err_scale
        assert abs(rb[i].value - r64[i].value) <= 1e-6 * r64[i].err_scale
        ref, S, _ = oracle.ustat_and_scale_einsum(W.CYCLE4, [oracle.rbf_matrix(Xh[i], 32.0)] * 4)
        say(f"large tiles batched dataset {i} n={ns[i]} vs oracle")
        assert abs(rb[i].value - ref) <= TOL["bf16x3"] * S
        assert abs(r64[i].value - ref) <= TOL["f64"] * S


def test_batched_workload_full_size_sampled(U):
    """The whole 256-dataset batch of the batched workload (n ~ U{128..4096},
    d = 32, Student-t(5) samples, 5-cycle plus chord, RBF divisor 64) in one
    split-bf16 evaluation with the launch shapes its benchmark uses; three
    datasets of it (the smallest, and those nearest n = 1024 and 2048) against
    the oracle, within 1e-6 S each."""
    import torch
    ns = [int(x) for x in W.ragged_sizes(256, 128, 4096, seed=4)]
    d, div = 32, 64.0
    Xh = [W.student_t_samples(n, d, seed=1000 + i) for i, n in enumerate(ns)]
    Xs = [dev(X, torch.float64) for X in Xh]
    P = U.Plan(5, W.CYCLE5_CHORD, precision="bf16x3", order="exhaustive")
    P.set_tuning(0, 1024)
    stream = torch.cuda.Stream()
    say("batched workload: 256 datasets, bf16x3, tuning 0,1024")
    r = P.eval_batched(Xs, div, stream=stream)
    torch.cuda.synchronize()
    picks = sorted({min(range(len(ns)), key=lambda i: ns[i]),
                    min(range(len(ns)), key=lambda i: abs(ns[i] - 1024)),
                    min(range(len(ns)), key=lambda i: abs(ns[i] - 2048))})
    for i in picks:
        K = oracle.rbf_matrix(Xh[i], div)
        ref, S, _ = oracle.ustat_and_scale_einsum(W.CYCLE5_CHORD, [K] * 6)
        err = abs(r[i].value - ref) / S
        say(f"batched workload dataset {i} n={ns[i]} err/S={err:.3e}")
        assert err <= TOL["bf16x3"], (i, ns[i], err)
        check_est(f"batched-{i}", r[i], err, "bf16x3")


@pytest.mark.parametrize("name", ["cycle4", "c5chord", "bowtie"])
def test_symmetric_factors_flag(U, name):
    """With symmetric factor matrices the symmetric flag (no transposed
    copies, orientation-merged steps) gives U within rounding of the default
    path in fp64 and bit-identical exact counts, and matches brute force."""
    import torch
    edges = GRAPHS[name]
    m = nverts(edges)
    n = 21
    (M,) = W.random_matrices(1, n, seed=31, lo=0.0, hi=1.0)
    M = 0.5 * (M + M.T)
    ref = oracle.ustat_bruteforce(edges, [M] * len(edges))
    Kd = dev(M, torch.float64)
    say(f"symmetric flag {name} n={n}")
    a = U.Plan(m, edges, precision="f64", symmetric=True).eval([Kd] * len(edges))
    b = U.Plan(m, edges, precision="f64").eval([Kd] * len(edges))
    assert abs(a.value - b.value) <= 1e-12 * b.err_scale
    assert abs(a.value - ref) <= 1e-12 * a.err_scale
    A = W.erdos_renyi(300, 0.1, seed=6)
    Ad = dev(A, torch.int8)
    ai = U.Plan(m, edges, precision="i8", symmetric=True).eval([Ad] * len(edges))
    bi = U.Plan(m, edges, precision="i8").eval([Ad] * len(edges))
    assert ai.exact == bi.exact


@pytest.mark.parametrize("name", ["cycle4", "c5chord", "bowtie"])
def test_row_reductions_span_segments(U, name):
    """Reductions over symmetric matrices run along rows in blocks of 32 rows
    by segments of up to 1024 columns.  At n = 1500 (two segments, 16-byte
    loads) and n = 1027 (two segments, element loads, a 3-column tail) the
    symmetric plan agrees with the column-strip plan on the same matrix in
    fp64 and bit for bit on the exact path; at a small size both match the
    oracle."""
    import torch
    edges = GRAPHS[name]
    m = nverts(edges)
    for n in (1500, 1027):
        (M,) = W.random_matrices(1, n, seed=41 + n, lo=0.0, hi=1.0)
        M = 0.5 * (M + M.T)
        Kd = dev(M, torch.float64)
        say(f"row reductions {name} n={n} f64")
        a = U.Plan(m, edges, precision="f64", symmetric=True).eval([Kd] * len(edges))
        b = U.Plan(m, edges, precision="f64").eval([Kd] * len(edges))
        assert abs(a.value - b.value) <= 1e-12 * b.err_scale
        A = W.erdos_renyi(n, 0.02, seed=n)
        Ad = dev(A, torch.int8)
        say(f"row reductions {name} n={n} i8")
        ai = U.Plan(m, edges, precision="i8", symmetric=True).eval([Ad] * len(edges))
        bi = U.Plan(m, edges, precision="i8").eval([Ad] * len(edges))
        assert ai.exact == bi.exact
    n = 37
    (M,) = W.random_matrices(1, n, seed=43, lo=0.0, hi=1.0)
    M = 0.5 * (M + M.T)
    ref = oracle.ustat_bruteforce(edges, [M] * len(edges))
    a = U.Plan(m, edges, precision="f64", symmetric=True).eval([dev(M, torch.float64)] * len(edges))
    assert abs(a.value - ref) <= 1e-12 * a.err_scale


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_autotune_and_forced_tilings_agree(U, prec):
    """The autotuner keeps one of its candidates, and every forced tiling
    (256-wide GEMM tiles whenever eligible, or never; coarse or fine column
    strips) gives U within the precision's tolerance of the f64 path."""
    import torch
    n, d = 1000, 16  # pads to 1024: 16 tiles of 256, so only a forced tiling uses them
    X = W.gaussian_samples(n, d, seed=23)
    K = U.ustat_build_rbf(dev(X, torch.float64), 32.0, "f32")  # split-bf16 reads fp32 factors
    K64 = U.ustat_build_rbf(dev(X, torch.float64), 32.0, "f64")
    ref = U.Plan(4, W.CYCLE4, precision="f64", symmetric=True).eval([K64] * 4)
    P = U.Plan(4, W.CYCLE4, precision=prec, symmetric=True)
    say(f"autotune cycle4 n={n} {prec}")
    ms = P.autotune([K] * 4, reps=2)
    t = P.tuning()
    assert ms > 0 and t["gemm_big_min"] in (256, 0, U.GEMM_BIG_NEVER)
    assert t["colred_blocks"] in (256, 1024, 4096)
    r = P.eval([K] * 4)
    assert abs(r.value - ref.value) <= TOL[prec] * ref.err_scale
    for gb in (0, U.GEMM_BIG_NEVER):
        for cb in (1, 4096):
            say(f"  forced tiling gemm_big_min={gb} colred_blocks={cb}")
            P.set_tuning(gb, cb)
            r = P.eval([K] * 4)
            assert abs(r.value - ref.value) <= TOL[prec] * ref.err_scale


def test_cycle5_er_full_size_exact(U):
    """Exact 5-cycle count of G(8192, 0.01) on the int8 path."""
    import torch
    n, p = 8192, 0.01
    A = W.erdos_renyi(n, p, seed=3)
    say("cycle5 ER n=8192 oracle...")
    ref = 10 * oracle.count_5cycles(A.astype(np.int64))
    say("cycle5 ER n=8192 gpu")
    r = U.Plan(5, W.CYCLE5, precision="i8").eval([dev(A, torch.int8)] * 5)
    assert r.exact == ref
    rs = U.Plan(5, W.CYCLE5, precision="i8", symmetric=True).eval([dev(A, torch.int8)] * 5)
    assert rs.exact == ref


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_lowrank_full_size(U, prec):
    """Rank-2 positive factors at n = 2048 on the 5-cycle-with-chord kernel:
    the oracle's subset DP gives the exact U at any n."""
    import torch
    n, r = 2048, 2
    edges = W.CYCLE5_CHORD
    (F, G), = W.lowrank_factors(1, n, r, seed=12, lo=0.1, hi=1.0)
    K = F @ G.T
    ref = oracle.ustat_lowrank(edges, [F] * 6, [G] * 6)
    say(f"lowrank c5chord n={n} {prec}")
    P = U.Plan(5, edges, precision=prec)
    res = P.eval([dev(K, P.factor_dtype)] * 6)
    # |U| <= S, so a relative-to-|U| bound is at least as strict
    assert abs(res.value - ref) <= TOL[prec] * abs(ref)
    check_est("lowrank-n2048", res, abs(res.value - ref) / res.err_scale, prec)


@pytest.mark.parametrize("name", ["cycle4", "c5chord", "bowtie"])
def test_cse_matches_separate_evaluation(U, name):
    """Merging equal steps across partitions gives the same U as evaluating
    every partition separately (fp64 to 1e-12 S; int8 exactly)."""
    import torch
    edges = GRAPHS[name]
    m = nverts(edges)
    n = 150
    (M,) = W.random_matrices(1, n, seed=17, lo=0.0, hi=1.0)
    Kd = dev(M, torch.float64)
    say(f"cse {name} n={n}")
    a = U.Plan(m, edges, precision="f64").eval([Kd] * len(edges))
    b = U.Plan(m, edges, precision="f64", cse=False).eval([Kd] * len(edges))
    assert abs(a.value - b.value) <= 1e-12 * b.err_scale
    A = W.erdos_renyi(n, 0.2, seed=5)
    Ad = dev(A, torch.int8)
    ai = U.Plan(m, edges, precision="i8").eval([Ad] * len(edges))
    bi = U.Plan(m, edges, precision="i8", cse=False).eval([Ad] * len(edges))
    assert ai.exact == bi.exact


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_batched_equals_single_and_oracle(U, prec):
    """Datasets of uneven n through ustat_eval_batched (one graph replay)
    give bitwise the results of one-by-one evaluation, and match the
    oracle's brute force on small datasets."""
    import torch
    edges = W.CYCLE5_CHORD
    ns = [int(x) for x in W.ragged_sizes(6, 17, 29, seed=4)]
    d, div = 3, 6.0
    Xs = [W.student_t_samples(n, d, seed=40 + i) for i, n in enumerate(ns)]
    P = U.Plan(5, edges, precision=prec)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Xd = [dev(X, torch.float64) for X in Xs]
        say(f"batched {prec} ns={ns}")
        rb = P.eval_batched(Xd, div, stream=s)
        rb2 = P.eval_batched(Xd, div, stream=s)  # replay
        singles = [P.eval_samples(X, div, stream=s) for X in Xd]
    for i, (X, n) in enumerate(zip(Xs, ns)):
        assert rb[i].value == singles[i].value
        assert rb2[i].value == rb[i].value
        K = oracle.rbf_matrix(X, div)
        ref = oracle.ustat_bruteforce(edges, [K] * 6)
        assert abs(rb[i].value - ref) <= TOL[prec] * rb[i].err_scale
        check_est(f"batched-{i}", rb[i], abs(rb[i].value - ref) / rb[i].err_scale, prec)


def test_batched_large_ragged(U):
    """A batch with n spanning several GEMM tiles and ragged tails: batched
    equals one-by-one evaluation bitwise."""
    import torch
    ns = [130, 257, 385, 512, 64, 1000]
    d, div = 32, 64.0
    Xs = [W.student_t_samples(n, d, seed=70 + i) for i, n in enumerate(ns)]
    P = U.Plan(5, W.CYCLE5_CHORD, precision="bf16x3")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Xd = [dev(X, torch.float64) for X in Xs]
        say(f"batched large ns={ns}")
        rb = P.eval_batched(Xd, div, stream=s)
        singles = [P.eval_samples(X, div, stream=s) for X in Xd]
    for i in range(len(ns)):
        assert rb[i].value == singles[i].value


K4 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_conditioned_treewidth3_small(U, prec):
    """Quotients of treewidth 3 are evaluated by conditioning on one vertex
    (a sum over its n values of width-2 eliminations): K4 and random m = 6
    workload graphs against brute force."""
    import torch
    graphs = [K4] + W.random_kernel_graphs(3, 6, 6, 10, seed=5)
    for edges in graphs:
        m = nverts(edges)
        n = {4: 37, 6: 13}[m]
        P = U.Plan(m, edges, precision=prec)
        assert P.info()["M"] >= 3
        mats = as_device_sees(W.random_matrices(len(edges), n, seed=8, lo=0.0, hi=1.0), prec)
        ref = oracle.ustat_bruteforce(edges, mats)
        say(f"conditioned {prec} m={m} n={n} edges={edges}")
        r = P.eval([dev(M, P.factor_dtype) for M in mats])
        assert abs(r.value - ref) <= TOL[prec] * r.err_scale
        check_est(f"conditioned-m{m}", r, abs(r.value - ref) / r.err_scale, prec)


def test_conditioned_exact_and_chunked(U):
    """Exact int8 counts through conditioning, and slice chunking giving the
    same result: a workspace limit equal to the one-slice workspace forces one
    slice per chunk, three times it a few slices per chunk with a ragged last
    chunk; a limit below the one-slice workspace is rejected as infeasible."""
    import torch
    A = W.erdos_renyi(40, 0.3, seed=9).astype(np.int64)
    Ad = dev(A, torch.int8)
    ref = oracle.ustat_bruteforce_int(K4, [A] * 6)
    say("conditioned int8 K4 n=40")
    r = U.Plan(4, K4, precision="i8").eval([Ad] * 6)
    assert r.exact == ref
    ws1 = U.Plan(4, K4, precision="i8").workspace([40])
    for lim in (ws1, 3 * ws1):
        say(f"conditioned int8 K4 n=40 workspace_limit={lim}")
        r2 = U.Plan(4, K4, precision="i8", workspace_limit=lim).eval([Ad] * 6)
        assert r2.exact == ref
    with pytest.raises(U.UstatError) as ei:
        U.Plan(4, K4, precision="i8", workspace_limit=1).eval([Ad] * 6)
    assert ei.value.code == 6
    X = W.gaussian_samples(150, 4, seed=3)
    Xd = dev(X, torch.float64)
    a = U.Plan(4, K4, precision="f64").eval_samples(Xd, 8.0)
    ws1 = U.Plan(4, K4, precision="f64").workspace([150])
    for lim in (ws1, 3 * ws1):
        say(f"conditioned f64 K4 n=150 workspace_limit={lim}")
        b = U.Plan(4, K4, precision="f64", workspace_limit=lim).eval_samples(Xd, 8.0)
        assert abs(a.value - b.value) <= 1e-12 * a.err_scale


@pytest.mark.parametrize("case", ["cycle4-samples", "c5chord-batched", "k4-conditioned"])
def test_second_stream_bitwise(U, case):
    """A level's reductions on a second stream beside its GEMMs (opt-in)
    give the results of the serial schedule bit for bit, on first evaluation and on
    graph replays (the 4-cycle on RBF factors at n = 2048, where the row
    reductions of K run beside the symmetric product; a ragged batch; a
    conditioned plan in slice chunks)."""
    import torch
    if case == "cycle4-samples":
        X = dev(W.gaussian_samples(2048, 16, seed=91), torch.float64)
        run = lambda P: [P.eval_samples(X, 32.0).value for _ in range(3)]
        mk = lambda ov: U.Plan(4, W.CYCLE4, precision="bf16x3", order="exhaustive", overlap=ov)
    elif case == "c5chord-batched":
        ns = [1100, 333, 2048, 700]
        Xs = [dev(W.gaussian_samples(n, 8, seed=92 + i), torch.float64) for i, n in enumerate(ns)]
        run = lambda P: [r.value for _ in range(2) for r in P.eval_batched(Xs, 16.0)]
        mk = lambda ov: U.Plan(5, W.CYCLE5_CHORD, precision="f32", overlap=ov)
    else:
        n = 300
        (M,) = W.random_matrices(1, n, seed=93, lo=0.0, hi=1.0)
        Kd = dev(0.5 * (M + M.T), torch.float64)
        run = lambda P: [P.eval([Kd] * 6).value for _ in range(2)]
        ws1 = U.Plan(4, K4, precision="f64", symmetric=True).workspace([n], shared_factor=False)
        mk = lambda ov: U.Plan(4, K4, precision="f64", symmetric=True, overlap=ov,
                               workspace_limit=40 * ws1)
    say(f"second stream {case}")
    a = run(mk(True))
    b = run(mk(False))
    assert a == b, (a, b)
