"""Benchmark: exact U-statistic evaluations per second on one MI355X.

Workload: the m = 4 four-cycle kernel h = k(x1,x2) k(x2,x3) k(x3,x4) k(x4,x1)
with the RBF factor k(x, y) = exp(-||x - y||^2 / (2 d)), n = 4096 samples in
R^16 drawn iid N(0, I) (seed 2), full Bell decomposition (15 restricted
V-statistics).  One step = one U-statistic evaluation from the samples
resident in HBM: factor build, every elimination step of every V-statistic,
the cross-tile reductions and the Moebius combination, replayed as one HIP
graph.  The headline precision is split-bf16 (hi*hi + hi*lo + lo*hi on MFMA,
fp32 accumulation, fp64 reductions); fp32-MFMA and fp64-MFMA runs of the same
workload are reported beside it with their errors relative to
S = sum |mu_pi V_pi|.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"bf16x3": 2.5e15, "f32": 157.3e12, "f64": 78.6e12}  # dense MFMA, FLOP/s
WORKLOAD = {"m": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "n": 4096, "d": 16, "seed": 2}


def timed_evals(plan, X, div, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        r = plan.eval_samples(X, div, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = plan.eval_samples(X, div, stream=stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


HBM_PEAK = 8.0e12  # bytes/s
KERNELS = {"gemm": "k_gemm", "elim1": "k_rowred/k_colred/k_elim1", "prep": "k_prep/k_transpose",
           "reduce": "k_reduce", "rbf": "k_rbf"}
PREC_INDEX = {"f64": 0, "f32": 1, "bf16x3": 2}
# HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (copy-calibrated) of the headline workload; used only while the kernel
# sources still hash to the value recorded with them.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cycle4_n4096_bf16x3.json")


LOWRANK_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_hoif_chains_n10000_r8.json")


def measured_lowrank_traffic(kernel, launches_per_step):
    """Counter-measured HBM bytes of one launch of a low-rank kernel (its
    bytes over the profiled steps divided by the launches), or None when no
    record exists or the low-rank kernels changed since it was taken."""
    try:
        with open(LOWRANK_TRAFFIC_FILE) as f:
            rec = json.load(f)
        from paper_2508_12627_amd.profsum import kernel_source_hash
    except (OSError, ValueError, ImportError):
        return None
    if rec.get("source_hash") != kernel_source_hash("lowrank"):
        return None
    for name, k in rec.get("kernels", {}).items():
        if kernel in name and k.get("bytes_per_launch") is not None:
            return k["bytes_per_launch"]
    return None


BATCHED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batched_c5chord_256.json")


def measured_traffic(kind, prec, path=TRAFFIC_FILE):
    """Counter-measured HBM bytes per launch of the kind's kernel, or None
    when no record exists or the kernels changed since it was taken."""
    try:
        with open(path) as f:
            rec = json.load(f)
        from paper_2508_12627_amd.profsum import kernel_source_hash
    except (OSError, ValueError, ImportError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("precision") != prec:
        return None
    frags = KERNELS[kind].split("/")
    if kind == "gemm":  # full products, symmetric ones (P P^T) and their fix-up
        frags = [f"k_gemm<{PREC_INDEX[prec]}", f"k_gemm_sym<{PREC_INDEX[prec]}",
                 f"k_gemm_symfix<{PREC_INDEX[prec]}"]
    # mean over the matching kernels' launches (a kind may span several
    # kernels, e.g. the row reductions over one and over two matrices); the
    # fix-up of a symmetric product belongs to its product's step, so its
    # bytes count and its launches do not
    tot, cnt = 0.0, 0
    for name, k in rec.get("kernels", {}).items():
        if any(fr in name for fr in frags) and k.get("bytes_per_launch") is not None:
            tot += k["bytes_per_launch"] * k["launches"]
            if "k_gemm_symfix" not in name:
                cnt += k["launches"]
    return tot / cnt if cnt else None


def kernel_rooflines(U, plan, X, div, stream, prec, reps=5, executed_share=1.0):
    """Per-kernel-kind durations from HIP events recorded around every
    launch on the launch stream (kernel-by-kernel launches, no graph)."""
    U.ustat_profile_enable(True)
    U.ustat_profile_reset()
    for _ in range(reps):
        plan.eval_samples(X, div, stream=stream)
    stats = {k: U.ustat_profile_read(k) for k in KERNELS}
    U.ustat_profile_enable(False)
    return summarize(stats, reps, prec, TRAFFIC_FILE, executed_share)


def summarize(stats, reps, prec, traffic_path=TRAFFIC_FILE, executed_share=1.0):
    """executed_share: the part of the GEMM's algorithmic products that its
    MFMA instructions compute (t(t+1)/2 of t^2 tiles for a symmetric product
    on t tiles a side, else 1); split-bf16 issues three products for each."""
    out = {}
    for k, g in stats.items():
        if g["launches"] == 0:
            continue
        sec = g["ms"] * 1e-3
        e = {"kernel": KERNELS[k] + (f"<{prec}>" if k == "gemm" else ""),
             "ms_per_eval": g["ms"] / reps, "launches_per_eval": g["launches"] / reps,
             "avg_launch_ms": g["ms"] / g["launches"],
             "traffic": measured_traffic(k, prec, traffic_path)}
        if k == "gemm":
            achieved = g["flops"] / sec
            e.update({"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAKS[prec] / 1e12,
                      "unit": "TFLOP/s", "frac": achieved / PEAKS[prec],
                      "flops_per_launch": g["flops"] / g["launches"],
                      "executed_frac": achieved * executed_share * (3 if prec == "bf16x3" else 1)
                      / PEAKS[prec]})
        elif g["bytes"] > 0:
            achieved = g["bytes"] / sec
            e.update({"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                      "unit": "GB/s", "frac": achieved / HBM_PEAK,
                      "bytes_per_launch": g["bytes"] / g["launches"]})
        out[k] = e
    dominant = max(out, key=lambda k: out[k]["ms_per_eval"])
    return dominant, out


def cpu_baseline(X, div, budget_s=15.0):
    """The oracle's brute-force sum over distinct ordered 4-tuples, timed on
    a bounded sample of (i0, i1) prefixes at the full n, scaled to evals/s."""
    import numpy as np
    import oracle
    edges = WORKLOAD["edges"]
    n = X.shape[0]
    K = oracle.rbf_matrix(X, div)
    items = 32
    t0 = time.perf_counter()
    oracle.ustat_bruteforce(edges, [K] * 4, items=(0, items))
    t = time.perf_counter() - t0
    if t < budget_s / 3:
        more = int(items * (budget_s - t) / max(t, 1e-3))
        t1 = time.perf_counter()
        oracle.ustat_bruteforce(edges, [K] * 4, items=(items, items + more))
        t += time.perf_counter() - t1
        items += more
    frac = items / float(n * n)
    cores = oracle.num_threads()
    # the same oracle on one core, over a smaller prefix sample
    oracle.set_num_threads(1)
    try:
        items1 = max(2, items // max(1, cores))
        t1 = time.perf_counter()
        oracle.ustat_bruteforce(edges, [K] * 4, items=(0, items1))
        t1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(cores)
    return {"value": frac / t, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "single_thread_value": items1 / float(n * n) / t1,
            "sample": f"brute-force sum over distinct ordered 4-tuples restricted to the first "
                      f"{items} (i0, i1) prefixes of {n * n} at n={n} ({t:.1f} s on {cores} "
                      f"threads), scaled by the prefix fraction; single thread: the first "
                      f"{items1} prefixes ({t1:.1f} s)"}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_batched(args):
    """256 independent datasets, n ~ U{128..4096} (seed 4), d = 32, iid
    Student-t(5) coordinates, kernel on the 5-cycle plus chord (0,2), RBF
    divisor 64; every (dataset, partition) pair in one HIP graph replay."""
    import numpy as np
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W
    ns = [int(x) for x in W.ragged_sizes(256, 128, 4096, seed=4)]
    d, div = 32, 64.0
    stream = torch.cuda.Stream()
    Xs = [torch.tensor(W.student_t_samples(n, d, seed=1000 + i), dtype=torch.float64,
                       device="cuda") for i, n in enumerate(ns)]
    out = {"metric": "datasets/s (batched U-statistics)", "unit": "datasets/s",
           "config": {"workload": "256 datasets, n~U{128..4096}, d=32, Student-t(5), "
                                  "5-cycle + chord kernel, 52 restricted V-statistics each",
                      "precision": args.precision, "second_stream": args.overlap_levels}}
    plan = U.Plan(5, W.CYCLE5_CHORD, precision=args.precision, order=args.order,
                  overlap=args.overlap_levels)
    if args.tuning:
        gb, cb = (int(v) for v in args.tuning.split(","))
        plan.set_tuning(gb, cb)
    else:
        # launch shapes tuned on the whole batch (outside the timed region)
        out["config"]["tune_ms"] = plan.autotune_batched(Xs, div, stream=stream, reps=2)
    out["config"]["tuning"] = plan.tuning()
    if args.profile_steps:
        for _ in range(args.profile_steps):
            r = plan.eval_batched(Xs, div, stream=stream)
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "value": r[0].value}))
        return
    steps = max(2, args.steps // 10)
    for _ in range(max(1, args.warmup // 2)):
        r = plan.eval_batched(Xs, div, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = plan.eval_batched(Xs, div, stream=stream)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    flops = sum(plan.cost(n)["flops"] for n in ns)
    out.update({"value": len(ns) / el, "ms_per_batch": 1e3 * el, "steps": steps,
                "algorithmic_flops_per_batch_without_cse": flops})
    # reference: f64 path of the same batch, error relative to S
    p64 = U.Plan(5, W.CYCLE5_CHORD, precision="f64", order=args.order)
    r64 = p64.eval_batched(Xs, div, stream=stream)
    out["max_err_vs_f64_over_S"] = max(abs(a.value - b.value) / b.err_scale for a, b in zip(r, r64))
    dom, kr = kernel_rooflines_batched(U, plan, Xs, div, stream, args.precision)
    out["roofline"] = dict(kr[dom])
    out["roofline"]["dominant_kind"] = dom
    out["kernels"] = kr
    print(json.dumps(out))


def kernel_rooflines_batched(U, plan, Xs, div, stream, prec, reps=1):
    U.ustat_profile_enable(True)
    U.ustat_profile_reset()
    for _ in range(reps):
        plan.eval_batched(Xs, div, stream=stream)
    stats = {k: U.ustat_profile_read(k) for k in KERNELS}
    U.ustat_profile_enable(False)
    return summarize(stats, reps, prec, BATCHED_TRAFFIC_FILE)


def bench_cycle5_exact(args):
    """Exact 5-cycle count of G(8192, 0.01) (seed 3) on the int8 path."""
    import numpy as np
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W
    A = W.erdos_renyi(8192, 0.01, seed=3)
    Ad = torch.tensor(A, dtype=torch.int8, device="cuda")
    torch.cuda.synchronize()
    # a side stream: the evaluation is captured as a graph and replayed
    stream = torch.cuda.Stream()
    out = {"metric": "exact 5-cycle count, G(8192, 0.01)", "unit": "evals/s",
           "config": {"workload": "G(8192,0.01) seed 3, 5-cycle kernel, int8 MFMA limbs"}}
    for sp in (False, True):
        plan = U.Plan(5, W.CYCLE5, precision="i8", sparsify=sp, symmetric=True,
                      overlap=args.overlap_levels)
        r = plan.eval([Ad] * 5, stream=stream)
        torch.cuda.synchronize()
        steps = max(3, args.steps // 5)
        t0 = time.perf_counter()
        for _ in range(steps):
            r = plan.eval([Ad] * 5, stream=stream)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        rec = {"ms_per_eval": 1e3 * el, "U": str(r.exact), "cycles": str(r.exact // 10),
               "num_vstats": r.num_vstats}
        # live GEMM timing (HIP events) of one evaluation: algorithmic
        # 2 n^3 integer multiply-adds per product against the int8 MFMA peak
        U.ustat_profile_enable(True)
        U.ustat_profile_reset()
        plan.eval([Ad] * 5)
        g = U.ustat_profile_read("gemm")
        U.ustat_profile_enable(False)
        if g["ms"] > 0:
            ach = g["flops"] / (g["ms"] * 1e-3)
            rec["roofline"] = {"kernel": "k_gemm<i8>", "bound": "mfma", "achieved": ach / 1e12,
                               "peak": 5000.0, "unit": "TOP/s", "frac": ach / 5.0e15,
                               "traffic": None, "launches_per_eval": g["launches"],
                               "avg_launch_ms": g["ms"] / max(1, g["launches"]),
                               "ops_per_eval": g["flops"]}
        out["sparsified" if sp else "full"] = rec
    # the sparsified program (Lemma 3) is the faster one; both are reported
    best = min(("full", "sparsified"), key=lambda k: out[k]["ms_per_eval"])
    out["value"] = 1e3 / out[best]["ms_per_eval"]
    out["value_from"] = best
    out["roofline"] = out[best].get("roofline")
    print(json.dumps(out))


# Published dense peaks of the MI355X (operations/s) for each MFMA kind the
# kernels use, and its HBM bandwidth (bytes/s).
SPEC_PEAKS = {"bf16": 2.5e15, "f64": 78.6e12, "i8": 5.0e15, "f32": 157.3e12}


def bench_peaks(args):
    """The rooflines' denominators measured on this device: back-to-back
    MFMAs of each kind the kernels use, and a streaming copy of 2 x 1 GiB;
    each next to the published figure."""
    from paper_2508_12627_amd import ustat as U
    out = {"metric": "measured peaks (MFMA kinds, streaming copy) against the published MI355X figures",
           "mfma": {}}
    for kind, spec in SPEC_PEAKS.items():
        # a few ms per timed launch (bf16 and int8 issue 16 384 / 32 768
        # operations per instruction, fp64 and fp32 2 048)
        iters = 40000 if kind in ("bf16", "i8") else 10000
        best = max(U.ustat_peak_mfma(kind, iters) for _ in range(3))
        out["mfma"][kind] = {"measured": best, "published": spec, "frac": best / spec}
        print(f"peaks: {kind} {best / 1e12:.1f} T/s ({best / spec:.3f} of published)", file=sys.stderr,
              flush=True)
    best = max(U.ustat_peak_copy(1 << 30) for _ in range(3))
    out["hbm_copy"] = {"measured": best, "published": HBM_PEAK, "frac": best / HBM_PEAK,
                       "unit": "bytes/s (read + write)"}
    print(f"peaks: copy {best / 1e9:.0f} GB/s", file=sys.stderr, flush=True)
    print(json.dumps(out))


def bench_motifs(args):
    """Induced motif counts of Erdos-Renyi graphs on the exact path at the
    sizes of the paper's motif tables: all 3-vertex motifs of G(20000, p)
    and all 4-vertex motifs of G(2000, p), p = 0.01 (seed 3); one
    evaluation counts every motif of a size (steps shared across motifs).
    The oracle (enumeration of connected induced subgraphs) is timed on the
    host cores beside it and must agree exactly."""
    import torch
    import oracle
    from paper_2508_12627_amd import ustat as U, workloads as W
    out = {"metric": "induced motif counts, seconds per graph (all motifs of a size)",
           "unit": "s", "higher_is_better": False,
           "config": {"workload": "G(20000, 0.01) 3-vertex motifs; G(2000, 0.01) 4-vertex motifs; "
                                  "seed 3; complete-graph kernels with A and 1 - A factors"}}
    for size, n, p in ((3, 20000, 0.01), (4, 2000, 0.01)):
        print(f"motifs: size {size}, G({n}, {p})", file=sys.stderr, flush=True)
        A = W.erdos_renyi(n, p, seed=3)
        Ad = torch.tensor(A, dtype=torch.int8, device="cuda")
        plan = U.MotifPlan(size)
        got = plan.counts(Ad)
        torch.cuda.synchronize()
        steps = max(2, args.steps // 40)
        U.ustat_profile_enable(True)
        U.ustat_profile_reset()
        t0 = time.perf_counter()
        for _ in range(steps):
            got = plan.counts(Ad)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        g = U.ustat_profile_read("gemm")
        U.ustat_profile_enable(False)
        rec = {"n": n, "p": p, "seconds": el, "counts": dict(zip(plan.names, got)),
               "gemm": {"ms_per_eval": g["ms"] / steps, "launches_per_eval": g["launches"] / steps,
                        "int8_tops_algorithmic": g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] else None}}
        print(f"  {el:.4f} s per evaluation; oracle...", file=sys.stderr, flush=True)
        if not args.no_cpu_baseline:
            t1 = time.perf_counter()
            if size == 3:
                ref = oracle.motifs3_closed_form(A)
                how = "whole graph (degrees and the trace formula for triangles)"
            else:
                ref = oracle.motifs_esu(A, size)
                how = "whole graph (enumeration of connected induced subgraphs)"
            rec["cpu_baseline"] = {"seconds": time.perf_counter() - t1, "cores": oracle.num_threads(),
                                   "kind": "oracle", "cpu_model": cpu_model(), "sample": how}
            rec["exact_match"] = ref == got
        out[f"size{size}"] = rec
    out["value"] = out["size4"]["seconds"]
    print(json.dumps(out))


# Table tab:HOIF_runtime of the paper, n = 10000, single RTX 5090, dense
# n x n factors (seconds per U-statistic, by order): context only.
HOIF_PAPER_GPU_S = {2: 0.04398, 3: 0.08977, 4: 0.17264, 5: 0.41339, 6: 1.66450, 7: 8.58869}


def bench_hoif(args):
    """Influence-function chains of Section 4.1 from low-rank panels: the
    U-statistics of h_j for orders j = 2..7 (g on the first j - 2 edges of
    the chain, f on the last) at n = 10000 with a rank-8 dictionary (panels
    P = A phi(Z), Q = Y phi(Z), seed 11).  One step = the six U-statistics
    from panels resident in HBM, no n x n matrix formed.  Beside it: the
    dense path on the materialised n x n factors (the form the paper's
    table times) in fp64, and the oracle on a bounded sample."""
    import numpy as np
    import torch
    import oracle
    from paper_2508_12627_amd import ustat as U, workloads as W
    n, k, orders = 10000, 8, list(range(2, 8))
    P, Q = W.hoif_panels(n, k, seed=11)
    Pd = torch.tensor(P, dtype=torch.float64, device="cuda")
    Qd = torch.tensor(Q, dtype=torch.float64, device="cuda")
    plans = {j: U.Plan(j, W.hoif_chain(j)) for j in orders}
    FG = {j: ([Pd] * (j - 1), [Pd] * (j - 2) + [Qd]) for j in orders}
    res = {}
    for j in orders:  # schedules built and uploaded outside the timed region
        res[j] = plans[j].eval_lowrank(*FG[j])
    print("hoif: schedules ready", file=sys.stderr, flush=True)
    if args.profile_steps:
        for _ in range(args.profile_steps):
            for j in orders:
                plans[j].eval_lowrank(*FG[j])
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "value": res[7].value}))
        return
    steps = max(3, args.steps // 10)
    warm = max(1, args.warmup // 10)
    for _ in range(warm):
        for j in orders:
            plans[j].eval_lowrank(*FG[j])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for j in orders:
            r = plans[j].eval_lowrank(*FG[j])
            assert r.value == res[j].value  # deterministic
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    per = {}
    for j in orders:
        t1 = time.perf_counter()
        for _ in range(steps):
            plans[j].eval_lowrank(*FG[j])
        per[j] = (time.perf_counter() - t1) / steps
    print(f"hoif: {1e3 * el:.3f} ms per step", file=sys.stderr, flush=True)
    # live kernel timing with HIP events (one step)
    U.ustat_profile_enable(True)
    U.ustat_profile_reset()
    for j in orders:
        plans[j].eval_lowrank(*FG[j])
    kinds = {kd: U.ustat_profile_read(kd) for kd in ("lowrank_step", "lowrank_outer", "lowrank_reduce")}
    U.ustat_profile_enable(False)
    # the dominant kernel: the GEMM steps (fp64 MFMA) or the vector steps
    dom = max(("lowrank_outer", "lowrank_step"), key=lambda kd: kinds[kd]["ms"])
    st = kinds[dom]
    flops, byts, ms = st["flops"], st["bytes"], st["ms"]
    if dom == "lowrank_outer":
        bound, peak, unit, achieved = "mfma", 78.6e12, "TFLOP/s", flops / (ms * 1e-3)
    else:
        alu_peak = 78.6e12  # fp64 vector FLOP/s
        bound = "alu" if flops / byts > alu_peak / HBM_PEAK else "hbm"
        achieved = flops / (ms * 1e-3) if bound == "alu" else byts / (ms * 1e-3)
        peak = alu_peak if bound == "alu" else HBM_PEAK
        unit = "TFLOP/s" if bound == "alu" else "GB/s"
    scale = 1e12 if unit == "TFLOP/s" else 1e9
    kname = "k_lr_kr" if dom == "lowrank_outer" else "k_lr_steps"
    roof = {"kernel": kname, "bound": bound,
            "achieved": achieved / scale, "peak": peak / scale, "unit": unit,
            "frac": achieved / peak,
            "traffic": measured_lowrank_traffic(kname, st["launches"]),
            "launches_per_step": st["launches"],
            "avg_launch_ms": ms / max(1, st["launches"]), "ms_per_step": ms,
            "flops_per_step": flops, "bytes_per_step": byts,
            "kernels": {kd: {"ms_per_step": v["ms"], "launches": v["launches"], "flops": v["flops"],
                             "bytes": v["bytes"]} for kd, v in kinds.items()}}
    info = {j: plans[j].lowrank_info(n, k, [0] * (2 * j - 3) + [1]) for j in orders}
    out = {"metric": "HOIF chain U-statistics, orders 2..7 at n=10000 from rank-8 panels, "
                     "steps/s (one step = all six orders)",
           "value": 1.0 / el, "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": warm,
           "ms_per_step": 1e3 * el, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64",
           "data": "synthetic: Z ~ U[0,1]^4, A ~ Bernoulli(expit(Z1+Z2-1)), Y = A + sum Z + N(0,1), "
                   "cosine dictionary of 8 functions, seed 11",
           "config": {"workload": "influence-function chains g..g f, orders 2-7, n=10000, rank 8, "
                                  "every partition (Bell(j)), low-rank panels",
                      "n": n, "rank": k, "orders": orders},
           "roofline": roof,
           "per_order": {str(j): {"ms": 1e3 * per[j], "U": res[j].value, "S": res[j].err_scale,
                                  "err_est": res[j].err_est, "num_vstats": res[j].num_vstats,
                                  "madds": info[j]["madds"], "steps": info[j]["num_steps"],
                                  "workspace_bytes": info[j]["workspace_bytes"],
                                  "paper_rtx5090_dense_s": HOIF_PAPER_GPU_S[j]}
                         for j in orders}}
    if not args.no_compare:
        # the same U-statistics through the dense path on n x n factors in fp64
        Tg = Pd @ Pd.T
        Tf = Pd @ Qd.T
        torch.cuda.synchronize()
        dense = {}
        for j in orders:
            fac = [Tg] * (j - 2) + [Tf]
            D = U.Plan(j, W.hoif_chain(j), precision="f64", order="exhaustive")
            D.eval(fac)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rdn = D.eval(fac)
            torch.cuda.synchronize()
            dense[str(j)] = {"ms": 1e3 * (time.perf_counter() - t1),
                             "diff_vs_lowrank_over_S": abs(rdn.value - res[j].value) / res[j].err_scale}
            print(f"hoif: dense order {j} {dense[str(j)]['ms']:.1f} ms", file=sys.stderr, flush=True)
            del D
        del Tg, Tf
        out["dense_f64_same_factors"] = dense
    if not args.no_cpu_baseline:
        # the oracle's cost is linear in n (one pass over the samples per
        # rank-index assignment): time it on the first ns rows, scale by n / ns
        ns = 3000
        Ps, Qs = np.ascontiguousarray(P[:ns]), np.ascontiguousarray(Q[:ns])
        t1 = time.perf_counter()
        for j in orders:
            F, G = W.hoif_factor_panels(j, Ps, Qs)
            oracle.ustat_lowrank(W.hoif_chain(j), F, G)
        t_s = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": 1.0 / (t_s * n / ns), "unit": "steps/s",
                               "cores": oracle.num_threads(), "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"subset dynamic programme over the first {ns} of {n} samples "
                                         f"for all six orders ({t_s:.1f} s), scaled by {n}/{ns} "
                                         "(its cost is linear in n)"}
    print(json.dumps(out))


def bench_learned_order(args):
    """Learned order choice, end to end.  64 random kernel graphs on 6
    vertices (6-10 edges, seed 5, draws with an isolated vertex rejected);
    graphs whose largest quotient treewidth M is 4 are skipped, M <= 2
    graphs run at n = 8192 and M = 3 graphs (conditioned steps, n^4 work)
    at n = 2048; x iid N(0, I_16), RBF divisor 32, split-bf16x3.  For each
    order policy the time is plan creation plus the first evaluation, and
    the U values of the policies must agree."""
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W
    graphs = W.random_kernel_graphs(64, 6, 6, 10, seed=5)
    lo, hi = (int(x) for x in args.graph_range.split(":"))
    policies = ["minfill", "exhaustive", "learned"]
    tot = {p: 0.0 for p in policies}
    per, skipped, worst = [], [], 0.0
    xs = {}
    for gi in range(lo, min(hi, len(graphs))):
        edges = graphs[gi]
        M = U.Plan(6, edges).info()["M"]
        if M > 3:
            skipped.append(gi)
            continue
        n = 8192 if M <= 2 else 2048
        if n not in xs:
            xs[n] = torch.tensor(W.gaussian_samples(n, 16, seed=50), dtype=torch.float64,
                                 device="cuda")
        rec = {"graph": gi, "M": M, "n": n}
        vals = {}
        for pol in policies:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = U.Plan(6, edges, precision="bf16x3", order=pol, n_hint=n)
            r = P.eval_samples(xs[n], 32.0)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            tot[pol] += el
            rec[pol + "_s"] = el
            vals[pol] = (r.value, r.err_scale)
            del P
        S = vals["minfill"][1]
        dev = max(abs(v[0] - vals["minfill"][0]) for v in vals.values()) / S
        worst = max(worst, dev)
        rec["max_policy_diff_over_S"] = dev
        per.append(rec)
        print(json.dumps(rec), file=sys.stderr, flush=True)
    out = {"metric": "end-to-end seconds (plan + eval) over the graphs, per order policy",
           "unit": "s", "higher_is_better": False,
           "config": {"workload": "64 random 6-vertex kernel graphs (6-10 edges, seed 5), "
                                  "203 restricted V-statistics each; n=8192 (M<=2) / 2048 (M=3), "
                                  "d=16, bf16x3", "graphs": f"{lo}:{hi}"},
           "value": tot["learned"], "totals_s": tot, "skipped_M4": skipped,
           "max_policy_diff_over_S": worst, "graphs_run": len(per), "per_graph": per}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "f32", "f64"])
    ap.add_argument("--order", default="exhaustive", choices=["minfill", "exhaustive"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--overlap-levels", action="store_true",
                    help="run a level's reductions on a second stream beside its GEMMs")
    ap.add_argument("--workload", default="cycle4",
                    choices=["cycle4", "batched", "cycle5-exact", "learned-order", "motifs", "hoif",
                             "peaks"],
                    help="cycle4: the headline line; the others print their own line")
    ap.add_argument("--graph-range", default="0:64",
                    help="learned-order workload: graphs lo:hi of the 64")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many plain steps (for external profilers)")
    ap.add_argument("--tuning", default=None, metavar="GEMM_BIG_MIN,COLRED_BLOCKS",
                    help="use these launch-shape settings instead of autotuning")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-mebibyte device buffer 4 times (the reference "
                         "kernel for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this engine has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "learned-order":
        # Switched off: one run of this workload after the symmetric stream-K
        # products and the other GEMM changes stopped on an illegal memory
        # access, and host-side checks of the schedules it builds (the
        # stream-K walk over whole slice chunks included) have not shown the
        # cause.  It stays off until one is found.
        print("bench.py: the learned-order workload is switched off: one run of it faulted the "
              "GPU and the cause has not been found (its last clean run: "
              "profiles/learned_order_e2e.json)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nb, "launches": 4}))
        return
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "cycle5-exact":
        return bench_cycle5_exact(args)
    if args.workload == "learned-order":
        return bench_learned_order(args)
    if args.workload == "motifs":
        return bench_motifs(args)
    if args.workload == "hoif":
        return bench_hoif(args)
    if args.workload == "peaks":
        return bench_peaks(args)
    m, edges, n, d = WORKLOAD["m"], WORKLOAD["edges"], WORKLOAD["n"], WORKLOAD["d"]
    div = 2.0 * d
    Xh = W.gaussian_samples(n, d, seed=WORKLOAD["seed"])
    X = torch.tensor(Xh, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    # symmetric: the same DAG as eval_samples builds for its RBF factor, so
    # that tuning on the factor matrix applies to the samples path
    plans = {p: U.Plan(m, edges, precision=p, order=args.order, symmetric=True,
                       overlap=args.overlap_levels)
             for p in ("bf16x3", "f32", "f64")}
    main_plan = plans[args.precision]
    if args.tuning:
        gb, cb = (int(v) for v in args.tuning.split(","))
        main_plan.set_tuning(gb, cb)
        tune_ms = None
    else:
        # autotuned launch shapes (outside the timed region)
        K = U.ustat_build_rbf(X, div, args.precision if args.precision != "bf16x3" else "f32")
        torch.cuda.synchronize()
        tune_ms = main_plan.autotune([K] * len(edges), stream=stream, reps=3)
        del K

    if args.profile_steps:
        for _ in range(args.profile_steps):
            r = main_plan.eval_samples(X, div, stream=stream)
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "value": r.value}))
        return

    elapsed, r = timed_evals(main_plan, X, div, args.steps, args.warmup, stream)
    value = args.steps / elapsed
    out = {"metric": "U-stat evals/s (m=4 4-cycle RBF kernel, n=4096, d=16)", "value": value,
           "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": {"bf16x3": "bf16x3-f32acc", "f32": "f32", "f64": "f64"}[args.precision],
           "data": "synthetic: X iid N(0, I_16), seed 2; factors built on the GPU",
           "config": {"workload": "4-cycle RBF U-statistic, m=4, n=4096, d=16, divisor 32, "
                                  "15 restricted V-statistics", "n": n, "d": d, "m": m,
                      "order": args.order, "precision": args.precision, "cse": True,
                      "second_stream": args.overlap_levels,
                      "num_vstats": r.num_vstats, "tuning": main_plan.tuning(),
                      "autotuned": tune_ms is not None}}
    # R = K K runs as a symmetric product on 256-wide tiles (n a multiple of
    # 256, 256-wide tiles chosen): t (t + 1) / 2 of the t^2 tiles are computed
    t = n // 256
    share = (t * (t + 1) / 2) / (t * t) if n % 256 == 0 and main_plan.tuning()["gemm_big_min"] <= t * t else 1.0
    dom, kr = kernel_rooflines(U, main_plan, X, div, stream, args.precision, executed_share=share)
    out["roofline"] = dict(kr[dom])
    out["roofline"]["dominant_kind"] = dom
    out["roofline_mfma_gemm"] = kr.get("gemm")
    out["kernels"] = kr
    if not args.no_compare:
        res = {}
        vals = {}
        for p in ("f64", "f32", "bf16x3"):
            steps = max(3, args.steps // (4 if p == "f64" else 2))
            el, rp = timed_evals(plans[p], X, div, steps, 2, stream)
            res[p] = {"evals_per_s": steps / el, "ms_per_eval": 1e3 * el / steps}
            vals[p] = rp
        S = vals["f64"].err_scale
        for p in res:
            res[p]["U"] = vals[p].value
            res[p]["err_vs_f64_over_S"] = abs(vals[p].value - vals["f64"].value) / S
        nc = U.Plan(m, edges, precision=args.precision, order=args.order, cse=False)
        steps = max(3, args.steps // 2)
        el, rnc = timed_evals(nc, X, div, steps, 2, stream)
        res["without_cse"] = {"evals_per_s": steps / el, "ms_per_eval": 1e3 * el / steps,
                              "err_vs_cse_over_S": abs(rnc.value - vals[args.precision].value) / S}
        res["speedup_bf16x3_over_f64"] = res["bf16x3"]["evals_per_s"] / res["f64"]["evals_per_s"]
        res["speedup_f32_over_f64"] = res["f32"]["evals_per_s"] / res["f64"]["evals_per_s"]
        res["S"] = S
        out["precision_comparison"] = res
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(Xh, div)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
