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


def gemm_roofline(U, plan, X, div, stream, prec, reps=3):
    """Per-launch GEMM durations from HIP events recorded on the launch
    stream (kernel-by-kernel launches, no graph)."""
    U.ustat_profile_enable(True)
    U.ustat_profile_reset()
    for _ in range(reps):
        plan.eval_samples(X, div, stream=stream)
    g = U.ustat_profile_read("gemm")
    others = {k: U.ustat_profile_read(k) for k in ("prep", "elim1", "reduce", "rbf")}
    U.ustat_profile_enable(False)
    achieved = g["flops"] / (g["ms"] * 1e-3)
    return {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAKS[prec] / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAKS[prec], "traffic": None,
            "kernel": f"k_gemm<{prec}>", "launches": g["launches"],
            "avg_launch_ms": g["ms"] / max(1, g["launches"]),
            "flops_per_launch": g["flops"] / max(1, g["launches"]),
            "executed_frac": achieved * (3 if prec == "bf16x3" else 1) / PEAKS[prec],
            "other_kernels_ms_per_eval": {k: v["ms"] / reps for k, v in others.items()},
            "gemm_ms_per_eval": g["ms"] / reps}


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
    return {"value": frac / t, "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"brute-force sum over distinct ordered 4-tuples restricted to the first "
                      f"{items} (i0, i1) prefixes of {n * n} at n={n} ({t:.1f} s), scaled by "
                      f"the prefix fraction"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "f32", "f64"])
    ap.add_argument("--order", default="exhaustive", choices=["minfill", "exhaustive"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many plain steps (for external profilers)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this engine has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W

    torch.cuda.set_device(0)
    m, edges, n, d = WORKLOAD["m"], WORKLOAD["edges"], WORKLOAD["n"], WORKLOAD["d"]
    div = 2.0 * d
    Xh = W.gaussian_samples(n, d, seed=WORKLOAD["seed"])
    X = torch.tensor(Xh, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    plans = {p: U.Plan(m, edges, precision=p, order=args.order) for p in ("bf16x3", "f32", "f64")}
    main_plan = plans[args.precision]

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
                      "num_vstats": r.num_vstats}}
    out["roofline"] = gemm_roofline(U, main_plan, X, div, stream, args.precision)
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
