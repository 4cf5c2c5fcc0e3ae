"""Harvest elimination-order timings on the GPU and train the order cost model.

For random kernel graphs, a sample of each partition's executable orders
(plain, or conditioned on one vertex when the quotient has treewidth 3) is
evaluated with ``vstat_eval_ordered`` and timed end to end (host scheduling
plus device work, best of a few calls).  Each sample is (features of the
lowered order, log seconds).  The MLP (18 -> H1 -> H2 -> 1) is then trained
on the GPU by the engine's own forward/backward/Adam kernels and written as
a cost-model file for ``order="learned"`` plans.  The paper notes, after
its complexity proposition for V-statistics (section "The Algorithm of
Computing V-Statistics"), that finding the treewidth-optimal order is
NP-complete and that heuristic orders are used in practice; the model ranks
the executable candidates by measured cost instead.

    python -m paper_2508_12627_amd.costmodel_train --out costmodel.txt
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import time

import numpy as np


WIDTH_FEATURE = 11  # index of the elimination width in the feature vector


def candidates(U, h, block_of, n: int):
    """The executable (order, slice_var) pairs of partition block_of that
    reach the smallest width: plain orders that stay within degree 2, else
    (conditioned vertex, order of the others) pairs.  Host only."""
    J = 1 + max(block_of)
    out = []
    for perm in itertools.permutations(range(J)):
        try:
            f = U.ustat_order_features(h, block_of, perm, n)
        except U.UstatError:
            continue
        out.append((list(perm), -1, f[WIDTH_FEATURE]))
    if not out:
        for c in range(J):
            rest = [q for q in range(J) if q != c]
            for perm in itertools.permutations(rest):
                try:
                    f = U.ustat_order_features(h, block_of, perm, n, c)
                except U.UstatError:
                    continue
                out.append((list(perm), c, f[WIDTH_FEATURE]))
    if not out:
        return []
    w = min(x[2] for x in out)
    return [(o, c) for o, c, wx in out if wx == w]


def wall_seconds(U, h, block_of, order, slice_var, n, fs, repeats: int) -> float:
    """Best-of-repeats wall time of one ordered V-statistic evaluation (host
    scheduling and device work), after one untimed warm-up call."""
    import torch
    U.vstat_eval_ordered(h, block_of, order, n, fs, slice_var=slice_var)
    torch.cuda.synchronize()
    best = math.inf
    for _ in range(repeats):
        t0 = time.perf_counter()
        U.vstat_eval_ordered(h, block_of, order, n, fs, slice_var=slice_var)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def harvest(graphs, ns_plain, ns_sliced, partitions_per_graph: int, orders_per_partition: int,
            seed: int, precision: str = "bf16x3", repeats: int = 2, log=print,
            sliced_per_graph: int = 8):
    """Returns X (samples x NUM_FEATURES float32), y (log seconds, float32) and the
    sample records (graph, partition, candidate, n, seconds)."""
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W
    rng = np.random.default_rng(seed)
    feats, targets, recs = [], [], []
    kmats = {}
    for n in sorted(set(ns_plain) | set(ns_sliced)):
        X = torch.tensor(W.gaussian_samples(n, 16, seed=seed + n), dtype=torch.float64, device="cuda")
        kmats[n] = U.ustat_build_rbf(X, 32.0, "f64" if precision == "f64" else "f32")
    torch.cuda.synchronize()
    for gi, edges in enumerate(graphs):
        m = 1 + max(max(e) for e in edges)
        P = U.Plan(m, edges, precision=precision)
        idx = [i for i in range(P.info()["num_vstats"]) if max(P.partition(i)["block_of"]) + 1 >= 3]
        # plain and conditioned partitions sampled separately: the latter
        # are few per graph but carry most of the time of wide graphs
        plain = [i for i in idx if P.slice_var(i) < 0]
        cond = [i for i in idx if P.slice_var(i) >= 0]
        if len(plain) > partitions_per_graph:
            plain = rng.choice(plain, partitions_per_graph, replace=False).tolist()
        if len(cond) > sliced_per_graph:
            cond = rng.choice(cond, sliced_per_graph, replace=False).tolist()
        for i in sorted(plain + cond):
            blk = P.partition(i)["block_of"]
            cands = candidates(U, P.h, blk, 1024)
            mf = (P.order(i), P.slice_var(i))
            if len(cands) > orders_per_partition:
                pick = rng.choice(len(cands), orders_per_partition, replace=False).tolist()
                cands = [cands[k] for k in sorted(pick)]
            if mf not in cands:
                cands.append(mf)
            sliced = cands[0][1] >= 0
            for n in (ns_sliced if sliced else ns_plain):
                fs = [kmats[n]] * len(edges)
                for order, sv in cands:
                    f = U.ustat_order_features(P.h, blk, order, n, sv)
                    t = wall_seconds(U, P.h, blk, order, sv, n, fs, repeats)
                    feats.append(f)
                    targets.append(math.log(max(t, 1e-7)))
                    recs.append({"graph": gi, "part": i, "order": order, "slice_var": sv, "n": n,
                                 "seconds": t})
        log(f"harvest graph {gi + 1}/{len(graphs)}: {len(targets)} samples", flush=True)
    return np.array(feats, dtype=np.float32), np.array(targets, dtype=np.float32), recs


def init_params(F: int, H1: int, H2: int, X, seed: int):
    """Standardisation from the data, He-normal weights (seeded)."""
    from paper_2508_12627_amd import ustat as U
    rng = np.random.default_rng(seed)
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    istd = np.where(std > 1e-6, 1.0 / np.maximum(std, 1e-6), 0.0)
    parts = [mean, istd,
             rng.normal(0, math.sqrt(2.0 / F), H1 * F), np.zeros(H1),
             rng.normal(0, math.sqrt(2.0 / H1), H2 * H1), np.zeros(H2),
             rng.normal(0, math.sqrt(1.0 / H2), H2), np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == U.ustat_mlp_num_params(F, H1, H2)
    return p


def compare_policies(graphs, n_for, model_path, precision: str = "bf16x3", max_candidates: int = 32,
          repeats: int = 2, seed: int = 0, log=print):
    """Brute-force comparison of the order policies.  For every partition of every
    graph with at least two executable candidates, times a sample of at most
    max_candidates candidates plus the picks of the min-fill, exhaustive
    (cost proxy) and learned policies, all at n = n_for(M) for the graph's
    largest quotient treewidth M.  Returns one record per partition."""
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W
    rng = np.random.default_rng(seed)
    kmats, recs = {}, []
    for gi, edges in enumerate(graphs):
        m = 1 + max(max(e) for e in edges)
        Pm = U.Plan(m, edges, precision=precision, order="minfill")
        n = int(n_for(Pm.info()["M"]))
        if n not in kmats:
            X = torch.tensor(W.gaussian_samples(n, 16, seed=seed + n), dtype=torch.float64,
                             device="cuda")
            kmats[n] = U.ustat_build_rbf(X, 32.0, "f64" if precision == "f64" else "f32")
            torch.cuda.synchronize()
        fs = [kmats[n]] * len(edges)
        Pe = U.Plan(m, edges, precision=precision, order="exhaustive", n_hint=n)
        Pl = U.Plan(m, edges, precision=precision, order="learned", cost_model_path=model_path,
                    n_hint=n)
        for i in range(Pm.info()["num_vstats"]):
            blk = Pm.partition(i)["block_of"]
            if max(blk) + 1 < 3:
                continue
            cands = [(tuple(o), sv) for o, sv in candidates(U, Pm.h, blk, n)]
            if len(cands) < 2:
                continue
            picks = {name: (tuple(P.order(i)), P.slice_var(i))
                     for name, P in (("minfill", Pm), ("exhaustive", Pe), ("learned", Pl))}
            if len(cands) > max_candidates:
                sel = rng.choice(len(cands), max_candidates, replace=False).tolist()
                cands = [cands[k] for k in sorted(sel)]
            pool = list(dict.fromkeys(cands + list(picks.values())))
            times = {c: wall_seconds(U, Pm.h, blk, list(c[0]), c[1], n, fs, repeats) for c in pool}
            rec = {"graph": gi, "part": i, "n": n, "candidates": len(pool),
                   "best": min(times.values())}
            for name, c in picks.items():
                rec[name] = times[c]
            recs.append(rec)
        log(f"policies graph {gi + 1}/{len(graphs)}: {len(recs)} partitions", flush=True)
    return recs


def policies_summary(recs, margin: float = 0.05) -> dict:
    """Totals over all compared partitions and over those where the best
    measured order beats min-fill by more than margin."""
    out = {}
    for name, sel in (("all", recs),
                      ("improvable", [r for r in recs if r["best"] < (1 - margin) * r["minfill"]])):
        out[name] = {"partitions": len(sel)}
        for k in ("best", "minfill", "exhaustive", "learned"):
            out[name][k + "_s"] = float(sum(r[k] for r in sel))
    return out


def _mse(a, b):
    return float(np.mean((np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) ** 2))


def fit(X, y, H1=64, H2=64, steps=3000, lr=2e-3, seed=0, holdout=0.2):
    """Train on the GPU; returns params and a summary with held-out MSE."""
    from paper_2508_12627_amd import ustat as U
    rng = np.random.default_rng(seed)
    N, F = X.shape
    perm = rng.permutation(N)
    nte = max(1, int(holdout * N))
    te, tr = perm[:nte], perm[nte:]
    p0 = init_params(F, H1, H2, X[tr], seed)
    base_te = _mse(np.full(nte, float(np.mean(y[tr]))), y[te])
    p, losses = U.ustat_mlp_train(F, H1, H2, p0, X[tr], y[tr], steps=steps, lr=lr)
    pred = U.ustat_mlp_predict(F, H1, H2, p, X[te])
    summary = {"samples": int(N), "train_loss_first": float(losses[0]),
               "train_loss_last": float(losses[-1]), "heldout_mse": _mse(pred, y[te]),
               "heldout_mse_constant_predictor": base_te, "H1": H1, "H2": H2, "steps": steps}
    return p, summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--graphs", type=int, default=16)
    ap.add_argument("--sizes", default="1024,2048,4096")
    ap.add_argument("--sliced-sizes", default="512,1024,2048")
    ap.add_argument("--sliced-partitions", type=int, default=8)
    ap.add_argument("--partitions", type=int, default=12)
    ap.add_argument("--orders", type=int, default=6)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--data-out", default=None)
    ap.add_argument("--compare-policies", default=None, metavar="LO:HI",
                    help="compare the policies on graphs LO:HI of the learned-order workload "
                         "(64 random 6-vertex graphs, seed 5) with the model --out, at "
                         "n = 2048 (M <= 2) / 512 (M = 3), instead of training")
    ap.add_argument("--compare-candidates", type=int, default=16)
    args = ap.parse_args()
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W
    torch.cuda.set_device(0)
    if args.compare_policies:
        lo, hi = (int(x) for x in args.compare_policies.split(":"))
        graphs = [e for e in W.random_kernel_graphs(64, 6, 6, 10, seed=5)[lo:hi]
                  if U.Plan(6, e).info()["M"] <= 3]
        recs = compare_policies(graphs, lambda M: 2048 if M <= 2 else 512, args.out,
                     max_candidates=args.compare_candidates, repeats=3)
        summary = policies_summary(recs)
        summary.update({"graphs": f"{lo}:{hi}", "model": os.path.basename(args.out)})
        if args.data_out:
            with open(args.data_out, "w") as f:
                json.dump(recs, f)
        print(json.dumps(summary))
        return
    # kernel graphs on 4, 5 and 6 vertices (6-10 edges on 6 vertices, as the
    # learned-order workload draws them), quotient treewidth at most 3
    graphs = []
    per_m = {4: args.graphs // 4, 5: args.graphs // 4}
    per_m[6] = args.graphs - per_m[4] - per_m[5]
    for m, cnt in per_m.items():
        lo, hi = (6, 10) if m == 6 else (m, min(10, m * (m - 1) // 2 - 1))
        pool = W.random_kernel_graphs(8 * cnt + 8, m, lo, hi, seed=args.seed + m)
        picked = [e for e in pool if U.Plan(m, e).info()["M"] <= 3][:cnt]
        graphs.extend(picked)
    t0 = time.time()
    X, y, recs = harvest(graphs, [int(s) for s in args.sizes.split(",")],
                         [int(s) for s in args.sliced_sizes.split(",")], args.partitions,
                         args.orders, args.seed, sliced_per_graph=args.sliced_partitions)
    t1 = time.time()
    p, summary = fit(X, y, steps=args.steps, seed=args.seed)
    U.ustat_mlp_save(args.out, X.shape[1], summary["H1"], summary["H2"], p)
    if args.data_out:
        np.savez(args.data_out, X=X, y=y)
        with open(args.data_out + ".json", "w") as f:
            json.dump(recs, f)
    summary.update({"graphs": len(graphs), "harvest_s": t1 - t0, "train_s": time.time() - t1,
                    "out": args.out})
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
