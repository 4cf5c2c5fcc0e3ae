"""Harvest elimination-order timings on the GPU and train the order cost model.

For random kernel graphs, every partition's candidate elimination orders are
evaluated with ``vstat_eval_ordered`` and timed with the engine's kernel
events (device time of all launches).  Each sample is (features of the
lowered order, log seconds).  The MLP (15 -> H1 -> H2 -> 1) is then trained
on the GPU by the engine's own forward/backward/Adam kernels and written as
a cost-model file for ``order="learned"`` plans.

    python -m paper_2508_12627_amd.costmodel_train --out costmodel.txt
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import time

import numpy as np


def candidate_orders(J: int, limit: int, rng) -> list:
    perms = list(itertools.permutations(range(J)))
    if len(perms) <= limit:
        return [list(p) for p in perms]
    idx = rng.choice(len(perms), size=limit, replace=False)
    return [list(perms[i]) for i in sorted(idx)]


def device_seconds(U) -> float:
    tot = 0.0
    for k in U.PROFILE_KINDS:
        tot += U.ustat_profile_read(k)["ms"]
    return tot * 1e-3


def harvest(graphs, ns, partitions_per_graph: int, orders_per_partition: int, seed: int,
            precision: str = "bf16x3", repeats: int = 2, log=print):
    """Returns X (samples x 15 float32) and y (log seconds, float32)."""
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W
    rng = np.random.default_rng(seed)
    feats, targets = [], []
    U.ustat_profile_enable(True)
    for n in ns:
        X = torch.tensor(W.gaussian_samples(n, 16, seed=seed + n), dtype=torch.float64, device="cuda")
        K = U.ustat_build_rbf(X, 32.0, "f64" if precision == "f64" else "f32")
        torch.cuda.synchronize()
        for gi, edges in enumerate(graphs):
            m = 1 + max(max(e) for e in edges)
            P = U.Plan(m, edges, precision=precision)
            parts = [p for p in P.partitions() if max(p["block_of"]) + 1 >= 3]
            if len(parts) > partitions_per_graph:
                parts = [parts[i] for i in sorted(rng.choice(len(parts), partitions_per_graph,
                                                             replace=False))]
            fs = [K] * len(edges)
            for p in parts:
                J = max(p["block_of"]) + 1
                for order in candidate_orders(J, orders_per_partition, rng):
                    try:
                        f = U.ustat_order_features(P.h, p["block_of"], order, n)
                    except U.UstatError:
                        continue  # needs a step of degree above 2
                    best = math.inf
                    for _ in range(repeats):
                        U.ustat_profile_reset()
                        U.vstat_eval_ordered(P.h, p["block_of"], order, n, fs)
                        best = min(best, device_seconds(U))
                    feats.append(f)
                    targets.append(math.log(max(best, 1e-7)))
            log(f"harvest n={n} graph {gi + 1}/{len(graphs)}: {len(targets)} samples")
    U.ustat_profile_enable(False)
    return np.array(feats, dtype=np.float32), np.array(targets, dtype=np.float32)


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
    ap.add_argument("--sizes", default="512,1024,2048,4096")
    ap.add_argument("--partitions", type=int, default=24)
    ap.add_argument("--orders", type=int, default=8)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--data-out", default=None)
    args = ap.parse_args()
    import torch
    from paper_2508_12627_amd import ustat as U, workloads as W
    torch.cuda.set_device(0)
    graphs = []
    per_m = {4: args.graphs // 4, 5: args.graphs // 2}
    per_m[6] = args.graphs - per_m[4] - per_m[5]
    for m, cnt in per_m.items():
        pool = W.random_kernel_graphs(8 * cnt + 8, m, m, min(10, m * (m - 1) // 2 - 1),
                                      seed=args.seed + m)
        picked = [e for e in pool if U.Plan(m, e).info()["M"] <= 2][:cnt]
        graphs.extend(picked)
    t0 = time.time()
    X, y = harvest(graphs, [int(s) for s in args.sizes.split(",")], args.partitions, args.orders,
                   args.seed)
    t1 = time.time()
    p, summary = fit(X, y, steps=args.steps, seed=args.seed)
    U.ustat_mlp_save(args.out, X.shape[1], summary["H1"], summary["H2"], p)
    if args.data_out:
        np.savez(args.data_out, X=X, y=y)
    summary.update({"graphs": len(graphs), "harvest_s": t1 - t0, "train_s": time.time() - t1,
                    "out": args.out})
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
