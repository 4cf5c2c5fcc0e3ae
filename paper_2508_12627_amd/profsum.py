"""Summaries of rocprofv3 results (its SQLite output) for the engine's kernels.

    python -m paper_2508_12627_amd.profsum kernels RESULTS.db
        per-kernel calls, total and average duration (kernel trace)
    python -m paper_2508_12627_amd.profsum traffic --fetch F.db --write W.db \\
        --cal-fetch CF.db --cal-write CW.db --cal-bytes B --kernel NAME [--out T.json]
        [--path dense|lowrank] [--meta KEY=VALUE ...]
        HBM bytes per launch of the kernels whose name contains NAME, from
        FETCH_SIZE and WRITE_SIZE runs, each scaled by what the same counter
        reads for a plain device copy of B bytes (the calibration runs)
    python -m paper_2508_12627_amd.profsum mfma RESULTS.db [--md OUT.md ...]
        per-kernel MFMA busy fraction, SQ_VALU_MFMA_BUSY_CYCLES over
        (GRBM_GUI_ACTIVE / 8 XCDs) x 1024 SIMDs, and the LDS bank-conflict
        rate SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE (a --pmc run)

The traffic record carries a hash of the kernel sources, so a reader can
tell whether the counters still describe the current kernels.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# Device code outside the dense evaluation path that traffic records cover:
# the cost-model network and the low-rank path (which has its own records).
_OTHER_PATHS = ("mlp.hip", "k_lowrank.hip")


def kernel_sources():
    """Every device-code source of the dense evaluation path: the kernel
    translation units and the headers they include."""
    d = os.path.join(HERE, "csrc")
    names = sorted(f for f in os.listdir(d)
                   if f.endswith(".hip") or f in ("kernels.hpp", "kdev.hpp") or f.endswith("_impl.hpp"))
    return [os.path.join(d, f) for f in names if f not in _OTHER_PATHS]


def lowrank_sources():
    """Device code of the low-rank path: its kernels and the descriptor
    header they include."""
    d = os.path.join(HERE, "csrc")
    return [os.path.join(d, f) for f in ("k_lowrank.hip", "lowrank.hpp")]


def kernel_source_hash(path: str = "dense") -> str:
    """Hash of the device sources of one evaluation path ("dense" or
    "lowrank")."""
    h = hashlib.sha256()
    for p in (lowrank_sources() if path == "lowrank" else kernel_sources()):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """Kernel name without its argument list (and without the anonymous
    namespace qualifier, whose parentheses would cut it short)."""
    return name.replace("(anonymous namespace)::", "").split("(")[0]


def kernel_stats(db: str):
    """[(name, calls, total_us, average_us, percent)] from a kernel trace."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels").fetchall()
    con.close()
    # the view reports microseconds
    return [(n, int(c), float(t), float(a), float(p)) for n, c, t, a, p in rows]


def dispatch_resources(db: str):
    """[(name, grid, workgroup, lds, vgpr, agpr, scratch)] for the first
    dispatch of each kernel."""
    con = sqlite3.connect(db)
    try:
        rows = con.execute("select name, grid_x, workgroup_x, lds_size, vgpr_count, "
                           "accum_vgpr_count, scratch_size from kernels order by start").fetchall()
    except sqlite3.Error:
        rows = []
    con.close()
    seen, out = set(), []
    for r in rows:
        if r[0] in seen:
            continue
        seen.add(r[0])
        out.append(r)
    return out


def counter_per_dispatch(db: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter."""
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, dispatch_id, value from counters_collection "
                       "where counter_name = ?", (counter,)).fetchall()
    con.close()
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for k, disp, v in rows:
        per[k][disp] += v
    return {k: list(d.values()) for k, d in per.items()}


def _mean(v):
    return sum(v) / len(v) if v else 0.0


SIMDS = 256 * 4   # MI355X: 256 compute units of 4 SIMDs
XCDS = 8          # GRBM_GUI_ACTIVE is summed over the 8 XCDs


def mfma_busy(db: str):
    """[(kernel, dispatches, mfma_busy_fraction, active_us, lds_conflict_rate)]
    from a --pmc run with SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE (and
    optionally SQ_LDS_BANK_CONFLICT, SQ_LDS_IDX_ACTIVE)."""
    busy = counter_per_dispatch(db, "SQ_VALU_MFMA_BUSY_CYCLES")
    gui = counter_per_dispatch(db, "GRBM_GUI_ACTIVE")
    conf = counter_per_dispatch(db, "SQ_LDS_BANK_CONFLICT")
    lds = counter_per_dispatch(db, "SQ_LDS_IDX_ACTIVE")
    out = []
    for k in sorted(gui):
        g = _mean(gui[k]) / XCDS
        b = _mean(busy.get(k, []))
        act = _mean(lds.get(k, []))
        rate = _mean(conf.get(k, [])) / act if act else None
        out.append((k, len(gui[k]), b / (g * SIMDS) if g else 0.0, g / 2.4e3, rate))
    return out


def traffic(fetch_db, write_db, cal_fetch_db, cal_write_db, cal_bytes, kernel, path="dense"):
    """Per-launch HBM bytes of the matching kernels, calibrated on a copy."""
    cf = counter_per_dispatch(cal_fetch_db, "FETCH_SIZE")
    cw = counter_per_dispatch(cal_write_db, "WRITE_SIZE")
    # the copy kernel is the one that moved the most bytes
    cf_kib = max((_mean(v) for v in cf.values()), default=0.0)
    cw_kib = max((_mean(v) for v in cw.values()), default=0.0)
    fs = cal_bytes / (cf_kib * 1024.0) if cf_kib else None
    ws = cal_bytes / (cw_kib * 1024.0) if cw_kib else None
    f = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    w = counter_per_dispatch(write_db, "WRITE_SIZE")
    out = {"calibration": {"copy_bytes": cal_bytes, "fetch_kib": cf_kib, "write_kib": cw_kib,
                           "fetch_scale": fs, "write_scale": ws},
           "source_hash": kernel_source_hash(path), "path": path, "kernels": {}}
    for name in sorted(set(f) | set(w)):
        if kernel not in name:
            continue
        fk, wk = _mean(f.get(name, [])), _mean(w.get(name, []))
        out["kernels"][name] = {
            "launches": max(len(f.get(name, [])), len(w.get(name, []))),
            "fetch_kib_raw": fk, "write_kib_raw": wk,
            "fetch_bytes": fk * 1024.0 * fs if fs else None,
            "write_bytes": wk * 1024.0 * ws if ws else None,
            "bytes_per_launch": (fk * 1024.0 * fs + wk * 1024.0 * ws) if fs and ws else None}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--md", default=None, help="also write a markdown summary here")
    k.add_argument("--title", default="kernel trace")
    k.add_argument("--command", default="", help="the rocprofv3 command that made the trace")
    k.add_argument("--note", default="")
    t = sub.add_parser("traffic")
    for a in ("--fetch", "--write", "--cal-fetch", "--cal-write"):
        t.add_argument(a, required=True)
    t.add_argument("--cal-bytes", type=float, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--path", default="dense", choices=["dense", "lowrank"],
                   help="whose device sources the record's hash covers")
    t.add_argument("--out", default=None)
    t.add_argument("--meta", action="append", default=[], metavar="KEY=VALUE",
                   help="extra fields of the record (workload, precision, command)")
    mf = sub.add_parser("mfma")
    mf.add_argument("db")
    mf.add_argument("--md", default=None)
    mf.add_argument("--title", default="MFMA busy")
    mf.add_argument("--command", default="")
    mf.add_argument("--note", default="")
    args = ap.parse_args(argv)
    if args.cmd == "mfma":
        rows = mfma_busy(args.db)
        lines = ["| kernel | dispatches | MFMA busy | active us (2.4 GHz) | LDS conflict rate |",
                 "|---|---|---|---|---|"]
        for k, nd, f, us, rate in rows:
            r = "-" if rate is None else f"{rate:.4f}"
            lines.append(f"| `{short_name(k)}` | {nd} | {f:.3f} | {us:.1f} | {r} |")
        print("\n".join(lines))
        if args.md:
            with open(args.md, "w") as f:
                f.write(f"# {args.title}\n\n")
                if args.command:
                    f.write("Command (from the repository root on the MI355X host):\n\n")
                    f.write(f"    {args.command}\n\n")
                if args.note:
                    f.write(args.note + "\n\n")
                f.write("\n".join(lines) + "\n")
        return 0
    if args.cmd == "kernels":
        stats = kernel_stats(args.db)
        print(f"{'kernel':<70} {'calls':>6} {'total_us':>11} {'avg_us':>9} {'pct':>6}")
        for n, c, tot, avg, pct in stats:
            print(f"{n[:70]:<70} {c:>6} {tot:>11.1f} {avg:>9.2f} {pct:>6.2f}")
        if args.md:
            with open(args.md, "w") as f:
                f.write(f"# {args.title}\n\n")
                if args.command:
                    f.write("Command (from the repository root on the MI355X host):\n\n")
                    f.write(f"    {args.command}\n\n")
                if args.note:
                    f.write(args.note + "\n\n")
                f.write("Durations in microseconds (rocprofv3 kernel trace).\n\n")
                f.write("| kernel | calls | total_us | avg_us | pct |\n|---|---|---|---|---|\n")
                for n, c, tot, avg, pct in stats:
                    f.write(f"| `{short_name(n)}` | {c} | {tot:.1f} | {avg:.2f} | {pct:.2f} |\n")
                res = dispatch_resources(args.db)
                if res:
                    f.write("\nPer-dispatch resources (first dispatch of each kernel):\n\n")
                    f.write("| kernel | grid | workgroup | lds | vgpr | agpr | scratch |\n"
                            "|---|---|---|---|---|---|---|\n")
                    for r in res:
                        f.write("| `" + short_name(r[0]) + "` | " + " | ".join(str(x) for x in r[1:]) + " |\n")
        return 0
    rec = traffic(args.fetch, args.write, args.cal_fetch, args.cal_write, args.cal_bytes,
                  args.kernel, args.path)
    for kv in args.meta:
        k, _, v = kv.partition("=")
        rec[k] = v
    text = json.dumps(rec, indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
