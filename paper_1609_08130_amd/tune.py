"""Autotuner of the launch plans (paper_1609_08130_amd/csrc/tuned_plans.inc).

The kernels of one colour choose their launch plan from a table indexed by the colour's box
count (buckets with lower bounds 1, 64, 256, 512, 1024 boxes).  This script measures the
candidates on the GPU: for one field at a time it factors the 2D Laplace grid workload with
every candidate value (set through RSS_TUNE for all buckets at once), reads the per-level
phase times the library reports (rss_info: ID, elimination and Schur time per level; the solve's
time for the sweep widths, one bucket at a time), assigns each level to the bucket of its
largest colour, and keeps per bucket the fastest value; fields are tuned in order, each
with the best values found so far.  It then writes the table and a JSON summary.

    python -m paper_1609_08130_amd.tune [--n 1024] [--tols 1e-6] [--reps 3] [--out csrc/tuned_plans.inc]

With several tolerances (--tols 1e-3,1e-6,1e-9) every candidate is measured at each, and a
bucket's score is the sum over tolerances of its phase time divided by the same bucket's
time with the starting table at that tolerance, so each tolerance weighs the same.
Buckets that no level of the workload falls into keep their previous values.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

BUCKET_LO = [1, 64, 256, 512, 1024]
FIELDS = ["gram_many", "gram_min_wg", "pchol_kc", "elim_tpw", "elim_tw", "inv_threads", "sweep_threads", "gram_i8", "schur_atomic",
          "schur_form"]
# the order in which the fields are tuned (the Gram kernel first: it decides the slicing)
ORDER = ["gram_i8", "gram_many", "gram_min_wg", "pchol_kc", "elim_tpw", "elim_tw", "inv_threads", "sweep_threads",
         "schur_atomic", "schur_form"]
DEFAULTS = [
    [0, 2048, 0, 1, 16, 1024, 1024, 0, 0, 0],
    [0, 2048, 0, 1, 16, 1024, 1024, 0, 0, 0],
    [0, 2048, 0, 1, 16, 256, 256, 0, 0, 0],
    [1, 2048, 16, 1, 16, 256, 256, 0, 0, 0],
    [1, 2048, 16, 4, 16, 256, 256, 0, 0, 0],
]
# candidate values and the phase each field is judged by
CANDIDATES = {
    "gram_many": ([0, 1], "id"),
    "gram_min_wg": ([1024, 2048, 4096, 8192], "id"),
    "pchol_kc": ([0, 8, 16, 32], "id"),
    "elim_tpw": ([1, 2, 4], "elim"),
    "elim_tw": ([8, 16, 32], "elim"),
    "inv_threads": ([256, 1024], "elim"),
    "sweep_threads": ([256, 1024], "solve"),
    "gram_i8": ([0, 1], "id"),
    "schur_atomic": ([0, 1], "schur"),
    "schur_form": ([0, 1], "schur"),
}


def bucket_of(nboxes: int) -> int:
    b = 0
    while b + 1 < len(BUCKET_LO) and nboxes >= BUCKET_LO[b + 1]:
        b += 1
    return b


def level_bucket(depth: int) -> int:
    nb = 2 ** depth
    return bucket_of(((nb + 2) // 3) ** 2)   # the largest colour of the 3 x 3 colouring


def env_of(table):
    return ",".join(f"b{b}.{f}={table[b][i]}" for b in range(len(table)) for i, f in enumerate(FIELDS))


def measure(rss, torch, W, n, tol, table, reps, solves=0):
    """Median per-level ID, elimination and Schur times (ms) by (depth, pass) and the median solve time."""
    os.environ["RSS_TUNE"] = env_of(table)
    prm = W.problem(n, tol)
    prm.pop("dim")
    pts = torch.tensor(W.grid_points(n), device="cuda")
    per = {}
    solve_ms = None
    for _ in range(reps):
        F = rss.Factor(pts, precision="mixed", **prm)
        info = F.info()
        for lv in info["levels"]:
            key = (lv["depth"], lv.get("pass", "strong"))
            per.setdefault(key, []).append((lv["ms_id"], lv["ms_elim"], lv["ms_schur"]))
        if solves:
            b = torch.tensor(W.rhs(n * n, seed=0), device="cuda")
            F.solve(b, use_fp32=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(solves):
                F.solve(b, use_fp32=True)
            torch.cuda.synchronize()
            solve_ms = (time.perf_counter() - t0) * 1e3 / solves
        F.close()
    med = {k: tuple(statistics.median(v[i] for v in vals) for i in range(3)) for k, vals in per.items()}
    return med, solve_ms


def combine(per_tol, base_tol):
    """Per bucket: sum over tolerances of time / the starting table's time (each tolerance
    weighs the same); per_tol and base_tol map tolerance -> {bucket: ms}."""
    out = {}
    for tol, per_bucket in per_tol.items():
        for b, t in per_bucket.items():
            ref = base_tol.get(tol, {}).get(b, 0.0)
            out[b] = out.get(b, 0.0) + (t / ref if ref > 0 else t)
    return out


def bucket_times(med, idx):
    """Phase idx (0 ID, 1 elimination, 2 Schur) summed per bucket of the levels."""
    per_bucket = {}
    for (d, p), t in med.items():
        per_bucket[level_bucket(d)] = per_bucket.get(level_bucket(d), 0.0) + t[idx]
    return per_bucket


def write_table(path, table, note):
    rows = ",\n".join("    {" + ", ".join(str(v) for v in row) + "}" for row in table)
    text = (f"// Launch-plan table, one row per bucket of boxes per colour (lower bounds kPlanBucketLo).\n"
            f"// Fields: {', '.join(FIELDS)}.\n"
            f"// Written by paper_1609_08130_amd/tune.py: {note}\n"
            f"const int kPlanBucketLo[kPlanBuckets] = {{{', '.join(str(b) for b in BUCKET_LO)}}};\n"
            f"static const PlanParams kPlanTable[kPlanBuckets] = {{\n{rows},\n}};\n")
    with open(path, "w") as fh:
        fh.write(text)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--tol", type=float, default=None, help="one tolerance (same as --tols T)")
    ap.add_argument("--tols", default="1e-6", help="comma-separated tolerances, weighed equally")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--solves", type=int, default=20)
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "tuned_plans.inc"))
    ap.add_argument("--summary", default=None)
    args = ap.parse_args()
    import torch

    from paper_1609_08130_amd import rss
    from paper_1609_08130_amd import workloads as W
    tols = [args.tol] if args.tol is not None else [float(t) for t in args.tols.split(",")]
    table = [list(r) for r in DEFAULTS]
    base_by_tol = {}
    base_phase = {}   # tolerance -> phase index -> {bucket: ms} with the starting table
    for tol in tols:
        base_by_tol[tol] = measure(rss, torch, W, args.n, tol, table, args.reps, args.solves)
        base_phase[tol] = {i: bucket_times(base_by_tol[tol][0], i) for i in range(3)}
    base, base_solve = base_by_tol[tols[0]]
    used = sorted({level_bucket(d) for tol in tols for d, _ in base_by_tol[tol][0]})
    log = {"n": args.n, "tols": tols, "reps": args.reps, "buckets_used": used, "baseline_solve_ms": base_solve,
           "baseline": {f"{d}/{p}": v for (d, p), v in base.items()}, "steps": []}
    print(f"[tune] tolerances {tols}; baseline solve {base_solve:.3f} ms; levels {sorted(base)}", flush=True)
    for field in ORDER:
        fi = FIELDS.index(field)
        cands, phase = CANDIDATES[field]
        if phase == "solve":
            for b in used:
                best_v, best_t = table[b][fi], None
                for v in cands:
                    trial = [list(r) for r in table]
                    trial[b][fi] = v
                    t = 0.0
                    for tol in tols:
                        _, ts = measure(rss, torch, W, args.n, tol, trial, 1, args.solves)
                        t += ts / base_by_tol[tol][1]
                    log["steps"].append({"field": field, "bucket": b, "value": v, "solve_score": t})
                    print(f"[tune] {field} bucket {b} = {v}: solve score {t:.4f}", flush=True)
                    if best_t is None or t < best_t:
                        best_v, best_t = v, t
                table[b][fi] = best_v
            continue
        idx = {"id": 0, "elim": 1, "schur": 2}[phase]
        results = {}
        for v in cands:
            trial = [list(r) for r in table]
            for b in range(len(trial)):
                trial[b][fi] = v
            per_tol = {}
            for tol in tols:
                med, _ = measure(rss, torch, W, args.n, tol, trial, args.reps)
                per_tol[tol] = bucket_times(med, idx)
            results[v] = combine(per_tol, {tol: base_phase[tol][idx] for tol in tols})
            log["steps"].append({"field": field, "value": v, "phase": phase,
                                 "ms_by_tol_bucket": {str(tol): {str(b): round(t, 4) for b, t in pb.items()}
                                                      for tol, pb in per_tol.items()},
                                 "score_by_bucket": {str(b): round(t, 4) for b, t in results[v].items()}})
            print(f"[tune] {field} = {v}: {phase} score by bucket "
                  f"{ {b: round(t, 4) for b, t in sorted(results[v].items())} }", flush=True)
        for b in used:
            table[b][fi] = min(cands, key=lambda v: results[v].get(b, float("inf")))
    final, final_solve = measure(rss, torch, W, args.n, tols[0], table, args.reps, args.solves)
    log["table"] = table
    log["final_solve_ms"] = final_solve
    log["final"] = {f"{d}/{p}": v for (d, p), v in final.items()}
    sid = lambda m: sum(v[0] for v in m.values())
    sel = lambda m: sum(v[1] for v in m.values())
    ssc = lambda m: sum(v[2] for v in m.values())
    print(f"[tune] ID {sid(base):.3f} -> {sid(final):.3f} ms, elimination {sel(base):.3f} -> {sel(final):.3f} ms, "
          f"Schur {ssc(base):.3f} -> {ssc(final):.3f} ms, solve {base_solve:.3f} -> {final_solve:.3f} ms", flush=True)
    write_table(args.out, table, f"{args.n}x{args.n} grid, tol {', '.join(f'{t:g}' for t in tols)}, mixed "
                f"precision, median of {args.reps} factorizations per candidate")
    if args.summary:
        with open(args.summary, "w") as fh:
            json.dump(log, fh, indent=1)
    print(json.dumps({"table": table}), flush=True)


if __name__ == "__main__":
    main()
