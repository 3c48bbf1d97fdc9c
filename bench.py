"""Benchmark: RS-S factor + solve of the 2D Laplace second-kind system on one MI355X.

A step = rss_factor_create (points resident in HBM -> factor ready, tree included)
followed by the refined solve of A x = b: FP64 GMRES with F^{-1} as right
preconditioner and the exact operator applied by FFT, to a relative residual of 1e-10;
then rss_factor_destroy.  The headline runs the mixed-precision factor (FP32 Schur
products, FP32 factor copy for the preconditioner); the FP64 factor is timed on the same
inputs for comparison.  Solves/s (plain x = F^{-1} b) are timed separately.

Prints one JSON line.  `roofline` is computed for the dominant kernel of the factor (the Schur update k_schur)
from the library's own HIP events (recorded on the launch stream around every launch of
the timed steps) and the algorithmic flop / byte counts of the realized box sizes;
`traffic` is the HBM bytes per launch measured with rocprofv3 counters (committed summary
under profiles/, null once the kernel source differs from the one measured).
`cpu_baseline` times the oracle on bounded samples of the same workload (corner sub-grids
with the same h, weight, leaf size and tolerance) at two sizes with one thread and with
every host core, and scales the cheapest per DOF linearly in N (the method's cost is linear
in N, Corollary 2; the two sizes show it on the host).  `e_a` is |A - F| / |A| by the power
method (Section 4) and `solve_roofline` the solve's algorithmic HBM bytes over its time.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1609_08130_amd import workloads as W  # noqa: E402

KEYS = ("ms_per_step", "factor_ms", "gmres_ms", "gmres_iters", "gmres_relres", "solve_ms", "solves_per_s",
        "solve8_ms", "rhs_per_s_nrhs8", "finv_f_err", "e_a", "solve_roofline")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6        # MI355X FP64 (vector and matrix)
FP32_PEAK_TFS = 157.3       # MI355X FP32 (vector and matrix)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024, help="grid side (N = n^2)")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--solves", type=int, default=100, help="solves timed for solves/s")
    ap.add_argument("--rtol", type=float, default=1e-10, help="GMRES relative residual target")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=256)
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: mixed factor + solve only, no baselines")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run only a device-to-device copy of MIB MiB (HBM counter calibration)")
    return ap.parse_args()


SCHUR_SRC = os.path.join(ROOT, "paper_1609_08130_amd", "csrc", "rss_schur.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_schur_grid1024_tol1e-6_hbm_counters.md")


def measured_traffic():
    """HBM bytes per k_schur launch from the committed counter summary, or None when the
    kernel source changed after the counters were taken (its SHA-256 is recorded there)."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        line = line.strip().strip("`")
        if "=" in line and not line.startswith("|"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    try:
        want = vals["source_sha256"]
        traffic = float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
    have = hashlib.sha256(open(SCHUR_SRC, "rb").read()).hexdigest()
    return traffic if have == want else None


def dominant_roofline(infos: list, mixed: bool) -> dict:
    """Roofline of k_schur, the factor kernel with the largest total time in the rocprofv3
    trace of this workload.  Durations come from the library's HIP events around every
    k_schur launch of the timed steps (on the launch stream); bytes and flops are the
    algorithmic counts of the realized |J| and |R| of every box."""
    t_ms = sum(i["phase_ms"]["schur"] for i in infos)
    nl = max(sum(i["launches"]["schur"] for i in infos), 1)
    byts = sum(sum(l["bytes_schur"] for l in i["levels"]) for i in infos)
    flops = sum(sum(l["flops_schur"] for l in i["levels"]) for i in infos)
    avg_ms = t_ms / nl
    ai = flops / byts
    peak_f = FP32_PEAK_TFS if mixed else FP64_PEAK_TFS
    ridge = peak_f * 1e12 / (HBM_PEAK_GBS * 1e9)
    traffic = measured_traffic()
    common = dict(kernel="k_schur<float, float>" if mixed else "k_schur<double, double>", launches=nl,
                  avg_launch_ms=avg_ms,
                  algorithmic_bytes_per_launch=byts / nl, algorithmic_flops_per_launch=flops / nl,
                  arithmetic_intensity=ai)
    if ai < ridge:
        ach = (byts / nl) / (avg_ms / 1e3) / 1e9
        return dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                    traffic=traffic, **common)
    ach = (flops / nl) / (avg_ms / 1e3) / 1e12
    return dict(bound="mfma", achieved=ach, peak=peak_f, unit="TFLOP/s", frac=ach / peak_f, traffic=traffic,
                **common)


def schur_level_roofline(l):
    """Schur update of one level against its attainable roofline: achieved flop rate over
    min(FP32 vector peak, arithmetic intensity x HBM peak), and over the FP32 peak alone
    (mixed factors multiply in FP32 on the vector units)."""
    ms = l["ms_schur"]
    if ms <= 0 or l["bytes_schur"] <= 0:
        return {}
    tflops = l["flops_schur"] / (ms / 1e3) / 1e12
    ai = l["flops_schur"] / l["bytes_schur"]
    attain = min(FP32_PEAK_TFS, ai * HBM_PEAK_GBS / 1e3)
    return {"schur_tflops": round(tflops, 3), "schur_ai": round(ai, 3),
            "schur_frac_attainable": round(tflops / attain, 4), "schur_frac_peak": round(tflops / FP32_PEAK_TFS, 4)}


def run_gpu(args, precision: str):
    import torch

    from paper_1609_08130_amd import rss
    n = args.n
    prm = W.problem(n, args.tol)
    prm.pop("dim")
    pts = torch.tensor(W.grid_points(n), device="cuda")
    b = torch.tensor(W.rhs(n * n, seed=0), device="cuda")
    use32 = precision == "mixed"
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        F = rss.Factor(pts, precision=precision, **prm)
        F.gmres(b, rtol=args.rtol, maxit=50, use_fp32=use32)
        torch.cuda.synchronize()
        F.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, gm = [], []
    for _ in range(args.steps):
        tf0 = time.perf_counter()
        F = rss.Factor(pts, precision=precision, **prm)
        tf1 = time.perf_counter()
        x, it, rr = F.gmres(b, rtol=args.rtol, maxit=50, use_fp32=use32)
        torch.cuda.synchronize()
        tf2 = time.perf_counter()
        gm.append((tf2 - tf1, it, rr))
        infos.append(F.info())
        F.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # separate solve rate on one factor
    F = rss.Factor(pts, precision=precision, **prm)
    info = F.info()
    x = F.solve(b, use_fp32=use32)
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(args.solves):
        x = F.solve(b, use_fp32=use32)
    e.record()
    torch.cuda.synchronize()
    solve_ms = s.elapsed_time(e) / args.solves
    # eight right-hand sides in one call (column-major N x 8)
    B8 = torch.stack([torch.tensor(W.rhs(n * n, seed=q), device="cuda") for q in range(8)], dim=1)
    B8 = B8.t().contiguous().t()
    F.solve(B8, use_fp32=use32)
    torch.cuda.synchronize()
    s.record()
    for _ in range(max(1, args.solves // 5)):
        F.solve(B8, use_fp32=use32)
    e.record()
    torch.cuda.synchronize()
    solve8_ms = s.elapsed_time(e) / max(1, args.solves // 5)
    # accuracy of the factor as an approximate inverse: F^{-1} applied to F x
    y = F.apply(b)
    z = F.solve(y, use_fp32=use32)
    inv_err = float(torch.linalg.norm(z - b) / torch.linalg.norm(b))
    e_a = approximation_error(F, n * n, torch)
    F.close()
    factor_ms = statistics.median(i["phase_ms"]["total"] for i in infos)
    return dict(precision=precision, ms_per_step=ms_step, factor_ms=factor_ms, solve_ms=solve_ms,
                solves_per_s=1e3 / solve_ms, solve8_ms=solve8_ms, rhs_per_s_nrhs8=8e3 / solve8_ms, info=info,
                infos=infos, finv_f_err=inv_err, e_a=e_a, solve_roofline=solve_roofline(info, solve_ms, use32, n * n),
                gmres_ms=statistics.median(g[0] for g in gm) * 1e3, gmres_iters=gm[-1][1], gmres_relres=gm[-1][2])


def run_level_graphs(args, stream_infos):
    """The mixed factorization with every level pass launched as one HIP graph
    (level_graphs = 1; the thread's executable graphs are updated in place from the second
    factorization on): median factor time and the time of the passes at depth <= 5 (the
    levels with at most 121 boxes per colour), against the same quantities of the
    kernel-by-kernel factorizations timed above."""
    import torch

    from paper_1609_08130_amd import rss
    n = args.n
    prm = W.problem(n, args.tol)
    prm.pop("dim")
    pts = torch.tensor(W.grid_points(n), device="cuda")
    infos = []
    for rep in range(args.warmup + args.steps):
        F = rss.Factor(pts, precision="mixed", level_graphs=1, **prm)
        if rep >= args.warmup:
            infos.append(F.info())
        F.close()
    torch.cuda.synchronize()

    def upper(info, key):
        return sum(key(l) for l in info["levels"] if l["depth"] <= 5)

    stream_pass = lambda l: l["ms_id"] + l["ms_elim"] + l["ms_schur"] + l["ms_schur_self"]
    return dict(factor_ms=statistics.median(i["phase_ms"]["total"] for i in infos),
                factor_ms_stream=statistics.median(i["phase_ms"]["total"] for i in stream_infos),
                passes_ms=statistics.median(i["phase_ms"]["level_graphs"] for i in infos),
                passes_ms_stream=statistics.median(sum(stream_pass(l) for l in i["levels"]) for i in stream_infos),
                upper_levels_ms=statistics.median(upper(i, lambda l: l["ms_graph"]) for i in infos),
                upper_levels_ms_stream=statistics.median(upper(i, stream_pass) for i in stream_infos))


def approximation_error(F, N, torch):
    """e_a = |A - F| / |A| by the power method to 1e-2 relative (Section 4), on the
    operators themselves (A symmetric, F symmetric up to its approximation error)."""
    gen = torch.Generator(device="cpu").manual_seed(1)
    x0 = torch.randn(N, generator=gen, dtype=torch.float64).cuda()

    def power(op):
        v = x0 / torch.linalg.norm(x0)
        lam = 0.0
        for _ in range(50):
            w = op(v)
            lam_new = float(torch.linalg.norm(w))
            v = w / lam_new
            if abs(lam_new - lam) <= 1e-2 * lam_new:
                return lam_new
            lam = lam_new
        return lam
    return power(lambda v: F.matvec(v) - F.apply(v)) / power(F.matvec)


def solve_roofline(info, solve_ms, use32, N):
    """The solve streams the factor once: per record 2|J||R| (X_JR, G) + 2|S||R| (T, read in
    both sweeps) + |R|^2 (X_RR^{-1}) entries, the top block's inverse, and the right-hand
    side in and the solution out (16 N bytes); HBM-bound."""
    key = "bytes_solve32" if use32 else "bytes_solve64"
    byts = sum(l[key] for l in info["levels"]) + (4 if use32 else 8) * info["n_top"] ** 2 + 16.0 * N
    ach = byts / (solve_ms / 1e3) / 1e9
    return dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                algorithmic_bytes=byts, ms=solve_ms)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """The oracle (plain numpy FP64) on corner sub-grids of the workload (same h, weight,
    leaf size, tolerance and proxies): factor + GMRES-refined solve at two sizes with one
    BLAS thread (the cost per DOF is constant, Corollary 2: the two sizes show it on this
    host), and at the larger size with every core; the faster of the two thread counts gives
    the value, scaled linearly to N."""
    from threadpoolctl import threadpool_limits

    from oracle import rss_oracle as O
    n = args.n
    h = 1.0 / n

    def run(m, threads):
        c = (np.arange(m) + 0.5) * h
        pts = np.empty((m * m, 2))
        pts[:, 0] = np.tile(c, m)
        pts[:, 1] = np.repeat(c, m)
        p = O.Params(weight=h * h, tol=args.tol, leaf_size=64, n_proxy=16, proxy_radius=1.25,
                     root_lo=(0.0, 0.0), root_side=m * h)
        b = W.rhs(m * m, seed=0)
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            F = O.factor(pts, p)
            t1 = time.perf_counter()
            _, its, rr = O.gmres(lambda v: O.matvec_grid_fft(m, p, v, h=h), lambda v: O.solve(F, v), b,
                                 rtol=args.rtol)
            t2 = time.perf_counter()
        return dict(m=m, threads=threads, factor_s=t1 - t0, solve_s=t2 - t1, step_s=t2 - t0, iters=its,
                    relres=rr, us_per_dof=(t2 - t0) / (m * m) * 1e6)

    m1 = min(args.cpu_sample_n, n)
    m0 = max(m1 // 2, 8)
    nproc = os.cpu_count() or 1
    runs = [run(m0, 1), run(m1, 1)]
    if nproc > 1:
        # every core at the smaller size first: many BLAS threads on the oracle's small
        # blocks can be slower than one; the larger size with every core only if not
        runs.append(run(m0, nproc))
        if runs[2]["step_s"] < runs[0]["step_s"]:
            runs.append(run(m1, nproc))
    best = min((r for r in runs if r["m"] == m1), key=lambda r: r["step_s"])
    scale = (n * n) / (best["m"] ** 2)
    step_s = best["step_s"] * scale
    desc = "; ".join(f"{r['m']}x{r['m']} ({r['m'] * r['m']} DOFs), {r['threads']} thread(s): factor "
                     f"{r['factor_s']:.2f} s + refined solve {r['solve_s']:.3f} s ({r['iters']} iterations) = "
                     f"{r['us_per_dof']:.1f} us/DOF" for r in runs)
    return dict(value=1.0 / step_s, unit="factor+refined-solve/s", cores=best["threads"], kind="oracle",
                sample=f"oracle factor + GMRES-refined solve (rtol {args.rtol:g}) on corner sub-grids of the "
                       f"{n}x{n} workload (same h=1/{n}, weight, leaf 64, tol {args.tol}, 16 proxies); the faster "
                       f"run at the larger size scaled linearly by N/{best['m'] ** 2} = {scale:.0f} (cost per DOF "
                       f"constant, Corollary 2: compare the two one-thread sizes); {desc}; "
                       f"numpy FP64 on {cpu_model()}, {nproc} cores visible",
                cpu_model=cpu_model(), nproc=nproc, runs=runs,
                factor_s_scaled=best["factor_s"] * scale, solve_s_scaled=best["solve_s"] * scale)


def copy_calibration(mib: int):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.profile:
        args.steps, args.warmup, args.solves = 1, 0, 1
        args.no_fp64 = True
        args.no_cpu_baseline = True
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 (multi-GPU sharding is a "
                                   "design note, not implemented)"}))
        sys.exit(2)
    mixed = run_gpu(args, "mixed")
    fp64 = None if args.no_fp64 else run_gpu(args, "fp64")
    graphs = None if args.profile else run_level_graphs(args, mixed["infos"])
    roof = dominant_roofline(mixed["infos"], True)
    out = {
        "metric": "RS-S factor s + solves/s, N=1M 2D Laplace ε=1e-6, mixed vs FP64, one GPU",
        "value": 1e3 / mixed["ms_per_step"],
        "unit": "factor+refined-solve/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"laplace2d_grid{args.n}_tol{args.tol:g}", "n": args.n * args.n,
                   "leaf_size": 64, "tol": args.tol, "n_proxy": 16, "proxy_radius": 1.25,
                   "precision": "mixed", "parallelism": "none"},
        "factor_s": mixed["factor_ms"] / 1e3,
        "solves_per_s": mixed["solves_per_s"],
        "mixed": {k: mixed[k] for k in KEYS},
        "fp64": None if fp64 is None else {k: fp64[k] for k in KEYS},
        "phase_ms_mixed": mixed["info"]["phase_ms"],
        "phase_ms_fp64": None if fp64 is None else fp64["info"]["phase_ms"],
        "level_graphs": graphs,
        "roofline": roof,
        "levels": [dict({k: (round(l[k], 3) if isinstance(l[k], float) else l[k])
                         for k in ("depth", "boxes", "nmax", "records", "sum_k", "max_k", "max_J", "ms_id", "ms_elim",
                                   "ms_schur")}, **schur_level_roofline(l))
                   for l in mixed["info"]["levels"]],
        "n_top": mixed["info"]["n_top"],
        "bytes_device": mixed["info"]["bytes_device"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
