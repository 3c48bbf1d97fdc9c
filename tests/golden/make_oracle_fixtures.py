"""Write the oracle's results for the large parity cases to tests/golden/ (compressed npz).

The oracle needs minutes for the 512 x 512 grids (a Python loop over ~22000 boxes), too
long to rerun inside every GPU test session, so its outputs are stored once.  This script
calls only the oracle and the seeded input generators; nothing here comes from the HIP
path.  Regenerate with

    python tests/golden/make_oracle_fixtures.py [name ...]

Each file holds, for the 2D Laplace grid problem of its name (cell-centre grid, leaf size,
tolerance, 16 proxies at 1.25 box sides, FP64):
  * the skeleton / redundant sets of every box of every skeletonized level
    (Section 3.1 eq. skelid; Algorithm 1),
  * the top set B_t (Section 3.3),
  * x = F^{-1} b and y = F b for b = rhs(N, seed 0) (Section 3.3),
  * (sign, log|det F|) (Section 3.3),
  * the full records (T, X_RR, X_JR = E X_RR, G, J) of one interior box of the last colour
    of every level (Section 3.1 eqs. zab, skelop).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import rss_oracle as O  # noqa: E402
from paper_1609_08130_amd import workloads as W  # noqa: E402

CASES = {
    # 16384 leaves of 16 points: ~1820 boxes per colour at depth 7, ~455 at depth 6
    "grid512_leaf16_tol1e-6": dict(n=512, leaf=16, tol=1e-6),
    # the 512 x 512 workload itself (leaf 64): ~455 boxes per colour at its leaves
    "grid512_leaf64_tol1e-6": dict(n=512, leaf=64, tol=1e-6),
}


def path_of(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.npz")


def record_sample(F, nb_of_depth):
    """One interior box of the last colour (8) per level: its blocks have seen the Schur
    updates of all eight earlier colours."""
    out = {}
    for r in F.records:
        nb = nb_of_depth[r.depth]
        bx, by = r.box % nb, r.box // nb
        if O.colour(r.box, nb) != 8 or not (2 <= bx < nb - 2 and 2 <= by < nb - 2):
            continue
        if r.depth not in out:
            out[r.depth] = r
    return [out[d] for d in sorted(out, reverse=True)]


def make(name: str) -> str:
    c = CASES[name]
    n = c["n"]
    pts = W.grid_points(n)
    prm = W.problem(n, c["tol"], leaf_size=c["leaf"])
    p = O.Params(**prm)
    t0 = time.perf_counter()
    F = O.factor(pts, p)
    t1 = time.perf_counter()
    b = W.rhs(n * n, seed=0)
    x = O.solve(F, b)
    y = O.apply(F, b)
    sg, ld = O.logdet(F)
    sk_t, sk_box, sk_ns, sk_nr, sk_idx = [], [], [], [], []
    for (t, box), (S, R) in F.skeletons.items():
        sk_t.append(t)
        sk_box.append(box)
        sk_ns.append(len(S))
        sk_nr.append(len(R))
        sk_idx.append(np.asarray(S, dtype=np.int32))
        sk_idx.append(np.asarray(R, dtype=np.int32))
    nb_of_depth = {t: 2 ** t for t in range(F.depth + 1)}
    recs = record_sample(F, nb_of_depth)
    arrays = dict(
        depth=np.int32(F.depth), top=np.asarray(F.top, dtype=np.int32),
        sk_t=np.asarray(sk_t, dtype=np.int32), sk_box=np.asarray(sk_box, dtype=np.int32),
        sk_ns=np.asarray(sk_ns, dtype=np.int32), sk_nr=np.asarray(sk_nr, dtype=np.int32),
        sk_idx=np.concatenate(sk_idx) if sk_idx else np.zeros(0, np.int32),
        x=x, y=y, logdet=np.array([sg, ld]),
        rec_depth=np.array([r.depth for r in recs], dtype=np.int32),
        rec_box=np.array([r.box for r in recs], dtype=np.int32),
    )
    for i, r in enumerate(recs):
        arrays[f"rec{i}_T"] = r.T
        arrays[f"rec{i}_XRR"] = r.XRR
        arrays[f"rec{i}_XJR"] = r.E @ r.XRR
        arrays[f"rec{i}_G"] = r.G
        arrays[f"rec{i}_J"] = np.asarray(r.J, dtype=np.int32)
    meta = dict(case=name, problem={k: (list(v) if isinstance(v, tuple) else v) for k, v in prm.items()},
                rhs="workloads.rhs(N, seed=0)", oracle_factor_seconds=round(t1 - t0, 1),
                levels=F.level_stats)
    arrays["meta_json"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    out = path_of(name)
    np.savez_compressed(out, **arrays)
    print(f"{name}: oracle factor {t1 - t0:.1f} s, depth {F.depth}, {len(F.records)} records, "
          f"top {len(F.top)} -> {out} ({os.path.getsize(out) / 1e6:.2f} MB)", flush=True)
    return out


def load(name: str) -> dict:
    z = np.load(path_of(name), allow_pickle=False)
    d = {k: z[k] for k in z.files}
    d["meta"] = json.loads(bytes(d.pop("meta_json")).decode())
    sk = {}
    off = 0
    for t, box, ns, nr in zip(d["sk_t"], d["sk_box"], d["sk_ns"], d["sk_nr"]):
        S = d["sk_idx"][off:off + ns].astype(np.int64)
        R = d["sk_idx"][off + ns:off + ns + nr].astype(np.int64)
        off += ns + nr
        sk[(int(t), int(box))] = (S, R)
    d["skeletons"] = sk
    d["records"] = [dict(depth=int(d["rec_depth"][i]), box=int(d["rec_box"][i]), T=d[f"rec{i}_T"],
                         XRR=d[f"rec{i}_XRR"], XJR=d[f"rec{i}_XJR"], G=d[f"rec{i}_G"],
                         J=d[f"rec{i}_J"].astype(np.int64)) for i in range(len(d["rec_depth"]))]
    return d


if __name__ == "__main__":
    from threadpoolctl import threadpool_limits
    names = sys.argv[1:] or list(CASES)
    with threadpool_limits(limits=1):
        for nm in names:
            make(nm)
