"""Writes full_size_oracle.json: the oracle's results on selected queries of the
full-size workloads (100,000 edge-edge; 1,000,000 simulation-shaped; the four
1,000,000-query minimum-separation runs), as per-class SHA-256 digests plus a
few stored results for diagnostics.  Only the oracle (Alg. 2 replayed on the
CPU) and the seeded input generators are called.

Selections (class codes of the generators):
  * edge-edge, 100,000 queries: every degenerate query (classes 2-7: parallel,
    coplanar, touching at t = 0 / t = 1, static, endpoint-on-edge; the parallel
    and coplanar ones run to the m_I = 1e6 cap) and 2,000 generic ones;
  * simulation-shaped, 1,000,000 queries: every near-contact (class 8) and
    grazing-contact (class 9) query and 5,000 generic ones;
  * minimum separation (d in {1e-4, 1e-3} x delta in {1e-6, 1e-4}): 150
    near-contact, 150 grazing, 300 band (pairs within 2 d) and 300 generic
    queries per run (under minimum separation the near and grazing pairs run
    to the cap: about 0.5 s each in the oracle).

Run:  python tests/golden/make_full_size.py [--procs 8]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "full_size_oracle.json")
MAX_ITER = 1_000_000


def digest(r: dict) -> str:
    """SHA-256 over the five result arrays in query order (floats as bits)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(r["toi"], dtype=np.float64).view(np.uint64).tobytes())
    h.update(np.ascontiguousarray(r["t_width"], dtype=np.float64).view(np.uint64).tobytes())
    h.update(np.ascontiguousarray(r["n_checks"]).astype(np.uint64).tobytes())
    h.update(np.ascontiguousarray(r["hit"]).astype(np.uint8).tobytes())
    h.update(np.ascontiguousarray(r["status"]).astype(np.uint8).tobytes())
    return h.hexdigest()


def workload(spec: dict) -> dict:
    from paper_2009_13349_amd import workloads as W
    fn = getattr(W, spec["fn"])
    return fn(**spec["args"])


def _solve(args):
    import oracle
    pos, kind, delta, min_sep = args
    r = oracle.solve_batch(pos, kind, delta=delta, max_iter=MAX_ITER, min_sep=min_sep)
    return {k: r[k] for k in ("toi", "t_width", "n_checks", "hit", "status")}


def solve_parallel(pool, w, idx, delta, min_sep, chunk=16):
    parts = [idx[i:i + chunk] for i in range(0, len(idx), chunk)]
    args = [(np.ascontiguousarray(w["pos"][:, p]), np.ascontiguousarray(w["kind"][p]), delta, min_sep)
            for p in parts]
    res = pool.map(_solve, args, chunksize=1)
    return {k: np.concatenate([r[k] for r in res]) for k in ("toi", "t_width", "n_checks", "hit", "status")}


def cases():
    ee = {"fn": "edge_edge_mixed", "args": {"n": 100_000, "seed": 1}}
    sim = {"fn": "simulation_mixed", "args": {"n": 1_000_000, "seed": 2}}
    out = []
    for c in range(2, 8):
        out.append({"workload": ee, "delta": 1e-6, "min_sep": 0.0, "class": c, "take": "all"})
    out.append({"workload": ee, "delta": 1e-6, "min_sep": 0.0, "class": [0, 1], "take": 2000})
    for c in (8, 9):
        out.append({"workload": sim, "delta": 1e-6, "min_sep": 0.0, "class": c, "take": "all"})
    out.append({"workload": sim, "delta": 1e-6, "min_sep": 0.0, "class": 0, "take": 5000})
    for d in (1e-4, 1e-3):
        for delta in (1e-6, 1e-4):
            ms = {"fn": "min_separation", "args": {"n": 1_000_000, "seed": 2, "d_min": d, "delta": delta}}
            for c, k in ((8, 150), (9, 150), (10, 300), (0, 300)):
                out.append({"workload": ms, "delta": delta, "min_sep": d, "class": c, "take": k})
    return out


def select(w: dict, case: dict, salt: int) -> np.ndarray:
    cls = case["class"] if isinstance(case["class"], list) else [case["class"]]
    idx = np.nonzero(np.isin(w["cls"], cls))[0]
    if case["take"] != "all" and len(idx) > case["take"]:
        rng = np.random.default_rng(1000 + salt)
        idx = np.sort(rng.choice(idx, size=case["take"], replace=False))
    return idx


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    import oracle
    oracle.lib()  # builds the oracle library once, before the workers load it
    ctx = mp.get_context("spawn")
    records = []
    cache = {}
    t0 = time.time()
    with ctx.Pool(args.procs) as pool:
        for salt, case in enumerate(cases()):
            key = json.dumps(case["workload"], sort_keys=True)
            if key not in cache:
                cache.clear()
                cache[key] = workload(case["workload"])
            w = cache[key]
            idx = select(w, case, salt)
            t = time.time()
            r = solve_parallel(pool, w, idx, case["delta"], case["min_sep"])
            keep = np.arange(min(8, len(idx)))
            rec = dict(case)
            rec.update(
                name=w["name"], indices=idx.tolist() if case["take"] != "all" else None,
                count=int(len(idx)), sha256=digest(r), hits=int(r["hit"].sum()),
                capped=int(np.count_nonzero(r["status"] & 1)),
                sample=[{"q": int(idx[i]), "toi": float(r["toi"][i]).hex(),
                         "t_width": float(r["t_width"][i]).hex(), "n_checks": int(r["n_checks"][i]),
                         "hit": int(r["hit"][i]), "status": int(r["status"][i])} for i in keep],
                salt=salt)
            records.append(rec)
            print(f"[{time.time() - t0:7.1f}s] {w['name']} class {case['class']}: {len(idx)} queries "
                  f"in {time.time() - t:.1f}s, {rec['hits']} hits, {rec['capped']} capped", flush=True)
    json.dump({"max_iter": MAX_ITER, "cases": records}, open(OUT, "w"), indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
