"""Benchmark of the MI355X CCD root finder.

One step = one ccd_batch call over the whole workload (all queries resident in
HBM before the timed region), i.e. the complete root finder for every query:
root pass (level 0 of every query), lane engine, group engine and block engine.  Default
workload: 1,000,000 simulation-shaped queries (60% vertex-face, 40%
edge-edge, 2% near-contacts, 1% grazing contacts), delta = 1e-6, m_I = 1e6,
no minimum separation.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CCD queries/s at delta=1e-6 (persistent vs plain kernel); p50/p99 serve latency"
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X: 256 CUs x 2.4 GHz x 128 FP64 FLOP/clk (FMA = 2)
FLOP_PER_CHECK = {0: 227.0, 1: 177.0}  # vertex-face, edge-edge box check (binary64 add/sub/mul)
KERNELS = ("root", "lane", "group", "block")


def make_workload(name: str, n: int | None):
    from paper_2009_13349_amd import workloads as W
    if name == "simulation":
        return W.simulation_mixed(n or 1_000_000, seed=2)
    if name == "edge_edge":
        return W.edge_edge_mixed(n or 100_000, seed=1)
    if name == "uniform_vf":
        return W.uniform_vf(n or 4096, seed=0)
    raise SystemExit(f"unknown workload {name}")


def run_engine(ctx, torch, pos, kind, w, engine, steps, warmup, timing=True, t_max=1.0):
    from paper_2009_13349_amd import ccd
    ctx.set_engine(engine)
    ctx.enable_timing(timing)
    out = None
    kw = dict(delta=w["delta"], max_iter=w["max_iter"], min_sep=w["min_sep"], t_max=t_max)
    for _ in range(warmup):
        out = ctx.batch_device(pos, kind, out=out, **kw)
        ctx.last_stats()
    torch.cuda.synchronize()
    per_step = []
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.batch_device(pos, kind, out=out, **kw)
        if timing:
            stats.append(ctx.last_stats())  # synchronises; reads the per-kernel HIP events
        per_step.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    del ccd
    return (t1 - t0), stats, out


def roofline(stats, kind_counts):
    """Dominant kernel (largest device time) and its achieved FP64 rate:
    algorithmic FLOPs (box checks executed by that kernel x FLOPs per check)
    per launch / average launch duration from HIP events."""
    ms = np.array([s["kernel_ms"] for s in stats])  # [steps, 4]
    avg = ms.mean(axis=0)
    k = int(np.argmax(avg[1:])) + 1
    tier = k - 1
    checks = np.array([s["checks"][tier] for s in stats], dtype=np.float64).mean(axis=0)
    flops = checks[0] * FLOP_PER_CHECK[0] + checks[1] * FLOP_PER_CHECK[1]
    achieved = flops / (avg[k] * 1e-3) / 1e12
    return {
        "bound": "alu",
        "kernel": KERNELS[k],
        "achieved": round(achieved, 3),
        "peak": FP64_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 5),
        "traffic": None,
        "avg_launch_ms": round(float(avg[k]), 4),
        "checks_per_launch": [int(checks[0]), int(checks[1])],
        "kernel_ms_avg": {KERNELS[i]: round(float(avg[i]), 4) for i in range(4)},
    }


def kernel_symbol(tier: int, tuning: dict) -> str:
    if tier == 0:
        return "ccd::k_lane<true>"
    if tier == 2:
        return "ccd::k_group<8, 1>"
    gw = tuning["group_waves"]
    return f"ccd::k_group<{gw}, {tuning['group_occupancy'] if gw == 1 else 1}>"


def hbm_record(symbol: str):
    """Per-launch HBM bytes {fetch_bytes, write_bytes} (FETCH_SIZE, WRITE_SIZE,
    copy-calibrated) recorded under profiles/ for these exact kernel sources,
    else None."""
    from paper_2009_13349_amd.rocprof_summary import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    k = rec["kernels"].get(symbol)
    if not k or k.get("fetch_bytes") is None or k.get("write_bytes") is None:
        return None
    return k


def hbm_traffic(symbol: str):
    k = hbm_record(symbol)
    return k["fetch_bytes"] + k["write_bytes"] if k else None


def query_streaming(stats, n: int):
    """The root pass reads every query's 24 coordinates and its kind once:
    its read rate against the 8 TB/s HBM peak."""
    ms = float(np.mean([s["kernel_ms"][0] for s in stats]))
    bytes_in = n * (24 * 8 + 1)
    gbps = bytes_in / (ms * 1e-3) / 1e9
    k = hbm_record("ccd::k_root")
    return {"kernel": "root", "algorithmic_bytes_read": bytes_in, "avg_launch_ms": round(ms, 4),
            "gbps": round(gbps, 1), "frac_of_hbm_peak": round(gbps / 8000.0, 3),
            "measured_read_bytes": round(k["fetch_bytes"]) if k else None}


def cpu_baseline(w, seconds: float):
    """The oracle (single thread, as it stands) on a seeded random sample of
    the same workload, scaled to queries/s."""
    import oracle
    from paper_2009_13349_amd import workloads as W
    n = w["pos"].shape[1]
    rng = np.random.default_rng(1234)
    perm = rng.permutation(n)
    done, t_used, chunk = 0, 0.0, 2000
    while t_used < seconds and done < n:
        idx = perm[done:done + chunk]
        ws = W.subset(w, idx)
        t0 = time.perf_counter()
        oracle.solve_batch(ws["pos"], ws["kind"], delta=w["delta"], max_iter=w["max_iter"],
                           min_sep=w["min_sep"])
        t_used += time.perf_counter() - t0
        done += len(idx)
    return {"value": round(done / t_used, 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} queries drawn uniformly at random (seed 1234) from the same "
                      f"{n}-query workload, single-threaded C++ oracle, {t_used:.1f} s"}


def serve_latency(w, torch, q_sat: float, requests: int, payloads: int = 64, load: float = 0.7,
                  seed: int = 4, streams: int = 2):
    """Poisson stream of requests (sizes log-uniform in [1e3, 1e6], delta
    log-uniform in [1e-6, 1e-4]) at `load` x the measured batch throughput,
    submitted to the continuous-batching server; latency = scheduled arrival ->
    results in the caller's arrays.  Request payloads are contiguous pinned
    slices of the benchmark workload (a fixed set of `payloads` of them,
    reused round robin)."""
    import math
    from paper_2009_13349_amd import ccd
    rng = np.random.default_rng(seed)
    N = w["pos"].shape[1]
    sizes = np.round(np.exp(rng.uniform(math.log(1e3), math.log(1e6), size=payloads))).astype(int)
    pay = []
    for n in sizes:
        off = int(rng.integers(0, N - n + 1))
        pos = torch.from_numpy(np.ascontiguousarray(w["pos"][:, off:off + n])).pin_memory()
        kind = torch.from_numpy(np.ascontiguousarray(w["kind"][off:off + n])).pin_memory()
        pay.append((int(n), pos, kind))
    mean_n = float(np.mean(sizes))
    lam = load * q_sat / mean_n  # requests per second
    gaps = rng.exponential(1.0 / lam, size=requests)
    deltas = np.exp(rng.uniform(math.log(1e-6), math.log(1e-4), size=requests))
    srv = ccd.Server(streams=streams, pool_bytes=16 << 30, scratch_bytes=12 << 30,
                     max_queries_per_launch=4_000_000)
    # warm-up: one request of each payload size, not timed
    for n, pos, kind in pay[:4]:
        srv.wait(srv.submit(pos, kind, delta=1e-6), 600_000)
    t0 = time.monotonic() + 0.05
    arrivals = t0 + np.cumsum(gaps)
    tickets = []
    for i in range(requests):
        dt = arrivals[i] - time.monotonic()
        if dt > 0:
            time.sleep(dt)
        n, pos, kind = pay[i % payloads]
        tickets.append((srv.submit(pos, kind, delta=float(deltas[i])), arrivals[i], n))
    lat, t_end, qsum = [], 0.0, 0
    for t, arr, n in tickets:
        srv.wait(t, 600_000)
        info = srv.info(t)
        lat.append(info["t_done"] - arr)
        t_end = max(t_end, info["t_done"])
        qsum += n
    st = srv.stats()
    srv.close()
    lat = np.array(lat[len(lat) // 20:]) * 1e3  # drop the first 5% (warm-up of the stream)
    return {"requests": requests, "offered_load": load, "offered_requests_per_s": round(lam, 2),
            "mean_request_queries": round(mean_n, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "max_ms": round(float(lat.max()), 3),
            "queries_per_s": round(qsum / (t_end - t0), 1), "launches": st["launches"],
            "pool_peak_bytes": st["pool_peak"],
            "latency": "scheduled arrival -> results in the caller's host arrays"}


def measure_extras(ctx, torch, pos, kind, w, n, steps):
    """The line search's shortened interval (Sec. 7.2): the same queries over t in
    [0, 0.5], then the batch-wide smallest toi (the step bound); the indexed
    form with a scene-wide filter; and the host-pointer form."""
    from paper_2009_13349_amd import ccd
    t_s, _, out_s = run_engine(ctx, torch, pos, kind, w, ccd.ENGINE_PERSISTENT, steps, 1,
                               timing=False, t_max=0.5)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mt = ctx.min_toi(out_s.toi)
    ev0.record()
    for _ in range(10):
        mt = ctx.min_toi(out_s.toi, out=mt)
    ev1.record()
    torch.cuda.synchronize()
    shortened = {"t_max": 0.5, "value": round(n * steps / t_s, 1),
                 "ms_per_step": round(1e3 * t_s / steps, 3),
                 "hits": int(out_s.hit.sum().item()), "min_toi": float(mt.item()),
                 "min_toi_ms": round(ev0.elapsed_time(ev1) / 10, 4)}
    return shortened, measure_indexed(ctx, torch, steps), measure_host(ctx, w, n)


def measure_host(ctx, w, n, runs: int = 2):
    """The host-pointer form of ccd_batch on the same queries (numpy arrays in
    pageable host memory): host validation, copies over PCIe both ways and the
    root finder, as a caller without device buffers sees it."""
    from paper_2009_13349_amd import ccd
    ctx.set_engine(ccd.ENGINE_PERSISTENT)
    ctx.enable_timing(False)
    pos = np.ascontiguousarray(w["pos"])
    kind = np.ascontiguousarray(w["kind"])
    r = ctx.batch_host(pos, kind, delta=w["delta"], max_iter=w["max_iter"], min_sep=w["min_sep"])
    t0 = time.perf_counter()
    for _ in range(runs):
        r = ctx.batch_host(pos, kind, delta=w["delta"], max_iter=w["max_iter"], min_sep=w["min_sep"])
    t = (time.perf_counter() - t0) / runs
    return {"value": round(n / t, 1), "ms_per_batch": round(1e3 * t, 3), "hits": int(r.hit.sum()),
            "note": "host arrays in, host arrays out (validation + PCIe copies included)"}


def measure_indexed(ctx, torch, steps, n_pairs=1_000_000):
    """Candidate pairs over shared vertex arrays with a scene-wide filter (the
    mesh form of Sec. 7): a two-sheet mesh scene of n_pairs broad-phase pairs,
    gamma from ccd_scene_gamma, then ccd_batch_indexed (gather + root finder)."""
    from paper_2009_13349_amd import ccd, workloads as W
    s = W.mesh_scene(n_pairs, seed=5)
    dev = torch.device("cuda:0")
    v0, v1 = torch.from_numpy(s["v0"]).to(dev), torch.from_numpy(s["v1"]).to(dev)
    ids, kind = torch.from_numpy(s["ids"]).to(dev), torch.from_numpy(s["kind"]).to(dev)
    ctx.set_engine(ccd.ENGINE_PERSISTENT)
    ctx.enable_timing(False)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    g = ctx.scene_gamma(v0, v1)
    ev[0].record()
    g = ctx.scene_gamma(v0, v1, out=g)
    ev[1].record()
    torch.cuda.synchronize()
    gamma_ms = ev[0].elapsed_time(ev[1])
    out = ctx.batch_indexed(v0, v1, ids, kind, gamma=g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.batch_indexed(v0, v1, ids, kind, gamma=g, out=out)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return {"workload": s["name"], "vertices": int(s["v0"].shape[0]), "value": round(n_pairs * steps / t, 1),
            "ms_per_step": round(1e3 * t / steps, 3), "hits": int(out.hit.sum().item()),
            "scene_gamma_ms": round(gamma_ms, 4), "gamma": [float(x) for x in g.cpu().numpy()]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="simulation", choices=["simulation", "edge_edge", "uniform_vf"])
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--tuning", default="", help="k=v,... overrides of ccd_tuning")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (default: tune once per device and workload, cached)")
    ap.add_argument("--tuning-cache", default=os.environ.get(
        "CCD_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ccd_mi355x_tuning.txt")))
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the serving measurement (0: skip)")
    ap.add_argument("--serve-streams", type=int, default=2,
                    help="compute streams of the serving measurement's server")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the benchmark workload's batches (for profiler runs): no "
                         "shortened-interval or indexed measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device-to-device copy first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: queries are independent, so several GPUs would "
              "each run the same batch call on a slice of the query index, with no cross-GPU "
              "step to measure.", file=sys.stderr)
        raise SystemExit(2)

    import torch
    from paper_2009_13349_amd import ccd

    w = make_workload(args.workload, args.n)
    n = w["pos"].shape[1]
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(w["pos"]).to(dev)
    kind = torch.from_numpy(w["kind"]).to(dev)
    torch.cuda.synchronize()
    kind_counts = np.bincount(w["kind"], minlength=2)

    if args.copy_calibration:
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = ccd.Context(0, mem_budget_bytes=32 << 30)
    autotune = None
    if args.tuning:
        ctx.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})
    elif not args.no_autotune:
        key = f"{w['name']}_delta{w['delta']:g}"
        if ctx.tuning_cache_load(args.tuning_cache, key):
            autotune = {"source": "cache", "tuning": ctx.tuning()}
        else:
            ctx.set_engine(ccd.ENGINE_PERSISTENT)
            t0 = time.perf_counter()
            best, best_ms = ctx.autotune(pos, kind, delta=w["delta"], max_iter=w["max_iter"],
                                         min_sep=w["min_sep"])
            autotune = {"source": "search", "seconds": round(time.perf_counter() - t0, 2),
                        "best_ms": round(best_ms, 3), "tuning": best}
            os.makedirs(os.path.dirname(args.tuning_cache) or ".", exist_ok=True)
            ctx.tuning_cache_store(args.tuning_cache, key)
    t_p, stats_p, out = run_engine(ctx, torch, pos, kind, w, ccd.ENGINE_PERSISTENT, args.steps,
                                   args.warmup)
    hits = int(out.hit.sum().item())
    # checks the sequential Alg. 2 performs (n_checks is exact unless capped)
    nck = out.n_checks.to(torch.float64)
    alg_checks = [float((nck * (kind == k)).sum().item()) for k in (0, 1)]
    value = n * args.steps / t_p
    # the same steps replaying the captured hipGraph (no per-kernel events)
    t_g, _, _ = run_engine(ctx, torch, pos, kind, w, ccd.ENGINE_PERSISTENT, args.steps, 1,
                           timing=False)
    graph_counts = ctx.graph_counts()
    plain = None
    if not args.no_plain:
        t_b, stats_b, _ = run_engine(ctx, torch, pos, kind, w, ccd.ENGINE_PLAIN, args.steps,
                                     args.warmup)
        plain = {"value": round(n * args.steps / t_b, 1), "ms_per_step": round(1e3 * t_b / args.steps, 3),
                 "kernel_ms_avg": {KERNELS[i]: round(float(np.mean([s["kernel_ms"][i] for s in stats_b])), 4)
                                   for i in range(4)}}
    shortened = indexed = host = None
    if not args.main_only:
        shortened, indexed, host = measure_extras(ctx, torch, pos, kind, w, n, args.steps)
    rl = roofline(stats_p, kind_counts)
    tier = KERNELS.index(rl["kernel"]) - 1
    rl["symbol"] = kernel_symbol(tier, ctx.tuning())
    tb = hbm_traffic(rl["symbol"])
    rl["traffic"] = round(tb) if tb else None
    rl["traffic_unit"] = "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    rl["hbm_gbps"] = round(tb / (rl["avg_launch_ms"] * 1e-3) / 1e9, 1) if tb else None
    streaming = query_streaming(stats_p, n)
    checks_total = int(sum(sum(c) for c in stats_p[-1]["checks"]))
    alg_flops = alg_checks[0] * FLOP_PER_CHECK[0] + alg_checks[1] * FLOP_PER_CHECK[1]
    path_alg_tflops = alg_flops / (t_p / args.steps) / 1e12
    ctx.close()

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_p / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "queries": n, "vf": int(kind_counts[0]),
                   "ee": int(kind_counts[1]), "delta": w["delta"], "max_iter": w["max_iter"],
                   "min_sep": w["min_sep"], "engine": "persistent", "parallelism": "single GPU"},
        "plain_kernel": plain,
        "speedup_vs_plain": round(value / plain["value"], 3) if plain else None,
        "graph_replay": {"value": round(n * args.steps / t_g, 1),
                         "ms_per_step": round(1e3 * t_g / args.steps, 3),
                         "graphs_built": graph_counts[0], "replays": graph_counts[1]},
        "autotune": autotune,
        "hits": hits,
        "box_checks_per_step": checks_total,
        "sequential_checks_per_step": int(sum(alg_checks)),
        "path_algorithmic_tflops": round(path_alg_tflops, 3),
        "promoted_per_step": stats_p[-1]["promoted"],
        "lane_utilization": [round(sum(stats_p[-1]["checks"][i]) / stats_p[-1]["lane_slots"][i], 3)
                             if stats_p[-1]["lane_slots"][i] else None for i in range(3)],
        "roofline": rl,
        "query_streaming": streaming,
        "shortened_interval": shortened,
        "indexed": indexed,
        "host_pointers": host,
    }
    line["serve"] = (serve_latency(w, torch, value, args.serve_requests, streams=args.serve_streams)
                     if args.serve_requests > 0 and args.workload == "simulation" else None)
    line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds) if args.cpu_seconds > 0 else None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
