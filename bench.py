"""Benchmark of the MI355X CCD root finder.

One step = one ccd_batch call over the whole workload (all queries resident in
HBM before the timed region), i.e. the complete root finder for every query:
root pass (level 0 of every query), lane engine, group engine and block
engine.  Default workload: 1,000,000 simulation-shaped queries (60%
vertex-face, 40% edge-edge, 2% near-contacts, 1% grazing contacts), delta =
1e-6, m_I = 1e6, no minimum separation.  Prints one JSON line, which also
carries per-workload lines for the other query sets (4,096 uniform
vertex-face; 100,000 edge-edge with 10% degenerate cases; the four
1,000,000-query minimum-separation runs), serving at three offered loads, and
the CPU oracle's rate on the host (one pinned core, and K pinned processes on
disjoint shards of the same sample).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CCD queries/s at delta=1e-6 (persistent vs plain kernel); p50/p99 serve latency"
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X: 256 CUs x 2.4 GHz x 128 FP64 FLOP/clk (FMA = 2)
FLOP_PER_CHECK = {0: 227.0, 1: 177.0}  # vertex-face, edge-edge box check (binary64 add/sub/mul)
FLOP_PER_CHECK_MS = 6.0                # enlargement by d (min_sep > 0)
KERNELS = ("root", "lane", "group", "block")
COMMITTED_TUNING = os.path.join(ROOT, "paper_2009_13349_amd", "tuning_mi355x.txt")


# ---------------------------------------------------------------------------
# CPU oracle workers.  They are forked before torch or the HIP library is
# loaded (so no GPU state is copied), each pinned to one core, and wait for
# work until the GPU measurements are over.

def _oracle_worker(conn, core):
    try:
        os.sched_setaffinity(0, {core})
    except OSError:
        pass
    import oracle
    oracle.lib()
    while True:
        msg = conn.recv()
        if msg is None:
            break
        pos, kind, kw = msg
        t0 = time.perf_counter()
        r = oracle.solve_batch(pos, kind, **kw)
        dt = time.perf_counter() - t0
        conn.send(({k: r[k] for k in ("toi", "t_width", "n_checks", "hit", "status")}, dt))


class OracleWorkers:
    def __init__(self, cores):
        ctx = mp.get_context("fork")
        self.cores = list(cores)
        self.conns, self.procs = [], []
        for c in self.cores:
            a, b = ctx.Pipe()
            p = ctx.Process(target=_oracle_worker, args=(b, c), daemon=True)
            p.start()
            self.conns.append(a)
            self.procs.append(p)

    def run(self, shards):
        """shards: list (at most one per worker) of (pos, kind, kw); returns the
        per-shard (results, seconds) and the wall time of the whole run."""
        t0 = time.perf_counter()
        for conn, sh in zip(self.conns, shards):
            conn.send(sh)
        out = [conn.recv() for conn, _ in zip(self.conns, shards)]
        return out, time.perf_counter() - t0

    def close(self):
        for c in self.conns:
            try:
                c.send(None)
            except OSError:
                pass
        for p in self.procs:
            p.join(timeout=5)


def _digest(parts):
    h = hashlib.sha256()
    for k in ("toi", "t_width", "n_checks", "hit", "status"):
        a = np.concatenate([p[k] for p in parts])
        if a.dtype == np.float64:
            a = a.view(np.uint64)
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workers: OracleWorkers, w, seconds: float):
    """The oracle (single-threaded C++, as it stands) on a seeded random sample
    of the same workload: one pinned core over the whole sample, then K pinned
    processes over disjoint shards of it; the two runs' results must hash the
    same."""
    from paper_2009_13349_amd import workloads as W
    n = w["pos"].shape[1]
    kw = dict(delta=w["delta"], max_iter=w["max_iter"], min_sep=w["min_sep"])
    perm = np.random.default_rng(1234).permutation(n)
    pilot = W.subset(w, perm[:2000])
    res, _ = workers.run([(pilot["pos"], pilot["kind"], kw)])
    t_pilot = res[0][1]
    m = int(min(n, max(2000, 2000 * seconds / max(t_pilot, 1e-3))))
    ws = W.subset(w, perm[:m])
    one, _ = workers.run([(ws["pos"], ws["kind"], kw)])
    k = len(workers.cores)
    cuts = np.array_split(np.arange(m), k)
    shards = [(np.ascontiguousarray(ws["pos"][:, c]), np.ascontiguousarray(ws["kind"][c]), kw) for c in cuts]
    many, tk = workers.run(shards)
    h1 = _digest([one[0][0]])
    hk = _digest([r[0] for r in many])
    return {"value": round(m / one[0][1], 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"{m} queries drawn uniformly at random (seed 1234) from the same {n}-query "
                      f"workload; single-threaded C++ oracle pinned to one core, {one[0][1]:.1f} s",
            "k_processes": {"value": round(m / tk, 2), "cores": k, "wall_s": round(tk, 2),
                            "note": "the same sample in K disjoint shards, one pinned process each"},
            "cpu_model": cpu_model(), "result_sha256": h1, "hash_equal": h1 == hk,
            "affinity_cores": len(os.sched_getaffinity(0))}


# ---------------------------------------------------------------------------
# GPU measurements

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
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.batch_device(pos, kind, out=out, **kw)
        if timing:
            stats.append(ctx.last_stats())  # synchronises; reads the per-kernel HIP events
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    del ccd
    return (t1 - t0), stats, out


def flop_per_check(kind: int, min_sep: float) -> float:
    return FLOP_PER_CHECK[kind] + (FLOP_PER_CHECK_MS if min_sep > 0 else 0.0)


def roofline(stats, min_sep: float = 0.0):
    """Dominant kernel (largest device time) and its achieved FP64 rate:
    algorithmic FLOPs (box checks executed by that kernel x FLOPs per check)
    per launch / average launch duration from HIP events."""
    ms = np.array([s["kernel_ms"] for s in stats])  # [steps, 4]
    avg = ms.mean(axis=0)
    k = int(np.argmax(avg[1:])) + 1
    tier = k - 1
    checks = np.array([s["checks"][tier] for s in stats], dtype=np.float64).mean(axis=0)
    flops = checks[0] * flop_per_check(0, min_sep) + checks[1] * flop_per_check(1, min_sep)
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
        "flop_per_check": [flop_per_check(0, min_sep), flop_per_check(1, min_sep)],
        "kernel_ms_avg": {KERNELS[i]: round(float(avg[i]), 4) for i in range(4)},
    }


BUDGET = [0]  # the measuring context's scratch budget (bytes)


def kernel_symbol(tier: int, tuning: dict, n: int = 1_000_000, max_iter: int = 1_000_000,
                  num_cu: int = 256) -> str:
    """The kernel a tier runs (the block tier: four-wave engines when the
    scratch plan has at least two block engines per CU)."""
    if tier == 0:
        return "ccd::k_lane<true>"
    if tier == 2:
        from paper_2009_13349_amd import ccd
        plan = ccd.plan_scratch(n, max_iter, num_cu, mem_budget_bytes=BUDGET[0], **tuning)
        if plan["block_count"] >= 2 * num_cu:
            return "ccd::k_group<4, 1, false>"
        return f"ccd::k_group<8, 1, {'true' if tuning['block_lds_words'] > 0 else 'false'}>"
    gw = tuning["group_waves"]
    occ = tuning["group_occupancy"] if gw == 1 else 1
    lds = tuning["group_lds_words"] > 0 and (gw == 8 or (gw == 1 and occ == 3))
    return f"ccd::k_group<{gw}, {occ}, {'true' if lds else 'false'}>"


def profile_record(fname: str, symbol: str, tuning: dict):
    """A per-kernel record under profiles/ taken with these exact kernel
    sources (else None), and whether its tuning is the one in use."""
    from paper_2009_13349_amd.rocprof_summary import kernel_source_hash
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None, False
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None, False
    k = rec.get("kernels", {}).get(symbol)
    same = rec.get("tuning") is not None and all(rec["tuning"].get(f) == v for f, v in tuning.items())
    return k, same


def executed_fp64(symbol: str, tuning: dict, avg_ms: float):
    """FP64 FLOP/s the dominant kernel executed (rocprofv3 counters of these
    kernel sources: 64 x (ADD_F64 + MUL_F64 + 2 FMA_F64) wave instructions per
    dispatch) over its launch time, and its VALU issue share."""
    k, same = profile_record("fp64_counters.json", symbol, tuning)
    if not k:
        return None
    add, mul, fma = (k.get("SQ_INSTS_VALU_ADD_F64", 0.0), k.get("SQ_INSTS_VALU_MUL_F64", 0.0),
                     k.get("SQ_INSTS_VALU_FMA_F64", 0.0))
    flops = 64.0 * (add + mul + 2.0 * fma)
    out = {"tflops": round(flops / (avg_ms * 1e-3) / 1e12, 3), "flop_per_launch": flops,
           "frac_of_peak": round(flops / (avg_ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 5),
           "counters_tuning_matches": same}
    valu, grbm = k.get("SQ_INSTS_VALU"), k.get("GRBM_GUI_ACTIVE")
    if valu and grbm:
        # 4 cycles per wave64 VALU instruction on 1,024 SIMDs; GRBM_GUI_ACTIVE
        # sums the dispatch's cycles over the 8 XCDs
        out["valu_busy"] = round(4.0 * valu / (1024.0 * grbm / 8.0), 3)
        out["fp64_share_of_valu"] = round((add + mul + fma) / valu, 3)
    return out


def query_streaming(stats, n: int, tuning: dict):
    """The root pass reads every query's 24 coordinates and its kind once:
    its read rate against the 8 TB/s HBM peak."""
    ms = float(np.mean([s["kernel_ms"][0] for s in stats]))
    bytes_in = n * (24 * 8 + 1)
    gbps = bytes_in / (ms * 1e-3) / 1e9
    k, _ = profile_record("hbm_traffic.json", "ccd::k_root", tuning)
    return {"kernel": "root", "algorithmic_bytes_read": bytes_in, "avg_launch_ms": round(ms, 4),
            "gbps": round(gbps, 1), "frac_of_hbm_peak": round(gbps / 8000.0, 3),
            "measured_read_bytes": round(k["fetch_bytes"]) if k else None}


def apply_tuning(ctx, args, key, w, pos, kind):
    """Tuning order: --tuning, the committed MI355X tuning file, the user cache,
    then a search (stored in the user cache)."""
    from paper_2009_13349_amd import ccd
    if args.tuning:
        ctx.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})
        return {"source": "command line", "tuning": ctx.tuning()}
    if not args.retune:
        if os.path.exists(COMMITTED_TUNING) and ctx.tuning_cache_load(COMMITTED_TUNING, key):
            return {"source": "committed tuning file (autotuner result on MI355X)", "key": key,
                    "tuning": ctx.tuning()}
        if ctx.tuning_cache_load(args.tuning_cache, key):
            return {"source": "cache", "key": key, "tuning": ctx.tuning()}
    if args.no_autotune:
        return {"source": "defaults", "tuning": ctx.tuning()}
    ctx.set_engine(ccd.ENGINE_PERSISTENT)
    t0 = time.perf_counter()
    best, best_ms = ctx.autotune(pos, kind, delta=w["delta"], max_iter=w["max_iter"], min_sep=w["min_sep"])
    os.makedirs(os.path.dirname(args.tuning_cache) or ".", exist_ok=True)
    ctx.tuning_cache_store(args.tuning_cache, key)
    return {"source": "search", "key": key, "seconds": round(time.perf_counter() - t0, 2),
            "best_ms": round(best_ms, 3), "tuning": best}


def measure_workload(ctx, torch, w, steps, warmup):
    """One query set: persistent engine, per-kernel events; its own roofline."""
    from paper_2009_13349_amd import ccd
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(w["pos"]).to(dev)
    kind = torch.from_numpy(w["kind"]).to(dev)
    n = w["pos"].shape[1]
    t, stats, out = run_engine(ctx, torch, pos, kind, w, ccd.ENGINE_PERSISTENT, steps, warmup)
    seq = float(out.n_checks.to(torch.float64).sum().item())
    rl = roofline(stats, w["min_sep"])
    tier = KERNELS.index(rl["kernel"]) - 1
    rl["symbol"] = kernel_symbol(tier, ctx.tuning(), n, w["max_iter"])
    res = {"queries": n, "value": round(n * steps / t, 1), "ms_per_step": round(1e3 * t / steps, 3),
           "steps": steps, "delta": w["delta"], "max_iter": w["max_iter"], "min_sep": w["min_sep"],
           "hits": int(out.hit.sum().item()),
           "capped": int(((out.status & 1) != 0).sum().item()),
           "overflowed": stats[-1]["overflowed"], "restarted": stats[-1]["restarted"],
           "handoff_pool_words_asked": stats[-1]["handoff_words"],
           "box_checks_per_step": int(sum(sum(c) for c in stats[-1]["checks"])),
           "sequential_checks_per_step": int(seq),
           "promoted_per_step": stats[-1]["promoted"], "level_probes_per_step": stats[-1]["probes"],
           "roofline": rl}
    del pos, kind, out
    torch.cuda.empty_cache()
    return res


def measure_configs(ctx, torch, steps):
    """The other query sets of the benchmark, each with its own entry of the
    committed MI355X tuning file when it has one (autotuner results, searched
    from the main workload's tuning with two block engines per CU), else the
    main workload's tuning with the library's default block engines (two
    four-wave engines per CU: these sets send thousands of capped queries to
    the block tier, where more engines at once beat eight waves per query;
    the main workload sends it a few hundred levels and keeps one eight-wave
    engine per CU): 4,096 uniform vertex-face queries; 100,000 edge-edge
    queries with 10% degenerate cases (their parallel and coplanar pairs run
    to the m_I cap); 1,000,000 minimum-separation queries at d in
    {1e-4, 1e-3} x delta in {1e-6, 1e-4}."""
    from paper_2009_13349_amd import workloads as W
    num_cu = torch.cuda.get_device_properties(0).multi_processor_count
    main = ctx.tuning()
    fallback = dict(main, block_count=2 * num_cu)
    out = {}

    def measure(w, steps_w, warm):
        key = f"{w['name']}_delta{w['delta']:g}"
        if ctx.tuning_cache_load(COMMITTED_TUNING, key):
            src = "committed tuning file (autotuner result on MI355X)"
        else:
            ctx.set_tuning(**fallback)
            src = "main workload's tuning, default block engines"
        res = measure_workload(ctx, torch, w, steps_w, warm)
        res["tuning_source"] = src
        res["tuning"] = ctx.tuning()
        return res

    w = W.uniform_vf(4096, seed=0)
    out[w["name"]] = measure(w, max(steps, 20), 3)
    w = W.edge_edge_mixed(100_000, seed=1)
    out[w["name"]] = measure(w, max(2, steps // 4), 1)
    for d in (1e-4, 1e-3):
        for delta in (1e-6, 1e-4):
            w = W.min_separation(1_000_000, seed=2, d_min=d, delta=delta)
            out[w["name"]] = measure(w, 2, 1)
            del w
    ctx.set_tuning(**main)
    return out


def serve_payloads(w, torch, rng, payloads: int):
    """Contiguous pinned slices of the benchmark workload, sizes log-uniform
    in [1e3, 1e6]."""
    N = w["pos"].shape[1]
    sizes = np.round(np.exp(rng.uniform(math.log(1e3), math.log(1e6), size=payloads))).astype(int)
    pay = []
    for n in sizes:
        off = int(rng.integers(0, N - n + 1))
        pos = torch.from_numpy(np.ascontiguousarray(w["pos"][:, off:off + n])).pin_memory()
        kind = torch.from_numpy(np.ascontiguousarray(w["kind"][off:off + n])).pin_memory()
        pay.append((int(n), pos, kind))
    return pay, float(np.mean(sizes))


def serve_saturation(w, torch, requests: int = 200, payloads: int = 64, seed: int = 4,
                     streams: int = 2, launch_target_us: int = 5000):
    """The serving path's own throughput: the same requests submitted back to
    back (closed loop, everything queued at once), queries per second from
    the first submission to the last result in host memory."""
    from paper_2009_13349_amd import ccd
    rng = np.random.default_rng(seed)
    pay, _ = serve_payloads(w, torch, rng, payloads)
    deltas = np.exp(rng.uniform(math.log(1e-6), math.log(1e-4), size=requests))
    srv = ccd.Server(streams=streams, pool_bytes=16 << 30, scratch_bytes=12 << 30,
                     max_queries_per_launch=4_000_000, launch_target_us=launch_target_us)
    for n, pos, kind in pay[:4]:
        srv.wait(srv.submit(pos, kind, delta=1e-6), 600_000)
    t0 = time.monotonic()
    tickets, qsum = [], 0
    for i in range(requests):
        n, pos, kind = pay[i % payloads]
        tickets.append(srv.submit(pos, kind, delta=float(deltas[i])))
        qsum += n
    for t in tickets:
        srv.wait(t, 600_000)
    dt = time.monotonic() - t0
    srv.close()
    return qsum / dt


def serve_latency(w, torch, q_sat: float, requests: int, payloads: int = 64, load: float = 0.7,
                  seed: int = 4, streams: int = 2, launch_target_us: int = 5000):
    """Poisson stream of requests (sizes log-uniform in [1e3, 1e6], delta
    log-uniform in [1e-6, 1e-4]) at `load` x q_sat (the serving path's own
    closed-loop throughput), submitted to the continuous-batching server;
    latency = scheduled arrival -> results in the caller's arrays.  Request
    payloads are contiguous pinned slices of the benchmark workload (a fixed
    set of `payloads` of them, reused round robin)."""
    from paper_2009_13349_amd import ccd
    rng = np.random.default_rng(seed)
    pay, mean_n = serve_payloads(w, torch, rng, payloads)
    lam = load * q_sat / mean_n  # requests per second
    gaps = rng.exponential(1.0 / lam, size=requests)
    deltas = np.exp(rng.uniform(math.log(1e-6), math.log(1e-4), size=requests))
    srv = ccd.Server(streams=streams, pool_bytes=16 << 30, scratch_bytes=12 << 30,
                     max_queries_per_launch=4_000_000, launch_target_us=launch_target_us)
    # warm-up: a few requests, not timed (they also seed the cost estimate)
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
            "launch_target_us": launch_target_us, "pool_peak_bytes": st["pool_peak"],
            "latency": "scheduled arrival -> results in the caller's host arrays"}


def measure_extras(ctx, torch, pos, kind, w, n, steps, args):
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
    return shortened, measure_indexed(ctx, torch, steps, args), measure_host(ctx, w, n)


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


def measure_indexed(ctx, torch, steps, args, n_pairs=1_000_000):
    """Candidate pairs over shared vertex arrays with a scene-wide filter (the
    mesh form of Sec. 7): a two-sheet mesh scene of n_pairs broad-phase pairs,
    gamma from ccd_scene_gamma, then ccd_batch_indexed (gather + root finder),
    with a tuning of its own (searched on the scene's pairs in
    structure-of-arrays form, stored under the scene's key)."""
    from paper_2009_13349_amd import ccd, workloads as W
    s = W.mesh_scene(n_pairs, seed=5)
    dev = torch.device("cuda:0")
    v0, v1 = torch.from_numpy(s["v0"]).to(dev), torch.from_numpy(s["v1"]).to(dev)
    ids, kind = torch.from_numpy(s["ids"]).to(dev), torch.from_numpy(s["kind"]).to(dev)
    main_tuning = ctx.tuning()
    tune = None
    if not args.tuning:
        # the pairs' coordinates as a structure-of-arrays batch for the tuner
        gathered = np.concatenate([s["v0"][s["ids"][:, k]].T for k in range(4)] +
                                  [s["v1"][s["ids"][:, k]].T for k in range(4)])
        pos = torch.from_numpy(np.ascontiguousarray(gathered)).to(dev)
        tune = apply_tuning(ctx, args, f"{s['name']}_delta1e-06",
                            {"delta": 1e-6, "max_iter": 1_000_000, "min_sep": 0.0}, pos, kind)
        del pos, gathered
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
    ctx.set_tuning(**main_tuning)
    return {"workload": s["name"], "vertices": int(s["v0"].shape[0]), "value": round(n_pairs * steps / t, 1),
            "ms_per_step": round(1e3 * t / steps, 3), "hits": int(out.hit.sum().item()),
            "scene_gamma_ms": round(gamma_ms, 4), "gamma": [float(x) for x in g.cpu().numpy()],
            "autotune": tune}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="simulation", choices=["simulation", "edge_edge", "uniform_vf"])
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="K of the K-process oracle run (capped by the cores this process may use)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the per-workload lines")
    ap.add_argument("--tuning", default="", help="k=v,... overrides of ccd_tuning")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library defaults when no stored tuning matches")
    ap.add_argument("--retune", action="store_true", help="search again instead of stored tunings")
    ap.add_argument("--tuning-cache", default=os.environ.get(
        "CCD_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ccd_mi355x_tuning.txt")))
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests per offered load of the serving measurement (0: skip)")
    ap.add_argument("--serve-loads", default="0.5,0.7,0.9")
    ap.add_argument("--budget-gib", type=int, default=160,
                    help="scratch budget of the measuring context (at most 60%% of free HBM)")
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--serve-target-us", type=int, default=5000,
                    help="server's launch latency target (0: launches bounded by size only)")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the benchmark workload's batches (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device-to-device copy first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: queries are independent, so several GPUs would "
              "each run the same batch call on a slice of the query index, with no cross-GPU "
              "step to measure.", file=sys.stderr)
        raise SystemExit(2)

    # the oracle's worker processes start before torch and the HIP library load
    workers = None
    if args.cpu_seconds > 0 and not args.main_only:
        cores = sorted(os.sched_getaffinity(0))[:max(1, args.cpu_procs)]
        workers = OracleWorkers(cores)

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

    # scratch budget: most of the 288 GB of HBM, so that the group -> block
    # hand-off pool holds every hand-off of the heaviest query sets (a
    # hand-off the pool cannot take restarts its query at level 0)
    free_bytes, _ = torch.cuda.mem_get_info(dev)
    budget = min(args.budget_gib << 30, int(free_bytes * 0.6))
    BUDGET[0] = budget
    ctx = ccd.Context(0, mem_budget_bytes=budget)
    key = f"{w['name']}_delta{w['delta']:g}"
    autotune = apply_tuning(ctx, args, key, w, pos, kind)
    tuning = ctx.tuning()
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
        kms = {KERNELS[i]: round(float(np.mean([s["kernel_ms"][i] for s in stats_b])), 4) for i in range(4)}
        handed = stats_b[-1]["promoted"][0]
        plain = {"value": round(n * args.steps / t_b, 1), "ms_per_step": round(1e3 * t_b / args.steps, 3),
                 "kernel_ms_avg": kms,
                 "lane_kernel_only": {
                     "ms": kms["lane"], "queries_finished": n - handed, "queries_handed_on": handed,
                     "note": "the plain kernel itself: one thread per query, a frontier of up to "
                             "lane_capacity boxes in LDS; a query whose level outgrows it goes to "
                             "the group tier, whose time is in the whole-path figure"}}
        ctx.set_engine(ccd.ENGINE_PERSISTENT)
    shortened = indexed = host = None
    if not args.main_only:
        shortened, indexed, host = measure_extras(ctx, torch, pos, kind, w, n, args.steps, args)
        ctx.set_tuning(**tuning)
    rl = roofline(stats_p)
    tier = KERNELS.index(rl["kernel"]) - 1
    rl["symbol"] = kernel_symbol(tier, tuning, n, w["max_iter"])
    tk, same = profile_record("hbm_traffic.json", rl["symbol"], tuning)
    tb = tk["fetch_bytes"] + tk["write_bytes"] if tk and tk.get("fetch_bytes") is not None else None
    rl["traffic"] = round(tb) if tb else None
    rl["traffic_unit"] = "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    rl["traffic_tuning_matches"] = same if tb else None
    rl["hbm_gbps"] = round(tb / (rl["avg_launch_ms"] * 1e-3) / 1e9, 1) if tb else None
    rl["executed"] = executed_fp64(rl["symbol"], tuning, rl["avg_launch_ms"])
    streaming = query_streaming(stats_p, n, tuning)
    checks_total = int(sum(sum(c) for c in stats_p[-1]["checks"]))
    alg_flops = alg_checks[0] * FLOP_PER_CHECK[0] + alg_checks[1] * FLOP_PER_CHECK[1]
    path_alg_tflops = alg_flops / (t_p / args.steps) / 1e12
    del pos, kind, out, nck
    torch.cuda.empty_cache()

    configs = None
    if not args.main_only and not args.no_configs and args.workload == "simulation":
        configs = measure_configs(ctx, torch, args.steps)
        ctx.set_tuning(**tuning)
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
        "level_probes_per_step": stats_p[-1]["probes"],
        "overflowed_per_step": stats_p[-1]["overflowed"],
        "restarted_per_step": stats_p[-1]["restarted"],
        "scratch_budget_bytes": budget,
        "lane_utilization": [round(sum(stats_p[-1]["checks"][i]) / stats_p[-1]["lane_slots"][i], 3)
                             if stats_p[-1]["lane_slots"][i] else None for i in range(3)],
        "roofline": rl,
        "query_streaming": streaming,
        "shortened_interval": shortened,
        "indexed": indexed,
        "host_pointers": host,
        "configs": configs,
    }
    loads = [float(x) for x in args.serve_loads.split(",") if x]
    if args.serve_requests > 0 and args.workload == "simulation" and not args.main_only:
        sat = serve_saturation(w, torch, streams=args.serve_streams, launch_target_us=args.serve_target_us)
        runs = [serve_latency(w, torch, sat, args.serve_requests, load=ld, streams=args.serve_streams,
                              launch_target_us=args.serve_target_us) for ld in loads]
        for r in runs:
            r["offered_load_of"] = "serving path's closed-loop throughput"
            r["serving_saturation_queries_per_s"] = round(sat, 1)
        line["serve"] = min(runs, key=lambda r: abs(r["offered_load"] - 0.7))
        line["serve_loads"] = runs
    else:
        line["serve"] = None
    line["cpu_baseline"] = cpu_baseline(workers, w, args.cpu_seconds) if workers else None
    if workers:
        workers.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
