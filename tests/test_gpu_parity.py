"""GPU <-> oracle parity of the HIP root finder, called through the C ABI.

Bar: hit and status bit-exact, toi and t_width bit-identical (which implies
the stated tolerance |toi_gpu - toi_oracle| <= 1e-6), n_checks identical.
Both sides compute in binary64 with the same operation order and no
contraction, so any difference is a bug."""
import math

import numpy as np
import pytest

import oracle
from paper_2009_13349_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("toi", "t_width", "hit", "n_checks", "status")
TOI_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def ccdmod():
    from paper_2009_13349_amd import ccd
    ccd.load()
    return ccd


@pytest.fixture()
def ctx(ccdmod, torch_dev):
    c = ccdmod.Context(0)
    yield c
    c.close()


def run_gpu(ctx, torch_dev, w, engine=0, **kw):
    torch, dev = torch_dev
    ctx.set_engine(engine)
    pos = torch.from_numpy(np.ascontiguousarray(w["pos"])).to(dev)
    kind = torch.from_numpy(np.ascontiguousarray(w["kind"])).to(dev)
    extra = {}
    for name, dt in (("delta_q", torch.float64), ("max_iter_q", torch.int64), ("min_sep_q", torch.float64)):
        if kw.get(name) is not None:
            extra[name] = torch.from_numpy(np.ascontiguousarray(kw.pop(name))).to(dev, dt)
        else:
            kw.pop(name, None)
    r = ctx.batch_device(pos, kind, **kw, **extra)
    torch.cuda.synchronize()
    out = {k: getattr(r, k).cpu().numpy() for k in FIELDS}
    out["n_checks"] = out["n_checks"].astype(np.uint64)
    return out


def run_oracle(w, delta=1e-6, max_iter=1_000_000, min_sep=0.0, literal=False, delta_q=None,
               max_iter_q=None, min_sep_q=None):
    return oracle.solve_batch(w["pos"], w["kind"], delta=delta if delta_q is None else delta_q,
                              max_iter=max_iter if max_iter_q is None else max_iter_q,
                              min_sep=min_sep if min_sep_q is None else min_sep_q, literal=literal)


def assert_same(got, ref, idx=None, what=""):
    for k in FIELDS:
        g = got[k] if idx is None else got[k][idx]
        r = ref[k]
        if k in ("toi", "t_width"):
            gb = np.ascontiguousarray(g, dtype=np.float64).view(np.int64)
            rb = np.ascontiguousarray(r, dtype=np.float64).view(np.int64)
            bad = np.nonzero(gb != rb)[0]
        else:
            bad = np.nonzero(np.asarray(g).astype(np.int64) != np.asarray(r).astype(np.int64))[0]
        assert len(bad) == 0, (f"{what}: field {k} differs at {len(bad)} queries, first "
                               f"{bad[:5].tolist()}: gpu {np.asarray(g)[bad[:5]]} oracle {np.asarray(r)[bad[:5]]}")
    fin = np.isfinite(ref["toi"])
    g = got["toi"] if idx is None else got["toi"][idx]
    assert np.all(np.abs(g[fin] - ref["toi"][fin]) <= TOI_TOL)


# ---------------------------------------------------------------------------

def test_single_queries_hand_cases(ccdmod, torch_dev):
    from tests.test_oracle_cases import CASES
    for name, kind, X, min_sep, _, _ in CASES:
        fn = ccdmod.vf if kind == 0 else ccdmod.ee
        g = fn(X, 1e-6, 1_000_000, min_sep)
        r = oracle.solve(kind, X, 1e-6, 1_000_000, min_sep)
        assert (g.toi, g.t_width, g.n_checks, g.hit, g.status) == \
            (r.toi, r.t_width, r.n_checks, r.hit, r.status), name


def test_single_queries_paper_examples(ccdmod, torch_dev):
    from tests.test_oracle_pins import _paper_examples
    for name, (_, kind, X, _) in _paper_examples().items():
        fn = ccdmod.vf if kind == 0 else ccdmod.ee
        g = fn(X)
        r = oracle.solve(kind, X)
        assert (g.toi, g.t_width, g.n_checks, g.hit, g.status) == \
            (r.toi, r.t_width, r.n_checks, r.hit, r.status), name


@pytest.mark.parametrize("engine", [0, 1], ids=["persistent", "plain"])
def test_uniform_vf_4096(ctx, torch_dev, engine):
    w = W.uniform_vf(4096, seed=0)
    got = run_gpu(ctx, torch_dev, w, engine)
    ref = run_oracle(w)
    assert_same(got, ref, what="uniform_vf_4096")
    assert ref["hit"][1::2].all()  # every constructed crossing is found


@pytest.mark.parametrize("engine", [0, 1], ids=["persistent", "plain"])
def test_edge_edge_degenerate(ctx, torch_dev, engine):
    w = W.edge_edge_mixed(3000, seed=1)
    got = run_gpu(ctx, torch_dev, w, engine, max_iter=100_000)
    ref = run_oracle(w, max_iter=100_000)
    assert_same(got, ref, what="edge_edge_mixed_3000")
    assert (ref["status"] & 1).sum() > 50  # the degenerate tail reaches the cap


def test_edge_edge_degenerate_paper_cap(ctx, torch_dev):
    w = W.edge_edge_mixed(400, seed=5, degenerate_frac=0.1)
    got = run_gpu(ctx, torch_dev, w, 0, max_iter=1_000_000)
    ref = run_oracle(w, max_iter=1_000_000)
    assert_same(got, ref, what="edge_edge_mixed_400 m_I=1e6")


@pytest.mark.parametrize("engine", [0, 1], ids=["persistent", "plain"])
def test_simulation_sample(ctx, torch_dev, engine):
    w = W.simulation_mixed(20000, seed=2)
    got = run_gpu(ctx, torch_dev, w, engine)
    ref = run_oracle(w)
    assert_same(got, ref, what="simulation_mixed_20000")


@pytest.mark.parametrize("seed", [7, 8])
def test_simulation_other_seeds(ctx, torch_dev, seed):
    """Other draws of the simulation-shaped generator, every output compared."""
    w = W.simulation_mixed(20000, seed=seed)
    got = run_gpu(ctx, torch_dev, w, 0)
    ref = run_oracle(w)
    assert_same(got, ref, what=f"simulation_mixed_20000 seed {seed}")


@pytest.mark.parametrize("d_min,delta", [(1e-4, 1e-6), (1e-3, 1e-4), (1e-4, 1e-4), (1e-3, 1e-6)])
def test_min_separation(ctx, torch_dev, d_min, delta):
    w = W.min_separation(1500, seed=3, d_min=d_min, delta=delta)
    got = run_gpu(ctx, torch_dev, w, 0, delta=delta, min_sep=d_min, max_iter=100_000)
    ref = run_oracle(w, delta=delta, min_sep=d_min, max_iter=100_000)
    assert_same(got, ref, what=f"min_sep d={d_min} delta={delta}")


def test_literal_mode(ctx, torch_dev):
    w = W.concat([W.edge_edge_mixed(1500, seed=7), W.uniform_vf(500, seed=8)])
    got = run_gpu(ctx, torch_dev, w, 0, max_iter=50_000, literal=True)
    ref = run_oracle(w, max_iter=50_000, literal=True)
    assert_same(got, ref, what="literal")


def test_per_query_parameters(ctx, torch_dev):
    w = W.concat([W.uniform_vf(800, seed=9), W.edge_edge_mixed(800, seed=10)])
    n = w["pos"].shape[1]
    rng = np.random.default_rng(0)
    dq = np.exp(rng.uniform(np.log(1e-6), np.log(1e-3), n))
    mq = rng.integers(1, 50_000, n).astype(np.int64)
    sq = np.where(rng.uniform(size=n) < 0.3, rng.uniform(1e-5, 1e-3, n), 0.0)
    got = run_gpu(ctx, torch_dev, w, 0, delta_q=dq, max_iter_q=mq, min_sep_q=sq)
    ref = run_oracle(w, delta_q=dq, max_iter_q=mq, min_sep_q=sq)
    assert_same(got, ref, what="per-query parameters")


def test_results_independent_of_tuning_and_engine(ctx, torch_dev):
    """Tiny lane arenas, a one-check budget and small group arenas force every
    query through the hand-off paths; the bits must not change."""
    w = W.concat([W.uniform_vf(1000, seed=11), W.edge_edge_mixed(1000, seed=12)])
    base = run_gpu(ctx, torch_dev, w, 0, max_iter=200_000)
    ref = run_oracle(w, max_iter=200_000)
    assert_same(base, ref, what="default tuning")
    for tune in ({"lane_capacity": 8, "lane_budget": 1},
                 {"lane_capacity": 8, "group_capacity": 256, "group_waves": 4},
                 {"lane_waves_per_cu": 1, "group_count": 3, "block_count": 2, "group_waves": 2},
                 {"lane_budget": 100000, "lane_capacity": 256, "group_waves": 8}):
        ctx.set_tuning(**tune)
        for engine in (0, 1):
            got = run_gpu(ctx, torch_dev, w, engine, max_iter=200_000)
            assert_same(got, ref, what=f"tuning {tune} engine {engine}")


def _hard_queries(count, seed):
    """Simulation-shaped queries whose sequential run takes more than 256
    checks (the ones the wide engines solve), chosen with the oracle."""
    w = W.simulation_mixed(20_000, seed=seed)
    ref = run_oracle(w, max_iter=1_000_000)
    idx = np.nonzero(ref["n_checks"] > 256)[0]
    vf = idx[w["kind"][idx] == 0][: count // 2]
    ee = idx[w["kind"][idx] == 1][: count - len(vf)]
    return W.subset(w, np.concatenate([vf, ee]))


@pytest.mark.parametrize("literal", [False, True])
def test_group_engine_every_small_cap(ctx, torch_dev, literal):
    """Hard queries forced into the group engines at every m_I from 1 to 600:
    the m_I stop lands on every position of the early levels, including the
    leading box of a level (the group engine's stop after one chunk) and the
    carried box (default mode)."""
    h = _hard_queries(8, seed=21)
    k = h["pos"].shape[1]
    caps = np.arange(1, 601, dtype=np.int64)
    w = W.subset(h, np.repeat(np.arange(k), len(caps)))
    mq = np.tile(caps, k)
    ref = run_oracle(w, max_iter_q=mq, literal=literal)
    for tune in ({"lane_capacity": 8, "lane_budget": 1},
                 {"lane_capacity": 8, "lane_budget": 1, "group_waves": 8}):
        ctx.set_tuning(**tune)
        got = run_gpu(ctx, torch_dev, w, 0, max_iter_q=mq, literal=literal)
        assert_same(got, ref, what=f"caps 1..600 literal={literal} tuning {tune}")


def test_group_engine_hard_queries(ctx, torch_dev):
    """Hard queries to the end (m_I = 1e6), default and literal modes, through
    the group engines with one- and eight-wave blocks."""
    w = _hard_queries(200, seed=22)
    for literal in (False, True):
        ref = run_oracle(w, max_iter=1_000_000, literal=literal)
        for tune in ({"lane_capacity": 8, "lane_budget": 1},
                     {"lane_capacity": 8, "lane_budget": 1, "group_waves": 8},
                     {"lane_capacity": 8, "lane_budget": 1, "group_capacity": 512}):
            ctx.set_tuning(**tune)
            got = run_gpu(ctx, torch_dev, w, 0, max_iter=1_000_000, literal=literal)
            assert_same(got, ref, what=f"hard literal={literal} tuning {tune}")


def test_group_engine_carried_returns(ctx, torch_dev):
    """Queries that end on a carried terminal box (delta = 1e-2 makes boxes of
    one level terminal at different depths), through the lane and group
    engines, with m_I at and around each query's own check count."""
    delta = 1e-2
    parts = []
    for w0 in (W.uniform_vf(20_000, seed=31), W.edge_edge_mixed(20_000, seed=33)):
        r0 = run_oracle(w0, delta=delta)
        parts.append(W.subset(w0, np.nonzero(r0["status"] & 2)[0]))
    w = W.concat(parts)
    k = w["pos"].shape[1]
    assert k >= 100
    r1 = run_oracle(w, delta=delta)
    rng = np.random.default_rng(3)
    offs = np.array([-3, -2, -1, 0, 1, 5], dtype=np.int64)
    base = r1["n_checks"].astype(np.int64)
    mq = np.concatenate([np.maximum(1, base + o) for o in offs] +
                        [rng.integers(1, np.maximum(2, base))])
    ww = W.subset(w, np.tile(np.arange(k), len(offs) + 1))
    for literal in (False, True):
        ref = run_oracle(ww, delta=delta, max_iter_q=mq, literal=literal)
        if not literal:
            assert np.count_nonzero(ref["status"] == 2) >= 50
        for tune in ({}, {"lane_capacity": 8, "lane_budget": 1},
                     {"lane_capacity": 8, "lane_budget": 1, "group_waves": 8}):
            if tune:
                ctx.set_tuning(**tune)
            got = run_gpu(ctx, torch_dev, ww, 0, delta=delta, max_iter_q=mq, literal=literal)
            assert_same(got, ref, what=f"carried returns literal={literal} tuning {tune}")


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 257, 1031])
def test_ragged_sizes(ctx, torch_dev, n):
    w = W.concat([W.uniform_vf(n, seed=13), W.edge_edge_mixed(n, seed=14)])
    w = W.subset(w, np.random.default_rng(n).permutation(2 * n)[:n])
    for engine in (0, 1):
        got = run_gpu(ctx, torch_dev, w, engine, max_iter=100_000)
        ref = run_oracle(w, max_iter=100_000)
        assert_same(got, ref, what=f"n={n} engine={engine}")


def test_empty_batches(ctx, torch_dev):
    """n = 0 on the device, host and indexed entry points returns without
    launching anything, and the context stays usable."""
    torch, dev = torch_dev
    for engine in (0, 1):
        ctx.set_engine(engine)
        r = ctx.batch_device(torch.empty((24, 0), dtype=torch.float64, device=dev),
                             torch.empty(0, dtype=torch.uint8, device=dev))
        torch.cuda.synchronize()
        assert r.toi.numel() == 0 and r.status.numel() == 0
    rh = ctx.batch_host(np.empty((24, 0)))
    assert rh.toi.size == 0
    v = torch.zeros((1, 3), dtype=torch.float64, device=dev)
    ri = ctx.batch_indexed(v, v, torch.empty((0, 4), dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    assert ri.toi.numel() == 0
    w = W.concat([W.uniform_vf(100, seed=21), W.edge_edge_mixed(100, seed=22)])
    for engine in (0, 1):
        got = run_gpu(ctx, torch_dev, w, engine, max_iter=100_000)
        assert_same(got, run_oracle(w, max_iter=100_000), what=f"after empty batches, engine {engine}")


def test_invalid_queries_on_device(ctx, torch_dev):
    w = W.uniform_vf(64, seed=15)
    w["pos"] = w["pos"].copy()
    w["pos"][3, 5] = np.nan
    w["pos"][7, 9] = np.inf
    w["pos"][0, 11] = 2e300
    dq = np.full(64, 1e-6)
    dq[20] = 0.0
    dq[21] = -1.0
    mq = np.full(64, 1000, np.int64)
    mq[30] = 0
    sq = np.zeros(64)
    sq[40] = 10.0  # not below gamma
    got = run_gpu(ctx, torch_dev, w, 0, delta_q=dq, max_iter_q=mq, min_sep_q=sq)
    ref = run_oracle(w, delta_q=dq, max_iter_q=mq, min_sep_q=sq)
    bad = np.array([5, 9, 11, 20, 21, 30, 40])
    assert np.all(got["status"][bad] == 0x80) and np.all(got["hit"][bad] == 0)
    assert np.all(np.isnan(got["toi"][bad]))
    ok = np.setdiff1d(np.arange(64), bad)
    assert np.all(ref["status"][bad] == 0xFF)
    sub = {k: ref[k][ok] for k in FIELDS}
    assert_same(got, sub, idx=ok, what="valid queries next to invalid ones")


def test_host_batch_validates_before_launch(ccdmod, ctx, torch_dev):
    w = W.uniform_vf(32, seed=16)
    res = ctx.batch_host(w["pos"], w["kind"], max_iter=10_000)
    ref = run_oracle(w, max_iter=10_000)
    assert_same({k: getattr(res, k) for k in FIELDS}, ref, what="host batch")
    pos = w["pos"].copy()
    pos[2, 3] = np.nan
    with pytest.raises(ccdmod.CCDError) as e:
        ctx.batch_host(pos, w["kind"])
    assert e.value.code == ccdmod.EINVAL
    with pytest.raises(ccdmod.CCDError):
        ctx.batch_host(w["pos"], w["kind"], delta=0.0)


def test_repeatable(ctx, torch_dev):
    w = W.simulation_mixed(50_000, seed=17)
    a = run_gpu(ctx, torch_dev, w, 0)
    b = run_gpu(ctx, torch_dev, w, 0)
    c = run_gpu(ctx, torch_dev, w, 1)
    assert_same(a, b, what="repeat")
    assert_same(a, c, what="plain vs persistent")


def test_full_size_simulation_sampled(ctx, torch_dev):
    """1M simulation-shaped queries at delta = 1e-6 in the benchmark's launch
    configuration; a seeded sample (every class represented) is checked
    against the oracle query by query."""
    w = W.simulation_mixed(1_000_000, seed=2)
    got = run_gpu(ctx, torch_dev, w, 0)
    rng = np.random.default_rng(99)
    idx = np.concatenate([rng.choice(np.nonzero(w["cls"] == c)[0], size=min(k, int((w["cls"] == c).sum())),
                                     replace=False) for c, k in ((0, 1500), (8, 40), (9, 200))])
    ws = W.subset(w, idx)
    ref = run_oracle(ws)
    assert_same(got, ref, idx=idx, what="simulation_mixed_1M sample")
    # every grazing contact (exact touching) is reported
    assert got["hit"][w["cls"] == 9].all()


def test_full_size_edge_edge_sampled(ctx, torch_dev):
    w = W.edge_edge_mixed(100_000, seed=1)
    got = run_gpu(ctx, torch_dev, w, 0)
    rng = np.random.default_rng(98)
    idx = np.concatenate([rng.choice(np.nonzero(w["cls"] == c)[0], size=k, replace=False)
                          for c, k in ((0, 400), (1, 400), (2, 8), (3, 8), (4, 8), (5, 8), (6, 8), (7, 8))])
    ws = W.subset(w, idx)
    ref = run_oracle(ws)
    assert_same(got, ref, idx=idx, what="edge_edge_mixed_100k sample")
    # constructed crossings are always found
    assert got["hit"][w["cls"] == 1].all()


@pytest.mark.parametrize("scale,delta", [(1.0, 1e-8), (64.0, 1e-7)])
def test_deep_levels(ctx, torch_dev, scale, delta):
    """Small delta / large coordinates drive the total bisection depth past 64,
    so the group engine moves from one-word to three-word box keys mid-query;
    a one-check lane budget sends every query there."""
    w = W.concat([W.uniform_vf(300, seed=31), W.edge_edge_mixed(300, seed=32, degenerate_frac=0.0)])
    w["pos"] = w["pos"] * scale
    ref = run_oracle(w, delta=delta)
    for tune in ({}, {"lane_budget": 1}, {"lane_budget": 1, "group_waves": 4}):
        if tune:
            ctx.set_tuning(**tune)
        got = run_gpu(ctx, torch_dev, w, 0, delta=delta)
        assert_same(got, ref, what=f"deep levels scale={scale} delta={delta} tuning={tune}")
    r = oracle.solve(0, w["pos"][:, 1], delta)
    assert sum(r.depth) > 64


def test_graph_replays_match_eager(ctx, torch_dev):
    """The captured launch sequence is replayed several times, with eager
    launches and synchronisations in between; every replay must equal the
    eager result (and the oracle)."""
    torch, dev = torch_dev
    w = W.concat([W.simulation_mixed(6000, seed=40), W.edge_edge_mixed(2000, seed=41)])
    ref = run_oracle(w, max_iter=200_000)
    ctx.enable_graphs(False)
    eager = run_gpu(ctx, torch_dev, w, 0, max_iter=200_000)
    assert_same(eager, ref, what="eager")
    ctx.enable_graphs(True)
    pos = torch.from_numpy(w["pos"]).to(dev)
    kind = torch.from_numpy(w["kind"]).to(dev)
    out = None
    for rep in range(4):
        out = ctx.batch_device(pos, kind, max_iter=200_000, out=out)
        torch.cuda.synchronize()
        got = {k: getattr(out, k).cpu().numpy() for k in FIELDS}
        got["n_checks"] = got["n_checks"].astype(np.uint64)
        assert_same(got, ref, what=f"graph replay {rep}")
        # eager work on the same stream between replays
        (pos * 2.0).sum().item()
        torch.cuda.synchronize()
    builds, replays = ctx.graph_counts()
    assert builds >= 1 and replays >= 3


def test_autotune_and_cache(ctx, torch_dev, tmp_path):
    torch, dev = torch_dev
    w = W.concat([W.simulation_mixed(20000, seed=50), W.edge_edge_mixed(2000, seed=51)])
    pos = torch.from_numpy(w["pos"]).to(dev)
    kind = torch.from_numpy(w["kind"]).to(dev)
    best, ms = ctx.autotune(pos, kind, max_trials=8)
    assert ms > 0 and best == ctx.tuning()
    ref = run_oracle(w)
    assert_same(run_gpu(ctx, torch_dev, w, 0), ref, what="after autotune")
    path = str(tmp_path / "tuning.txt")
    ctx.tuning_cache_store(path, "sim22k")
    from paper_2009_13349_amd import ccd
    with ccd.Context(0) as c2:
        assert not c2.tuning_cache_load(path, "other")
        assert c2.tuning_cache_load(path, "sim22k")
        assert c2.tuning() == best
