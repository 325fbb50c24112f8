"""Frontier storage and hand-offs between the engines, on the GPU through the C
ABI: the lane engine's LDS frontier (including the hand-off when a level's keys
would pass 64 bits), the group -> block hand-off that continues a wide query at
its current level, the restart fallback when the hand-off pool is full, and
the flagged overflow return when even the block engine's arena is too small.

Bar: bit-identical to the oracle (Alg. 2 replayed sequentially) wherever the
path completes; an overflowed query must carry CCD_ST_OVERFLOW, report a hit
and a toi no later than the oracle's (which is itself never later than the
first root), and no more checks than the oracle."""
import numpy as np
import pytest

from paper_2009_13349_amd import workloads as W

from test_gpu_parity import FIELDS, assert_same, ccdmod, ctx, run_gpu, run_oracle, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wide():
    """Simulation-shaped queries whose sequential run takes more than 2,000
    checks (levels of hundreds to thousands of boxes), with their oracle
    results, plus some light ones."""
    w = W.simulation_mixed(20_000, seed=41)
    ref = run_oracle(w)
    heavy = np.nonzero(ref["n_checks"] > 2000)[0]
    light = np.nonzero(ref["n_checks"] <= 2000)[0][:300]
    idx = np.concatenate([heavy[:160], light])
    ws = W.subset(w, idx)
    rs = {k: ref[k][idx] for k in FIELDS}
    assert len(heavy) >= 40
    return ws, rs


def test_group_to_block_continues_at_the_level(ctx, torch_dev, wide):
    """Small group arenas hand wide queries to the block engine at their
    current level (pool records), which goes on from there."""
    w, ref = wide
    ctx.set_tuning(lane_capacity=8, lane_budget=1, group_capacity=256)
    got = run_gpu(ctx, torch_dev, w, 0)
    st = ctx.last_stats()
    assert_same(got, ref, what="group -> block continuation")
    assert st["promoted"][1] > 0 and st["restarted"] == 0 and st["overflowed"] == 0
    assert st["handoff_words"] > 0
    # a continued query checks only its hand-off level twice; a restart redoes
    # every level before it.  (Which queries are handed on depends on timing:
    # a single-wave group also hands on a level of cap / 16 words or more
    # once its engine's records are all taken.)
    ctx.set_tuning(handoff_words=1)
    got_r = run_gpu(ctx, torch_dev, w, 0)
    st_r = ctx.last_stats()
    assert_same(got_r, ref, what="restart fallback")
    assert st_r["restarted"] == st_r["promoted"][1] > 0
    block_cont = sum(st["checks"][2]) / st["promoted"][1]
    block_restart = sum(st_r["checks"][2]) / st_r["promoted"][1]
    assert block_cont < block_restart, (block_cont, block_restart)


def test_four_wave_block_engines(ctx, torch_dev, wide):
    """Two block engines per CU (small block arenas so that they fit the
    budget) run as four-wave workgroups; same results."""
    w, ref = wide
    ctx.set_tuning(lane_capacity=8, lane_budget=1, group_capacity=256, block_capacity=65536,
                   block_count=2 * torch_dev[0].cuda.get_device_properties(0).multi_processor_count)
    got = run_gpu(ctx, torch_dev, w, 0)
    st = ctx.last_stats()
    assert_same(got, ref, what="four-wave block engines")
    assert st["promoted"][1] > 0 and st["restarted"] == 0 and st["overflowed"] == 0


def test_drained_group_queue_hands_wide_levels_on(ctx, torch_dev, wide):
    """Every record of the group engine is taken at once (fewer queries than
    groups): a level of at least cap / 16 words goes to the block engine
    before it is checked, with the same results."""
    w, ref = wide
    ctx.set_tuning(lane_capacity=8, lane_budget=1, group_capacity=4096)
    got = run_gpu(ctx, torch_dev, w, 0)
    st = ctx.last_stats()
    assert_same(got, ref, what="tail hand-off")
    assert st["promoted"][1] > 0 and st["restarted"] == 0 and st["overflowed"] == 0


def test_overflow_is_flagged_and_conservative(ctx, torch_dev, wide):
    """A block arena as small as a group arena: queries whose next level does
    not fit return at their current level's first colliding box, flagged."""
    w, ref = wide
    ctx.set_tuning(lane_capacity=8, lane_budget=1, group_capacity=256, block_capacity=256)
    for engine in (0, 1):
        got = run_gpu(ctx, torch_dev, w, engine)
        st = ctx.last_stats()
        flagged = (got["status"] & 0x08) != 0
        assert flagged.sum() > 0 and st["overflowed"] == int(flagged.sum())
        ok = np.nonzero(~flagged)[0]
        assert_same({k: got[k][ok] for k in FIELDS}, {k: ref[k][ok] for k in FIELDS},
                    what=f"unflagged queries, engine {engine}")
        f = np.nonzero(flagged)[0]
        assert np.all(got["hit"][f] == 1)
        assert np.all(got["toi"][f] <= ref["toi"][f])
        assert np.all(got["n_checks"][f] <= ref["n_checks"][f])
        assert np.all(got["t_width"][f] > 0)
        assert np.all((got["status"][f] & 0x07) == 0)


def test_lane_hands_on_levels_past_64_bits(ctx, torch_dev):
    """delta = 1e-10 drives converging queries past level 64 while their
    frontier is still narrow: the lane engine (one-word keys in LDS) hands them
    on at level 64 and the group engine finishes them with three-word boxes."""
    w = W.uniform_vf(1500, seed=43)
    ref = run_oracle(w, delta=1e-10, max_iter=200_000)
    for engine in (0, 1):
        ctx.set_tuning(lane_capacity=32, lane_budget=100_000)
        got = run_gpu(ctx, torch_dev, w, engine, delta=1e-10, max_iter=200_000)
        st = ctx.last_stats()
        assert_same(got, ref, what=f"deep levels, engine {engine}")
        assert st["deep"] > 0


@pytest.mark.parametrize("cap", [8, 16, 32])
def test_lane_capacities(ctx, torch_dev, cap):
    """Every lane capacity the LDS frontier supports, both engines."""
    w = W.concat([W.uniform_vf(600, seed=44), W.edge_edge_mixed(600, seed=45),
                  W.simulation_mixed(3000, seed=46)])
    ref = run_oracle(w, max_iter=100_000)
    ctx.set_tuning(lane_capacity=cap, lane_budget=512)
    for engine in (0, 1):
        got = run_gpu(ctx, torch_dev, w, engine, max_iter=100_000)
        assert_same(got, ref, what=f"lane capacity {cap}, engine {engine}")


@pytest.mark.parametrize("tune", [
    {"group_lds_words": 64},                       # levels of more than one chunk spill to HBM
    {"group_lds_words": 512},
    {"group_lds_words": 512, "group_capacity": 256, "block_lds_words": 64},
    {"group_lds_words": 0, "group_capacity": 256, "block_lds_words": 4096},
    {"group_lds_words": 512, "group_waves": 8},
    {"group_lds_words": 512, "group_occupancy": 2},  # no LDS variant: plain HBM arena
])
def test_group_levels_staged_in_lds(ctx, torch_dev, wide, tune):
    """The first words of every level in LDS, the rest in the HBM arena, at
    sizes that make most levels straddle the boundary, in the group and the
    block engine (with the lane engine handing everything on)."""
    w, ref = wide
    ctx.set_tuning(lane_capacity=8, lane_budget=1, **tune)
    for engine in (0, 1):
        got = run_gpu(ctx, torch_dev, w, engine)
        assert_same(got, ref, what=f"LDS-staged levels {tune}, engine {engine}")
        assert ctx.last_stats()["overflowed"] == 0
