"""The allocation-free entry point (ccd_batch_noalloc) against ccd_batch,
through the C ABI: two calls in a row on the same GPU, the second with fewer
queries (the static scratch keeps the first call's contents), every output
field identical bit for bit to ccd_batch's on the same inputs."""
import numpy as np
import pytest

from paper_2009_13349_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("toi", "t_width", "hit", "n_checks", "status")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def _host(r):
    return {k: getattr(r, k).cpu().numpy() for k in FIELDS}


def _same(a, b, what):
    for k in FIELDS:
        x, y = np.ascontiguousarray(a[k]), np.ascontiguousarray(b[k])
        if k in ("toi", "t_width"):
            x, y = x.view(np.int64), y.view(np.int64)
        bad = np.nonzero(x != y)[0]
        assert len(bad) == 0, f"{what}: {k} differs at {len(bad)} queries, first {bad[:5].tolist()}"


def test_noalloc_matches_batch_twice(torch_dev):
    from paper_2009_13349_amd import ccd
    torch, dev = torch_dev
    big = W.concat([W.simulation_mixed(40_000, seed=61), W.edge_edge_mixed(4_000, seed=62)])
    small = W.concat([W.uniform_vf(3_000, seed=63), W.simulation_mixed(5_000, seed=64)])
    with ccd.Context(0) as ctx:
        for w, what in ((big, "first call, 44,000 queries"), (small, "second call, 8,000 queries")):
            pos = torch.from_numpy(np.ascontiguousarray(w["pos"])).to(dev)
            kind = torch.from_numpy(np.ascontiguousarray(w["kind"])).to(dev)
            ref = _host(ctx.batch_device(pos, kind, max_iter=300_000))
            torch.cuda.synchronize()
            got = _host(ctx.batch_noalloc(pos, kind, max_iter=300_000))
            torch.cuda.synchronize()
            assert np.count_nonzero(ref["hit"]) > 0
            _same(got, ref, what)
        # per-query parameters and the plain engine on the same array
        w = small
        n = w["pos"].shape[1]
        rng = np.random.default_rng(5)
        dq = torch.from_numpy(np.exp(rng.uniform(np.log(1e-6), np.log(1e-4), n))).to(dev)
        mq = torch.from_numpy(rng.integers(1, 100_000, n).astype(np.int64)).to(dev)
        pos = torch.from_numpy(np.ascontiguousarray(w["pos"])).to(dev)
        kind = torch.from_numpy(np.ascontiguousarray(w["kind"])).to(dev)
        for engine in (ccd.ENGINE_PERSISTENT, ccd.ENGINE_PLAIN):
            ctx.set_engine(engine)
            ref = _host(ctx.batch_device(pos, kind, delta_q=dq, max_iter_q=mq))
            got = _host(ctx.batch_noalloc(pos, kind, delta_q=dq, max_iter_q=mq))
            torch.cuda.synchronize()
            _same(got, ref, f"per-query parameters, engine {engine}")


def test_noalloc_rejects_oversized_batches(torch_dev):
    """A batch whose plan does not fit the static array is refused before any
    launch (checked on the host; the inputs are never read)."""
    from paper_2009_13349_amd import ccd
    torch, dev = torch_dev
    n = 3_000_000
    pos = torch.zeros((24, n), dtype=torch.float64, device=dev)
    with ccd.Context(0) as ctx:
        with pytest.raises(ccd.CCDError) as e:
            ctx.batch_noalloc(pos, None)
        assert e.value.code == ccd.ENOMEM
        # the context and the array stay usable
        w = W.uniform_vf(500, seed=65)
        p = torch.from_numpy(np.ascontiguousarray(w["pos"])).to(dev)
        k = torch.from_numpy(np.ascontiguousarray(w["kind"])).to(dev)
        ref = _host(ctx.batch_device(p, k))
        got = _host(ctx.batch_noalloc(p, k))
        torch.cuda.synchronize()
        _same(got, ref, "after a rejected batch")
