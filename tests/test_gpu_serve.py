"""Serving (ccd_serve_*): continuous batching, admission by device memory,
results identical alone and in the mix."""
import numpy as np
import pytest

import oracle
from paper_2009_13349_amd import workloads as W

pytestmark = pytest.mark.gpu
FIELDS = ("toi", "t_width", "hit", "n_checks", "status")


@pytest.fixture(scope="module")
def ccdmod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_13349_amd import ccd
    ccd.load()
    return ccd


def same(a, b):
    for k in FIELDS:
        x, y = np.asarray(getattr(a, k) if not isinstance(a, dict) else a[k]), \
            np.asarray(getattr(b, k) if not isinstance(b, dict) else b[k])
        if k in ("toi", "t_width"):
            x, y = x.astype(np.float64).view(np.int64), y.astype(np.float64).view(np.int64)
        else:
            x, y = x.astype(np.int64), y.astype(np.int64)
        if not np.array_equal(x, y):
            return False
    return True


def requests(count, seed):
    rng = np.random.default_rng(seed)
    big = W.simulation_mixed(60_000, seed=seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(50), np.log(20_000))))
        off = int(rng.integers(0, 60_000 - n))
        w = W.subset(big, np.arange(off, off + n))
        delta = float(np.exp(rng.uniform(np.log(1e-6), np.log(1e-4))))
        out.append((w, delta))
    return out


def test_serve_mix_invariance_and_oracle(ccdmod):
    reqs = requests(24, seed=60)
    with ccdmod.Context(0) as ctx:
        alone = [ctx.batch_host(w["pos"], w["kind"], delta=d) for w, d in reqs]
    # a pool of ~1.5 of the largest request forces admission to wait for memory
    with ccdmod.Server(pool_bytes=6 << 20, streams=2, scratch_bytes=4 << 30,
                       max_queries_per_launch=30_000) as srv:
        tickets = [srv.submit(w["pos"], w["kind"], delta=d) for w, d in reqs]
        for t in tickets:
            srv.wait(t, timeout_ms=120_000)
        st = srv.stats()
        infos = [srv.info(t) for t in tickets]
    assert st["completed"] == len(reqs) and st["launches"] >= 2
    for (w, d), t, a in zip(reqs, tickets, alone):
        assert same(t.result, a)
    for (w, d), t in list(zip(reqs, tickets))[:6]:
        ref = oracle.solve_batch(w["pos"], w["kind"], delta=d)
        assert same(t.result, ref)
    for i in infos:
        assert i["state"] == 3 and i["rc"] == 0
        assert i["t_submit"] <= i["t_admit"] <= i["t_launch"] <= i["t_done"]


def test_serve_keeps_buffers_of_dropped_tickets(ccdmod):
    """A caller that drops its ticket references (here: an exception in the
    middle of submitting) must not leave the server writing into freed
    arrays; close() finishes the submitted requests."""
    reqs = requests(8, seed=64)
    with ccdmod.Server(pool_bytes=64 << 20, streams=2, scratch_bytes=4 << 30) as srv:
        def submit_all():
            ts = [srv.submit(w["pos"], w["kind"], delta=d) for w, d in reqs]
            raise RuntimeError("caller error after submitting")
        with pytest.raises(RuntimeError):
            submit_all()
        import gc
        gc.collect()
    assert True


def test_serve_errors(ccdmod):
    w = W.uniform_vf(64, seed=61)
    with ccdmod.Server(pool_bytes=64 << 10, streams=1, scratch_bytes=2 << 30,
                       max_queries_per_launch=10_000) as srv:
        big = W.uniform_vf(2000, seed=62)
        with pytest.raises(ccdmod.CCDError) as e:
            srv.submit(big["pos"], big["kind"])
        assert e.value.code == ccdmod.ENOMEM
        bad = w["pos"].copy()
        bad[0, 0] = np.nan
        with pytest.raises(ccdmod.CCDError) as e:
            srv.submit(bad, w["kind"])
        assert e.value.code == ccdmod.EINVAL
        t = srv.submit(w["pos"], w["kind"])
        srv.wait(t, 60_000)
        ref = oracle.solve_batch(w["pos"], w["kind"])
        assert same(t.result, ref)
        assert srv.release(t) == 0


def test_serve_many_small_concurrent(ccdmod):
    """Requests submitted from several threads while launches are running."""
    import threading
    reqs = requests(40, seed=63)
    results = [None] * len(reqs)
    with ccdmod.Server(streams=2, pool_bytes=256 << 20, scratch_bytes=4 << 30) as srv:
        def worker(idx):
            for i in idx:
                w, d = reqs[i]
                t = srv.submit(w["pos"], w["kind"], delta=d)
                results[i] = srv.wait(t, 120_000)
        th = [threading.Thread(target=worker, args=(range(k, len(reqs), 4),)) for k in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
    with ccdmod.Context(0) as ctx:
        for (w, d), r in zip(reqs, results):
            assert same(r, ctx.batch_host(w["pos"], w["kind"], delta=d))
