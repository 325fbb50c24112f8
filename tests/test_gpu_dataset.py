"""GPU evaluation of a query file in the paper's format: the false positive and
false negative counts equal the oracle's, and there are no false negatives."""
import numpy as np
import pytest

import oracle
from paper_2009_13349_amd import dataset, workloads as W
from tests.test_dataset_cpu import synthetic_file

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_13349_amd import ccd
    c = ccd.Context(0)
    yield c
    c.close()


def test_evaluate_matches_oracle(ctx, tmp_path):
    p = str(tmp_path / "vf.csv")
    synthetic_file(p, n=60, seed=94)
    got = dataset.evaluate(ctx, p, kind=0)
    pos, t = dataset.read_queries(p)
    r = oracle.solve_batch(pos, None, default_kind=0)
    hit, gt = r["hit"].astype(bool), t.astype(bool)
    assert got["queries"] == 60 and got["collisions"] == int(gt.sum())
    assert got["false_negatives"] == 0 == int((~hit & gt).sum())
    assert got["false_positives"] == int((hit & ~gt).sum())
    assert got["hits"] == int(hit.sum()) and got["invalid"] == 0
