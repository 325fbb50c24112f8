"""The paper's query-file format (appendix "Dataset Format"): exact rational
round trip, conversion of rationals that are not doubles, malformed files, and
false-negative-free evaluation by the oracle on a file whose ground truth comes
from exact first contacts.  CPU-only."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2009_13349_amd import dataset, workloads as W


def test_round_trip_is_exact(tmp_path):
    w = W.concat([W.uniform_vf(50, seed=91), W.edge_edge_mixed(50, seed=92)])
    truth = np.arange(100) % 2
    p = tmp_path / "q.csv"
    dataset.write_queries(str(p), w["pos"], truth)
    pos, t = dataset.read_queries(str(p))
    assert np.array_equal(pos.view(np.int64), w["pos"].view(np.int64))
    assert np.array_equal(t, truth)


def test_rationals_convert_to_nearest_double(tmp_path):
    big = 2 ** 200 + 1
    rows = [["1", "3", "-2", "7", str(big), str(2 ** 199), "1"]] + \
           [["0", "1", "5", "2", "-1", "1048576", "1"]] * 7
    p = tmp_path / "r.csv"
    p.write_text("\n".join(",".join(r) for r in rows) + "\n")
    pos, t = dataset.read_queries(str(p))
    assert pos.shape == (24, 1) and t.tolist() == [1]
    assert pos[0, 0] == 1 / 3 and pos[1, 0] == -2 / 7
    assert pos[2, 0] == float(Fraction(big, 2 ** 199)) == 2.0
    assert pos[3:6, 0].tolist() == [0.0, 2.5, -1 / 1048576]


@pytest.mark.parametrize("bad", ["cols", "rows", "truth", "zero"])
def test_malformed_files_rejected(tmp_path, bad):
    row = ["1", "2", "1", "2", "1", "2", "0"]
    rows = [list(row) for _ in range(8)]
    if bad == "cols":
        rows[3] = rows[3][:6]
    elif bad == "rows":
        rows = rows[:7]
    elif bad == "truth":
        rows[5][6] = "1"
    else:
        rows[2][1] = "0"
    p = tmp_path / "bad.csv"
    p.write_text("\n".join(",".join(r) for r in rows) + "\n")
    with pytest.raises(ValueError):
        dataset.read_queries(str(p))


def synthetic_file(path, n=40, seed=93):
    """Uniform vertex-face queries (half constructed to cross) with the ground
    truth of the exact univariate route."""
    w = W.uniform_vf(n, seed=seed)
    truth = np.array([exact.first_contact_univariate(0, w["pos"][:, i])[0] == "contact"
                      for i in range(n)], np.uint8)
    dataset.write_queries(path, w["pos"], truth)
    return truth


def test_oracle_on_a_file_has_no_false_negatives(tmp_path):
    p = str(tmp_path / "vf.csv")
    truth = synthetic_file(p)
    pos, t = dataset.read_queries(p)
    r = oracle.solve_batch(pos, None, default_kind=0)
    hit = r["hit"].astype(bool)
    assert t.sum() >= 15
    assert not np.any(~hit & t.astype(bool))  # no false negatives
