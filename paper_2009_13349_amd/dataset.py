"""Reader, writer and evaluator for the paper's CCD query files (appendix
"Dataset Format").

One query is an 8 x 7 block of CSV rows: row k is input point k (points
0..3 at t = 0, 4..7 at t = 1), columns are the numerator and denominator of
x, y and z, as decimal integer strings of any length, and the last column is
the ground truth (1: the pair collides).  Several blocks follow each other in
one file.  The coordinates are stored as exact rationals; converting one to a
double rounds to nearest, which is exact for the dataset's values (they were
doubles to begin with).

`evaluate` runs a file through the GPU root finder and counts false positives
(hit without a ground-truth collision) and false negatives (ground-truth
collision missed), the two error columns of the paper's benchmark.
"""
from __future__ import annotations

import csv
from fractions import Fraction

import numpy as np


def _to_double(num: str, den: str) -> float:
    return float(Fraction(int(num), int(den)))


def read_queries(path: str):
    """Returns (pos float64 [24, n], truth uint8 [n]) from one query file.
    Raises ValueError on a malformed block (wrong row or column count, zero
    denominator, ground truth not constant within a block)."""
    rows = []
    with open(path, newline="") as f:
        for r in csv.reader(f):
            r = [c.strip() for c in r]
            if not r or all(c == "" for c in r):
                continue
            if len(r) != 7:
                raise ValueError(f"{path}: a row has {len(r)} columns, expected 7")
            rows.append(r)
    if len(rows) % 8:
        raise ValueError(f"{path}: {len(rows)} rows is not a multiple of 8")
    n = len(rows) // 8
    pos = np.empty((24, n))
    truth = np.empty(n, np.uint8)
    for q in range(n):
        block = rows[8 * q: 8 * q + 8]
        t = {int(r[6]) for r in block}
        if len(t) != 1 or not t <= {0, 1}:
            raise ValueError(f"{path}: query {q}: ground truth {sorted(t)} is not one 0/1 value")
        truth[q] = t.pop()
        for k, r in enumerate(block):
            for c in range(3):
                if int(r[2 * c + 1]) == 0:
                    raise ValueError(f"{path}: query {q}: zero denominator")
                pos[3 * k + c, q] = _to_double(r[2 * c], r[2 * c + 1])
    return pos, truth


def write_queries(path: str, pos: np.ndarray, truth) -> None:
    """Writes queries in the same format (exact rationals of the doubles)."""
    pos = np.asarray(pos, dtype=np.float64)
    truth = np.asarray(truth).astype(np.uint8)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        for q in range(pos.shape[1]):
            for k in range(8):
                row = []
                for c in range(3):
                    fr = Fraction(float(pos[3 * k + c, q]))
                    row += [str(fr.numerator), str(fr.denominator)]
                w.writerow(row + [str(int(truth[q]))])


def evaluate(ctx, path: str, kind: int, delta: float = 1e-6, max_iter: int = 1_000_000,
             min_sep: float = 0.0) -> dict:
    """Runs one query file (all queries of one kind, as in the dataset's
    vertex-face and edge-edge folders) on the GPU and counts FP / FN."""
    import torch
    pos, truth = read_queries(path)
    n = pos.shape[1]
    dev = torch.device("cuda", ctx.device) if hasattr(ctx, "device") else torch.device("cuda:0")
    p = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    r = ctx.batch_device(p, None, default_kind=kind, delta=delta, max_iter=max_iter,
                         min_sep=min_sep)
    torch.cuda.synchronize()
    hit = r.hit.cpu().numpy().astype(bool)
    gt = truth.astype(bool)
    return {"queries": n, "collisions": int(gt.sum()), "hits": int(hit.sum()),
            "false_positives": int((hit & ~gt).sum()), "false_negatives": int((~hit & gt).sum()),
            "invalid": int((r.status.cpu().numpy() & 0x80).astype(bool).sum())}
