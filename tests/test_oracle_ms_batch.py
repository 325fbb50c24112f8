"""Pins of two oracle rules that GPU parity alone cannot check (CPU-only).

1. Minimum separation (Sec. 6.1, eq. msccd-error): the box is enlarged by d
   for the filter test, but its width is measured on the un-enlarged box
   B = B_F(I).  Were the width taken on the enlarged box (w(B) + 2d), no
   colliding query with 2d >= delta could ever end by the width test and every
   one would run into m_I; with the un-enlarged width the returns below end by
   width after few checks, and their boxes obey the exact accuracy bound that
   follows from the filter and the width test.
2. The batch driver's per-query parameter arrays (Alg. 2 inputs delta and m_I,
   Sec. 6.1's d per query): the batch result equals a loop of single solves
   with each query's own parameters.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact

VF, EE = 0, 1
U = Fraction(1, 2 ** 52)

TRI = [[0, 0, 0], [1, 0, 0], [0, 1, 0]]


def q(p0, p1):
    return np.array(list(p0) + list(p1), dtype=float).reshape(24)


def _accuracy_bound_holds(orc, kind, X, r, delta, d):
    """At the 8 corners of the returned box every exact F^c satisfies
    |F^c| <= (d + delta + 2 eps_c)(1 + 2^-52).  The filter admits the box when
    fl(m - d) <= eps and fl(M + d) >= -eps; the width test gives
    fl(M - m) < delta; each computed corner value is within eps_c of the exact
    one (the filter's own bound, Sec. 5.2)."""
    eps = orc.filter_eps(kind, X, d)
    P = exact.frac_query(X)
    box = [Fraction(b) for b in r.box]
    lo, hi = exact.corner_hull(kind, P, box)
    for c in range(3):
        lim = (Fraction(d) + Fraction(delta) + 2 * Fraction(float(eps[c]))) * (1 + U)
        if not (-lim <= lo[c] and hi[c] <= lim):
            return False
    return True


@pytest.mark.parametrize("kind,X", [
    # H14: the point of H1 crosses the static triangle's interior at t = 1/2;
    # with d the L-infinity distance |z| = |1 - 2t| <= d first holds at
    # t* = 1/2 - d/2.
    (VF, q([[.25, .25, 1]] + TRI, [[.25, .25, -1]] + TRI)),
    # H15: the edges of H7 (B passes through A's midpoint at t = 1/2): again
    # |F_z| = |1 - 2t| <= d from t* = 1/2 - d/2 on.
    (EE, q([[-1, 0, 0], [1, 0, 0], [0, -1, 1], [0, 1, 1]],
           [[-1, 0, 0], [1, 0, 0], [0, -1, -1], [0, 1, -1]])),
], ids=["H14_vf_ms_width", "H15_ee_ms_width"])
@pytest.mark.parametrize("d", [2.0 ** -10, 2.0 ** -14])
def test_ms_hand_case_ends_by_width(orc, kind, X, d):
    # delta = d < 2d: a width taken on the enlarged box (w(B) + 2d) could never
    # pass; the colliding region {|F| <= d} is a solid block of about (2d)^2 d
    # in (u, v, t), so an accuracy delta much finer than d would need far more
    # than m_I boxes
    delta = d
    r = orc.solve(kind, X, delta, 100_000, d)
    t_star = 0.5 - d / 2
    eps = max(orc.filter_eps(kind, X, d))
    assert r.hit == 1
    assert r.status == 0, "must end by the width test on the un-enlarged box"
    assert r.n_checks < 5_000
    # F_z moves at speed 2: the first box whose enlarged image reaches the
    # filter starts at most (delta + 2 eps) / 2 before t*
    assert t_star - delta - 2 * eps <= r.toi <= t_star
    assert _accuracy_bound_holds(orc, kind, X, r, delta, d)


def test_ms_width_terminated_returns_on_generator(orc):
    """Config-3 geometry (the simulation-shaped generator with pairs passing
    within U(0, 2 d) of each other), d = 1e-4 and delta = 1e-4 < 2d: most
    band pairs end by the width test after about a thousand checks, and every
    such return meets the exact accuracy bound."""
    from paper_2009_13349_amd import workloads as W
    d, delta, mI = 1e-4, 1e-4, 1_000_000
    w = W.min_separation(4000, seed=2, d_min=d, delta=delta)
    band = np.nonzero(w["cls"] == 10)[0]
    assert len(band) > 150
    width_ends = 0
    for i in band:
        kind, X = int(w["kind"][i]), w["pos"][:, i]
        r = orc.solve(kind, X, delta, mI, d)
        if r.hit and r.status == 0:
            assert r.n_checks < mI // 100
            assert _accuracy_bound_holds(orc, kind, X, r, delta, d)
            width_ends += 1
        if not r.hit:
            assert exact.exclusion_proof(kind, X, d=d, max_boxes=100_000) is not False
    assert width_ends > len(band) // 2


def _mixed_queries(n_each=120):
    from paper_2009_13349_amd import workloads as W
    return W.concat([W.uniform_vf(n_each, seed=31), W.edge_edge_mixed(n_each, seed=32),
                     W.simulation_mixed(n_each, seed=33)])


def test_solve_batch_per_query_parameters_equal_single_solves(orc):
    """Alg. 2's inputs per query: delta, m_I and d drawn per query (d = 0 for
    some); every output field of the batch driver equals the single solve."""
    w = _mixed_queries()
    n = w["pos"].shape[1]
    rng = np.random.default_rng(77)
    delta = np.exp(rng.uniform(np.log(1e-8), np.log(1e-2), size=n))
    max_iter = rng.choice(np.array([1, 2, 3, 7, 40, 500, 20_000], np.int64), size=n)
    min_sep = np.where(rng.uniform(size=n) < 0.5, 0.0, 2.0 ** rng.integers(-14, -6, size=n))
    b = orc.solve_batch(w["pos"], w["kind"], delta=delta, max_iter=max_iter, min_sep=min_sep)
    assert b["invalid"] == 0
    for i in range(n):
        r = orc.solve(int(w["kind"][i]), w["pos"][:, i], float(delta[i]), int(max_iter[i]),
                      float(min_sep[i]))
        assert b["toi"][i] == r.toi or (np.isnan(b["toi"][i]) and np.isnan(r.toi)), i
        assert b["t_width"][i] == r.t_width, i
        assert b["hit"][i] == r.hit and b["status"][i] == r.status, i
        assert int(b["n_checks"][i]) == r.n_checks, i
    # the parameters matter: a batch with the parameters of query 0 for all
    # differs on many queries
    s = orc.solve_batch(w["pos"], w["kind"], delta=float(delta[0]), max_iter=int(max_iter[0]),
                        min_sep=float(min_sep[0]))
    assert np.count_nonzero(s["n_checks"] != b["n_checks"]) > n // 4


def test_solve_batch_per_query_delta_alone(orc):
    """Only delta varies per query (m_I and d scalar): queries with a wide
    delta end after fewer checks than with a narrow one, as single solves say."""
    w = _mixed_queries(60)
    n = w["pos"].shape[1]
    delta = np.where(np.arange(n) % 2 == 0, 1e-2, 1e-8)
    b = orc.solve_batch(w["pos"], w["kind"], delta=delta, max_iter=200_000)
    for i in range(n):
        r = orc.solve(int(w["kind"][i]), w["pos"][:, i], float(delta[i]), 200_000)
        assert int(b["n_checks"][i]) == r.n_checks and b["toi"][i] == r.toi, i
