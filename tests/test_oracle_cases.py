"""Hand-built CCD cases with answers derived by hand, and exact-arithmetic
properties of the oracle (zero false negatives, toi <= first contact, accuracy
of width-terminated returns).  CPU-only."""
import math
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import exact

VF, EE = 0, 1
DELTA = 1e-6
D = 2.0 ** -10  # minimum separation used by the MS cases


def q(p0, p1):
    return np.array(list(p0) + list(p1), dtype=float).reshape(24)


TRI = [[0, 0, 0], [1, 0, 0], [0, 1, 0]]

# (name, kind, X, min_sep, expectation, t_star)
#  expectation: "hit_at" (toi in [t* - delta - slack, t*]), "hit_le" (toi <= t*),
#               "zero" (toi == 0), "miss".
#  H10 and H11 have one-dimensional root sets after t* (B keeps passing through
#  A), and the set where |F| <= d in H12 is a solid box, so those searches may
#  end by the m_I cap; only toi <= t* is guaranteed.
CASES = [
    ("H1_vf_crossing", VF, q([[.25, .25, 1]] + TRI, [[.25, .25, -1]] + TRI), 0.0, "hit_at", 0.5),
    ("H2_vf_miss", VF, q([[.75, .75, 1]] + TRI, [[.75, .75, -1]] + TRI), 0.0, "miss", None),
    ("H3_vf_touch_t0", VF, q([[.25, .25, 0]] + TRI, [[.25, .25, -1]] + TRI), 0.0, "zero", 0.0),
    ("H4_vf_touch_t1", VF, q([[.25, .25, 1]] + TRI, [[.25, .25, 0]] + TRI), 0.0, "hit_at", 1.0),
    ("H5_vf_static_apart", VF, q([[.25, .25, .5]] + TRI, [[.25, .25, .5]] + TRI), 0.0, "miss", None),
    ("H6_vf_static_touch", VF, q([[.25, .25, 0]] + TRI, [[.25, .25, 0]] + TRI), 0.0, "zero", 0.0),
    ("H7_ee_crossing", EE, q([[-1, 0, 0], [1, 0, 0], [0, -1, 1], [0, 1, 1]],
                             [[-1, 0, 0], [1, 0, 0], [0, -1, -1], [0, 1, -1]]), 0.0, "hit_at", 0.5),
    ("H8_ee_parallel_apart", EE, q([[-1, 0, 0], [1, 0, 0], [-1, 1, 0], [1, 1, 0]],
                                   [[-1, 0, 0], [1, 0, 0], [-1, .5, 0], [1, .5, 0]]), 0.0, "miss", None),
    ("H9_ee_collinear_overlap", EE, q([[0, 0, 0], [1, 0, 0], [.5, 0, 0], [1.5, 0, 0]],
                                      [[0, 0, 0], [1, 0, 0], [.5, 0, 0], [1.5, 0, 0]]), 0.0, "zero", 0.0),
    ("H10_ee_endpoint_on_edge", EE, q([[-1, 0, 0], [1, 0, 0], [.25, 0, 1], [.25, 0, 2]],
                                      [[-1, 0, 0], [1, 0, 0], [.25, 0, -1], [.25, 0, 0]]), 0.0,
     "hit_le", 0.5),
    ("H11_ee_coplanar_slide", EE, q([[0, 0, 0], [1, 0, 0], [.5, 1, 0], [.5, 2, 0]],
                                    [[0, 0, 0], [1, 0, 0], [.5, -1, 0], [.5, 0, 0]]), 0.0,
     "hit_le", 0.5),
    # L-infinity minimum separation (Sec. 6): the point passes the vertex v1 at
    # (-7/8 d, -7/8 d) in the plane z = 0: Euclidean distance 1.24 d > d, but
    # L-infinity distance 7/8 d <= d, reached for |z| <= d, i.e. t >= 1/2 - d/2.
    ("H12_ms_linf_hit", VF, q([[-.875 * D, -.875 * D, 1]] + TRI, [[-.875 * D, -.875 * D, -1]] + TRI),
     D, "hit_le", 0.5 - D / 2),
    ("H13_ms_linf_miss", VF, q([[-1.5 * D, -1.5 * D, 1]] + TRI, [[-1.5 * D, -1.5 * D, -1]] + TRI),
     D, "miss", None),
]


@pytest.mark.parametrize("name,kind,X,min_sep,expect,t_star", CASES, ids=[c[0] for c in CASES])
def test_hand_cases(orc, name, kind, X, min_sep, expect, t_star):
    r = orc.solve(kind, X, DELTA, 1_000_000, min_sep)
    if expect == "miss":
        assert r.hit == 0 and r.toi == math.inf and r.t_width == 0.0
        assert exact.exclusion_proof(kind, X, d=min_sep) is True
        return
    assert r.hit == 1
    if expect == "zero":
        assert r.toi == 0.0
    elif expect == "hit_le":
        assert r.toi <= t_star
    else:
        eps = max(orc.filter_eps(kind, X, min_sep))
        assert t_star - DELTA - 2 * eps <= r.toi <= t_star


def test_h9_terminates_by_cap(orc):
    # collinear overlapping static edges: the root set is two-dimensional, the
    # search runs into m_I and returns the first colliding box of that level.
    r = orc.solve(EE, CASES[8][2], DELTA, 10_000)
    assert r.toi == 0.0 and r.status & orc.ST_CAP and r.n_checks == 10_000


# ---------------------------------------------------------------------------
# Exact properties on small dyadic inputs

coord = st.integers(min_value=-16, max_value=16).map(lambda k: k / 16)
query = st.lists(coord, min_size=24, max_size=24)


def _check_no_false_negative_and_first_root(orc, kind, X, delta, min_sep=0.0):
    r = orc.solve(kind, np.array(X), delta, 200_000, min_sep)
    if r.hit == 0:
        # zero false negatives: an exact proof that there is no contact
        assert exact.exclusion_proof(kind, X, d=min_sep, max_boxes=400_000) is True
    if min_sep == 0.0:
        status, t_first = exact.first_contact_univariate(kind, X)
        if status == "contact":
            assert r.hit == 1
            assert Fraction(r.toi) <= Fraction(str(t_first.evalf(60))) + Fraction(1, 10 ** 50)
    return r


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(query, st.sampled_from([VF, EE]))
def test_zero_false_negatives_random_dyadic(orc, X, kind):
    _check_no_false_negative_and_first_root(orc, kind, X, 1e-3)


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.lists(st.integers(-8, 8).map(lambda k: k / 8), min_size=12, max_size=12),
       st.lists(st.integers(-8, 8).map(lambda k: k / 8), min_size=12, max_size=12),
       st.sampled_from([VF, EE]), st.integers(0, 3))
def test_zero_false_negatives_degenerate_families(orc, a, b, kind, fam):
    """Static (b ignored), coplanar (z = 0 everywhere), shared-vertex and
    translated-copy families."""
    P0 = np.array(a, dtype=float).reshape(4, 3)
    P1 = np.array(b, dtype=float).reshape(4, 3)
    if fam == 0:
        P1 = P0.copy()
    elif fam == 1:
        P0[:, 2] = 0
        P1[:, 2] = 0
    elif fam == 2:
        P0[0] = P0[1]
        P1[0] = P1[1] + 0.125
    else:
        P1 = P0 + P1[0]
    X = q(P0, P1)
    _check_no_false_negative_and_first_root(orc, kind, X, 1e-3)


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(query, st.sampled_from([VF, EE]))
def test_min_separation_no_false_negatives(orc, X, kind):
    _check_no_false_negative_and_first_root(orc, kind, X, 1e-3, min_sep=2.0 ** -6)


def test_accuracy_of_width_terminated_returns(orc):
    """A box returned by the width or inside test satisfies, exactly at its 8
    corners, |F^c| <= d + delta (1 + 2^-52) + 2 eps_c (filter bound of Sec. 5.2)."""
    from paper_2009_13349_amd import workloads as W
    w = W.uniform_vf(256, seed=7)
    checked = 0
    for i in range(w["pos"].shape[1]):
        X = w["pos"][:, i]
        r = orc.solve(VF, X, 1e-4, 1_000_000)
        if not r.hit or r.status != 0:
            continue
        eps = orc.filter_eps(VF, X)
        P = exact.frac_query(X)
        box = [Fraction(b) for b in r.box]
        lim = [Fraction(1e-4) * (1 + Fraction(1, 2 ** 52)) + 2 * Fraction(e) for e in eps]
        lo, hi = exact.corner_hull(VF, P, box)
        for c in range(3):
            assert -lim[c] <= lo[c] and hi[c] <= lim[c]
        checked += 1
    assert checked > 50


def test_carry_never_later_than_literal(orc):
    """The carried pending box is the earliest candidate of its level, and the
    first colliding box of later levels never moves earlier, so the carry
    reading returns a toi no later than the literal algorithm (and flags the
    returns where it differs)."""
    from paper_2009_13349_amd import workloads as W
    w = W.edge_edge_mixed(2000, seed=3)
    diff = 0
    for i in range(w["pos"].shape[1]):
        X = w["pos"][:, i]
        rc = orc.solve(EE, X, 1e-6, 20_000, 0.0, literal=False)
        rl = orc.solve(EE, X, 1e-6, 20_000, 0.0, literal=True)
        assert rc.toi <= rl.toi
        if rc.toi != rl.toi:
            diff += 1
            assert rc.status & orc.ST_CARRY
    # the two readings agree on the overwhelming majority of queries
    assert diff <= 20


@pytest.mark.parametrize("which", ["uniform_vf", "edge_edge_generic"])
def test_first_contact_on_generated_crossings(orc, which):
    """On generated queries (half constructed to cross), the earliest contact
    found exactly by the univariate route is never before the oracle's toi,
    and every query with a contact is reported as a hit."""
    from paper_2009_13349_amd import workloads as W
    if which == "uniform_vf":
        w, kind = W.uniform_vf(48, seed=11), VF
    else:
        w, kind = W.edge_edge_mixed(48, seed=12, degenerate_frac=0.0), EE
    contacts = 0
    for i in range(w["pos"].shape[1]):
        X = w["pos"][:, i]
        r = orc.solve(kind, X, 1e-6, 1_000_000)
        status, t_first = exact.first_contact_univariate(kind, X)
        if status == "contact":
            contacts += 1
            assert r.hit == 1
            assert Fraction(r.toi) <= Fraction(str(t_first.evalf(60))) + Fraction(1, 10 ** 50)
        if r.hit == 0:
            assert status == "none"
            assert exact.exclusion_proof(kind, X, max_boxes=100_000) is True
    assert contacts >= 20
