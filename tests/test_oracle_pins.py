"""Pins of the CPU oracle against facts that do not come from the oracle itself:
numbers printed in the paper, closed forms derived by hand, the paper's
propositions as invariants, special cases of the algorithm, and exact
rational arithmetic.  All CPU-only."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact

HERE = os.path.dirname(os.path.abspath(__file__))
VF, EE = 0, 1


def q(p0, p1):
    """4 points at t0 and the same 4 at t1 -> 24 doubles."""
    return np.array(list(p0) + list(p1), dtype=float).reshape(24)


# ---------------------------------------------------------------------------
# Filter constants (Sec. 5.2 eq. ccd-error, Sec. 6.1 eq. msccd-error)

def _golden_constants():
    out = {}
    with open(os.path.join(HERE, "golden", "filter_constants.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            mode, kind, val = line.split()
            out[(mode, kind)] = float(val)
    return out


@pytest.mark.parametrize("mode,kind", [("ccd", "ee"), ("ccd", "vf"), ("msccd", "ee"), ("msccd", "vf")])
def test_filter_constant_matches_paper(orc, mode, kind):
    K = _golden_constants()[(mode, kind)]
    X = np.zeros(24)  # gamma = 1 on every axis
    d = 1e-3 if mode == "msccd" else 0.0
    eps = orc.filter_eps(EE if kind == "ee" else VF, X, d)
    assert np.all(eps == K)


def test_filter_gamma_cubed_per_axis(orc):
    # gamma_c = max(1, max_k |x_k^c|) over the 8 input points, per axis.
    X = np.zeros(24)
    X[3 * 5 + 0] = -2.0   # point 5 (t1), x: gamma_x = 2
    X[3 * 1 + 1] = 0.5    # gamma_y stays 1
    X[3 * 7 + 2] = 10.0   # gamma_z = 10
    K = _golden_constants()[("ccd", "vf")]
    eps = orc.filter_eps(VF, X)
    assert eps[0] == K * 8
    assert eps[1] == K
    assert eps[2] == pytest.approx(K * 1000, rel=4e-16)


# ---------------------------------------------------------------------------
# F: closed forms derived by hand for specific geometry (Sec. 3)

def test_F_vf_closed_form(orc):
    # static triangle (0,0,0),(1,0,0),(0,1,0); p from (1/4,1/4,1) to (1/4,1/4,-1):
    # F(t,u,v) = (1/4 - u, 1/4 - v, 1 - 2t).
    X = q([[.25, .25, 1], [0, 0, 0], [1, 0, 0], [0, 1, 0]],
          [[.25, .25, -1], [0, 0, 0], [1, 0, 0], [0, 1, 0]])
    rng = np.random.default_rng(5)
    for _ in range(200):
        t, u, v = (rng.integers(0, 2 ** 20, 3) / 2 ** 20)
        got = orc.F(VF, X, t, u, v)
        assert list(got) == [0.25 - u, 0.25 - v, 1 - 2 * t]


def test_F_ee_closed_form(orc):
    # A = (-1,0,0)-(1,0,0) static; B = (0,-1,z)-(0,1,z), z: 1 -> -1:
    # F(t,u,v) = (2u - 1, 1 - 2v, 2t - 1).
    X = q([[-1, 0, 0], [1, 0, 0], [0, -1, 1], [0, 1, 1]],
          [[-1, 0, 0], [1, 0, 0], [0, -1, -1], [0, 1, -1]])
    rng = np.random.default_rng(6)
    for _ in range(200):
        t, u, v = (rng.integers(0, 2 ** 20, 3) / 2 ** 20)
        got = orc.F(EE, X, t, u, v)
        assert list(got) == [2 * u - 1, 1 - 2 * v, 2 * t - 1]


def test_F_vf_matches_printed_cubic(orc):
    """App. C prints the coplanarity cubic -72t^3 + 120t^2 - 44t + 3 of its first
    example.  For fixed t, F_vf is affine in (u, v): F = q - u e1 - v e2 with
    q = p - v1, e1 = v2 - v1, e2 = v3 - v1, and det[e1, e2, q] is that cubic.
    The inputs are small integers, so at dyadic t every operation is exact."""
    X = q([[1, 1, 0], [0, 0, 5], [2, 0, 2], [0, 1, 0]],
          [[1, 1, 0], [0, 0, -1], [0, 0, -2], [0, 7, 0]])
    for k in range(0, 33):
        t = k / 32
        F00 = orc.F(VF, X, t, 0, 0)
        F10 = orc.F(VF, X, t, 1, 0)
        F01 = orc.F(VF, X, t, 0, 1)
        qv = [Fraction(x) for x in F00]
        e1 = [Fraction(a) - Fraction(b) for a, b in zip(F00, F10)]
        e2 = [Fraction(a) - Fraction(b) for a, b in zip(F00, F01)]
        det = (e1[0] * (e2[1] * qv[2] - e2[2] * qv[1])
               - e1[1] * (e2[0] * qv[2] - e2[2] * qv[0])
               + e1[2] * (e2[0] * qv[1] - e2[1] * qv[0]))
        tf = Fraction(t)
        cubic = -72 * tf ** 3 + 120 * tf ** 2 - 44 * tf + 3
        assert det == cubic


def _dyadic(rng, shape, bits):
    return rng.integers(-2 ** bits, 2 ** bits, size=shape) / 2 ** bits


@pytest.mark.parametrize("kind", [VF, EE])
def test_F_vanishes_at_constructed_root(orc, kind):
    """Geometry built so that the primitives touch at a chosen (t*, u*, v*):
    F(t*, u*, v*) is exactly zero (all inputs dyadic with few bits, so the
    binary64 evaluation is exact), and moving any one parameter off the root
    makes F nonzero in general."""
    rng = np.random.default_rng(10 + kind)
    for _ in range(300):
        P0 = _dyadic(rng, (4, 3), 6)
        P1 = _dyadic(rng, (4, 3), 6)
        t, u, v = rng.integers(1, 16, 3) / 16
        if kind == VF:
            if u + v > 1:
                u, v = 1 - u, 1 - v
            pos_t = (1 - t) * P0 + t * P1
            target = (1 - u - v) * pos_t[1] + u * pos_t[2] + v * pos_t[3]
            shift = target - pos_t[0]
            P0[0] += shift
            P1[0] += shift
        else:
            pos_t = (1 - t) * P0 + t * P1
            a = (1 - u) * pos_t[0] + u * pos_t[1]
            b = (1 - v) * pos_t[2] + v * pos_t[3]
            P0[2:] += a - b
            P1[2:] += a - b
        X = q(P0, P1)
        assert list(orc.F(kind, X, t, u, v)) == [0.0, 0.0, 0.0]
        r = orc.solve(kind, X)
        assert r.hit == 1 and r.toi <= t


# ---------------------------------------------------------------------------
# Error bound of the filter (Sec. 5.2): |fl(F) - F| <= eps on every axis

@pytest.mark.parametrize("kind", [VF, EE])
def test_filter_bounds_rounding_error(orc, kind):
    rng = np.random.default_rng(20 + kind)
    worst = 0.0
    for trial in range(300):
        scale = 10.0 ** rng.uniform(0, 3)
        X = rng.uniform(-scale, scale, 24)
        if trial % 3 == 0:
            # near cancellation: all points close to one another
            X = np.tile(rng.uniform(-scale, scale, 3), 8) + rng.uniform(-1e-3, 1e-3, 24)
        eps = orc.filter_eps(kind, X)
        P = exact.frac_query(X)
        for _ in range(4):
            t, u, v = (rng.integers(0, 2 ** 30, 3) / 2 ** 30)
            got = orc.F(kind, X, t, u, v)
            ex = exact.F_exact(kind, P, Fraction(t), Fraction(u), Fraction(v))
            for c in range(3):
                err = abs(Fraction(got[c]) - ex[c])
                assert err <= Fraction(eps[c])
                worst = max(worst, float(err / Fraction(eps[c])))
    assert worst < 1.0


# ---------------------------------------------------------------------------
# Propositions of Sec. 5.2 as invariants

@pytest.mark.parametrize("kind", [VF, EE])
def test_prop1_corner_box_encloses_F(orc, kind):
    """Prop. 1: F on a box lies in the AABB of its 8 corner values (checked
    exactly at random interior points)."""
    rng = np.random.default_rng(30 + kind)
    for _ in range(100):
        X = rng.uniform(-1, 1, 24)
        P = exact.frac_query(X)
        lo = np.sort(rng.integers(0, 2 ** 10, (3, 2)) / 2 ** 10, axis=1)
        lo[:, 1] += 2 ** -10
        box = [lo[0, 0], lo[0, 1], lo[1, 0], lo[1, 1], lo[2, 0], lo[2, 1]]
        fbox = [Fraction(b) for b in box]
        hlo, hhi = exact.corner_hull(kind, P, fbox)
        for _ in range(5):
            pt = [fbox[2 * a] + Fraction(int(rng.integers(0, 1000)), 999) * (fbox[2 * a + 1] - fbox[2 * a])
                  for a in range(3)]
            val = exact.F_exact(kind, P, *pt)
            for c in range(3):
                assert hlo[c] <= val[c] <= hhi[c]
        # the oracle's floating-point box matches the exact hull within eps
        eps = orc.filter_eps(kind, X)
        _, _, _, flo, fhi = orc.box_check(kind, X, box, eps)
        for c in range(3):
            assert abs(Fraction(flo[c]) - hlo[c]) <= Fraction(eps[c])
            assert abs(Fraction(fhi[c]) - hhi[c]) <= Fraction(eps[c])


@pytest.mark.parametrize("kind", [VF, EE])
def test_prop2_codomain_width_bound(orc, kind):
    """Prop. 2: w(B_F(I)) <= (w_t k_t + w_u k_u + w_v k_v) / 3 (plus rounding)."""
    rng = np.random.default_rng(40 + kind)
    for _ in range(300):
        X = rng.uniform(-1, 1, 24) * 10.0 ** rng.uniform(0, 2)
        kap = orc.kappa(kind, X)
        eps = orc.filter_eps(kind, X)
        d = rng.integers(0, 12, 3)
        idx = [rng.integers(0, 2 ** int(di)) for di in d]
        w = [2.0 ** -int(di) for di in d]
        box = [idx[0] * w[0], (idx[0] + 1) * w[0], idx[1] * w[1], (idx[1] + 1) * w[1],
               idx[2] * w[2], (idx[2] + 1) * w[2]]
        _, _, width, _, _ = orc.box_check(kind, X, box, eps)
        bound = (w[0] * kap[0] + w[1] * kap[1] + w[2] * kap[2]) / 3
        assert width <= bound * (1 + 1e-12) + 2 * max(eps)


def test_kappa_closed_forms(orc):
    # eq. kappas on hand-built queries with F known in closed form
    X = q([[.25, .25, 1], [0, 0, 0], [1, 0, 0], [0, 1, 0]],
          [[.25, .25, -1], [0, 0, 0], [1, 0, 0], [0, 1, 0]])
    assert list(orc.kappa(VF, X)) == [6.0, 3.0, 3.0]   # F = (1/4-u, 1/4-v, 1-2t)
    X = q([[-1, 0, 0], [1, 0, 0], [0, -1, 1], [0, 1, 1]],
          [[-1, 0, 0], [1, 0, 0], [0, -1, -1], [0, 1, -1]])
    assert list(orc.kappa(EE, X)) == [6.0, 6.0, 6.0]   # F = (2u-1, 1-2v, 2t-1)
    Xs = q([[.25, .25, .5], [0, 0, 0], [1, 0, 0], [0, 1, 0]],
           [[.25, .25, .5], [0, 0, 0], [1, 0, 0], [0, 1, 0]])
    assert orc.kappa(VF, Xs)[0] == 0.0                  # static: no t dependence


def test_split_rule_tie_order(orc):
    # Alg. 2 SPLIT: largest w * kappa wins; ties go to t, then u, then v.
    assert orc.split_axis([1, 1, 1], [1, 1, 1]) == 0
    assert orc.split_axis([1, 1, 1], [0.5, 1, 1]) == 1
    assert orc.split_axis([1, 1, 1], [0.5, 0.5, 1]) == 2
    assert orc.split_axis([1, 1, 1], [0.5, 0.5, 0.5]) == 0
    assert orc.split_axis([2, 4, 4], [1, 0.5, 0.5]) == 0
    assert orc.split_axis([0, 3, 3], [1, 1, 1]) == 1
    assert orc.split_axis([0, 0, 0], [1, 1, 1]) == 0
    assert orc.split_axis([1, 2, 3], [1, 1, 1]) == 2


# ---------------------------------------------------------------------------
# Special cases of Alg. 2 with a closed-form answer

def test_max_iter_one_is_level_zero_decision(orc):
    rng = np.random.default_rng(50)
    for _ in range(200):
        kind = int(rng.integers(0, 2))
        X = rng.uniform(0, 1, 24)
        r = orc.solve(kind, X, 1e-6, 1)
        eps = orc.filter_eps(kind, X)
        col, _, _, _, _ = orc.box_check(kind, X, [0, 1, 0, 1, 0, 1], eps)
        if col:
            assert (r.toi, r.t_width, r.n_checks) == (0.0, 1.0, 1)
        else:
            assert (r.toi, r.t_width, r.hit) == (math.inf, 0.0, 0)


def test_static_query_never_splits_time(orc):
    rng = np.random.default_rng(51)
    for _ in range(100):
        kind = int(rng.integers(0, 2))
        P = rng.uniform(0, 1, (4, 3))
        X = q(P, P)
        r = orc.solve(kind, X, 1e-6, 10_000)
        assert r.toi in (0.0, math.inf)
        if r.hit:
            assert r.t_width == 1.0


def test_huge_delta_returns_zero_when_level0_collides(orc):
    X = q([[.25, .25, 1], [0, 0, 0], [1, 0, 0], [0, 1, 0]],
          [[.25, .25, -1], [0, 0, 0], [1, 0, 0], [0, 1, 0]])
    r = orc.solve(VF, X, 100.0, 1000)
    assert (r.toi, r.t_width, r.n_checks) == (0.0, 1.0, 1)


def test_invalid_inputs_rejected(orc):
    X = np.zeros(24)
    assert orc.validate(X, 1e-6, 10)
    assert not orc.validate(X, 0.0, 10)
    assert not orc.validate(X, -1.0, 10)
    assert not orc.validate(X, float("nan"), 10)
    assert not orc.validate(X, 1e-6, 0)
    assert not orc.validate(X, 1e-6, 10, -1e-3)
    assert not orc.validate(X, 1e-6, 10, 1.0)   # d must be below gamma (>= 1)
    Xn = X.copy()
    Xn[7] = float("inf")
    assert not orc.validate(Xn, 1e-6, 10)
    with pytest.raises(ValueError):
        orc.solve(VF, Xn)


# ---------------------------------------------------------------------------
# Worked examples printed in the paper (App. B and C)

def _paper_examples():
    rows = []
    with open(os.path.join(HERE, "golden", "paper_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, kind, a, b, expect = [s.strip() for s in line.split("|")]
            p0 = [float(x) for x in a.split()]
            p1 = [float(x) for x in b.split()]
            rows.append((name, VF if kind == "vf" else EE, np.array(p0 + p1), expect))
    return {r[0]: r for r in rows}


def test_app_b_hourglass(orc):
    _, kind, X, expect = _paper_examples()["app_b"]
    assert expect.startswith("hit")
    t_star = Fraction(1) - Fraction(0.1)
    assert t_star == Fraction(32425917317067571, 2 ** 55)
    # F vanishes at (t*, fl(0.1), fl(0.1)) in exact arithmetic
    P = exact.frac_query(X)
    assert exact.F_exact(kind, P, t_star, Fraction(0.1), Fraction(0.1)) == [0, 0, 0]
    r = orc.solve(kind, X)
    assert r.hit == 1 and r.status == 0
    assert Fraction(r.toi) <= t_star and float(t_star) - r.toi <= 1e-5
    # no contact at t = 1/2 (the triangle is a segment there)
    assert exact.exclusion_proof(kind, X, t_max=Fraction(1, 2)) is True


def test_app_c1_inflection_no_contact(orc):
    _, kind, X, expect = _paper_examples()["app_c1"]
    assert expect.startswith("nohit")
    coeffs = [int(c) for c in expect.split("=")[1].split(",")]
    poly = exact.coplanarity_cubic(kind, X)
    assert [int(c) for c in poly.all_coeffs()] == coeffs
    r = orc.solve(kind, X)
    assert r.hit == 0 and r.toi == math.inf and r.t_width == 0.0
    assert exact.first_contact_univariate(kind, X)[0] == "none"
    assert exact.exclusion_proof(kind, X) is True


def test_app_c2_coplanar_degenerate(orc):
    _, kind, X, expect = _paper_examples()["app_c2"]
    t_star = (Fraction(0.57) - Fraction(0.5)) / (Fraction(0.57) - Fraction(0.28))
    assert t_star == Fraction(630503947831869, 2612087783874887)
    assert exact.coplanarity_cubic(kind, X).is_zero   # all 8 points in z = 1
    r = orc.solve(kind, X)
    assert r.hit == 1 and Fraction(r.toi) <= t_star
    # no contact before t*: exclusion on [0, t* - 2^-20]
    assert exact.exclusion_proof(kind, X, t_max=t_star - Fraction(1, 2 ** 20)) is True
