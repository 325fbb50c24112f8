"""Pins of the oracle's shortened time interval I_t = [0, t_max] (Sec. 7.2: the
line search changes only the initial interval of Alg. 2).  Reading: the time
axis is bisected in s = t / t_max and a box's time endpoints are
fl(t_max * s).  The pins use exact arithmetic, exact first contacts and a
closed form, none of which comes from the oracle.  CPU-only."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact

VF, EE = 0, 1


def q(p0, p1):
    return np.array(list(p0) + list(p1), dtype=float).reshape(24)


TRI = [[0, 0, 0], [1, 0, 0], [0, 1, 0]]


def test_tmax_one_is_the_full_interval(orc):
    from paper_2009_13349_amd import workloads as W
    w = W.concat([W.uniform_vf(300, seed=41), W.edge_edge_mixed(300, seed=42)])
    a = orc.solve_batch(w["pos"], w["kind"])
    b = orc.solve_batch(w["pos"], w["kind"], t_max=1.0)
    for k in ("toi", "t_width"):
        assert np.array_equal(a[k].view(np.int64), b[k].view(np.int64))
    for k in ("hit", "n_checks", "status"):
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("kind", [VF, EE])
def test_filter_bounds_rounding_error_scaled_time(orc, kind):
    """eq. ccd-error bounds the rounding error of F at time values that are not
    dyadic (t = fl(t_max * s)), where 1 - t is itself rounded: exact rational
    evaluation at random corners."""
    rng = np.random.default_rng(60 + kind)
    worst = 0.0
    for trial in range(200):
        scale = 10.0 ** rng.uniform(0, 3)
        X = rng.uniform(-scale, scale, 24)
        if trial % 3 == 0:
            X = np.tile(rng.uniform(-scale, scale, 3), 8) + rng.uniform(-1e-3, 1e-3, 24)
        eps = orc.filter_eps(kind, X)
        P = exact.frac_query(X)
        for _ in range(4):
            t_max = float(rng.uniform(1e-3, 1.0))
            s, u, v = rng.integers(0, 2 ** 30, 3) / 2 ** 30
            t = t_max * s
            got = orc.F(kind, X, t, u, v)
            ex = exact.F_exact(kind, P, Fraction(t), Fraction(u), Fraction(v))
            for c in range(3):
                err = abs(Fraction(got[c]) - ex[c])
                assert err <= Fraction(eps[c])
                worst = max(worst, float(err / Fraction(eps[c])))
    assert worst < 1.0


@pytest.mark.parametrize("which", ["uniform_vf", "edge_edge_generic"])
def test_tmax_first_contact(orc, which):
    """Against the exact earliest contact t* (univariate route): with
    t* <= t_max the shortened search reports a hit no later than t*; with
    t_max < t* there is no contact in [0, t_max], and a reported miss must then
    be provable by exact exclusion on [0, t_max] (no false negatives)."""
    from paper_2009_13349_amd import workloads as W
    if which == "uniform_vf":
        w, kind = W.uniform_vf(40, seed=13), VF
    else:
        w, kind = W.edge_edge_mixed(40, seed=14, degenerate_frac=0.0), EE
    rng = np.random.default_rng(7)
    above = below = 0
    for i in range(w["pos"].shape[1]):
        X = w["pos"][:, i]
        status, t_first = exact.first_contact_univariate(kind, X)
        if status != "contact":
            continue
        t_star = Fraction(str(t_first.evalf(60)))
        ts = float(t_star)
        # t_max above t*: the contact is inside the shortened interval
        t_max = float(rng.uniform(min(1.0, ts * 1.05 + 1e-3), 1.0)) if ts < 0.95 else 1.0
        r = orc.solve(kind, X, 1e-6, 1_000_000, t_max=t_max)
        assert r.hit == 1 and Fraction(r.toi) <= t_star + Fraction(1, 10 ** 50)
        assert r.toi <= t_max
        above += 1
        # t_max below t*: nothing to find in [0, t_max]
        if ts > 0.05:
            t_max = float(rng.uniform(0.01, ts * 0.9))
            r = orc.solve(kind, X, 1e-6, 1_000_000, t_max=t_max)
            if r.hit == 0:
                assert exact.exclusion_proof(kind, X, t_max=Fraction(t_max),
                                             max_boxes=100_000) is True
            else:
                assert r.toi <= t_max
            below += 1
    assert above >= 15 and below >= 10


@pytest.mark.parametrize("t_max", [1.0, 0.75, 0.3, 2.0 ** -20, 1e-3])
def test_static_touching_query_closed_form(orc, t_max):
    """A static query touching at every t: F does not depend on t, kappa_t = 0,
    the time axis is never split, so every t_max gives the t_max = 1 result
    with toi = 0 and w(I_t) = t_max."""
    X = q([[.25, .25, 0]] + TRI, [[.25, .25, 0]] + TRI)
    ref = orc.solve(VF, X, 1e-6, 1_000_000)
    r = orc.solve(VF, X, 1e-6, 1_000_000, t_max=t_max)
    assert r.toi == 0.0 and r.hit == 1
    assert r.t_width == t_max
    assert (r.n_checks, r.status) == (ref.n_checks, ref.status)


@pytest.mark.parametrize("t_max", [0.0, -0.5, 1.0000000000000002, float("nan"), float("inf")])
def test_invalid_tmax_rejected(orc, t_max):
    X = q([[.25, .25, 1]] + TRI, [[.25, .25, -1]] + TRI)
    with pytest.raises(ValueError):
        orc.solve(VF, X, 1e-6, 1_000_000, t_max=t_max)
