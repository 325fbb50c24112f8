"""Pins of the oracle's scene-wide filter (Sec. 7: the tolerances eq.
ccd-error / msccd-error computed from the maximum over all the vertices of the
scene).  Reading: a gamma per axis replaces the query's own, and must be at
least the query's own for the filter's bound to cover the query.  CPU-only."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact

VF, EE = 0, 1


def own_gamma(X):
    """gamma_c = max(1, max over the 8 points of |x^c|), from the coordinates."""
    return np.maximum(1.0, np.abs(np.asarray(X, dtype=float).reshape(8, 3)).max(axis=0))


def test_own_gamma_is_the_per_query_filter(orc):
    from paper_2009_13349_amd import workloads as W
    w = W.concat([W.uniform_vf(200, seed=71), W.edge_edge_mixed(200, seed=72)])
    for i in range(w["pos"].shape[1]):
        X = w["pos"][:, i]
        k = int(w["kind"][i])
        a = orc.solve(k, X, 1e-6, 100_000)
        b = orc.solve(k, X, 1e-6, 100_000, gamma=own_gamma(X))
        assert (a.toi, a.t_width, a.n_checks, a.hit, a.status) == \
            (b.toi, b.t_width, b.n_checks, b.hit, b.status)


@pytest.mark.parametrize("kind,min_sep", [(VF, 0.0), (EE, 0.0), (VF, 1e-3), (EE, 1e-3)])
def test_filter_scales_with_gamma_cubed(orc, kind, min_sep):
    g = np.array([1.0, 3.0, 10.0])
    e1 = orc.filter_eps_gamma(kind, g, min_sep)
    e2 = orc.filter_eps_gamma(kind, 2 * g, min_sep)
    assert np.array_equal(e2, 8 * e1)  # powers of two: exact
    # and the per-axis constant is the paper's K * gamma^3 at gamma = 1
    e0 = orc.filter_eps_gamma(kind, np.ones(3), min_sep)
    assert np.array_equal(e0, orc.filter_eps(kind, np.zeros(24), min_sep))


@pytest.mark.parametrize("which", ["uniform_vf", "edge_edge_generic"])
def test_scene_gamma_keeps_first_contact(orc, which):
    """A scene gamma 4x the query's own (a wider filter) stays conservative:
    every exact contact is a hit no later than t*, every miss is provable."""
    from paper_2009_13349_amd import workloads as W
    if which == "uniform_vf":
        w, kind = W.uniform_vf(40, seed=15), VF
    else:
        w, kind = W.edge_edge_mixed(40, seed=16, degenerate_frac=0.0), EE
    contacts = 0
    for i in range(w["pos"].shape[1]):
        X = w["pos"][:, i]
        r = orc.solve(kind, X, 1e-6, 1_000_000, gamma=4 * own_gamma(X))
        status, t_first = exact.first_contact_univariate(kind, X)
        if status == "contact":
            contacts += 1
            assert r.hit == 1
            assert Fraction(r.toi) <= Fraction(str(t_first.evalf(60))) + Fraction(1, 10 ** 50)
        if r.hit == 0:
            assert exact.exclusion_proof(kind, X, max_boxes=100_000) is True
    assert contacts >= 15


def test_scene_gamma_validation(orc):
    X = np.array([.25, .25, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0,
                  .25, .25, -1, 0, 0, 0, 1, 0, 0, 0, 1, 0], dtype=float) * 3.0
    g = own_gamma(X)
    orc.solve(VF, X, 1e-6, 1000, gamma=g)              # equal: valid
    orc.solve(VF, X, 1e-6, 1000, gamma=g * 1.5)        # larger: valid
    for bad in (g * np.array([1, 1, 0.5]), np.array([np.nan, 1, 1]), np.array([np.inf] * 3)):
        with pytest.raises(ValueError):
            orc.solve(VF, X, 1e-6, 1000, gamma=bad)
    with pytest.raises(ValueError):                    # d < min_c gamma_c
        orc.solve(VF, X, 1e-6, 1000, min_sep=float(g.min()), gamma=g)
