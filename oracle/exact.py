"""Exact-rational checks for the CCD problem (test infrastructure).

Nothing here uses floating-point arithmetic on the method's quantities: inputs
(binary64 numbers) are converted exactly to `fractions.Fraction`, and every
predicate is decided exactly.  Two independent routes are provided:

* the multivariate definition (Sec. 3, eqs. F-vf / F-ee): a root of F in the
  domain Omega means contact.  `exclusion_proof` bisects the parameter box and
  uses the exact corner hull of F (F is affine in each of t, u, v separately, so
  on a box each coordinate of F attains its extremes at the 8 corners, Sec. 5.2
  Prop. 1) to certify that no root exists;
* the univariate coplanarity formulation (Sec. 3, eq. univariate): contact can
  only happen at a root of the cubic f(t) = <n(t), q(t)>, followed by an
  inside test.  `first_contact_univariate` finds the earliest contact this way
  with sympy's exact real-root isolation.  It is independent of F's code and
  is used to pin the oracle on non-degenerate inputs.
"""
from __future__ import annotations

from fractions import Fraction

import sympy

VF, EE = 0, 1


def frac_query(X):
    """24 doubles -> 8 points x 3 exact Fractions (points 0..3 at t0, 4..7 at t1)."""
    flat = [Fraction(float(x)) for x in list(_flatten(X))]
    assert len(flat) == 24
    return [flat[3 * k:3 * k + 3] for k in range(8)]


def _flatten(X):
    try:
        import numpy as np
        return np.asarray(X, dtype=float).reshape(24).tolist()
    except Exception:  # pragma: no cover
        return X


def _pos(P, k, t):
    """p_k(t) = (1-t) p_k^0 + t p_k^1 (Sec. 3), exactly."""
    return [(1 - t) * P[k][c] + t * P[k + 4][c] for c in range(3)]


def F_exact(kind, P, t, u, v):
    """Exact F_vf / F_ee at (t, u, v) (Sec. 3 eqs. F-vf, F-ee)."""
    p0, p1, p2, p3 = (_pos(P, k, t) for k in range(4))
    if kind == EE:
        return [((1 - u) * p0[c] + u * p1[c]) - ((1 - v) * p2[c] + v * p3[c]) for c in range(3)]
    return [p0[c] - ((1 - u - v) * p1[c] + u * p2[c] + v * p3[c]) for c in range(3)]


def corner_hull(kind, P, box):
    """Exact per-axis [min, max] of F over the 8 corners of box=(t0,t1,u0,u1,v0,v1)."""
    vals = [F_exact(kind, P, t, u, v)
            for t in (box[0], box[1]) for u in (box[2], box[3]) for v in (box[4], box[5])]
    lo = [min(f[c] for f in vals) for c in range(3)]
    hi = [max(f[c] for f in vals) for c in range(3)]
    return lo, hi


def _excluded(lo, hi, d):
    # F(box) misses the cube [-d, d]^3 (L-infinity distance d, Sec. 6.1).
    return any(lo[c] > d or hi[c] < -d for c in range(3))


def exclusion_proof(kind, X, d=0.0, t_max=Fraction(1), max_boxes=200_000):
    """Try to prove that F has no root (|F|_inf <= d) in Omega with t <= t_max.

    Returns True if proved, False if a box that cannot be excluded shrank to a
    point-like size (a root is likely), None if the box budget ran out."""
    P = frac_query(X)
    d = Fraction(float(d))
    t_max = Fraction(t_max)
    stack = [((Fraction(0), t_max, Fraction(0), Fraction(1), Fraction(0), Fraction(1)), 0)]
    used = 0
    while stack:
        box, depth = stack.pop()
        used += 1
        if used > max_boxes:
            return None
        if kind == VF and box[2] + box[4] > 1:
            continue  # outside the prism u + v <= 1
        lo, hi = corner_hull(kind, P, box)
        if _excluded(lo, hi, d):
            continue
        if depth >= 60:
            return False
        axis = depth % 3
        a, b = box[2 * axis], box[2 * axis + 1]
        m = (a + b) / 2
        b0 = list(box)
        b1 = list(box)
        b0[2 * axis + 1] = m
        b1[2 * axis] = m
        stack.append((tuple(b1), depth + 1))
        stack.append((tuple(b0), depth + 1))
    return True


# ---------------------------------------------------------------------------
# Univariate route (Sec. 3, eq. univariate).

def _poly_coeffs(P, kind):
    t = sympy.Symbol("t")
    pts = [[sympy.Rational(x.numerator, x.denominator) * (1 - t)
            + sympy.Rational(y.numerator, y.denominator) * t
            for x, y in zip(P[k], P[k + 4])] for k in range(4)]
    M = sympy.Matrix
    if kind == VF:
        p, v1, v2, v3 = (M(q) for q in pts)
        n = (v2 - v1).cross(v3 - v1)
        q = p - v1
    else:
        p1, p2, p3, p4 = (M(q) for q in pts)
        n = (p2 - p1).cross(p4 - p3)
        q = p3 - p1
    f = sympy.expand(n.dot(q))
    return t, f, pts


def coplanarity_cubic(kind, X):
    """The cubic f(t) of eq. univariate as a sympy Poly in t (exact)."""
    P = frac_query(X)
    t, f, _ = _poly_coeffs(P, kind)
    return sympy.Poly(f, t)


def _inside_at(kind, P, root, prec=120):
    """Decide, at coplanar time `root`, whether the primitives touch.

    Positions are evaluated from the exact inputs at `root` with `prec` decimal
    digits.  Returns True/False, or None when the decision is too close to call
    (the touching point lies on a boundary to within 10^-(prec/2)) or the
    primitives are degenerate at that time."""
    import mpmath
    mpmath.mp.dps = prec
    tv = mpmath.mpf(str(sympy.N(root, prec + 10)))

    def mp(x):
        return mpmath.mpf(x.numerator) / x.denominator

    Q = [[(1 - tv) * mp(P[k][c]) + tv * mp(P[k + 4][c]) for c in range(3)] for k in range(4)]
    tol = mpmath.mpf(10) ** (-(prec // 2))

    def dot(a, b):
        return sum(a[i] * b[i] for i in range(3))

    if kind == VF:
        p, a, b, c = Q
        e1 = [b[i] - a[i] for i in range(3)]
        e2 = [c[i] - a[i] for i in range(3)]
        r = [p[i] - a[i] for i in range(3)]
        d11, d12, d22 = dot(e1, e1), dot(e1, e2), dot(e2, e2)
        r1, r2 = dot(r, e1), dot(r, e2)
        den = d11 * d22 - d12 * d12
        if abs(den) < tol:
            return None  # degenerate triangle
        u = (r1 * d22 - r2 * d12) / den
        v = (r2 * d11 - r1 * d12) / den
        vals = [u, v, 1 - u - v]
    else:
        p1, p2, p3, p4 = Q
        e1 = [p2[i] - p1[i] for i in range(3)]
        e2 = [p4[i] - p3[i] for i in range(3)]
        r = [p3[i] - p1[i] for i in range(3)]
        d11, d12, d22 = dot(e1, e1), dot(e1, e2), dot(e2, e2)
        r1, r2 = dot(r, e1), dot(r, e2)
        den = d11 * d22 - d12 * d12
        if abs(den) < tol:
            return None  # parallel edges
        # p1 + u e1 = p3 + v e2
        u = (r1 * d22 - r2 * d12) / den
        v = (r1 * d12 - r2 * d11) / den
        vals = [u, 1 - u, v, 1 - v]
    if any(abs(x) < tol for x in vals):
        return None
    return all(x > 0 for x in vals)


def first_contact_univariate(kind, X):
    """Earliest contact time in [0, 1] by the univariate route.

    Returns (status, t) with status in {"contact", "none", "degenerate"}; t is
    a sympy exact algebraic number for "contact"."""
    P = frac_query(X)
    t, f, pts = _poly_coeffs(P, kind)
    poly = sympy.Poly(f, t)
    if poly.is_zero:
        return "degenerate", None
    roots = [r for r in sympy.real_roots(poly) if 0 <= r <= 1]
    roots = sorted(set(roots), key=lambda r: sympy.N(r, 50))
    for r in roots:
        ins = _inside_at(kind, P, r)
        if ins is None:
            return "degenerate", r
        if ins:
            return "contact", r
    return "none", None
