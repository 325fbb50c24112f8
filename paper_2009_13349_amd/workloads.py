"""Seeded synthetic CCD workloads.

The paper's handcrafted and simulation query sets are not available, so every
workload here is generated from a seed with numpy's PCG64.  The generators only
place points; they contain none of the root finder's arithmetic.  A workload is
a dict with

* ``pos``   float64[24, n]: structure-of-arrays positions, row 3k+c is coordinate
  c of point k; points 0..3 are at t0, points 4..7 are the same vertices at t1
  (vertex-face: p, v1, v2, v3; edge-edge: p1, p2, p3, p4);
* ``kind``  uint8[n]: 0 vertex-face, 1 edge-edge;
* ``delta``, ``max_iter``, ``min_sep``: scalar parameters;
* ``cls``   uint8[n]: generator class of each query (see CLASS_NAMES).

Shapes follow the paper's two datasets (Sec. 4.1): a handcrafted-like set rich
in degenerate configurations (parallel, coplanar, touching at t=0 or t=1,
static, vertex-on-edge) and a simulation-like set of broad-phase candidates
moving ~1e-3 per step on an object of size 1 with ~1e-2 elements, including
near-contacts and exact grazing contacts.
"""
from __future__ import annotations

import math

import numpy as np

VF, EE = 0, 1

CLASS_NAMES = {
    0: "generic",
    1: "constructed_crossing",
    2: "parallel",
    3: "coplanar",
    4: "touch_t0",
    5: "touch_t1",
    6: "static",
    7: "endpoint_on_edge",
    8: "near_contact",
    9: "grazing",
    10: "min_sep_band",
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _pack(P0: np.ndarray, P1: np.ndarray) -> np.ndarray:
    """P0, P1: [n, 4, 3] positions at t0 and t1 -> pos[24, n]."""
    n = P0.shape[0]
    allp = np.concatenate([P0, P1], axis=1)  # [n, 8, 3]
    return np.ascontiguousarray(allp.reshape(n, 24).T.astype(np.float64))


def unpack(pos: np.ndarray, q: int) -> np.ndarray:
    """Query q of a workload as 24 doubles (X[3k+c])."""
    return np.ascontiguousarray(pos[:, q])


def _lerp(a, b, t):
    t = np.asarray(t)[..., None]
    return (1.0 - t) * a + t * b


def _rand_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _rand_rot(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _dirichlet_min(rng, n, lo=0.05):
    out = np.empty((n, 3))
    filled = 0
    while filled < n:
        b = rng.dirichlet((1.0, 1.0, 1.0), size=2 * (n - filled) + 8)
        b = b[b.min(axis=1) >= lo]
        take = min(len(b), n - filled)
        out[filled:filled + take] = b[:take]
        filled += take
    return out


# ---------------------------------------------------------------------------
# Uniform workloads (small: the oracle finishes them in seconds)

def uniform_vf(n: int = 4096, seed: int = 0) -> dict:
    """n vertex-face queries: all points uniform in [0,1)^3 at t0, displacement
    uniform in [-0.5,0.5)^3; odd indices are built to cross the triangle at
    t* ~ U(0.001, 0.999) at barycentric weights ~ Dirichlet(1,1,1) (min 0.05)."""
    rng = _rng(seed)
    P0 = rng.uniform(0.0, 1.0, size=(n, 4, 3))
    D = rng.uniform(-0.5, 0.5, size=(n, 4, 3))
    P1 = P0 + D
    cls = np.zeros(n, np.uint8)
    odd = np.arange(1, n, 2)
    m = len(odd)
    ts = rng.uniform(0.001, 0.999, size=m)
    beta = _dirichlet_min(rng, m)
    tri_t = _lerp(P0[odd, 1:4], P1[odd, 1:4], ts[:, None])  # [m, 3, 3]
    target = np.einsum("mj,mjc->mc", beta, tri_t)
    dp = D[odd, 0]
    P0[odd, 0] = target - ts[:, None] * dp
    P1[odd, 0] = P0[odd, 0] + dp
    cls[odd] = 1
    return {"name": f"uniform_vf_{n}", "pos": _pack(P0, P1), "kind": np.zeros(n, np.uint8),
            "cls": cls, "delta": 1e-6, "max_iter": 1_000_000, "min_sep": 0.0, "seed": seed}


def _grid(rng, shape, bits=10, lo=0.0, hi=1.0):
    """Dyadic grid values k * 2^-bits in [lo, hi)."""
    k = rng.integers(int(lo * 2 ** bits), int(hi * 2 ** bits), size=shape)
    return k.astype(np.float64) / 2 ** bits


def _dyadic_t(rng, shape, bits=4, lo=1, hi=None):
    hi = 2 ** bits if hi is None else hi
    return rng.integers(lo, hi, size=shape).astype(np.float64) / 2 ** bits


def edge_edge_mixed(n: int = 100_000, seed: int = 1, degenerate_frac: float = 0.1) -> dict:
    """n edge-edge queries: (1 - degenerate_frac) generic (uniform like
    uniform_vf, half constructed to cross at t*, u*, v* ~ U(0.05, 0.95) by
    translating edge B), and degenerate_frac split evenly over five classes on
    a dyadic grid: parallel (half collinear-overlapping), coplanar (half
    crossing), touching exactly at t=0 or t=1, static (half intersecting) and
    endpoint-on-edge contact at a dyadic t*."""
    rng = _rng(seed)
    n_deg = int(round(n * degenerate_frac))
    n_gen = n - n_deg
    P0 = np.empty((n, 4, 3))
    P1 = np.empty((n, 4, 3))
    cls = np.zeros(n, np.uint8)

    # generic
    G0 = rng.uniform(0.0, 1.0, size=(n_gen, 4, 3))
    GD = rng.uniform(-0.5, 0.5, size=(n_gen, 4, 3))
    G1 = G0 + GD
    cr = np.arange(1, n_gen, 2)
    m = len(cr)
    ts = rng.uniform(0.05, 0.95, size=m)
    us = rng.uniform(0.05, 0.95, size=m)
    vs = rng.uniform(0.05, 0.95, size=m)
    A = _lerp(_lerp(G0[cr, 0], G1[cr, 0], ts), _lerp(G0[cr, 1], G1[cr, 1], ts), us)
    B = _lerp(_lerp(G0[cr, 2], G1[cr, 2], ts), _lerp(G0[cr, 3], G1[cr, 3], ts), vs)
    shift = A - B
    G0[cr, 2:4] += shift[:, None, :]
    G1[cr, 2:4] += shift[:, None, :]
    P0[:n_gen], P1[:n_gen] = G0, G1
    cls[cr] = 1

    # degenerate classes on a dyadic grid (all constructions exact in binary64)
    per = n_deg // 5
    counts = [per] * 5
    counts[-1] += n_deg - 5 * per
    base = n_gen
    builders = [_ee_parallel, _ee_coplanar, _ee_touch_end, _ee_static, _ee_endpoint_on_edge]
    for b, cnt in zip(builders, counts):
        if cnt == 0:
            continue
        Q0, Q1, c = b(rng, cnt)
        P0[base:base + cnt], P1[base:base + cnt], cls[base:base + cnt] = Q0, Q1, c
        base += cnt
    return {"name": f"edge_edge_mixed_{n}", "pos": _pack(P0, P1), "kind": np.ones(n, np.uint8),
            "cls": cls, "delta": 1e-6, "max_iter": 1_000_000, "min_sep": 0.0, "seed": seed}


def _grid_dir(rng, n, bits=6):
    """Nonzero dyadic direction vectors with components in [-1, 1)."""
    d = _grid(rng, (n, 3), bits, -1.0, 1.0)
    bad = np.all(d == 0, axis=1)
    d[bad, 0] = 0.5
    return d


def _ee_parallel(rng, n):
    a = _grid(rng, (n, 3), 10, 0.0, 1.0)
    d = _grid_dir(rng, n) * 0.25
    P0 = np.empty((n, 4, 3))
    P1 = np.empty((n, 4, 3))
    mv = _grid(rng, (n, 3), 10, -0.25, 0.25)
    half = n // 2
    # collinear, overlapping, moving together: contact for every t
    al = _dyadic_t(rng, half, 4, 1, 12)
    P0[:half, 0] = a[:half]
    P0[:half, 1] = a[:half] + d[:half]
    P0[:half, 2] = a[:half] + al[:, None] * d[:half]
    P0[:half, 3] = P0[:half, 2] + d[:half]
    P1[:half] = P0[:half] + mv[:half, None, :]
    # parallel with an offset; B moves toward A's line and reaches it at
    # t* in {1/8, 1/4, 1/2, 1} (or would at t* = 2, i.e. never within [0, 1])
    r = n - half
    off = _grid_dir(rng, r) * 0.125
    ts = np.array([0.125, 0.25, 0.5, 1.0, 2.0])[rng.integers(0, 5, size=r)]
    al = _dyadic_t(rng, r, 4, 1, 12)
    A0 = a[half:]
    P0[half:, 0] = A0
    P0[half:, 1] = A0 + d[half:]
    P0[half:, 2] = A0 + al[:, None] * d[half:] + off
    P0[half:, 3] = P0[half:, 2] + d[half:]
    P1[half:, 0:2] = P0[half:, 0:2]
    step = off / ts[:, None]  # exact: ts is a power of two
    P1[half:, 2] = P0[half:, 2] - step
    P1[half:, 3] = P0[half:, 3] - step
    return P0, P1, np.full(n, 2, np.uint8)


def _ee_coplanar(rng, n):
    z = _grid(rng, (n,), 10, 0.0, 1.0)
    P0 = _grid(rng, (n, 4, 3), 10, 0.0, 1.0)
    P1 = P0 + _grid(rng, (n, 4, 3), 10, -0.25, 0.25)
    P0[:, :, 2] = z[:, None]
    P1[:, :, 2] = z[:, None]
    half = n // 2
    # crossing half: shift B so that A(t*, u*) = B(t*, v*) with dyadic t*, u*, v*
    ts = _dyadic_t(rng, half, 4, 1, 16)
    us = _dyadic_t(rng, half, 4, 1, 16)
    vs = _dyadic_t(rng, half, 4, 1, 16)
    A = _lerp(_lerp(P0[:half, 0], P1[:half, 0], ts), _lerp(P0[:half, 1], P1[:half, 1], ts), us)
    B = _lerp(_lerp(P0[:half, 2], P1[:half, 2], ts), _lerp(P0[:half, 3], P1[:half, 3], ts), vs)
    sh = A - B
    P0[:half, 2:4] += sh[:, None, :]
    P1[:half, 2:4] += sh[:, None, :]
    return P0, P1, np.full(n, 3, np.uint8)


def _ee_touch_end(rng, n):
    P0 = _grid(rng, (n, 4, 3), 10, 0.0, 1.0)
    P1 = P0 + _grid(rng, (n, 4, 3), 10, -0.25, 0.25)
    half = n // 2
    ts = np.where(np.arange(n) < half, 0.0, 1.0)
    us = _dyadic_t(rng, n, 4, 1, 16)
    vs = _dyadic_t(rng, n, 4, 1, 16)
    A = _lerp(_lerp(P0[:, 0], P1[:, 0], ts), _lerp(P0[:, 1], P1[:, 1], ts), us)
    B = _lerp(_lerp(P0[:, 2], P1[:, 2], ts), _lerp(P0[:, 3], P1[:, 3], ts), vs)
    sh = A - B
    P0[:, 2:4] += sh[:, None, :]
    P1[:, 2:4] += sh[:, None, :]
    cls = np.where(np.arange(n) < half, 4, 5).astype(np.uint8)
    return P0, P1, cls


def _ee_static(rng, n):
    P0 = _grid(rng, (n, 4, 3), 10, 0.0, 1.0)
    half = n // 2
    us = _dyadic_t(rng, half, 4, 1, 16)
    vs = _dyadic_t(rng, half, 4, 1, 16)
    A = _lerp(P0[:half, 0], P0[:half, 1], us)
    B = _lerp(P0[:half, 2], P0[:half, 3], vs)
    P0[:half, 2:4] += (A - B)[:, None, :]
    P1 = P0.copy()
    return P0, P1, np.full(n, 6, np.uint8)


def _ee_endpoint_on_edge(rng, n):
    P0 = _grid(rng, (n, 4, 3), 10, 0.0, 1.0)
    P1 = P0 + _grid(rng, (n, 4, 3), 10, -0.25, 0.25)
    ts = _dyadic_t(rng, n, 4, 1, 16)
    us = _dyadic_t(rng, n, 4, 1, 16)
    A = _lerp(_lerp(P0[:, 0], P1[:, 0], ts), _lerp(P0[:, 1], P1[:, 1], ts), us)
    B = _lerp(P0[:, 2], P1[:, 2], ts)  # endpoint p3 (v = 0)
    sh = A - B
    P0[:, 2:4] += sh[:, None, :]
    P1[:, 2:4] += sh[:, None, :]
    return P0, P1, np.full(n, 7, np.uint8)


# ---------------------------------------------------------------------------
# Simulation-shaped workload

def _displacements(rng, n, mean=1e-3, sigma=3e-4):
    mag = np.maximum(rng.normal(mean, sigma, size=n), 0.0)
    d = _rand_unit(rng, n) * mag[:, None]
    return d, mag


def simulation_mixed(n: int = 1_000_000, seed: int = 2, vf_frac: float = 0.6,
                     near_frac: float = 0.02, graze_frac: float = 0.01,
                     band_frac: float = 0.0, band_dmin: float = 0.0, h: float = 1e-2) -> dict:
    """Broad-phase-like candidate pairs on an object of size 1 with element
    size h: equilateral triangles / edges of length h with random orientation,
    partners at separation s ~ U[0, 2h], per-primitive displacement of
    magnitude ~ N(1e-3, 3e-4) (truncated at 0) in a random direction plus a 10%
    per-vertex jitter.  near_frac of the pairs move parallel to each other at
    a normal distance ~ logU[1e-12, 1e-8] (no true contact), graze_frac touch
    at exactly one instant on a dyadic grid (a point sliding in the triangle
    plane through a vertex; two coplanar edges meeting at an endpoint), and
    band_frac come within ~U(0, 2*band_dmin) of each other (min-separation
    workloads)."""
    rng = _rng(seed)
    n_vf = int(round(n * vf_frac))
    kind = np.zeros(n, np.uint8)
    kind[n_vf:] = 1
    P0 = np.empty((n, 4, 3))
    P1 = np.empty((n, 4, 3))
    cls = np.zeros(n, np.uint8)

    cat = rng.uniform(size=n)
    near = cat < near_frac
    graze = (cat >= near_frac) & (cat < near_frac + graze_frac)
    band = (cat >= near_frac + graze_frac) & (cat < near_frac + graze_frac + band_frac)
    generic = ~(near | graze | band)

    vf = kind == VF
    ee = ~vf
    for sel_kind, builder in ((vf, _sim_vf), (ee, _sim_ee)):
        idx = np.nonzero(sel_kind & generic)[0]
        if len(idx):
            Q0, Q1 = builder(rng, len(idx), h)
            P0[idx], P1[idx] = Q0, Q1
            cls[idx] = 0
    for sel_kind, builder in ((vf, _near_vf), (ee, _near_ee)):
        idx = np.nonzero(sel_kind & near)[0]
        if len(idx):
            gap = np.exp(rng.uniform(math.log(1e-12), math.log(1e-8), size=len(idx)))
            Q0, Q1 = builder(rng, len(idx), h, gap)
            P0[idx], P1[idx] = Q0, Q1
            cls[idx] = 8
        idx = np.nonzero(sel_kind & band)[0]
        if len(idx):
            gap = rng.uniform(0.0, 2.0 * band_dmin, size=len(idx))
            Q0, Q1 = builder(rng, len(idx), h, gap)
            P0[idx], P1[idx] = Q0, Q1
            cls[idx] = 10
    for sel_kind, builder in ((vf, _graze_vf), (ee, _graze_ee)):
        idx = np.nonzero(sel_kind & graze)[0]
        if len(idx):
            Q0, Q1 = builder(rng, len(idx))
            P0[idx], P1[idx] = Q0, Q1
            cls[idx] = 9
    return {"name": f"simulation_mixed_{n}", "pos": _pack(P0, P1), "kind": kind, "cls": cls,
            "delta": 1e-6, "max_iter": 1_000_000, "min_sep": 0.0, "seed": seed}


def _triangle(rng, n, h):
    R = _rand_rot(rng, n)
    r = h / math.sqrt(3.0)  # circumradius of an equilateral triangle of edge h
    ang = np.array([0.0, 2 * math.pi / 3, 4 * math.pi / 3])
    local = np.stack([r * np.cos(ang), r * np.sin(ang), np.zeros(3)], axis=1)  # [3, 3]
    c = rng.uniform(0.0, 1.0, size=(n, 3))
    tri = c[:, None, :] + np.einsum("nij,kj->nki", R, local)
    normal = R[:, :, 2]
    inplane = (R[:, :, 0], R[:, :, 1])
    return tri, normal, inplane, c, r


def _move(rng, n, npts):
    d, mag = _displacements(rng, n)
    jitter = _rand_unit(rng, n * npts).reshape(n, npts, 3) * (0.1 * mag)[:, None, None]
    return d[:, None, :] + jitter


def _sim_vf(rng, n, h):
    tri, normal, (ex, ey), c, r = _triangle(rng, n, h)
    s = rng.uniform(0.0, 2 * h, size=n) * rng.choice([-1.0, 1.0], size=n)
    rad = 1.5 * r * np.sqrt(rng.uniform(size=n))
    th = rng.uniform(0, 2 * math.pi, size=n)
    p = c + s[:, None] * normal + (rad * np.cos(th))[:, None] * ex + (rad * np.sin(th))[:, None] * ey
    P0 = np.concatenate([p[:, None, :], tri], axis=1)
    mv_p = _move(rng, n, 1)
    mv_t = _move(rng, n, 3)
    P1 = P0 + np.concatenate([mv_p, mv_t], axis=1)
    return P0, P1


def _sim_ee(rng, n, h):
    ca = rng.uniform(0.0, 1.0, size=(n, 3))
    da = _rand_unit(rng, n) * (h / 2)
    s = rng.uniform(0.0, 2 * h, size=n)
    cb = ca + _rand_unit(rng, n) * s[:, None]
    db = _rand_unit(rng, n) * (h / 2)
    P0 = np.stack([ca - da, ca + da, cb - db, cb + db], axis=1)
    mv_a = _move(rng, n, 2)
    mv_b = _move(rng, n, 2)
    P1 = P0 + np.concatenate([mv_a, mv_b], axis=1)
    return P0, P1


def _near_vf(rng, n, h, gap):
    """Point gliding parallel to the triangle's plane at normal distance gap,
    over the triangle's interior."""
    tri, normal, (ex, ey), c, r = _triangle(rng, n, h)
    side = rng.choice([-1.0, 1.0], size=n)
    d, _ = _displacements(rng, n)
    d_in = d - np.sum(d * normal, axis=1, keepdims=True) * normal  # in-plane motion
    beta = _dirichlet_min(rng, n, 0.1)
    mid = np.einsum("nj,njc->nc", beta, tri)  # interior point crossed at t=1/2
    p_mid = mid + (side * gap)[:, None] * normal
    p0 = p_mid - 0.5 * d_in
    p1 = p_mid + 0.5 * d_in
    P0 = np.concatenate([p0[:, None, :], tri], axis=1)
    P1 = np.concatenate([p1[:, None, :], tri], axis=1)
    return P0, P1


def _near_ee(rng, n, h, gap):
    """Two edges in parallel planes a distance gap apart, sliding across each
    other: no contact, minimum distance gap."""
    ca = rng.uniform(0.0, 1.0, size=(n, 3))
    R = _rand_rot(rng, n)
    ex, ey, nz = R[:, :, 0], R[:, :, 1], R[:, :, 2]
    A0 = ca - ex * (h / 2)
    A1 = ca + ex * (h / 2)
    side = rng.choice([-1.0, 1.0], size=n)
    u = rng.uniform(0.2, 0.8, size=n)
    cross = _lerp(A0, A1, u)
    b_mid = cross + (side * gap)[:, None] * nz
    d, _ = _displacements(rng, n)
    d_in = d - np.sum(d * nz, axis=1, keepdims=True) * nz
    Bm0 = b_mid - 0.5 * d_in
    Bm1 = b_mid + 0.5 * d_in
    B_a0 = Bm0 - ey * (h / 2)
    B_b0 = Bm0 + ey * (h / 2)
    P0 = np.stack([A0, A1, B_a0, B_b0], axis=1)
    P1 = np.stack([A0, A1, Bm1 - ey * (h / 2), Bm1 + ey * (h / 2)], axis=1)
    return P0, P1


def _signed_perm(rng, n):
    """Random axis permutations with sign flips (exact on dyadic data)."""
    perms = np.array([[0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]])
    p = perms[rng.integers(0, 6, size=n)]
    s = rng.choice([-1.0, 1.0], size=(n, 3))
    return p, s


def _apply_perm(P, p, s, origin):
    out = np.empty_like(P)
    for i in range(P.shape[0]):
        out[i] = P[i][..., p[i]] * s[i] + origin[i]
    return out


def _graze_vf(rng, n):
    """A point sliding in the triangle's plane that touches only the vertex v1
    at a dyadic instant t*: v1 = 0, v2 = a e_x, v3 = b e_y, p(t) = v1 + (t - t*)
    (c, -c, 0); then a signed axis permutation and a dyadic translation."""
    a = _grid(rng, (n,), 10, 2 ** -7, 2 ** -5)
    b = _grid(rng, (n,), 10, 2 ** -7, 2 ** -5)
    cc = _grid(rng, (n,), 12, 2 ** -10, 2 ** -8)
    ts = _dyadic_t(rng, n, 4, 1, 16)
    P0 = np.zeros((n, 4, 3))
    P0[:, 2, 0] = a
    P0[:, 3, 1] = b
    P0[:, 0, 0] = -ts * cc
    P0[:, 0, 1] = ts * cc
    P1 = P0.copy()
    P1[:, 0, 0] = (1 - ts) * cc
    P1[:, 0, 1] = -(1 - ts) * cc
    p, s = _signed_perm(rng, n)
    origin = _grid(rng, (n, 3), 10, 0.0, 1.0)
    return _apply_perm(P0, p, s, origin), _apply_perm(P1, p, s, origin)


def _graze_ee(rng, n):
    """Coplanar edges A = [0, a e_x] (static) and B = [q(t), q(t) + b e_y] with
    q(t) = (t* - t) (c, c, 0): they touch only at t = t*, where B's endpoint
    meets A's endpoint."""
    a = _grid(rng, (n,), 10, 2 ** -7, 2 ** -5)
    b = _grid(rng, (n,), 10, 2 ** -7, 2 ** -5)
    cc = _grid(rng, (n,), 12, 2 ** -10, 2 ** -8)
    ts = _dyadic_t(rng, n, 4, 1, 16)
    P0 = np.zeros((n, 4, 3))
    P0[:, 1, 0] = a
    P0[:, 2, 0] = ts * cc
    P0[:, 2, 1] = ts * cc
    P0[:, 3] = P0[:, 2]
    P0[:, 3, 1] += b
    P1 = P0.copy()
    P1[:, 2, 0] = (ts - 1) * cc
    P1[:, 2, 1] = (ts - 1) * cc
    P1[:, 3] = P1[:, 2]
    P1[:, 3, 1] += b
    p, s = _signed_perm(rng, n)
    origin = _grid(rng, (n, 3), 10, 0.0, 1.0)
    return _apply_perm(P0, p, s, origin), _apply_perm(P1, p, s, origin)


def min_separation(n: int = 1_000_000, seed: int = 2, d_min: float = 1e-4,
                   delta: float = 1e-6) -> dict:
    """The simulation-shaped generator with 5% of pairs placed at a distance
    ~ U(0, 2 d_min) along their trajectory; minimum separation d_min."""
    w = simulation_mixed(n, seed, band_frac=0.05, band_dmin=d_min)
    w.update(name=f"min_separation_{n}_d{d_min:g}_delta{delta:g}", min_sep=float(d_min),
             delta=float(delta))
    return w


def serving_requests(count: int = 2000, seed: int = 4, n_lo: int = 1000,
                     n_hi: int = 1_000_000) -> list:
    """Request descriptors of the serving workload: sizes log-uniform in
    [n_lo, n_hi], delta log-uniform in [1e-6, 1e-4], per-request seed 1000 + i.
    Queries are generated lazily with `request_queries`."""
    rng = _rng(seed)
    sizes = np.round(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(int)
    deltas = np.exp(rng.uniform(math.log(1e-6), math.log(1e-4), size=count))
    return [{"id": i, "n": int(sizes[i]), "delta": float(deltas[i]), "seed": 1000 + i,
             "max_iter": 1_000_000, "min_sep": 0.0} for i in range(count)]


def request_queries(req: dict) -> dict:
    w = simulation_mixed(req["n"], req["seed"])
    w.update(delta=req["delta"], max_iter=req["max_iter"], min_sep=req["min_sep"])
    return w


def subset(w: dict, idx) -> dict:
    idx = np.asarray(idx)
    out = dict(w)
    out["pos"] = np.ascontiguousarray(w["pos"][:, idx])
    out["kind"] = np.ascontiguousarray(w["kind"][idx])
    out["cls"] = np.ascontiguousarray(w["cls"][idx])
    return out


def concat(ws) -> dict:
    out = dict(ws[0])
    out["pos"] = np.ascontiguousarray(np.concatenate([w["pos"] for w in ws], axis=1))
    out["kind"] = np.concatenate([w["kind"] for w in ws])
    out["cls"] = np.concatenate([w["cls"] for w in ws])
    return out


# ---------------------------------------------------------------------------
# Candidate pairs over shared vertex arrays (the mesh form the active-set and
# line-search drivers of Sec. 7 work on).

def as_indexed(w: dict) -> dict:
    """The queries of a structure-of-arrays workload as vertex arrays and ids:
    query q's 4 points become vertices 4q..4q+3 (no sharing), so an indexed
    batch must reproduce the workload's results exactly."""
    n = w["pos"].shape[1]
    P = w["pos"].T.reshape(n, 8, 3)
    v0 = np.ascontiguousarray(P[:, :4, :].reshape(4 * n, 3))
    v1 = np.ascontiguousarray(P[:, 4:, :].reshape(4 * n, 3))
    ids = np.arange(4 * n, dtype=np.int32).reshape(n, 4)
    return {"v0": v0, "v1": v1, "ids": ids, "kind": w["kind"].copy(), "name": w.get("name", "") + "_indexed",
            "delta": w.get("delta", 1e-6), "max_iter": w.get("max_iter", 1_000_000),
            "min_sep": w.get("min_sep", 0.0)}


def gather(scene: dict) -> np.ndarray:
    """Structure-of-arrays positions pos[24, n] of an indexed scene."""
    ids = scene["ids"]
    P = np.concatenate([scene["v0"][ids], scene["v1"][ids]], axis=1)  # [n, 8, 3]
    return np.ascontiguousarray(P.reshape(ids.shape[0], 24).T)


def mesh_scene(n_pairs: int = 100_000, seed: int = 5, h: float = 2e-3, vf_frac: float = 0.6) -> dict:
    """Two triangulated g x g sheets on [0,1]^2: sheet A static at z = 0, sheet B
    (offset by half a cell) moving from z = +h to z = -h through A, with small
    in-plane jitter.  Candidate pairs as a broad phase would give them: VF =
    (vertex of B, triangle of A under it), EE = (edge of B, edge of A in the
    same cell).  Vertices are shared by many pairs."""
    rng = _rng(seed)
    g = max(4, int(math.ceil(math.sqrt(n_pairs / 4.0))) + 2)
    cell = 1.0 / (g - 1)
    ii, jj = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
    base = np.stack([ii.ravel() * cell, jj.ravel() * cell], axis=1)
    A0 = np.concatenate([base + rng.uniform(-0.1, 0.1, base.shape) * cell, np.zeros((g * g, 1))], axis=1)
    A1 = A0.copy()
    B0 = np.concatenate([base + 0.5 * cell + rng.uniform(-0.1, 0.1, base.shape) * cell,
                         np.full((g * g, 1), h)], axis=1)
    B1 = B0 + np.concatenate([rng.normal(0, 0.02, (g * g, 2)) * cell,
                              -2 * h * np.ones((g * g, 1)) + rng.normal(0, 0.1 * h, (g * g, 1))], axis=1)
    v0 = np.ascontiguousarray(np.concatenate([A0, B0]))
    v1 = np.ascontiguousarray(np.concatenate([A1, B1]))
    nA = g * g
    idx = lambda i, j: i * g + j  # noqa: E731
    n_vf = int(round(n_pairs * vf_frac))
    n_ee = n_pairs - n_vf
    # VF: vertex (i, j) of B lies over cell (i, j) of A, whose two triangles are tried
    ci = rng.integers(0, g - 1, n_vf)
    cj = rng.integers(0, g - 1, n_vf)
    upper = rng.integers(0, 2, n_vf).astype(bool)
    a00, a10, a01, a11 = idx(ci, cj), idx(ci + 1, cj), idx(ci, cj + 1), idx(ci + 1, cj + 1)
    tri = np.where(upper[:, None], np.stack([a10, a11, a01], 1), np.stack([a00, a10, a01], 1))
    vf = np.concatenate([(nA + idx(ci, cj))[:, None], tri], axis=1)
    # EE: an edge of B's cell against an edge of A's cell
    ci = rng.integers(0, g - 1, n_ee)
    cj = rng.integers(0, g - 1, n_ee)

    def cell_edge(off, i, j, which):
        e0 = np.where(which == 0, idx(i, j), np.where(which == 1, idx(i, j), idx(i + 1, j)))
        e1 = np.where(which == 0, idx(i + 1, j), np.where(which == 1, idx(i, j + 1), idx(i, j + 1)))
        return off + e0, off + e1

    ea0, ea1 = cell_edge(0, ci, cj, rng.integers(0, 3, n_ee))
    eb0, eb1 = cell_edge(nA, ci, cj, rng.integers(0, 3, n_ee))
    ee = np.stack([eb0, eb1, ea0, ea1], axis=1)
    ids = np.ascontiguousarray(np.concatenate([vf, ee]).astype(np.int32))
    kind = np.concatenate([np.full(n_vf, VF, np.uint8), np.full(n_ee, EE, np.uint8)])
    return {"v0": v0, "v1": v1, "ids": ids, "kind": kind, "name": f"mesh_scene_{n_pairs}",
            "delta": 1e-6, "max_iter": 1_000_000, "min_sep": 0.0}
