"""Pins of the oracle's extruded geometry (Sec. VI, the evaluation environment:
the outer disk and the obstacle disks are extruded and further unbounded
dimensions are appended, the distance being taken in the first two
coordinates), on the CPU: distances against brute force over sampled surface
points of the extruded boundary in full d-space, empty-ball membership and
closest points, the extruded annulus whose exact solution is the
two-dimensional one in every d (Laplace and screened), affine data with
slopes along the free coordinates, and translation invariance along them."""
import math

import numpy as np
import pytest

from paper_2406_01713_amd import scenes as S


def _interior_points(s, n, seed, spread=5.0):
    """Points whose first two coordinates are clear of the 2-D geometry by
    0.05, free coordinates uniform in [-spread, spread]."""
    rng = np.random.default_rng(seed)
    d = s["d"]
    out = []
    while len(out) < n:
        p = np.zeros(d)
        p[:2] = rng.uniform(-10, 10, size=2)
        p[2:] = rng.uniform(-spread, spread, size=d - 2)
        if S.is_clear(p, s, 0.05):
            out.append(p)
    return np.array(out)


def _circles(s):
    """(centre (2,), radius, class, index) of every boundary circle of an
    extruded scene with a ball outer boundary."""
    out = [(np.asarray(s["sph_c"][j][:2]), float(s["sph_r"][j]), 1, j) for j in range(len(s["sph_r"]))]
    out.append((np.asarray(s["outer"]["c"][:2]), float(s["outer"]["r"]), 3, 0))
    return out


@pytest.mark.parametrize("d", [3, 5])
def test_distance_matches_brute_force_over_extruded_surfaces(oracle, d):
    """The boundary is {circle} x R^(d-2) for every circle; sample it in full
    d-space (dense angles, free coordinates offset from the point's own by a
    grid that contains 0 and by random offsets) and take the nearest sample.
    The oracle's distance must lie within the angular sampling gap of it and
    never above it, and name the same component."""
    s = S.scene_eval_env(d, k_r=0.3)
    dom = oracle.Domain(s)
    P = _interior_points(s, 40, seed=d)
    rng = np.random.default_rng(7)
    th = np.linspace(0.0, 2 * np.pi, 20000, endpoint=False)
    ring = np.stack([np.cos(th), np.sin(th)], axis=1)
    offs = np.concatenate([np.zeros((1, d - 2)), rng.normal(scale=0.5, size=(15, d - 2))])
    for x in P:
        best, arg = np.inf, None
        for c2, r, cls, idx in _circles(s):
            pts2 = c2 + r * ring
            for o in offs:
                diff = np.concatenate([pts2 - x[:2], np.broadcast_to(o, (len(ring), d - 2))], axis=1)
                m = np.sqrt((diff ** 2).sum(axis=1)).min()
                if m < best:
                    best, arg = m, (cls, idx)
        R, cls, idx = oracle.distance(dom, x)
        gap = 2 * np.pi * 10.0 / len(th)  # largest chord between samples
        assert R <= best + 1e-12 and best - R <= gap, (x, R, best)
        assert (cls, idx) == arg, (x, cls, idx, arg)


@pytest.mark.parametrize("d", [3, 4])
def test_empty_ball_and_closest_point(oracle, d):
    """B(x, R) holds no boundary point (membership by the 2-D disks), and the
    closest point lies on the absorbing circle at distance R with the free
    coordinates of x."""
    s = S.scene_eval_env(d, k_r=0.45)
    dom = oracle.Domain(s)
    rng = np.random.default_rng(11)
    for x in _interior_points(s, 25, seed=100 + d):
        R, cls, idx = oracle.distance(dom, x)
        v = rng.normal(size=(3000, d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        y = x + v * (R * rng.uniform(0, 1, size=(3000, 1)) ** (1.0 / d)) * (1 - 1e-9)
        y2 = y[:, :2]
        assert np.all((y2 ** 2).sum(1) < 100.0)
        for c, r in zip(s["sph_c"], s["sph_r"]):
            assert np.all(((y2 - c[:2]) ** 2).sum(1) > r * r)
        xb = oracle.closest_point(dom, x, cls, idx)
        assert np.allclose(xb[2:], x[2:], rtol=0, atol=0)
        assert abs(np.linalg.norm(xb - x) - R) < 1e-9
        c2, r = ((s["sph_c"][idx][:2], s["sph_r"][idx]) if cls == 1 else (np.zeros(2), 10.0))
        assert abs(np.linalg.norm(xb[:2] - c2) - r) < 1e-9


def _annulus_exact(rho, r_in, r_out, sigma):
    if sigma == 0.0:
        return math.log(r_out / rho) / math.log(r_out / r_in)
    from scipy.special import i0, k0
    k = math.sqrt(sigma)
    f = lambda t: k0(k * r_out) * i0(k * t) - i0(k * r_out) * k0(k * t)
    return f(rho) / f(r_in)


@pytest.mark.parametrize("d,sigma", [(3, 0.0), (4, 0.0), (3, 2.0)])
def test_extruded_annulus_is_the_planar_solution(oracle, d, sigma):
    """The solution on an annulus extruded along d - 2 free coordinates does
    not depend on them, so it is the 2-D annulus solution; the d-dimensional
    walk with d-dimensional screening weights reproduces it within 4 SE (plus
    the O(eps) shell bias)."""
    q = np.zeros((3, d))
    q[0, :2] = [0.8, 0.0]
    q[1, :2] = [-0.9, 0.6]
    q[2, :2] = [0.0, -1.5]
    q[:, 2:] = np.linspace(-3, 3, 3)[:, None]
    s = S.scene_extruded_annulus(d, sigma=sigma, queries=q, n_walks=6000, seed=3)
    u, g, st = oracle.estimate(s)
    for i, x in enumerate(q):
        ex = _annulus_exact(np.linalg.norm(x[:2]), 0.5, 2.0, sigma)
        assert abs(u[i] - ex) <= 4 * st[i, 0] + 2e-3, (i, u[i], ex, st[i, 0])


def test_affine_data_along_free_coordinates(oracle):
    """sigma = 0, g(y) = a.y + b on the extruded annulus with a slope along a
    free coordinate: u = a.x + b exactly (harmonic), which holds only if the
    closest boundary point keeps the walker's free coordinates."""
    d = 3
    q = np.array([[0.9, 0.3, 1.5], [-1.2, -0.4, -2.0]])
    s = S.scene_extruded_annulus(d, queries=q, n_walks=8000, seed=5)
    a = np.array([0.3, -0.2, 0.7])
    s["bdata"] = S._bdata(1, d, ak=a, b=0.25)
    u, g, st = oracle.estimate(s)
    for i, x in enumerate(q):
        assert abs(u[i] - (a @ x + 0.25)) <= 4 * st[i, 0] + 1e-3, (i, u[i], a @ x + 0.25)


def test_walks_are_invariant_along_free_coordinates(oracle):
    """Shifting the query and the source by t along a free coordinate leaves
    every walk's steps, status and estimates unchanged (the geometry does not
    see that coordinate)."""
    d = 3
    s0 = S.scene_eval_env(d, k_r=0.3, n_walks=64)
    s0["queries"] = np.array([[6.5, 0.5, 0.0]])
    s1 = dict(s0)
    t = 2.75
    s1["queries"] = s0["queries"] + np.array([0.0, 0.0, t])
    s1["source"] = dict(s0["source"], z=s0["source"]["z"] + np.array([0.0, 0.0, t]))
    d0, d1 = oracle.Domain(s0), oracle.Domain(s1)
    hits = 0
    for w in range(64):
        r0 = oracle.walk(s0, s0["queries"][0], w, 0, dom=d0)
        r1 = oracle.walk(s1, s1["queries"][0], w, 0, dom=d1)
        assert r0["steps"] == r1["steps"] and r0["status"] == r1["status"]
        assert r0["u"] == pytest.approx(r1["u"], rel=1e-9, abs=1e-300)
        assert np.allclose(r0["grad"], r1["grad"], rtol=1e-9, atol=1e-300)
        hits += r0["u"] > 0
    assert hits > 0


def test_full_geometry_dimension_is_the_plain_domain(oracle):
    """geom_d = d is the ordinary domain: identical walks to geom_d unset."""
    s0 = S.scene_c5(n_starts=2, n_walks=32)
    s1 = dict(s0, geom_d=s0["d"])
    d0, d1 = oracle.Domain(s0), oracle.Domain(s1)
    for w in range(32):
        r0 = oracle.walk(s0, s0["queries"][0], w, 0, dom=d0)
        r1 = oracle.walk(s1, s1["queries"][0], w, 0, dom=d1)
        assert r0["steps"] == r1["steps"] and r0["status"] == r1["status"]
        assert r0["u"] == r1["u"] and np.array_equal(r0["grad"], r1["grad"])
