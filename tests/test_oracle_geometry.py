"""Pins of the oracle's distance-to-boundary function, closest points and
boundary data against brute force on tiny scenes (dense surface sampling and
point-membership tests written independently of the oracle)."""
import numpy as np
import pytest

from paper_2406_01713_amd import scenes as S


def _tiny_scene(d, seed):
    rng = np.random.default_rng(seed)
    s = S._empty(d)
    s.update(d=d, sph_c=rng.uniform(-2, 2, size=(3, d)), sph_r=rng.uniform(0.2, 0.6, size=3),
             box_c=rng.uniform(-2, 2, size=(2, d)), box_h=rng.uniform(0.1, 0.5, size=(2, d)),
             goal_c=rng.uniform(-2, 2, size=d), goal_r=0.3, outer=S.box_outer(d),
             bdata=S._bdata(0, d), sigma=1.0, eps=1e-3, n_walks=16, seed=seed)
    return s


def _surface_samples(s, n_per=20000, rng=None):
    """Points on every boundary component, with their (class, index) labels."""
    rng = rng or np.random.default_rng(0)
    d = s["d"]
    pts, lab = [], []

    def sphere_pts(c, r):
        v = rng.normal(size=(n_per, d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        return c + r * v

    pts.append(sphere_pts(s["goal_c"], s["goal_r"]))
    lab += [(0, 0)] * n_per
    for j, (c, r) in enumerate(zip(s["sph_c"], s["sph_r"])):
        pts.append(sphere_pts(c, r))
        lab += [(1, j)] * n_per
    for j, (c, h) in enumerate(zip(s["box_c"], s["box_h"])):
        p = rng.uniform(-1, 1, size=(n_per, d))
        ax = rng.integers(0, d, size=n_per)
        p[np.arange(n_per), ax] = np.sign(rng.uniform(-1, 1, size=n_per))
        pts.append(c + h * p)
        lab += [(2, j)] * n_per
    lo, hi = s["outer"]["lo"], s["outer"]["hi"]
    p = rng.uniform(lo, hi, size=(n_per, d))
    ax = rng.integers(0, d, size=n_per)
    side = rng.integers(0, 2, size=n_per)
    p[np.arange(n_per), ax] = np.where(side == 1, hi[ax], lo[ax])
    pts.append(p)
    lab += [(3, 0)] * n_per
    return np.concatenate(pts), lab


def _inside_any_obstacle(s, p):
    if np.any(((p[:, None, :] - s["sph_c"][None]) ** 2).sum(-1) < s["sph_r"][None] ** 2):
        return True
    if np.any(np.all(np.abs(p[:, None, :] - s["box_c"][None]) < s["box_h"][None], axis=-1)):
        return True
    if np.any(((p - s["goal_c"]) ** 2).sum(-1) < s["goal_r"] ** 2):
        return True
    lo, hi = s["outer"]["lo"], s["outer"]["hi"]
    return bool(np.any((p < lo) | (p > hi)))


@pytest.mark.parametrize("d", [2, 3])
def test_distance_against_brute_force(oracle, d):
    s = _tiny_scene(d, seed=d)
    dom = oracle.Domain(s)
    surf, lab = _surface_samples(s)
    rng = np.random.default_rng(5)
    checked = 0
    for x in rng.uniform(-3, 3, size=(60, d)):
        R, cls, idx = oracle.distance(dom, x)
        if R <= 0:
            continue
        checked += 1
        dist = np.linalg.norm(surf - x, axis=1)
        # every sampled boundary point is at least R away; the nearest is about R
        assert dist.min() >= R - 1e-12
        tol = 0.08 if d == 3 else 5e-3
        assert dist.min() <= R + tol
        # the ball of radius R is empty: random points inside it hit no obstacle
        v = rng.normal(size=(4000, d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        inner = x + (R * rng.uniform(0, 1, size=(4000, 1)) ** (1.0 / d)) * v * (1 - 1e-12)
        assert not _inside_any_obstacle(s, inner)
        # the closest point lies at distance R on the reported component
        xb = oracle.closest_point(dom, x, cls, idx)
        assert np.linalg.norm(xb - x) == pytest.approx(R, rel=1e-12, abs=1e-12)
        R2, _, _ = oracle.distance(dom, xb)
        assert abs(R2) < 1e-12
    assert checked > 20


def test_box_sdf_inside_is_minus_face_distance(oracle):
    d = 3
    s = S._empty(d)
    s.update(d=d, box_c=np.array([[0.0, 0.0, 0.0]]), box_h=np.array([[1.0, 0.5, 2.0]]),
             goal_c=None, goal_r=None, outer=S.box_outer(d, 10.0), bdata=S._bdata(0, d))
    R, cls, idx = oracle.distance(s, [0.2, -0.1, 0.3])
    assert cls == 2 and R == pytest.approx(-0.4)
    xb = oracle.closest_point(s, [0.2, -0.1, 0.3], cls, idx)
    assert np.allclose(xb, [0.2, -0.5, 0.3])
    # outside near a corner: Euclidean distance to the corner
    R, cls, _ = oracle.distance(s, [2.0, 1.5, 3.0])
    assert R == pytest.approx(np.sqrt(1 + 1 + 1))


def test_tie_prefers_goal_then_obstacles_in_order(oracle):
    d = 2
    s = S._empty(d)
    s.update(d=d, sph_c=np.array([[2.0, 0.0], [-2.0, 0.0]]), sph_r=np.array([1.0, 1.0]),
             goal_c=np.array([0.0, 2.0]), goal_r=1.0, outer=S.box_outer(d, 50.0), bdata=S._bdata(0, d))
    R, cls, idx = oracle.distance(s, [0.0, 0.0])
    assert R == pytest.approx(1.0) and cls == 0
    s["goal_c"] = np.array([0.0, 5.0])
    R, cls, idx = oracle.distance(s, [0.0, 0.0])
    assert cls == 1 and idx == 0


def test_outer_box_and_ball_distance(oracle):
    d = 4
    s = S._empty(d)
    s.update(d=d, goal_c=None, goal_r=None, outer=S.box_outer(d), bdata=S._bdata(0, d))
    R, cls, _ = oracle.distance(s, [3.0, 0, 0, -1.0])
    assert cls == 3 and R == pytest.approx(np.pi - 3.0)
    xb = oracle.closest_point(s, [3.0, 0, 0, -1.0], 3, 0)
    assert np.allclose(xb, [np.pi, 0, 0, -1.0])
    b = S.scene_ball(d, R=2.0)
    R, cls, _ = oracle.distance(b, [0.5, 0.5, 0.5, 0.5])
    assert cls == 3 and R == pytest.approx(1.0)


def test_boundary_value_modes(oracle):
    d = 3
    s = _tiny_scene(d, 1)
    x = np.array([2.9, 0.0, 0.1])
    R, cls, idx = oracle.distance(s, x)
    assert cls == 3
    assert oracle.boundary_value(s, x, cls, idx) == s["bdata"]["g_outer"]
    a = np.array([0.3, -1.0, 2.0])
    s1 = S.with_bdata(s, 1, ak=a, b=0.7)
    xb = oracle.closest_point(s, x, cls, idx)
    assert oracle.boundary_value(s1, x, cls, idx) == pytest.approx(a @ xb + 0.7)
    s2 = S.with_bdata(s, 2, ak=a)
    assert oracle.boundary_value(s2, x, cls, idx) == pytest.approx(np.exp(a @ xb))
