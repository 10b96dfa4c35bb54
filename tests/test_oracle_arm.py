"""Pins of the oracle's planar-arm distance (Sec. V-A: the joint-space
distance to collision bounded below by the task-space distance over a
Lipschitz constant of the forward kinematics) and of the IK-based collision
points of the RR task (Sec. VII), on the CPU.  Forward kinematics here is
written independently of the oracle and evaluated by dense sampling along
the links."""
import numpy as np
import pytest

from paper_2406_01713_amd import scenes as S


def fk_samples(q, links, n=4001):
    """Points sampled densely along every link of the planar arm."""
    out = []
    base = np.zeros(2)
    th = 0.0
    for qi, li in zip(q, links):
        th += qi
        tip = base + li * np.array([np.cos(th), np.sin(th)])
        s = np.linspace(0.0, 1.0, n)[:, None]
        out.append(base + s * (tip - base))
        base = tip
    return np.concatenate(out)


def task_distance_brute(q, links, pts):
    P = fk_samples(q, links)
    return np.sqrt(((P[:, None, :] - np.asarray(pts)[None]) ** 2).sum(-1)).min()


def arm_scene(links, pts, half=np.pi):
    d = len(links)
    s = S._empty(d)
    s.update(d=d, goal_c=None, goal_r=None, arm={"l": np.array(links, float), "pts": np.array(pts, float)},
             outer={"kind": "box", "lo": np.full(d, -50.0), "hi": np.full(d, 50.0)},
             bdata=S._bdata(0, d, g_goal=0.0, g_obs=0.0, g_outer=1.0), sigma=1.0, eps=1e-3,
             queries=np.zeros((1, d)), n_walks=64, seed=0)
    return s


ARMS = [((1.0, 1.0), [(0.0, 1.3)]),
        ((0.3, 1.0, 0.7), [(0.5, 1.2), (-1.1, 0.4), (0.9, -0.9)]),
        ((0.5, 0.4, 0.3, 0.6, 0.2), [(1.0, 1.0), (-0.4, 1.5)])]


@pytest.mark.parametrize("links,pts", ARMS)
def test_task_distance_matches_brute_force(oracle, links, pts):
    s = arm_scene(links, pts)
    dom = oracle.Domain(s)
    rng = np.random.default_rng(len(links))
    gap = max(links) / 4000
    for _ in range(30):
        q = rng.uniform(-np.pi, np.pi, size=len(links))
        dt = oracle.arm_task_distance(dom, q)
        bf = task_distance_brute(q, links, pts)
        assert dt <= bf + 1e-12 and bf - dt <= gap, (q, dt, bf)
        R, cls, _ = oracle.distance(dom, q)  # the box is far: the arm term decides
        assert cls == oracle.ARM and R == pytest.approx(dt / oracle.arm_K(dom), rel=1e-14)


@pytest.mark.parametrize("links,pts", ARMS)
def test_K_bounds_every_arm_point_speed(oracle, links, pts):
    """K is at least the spectral norm of the Jacobian of every point of the
    arm (central differences), and is attained by the straight arm's tip for
    motions of all joints together."""
    s = arm_scene(links, pts)
    K = oracle.arm_K(oracle.Domain(s))
    rng = np.random.default_rng(3)
    d = len(links)
    h = 1e-6
    worst = 0.0
    for _ in range(200):
        q = rng.uniform(-np.pi, np.pi, size=d)
        k = rng.integers(d)
        f = rng.uniform(0, 1)

        def point(qq):
            base = np.zeros(2)
            th = 0.0
            for i in range(k + 1):
                th += qq[i]
                step = links[i] * np.array([np.cos(th), np.sin(th)])
                if i == k:
                    return base + f * step
                base = base + step

        J = np.stack([(point(q + h * e) - point(q - h * e)) / (2 * h) for e in np.eye(d)], axis=1)
        worst = max(worst, np.linalg.norm(J, 2))
    assert worst <= K * (1 + 1e-6)
    reach = np.cumsum(np.asarray(links)[::-1])[::-1]  # joint n to the tip, straight arm
    assert K == pytest.approx(np.sqrt((reach ** 2).sum()), rel=1e-14)


@pytest.mark.parametrize("links,pts", ARMS)
def test_safe_ball_holds_no_collision(oracle, links, pts):
    """Sec. V, eq. safe_ball: every configuration in B(q, d_tau(q) / K)
    keeps the arm off every obstacle point."""
    s = arm_scene(links, pts)
    dom = oracle.Domain(s)
    rng = np.random.default_rng(11)
    d = len(links)
    for _ in range(12):
        q = rng.uniform(-np.pi, np.pi, size=d)
        R, cls, _ = oracle.distance(dom, q)
        v = rng.normal(size=(60, d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        for qq in q + R * v * rng.uniform(0, 1, size=(60, 1)) ** (1.0 / d):
            assert task_distance_brute(qq, links, pts) > 0.0


def test_ik_points_sit_on_the_collision_set():
    """The N_col = 200 IK points put the obstacle point on link 2, and their
    spacing lies in the range the paper prints (0.017 to 0.0235)."""
    P = S.rr_collision_points()
    assert P.shape == (200, 2)
    for q in P:
        assert task_distance_brute(q, S.RR_LINKS, [S.RR_X_OBS]) < 2e-4
    sp = np.linalg.norm(np.diff(P, axis=0), axis=1)
    assert sp.min() >= 0.017 and sp.max() <= 0.0235
    lo, hi = np.array(S.RR_Q_LO), np.array(S.RR_Q_HI)
    assert np.all(P > lo) and np.all(P < hi)


def test_lipschitz_distance_underestimates_the_ik_distance(oracle):
    """The bound never exceeds the joint-space distance to the IK points,
    which lie on the collision set."""
    s = S.scene_rr("lipschitz", n_walks=16)
    dom = oracle.Domain(s)
    P = S.rr_collision_points()
    rng = np.random.default_rng(5)
    for _ in range(300):
        q = rng.uniform(S.RR_Q_LO, S.RR_Q_HI)
        dt = oracle.arm_task_distance(dom, q) / oracle.arm_K(dom)
        assert dt <= np.linalg.norm(P - q, axis=1).min() + 1e-12


def test_unreachable_arm_obstacle_leaves_the_solution(oracle):
    """An obstacle point beyond the arm's reach never absorbs a walk (the
    bound stays above eps); it only shrinks the balls, so the estimate
    matches the one without the arm within 4 SE of both."""
    links = (1.0, 1.0)
    s = arm_scene(links, [(0.0, 2.6)], half=1.0)
    s["outer"] = {"kind": "box", "lo": np.full(2, -1.0), "hi": np.full(2, 1.0)}
    s["queries"] = np.array([[0.3, -0.2], [-0.5, 0.6]])
    s["n_walks"] = 20000
    s0 = dict(s)
    s0.pop("arm")
    u, g, st = oracle.estimate(s)
    u0, g0, st0 = oracle.estimate(s0)
    assert np.all(np.abs(u - u0) <= 4 * np.hypot(st[:, 0], st0[:, 0])), (u, u0)
    assert np.all(np.abs(g - g0) <= 4 * np.hypot(st[:, 1:3], st0[:, 1:3]))
