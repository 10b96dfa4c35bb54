"""GPU parity of the planar-arm distance bound (Sec. V-A) and the RR task of
Sec. VII against the FP64 oracle on identical Philox streams: per-walk
records with the Lipschitz bound (RR and longer arms), FP32 means within
4 SE, batched vs plain, and the RR planning task with the IK-point and
Lipschitz distances (the captured planning graph follows the oracle's
steps; with 1e5 walks per step the path reaches the goal, and a larger
screening coefficient gives a shorter path, as the paper reports)."""
import numpy as np
import pytest

from paper_2406_01713_amd import scenes as S
from tests.walkmatch import check_rate
from tests.test_gpu_parity import assert_within_4se, dev, gpu_batch, gpu_estimate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_01713_amd import binding
    return binding


def arm_env(links, pts, nw=256, seed=0, sigma=1.0, nq=4):
    """A planar arm with class data: g = 1 on collisions with the obstacle
    points, 0 on the joint box [-pi, pi]^d; queries at random joint angles
    whose Lipschitz bound exceeds 0.05."""
    d = len(links)
    s = S._empty(d)
    s.update(d=d, goal_c=None, goal_r=None, arm={"l": np.array(links, float), "pts": np.array(pts, float)},
             outer={"kind": "box", "lo": np.full(d, -np.pi), "hi": np.full(d, np.pi)},
             bdata=S._bdata(0, d, g_goal=0.0, g_obs=1.0, g_outer=0.0), sigma=sigma, eps=2e-3,
             n_walks=nw, seed=seed, name=f"arm{d}")
    return s


def with_queries(oracle, s, nq, seed=1):
    dom = oracle.Domain(s)
    rng = np.random.default_rng(seed)
    qs = []
    while len(qs) < nq:
        q = rng.uniform(-2.5, 2.5, size=s["d"])
        if oracle.distance(dom, q)[0] > 0.05:
            qs.append(q)
    s["queries"] = np.array(qs)
    return s


ARMS = {"rr": ((1.0, 1.0), [(0.0, 1.3)]),
        "r3": ((0.3, 1.0, 0.7), [(0.5, 1.2), (-1.1, 0.4), (0.9, -0.9)]),
        "r6": ((0.4, 0.35, 0.3, 0.3, 0.25, 0.2), [(1.0, 0.6), (-0.7, 1.0), (0.2, -1.1), (1.3, -0.2)])}


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("which", ["rr", "r3", "r6"])
def test_arm_walk_level_parity(B, oracle, which, fp64):
    s = with_queries(oracle, arm_env(*ARMS[which], nw=128), 4)
    dom = B.Domain(s)
    odom = oracle.Domain(s)
    d = s["d"]
    n = s["n_walks"]
    tol = 1e-9 if fp64 else 2e-4
    same = arm_hits = 0
    for qi, x in enumerate(s["queries"]):
        rec = B.wos_debug_walks(dom, x, qi, 0, n, s["sigma"], s["eps"], s["seed"], B.options(fp64))
        for w in range(n):
            r = oracle.walk(s, x, w, qi, dom=odom)
            if int(rec[w, d + 3]) != r["steps"]:
                continue
            same += 1
            arm_hits += r["cls"] == oracle.ARM
            assert abs(rec[w, 0] - r["u"]) <= tol * max(1.0, abs(r["u"])), (qi, w, rec[w, 0], r["u"])
            assert np.allclose(rec[w, 1:1 + d], r["grad"], rtol=10 * tol, atol=10 * tol), (qi, w)
            assert int(rec[w, d + 4]) == r["status"]
            assert int(rec[w, d + 5]) == r["cls"], (qi, w)
    total = n * len(s["queries"])
    check_rate(f"arm {which}", fp64, same, total)
    assert arm_hits >= 0.05 * total, arm_hits


@pytest.mark.parametrize("which", ["rr", "r3"])
def test_arm_fp32_estimate_vs_oracle(B, oracle, which):
    s = with_queries(oracle, arm_env(*ARMS[which], nw=4096, seed=3), 3, seed=2)
    u, g, st = gpu_estimate(B, s)
    uc, gc, stc = oracle.estimate(s)
    assert_within_4se(u, g, uc, gc, stc, s["d"])


def test_arm_batch_matches_plain(B, oracle):
    envs = [with_queries(oracle, arm_env(*ARMS["r3"], nw=256), 5), S.scene_rr("lipschitz", n_walks=256),
            S.scene_rr("ik", n_walks=256), S.scene_c4_env(2, n_walks=256, seed=7, q_cap=6)]
    for s in envs:
        s["seed"] = 7
    out = gpu_batch(B, envs, 256, 7)
    off = out["off"]
    for e, s in enumerate(envs):
        d = s["d"]
        sl = slice(off[e], off[e + 1])
        u, g, st = gpu_estimate(B, s, n_walks=256, seed=7, env_id=e)
        assert np.allclose(out["u"][sl], u, rtol=2e-5, atol=1e-12), e
        assert np.allclose(out["g"][sl, :d], g, rtol=2e-5, atol=1e-9), e
        assert np.allclose(out["st"][sl, 9], st[:, d + 1], rtol=1e-12), e


@pytest.mark.parametrize("distance", ["ik", "lipschitz"])
def test_rr_plan_follows_the_oracle(B, oracle, distance):
    """Three captured planning steps from q_start and two nearby starts
    (512 walks per gradient) reproduce the oracle's steps."""
    import torch
    s = S.scene_rr(distance, sigma=5.0, n_walks=512)
    x0 = np.array([S.RR_Q_START, [0.6, 1.2], [1.9, 0.9]])
    x = dev(x0, torch.float32)
    dom = B.Domain(s)
    plan = B.Plan(dom, x, 512, s["sigma"], s["eps"], s["s_ub"], s["seed"])
    xo = np.ascontiguousarray(x0.astype(np.float32).astype(np.float64))
    path = np.zeros(3)
    stalls = np.zeros(3, dtype=np.int32)
    status = np.zeros(3, dtype=np.int32)
    for t in range(3):
        plan.step(1)
        sts = plan.read()[4]
        oracle.plan_step(s, xo, t, path, stalls, status)
        xg = x.cpu().numpy().astype(np.float64)
        assert np.array_equal(sts, status)
        assert np.allclose(xg, xo, atol=2e-4), (t, np.abs(xg - xo).max())
    del plan


def rr_path(B, distance, sigma, n_walks=100000, max_steps=300):
    import torch
    s = S.scene_rr(distance, sigma=sigma, n_walks=n_walks)
    x = dev(np.array([S.RR_Q_START]), torch.float32)
    plan = B.Plan(B.Domain(s), x, n_walks, s["sigma"], s["eps"], s["s_ub"], s["seed"])
    plan.step(max_steps)
    u, g, path, stalls, status, step = plan.read()
    del plan
    return float(path[0]), int(status[0]), x.cpu().numpy()[0]


def test_rr_paths_reach_the_goal_and_screening_shortens_them(B):
    """Sec. VII: with 1e5 walks per step, s = min(0.1, d/2) and eps = 0.02 the
    path from q_start reaches q_goal with either distance function, and the
    screened path (c = 5) is shorter than the harmonic one (c = 0)."""
    res = {}
    for distance in ("ik", "lipschitz"):
        for sigma in (0.0, 5.0):
            L, st, xe = rr_path(B, distance, sigma)
            print(f"RR {distance} c={sigma:g}: path length {L:.3f}, status {st}, end {xe}")
            assert st == 1, (distance, sigma, st, xe)
            assert np.linalg.norm(xe - np.array(S.RR_Q_GOAL)) <= 0.1 + 1e-6
            res[distance, sigma] = L
    for distance in ("ik", "lipschitz"):
        assert res[distance, 5.0] < res[distance, 0.0], res


def test_rr_ik_points_culling_is_exact(B):
    """The RR task's 200 IK points (radius-0 obstacles, clustered): the
    culled scan, with the pair scan's bounding-box test by default (off in
    two dimensions), forced on, or forced off, gives bitwise the walks of a
    full scan."""
    s = S.scene_rr("ik", sigma=5.0, n_walks=2048)
    rng = np.random.default_rng(3)
    q = np.concatenate([np.asarray(s["queries"]),
                        rng.uniform([-np.pi / 2 + 0.2, -np.pi + 0.2], [3 * np.pi / 2 - 0.2, np.pi - 0.2], size=(7, 2))])
    a = gpu_estimate(B, s, queries=q)
    for kw in (dict(full_scan=True), dict(box_test=True), dict(no_box_test=True)):
        b = gpu_estimate(B, s, queries=q, **kw)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), kw
