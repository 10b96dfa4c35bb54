"""Pins of the oracle's estimator (u, grad u, backward, planning step) against
exact PDE solutions, a finite-difference solve, the O(1/sqrt(n)) law and
exact invariants.  Every tolerance is 4 standard errors plus the eps-shell
bias bound derived in the test (the estimator reads g at the closest point of
a walker within eps of the boundary, so its bias is at most eps |grad u|)."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from paper_2406_01713_amd import scenes as S
from tests.pins import closed_forms as CF


# ----------------------------------------------------------------- balls ----

@pytest.mark.parametrize("d", [2, 3, 5, 7])
@pytest.mark.parametrize("sigma", [0.5, 2.0, 8.0])
def test_ball_value_and_gradient(oracle, d, sigma):
    R = 1.0
    eps = 1e-4
    pts = []
    for i, frac in enumerate([0.25, 0.5, 0.9]):
        x = np.zeros(d)
        x[i % d] = frac * R
        x[(i + 1) % d] = 0.1 * frac * R
        pts.append(x)
    s = S.scene_ball(d, R=R, sigma=sigma, eps=eps, queries=np.array(pts), n_walks=4096, seed=7)
    u, g, st_ = oracle.estimate(s)
    for q, x in enumerate(pts):
        ue = CF.ball_u(d, sigma, R, x)
        ge = CF.ball_grad(d, sigma, R, x)
        gmax = np.linalg.norm(CF.ball_grad(d, sigma, R, np.r_[R, np.zeros(d - 1)]))
        r0 = R - np.linalg.norm(x)
        assert abs(u[q] - ue) <= 4 * st_[q, 0] + 2 * eps * gmax, (q, u[q], ue)
        assert np.all(np.abs(g[q] - ge) <= 4 * st_[q, 1:1 + d] + 2 * d * eps * gmax / r0), (q, g[q], ge)


@pytest.mark.parametrize("d", [2, 4, 7])
def test_ball_at_sigma_zero_is_exactly_one(oracle, d):
    s = S.scene_ball(d, sigma=0.0, queries=np.full((1, d), 0.2), n_walks=512)
    u, g, st_ = oracle.estimate(s)
    assert u[0] == 1.0 and st_[0, 0] == 0.0


@pytest.mark.parametrize("d", [2, 3, 6, 8])
def test_ball_centre_is_one_exact_jump(oracle, d):
    """From the centre the first ball is the whole ball: every walk makes one
    jump and lands on the sphere, so u_hat = C(R) with zero variance."""
    from tests.test_oracle_rng_series import _C_bessel
    for sigma in [0.5, 3.0]:
        s = S.scene_ball(d, R=1.3, sigma=sigma, n_walks=256)
        u, g, st_ = oracle.estimate(s)
        assert u[0] == pytest.approx(_C_bessel(d, sigma, 1.3), rel=1e-12)
        assert st_[0, 0] < 1e-15
        assert st_[0, d + 1] == 2.0  # one jump plus the absorbing evaluation


@pytest.mark.parametrize("d", [2, 5, 7])
def test_plane_wave_in_ball_pins_gradient_factor(oracle, d):
    """u = exp(k.x) with |k|^2 = sigma.  Without the screening factor C1 the
    first-sphere gradient estimate would be biased by 20-40 % here."""
    sigma = 8.0
    k = S.plane_wave_k(d, sigma, seed=d)
    x = np.zeros(d)
    x[0] = 0.2
    s = S.scene_ball(d, R=1.0, sigma=sigma, eps=1e-4, queries=x[None], n_walks=40000, seed=3,
                     mode=2, ak=k)
    u, g, st_ = oracle.estimate(s)
    ue, ge = CF.plane_wave(k, x)
    kn = math.sqrt(sigma)
    emax = math.exp(kn)  # largest boundary value on the unit sphere
    assert abs(u[0] - ue) <= 4 * st_[0, 0] + 2e-4 * kn * emax
    assert np.all(np.abs(g[0] - ge) <= 4 * st_[0, 1:1 + d] + 2e-4 * d * kn * emax / 0.8)
    # the literal first-sphere form (no C1) misses by several standard errors
    from tests.test_oracle_rng_series import _C_bessel
    c1 = _C_bessel(d + 2, sigma, 0.8)
    assert np.linalg.norm(g[0] / c1 - ge) > 4 * np.linalg.norm(st_[0, 1:1 + d]) / c1


@pytest.mark.parametrize("d,sigma", [(2, 0.0), (3, 0.0), (6, 0.0), (2, 2.0), (3, 4.0), (6, 2.0)])
def test_annulus(oracle, d, sigma):
    r_in, R = 0.3, 1.0
    pts = []
    for i, r in enumerate([0.4, 0.6, 0.85]):
        v = np.zeros(d)
        v[i % d] = 1.0
        v[(i + 1) % d] = 0.5
        pts.append(r * v / np.linalg.norm(v))
    s = S.scene_annulus(d, r_goal=r_in, R=R, sigma=sigma, eps=1e-4, queries=np.array(pts),
                        n_walks=8192, seed=11)
    u, g, st_ = oracle.estimate(s)
    for q, x in enumerate(pts):
        ue = CF.annulus_u(d, sigma, r_in, R, x)
        h = 1e-6
        gmax = abs(CF.annulus_u(d, sigma, r_in, R, np.r_[r_in + h, np.zeros(d - 1)]) - 1.0) / h
        assert abs(u[q] - ue) <= 4 * st_[q, 0] + 2e-4 * gmax, (q, u[q], ue)


# ------------------------------------------- affine / plane wave on scenes ----

def _scene_subset(name, nq):
    if name == "c1":
        s = S.scene_c1()
        free = [i for i, x in enumerate(s["queries"]) if S.is_clear(x, s, 0.05)]
        s["queries"] = s["queries"][free[:nq]]
    elif name == "c2":
        s = S.scene_c2(n_queries=nq)
    elif name == "c3":
        s = S.scene_c3()
        s["queries"] = s["queries"][::1024 // nq][:nq]
    else:
        s = S.scene_c5(n_starts=nq)
    return s


@pytest.mark.parametrize("name,nq,nw", [("c1", 6, 4096), ("c2", 3, 2048), ("c3", 3, 2048),
                                        ("c5", 2, 1024)])
def test_affine_data_at_sigma_zero(oracle, name, nq, nw):
    """Kakutani (Sec. IV): at sigma = 0, E[g(first exit)] = a.x + b for affine
    data in any geometry; the gradient is a."""
    s = _scene_subset(name, nq)
    d = s["d"]
    rng = np.random.default_rng(1)
    a = rng.normal(size=d)
    s = S.with_bdata(s, 1, ak=a, b=0.5)
    s.update(sigma=0.0, n_walks=nw, seed=5)
    u, g, st_ = oracle.estimate(s)
    an = np.linalg.norm(a)
    for q, x in enumerate(s["queries"]):
        R0 = oracle.distance(s, x)[0]
        assert abs(u[q] - (a @ x + 0.5)) <= 4 * st_[q, 0] + an * s["eps"]
        assert np.all(np.abs(g[q] - a) <= 4 * st_[q, 1:1 + d] + d * an * s["eps"] / R0)
        assert st_[q, d + 2] == 0  # nothing truncated


@pytest.mark.parametrize("name,nq,nw", [("c1", 6, 4096), ("c2", 3, 2048), ("c3", 3, 2048),
                                        ("c5", 2, 1024)])
def test_plane_wave_data_on_scenes(oracle, name, nq, nw):
    """u = exp(k.x), |k|^2 = sigma, solves the screened equation in any
    geometry: pins C, C1 and every obstacle type on the workload scenes."""
    s = _scene_subset(name, nq)
    d = s["d"]
    k = S.plane_wave_k(d, s["sigma"], seed=2)
    s = S.with_bdata(s, 2, ak=k)
    s.update(n_walks=nw, seed=9)
    u, g, st_ = oracle.estimate(s)
    kn = np.linalg.norm(k)
    for q, x in enumerate(s["queries"]):
        ue, ge = CF.plane_wave(k, x)
        R0 = oracle.distance(s, x)[0]
        bias = 2 * s["eps"] * kn * ue
        assert abs(u[q] - ue) <= 4 * st_[q, 0] + bias, (q, u[q], ue, st_[q, 0])
        assert np.all(np.abs(g[q] - ge) <= 4 * st_[q, 1:1 + d] + d * bias / R0), (q, g[q], ge)


# --------------------------------------------------------- FD solve, d = 2 ----

@pytest.mark.slow
def test_fd_solve_on_rr_scene(oracle):
    """C1 geometry (8 discs, goal disc, box) against a Shortley-Weller FD solve
    at h and h/2: |u_wos - u_fd| <= 4 SE + (4/3)|u_h - u_h/2| + eps-shell bias."""
    from tests.pins import fd2d
    s = S.scene_c1()
    s["eps"] = 1e-4
    N1, N2 = 256, 512
    _, U1 = fd2d.solve(fd2d.c1_discs(s), s["sigma"], N1)
    xs, U2 = fd2d.solve(fd2d.c1_discs(s), s["sigma"], N2)
    h = xs[1] - xs[0]
    gi, gj = np.round((s["goal_c"] + np.pi) / h).astype(int)
    cand = [(gi + di, gj + dj) for di, dj in [(-20, 0), (-40, 10), (0, 30), (25, -25), (-60, -60),
                                              (10, 60), (-90, 20), (0, -45)]]
    pts, ref, err = [], [], []
    for i, j in cand:
        x = np.array([xs[i], xs[j]])
        if not S.is_clear(x, s, 0.02) or i % 2 or j % 2:
            continue
        pts.append(x)
        ref.append(U2[i, j])
        err.append(abs(U2[i, j] - U1[i // 2, j // 2]) * 4.0 / 3.0)
    assert len(pts) >= 5
    s.update(queries=np.array(pts), n_walks=1 << 15, seed=21)
    u, g, st_ = oracle.estimate(s)
    for q in range(len(pts)):
        tol = 4 * st_[q, 0] + err[q] + 5 * s["eps"]
        assert abs(u[q] - ref[q]) <= tol, (pts[q], u[q], ref[q], st_[q, 0], err[q])


# ------------------------------------------------------ convergence order ----

def test_standard_error_decays_as_inverse_sqrt_n(oracle):
    """Sec. IV-B: the standard deviation of the mean falls as O(1/sqrt(n))."""
    s = _scene_subset("c1", 1)
    ns = [2 ** p for p in range(8, 15)]
    ses = []
    for n in ns:
        s.update(n_walks=n, seed=n)
        _, _, st_ = oracle.estimate(s)
        ses.append(st_[0, 0])
    slope = np.polyfit(np.log(ns), np.log(ses), 1)[0]
    assert -0.55 <= slope <= -0.45, slope


def _se_scale_case(name):
    if name == "c1":  # the three clear grid points nearest the goal (signal on many walks)
        s = S.scene_c1()
        free = [i for i, x in enumerate(s["queries"]) if S.is_clear(x, s, 0.05)]
        near = sorted(free, key=lambda i: np.linalg.norm(s["queries"][i] - s["goal_c"]))[:3]
        s["queries"] = s["queries"][near]
    elif name == "ball3":
        s = S.scene_ball(3, R=1.0, sigma=2.0, eps=1e-4, queries=[[0.5, 0.0, 0.0], [0.1, -0.6, 0.3]])
    else:  # plane-wave data in a 5-D ball: u = exp(k.x), a gradient in every coordinate
        k = S.plane_wave_k(5, 2.0, seed=3)
        s = S.scene_ball(5, R=1.0, sigma=2.0, eps=1e-4, queries=[[0.3, -0.2, 0.1, 0.0, 0.4]], mode=2, ak=k)
    return s


@pytest.mark.parametrize("name", ["c1", "ball3", "plane_d5"])
def test_standard_error_scale_matches_spread_of_estimates(oracle, name):
    """Sec. IV-B: the reported standard error is the standard deviation of the
    mean of n walks.  K = 256 independent estimates (distinct seeds, n = 256
    walks each): the empirical standard deviation of their values must agree
    with the root mean square of their reported SEs (SE^2 is unbiased for
    sigma^2 / n; SE itself is biased low for skewed walk values), for u and
    every gradient component.  The estimates are near-normal means, so
    (K - 1) s^2 / sigma^2 is chi-square with K - 1 degrees of freedom
    (relative spread of s about 1 / sqrt(2 (K - 1)) = 4.4 %); the mean of the
    K squared SEs adds its own spread.  The bar is 4 of the combined
    relative spreads (about 20 %): a constant-factor error of 1.5 in the SE
    fails it."""
    s = _se_scale_case(name)
    d = s["d"]
    K, n = 256, 256
    vals, ses = [], []
    for k in range(K):
        u, g, st_ = oracle.estimate(s, n_walks=n, seed=1000 + k)
        vals.append(np.concatenate([u[:, None], g], axis=1))
        ses.append(st_[:, :1 + d])
    vals, ses = np.array(vals), np.array(ses)  # (K, Q, 1 + d)
    emp = vals.std(axis=0, ddof=1)
    se2 = ses ** 2
    rep = np.sqrt(se2.mean(axis=0))
    spread = np.sqrt(1.0 / (2 * (K - 1)) + 0.25 * se2.var(axis=0, ddof=1) / (K * rep ** 4))
    ratio = emp / rep
    print(f"{name}: empirical sd / rms reported SE per (query, component):\n{np.round(ratio, 3)}\n"
          f"bars: {np.round(4 * spread, 3)}")
    assert np.all(rep > 0)
    assert np.all(np.abs(ratio - 1.0) <= 4 * spread), (ratio, spread)


# ------------------------------------------------------------- invariants ----

def _random_scene(d, seed, sigma):
    rng = np.random.default_rng(seed)
    s = S._empty(d)
    s.update(d=d, sph_c=rng.uniform(-2.5, 2.5, size=(4, d)), sph_r=rng.uniform(0.2, 0.6, size=4),
             box_c=rng.uniform(-2.5, 2.5, size=(2, d)), box_h=rng.uniform(0.1, 0.4, size=(2, d)),
             goal_c=rng.uniform(-2, 2, size=d), goal_r=0.4, outer=S.box_outer(d),
             bdata=S._bdata(0, d), sigma=sigma, eps=1e-3, n_walks=64, seed=seed)
    s["queries"] = S._free_points(rng, s, 2, 0.05)
    return s


@settings(max_examples=20, deadline=None)
@given(d=st.integers(2, 6), seed=st.integers(0, 10_000), sigma=st.floats(0.1, 6.0))
def test_walk_invariants(oracle, d, seed, sigma):
    s = _random_scene(d, seed, sigma)
    dom = oracle.Domain(s)
    s0 = dict(s, sigma=0.0)
    s_hi = dict(s, sigma=sigma * 1.5)
    ones = dict(s0, bdata=S._bdata(0, d, g_goal=1.0, g_obs=1.0, g_outer=1.0))
    dom1 = oracle.Domain(ones)
    for q, x in enumerate(s["queries"]):
        for w in range(16):
            r = oracle.walk(s, x, w, q, dom=dom)
            assert 0.0 <= r["u"] <= 1.0
            assert r["status"] in (0, 1)
            rh = oracle.walk(s_hi, x, w, q, dom=dom)
            # same path (law independent of sigma), larger sigma -> smaller weight
            assert rh["steps"] == r["steps"] and rh["cls"] == r["cls"]
            assert rh["u"] <= r["u"] + 1e-15
            # at sigma = 0 with g = 1 everywhere the absorption weights sum to 1
            assert oracle.walk(ones, x, w, q, dom=dom1)["u"] == 1.0
            # d u_hat / d sigma = u_hat * S <= 0
            assert r["u"] * r["dlnC_sum"] <= 0.0


def test_truncation_and_degenerate_queries(oracle):
    s = _scene_subset("c1", 2)
    s.update(n_walks=256)
    u, g, st_ = oracle.estimate(s, max_steps=2)
    d = 2
    assert np.all(st_[:, d + 2] > 0)  # walks hit the cap
    full = oracle.estimate(s)
    assert np.all(u <= full[0] + 1e-15)
    # a query inside obstacle 0: every walk is degenerate, u = g_obs, grad = 0
    c = S.scene_c1()
    c["queries"] = c["sph_c"][:1].copy()
    c["n_walks"] = 32
    u, g, st_ = oracle.estimate(c)
    assert u[0] == 0.0 and np.all(g == 0.0) and st_[0, d + 3] == 32
    # a query inside the goal: u = g_goal
    c["queries"] = c["goal_c"][None].copy()
    u, g, st_ = oracle.estimate(c)
    assert u[0] == 1.0 and st_[0, d + 3] == 32


# --------------------------------------------------------------- backward ----

def test_backward_matches_common_random_number_differences(oracle):
    s = _scene_subset("c3", 2)
    s.update(n_walks=512, seed=4)
    d = s["d"]
    ubar = np.array([0.7, -1.3])
    dx, dsig, dg = oracle.backward(s, ubar)
    u, g, st_, dq = oracle.estimate(s, dq=True)
    assert np.allclose(dx, ubar[:, None] * g, rtol=0, atol=1e-15)
    # sigma: same walks at sigma +- h, O(h^2) central difference
    h = 1e-4
    up = oracle.estimate(s, sigma=s["sigma"] + h)[0]
    um = oracle.estimate(s, sigma=s["sigma"] - h)[0]
    fd = (up - um) / (2 * h)
    assert np.allclose(dq[:, 0], fd, rtol=1e-6, atol=1e-12)
    assert dsig == pytest.approx(float(ubar @ fd), rel=1e-6, abs=1e-12)
    # goal value: u is linear in g_goal, so the difference is exact
    s1 = dict(s, bdata=dict(s["bdata"], g_goal=2.0))
    fdg = oracle.estimate(s1)[0] - u
    assert np.allclose(dq[:, 1], fdg, rtol=1e-12, atol=1e-15)
    assert dg == pytest.approx(float(ubar @ fdg), rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("d,sigma", [(3, 2.0), (7, 2.0), (2, 0.5)])
def test_dsigma_matches_ball_closed_form(oracle, d, sigma):
    x = np.zeros(d)
    x[0] = 0.45
    s = S.scene_ball(d, R=1.0, sigma=sigma, eps=1e-4, queries=x[None], n_walks=4000, seed=13)
    dom = oracle.Domain(s)
    vals = np.array([(lambda r: r["u"] * r["dlnC_sum"])(oracle.walk(s, x, w, 0, dom=dom))
                     for w in range(s["n_walks"])])
    want = CF.ball_du_dsigma(d, sigma, 1.0, x)
    se = vals.std(ddof=1) / math.sqrt(len(vals))
    assert abs(vals.mean() - want) <= 4 * se + 1e-4
    _, _, _, dq = oracle.estimate(s, dq=True)
    assert dq[0, 0] == pytest.approx(vals.mean(), rel=1e-12)


# ----------------------------------------------------------- planning step ----

def test_plan_step_rule_and_forward_invariance(oracle):
    """Starts 0.1 outside the goal sphere (in d = 7 far starts see no goal hits
    at this walk count): each move has length min(s_ub, d(x)/2) along the
    normalised mean gradient of the walks keyed by the start index and the
    step's seed, and the path stays in the domain."""
    s = S.scene_c5(n_starts=3, n_walks=512)
    rng = np.random.default_rng(3)
    starts = []
    while len(starts) < 3:
        v = rng.normal(size=7)
        p = s["goal_c"] + (s["goal_r"] + 0.1) * v / np.linalg.norm(v)
        if S.is_clear(p, s, 0.05):
            starts.append(p)
    x = np.ascontiguousarray(np.array(starts))
    S_ = len(x)
    path = np.zeros(S_)
    stalls = np.zeros(S_, dtype=np.int32)
    status = np.zeros(S_, dtype=np.int32)
    dom = oracle.Domain(s)
    moves = 0
    for t in range(3):
        before = x.copy()
        R_before = np.array([oracle.distance(s, p)[0] for p in before])
        oracle.plan_step(s, x, t, path, stalls, status)
        for i in range(S_):
            step = x[i] - before[i]
            moved = np.linalg.norm(step)
            if moved > 0:
                moves += 1
                assert moved == pytest.approx(min(s["s_ub"], 0.5 * R_before[i]), rel=1e-12)
                g = np.mean([oracle.walk(s, before[i], w, i, seed=s["seed"] + t, dom=dom)["grad"]
                             for w in range(s["n_walks"])], axis=0)
                assert np.allclose(step / moved, g / np.linalg.norm(g), atol=1e-12)
            assert oracle.distance(s, x[i])[0] > 0.0
    assert moves > 0 and path.sum() > 0


def test_plan_step_stalls_on_zero_gradient(oracle):
    s = S.scene_c5(n_starts=2, n_walks=64)
    s["bdata"] = S._bdata(0, 7, g_goal=0.0)  # g = 0 everywhere: grad u_hat == 0
    x = np.ascontiguousarray(s["queries"].copy())
    path = np.zeros(2)
    stalls = np.zeros(2, dtype=np.int32)
    status = np.zeros(2, dtype=np.int32)
    oracle.plan_step(s, x, 0, path, stalls, status)
    assert np.array_equal(x, s["queries"]) and np.all(stalls == 1) and np.all(path == 0)
