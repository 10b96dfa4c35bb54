"""Pins of the oracle's point-source terms (Sec. IV-A volume and gradient
terms; Sec. VI unit impulse at the goal): the Bessel function K_nu against
SciPy, the ball Green's function against its elementary d = 3 form, the
radial equations it must solve with their boundary and flux conditions, the
Laplace image construction, the sigma derivative against finite differences,
and the whole estimator against the exact solution on a ball with a central
source.  All CPU."""
import math

import numpy as np
import pytest
from scipy import special

from paper_2406_01713_amd import scenes as S


def area(d):
    return 2 * math.pi ** (d / 2) / math.gamma(d / 2)


@pytest.mark.parametrize("nu", [0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0])
def test_bessel_k_matches_scipy(oracle, nu):
    for z in np.geomspace(1e-4, 40.0, 23):
        ref = special.kv(nu, z)
        assert oracle.bessel_k(nu, z) == pytest.approx(ref, rel=1e-12), (nu, z)


def test_free_space_solution_d3_and_laplace(oracle):
    for sig in (0.5, 2.0, 8.0):
        for r in (0.01, 0.3, 2.0):
            assert oracle.yukawa_free(3, sig, r) == pytest.approx(math.exp(-math.sqrt(sig) * r) / (4 * math.pi * r),
                                                                 rel=1e-12)
    for d in range(3, 9):
        assert oracle.yukawa_free(d, 0.0, 0.7) == pytest.approx(0.7 ** (2 - d) / ((d - 2) * area(d)), rel=1e-14)
    assert oracle.yukawa_free(2, 0.0, 0.7) == pytest.approx(-math.log(0.7) / (2 * math.pi), rel=1e-14)


def test_ball_green_d3_elementary(oracle):
    """d = 3: G_B(r; R) = [e^{-ar}/r - (e^{-aR}/R) (sinh(ar)/r) / (sinh(aR)/R)] / (4 pi)."""
    for sig in (0.5, 2.0, 8.0):
        a = math.sqrt(sig)
        for R in (0.4, 1.0, 2.5):
            for r in (0.05 * R, 0.5 * R, 0.95 * R):
                ref = (math.exp(-a * r) / r - math.exp(-a * R) / R * (math.sinh(a * r) / r) / (math.sinh(a * R) / R)) / (4 * math.pi)
                assert oracle.ball_green(3, sig, r, R) == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("sig", [0.0, 0.5, 2.0, 8.0])
def test_ball_green_solves_radial_problem(oracle, d, sig):
    """G'' + (d-1)/r G' - sigma G = 0 inside, G(R) = 0, and the flux
    -|S| r^{d-1} G'(r) -> 1 at the source (a unit impulse)."""
    R = 1.3
    G = lambda r: oracle.ball_green(d, sig, r, R)
    for r in (0.2, 0.5, 0.9, 1.2):
        h = 1e-3 * r
        g0, gp, gm = G(r), G(r + h), G(r - h)
        d2 = (gp - 2 * g0 + gm) / h ** 2
        d1 = (gp - gm) / (2 * h)
        lhs = d2 + (d - 1) / r * d1 - sig * g0
        scale = abs(d2) + abs((d - 1) / r * d1) + abs(sig * g0)
        assert abs(lhs) <= 1e-5 * scale + 1e-9, (r, lhs, scale)
    assert abs(G(R * (1 - 1e-12))) < 1e-9
    r = 1e-4
    h = 1e-3 * r
    flux = -area(d) * r ** (d - 1) * (G(r + h) - G(r - h)) / (2 * h)
    assert flux == pytest.approx(1.0, rel=2e-5)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("sig", [0.0, 0.5, 2.0, 8.0])
def test_ball_green_gradient_solves_l1_problem(oracle, d, sig):
    """The centre gradient towards a source at distance r is the l = 1 radial
    mode: q'' + (d-1)/r q' - (d-1)/r^2 q - sigma q = 0, q(R) = 0, and
    |S| r^{d-1} q(r) -> 1 at the source (the free-space gradient)."""
    R = 1.3
    q = lambda r: oracle.ball_green_grad(d, sig, r, R)
    for r in (0.2, 0.5, 0.9, 1.2):
        h = 1e-3 * r
        q0, qp, qm = q(r), q(r + h), q(r - h)
        d2 = (qp - 2 * q0 + qm) / h ** 2
        d1 = (qp - qm) / (2 * h)
        lhs = d2 + (d - 1) / r * d1 - (d - 1) / r ** 2 * q0 - sig * q0
        scale = abs(d2) + abs((d - 1) / r * d1) + abs((d - 1) / r ** 2 * q0) + abs(sig * q0)
        assert abs(lhs) <= 1e-5 * scale + 1e-9, (r, lhs, scale)
    assert abs(q(R * (1 - 1e-12))) < 1e-9
    assert area(d) * 1e-4 ** (d - 1) * q(1e-4) == pytest.approx(1.0, rel=1e-6)


@pytest.mark.parametrize("d", [3, 4, 7])
def test_ball_green_gradient_matches_kelvin_image(oracle, d):
    """Laplace: G_B(x, y) = Phi(|x - y|) - Phi(|y| |x - y*| / R), y* = R^2 y / |y|^2
    (the Kelvin image), differentiated in x at the centre by finite differences."""
    R = 1.0
    phi = lambda r: r ** (2 - d) / ((d - 2) * area(d))
    y = np.zeros(d)
    y[0] = 0.37
    y[1] = -0.21
    r = np.linalg.norm(y)
    ys = R ** 2 * y / r ** 2
    G = lambda x: phi(np.linalg.norm(x - y)) - phi(r * np.linalg.norm(x - ys) / R)
    h = 1e-5
    grad = np.array([(G(h * e) - G(-h * e)) / (2 * h) for e in np.eye(d)])
    ref = oracle.ball_green_grad(d, 0.0, r, R) * y / r
    assert np.allclose(grad, ref, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_ball_green_dsigma_matches_finite_difference(oracle, d):
    R = 1.1
    for sig in (0.5, 2.0, 8.0):
        for r in (0.05, 0.4, 0.9):
            h = 1e-4 * sig
            fd = (oracle.ball_green(d, sig + h, r, R) - oracle.ball_green(d, sig - h, r, R)) / (2 * h)
            assert oracle.ball_green_dsigma(d, sig, r, R) == pytest.approx(fd, rel=2e-6, abs=1e-12)


def test_small_sigma_tends_to_laplace(oracle):
    for d in (2, 3, 6):
        for r in (0.1, 0.6):
            assert oracle.ball_green(d, 1e-9, r, 1.0) == pytest.approx(oracle.ball_green(d, 0.0, r, 1.0), rel=1e-6)
            assert oracle.ball_green_grad(d, 1e-9, r, 1.0) == pytest.approx(oracle.ball_green_grad(d, 0.0, r, 1.0),
                                                                           rel=1e-6)


# ------------------------------------------------------------ estimator ----

def _radial_derivative(oracle, d, sig, r, R):
    h = 1e-6
    return (oracle.ball_green(d, sig, r + h, R) - oracle.ball_green(d, sig, r - h, R)) / (2 * h)


@pytest.mark.parametrize("d,sig", [(2, 0.0), (2, 2.0), (3, 0.0), (3, 2.0)])
def test_estimator_matches_ball_green_function(oracle, d, sig):
    """Ball of radius 1 with a unit source at its centre, zero data: the
    estimate of u and grad u at off-centre queries matches G_B(|x|; 1) and
    its radial derivative within 4 SE (finite variance for d <= 3).  The
    query at |x| = 0.3 has the source in its first ball, which exercises the
    source-gradient term; the one at 0.7 does not."""
    qs = np.zeros((2, d))
    qs[0, 0] = 0.3
    qs[1, 0] = -0.5
    qs[1, 1] = 0.5
    s = S.scene_ball_source(d, R=1.0, sigma=sig, eps=1e-4, queries=qs, n_walks=1 << 14, seed=3)
    u, g, st = oracle.estimate(s)
    for q in range(2):
        r = np.linalg.norm(qs[q])
        exact = oracle.ball_green(d, sig, r, 1.0)
        assert abs(u[q] - exact) <= 4 * st[q, 0] + 1e-9, (q, u[q], exact, st[q, 0])
        gexact = _radial_derivative(oracle, d, sig, r, 1.0) * qs[q] / r
        assert np.all(np.abs(g[q] - gexact) <= 4 * st[q, 1:1 + d] + 1e-9), (q, g[q], gexact)


def test_source_is_linear_and_superposes(oracle):
    """Same geometry, same walks: doubling the amplitude doubles u_hat and
    grad_hat, and the estimate with goal data and a source is the sum of the
    goal-data estimate and the source-only one (u is linear in (g, f))."""
    base = S.scene_c3(n_walks=64)
    qs = base["queries"][::200][:5]
    z = base["goal_c"] + np.r_[0.4, np.zeros(6)]
    both = S.with_source(base, z, amp=1.0, keep_goal=True)
    only_src = S.with_source(base, z, amp=1.0, keep_goal=True, g_goal=0.0)
    only_src2 = S.with_source(base, z, amp=2.0, keep_goal=True, g_goal=0.0)
    for qi, x in enumerate(qs):
        for w in range(64):
            a = oracle.walk(only_src, x, w, qi)
            b = oracle.walk(only_src2, x, w, qi)
            c = oracle.walk(both, x, w, qi)
            g = oracle.walk(base, x, w, qi)
            assert b["u"] == pytest.approx(2 * a["u"], rel=1e-14, abs=1e-300)
            assert np.allclose(b["grad"], 2 * a["grad"], rtol=1e-14, atol=0)
            assert a["steps"] == g["steps"] == c["steps"]
            assert c["u"] == pytest.approx(a["u"] + g["u"], rel=1e-12, abs=1e-300)
            assert np.allclose(c["grad"], a["grad"] + g["grad"], rtol=1e-12, atol=1e-300)


def test_source_gradient_term_only_inside_first_ball(oracle):
    """The deterministic c_imp grad G_B term appears iff the source lies in
    the first ball, and scales with c_imp."""
    s0 = S.scene_ball_source(3, R=1.0, sigma=2.0, n_walks=8)
    s1 = dict(s0)
    s1["source"] = dict(s0["source"], c_imp=3.0)
    near = np.array([0.2, 0.0, 0.0])   # |z - x0| = 0.2 < R0 = 0.8
    far = np.array([0.6, 0.0, 0.0])    # |z - x0| = 0.6 > R0 = 0.4
    for w in range(8):
        a, b = oracle.walk(s0, near, w), oracle.walk(s1, near, w)
        term = oracle.ball_green_grad(3, 2.0, 0.2, 0.8) * (-near) / 0.2
        assert np.allclose(b["grad"] - a["grad"], 2 * term, rtol=1e-10)
        a, b = oracle.walk(s0, far, w), oracle.walk(s1, far, w)
        assert np.array_equal(a["grad"], b["grad"])


def test_source_backward_matches_crn_finite_difference(oracle):
    """du_hat/dsigma with a source (weights and Green's functions both depend
    on sigma) against central differences on the same walks."""
    base = S.scene_c3(n_walks=32)
    z = base["goal_c"] + np.r_[0.3, np.zeros(6)]
    s = S.with_source(base, z)
    x = base["queries"][-3]
    h = 1e-4
    for w in range(32):
        r = oracle.walk(s, x, w, 0)
        up = oracle.walk(s, x, w, 0, sigma=s["sigma"] + h)["u"]
        dn = oracle.walk(s, x, w, 0, sigma=s["sigma"] - h)["u"]
        assert r["du_dsigma"] == pytest.approx((up - dn) / (2 * h), rel=1e-5, abs=1e-10)


def test_planning_arrives_at_point_source(oracle):
    """With a point-source goal a start within one nominal step of the source
    is reported as arrived."""
    s = S.with_source(S.scene_c5(n_starts=2, n_walks=16), np.zeros(7))
    s["queries"] = np.zeros((2, 7))
    x = np.array([[0.01, 0, 0, 0, 0, 0, 0], [0.5, 0, 0, 0, 0, 0, 0]], dtype=np.float64)
    pl = np.zeros(2)
    st = np.zeros(2, np.int32)
    status = np.zeros(2, np.int32)
    R0 = oracle.distance(s, x[1])[0]
    if R0 < s["eps"]:
        pytest.skip("start inside an obstacle")
    oracle.plan_step(s, x, 0, pl, st, status)
    assert status[0] == 1
    assert status[1] in (0, 2)
