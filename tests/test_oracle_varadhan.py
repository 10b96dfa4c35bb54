"""Pins of the Varadhan read-out w = -sqrt(t) ln u, t = 1/sigma (Sec. III, eq.
transformation_varadhan), on the CPU: with plane-wave boundary data the
estimated w is the signed distance to a plane; at the centre of a ball with
unit data w tends to the radius as t -> 0 with the known correction terms; the
transformed ball solution solves the regularized eikonal equation of Sec. III;
no signal (u <= 0) reads as an infinite distance."""
import math

import numpy as np
import pytest

from paper_2406_01713_amd import scenes as S


def test_plane_wave_reads_out_a_signed_distance(oracle):
    """u = exp(k.x), |k|^2 = sigma, solves the screened equation; w = -k.x /
    sqrt(sigma) is the signed distance to the plane k.x = 0 along -k/|k|.
    The estimator's u gives that w within 4 SE (delta method: SE_w = SE_u /
    (u sqrt(sigma)))."""
    base = S.scene_c1(n_walks=4096, seed=2)
    k = S.plane_wave_k(2, base["sigma"], seed=4)
    s = S.with_bdata(base, 2, ak=k)
    qs = s["queries"][[9, 20, 35, 50]]
    u, g, st = oracle.estimate(s, queries=qs)
    for q, x in enumerate(qs):
        w, gw = oracle.varadhan(s["sigma"], u[q], g[q])
        exact = -float(k @ x) / math.sqrt(s["sigma"])
        se_w = st[q, 0] / (u[q] * math.sqrt(s["sigma"]))
        assert abs(w - exact) <= 4 * se_w + 1e-12, (q, w, exact, se_w)
        # grad w = -grad u / (u sqrt(sigma)) -> -k / sqrt(sigma), a unit vector
        assert np.allclose(gw, -k / math.sqrt(s["sigma"]), atol=4 * np.abs(st[q, 1:3]).max() / (u[q] * math.sqrt(s["sigma"])) + 0.05)


@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_ball_centre_tends_to_the_radius(oracle, d):
    """u(0) = 1 / 0F1(; d/2; sigma R^2 / 4) on a ball with unit data, so
    w(0) = ln 0F1 / sqrt(sigma).  With I_nu's expansion at large argument,
    sqrt(sigma) (w - R) = -(nu + 1/2) ln(sqrt(sigma) R) + ln(Gamma(nu+1) 2^nu / sqrt(2 pi)) + o(1)."""
    R = 1.3
    nu = d / 2 - 1
    c = math.log(math.gamma(nu + 1) * 2 ** nu / math.sqrt(2 * math.pi))
    errs = []
    for sigma in (1e2, 1e3, 1e4, 1e5):
        u0 = oracle.screening_C(d, sigma, R)
        w = oracle.varadhan(sigma, u0)
        errs.append(abs(w - R))
        rem = math.sqrt(sigma) * (w - R) + (nu + 0.5) * math.log(math.sqrt(sigma) * R) - c
        if sigma == 1e5:  # next term of the expansion: O(1 / (sqrt(sigma) R)) < 1e-2
            assert abs(rem) < 2e-2, rem
    assert errs[0] > errs[1] > errs[2] > errs[3]


@pytest.mark.parametrize("d", [2, 3, 7])
@pytest.mark.parametrize("sigma", [0.5, 4.0, 50.0])
def test_ball_solution_solves_regularized_eikonal(oracle, d, sigma):
    """u(r) = p(r) / p(R), p(r) = 0F1(; d/2; sigma r^2 / 4), is the ball
    solution with unit data; w = -sqrt(t) ln u satisfies
    (1 - |w'|^2) + sqrt(t) (w'' + (d-1)/r w') = 0 (Sec. III)."""
    R = 1.0
    t = 1.0 / sigma
    pR = oracle.hyp0f1(d / 2, sigma * R * R / 4)
    w = lambda r: oracle.varadhan(sigma, oracle.hyp0f1(d / 2, sigma * r * r / 4) / pR)
    for r in (0.2, 0.5, 0.8):
        h = 1e-4
        w0, wp, wm = w(r), w(r + h), w(r - h)
        d1 = (wp - wm) / (2 * h)
        d2 = (wp - 2 * w0 + wm) / h ** 2
        res = (1 - d1 ** 2) + math.sqrt(t) * (d2 + (d - 1) / r * d1)
        assert abs(res) < 1e-5, (r, res)


def test_no_signal_reads_as_infinite_distance(oracle):
    w, gw = oracle.varadhan(2.0, 0.0, np.array([0.3, -0.1]))
    assert w == math.inf and np.all(gw == 0)
    assert oracle.varadhan(2.0, -1e-3) == math.inf
