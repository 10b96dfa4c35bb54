"""GPU Varadhan read-out (Sec. III, eq. transformation_varadhan) against the
oracle's formula, and end to end: estimate, then read out a distance."""
import math

import numpy as np
import pytest

from paper_2406_01713_amd import scenes as S
from tests.test_gpu_parity import dev, gpu_estimate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_01713_amd import binding
    return binding


@pytest.mark.parametrize("fp64", [False, True])
def test_readout_matches_oracle_formula(B, oracle, fp64):
    import torch
    dt = torch.float64 if fp64 else torch.float32
    rng = np.random.default_rng(0)
    n, d, sigma = 1000, 7, 2.5
    u = rng.uniform(1e-30, 1.0, n)
    u[::17] = 0.0
    u[5] = -0.5
    g = rng.normal(size=(n, 8))
    w, gw = B.wos_varadhan(dev(u, dt), sigma, grad_u=dev(g, dt))
    import torch as T
    T.cuda.synchronize()
    w, gw = w.cpu().numpy(), gw.cpu().numpy()
    rtol = 1e-13 if fp64 else 2e-6
    for q in range(n):
        uq = float(dev(u[q:q + 1], dt).cpu().numpy()[0])
        wq, gq = oracle.varadhan(sigma, uq, g[q].astype(np.float32 if not fp64 else np.float64).astype(np.float64))
        if math.isinf(wq):
            assert math.isinf(w[q]) and np.all(gw[q] == 0)
        else:
            assert w[q] == pytest.approx(wq, rel=rtol, abs=rtol)
            assert np.allclose(gw[q], gq, rtol=rtol * 10, atol=rtol * np.abs(gq).max())
    assert B.wos_varadhan(dev(np.zeros(0), dt), sigma).shape[0] == 0


def test_estimate_then_read_out_a_plane_distance(B):
    """Plane-wave data exp(k.x) on the 6-D scene: the read-out of the GPU
    estimate is the signed distance -k.x / |k| within 4 SE (delta method)."""
    base = S.scene_c2(n_queries=16, n_walks=16384, seed=3)
    k = S.plane_wave_k(6, base["sigma"], seed=1)
    s = S.with_bdata(base, 2, ak=k)
    u, g, st = gpu_estimate(B, s, fp64=True)
    w = B.wos_varadhan(dev(u, __import__("torch").float64), s["sigma"]).cpu().numpy()
    exact = -(s["queries"] @ k) / math.sqrt(s["sigma"])
    se_w = st[:, 0] / (u * math.sqrt(s["sigma"]))
    assert np.all(np.abs(w - exact) <= 4 * se_w + 1e-9), np.abs(w - exact) / se_w


def test_screening_sweep_approaches_the_distance(B, oracle):
    """Ball of radius 1 with unit data, query at |x| = 0.5 (d = 5): the GPU
    read-out matches the exact one, -ln(p(0.5)/p(1))/sqrt(sigma) with
    p(r) = 0F1(; 5/2; sigma r^2/4), within 4 SE, and as sigma grows (t -> 0)
    it approaches the distance to the sphere, 0.5."""
    errs = []
    for sigma in (1.0, 10.0, 100.0, 1000.0):
        s = S.scene_ball(5, R=1.0, sigma=sigma, queries=np.array([[0.5, 0, 0, 0, 0]]), n_walks=1 << 16, seed=1)
        u, g, st = gpu_estimate(B, s, fp64=True)
        w = float(B.wos_varadhan(dev(u, __import__("torch").float64), sigma).cpu().numpy()[0])
        exact = -math.log(oracle.hyp0f1(2.5, sigma / 16) / oracle.hyp0f1(2.5, sigma / 4)) / math.sqrt(sigma)
        se_w = st[0, 0] / (u[0] * math.sqrt(sigma))
        assert abs(w - exact) <= 4 * se_w + 1e-12, (sigma, w, exact, se_w)
        errs.append(abs(w - 0.5))
    assert errs[0] > errs[1] > errs[2] > errs[3], errs
