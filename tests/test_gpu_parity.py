"""GPU parity: the HIP path, called through the C ABI, against the FP64 CPU
oracle on identical Philox streams.  Bar: per query |u_gpu - u_cpu| <= 4 SE_cpu
+ 1e-7 (same for each gradient component); walk-level agreement where the
walks coincide; FP32 bias against the closed-form ball solution < 1e-3
relative; batched and plain paths agree up to summation order."""
import math
import os
import tempfile

import numpy as np
import pytest

from paper_2406_01713_amd import scenes as S
from tests.pins import closed_forms as CF
from tests.walkmatch import check_rate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_01713_amd import binding
    return binding


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def gpu_estimate(B, scene, fp64=False, queries=None, n_walks=None, seed=None, env_id=0,
                 max_steps=0, sigma=None, eps=None, full_scan=False, scalar_cull=False, wave_scan=False,
                 no_box_test=False, box_test=False):
    import torch
    dt = torch.float64 if fp64 else torch.float32
    dom = B.Domain(scene)
    q = dev(scene["queries"] if queries is None else queries, dt)
    Q, d = q.shape
    u = torch.empty(Q, dtype=dt, device="cuda")
    g = torch.empty(Q, d, dtype=dt, device="cuda")
    st = torch.empty(Q, d + 4, dtype=torch.float64, device="cuda")
    B.wos_estimate(dom, q, scene["n_walks"] if n_walks is None else n_walks,
                   scene["sigma"] if sigma is None else sigma, scene["eps"] if eps is None else eps,
                   scene["seed"] if seed is None else seed, u, g, st,
                   opt=B.options(fp64, env_id, max_steps, full_scan=full_scan, scalar_cull=scalar_cull,
                                 wave_scan=wave_scan, no_box_test=no_box_test, box_test=box_test))
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64), st.cpu().numpy()


def gpu_backward(B, scene, ubar, fp64=False, queries=None, n_walks=None, seed=None, env_id=0):
    import torch
    dt = torch.float64 if fp64 else torch.float32
    dom = B.Domain(scene)
    q = dev(scene["queries"] if queries is None else queries, dt)
    Q, d = q.shape
    dx = torch.empty(Q, d, dtype=dt, device="cuda")
    ds = torch.empty(1, dtype=torch.float64, device="cuda")
    dg = torch.empty(1, dtype=torch.float64, device="cuda")
    dq = torch.empty(Q, 2, dtype=torch.float64, device="cuda")
    B.wos_backward(dom, q, scene["n_walks"] if n_walks is None else n_walks, scene["sigma"],
                   scene["eps"], scene["seed"] if seed is None else seed, dev(ubar, dt), dx, ds, dg,
                   dq, opt=B.options(fp64, env_id))
    torch.cuda.synchronize()
    return dx.cpu().numpy().astype(np.float64), float(ds.item()), float(dg.item()), dq.cpu().numpy()


def assert_within_4se(u_gpu, g_gpu, u_cpu, g_cpu, st_cpu, d, extra=0.0, rel=0.0):
    """Per query and gradient component: |gpu - oracle| <= 4 SE_oracle + 1e-7
    + extra + rel |oracle| (rel covers FP32 rounding of large plane-wave
    values; for a gradient it scales with the larger of |u| and |grad u|)."""
    tol_u = 4 * st_cpu[:, 0] + 1e-7 + extra + rel * np.abs(u_cpu)
    bad = np.abs(u_gpu - u_cpu) > tol_u
    assert not bad.any(), (np.nonzero(bad)[0], u_gpu[bad], u_cpu[bad], tol_u[bad])
    scale = np.maximum(np.abs(u_cpu), np.abs(g_cpu).max(axis=1)) if len(u_cpu) else np.zeros(0)
    tol_g = 4 * st_cpu[:, 1:1 + d] + 1e-7 + extra + rel * scale[:, None]
    badg = np.abs(g_gpu - g_cpu) > tol_g
    assert not badg.any(), (np.argwhere(badg)[:5], g_gpu[badg][:5], g_cpu[badg][:5])


def assert_signal(u_cpu, g_cpu=None, min_frac=0.95, what=""):
    """A parity comparison must be made on non-zero values: at least min_frac
    of the oracle's query means (and gradient means) are non-zero."""
    fu = float(np.mean(u_cpu != 0)) if len(u_cpu) else 0.0
    assert fu >= min_frac, f"{what}: only {fu:.2f} of the oracle's u are non-zero"
    if g_cpu is not None:
        fg = float(np.mean(np.linalg.norm(np.atleast_2d(g_cpu), axis=1) > 0))
        assert fg >= min_frac, f"{what}: only {fg:.2f} of the oracle's grad u are non-zero"


def plane_wave(s, seed=4):
    """Plane-wave boundary data g = exp(k.y), |k|^2 = sigma, on the scene's
    geometry: u = exp(k.x) everywhere, so every walk carries signal."""
    return S.with_bdata(s, 2, ak=S.plane_wave_k(s["d"], s["sigma"], seed=seed))


def subset(name, nq, nw, seed=0, pw=False):
    """Reduced copies of the workloads: c1 (d = 2), c2 (d = 6), c3 (d = 7
    segments), c5 (d = 7, spheres and boxes), d4 / d8 (sphere-cluttered
    boxes of that dimension), and c3_near / d8_near (queries 0.02-0.1
    outside the goal sphere, so goal-indicator data has signal).  pw: with
    plane-wave data."""
    if name == "c1":
        s = S.scene_c1(n_walks=nw, seed=seed)
        s["queries"] = s["queries"][:nq]
    elif name == "c2":
        s = S.scene_c2(n_queries=nq, n_walks=nw, seed=seed)
    elif name == "c3":
        s = S.scene_c3(n_walks=nw, seed=seed)
        s["queries"] = s["queries"][::max(1, 1024 // nq)][:nq]
    elif name == "c5":
        s = S.scene_c5(n_starts=nq, n_walks=nw, seed=seed)
    elif name in ("d4", "d8"):
        s = S.scene_spheres(int(name[1]), n_queries=nq, n_walks=nw, seed=seed)
    elif name in ("c3_near", "d8_near"):
        s = S.scene_c3(n_walks=nw, seed=seed) if name == "c3_near" else \
            S.scene_spheres(8, n_queries=1, n_walks=nw, seed=seed)
        s["queries"] = S.near_goal_points(s, nq, seed=seed + 5)
    else:
        raise ValueError(name)
    return plane_wave(s) if pw else s


# --------------------------------------------------------------- walks ----

@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("name", ["c1", "c3", "c5", "d8", "c3_near"])
def test_walk_level_parity(B, oracle, name, fp64):
    """Same Philox counters -> same walks: step counts agree for almost every
    walk; where they agree the one-point estimates agree to rounding.  The
    data is plane-wave (or goal-indicator data next to the goal), so every
    compared value is non-zero.  FP32 positions drift from the FP64 walk's
    as rounding compounds over the steps (an 8-D walk of ~100 steps ends up
    to ~1e-3 away in relative terms): 95 % of the matched FP32 walks agree
    within 2e-4, every one within 2e-3."""
    s = subset(name, 2, 128, seed=11, pw=(name != "c3_near"))
    dom = B.Domain(s)
    odom = oracle.Domain(s)
    n = 128
    d = s["d"]
    tol, tol_all = (1e-9, 1e-9) if fp64 else (2e-4, 2e-3)
    for qi, x in enumerate(s["queries"]):
        rec = B.wos_debug_walks(dom, x, qi, 0, n, s["sigma"], s["eps"], s["seed"], B.options(fp64))
        same = nonzero = close = 0
        for w in range(n):
            r = oracle.walk(s, x, w, qi, dom=odom)
            gsteps = int(rec[w, d + 3])
            if gsteps != r["steps"]:
                continue
            same += 1
            nonzero += r["u"] != 0
            us = max(1.0, abs(r["u"]))
            gsc = max(1.0, np.abs(r["grad"]).max())
            err = max(abs(rec[w, 0] - r["u"]) / us, np.abs(rec[w, 1:1 + d] - r["grad"]).max() / (10 * gsc),
                      abs(rec[w, d + 2] - r["goal_w"]) / max(1.0, abs(r["goal_w"])),
                      abs(rec[w, d + 6] - r["du_dsigma"]) / (10 * max(1.0, abs(r["du_dsigma"]))))
            close += err <= tol
            assert err <= tol_all, (w, err, rec[w, 0], r["u"])
            assert int(rec[w, d + 4]) == r["status"]
            if r["status"] != 2:
                assert int(rec[w, d + 5]) == r["cls"]
        check_rate(f"{name} query {qi}", fp64, same, n)
        print(f"  {close} of them within {tol:g}, {nonzero} with a non-zero estimate")
        assert close >= 0.95 * same, (close, same)
        assert nonzero >= 0.1 * n, nonzero


# ------------------------------------------------------------- queries ----

def test_rr_config_fp64_full(B, oracle):
    """The d = 2 RR configuration at full size (64 grid queries x 1024 walks,
    FP64 plain kernel)."""
    s = S.scene_c1()
    u, g, st = gpu_estimate(B, s, fp64=True)
    uc, gc, stc = oracle.estimate(s)
    assert_within_4se(u, g, uc, gc, stc, 2)
    assert np.array_equal(st[:, 2 + 3], stc[:, 2 + 3])  # degenerate counts
    assert np.allclose(st[:, 0], stc[:, 0], rtol=0.05, atol=1e-9)


@pytest.mark.parametrize("name,nq,nw,pw,min_signal", [
    ("c1", 16, 2048, False, 0.8),      # goal data; 2 of the 16 grid points lie in obstacles
    ("c2", 24, 1024, True, 1.0), ("c3", 16, 1024, True, 1.0), ("c5", 6, 512, True, 1.0),
    ("d4", 16, 1024, True, 1.0), ("d8", 12, 1024, True, 1.0),
    ("c3_near", 12, 1024, False, 1.0), ("d8_near", 8, 1024, False, 1.0)])
def test_fp32_plain_vs_oracle(B, oracle, name, nq, nw, pw, min_signal):
    """FP32 plain kernel against the FP64 oracle on the same streams, every
    query and gradient component within 4 SE, on data with signal: plane-wave
    data (u = exp(k.x) > 0) on the 6-, 7- and 8-D sphere and box scenes, and
    goal-indicator data at 2-D grid points and next to the goal in 7 and 8
    dimensions."""
    s = subset(name, nq, nw, seed=3, pw=pw)
    u, g, st = gpu_estimate(B, s)
    uc, gc, stc = oracle.estimate(s)
    assert_signal(uc, gc, min_signal, name)
    assert_within_4se(u, g, uc, gc, stc, s["d"], rel=2e-5)
    assert np.allclose(st[:, s["d"] + 1], stc[:, s["d"] + 1], rtol=0.05)  # mean walk length


@pytest.mark.parametrize("name,pw", [("d8", True), ("d8_near", False), ("c2", True)])
def test_fp64_plain_vs_oracle(B, oracle, name, pw):
    """FP64 plain kernel against the FP64 oracle in 6 and 8 dimensions."""
    s = subset(name, 6, 512, seed=6, pw=pw)
    u, g, st = gpu_estimate(B, s, fp64=True)
    uc, gc, stc = oracle.estimate(s)
    assert_signal(uc, gc, 1.0, name)
    assert_within_4se(u, g, uc, gc, stc, s["d"], rel=1e-9)
    assert np.allclose(st[:, s["d"] + 1], stc[:, s["d"] + 1], rtol=0.02)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("name", ["c3", "c5"])
def test_fp32_affine_and_plane_wave_vs_oracle(B, oracle, name, mode):
    s = subset(name, 6, 1024, seed=5)
    d = s["d"]
    if mode == 1:
        s = S.with_bdata(s, 1, ak=np.linspace(-1, 1, d), b=0.3)
        s["sigma"] = 0.0
    else:
        s = S.with_bdata(s, 2, ak=S.plane_wave_k(d, s["sigma"], seed=4))
    u, g, st = gpu_estimate(B, s)
    uc, gc, stc = oracle.estimate(s)
    scale = np.maximum(1.0, np.abs(uc))
    assert_within_4se(u, g, uc, gc, stc, d, extra=2e-5 * scale[:, None].max())


@pytest.mark.parametrize("d", [2, 5, 7])
def test_fp32_bias_vs_ball_closed_form(B, d):
    """FP32 walks, 2^22 per point: |u - u_exact| < 1e-3 u_exact."""
    sigma = 2.0
    pts = np.zeros((2, d))
    pts[0, 0] = 0.5
    pts[1, d - 1] = -0.3
    pts[1, 0] = 0.2
    s = S.scene_ball(d, R=1.0, sigma=sigma, eps=1e-4, queries=pts, n_walks=1 << 22, seed=17)
    u, g, st = gpu_estimate(B, s)
    for q, x in enumerate(pts):
        ue = CF.ball_u(d, sigma, 1.0, x)
        print(f"d={d} point {q}: u {u[q]:.6f}, exact {ue:.6f}, relative bias {(u[q] - ue) / ue:+.2e}, "
              f"SE / u {st[q, 0] / ue:.1e}")
        assert abs(u[q] - ue) < 1e-3 * ue, (q, u[q], ue, st[q, 0])
        assert abs(u[q] - ue) <= 4 * st[q, 0] + 2e-4 * ue
        ge = CF.ball_grad(d, sigma, 1.0, x)
        assert np.all(np.abs(g[q] - ge) <= 4 * st[q, 1:1 + d] + 1e-3 * np.linalg.norm(ge))


def test_fp64_gpu_ball_centre_exact(B):
    from tests.test_oracle_rng_series import _C_bessel
    for d in (3, 7):
        s = S.scene_ball(d, R=1.3, sigma=3.0, n_walks=4096)
        u, g, st = gpu_estimate(B, s, fp64=True)
        assert u[0] == pytest.approx(_C_bessel(d, 3.0, 1.3), rel=1e-12)
        assert st[0, 0] < 1e-14 and st[0, d + 1] == 2.0


# ------------------------------------------------------------ backward ----

def _oracle_walk_stats(oracle, s, n_walks=None, env=0):
    """Per query: oracle means and standard errors of u_hat, d u_hat / d sigma
    and W 1{goal}, from its individual walks."""
    dom = oracle.Domain(s)
    n = s["n_walks"] if n_walks is None else n_walks
    out = []
    for q, x in enumerate(s["queries"]):
        rs = [oracle.walk(s, x, w, q, env=env, dom=dom) for w in range(n)]
        a = np.array([[r["u"], r["du_dsigma"], r["goal_w"]] for r in rs])
        out.append((a.mean(0), a.std(0, ddof=1) / math.sqrt(n)))
    return np.array([o[0] for o in out]), np.array([o[1] for o in out])


@pytest.mark.parametrize("fp64", [True, False])
def test_backward_vs_oracle(B, oracle, fp64):
    """wos_backward next to the goal in 7-D (goal-indicator data, about a
    quarter to three quarters of the walks reach the goal): per-query
    du/dsigma and du/dg_goal and the u-bar-weighted sums agree with the
    oracle within 4 SE of its walks; dx = u-bar grad u within 4 SE."""
    s = subset("c3_near", 6, 512, seed=8)
    rng = np.random.default_rng(0)
    ubar = rng.normal(size=6)
    dx, ds, dg, dq = gpu_backward(B, s, ubar, fp64=fp64)
    dxc, dsc, dgc = oracle.backward(s, ubar)
    _, gc, stc, dqc = oracle.estimate(s, dq=True)
    mean, se = _oracle_walk_stats(oracle, s)
    assert np.allclose(mean[:, 1:], dqc, rtol=1e-12, atol=1e-15)
    assert_signal(dqc[:, 0], None, 1.0, "du/dsigma")
    assert_signal(dqc[:, 1], gc, 1.0, "du/dg_goal")
    d = s["d"]
    rel = 1e-9 if fp64 else 2e-5
    tol_dx = 4 * np.abs(ubar)[:, None] * stc[:, 1:1 + d] + 1e-9 + rel * np.abs(dxc).max()
    assert np.all(np.abs(dx - dxc) <= tol_dx), np.abs(dx - dxc) / tol_dx
    tol = 4 * se[:, 1:] + 1e-9 + rel * np.abs(dqc)
    assert np.all(np.abs(dq - dqc) <= tol), (dq, dqc, se[:, 1:])
    se_ds = math.sqrt(float(np.sum((ubar * se[:, 1]) ** 2)))
    se_dg = math.sqrt(float(np.sum((ubar * se[:, 2]) ** 2)))
    print(f"d sigma: {ds:.6g} vs oracle {dsc:.6g} (SE {se_ds:.2g}); d g_goal: {dg:.6g} vs {dgc:.6g} "
          f"(SE {se_dg:.2g})")
    assert abs(ds - dsc) <= 4 * se_ds + 1e-9 + rel * abs(dsc)
    assert abs(dg - dgc) <= 4 * se_dg + 1e-9 + rel * abs(dgc)


def test_backward_matches_crn_finite_differences_fp64(B):
    """Next to the goal in 7-D: du/dsigma equals central differences in sigma
    on the same walks (the walk law does not depend on sigma), and
    du/dg_goal equals the exact difference quotient (u is linear in g)."""
    s = subset("c3_near", 4, 1024, seed=9)
    ubar = np.ones(4)
    _, _, _, dq = gpu_backward(B, s, ubar, fp64=True)
    assert_signal(dq[:, 0], None, 1.0, "du/dsigma")
    assert_signal(dq[:, 1], None, 1.0, "du/dg_goal")
    h = 1e-4
    up = gpu_estimate(B, s, fp64=True, sigma=s["sigma"] + h)[0]
    um = gpu_estimate(B, s, fp64=True, sigma=s["sigma"] - h)[0]
    assert np.allclose(dq[:, 0], (up - um) / (2 * h), rtol=1e-5, atol=1e-10)
    s1 = dict(s, bdata=dict(s["bdata"], g_goal=3.0))
    u1 = gpu_estimate(B, s1, fp64=True)[0]
    u0 = gpu_estimate(B, s, fp64=True)[0]
    assert np.allclose(dq[:, 1], (u1 - u0) / 2.0, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("case", ["plane_wave", "goal_near"])
def test_dx_matches_crn_finite_differences(B, case):
    """d u / d x from the first-sphere estimator (the backward's dx) against
    central differences of the u estimator in x on common random numbers:
    per walk (u_hat(x + h e_i) - u_hat(x - h e_i)) / 2h with the walk's own
    Philox stream, 2^18 walks per point (FP64 walks), 7-D segment geometry.
    Both are unbiased for grad u (the difference up to O(h^2)); the bar is 4
    standard errors of the paired difference of the two per-walk
    estimators."""
    if case == "plane_wave":
        # the segment query where u = exp(k.x) is largest, and the coordinates
        # with the largest |k_i|: grad u = k u stands well above its SE
        s = subset("c3", 1024, 1024, seed=4, pw=True)
        k = s["bdata"]["ak"]
        x = s["queries"][int(np.argmax(s["queries"] @ k))]
        coords = [int(i) for i in np.argsort(-np.abs(k))[:3]]
    else:
        s = subset("c3_near", 1, 1024, seed=4)
        x = s["queries"][0]
        coords = [0, 3, 6]
    d, n, h = s["d"], 1 << 18, 1e-2
    dom = B.Domain(s)
    opt = B.options(True)

    def walks(p):
        return B.wos_debug_walks(dom, p, 0, 0, n, s["sigma"], s["eps"], s["seed"], opt)

    r0 = walks(x)
    strong = 0
    for i in coords:
        e = np.zeros(d)
        e[i] = h
        fd = (walks(x + e)[:, 0] - walks(x - e)[:, 0]) / (2 * h)
        gi = r0[:, 1 + i]
        diff = gi - fd
        se = diff.std(ddof=1) / math.sqrt(n)
        print(f"{case} coordinate {i}: first-sphere {gi.mean():.5g} (SE {gi.std(ddof=1) / math.sqrt(n):.2g}), "
              f"CRN difference {fd.mean():.5g} (SE {fd.std(ddof=1) / math.sqrt(n):.2g}), paired SE {se:.2g}")
        assert abs(diff.mean()) <= 4 * se, (i, gi.mean(), fd.mean(), se)
        strong += abs(gi.mean()) > 8 * se
    assert strong >= 1  # the test has power: some component is far from 0


def test_backward_vs_ball_closed_form(B):
    d, sigma = 5, 2.0
    x = np.zeros((1, d))
    x[0, 1] = 0.4
    s = S.scene_ball(d, R=1.0, sigma=sigma, eps=1e-4, queries=x, n_walks=1 << 20, seed=2)
    dx, ds, dg, dq = gpu_backward(B, s, np.ones(1))
    want = CF.ball_du_dsigma(d, sigma, 1.0, x[0])
    assert dq[0, 0] == pytest.approx(want, rel=1e-2)
    _, _, st = gpu_estimate(B, s)  # same walks: their gradient standard errors
    ge = CF.ball_grad(d, sigma, 1.0, x[0])
    assert np.all(np.abs(dx[0] - ge) <= 4 * st[0, 1:1 + d] + 1e-4), (dx[0], ge, st[0, 1:1 + d])


def test_autograd_function(B):
    import torch
    from paper_2406_01713_amd.autograd import WoSFunction
    s = subset("c3_near", 8, 512, seed=1)
    x = dev(s["queries"], torch.float64).requires_grad_(True)
    sig = torch.tensor(s["sigma"], dtype=torch.float64, requires_grad=True)
    gg = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    u, g = WoSFunction.apply(x, sig, gg, s, s["n_walks"], s["eps"], s["seed"])
    w = torch.linspace(-1, 1, 8, dtype=torch.float64, device="cuda")
    (u * w).sum().backward()
    dx, ds, dgv, dq = gpu_backward(B, s, w.cpu().numpy(), fp64=True)
    assert_signal(u.detach().cpu().numpy(), dx, 1.0, "u")
    assert_signal(dq[:, 0], None, 1.0, "du/dsigma")
    assert_signal(dq[:, 1], None, 1.0, "du/dg_goal")
    assert np.allclose(x.grad.cpu().numpy(), dx, rtol=1e-12, atol=1e-15)
    assert sig.grad.item() == pytest.approx(ds, rel=1e-12)
    assert gg.grad.item() == pytest.approx(dgv, rel=1e-12)
    assert np.allclose(g.detach().cpu().numpy(), gpu_estimate(B, s, fp64=True)[1], rtol=1e-12)


# --------------------------------------------------------------- batch ----

def _ragged(n_envs=10, q_cap=24, n_walks=512):
    envs = [S.scene_c4_env(e, n_walks=n_walks, seed=7, q_cap=q_cap) for e in range(n_envs)]
    return envs


def gpu_batch(B, envs, n_walks, seed, ubar=None, torch_dtype=None, full_scan=False, scalar_cull=False,
              wave_scan=False, no_box_test=False, box_test=False):
    import torch
    doms = [B.Domain(e) for e in envs]
    Qs = [len(e["queries"]) for e in envs]
    off = np.concatenate([[0], np.cumsum(Qs)]).astype(np.int64)
    qp = np.zeros((off[-1], 8), dtype=np.float32)
    for e, s in enumerate(envs):
        qp[off[e]:off[e + 1], :s["d"]] = s["queries"]
    q = dev(qp, torch.float32)
    n = int(off[-1])
    u = torch.empty(n, device="cuda")
    g = torch.empty(n, 8, device="cuda")
    st = torch.empty(n, B.BATCH_STATS, dtype=torch.float64, device="cuda")
    kw = {}
    if ubar is not None:
        kw = dict(grad_u=dev(ubar, torch.float32), out_dx=torch.empty(n, 8, device="cuda"),
                  out_dsigma=torch.empty(len(envs), dtype=torch.float64, device="cuda"),
                  out_dg=torch.empty(len(envs), dtype=torch.float64, device="cuda"))
    B.wos_estimate_batch(doms, q, off, [e["sigma"] for e in envs], [e["eps"] for e in envs], n_walks,
                         seed, u, g, st, opt=B.options(full_scan=full_scan, scalar_cull=scalar_cull,
                                                       wave_scan=wave_scan, no_box_test=no_box_test,
                                                       box_test=box_test), **kw)
    torch.cuda.synchronize()
    out = {"u": u.cpu().numpy(), "g": g.cpu().numpy(), "st": st.cpu().numpy(), "off": off}
    if ubar is not None:
        out.update(dx=kw["out_dx"].cpu().numpy(), ds=kw["out_dsigma"].cpu().numpy(),
                   dg=kw["out_dg"].cpu().numpy())
    return out


def test_batch_matches_plain_per_env(B):
    """One persistent fused launch over a ragged batch (d in 2..7, uneven M and
    Q) reproduces per-env plain forward and backward calls with env_id = e."""
    envs = _ragged()
    n_walks, seed = 512, 7
    rng = np.random.default_rng(3)
    Qt = sum(len(e["queries"]) for e in envs)
    ubar = rng.normal(size=Qt).astype(np.float32)
    out = gpu_batch(B, envs, n_walks, seed, ubar=ubar)
    off = out["off"]
    for e, s in enumerate(envs):
        d = s["d"]
        sl = slice(off[e], off[e + 1])
        u, g, st = gpu_estimate(B, s, n_walks=n_walks, seed=seed, env_id=e)
        assert np.allclose(out["u"][sl], u, rtol=2e-5, atol=1e-7), e
        assert np.allclose(out["g"][sl, :d], g, rtol=2e-5, atol=1e-6), e
        assert np.all(out["g"][sl, d:] == 0)
        assert np.allclose(out["st"][sl, 9], st[:, d + 1], rtol=1e-12)  # mean steps: identical walks
        assert np.array_equal(out["st"][sl, 11], st[:, d + 3])
        dx, ds, dg, dq = gpu_backward(B, s, ubar[sl], n_walks=n_walks, seed=seed, env_id=e)
        assert np.allclose(out["dx"][sl, :d], dx, rtol=2e-5, atol=1e-6), e
        assert out["ds"][e] == pytest.approx(ds, rel=1e-4, abs=1e-8)
        assert out["dg"][e] == pytest.approx(dg, rel=1e-4, abs=1e-8)


def _cull_scenes():
    big = S.scene_c4_env(5, n_walks=256, seed=2, q_cap=6)
    return [subset("c3", 8, 256, seed=2), subset("c5", 6, 256, seed=2), big, subset("d8", 6, 256, seed=2)]


@pytest.mark.parametrize("fp64", [False, True])
def test_culling_changes_no_result_plain(B, fp64):
    """Cluster culling skips only obstacles that cannot be nearest: every
    walk, hence every output, is bitwise the one a scan of every obstacle
    gives (spheres and boxes, FP32 and FP64)."""
    for s in _cull_scenes():
        assert len(s["sph_r"]) >= 64
        a = gpu_estimate(B, s, fp64=fp64)
        b = gpu_estimate(B, s, fp64=fp64, full_scan=True)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), s["name"]
        dom = B.Domain(s)
        for q in range(2):
            ra = B.wos_debug_walks(dom, s["queries"][q], q, 0, 256, s["sigma"], s["eps"], s["seed"],
                                   opt=B.options(fp64))
            rb = B.wos_debug_walks(dom, s["queries"][q], q, 0, 256, s["sigma"], s["eps"], s["seed"],
                                   opt=B.options(fp64, full_scan=True))
            assert np.array_equal(ra, rb), (s["name"], q)


def test_culling_changes_no_result_batch(B):
    """Same in the persistent kernel, and the work columns of the stats
    count what the scans did: a full scan evaluates M obstacles per step, a
    culled one at most that plus one bound per cluster, and at most one
    bounding-box test per cluster and step (made only for pairs the cluster
    bound keeps)."""
    envs = _ragged(n_envs=12, q_cap=16, n_walks=256)
    rng = np.random.default_rng(9)
    ubar = rng.normal(size=sum(len(e["queries"]) for e in envs)).astype(np.float32)
    a = gpu_batch(B, envs, 256, 5, ubar=ubar)
    b = gpu_batch(B, envs, 256, 5, ubar=ubar, full_scan=True)
    for k in ("u", "g", "dx", "ds", "dg"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["st"][:, :12], b["st"][:, :12])
    saved = done = full = 0.0
    for e, s in enumerate(envs):
        sl = slice(a["off"][e], a["off"][e + 1])
        M = len(s["sph_r"])
        steps = b["st"][sl, 9]
        assert np.allclose(b["st"][sl, 12], steps * M, rtol=1e-12)
        assert np.all(b["st"][sl, 13] == 0) and np.all(b["st"][sl, 14] == 0) and np.all(b["st"][sl, 15] == 0)
        if M < 64:
            assert np.array_equal(a["st"][sl, 12:], b["st"][sl, 12:]), e
        else:
            assert np.allclose(a["st"][sl, 14], steps * -(-M // 8), rtol=1e-12)
            assert np.all(a["st"][sl, 12] <= (-(-M // 8) * 8) * steps * (1 + 1e-12))
            assert np.all(a["st"][sl, 15] <= -(-M // 8) * steps * (1 + 1e-12))
            # the box test runs by default where the obstacles depend on 6 or
            # more coordinates
            if s["d"] < 6:
                assert np.all(a["st"][sl, 15] == 0), e
            elif M >= 128:
                assert np.any(a["st"][sl, 15] > 0), e
            saved += (b["st"][sl, 12] - a["st"][sl, 12]).sum()
            done += (a["st"][sl, 12] + a["st"][sl, 14]).sum()
            full += b["st"][sl, 12].sum()
    assert saved > 0
    print(f"work fraction of the clustered envs: {done / full:.3f}")


def test_matrix_core_cull_matches_vector_cull(B):
    """The FP32 cluster test on the matrix cores (members scanned pair by
    pair, with the bounding-box test in every dimension, by dimension or
    never, or by every lane of the wave) and on the vector ALUs skip
    different (always non-minimal) clusters; walks and outputs are
    identical, and the more pairs the box test sees the fewer member
    distances are evaluated."""
    for s in _cull_scenes():
        a = gpu_estimate(B, s)
        b = gpu_estimate(B, s, scalar_cull=True)
        c = gpu_estimate(B, s, wave_scan=True)
        n = gpu_estimate(B, s, no_box_test=True)
        f = gpu_estimate(B, s, box_test=True)
        for x, y, z, w, v in zip(a, b, c, n, f):
            assert np.array_equal(x, y), s["name"]
            assert np.array_equal(x, z), s["name"]
            assert np.array_equal(x, w), s["name"]
            assert np.array_equal(x, v), s["name"]
        dom = B.Domain(s)
        for q in range(2):
            ra = B.wos_debug_walks(dom, s["queries"][q], q, 0, 128, s["sigma"], s["eps"], s["seed"],
                                   opt=B.options())
            rb = B.wos_debug_walks(dom, s["queries"][q], q, 0, 128, s["sigma"], s["eps"], s["seed"],
                                   opt=B.options(full_scan=True))
            assert np.array_equal(ra, rb), (s["name"], q)
    envs = _ragged(n_envs=12, q_cap=16, n_walks=256)
    rng = np.random.default_rng(10)
    ubar = rng.normal(size=sum(len(e["queries"]) for e in envs)).astype(np.float32)
    a = gpu_batch(B, envs, 256, 5, ubar=ubar)
    b = gpu_batch(B, envs, 256, 5, ubar=ubar, scalar_cull=True)
    c = gpu_batch(B, envs, 256, 5, ubar=ubar, wave_scan=True)
    n = gpu_batch(B, envs, 256, 5, ubar=ubar, no_box_test=True)
    f = gpu_batch(B, envs, 256, 5, ubar=ubar, box_test=True)
    for k in ("u", "g", "dx", "ds", "dg"):
        for o in (b, c, n, f):
            assert np.array_equal(a[k], o[k]), k
    for o in (b, c, n, f):
        assert np.array_equal(a["st"][:, :12], o["st"][:, :12])
    ma, mb, mc, mn, mf = (o["st"][:, 12].sum() for o in (a, b, c, n, f))
    print(f"member distances per walk, pairs with the box test everywhere / by dimension / never, wave scan, "
          f"vector cull: {mf:.4g} / {ma:.4g} / {mn:.4g} / {mc:.4g} / {mb:.4g}")
    assert mf <= ma <= mn <= mc and mn <= mb
    assert np.all(n["st"][:, 15] == 0) and f["st"][:, 15].sum() >= a["st"][:, 15].sum() > 0


def _dense_cloud(seed=21, boxes=False):
    """d = 3: 1024 spheres (r 0.01-0.02) or boxes (half-widths 0.01-0.02)
    packed in [-0.5, 0.5]^3 plus 512 sparse ones (0.05-0.1) in the rest of
    the box [-3, 3]^3, no goal; g = 1 on obstacles.  Queries inside the cloud
    see every cloud cluster within the outer-box distance, so all 64 walkers
    of a wave need every cluster of a cloud tile: 1024 pairs per tile, more
    than the queue takes at once."""
    rng = np.random.default_rng(seed)
    d = 3
    dense = rng.uniform(-0.5, 0.5, size=(1024, d))
    sparse = []
    while len(sparse) < 512:
        p = rng.uniform(-2.8, 2.8, size=d)
        if np.abs(p).max() > 0.8:
            sparse.append(p)
    c = np.concatenate([dense, np.array(sparse)])
    r = np.concatenate([rng.uniform(0.01, 0.02, 1024), rng.uniform(0.05, 0.1, 512)])
    s = S._empty(d)
    if boxes:
        s.update(box_c=c, box_h=np.repeat(r[:, None], d, axis=1) * rng.uniform(0.6, 1.0, size=(len(r), d)))
    else:
        s.update(sph_c=c, sph_r=r)
    s.update(d=d, goal_c=None, goal_r=None, outer=S.box_outer(d, 3.0),
             bdata=S._bdata(0, d, g_goal=0.0, g_obs=1.0, g_outer=0.0), sigma=1.0, eps=1e-3,
             n_walks=128, seed=seed, name="dense_box_cloud" if boxes else "dense_cloud")
    qs = []
    while len(qs) < 4:
        p = rng.uniform(-0.4, 0.4, size=d)
        if S.is_clear(p, s, 0.005):
            qs.append(p)
    qs += [np.array([1.5, -1.2, 2.0]), np.array([-2.0, 1.0, -1.5])]
    s["queries"] = np.array(qs)
    return s


@pytest.mark.parametrize("boxes", [False, True])
def test_pair_queue_overflow_is_exact(B, boxes):
    """A tile whose (walker, cluster) pairs overflow the per-wave queue is
    queued two need bits at a time after the waiting pairs are tested: walks
    and outputs stay bitwise those of the wave-uniform, vector-ALU and full
    scans, and of the pair scan with the bounding-box test forced on or off,
    in the plain, debug-walk and batched launches (sphere and box
    obstacles)."""
    s = _dense_cloud(boxes=boxes)
    # precondition: at step 0 the 64 walkers of query 0 need more than
    # 256 - 63 pairs in some tile (they all sit at the query point)
    if boxes:
        cl = B.wos_debug_clusters(3, box_c=s["box_c"], box_h=s["box_h"])["box"][1]
    else:
        cl = B.wos_debug_clusters(3, s["sph_c"], s["sph_r"])["sph"][1]
    x0 = s["queries"][0]
    thr = np.min(np.minimum(x0 - s["outer"]["lo"], s["outer"]["hi"] - x0))
    need = np.linalg.norm(cl[:, :3] - x0, axis=1) - cl[:, 3] <= thr
    per_tile = [need[t:t + 16].sum() for t in range(0, len(need), 16)]
    assert 64 * max(per_tile) > 256 - 63, per_tile
    a = gpu_estimate(B, s)
    for kw in (dict(full_scan=True), dict(wave_scan=True), dict(scalar_cull=True), dict(no_box_test=True),
               dict(box_test=True)):
        b = gpu_estimate(B, s, **kw)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), kw
    dom = B.Domain(s)
    for q in (0, 1, 4):
        ra = B.wos_debug_walks(dom, s["queries"][q], q, 0, 128, s["sigma"], s["eps"], s["seed"],
                               opt=B.options())
        rb = B.wos_debug_walks(dom, s["queries"][q], q, 0, 128, s["sigma"], s["eps"], s["seed"],
                               opt=B.options(full_scan=True))
        assert np.array_equal(ra, rb), q
    envs = [s, S.scene_c4_env(3, n_walks=128, seed=4, q_cap=6)]
    rng = np.random.default_rng(12)
    ubar = rng.normal(size=sum(len(e["queries"]) for e in envs)).astype(np.float32)
    a = gpu_batch(B, envs, 128, 5, ubar=ubar)
    b = gpu_batch(B, envs, 128, 5, ubar=ubar, full_scan=True)
    for k in ("u", "g", "dx", "ds", "dg"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["st"][:, :12], b["st"][:, :12])
    assert np.all(a["u"][:4] > 0)  # the cloud absorbs walks


def _env_per_d(n_walks, seed, q_cap, dims=range(2, 8)):
    """The first environment of the ragged batch of each dimension."""
    out = []
    for d in dims:
        e = 0
        while True:
            s = S.scene_c4_env(e, n_walks=n_walks, seed=seed, q_cap=q_cap, dims={d})
            if s is not None:
                out.append(s)
                break
            e += 1
    return out


def test_batch_vs_oracle(B, oracle):
    """A mixed-dimension batch in one persistent launch (one env of each d in
    2..7 from the ragged batch plus an 8-D sphere scene), plane-wave data so
    every query has signal, against the oracle with env_id = the batch
    position: every query and gradient component within 4 SE."""
    envs = _env_per_d(256, 7, 4) + [S.scene_spheres(8, n_queries=4, n_walks=256, seed=7)]
    envs = [plane_wave(e, seed=i) for i, e in enumerate(envs)]
    assert sorted(e["d"] for e in envs) == list(range(2, 9))
    out = gpu_batch(B, envs, 256, 7)
    for e, s in enumerate(envs):
        sl = slice(out["off"][e], out["off"][e + 1])
        uc, gc, stc = oracle.estimate(s, n_walks=256, seed=7, env=e)
        assert_signal(uc, gc, 1.0, s["name"])
        assert_within_4se(out["u"][sl].astype(np.float64), out["g"][sl, :s["d"]].astype(np.float64),
                          uc, gc, stc, s["d"], rel=2e-5)
        assert np.all(out["g"][sl, s["d"]:] == 0)
        assert np.allclose(out["st"][sl, 9], stc[:, s["d"] + 1], rtol=0.05)  # mean walk length


def test_batch_is_deterministic(B):
    envs = _ragged(n_envs=5, q_cap=16, n_walks=256)
    a = gpu_batch(B, envs, 256, 3, ubar=np.ones(sum(len(e["queries"]) for e in envs), np.float32))
    b = gpu_batch(B, envs, 256, 3, ubar=np.ones(sum(len(e["queries"]) for e in envs), np.float32))
    for k in ("u", "g", "st", "dx", "ds", "dg"):
        assert np.array_equal(a[k], b[k]), k


def test_autotune_writes_cache_and_batch_uses_it(B):
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "tune.json")
        B.wos_autotune(7, 64, 32, 256, path)
        txt = open(path).read()
        assert "units_per_wave" in txt and "walks_per_lane" in txt and "waves_per_block" in txt and "d7_" in txt
        B.wos_set_autotune_cache(path)
        envs = _ragged(n_envs=3, q_cap=8, n_walks=256)
        a = gpu_batch(B, envs, 256, 5)
        B.wos_set_autotune_cache(None)
        b = gpu_batch(B, envs, 256, 5)
        assert np.allclose(a["u"], b["u"], rtol=2e-5, atol=1e-7)


def _batch_args(B, envs):
    import torch
    Qs = [len(e["queries"]) for e in envs]
    off = np.concatenate([[0], np.cumsum(Qs)]).astype(np.int64)
    qp = np.zeros((off[-1], 8), dtype=np.float32)
    for e, s in enumerate(envs):
        qp[off[e]:off[e + 1], :s["d"]] = s["queries"]
    return [B.Domain(e) for e in envs], dev(qp, torch.float32), off


def test_autotune_batch_and_every_block_shape(B):
    """The batch tuner times launch shapes on the caller's own batch and
    records the best under the batch's mix key; every block shape (1, 2 and 4
    waves per block), with other unit and walk-range splits and 1, 2, 4 or 64
    lanes per walker, gives the same walks as the built-in shape (identical step and degenerate counts, means
    equal up to summation order)."""
    import json
    envs = _ragged(n_envs=6, q_cap=24, n_walks=512)
    rng = np.random.default_rng(4)
    ubar = rng.normal(size=sum(len(e["queries"]) for e in envs)).astype(np.float32)
    B.wos_set_autotune_cache(None)
    ref = gpu_batch(B, envs, 512, 5, ubar=ubar)
    doms, q, off = _batch_args(B, envs)
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "tune.json")
        r = B.wos_autotune_batch(doms, q, off, [e["sigma"] for e in envs], [e["eps"] for e in envs], 512, 5,
                                 fused=True, cache_path=path)
        print("tuned shape:", r)
        assert r["waves_per_block"] in (1, 2, 4) and r["units_per_wave"] in (1, 2, 4, 8, 16)
        assert r["grid_mult"] in (1, 2) and r["walks_per_lane"] in (1, 2, 4) and r["lanes_per_walker"] in (1, 2, 4, 8, 16, 32, 64)
        assert 0 < r["ms_best"] <= r["ms_default"] and r["tried"] >= 11
        cache = json.load(open(path))
        keys = [k for k in cache if k.startswith("mix_6_")]
        assert len(keys) == 1
        key = keys[0]
        order = ("units_per_wave", "grid_mult", "walks_per_lane", "waves_per_block",
                 "lanes_per_walker")  # the file's key order
        for shape in ({"waves_per_block": 1, "units_per_wave": 2, "grid_mult": 1, "walks_per_lane": 1,
                       "lanes_per_walker": 2},
                      {"waves_per_block": 2, "units_per_wave": 8, "grid_mult": 2, "walks_per_lane": 4,
                       "lanes_per_walker": 1},
                      {"waves_per_block": 4, "units_per_wave": 1, "grid_mult": 2, "walks_per_lane": 2,
                       "lanes_per_walker": 4},
                      {"waves_per_block": 4, "units_per_wave": 4, "grid_mult": 1, "walks_per_lane": 1,
                       "lanes_per_walker": 64},
                      cache[key]):
            with open(path, "w") as f:
                f.write("{\n  \"%s\": %s\n}\n" % (key, json.dumps({k: shape[k] for k in order})))
            B.wos_set_autotune_cache(path)
            out = gpu_batch(B, envs, 512, 5, ubar=ubar)
            for k in ("u", "g", "dx"):
                assert np.allclose(out[k], ref[k], rtol=1e-5, atol=1e-7), (shape, k)
            assert np.allclose(out["ds"], ref["ds"], rtol=1e-5, atol=1e-9) and np.allclose(out["dg"], ref["dg"],
                                                                                            rtol=1e-5, atol=1e-9)
            assert np.array_equal(out["st"][:, 9], ref["st"][:, 9]), shape   # same walks: same step counts
            assert np.array_equal(out["st"][:, 10:12], ref["st"][:, 10:12]), shape
    B.wos_set_autotune_cache(None)


# ------------------------------------------------------------ planning ----

@pytest.mark.parametrize("n_walks", [512, 2048])
def test_plan_graph_matches_oracle_steps(B, oracle, n_walks):
    """Three captured planning steps on the full C5 scene (512 spheres + 512
    boxes) from four starts near the goal follow the oracle's steps; 2048
    walks per gradient is the benchmark's planning configuration."""
    import torch
    s = S.scene_c5(n_starts=3, n_walks=n_walks)
    rng = np.random.default_rng(3)
    starts = []
    while len(starts) < 4:
        v = rng.normal(size=7)
        p = s["goal_c"] + (s["goal_r"] + 0.1) * v / np.linalg.norm(v)
        if S.is_clear(p, s, 0.05):
            starts.append(p)
    x0 = np.array(starts)
    x = dev(x0, torch.float32)
    dom = B.Domain(s)
    plan = B.Plan(dom, x, n_walks, s["sigma"], s["eps"], s["s_ub"], s["seed"])
    xo = np.ascontiguousarray(x0.astype(np.float32).astype(np.float64))
    path = np.zeros(4)
    stalls = np.zeros(4, dtype=np.int32)
    status = np.zeros(4, dtype=np.int32)
    for t in range(3):
        plan.step(1)
        u, g, pl, stl, sts, step = plan.read()
        oracle.plan_step(s, xo, t, path, stalls, status)
        xg = x.cpu().numpy().astype(np.float64)
        assert step[0] == t + 1
        assert np.array_equal(stl, stalls) and np.array_equal(sts, status)
        assert np.allclose(xg, xo, atol=2e-4), (t, np.abs(xg - xo).max())
        assert np.allclose(pl, path, rtol=1e-4, atol=1e-6)
    del plan


# ---------------------------------------------------------- edge cases ----

def test_edge_cases(B, oracle):
    import torch
    s = subset("c1", 4, 100, seed=2)  # 100 walks: a ragged 64-walk chunk
    u, g, st = gpu_estimate(B, s, fp64=True)
    uc, gc, stc = oracle.estimate(s)
    assert_within_4se(u, g, uc, gc, stc, 2)
    # one walk per query: SE = 0 and the value is that walk's
    u1, _, st1 = gpu_estimate(B, s, fp64=True, n_walks=1)
    assert np.all(st1[:, 0] == 0)
    for q, x in enumerate(s["queries"]):
        assert u1[q] == pytest.approx(oracle.walk(s, x, 0, q)["u"], rel=1e-9, abs=1e-12)
    # degenerate queries: inside an obstacle, inside the goal, outside the box
    c = S.scene_c1(n_walks=64)
    qs = np.array([c["sph_c"][0], c["goal_c"], [4.0, 0.0]])
    u, g, st = gpu_estimate(B, c, fp64=True, queries=qs)
    assert u[0] == 0.0 and u[1] == 1.0 and u[2] == 0.0 and np.all(g == 0)
    assert np.all(st[:, 2 + 3] == 64) and np.all(st[:, 2 + 1] == 1.0)
    # truncation with a tiny step cap matches the oracle's count
    u, g, st = gpu_estimate(B, s, fp64=True, max_steps=3)
    uc, gc, stc = oracle.estimate(s, max_steps=3)
    assert np.array_equal(st[:, 2 + 2], stc[:, 2 + 2])
    # no queries: nothing launched, no error
    dom = B.Domain(s)
    q0 = torch.empty(0, 2, device="cuda")
    B.wos_estimate(dom, q0, 64, 1.0, 1e-3, 0, torch.empty(0, device="cuda"))
    # invalid arguments come back as errors
    with pytest.raises(B.WosError):
        B.wos_estimate(dom, dev(s["queries"], torch.float32), 0, 1.0, 1e-3, 0,
                       torch.empty(4, device="cuda"))
    with pytest.raises(B.WosError):
        B.wos_estimate(dom, dev(s["queries"], torch.float32), 64, -1.0, 1e-3, 0,
                       torch.empty(4, device="cuda"))
    with pytest.raises(B.WosError):
        B.wos_estimate(dom, dev(s["queries"], torch.float32), 64, 1.0, 0.0, 0,
                       torch.empty(4, device="cuda"))
    aff = B.Domain(S.with_bdata(s, 1, ak=[1.0, 0.0]))
    with pytest.raises(B.WosError):
        B.wos_estimate(aff, dev(s["queries"], torch.float32), 64, 1.0, 1e-3, 0,
                       torch.empty(4, device="cuda"))


def test_batch_rejects_counts_beyond_its_indices(B):
    """Query and work-unit counts past what the kernels index (32-bit query
    counters, a 32-bit unit counter) come back as errors before any device
    work: an env with 2^31 queries, and three envs of 2^31 - 1 queries (about
    6.4e9 work units)."""
    import torch
    s = subset("c3", 4, 64, seed=1)
    dom = B.Domain(s)
    q = torch.zeros(4, 8, device="cuda")
    u = torch.empty(4, device="cuda")
    with pytest.raises(B.WosError, match="queries"):
        B.wos_estimate_batch([dom], q, [0, 2 ** 31], [2.0], [1e-4], 64, 0, u)
    n = 2 ** 31 - 1
    with pytest.raises(B.WosError, match="work units"):
        B.wos_estimate_batch([dom] * 3, q, [0, n, 2 * n, 3 * n], [2.0] * 3, [1e-4] * 3, 64, 0, u)
    B.wos_estimate_batch([dom], q, [0, 4], [2.0], [1e-4], 64, 0, u)  # the library still works
    torch.cuda.synchronize()


# -------------------------------------------- full-size sampled parity ----

@pytest.mark.parametrize("fused", [False, True])
def test_d6_forward_full_size_sampled(B, oracle, fused):
    """4096 queries x 4096 walks (d = 6), plane-wave data on its geometry:
    the full launch, checked on sampled queries that the oracle recomputes
    walk by walk on the same streams."""
    s = plane_wave(S.scene_c2())
    if fused:
        out = gpu_batch(B, [s], s["n_walks"], s["seed"])
        u, g = out["u"].astype(np.float64), out["g"][:, :6].astype(np.float64)
        env = 0
    else:
        u, g, _ = gpu_estimate(B, s)
        env = 0
    idx = [0, 1777, 4095]
    for q in idx:
        # the oracle keys walks by the query's index: evaluate row q alone
        dom = oracle.Domain(s)
        vals = [oracle.walk(s, s["queries"][q], w, q, env=env, dom=dom) for w in range(s["n_walks"])]
        uw = np.array([v["u"] for v in vals])
        gw = np.array([v["grad"] for v in vals])
        se_u = uw.std(ddof=1) / math.sqrt(len(uw))
        se_g = gw.std(axis=0, ddof=1) / math.sqrt(len(uw))
        assert np.mean(uw != 0) >= 0.95  # signal
        print(f"C2 query {q}: |u - u_oracle| / SE = {abs(u[q] - uw.mean()) / se_u:.3f}, "
              f"max |grad - grad_oracle| / SE = {np.max(np.abs(g[q] - gw.mean(0)) / se_g):.3f}")
        assert abs(u[q] - uw.mean()) <= 4 * se_u + 1e-7 + 2e-5 * abs(uw.mean())
        assert np.all(np.abs(g[q] - gw.mean(0)) <= 4 * se_g + 1e-7 + 2e-5 * np.abs(gw.mean(0)).max())


def _fused_full_launch(B, envs):
    """One fused forward + backward persistent launch over envs (u-bar = 1),
    env e with env_id = e.  Returns host copies of u, grad, stats, dx and
    the row offsets."""
    import torch
    seed = envs[0]["seed"]
    Qs = [len(e["queries"]) for e in envs]
    off = np.concatenate([[0], np.cumsum(Qs)]).astype(np.int64)
    n = int(off[-1])
    qp = np.zeros((n, 8), dtype=np.float32)
    for e, s in enumerate(envs):
        qp[off[e]:off[e + 1], :s["d"]] = s["queries"]
    q = dev(qp, torch.float32)
    u = torch.empty(n, device="cuda")
    g = torch.empty(n, 8, device="cuda")
    st = torch.empty(n, B.BATCH_STATS, dtype=torch.float64, device="cuda")
    ubar = torch.ones(n, device="cuda")
    dx = torch.empty(n, 8, device="cuda")
    ds = torch.empty(len(envs), dtype=torch.float64, device="cuda")
    dg = torch.empty(len(envs), dtype=torch.float64, device="cuda")
    B.wos_estimate_batch([B.Domain(e) for e in envs], q, off, [e["sigma"] for e in envs],
                         [e["eps"] for e in envs], np.array([e["n_walks"] for e in envs]), seed, u, g, st,
                         ubar, dx, ds, dg)
    torch.cuda.synchronize()
    return u.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy(), dx.cpu().numpy(), off


def _check_sampled(oracle, envs, out, picks, what):
    """Sampled queries (env, local query) of a full launch recomputed by the
    oracle walk by walk on the same streams: u, grad u within 4 SE of the
    oracle's walks (+ FP32 rounding of large plane-wave values), dx = grad
    (u-bar = 1), padding columns 0, mean walk length within 5 %."""
    u, g, st, dx, off = out
    for e, ql in picks:
        s = envs[e]
        d = s["d"]
        dom = oracle.Domain(s)
        vals = [oracle.walk(s, s["queries"][ql], w, ql, env=e, dom=dom) for w in range(s["n_walks"])]
        uw = np.array([v["u"] for v in vals])
        gw = np.array([v["grad"] for v in vals])
        steps = np.array([v["steps"] for v in vals], dtype=np.float64)
        se_u = uw.std(ddof=1) / math.sqrt(len(uw))
        se_g = gw.std(axis=0, ddof=1) / math.sqrt(len(uw))
        r = off[e] + ql
        print(f"{what}: env {e} (d = {d}, M = {len(s['sph_r'])}) query {ql}: "
              f"|u - u_oracle| / SE = {abs(u[r] - uw.mean()) / se_u:.3f}, "
              f"max |grad - grad_oracle| / SE = {np.max(np.abs(g[r, :d] - gw.mean(0)) / se_g):.3f}, "
              f"steps {st[r, 9]:.2f} vs {steps.mean():.2f}")
        assert np.mean(uw != 0) >= 0.95, (e, ql)  # signal
        assert abs(u[r] - uw.mean()) <= 4 * se_u + 1e-6 + 2e-5 * abs(uw.mean()), (e, ql, u[r], uw.mean(), se_u)
        tol_g = 4 * se_g + 1e-6 + 2e-5 * max(abs(uw.mean()), np.abs(gw.mean(0)).max())
        assert np.all(np.abs(g[r, :d] - gw.mean(0)) <= tol_g), (e, ql)
        assert np.allclose(dx[r, :d], g[r, :d], rtol=1e-6, atol=1e-9), (e, ql)
        assert np.all(g[r, d:] == 0) and np.all(dx[r, d:] == 0)
        assert abs(st[r, 9] - steps.mean()) <= 0.05 * steps.mean()


def test_d7_bench_launch_sampled(B, oracle):
    """The d = 7 workload in the benchmark's launch (the 7-D segment queries
    plus the 83 7-D environments of the ragged batch, one fused forward +
    backward persistent launch, u_bar = 1), with plane-wave boundary data so
    that every query has signal: sampled queries recomputed by the oracle
    walk by walk on the same streams, within 4 SE (u, grad u, dx)."""
    envs = [S.scene_c3()] + S.scene_c4(dims={7})
    envs = [plane_wave(e, seed=i) for i, e in enumerate(envs)]
    out = _fused_full_launch(B, envs)
    Qs = [len(e["queries"]) for e in envs]
    heavy = max(range(1, len(envs)), key=lambda e: len(envs[e]["sph_r"]))
    rng = np.random.default_rng(17)
    picks = [(0, 5), (heavy, 0)] + [(e, int(rng.integers(Qs[e]))) for e in rng.choice(np.arange(1, len(envs)), 2)]
    assert np.all(out[0] > 0) and np.all(np.isfinite(out[0]))
    _check_sampled(oracle, envs, out, picks, "d7 launch")


def test_c4_full_launch_sampled(B, oracle):
    """The full ragged batch: 512 environments, d uniform in 2..7, 16-2048
    spheres, 1-4096 queries each (266081 queries x 2048 walks), in ONE fused
    forward + backward persistent launch, with plane-wave data on each
    environment's geometry so that every query has signal.  Every query's u
    is positive and finite; for each dimension, a query of the environment
    with the most obstacles and one of another environment are recomputed by
    the oracle walk by walk and agree within 4 SE."""
    envs = S.scene_c4()
    assert len(envs) == 512
    envs = [plane_wave(e, seed=i) for i, e in enumerate(envs)]
    out = _fused_full_launch(B, envs)
    u, g, st = out[0], out[1], out[2]
    assert np.all(u > 0) and np.all(np.isfinite(u)) and np.all(np.isfinite(g))
    assert np.all(st[:, 10] == 0)  # no truncated walk
    rng = np.random.default_rng(23)
    picks = []
    for d in range(2, 8):
        es = [e for e, s in enumerate(envs) if s["d"] == d]
        heavy = max(es, key=lambda e: len(envs[e]["sph_r"]))
        other = int(rng.choice([e for e in es if e != heavy]))
        for e in (heavy, other):
            picks.append((e, int(rng.integers(len(envs[e]["queries"])))))
    _check_sampled(oracle, envs, out, picks, "C4 launch")
