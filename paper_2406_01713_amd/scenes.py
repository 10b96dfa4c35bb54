"""Seeded synthetic scenes for the Walk-on-Spheres path.

This module only draws inputs: obstacle sets, goal balls, outer boxes and query
points, from ``numpy.random.default_rng(seed)`` in a fixed, documented order.
It holds none of the estimator's arithmetic.  The one geometric test it needs,
"is this point at least ``delta`` away from every obstacle", is a conservative
membership test (squared-radius test for balls, an L-infinity inflation for
boxes) written for input construction only; it is not the signed distance that
the walks use.

Both the HIP path and the CPU oracle take their inputs from here, so every
scene is a plain dict of float64 numpy arrays:

    d            dimension of configuration space
    sph_c, sph_r sphere obstacles, (Ms, d) and (Ms,)
    box_c, box_h axis-aligned box obstacles, centres and half-widths (Mb, d)
    goal_c, goal_r   goal ball (g = g_goal on its boundary), or goal_r = None
    outer        {"kind": "box", "lo": (d,), "hi": (d,)} or
                 {"kind": "ball", "c": (d,), "r": float}
    bdata        {"mode": 0|1|2, "g_goal", "g_obs", "g_outer", "ak": (d,), "b"}
    sigma, eps   screening coefficient (the paper's c = 1/t) and shell width
    queries      (Q, d)
    n_walks, seed

The workloads follow the paper's synthetic settings: a 2-D RR-arm-like box
(Table I gives the joint-space goal), sphere-cluttered boxes in 6 and 7
dimensions, a ragged batch of environments and a planning set of starts.
"""
from __future__ import annotations

import math

import numpy as np

PI = math.pi
CLEAR = 1e-2          # query clearance used by the workloads
GOAL_KEEPOUT = 0.05   # obstacles are redrawn if they come this close to goal/start


def _bdata(mode=0, d=2, g_goal=1.0, g_obs=0.0, g_outer=0.0, ak=None, b=0.0):
    a = np.zeros(d) if ak is None else np.asarray(ak, dtype=np.float64)
    return {"mode": int(mode), "g_goal": float(g_goal), "g_obs": float(g_obs),
            "g_outer": float(g_outer), "ak": a, "b": float(b)}


def box_outer(d, half=PI):
    return {"kind": "box", "lo": np.full(d, -half), "hi": np.full(d, half)}


def clear_mask(P, scene, delta, chunk=256):
    """Conservative clearance test for input construction, one flag per row of
    ``P``: True when the point is at least ``delta`` away from every obstacle,
    the goal ball and the outer boundary.  Spheres use a squared-radius test;
    boxes are tested against their L-infinity inflation, which contains their
    Euclidean ``delta``-neighbourhood."""
    P = np.atleast_2d(np.asarray(P, dtype=np.float64))
    ok = np.ones(len(P), dtype=bool)
    o = scene["outer"]
    k = int(scene.get("geom_d") or scene["d"])  # extruded geometry: leading k coordinates
    for i in range(0, len(P), chunk):
        p = P[i:i + chunk]
        pg = p[:, :k]
        m = np.ones(len(p), dtype=bool)
        if scene["sph_r"].size:
            sq = ((pg[:, None, :] - scene["sph_c"][None, :, :k]) ** 2).sum(axis=-1)
            m &= ~(sq < (scene["sph_r"][None] + delta) ** 2).any(axis=1)
        if scene["box_h"].size:
            away = (np.abs(p[:, None, :] - scene["box_c"][None])
                    >= scene["box_h"][None] + delta).any(axis=-1)
            m &= away.all(axis=1)
        if scene.get("goal_r") is not None:
            m &= ((p - scene["goal_c"]) ** 2).sum(axis=1) >= (scene["goal_r"] + delta) ** 2
        if o["kind"] == "box":
            m &= np.all(pg >= o["lo"][:k] + delta, axis=1) & np.all(pg <= o["hi"][:k] - delta, axis=1)
        else:
            m &= ((pg - o["c"][:k]) ** 2).sum(axis=1) <= max(o["r"] - delta, 0.0) ** 2
        ok[i:i + chunk] = m
    return ok


def is_clear(p, scene, delta):
    return bool(clear_mask(p, scene, delta)[0])


def _too_close(c, r, centre, rad, gap):
    return ((c - centre) ** 2).sum() < (r + rad + gap) ** 2


def _draw_spheres(rng, d, m, rlo, rhi, keep_clear, lo=-PI, hi=PI):
    """Centres (m, d) uniform in the box, then radii (m,) uniform; an obstacle
    that comes within GOAL_KEEPOUT of a keep-clear ball is redrawn (centre then
    radius) until it does not."""
    c = rng.uniform(lo, hi, size=(m, d))
    r = rng.uniform(rlo, rhi, size=m)
    for j in range(m):
        while any(_too_close(c[j], r[j], kc, kr, GOAL_KEEPOUT) for kc, kr in keep_clear):
            c[j] = rng.uniform(lo, hi, size=d)
            r[j] = rng.uniform(rlo, rhi)
    return c, r


def _draw_boxes(rng, d, m, hlo, hhi, keep_clear, lo=-PI, hi=PI):
    """Centres (m, d) uniform, half-widths (m, d) uniform per axis; redraw a box
    whose L-infinity inflation reaches a keep-clear ball's bounding box."""
    c = rng.uniform(lo, hi, size=(m, d))
    h = rng.uniform(hlo, hhi, size=(m, d))

    def bad(j):
        for kc, kr in keep_clear:
            if np.all(np.abs(kc - c[j]) < h[j] + kr + GOAL_KEEPOUT):
                return True
        return False

    for j in range(m):
        while bad(j):
            c[j] = rng.uniform(lo, hi, size=d)
            h[j] = rng.uniform(hlo, hhi, size=d)
    return c, h


def _free_points(rng, scene, n, delta=CLEAR, max_tries=None):
    """Uniform points in the outer box, redrawn while not clear by ``delta``.
    Round t redraws, in index order, every point still unclear after round
    t - 1.  With ``max_tries`` set, a point still unclear after that many
    rounds is kept as drawn (it starts inside or next to an obstacle: a
    degenerate query)."""
    o = scene["outer"]
    d = scene["d"]
    out = rng.uniform(o["lo"], o["hi"], size=(n, d))
    todo = np.nonzero(~clear_mask(out, scene, delta))[0]
    tries = 1
    while todo.size and (max_tries is None or tries < max_tries):
        out[todo] = rng.uniform(o["lo"], o["hi"], size=(todo.size, d))
        todo = todo[~clear_mask(out[todo], scene, delta)]
        tries += 1
    return out


def _empty(d):
    return {"sph_c": np.zeros((0, d)), "sph_r": np.zeros(0),
            "box_c": np.zeros((0, d)), "box_h": np.zeros((0, d))}


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def scene_c1(n_walks=1024, seed=0):
    """d = 2 RR-arm configuration box [-pi, pi]^2 with 8 circular C-obstacles
    (centres uniform, radii U[0.2, 0.5], seed 0), goal ball r = 0.1 centred at
    the joint-space goal of Table I (2.042, 0.200), sigma = 1, eps = 1e-3,
    an 8 x 8 cell-centre grid of queries (those inside obstacles are
    degenerate), FP64."""
    d = 2
    rng = np.random.default_rng(0)
    goal_c = np.array([2.042, 0.200])
    goal_r = 0.1
    c, r = _draw_spheres(rng, d, 8, 0.2, 0.5, [(goal_c, goal_r)])
    g = (np.arange(8) + 0.5) * (2 * PI / 8) - PI
    qx, qy = np.meshgrid(g, g, indexing="ij")
    queries = np.stack([qx.ravel(), qy.ravel()], axis=1)
    s = _empty(d)
    s.update(d=d, sph_c=c, sph_r=r, goal_c=goal_c, goal_r=goal_r, outer=box_outer(d),
             bdata=_bdata(0, d), sigma=1.0, eps=1e-3, queries=queries,
             n_walks=n_walks, seed=seed, name="c1_d2_rr")
    return s


def _cluttered(d, m_sph, m_box, seed, r_goal=0.15, rlo=0.1, rhi=0.4, hlo=0.05, hhi=0.3,
               goal_margin=0.5):
    """Goal centre then start point uniform in [-pi+0.5, pi-0.5]^d, then
    sphere obstacles (centres, radii), then box obstacles, all kept
    GOAL_KEEPOUT away from the goal ball and the start ball (radius r_goal)."""
    rng = np.random.default_rng(seed)
    goal_c = rng.uniform(-PI + goal_margin, PI - goal_margin, size=d)
    start = rng.uniform(-PI + goal_margin, PI - goal_margin, size=d)
    keep = [(goal_c, r_goal), (start, r_goal)]
    sc, sr = _draw_spheres(rng, d, m_sph, rlo, rhi, keep)
    if m_box:
        bc, bh = _draw_boxes(rng, d, m_box, hlo, hhi, keep)
    else:
        bc, bh = np.zeros((0, d)), np.zeros((0, d))
    s = {"d": d, "sph_c": sc, "sph_r": sr, "box_c": bc, "box_h": bh, "goal_c": goal_c,
         "goal_r": r_goal, "start": start, "outer": box_outer(d), "bdata": _bdata(0, d)}
    return s, rng


def scene_c2(n_queries=4096, n_walks=4096, seed=0):
    """d = 6 box [-pi, pi]^6, 256 spheres r U[0.1, 0.4] (scene seed 0), goal
    r = 0.15, sigma = 4, eps = 1e-4, uniform free queries (query seed 1,
    clearance 1e-2), FP32 forward u and grad u."""
    s, _ = _cluttered(6, 256, 0, 0)
    qrng = np.random.default_rng(1)
    s.update(sigma=4.0, eps=1e-4, queries=_free_points(qrng, s, n_queries),
             n_walks=n_walks, seed=seed, name="c2_d6_fwd")
    return s


def segment_queries(rng, s, n_seg=32, per_seg=32, delta=CLEAR):
    """Straight segments from uniform free starts towards the goal: points at
    t = (j + 1/2) / per_seg of the segment from the start to the goal sphere's
    point facing it; a segment is kept only if all its points are clear."""
    out = []
    while len(out) < n_seg:
        st = _free_points(rng, s, 1, delta)[0]
        dvec = st - s["goal_c"]
        end = s["goal_c"] + s["goal_r"] * dvec / np.sqrt((dvec ** 2).sum())
        t = (np.arange(per_seg) + 0.5) / per_seg
        pts = st[None, :] + t[:, None] * (end - st)[None, :]
        if clear_mask(pts, s, delta).all():
            out.append(pts)
    return np.concatenate(out, axis=0)


def scene_c3(n_walks=16384, seed=0, n_seg=32, per_seg=32):
    """d = 7, 256 spheres r U[0.1, 0.4], sigma = 2, eps = 1e-4, goal r = 0.15;
    1024 queries on 32 straight segments towards the goal; 16384 walks;
    differentiated (d/dx, d/dsigma, d/dg_goal)."""
    s, rng = _cluttered(7, 256, 0, 0)
    s.update(sigma=2.0, eps=1e-4, queries=segment_queries(rng, s, n_seg, per_seg),
             n_walks=n_walks, seed=seed, name="c3_d7_diff")
    return s


def scene_c4_env(e, n_walks=2048, seed=0, q_cap=None, dims=None):
    """Environment ``e`` of the ragged batch (rng seed e): d ~ U{2..7},
    M = round(exp(U[ln 16, ln 2048])) spheres r U[0.05, 0.4],
    Q = round(exp(U[0, ln 4096])) queries, sigma ~ U[0.5, 8], eps = 1e-4,
    goal r = 0.15 (0.1 for d = 2).  Queries are uniform free points; a query
    that stays unclear for 64 draws is kept (packed low-d scenes).  With
    ``dims`` given, an environment of another dimension is not drawn further
    and None is returned (every environment has its own generator)."""
    rng = np.random.default_rng(e)
    d = int(rng.integers(2, 8))
    if dims is not None and d not in dims:
        return None
    m = int(round(math.exp(rng.uniform(math.log(16), math.log(2048)))))
    q = int(round(math.exp(rng.uniform(0.0, math.log(4096)))))
    sigma = float(rng.uniform(0.5, 8.0))
    r_goal = 0.1 if d == 2 else 0.15
    goal_c = rng.uniform(-PI + 0.5, PI - 0.5, size=d)
    start = rng.uniform(-PI + 0.5, PI - 0.5, size=d)
    keep = [(goal_c, r_goal), (start, r_goal)]
    sc, sr = _draw_spheres(rng, d, m, 0.05, 0.4, keep)
    s = _empty(d)
    s.update(d=d, sph_c=sc, sph_r=sr, goal_c=goal_c, goal_r=r_goal, start=start,
             outer=box_outer(d), bdata=_bdata(0, d), sigma=sigma, eps=1e-4,
             n_walks=n_walks, seed=seed, name=f"c4_env{e}")
    if q_cap is not None:
        q = min(q, q_cap)
    s["queries"] = _free_points(rng, s, q, CLEAR, max_tries=64)
    return s


def scene_c4(n_envs=512, n_walks=2048, seed=0, dims=None, q_cap=None):
    """Ragged batch: environments 0..n_envs-1, optionally only those whose
    dimension is in ``dims``."""
    envs = []
    for e in range(n_envs):
        s = scene_c4_env(e, n_walks, seed, q_cap, dims)
        if s is not None:
            s["env_id"] = e
            envs.append(s)
    return envs


def scene_spheres(d, m_sph=256, n_queries=16, n_walks=1024, sigma=2.0, eps=1e-4, seed=0,
                  scene_seed=None):
    """A sphere-cluttered box [-pi, pi]^d of any dimension 2..8 in the form
    of the 6-D and 7-D workloads: m_sph spheres r U[0.1, 0.4], goal r = 0.15,
    uniform free queries drawn after the obstacles.  scene_seed (default d)
    keys the generator."""
    s, rng = _cluttered(d, m_sph, 0, d if scene_seed is None else scene_seed)
    s.update(sigma=float(sigma), eps=float(eps), queries=_free_points(rng, s, n_queries),
             n_walks=n_walks, seed=seed, name=f"spheres_d{d}_m{m_sph}")
    return s


def near_goal_points(scene, n, gap_lo=0.02, gap_hi=0.1, seed=5, delta=0.01):
    """n points at a distance U[gap_lo, gap_hi] outside the goal sphere in
    uniformly random directions, each clear of the obstacles and the outer
    boundary by delta (redrawn otherwise): queries whose walks reach the
    goal often, also in 6 and 7 dimensions."""
    rng = np.random.default_rng(seed)
    d = scene["d"]
    out = []
    while len(out) < n:
        v = rng.normal(size=d)
        p = scene["goal_c"] + (scene["goal_r"] + rng.uniform(gap_lo, gap_hi)) * v / np.sqrt((v ** 2).sum())
        if is_clear(p, scene, delta):
            out.append(p)
    return np.array(out)


def scene_c5(n_starts=256, n_walks=2048, seed=0):
    """Planning in d = 7: 512 spheres r U[0.1, 0.4] + 512 axis-aligned boxes
    (half-widths U[0.05, 0.3] per axis), sigma = 2, eps = 1e-4, goal r = 0.15,
    256 uniform free starts; steps s = min(0.02, d(x)/2), 200 steps."""
    s, rng = _cluttered(7, 512, 512, 0)
    s.update(sigma=2.0, eps=1e-4, queries=_free_points(rng, s, n_starts),
             n_walks=n_walks, seed=seed, s_ub=0.02, n_steps=200, name="c5_d7_plan")
    return s


# --------------------------------------------------------------------------
# Scenes with closed-form solutions (used to pin the estimator)
# --------------------------------------------------------------------------

def scene_ball(d, R=1.0, sigma=0.0, eps=1e-4, queries=None, n_walks=4096, seed=0,
               mode=0, ak=None, b=0.0):
    """Empty ball of radius R centred at the origin, boundary value 1 on the
    sphere (mode 0), or affine / plane-wave data (modes 1 / 2)."""
    s = _empty(d)
    s.update(d=d, goal_c=None, goal_r=None,
             outer={"kind": "ball", "c": np.zeros(d), "r": float(R)},
             bdata=_bdata(mode, d, g_goal=0.0, g_obs=0.0, g_outer=1.0, ak=ak, b=b),
             sigma=float(sigma), eps=float(eps),
             queries=np.zeros((1, d)) if queries is None else np.asarray(queries, float),
             n_walks=n_walks, seed=seed, name=f"ball_d{d}")
    return s


def scene_annulus(d, r_goal=0.3, R=1.0, sigma=0.0, eps=1e-4, queries=None, n_walks=4096,
                  seed=0):
    """Goal ball of radius r_goal at the origin inside an outer ball of radius
    R: g = 1 on the goal sphere, 0 on the outer sphere."""
    s = _empty(d)
    s.update(d=d, goal_c=np.zeros(d), goal_r=float(r_goal),
             outer={"kind": "ball", "c": np.zeros(d), "r": float(R)},
             bdata=_bdata(0, d), sigma=float(sigma), eps=float(eps),
             queries=np.zeros((1, d)) if queries is None else np.asarray(queries, float),
             n_walks=n_walks, seed=seed, name=f"annulus_d{d}")
    return s


def with_bdata(scene, mode, ak=None, b=0.0):
    """Copy of ``scene`` with affine (mode 1) or plane-wave (mode 2) data."""
    s = dict(scene)
    s["bdata"] = _bdata(mode, scene["d"], ak=ak, b=b)
    return s


def with_source(scene, z, amp=1.0, c_imp=1.0, keep_goal=False, g_goal=None):
    """Copy of ``scene`` with a point source amp * delta_z (Sec. VI: a unit
    impulse at the goal point).  By default the goal ball is dropped and all
    boundary data are zero, the paper's point-source formulation; with
    keep_goal the goal ball and boundary data stay (g_goal overrides the goal
    value)."""
    s = dict(scene)
    s["source"] = {"z": np.asarray(z, dtype=np.float64).copy(), "amp": float(amp), "c_imp": float(c_imp)}
    if not keep_goal:
        s["goal_c"], s["goal_r"] = None, None
        s["bdata"] = _bdata(0, scene["d"], g_goal=0.0, g_obs=0.0, g_outer=0.0)
    elif g_goal is not None:
        s["bdata"] = dict(scene["bdata"], g_goal=float(g_goal))
    return s


def scene_ball_source(d, R=1.0, sigma=1.0, eps=1e-4, queries=None, n_walks=4096, seed=0):
    """Ball of radius R around the origin with a unit source at the centre and
    zero boundary data: u(x) = G_B(|x|; R), the ball's Green's function."""
    s = scene_ball(d, R=R, sigma=sigma, eps=eps, queries=queries, n_walks=n_walks, seed=seed)
    s["bdata"] = _bdata(0, d, g_goal=0.0, g_obs=0.0, g_outer=0.0)
    s["source"] = {"z": np.zeros(d), "amp": 1.0, "c_imp": 1.0}
    s["name"] = f"ball_src_d{d}"
    return s


def scene_eval_env(d, k_r=0.3, sigma=1.0, eps=1e-2, queries=None, n_walks=4096, seed=0,
                   goal=(8.0, 0.0)):
    """The paper's evaluation environment (Sec. VI): an outer disk of radius
    r_o = 10 at the origin, an upper obstacle disk of radius r_u = k_r r_o and
    a lower one of radius r_l = r_u / 2 whose circles touch only at the
    origin, extruded: the geometry depends on (x_1, x_2) only and every
    further coordinate is unbounded.  A unit impulse at the goal point with
    zero boundary data; the goal point (8, 0) and the query x_start,1 = (-8, 0)
    (extra coordinates 0) are read off the paper's figures."""
    r_o = 10.0
    r_u = k_r * r_o
    r_l = 0.5 * r_u
    c = np.zeros((2, d))
    c[0, 1] = r_u
    c[1, 1] = -r_l
    s = {"sph_c": c, "sph_r": np.array([r_u, r_l]),
         "box_c": np.zeros((0, d)), "box_h": np.zeros((0, d))}
    z = np.zeros(d)
    z[:2] = goal
    if queries is None:
        queries = np.zeros((1, d))
        queries[0, 0] = -8.0
    s.update(d=d, geom_d=2, goal_c=None, goal_r=None,
             outer={"kind": "ball", "c": np.zeros(d), "r": r_o},
             bdata=_bdata(0, d, g_goal=0.0, g_obs=0.0, g_outer=0.0),
             source={"z": z, "amp": 1.0, "c_imp": 1.0},
             sigma=float(sigma), eps=float(eps), queries=np.asarray(queries, float),
             n_walks=n_walks, seed=seed, name=f"eval_env_d{d}_kr{k_r:g}")
    return s


def scene_extruded_annulus(d, r_in=0.5, r_out=2.0, sigma=0.0, eps=1e-4, queries=None,
                           n_walks=4096, seed=0):
    """An annulus in (x_1, x_2) extruded along every further coordinate: the
    inner disk is an obstacle carrying g = 1, the outer circle carries g = 0.
    The solution does not depend on the extra coordinates, so it is the
    two-dimensional one for every d: ln(r_out / rho) / ln(r_out / r_in) at
    sigma = 0, rho = |(x_1, x_2)|."""
    s = {"sph_c": np.zeros((1, d)), "sph_r": np.array([float(r_in)]),
         "box_c": np.zeros((0, d)), "box_h": np.zeros((0, d))}
    s.update(d=d, geom_d=2, goal_c=None, goal_r=None,
             outer={"kind": "ball", "c": np.zeros(d), "r": float(r_out)},
             bdata=_bdata(0, d, g_goal=0.0, g_obs=1.0, g_outer=0.0),
             sigma=float(sigma), eps=float(eps),
             queries=np.zeros((1, d)) if queries is None else np.asarray(queries, float),
             n_walks=n_walks, seed=seed, name=f"ext_annulus_d{d}")
    return s


RR_LINKS = (1.0, 1.0)  # link lengths: not given in the paper (unit links)
RR_X_OBS = (0.0, 1.3)  # task-space point obstacle (Table II)
RR_Q_LO = (-0.5 * PI, -PI)  # joint lower bounds: not given (each joint spans 2 pi)
RR_Q_HI = (1.5 * PI, PI)  # joint upper bounds q_ub (Table II)
RR_Q_START = (0.785, 0.800)
RR_Q_GOAL = (2.042, 0.200)


def rr_collision_points(links=RR_LINKS, x_obs=RR_X_OBS, n_col=200, n_dense=200001):
    """N_col points, equally spaced in arc length, on the set of RR joint
    configurations whose second link passes through the task-space point
    x_obs (Sec. VII, IK-based distance): with the point at distance t along
    link 2, the elbow angle q2 and the law of cosines give
    t = -l1 cos q2 + sqrt(rho^2 - l1^2 sin^2 q2), q1 = atan2(x_obs) -
    atan2(t sin q2, l1 + t cos q2), for |q2| up to the angle where t = l2.
    Link 1 cannot touch the point (l1 < |x_obs|)."""
    l1, l2 = links
    rho = math.hypot(*x_obs)
    if not (l1 < rho <= l1 + l2):
        raise ValueError("the point must lie beyond link 1 and within reach")
    a = math.acos((rho * rho - l1 * l1 - l2 * l2) / (2 * l1 * l2))
    q2 = np.linspace(-a, a, n_dense)
    t = -l1 * np.cos(q2) + np.sqrt(rho * rho - (l1 * np.sin(q2)) ** 2)
    q1 = math.atan2(x_obs[1], x_obs[0]) - np.arctan2(t * np.sin(q2), l1 + t * np.cos(q2))
    P = np.stack([q1, q2], axis=1)
    s = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(P, axis=0), axis=1))])
    tgt = np.linspace(0.0, s[-1], n_col)
    return np.stack([np.interp(tgt, s, q1), np.interp(tgt, s, q2)], axis=1)


def scene_rr(distance="ik", sigma=0.0, n_walks=100000, seed=0, eps=0.02, links=RR_LINKS):
    """The RR validation task (Sec. VII, Table II): joint box [q_lo, q_ub], a
    task-space point obstacle, a unit impulse at q_goal with zero boundary
    data, query q_start.  distance "ik": the collision set as N_col = 200
    point obstacles (radius 0); "lipschitz": the planar-arm bound
    d_tau / K."""
    d = 2
    s = _empty(d)
    if distance == "ik":
        P = rr_collision_points(links)
        s.update(sph_c=P, sph_r=np.zeros(len(P)))
    elif distance == "lipschitz":
        s["arm"] = {"l": np.array(links, dtype=np.float64), "pts": np.array([RR_X_OBS], dtype=np.float64)}
    else:
        raise ValueError(distance)
    s.update(d=d, goal_c=None, goal_r=None,
             outer={"kind": "box", "lo": np.array(RR_Q_LO), "hi": np.array(RR_Q_HI)},
             bdata=_bdata(0, d, g_goal=0.0, g_obs=0.0, g_outer=0.0),
             source={"z": np.array(RR_Q_GOAL), "amp": 1.0, "c_imp": 1.0},
             sigma=float(sigma), eps=float(eps), queries=np.array([RR_Q_START]),
             n_walks=n_walks, seed=seed, s_ub=0.1, name=f"rr_{distance}_c{sigma:g}")
    return s


def plane_wave_k(d, sigma, seed=0):
    """A wave vector k with |k|^2 = sigma, direction drawn from the seed."""
    rng = np.random.default_rng(1000 + seed)
    v = rng.normal(size=d)
    return math.sqrt(sigma) * v / np.sqrt((v ** 2).sum())


def walk_steps_hint(d):
    """Rough mean walk length used only to order work before it runs."""
    return {2: 12, 3: 25, 4: 40, 5: 55, 6: 71, 7: 85, 8: 95}.get(d, 85)
