"""ctypes binding of the FP64 CPU oracle (``wos_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.
Scenes are the dicts produced by ``paper_2406_01713_amd.scenes``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wos_oracle.c")
LIB = os.path.join(HERE, "libwos_oracle.so")
MAXD = 8
GOAL, SPHERE, BOX, OUTER, ARM = 0, 1, 2, 3, 4
ABSORBED, DEGENERATE, TRUNCATED = 0, 1, 2
DEFAULT_MAX_STEPS = 1 << 16


def build():
    """Compile the oracle with gcc (plain C99, -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", SRC, "-o", LIB, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB


class OrDomain(C.Structure):
    _fields_ = [
        ("d", C.c_int),
        ("has_src", C.c_int), ("src_z", C.c_double * MAXD), ("src_amp", C.c_double), ("c_imp", C.c_double),
        ("n_sph", C.c_int), ("sph_c", C.POINTER(C.c_double)), ("sph_r", C.POINTER(C.c_double)),
        ("n_box", C.c_int), ("box_c", C.POINTER(C.c_double)), ("box_h", C.POINTER(C.c_double)),
        ("has_goal", C.c_int), ("goal_c", C.c_double * MAXD), ("goal_r", C.c_double),
        ("outer_kind", C.c_int), ("lo", C.c_double * MAXD), ("hi", C.c_double * MAXD),
        ("outer_c", C.c_double * MAXD), ("outer_r", C.c_double),
        ("mode", C.c_int), ("g_goal", C.c_double), ("g_obs", C.c_double),
        ("g_outer", C.c_double), ("ak", C.c_double * MAXD), ("b", C.c_double),
        ("geom_d", C.c_int),
        ("n_arm", C.c_int), ("arm_pts", C.POINTER(C.c_double)), ("arm_l", C.c_double * MAXD),
    ]


class OrWalk(C.Structure):
    _fields_ = [("u", C.c_double), ("grad", C.c_double * MAXD), ("dlnC_sum", C.c_double),
                ("du_dsigma", C.c_double), ("goal_w", C.c_double), ("steps", C.c_int), ("status", C.c_int),
                ("cls", C.c_int), ("idx", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        u32 = C.c_uint32
        L.or_philox4x32_10.argtypes = [C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
        L.or_uniform.argtypes = [u32]
        L.or_uniform.restype = C.c_double
        L.or_direction.argtypes = [C.c_int, C.c_uint64, u32, u32, u32, u32, dp]
        L.or_distance.argtypes = [C.POINTER(OrDomain), dp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.or_distance.restype = C.c_double
        L.or_closest_point.argtypes = [C.POINTER(OrDomain), dp, C.c_int, C.c_int, dp]
        L.or_arm_K.argtypes = [C.POINTER(OrDomain)]
        L.or_arm_K.restype = C.c_double
        L.or_arm_task_distance.argtypes = [C.POINTER(OrDomain), dp]
        L.or_arm_task_distance.restype = C.c_double
        L.or_boundary_value.argtypes = [C.POINTER(OrDomain), dp, C.c_int, C.c_int]
        L.or_boundary_value.restype = C.c_double
        for f in ("or_screening_C", "or_screening_C1", "or_dlnC_dsigma"):
            getattr(L, f).argtypes = [C.c_int, C.c_double, C.c_double]
            getattr(L, f).restype = C.c_double
        L.or_hyp0f1.argtypes = [C.c_double, C.c_double]
        L.or_hyp0f1.restype = C.c_double
        L.or_bessel_k.argtypes = [C.c_double, C.c_double]
        L.or_bessel_k.restype = C.c_double
        L.or_varadhan.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.or_yukawa_free.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_yukawa_free.restype = C.c_double
        for f in ("or_ball_green", "or_ball_green_grad", "or_ball_green_dsigma"):
            getattr(L, f).argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
            getattr(L, f).restype = C.c_double
        L.or_walk.argtypes = [C.POINTER(OrDomain), dp, C.c_double, C.c_double, C.c_uint64,
                              u32, u32, u32, C.c_int, C.POINTER(OrWalk)]
        L.or_estimate.argtypes = [C.POINTER(OrDomain), dp, C.c_int64, C.c_int64, C.c_double,
                                  C.c_double, C.c_uint64, u32, C.c_int, dp, dp, dp, dp]
        L.or_estimate.restype = C.c_int
        L.or_backward.argtypes = [C.POINTER(OrDomain), dp, C.c_int64, C.c_int64, C.c_double,
                                  C.c_double, C.c_uint64, u32, C.c_int, dp, dp, dp, dp]
        L.or_backward.restype = C.c_int
        L.or_plan_step.argtypes = [C.POINTER(OrDomain), dp, C.c_int64, C.c_int64, C.c_double,
                                   C.c_double, C.c_double, C.c_uint64, C.c_uint64, C.c_int, dp,
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.or_plan_step.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Domain:
    """Oracle view of a scene dict (keeps the numpy arrays alive)."""

    def __init__(self, scene):
        d = int(scene["d"])
        self.d = d
        self._keep = []
        D = OrDomain()
        D.d = d

        def arr(a, shape):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))
            self._keep.append(a)
            return a

        sc = arr(scene["sph_c"], (-1, d)) if len(scene["sph_r"]) else arr(np.zeros((1, d)), (1, d))
        sr = arr(scene["sph_r"], (-1,)) if len(scene["sph_r"]) else arr(np.zeros(1), (1,))
        D.n_sph = len(scene["sph_r"])
        D.sph_c, D.sph_r = _dp(sc), _dp(sr)
        nb = len(scene["box_h"])
        bc = arr(scene["box_c"], (-1, d)) if nb else arr(np.zeros((1, d)), (1, d))
        bh = arr(scene["box_h"], (-1, d)) if nb else arr(np.zeros((1, d)), (1, d))
        D.n_box = nb
        D.box_c, D.box_h = _dp(bc), _dp(bh)
        if scene.get("goal_r") is not None:
            D.has_goal = 1
            for i in range(d):
                D.goal_c[i] = float(scene["goal_c"][i])
            D.goal_r = float(scene["goal_r"])
        D.geom_d = int(scene.get("geom_d") or 0)  # 0: the full space
        arm = scene.get("arm")
        if arm is not None:
            ap = arr(arm["pts"], (-1, 2))
            D.n_arm = len(ap)
            D.arm_pts = _dp(ap)
            for i in range(d):
                D.arm_l[i] = float(arm["l"][i])
        o = scene["outer"]
        if o["kind"] == "box":
            D.outer_kind = 0
            for i in range(d):
                D.lo[i], D.hi[i] = float(o["lo"][i]), float(o["hi"][i])
        else:
            D.outer_kind = 1
            for i in range(d):
                D.outer_c[i] = float(o["c"][i])
            D.outer_r = float(o["r"])
        b = scene["bdata"]
        D.mode = int(b["mode"])
        D.g_goal, D.g_obs, D.g_outer = b["g_goal"], b["g_obs"], b["g_outer"]
        for i in range(d):
            D.ak[i] = float(b["ak"][i])
        D.b = float(b["b"])
        src = scene.get("source")
        if src is not None:
            D.has_src = 1
            for i in range(d):
                D.src_z[i] = float(src["z"][i])
            D.src_amp = float(src.get("amp", 1.0))
            D.c_imp = float(src.get("c_imp", 1.0))
        self.s = D

    @property
    def ref(self):
        return C.byref(self.s)


def philox(ctr, key):
    L = lib()
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    L.or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(x):
    return lib().or_uniform(int(x) & 0xFFFFFFFF)


def direction(d, seed, k, w, q, env=0):
    v = np.zeros(MAXD)
    lib().or_direction(d, seed, k, w, q, env, _dp(v))
    return v[:d].copy()


def distance(scene_or_dom, x):
    dom = scene_or_dom if isinstance(scene_or_dom, Domain) else Domain(scene_or_dom)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    cls, idx = C.c_int(), C.c_int()
    R = lib().or_distance(dom.ref, _dp(x), C.byref(cls), C.byref(idx))
    return R, cls.value, idx.value


def closest_point(scene_or_dom, x, cls, idx):
    dom = scene_or_dom if isinstance(scene_or_dom, Domain) else Domain(scene_or_dom)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.zeros(dom.d)
    lib().or_closest_point(dom.ref, _dp(x), cls, idx, _dp(out))
    return out


def arm_K(scene_or_dom):
    dom = scene_or_dom if isinstance(scene_or_dom, Domain) else Domain(scene_or_dom)
    return lib().or_arm_K(dom.ref)


def arm_task_distance(scene_or_dom, q):
    dom = scene_or_dom if isinstance(scene_or_dom, Domain) else Domain(scene_or_dom)
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    return lib().or_arm_task_distance(dom.ref, _dp(q))


def boundary_value(scene_or_dom, x, cls, idx):
    dom = scene_or_dom if isinstance(scene_or_dom, Domain) else Domain(scene_or_dom)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return lib().or_boundary_value(dom.ref, _dp(x), cls, idx)


def hyp0f1(b, y):
    return lib().or_hyp0f1(float(b), float(y))


def varadhan(sigma, u, grad_u=None):
    """(w, grad_w) = (-sqrt(t) ln u, -sqrt(t) grad_u / u), t = 1 / sigma."""
    g = np.ascontiguousarray(np.zeros(1) if grad_u is None else np.asarray(grad_u, dtype=np.float64))
    d = len(g) if grad_u is not None else 0
    w = C.c_double()
    gw = np.zeros(max(d, 1))
    lib().or_varadhan(d, float(sigma), float(u), _dp(g), C.byref(w), _dp(gw) if grad_u is not None else None)
    return (w.value, gw[:d].copy()) if grad_u is not None else w.value


def bessel_k(nu, z):
    return lib().or_bessel_k(float(nu), float(z))


def yukawa_free(d, sigma, r):
    return lib().or_yukawa_free(int(d), float(sigma), float(r))


def ball_green(d, sigma, r, R):
    return lib().or_ball_green(int(d), float(sigma), float(r), float(R))


def ball_green_grad(d, sigma, r, R):
    return lib().or_ball_green_grad(int(d), float(sigma), float(r), float(R))


def ball_green_dsigma(d, sigma, r, R):
    return lib().or_ball_green_dsigma(int(d), float(sigma), float(r), float(R))


def screening_C(d, sigma, R):
    return lib().or_screening_C(d, float(sigma), float(R))


def screening_C1(d, sigma, R):
    return lib().or_screening_C1(d, float(sigma), float(R))


def dlnC_dsigma(d, sigma, R):
    return lib().or_dlnC_dsigma(d, float(sigma), float(R))


def walk(scene, x, w, q=0, env=0, sigma=None, eps=None, seed=None, max_steps=DEFAULT_MAX_STEPS,
         dom=None):
    dom = dom or Domain(scene)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    r = OrWalk()
    lib().or_walk(dom.ref, _dp(x), scene["sigma"] if sigma is None else sigma,
                  scene["eps"] if eps is None else eps, scene["seed"] if seed is None else seed,
                  w, q, env, max_steps, C.byref(r))
    return {"u": r.u, "grad": np.array(r.grad[:dom.d]), "dlnC_sum": r.dlnC_sum,
            "du_dsigma": r.du_dsigma, "goal_w": r.goal_w, "steps": r.steps, "status": r.status, "cls": r.cls,
            "idx": r.idx}


def estimate(scene, queries=None, n_walks=None, sigma=None, eps=None, seed=None, env=0,
             max_steps=DEFAULT_MAX_STEPS, dq=False):
    """Returns (u[Q], grad[Q, d], stats[Q, d + 4]) and, with dq=True, also
    dq[Q, 2] = (du/dsigma, du/dg_goal) per query."""
    dom = Domain(scene)
    d = dom.d
    Qs = np.ascontiguousarray(np.asarray(scene["queries"] if queries is None else queries,
                                         dtype=np.float64).reshape(-1, d))
    Q = len(Qs)
    u = np.zeros(Q)
    g = np.zeros((Q, d))
    st = np.zeros((Q, d + 4))
    dqa = np.zeros((Q, 2))
    rc = lib().or_estimate(dom.ref, _dp(Qs), Q, scene["n_walks"] if n_walks is None else n_walks,
                           scene["sigma"] if sigma is None else sigma,
                           scene["eps"] if eps is None else eps,
                           scene["seed"] if seed is None else seed, env, max_steps,
                           _dp(u), _dp(g), _dp(st), _dp(dqa))
    if rc:
        raise RuntimeError(f"or_estimate failed: {rc}")
    return (u, g, st, dqa) if dq else (u, g, st)


def backward(scene, ubar, queries=None, n_walks=None, sigma=None, eps=None, seed=None, env=0,
             max_steps=DEFAULT_MAX_STEPS):
    dom = Domain(scene)
    d = dom.d
    Qs = np.ascontiguousarray(np.asarray(scene["queries"] if queries is None else queries,
                                         dtype=np.float64).reshape(-1, d))
    Q = len(Qs)
    ub = np.ascontiguousarray(np.asarray(ubar, dtype=np.float64).reshape(Q))
    dx = np.zeros((Q, d))
    ds, dg = C.c_double(), C.c_double()
    rc = lib().or_backward(dom.ref, _dp(Qs), Q, scene["n_walks"] if n_walks is None else n_walks,
                           scene["sigma"] if sigma is None else sigma,
                           scene["eps"] if eps is None else eps,
                           scene["seed"] if seed is None else seed, env, max_steps, _dp(ub),
                           _dp(dx), C.byref(ds), C.byref(dg))
    if rc:
        raise RuntimeError(f"or_backward failed: {rc}")
    return dx, ds.value, dg.value


def plan_step(scene, x, t, path_len, stalls, status, n_walks=None, s_ub=None, seed=None,
              max_steps=DEFAULT_MAX_STEPS):
    """One planning step in place on x (S, d), path_len (S,), stalls, status (S,) int32."""
    dom = Domain(scene)
    assert x.dtype == np.float64 and x.flags.c_contiguous
    rc = lib().or_plan_step(dom.ref, _dp(x), len(x),
                            scene["n_walks"] if n_walks is None else n_walks, scene["sigma"],
                            scene["eps"], scene["s_ub"] if s_ub is None else s_ub,
                            scene["seed"] if seed is None else seed, t, max_steps, _dp(path_len),
                            stalls.ctypes.data_as(C.POINTER(C.c_int32)),
                            status.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc:
        raise RuntimeError(f"or_plan_step failed: {rc}")
