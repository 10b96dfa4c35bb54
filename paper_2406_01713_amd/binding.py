"""Thin ctypes binding of libwos (include/wos.h).

Argument marshalling only: every step of the estimator runs in the HIP
kernels of libwos.so.  Functions keep the C names (wos_create_domain,
wos_estimate, wos_backward, wos_estimate_batch, wos_plan_*, wos_autotune,
wos_debug_walks, wos_last_error); torch tensors provide device memory and
the current HIP stream.  If libwos.so is missing the import of this module
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libwos.so")

WOS_OK, WOS_EINVAL, WOS_EDIM, WOS_ENOMEM, WOS_EHIP, WOS_ENOTSUP = 0, -1, -2, -3, -4, -5
WOS_FP32, WOS_FP64, WOS_FULL_SCAN, WOS_SCALAR_CULL, WOS_WAVE_SCAN = 0, 1, 2, 4, 8
WOS_OUT_FP64 = 16
WOS_NO_BOX_TEST = 32
WOS_BOX_TEST = 64
WOS_NOALLOC_SCRATCH_BYTES = 64 << 20
WOS_NOALLOC_MAX_ENVS = 1024
WOS_CLUSTER_ROWS = 8  # obstacle rows per cluster (wos_debug_clusters capacities)
CLUSTER = WOS_CLUSTER_ROWS
WOS_BATCH_STATS = 16  # columns of a batched stats row
BATCH_STATS = WOS_BATCH_STATS
WOS_OUTER_BOX, WOS_OUTER_BALL = 0, 1
WOS_BATCH_STRIDE = 8
BATCH_STRIDE = WOS_BATCH_STRIDE
MAX_DIM = 8

EXPORTED = ["wos_create_domain", "wos_destroy_domain", "wos_domain_dim", "wos_estimate",
            "wos_backward", "wos_estimate_batch", "wos_estimate_batch_noalloc", "wos_plan_create", "wos_plan_step",
            "wos_plan_buffers", "wos_plan_read", "wos_plan_destroy", "wos_autotune", "wos_autotune_batch",
            "wos_set_autotune_cache",
            "wos_debug_walks", "wos_debug_clusters", "wos_debug_cluster_boxes", "wos_varadhan", "wos_microbench",
            "wos_last_error"]


class WosError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libwos error {code}: {msg}")
        self.code = code


class Spheres(C.Structure):
    _fields_ = [("n", C.c_int64), ("centers", C.POINTER(C.c_double)), ("radii", C.POINTER(C.c_double))]


class Boxes(C.Structure):
    _fields_ = [("n", C.c_int64), ("centers", C.POINTER(C.c_double)),
                ("half_widths", C.POINTER(C.c_double))]


class Ball(C.Structure):
    _fields_ = [("center", C.POINTER(C.c_double)), ("radius", C.c_double)]


class Outer(C.Structure):
    _fields_ = [("kind", C.c_int), ("lo", C.POINTER(C.c_double)), ("hi", C.POINTER(C.c_double)),
                ("center", C.POINTER(C.c_double)), ("radius", C.c_double), ("geom_d", C.c_int)]


class BData(C.Structure):
    _fields_ = [("mode", C.c_int), ("g_goal", C.c_double), ("g_obstacle", C.c_double),
                ("g_outer", C.c_double), ("a_or_k", C.POINTER(C.c_double)), ("b", C.c_double)]


class Arm(C.Structure):
    _fields_ = [("lengths", C.POINTER(C.c_double)), ("n_points", C.c_int64), ("points", C.POINTER(C.c_double))]


class Source(C.Structure):
    _fields_ = [("z", C.POINTER(C.c_double)), ("amplitude", C.c_double), ("c_imp", C.c_double)]


class Options(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("env_id", C.c_uint32), ("max_steps", C.c_uint32),
                ("reserved", C.c_uint32)]


class TuneResult(C.Structure):
    _fields_ = [("waves_per_block", C.c_int), ("units_per_wave", C.c_int), ("grid_mult", C.c_int),
                ("walks_per_lane", C.c_int), ("lanes_per_walker", C.c_int), ("ms_default", C.c_double),
                ("ms_best", C.c_double), ("tried", C.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2406_01713_amd.build` "
                          "(the estimator has no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i64, u64, u32, dp = C.c_void_p, C.c_int64, C.c_uint64, C.c_uint32, C.POINTER(C.c_double)
    L.wos_create_domain.argtypes = [C.c_int, C.POINTER(Spheres), C.POINTER(Boxes), C.POINTER(Arm),
                                    C.POINTER(Ball), C.POINTER(Outer), C.POINTER(BData), C.POINTER(Source),
                                    C.POINTER(vp)]
    L.wos_destroy_domain.argtypes = [vp]
    L.wos_destroy_domain.restype = None
    L.wos_domain_dim.argtypes = [vp]
    L.wos_estimate.argtypes = [vp, vp, i64, i64, C.c_double, C.c_double, u64, vp, vp, vp,
                               C.POINTER(Options), vp]
    L.wos_backward.argtypes = [vp, vp, i64, i64, C.c_double, C.c_double, u64, vp, vp, vp, vp, vp,
                               C.POINTER(Options), vp]
    L.wos_estimate_batch.argtypes = [C.POINTER(vp), C.c_int, vp, C.POINTER(i64), dp, dp, C.POINTER(i64), u64,
                                     vp, vp, vp, vp, vp, vp, vp, C.POINTER(Options), vp]
    L.wos_estimate_batch_noalloc.argtypes = L.wos_estimate_batch.argtypes
    L.wos_plan_create.argtypes = [vp, vp, i64, i64, C.c_double, C.c_double, C.c_double, u64,
                                  C.POINTER(Options), vp, C.POINTER(vp)]
    L.wos_plan_step.argtypes = [vp, C.c_int]
    L.wos_plan_buffers.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                   C.POINTER(vp), C.POINTER(vp)]
    L.wos_plan_read.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.wos_plan_destroy.argtypes = [vp]
    L.wos_plan_destroy.restype = None
    L.wos_autotune.argtypes = [C.c_int, i64, i64, i64, C.c_char_p]
    L.wos_autotune_batch.argtypes = [C.POINTER(vp), C.c_int, vp, C.POINTER(i64), dp, dp, C.POINTER(i64), u64,
                                     C.c_int, C.c_char_p, C.POINTER(TuneResult)]
    L.wos_set_autotune_cache.argtypes = [C.c_char_p]
    L.wos_debug_walks.argtypes = [vp, dp, u32, i64, i64, C.c_double, C.c_double, u64,
                                  C.POINTER(Options), dp]
    L.wos_debug_clusters.argtypes = [C.c_int, C.POINTER(Spheres), C.POINTER(Boxes), C.c_int,
                                     C.POINTER(i64), C.POINTER(i64), dp, C.POINTER(i64), dp]
    L.wos_debug_cluster_boxes.argtypes = [C.c_int, C.POINTER(Spheres), C.POINTER(Boxes), C.POINTER(i64), dp, dp]
    L.wos_microbench.argtypes = [C.c_int, dp, dp]
    L.wos_varadhan.argtypes = [vp, vp, i64, C.c_int, C.c_int, C.c_double, vp, vp, C.POINTER(Options), vp]
    L.wos_last_error.restype = C.c_char_p
    return L


lib = _load()


def check(rc):
    if rc != WOS_OK:
        raise WosError(rc, lib.wos_last_error().decode())
    return rc


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.reshape(shape) if shape is not None else a


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libwos needs device tensors")
    if not t.is_contiguous():
        raise ValueError("libwos needs contiguous tensors")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def options(fp64=False, env_id=0, max_steps=0, full_scan=False, scalar_cull=False, wave_scan=False,
            out_fp64=False, no_box_test=False, box_test=False):
    flags = (WOS_FP64 if fp64 else WOS_FP32) | (WOS_FULL_SCAN if full_scan else 0) | \
        (WOS_SCALAR_CULL if scalar_cull else 0) | (WOS_WAVE_SCAN if wave_scan else 0) | \
        (WOS_OUT_FP64 if out_fp64 else 0) | (WOS_NO_BOX_TEST if no_box_test else 0) | \
        (WOS_BOX_TEST if box_test else 0)
    return Options(flags, int(env_id), int(max_steps), 0)


# ---------------------------------------------------------------------------
# Domain
# ---------------------------------------------------------------------------

class Domain:
    """Owns a wos_domain built from a scene dict (see scenes.py)."""

    def __init__(self, scene):
        d = int(scene["d"])
        self.d = d
        keep = []

        def arr(a, shape):
            a = _f64(a, shape)
            keep.append(a)
            return a

        ns = len(scene["sph_r"])
        nb = len(scene["box_h"])
        sc, sr = arr(scene["sph_c"], (-1, d)) if ns else None, arr(scene["sph_r"], (-1,)) if ns else None
        bc, bh = arr(scene["box_c"], (-1, d)) if nb else None, arr(scene["box_h"], (-1, d)) if nb else None
        sph = Spheres(ns, _dp(sc) if ns else None, _dp(sr) if ns else None)
        box = Boxes(nb, _dp(bc) if nb else None, _dp(bh) if nb else None)
        goal = None
        if scene.get("goal_r") is not None:
            gc = arr(scene["goal_c"], (d,))
            goal = Ball(_dp(gc), float(scene["goal_r"]))
        o = scene["outer"]
        gd = int(scene.get("geom_d") or 0)  # 0: the full space
        if o["kind"] == "box":
            lo, hi = arr(o["lo"], (d,)), arr(o["hi"], (d,))
            outer = Outer(WOS_OUTER_BOX, _dp(lo), _dp(hi), None, 0.0, gd)
        else:
            oc = arr(o["c"], (d,))
            outer = Outer(WOS_OUTER_BALL, None, None, _dp(oc), float(o["r"]), gd)
        b = scene["bdata"]
        ak = arr(b["ak"], (d,))
        bd = BData(int(b["mode"]), float(b["g_goal"]), float(b["g_obs"]), float(b["g_outer"]),
                   _dp(ak), float(b["b"]))
        src = None
        if scene.get("source") is not None:
            z = arr(scene["source"]["z"], (d,))
            src = Source(_dp(z), float(scene["source"].get("amp", 1.0)),
                         float(scene["source"].get("c_imp", 1.0)))
        arm = None
        if scene.get("arm") is not None:
            al = arr(scene["arm"]["l"], (d,))
            ap = arr(scene["arm"]["pts"], (-1, 2))
            arm = Arm(_dp(al), len(ap), _dp(ap))
        h = C.c_void_p()
        check(lib.wos_create_domain(d, C.byref(sph), C.byref(box), C.byref(arm) if arm else None,
                                    C.byref(goal) if goal else None,
                                    C.byref(outer), C.byref(bd), C.byref(src) if src else None, C.byref(h)))
        self.handle = h
        self.n_obstacles = ns + nb
        self.has_source = src is not None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:  # lib is None during interpreter exit
            lib.wos_destroy_domain(h)
            self.handle = None


# ---------------------------------------------------------------------------
# Calls (device tensors in, device tensors out)
# ---------------------------------------------------------------------------

def wos_estimate(dom, queries, n_walks, sigma, eps, seed, out_u, out_grad=None, out_stats=None,
                 opt=None, stream=None):
    check(lib.wos_estimate(dom.handle, _ptr(queries), queries.shape[0], int(n_walks), float(sigma),
                           float(eps), int(seed), _ptr(out_u), _ptr(out_grad), _ptr(out_stats),
                           C.byref(opt) if opt is not None else None, _stream(stream)))


def wos_backward(dom, queries, n_walks, sigma, eps, seed, grad_u, out_dx, out_dsigma, out_dg,
                 out_dq=None, opt=None, stream=None):
    check(lib.wos_backward(dom.handle, _ptr(queries), queries.shape[0], int(n_walks), float(sigma),
                           float(eps), int(seed), _ptr(grad_u), _ptr(out_dx), _ptr(out_dsigma),
                           _ptr(out_dg), _ptr(out_dq), C.byref(opt) if opt is not None else None,
                           _stream(stream)))


def wos_estimate_batch(doms, queries, q_offsets, sigma, eps, n_walks, seed, out_u, out_grad=None,
                       out_stats=None, grad_u=None, out_dx=None, out_dsigma=None, out_dg=None,
                       opt=None, stream=None, noalloc=False):
    """The batched call; noalloc=True calls wos_estimate_batch_noalloc (the
    same launch with the library's fixed per-device scratch array)."""
    n = len(doms)
    fn = lib.wos_estimate_batch_noalloc if noalloc else lib.wos_estimate_batch
    hs = (C.c_void_p * n)(*[dm.handle.value for dm in doms])
    qo = np.ascontiguousarray(np.asarray(q_offsets, dtype=np.int64))
    sg = _f64(sigma)
    ep = _f64(eps)
    nw = np.ascontiguousarray(np.broadcast_to(np.asarray(n_walks, dtype=np.int64), (n,)))
    check(fn(hs, n, _ptr(queries), qo.ctypes.data_as(C.POINTER(C.c_int64)),
             _dp(sg), _dp(ep), nw.ctypes.data_as(C.POINTER(C.c_int64)), int(seed),
             _ptr(out_u), _ptr(out_grad), _ptr(out_stats), _ptr(grad_u), _ptr(out_dx),
             _ptr(out_dsigma), _ptr(out_dg), C.byref(opt) if opt is not None else None, _stream(stream)))


def wos_debug_walks(dom, query, q_index, w0, n, sigma, eps, seed, opt=None):
    q = _f64(query, (dom.d,))
    out = np.zeros((int(n), dom.d + 7))
    check(lib.wos_debug_walks(dom.handle, _dp(q), int(q_index), int(w0), int(n), float(sigma),
                              float(eps), int(seed), C.byref(opt) if opt is not None else None,
                              _dp(out)))
    return out


def wos_debug_cluster_boxes(d, sph_c=None, sph_r=None, box_c=None, box_h=None):
    """Host-only cluster bounding boxes of an obstacle set: dict with, per
    kind ('sph', 'box'), an n_cl x 2d array of lo then hi per cluster (the
    FP32 values of the device table), clusters in wos_debug_clusters order."""
    keep = []
    sp = bx = None
    if sph_c is not None and len(sph_r):
        c, r = _f64(sph_c), _f64(sph_r)
        keep += [c, r]
        sp = Spheres(len(r), _dp(c), _dp(r))
    if box_c is not None and len(box_c):
        c, h = _f64(box_c), _f64(box_h)
        keep += [c, h]
        bx = Boxes(len(c), _dp(c), _dp(h))
    n_cl = (C.c_int64 * 2)()
    args = (int(d), C.byref(sp) if sp else None, C.byref(bx) if bx else None)
    check(lib.wos_debug_cluster_boxes(*args, n_cl, None, None))
    b_s = np.zeros((n_cl[0], 2 * d))
    b_b = np.zeros((n_cl[1], 2 * d))
    check(lib.wos_debug_cluster_boxes(*args, n_cl, _dp(b_s), _dp(b_b)))
    return {"sph": b_s, "box": b_b}


def wos_debug_clusters(d, sph_c=None, sph_r=None, box_c=None, box_h=None, fp64=False):
    """Host-only cluster layout of an obstacle set: dict with, per kind
    ('sph', 'box'), the caller index of each clustered row (-1: padding) and
    the bounding spheres (n_cl x (d + 1): centre, enlarged radius)."""
    keep = []
    sp = bx = None
    if sph_c is not None and len(sph_r):
        c, r = _f64(sph_c), _f64(sph_r)
        keep += [c, r]
        sp = Spheres(len(r), _dp(c), _dp(r))
    if box_c is not None and len(box_c):
        c, h = _f64(box_c), _f64(box_h)
        keep += [c, h]
        bx = Boxes(len(c), _dp(c), _dp(h))
    n_cl = (C.c_int64 * 2)()
    args = (int(d), C.byref(sp) if sp else None, C.byref(bx) if bx else None, int(bool(fp64)))
    check(lib.wos_debug_clusters(*args, n_cl, None, None, None, None))
    ns, nb = n_cl[0], n_cl[1]
    o_s = np.zeros(ns * CLUSTER, np.int64)
    o_b = np.zeros(nb * CLUSTER, np.int64)
    b_s = np.zeros((ns, d + 1))
    b_b = np.zeros((nb, d + 1))
    p64 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
    check(lib.wos_debug_clusters(*args, n_cl, p64(o_s), _dp(b_s), p64(o_b), _dp(b_b)))
    return {"sph": (o_s, b_s), "box": (o_b, b_b)}


def wos_varadhan(u, sigma, grad_u=None, out_w=None, out_grad_w=None, opt=None, stream=None):
    """Varadhan read-out w = -sqrt(1/sigma) ln u (and grad w) on device tensors."""
    import torch
    if opt is None:
        opt = options(fp64=(u.dtype == torch.float64))
    out_w = torch.empty_like(u) if out_w is None else out_w
    d = stride = 0
    if grad_u is not None:
        stride = grad_u.shape[1]
        d = stride if stride <= MAX_DIM else MAX_DIM
        out_grad_w = torch.empty_like(grad_u) if out_grad_w is None else out_grad_w
    check(lib.wos_varadhan(_ptr(u), _ptr(grad_u), u.shape[0], d, stride, float(sigma), _ptr(out_w),
                           _ptr(out_grad_w), C.byref(opt) if opt is not None else None, _stream(stream)))
    return (out_w, out_grad_w) if grad_u is not None else out_w


def wos_microbench(which):
    """(rate, ms): 0 FP32 FMA FLOP/s, 1 sqrt/s, 2 7-D sphere evaluations/s."""
    r = C.c_double()
    ms = C.c_double()
    check(lib.wos_microbench(int(which), C.byref(r), C.byref(ms)))
    return r.value, ms.value


def wos_autotune(d, n_obstacles, n_queries, n_walks, cache_path):
    check(lib.wos_autotune(int(d), int(n_obstacles), int(n_queries), int(n_walks),
                           str(cache_path).encode()))


def wos_autotune_batch(doms, queries, q_offsets, sigma, eps, n_walks, seed, fused=True, cache_path=None):
    """Search the persistent launch's shape on this batch (wos_autotune_batch);
    returns the chosen shape and the launch times (ms) of the built-in and
    the chosen shape."""
    n = len(doms)
    hs = (C.c_void_p * n)(*[dm.handle.value for dm in doms])
    qo = np.ascontiguousarray(np.asarray(q_offsets, dtype=np.int64))
    sg = _f64(sigma)
    ep = _f64(eps)
    nw = np.ascontiguousarray(np.broadcast_to(np.asarray(n_walks, dtype=np.int64), (n,)))
    r = TuneResult()
    check(lib.wos_autotune_batch(hs, n, _ptr(queries), qo.ctypes.data_as(C.POINTER(C.c_int64)), _dp(sg), _dp(ep),
                                 nw.ctypes.data_as(C.POINTER(C.c_int64)), int(seed), int(bool(fused)),
                                 None if cache_path is None else str(cache_path).encode(), C.byref(r)))
    return {k: getattr(r, k) for k, _ in TuneResult._fields_}


def wos_set_autotune_cache(cache_path):
    check(lib.wos_set_autotune_cache(None if cache_path is None else str(cache_path).encode()))


class Plan:
    """Planning loop captured as a HIP graph (wos_plan_*)."""

    def __init__(self, dom, x, n_walks, sigma, eps, s_ub, seed, opt=None, stream=None):
        self.x = x
        self.d = dom.d
        self._dom = dom
        h = C.c_void_p()
        check(lib.wos_plan_create(dom.handle, _ptr(x), x.shape[0], int(n_walks), float(sigma),
                                  float(eps), float(s_ub), int(seed),
                                  C.byref(opt) if opt is not None else None, _stream(stream),
                                  C.byref(h)))
        self.handle = h
        ptrs = [C.c_void_p() for _ in range(6)]
        check(lib.wos_plan_buffers(h, *[C.byref(p) for p in ptrs]))
        self.device_ptrs = [p.value for p in ptrs]

    def step(self, n=1):
        check(lib.wos_plan_step(self.handle, int(n)))

    def read(self):
        """Host copies of (u[S], grad[S, 8], path_len[S], stalls[S], status[S], step)."""
        S = self.x.shape[0]
        out = [np.zeros(S, np.float32), np.zeros((S, 8), np.float32), np.zeros(S, np.float64),
               np.zeros(S, np.int32), np.zeros(S, np.int32), np.zeros(1, np.uint64)]
        check(lib.wos_plan_read(self.handle, *[C.c_void_p(a.ctypes.data) for a in out]))
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:  # lib is None during interpreter exit
            lib.wos_plan_destroy(h)
            self.handle = None
