"""torch.autograd.Function over the WoS estimator.

Forward: u(x) and grad u(x) at the query rows of x (wos_estimate).  Only the
seed is kept for the backward pass; the backward kernel (wos_backward)
regenerates the same walks from their Philox counters and returns
dL/dx = ubar * grad u, dL/dsigma and dL/dg_goal.  The returned grad u is not
differentiable (its cotangent is ignored).
"""
from __future__ import annotations

import hashlib

import numpy as np
import torch

from . import binding as B


class WoSFunction(torch.autograd.Function):
    """u, grad_u = WoSFunction.apply(x, sigma, g_goal, scene, n_walks, eps, seed)

    x       (Q, d) float32 or float64 device tensor
    sigma   scalar tensor (screening coefficient c = 1/t)
    g_goal  scalar tensor (boundary value on the goal sphere, class mode)
    scene   scene dict (scenes.py) describing obstacles, goal and box
    """

    _cache = {}

    @staticmethod
    def _digest(obj, h):
        """Feed the scene's contents (arrays by value, nested dicts in key
        order) into the hash h."""
        if isinstance(obj, dict):
            for k in sorted(obj):
                h.update(repr(k).encode())
                WoSFunction._digest(obj[k], h)
        elif isinstance(obj, (np.ndarray, list, tuple)):
            a = np.ascontiguousarray(np.asarray(obj, dtype=np.float64))
            h.update(repr(a.shape).encode())
            h.update(a.tobytes())
        else:
            h.update(repr(obj).encode())

    @staticmethod
    def _domain(scene, g_goal):
        """The device domain of (scene, g_goal), cached by the scene's contents:
        a scene changed in place, or a new scene at a recycled address, gets
        its own domain."""
        h = hashlib.sha256()
        WoSFunction._digest({k: v for k, v in scene.items() if k != "queries"}, h)
        key = (h.hexdigest(), float(g_goal))
        dom = WoSFunction._cache.get(key)
        if dom is None:
            sc = dict(scene)
            sc["bdata"] = dict(scene["bdata"], g_goal=float(g_goal))
            dom = B.Domain(sc)
            if len(WoSFunction._cache) > 64:
                WoSFunction._cache.clear()
            WoSFunction._cache[key] = dom
        return dom

    @staticmethod
    def forward(ctx, x, sigma, g_goal, scene, n_walks, eps, seed):
        if x.dtype not in (torch.float32, torch.float64):
            raise TypeError("x must be float32 or float64")
        x = x.contiguous()
        fp64 = x.dtype == torch.float64
        dom = WoSFunction._domain(scene, float(g_goal))
        Q, d = x.shape
        u = torch.empty(Q, dtype=x.dtype, device=x.device)
        g = torch.empty(Q, d, dtype=x.dtype, device=x.device)
        B.wos_estimate(dom, x, n_walks, float(sigma), eps, seed, u, g, opt=B.options(fp64=fp64))
        ctx.save_for_backward(x)
        ctx.meta = (dom, float(sigma), n_walks, eps, seed, fp64)
        ctx.mark_non_differentiable(g)
        return u, g

    @staticmethod
    def backward(ctx, du, dgrad):
        (x,) = ctx.saved_tensors
        dom, sigma, n_walks, eps, seed, fp64 = ctx.meta
        if du is None:
            return None, None, None, None, None, None, None
        du = du.contiguous().to(x.dtype)
        dx = torch.empty_like(x)
        ds = torch.empty(1, dtype=torch.float64, device=x.device)
        dg = torch.empty(1, dtype=torch.float64, device=x.device)
        B.wos_backward(dom, x, n_walks, sigma, eps, seed, du, dx, ds, dg, opt=B.options(fp64=fp64))
        return dx, ds[0].to(x.dtype), dg[0].to(x.dtype), None, None, None, None


def wos_u(x, sigma, g_goal, scene, n_walks, eps, seed):
    return WoSFunction.apply(x, sigma, g_goal, scene, n_walks, eps, seed)
