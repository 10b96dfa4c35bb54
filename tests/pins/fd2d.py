"""Second-order finite-difference solve of the screened Poisson problem in 2-D,
used as an independent pin of the Walk-on-Spheres oracle.

Problem: Laplacian(u) - sigma u = 0 in the box [lo, hi]^2 minus a set of discs,
u = g on the boundary (g = 1 on the goal disc, 0 on obstacle discs and box).
Discretisation: five-point stencil on an (N + 1)^2 node grid; where a stencil
arm crosses a disc before the neighbouring node, the arm is shortened to the
crossing point and the boundary value is used there (Shortley & Weller, 1938),
which keeps the scheme O(h^2) at curved boundaries.  Solved with SuperLU.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def solve(discs, sigma, N, lo=-np.pi, hi=np.pi):
    """discs: list of (cx, cy, r, g).  Returns (xs, U) with U[i, j] the value at
    node (xs[i], xs[j]); nodes inside a disc hold that disc's g (nan when not
    in any disc but on the box, where g = 0)."""
    h = (hi - lo) / N
    xs = lo + h * np.arange(N + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    inside_disc = np.zeros(X.shape, dtype=bool)
    disc_val = np.zeros(X.shape)
    for cx, cy, r, g in discs:
        m = (X - cx) ** 2 + (Y - cy) ** 2 <= r * r
        disc_val[m & ~inside_disc] = g
        inside_disc |= m
    unknown = ~inside_disc
    unknown[0, :] = unknown[-1, :] = unknown[:, 0] = unknown[:, -1] = False
    idx = -np.ones(X.shape, dtype=np.int64)
    idx[unknown] = np.arange(unknown.sum())
    n = int(unknown.sum())
    I, J = np.nonzero(unknown)
    px, py = X[I, J], Y[I, J]

    diag = np.full(n, sigma, dtype=np.float64)
    rhs = np.zeros(n)
    arms = []  # per direction: (arm length, boundary value or nan, neighbour i, j)
    for (ex, ey, di, dj) in ((1, 0, 1, 0), (-1, 0, -1, 0), (0, 1, 0, 1), (0, -1, 0, -1)):
        arm = np.full(n, h)
        bval = np.full(n, np.nan)
        for cx, cy, r, g in discs:
            bx, by = px - cx, py - cy
            b = ex * bx + ey * by
            cc = bx * bx + by * by - r * r
            disc = b * b - cc
            ok = disc >= 0
            t = np.full(n, np.inf)
            t[ok] = -b[ok] - np.sqrt(disc[ok])
            hit = ok & (t > 0) & (t <= h) & (t < arm)
            arm[hit] = t[hit]
            bval[hit] = g
        arms.append((arm, bval, I + di, J + dj))
    A_r, A_c, A_v = [], [], []
    for axis in (0, 1):
        plus, minus = arms[2 * axis], arms[2 * axis + 1]
        for (harm, bval, ni, nj), hother in ((plus, minus[0]), (minus, plus[0])):
            w = 2.0 / (harm * (harm + hother))
            diag += w
            cut = ~np.isnan(bval)
            m_unk = (~cut) & unknown[ni, nj]
            A_r.append(np.nonzero(m_unk)[0])
            A_c.append(idx[ni[m_unk], nj[m_unk]])
            A_v.append(-w[m_unk])
            rhs[cut] += w[cut] * bval[cut]
            # an uncut arm ending on a box node contributes g_outer = 0
    r_all = np.concatenate(A_r + [np.arange(n)])
    c_all = np.concatenate(A_c + [np.arange(n)])
    v_all = np.concatenate(A_v + [diag])
    A = sp.csr_matrix((v_all, (r_all, c_all)), shape=(n, n))
    u = spla.spsolve(A.tocsc(), rhs)
    U = np.where(inside_disc, disc_val, 0.0)
    U[unknown] = u
    return xs, U


def c1_discs(scene):
    discs = [(float(c[0]), float(c[1]), float(r), scene["bdata"]["g_obs"])
             for c, r in zip(scene["sph_c"], scene["sph_r"])]
    discs.insert(0, (float(scene["goal_c"][0]), float(scene["goal_c"][1]),
                     float(scene["goal_r"]), scene["bdata"]["g_goal"]))
    return discs
