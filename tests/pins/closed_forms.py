"""Exact solutions of Laplacian(u) - sigma u = 0 used to pin the estimator.

All are textbook separable solutions written with scipy's modified Bessel
functions (DLMF 10.25): with nu = d/2 - 1 and z = sqrt(sigma),
r^-nu I_nu(z r) and r^-nu K_nu(z r) are the radial solutions in d dimensions;
exp(k.x) with |k|^2 = sigma solves the equation everywhere; at sigma = 0 any
affine function is harmonic."""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def _f_I(nu, z, r):
    """r^-nu I_nu(z r), continuous at r = 0."""
    if r == 0.0:
        return (z / 2.0) ** nu / special.gamma(nu + 1.0)
    return r ** (-nu) * special.iv(nu, z * r)


def ball_u(d, sigma, R, x):
    """Solution in the ball |x| < R with u = 1 on the sphere."""
    r = float(np.linalg.norm(x))
    if sigma == 0.0:
        return 1.0
    nu = d / 2.0 - 1.0
    z = math.sqrt(sigma)
    return _f_I(nu, z, r) / _f_I(nu, z, R)


def ball_grad(d, sigma, R, x):
    """Gradient of ball_u: d/dr [r^-nu I_nu(z r)] = z r^-nu I_{nu+1}(z r)."""
    x = np.asarray(x, dtype=float)
    r = float(np.linalg.norm(x))
    if sigma == 0.0 or r == 0.0:
        return np.zeros_like(x)
    nu = d / 2.0 - 1.0
    z = math.sqrt(sigma)
    dudr = z * r ** (-nu) * special.iv(nu + 1.0, z * r) / _f_I(nu, z, R)
    return dudr * x / r


def ball_du_dsigma(d, sigma, R, x, h=1e-5):
    """d u / d sigma of ball_u by a central difference of the exact form."""
    if sigma <= h:
        return (ball_u(d, sigma + h, R, x) - ball_u(d, sigma, R, x)) / h
    return (ball_u(d, sigma + h, R, x) - ball_u(d, sigma - h, R, x)) / (2 * h)


def annulus_u(d, sigma, r_in, R, x):
    """Solution in r_in < |x| < R with u = 1 at r_in and u = 0 at R."""
    r = float(np.linalg.norm(x))
    if sigma == 0.0:
        if d == 2:
            return math.log(r / R) / math.log(r_in / R)
        p = 2.0 - d
        return (r ** p - R ** p) / (r_in ** p - R ** p)
    nu = d / 2.0 - 1.0
    z = math.sqrt(sigma)

    def fI(s):
        return s ** (-nu) * special.iv(nu, z * s)

    def fK(s):
        return s ** (-nu) * special.kv(nu, z * s)

    M = np.array([[fI(r_in), fK(r_in)], [fI(R), fK(R)]])
    A, B = np.linalg.solve(M, np.array([1.0, 0.0]))
    return A * fI(r) + B * fK(r)


def plane_wave(k, x):
    k = np.asarray(k, dtype=float)
    x = np.asarray(x, dtype=float)
    u = math.exp(float(k @ x))
    return u, k * u
