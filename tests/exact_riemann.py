"""Exact solution of the one-dimensional Riemann problem for the Euler
equations of an ideal gas (the classical construction: a nonlinear equation
for the star pressure, each side a shock or a rarefaction, sampled along
x/t).  Test infrastructure: used to check shock-capturing results against
the physics, independently of the oracle.
"""
from __future__ import annotations

import math

import numpy as np


def _side(p, rho, pk, gamma):
    """Velocity jump across the wave of one side for star pressure p, and its
    derivative in p."""
    c = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        a = 2.0 / ((gamma + 1.0) * rho)
        b = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(a / (p + b))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + b))
    # rarefaction
    e = (gamma - 1.0) / (2.0 * gamma)
    f = 2.0 * c / (gamma - 1.0) * ((p / pk) ** e - 1.0)
    return f, (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * c)


def star_state(left, right, gamma=1.4, tol=1e-14):
    """(p*, u*) for primitive states left = (rho, u, p), right = (rho, u, p),
    by Newton's method on f_L(p) + f_R(p) + u_R - u_L = 0."""
    rl, ul, pl = left
    rr, ur, pr = right
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _side(p, rl, pl, gamma)
        fr, dr = _side(p, rr, pr, gamma)
        step = (fl + fr + ur - ul) / (dl + dr)
        p_new = max(1e-14, p - step)
        if abs(p_new - p) <= tol * p_new:
            p = p_new
            break
        p = p_new
    fl, _ = _side(p, rl, pl, gamma)
    fr, _ = _side(p, rr, pr, gamma)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, s, gamma=1.4):
    """Primitive (rho, u, p) of the solution at x/t = s (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    s = np.asarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)

    def one_side(mask, rk, uk, pk, sign):
        # sign = +1 for the left wave (moving left), -1 for the right wave;
        # written for the left side, mirrored for the right
        ck = math.sqrt(gamma * pk / rk)
        ss = sign * s
        uu = sign * uk
        usr = sign * us
        if ps > pk:  # shock
            rstar = rk * ((ps / pk + g1) / (ps / pk * g1 + 1.0))
            speed = uu - ck * math.sqrt((gamma + 1) / (2 * gamma) * ps / pk + (gamma - 1) / (2 * gamma))
            before = ss < speed
            r_ = np.where(before, rk, rstar)
            v_ = np.where(before, uu, usr)
            p_ = np.where(before, pk, ps)
        else:  # rarefaction
            cstar = ck * (ps / pk) ** ((gamma - 1) / (2 * gamma))
            head, tail = uu - ck, usr - cstar
            fan_u = 2.0 / (gamma + 1) * (ck + (gamma - 1) / 2 * uu + ss)
            fan_c = 2.0 / (gamma + 1) * (ck + (gamma - 1) / 2 * (uu - ss))
            fan_r = rk * (np.maximum(fan_c, 0.0) / ck) ** (2 / (gamma - 1))
            fan_p = pk * (np.maximum(fan_c, 0.0) / ck) ** (2 * gamma / (gamma - 1))
            rstar = rk * (ps / pk) ** (1 / gamma)
            r_ = np.where(ss < head, rk, np.where(ss > tail, rstar, fan_r))
            v_ = np.where(ss < head, uu, np.where(ss > tail, usr, fan_u))
            p_ = np.where(ss < head, pk, np.where(ss > tail, ps, fan_p))
        rho[mask] = r_[mask]
        u[mask] = sign * v_[mask]
        p[mask] = p_[mask]

    left_of_contact = s <= us
    one_side(left_of_contact, rl, ul, pl, 1.0)
    one_side(~left_of_contact, rr, ur, pr, -1.0)
    return rho, u, p
