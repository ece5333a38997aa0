"""Exact solution of the 1D Riemann problem for an ideal gas (test tool).

Written from the gas-dynamics definitions, independently of the oracle, to pin
it: the star pressure is the root of f(p) = f_L(p) + f_R(p) + (u_R - u_L) with
the exact wave curves

  shock (p > p_K):        f_K = (p - p_K) sqrt(A_K / (p + B_K)),
                          A_K = 2 / ((gamma+1) rho_K), B_K = (gamma-1)/(gamma+1) p_K
  rarefaction (p <= p_K): f_K = 2 c_K/(gamma-1) ((p/p_K)^((gamma-1)/(2 gamma)) - 1)

found by bracketing (scipy brentq) rather than Newton, and the self-similar
solution is sampled at x/t from the Rankine-Hugoniot and isentropic relations.
States are (rho, u, p) along the normal direction.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _fK(p, rho, pK, gamma):
    if p > pK:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        return (p - pK) * math.sqrt(A / (p + B))
    c = math.sqrt(gamma * pK / rho)
    return 2.0 * c / (gamma - 1.0) * ((p / pK) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def wave_function(p, L, R, gamma):
    return _fK(p, L[0], L[2], gamma) + _fK(p, R[0], R[2], gamma) + (R[1] - L[1])


def star(L, R, gamma=1.4, xtol=1e-15):
    """(p*, u*) of the exact solution.  L, R = (rho, u, p)."""
    cL = math.sqrt(gamma * L[2] / L[0])
    cR = math.sqrt(gamma * R[2] / R[0])
    if 2.0 / (gamma - 1.0) * (cL + cR) <= R[1] - L[1]:
        raise ValueError("vacuum is generated")
    lo = 1e-300
    hi = max(L[2], R[2])
    while wave_function(hi, L, R, gamma) < 0.0:
        hi *= 2.0
    p = brentq(lambda x: wave_function(x, L, R, gamma), lo, hi, xtol=1e-300, rtol=8.9e-16,
               maxiter=500)
    u = 0.5 * (L[1] + R[1]) + 0.5 * (_fK(p, R[0], R[2], gamma) - _fK(p, L[0], L[2], gamma))
    return p, u


def sample(L, R, xi, gamma=1.4, ps=None):
    """Exact (rho, u, p) at x/t = xi."""
    if ps is None:
        ps, us = star(L, R, gamma)
    else:
        ps, us = ps
    g = gamma
    if xi <= us:  # left of the contact
        rho, u, p = L
        c = math.sqrt(g * p / rho)
        if ps > p:
            S = u - c * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
            if xi <= S:
                return (rho, u, p)
            G = (g - 1) / (g + 1)
            return (rho * (ps / p + G) / (G * ps / p + 1.0), us, ps)
        head = u - c
        if xi <= head:
            return (rho, u, p)
        cs = c * (ps / p) ** ((g - 1) / (2 * g))
        tail = us - cs
        if xi > tail:
            return (rho * (ps / p) ** (1.0 / g), us, ps)
        uf = 2.0 / (g + 1) * (c + (g - 1) / 2.0 * u + xi)
        cf = 2.0 / (g + 1) * (c + (g - 1) / 2.0 * (u - xi))
        return (rho * (cf / c) ** (2.0 / (g - 1)), uf, p * (cf / c) ** (2.0 * g / (g - 1)))
    rho, u, p = R
    c = math.sqrt(g * p / rho)
    if ps > p:
        S = u + c * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
        if xi >= S:
            return (rho, u, p)
        G = (g - 1) / (g + 1)
        return (rho * (ps / p + G) / (G * ps / p + 1.0), us, ps)
    head = u + c
    if xi >= head:
        return (rho, u, p)
    cs = c * (ps / p) ** ((g - 1) / (2 * g))
    tail = us + cs
    if xi < tail:
        return (rho * (ps / p) ** (1.0 / g), us, ps)
    uf = 2.0 / (g + 1) * (-c + (g - 1) / 2.0 * u + xi)
    cf = 2.0 / (g + 1) * (c - (g - 1) / 2.0 * (u - xi))
    return (rho * (cf / c) ** (2.0 / (g - 1)), uf, p * (cf / c) ** (2.0 * g / (g - 1)))


def profile(L, R, x, t, x0=0.5, gamma=1.4):
    """Exact (rho, u, p) arrays at positions x and time t > 0."""
    st = star(L, R, gamma)
    out = np.array([sample(L, R, (xi - x0) / t, gamma, st) for xi in x])
    return out[:, 0], out[:, 1], out[:, 2]


def cell_averages(L, R, edges, t, x0=0.5, gamma=1.4, sub=16):
    """Exact cell averages of (rho, rho u, E) over cells [edges[i], edges[i+1]],
    by the midpoint rule on `sub` sub-cells (the exact solution is piecewise
    smooth, so this converges to the average)."""
    st = star(L, R, gamma)
    n = len(edges) - 1
    acc = np.zeros((3, n))
    for s in range(sub):
        xs = edges[:-1] + (s + 0.5) / sub * (edges[1:] - edges[:-1])
        vals = np.array([sample(L, R, (xi - x0) / t, gamma, st) for xi in xs])
        rho, u, p = vals[:, 0], vals[:, 1], vals[:, 2]
        acc[0] += rho
        acc[1] += rho * u
        acc[2] += p / (gamma - 1) + 0.5 * rho * u * u
    return acc / sub
