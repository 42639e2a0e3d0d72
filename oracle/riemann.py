"""Exact solution of the 1D Euler Riemann problem (ideal gas).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper cites Toro's book for approximate Riemann solvers (Section 2.2); the
exact solver of that book (star-region pressure from the two wave functions,
then sampling of the self-similar solution) provides a closed form that pins
the discrete scheme on shock tubes.  Written from the mathematics:

* wave function of side K at pressure p:
    shock (p > p_K):       (p - p_K) sqrt(A_K / (p + B_K)),
                            A_K = 2 / ((gamma + 1) rho_K), B_K = p_K (gamma - 1) / (gamma + 1)
    rarefaction (p <= p_K): 2 c_K / (gamma - 1) ((p / p_K)^((gamma - 1) / (2 gamma)) - 1)
* p* solves f_L(p) + f_R(p) + (u_R - u_L) = 0 (Newton's method),
  u* = (u_L + u_R) / 2 + (f_R(p*) - f_L(p*)) / 2;
* shocks move with the Rankine-Hugoniot speed, rarefactions are centred fans.
"""
from __future__ import annotations

import math

import numpy as np


def _wave(p, rho_k, p_k, c_k, g):
    if p > p_k:
        A = 2.0 / ((g + 1.0) * rho_k)
        B = p_k * (g - 1.0) / (g + 1.0)
        s = math.sqrt(A / (p + B))
        return (p - p_k) * s, s * (1.0 - 0.5 * (p - p_k) / (B + p))
    r = p / p_k
    f = 2.0 * c_k / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho_k * c_k) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma=1.4, tol=1e-15, maxit=200):
    """(p*, u*) of the Riemann problem; raises if a vacuum would form."""
    g = gamma
    c_l = math.sqrt(g * p_l / rho_l)
    c_r = math.sqrt(g * p_r / rho_r)
    if 2.0 * (c_l + c_r) / (g - 1.0) <= u_r - u_l:
        raise ValueError("vacuum generated")
    p = 0.5 * (p_l + p_r) - 0.125 * (u_r - u_l) * (rho_l + rho_r) * (c_l + c_r)
    p = max(p, 1e-10 * min(p_l, p_r))
    for _ in range(maxit):
        fl, dl = _wave(p, rho_l, p_l, c_l, g)
        fr, dr = _wave(p, rho_r, p_r, c_r, g)
        pn = p - (fl + fr + u_r - u_l) / (dl + dr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _wave(p, rho_l, p_l, c_l, g)
    fr, _ = _wave(p, rho_r, p_r, c_r, g)
    u = 0.5 * (u_l + u_r) + 0.5 * (fr - fl)
    return p, u


def star_densities(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma=1.4):
    p, u = star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma)
    return p, u, _star_rho(p, rho_l, p_l, gamma), _star_rho(p, rho_r, p_r, gamma)


def _star_rho(p, rho_k, p_k, g):
    if p > p_k:
        G6 = (g - 1.0) / (g + 1.0)
        r = p / p_k
        return rho_k * (r + G6) / (G6 * r + 1.0)
    return rho_k * (p / p_k) ** (1.0 / g)


def sample(xi, rho_l, u_l, p_l, rho_r, u_r, p_r, gamma=1.4):
    """(rho, u, p) of the self-similar solution at xi = (x - x0) / t (arrays)."""
    g = gamma
    ps, us = star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, g)
    c_l = math.sqrt(g * p_l / rho_l)
    c_r = math.sqrt(g * p_r / rho_r)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for idx, s in np.ndenumerate(xi):
        if s <= us:
            if ps > p_l:
                S = u_l - c_l * math.sqrt((g + 1.0) / (2.0 * g) * ps / p_l + (g - 1.0) / (2.0 * g))
                w = (rho_l, u_l, p_l) if s <= S else (_star_rho(ps, rho_l, p_l, g), us, ps)
            else:
                shead = u_l - c_l
                cs = c_l * (ps / p_l) ** ((g - 1.0) / (2.0 * g))
                stail = us - cs
                if s <= shead:
                    w = (rho_l, u_l, p_l)
                elif s > stail:
                    w = (_star_rho(ps, rho_l, p_l, g), us, ps)
                else:
                    c = 2.0 / (g + 1.0) * (c_l + 0.5 * (g - 1.0) * (u_l - s))
                    w = (rho_l * (c / c_l) ** (2.0 / (g - 1.0)),
                         2.0 / (g + 1.0) * (c_l + 0.5 * (g - 1.0) * u_l + s),
                         p_l * (c / c_l) ** (2.0 * g / (g - 1.0)))
        else:
            if ps > p_r:
                S = u_r + c_r * math.sqrt((g + 1.0) / (2.0 * g) * ps / p_r + (g - 1.0) / (2.0 * g))
                w = (rho_r, u_r, p_r) if s >= S else (_star_rho(ps, rho_r, p_r, g), us, ps)
            else:
                shead = u_r + c_r
                cs = c_r * (ps / p_r) ** ((g - 1.0) / (2.0 * g))
                stail = us + cs
                if s >= shead:
                    w = (rho_r, u_r, p_r)
                elif s <= stail:
                    w = (_star_rho(ps, rho_r, p_r, g), us, ps)
                else:
                    c = 2.0 / (g + 1.0) * (c_r - 0.5 * (g - 1.0) * (u_r - s))
                    w = (rho_r * (c / c_r) ** (2.0 / (g - 1.0)),
                         2.0 / (g + 1.0) * (-c_r + 0.5 * (g - 1.0) * u_r + s),
                         p_r * (c / c_r) ** (2.0 * g / (g - 1.0)))
        rho[idx], u[idx], p[idx] = w
    return rho, u, p
