"""Exact solution of the 1-D Riemann problem for the ideal-gas Euler equations.

Textbook construction (E. F. Toro, "Riemann Solvers and Numerical Methods for
Fluid Dynamics", ch. 4): the star pressure solves f_L(p) + f_R(p) + (u_R - u_L)
= 0 with shock (Rankine-Hugoniot) or rarefaction (isentropic) branches, and the
self-similar solution is sampled at x/t.  Used only as an independent pin of
the oracle (shock-tube convergence).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _f_branch(p, rho, pk, c, gamma):
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(left, right, gamma):
    """Return (p*, u*) for primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)

    def f(p):
        return _f_branch(p, rl, pl, cl, gamma) + _f_branch(p, rr, pr, cr, gamma) + (ur - ul)

    lo, hi = 1e-14, max(pl, pr)
    while f(hi) < 0.0:
        hi *= 2.0
    p_star = brentq(f, lo, hi, xtol=1e-15, rtol=1e-14, maxiter=500)
    u_star = 0.5 * (ul + ur) + 0.5 * (_f_branch(p_star, rr, pr, cr, gamma)
                                      - _f_branch(p_star, rl, pl, cl, gamma))
    return p_star, u_star


def sample(left, right, gamma, s):
    """Primitive solution (rho, u, p) at similarity coordinates s = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    ps, us = star_state(left, right, gamma)
    g1 = (gamma - 1.0) / (2.0 * gamma)
    g6 = (gamma - 1.0) / (gamma + 1.0)
    out = np.zeros((3, len(s)))
    for n, S in enumerate(np.asarray(s, dtype=float)):
        if S <= us:
            if ps > pl:
                SL = ul - cl * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl + g1)
                if S <= SL:
                    W = (rl, ul, pl)
                else:
                    W = (rl * (ps / pl + g6) / (g6 * ps / pl + 1.0), us, ps)
            else:
                SHL = ul - cl
                STL = us - cl * (ps / pl) ** g1
                if S <= SHL:
                    W = (rl, ul, pl)
                elif S >= STL:
                    W = (rl * (ps / pl) ** (1.0 / gamma), us, ps)
                else:
                    u = 2.0 / (gamma + 1.0) * (cl + 0.5 * (gamma - 1.0) * ul + S)
                    c = 2.0 / (gamma + 1.0) * (cl + 0.5 * (gamma - 1.0) * (ul - S))
                    W = (rl * (c / cl) ** (2.0 / (gamma - 1.0)), u,
                         pl * (c / cl) ** (2.0 * gamma / (gamma - 1.0)))
        else:
            if ps > pr:
                SR = ur + cr * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr + g1)
                if S >= SR:
                    W = (rr, ur, pr)
                else:
                    W = (rr * (ps / pr + g6) / (g6 * ps / pr + 1.0), us, ps)
            else:
                SHR = ur + cr
                STR = us + cr * (ps / pr) ** g1
                if S >= SHR:
                    W = (rr, ur, pr)
                elif S <= STR:
                    W = (rr * (ps / pr) ** (1.0 / gamma), us, ps)
                else:
                    u = 2.0 / (gamma + 1.0) * (-cr + 0.5 * (gamma - 1.0) * ur + S)
                    c = 2.0 / (gamma + 1.0) * (cr - 0.5 * (gamma - 1.0) * (ur - S))
                    W = (rr * (c / cr) ** (2.0 / (gamma - 1.0)), u,
                         pr * (c / cr) ** (2.0 * gamma / (gamma - 1.0)))
        out[:, n] = W
    return out
