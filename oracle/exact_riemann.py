"""Exact solution of the relativistic shock tube for p = e/3.

TEST INFRASTRUCTURE ONLY (like the rest of this package).  Independent of the
C oracle and of the GPU path: written from the textbook
theory of the one-dimensional relativistic Riemann problem for an
ultra-relativistic ideal gas (c_s^2 = 1/3), both states initially at rest,
e_L > e_R.  The solution is a left-moving rarefaction, a contact and a
right-moving shock.

  rarefaction:  artanh(v) = (sqrt(3)/4) ln(e_L / e)   (Riemann invariant)
                x/t = (v - c_s) / (1 - v c_s)         (C- characteristic)
  shock (Taub): v^2 = (p - p_R)(e - e_R) / ((e_R + p)(e + p_R))
                V_s = M* / (E* - E_R)                 (energy jump)
  baryons:      n ∝ e^{3/4} across the rarefaction (isentropic),
                N* = N_R V_s / (V_s - v*) behind the shock (baryon jump).
"""
from __future__ import annotations

import math

import numpy as np

CS = 1.0 / math.sqrt(3.0)


def v_rarefaction(e, e_left):
    return math.tanh(math.sqrt(3.0) / 4.0 * math.log(e_left / e))


def v_shock(e, e_right):
    p, pR = e / 3.0, e_right / 3.0
    return math.sqrt((p - pR) * (e - e_right) / ((e_right + p) * (e + pR)))


def star_state(e_left=10.0, e_right=1.0):
    lo, hi = e_right, e_left
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if v_rarefaction(mid, e_left) - v_shock(mid, e_right) > 0.0:
            lo = mid
        else:
            hi = mid
    e_star = 0.5 * (lo + hi)
    v_star = v_shock(e_star, e_right)
    p_star = e_star / 3.0
    g2 = 1.0 / (1.0 - v_star ** 2)
    E_star = (e_star + p_star) * g2 - p_star
    M_star = (e_star + p_star) * g2 * v_star
    V_s = M_star / (E_star - e_right)
    V_s_momentum = (M_star * v_star + p_star - e_right / 3.0) / M_star
    return dict(e=e_star, v=v_star, E=E_star, M=M_star, V_shock=V_s,
                V_shock_momentum=V_s_momentum,
                tail=(v_star - CS) / (1.0 - v_star * CS), head=-CS)


def solution(x, t, e_left=10.0, e_right=1.0, n_over_e=0.1):
    """Exact e, v, n at positions x (array) and time t > 0; the initial jump
    sits at x = 0."""
    st = star_state(e_left, e_right)
    xi = np.asarray(x, dtype=np.float64) / t
    e = np.empty_like(xi)
    v = np.empty_like(xi)
    n = np.empty_like(xi)
    nL, nR = n_over_e * e_left, n_over_e * e_right
    n_star_left = nL * (st["e"] / e_left) ** 0.75
    g_star = 1.0 / math.sqrt(1.0 - st["v"] ** 2)
    N_star = nR * st["V_shock"] / (st["V_shock"] - st["v"])
    n_star_right = N_star / g_star
    for i, s in enumerate(xi):
        if s <= st["head"]:
            e[i], v[i], n[i] = e_left, 0.0, nL
        elif s <= st["tail"]:
            vv = (s + CS) / (1.0 + s * CS)
            ee = e_left * math.exp(-4.0 / math.sqrt(3.0) * math.atanh(vv))
            e[i], v[i], n[i] = ee, vv, nL * (ee / e_left) ** 0.75
        elif s <= st["v"]:
            e[i], v[i], n[i] = st["e"], st["v"], n_star_left
        elif s <= st["V_shock"]:
            e[i], v[i], n[i] = st["e"], st["v"], n_star_right
        else:
            e[i], v[i], n[i] = e_right, 0.0, nR
    return e, v, n
