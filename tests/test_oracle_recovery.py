"""Pins of the oracle's eigenframe recovery (Sec. 3, last paragraph) against
closed forms derived independently of the fixed-point iteration.

For a piecewise linear EOS p = a e + b the recovery condition
v (E + p(E - M v)) = M is the quadratic  -a M v^2 + ((1+a)E + b) v - M = 0,
whose physical root is v = 2M / (K + sqrt(K^2 - 4 a M^2)), K = (1+a)E + b
(v = M/(E+b) for a = 0).  For p = e/3 this is v = 3M/(2E + sqrt(4E^2-3M^2)).
"""
import math

import numpy as np
import pytest

from conftest import to_cons


def closed_form_v(E, M, branches):
    """branches: list of (a, b, e_lo, e_hi); returns v of the branch whose
    e = E - M v lies in [e_lo, e_hi]."""
    for a, b, lo, hi in branches:
        K = (1.0 + a) * E + b
        if M == 0.0:
            v = 0.0
        elif a == 0.0:
            v = M / K
        else:
            v = 2.0 * M / (K + math.sqrt(K * K - 4.0 * a * M * M))
        e = E - M * v
        if lo <= e <= hi:
            return v, e
    raise AssertionError("no branch")


def _samples(seed, n=400):
    rng = np.random.default_rng(seed)
    E = 10.0 ** rng.uniform(-6, 3, n)
    r = rng.uniform(0.0, 0.999, n)
    r[:5] = [0.0, 1e-12, 0.5, 0.99, 0.999]
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return E, r, d


def test_recovery_ideal_closed_form(orc):
    E, r, d = _samples(1)
    for Ei, ri, di in zip(E, r, d):
        M = ri * Ei
        res = orc.recover(Ei, *(M * di))
        v_ex, e_ex = closed_form_v(Ei, M, [(1 / 3, 0.0, -np.inf, np.inf)])
        assert res["converged"] and not res["clamped"] and not res["floored"]
        assert abs(res["v"] - v_ex) <= 2e-15 * max(v_ex, 1e-300) + 1e-300
        assert abs(res["e"] - e_ex) <= 1e-14 * Ei
        assert abs(res["p"] - res["e"] / 3.0) <= 1e-16 * Ei
        # velocity points along M (eq. cf-momentum)
        vel = np.array([res["vx"], res["vy"], res["vz"]])
        assert np.allclose(vel, res["v"] * di, rtol=0, atol=1e-15)


def test_recovery_bag_closed_form(orc_bag):
    o = orc_bag
    B, e_H = o.eos.B, o.eos.e_H
    e_Q = e_H + 4 * B
    p_c = e_H / 3
    branches = [(1 / 3, 0.0, -np.inf, e_H), (0.0, p_c, e_H, e_Q),
                (1 / 3, -4 * B / 3, e_Q, np.inf)]
    # EOS: continuity at both edges of the mixed phase
    assert o.pressure(e_H) == pytest.approx(p_c, rel=1e-15)
    assert o.pressure(e_Q) == pytest.approx(p_c, rel=1e-15)
    assert o.pressure(e_Q * 2) == pytest.approx((2 * e_Q - 4 * B) / 3, rel=1e-15)
    rng = np.random.default_rng(3)
    E = np.concatenate([10 ** rng.uniform(-3, 2, 300),
                        rng.uniform(0.5 * e_H, 2 * e_Q, 300)])
    r = rng.uniform(0, 0.99, E.size)
    hit = set()
    for Ei, ri in zip(E, r):
        M = ri * Ei
        res = o.recover(Ei, M, 0.0, 0.0)
        v_ex, e_ex = closed_form_v(Ei, M, branches)
        hit.add(0 if e_ex <= e_H else (1 if e_ex < e_Q else 2))
        assert res["converged"]
        assert abs(res["v"] - v_ex) <= 4e-15 * max(v_ex, 1e-300) + 1e-300
        assert abs(res["e"] - e_ex) <= 1e-14 * Ei
    assert hit == {0, 1, 2}


def test_guard_clamp_and_floor(orc):
    # |M| >= E: clamped to (1 - 1e-10) E, direction kept, counted
    res = orc.recover(1.0, 2.0, 0.0, 0.0)
    assert res["clamped"] == 1 and res["converged"]
    v_ex, _ = closed_form_v(1.0, 1.0 - 1e-10, [(1 / 3, 0.0, -np.inf, np.inf)])
    assert res["v"] == pytest.approx(v_ex, rel=1e-14) and res["v"] < 1.0
    # E <= 0: floored, still finite
    res = orc.recover(-1.0, 0.0, 0.0, 0.0)
    assert res["floored"] == 1 and res["v"] == 0.0 and math.isfinite(res["e"])


def test_prim_cons_round_trip(orc):
    rng = np.random.default_rng(5)
    n = 2000
    e = 10 ** rng.uniform(-4, 2, n)
    v = rng.uniform(0, 0.99, n)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    vel = v[:, None] * d
    nb = rng.uniform(0, 1, n)
    E, Mx, My, Mz, R = orc.prim_to_cons(e, vel[:, 0], vel[:, 1], vel[:, 2], nb)
    # eq. cf-energy: E = (e+p) gamma^2 - p, so E > |M| and E > 0
    assert np.all(E > np.sqrt(Mx ** 2 + My ** 2 + Mz ** 2))
    back = orc.cons_to_prim(E, Mx, My, Mz, R)
    g2 = 1 / (1 - v ** 2)
    assert np.allclose(back["e"], e, rtol=2e-14 * g2.max(), atol=0)
    for k, i in (("vx", 0), ("vy", 1), ("vz", 2)):
        assert np.allclose(back[k], vel[:, i], rtol=0, atol=1e-14)
    assert np.allclose(back["n"], nb, rtol=1e-12, atol=1e-15)
