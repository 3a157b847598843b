"""Pins of the oracle's reductions (compensated sums, conservation ledger,
largest Courant number), of the exact shock-tube solution the physics pins
use, and of the convergence domain of the tabled EOS recovery."""
import json
import math
import os

import numpy as np
import pytest

from conftest import to_cons
from oracle import exact_riemann as er
from paper_1206_0919_amd import inputs

LAM = 0.4
DX = 0.2
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_sum_is_compensated(orc):
    # Terms that plain summation, and Kahan's compensation, lose: the exact
    # total is 2 (Neumaier's compensation keeps the small terms).
    assert orc.total(np.array([1e16, 1.0, -1e16, 1.0])) == 2.0
    assert orc.total(np.array([1.0, 1e100, 1.0, -1e100])) == 2.0
    rng = np.random.default_rng(3)
    a = rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, 10000)
    assert orc.total(a) == pytest.approx(math.fsum(a), rel=1e-15, abs=1e-300)


def _pencil_shock_tubes(jumps, N=16):
    """One x pencil per (e_left, e_right): e at rest, jump at the centre."""
    ny, nz = 2, len(jumps) // 2
    e = np.empty((nz, ny, N))
    for k, (eL, eR) in enumerate(jumps):
        y, z = k % ny, k // ny
        e[z, y] = np.where(np.arange(N) < N // 2, eL, eR)
    z0 = np.zeros_like(e)
    return inputs.Primitive(e, z0, z0, z0, 0.1 * e)


def test_ledger_sum_over_pencils_is_compensated(orc):
    # Before waves reach the faces, the M_x outflow of a pencil at rest is
    # lambda (p_R - p_L).  Pencils of wildly different scale cancel in the
    # ledger's sum over pencils: it must equal the exactly rounded sum of the
    # pencils' own ledgers (naive summation loses the O(1) pencils).
    jumps = [(3e16, 3.0), (3.0, 6.0), (3.0, 3e16), (3.0, 6.0)]
    U = to_cons(orc, _pencil_shock_tubes(jumps))
    single = []
    for eL, eR in jumps:
        V = to_cons(orc, _pencil_shock_tubes([(eL, eR), (eL, eR)]))
        V = [np.ascontiguousarray(a[:1, :1]) for a in V]
        led, _, _ = orc.sweep(V, 0, LAM)
        single.append(led[1])
    ledger, _, _ = orc.sweep(U, 0, LAM)
    exact = math.fsum(single)
    assert abs(exact) < 10.0   # the large pencils cancel
    assert ledger[1] == exact


def test_max_eps_is_the_corrector_courant_number(orc):
    # Uniform flow is steady, so the half-step velocity equals the initial one
    # and the largest |lambda v_d| over the sweeps of a step is lambda max|v_i|
    # (the predictor's lambda/2 would halve it).
    dims = (8, 7, 6)
    shape = dims[::-1]
    e = np.full(shape, 2.0)
    v = (0.21, -0.47, 0.3)
    prim = inputs.Primitive(e, *(np.full(shape, c) for c in v), 0.3 * e)
    U = to_cons(orc, prim)
    _, maxeps, _ = orc.run(U, LAM, 1)
    assert maxeps == pytest.approx(LAM * 0.47, rel=1e-14)


def test_exact_shock_tube_jump_conditions():
    # Rankine-Hugoniot at the shock for energy, momentum and baryon number
    # with one shock speed, and the rarefaction's Riemann invariant at the
    # star state: fixes the Taub relation and the rarefaction law.
    st = er.star_state(10.0, 1.0)
    eR, pR = 1.0, 1.0 / 3.0
    e, v = st["e"], st["v"]
    p = e / 3.0
    g2 = 1.0 / (1.0 - v * v)
    E, M = (e + p) * g2 - p, (e + p) * g2 * v
    Vs = st["V_shock"]
    assert Vs * (E - eR) == pytest.approx(M, rel=1e-13)                 # energy
    assert Vs * M == pytest.approx(M * v + p - pR, rel=1e-13)           # momentum
    assert st["V_shock_momentum"] == pytest.approx(Vs, rel=1e-12)
    nR = 0.1 * eR
    N_star = nR * Vs / (Vs - v)
    assert Vs * (N_star - nR) == pytest.approx(N_star * v, rel=1e-13)    # baryons
    assert math.atanh(v) == pytest.approx(math.sqrt(3.0) / 4.0 * math.log(10.0 / e),
                                          rel=1e-13)
    assert 0.0 < v < Vs < 1.0 and eR < e < 10.0


def test_exact_shock_tube_conserves_energy_and_momentum():
    # The exact profile at time t, integrated over a box the waves have not
    # left, holds the initial energy, and its momentum grew by t (p_L - p_R)
    # (the pressure difference across the box).  Fixes the fan, the plateau
    # and the shock position together.
    t = 4.0
    x = np.linspace(-4.0, 4.0, 2_000_001)
    e, v, n = er.solution(x, t)
    p = e / 3.0
    g2 = 1.0 / (1.0 - v * v)
    E, M = (e + p) * g2 - p, (e + p) * g2 * v
    w = np.full(x.size, x[1] - x[0])
    w[0] = w[-1] = 0.5 * w[0]
    E0 = 10.0 * 4.0 + 1.0 * 4.0
    assert (w * E).sum() == pytest.approx(E0, rel=2e-6)
    assert (w * M).sum() == pytest.approx(t * (10.0 - 1.0) / 3.0, rel=2e-6)
    N0 = 0.1 * 10.0 * 4.0 + 0.1 * 1.0 * 4.0
    assert (w * n * np.sqrt(g2)).sum() == pytest.approx(N0, rel=2e-6)


def test_exact_shock_tube_star_state_golden():
    with open(os.path.join(GOLDEN, "shock_tube_star.json")) as fh:
        g = json.load(fh)
    st = er.star_state(10.0, 1.0)
    for k in ("e", "v", "E", "M", "V_shock"):
        key = k if k == "V_shock" else f"{k}_star"
        assert st[k] == pytest.approx(g[key], rel=1e-13)
    # ten digits quoted in the survey of the method's test cases
    assert g["e_star"] == pytest.approx(3.1398315582, abs=1e-10)
    assert g["v_star"] == pytest.approx(0.4633814654, abs=1e-10)
    assert g["V_shock"] == pytest.approx(0.7521153854, abs=1e-10)


def test_table_fixed_point_converges_at_steepest_slope():
    # The fixed point v <- M / (E + p(E - M v)) contracts by p'(e) v^2 <= the
    # slope per iteration, so with slopes <= 3/4 the 200 iterations reach the
    # 2^-50 step even at the guard's largest |M|/E.
    import oracle
    te = np.array([0.0, 1.0, 5.0])
    tp = np.array([0.0, 0.75, 3.75])
    o = oracle.Oracle(oracle.EOS_TABLE, table=(te, tp))
    for E, r in ((1.0, 1.0 - 1e-10), (3.0, 0.999999), (50.0, 0.99), (0.5, 0.9)):
        res = o.recover(E, r * E, 0.0, 0.0)
        assert res["converged"] and res["iters"] <= 200
        K = 1.75 * E
        v_ex = 2.0 * (r * E) / (K + math.sqrt(K * K - 3.0 * (r * E) ** 2))
        assert res["v"] == pytest.approx(v_ex, rel=1e-13)
