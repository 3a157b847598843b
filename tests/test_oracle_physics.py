"""Pins of the oracle's 3+1D time step against the exact relativistic shock
tube, conservation, axis-permutation invariance and spherical symmetry."""
import numpy as np
import pytest

from oracle import exact_riemann as er
from conftest import to_cons
from paper_1206_0919_amd import inputs

LAM = 0.4
DX = 0.2
DT = LAM * DX  # 0.08 fm/c: 200 steps = 16 fm/c (Sec. 4)


def _shock_profile(orc, steps, dims=(64, 2, 2)):
    U = to_cons(orc, inputs.shock_tube(dims, DX))
    orc.run(U, LAM, steps)
    P = orc.cons_to_prim(*U)
    sh = U[0].shape
    return {k: P[k].reshape(sh)[0, 0] for k in ("e", "vx", "n")}, U


@pytest.mark.parametrize("steps", [50, 100])
def test_shock_tube_vs_exact(orc, steps):
    prof, _ = _shock_profile(orc, steps)
    t = steps * DT
    xc = inputs.centres(64, DX)
    e_ex, v_ex, n_ex = er.solution(xc, t)
    st = er.star_state()
    L1 = lambda a, b: np.abs(a - b).sum() / np.abs(b).sum()
    assert L1(prof["e"], e_ex) <= 0.03
    assert L1(prof["n"], n_ex) <= 0.03
    assert L1(prof["vx"], v_ex) <= (0.07 if steps == 50 else 0.04)
    plateau = (xc > st["tail"] * t + 0.2) & (xc < st["V_shock"] * t - 0.4)
    assert plateau.sum() >= 10
    assert prof["e"][plateau].mean() == pytest.approx(st["e"], rel=0.01)
    assert prof["vx"][plateau].mean() == pytest.approx(st["v"], rel=0.01)
    # shock position: where e crosses the mean of e* and e_R
    half = 0.5 * (st["e"] + 1.0)
    e = prof["e"]
    i = np.where((e[:-1] > half) & (e[1:] <= half))[0][-1]
    xs = xc[i] + (e[i] - half) / (e[i] - e[i + 1]) * DX
    assert abs(xs - st["V_shock"] * t) <= 2 * DX
    # nearly undisturbed states beyond the waves (the scheme's precursors
    # decay exponentially ahead of each front)
    assert np.all(np.abs(e[xc < st["head"] * t - 1.0] - 10.0) < 0.01)
    assert np.all(np.abs(e[xc > st["V_shock"] * t + 0.5] - 1.0) < 1e-6)


def test_shock_tube_boundary_pressure_flux(orc):
    # Before any wave reaches a wall, each x sweep changes sum M_x of a pencil
    # by exactly lambda (p_L - p_R) (the pressure flux through the two outflow
    # faces), while sum E and sum R stay fixed.
    U = to_cons(orc, inputs.shock_tube((64, 2, 2), DX))
    E0, R0 = orc.total(U[0]), orc.total(U[4])
    steps = 30
    orc.run(U, LAM, steps)
    per_pencil = orc.total(U[1]) / 4
    assert per_pencil == pytest.approx(steps * LAM * (10.0 / 3 - 1.0 / 3), rel=1e-14)
    assert orc.total(U[0]) == pytest.approx(E0, rel=1e-14)
    assert orc.total(U[4]) == pytest.approx(R0, rel=1e-14)
    assert np.all(U[2] == 0.0) and np.all(U[3] == 0.0)


def test_planar_invariance_bitwise(orc):
    # x-, y- and z-planar versions of the shock tube give identical profiles:
    # sweeps across a planar state with no transverse velocity are exact
    # identities, whatever their order in the permutation cycle.
    steps = 25
    runs = []
    for axis, dims in ((0, (48, 3, 2)), (1, (2, 48, 3)), (2, (3, 2, 48))):
        U = to_cons(orc, inputs.shock_tube(dims, DX, axis=axis))
        orc.run(U, LAM, steps)
        mom = U[1 + axis]
        line = [np.moveaxis(a, 2 - axis, 2).reshape(-1, 48) for a in (U[0], mom, U[4])]
        for a in line:
            assert np.all(a == a[0])  # planar: every pencil identical
        for q in range(3):
            if q != axis:
                assert np.all(U[1 + q] == 0.0)
        runs.append([a[0] for a in line])
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert np.array_equal(a, b)


def _random_state(orc, dims, seed):
    rng = np.random.default_rng(seed)
    pr = inputs.hotspots(dims, DX, 6, seed=seed, radius=8.0)
    shape = pr.e.shape
    v = rng.uniform(-0.3, 0.3, (3,) + shape)
    return to_cons(orc, inputs.Primitive(pr.e, v[0], v[1], v[2], pr.n))


@pytest.mark.parametrize("pair", [(0, 1), (0, 2), (1, 2)])
def test_sweep_axis_permutation_equivariance(orc, pair):
    a, b = pair
    U = _random_state(orc, (14, 12, 10), 11)
    # swapping grid axes a and b of a (z, y, x) array
    ta, tb = 2 - a, 2 - b
    perm = [0, 1, 2]
    perm[ta], perm[tb] = perm[tb], perm[ta]
    T = [np.ascontiguousarray(x.transpose(perm)) for x in U]
    T[1 + a], T[1 + b] = T[1 + b], T[1 + a]
    la, _, _ = orc.sweep(U, a, LAM)
    lb, _, _ = orc.sweep(T, b, LAM)
    back = [np.ascontiguousarray(x.transpose(perm)) for x in T]
    back[1 + a], back[1 + b] = back[1 + b], back[1 + a]
    for q in range(5):
        assert np.array_equal(U[q], back[q])
    lb = list(lb)
    lb[1 + a], lb[1 + b] = lb[1 + b], lb[1 + a]
    np.testing.assert_allclose(la, lb, rtol=1e-15, atol=1e-15)


def test_conservation_ledger(orc):
    # sum U(t) + accumulated boundary outflow = sum U(0) for all five fields,
    # with waves crossing the outflow boundaries of an anisotropic grid.
    U = _random_state(orc, (24, 20, 16), 7)
    s0 = np.array([orc.total(x) for x in U])
    scale = np.array([orc.total(np.abs(x)) for x in U])
    ledger, maxeps, cnt = orc.run(U, LAM, 30)
    s1 = np.array([orc.total(x) for x in U])
    assert np.all(np.abs(ledger) > 1e-3 * scale)  # fluxes really left the box
    np.testing.assert_allclose(s1 + ledger - s0, 0.0, atol=1e-12 * scale.max())
    assert 0 < maxeps < 0.5 and cnt[:3] == [0, 0, 0]


def test_ball_mirror_symmetry_bitwise(orc):
    # Expanding sphere of r = 2 fm: the grid and the scheme are symmetric
    # under each reflection x -> -x (with M_x -> -M_x), exactly.
    U = to_cons(orc, inputs.ball((32, 30, 28), DX, radius=2.0))
    orc.run(U, LAM, 20)
    E, Mx, My, Mz, R = U
    for ax, M in ((2, Mx), (1, My), (0, Mz)):
        for F in (E, R):
            assert np.array_equal(F, np.flip(F, ax))
        assert np.array_equal(M, -np.flip(M, ax))
        for Mo in (Mx, My, Mz):
            if Mo is not M:
                assert np.array_equal(Mo, np.flip(Mo, ax))


def test_ball_isotropy_bounded(orc):
    # Parity unpinned: dimensional splitting breaks the x<->y symmetry of the
    # sphere slightly (the axis order differs); the deviation stays small and
    # the radial outflow is monotone in |M| near the front.
    U = to_cons(orc, inputs.ball((32, 32, 32), DX, radius=2.0))
    orc.run(U, LAM, 20)
    E = U[0]
    assert np.abs(E - E.transpose(0, 2, 1)).max() <= 0.05 * E.max()
    assert np.abs(E - E.transpose(2, 1, 0)).max() <= 0.05 * E.max()


def test_schedule_is_listing_2_table(orc):
    # permutation table of the enqueueing listing (Appendix A)
    table = [0, 1, 2, 0, 2, 1, 2, 0, 1, 2, 1, 0, 1, 2, 0, 1, 0, 2]
    got = [orc.axis_of(k, w) for k in range(12) for w in range(3)]
    assert got == table + table


def test_thread_count_does_not_change_results(orc):
    U1 = _random_state(orc, (20, 18, 16), 3)
    U8 = [x.copy() for x in U1]
    l1, _, _ = orc.run(U1, LAM, 4, nthreads=1)
    l8, _, _ = orc.run(U8, LAM, 4, nthreads=8)
    for a, b in zip(U1, U8):
        assert np.array_equal(a, b)
    assert np.array_equal(l1, l8)


def test_uniform_flow_is_steady_through_outflow_faces(orc):
    # A uniform state moving obliquely through the box is steady: every ghost
    # cell repeats its edge cell, so each pencil with its halo is uniform and
    # the sweep returns it unchanged (the geometric factors sum to one), also
    # in the cells next to the faces where the flow leaves or enters.
    dims = (10, 9, 8)
    shape = dims[::-1]
    e = np.full(shape, 1.3)
    prim = inputs.Primitive(e, np.full(shape, 0.31), np.full(shape, -0.22),
                            np.full(shape, 0.13), 0.4 * e)
    U = to_cons(orc, prim)
    U0 = [a.copy() for a in U]
    ledger, maxeps, cnt = orc.run(U, LAM, 6)
    for a, b in zip(U, U0):
        np.testing.assert_allclose(a, b, rtol=1e-14, atol=0)
    assert cnt[:3] == [0, 0, 0]


def _sweep_by_parts(orc, U, lam):
    """One x sweep of a single pencil assembled from separately pinned parts:
    the halo as numpy's edge padding (three copies of the edge cell), the
    recovery of each padded cell, and the one-dimensional FCT operator."""
    pad = lambda a: np.pad(a, 3, mode="edge")

    guards = [0, 0]   # clamped, floored: interior cells of both time levels

    def level(V):
        Vp = [pad(a) for a in V]
        rec = [orc.recover(Vp[0][i], Vp[1][i], Vp[2][i], Vp[3][i], Vp[4][i])
               for i in range(Vp[0].size)]
        for r in rec[3:-3]:
            guards[0] += r["clamped"]
            guards[1] += r["floored"]
        v = np.array([r["vx"] for r in rec])
        p = np.array([r["p"] for r in rec])
        return Vp, v, p

    Up, v, p = level(U)
    half = [orc.fct_1d(Up[q], 0.5 * lam * v, (p * v if q == 0 else p) if q in (0, 1) else None,
                       0.5 * lam)[0] for q in range(5)]
    _, vh, ph = level(half)
    return [orc.fct_1d(Up[q], lam * vh, (ph * vh if q == 0 else ph) if q in (0, 1) else None,
                       lam)[0] for q in range(5)], guards


def test_sweep_is_the_composition_of_its_parts(orc):
    # Pins the halo rule (three ghost cells copying the edge cell, before each
    # half step) and the time levels of the sweep, including the cells next
    # to the outflow faces, where the limiter reads the outermost ghost.
    rng = np.random.default_rng(31)
    N = 18
    e = 1.0 + 9.0 * rng.uniform(size=N) ** 3
    vx = rng.uniform(-0.6, 0.6, N)
    vy = rng.uniform(-0.2, 0.2, N)
    z = np.zeros(N)
    U = [a.reshape(1, 1, N) for a in orc.prim_to_cons(e, vx, vy, z, 0.2 * e)]
    want, guards = _sweep_by_parts(orc, [a.ravel() for a in U], LAM)
    _, _, cnt = orc.sweep(U, 0, LAM)
    for q in range(5):
        assert np.array_equal(U[q].ravel(), want[q])
    assert guards == [0, 0] and cnt[:3] == [0, 0, 0]


def test_guard_counts_interior_cells_of_both_levels(orc):
    # Inadmissible conserved states (E <= 0 at one face, |M| >= E at the other
    # face and inside): the guard acts inside the recovery only, so the fields
    # follow the same composition of parts, and each interior cell counts
    # once per time level (the ghost copies of a guarded edge cell do not).
    rng = np.random.default_rng(5)
    N = 16
    E = 1.0 + rng.uniform(size=N)
    Mx = rng.uniform(-0.5, 0.5, N) * E
    Mx[[3, 9, N - 1]] = [1.2 * E[3], -1.0 * E[9], 1.5 * E[N - 1]]
    E[0] = -0.3
    U = [a.reshape(1, 1, N).copy() for a in (E, Mx, np.zeros(N), np.zeros(N), 0.1 * np.abs(E))]
    want, guards = _sweep_by_parts(orc, [a.ravel() for a in U], LAM)
    _, _, cnt = orc.sweep(U, 0, LAM)
    for q in range(5):
        assert np.array_equal(U[q].ravel(), want[q])
    assert guards[0] >= 3 and guards[1] >= 1
    assert cnt[:2] == guards
