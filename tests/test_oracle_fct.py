"""Pins of the oracle's one-dimensional SHASTA operator (Sec. 3, eqs.
shasta-diff, shasta-geo, phoenical antidiffusion, flux limiter, eq.
shasta-n) against exact identities and textbook properties."""
import numpy as np
import pytest


def with_halo(u):
    """Outflow halo: three copies of each edge cell."""
    u = np.asarray(u, dtype=np.float64)
    return np.concatenate([[u[0]] * 3, u, [u[-1]] * 3])


def test_phoenical_identity_at_rest(orc):
    # With v = 0 the diffusion of eq. shasta-geo is 1/8 of the second
    # difference and the phoenical antiflux is exactly 1/8 Delta_j, so on data
    # where the limiter is inactive the step returns U unchanged.
    x = np.linspace(-1.0, 1.0, 48)
    for u in (np.tanh(x) + 2.0, 3.0 + x + 0.1 * x ** 3, np.exp(x)):
        out, _ = orc.fct_1d(with_halo(u), np.zeros(u.size + 6), None, 0.0)
        np.testing.assert_allclose(out[3:-3], u[3:-3], rtol=4e-16, atol=0)


@pytest.mark.parametrize("diff", [0.0, 0.25, 0.5, 1.0])
def test_antidiffusion_scale_at_rest(orc, diff):
    # At rest hat U = U + D2/8 (D2 = U_{j+1} - 2 U_j + U_{j-1}) and the
    # phoenical antiflux is diff/8 Delta_j; on smooth monotone data the
    # limiter is inactive, so U^{n+1} = U + (1 - diff) D2 / 8: diff = 0 is
    # the bare SHASTA diffusion with coefficient 1/8, diff = 1 removes it.
    x = np.linspace(-1.0, 1.0, 48)
    for u in (np.tanh(x) + 2.0, 3.0 + x + 0.1 * x ** 3, np.exp(x)):
        out, _ = orc.fct_1d(with_halo(u), np.zeros(u.size + 6), None, 0.0, diff=diff)
        d2 = u[4:-2] - 2.0 * u[3:-3] + u[2:-4]
        np.testing.assert_allclose(out[3:-3], u[3:-3] + (1.0 - diff) * d2 / 8.0,
                                   rtol=1e-15, atol=1e-15)


def test_step_at_rest_is_preserved_exactly(orc):
    # Hand-derived worked example: a step at rest gets hat U = (..,1/8,7/8,..)
    # and antiflux A = 1/8 at the jump, so U^{n+1} equals U^n exactly.
    u = np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.float64)
    out, flux = orc.fct_1d(with_halo(u), np.zeros(14), None, 0.0)
    assert np.array_equal(out, u)
    assert np.array_equal(flux, [0.0, 0.0])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("has_src", [False, True])
def test_boundary_flux_closes_the_sum(orc, seed, has_src):
    # Because Q+_j + Q-_{j+1} = 1, eq. shasta-geo is a flux difference; with
    # outflow halos the only fluxes left are eps_0 U_0 + lam f_0 at the left
    # and eps_{N-1} U_{N-1} + lam f_{N-1} at the right end.
    rng = np.random.default_rng(seed)
    N = 37
    u = rng.uniform(0.5, 2.0, N)
    lam = 0.4
    eps = lam * rng.uniform(-0.9, 0.9, N)
    f = rng.uniform(0.0, 1.0, N)
    out, flux = orc.fct_1d(with_halo(u), with_halo(eps),
                           with_halo(f) if has_src else None, lam)
    left = eps[0] * u[0] + (lam * f[0] if has_src else 0.0)
    right = eps[-1] * u[-1] + (lam * f[-1] if has_src else 0.0)
    assert out.sum() - u.sum() == pytest.approx(left - right, abs=1e-13 * N)
    assert flux == pytest.approx([left, right], abs=1e-15)


@pytest.mark.parametrize("eps", [0.2, -0.2, 0.05])
def test_passive_scalar_no_new_extrema(orc, eps):
    # Boris-Book: a square wave advected at constant Courant number keeps its
    # bounds and its total.
    N = 120
    u = np.zeros(N)
    u[45:60] = 1.0
    tot = u.sum()
    e = np.full(N + 6, eps)
    for _ in range(150):
        u, _ = orc.fct_1d(with_halo(u), e, None, 0.0)
        assert u.min() >= -1e-14 and u.max() <= 1.0 + 1e-14
    assert u.sum() == pytest.approx(tot, rel=1e-13)
    # centre of mass moved by eps per step (symmetric profile, no walls hit)
    com = (np.arange(N) * u).sum() / u.sum()
    assert com == pytest.approx(52.0 + 150 * eps, abs=0.05)
    # the wave stays sharp: >= 90% of the mass within the original width + 4
    c = int(round(com))
    assert u[c - 9:c + 10].sum() >= 0.9 * tot


def test_uniform_state_is_fixed_point(orc):
    # A uniform state at any velocity is invariant (no gradients, no source
    # difference): hat U = (Q+ + Q-) U with Q+ + Q- = 1 for constant eps.
    for eps in (0.0, 0.1, -0.23):
        out, _ = orc.fct_1d(np.full(26, 1.7), np.full(26, eps), np.full(26, 0.4), 0.4)
        np.testing.assert_allclose(out, 1.7, rtol=4e-16)
