"""Seeded synthetic initial states (primitive fields only).

This module is shared by the GPU path and by the CPU oracle in the tests.  It
holds none of the method's arithmetic: it only draws random numbers and
evaluates the prescribed initial profiles of e, v and n on the grid.  Each
side converts primitives to conserved fields with its own code.

Arrays are float64, shape (nz, ny, nx), x fastest.  Cell centres sit at
x_i = (i + 1/2 - N/2) dx on every axis, so the grid centre is a cell corner.

The paper measures on a sphere of constant energy density and on UrQMD Au+Au
initial states (Sec. 4); the latter are not available, so seeded sums of
Gaussian hot spots on grids of the paper's size (~200^3 cells, Sec. 3.1)
stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

HBARC = 0.1973269804  # GeV fm


@dataclass
class Primitive:
    e: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    n: np.ndarray

    @property
    def shape(self):
        return self.e.shape

    def as_tuple(self):
        return (self.e, self.vx, self.vy, self.vz, self.n)


def centres(N: int, dx: float) -> np.ndarray:
    return (np.arange(N, dtype=np.float64) + 0.5 - N / 2.0) * dx


def _zeros(shape):
    return np.zeros(shape, dtype=np.float64)


def shock_tube(dims=(64, 64, 64), dx=0.2, e_left=10.0, e_right=1.0,
               n_over_e=0.1, axis=0) -> Primitive:
    """Planar Riemann problem: e = e_left where the coordinate along `axis`
    is negative, e_right elsewhere; v = 0; n = n_over_e * e."""
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    coord = centres(dims[axis], dx)
    prof = np.where(coord < 0.0, e_left, e_right)
    bshape = [1, 1, 1]
    bshape[2 - axis] = dims[axis]
    e = np.broadcast_to(prof.reshape(bshape), shape).copy()
    return Primitive(e, _zeros(shape), _zeros(shape), _zeros(shape), n_over_e * e)


def ball(dims=(64, 64, 64), dx=0.2, radius=2.0, e_in=10.0, e_out=1.0,
         n_over_e=0.1) -> Primitive:
    """Sphere of constant energy density (the paper's 'ball' geometry)."""
    nx, ny, nz = dims
    X = centres(nx, dx)[None, None, :]
    Y = centres(ny, dx)[None, :, None]
    Z = centres(nz, dx)[:, None, None]
    r2 = X * X + Y * Y + Z * Z
    e = np.where(r2 < radius * radius, e_in, e_out) * np.ones((nz, ny, nx))
    shape = e.shape
    return Primitive(e, _zeros(shape), _zeros(shape), _zeros(shape), n_over_e * e)


def hotspot_list(rng: np.random.Generator, n_spots: int, dims, dx,
                 amp=(1.0, 20.0), radius=8.0):
    """Draw hot-spot centres uniformly inside the ellipsoid with semi-axes
    r_a = min(radius, N_a dx / 4) around the grid centre (rejection from the
    bounding box), and amplitudes uniform in [amp0, amp1]."""
    semi = np.array([min(radius, d * dx / 4.0) for d in dims], dtype=np.float64)
    cents = []
    while len(cents) < n_spots:
        c = rng.uniform(-1.0, 1.0, size=3)
        if float(np.dot(c, c)) <= 1.0:
            cents.append(c * semi)
    amps = rng.uniform(amp[0], amp[1], size=n_spots)
    return np.array(cents, dtype=np.float64), amps


def hotspots(dims=(200, 200, 200), dx=0.2, n_spots=64, seed=2, sigma=1.0,
             amp=(1.0, 20.0), radius=8.0, e_bg=1e-3, n_over_e=0.15,
             vz_profile=None) -> Primitive:
    """e = e_bg + sum_k A_k exp(-|x - c_k|^2 / (2 sigma^2)), v = 0 (or the
    longitudinal profile vz_profile(z)), n = n_over_e * e."""
    rng = np.random.default_rng(seed)
    cents, amps = hotspot_list(rng, n_spots, dims, dx, amp, radius)
    return hotspots_from_list(dims, dx, cents, amps, sigma, e_bg, n_over_e,
                              vz_profile)


def hotspots_from_list(dims, dx, cents, amps, sigma=1.0, e_bg=1e-3,
                       n_over_e=0.15, vz_profile=None) -> Primitive:
    nx, ny, nz = dims
    X, Y, Z = centres(nx, dx), centres(ny, dx), centres(nz, dx)
    e = np.full((nz, ny, nx), e_bg, dtype=np.float64)
    inv = 1.0 / (2.0 * sigma * sigma)
    for c, a in zip(cents, amps):
        gx = np.exp(-(X - c[0]) ** 2 * inv)
        gy = np.exp(-(Y - c[1]) ** 2 * inv)
        gz = np.exp(-(Z - c[2]) ** 2 * inv)
        e += a * (gz[:, None, None] * gy[None, :, None]) * gx[None, None, :]
    shape = e.shape
    vz = _zeros(shape)
    if vz_profile is not None:
        vz = np.broadcast_to(vz_profile(Z)[:, None, None], shape).copy()
    return Primitive(e, _zeros(shape), _zeros(shape), vz, n_over_e * e)


def longitudinal_flow(z: np.ndarray, scale=0.1, cap=0.9) -> np.ndarray:
    """v_z = sgn(z) min(tanh(scale |z|), cap)."""
    return np.sign(z) * np.minimum(np.tanh(scale * np.abs(z)), cap)


def bag_parameters(B_quarter_GeV=0.235, d_H=3.0, d_Q=37.0):
    """Bag constant B [GeV/fm^3] from B^{1/4} and the hadron-side edge of the
    mixed phase e_H = 3 B d_H / (d_Q - d_H) (massless pions / quark-gluon
    gas with the given degeneracies)."""
    B = B_quarter_GeV ** 4 / HBARC ** 3
    e_H = 3.0 * B * d_H / (d_Q - d_H)
    return B, e_H


def crossover_eos_table(n_nodes=48, B=None, e_c=1.0, width=1.0, e_max=1.0e3):
    """Synthetic tabled EOS (node energy densities, node pressures), GeV/fm^3.

    A smooth crossover from the massless gas p = e/3 to the bag-shifted
    plasma p = (e - 4B)/3: p(e) = e/3 - (4B/3) (s(e) - s(0)) with the step
    s(e) = (1 + tanh((e - e_c)/width)) / 2, sampled at e = 0 and at
    n_nodes - 1 log-spaced points in [1e-3, e_max].  For width >= 2B the
    slope dp/de stays in (0, 1/3], so the table is causal and p increases.
    """
    if B is None:
        B, _ = bag_parameters()
    e = np.concatenate([[0.0], np.geomspace(1e-3, e_max, n_nodes - 1)])
    step = lambda x: 0.5 * (1.0 + np.tanh((x - e_c) / width))
    p = e / 3.0 - (4.0 * B / 3.0) * (step(e) - step(0.0))
    return e, p


def steep_eos_table():
    """A causal table whose segments alternate soft and stiff slopes, up to
    dp/de = 3/4 (nodes in GeV/fm^3): the steepest EOS on which the
    recovery's fixed point is pinned to converge at the guard's largest
    |M|/E."""
    e = np.array([0.0, 0.5, 2.0, 10.0, 100.0, 1000.0])
    slopes = np.array([0.2, 0.75, 0.1, 0.75, 1.0 / 3.0])
    p = np.concatenate([[0.0], np.cumsum(slopes * np.diff(e))])
    return e, p


def bag_eos_table(B, e_H, e_top=1.0e3):
    """The bag model of bag_parameters() as a table: its break points e_H and
    e_Q = e_H + 4B plus one node far in the plasma phase (the last segment,
    extended, is the plasma line p = (e - 4B)/3)."""
    e_Q = e_H + 4.0 * B
    e = np.array([0.0, e_H, e_Q, e_top])
    p = np.array([0.0, e_H / 3.0, e_H / 3.0, (e_top - 4.0 * B) / 3.0])
    return e, p


# ---------------------------------------------------------------- workloads
# The five synthetic workloads, by name.  Each returns dims, dx, dt/dx, steps,
# precision, EOS, and a callable producing the primitive state.

def workload(name: str):
    if name == "shock64":
        dims = (64, 64, 64)
        return dict(name=name, dims=dims, dx=0.2, lam=0.4, steps=100,
                    precision="fp64", eos=("ideal", ()),
                    init=lambda: shock_tube(dims, 0.2))
    if name == "hotspots200":
        dims = (200, 200, 200)
        return dict(name=name, dims=dims, dx=0.2, lam=0.4, steps=500,
                    precision="fp64", eos=("ideal", ()),
                    init=lambda: hotspots(dims, 0.2, 64, seed=2))
    if name == "shock256_mixed":
        dims = (256, 256, 256)
        return dict(name=name, dims=dims, dx=0.2, lam=0.4, steps=100,
                    precision="fp32", eos=("ideal", ()),
                    init=lambda: shock_tube(dims, 0.2))
    if name == "batch96":
        evs = batch_events()
        return dict(name=name, dims=[ev["dims"] for ev in evs], dx=0.2, lam=0.4,
                    steps=200, precision="fp32", eos=("ideal", ()),
                    init=lambda: [ev["init"]() for ev in evs])
    if name == "bag400":
        dims = (400, 400, 400)
        B, e_H = bag_parameters()
        return dict(name=name, dims=dims, dx=0.1, lam=0.4, steps=300,
                    precision="fp32", eos=("bag", (B, e_H)),
                    init=lambda: hotspots(dims, 0.1, 64, seed=5,
                                          vz_profile=longitudinal_flow))
    raise KeyError(name)


def batch_events(n_events=96, sizes=(48, 64, 96, 128), seed0=4000, dx=0.2):
    """Uneven events: each axis length drawn from `sizes`, 8..32 hot spots,
    seed seed0 + k per event."""
    evs = []
    for k in range(n_events):
        rng = np.random.default_rng(seed0 + k)
        dims = tuple(int(s) for s in rng.choice(sizes, size=3))
        nsp = int(rng.integers(8, 33))
        cents, amps = hotspot_list(rng, nsp, dims, dx)
        evs.append(dict(dims=dims, n_spots=nsp,
                        init=(lambda d=dims, c=cents, a=amps:
                              hotspots_from_list(d, dx, c, a))))
    return evs
