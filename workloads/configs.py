"""The five workloads of the build, as seeded generators.

Each generator takes an optional size reduction so the same recipe yields the
parity-test case (small enough for the FP64 oracle) and the full-size case.
Defaults: tau = 1, rest state f = 0, Ricker period 40 and delay 60, unit
amplitude, "vertical" means direction (0, +1) (down, into the solid).

Lame units: mu = rho0 * 0.2^2 (the stated S-wave speed 0.2 fixes the unit of
lambda and mu; only lambda/mu enters the lattice scheme).

Free surfaces use the zero-order extrapolation (BC_FREE0) by default: the
printed linear extrapolation makes short surface modes grow at every tau, which
the long runs of these workloads would amplify from rounding noise. Layered
media draw lambda so that the Poisson ratio stays in [0.1, 0.33], the range in
which the step with that surface and tau = 1 has spectral radius <= 1.
"""
from __future__ import annotations

import numpy as np

from .problem import (BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source,
                      default_sponge_profile, ring_receivers, row_receivers)

CONFIG_NAMES = ("plain_small", "plain_large", "hbm_scale", "batched_shots",
                "adjoint_shots")

MU_UNIT = 0.04  # rho0 * 0.2^2


def lame_from_poisson(nu: float, mu: float = MU_UNIT):
    """lambda for a given Poisson ratio nu = lambda / (2 (lambda + mu))."""
    return 2.0 * nu * mu / (1.0 - 2.0 * nu), mu


def plain_small(n: int = 128, nsteps: int = 600, dtype: str = "f64",
                nu: float = 0.25, tau: float = 1.0) -> Problem:
    """128x128 periodic box, homogeneous Poisson solid, centred x-directed
    Gaussian force (sigma 4), 16 receivers on a radius-30 ring."""
    lam, mu = lame_from_poisson(nu)
    c = n / 2.0
    radius = 30.0 * n / 128.0
    return Problem(
        nx=n, ny=n, bc=(BC_PERIODIC,) * 4,
        medium=Medium("homogeneous", lam, mu, 1.0), tau=tau,
        sources=[Source(c, c, 4.0, 1.0, 0.0, 1.0, 40.0, 60.0)],
        receivers=ring_receivers(c, c, radius, 16), comp_mask=3,
        nsteps=nsteps, dtype=dtype, name="plain_small")


def _sponged(nx, ny, thick, bottom_bc=BC_RIGID, top_bc=BC_FREE0):
    prof = default_sponge_profile(thick)
    return dict(bc=(top_bc, bottom_bc, BC_PERIODIC, BC_PERIODIC),
                sponge_thick=(0, thick, thick, thick),
                sponge_profiles=(None, prof, prof, prof))


def plain_large(n: int = 4096, nsteps: int = 12000, dtype: str = "f32",
                nu: float = 0.33, sponge: int = 96, src_depth: int = 20,
                top_bc: int = BC_FREE0) -> Problem:
    """Free surface on top, sponges on the other three sides (bottom rigid
    behind its sponge, sides periodic behind theirs), homogeneous nu = 0.33,
    vertical source sigma 3 at depth 20, a receiver on every surface cell
    recording v_y (the Rayleigh-wave case)."""
    lam, mu = lame_from_poisson(nu)
    return Problem(
        nx=n, ny=n, medium=Medium("homogeneous", lam, mu, 1.0), tau=1.0,
        sources=[Source(n / 2.0, float(src_depth), 3.0, 0.0, 1.0, 1.0, 40.0, 60.0)],
        receivers=row_receivers(n, 0), comp_mask=2, nsteps=nsteps, dtype=dtype,
        name="plain_large", **_sponged(n, n, sponge, top_bc=top_bc))


def _layers(rng, ny: int, nlayers: int):
    rows = ny // nlayers
    lam = np.empty(ny)
    mu = np.empty(ny)
    for l in range(nlayers):
        m = rng.uniform(0.036, 0.044)
        a = rng.uniform(0.011, 0.0684)      # nu in [0.1, 0.33]
        lo = l * rows
        hi = ny if l == nlayers - 1 else (l + 1) * rows
        lam[lo:hi] = a
        mu[lo:hi] = m
    return lam, mu


def hbm_scale(n: int = 16384, nsteps: int = 4000, dtype: str = "f32",
              sponge: int = 128, seed: int = 3, src_seed: int = 33) -> Problem:
    """8 horizontal layers with seeded lambda, mu (nu in [0, 0.33]), a rigid
    interface at depth 12000/16384 of the grid, free surface on top, sponges
    on the other sides, 3 seeded vertical sources."""
    rng = np.random.default_rng(seed)
    lam, mu = _layers(rng, n, 8)
    rigid_row = int(round(12000 * n / 16384))
    srng = np.random.default_rng(src_seed)
    srcs = []
    x_lo = max(1, int(round(160 * n / 16384)))
    for _ in range(3):
        x = float(srng.integers(x_lo, n - x_lo))
        y = float(srng.integers(20, max(21, rigid_row - 33)))
        srcs.append(Source(x, y, 3.0, 0.0, 1.0, 1.0, 40.0, 60.0))
    return Problem(
        nx=n, ny=n, medium=Medium("layered", lam, mu, np.ones(n)), tau=1.0,
        rigid_row=rigid_row, sources=srcs, nsteps=nsteps, dtype=dtype,
        comp_mask=2, name="hbm_scale", **_sponged(n, n, sponge))


def batched_shots(count: int = 512, nsteps: int = 3000, dtype: str = "f32",
                  seed: int = 4, sponge: int = 64, sides=None):
    """count independent grids, square side 256 + 64 U{0..28} (seeded), each
    with its own 8-layer medium, free top, 64-cell sponges, one source."""
    rng = np.random.default_rng(seed)
    if sides is None:
        sides = 256 + 64 * rng.integers(0, 29, size=count)
    probs = []
    for g, s in enumerate(sides):
        s = int(s)
        grng = np.random.default_rng(4000 + g)
        lam, mu = _layers(grng, s, 8)
        edge = min(80, s // 4)
        x = float(grng.integers(edge, s - edge))
        y = float(grng.integers(min(20, s // 8), s - edge))
        probs.append(Problem(
            nx=s, ny=s, medium=Medium("layered", lam, mu, np.ones(s)), tau=1.0,
            sources=[Source(x, y, 3.0, 0.0, 1.0, 1.0, 40.0, 60.0)],
            nsteps=nsteps, dtype=dtype, comp_mask=2, name=f"batched_{g}",
            **_sponged(s, s, min(sponge, s // 4))))
    return probs


def gaussian_random_field(rng, n: int, corr: float, max_abs: float) -> np.ndarray:
    """White N(0,1) noise filtered by exp(-|k|^2 l^2 / 4), scaled to max|d|."""
    w = rng.standard_normal((n, n))
    k = 2 * np.pi * np.fft.fftfreq(n)
    kk = k[:, None] ** 2 + k[None, :] ** 2
    d = np.real(np.fft.ifft2(np.fft.fft2(w) * np.exp(-kk * corr * corr / 4.0)))
    return d * (max_abs / np.max(np.abs(d)))


def adjoint_shots(n: int = 1024, shots: int = 16, nsteps: int = 5000,
                  dtype: str = "f32", corr: float = 40.0, sponge: int = 64,
                  homogeneous: bool = False):
    """Seeded +/-10% Gaussian-random-field perturbation of lambda and mu about
    a Poisson-0.25 background, free top with a receiver on every surface cell,
    shot s has a vertical source at (32 + 64 s, 20) (scaled to the grid)."""
    lam0 = mu0 = MU_UNIT
    if homogeneous:
        lam = np.full((n, n), lam0)
        mu = np.full((n, n), mu0)
    else:
        dl = gaussian_random_field(np.random.default_rng(5), n, corr * n / 1024, 0.10)
        dm = gaussian_random_field(np.random.default_rng(55), n, corr * n / 1024, 0.10)
        lam = lam0 * (1.0 + dl)
        mu = mu0 * (1.0 + dm)
    spacing = n / shots
    probs = []
    for s in range(shots):
        x = float(int(spacing / 2 + spacing * s))
        probs.append(Problem(
            nx=n, ny=n, medium=Medium("field", lam, mu, np.ones((n, n))), tau=1.0,
            sources=[Source(x, 20.0, 3.0, 0.0, 1.0, 1.0, 40.0, 60.0)],
            receivers=row_receivers(n, 0), comp_mask=2, nsteps=nsteps,
            dtype=dtype, name=f"adjoint_shot{s}",
            **_sponged(n, n, min(sponge, n // 4))))
    return probs
