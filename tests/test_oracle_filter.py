"""Pins of the oracle's high-wavenumber filter (oracle/filter.py) against what
the mathematics fixes, and of the library's filtered stability factor
against the oracle's von Neumann matrix (host code, no GPU)."""
import math

import numpy as np
import pytest

import workloads as w
from workloads import BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem
from oracle import stepper, theory as T
from oracle.filter import filter_state


def _box(nx, ny, bc=(BC_PERIODIC,) * 4, rr=-1, nu=0.25, tau=1.0):
    lam = 0.04 * T.lame_ratio(nu)
    return Problem(nx=nx, ny=ny, bc=bc, rigid_row=rr, medium=Medium("homogeneous", lam, 0.04, 1.0), tau=tau)


@pytest.mark.parametrize("mx,my", [(1, 0), (3, 2), (8, 5), (16, 12), (15, 11)])
def test_plane_wave_factor(mx, my):
    """On a periodic grid a lattice plane wave is an eigenfunction, with factor
    1 - 16 sigma (sin^4(kx/2) + sin^4(ky/2)) (the symbol of the fourth difference
    is (2 sin(k/2))^4)."""
    nx, ny, sigma = 32, 24, 0.03
    kx, ky = 2 * math.pi * mx / nx, 2 * math.pi * my / ny
    x, y = np.meshgrid(np.arange(nx), np.arange(ny))
    a = np.random.default_rng(mx + 10 * my).standard_normal(9)
    f = a[:, None, None] * np.cos(kx * x + ky * y + 0.3)[None]
    g = filter_state(_box(nx, ny), f, sigma)
    fac = 1 - 16 * sigma * (math.sin(kx / 2) ** 4 + math.sin(ky / 2) ** 4)
    assert np.max(np.abs(g - fac * f)) < 1e-13


def test_periodic_sums_are_conserved():
    f = np.random.default_rng(1).standard_normal((9, 20, 28))
    g = filter_state(_box(28, 20), f, 1 / 16)
    assert np.allclose(g.sum(axis=(1, 2)), f.sum(axis=(1, 2)), atol=1e-12)
    assert np.linalg.norm(g) < np.linalg.norm(f)          # it only damps


def test_cubic_fields_unchanged_with_walls_and_rigid_row():
    """Fourth differences of a cubic vanish, and the left-out terms near walls
    change nothing either: a cubic state is a fixed point on any grid."""
    nx, ny = 23, 19
    x, y = np.meshgrid(np.arange(nx, dtype=float), np.arange(ny, dtype=float))
    cub = 0.3 + 0.1 * x - 0.02 * y + 1e-3 * x * y + 2e-4 * x ** 3 - 3e-4 * y ** 3 + 1e-4 * x * x * y
    f = np.stack([cub * (i + 1) for i in range(9)])
    p = _box(nx, ny, bc=(BC_FREE0, BC_RIGID, BC_RIGID, BC_RIGID), rr=9)
    g = filter_state(p, f, 0.05)
    assert np.max(np.abs(g - f)) < 1e-12 * np.max(np.abs(f))


def test_terms_left_out_at_walls_and_across_the_rigid_row():
    """A single nonzero cell: cells whose x stencil would leave through a
    rigid side keep no x term, cells within two rows of the internal wall
    keep no y term, and nothing couples across that wall."""
    nx, ny, rr = 12, 16, 8
    p = _box(nx, ny, bc=(BC_PERIODIC, BC_PERIODIC, BC_RIGID, BC_RIGID), rr=rr)
    f = np.zeros((9, ny, nx))
    f[0, rr, 1] = 1.0                       # first row below the wall, column 1
    g = filter_state(p, f, 0.05)
    # column 1 has no x term (x-2 < 0) and row rr no y term (within 2 of the wall)
    assert g[0, rr, 1] == 1.0
    # x neighbours 2 and 3 keep their x terms: -4 and +1 times the impulse
    assert abs(g[0, rr, 2] - (0.05 * 4)) < 1e-15 and abs(g[0, rr, 3] + 0.05) < 1e-15
    # rows rr+1 (no y term) and above the wall see nothing; rows rr+2, rr+3 do
    assert g[0, rr + 1, 1] == 0.0 and np.all(g[0, :rr, :] == 0.0)
    assert abs(g[0, rr + 2, 1] + 0.05) < 1e-15 and g[0, rr + 3, 1] == 0.0
    # only population 0 was touched
    assert np.all(g[1:] == 0.0)


@pytest.mark.parametrize("nu,tau,sigma,every", [(0.37, 1.0, 0.005, 1), (0.3, 0.55, 0.005, 1),
                                                (0.0, 0.55, 0.01, 1), (0.37, 1.0, 0.02, 4),
                                                (0.4, 1.0, 0.04, 1), (0.25, 1.0, 0.01, 2)])
def test_library_filtered_factor_matches_oracle_theory(nu, tau, sigma, every):
    from paper_2009_06404_amd import _lib as L
    ks = np.linspace(0, math.pi, 17)
    ref = 0.0
    for kx in ks:
        for ky in ks:
            F = 1 - 16 * sigma * (math.sin(kx / 2) ** 4 + math.sin(ky / 2) ** 4)
            A = F * np.linalg.matrix_power(T.vn_matrix(kx, ky, nu, tau), every)
            ref = max(ref, np.abs(np.linalg.eigvals(A)).max() ** (1 / every))
    g = L.lbm_vn_growth_filtered(nu, tau, sigma, every, 17)
    assert abs(g - ref) < 1e-7, (g, ref)


def test_filter_restores_stability_of_a_growing_run():
    """nu = 0.37 at tau = 1 is unstable: its fastest modes, near
    k = 0.55 pi along both axes, grow about 0.85% per step, and a 22-cell
    periodic box holds k = 6/11 pi. The same oracle run filtered every 4 steps
    with sigma = 0.02 (factor <= 1 by the von Neumann analysis) decays."""
    from paper_2009_06404_amd import _lib as L
    assert L.lbm_vn_growth(0.37, 1.0, 33) > 1.007
    assert L.lbm_vn_growth_filtered(0.37, 1.0, 0.02, 4, 33) <= 1.0 + 1e-9
    p = _box(22, 22, nu=0.37)
    f0 = np.random.default_rng(7).standard_normal((9, 22, 22))
    a = stepper.run(p, nsteps=400, fstar_init=f0, want_trace=False)["fstar"]
    assert np.linalg.norm(a) > 2 * np.linalg.norm(f0)
    f, t = f0, 0
    for _ in range(100):
        f = stepper.run(p, nsteps=4, fstar_init=f, t0=t, want_trace=False)["fstar"]
        t += 4
        f = filter_state(p, f, 0.02)
    assert np.linalg.norm(f) < 0.5 * np.linalg.norm(f0)
