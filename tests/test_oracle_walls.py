"""Pins of the oracle's internal rigid wall and of its density-gradient rule at
walls, against what the scheme's own definitions fix:

* a rigid wall between rows r-1 and r (eq. BB of Sec. 6.1, placed inside the
  grid) decouples the two sides completely: a grid with the wall must equal,
  bit for bit, the two independent grids of rows 0..r-1 (rigid bottom edge)
  and rows r..ny-1 (rigid top edge), fields, populations and traces, in the
  forward and in the adjoint. On a grid periodic in y the wall instead turns
  the grid into one grid of rows r..ny-1, 0..r-1 with rigid edges on both
  ends;
* the centred difference of eq. FDrho (Sec. 2), completed at a non-periodic
  edge or beside the internal wall by the linearly extrapolated ghost density,
  is exact for a density that is linear on each side of the wall: from
  populations holding only a rest part, one collision must add kappa times the
  exact slope to sum_i f_i c_i at every cell, corners, edges and both faces of
  the wall included.

A zero-order ghost, or a wall missing from the streaming or from the
gradient, fails one of these.
"""
import numpy as np
import pytest

from workloads import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
from workloads.problem import default_sponge_profile
from oracle import stepper


def _field_medium(rng, ny, nx):
    mu = rng.uniform(0.036, 0.044, (ny, nx))
    nu = rng.uniform(0.1, 0.33, (ny, nx))
    lam = 2 * nu * mu / (1 - 2 * nu)
    rho = rng.uniform(0.9, 1.1, (ny, nx))
    return lam, mu, rho


def _sub(p, lam, mu, rho, rows, bc_top, bc_bottom, thick_top, thick_bottom, y_shift,
         rec_sel):
    """The rows `rows` of problem p as a grid of its own, with the given top
    and bottom edges and sponge thicknesses; sources keep their absolute
    position (shifted into the new coordinates), so their tails are the same."""
    ny = len(rows)
    prof = p.sponge_profiles
    thick = (thick_top, thick_bottom, p.sponge_thick[2], p.sponge_thick[3])
    yn = p.ny if p.bc[0] == BC_PERIODIC else None
    srcs = [Source(s.x, (s.y - y_shift) % yn if yn else s.y - y_shift, s.sigma, s.dir_x,
                   s.dir_y, s.amp, s.period, s.t0) for s in p.sources]
    rec = p.receivers[rec_sel].copy()
    if rec.size:
        rec[:, 1] = (rec[:, 1] - y_shift) % p.ny
    sub = Problem(nx=p.nx, ny=ny, bc=(bc_top, bc_bottom, p.bc[2], p.bc[3]),
                  medium=Medium("field", lam[rows], mu[rows], rho[rows]), tau=p.tau,
                  rigid_row=-1, sponge_thick=thick,
                  sponge_profiles=(prof[0], prof[1], prof[2], prof[3]),
                  sources=srcs, receivers=rec.reshape(-1, 2).astype(np.int32),
                  comp_mask=p.comp_mask, nsteps=p.nsteps)
    return sub


def _walled(bc, nx=13, ny=17, rr=7, seed=0, tau=0.8, thick=(3, 4, 2, 3), sigma=1.3,
            src_y=None):
    rng = np.random.default_rng(seed)
    lam, mu, rho = _field_medium(rng, ny, nx)
    profs = tuple(default_sponge_profile(t) * 2.0 if t else None for t in thick)
    # sources on both sides, by default one next to the wall so that its tail
    # crosses it
    sy = (3.0, rr - 1.0, rr + 4.0) if src_y is None else src_y
    srcs = [Source(4.0, sy[0], sigma, 0.3, 1.0, 1.0, 8.0, 6.0),
            Source(9.0, sy[1], sigma, 1.0, -0.4, -0.7, 9.0, 5.0),
            Source(6.0, sy[2], sigma, -0.6, 0.8, 1.4, 7.0, 4.0)]
    rec = np.array([[1, 0], [5, rr - 1], [11, 2], [2, rr], [8, ny - 1], [12, rr + 3]],
                   np.int32)
    p = Problem(nx=nx, ny=ny, bc=bc, medium=Medium("field", lam, mu, rho), tau=tau,
                rigid_row=rr, sponge_thick=thick, sponge_profiles=profs, sources=srcs,
                receivers=rec, comp_mask=3, nsteps=9)
    return p, (lam, mu, rho), rng


def _split(p, lam, mu, rho):
    """The independent grids a wall between rows r-1 and r must be equal to."""
    r, ny = p.rigid_row, p.ny
    rec_y = p.receivers[:, 1]
    if p.bc[0] != BC_PERIODIC:
        up = _sub(p, lam, mu, rho, np.arange(0, r), p.bc[0], BC_RIGID, p.sponge_thick[0], 0,
                  0, rec_y < r)
        lo = _sub(p, lam, mu, rho, np.arange(r, ny), BC_RIGID, p.bc[1], 0, p.sponge_thick[1],
                  r, rec_y >= r)
        return [(up, np.arange(0, r), rec_y < r), (lo, np.arange(r, ny), rec_y >= r)]
    # periodic in y: one grid of rows r..ny-1 then 0..r-1, rigid at both ends
    rows = np.concatenate([np.arange(r, ny), np.arange(0, r)])
    one = _sub(p, lam, mu, rho, rows, BC_RIGID, BC_RIGID, 0, 0, r, np.ones(len(rec_y), bool))
    return [(one, rows, np.ones(len(rec_y), bool))]


WALL_CASES = [
    ("free_top_rigid_bottom_periodic_sides", (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC)),
    ("free0_top_free_bottom_rigid_sides", (BC_FREE0, BC_FREE, BC_RIGID, BC_RIGID)),
    ("rigid_box", (BC_RIGID, BC_RIGID, BC_RIGID, BC_RIGID)),
]


@pytest.mark.parametrize("name,bc", WALL_CASES, ids=[c[0] for c in WALL_CASES])
def test_internal_rigid_wall_equals_two_independent_grids(name, bc):
    p, (lam, mu, rho), rng = _walled(bc)
    fs0 = rng.standard_normal((9, p.ny, p.nx))
    whole = stepper.run(p, fstar_init=fs0, t0=3)
    for sub, rows, sel in _split(p, lam, mu, rho):
        part = stepper.run(sub, fstar_init=fs0[:, rows], t0=3)
        for key in ("fstar", "f", "mom"):
            assert np.array_equal(whole[key][:, rows], part[key]), key
        assert np.array_equal(whole["trace"][:, sel], part["trace"])


def test_internal_rigid_wall_on_a_y_periodic_grid_is_a_rotated_rigid_channel():
    """With periodic top and bottom, the wall is the only place the rows meet
    a wall: the grid equals rows r..ny-1, 0..r-1 between two rigid edges.
    The body force is geometric and ignores walls, so the sources sit more
    than 9 sigma from the wall (one of them across the wrap): there the
    minimum image of the periodic grid and the plain distance in the channel
    agree on every cell they reach."""
    bc = (BC_PERIODIC, BC_PERIODIC, BC_RIGID, BC_RIGID)
    p, (lam, mu, rho), rng = _walled(bc, ny=24, rr=9, thick=(0, 0, 2, 3), sigma=0.6,
                                     src_y=(1.0, 22.0, 15.0))
    fs0 = rng.standard_normal((9, p.ny, p.nx))
    whole = stepper.run(p, fstar_init=fs0, t0=2)
    [(sub, rows, sel)] = _split(p, lam, mu, rho)
    # receivers were re-expressed in the rotated rows; order is unchanged
    part = stepper.run(sub, fstar_init=fs0[:, rows], t0=2)
    for key in ("fstar", "f", "mom"):
        assert np.array_equal(whole[key][:, rows], part[key]), key
    assert np.array_equal(whole["trace"], part["trace"])


@pytest.mark.parametrize("name,bc", WALL_CASES[:2], ids=[c[0] for c in WALL_CASES[:2]])
def test_internal_rigid_wall_splits_the_adjoint(name, bc):
    """The same decoupling for the oracle's adjoint: the adjoint state and
    dL/dkappa equal those of the two grids bit for bit; dL/damp, a sum over
    cells, is the sum of the two grids' values (to rounding)."""
    p, (lam, mu, rho), rng = _walled(bc, seed=4)
    n = p.nsteps
    fs0 = rng.standard_normal((9, p.ny, p.nx))
    ai = rng.standard_normal((9, p.ny, p.nx))
    res = rng.standard_normal((n, p.nrec, p.ncomp))
    whole = stepper.adjoint(p, residual=res, adj_init=ai, fstar_init=fs0, t0=1)
    amp = np.zeros(len(p.sources))
    for sub, rows, sel in _split(p, lam, mu, rho):
        part = stepper.adjoint(sub, residual=res[:, sel], adj_init=ai[:, rows],
                               fstar_init=fs0[:, rows], t0=1)
        assert np.array_equal(whole["adj"][:, rows], part["adj"])
        assert np.array_equal(whole["grad_kappa"][rows], part["grad_kappa"])
        assert np.array_equal(whole["trace"][:, sel], part["trace"])
        amp += part["grad_amp"]
    assert np.abs(whole["grad_amp"] - amp).max() <= 1e-13 * np.abs(amp).max()


GHOST_CASES = [
    ("free_top_rigid_bottom", (BC_FREE, BC_RIGID, BC_RIGID, BC_RIGID), 6),
    ("free0_top_free_bottom", (BC_FREE0, BC_FREE, BC_RIGID, BC_RIGID), 5),
    ("rigid_box_no_wall", (BC_RIGID, BC_RIGID, BC_RIGID, BC_RIGID), -1),
    ("periodic_y_with_wall", (BC_PERIODIC, BC_PERIODIC, BC_RIGID, BC_RIGID), 4),
]


@pytest.mark.parametrize("name,bc,rr", GHOST_CASES, ids=[c[0] for c in GHOST_CASES])
def test_density_gradient_exact_for_linear_density_up_to_walls(name, bc, rr):
    """f_i = w_i rho(x, y) with rho linear in x and linear in y on each side
    of the wall (its own slope and offset on each side). The moments are
    rho, m = 0, P = b^2 rho I, so with no sponge and no force one collision
    adds S = kappa D rho to sum_i f_i c_i; eq. FDrho with the extrapolated
    ghost gives the exact slopes at every cell. On a grid periodic in y the
    density is linear along the channel the wall leaves (rows r..ny-1, then
    0..r-1 across the wrap)."""
    nx, ny = 11, 12
    rng = np.random.default_rng(7)
    lam, mu, rho0 = _field_medium(rng, ny, nx)
    p = Problem(nx=nx, ny=ny, bc=bc, medium=Medium("field", lam, mu, rho0), tau=0.7,
                rigid_row=rr, nsteps=1)
    _, _, wt, _ = stepper.lattice()
    cx, cy, _, _ = stepper.lattice()
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    x = np.ones((ny, 1)) * np.arange(nx)[None, :]
    sx = 0.031
    if bc[0] == BC_PERIODIC:
        # the rows meet across the wrap: linear along the channel r..ny-1, 0..r-1
        y = (y - rr) % ny
        below = np.zeros_like(y, bool)
    else:
        below = y >= rr if rr > 0 else np.zeros_like(y, bool)
    sy = np.where(below, -0.047, 0.022)
    off = np.where(below, 0.9, -0.35)
    rho = off + sx * x + sy * y
    f0 = wt[:, None, None] * rho[None]
    out = stepper.run(p, f_init=f0, t0=0)
    fs = out["fstar"]
    kappa = (mu - lam) / mu / 3.0
    gx = np.tensordot(cx.astype(float), fs, axes=(0, 0))
    gy = np.tensordot(cy.astype(float), fs, axes=(0, 0))
    assert np.abs(gx - kappa * sx).max() <= 1e-15
    assert np.abs(gy - kappa * sy).max() <= 1e-15
    # the rest part itself is untouched: density and P = b^2 rho I conserved
    assert np.abs(fs.sum(0) - rho).max() <= 1e-15
