"""Pins of the oracle's discrete adjoint against what the forward oracle and the
mathematics fix, with no reference to the adjoint's own formulas:

* the transpose of one step, and of the receiver read-out, equals the step's
  Jacobian built column by column from the (already pinned) forward oracle, on
  tiny grids for every boundary type, heterogeneous kappa and a sponge;
* the dot-product identity over several steps with receivers and a final-state
  term;
* central finite differences of the misfit with respect to lambda, mu and the
  source amplitude, taken with the forward oracle alone;
* for one source from rest, dL/damp = <e, v> / amp exactly (linearity);
* the forward depends on lambda/mu only (reading of Sec. 4's Lambda), so the
  misfit is flat along (lambda, mu) -> s (lambda, mu) and the per-cell
  gradients satisfy lambda dL/dlambda + mu dL/dmu = 0.
"""
import numpy as np
import pytest

from workloads import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
from workloads.problem import default_sponge_profile
from oracle import stepper

BC_CASES = [
    ("periodic", (BC_PERIODIC,) * 4, -1),
    ("free_rigid_interface", (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC), 3),
    ("free0_both_rigid_sides", (BC_FREE0, BC_FREE0, BC_RIGID, BC_RIGID), -1),
    ("rigid_box_interface", (BC_RIGID,) * 4, 3),
    ("rigid_top_free_bottom", (BC_RIGID, BC_FREE, BC_PERIODIC, BC_PERIODIC), -1),
]


def _medium(rng, ny, nx):
    mu = rng.uniform(0.036, 0.044, (ny, nx))
    nu = rng.uniform(0.1, 0.3, (ny, nx))
    lam = 2 * nu * mu / (1 - 2 * nu)
    rho = rng.uniform(0.9, 1.1, (ny, nx))
    return Medium("field", lam, mu, rho)


def _problem(bc, rr, nx=6, ny=7, seed=0, sources=(), receivers=None, comp_mask=3, tau=0.8,
             sponge=2):
    rng = np.random.default_rng(seed)
    prof = default_sponge_profile(sponge) * 3.0 if sponge else None
    thick = (0, sponge, sponge, 0)               # uneven layers, one over a wall
    rec = np.zeros((0, 2), np.int32) if receivers is None else np.asarray(receivers, np.int32)
    return Problem(nx=nx, ny=ny, bc=bc, medium=_medium(rng, ny, nx), tau=tau, rigid_row=rr,
                   sponge_thick=thick,
                   sponge_profiles=tuple(prof if t else None for t in thick),
                   sources=list(sources), receivers=rec, comp_mask=comp_mask, nsteps=1)


@pytest.mark.parametrize("name,bc,rr", BC_CASES, ids=[c[0] for c in BC_CASES])
def test_adjoint_step_is_transpose_of_step_jacobian(name, bc, rr):
    p = _problem(bc, rr)
    n = 9 * p.ny * p.nx
    J = np.zeros((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        J[:, col] = stepper.run(p, nsteps=1, f_init=e.reshape(9, p.ny, p.nx),
                                want_trace=False)["f"].ravel()
    JT = np.zeros((n, n))
    for row in range(n):
        e = np.zeros(n)
        e[row] = 1.0
        JT[row, :] = stepper.adjoint(p, nsteps=1, adj_init=e.reshape(9, p.ny, p.nx))["adj"].ravel()
    assert np.max(np.abs(J)) > 0.1
    assert np.max(np.abs(JT - J)) <= 1e-14, f"{name}: {np.max(np.abs(JT - J)):.3e}"


def test_adjoint_of_receiver_readout_is_its_transpose():
    bc = (BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC)
    rec = [(0, 0), (3, 0), (5, 2), (2, 4), (3, 0)]          # one cell twice
    p = _problem(bc, -1, receivers=rec, comp_mask=3)
    n = 9 * p.ny * p.nx
    m = len(rec) * 2
    Cm = np.zeros((m, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        Cm[:, col] = stepper.run(p, nsteps=1, f_init=e.reshape(9, p.ny, p.nx))["trace"][0].ravel()
    CT = np.zeros((m, n))
    for row in range(m):
        r = np.zeros(m)
        r[row] = 1.0
        CT[row, :] = stepper.adjoint(p, nsteps=1, residual=r.reshape(1, len(rec), 2))["adj"].ravel()
    assert np.max(np.abs(Cm)) > 0.1
    assert np.max(np.abs(CT - Cm)) <= 1e-14


@pytest.mark.parametrize("name,bc,rr", BC_CASES, ids=[c[0] for c in BC_CASES])
def test_dot_product_identity_over_several_steps(name, bc, rr):
    """<fh(t0), f(t0)> = <a, f(T)> + sum_t <e(t), v(t)> for the linear step."""
    rec = [(1, 1), (4, 0), (2, 5)]
    p = _problem(bc, rr, nx=8, ny=9, seed=3, receivers=rec, comp_mask=3)
    rng = np.random.default_rng(11)
    T = 6
    f0 = rng.standard_normal((9, p.ny, p.nx))
    a = rng.standard_normal((9, p.ny, p.nx))
    e = rng.standard_normal((T, len(rec), 2))
    fw = stepper.run(p, nsteps=T, f_init=f0)
    lhs = np.sum(a * fw["f"]) + np.sum(e * fw["trace"])
    rhs = np.sum(stepper.adjoint(p, nsteps=T, residual=e, adj_init=a)["adj"] * f0)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.sum(np.abs(e)) * 1e-3 + 1.0), (lhs, rhs)


def _misfit_case(seed=5, T=70):
    bc = (BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC)
    src = [Source(9.0, 4.0, 1.5, 0.0, 1.0, 1.0, 12.0, 16.0),
           Source(4.0, 8.0, 1.5, 0.6, 0.8, 0.7, 14.0, 20.0)]
    rec = [(x, 0) for x in range(0, 20, 2)] + [(x, 10) for x in range(1, 20, 3)]
    p = _problem(bc, -1, nx=20, ny=16, seed=seed, sources=src, receivers=rec, comp_mask=3,
                 tau=1.0, sponge=3)
    lam, mu, rho = p.medium.full(p.ny, p.nx)
    # "observed" data: the same shots through a homogeneous background
    bg = (np.full_like(lam, lam.mean()), np.full_like(mu, mu.mean()), rho)
    d_obs = stepper.run(p, nsteps=T, medium=bg)["trace"]
    return p, (lam, mu, rho), d_obs, T


def _L(p, med, d_obs, T):
    return stepper.misfit(stepper.run(p, nsteps=T, medium=med)["trace"], d_obs)[0]


def test_lame_gradients_match_central_differences():
    p, (lam, mu, rho), d_obs, T = _misfit_case()
    fw = stepper.run(p, nsteps=T, medium=(lam, mu, rho))
    L0, e = stepper.misfit(fw["trace"], d_obs)
    assert L0 > 0
    ad = stepper.adjoint(p, nsteps=T, residual=e, medium=(lam, mu, rho))
    assert np.allclose(ad["trace"], fw["trace"], rtol=0, atol=1e-15)
    g_lam, g_mu = stepper.lame_gradients(ad["grad_kappa"], lam, mu)
    rng = np.random.default_rng(21)
    for trial in range(2):
        dl = rng.standard_normal(lam.shape) * lam * 0.1
        dm = rng.standard_normal(mu.shape) * mu * 0.1
        eps = 1e-4
        fd_l = (_L(p, (lam + eps * dl, mu, rho), d_obs, T)
                - _L(p, (lam - eps * dl, mu, rho), d_obs, T)) / (2 * eps)
        fd_m = (_L(p, (lam, mu + eps * dm, rho), d_obs, T)
                - _L(p, (lam, mu - eps * dm, rho), d_obs, T)) / (2 * eps)
        an_l = float(np.sum(g_lam * dl))
        an_m = float(np.sum(g_mu * dm))
        assert abs(fd_l - an_l) <= 1e-6 * abs(fd_l), (trial, fd_l, an_l)
        assert abs(fd_m - an_m) <= 1e-6 * abs(fd_m), (trial, fd_m, an_m)


def test_amplitude_gradient_matches_differences_and_linearity():
    p, med, d_obs, T = _misfit_case(seed=8)
    L0, e = stepper.misfit(stepper.run(p, nsteps=T, medium=med)["trace"], d_obs)
    ga = stepper.adjoint(p, nsteps=T, residual=e, medium=med)["grad_amp"]
    for s in range(len(p.sources)):
        eps = 1e-4
        def L_at(da):
            srcs = list(p.sources)
            q = srcs[s]
            srcs[s] = Source(q.x, q.y, q.sigma, q.dir_x, q.dir_y, q.amp + da, q.period, q.t0)
            return _L(p.replace(sources=srcs), med, d_obs, T)
        fd = (L_at(eps) - L_at(-eps)) / (2 * eps)
        assert abs(fd - ga[s]) <= 1e-7 * abs(fd), (s, fd, ga[s])
    # one source from rest: v = amp * v_unit, so dL/damp = <e, v> / amp
    one = p.replace(sources=[p.sources[1]])
    tr = stepper.run(one, nsteps=T, medium=med)["trace"]
    _, e1 = stepper.misfit(tr, d_obs)
    g1 = stepper.adjoint(one, nsteps=T, residual=e1, medium=med)["grad_amp"][0]
    want = float(np.sum(e1 * tr)) / one.sources[0].amp
    assert abs(g1 - want) <= 1e-12 * abs(want)


def test_misfit_depends_on_lame_ratio_only():
    p, (lam, mu, rho), d_obs, T = _misfit_case(seed=9)
    L0, e = stepper.misfit(stepper.run(p, nsteps=T, medium=(lam, mu, rho))["trace"], d_obs)
    for s in (0.5, 1.7):
        Ls = _L(p, (lam * s, mu * s, rho), d_obs, T)
        assert abs(Ls - L0) <= 1e-12 * L0
    gk = stepper.adjoint(p, nsteps=T, residual=e, medium=(lam, mu, rho))["grad_kappa"]
    g_lam, g_mu = stepper.lame_gradients(gk, lam, mu)
    scale = np.max(np.abs(lam * g_lam))
    assert scale > 0
    assert np.max(np.abs(lam * g_lam + mu * g_mu)) <= 1e-13 * scale
