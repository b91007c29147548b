"""Pins of the C oracle (the scheme itself) against what the paper and the
mathematics fix: lattice isotropy, the moments of the equilibrium, collision
invariants, exact plane-wave evolution under the independently built von
Neumann matrix, conservation, linearity, rest states, symmetry, the exact image
equivalence of a bounce-back wall, the spectral Navier reference, wave speeds,
the Rayleigh speed and the reflection polarity of the two walls."""
import math

import numpy as np
import pytest

import workloads as w
from workloads import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source
from oracle import spectral, stepper, theory as T
from _golden import TABLE1_NUS, paper_values, table1

RNG = np.random.default_rng(1234)


def _lattice():
    cx, cy, wt, opp = stepper.lattice()
    return cx.astype(float), cy.astype(float), wt, opp


def _delta(a, b):
    return 1.0 if a == b else 0.0


def test_lattice_isotropy():
    """eq. isotropy up to sixth order, including the -6 delta defect."""
    cx, cy, wt, opp = _lattice()
    c = np.stack([cx, cy], 1)
    b2 = 1.0 / 3.0
    assert abs(wt.sum() - 1) < 1e-15
    for i in range(9):
        assert cx[opp[i]] == -cx[i] and cy[opp[i]] == -cy[i]
    idx = range(2)
    for a in idx:
        assert abs(np.sum(wt * c[:, a])) < 1e-16
        for b in idx:
            assert abs(np.sum(wt * c[:, a] * c[:, b]) - b2 * _delta(a, b)) < 1e-15
            for g in idx:
                assert abs(np.sum(wt * c[:, a] * c[:, b] * c[:, g])) < 1e-16
                for k in idx:
                    d4 = _delta(a, b) * _delta(g, k) + _delta(a, g) * _delta(b, k) + _delta(a, k) * _delta(b, g)
                    assert abs(np.sum(wt * c[:, a] * c[:, b] * c[:, g] * c[:, k]) - b2 ** 2 * d4) < 1e-15
    # sixth order: b^6 (Delta6 - 6 delta_abgkps)
    import itertools
    for ind in itertools.product(idx, repeat=6):
        lhs = np.sum(wt * np.prod([c[:, q] for q in ind], axis=0))
        # Delta6 = sum over the 15 pairings of delta products
        def pairings(s):
            if not s:
                yield []
                return
            a = s[0]
            for j in range(1, len(s)):
                rest = s[1:j] + s[j + 1:]
                for p in pairings(rest):
                    yield [(a, s[j])] + p
        d6 = sum(np.prod([_delta(ind[p], ind[q]) for p, q in pr]) for pr in pairings(list(range(6))))
        allsame = 1.0 if len(set(ind)) == 1 else 0.0
        assert abs(lhs - b2 ** 3 * (d6 - 6 * allsame)) < 1e-15


@pytest.mark.parametrize("A", ["0", "1/10"])
@pytest.mark.parametrize("tau", ["1", "11/20"])
def test_single_cell_collision_exact_rationals(A, tau):
    """One cell's collision (Sec. 2 moments, the implicit sponge flux of
    Sec. 6.3, the equilibrium with P^n = P - b^2 rho I and the forcing term)
    evaluated in exact rational arithmetic for a hand-picked population
    vector, gradient force G = kappa D rho + F with kappa = -1/5, D rho =
    (1/2, -1/4) and F = (0, 0); the oracle must agree to rounding."""
    from fractions import Fraction as Fr
    cx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    cy = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    wt = [Fr(4, 9)] + [Fr(1, 9)] * 4 + [Fr(1, 36)] * 4
    b2 = Fr(1, 3)
    A, tau = Fr(A), Fr(tau)
    f = [Fr(i + 1, 100) for i in range(9)]
    kappa = Fr(-1, 5)
    G = (kappa * Fr(1, 2), kappa * Fr(-1, 4))
    rho = sum(f)
    m = (sum(fi * c for fi, c in zip(f, cx)), sum(fi * c for fi, c in zip(f, cy)))
    P = [[sum(fi * a * b for fi, a, b in zip(f, ca, cb)) for cb in (cx, cy)] for ca in (cx, cy)]
    j = tuple((m[a] + G[a] / 2) / (1 + A / 2) for a in range(2))
    S = tuple(G[a] - A * j[a] for a in range(2))
    Pn = [[P[a][b] - (b2 * rho if a == b else 0) for b in range(2)] for a in range(2)]
    want = []
    for i in range(9):
        c = (cx[i], cy[i])
        q = sum(Pn[a][b] * (c[a] * c[b] - (b2 if a == b else 0)) for a in range(2) for b in range(2))
        feq = wt[i] * (rho + (j[0] * c[0] + j[1] * c[1]) / b2 + q / (2 * b2 * b2))
        force = (1 - 1 / (2 * tau)) * wt[i] * (c[0] * S[0] + c[1] * S[1]) / b2
        want.append(f[i] - (f[i] - feq) / tau + force)
    fs, jo, So = stepper.collide_cell(np.array([float(x) for x in f]),
                                      np.array([float(g) for g in G]), float(A), float(tau))
    want = np.array([float(x) for x in want])
    assert np.max(np.abs(fs - want)) <= 1e-15 * np.max(np.abs(want))
    assert np.allclose(jo, [float(x) for x in j], rtol=1e-15, atol=0)
    assert np.allclose(So, [float(x) for x in S], rtol=1e-15, atol=1e-18)


def test_equilibrium_moments():
    """eq. MomentsFeq: moments 0-3 of f^eq are rho, j, P and
    Q^eq = b^2 (j d + j d + j d) (the paper's first moment read as j)."""
    cx, cy, _, _ = _lattice()
    c = np.stack([cx, cy], 1)
    for _ in range(20):
        rho = RNG.normal()
        j = RNG.normal(size=2)
        P = RNG.normal(size=3)
        feq = stepper.equilibrium(rho, j, P)
        Pm = np.array([[P[0], P[1]], [P[1], P[2]]])
        assert abs(feq.sum() - rho) < 1e-14
        assert np.allclose(c.T @ feq, j, atol=1e-14)
        assert np.allclose(np.einsum("i,ia,ib->ab", feq, c, c), Pm, atol=1e-14)
        Q = np.einsum("i,ia,ib,ig->abg", feq, c, c, c)
        for a in range(2):
            for b in range(2):
                for g in range(2):
                    ref = (j[a] * _delta(b, g) + j[b] * _delta(a, g) + j[g] * _delta(a, b)) / 3.0
                    assert abs(Q[a, b, g] - ref) < 1e-14


@pytest.mark.parametrize("tau", [0.55, 1.0, 1.7])
@pytest.mark.parametrize("A", [0.0, 0.1])
def test_collision_invariants(tau, A):
    """Solvability conditions (Sec. 3): the collision conserves rho and P and
    adds exactly S to the first moment, S = G - A j, j = sum f c + S/2."""
    cx, cy, _, _ = _lattice()
    c = np.stack([cx, cy], 1)
    for _ in range(50):
        f = RNG.normal(size=9)
        G = RNG.normal(size=2)
        fs, j, S = stepper.collide_cell(f, G, A, tau)
        m = c.T @ f
        assert abs(fs.sum() - f.sum()) < 1e-13
        assert np.allclose(np.einsum("i,ia,ib->ab", fs, c, c), np.einsum("i,ia,ib->ab", f, c, c), atol=1e-13)
        assert np.allclose(c.T @ fs, m + S, atol=1e-13)
        assert np.allclose(j, m + S / 2, atol=1e-13)
        assert np.allclose(S, G - A * j, atol=1e-13)


def test_collision_of_equilibrium_state():
    """A cell already at equilibrium only receives the forcing populations:
    f* = f^eq + (1 - 1/(2 tau)) w_i c_i.S / b^2 (eqs. LBGK, Si)."""
    cx, cy, wt, _ = _lattice()
    tau = 0.7
    rho, m, P = 0.3, np.array([0.1, -0.2]), np.array([0.05, 0.02, -0.03])
    G = np.array([0.04, -0.01])
    j = m + G / 2
    feq = stepper.equilibrium(rho, j, P)
    # feq has first moment j; shift it back so that sum f c = m
    f = feq - 0.0
    f_m = f.copy()
    f_m += wt * (cx * (m[0] - j[0]) + cy * (m[1] - j[1])) * 3.0  # first-moment shift
    fs, jj, S = stepper.collide_cell(f_m, G, 0.0, tau)
    assert np.allclose(jj, j, atol=1e-15)
    feq2 = stepper.equilibrium(rho, j, np.array([
        np.sum(f_m * cx * cx), np.sum(f_m * cx * cy), np.sum(f_m * cy * cy)]))
    expect = f_m - (f_m - feq2) / tau + (1 - 0.5 / tau) * wt * (cx * S[0] + cy * S[1]) * 3.0
    assert np.allclose(fs, expect, atol=1e-15)


def _periodic_problem(n, nu, tau, sources=(), A_uniform=0.0, nx=None):
    lam_mu = T.lame_ratio(nu)
    ny = n
    nx = n if nx is None else nx
    thick = (ny, 0, 0, 0) if A_uniform else (0, 0, 0, 0)
    prof = (np.full(ny, A_uniform), None, None, None) if A_uniform else (None,) * 4
    return Problem(nx=nx, ny=ny, bc=(BC_PERIODIC,) * 4,
                   medium=Medium("homogeneous", 0.04 * lam_mu, 0.04, 1.0), tau=tau,
                   sponge_thick=thick, sponge_profiles=prof, sources=list(sources),
                   receivers=np.zeros((0, 2), np.int32), nsteps=0)


@pytest.mark.parametrize("nu,tau,A", [(0.1, 0.8, 0.0), (0.25, 0.55, 0.0), (0.33, 1.0, 0.0), (0.2, 0.9, 0.05)])
def test_plane_wave_eigen_evolution(nu, tau, A):
    """A Bloch wave F exp(i k.x), F an eigenvector of the von Neumann matrix
    M(k) with eigenvalue l, evolves into l^n F exp(i k.x) under the oracle
    (the real part of it, since the scheme is real and linear)."""
    n = 16
    p = _periodic_problem(n, nu, tau, A_uniform=A)
    y, x = np.mgrid[0:n, 0:n]
    for (mx, my) in [(1, 0), (2, 3), (5, 5), (7, 2)]:
        kx, ky = 2 * math.pi * mx / n, 2 * math.pi * my / n
        lam, V = np.linalg.eig(T.vn_matrix(kx, ky, nu, tau, A))
        phase = np.exp(1j * (kx * x + ky * y))
        for e in range(9):
            F = V[:, e]
            f0 = np.real(F[:, None, None] * phase[None])
            steps = 5
            out = stepper.run(p, nsteps=steps, f_init=f0)["f"]
            ref = np.real((lam[e] ** steps) * F[:, None, None] * phase[None])
            scale = np.abs(f0).max()
            assert np.abs(out - ref).max() / scale < 1e-12


def test_periodic_conservation():
    """Periodic box, homogeneous medium, no sponge: sum rho and sum P are
    invariant and sum m grows by exactly sum F per step (the elastic term
    kappa D rho telescopes)."""
    n = 24
    src = Source(9.3, 13.7, 2.0, 0.6, 0.8, 1.0, 8.0, 6.0)
    p = _periodic_problem(n, 0.1, 0.8, sources=[src])
    cx, cy, _, _ = _lattice()
    f = RNG.normal(size=(9, n, n)) * 1e-2
    prev = None
    for t in range(12):
        out = stepper.run(p, nsteps=1, t0=t, f_init=f)
        f1 = out["f"]
        rho0, rho1 = f.sum(), f1.sum()
        assert abs(rho1 - rho0) < 1e-13
        for a, b in ((cx, cx), (cx, cy), (cy, cy)):
            assert abs(np.einsum("iyx,i->", f1, a * b) - np.einsum("iyx,i->", f, a * b)) < 1e-13
        # sum F at time t, written out from the source definition (Sec. 5)
        y, x = np.mgrid[0:n, 0:n].astype(float)
        dx = (x - src.x + n / 2) % n - n / 2
        dy = (y - src.y + n / 2) % n - n / 2
        a = math.pi * (t - src.t0) / src.period
        g = np.exp(-(dx ** 2 + dy ** 2) / (2 * src.sigma ** 2)) * (1 - 2 * a * a) * math.exp(-a * a)
        for c, d in ((cx, src.dir_x), (cy, src.dir_y)):
            dm = np.einsum("iyx,i->", f1, c) - np.einsum("iyx,i->", f, c)
            assert abs(dm - d * g.sum()) < 1e-12
        f = f1


def test_linearity_and_superposition():
    base = w.plain_large(n=96, nsteps=40, dtype="f64", sponge=16, src_depth=10)
    s1 = Source(30.0, 10.0, 3.0, 0.0, 1.0, 1.0, 10.0, 12.0)
    s2 = Source(70.0, 40.0, 2.0, 0.7, -0.3, 1.0, 14.0, 9.0)
    p1 = base.replace(sources=[s1])
    p2 = base.replace(sources=[s2])
    s1b = Source(**{**s1.__dict__, "amp": 2.5})
    s2b = Source(**{**s2.__dict__, "amp": -1.5})
    p12 = base.replace(sources=[s1b, s2b])
    r1, r2, r12 = stepper.run(p1), stepper.run(p2), stepper.run(p12)
    for key in ("f", "mom", "trace"):
        ref = 2.5 * r1[key] - 1.5 * r2[key]
        assert np.abs(r12[key] - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("bc", [(BC_PERIODIC,) * 4, (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                                (BC_RIGID, BC_FREE, BC_RIGID, BC_RIGID), (BC_FREE, BC_FREE, BC_PERIODIC, BC_PERIODIC)])
def test_rest_state_is_fixed(bc):
    p = Problem(nx=12, ny=10, bc=bc, medium=Medium("homogeneous", 0.02, 0.04, 1.0),
                rigid_row=5, nsteps=7)
    out = stepper.run(p)
    assert np.all(out["f"] == 0.0) and np.all(out["mom"] == 0.0)


def test_uniform_density_state_fixed_under_periodic_and_rigid():
    """f = w rho0 is a fixed point of collision, streaming and bounce-back."""
    _, _, wt, _ = _lattice()
    f0 = np.broadcast_to(0.7 * wt[:, None, None], (9, 10, 12)).copy()
    for bc in [(BC_PERIODIC,) * 4, (BC_RIGID, BC_RIGID, BC_RIGID, BC_RIGID),
               (BC_RIGID, BC_RIGID, BC_PERIODIC, BC_PERIODIC)]:
        p = Problem(nx=12, ny=10, bc=bc, medium=Medium("homogeneous", 0.02, 0.04, 1.0), rigid_row=4)
        out = stepper.run(p, nsteps=9, f_init=f0)
        assert np.abs(out["f"] - f0).max() < 1e-15


@pytest.mark.parametrize("free", [BC_FREE, BC_FREE0])
def test_traction_free_uniform_state_fixed_at_free_surface(free):
    """A uniform equilibrium with zero flux and P.n = 0 at the free surface
    (P_yy = P_xy = 0, any rho and P_xx) is a fixed point of the anti-bounce-back
    rule (Sec. 6.2); a uniform state with P_yy != 0 is not."""
    ny, nx = 9, 8
    bc = (free, BC_RIGID, BC_PERIODIC, BC_PERIODIC)
    p = Problem(nx=nx, ny=ny, bc=bc, medium=Medium("homogeneous", 0.03, 0.04, 1.0))
    feq = stepper.equilibrium(0.3, [0.0, 0.0], [0.7, 0.0, 0.0])
    f0 = np.broadcast_to(feq[:, None, None], (9, ny, nx)).copy()
    out = stepper.run(p, nsteps=6, f_init=f0)
    assert np.abs(out["f"] - f0).max() < 1e-14
    feq_bad = stepper.equilibrium(0.3, [0.0, 0.0], [0.7, 0.0, 0.2])
    fb = np.broadcast_to(feq_bad[:, None, None], (9, ny, nx)).copy()
    out = stepper.run(p, nsteps=1, f_init=fb)
    assert np.abs(out["f"] - fb).max() > 1e-3


def test_mirror_symmetry_of_centred_x_force():
    """A centred x-directed source gives j_x even and j_y odd about both
    symmetry lines of the periodic box (Sec. 5 set-up)."""
    p = w.plain_small(n=64, nsteps=60, nu=0.1, tau=0.8)
    p = p.replace(sources=[Source(32.0, 32.0, 4.0, 1.0, 0.0, 1.0, 20.0, 30.0)])
    m = stepper.run(p)["mom"]
    jx, jy = m[1], m[2]
    # reflection x -> 64 - x about x = 32 (periodic: index (64 - i) % 64)
    rx = lambda a: a[:, (-np.arange(64)) % 64 + 0][:, :]
    ix = (64 - np.arange(64)) % 64
    sc = np.abs(jx).max()
    assert np.abs(jx - jx[:, ix]).max() < 1e-13 * sc
    assert np.abs(jx - jx[ix, :]).max() < 1e-13 * sc
    assert np.abs(jy + jy[:, ix]).max() < 1e-13 * sc
    assert np.abs(jy + jy[ix, :]).max() < 1e-13 * sc


def test_bounce_back_equals_image_domain():
    """Halfway bounce-back (eq. BB) between two rigid walls is exactly the
    doubled periodic domain holding the point-reflected image state, for an
    x-uniform Poisson solid (no elastic force, so no boundary rule for D rho
    is involved)."""
    H, nx = 11, 3
    _, _, _, opp = _lattice()
    f = RNG.normal(size=(9, H, 1)) * np.ones((1, 1, nx))
    walls = Problem(nx=nx, ny=H, bc=(BC_RIGID, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                    medium=Medium("homogeneous", 0.04, 0.04, 1.0), tau=0.7)
    img = np.zeros((9, 2 * H, nx))
    img[:, :H] = f
    img[:, H:] = f[opp][:, ::-1]
    doubled = walls.replace(ny=2 * H, bc=(BC_PERIODIC,) * 4)
    a = stepper.run(walls, nsteps=25, f_init=f)["f"]
    b = stepper.run(doubled, nsteps=25, f_init=img)["f"]
    assert np.abs(a - b[:, :H]).max() < 1e-13 * np.abs(f).max()


def test_spectral_reference_table1_128():
    """Relative L2 misfit of j_x against the App. B spectral solution at the
    paper's 128x128 case is of the size the paper prints (Table errorL2)."""
    tab = table1()[128]
    for nu, printed in zip(TABLE1_NUS, tab):
        p = w.plain_small(n=128, nsteps=70, nu=nu, tau=0.55)
        p = p.replace(sources=[Source(64.0, 64.0, 4.0, 1.0, 0.0, 1.0, 20.0, 30.0)])
        jx = stepper.run(p)["mom"][1]
        jx_ref, _ = spectral.solve(128, nu, 70, p.sources[0])
        err = spectral.rel_l2(jx, jx_ref)
        assert printed / 1.5 < err < printed * 1.5, (nu, err, printed)


def test_spectral_convergence_with_refinement():
    """At a fixed physical source the misfit falls as the grid is refined
    (Sec. 5: the scheme converges to the Navier solution)."""
    errs = []
    for n in (64, 128, 256):
        s = n / 128
        p = w.plain_small(n=n, nsteps=int(round(70 * s)), nu=0.1, tau=0.55)
        p = p.replace(sources=[Source(n / 2, n / 2, 4.0 * s, 1.0, 0.0, 1.0, 20.0 * s, 30.0 * s)])
        jx = stepper.run(p)["mom"][1]
        jx_ref, _ = spectral.solve(n, 0.1, p.nsteps, p.sources[0])
        errs.append(spectral.rel_l2(jx, jx_ref))
    assert errs[0] > 1.8 * errs[1] > 1.8 * 1.8 * errs[2]


def _peak_time(tr):
    a = np.abs(tr)
    i = int(np.argmax(a))
    if 0 < i < len(a) - 1:
        den = a[i - 1] - 2 * a[i] + a[i + 1]
        if den != 0:
            return i + 0.5 * (a[i - 1] - a[i + 1]) / den
    return float(i)


@pytest.mark.parametrize("nu", [0.0, 0.1, 0.2, 0.25, 0.3])
def test_wave_speeds_from_travel_times(nu):
    """P and S speeds from the arrival times of a plane pulse at two stations
    (a line source in a one-column periodic box, so no geometric spreading
    bends the waveform). Sec. 5 reports travel-time speeds within 1.1%."""
    ny, ys, d1, d2 = 900, 100.0, 60, 360
    lam_mu = T.lame_ratio(nu)
    rec = np.array([[0, int(ys) + d1], [0, int(ys) + d2]], np.int32)
    vp, vs = T.wave_speeds(nu)
    tol = paper_values()["wave_speed_max_rel_error"]
    for direction, v in (((0.0, 1.0), vp), ((1.0, 0.0), vs)):
        p = Problem(nx=1, ny=ny, bc=(BC_PERIODIC,) * 4,
                    medium=Medium("homogeneous", 0.04 * lam_mu, 0.04, 1.0), tau=0.55,
                    sources=[Source(0.0, ys, 4.0, direction[0], direction[1], 1.0, 20.0, 30.0)],
                    receivers=rec, comp_mask=3)
        nsteps = int(30 + d2 / v + 60)
        tr = stepper.run(p, nsteps=nsteps)["trace"]
        comp = 1 if direction[1] else 0
        t1 = _peak_time(tr[:, 0, comp])
        t2 = _peak_time(tr[:, 1, comp])
        vm = (d2 - d1) / (t2 - t1)
        assert abs(vm - v) / v < tol, (nu, direction, vm, v)


def _peak_in(tr, lo, hi):
    a = np.abs(tr)
    lo, hi = max(int(lo), 1), min(int(hi), len(a) - 2)
    i = lo + int(np.argmax(a[lo:hi]))
    den = a[i - 1] - 2 * a[i] + a[i + 1]
    return i + 0.5 * (a[i - 1] - a[i + 1]) / den


@pytest.mark.parametrize("free", [BC_FREE, BC_FREE0])
@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_rayleigh_wave_speed(free, tau):
    """Surface-wave speed under the free-surface rule versus the root of the
    Rayleigh equation, from the arrival of the surface pulse at two stations
    (Sec. 7: 0.5315 measured against 0.5308 for nu = 0.25)."""
    nu = 0.25
    nx, ny, xs, d1, d2 = 1024, 200, 100, 200, 450
    lam_mu = T.lame_ratio(nu)
    prof = w.default_sponge_profile(60)
    vr = T.rayleigh_speed(nu)
    p = Problem(nx=nx, ny=ny, bc=(free, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                medium=Medium("homogeneous", 0.04 * lam_mu, 0.04, 1.0), tau=tau,
                sponge_thick=(0, 60, 0, 0), sponge_profiles=(None, prof, None, None),
                sources=[Source(float(xs), 2.0, 3.0, 0.0, 1.0, 1.0, 20.0, 30.0)],
                receivers=np.array([[xs + d1, 0], [xs + d2, 0]], np.int32), comp_mask=2)
    tr = stepper.run(p, nsteps=int(30 + d2 / vr + 40))["trace"][:, :, 0]
    # arrival picked within +-12 steps of the predicted time (the S pulse
    # arrives ~30 steps earlier at the near station)
    t1 = _peak_in(tr[:, 0], 30 + d1 / vr - 12, 30 + d1 / vr + 12)
    t2 = _peak_in(tr[:, 1], 30 + d2 / vr - 12, 30 + d2 / vr + 12)
    v = (d2 - d1) / (t2 - t1)
    assert abs(v - vr) / vr < 0.01, (v, vr)


def _growth_per_step(p, steps, seed=0):
    """Geometric-mean growth of a random state's norm per step (sources off)."""
    rng = np.random.default_rng(seed)
    f0 = rng.normal(size=(9, p.ny, p.nx))
    q = p.replace(sources=[], receivers=np.zeros((0, 2), np.int32))
    a = stepper.run(q, nsteps=steps // 2, fstar_init=f0, want_trace=False)["fstar"]
    b = stepper.run(q, nsteps=steps - steps // 2, fstar_init=a, want_trace=False)["fstar"]
    return (np.linalg.norm(b) / np.linalg.norm(a)) ** (1.0 / (steps - steps // 2))


def test_free_surface_rule_as_printed_is_unstable_zero_order_is_not():
    """The linear extrapolation of rho_air and P_xx,air printed in Sec. 6.2
    makes short-wavelength surface modes grow (4.6% per step at nu = 0.25,
    tau = 1); with the boundary cell's own values (zero order) the same grid
    is stable for nu in [0.1, 0.33]."""
    lam_mu = T.lame_ratio(0.25)
    base = Problem(nx=32, ny=24, bc=(BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                   medium=Medium("homogeneous", 0.04 * lam_mu, 0.04, 1.0), tau=1.0)
    assert _growth_per_step(base, 400) > 1.03
    for nu in (0.1, 0.25, 0.33):
        q = base.replace(bc=(BC_FREE0, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                         medium=Medium("homogeneous", 0.04 * T.lame_ratio(nu), 0.04, 1.0))
        assert _growth_per_step(q, 400) <= 1.0 + 1e-6, nu


@pytest.mark.parametrize("free", [BC_FREE, BC_FREE0])
def test_reflection_polarity_rigid_versus_free(free):
    """Sec. 6.3: a free surface reflects the vertical flux without a phase
    change (constructive at the surface), a rigid wall with a phase inversion
    (destructive). Compared with the same source in a periodic column."""
    nx, ny, depth = 64, 160, 30
    lam_mu = T.lame_ratio(0.25)
    med = Medium("homogeneous", 0.04 * lam_mu, 0.04, 1.0)
    src = Source(32.0, float(depth), 3.0, 0.0, 1.0, 1.0, 20.0, 30.0)
    rec = np.array([[32, 0]], np.int32)
    amps = {}
    for name, bc in (("free", (free, BC_PERIODIC)), ("rigid", (BC_RIGID, BC_PERIODIC)),
                     ("none", (BC_PERIODIC, BC_PERIODIC))):
        top = bc[0]
        # a periodic column cannot have a lone wall: close it far below
        bottom = BC_RIGID if top != BC_PERIODIC else BC_PERIODIC
        p = Problem(nx=nx, ny=ny, bc=(top, bottom, BC_PERIODIC, BC_PERIODIC), medium=med, tau=0.8,
                    sources=[src], receivers=rec, comp_mask=2)
        if top == BC_PERIODIC:
            # the reference: source placed mid-column, station at the same offset
            p = p.replace(sources=[Source(32.0, 80.0, 3.0, 0.0, 1.0, 1.0, 20.0, 30.0)],
                          receivers=np.array([[32, 80 - depth]], np.int32))
        tr = stepper.run(p, nsteps=110)["trace"][:, 0, 0]
        amps[name] = tr
    ref = np.abs(amps["none"]).max()
    assert np.abs(amps["free"]).max() > 1.6 * ref
    assert np.abs(amps["rigid"]).max() < 0.6 * ref


def test_rayleigh_protocol_two_turns_and_depth_profile():
    """Sec. 7's surface-wave experiment on the oracle: the speed from two
    complete turns around the periodic surface lies within 0.5% of the root
    of the Rayleigh equation (the paper: 0.14%), and the depth profile of j_y
    at step 1800 follows the half-space Rayleigh profile far better than a
    plain exponential or the printed form with a_P and a_S exchanged."""
    import _rayleigh as RY
    p1, p2 = RY.problems()
    a = stepper.run(p1, nsteps=RY.SWITCH)
    b = stepper.run(p2, nsteps=RY.PROFILE_STEP - RY.SWITCH, t0=RY.SWITCH, fstar_init=a["fstar"])
    c = stepper.run(p2, nsteps=RY.END - RY.PROFILE_STEP, t0=RY.PROFILE_STEP, fstar_init=b["fstar"])
    trace = np.concatenate([a["trace"][:, :, 0], b["trace"][:, :, 0], c["trace"][:, :, 0]])
    vr, _, _ = RY.speeds()
    v, spread, n = RY.two_turn_speed(trace)
    assert n >= 20 and abs(v - vr) / vr < 0.005, (v, vr, spread)
    fits = RY.depth_fits(b["mom"][2])
    assert fits["rayleigh"][1] < 0.5 * fits["exp"][1], fits
    assert fits["rayleigh"][1] < 0.1 * fits["printed"][1], fits
