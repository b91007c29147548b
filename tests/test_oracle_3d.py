"""Pins of the three-dimensional oracle (oracle/lbm3d_oracle.c), on both its
lattices (D3Q19 and D3Q27), to what the paper and the mathematics fix,
independently of the oracle's own formulas:

* the lattice: the isotropy conditions of the Chapman-Enskog analysis (Sec. 3)
  up to fourth order, opposite vectors, odd moments; the printed sixth-order
  condition, which D3Q27 meets and D3Q19 misses exactly on the components
  with three distinct index pairs (it has no (1,1,1) vectors);
* the equilibrium's moments: rho, j, P and the third moment b^2 (j d + ...)
  that closes the wave equation (Sec. 3);
* the collision's invariants and the momentum it adds (Sec. 2: rho and P
  conserved, m -> m + S with the implicit sponge);
* small-k phase speeds of the whole step on periodic volumes along three
  directions: shear b and compressional sqrt(3 b^2 - kappa), i.e.
  sqrt(mu/rho0) and sqrt((lambda + 2 mu)/rho0) (Sec. 2 and 4), extrapolated to
  k -> 0 from two wavenumbers;
* exact conservation of the totals of rho, m and P on periodic volumes and of
  rho and P in a closed rigid box (streaming permutes populations, bounce-back
  reverses them);
* uniform traction-free stress states as exact steady states of the free
  surface (Sec. 6.2), and a uniform state with P_zz != 0 not one;
* symmetry under the exchange of x and y and under the reflection z -> -z;
* the Gaussian x Ricker force's total impulse (Sec. 5) against its integral
  (2 pi sigma^2)^(3/2);
* receivers reading j / rho0 at their cells.
"""
import math

import numpy as np
import pytest

from oracle import stepper3d as O3
from workloads.problem import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID
from workloads.problem3 import Problem3, Source3, volume_field
from workloads.configs import lame_from_poisson

B2 = 1.0 / 3.0


Q = [19, 27]


def _lat(q):
    c, w, opp = O3.lattice(q)
    return c.astype(np.float64), w, opp


@pytest.mark.parametrize("q", Q)
def test_lattice_isotropy_and_opposites(q):
    c, w, opp = _lat(q)
    assert len({tuple(v) for v in c.astype(int)}) == q
    assert np.all(np.abs(c).sum(1) <= (2 if q == 19 else 3))
    assert np.array_equal(c[opp], -c)
    d = np.eye(3)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), B2 * d, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    d4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
          + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), B2 ** 2 * d4, atol=1e-16)
    # weights by speed class: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216
    s = np.abs(c).sum(1)
    want = {19: (1 / 3, 1 / 18, 1 / 36), 27: (8 / 27, 2 / 27, 1 / 54, 1 / 216)}[q]
    for k, wk in enumerate(want):
        assert np.allclose(w[s == k], wk)
    # the first 19 vectors of D3Q27 are D3Q19's, in the same order
    if q == 27:
        assert np.array_equal(c[:19], _lat(19)[0])


@pytest.mark.parametrize("q", Q)
def test_sixth_order_isotropy(q):
    """sum_i w c^6 = b^6 (Delta6 - 6 delta6) (Sec. 3): Delta6 is the sum over
    the 15 pairings of the six indices of products of deltas, delta6 = 1 when
    all six indices are equal."""
    import itertools
    c, w, _ = _lat(q)
    m6 = np.einsum("i,ia,ib,ic,id,ie,if->abcdef", w, c, c, c, c, c, c)
    ref = np.zeros((3,) * 6)
    distinct = np.zeros((3,) * 6, bool)
    for idx in itertools.product(range(3), repeat=6):
        counts = [idx.count(a) for a in range(3)]
        if any(k % 2 for k in counts):
            continue
        # pairings of equal indices: prod over axes of (count - 1)!!
        pairings = 1
        for k in counts:
            pairings *= {0: 1, 2: 1, 4: 3, 6: 15}[k]
        ref[idx] = B2 ** 3 * (pairings - (6 if max(counts) == 6 else 0))
        distinct[idx] = all(k == 2 for k in counts)
    if q == 27:
        assert np.allclose(m6, ref, atol=1e-16)
    else:
        assert np.allclose(m6[~distinct], ref[~distinct], atol=1e-16)
        assert np.allclose(m6[distinct], 0.0) and np.allclose(ref[distinct], B2 ** 3)


def _sym(P6):
    xx, xy, xz, yy, yz, zz = P6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


@pytest.mark.parametrize("q", Q)
def test_equilibrium_moments(q):
    c, w, _ = _lat(q)
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.normal()
        j = rng.normal(size=3)
        P6 = rng.normal(size=6)
        feq = O3.equilibrium(rho, j, P6, q)
        assert abs(feq.sum() - rho) < 1e-13
        assert np.allclose(feq @ c, j, atol=1e-13)
        assert np.allclose(np.einsum("i,ia,ib->ab", feq, c, c), _sym(P6), atol=1e-13)
        Q = np.einsum("i,ia,ib,ic->abc", feq, c, c, c)
        d = np.eye(3)
        Qref = B2 * (np.einsum("a,bc->abc", j, d) + np.einsum("b,ac->abc", j, d)
                     + np.einsum("c,ab->abc", j, d))
        assert np.allclose(Q, Qref, atol=1e-13)


@pytest.mark.parametrize("q", Q)
def test_collision_invariants_and_momentum_gain(q):
    c, w, _ = _lat(q)
    rng = np.random.default_rng(2)
    for tau in (0.55, 0.8, 1.0, 1.7):
        for A in (0.0, 0.05, 0.3):
            f = rng.normal(size=q)
            G = rng.normal(size=3)
            fs, j, S = O3.collide_cell(f, G, A, tau)
            m = f @ c
            assert abs(fs.sum() - f.sum()) < 1e-13
            assert np.allclose(np.einsum("i,ia,ib->ab", fs, c, c),
                               np.einsum("i,ia,ib->ab", f, c, c), atol=1e-13)
            assert np.allclose(fs @ c, m + S, atol=1e-13)
            # implicit sponge: j = m + S/2 with S = G - A j
            assert np.allclose(j, m + 0.5 * S, atol=1e-14)
            assert np.allclose(S, G - A * j, atol=1e-14)
            if A == 0.0:
                assert np.allclose(S, G, atol=0)


def _periodic(n, lam, mu, tau=1.0, shape=None, q=19):
    nz, ny, nx = shape if shape is not None else (n, n, n)
    return Problem3(nx=nx, ny=ny, nz=nz, faces=(BC_PERIODIC,) * 6, lam=lam, mu=mu, tau=tau, q=q)


def _step_matrix(kvec_int, shape, lam, mu, tau, q=19):
    """M(k): pre-collision populations at t+1 from those at t, for the plane
    wave exp(i k.x) with k = 2 pi kvec_int / (nx, ny, nz), read off one oracle
    step of cos and sin inputs."""
    nz, ny, nx = shape
    p = _periodic(0, lam, mu, tau, shape, q)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = 2 * np.pi * (kvec_int[0] * x / nx + kvec_int[1] * y / ny + kvec_int[2] * z / nz)
    M = np.zeros((q, q), complex)
    for jcol in range(q):
        out = []
        for wave in (np.cos(ph), np.sin(ph)):
            f0 = np.zeros((q,) + shape)
            f0[jcol] = wave
            out.append(O3.run(p, 1, f_init=f0, want_trace=False)["f"][:, 0, 0, 0])
        M[:, jcol] = out[0] + 1j * out[1]
    return M


def _speeds(M, kabs):
    lam = np.linalg.eigvals(M)
    # the slow modes (|lambda| near 1; the kinetic ones decay like 1 - 1/tau)
    # that propagate
    prop = lam[(np.abs(lam) > 0.5) & (np.abs(np.angle(lam)) > 1e-9)]
    assert prop.size == 6, lam
    sp = np.sort(np.abs(np.angle(prop)) / kabs)
    return sp


@pytest.mark.parametrize("q", Q)
@pytest.mark.parametrize("nu", [0.1, 0.33])
@pytest.mark.parametrize("direction,sizes", [((1, 0, 0), ((3, 3, 40), (3, 3, 80))),
                                              ((1, 1, 0), ((3, 32, 32), (3, 64, 64))),
                                              ((1, 1, 1), ((16, 16, 16), (32, 32, 32)))])
def test_small_k_phase_speeds(direction, sizes, nu, q):
    lam, mu = lame_from_poisson(nu)
    kappa = B2 * (mu - lam) / mu
    cs, cp = math.sqrt(B2), math.sqrt(3 * B2 - kappa)
    assert abs(cp - math.sqrt((lam + 2 * mu) / (mu / B2))) < 1e-14
    got = []
    for shape in sizes:
        n = shape[2]
        kabs = 2 * np.pi / n * math.sqrt(sum(d * d for d in direction))
        sp = _speeds(_step_matrix(direction, shape, lam, mu, 1.0, q), kabs)
        # the propagating pairs: 2 compressional, 4 shear (two polarisations)
        fast = sp[4:]
        slow = sp[:4]
        # each pair is one mode; the two shear polarisations may differ at
        # finite k (lattice anisotropy of the O(k^2) dispersion), by < 1e-3
        assert np.allclose(fast, fast[0], rtol=1e-9) and np.allclose(slow, slow[0], rtol=1e-3)
        got.append((fast.mean(), slow.mean()))
        assert abs(got[-1][0] / cp - 1) < 0.03 and abs(got[-1][1] / cs - 1) < 0.03, (shape, fast, slow)
    # second order in k: Richardson extrapolation to k -> 0
    for which, ref in ((0, cp), (1, cs)):
        c0 = (4 * got[1][which] - got[0][which]) / 3
        assert abs(c0 / ref - 1) < 2e-4, (which, got, c0, ref)


def _totals(f, c):
    tot = f.reshape(f.shape[0], -1).sum(1)
    return tot.sum(), tot @ c, np.einsum("i,ia,ib->ab", tot, c, c)


@pytest.mark.parametrize("q", Q)
def test_periodic_volume_conserves_rho_m_P(q):
    c, _, _ = _lat(q)
    lam, mu = lame_from_poisson(0.2)
    p = _periodic(0, lam, mu, tau=0.8, shape=(9, 11, 13), q=q)
    f0 = np.random.default_rng(3).normal(size=(q, 9, 11, 13)) * 1e-2
    out = O3.run(p, 12, f_init=f0, want_trace=False)["f"]
    a, b = _totals(f0, c), _totals(out, c)
    assert abs(a[0] - b[0]) < 1e-12
    assert np.allclose(a[1], b[1], atol=1e-12)
    assert np.allclose(a[2], b[2], atol=1e-12)


@pytest.mark.parametrize("q", Q)
def test_closed_rigid_box_conserves_rho_and_P(q):
    c, _, _ = _lat(q)
    lam, mu = lame_from_poisson(0.25)
    p = Problem3(nx=12, ny=10, nz=9, faces=(BC_RIGID,) * 6, lam=lam, mu=mu, tau=0.9, q=q)
    f0 = np.random.default_rng(4).normal(size=(q, 9, 10, 12)) * 1e-2
    out = O3.run(p, 10, f_init=f0, want_trace=False)["f"]
    a, b = _totals(f0, c), _totals(out, c)
    assert abs(a[0] - b[0]) < 1e-12
    assert np.allclose(a[2], b[2], atol=1e-12)
    assert not np.allclose(a[1], b[1], atol=1e-6)   # walls take momentum


@pytest.mark.parametrize("q", Q)
@pytest.mark.parametrize("top,bottom", [(BC_FREE0, BC_FREE0), (BC_FREE, BC_FREE0), (BC_FREE, BC_RIGID)])
def test_traction_free_uniform_stress_is_steady(top, bottom, q):
    """f = feq(rho, 0, P) with P n = 0 on the z faces (P_xz = P_yz = P_zz = 0)
    is left unchanged by the free surfaces; with P_zz != 0 it is not."""
    lam, mu = lame_from_poisson(0.25)
    shape = (8, 7, 9)
    p = Problem3(nx=9, ny=7, nz=8, faces=(top, bottom, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC,
                                          BC_PERIODIC), lam=lam, mu=mu, tau=0.9, q=q)
    rho = 0.013
    P_free = np.array([0.004, -0.002, 0.0, 0.003, 0.0, 0.0])
    feq = O3.equilibrium(rho, np.zeros(3), P_free, q)
    f0 = np.broadcast_to(feq[:, None, None, None], (q,) + shape).copy()
    out = O3.run(p, 6, f_init=f0, want_trace=False)["f"]
    assert np.max(np.abs(out - f0)) < 1e-15
    P_loaded = P_free + np.array([0, 0, 0, 0, 0, 0.002])
    feq = O3.equilibrium(rho, np.zeros(3), P_loaded, q)
    f1 = np.broadcast_to(feq[:, None, None, None], (q,) + shape).copy()
    out = O3.run(p, 1, f_init=f1, want_trace=False)["f"]
    assert np.max(np.abs(out - f1)) > 1e-5
    if q == 27:
        # the corner links through a z face carry the tangential shear P_xy:
        # a uniform state whose air state lacked it would not be steady
        P_shear = np.array([0.0, 0.003, 0.0, 0.0, 0.0, 0.0])
        feq = O3.equilibrium(rho, np.zeros(3), P_shear, q)
        f2 = np.broadcast_to(feq[:, None, None, None], (q,) + shape).copy()
        out = O3.run(p, 4, f_init=f2, want_trace=False)["f"]
        assert np.max(np.abs(out - f2)) < 1e-15
    # a rigid box keeps any uniform state at rest
    q = p.replace(faces=(BC_RIGID,) * 6)
    out = O3.run(q, 6, f_init=f1, want_trace=False)["f"]
    assert np.max(np.abs(out - f1)) < 1e-15


def _perm_index(c, mapc):
    """Index map k -> i with c_i = mapc(c_k)."""
    lut = {tuple(v): i for i, v in enumerate(c.astype(int))}
    return np.array([lut[tuple(mapc(v))] for v in c.astype(int)])


@pytest.mark.parametrize("q", Q)
def test_exchange_of_x_and_y(q):
    c, _, _ = _lat(q)
    p = volume_field(nx=14, ny=11, nz=9, seed=6, nsteps=8,
                     faces=(BC_FREE0, BC_RIGID, BC_RIGID, BC_RIGID, BC_PERIODIC, BC_PERIODIC), q=q)
    p = p.replace(sponge_thick=(0, 3, 2, 0, 0, 0),
                  sponge_profiles=(None, np.array([0.3, 0.2, 0.1]), np.array([0.2, 0.1]), None, None, None))
    f0 = np.random.default_rng(7).normal(size=(q, 9, 11, 14)) * 1e-3
    a = O3.run(p, 8, fstar_init=f0)
    sw = lambda arr: np.swapaxes(arr, -1, -2)
    s = p.sources[0]
    pq = Problem3(nx=p.ny, ny=p.nx, nz=p.nz,
                 faces=(p.faces[0], p.faces[1], p.faces[4], p.faces[5], p.faces[2], p.faces[3]),
                 lam=sw(p.lam), mu=sw(p.mu), rho0=sw(p.rho0), tau=p.tau,
                 sponge_thick=(0, 3, 0, 0, 2, 0),
                 sponge_profiles=(None, np.array([0.3, 0.2, 0.1]), None, None, np.array([0.2, 0.1]), None),
                 sources=[Source3(s.y, s.x, s.z, s.sigma, s.dir_y, s.dir_x, s.dir_z, s.amp, s.period, s.t0)],
                 receivers=p.receivers[:, [1, 0, 2]].copy(), comp_mask=7, q=q)
    k = _perm_index(c, lambda v: (v[1], v[0], v[2]))   # population k of p -> k[...] of pq
    g0 = np.zeros((q, 9, 14, 11))
    g0[k] = sw(f0)
    b = O3.run(pq, 8, fstar_init=g0)
    assert np.allclose(b["fstar"][k], sw(a["fstar"]), atol=1e-15, rtol=0)
    assert np.allclose(b["trace"][:, :, [1, 0, 2]], a["trace"], atol=1e-15, rtol=0)
    mom_perm = [0, 2, 1, 3, 7, 5, 8, 4, 6, 9]   # where each field of p sits in pq
    assert np.allclose(b["mom"][mom_perm], sw(a["mom"]), atol=1e-15, rtol=0)


@pytest.mark.parametrize("q", Q)
def test_reflection_of_z(q):
    c, _, _ = _lat(q)
    p = volume_field(nx=10, ny=9, nz=12, seed=8, nsteps=7,
                     faces=(BC_FREE, BC_FREE0, BC_PERIODIC, BC_PERIODIC, BC_RIGID, BC_RIGID), q=q)
    f0 = np.random.default_rng(9).normal(size=(q, 12, 9, 10)) * 1e-3
    a = O3.run(p, 7, fstar_init=f0)
    fl = lambda arr: arr[..., ::-1, :, :].copy()
    s = p.sources[0]
    pq = p.replace(faces=(BC_FREE0, BC_FREE) + p.faces[2:], lam=fl(p.lam), mu=fl(p.mu), rho0=fl(p.rho0),
                  sources=[Source3(s.x, s.y, p.nz - 1 - s.z, s.sigma, s.dir_x, s.dir_y, -s.dir_z,
                                   s.amp, s.period, s.t0)],
                  receivers=np.stack([p.receivers[:, 0], p.receivers[:, 1], p.nz - 1 - p.receivers[:, 2]],
                                     1).astype(np.int32))
    k = _perm_index(c, lambda v: (v[0], v[1], -v[2]))
    g0 = np.zeros_like(f0)
    g0[k] = fl(f0)
    b = O3.run(pq, 7, fstar_init=g0)
    assert np.allclose(b["fstar"][k], fl(a["fstar"]), atol=1e-15, rtol=0)
    assert np.allclose(b["trace"] * np.array([1, 1, -1]), a["trace"], atol=1e-15, rtol=0)
    sign = np.array([1, 1, 1, -1, 1, 1, -1, 1, -1, 1])[:, None, None, None]
    assert np.allclose(sign * b["mom"], fl(a["mom"]), atol=1e-15, rtol=0)


@pytest.mark.parametrize("q", Q)
def test_source_impulse_matches_the_gaussian_integral(q):
    """From rest, one step at the Ricker peak adds total momentum
    amp (2 pi sigma^2)^(3/2) dir (the lattice sum of a Gaussian of sigma >= 2
    equals its integral to far below 1e-12; the 9-sigma cut drops e^-40)."""
    c, _, _ = _lat(q)
    lam, mu = lame_from_poisson(0.25)
    sig, amp = 2.0, 0.7
    d = np.array([0.48, 0.6, 0.64])
    p = Problem3(nx=40, ny=40, nz=40, faces=(BC_PERIODIC,) * 6, lam=lam, mu=mu,
                 sources=[Source3(19.3, 20.6, 21.1, sig, d[0], d[1], d[2], amp, 30.0, 5.0)], q=q)
    out = O3.run(p, 1, t0=5, want_trace=False)["f"]
    m = out.reshape(q, -1).sum(1) @ c
    ref = amp * (2 * math.pi * sig * sig) ** 1.5 * d
    assert np.allclose(m, ref, rtol=1e-12, atol=0), (m, ref)
    # one step earlier the Ricker factor is (1 - 2 a^2) exp(-a^2), a = pi / 30
    out = O3.run(p, 1, t0=4, want_trace=False)["f"]
    a = math.pi / 30.0
    assert np.allclose(out.reshape(q, -1).sum(1) @ c,
                       ref * (1 - 2 * a * a) * math.exp(-a * a), rtol=1e-12, atol=0)


@pytest.mark.parametrize("q", Q)
def test_receivers_read_the_flux_over_rho0(q):
    p = volume_field(nx=12, ny=10, nz=8, seed=10, nsteps=9,
                     faces=(BC_FREE0, BC_RIGID) + (BC_PERIODIC,) * 4, q=q)
    p = p.replace(sponge_thick=(0, 3, 0, 0, 0, 0), sponge_profiles=(None, np.array([0.3, 0.2, 0.1]),
                                                                    None, None, None, None))
    full = O3.run(p, 9)
    part = O3.run(p, 8)
    _, _, rho0 = p.full()
    r = p.receivers
    want = part["mom"][1:4][:, r[:, 2], r[:, 1], r[:, 0]].T / rho0[r[:, 2], r[:, 1], r[:, 0]][:, None]
    assert np.allclose(full["trace"][8], want, rtol=1e-14, atol=1e-18)
    assert np.array_equal(full["trace"][:8], part["trace"])


@pytest.mark.parametrize("q", Q)
@pytest.mark.parametrize("faces", [(BC_RIGID, BC_FREE0, BC_RIGID, BC_RIGID, BC_PERIODIC, BC_PERIODIC),
                                   (BC_FREE, BC_RIGID, BC_PERIODIC, BC_PERIODIC, BC_RIGID, BC_RIGID)])
def test_density_gradient_exact_for_linear_density_up_to_the_faces(faces, q):
    """The centred difference of eq. FDrho with the linearly extrapolated ghost
    beyond non-periodic faces is exact for a density linear along those axes:
    the flux the state carries at rest is j = G/2 = kappa grad(rho)/2 in every
    cell, boundary cells included."""
    lam, mu = lame_from_poisson(0.1)
    kappa = B2 * (mu - lam) / mu
    nz, ny, nx = 7, 6, 8
    p = Problem3(nx=nx, ny=ny, nz=nz, faces=faces, lam=lam, mu=mu, tau=0.9, q=q)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    slope = np.array([0.0, 0.0, 0.0])
    per = [faces[2] == BC_PERIODIC, faces[4] == BC_PERIODIC, faces[0] == BC_PERIODIC]
    slope[[a for a in range(3) if not per[a]]] = [3e-3, -2e-3, 1.5e-3][:sum(not q for q in per)]
    rho = 0.01 + slope[0] * x + slope[1] * y + slope[2] * z
    f0 = np.zeros((q,) + rho.shape)
    for k in np.ndindex(rho.shape):
        f0[(slice(None),) + k] = O3.equilibrium(rho[k], np.zeros(3), np.array([B2, 0, 0, B2, 0, B2]) * rho[k], q)
    mom = O3.run(p, 0, f_init=f0, want_trace=False)["mom"]
    assert np.allclose(mom[0], rho, atol=1e-16)
    for a in range(3):
        assert np.allclose(mom[1 + a], 0.5 * kappa * slope[a], atol=1e-15, rtol=0), a
