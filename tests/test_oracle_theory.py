"""Pins of the analysis tools against what the paper fixes in closed form.

The von Neumann matrix M(k) is rebuilt from the scheme; here it is tied to the
paper's own continuum results: the Navier wave speeds (Sec. 2), the dissipative
modified moment chain of the Chapman-Enskog analysis (Sec. 3, Appendix A), the
stability statements of Sec. 4, and the damped Navier equation of Sec. 6.4.
"""
import math

import numpy as np
import pytest

from oracle import theory as T
from _golden import paper_values


def test_rayleigh_root_matches_printed_value():
    pv = paper_values()
    vp, vs = T.wave_speeds(0.25)
    vr = T.rayleigh_speed(0.25)
    # printed: v_R = sqrt(0.8453/3) = 0.5308 (Sec. 7, eq. vR)
    assert abs(vr - pv["rayleigh_speed_theory_nu025"]) < 5e-5
    assert abs((vr / vs) ** 2 - pv["rayleigh_ratio_sq_nu025"]) < 5e-5
    # closed form for a Poisson solid: (v_R/v_S)^2 = 2 - 2/sqrt(3)
    assert abs((vr / vs) ** 2 - (2.0 - 2.0 / math.sqrt(3.0))) < 1e-12


def test_wave_speed_relations():
    for nu in (0.0, 0.1, 0.25, 0.33, 0.4):
        vp, vs = T.wave_speeds(nu)
        assert abs(vs - 1.0 / math.sqrt(3.0)) < 1e-15        # v_S = b
        lam_mu = T.lame_ratio(nu)
        assert abs(T.poisson_ratio(lam_mu, 1.0) - nu) < 1e-14  # eq. nu
        # eq. VpVs with mu/rho0 = b^2: v_P^2 = b^2 (lambda/mu + 2)
        assert abs(vp * vp - T.B2 * (lam_mu + 2.0)) < 1e-14
        # Lambda = (mu - lambda)/(rho0 b^2) = (1 - 4 nu)/(1 - 2 nu)
        assert abs(T.Lambda(nu) - (1.0 - lam_mu)) < 1e-13
    assert abs(T.wave_speeds(0.25)[0] - 1.0) < 1e-15          # v_P = 1 at nu = 1/4
    assert abs(T.nu_limit() - paper_values()["nu_limit"]) < 1e-15


@pytest.mark.parametrize("nu", [0.0, 0.1, 0.25, 0.33])
@pytest.mark.parametrize("tau", [0.55, 1.0])
def test_vn_small_k_matches_navier_and_modified_chain(nu, tau):
    """Small-k eigenvalues of M(k): phase speeds are the Navier speeds, and
    damping rates equal those of the paper's modified moment chain."""
    vp, vs = T.wave_speeds(nu)
    k = 0.02
    for theta in (0.0, 0.3, math.pi / 4, 1.1):
        kx, ky = k * math.cos(theta), k * math.sin(theta)
        lam_vn = T.vn_eigs(kx, ky, nu, tau)
        s_macro = np.linalg.eigvals(T.macro_matrix(kx, ky, nu, tau))
        speeds = sorted(abs(np.angle(l)) / k for l in lam_vn if abs(l) > 0.9)
        # four propagating modes: +-v_S and +-v_P
        prop = [v for v in speeds if v > 0.1]
        assert len(prop) == 4
        assert abs(prop[0] - vs) / vs < 1e-4 and abs(prop[1] - vs) / vs < 1e-4
        assert abs(prop[2] - vp) / vp < 1e-4 and abs(prop[3] - vp) / vp < 1e-4
        scale = (tau - 0.5) * T.B2 * k * k
        for s in s_macro:
            lv = lam_vn[np.argmin(abs(lam_vn - np.exp(s)))]
            assert abs(-math.log(abs(lv)) - (-s.real)) < 2e-3 * scale + 1e-12


def test_vn_decay_coefficients_of_survey_probe():
    """Decay -ln|l| = c (tau - 1/2) b^2 k^2 of the acoustic pairs: S on an
    axis c = 1, P on an axis c = 0, S at 45 degrees c = 1/4, P at 45 degrees
    c = 3/4 for a Poisson solid (all from eq. MomentChain2)."""
    k, tau, nu = 0.02, 0.8, 0.25
    scale = (tau - 0.5) * T.B2 * k * k

    def coeffs(theta):
        l = T.vn_eigs(k * math.cos(theta), k * math.sin(theta), nu, tau)
        out = {}
        for v in l:
            sp = abs(np.angle(v)) / k
            if sp > 0.1:
                out[round(sp, 2)] = -math.log(abs(v)) / scale
        return out

    ax = coeffs(0.0)
    assert abs(ax[0.58] - 1.0) < 1e-3 and abs(ax[1.0]) < 1e-3
    dg = coeffs(math.pi / 4)
    assert abs(dg[0.58] - 0.25) < 1e-3 and abs(dg[1.0] - 0.75) < 1e-3


@pytest.mark.parametrize("tau", [0.51, 0.55, 1.0, 2.0, 10.0])
def test_poisson_solid_unconditionally_stable(tau):
    """Sec. 4: unconditionally stable for nu = 0.25."""
    assert T.max_growth(0.25, tau, n=33) <= 1.0 + 1e-12


def test_low_nu_instability_is_45_degree_high_k():
    """Sec. 4: at low nu the unstable wave vectors sit near 45 degrees and
    near |k| = pi; the 45-degree stripes are 2.1 cells apart."""
    ks = np.linspace(0.05, math.pi, 90)
    worst, arg = 0.0, None
    unstable = []
    for kx in ks:
        for ky in ks:
            g = np.abs(T.vn_eigs(kx, ky, 0.0, 0.55)).max()
            if g > 1 + 1e-9:
                unstable.append((kx, ky))
            if g > worst:
                worst, arg = g, (kx, ky)
    assert worst > 1.01
    for kx, ky in unstable:
        assert abs(math.degrees(math.atan2(ky, kx)) - 45.0) < 20.0
        assert math.hypot(kx, ky) > 2.0
    spacing = 2 * math.pi / math.hypot(*arg)
    assert abs(spacing - paper_values()["stripe_spacing"]) / 2.1 < 0.05


def test_high_nu_instability_all_directions_but_not_low_k():
    """Sec. 4: at nu = 0.4 every direction is unstable at high enough k, and
    only |k| > pi/3 is unstable. (Exactly on an axis the growth is marginal,
    |l| = 1; every oblique direction has unstable wave vectors.)"""
    kthr = paper_values()["unstable_k_threshold_nu04"]
    for theta in np.radians(np.linspace(5.0, 85.0, 9)):
        kmax = math.pi / max(math.cos(theta), math.sin(theta))
        ks = np.linspace(0.02, kmax, 120)
        g = [np.abs(T.vn_eigs(k * math.cos(theta), k * math.sin(theta), 0.4, 0.55)).max()
             for k in ks]
        assert max(g) > 1 + 1e-9
        for k, gk in zip(ks, g):
            if k < kthr:
                assert gk <= 1 + 1e-9


def test_sponge_zero_k_is_trapezoidal_damping():
    """The -A j term handled as a forcing with the half-step correction damps
    the k = 0 flux by (1 - A/2)/(1 + A/2) per step (trapezoidal rule for
    d_t j = -A j, Sec. 6.4)."""
    for A in (0.01, 0.1, 0.5):
        lam = T.vn_eigs(0.0, 0.0, 0.1, 0.8, A)
        target = (1 - A / 2) / (1 + A / 2)
        assert np.min(abs(lam - target)) < 1e-13
        assert np.sum(abs(lam - target) < 1e-12) == 2   # j_x and j_y


def test_sponge_small_k_matches_damped_navier():
    """Small-k propagating modes with a uniform sponge solve the damped Navier
    dispersion relation w^2 + i A w = v^2 k^2 (eq. RelaxationNavierJ)."""
    nu, tau, A, k = 0.25, 0.55, 0.02, 0.03
    vp, vs = T.wave_speeds(nu)
    lam = T.vn_eigs(k, 0.0, nu, tau, A)
    for v in (vp, vs):
        # root with positive real frequency: w = -iA/2 + sqrt(v^2 k^2 - A^2/4)
        w = -0.5j * A + math.sqrt(v * v * k * k - A * A / 4)
        target = np.exp(-1j * w)
        best = lam[np.argmin(abs(lam - target))]
        assert abs(best - target) < 2e-4
