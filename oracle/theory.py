"""Closed forms and linear analyses of the paper (test infrastructure).

* Navier wave speeds (Sec. 2, eqs. VpVs, VpVsRatio, nu) in lattice units,
  where the S-wave speed equals b = 1/sqrt(3) (Sec. 2, after eq. MomentsFeq).
* Lambda(nu) of Sec. 4.
* The von Neumann amplification matrix M(k) of Sec. 4, rebuilt from the scheme
  (the printed matrix of eq. VN mixes sign conventions): for a plane wave
  f_i(x, t) = F_i exp(i k.x), one step maps F to
      M(k) F = diag(exp(-i k.c_l)) [ (1 - 1/tau) I + (1/tau) E(k)
                                     + (1 - 1/(2 tau)) Phi(k) ] F,
  where E(k) maps F to f^eq and Phi(k) to the forcing populations; the
  centred difference of eq. FDrho has the symbol i sin(k_alpha).
* The paper's modified moment chain (eq. MomentChain2 with the dissipative
  term of Appendix A, eq. Q1) as a 6x6 linear system in Fourier space.
* The Rayleigh equation (Sec. 7) in the form eta^3 - 8 eta^2 + (24 - 16 g) eta
  - 16 (1 - g) = 0, eta = (v_R/v_S)^2, g = v_S^2/v_P^2.
"""
from __future__ import annotations

import math

import numpy as np

B2 = 1.0 / 3.0
# D2Q9 in the ordering used throughout: rest, 4 axis links, 4 diagonals.
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def poisson_ratio(lam: float, mu: float) -> float:
    """eq. nu."""
    return lam / (2.0 * (lam + mu))


def lame_ratio(nu: float) -> float:
    """lambda / mu for a given Poisson ratio (inverse of eq. nu)."""
    return 2.0 * nu / (1.0 - 2.0 * nu)


def Lambda(nu: float) -> float:
    """Lambda = (mu - lambda)/(rho0 b^2) = (1 - 4 nu)/(1 - 2 nu), Sec. 4."""
    return (1.0 - 4.0 * nu) / (1.0 - 2.0 * nu)


def kappa(nu: float) -> float:
    """Elastic-force coefficient (mu - lambda)/rho0 in lattice units."""
    return B2 * Lambda(nu)


def wave_speeds(nu: float):
    """(v_P, v_S) in lattice units: v_S = b, v_P/v_S from eq. VpVsRatio."""
    vs = math.sqrt(B2)
    return vs * math.sqrt((2.0 - 2.0 * nu) / (1.0 - 2.0 * nu)), vs


def rayleigh_speed(nu: float) -> float:
    """Rayleigh-wave speed: the root eta in (0, 1) of the Rayleigh cubic."""
    vp, vs = wave_speeds(nu)
    g = (vs / vp) ** 2
    roots = np.roots([1.0, -8.0, 24.0 - 16.0 * g, -16.0 * (1.0 - g)])
    good = [r.real for r in roots if abs(r.imag) < 1e-12 and 0.0 < r.real < 1.0]
    if len(good) != 1:
        raise ValueError("no unique Rayleigh root")
    return vs * math.sqrt(good[0])


def nu_limit() -> float:
    """Poisson ratio at which v_P reaches 2 (the centred difference lets
    information travel two cells per step), Sec. 4: v_P/v_S = 2 sqrt(3)."""
    r2 = 12.0  # (v_P/v_S)^2 = (2 - 2 nu)/(1 - 2 nu)
    return (r2 - 2.0) / (2.0 * r2 - 2.0)


def vn_matrix(kx: float, ky: float, nu: float, tau: float, A: float = 0.0) -> np.ndarray:
    """9x9 amplification matrix of one step for the plane wave exp(i k.x)."""
    kap = kappa(nu)
    one = np.ones(9)
    # Linear functionals of the populations (rows): moments of eq. MomentsFeq.
    rho = one.astype(complex)
    mx, my = CX.astype(complex), CY.astype(complex)
    pxx, pxy, pyy = CX * CX, CX * CY, CY * CY
    # Elastic source G = kappa D rho with D = i sin k (eq. FDrho, eq. S).
    gx = kap * 1j * math.sin(kx) * rho
    gy = kap * 1j * math.sin(ky) * rho
    # Flux and sponge-corrected source (implicit sponge).
    jx = (mx + 0.5 * gx) / (1.0 + 0.5 * A)
    jy = (my + 0.5 * gy) / (1.0 + 0.5 * A)
    sx = gx - A * jx
    sy = gy - A * jy
    pnxx = pxx - B2 * rho
    pnyy = pyy - B2 * rho
    pnxy = pxy.astype(complex)
    E = np.zeros((9, 9), complex)
    Phi = np.zeros((9, 9), complex)
    for l in range(9):
        cx, cy = CX[l], CY[l]
        E[l] = W[l] * (rho + (jx * cx + jy * cy) / B2 +
                       (pnxx * (cx * cx - B2) + 2 * pnxy * cx * cy + pnyy * (cy * cy - B2)) / (2 * B2 * B2))
        Phi[l] = W[l] * (cx * sx + cy * sy) / B2
    coll = (1.0 - 1.0 / tau) * np.eye(9) + E / tau + (1.0 - 0.5 / tau) * Phi
    shift = np.exp(-1j * (kx * CX + ky * CY))
    return shift[:, None] * coll


def vn_eigs(kx, ky, nu, tau, A=0.0):
    return np.linalg.eigvals(vn_matrix(kx, ky, nu, tau, A))


def max_growth(nu: float, tau: float, n: int = 64, kmax: float = math.pi) -> float:
    """max |eigenvalue| over a uniform n x n grid of k in [0, kmax]^2."""
    ks = np.linspace(0.0, kmax, n)
    m = 0.0
    for kx in ks:
        for ky in ks:
            m = max(m, np.abs(vn_eigs(kx, ky, nu, tau)).max())
    return m


def macro_matrix(kx: float, ky: float, nu: float, tau: float) -> np.ndarray:
    """Right-hand side L(k) of dU/dt = L U for U = (rho, j_x, j_y, P_xx, P_xy,
    P_yy) under the modified moment chain (eq. MomentChain2): mass and flux
    equations exact, stress equation with the dissipative term
    (tau - 1/2) b^2 d_g (d_a Pn_bg + d_b Pn_ag + d_g Pn_ab - 3 delta_abgk d_k Pn_kk)
    and d -> i k."""
    kap = kappa(nu)
    k = np.array([kx, ky])
    nud = (tau - 0.5) * B2
    R, JX, JY, XX, XY, YY = range(6)
    L = np.zeros((6, 6), complex)
    ik = 1j * k
    # d_t rho = -d_a j_a
    L[R, JX] = -ik[0]
    L[R, JY] = -ik[1]
    # d_t j_a = -d_b P_ab + kappa d_a rho
    L[JX, XX] = -ik[0]; L[JX, XY] = -ik[1]; L[JX, R] = kap * ik[0]
    L[JY, XY] = -ik[0]; L[JY, YY] = -ik[1]; L[JY, R] = kap * ik[1]
    # d_t P_ab = -b^2 (d_a j_b + d_b j_a + delta_ab d_g j_g) + dissipation
    pidx = {(0, 0): XX, (0, 1): XY, (1, 0): XY, (1, 1): YY}
    jidx = [JX, JY]
    for (a, b), row in ((( 0, 0), XX), ((0, 1), XY), ((1, 1), YY)):
        L[row, jidx[b]] += -B2 * ik[a]
        L[row, jidx[a]] += -B2 * ik[b]
        if a == b:
            L[row, JX] += -B2 * ik[0]
            L[row, JY] += -B2 * ik[1]

    # Dissipation acts on P^n = P - b^2 rho I: build the map U -> P^n_cd.
    def pn(c, d):
        v = np.zeros(6, complex)
        v[pidx[(c, d)]] = 1.0
        if c == d:
            v[R] -= B2
        return v

    for (a, b), row in (((0, 0), XX), ((0, 1), XY), ((1, 1), YY)):
        acc = np.zeros(6, complex)
        for g in range(2):
            acc += ik[g] * ik[a] * pn(b, g) + ik[g] * ik[b] * pn(a, g) + ik[g] * ik[g] * pn(a, b)
        if a == b:
            acc -= 3.0 * ik[a] * ik[a] * pn(a, a)
        L[row] += nud * acc
    return L
