"""Fourier spectral / Crank-Nicolson reference for the Navier equation on a
periodic box (Appendix B; test infrastructure).

State per wave vector: J = (j_x, j_y, d_t j_x, d_t j_y) (eq. J). The Navier
equation for j in Fourier space (eq. NavierFourier) is integrated with the
Crank-Nicolson rule (eq. Crank-Nicholson) written as M J_{n+1} = N (J_n, G_x,
G_y) (eqs. MatrixFourier, M, N, ABC), with G = (d_t F_n + d_t F_{n+1}) / rho0.
Coefficients in lattice units: b^2 = mu/rho0 = 1/3, a^2 = (lambda + 2 mu)/rho0,
d^2 = (lambda + mu)/rho0, with lambda/mu fixed by the Poisson ratio.
"""
from __future__ import annotations

import math

import numpy as np

from . import theory


def ricker_dt(t: float, period: float, t0: float) -> float:
    """Time derivative of the Ricker wavelet (1 - 2 a^2) exp(-a^2), a = pi (t - t0)/T."""
    a = math.pi * (t - t0) / period
    da = math.pi / period
    return (-4.0 * a * da) * math.exp(-a * a) + (1.0 - 2.0 * a * a) * (-2.0 * a * da) * math.exp(-a * a)


def gaussian_field(n: int, xs: float, ys: float, sigma: float) -> np.ndarray:
    """exp(-r^2 / (2 sigma^2)) on an n x n periodic grid (minimum image),
    set to 0 beyond 9 sigma -- the spatial factor of the body force."""
    x = np.arange(n, dtype=float)
    dx = x - xs
    dx = np.where(dx > n / 2, dx - n, dx)
    dx = np.where(dx < -n / 2, dx + n, dx)
    dy = x - ys
    dy = np.where(dy > n / 2, dy - n, dy)
    dy = np.where(dy < -n / 2, dy + n, dy)
    r2 = dy[:, None] ** 2 + dx[None, :] ** 2
    g = np.exp(-r2 / (2.0 * sigma * sigma))
    return np.where(r2 > 81.0 * sigma * sigma, 0.0, g)


def solve(n: int, nu: float, nsteps: int, src, rho0: float = 1.0):
    """j_x, j_y (each n x n) at time nsteps for a single Gaussian x Ricker
    source ``src`` (a workloads.Source) on an n x n periodic box."""
    lam_over_mu = theory.lame_ratio(nu)
    b2 = theory.B2
    a2 = b2 * (lam_over_mu + 2.0)
    d2 = b2 * (lam_over_mu + 1.0)
    k = 2.0 * np.pi * np.fft.fftfreq(n)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    A = a2 * kx ** 2 + b2 * ky ** 2
    B = d2 * kx * ky
    Cc = a2 * ky ** 2 + b2 * kx ** 2
    dt = 1.0
    g = gaussian_field(n, src.x, src.y, src.sigma) * src.amp
    gh = np.fft.fft2(g)
    fxh = gh * src.dir_x
    fyh = gh * src.dir_y
    # Per-k 4x4 systems: M J_{n+1} = N (J_n, Gx, Gy).
    shape = kx.shape
    M = np.zeros(shape + (4, 4))
    M[..., 0, 0] = 1; M[..., 0, 2] = -dt / 2
    M[..., 1, 1] = 1; M[..., 1, 3] = -dt / 2
    M[..., 2, 0] = A * dt / 2; M[..., 2, 1] = B * dt / 2; M[..., 2, 2] = 1
    M[..., 3, 0] = B * dt / 2; M[..., 3, 1] = Cc * dt / 2; M[..., 3, 3] = 1
    N = np.zeros(shape + (4, 6))
    N[..., 0, 0] = 1; N[..., 0, 2] = dt / 2
    N[..., 1, 1] = 1; N[..., 1, 3] = dt / 2
    N[..., 2, 0] = -A * dt / 2; N[..., 2, 1] = -B * dt / 2; N[..., 2, 2] = 1; N[..., 2, 4] = dt / 2
    N[..., 3, 0] = -B * dt / 2; N[..., 3, 1] = -Cc * dt / 2; N[..., 3, 3] = 1; N[..., 3, 5] = dt / 2
    MinvN = np.linalg.solve(M, N)
    J = np.zeros(shape + (4,), complex)
    for step in range(nsteps):
        r0 = ricker_dt(step, src.period, src.t0)
        r1 = ricker_dt(step + 1, src.period, src.t0)
        gx = (fxh * r0 + fxh * r1) / rho0
        gy = (fyh * r0 + fyh * r1) / rho0
        rhs = np.concatenate([J, gx[..., None], gy[..., None]], axis=-1)
        J = np.einsum("...ij,...j->...i", MinvN, rhs)
    jx = np.real(np.fft.ifft2(J[..., 0]))
    jy = np.real(np.fft.ifft2(J[..., 1]))
    return jx, jy


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    """Relative L2 misfit of eq. pmisfit."""
    return float(np.sqrt(np.sum((a - ref) ** 2) / np.sum(ref ** 2)))
