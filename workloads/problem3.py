"""Problem description for one D3Q19 elastic-wave run: volume, face flags,
medium, sponges, sources, receivers, and the seeded volume workloads. Inputs
only -- no scheme arithmetic.

Faces are ordered top (z = 0), bottom (z = nz-1), left (x = 0), right
(x = nx-1), front (y = 0), back (y = ny-1); x is the fast index and z grows
with depth. Free surfaces are allowed on the top and bottom faces only.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

from .problem import BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, default_sponge_profile
from .configs import lame_from_poisson

FACES = ("top", "bottom", "left", "right", "front", "back")


@dataclasses.dataclass
class Source3:
    """Gaussian-in-space, Ricker-in-time body force (paper Sec. 5) in 3-D."""
    x: float
    y: float
    z: float
    sigma: float
    dir_x: float
    dir_y: float
    dir_z: float
    amp: float = 1.0
    period: float = 40.0
    t0: float = 60.0

    def as_tuple(self) -> Tuple[float, ...]:
        return (self.x, self.y, self.z, self.sigma, self.dir_x, self.dir_y, self.dir_z,
                self.amp, self.period, self.t0)


@dataclasses.dataclass
class Problem3:
    nx: int
    ny: int
    nz: int
    faces: Tuple[int, int, int, int, int, int]
    lam: object                               # scalar or (nz, ny, nx)
    mu: object
    rho0: object = 1.0
    tau: float = 1.0
    sponge_thick: Tuple[int, ...] = (0, 0, 0, 0, 0, 0)
    sponge_profiles: Tuple[Optional[np.ndarray], ...] = (None,) * 6
    sources: List[Source3] = dataclasses.field(default_factory=list)
    receivers: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros((0, 3), np.int32))
    comp_mask: int = 7                        # bit0 v_x, bit1 v_y, bit2 v_z
    nsteps: int = 0
    name: str = ""
    q: int = 19                               # lattice: D3Q19 or D3Q27

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def ncomp(self) -> int:
        return sum((self.comp_mask >> a) & 1 for a in range(3))

    @property
    def nrec(self) -> int:
        return int(self.receivers.shape[0])

    def full(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        out = []
        for v in (self.lam, self.mu, self.rho0):
            a = np.asarray(v, dtype=np.float64)
            if a.ndim == 0:
                a = np.full(self.shape, float(a))
            elif a.shape != self.shape:
                raise ValueError("medium field has the wrong shape")
            out.append(np.ascontiguousarray(a))
        return out[0], out[1], out[2]

    def profile(self, face: int) -> np.ndarray:
        t = self.sponge_thick[face]
        if t == 0:
            return np.zeros(0)
        return np.asarray(self.sponge_profiles[face], dtype=np.float64)[:t]

    def replace(self, **kw) -> "Problem3":
        return dataclasses.replace(self, **kw)


def surface_receivers(nx: int, ny: int, stride: int = 1, z: int = 0) -> np.ndarray:
    """A receiver every ``stride`` cells of the plane z, x fastest."""
    ys, xs = np.meshgrid(np.arange(0, ny, stride), np.arange(0, nx, stride), indexing="ij")
    zs = np.full(xs.size, z)
    return np.stack([xs.ravel(), ys.ravel(), zs], axis=1).astype(np.int32)


def volume_half_space(n: int = 256, nz: Optional[int] = None, nsteps: int = 2000,
                      nu: float = 0.25, sponge: int = 24, src_depth: int = 12,
                      top: int = BC_FREE0, stride: int = 4, q: int = 19) -> Problem3:
    """The plain workload in three dimensions: an n x n x nz half-space with a
    free surface on top, sponges on the bottom (rigid behind it) and the four
    sides (periodic behind them), homogeneous solid, a vertical Ricker source
    (sigma 3) at depth src_depth under the centre, receivers on every
    ``stride``-th surface cell recording v_z."""
    nz = n if nz is None else nz
    lam, mu = lame_from_poisson(nu)
    prof = default_sponge_profile(sponge)
    return Problem3(
        nx=n, ny=n, nz=nz,
        faces=(top, BC_RIGID, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC),
        lam=lam, mu=mu, rho0=1.0, tau=1.0,
        sponge_thick=(0, sponge, sponge, sponge, sponge, sponge),
        sponge_profiles=(None, prof, prof, prof, prof, prof),
        sources=[Source3(n / 2.0, n / 2.0, float(src_depth), 3.0, 0.0, 0.0, 1.0, 1.0, 40.0, 60.0)],
        receivers=surface_receivers(n, n, stride), comp_mask=4, nsteps=nsteps,
        name="volume_half_space", q=q)


def volume_field(nx: int = 72, ny: int = 40, nz: int = 34, seed: int = 5, nsteps: int = 40,
                 faces=(BC_PERIODIC,) * 6, tau: float = 0.9, q: int = 19) -> Problem3:
    """A cell-wise random solid (mu in [0.036, 0.044], nu in [0.1, 0.3]) with
    an oblique source and scattered receivers recording all three components."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    mu = rng.uniform(0.036, 0.044, shape)
    nu = rng.uniform(0.1, 0.3, shape)
    lam = 2 * nu * mu / (1 - 2 * nu)
    rho0 = rng.uniform(0.8, 1.2, shape)
    rec = np.stack([rng.integers(0, nx, 24), rng.integers(0, ny, 24),
                    rng.integers(0, nz, 24)], axis=1).astype(np.int32)
    d = np.array([0.6, -0.3, 0.74])
    d /= np.linalg.norm(d)
    return Problem3(nx=nx, ny=ny, nz=nz, faces=tuple(faces), lam=lam, mu=mu, rho0=rho0,
                    tau=tau, sources=[Source3(nx * 0.4, ny * 0.55, nz * 0.45, 2.5, d[0], d[1], d[2],
                                              1.0, 10.0, 12.0)],
                    receivers=rec, comp_mask=7, nsteps=nsteps, name="volume_field", q=q)


__all__ = ["FACES", "Source3", "Problem3", "surface_receivers", "volume_half_space",
           "volume_field", "BC_FREE", "BC_FREE0", "BC_PERIODIC", "BC_RIGID"]
