"""Problem description for one D2Q9 elastic-wave run: grid, boundary flags,
medium, sponge, sources, receivers. Inputs only -- no scheme arithmetic."""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

BC_PERIODIC = 0
BC_FREE = 1        # free surface, linear extrapolation to the interface (as printed)
BC_RIGID = 2
BC_FREE0 = 3       # free surface, zero-order extrapolation (stabilised variant)

EDGES = ("top", "bottom", "left", "right")


@dataclasses.dataclass
class Source:
    """Gaussian-in-space, Ricker-in-time body force (paper Sec. 5)."""
    x: float
    y: float
    sigma: float
    dir_x: float
    dir_y: float
    amp: float = 1.0
    period: float = 40.0
    t0: float = 60.0

    def as_tuple(self) -> Tuple[float, ...]:
        return (self.x, self.y, self.sigma, self.dir_x, self.dir_y, self.amp,
                self.period, self.t0)


@dataclasses.dataclass
class Medium:
    """Lame coefficients and density.

    ``kind`` is ``"homogeneous"`` (scalars), ``"layered"`` (one value per row,
    arrays of length ny) or ``"field"`` (arrays of shape (ny, nx)).
    """
    kind: str
    lam: object
    mu: object
    rho0: object

    def full(self, ny: int, nx: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        out = []
        for v in (self.lam, self.mu, self.rho0):
            a = np.asarray(v, dtype=np.float64)
            if a.ndim == 0:
                a = np.full((ny, nx), float(a))
            elif a.ndim == 1:
                if a.shape[0] != ny:
                    raise ValueError("layered medium needs one value per row")
                a = np.repeat(a[:, None], nx, axis=1)
            elif a.shape != (ny, nx):
                raise ValueError("medium field has the wrong shape")
            out.append(np.ascontiguousarray(a))
        return out[0], out[1], out[2]

    def rows(self, ny: int) -> Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]]:
        """Per-row values when the medium depends on depth only, else None."""
        if self.kind == "field":
            return None
        res = []
        for v in (self.lam, self.mu, self.rho0):
            a = np.asarray(v, dtype=np.float64)
            res.append(np.full(ny, float(a)) if a.ndim == 0 else a.copy())
        return res[0], res[1], res[2]


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    bc: Tuple[int, int, int, int]            # top, bottom, left, right
    medium: Medium
    tau: float = 1.0
    rigid_row: int = -1                       # wall between rows r-1 and r
    sponge_thick: Tuple[int, int, int, int] = (0, 0, 0, 0)
    sponge_profiles: Tuple[Optional[np.ndarray], ...] = (None, None, None, None)
    sources: List[Source] = dataclasses.field(default_factory=list)
    receivers: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros((0, 2), np.int32))
    comp_mask: int = 3                        # bit0 v_x, bit1 v_y
    nsteps: int = 0
    dtype: str = "f64"
    name: str = ""

    @property
    def ncomp(self) -> int:
        return (self.comp_mask & 1) + ((self.comp_mask >> 1) & 1)

    @property
    def nrec(self) -> int:
        return int(self.receivers.shape[0])

    def profile(self, edge: int) -> np.ndarray:
        p = self.sponge_profiles[edge]
        t = self.sponge_thick[edge]
        if t == 0:
            return np.zeros(0)
        return np.asarray(p, dtype=np.float64)[:t]

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def default_sponge_profile(thick: int, a_max: float = 0.1) -> np.ndarray:
    """Smoothly increasing damping A[k] = a_max ((L - k)/L)^2, k = cells from
    the outer edge (the paper asks only for a smooth increase, Sec. 6.4)."""
    if thick <= 0:
        return np.zeros(0)
    k = np.arange(thick, dtype=np.float64)
    return a_max * ((thick - k) / thick) ** 2


def round_half_away(v: float) -> int:
    return int(math.floor(v + 0.5)) if v >= 0 else -int(math.floor(-v + 0.5))


def ring_receivers(cx: float, cy: float, radius: float, n: int) -> np.ndarray:
    """n stations on a circle, snapped to the nearest cell (half away from 0)."""
    pts = []
    for k in range(n):
        a = 2.0 * math.pi * k / n
        pts.append((round_half_away(cx + radius * math.cos(a)),
                    round_half_away(cy + radius * math.sin(a))))
    return np.asarray(pts, dtype=np.int32).reshape(-1, 2)


def row_receivers(nx: int, row: int = 0, x0: int = 0, stride: int = 1) -> np.ndarray:
    xs = np.arange(x0, nx, stride, dtype=np.int32)
    return np.stack([xs, np.full_like(xs, row)], axis=1).astype(np.int32)
